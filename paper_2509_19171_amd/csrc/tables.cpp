// Host construction of the spectral-element tables: GLL nodes and weights,
// the 1D derivative matrix, the modal filter matrix and the lattice.
#include <cmath>
#include <cstring>

#include "sel_internal.h"

namespace sel {

// Legendre values P_0..P_n at x by the three-term recurrence.
static void legendre_all(int n, double x, double *P)
{
    P[0] = 1.0;
    if (n >= 1) P[1] = x;
    for (int k = 2; k <= n; ++k) P[k] = ((2.0 * k - 1.0) * x * P[k - 1] - (k - 1.0) * P[k - 2]) / k;
}

// GLL nodes (Sec. 2.2): the zeros of (1 - x^2) P_N'(x). Newton's method on
// x P_N - P_{N-1}, which has the same zeros (it equals (x^2 - 1) P_N' / N), with
// derivative (N + 1) P_N, started from the Chebyshev-Gauss-Lobatto points.
// Weights rho_i = 2 / (N (N + 1) P_N(x_i)^2). Derivative matrix from the
// closed form of the GLL Lagrange basis:
//   D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j)), D_00 = -N(N+1)/4, D_NN = N(N+1)/4.
int build_gll(int N, Tables &t)
{
    if (N < 1 || N + 1 > kMaxN1) return -1;
    int n1 = N + 1;
    double x[kMaxN1], P[kMaxN1];
    for (int i = 0; i < n1; ++i) x[i] = -std::cos(M_PI * i / N);
    for (int it = 0; it < 200; ++it) {
        double dmax = 0.0;
        for (int i = 0; i < n1; ++i) {
            legendre_all(N, x[i], P);
            double dx = (x[i] * P[N] - P[N - 1]) / (n1 * P[N]);
            x[i] -= dx;
            dmax = std::fmax(dmax, std::fabs(dx));
        }
        if (dmax < 1e-16) break;
    }
    x[0] = -1.0;
    x[N] = 1.0;
    t.N = N;
    double PN[kMaxN1];
    for (int i = 0; i < n1; ++i) {
        legendre_all(N, x[i], P);
        PN[i] = P[N];
        t.xi[i] = x[i];
        t.w[i] = 2.0 / (N * (N + 1.0) * P[N] * P[N]);
    }
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            double v = 0.0;
            if (i != j) v = PN[i] / (PN[j] * (x[i] - x[j]));
            else if (i == 0) v = -N * (N + 1.0) / 4.0;
            else if (i == N) v = N * (N + 1.0) / 4.0;
            t.D[i * n1 + j] = v;
        }
    for (int i = 0; i < n1 * n1; ++i) t.F[i] = 0.0;
    for (int i = 0; i < n1; ++i) t.F[i * n1 + i] = 1.0;
    return 0;
}

// Filter matrix (Sec. 2.2.3). The nodal values are expanded in the basis
// phi_0 = P_0, phi_1 = P_1, phi_k = P_k - P_{k-2}, each coefficient is scaled
// by sigma_k, and the result is evaluated at the nodes. The expansion goes
// through the discrete Legendre transform on the GLL nodes:
//   a_k = (sum_i w_i u_i P_k(x_i)) / g_k, g_k = 2/(2k+1) (k < N), g_N = 2/N;
//   phi coefficients p_k = a_k + p_{k+2} from k = N down (p_{N+1} = p_{N+2} = 0).
// Rows 0 and N of the exact matrix are unit vectors (phi_k vanishes at +-1 for
// k >= 2) and the matrix is reversal-symmetric; both are imposed exactly so
// that face values of neighbouring elements stay bit-identical.
int build_filter(int N, int type, int kc, double amp, double order, Tables &t)
{
    int n1 = N + 1;
    if (type == SEL_FILTER_NONE) {
        for (int i = 0; i < n1 * n1; ++i) t.F[i] = 0.0;
        for (int i = 0; i < n1; ++i) t.F[i * n1 + i] = 1.0;
        return 0;
    }
    if (kc < 0 || kc >= N) return -1;
    double sigma[kMaxN1];
    for (int k = 0; k < n1; ++k) {
        double q = (k > kc) ? double(k - kc) / double(N - kc) : 0.0;
        if (k <= kc) sigma[k] = 1.0;
        else if (type == SEL_FILTER_QUAD) sigma[k] = 1.0 - amp * q * q;
        else if (type == SEL_FILTER_EXP) sigma[k] = std::exp(-amp * std::pow(q, order));
        else return -1;
    }
    double Pn[kMaxN1][kMaxN1];  // Pn[i][k] = P_k(x_i)
    for (int i = 0; i < n1; ++i) legendre_all(N, t.xi[i], Pn[i]);
    double F[kMaxN1 * kMaxN1];
    for (int j = 0; j < n1; ++j) {  // column j: filtered unit vector e_j
        double a[kMaxN1 + 2] = {}, p[kMaxN1 + 2] = {}, ap[kMaxN1 + 2] = {};
        for (int k = 0; k < n1; ++k) {
            double gk = (k < N) ? 2.0 / (2.0 * k + 1.0) : 2.0 / N;
            a[k] = t.w[j] * Pn[j][k] / gk;
        }
        for (int k = N; k >= 0; --k) p[k] = a[k] + p[k + 2];
        for (int k = 0; k < n1; ++k) p[k] *= sigma[k];
        for (int k = 0; k < n1; ++k) ap[k] = p[k] - p[k + 2];
        for (int i = 0; i < n1; ++i) {
            double s = 0.0;
            for (int k = 0; k < n1; ++k) s += ap[k] * Pn[i][k];
            F[i * n1 + j] = s;
        }
    }
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j)
            t.F[i * n1 + j] = 0.5 * (F[i * n1 + j] + F[(N - i) * n1 + (N - j)]);
    for (int j = 0; j < n1; ++j) {
        t.F[0 * n1 + j] = (j == 0) ? 1.0 : 0.0;
        t.F[N * n1 + j] = (j == N) ? 1.0 : 0.0;
    }
    return 0;
}

// Lattice (Sec. 2.1): a = a0 + 3 a1 (+ 9 a2), component values {0, +1, -1};
// D3Q19 keeps the |e|^2 <= 2 entries. Weights by |e|^2.
int build_lattice(int dim, int Q, HostLattice &L)
{
    static const int comp[3] = {0, 1, -1};
    int n = 0;
    int full = (dim == 2) ? 9 : 27;
    if (!((dim == 2 && Q == 9) || (dim == 3 && (Q == 19 || Q == 27)))) return -1;
    for (int f = 0; f < full; ++f) {
        int c[3] = {comp[f % 3], comp[(f / 3) % 3], dim == 3 ? comp[f / 9] : 0};
        int s2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        if (Q == 19 && s2 > 2) continue;
        for (int k = 0; k < 3; ++k) L.e[n][k] = c[k];
        static const double w9[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
        static const double w19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
        static const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
        L.t[n] = (Q == 9) ? w9[s2] : (Q == 19) ? w19[s2] : w27[s2];
        ++n;
    }
    L.Q = n;
    for (int a = 0; a < n; ++a) {
        L.opp[a] = -1;
        for (int b = 0; b < n; ++b)
            if (L.e[b][0] == -L.e[a][0] && L.e[b][1] == -L.e[a][1] && L.e[b][2] == -L.e[a][2]) L.opp[a] = b;
    }
    return 0;
}

}  // namespace sel

namespace sel {

// Projection of an Nf-nodal line onto the Nc-nodal line of the same element
// (learned-closure coarse graining): expansion in the basis phi_0 = P_0,
// phi_1 = P_1, phi_k = P_k - P_{k-2} through the discrete Legendre transform,
// truncation to k <= Nc, evaluation at the Nc GLL nodes. Pm[ic][jf].
// phi_k vanishes at +-1 for k >= 2 and phi_0, phi_1 are kept, so the end rows
// are unit vectors; they are set exactly, which keeps coarse face values a
// function of the fine face values alone (identical on both sides of a face).
int build_projection(int Nf, int Nc, double *Pm)
{
    if (Nc > Nf || Nc < 1) return -1;
    Tables tf, tc;
    if (build_gll(Nf, tf) || build_gll(Nc, tc)) return -1;
    const int nf1 = Nf + 1, nc1 = Nc + 1;
    double Pf[kMaxN1][kMaxN1], Pc[kMaxN1][kMaxN1];
    for (int i = 0; i < nf1; ++i) legendre_all(Nf, tf.xi[i], Pf[i]);
    for (int i = 0; i < nc1; ++i) legendre_all(Nf, tc.xi[i], Pc[i]);
    for (int j = 0; j < nf1; ++j) {
        double a[kMaxN1 + 2] = {}, p[kMaxN1 + 2] = {};
        for (int k = 0; k < nf1; ++k) {
            double gk = (k < Nf) ? 2.0 / (2.0 * k + 1.0) : 2.0 / Nf;
            a[k] = tf.w[j] * Pf[j][k] / gk;
        }
        for (int k = Nf; k >= 0; --k) p[k] = a[k] + p[k + 2];
        for (int i = 0; i < nc1; ++i) {
            double s = 0.0;
            for (int k = 0; k <= Nc; ++k) {
                double phi = (k >= 2) ? Pc[i][k] - Pc[i][k - 2] : Pc[i][k];
                s += p[k] * phi;
            }
            Pm[i * nf1 + j] = s;
        }
    }
    for (int j = 0; j < nf1; ++j) {
        Pm[0 * nf1 + j] = (j == 0) ? 1.0 : 0.0;
        Pm[Nc * nf1 + j] = (j == Nf) ? 1.0 : 0.0;
    }
    return 0;
}

}  // namespace sel
