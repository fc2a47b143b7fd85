/*
 * sel_oracle.c -- plain, slow, FP64 CPU oracle of the filtered spectral-element
 * lattice Boltzmann (SELBM) time step with flux bounce-back (FBB) walls of
 * Zhao, Patel, Lin, Min & Lee, "A flux bounce-back scheme for the filtered
 * Spectral Element Lattice Boltzmann Method" (arXiv:2509.19171).
 *
 * THIS FILE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load the library built from it.
 * The HIP library never links, loads or calls it, and the two share no code,
 * header, table or constant generator.
 *
 * Every routine states the passage of the paper it follows. Readings taken
 * where the paper is silent or garbled are stated where they are used:
 *   R1  D-hat is the derivative of the Lagrange basis through the GLL nodes,
 *       D_ij = l_j'(xi_i) (Sec. 2.2 names the 1D derivative matrix but does
 *       not print it); evaluated with the barycentric product formula.
 *   R2  The convection matrix is evaluated with nodal GLL quadrature at the
 *       solution nodes (the same quadrature as the lumped mass of Sec. 2.2),
 *       so (C_a f)_i = wJ_i e_a . grad f(x_i).
 *   R3  The geometric factor G_ij of Sec. 2.2 (printed with a stray sum) is
 *       read as G_mk = w w w J dr_m/dx_k, one diagonal block per (m,k).
 *   R4  Elements are coupled by continuous-Galerkin assembly (direct
 *       stiffness summation): the element contributions C_a f and R(n.j) are
 *       summed at shared nodes and divided by the assembled lumped mass
 *       (Sec. 2.2.1: the flux is integrated only on the outer boundary).
 *   R5  The FBB surface term uses the outward unit normal n and the surface
 *       GLL quadrature w_s J_s of the wall face; the flux enters only for
 *       incoming directions n.e_a < 0 (Sec. 2.2.1, Lax-Friedrichs flux and
 *       bounce-back jump with wall velocity u_b, reference density rho0).
 *   R6  The spatial operator of Sec. 2.2.2, printed as I + M^-1 (R - C), is
 *       read as L f = M^-1 (R(n.j) - C f) + F*: the "I" is the leading-order
 *       force F* of the streaming equation. F = rho g is frozen at the
 *       collision of the step.
 *   R7  Time marching: the text names the third-order SSP Runge-Kutta method;
 *       rk = 0 is the Shu-Osher SSPRK3. The four printed stage formulas are
 *       rk = 1, with L applied linearly to the printed combinations of stage
 *       values, i.e. L(sum c_k f_k) := sum c_k L(f_k), which weights the
 *       constant part of the affine L by sum c_k.
 *   R8  Filter basis (Sec. 2.2.3 defers to the cited filter paper): phi_0 = L_0,
 *       phi_1 = L_1, phi_k = L_k - L_{k-2}; the filter F = Phi diag(sigma)
 *       Phi^-1 acts per direction, mode index k per direction.
 *   R9  Step order (Sec. 2.2, scheme summary): collide -> SSPRK streaming with
 *       F* and the wall flux -> filter -> moments. The stage-0 state of the
 *       streaming is the post-collision f* (Eq. perfect1).
 *   R10 Moments carry no half-force shift: rho u = sum e f-bar (Eq. momentum).
 *   R11 Discontinuous-Galerkin coupling (the alternative the introduction
 *       sets the method against, with the flux of the cited DG-LBM work):
 *       every element keeps its own copy of its face nodes, the mass is the
 *       element's own lumped wJ (no assembly), and every face that is not a
 *       wall adds the upwind flux of the velocities entering the element,
 *       (n.e_a) w_s J_s (f_a - f_a^out) for n.e_a < 0, with f^out the value
 *       at the coincident node of the element across the face (same node
 *       id); wall faces keep the FBB term of R5. A face whose nodes repeat an
 *       id (one element along a periodic direction) is rejected: its
 *       coincident nodes would be ambiguous.
 *   R12 The force density of Sec. 2.1 is F = rho g + F_n(x): a body
 *       acceleration plus an optional force density per node (the pipe case
 *       of Sec. 3.5 adds a perturbation force of this kind). Like rho g it
 *       is taken at the collision of the step and frozen for its stages.
 *
 * Conventions shared with the public interface (the interface documents
 * them; this file re-states them in its own code):
 *   node index  i + (N+1) j + (N+1)^2 k, r fastest;
 *   xyz [E][np][dim], rho [E][np], u [E][np][dim], f [E][Q][np];
 *   faces ordered (r-, r+, s-, s+, t-, t+); tag 0 = interior/periodic,
 *   tag k >= 1 = wall k with velocity wall_u[k-1][dim];
 *   velocity a = a0 + 3 a1 (+ 9 a2) with component value {0, +1, -1}[a_i];
 *   D3Q19 keeps the D3Q27 entries with |e|^2 <= 2 in the same order.
 * Units: lattice speed 1, c_s^2 = 1/3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN1 24 /* N <= 23 */
#define OR_MAXQ 27

/* ------------------------------------------------------------------------ */
/* Legendre polynomials by the three-term recurrence.                       */
/* ------------------------------------------------------------------------ */
static void or_legendre(int n, double x, double *Ln, double *dLn)
{
    /* (k+1) L_{k+1} = (2k+1) x L_k - k L_{k-1};  L'_{k+1} = L'_{k-1} + (2k+1) L_k */
    double L0 = 1.0, L1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) {
        *Ln = 1.0;
        *dLn = 0.0;
        return;
    }
    for (int k = 1; k < n; ++k) {
        double L2 = ((2.0 * k + 1.0) * x * L1 - k * L0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * L1;
        L0 = L1;
        L1 = L2;
        d0 = d1;
        d1 = d2;
    }
    *Ln = L1;
    *dLn = d1;
}

int oracle_legendre(int n, double x, double *Ln, double *dLn)
{
    if (n < 0) return -1;
    or_legendre(n, x, Ln, dLn);
    return 0;
}

/* GLL nodes and weights (Sec. 2.2): the nodes are -1, +1 and the roots of
 * L_N'; the weights are rho_i = 2 / (N (N+1) L_N(xi_i)^2).
 * The roots are found by Newton's method on L_N', with L_N'' taken from the
 * Legendre differential equation (1-x^2) L'' = 2x L' - N(N+1) L. */
int oracle_gll(int N, double *xi, double *w)
{
    if (N < 1 || N + 1 > OR_MAXN1) return -1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double L, dL;
            or_legendre(N, x, &L, &dL);
            double d2L = (2.0 * x * dL - N * (N + 1.0) * L) / (1.0 - x * x);
            double dx = dL / d2L;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double L, dL;
        or_legendre(N, xi[i], &L, &dL);
        w[i] = 2.0 / (N * (N + 1.0) * L * L);
    }
    return 0;
}

/* 1D derivative matrix (reading R1): D_ij = l_j'(xi_i) for the Lagrange
 * basis through the nodes, barycentric form:
 *   c_i = prod_{m != i} (xi_i - xi_m);
 *   D_ij = (c_i / c_j) / (xi_i - xi_j)  (i != j);  D_ii = sum_{m != i} 1/(xi_i - xi_m). */
int oracle_dmat(int N, const double *xi, double *D)
{
    int n1 = N + 1;
    double c[OR_MAXN1];
    if (N < 1 || n1 > OR_MAXN1) return -1;
    for (int i = 0; i < n1; ++i) {
        c[i] = 1.0;
        for (int m = 0; m < n1; ++m)
            if (m != i) c[i] *= (xi[i] - xi[m]);
    }
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            if (i != j) {
                D[i * n1 + j] = (c[i] / c[j]) / (xi[i] - xi[j]);
            } else {
                double s = 0.0;
                for (int m = 0; m < n1; ++m)
                    if (m != i) s += 1.0 / (xi[i] - xi[m]);
                D[i * n1 + j] = s;
            }
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Lattice (Sec. 2.1): velocities e_a, weights t_a, opposite index.          */
/* D2Q9 weights 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27,      */
/* 1/54, 1/216 by |e|^2 (textbook values of the lattices the paper names).   */
/* ------------------------------------------------------------------------ */
int oracle_lattice(int dim, int Q, double *e /*[Q][3]*/, double *t, int *opp)
{
    static const int comp[3] = {0, 1, -1};
    int cnt = 0;
    int ev[OR_MAXQ][3];
    if (dim == 2 && Q == 9) {
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                ev[cnt][0] = comp[a];
                ev[cnt][1] = comp[b];
                ev[cnt][2] = 0;
                ++cnt;
            }
    } else if (dim == 3 && (Q == 27 || Q == 19)) {
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    int s = comp[a] * comp[a] + comp[b] * comp[b] + comp[c] * comp[c];
                    if (Q == 19 && s > 2) continue;
                    ev[cnt][0] = comp[a];
                    ev[cnt][1] = comp[b];
                    ev[cnt][2] = comp[c];
                    ++cnt;
                }
    } else {
        return -1;
    }
    for (int a = 0; a < Q; ++a) {
        int s = ev[a][0] * ev[a][0] + ev[a][1] * ev[a][1] + ev[a][2] * ev[a][2];
        double wt;
        if (Q == 9) wt = (s == 0) ? 4.0 / 9.0 : (s == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
        else if (Q == 19) wt = (s == 0) ? 1.0 / 3.0 : (s == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        else wt = (s == 0) ? 8.0 / 27.0 : (s == 1) ? 2.0 / 27.0 : (s == 2) ? 1.0 / 54.0 : 1.0 / 216.0;
        t[a] = wt;
        for (int k = 0; k < 3; ++k) e[3 * a + k] = (double)ev[a][k];
        opp[a] = -1;
        for (int b = 0; b < Q; ++b)
            if (ev[b][0] == -ev[a][0] && ev[b][1] == -ev[a][1] && ev[b][2] == -ev[a][2]) opp[a] = b;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Explicit modal filter (Sec. 2.2.3), reading R8.                           */
/*   sigma_k = 1 - gamma ((k - kc)/(N - kc))^2 for k > kc, else 1  (type 1)  */
/*   sigma_k = exp(-alpha ((k - kc)/(N - kc))^s) for k > kc, else 1 (type 2) */
/*   F = Phi diag(sigma) Phi^-1, Phi_ik = phi_k(xi_i).                       */
/* ------------------------------------------------------------------------ */
int oracle_filter_sigma(int N, int type, int kc, double amp, double order, double *sigma)
{
    for (int k = 0; k <= N; ++k) {
        double s = 1.0;
        if (type != 0 && k > kc && N > kc) {
            double q = (double)(k - kc) / (double)(N - kc);
            if (type == 1) s = 1.0 - amp * q * q;
            else if (type == 2) s = exp(-amp * pow(q, order));
            else return -1;
        }
        sigma[k] = s;
    }
    return 0;
}

/* Gauss-Jordan inverse with partial pivoting of an n x n matrix. */
static int or_invert(int n, const double *A, double *Ainv)
{
    double M[OR_MAXN1][2 * OR_MAXN1];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) M[i][j] = (j < n) ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(M[i][c]) > fabs(M[p][c])) p = i;
        if (M[p][c] == 0.0) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double tmp = M[c][j];
                M[c][j] = M[p][j];
                M[p][j] = tmp;
            }
        double piv = M[c][c];
        for (int j = 0; j < 2 * n; ++j) M[c][j] /= piv;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            double fac = M[i][c];
            for (int j = 0; j < 2 * n; ++j) M[i][j] -= fac * M[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = M[i][n + j];
    return 0;
}

int oracle_filter_matrix(int N, const double *xi, int type, int kc, double amp, double order,
                         double *F)
{
    int n1 = N + 1;
    double Phi[OR_MAXN1 * OR_MAXN1], Pinv[OR_MAXN1 * OR_MAXN1], sigma[OR_MAXN1];
    if (N < 1 || n1 > OR_MAXN1) return -1;
    if (oracle_filter_sigma(N, type, kc, amp, order, sigma)) return -1;
    for (int i = 0; i < n1; ++i)
        for (int k = 0; k < n1; ++k) {
            double Lk, dLk, Lk2, dLk2;
            or_legendre(k, xi[i], &Lk, &dLk);
            if (k >= 2) {
                or_legendre(k - 2, xi[i], &Lk2, &dLk2);
                Phi[i * n1 + k] = Lk - Lk2;
            } else {
                Phi[i * n1 + k] = Lk;
            }
        }
    if (or_invert(n1, Phi, Pinv)) return -1;
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            double s = 0.0;
            for (int k = 0; k < n1; ++k) s += Phi[i * n1 + k] * sigma[k] * Pinv[k * n1 + j];
            F[i * n1 + j] = s;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Simulation state.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct oracle_sim {
    int dim, N, n1, np, Q, nface;
    int64_t E;
    double xi[OR_MAXN1], w[OR_MAXN1], D[OR_MAXN1 * OR_MAXN1];
    double e[OR_MAXQ * 3], t[OR_MAXQ];
    int opp[OR_MAXQ];
    double cs2;
    double rho0, nu, dt, tau, g[3];
    int rk;
    int filter_on;
    double Ff[OR_MAXN1 * OR_MAXN1];
    /* mesh */
    int64_t *gid;     /* [E][np] */
    int32_t *ftag;    /* [E][2 dim] */
    int ntags;
    double *wall_u;   /* [ntags][3] */
    double *J;        /* [E][np] */
    double *wJ;       /* [E][np] */
    double *G;        /* [E][np][3][3]  wJ dr_m/dx_k */
    double *Mg;       /* [E np] assembled lumped mass, indexed by global id */
    int dg;           /* coupling: 0 continuous (R4), 1 discontinuous (R11) */
    int nfn;          /* nodes per face */
    int *fnode;       /* [2 dim][nfn] local index of the k-th node of each face (increasing) */
    int64_t *if_el2;  /* [E][2 dim] element across each face (R11), -1 for wall faces */
    int32_t *if_p2;   /* [E][2 dim][nfn] its local index of the coincident node */
    double *if_A;     /* [E][2 dim][nfn][3] w_s J_s n at the face nodes */
    int64_t nwf;      /* wall faces */
    int64_t *wf_el;   /* [nwf] element */
    int *wf_fc;       /* [nwf] face 0..2dim-1 */
    int *wf_tag;      /* [nwf] wall tag >= 1 */
    double *wf_A;     /* [nwf][np][3] w_s J_s n at the face nodes, 0 elsewhere */
    /* state */
    double *f;        /* [E][Q][np] f-bar */
    double *f0, *w1, *w2, *L0, *L1, *L2, *L3; /* work arrays [E][Q][np] */
    double *rt;       /* [E][Q][np] element contributions */
    double *rg;       /* [Q][E np] assembled sums by global id */
    double *rhoc;     /* [E][np] density at the collision of the step */
    double *dtau;     /* [E][np] relaxation-time increments (learned closure), NULL = 0 */
    double *Fn;       /* [E][np][3] force density added to rho g (reading R12), NULL = 0 */
    double time;
    int64_t nstep;
} oracle_sim;

static int64_t or_nv(const oracle_sim *s) { return s->E * (int64_t)s->Q * s->np; }

static void or_node_ijk(const oracle_sim *s, int p, int *ijk)
{
    ijk[0] = p % s->n1;
    ijk[1] = (p / s->n1) % s->n1;
    ijk[2] = (s->dim == 3) ? p / (s->n1 * s->n1) : 0;
}

static int or_node_index(const oracle_sim *s, const int *ijk)
{
    return ijk[0] + s->n1 * ijk[1] + (s->dim == 3 ? s->n1 * s->n1 * ijk[2] : 0);
}

/* Derivative of a nodal element field v (stride 'stride' between nodes)
 * along reference direction m at node p: (D_m v)_p, where D_r = I (x) D-hat
 * acts on the fastest index, D_s on the middle, D_t on the slowest
 * (Sec. 2.2, tensor-product derivative operators). */
static double or_dref(const oracle_sim *s, const double *v, int stride, int p, int m)
{
    int ijk[3], q[3];
    or_node_ijk(s, p, ijk);
    double acc = 0.0;
    for (int a = 0; a < s->n1; ++a) {
        q[0] = ijk[0];
        q[1] = ijk[1];
        q[2] = ijk[2];
        q[m] = a;
        acc += s->D[ijk[m] * s->n1 + a] * v[(int64_t)or_node_index(s, q) * stride];
    }
    return acc;
}

static double or_wprod(const oracle_sim *s, int p)
{
    int ijk[3];
    or_node_ijk(s, p, ijk);
    double wp = s->w[ijk[0]] * s->w[ijk[1]];
    if (s->dim == 3) wp *= s->w[ijk[2]];
    return wp;
}

/* Geometry (Sec. 2.2): A_km = dx_k/dr_m from the isoparametric map through
 * the given nodes, J = det A, dr/dx = A^-1, wJ = w w w J, and (reading R3)
 * G_mk = wJ dr_m/dx_k. Returns -2 if some J <= 0. */
static int or_geometry(oracle_sim *s, const double *xyz)
{
    int d = s->dim, np = s->np;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t el = 0; el < s->E; ++el) {
        const double *xe = xyz + el * (int64_t)np * d;
        for (int p = 0; p < np; ++p) {
            double A[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, B[3][3];
            for (int k = 0; k < d; ++k)
                for (int m = 0; m < d; ++m) A[k][m] = or_dref(s, xe + k, d, p, m);
            double J;
            if (d == 2) {
                J = A[0][0] * A[1][1] - A[0][1] * A[1][0];
                B[0][0] = A[1][1] / J;
                B[0][1] = -A[0][1] / J;
                B[1][0] = -A[1][0] / J;
                B[1][1] = A[0][0] / J;
            } else {
                J = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                    A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                    A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
                /* inverse = adjugate / det */
                B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / J;
                B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / J;
                B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / J;
                B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / J;
                B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / J;
                B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / J;
                B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / J;
                B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / J;
                B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / J;
            }
            if (!(J > 0.0)) bad += 1;
            int64_t ip = el * np + p;
            double wJ = or_wprod(s, p) * J;
            s->J[ip] = J;
            s->wJ[ip] = wJ;
            for (int m = 0; m < 3; ++m)
                for (int k = 0; k < 3; ++k)
                    s->G[ip * 9 + m * 3 + k] = (m < d && k < d) ? wJ * B[m][k] : 0.0;
        }
    }
    return bad ? -2 : 0;
}

/* Outward area-weighted normal w_s J_s n at node p of face fc of element el
 * (reading R5): the surface Jacobian vector is the cross product of the
 * tangent vectors of the face parametrisation (2D: the rotated tangent), with
 * the GLL weights of the tangential indices. */
static void or_face_normal(const oracle_sim *s, const double *xyz, int64_t el, int fc, int p,
                           double *An)
{
    int d = s->dim, m = fc / 2, side = fc % 2;
    const double *xe = xyz + el * (int64_t)s->np * d;
    int ijk[3];
    or_node_ijk(s, p, ijk);
    double T[3][3] = {{0}}; /* T[m'][k] = dx_k/dr_m' */
    for (int mm = 0; mm < d; ++mm)
        for (int k = 0; k < d; ++k) T[mm][k] = or_dref(s, xe + k, d, p, mm);
    double v[3] = {0, 0, 0}, wt = 1.0;
    if (d == 2) {
        int tdir = 1 - m;
        /* face r = const: cofactor (y_s, -x_s); face s = const: (-y_r, x_r) */
        if (m == 0) {
            v[0] = T[1][1];
            v[1] = -T[1][0];
        } else {
            v[0] = -T[0][1];
            v[1] = T[0][0];
        }
        wt = s->w[ijk[tdir]];
    } else {
        int a = (m + 1) % 3, b = (m + 2) % 3; /* cyclic: x_s x x_t, x_t x x_r, x_r x x_s */
        v[0] = T[a][1] * T[b][2] - T[a][2] * T[b][1];
        v[1] = T[a][2] * T[b][0] - T[a][0] * T[b][2];
        v[2] = T[a][0] * T[b][1] - T[a][1] * T[b][0];
        wt = s->w[ijk[a]] * s->w[ijk[b]];
    }
    double sg = side ? 1.0 : -1.0;
    for (int k = 0; k < 3; ++k) An[k] = sg * wt * v[k];
}


/* A node p lies on face fc when its index along the face's normal
 * direction is 0 (minus face) or N (plus face). */
static int or_on_face(const oracle_sim *s, int p, int fc)
{
    int ijk[3];
    or_node_ijk(s, p, ijk);
    return ijk[fc / 2] == ((fc % 2) ? s->N : 0);
}

/* Sorting of the faces by their node ids (reading R11): the ids of each face
 * are sorted, and faces compare lexicographically on them. */
static const int64_t *or_fkeys;
static int or_fkey_n;
static int or_cmp_face(const void *a, const void *b)
{
    const int64_t *x = or_fkeys + *(const int64_t *)a * or_fkey_n;
    const int64_t *y = or_fkeys + *(const int64_t *)b * or_fkey_n;
    for (int k = 0; k < or_fkey_n; ++k)
        if (x[k] != y[k]) return x[k] < y[k] ? -1 : 1;
    return 0;
}
static int or_cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Interface faces of the discontinuous coupling (reading R11): every face
 * that is not a wall is matched with the one other face carrying the same
 * node ids, and each of its nodes with the node of the same id there. The
 * area-weighted outward normals come from the face parametrisation (R5).
 * Returns nonzero for an unmatched face, a face matched more than once or a
 * face with a repeated node id. */
static int or_dg_faces(oracle_sim *s, const double *xyz)
{
    int nface = s->nface, np = s->np, n1 = s->n1;
    int nfn = (s->dim == 2) ? n1 : n1 * n1;
    int64_t nf = s->E * nface;
    s->nfn = nfn;
    s->fnode = (int *)malloc(sizeof(int) * nface * nfn);
    s->if_el2 = (int64_t *)malloc(sizeof(int64_t) * nf);
    s->if_p2 = (int32_t *)malloc(sizeof(int32_t) * nf * nfn);
    s->if_A = (double *)calloc((size_t)nf * nfn * 3, sizeof(double));
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * nf * nfn);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * nf);
    int rc = 1;
    if (!s->fnode || !s->if_el2 || !s->if_p2 || !s->if_A || !keys || !order) goto done;
    for (int fc = 0; fc < nface; ++fc) {
        int k = 0;
        for (int p = 0; p < np; ++p)
            if (or_on_face(s, p, fc)) s->fnode[fc * nfn + k++] = p;
    }
    int64_t nin = 0;
    for (int64_t f = 0; f < nf; ++f) {
        int64_t el = f / nface;
        int fc = (int)(f % nface);
        s->if_el2[f] = -1;
        if (s->ftag[f] > 0) continue;
        int64_t *kf = keys + nin * nfn;
        for (int k = 0; k < nfn; ++k) kf[k] = s->gid[el * np + s->fnode[fc * nfn + k]];
        qsort(kf, (size_t)nfn, sizeof(int64_t), or_cmp_i64);
        for (int k = 1; k < nfn; ++k)
            if (kf[k] == kf[k - 1]) goto done; /* repeated id on one face */
        order[nin++] = f;
    }
    /* sort the face numbers by key; keys are stored in face-list order */
    {
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (nin > 0 ? nin : 1));
        if (!idx) goto done;
        for (int64_t i = 0; i < nin; ++i) idx[i] = i;
        or_fkeys = keys;
        or_fkey_n = nfn;
        qsort(idx, (size_t)nin, sizeof(int64_t), or_cmp_face);
        for (int64_t i = 0; i < nin;) {
            int64_t j = i + 1;
            while (j < nin && or_cmp_face(&idx[i], &idx[j]) == 0) ++j;
            if (j - i != 2) {
                free(idx);
                goto done; /* unmatched, or more than two faces with these ids */
            }
            int64_t fa = order[idx[i]], fb = order[idx[i + 1]];
            s->if_el2[fa] = fb / nface;
            s->if_el2[fb] = fa / nface;
            for (int side = 0; side < 2; ++side) {
                int64_t f1 = side ? fb : fa, f2 = side ? fa : fb;
                int64_t el1 = f1 / nface, el2 = f2 / nface;
                int fc1 = (int)(f1 % nface), fc2 = (int)(f2 % nface);
                for (int k = 0; k < nfn; ++k) {
                    int p = s->fnode[fc1 * nfn + k];
                    int64_t gk = s->gid[el1 * np + p];
                    int found = -1;
                    for (int k2 = 0; k2 < nfn; ++k2) {
                        int p2 = s->fnode[fc2 * nfn + k2];
                        if (s->gid[el2 * np + p2] == gk) found = p2;
                    }
                    s->if_p2[f1 * nfn + k] = found;
                    or_face_normal(s, xyz, el1, fc1, p, s->if_A + (f1 * nfn + k) * 3);
                }
            }
            i = j;
        }
        free(idx);
    }
    rc = 0;
done:
    free(keys);
    free(order);
    return rc;
}

void oracle_destroy(oracle_sim *s)
{
    if (!s) return;
    free(s->gid);
    free(s->ftag);
    free(s->wall_u);
    free(s->J);
    free(s->wJ);
    free(s->G);
    free(s->Mg);
    free(s->fnode);
    free(s->if_el2);
    free(s->if_p2);
    free(s->if_A);
    free(s->wf_el);
    free(s->wf_fc);
    free(s->wf_tag);
    free(s->wf_A);
    free(s->f);
    free(s->f0);
    free(s->w1);
    free(s->w2);
    free(s->L0);
    free(s->L1);
    free(s->L2);
    free(s->L3);
    free(s->rt);
    free(s->rg);
    free(s->rhoc);
    free(s->dtau);
    free(s->Fn);
    free(s);
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Create the oracle for a mesh and the physical parameters.
 *   filter_type 0 none, 1 quadratic, 2 exponential (reading R8);
 *   rk 0 SSPRK3, 1 printed four-stage form (reading R7);
 *   coupling 0 continuous Galerkin (R4), 1 discontinuous Galerkin (R11).
 * Returns NULL on invalid input, J <= 0 or allocation failure. */
oracle_sim *oracle_create(int dim, int N, int64_t E, const double *xyz, const int64_t *gid,
                          const int32_t *face_tag, int ntags, const double *wall_u, int Q,
                          double rho0, double nu, double dt, const double *g, int filter_type,
                          int kc, double famp, double forder, int rk, int coupling)
{
    if ((dim != 2 && dim != 3) || N < 1 || N + 1 > OR_MAXN1 || E < 1 || dt <= 0.0 || nu <= 0.0)
        return NULL;
    if (rk != 0 && rk != 1) return NULL;
    if (coupling != 0 && coupling != 1) return NULL;
    oracle_sim *s = (oracle_sim *)calloc(1, sizeof(oracle_sim));
    if (!s) return NULL;
    s->dim = dim;
    s->N = N;
    s->n1 = N + 1;
    s->np = (dim == 2) ? s->n1 * s->n1 : s->n1 * s->n1 * s->n1;
    s->Q = Q;
    s->E = E;
    s->nface = 2 * dim;
    s->cs2 = 1.0 / 3.0;
    s->rho0 = rho0;
    s->nu = nu;
    s->dt = dt;
    /* nu = lambda c_s^2 and tau = lambda / dt (Sec. 2.1) */
    s->tau = (nu / s->cs2) / dt;
    for (int k = 0; k < 3; ++k) s->g[k] = (g && k < dim) ? g[k] : 0.0;
    s->rk = rk;
    if (oracle_lattice(dim, Q, s->e, s->t, s->opp)) goto fail;
    if (oracle_gll(N, s->xi, s->w)) goto fail;
    if (oracle_dmat(N, s->xi, s->D)) goto fail;
    s->filter_on = (filter_type != 0);
    if (s->filter_on && oracle_filter_matrix(N, s->xi, filter_type, kc, famp, forder, s->Ff)) goto fail;

    int64_t nl = E * s->np, nv = nl * Q;
    s->gid = (int64_t *)malloc(sizeof(int64_t) * nl);
    s->ftag = (int32_t *)malloc(sizeof(int32_t) * E * s->nface);
    s->ntags = ntags;
    s->wall_u = (double *)calloc((size_t)(ntags > 0 ? ntags : 1) * 3, sizeof(double));
    s->J = (double *)malloc(sizeof(double) * nl);
    s->wJ = (double *)malloc(sizeof(double) * nl);
    s->G = (double *)malloc(sizeof(double) * nl * 9);
    s->Mg = (double *)calloc((size_t)nl, sizeof(double));
    s->f = (double *)calloc((size_t)nv, sizeof(double));
    s->f0 = (double *)malloc(sizeof(double) * nv);
    s->w1 = (double *)malloc(sizeof(double) * nv);
    s->w2 = (double *)malloc(sizeof(double) * nv);
    s->L0 = (double *)malloc(sizeof(double) * nv);
    s->L1 = (double *)malloc(sizeof(double) * nv);
    s->L2 = (double *)malloc(sizeof(double) * nv);
    s->rt = (double *)malloc(sizeof(double) * nv);
    s->rg = (double *)malloc(sizeof(double) * nv);
    s->rhoc = (double *)malloc(sizeof(double) * nl);
    if (!s->gid || !s->ftag || !s->wall_u || !s->J || !s->wJ || !s->G || !s->Mg || !s->f ||
        !s->f0 || !s->w1 || !s->w2 || !s->L0 || !s->L1 || !s->L2 || !s->rt || !s->rg || !s->rhoc)
        goto fail;
    if (rk == 1) {
        s->L3 = (double *)malloc(sizeof(double) * nv);
        if (!s->L3) goto fail;
    }
    for (int64_t i = 0; i < nl; ++i) {
        if (gid[i] < 0 || gid[i] >= nl) goto fail;
        s->gid[i] = gid[i];
    }
    for (int64_t i = 0; i < E * s->nface; ++i) {
        int32_t tg = face_tag ? face_tag[i] : 0;
        if (tg < 0 || tg > ntags) goto fail;
        s->ftag[i] = tg;
    }
    for (int k = 0; k < ntags; ++k)
        for (int c = 0; c < dim; ++c) s->wall_u[3 * k + c] = wall_u[k * dim + c];

    if (or_geometry(s, xyz)) goto fail;

    /* Discontinuous coupling (reading R11): the elements across the faces,
     * then one assembly id per local node (no sharing). */
    s->dg = coupling;
    if (s->dg) {
        if (or_dg_faces(s, xyz)) goto fail;
        for (int64_t i = 0; i < nl; ++i) s->gid[i] = i;
    }

    /* Assembled lumped mass by global node (reading R4). */
    for (int64_t i = 0; i < nl; ++i) s->Mg[s->gid[i]] += s->wJ[i];

    /* Wall faces and their area-weighted outward normals (reading R5). */
    s->nwf = 0;
    for (int64_t i = 0; i < E * s->nface; ++i)
        if (s->ftag[i] > 0) s->nwf++;
    if (s->nwf > 0) {
        s->wf_el = (int64_t *)malloc(sizeof(int64_t) * s->nwf);
        s->wf_fc = (int *)malloc(sizeof(int) * s->nwf);
        s->wf_tag = (int *)malloc(sizeof(int) * s->nwf);
        s->wf_A = (double *)calloc((size_t)s->nwf * s->np * 3, sizeof(double));
        if (!s->wf_el || !s->wf_fc || !s->wf_tag || !s->wf_A) goto fail;
        int64_t c = 0;
        for (int64_t el = 0; el < E; ++el)
            for (int fc = 0; fc < s->nface; ++fc) {
                int tg = s->ftag[el * s->nface + fc];
                if (tg <= 0) continue;
                s->wf_el[c] = el;
                s->wf_fc[c] = fc;
                s->wf_tag[c] = tg;
                for (int p = 0; p < s->np; ++p)
                    if (or_on_face(s, p, fc)) or_face_normal(s, xyz, el, fc, p, s->wf_A + (c * s->np + p) * 3);
                ++c;
            }
    }
    return s;
fail:
    oracle_destroy(s);
    return NULL;
}

/* Equilibrium (Sec. 2.1, Eq. geq_s). */
static double or_feq(const oracle_sim *s, int a, double rho, const double *u)
{
    const double *e = s->e + 3 * a;
    double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double cs2 = s->cs2;
    return s->t[a] * rho * (1.0 + eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

/* Higher-order force F** (Sec. 2.1, Eq. f_c): t_a ((e.u) e / c_s^4 - u / c_s^2) . F */
static double or_fss(const oracle_sim *s, int a, const double *u, const double *F)
{
    const double *e = s->e + 3 * a;
    double cs2 = s->cs2;
    double acc = 0.0;
    double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
    for (int k = 0; k < 3; ++k) acc += (eu * e[k] / (cs2 * cs2) - u[k] / cs2) * F[k];
    return s->t[a] * acc;
}

/* Leading-order force F* (Sec. 2.1, Eq. body): t_a (e / c_s^2) . F */
static double or_fs(const oracle_sim *s, int a, const double *F)
{
    const double *e = s->e + 3 * a;
    return s->t[a] * (e[0] * F[0] + e[1] * F[1] + e[2] * F[2]) / s->cs2;
}

/* Moments of one node (Eqs. pressure, momentum; reading R10). */
static void or_moments_node(const oracle_sim *s, const double *fn, int64_t stride, double *rho,
                            double *u)
{
    double r = 0.0, m[3] = {0, 0, 0};
    for (int a = 0; a < s->Q; ++a) {
        double fa = fn[a * stride];
        r += fa;
        for (int k = 0; k < 3; ++k) m[k] += s->e[3 * a + k] * fa;
    }
    *rho = r;
    for (int k = 0; k < 3; ++k) u[k] = m[k] / r;
}

/* BGK collision with the higher-order force (Sec. 2.1):
 *   f-bar^eq = f^eq - dt F** / 2,  f* = f-bar - (f-bar - f-bar^eq)/(tau + 1/2) + dt F**,
 * with F = rho g. Writes f* and the density used for F. */
static void or_collide_all(const oracle_sim *s, const double *fb, double *fs, double *rhoc)
{
    int np = s->np, Q = s->Q;
#pragma omp parallel for schedule(static)
    for (int64_t el = 0; el < s->E; ++el)
        for (int p = 0; p < np; ++p) {
            const double *fn = fb + el * (int64_t)Q * np + p;
            double rho, u[3], F[3];
            or_moments_node(s, fn, np, &rho, u);
            for (int k = 0; k < 3; ++k) F[k] = rho * s->g[k] + (s->Fn ? s->Fn[(el * np + p) * 3 + k] : 0.0);
            /* relaxation time, plus the closure's increment when one is set */
            double tau = s->tau + (s->dtau ? s->dtau[el * np + p] : 0.0);
            for (int a = 0; a < Q; ++a) {
                double fss = or_fss(s, a, u, F);
                double fbeq = or_feq(s, a, rho, u) - 0.5 * s->dt * fss;
                double fa = fn[(int64_t)a * np];
                fs[el * (int64_t)Q * np + (int64_t)a * np + p] =
                    fa - (fa - fbeq) / (tau + 0.5) + s->dt * fss;
            }
            if (rhoc) rhoc[el * np + p] = rho;
        }
}

/* Element contributions (Sec. 2.2, Eqs. full, advection2; Sec. 2.2.1, Eq. entire):
 *   rt_a = -(C_a f_a) + R (n . j_a)
 *   (C_a f)_p = sum_k e_ak sum_m G_mk(p) (D_m f_a)_p       (readings R2, R3)
 *   R (n . j_a) at wall-face nodes = (w_s J_s n . e_a) [f_a]_bc for n . e_a < 0,
 *   [f_a]_bc = f_a - f_b - 2 t_a rho0 (e_a . u_b) / c_s^2, b = opposite(a). */
static void or_rhs_local(const oracle_sim *s, const double *f, double *rt)
{
    int np = s->np, Q = s->Q, d = s->dim;
#pragma omp parallel for schedule(static)
    for (int64_t el = 0; el < s->E; ++el)
        for (int a = 0; a < Q; ++a) {
            const double *fa = f + el * (int64_t)Q * np + (int64_t)a * np;
            const double *e = s->e + 3 * a;
            for (int p = 0; p < np; ++p) {
                const double *Gp = s->G + (el * np + p) * 9;
                double acc = 0.0;
                for (int m = 0; m < d; ++m) {
                    double dm = or_dref(s, fa, 1, p, m);
                    for (int k = 0; k < d; ++k) acc += e[k] * Gp[m * 3 + k] * dm;
                }
                rt[el * (int64_t)Q * np + (int64_t)a * np + p] = -acc;
            }
        }
    /* wall flux: serial over wall faces (few) */
    for (int64_t c = 0; c < s->nwf; ++c) {
        int64_t el = s->wf_el[c];
        int fc = s->wf_fc[c];
        const double *ub = s->wall_u + 3 * (s->wf_tag[c] - 1);
        for (int p = 0; p < np; ++p) {
            if (!or_on_face(s, p, fc)) continue;
            const double *A = s->wf_A + (c * np + p) * 3;
            for (int a = 0; a < Q; ++a) {
                const double *e = s->e + 3 * a;
                double ne = A[0] * e[0] + A[1] * e[1] + A[2] * e[2];
                if (ne < 0.0) {
                    int b = s->opp[a];
                    double fa = f[el * (int64_t)Q * np + (int64_t)a * np + p];
                    double fb = f[el * (int64_t)Q * np + (int64_t)b * np + p];
                    double eub = e[0] * ub[0] + e[1] * ub[1] + e[2] * ub[2];
                    double jump = fa - fb - 2.0 * s->t[a] * s->rho0 * eub / s->cs2;
                    rt[el * (int64_t)Q * np + (int64_t)a * np + p] += ne * jump;
                }
            }
        }
    }
    if (!s->dg) return;
    /* discontinuous coupling (reading R11): upwind flux of the entering
     * velocities on every interface face */
#pragma omp parallel for schedule(static)
    for (int64_t el = 0; el < s->E; ++el)
        for (int fc = 0; fc < s->nface; ++fc) {
            int64_t fi = el * s->nface + fc, el2 = s->if_el2[fi];
            if (el2 < 0) continue;
            for (int k = 0; k < s->nfn; ++k) {
                int p = s->fnode[fc * s->nfn + k], p2 = s->if_p2[fi * s->nfn + k];
                const double *A = s->if_A + (fi * s->nfn + k) * 3;
                for (int a = 0; a < Q; ++a) {
                    const double *e = s->e + 3 * a;
                    double ne = A[0] * e[0] + A[1] * e[1] + A[2] * e[2];
                    if (ne < 0.0) {
                        double fin = f[el * (int64_t)Q * np + (int64_t)a * np + p];
                        double fout = f[el2 * (int64_t)Q * np + (int64_t)a * np + p2];
                        rt[el * (int64_t)Q * np + (int64_t)a * np + p] += ne * (fin - fout);
                    }
                }
            }
        }
}

/* Direct stiffness summation (reading R4): r = (sum over copies of rt) /
 * (sum over copies of wJ) at every copy of every global node. */
static void or_assemble(const oracle_sim *s, const double *rt, double *r)
{
    int np = s->np, Q = s->Q;
    int64_t nl = s->E * np;
    memset(s->rg, 0, sizeof(double) * nl * Q);
    for (int64_t el = 0; el < s->E; ++el)
        for (int a = 0; a < Q; ++a)
            for (int p = 0; p < np; ++p)
                s->rg[(int64_t)a * nl + s->gid[el * np + p]] += rt[el * (int64_t)Q * np + (int64_t)a * np + p];
#pragma omp parallel for schedule(static)
    for (int64_t el = 0; el < s->E; ++el)
        for (int a = 0; a < Q; ++a)
            for (int p = 0; p < np; ++p) {
                int64_t g = s->gid[el * np + p];
                r[el * (int64_t)Q * np + (int64_t)a * np + p] = s->rg[(int64_t)a * nl + g] / s->Mg[g];
            }
}

/* Spatial operator (reading R6): L f = M^-1 (R(n.j) - C f) + F*, F = rhoc g. */
static void or_L(oracle_sim *s, const double *f, double *Lf, int with_force)
{
    int np = s->np, Q = s->Q;
    or_rhs_local(s, f, s->rt);
    or_assemble(s, s->rt, Lf);
    if (!with_force) return;
#pragma omp parallel for schedule(static)
    for (int64_t el = 0; el < s->E; ++el)
        for (int p = 0; p < np; ++p) {
            double F[3];
            for (int k = 0; k < 3; ++k)
                F[k] = s->rhoc[el * np + p] * s->g[k] + (s->Fn ? s->Fn[(el * np + p) * 3 + k] : 0.0);
            for (int a = 0; a < Q; ++a) Lf[el * (int64_t)Q * np + (int64_t)a * np + p] += or_fs(s, a, F);
        }
}

/* Time marching over one step of size dt (Sec. 2.2.2, reading R7), from the
 * stage-0 state y (overwritten by the result). */
static void or_rk(oracle_sim *s, double *y, int with_force)
{
    int64_t nv = or_nv(s);
    double dt = s->dt;
    if (s->rk == 0) {
        /* Shu-Osher SSPRK3 */
        or_L(s, y, s->L0, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) s->w1[i] = y[i] + dt * s->L0[i];
        or_L(s, s->w1, s->L1, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) s->w2[i] = 0.75 * y[i] + 0.25 * (s->w1[i] + dt * s->L1[i]);
        or_L(s, s->w2, s->L2, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) y[i] = y[i] / 3.0 + (2.0 / 3.0) * (s->w2[i] + dt * s->L2[i]);
    } else {
        /* printed four-stage form */
        or_L(s, y, s->L0, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) s->w1[i] = y[i] + (dt / 3.0) * s->L0[i];
        or_L(s, s->w1, s->L1, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i) s->w2[i] = s->w1[i] - (3.0 * dt / 4.0) * (s->L0[i] - s->L1[i]);
        or_L(s, s->w2, s->L2, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i)
            s->w1[i] = s->w2[i] + (2.0 * dt / 3.0) * (s->L0[i] - s->L1[i] + s->L2[i]);
        /* w1 now holds stage 3 */
        or_L(s, s->w1, s->L3, with_force);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; ++i)
            y[i] = s->w1[i] - (dt / 4.0) * (s->L0[i] - s->L1[i] + s->L2[i] - s->L3[i]);
    }
}

/* Filter (Sec. 2.2.3): f <- (F (x) F (x) F) f per element and velocity, as
 * the product of its one-direction factors. */
static void or_filter(const oracle_sim *s, const double *fin, double *fout)
{
    int np = s->np, Q = s->Q, n1 = s->n1, d = s->dim;
#pragma omp parallel for schedule(static)
    for (int64_t el = 0; el < s->E; ++el) {
        double tmp[2][OR_MAXN1 * OR_MAXN1 * OR_MAXN1];
        for (int a = 0; a < Q; ++a) {
            const double *src = fin + el * (int64_t)Q * np + (int64_t)a * np;
            memcpy(tmp[0], src, sizeof(double) * np);
            int cur = 0;
            for (int m = 0; m < d; ++m) {
                for (int p = 0; p < np; ++p) {
                    int ijk[3], q[3];
                    or_node_ijk(s, p, ijk);
                    double acc = 0.0;
                    for (int c = 0; c < n1; ++c) {
                        q[0] = ijk[0];
                        q[1] = ijk[1];
                        q[2] = ijk[2];
                        q[m] = c;
                        acc += s->Ff[ijk[m] * n1 + c] * tmp[cur][or_node_index(s, q)];
                    }
                    tmp[1 - cur][p] = acc;
                }
                cur = 1 - cur;
            }
            memcpy(fout + el * (int64_t)Q * np + (int64_t)a * np, tmp[cur], sizeof(double) * np);
        }
    }
}

/* Initial state (Sec. 2.1 with f = f^eq): f-bar = f^eq(rho, u) - dt F** / 2. */
int oracle_init(oracle_sim *s, const double *rho, const double *u)
{
    int np = s->np, Q = s->Q, d = s->dim;
    for (int64_t el = 0; el < s->E; ++el)
        for (int p = 0; p < np; ++p) {
            int64_t ip = el * np + p;
            double uu[3] = {0, 0, 0}, F[3];
            for (int k = 0; k < d; ++k) uu[k] = u[ip * d + k];
            for (int k = 0; k < 3; ++k) F[k] = rho[ip] * s->g[k];
            for (int a = 0; a < Q; ++a)
                s->f[el * (int64_t)Q * np + (int64_t)a * np + p] =
                    or_feq(s, a, rho[ip], uu) - 0.5 * s->dt * or_fss(s, a, uu, F);
        }
    s->time = 0.0;
    s->nstep = 0;
    return 0;
}

/* One full step in the order of the scheme summary (reading R9). */
int oracle_step(oracle_sim *s, int64_t nsteps)
{
    int64_t nv = or_nv(s);
    for (int64_t n = 0; n < nsteps; ++n) {
        or_collide_all(s, s->f, s->f0, s->rhoc);
        or_rk(s, s->f0, 1);
        if (s->filter_on) or_filter(s, s->f0, s->f);
        else memcpy(s->f, s->f0, sizeof(double) * nv);
        s->time += s->dt;
        s->nstep++;
    }
    return 0;
}

/* Streaming only (no collision, no force, no filter): advances f-bar by the
 * time marching of the streaming equation with the wall flux. Used to check
 * the advection operator against exact transport. */
int oracle_advect(oracle_sim *s, int64_t nsteps)
{
    for (int64_t n = 0; n < nsteps; ++n) {
        or_rk(s, s->f, 0);
        s->time += s->dt;
        s->nstep++;
    }
    return 0;
}

int oracle_moments(const oracle_sim *s, double *rho, double *u)
{
    int np = s->np, d = s->dim;
    for (int64_t el = 0; el < s->E; ++el)
        for (int p = 0; p < np; ++p) {
            double r, uu[3];
            or_moments_node(s, s->f + el * (int64_t)s->Q * np + p, np, &r, uu);
            rho[el * np + p] = r;
            for (int k = 0; k < d; ++k) u[(el * np + p) * d + k] = uu[k];
        }
    return 0;
}

/* Integrals with the lumped mass: out = [sum wJ rho, sum wJ rho u (dim),
 * sum wJ rho0 |u|^2 / 2]. */
int oracle_reduce(const oracle_sim *s, double *out)
{
    int np = s->np, d = s->dim;
    double m = 0.0, mom[3] = {0, 0, 0}, ke = 0.0;
    for (int64_t el = 0; el < s->E; ++el)
        for (int p = 0; p < np; ++p) {
            double r, uu[3];
            or_moments_node(s, s->f + el * (int64_t)s->Q * np + p, np, &r, uu);
            double wj = s->wJ[el * np + p];
            m += wj * r;
            for (int k = 0; k < d; ++k) mom[k] += wj * r * uu[k];
            ke += wj * 0.5 * s->rho0 * (uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
        }
    out[0] = m;
    for (int k = 0; k < d; ++k) out[1 + k] = mom[k];
    out[1 + d] = ke;
    return 0;
}

int oracle_get_f(const oracle_sim *s, double *f)
{
    memcpy(f, s->f, sizeof(double) * or_nv(s));
    return 0;
}

int oracle_set_f(oracle_sim *s, const double *f)
{
    memcpy(s->f, f, sizeof(double) * or_nv(s));
    return 0;
}

double oracle_time(const oracle_sim *s) { return s->time; }
double oracle_tau(const oracle_sim *s) { return s->tau; }

/* Geometry export: wJ [E][np], G [E][np][3][3], J [E][np]. */
int oracle_geometry(const oracle_sim *s, double *wJ, double *G, double *J)
{
    int64_t nl = s->E * s->np;
    if (wJ) memcpy(wJ, s->wJ, sizeof(double) * nl);
    if (G) memcpy(G, s->G, sizeof(double) * nl * 9);
    if (J) memcpy(J, s->J, sizeof(double) * nl);
    return 0;
}

/* Assembled lumped mass at every local node [E][np]. */
int oracle_mass(const oracle_sim *s, double *M)
{
    int64_t nl = s->E * s->np;
    for (int64_t i = 0; i < nl; ++i) M[i] = s->Mg[s->gid[i]];
    return 0;
}

/* Operator pieces on a caller-given state f [E][Q][np]:
 *   oracle_rhs_local: element contributions rt (with wall flux, before DSS);
 *   oracle_rhs:       assembled M^-1 (R(n.j) - C f), without F*;
 *   oracle_collide:   post-collision f*;
 *   oracle_filter:    filtered f. */
int oracle_rhs_local(oracle_sim *s, const double *f, double *rt)
{
    or_rhs_local(s, f, rt);
    return 0;
}

int oracle_rhs(oracle_sim *s, const double *f, double *r)
{
    or_rhs_local(s, f, s->rt);
    or_assemble(s, s->rt, r);
    return 0;
}

int oracle_collide(oracle_sim *s, const double *f, double *fs)
{
    or_collide_all(s, f, fs, NULL);
    return 0;
}

int oracle_filter(oracle_sim *s, const double *f, double *out)
{
    if (!s->filter_on) {
        memcpy(out, f, sizeof(double) * or_nv(s));
        return 0;
    }
    or_filter(s, f, out);
    return 0;
}

/* Time marching of a scalar affine ODE y' = lam y + b with the same stage
 * formulas as the field integrator (reading R7). */
int oracle_rk_scalar(int rk, double lam, double b, double y0, double dt, int64_t nsteps, double *y)
{
    double v = y0;
    for (int64_t n = 0; n < nsteps; ++n) {
        if (rk == 0) {
            double l0 = lam * v + b;
            double w1 = v + dt * l0;
            double l1 = lam * w1 + b;
            double w2 = 0.75 * v + 0.25 * (w1 + dt * l1);
            double l2 = lam * w2 + b;
            v = v / 3.0 + (2.0 / 3.0) * (w2 + dt * l2);
        } else if (rk == 1) {
            double l0 = lam * v + b;
            double w1 = v + (dt / 3.0) * l0;
            double l1 = lam * w1 + b;
            double w2 = w1 - (3.0 * dt / 4.0) * (l0 - l1);
            double l2 = lam * w2 + b;
            double w3 = w2 + (2.0 * dt / 3.0) * (l0 - l1 + l2);
            double l3 = lam * w3 + b;
            v = w3 - (dt / 4.0) * (l0 - l1 + l2 - l3);
        } else {
            return -1;
        }
    }
    *y = v;
    return 0;
}

/* Force density per node [E][np][dim] added to rho g from the next step on
 * (reading R12); NULL removes it. */
int oracle_set_force(oracle_sim *s, const double *F)
{
    int64_t nl = s->E * s->np;
    if (!F) {
        free(s->Fn);
        s->Fn = NULL;
        return 0;
    }
    if (!s->Fn) {
        s->Fn = (double *)calloc((size_t)nl * 3, sizeof(double));
        if (!s->Fn) return -1;
    }
    for (int64_t i = 0; i < nl; ++i)
        for (int k = 0; k < 3; ++k) s->Fn[i * 3 + k] = k < s->dim ? F[i * s->dim + k] : 0.0;
    return 0;
}

/* Per-node relaxation-time increments [E][np] used by the following
 * collisions (learned closure); NULL or all zero restores the plain method. */
int oracle_set_dtau(oracle_sim *s, const double *dtau)
{
    int64_t nl = s->E * s->np;
    if (!dtau) {
        free(s->dtau);
        s->dtau = NULL;
        return 0;
    }
    if (!s->dtau) s->dtau = (double *)malloc(sizeof(double) * nl);
    if (!s->dtau) return -1;
    memcpy(s->dtau, dtau, sizeof(double) * nl);
    return 0;
}
