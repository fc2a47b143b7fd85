// HIP kernels of the SELBM time step for gfx950, templated on the dimension,
// the order N, the lattice Q, the storage type T and the deviation form DEV.
//
// Data layout (all device, one workspace):
//   state arrays: element interiors [E][Q][NI] (node id e*NI + s), then the
//     shared element-boundary nodes, one entry per node group, in tiles of 64
//     groups [ceil(ngrp/64)][Q][64] (node id Gi + g). Every block touches a
//     few contiguous regions; per velocity the accesses stay coalesced.
//   element contributions of boundary nodes rtb [E][Q][NB].
//   metric Gm [E][DIM*DIM][NP] = wJ dr_m/dx_k, interior 1/wJ [E][NI],
//   assembled inverse mass of boundary groups [ngrp].
// One workgroup handles EPB elements with one thread per node; a velocity
// plane of each element is staged in LDS for the tensor-product derivatives.
#pragma once

#include <type_traits>

#include "sel_internal.h"

namespace sel {

constexpr double kCs2 = 1.0 / 3.0;

// velocity planes staged in LDS per barrier in the element kernels
#ifndef SEL_CHUNK
#define SEL_CHUNK 3
#endif


__host__ __device__ constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }

// ---------------------------------------------------------------- lattice --
// a = a0 + 3 a1 (+ 9 a2), component values {0, +1, -1}; D3Q19 keeps |e|^2 <= 2.
template <int DIM, int Q>
__host__ __device__ constexpr int lat_full(int a)
{
    if (Q != 19) return a;
    int cnt = 0;
    for (int f = 0; f < 27; ++f) {
        int s = (f % 3 != 0) + ((f / 3) % 3 != 0) + (f / 9 != 0);
        if (s > 2) continue;
        if (cnt == a) return f;
        ++cnt;
    }
    return 0;
}
template <int DIM, int Q>
__host__ __device__ constexpr int lat_e(int a, int k)
{
    if (k >= DIM) return 0;
    int f = lat_full<DIM, Q>(a);
    int c = (k == 0) ? f % 3 : (k == 1) ? (f / 3) % 3 : f / 9;
    return c == 0 ? 0 : (c == 1 ? 1 : -1);
}
template <int DIM, int Q>
__host__ __device__ constexpr int lat_s2(int a)
{
    return lat_e<DIM, Q>(a, 0) * lat_e<DIM, Q>(a, 0) + lat_e<DIM, Q>(a, 1) * lat_e<DIM, Q>(a, 1) +
           lat_e<DIM, Q>(a, 2) * lat_e<DIM, Q>(a, 2);
}
template <int DIM, int Q>
__host__ __device__ constexpr double lat_t(int a)
{
    int s = lat_s2<DIM, Q>(a);
    if (Q == 9) return s == 0 ? 4.0 / 9.0 : s == 1 ? 1.0 / 9.0 : 1.0 / 36.0;
    if (Q == 19) return s == 0 ? 1.0 / 3.0 : s == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
    return s == 0 ? 8.0 / 27.0 : s == 1 ? 2.0 / 27.0 : s == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}
template <int DIM, int Q>
__host__ __device__ constexpr int lat_opp(int a)
{
    for (int b = 0; b < Q; ++b)
        if (lat_e<DIM, Q>(b, 0) == -lat_e<DIM, Q>(a, 0) && lat_e<DIM, Q>(b, 1) == -lat_e<DIM, Q>(a, 1) &&
            lat_e<DIM, Q>(b, 2) == -lat_e<DIM, Q>(a, 2))
            return b;
    return 0;
}

template <int I, int END, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < END) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, END>(f);
    }
}

template <int DIM, int N>
struct Geo {
    static constexpr int n1 = N + 1;
    static constexpr int NP = ipow_c(n1, DIM);
    static constexpr int NI = ipow_c(N - 1, DIM);
    static constexpr int NB = NP - NI;
    static constexpr int EPB = (NP >= 256) ? 1 : 256 / NP;
    static constexpr int BLOCK = EPB * NP;
};

// State index of node id gix for velocity a is base + a * stride.
constexpr int kTile = 64;
struct SIdx {
    int64_t base;
    int stride;
};
__device__ __forceinline__ SIdx sidx_interior(int64_t e, int s, int Q, int NI)
{
    return {e * (int64_t)Q * NI + s, NI};
}
__device__ __forceinline__ SIdx sidx_group(int64_t g, int Q, int64_t QGi)
{
    return {QGi + (g / kTile) * (int64_t)Q * kTile + (g % kTile), kTile};
}

// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of element blocks so that neighbours share its L2.
__device__ __forceinline__ int64_t xcd_block(int64_t nblk)
{
    const int64_t x = blockIdx.x;
    const int64_t per = (nblk + 7) / 8;
    return (x % 8) * per + x / 8;
}
inline int64_t xcd_grid(int64_t nblk) { return 8 * ((nblk + 7) / 8); }

// --------------------------------------------------------- local physics --
// e . x over the nonzero components of a lattice velocity (each +-1, so the
// products are exact): no additions of zero terms.
template <int ex, int ey, int ez, typename T>
__device__ __forceinline__ T edot(T x, T y, T z)
{
    T r = T(0);
    if constexpr (ex != 0) r = T(ex) * x;
    if constexpr (ey != 0) r = (ex != 0) ? r + T(ey) * y : T(ey) * y;
    if constexpr (ez != 0) r = (ex != 0 || ey != 0) ? r + T(ez) * z : T(ez) * z;
    return r;
}

// BGK collision with the higher-order force F** (Sec. 2.1): from the node's
// values v[a] (full f, or the deviation g = f - t_a rho0 when DEV) compute
// rho, u = sum e f / rho, F = rho g and
//   f* = f - omega (f - (f^eq - dt F**/2)) + dt F**,  omega = 1 / (tau + 1/2).
template <int DIM, int Q, typename T, bool DEV>
__device__ __forceinline__ void collide_node(T (&v)[Q], T rho0, T omega, T dt, const T (&g)[3], T &rho_out)
{
    T m0 = 0, j0 = 0, j1 = 0, j2 = 0;
    static_for<0, Q>([&](auto A) {
        constexpr int a = decltype(A)::value;
        m0 += v[a];
        if constexpr (lat_e<DIM, Q>(a, 0) != 0) j0 += T(lat_e<DIM, Q>(a, 0)) * v[a];
        if constexpr (lat_e<DIM, Q>(a, 1) != 0) j1 += T(lat_e<DIM, Q>(a, 1)) * v[a];
        if constexpr (lat_e<DIM, Q>(a, 2) != 0) j2 += T(lat_e<DIM, Q>(a, 2)) * v[a];
    });
    const T rho = DEV ? rho0 + m0 : m0;
    const T inv = T(1) / rho;
    const T u0 = j0 * inv, u1 = j1 * inv, u2 = j2 * inv;
    const T F0 = rho * g[0], F1 = rho * g[1], F2 = rho * g[2];
    const T uu = u0 * u0 + u1 * u1 + u2 * u2;
    const T uF = u0 * F0 + u1 * F1 + u2 * F2;
    const T c1 = T(3), c2 = T(4.5), c3 = T(1.5);  // 1/cs2, 1/(2 cs4), 1/(2 cs2)
    const T half_dt = T(0.5) * dt;
    if constexpr (!std::is_same<T, float>::value) {
        static_for<0, Q>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
            const T t = T(lat_t<DIM, Q>(a));
            const T eu = T(ex) * u0 + T(ey) * u1 + T(ez) * u2;
            const T eF = T(ex) * F0 + T(ey) * F1 + T(ez) * F2;
            const T poly = c1 * eu + c2 * eu * eu - c3 * uu;
            // equilibrium (Eq. geq_s), as a deviation from t rho0 when DEV
            const T feq = DEV ? t * (m0 + rho * poly) : t * rho * (T(1) + poly);
            // higher-order force (Eq. f_c): t ((e.u)(e.F)/cs4 - (u.F)/cs2)
            const T fss = t * (T(9) * eu * eF - T(3) * uF);
            const T fbeq = feq - half_dt * fss;
            v[a] = v[a] - omega * (v[a] - fbeq) + dt * fss;
        });
    } else {
        // FP32: the rounded equilibrium does not reproduce rho and j exactly,
        // and relaxing towards it would leak mass and momentum with a sign
        // set by the state (a drift over many steps). The non-equilibrium
        // part n = f - f-bar-eq has zero mass and momentum in exact
        // arithmetic; its computed moments are sums of small numbers, so
        // they are accurate, and they are projected out before relaxing:
        //   n' = n - t (S0 + e.S1 / cs2), f* = f-bar-eq + dt F** + (1 - omega) n + omega (n - n').
        // Dot products with e_a take only its nonzero components (+-1), and
        // the weight's products t m0, t rho, omega t are formed once per weight.
        T base[Q];
        T S0 = 0, S1x = 0, S1y = 0, S1z = 0;
        // without a body force F** vanishes: the same values without its terms
        const bool forced = (g[0] != T(0)) | (g[1] != T(0)) | (g[2] != T(0));
        const T c3uu = c3 * uu;
        auto pass1 = [&](auto FORCED) {
            static_for<0, Q>([&](auto A) {
                constexpr int a = decltype(A)::value;
                constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
                const T t = T(lat_t<DIM, Q>(a));
                const T eu = edot<ex, ey, ez>(u0, u1, u2);
                const T poly = eu * (c1 + c2 * eu) - c3uu;  // e.u/cs2 + (e.u)^2/(2 cs4) - u.u/(2 cs2)
                const T feq = DEV ? (t * m0 + (t * rho) * poly) : (t * rho) * (T(1) + poly);
                T fbeq = feq;
                if constexpr (decltype(FORCED)::value) {
                    const T eF = edot<ex, ey, ez>(F0, F1, F2);
                    const T fss = t * (T(9) * eu * eF - T(3) * uF);
                    fbeq = feq - half_dt * fss;
                    base[a] = fbeq + dt * fss;
                } else {
                    base[a] = fbeq;
                }
                const T n = v[a] - fbeq;
                v[a] = n;
                S0 += n;
                if constexpr (ex != 0) S1x += T(ex) * n;
                if constexpr (ey != 0) S1y += T(ey) * n;
                if constexpr (ez != 0) S1z += T(ez) * n;
            });
        };
        if (forced) pass1(std::true_type{});
        else pass1(std::false_type{});
        const T keep = T(1) - omega;
        const T S3x = T(3) * S1x, S3y = T(3) * S1y, S3z = T(3) * S1z;
        static_for<0, Q>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
            const T t = T(lat_t<DIM, Q>(a));
            const T es = S0 + edot<ex, ey, ez>(S3x, S3y, S3z);
            v[a] = base[a] + (keep * v[a] + (omega * t) * es);
        });
    }
    rho_out = rho;
}

// SSPRK stage output ca f0 + cb fk + cc L with ca + cb = 1. FP32 takes the
// increment form fk + (ca (f0 - fk) + cc L): the weights then sum to one
// exactly (float(1/3) + float(2/3) exceeds 1 by 3e-8, which would scale the
// state by that much every step) and only one rounding acts at the size of f.
// (incr = 0: general weights, as for the single-operator entry point.)
template <typename T>
__device__ __forceinline__ T rk_combine(T ca, T cb, T cc, T f0, T fk, T L, int incr)
{
    if constexpr (std::is_same<T, float>::value) {
        if (incr) return fk + (ca * (f0 - fk) + cc * L);
    }
    return ca * f0 + cb * fk + cc * L;
}

// Volume part of the streaming operator of velocity a at one node (Sec. 2.2),
//   rt = -wJ e_a . grad f_a = -sum_m c_m d f_a / d r_m,  c_m = sum_k e_k G_mk,
// with the reference derivatives from the element's plane P of f_a in LDS
// (rows of D-hat). FP32 (DIF) takes the line contractions around the node's
// own value v.
template <int DIM, int N, int Q, int a, bool DIF, typename T>
__device__ __forceinline__ T stream_volume(const T *P, T v, const T (&Di)[N + 1], const T (&Dj)[N + 1],
                                           const T (&Dk)[N + 1], const T (&Gr)[DIM][DIM], int rowr, int rows,
                                           int rowt)
{
    constexpr int n1 = N + 1;
    constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
    // the rest velocity does not stream (e = 0); without this the products
    // 0 * (derivative) would still be evaluated
    if constexpr (ex == 0 && ey == 0 && ez == 0) return T(0);
    T dr = 0, ds = 0, dtt = 0;
    if constexpr (DIF) {
#pragma unroll
        for (int q = 0; q < n1; ++q) dr += Di[q] * (P[rowr + q] - v);
#pragma unroll
        for (int q = 0; q < n1; ++q) ds += Dj[q] * (P[rows + n1 * q] - v);
        if constexpr (DIM == 3) {
#pragma unroll
            for (int q = 0; q < n1; ++q) dtt += Dk[q] * (P[rowt + n1 * n1 * q] - v);
        }
    } else {
#pragma unroll
        for (int q = 0; q < n1; ++q) dr += Di[q] * P[rowr + q];
#pragma unroll
        for (int q = 0; q < n1; ++q) ds += Dj[q] * P[rows + n1 * q];
        if constexpr (DIM == 3) {
#pragma unroll
            for (int q = 0; q < n1; ++q) dtt += Dk[q] * P[rowt + n1 * n1 * q];
        }
    }
    // c_m = sum_k e_k G_mk
    T cr = 0, cs = 0, ct = 0;
    if constexpr (ex != 0) {
        cr += T(ex) * Gr[0][0];
        cs += T(ex) * Gr[1][0];
        if constexpr (DIM == 3) ct += T(ex) * Gr[2][0];
    }
    if constexpr (ey != 0) {
        cr += T(ey) * Gr[0][1];
        cs += T(ey) * Gr[1][1];
        if constexpr (DIM == 3) ct += T(ey) * Gr[2][1];
    }
    if constexpr (DIM == 3 && ez != 0) {
        cr += T(ez) * Gr[0][2];
        cs += T(ez) * Gr[1][2];
        ct += T(ez) * Gr[2][2];
    }
    return -(cr * dr + cs * ds + ct * dtt);
}

// Flux bounce-back term of velocity a (Sec. 2.2.1) added to rt: on each wall
// face through the node where e_a is incoming, the population is replaced
// by the reflected one, f_a - f_b - 2 t_a rho0 (e_a . u_w)/c_s^2 with b the
// opposite velocity (node values v and vb), times the outward area vector
// w_s J_s n = +-(w_end)^-1 wJ dr_m/dx of the face r_m = +-1, taken from the
// same metric as the volume term. wcode: 8 bits per reference direction m,
// the wall tag (0 = none) and bit 7 for the face r_m = +1.
template <int DIM, int N, int Q, int a, typename T>
__device__ __forceinline__ void wall_flux(T &rt, T v, T vb, const T (&Gr)[DIM][DIM], uint32_t wcode,
                                          const T *wallu, T rho0)
{
    constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
    const T t = T(lat_t<DIM, Q>(a));
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        const uint32_t code = (wcode >> (8 * m)) & 0xffu;
        if (code) {
            const T sc = ((code & 0x80u) ? T(1) : T(-1)) * T(N * (N + 1)) / T(2);
            T ne = T(ex) * Gr[m][0] + T(ey) * Gr[m][1];
            if constexpr (DIM == 3) ne += T(ez) * Gr[m][2];
            ne *= sc;
            if (ne < T(0)) {
                const T *ub = wallu + 3 * (code & 0x7fu);
                const T eub = T(ex) * ub[0] + T(ey) * ub[1] + T(ez) * ub[2];
                rt += ne * (v - vb - T(2) * t * rho0 * eub * T(3));
            }
        }
    }
}

// Upwind interface flux of velocity a under the discontinuous coupling,
// added to rt: on each face through the node that is not a wall (icode:
// bit 2m set for direction m, bit 2m+1 for the face r_m = +1) and where e_a
// enters the element, (n.e_a) w_s J_s (v - f_out), with f_out the value of
// the coincident node of the element across the face (its group gnb[m] in
// the state op) and the area vector as in wall_flux.
template <int DIM, int N, int Q, int a, typename T>
__device__ __forceinline__ void interface_flux(T &rt, T v, const T (&Gr)[DIM][DIM], uint32_t icode,
                                               const int32_t (&gnb)[DIM], const T *op, int64_t QGi)
{
    constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        if ((icode >> (2 * m)) & 1u) {
            const T sc = (((icode >> (2 * m + 1)) & 1u) ? T(1) : T(-1)) * T(N * (N + 1)) / T(2);
            T ne = T(ex) * Gr[m][0] + T(ey) * Gr[m][1];
            if constexpr (DIM == 3) ne += T(ez) * Gr[m][2];
            ne *= sc;
            if (ne < T(0)) {
                const SIdx so = sidx_group(gnb[m], Q, QGi);
                rt += ne * (v - op[so.base + (int64_t)a * so.stride]);
            }
        }
    }
}

// ----------------------------------------------------------- stage kernel --
enum { M_STAGE1 = 0, M_STAGE23 = 1, M_LOCAL = 2, M_FILTER = 3 };

template <typename T>
struct StageArgs {
    const T *op;     // operand state
    const T *f0in;   // post-collision state (stages 2, 3)
    T *f0out;        // stage 1: post-collision state written here
    T *rhoc;         // density at the collision [Gtot]
    T *out;          // output state (interior nodes; all owned nodes for M_FILTER)
    T *rtb;          // element contributions of boundary nodes [Q][plane]
    const int32_t *posmap;  // [E][NB] contribution slot of each boundary node
    int64_t plane;
    T *local;        // M_LOCAL: element contributions [Q][E][NP]
    const T *Gm, *invw, *D, *F;
    const int32_t *pcode, *bmap, *ftag;
    const int32_t *bpos;  // [NB] node index of each boundary slot
    const uint8_t *bown;
    const T *wallu;  // [ntags+1][3]
    int64_t E, nblk, Gi, QGi;
    T dt, omega, rho0, ca, cb, cc;  // output = ca f0 + cb f_k + cc L(f_k)
    int incr;                       // ca + cb = 1 (time steps): FP32 increment form
    T g[3];
    T fsc[kMaxQ];  // F* per unit density: t_a (e_a . g) / cs2
    int filter;    // M_STAGE1: filter the operand first
    T tau;                // relaxation time
    const float *dtau;    // learned-closure increments per node id (nullptr: plain method)
    const int32_t *nbr;   // discontinuous coupling: [E][2 dim][(N+1)^(dim-1)] group across each face (nullptr: continuous)
    int collide_only;     // M_STAGE1: stop after writing the post-collision state
};

// DGC: the discontinuous coupling's interface flux is compiled in (a
// separate instantiation, so the continuous kernels carry none of it).
template <int DIM, int N, int Q, typename T, bool DEV, int MODE, bool DGC = false>
__global__ void __launch_bounds__((Geo<DIM, N>::BLOCK), (((MODE == M_STAGE23 || MODE == M_STAGE1) && sizeof(T) == 4) ? 4 : 1)) k_stage(StageArgs<T> A)
{
    using GG = Geo<DIM, N>;
    constexpr int n1 = GG::n1, NP = GG::NP, NI = GG::NI, NB = GG::NB, EPB = GG::EPB;
    // first stage and filter keep all velocities of the node in registers
    // (collision and filter need them); later stages stream the velocities
    // with a software prefetch one chunk ahead. Velocities are processed in
    // chunks of NA planes per LDS barrier.
    constexpr bool ALLQ = (MODE == M_STAGE1 || MODE == M_FILTER);
    // FP32: line contractions are taken around the node's own value,
    // sum_q W_q (P_q - x) (+ x for filter rows, which sum to one), so that a
    // large common level of the populations adds no rounding bias (the
    // rounded rows of D-hat and F do not sum exactly to 0 and 1)
    constexpr bool DIF = std::is_same<T, float>::value;
    constexpr int NA = SEL_CHUNK;
    constexpr int NC = (Q + NA - 1) / NA;
    // whole-element staging (FP32, one element per workgroup): all Q values
    // of the node are loaded at once (every load in flight together), all Q
    // planes of the element go to LDS behind one barrier, and the velocities
    // are then processed without further waits on global memory
    constexpr bool FULL = DIF && EPB == 1 && MODE != M_FILTER && Q * NP * 4 <= 80 * 1024;
    // FP32 filter with all Q planes in LDS (first stage and filter-only
    // launch); FP64 uses it for the filter-only launch (110 KB of LDS at
    // N = 7, Q = 27: one workgroup per CU, which costs the stages more than
    // the chunked passes)
    constexpr bool FF = EPB == 1 && ALLQ && (DIF ? Q * NP * 4 <= 80 * 1024 : (MODE == M_FILTER && Q * NP * 8 <= 120 * 1024));
    // later stages also stage their results through LDS for coalesced stores
    constexpr bool STG = FULL && (MODE == M_STAGE23 || MODE == M_STAGE1);
    constexpr int PL_N = (ALLQ ? 3 : 2) * NA * EPB * NP;
    constexpr int LDS_N = (FULL || FF) ? (ALLQ ? (Q * NP > PL_N ? Q * NP : PL_N) : Q * NP) : PL_N;
    __shared__ __attribute__((aligned(16))) T lds[LDS_N];
    T(*pl)[EPB * NP] = reinterpret_cast<T(*)[EPB * NP]>(lds);
    __shared__ T sF[ALLQ ? n1 * n1 : 1];
    // FP32 first stage: D-hat in LDS as well (its rows are read after the
    // collision, where global loads would add a memory latency)
    constexpr bool SD = MODE == M_STAGE1 && FULL;
    __shared__ T sD[SD ? n1 * n1 : 1];

    const int tid = threadIdx.x;
    const int le = tid / NP;
    const int p = tid - le * NP;
    const int64_t eb = xcd_block(A.nblk);
    if (eb >= A.nblk) return;  // whole workgroup
    const int64_t e = eb * EPB + le;
    const bool valid = e < A.E;
    const bool filt = (MODE == M_FILTER) || (MODE == M_STAGE1 && A.filter);
    if constexpr (ALLQ) {
        if (filt)
            for (int q = tid; q < n1 * n1; q += GG::BLOCK) sF[q] = A.F[q];
    }
    if constexpr (SD) {
        for (int q = tid; q < n1 * n1; q += GG::BLOCK) sD[q] = A.D[q];
        if (!filt) __syncthreads();  // else the filter's first barrier makes it visible
    }
    const int i = p % n1;
    const int j = (p / n1) % n1;
    int k = (DIM == 3) ? p / (n1 * n1) : 0;
    // a k-slice of the N = 7 element is exactly one wavefront: k is uniform
    if constexpr (DIM == 3 && n1 * n1 == 64 && EPB == 1) k = __builtin_amdgcn_readfirstlane(k);
    const int pc = A.pcode[p];
    const bool inner = pc >= 0;
    const int bsl = inner ? 0 : -pc - 1;
    int64_t gix = 0;
    bool own = false;
    SIdx si{0, 0};
    if (valid) {
        if (inner) {
            gix = e * NI + pc;
            own = true;
            si = sidx_interior(e, pc, Q, NI);
        } else {
            const int64_t g = A.bmap[e * NB + bsl];
            gix = A.Gi + g;
            own = A.bown[e * NB + bsl] != 0;
            si = sidx_group(g, Q, A.QGi);
        }
    }
    int32_t slot = 0;  // contribution slot of a boundary node
    if constexpr (MODE != M_LOCAL && MODE != M_FILTER) {
        if (valid && !inner) slot = A.posmap[e * NB + bsl];
    }
    const int base = le * NP;
    const int rowr = base + n1 * j + n1 * n1 * k;  // + c       (r line)
    const int rows = base + i + n1 * n1 * k;       // + n1 c    (s line)
    const int rowt = base + i + n1 * j;            // + n1^2 c  (t line)

    T fq[(ALLQ || FULL) ? Q : 1];
    T f0q[(FULL && MODE == M_STAGE23) ? Q : 1];
    // prefetch ring: even chunks in (roA, r0A), odd chunks in (roB, r0B)
    T roA[NA] = {}, r0A[NA] = {}, roB[NA] = {}, r0B[NA] = {};
    auto prefetch = [&](auto CC) {
        constexpr int c = decltype(CC)::value;
        if constexpr (!ALLQ && !FULL && c < NC) {
            static_for<0, NA>([&](auto UU) {
                constexpr int u = decltype(UU)::value, a = c * NA + u;
                if constexpr (a < Q) {
                    const T vo = valid ? A.op[si.base + (int64_t)a * si.stride] : T(0);
                    const T v0 = (MODE == M_STAGE23 && valid && inner) ? A.f0in[si.base + (int64_t)a * si.stride] : T(0);
                    if constexpr (c & 1) {
                        roB[u] = vo;
                        r0B[u] = v0;
                    } else {
                        roA[u] = vo;
                        r0A[u] = v0;
                    }
                }
            });
        }
    };
    // first stage with the filter, and the later stages (FP32, one element
    // per workgroup): the element's values go straight to the planes, one slot
    // per thread (interior slots contiguous per velocity, boundary slots
    // through their node group)
    constexpr bool SLOT = FULL && EPB == 1 && NB + NI == NP && ((MODE == M_STAGE1 && FF) || MODE == M_STAGE23);
    bool slotted = false;
    // the node's metric terms and inverse mass: with the slot loads they are
    // issued together with the element's values and parked in LDS (18 KB at
    // N = 7; two elements per CU still fit), so that their latency is hidden
    // behind the filter and they hold no registers through it (else they are
    // read after the collision)
    T Gr[DIM][DIM];
    T invw = 0;
    bool have_metric = false;
    __shared__ T sG[SLOT ? (DIM * DIM + 1) * NP : 1];
    if constexpr (SLOT) {
        if (MODE == M_STAGE23 || filt) {
            slotted = true;
            const T *src;
            int node, stride;
            if (tid < NI) {
                src = A.op + e * (int64_t)Q * NI + tid;
                stride = NI;
                node = (tid % (N - 1) + 1) + n1 * ((tid / (N - 1)) % (N - 1) + 1) + n1 * n1 * (tid / ((N - 1) * (N - 1)) + 1);
            } else {
                const int b = tid - NI;
                const int64_t g = A.bmap[e * NB + b];
                src = A.op + A.QGi + (g / kTile) * (int64_t)Q * kTile + (g % kTile);
                stride = kTile;
                node = A.bpos[b];
            }
            T v[Q];
            static_for<0, Q>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                v[a] = src[a * stride];
            });
            T gt[DIM * DIM];
#pragma unroll
            for (int m = 0; m < DIM * DIM; ++m) gt[m] = __builtin_nontemporal_load(A.Gm + (e * DIM * DIM + m) * NP + p);
            const T iw = inner ? A.invw[e * NI + pc] : T(0);
            have_metric = true;
            static_for<0, Q>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                pl[a][node] = v[a];
            });
#pragma unroll
            for (int m = 0; m < DIM * DIM; ++m) sG[m * NP + p] = gt[m];
            sG[DIM * DIM * NP + p] = iw;
        }
    }
    if constexpr (ALLQ || FULL) {
        if (!slotted) {
            static_for<0, Q>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                fq[a] = valid ? A.op[si.base + (int64_t)a * si.stride] : T(0);
            });
        }
        if constexpr (FULL && MODE == M_STAGE23) {
            static_for<0, Q>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                // read once per stage: non-temporal, like the metric
                f0q[a] = (valid && inner) ? __builtin_nontemporal_load(A.f0in + si.base + (int64_t)a * si.stride) : T(0);
            });
        }
    } else {
        prefetch(std::integral_constant<int, 0>{});
    }

    if constexpr (ALLQ) {
        if (filt && FF) {
            // explicit modal filter (Sec. 2.2.3), all velocities per pass: the
            // node's values go to the Q planes, each pass is computed into
            // registers and written back (two barriers per pass)
            if (!slotted) {
                static_for<0, Q>([&](auto AA) {
                    constexpr int a = decltype(AA)::value;
                    pl[a][p] = fq[a];
                });
            }
            __syncthreads();  // planes and sF visible
            if (slotted) {
                static_for<0, Q>([&](auto AA) {
                    constexpr int a = decltype(AA)::value;
                    fq[a] = pl[a][p];
                });
            }
            static_for<0, DIM>([&](auto MM) {
                constexpr int m = decltype(MM)::value;
                const int row = (m == 0) ? rowr : (m == 1) ? rows : rowt;
                constexpr int st = (m == 0) ? 1 : (m == 1) ? n1 : n1 * n1;
                const int ir = (m == 0) ? i : (m == 1) ? j : k;
                // rows 0 and N of F are unit vectors: nodes at the ends of
                // the line keep their value (exactly); along t in 3D at N = 7
                // these are whole wavefronts (k is uniform)
                if (!(m == DIM - 1 && (ir == 0 || ir == N))) {
                    static_for<0, Q>([&](auto AA) {
                        constexpr int a = decltype(AA)::value;
                        const T x = fq[a];
                        T t = 0;
#pragma unroll
                        for (int q = 0; q < n1; ++q) t += sF[ir * n1 + q] * (pl[a][row + st * q] - x);
                        fq[a] = t + x;
                    });
                }
                if constexpr (m + 1 < DIM) {
                    __syncthreads();  // every read of this pass done
                    static_for<0, Q>([&](auto AA) {
                        constexpr int a = decltype(AA)::value;
                        pl[a][p] = fq[a];
                    });
                    __syncthreads();
                }
            });
        } else if (filt) {
            __syncthreads();  // sF visible
            // explicit modal filter (Sec. 2.2.3): (F x F x F) applied one direction at a time
            static_for<0, NC>([&](auto CC) {
                constexpr int c = decltype(CC)::value;
                T t1v[NA], t2v[NA];
                static_for<0, NA>([&](auto UU) {
                    constexpr int u = decltype(UU)::value, a = c * NA + u;
                    if constexpr (a < Q) pl[u][base + p] = fq[a];
                });
                __syncthreads();
                static_for<0, NA>([&](auto UU) {
                    constexpr int u = decltype(UU)::value, a = c * NA + u;
                    if constexpr (a < Q) {
                        const T x = fq[a];
                        T t1 = 0;
#pragma unroll
                        for (int q = 0; q < n1; ++q) {
                            if constexpr (DIF) t1 += sF[i * n1 + q] * (pl[u][rowr + q] - x);
                            else t1 += sF[i * n1 + q] * pl[u][rowr + q];
                        }
                        if constexpr (DIF) t1 += x;
                        t1v[u] = t1;
                        pl[NA + u][base + p] = t1;
                    }
                });
                __syncthreads();
                static_for<0, NA>([&](auto UU) {
                    constexpr int u = decltype(UU)::value, a = c * NA + u;
                    if constexpr (a < Q) {
                        const T x = t1v[u];
                        T t2 = 0;
#pragma unroll
                        for (int q = 0; q < n1; ++q) {
                            if constexpr (DIF) t2 += sF[j * n1 + q] * (pl[NA + u][rows + n1 * q] - x);
                            else t2 += sF[j * n1 + q] * pl[NA + u][rows + n1 * q];
                        }
                        if constexpr (DIF) t2 += x;
                        t2v[u] = t2;
                        if constexpr (DIM == 3) pl[2 * NA + u][base + p] = t2;
                        else fq[a] = t2;
                    }
                });
                if constexpr (DIM == 3) {
                    __syncthreads();
                    static_for<0, NA>([&](auto UU) {
                        constexpr int u = decltype(UU)::value, a = c * NA + u;
                        if constexpr (a < Q) {
                            const T x = t2v[u];
                            T t3 = 0;
#pragma unroll
                            for (int q = 0; q < n1; ++q) {
                                if constexpr (DIF) t3 += sF[k * n1 + q] * (pl[2 * NA + u][rowt + n1 * n1 * q] - x);
                                else t3 += sF[k * n1 + q] * pl[2 * NA + u][rowt + n1 * n1 * q];
                            }
                            if constexpr (DIF) t3 += x;
                            fq[a] = t3;
                        }
                    });
                }
            });
        }
        if constexpr (MODE == M_FILTER) {
            if (valid && own) {
                static_for<0, Q>([&](auto AA) {
                    constexpr int a = decltype(AA)::value;
                    A.out[si.base + (int64_t)a * si.stride] = fq[a];
                });
            }
            return;
        }
    }

    T rho = 0;
    if constexpr (MODE == M_STAGE1) {
        if (valid) {
            T om = A.omega;
            if (A.dtau) om = T(1) / (A.tau + T(A.dtau[gix]) + T(0.5));
            collide_node<DIM, Q, T, DEV>(fq, A.rho0, om, A.dt, A.g, rho);
            if (own) {
                static_for<0, Q>([&](auto AA) {
                    constexpr int a = decltype(AA)::value;
                    A.f0out[si.base + (int64_t)a * si.stride] = fq[a];
                });
                A.rhoc[gix] = rho;
            }
        }
        if (A.collide_only) return;  // whole workgroup
    } else if constexpr (MODE == M_STAGE23) {
        if (valid && inner) rho = A.rhoc[gix];
    }

    // D-hat rows of this node and its metric terms
    T Di[n1], Dj[n1], Dk[n1];
#pragma unroll
    for (int c = 0; c < n1; ++c) {
        const T *Dt = SD ? sD : A.D;
        Di[c] = Dt[i * n1 + c];
        Dj[c] = Dt[j * n1 + c];
        Dk[c] = (DIM == 3) ? Dt[k * n1 + c] : T(0);
    }
    if (have_metric) {
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int q = 0; q < DIM; ++q) Gr[m][q] = sG[(m * DIM + q) * NP + p];
        invw = sG[DIM * DIM * NP + p];
    } else {
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int q = 0; q < DIM; ++q)
                Gr[m][q] = valid ? __builtin_nontemporal_load(A.Gm + (e * DIM * DIM + m * DIM + q) * NP + p) : T(0);
        if (MODE != M_LOCAL && valid && inner) invw = A.invw[e * NI + pc];
    }

    // wall faces through this node (flux bounce-back, Sec. 2.2.1): at most
    // one per reference direction m; 8 bits per direction hold the wall tag
    // (0 = none) and bit 7 the side (plus face r_m = +1)
    uint32_t wcode = 0;
    if (valid && !inner) {
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            const int idx = (m == 0) ? i : (m == 1) ? j : k;
            if (idx == 0 || idx == N) {
                const int fc = 2 * m + (idx == N ? 1 : 0);
                const uint32_t tag = (uint32_t)A.ftag[e * 2 * DIM + fc];
                if (tag > 0) wcode |= (tag | (idx == N ? 0x80u : 0u)) << (8 * m);
            }
        }
    }

    // interface faces through this node under the discontinuous coupling
    // (faces that are not walls) and the group of the coincident node across
    // each; face nodes are numbered in increasing node index
    uint32_t icode = 0;
    int32_t gnb[DIM] = {};
    if (DGC && valid && !inner) {
        constexpr int nfn = (DIM == 2) ? n1 : n1 * n1;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            const int idx = (m == 0) ? i : (m == 1) ? j : k;
            if (idx == 0 || idx == N) {
                const int fc = 2 * m + (idx == N ? 1 : 0);
                if (A.ftag[e * 2 * DIM + fc] == 0) {
                    const int t0 = (m == 0) ? j : i;
                    const int t1 = (DIM == 2) ? 0 : (m == 2) ? j : k;
                    gnb[m] = A.nbr[(e * 2 * DIM + fc) * nfn + t0 + n1 * t1];
                    icode |= (1u | (idx == N ? 2u : 0u)) << (2 * m);
                }
            }
        }
    }

    // streaming operator per velocity (Sec. 2.2): P is the velocity's plane in
    // LDS, v and f0v the node's operand and post-collision values
    auto velocity = [&](auto AA, const T *P, T v, T f0v) {
        constexpr int a = decltype(AA)::value;
        T rt = stream_volume<DIM, N, Q, a, DIF>(P, v, Di, Dj, Dk, Gr, rowr, rows, rowt);
        if (wcode) {
            constexpr int b = lat_opp<DIM, Q>(a);
            T vb;
            if constexpr (STG) vb = pl[b][p];
            else if constexpr (ALLQ || FULL) vb = fq[b];
            else vb = A.op[si.base + (int64_t)b * si.stride];
            wall_flux<DIM, N, Q, a>(rt, v, vb, Gr, wcode, A.wallu, A.rho0);
        }
        if constexpr (DGC) {
            if (icode) interface_flux<DIM, N, Q, a>(rt, v, Gr, icode, gnb, A.op, A.QGi);
        }
        if constexpr (STG) {
            // kept in the register of the consumed operand, stored after the loop
            if (inner) fq[a] = rk_combine(A.ca, A.cb, A.cc, f0v, v, rt * invw + A.fsc[a] * rho, A.incr);
            else fq[a] = rt;
        } else if (valid) {
            if constexpr (MODE == M_LOCAL) {
                A.local[((int64_t)a * A.E + e) * NP + p] = rt;
            } else {
                if (inner) {
                    const T L = rt * invw + A.fsc[a] * rho;
                    A.out[si.base + (int64_t)a * si.stride] = rk_combine(A.ca, A.cb, A.cc, f0v, v, L, A.incr);
                } else {
                    A.rtb[(int64_t)a * A.plane + slot] = rt;
                }
            }
        }
    };

    if constexpr (FULL) {
        if (MODE == M_STAGE23 && slotted) {
            // the planes already hold the operand (filled slot by slot)
            __syncthreads();
            static_for<0, Q>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                fq[a] = pl[a][p];
            });
        } else {
            // the filter passes of the first stage used the same LDS
            if constexpr (ALLQ) __syncthreads();
            static_for<0, Q>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                pl[a][p] = fq[a];
            });
            __syncthreads();
        }
        static_for<0, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            T f0v;
            if constexpr (MODE == M_STAGE23) f0v = f0q[a];
            else f0v = fq[a];
            velocity(AA, pl[a], fq[a], f0v);
        });
        if constexpr (STG) {
            // results go through LDS: the element's interior block [Q][NI]
            // is stored as one contiguous run, and the boundary
            // contributions slot by slot in face order. The
            // interior block is written non-temporally (whole lines, not read
            // again in this stage) so that L2 keeps the contribution slots,
            // which neighbouring elements fill line by line, and the shared
            // operand values.
            __syncthreads();  // every plane read done
            // staging [Q][NP] in slot order (interior slots, then boundary
            // slots): one store per velocity for every node, whichever kind
            {
                const int slot = inner ? pc : NI + bsl;
                static_for<0, Q>([&](auto AA) {
                    constexpr int a = decltype(AA)::value;
                    lds[a * NP + slot] = fq[a];
                });
            }
            __syncthreads();
            T *dst = A.out + e * (int64_t)Q * NI;
            if constexpr (NI % 4 == 0 && NP % 4 == 0) {
                typedef T v4 __attribute__((ext_vector_type(4)));
                for (int q = tid; q < Q * NI / 4; q += GG::BLOCK) {
                    const int a = (4 * q) / NI, s0 = 4 * q - a * NI;
                    __builtin_nontemporal_store(*reinterpret_cast<const v4 *>(lds + a * NP + s0),
                                                reinterpret_cast<v4 *>(dst) + q);
                }
            } else {
                for (int q = tid; q < Q * NI; q += GG::BLOCK) {
                    const int a = q / NI;
                    dst[q] = lds[a * NP + q - a * NI];
                }
            }
            const int32_t *pm = A.posmap + e * NB;
            if constexpr (MODE == M_STAGE23) {
                // later stages: one slot per thread (its rank-plane position
                // read once); the rest velocity's contributions are zero and
                // the assembly does not read them
                if (tid < NB) {
                    T *dst = A.rtb + pm[tid];
                    static_for<1, Q>([&](auto AA) {
                        constexpr int a = decltype(AA)::value;
                        dst[(int64_t)a * A.plane] = lds[a * NP + NI + tid];
                    });
                }
            } else {
                for (int q = tid; q < Q * NB; q += GG::BLOCK) {
                    const int a = q / NB, b = q - a * NB;
                    A.rtb[(int64_t)a * A.plane + pm[b]] = lds[a * NP + NI + b];
                }
            }
        }
    } else {
        static_for<0, NC>([&](auto CC) {
            constexpr int c = decltype(CC)::value;
            prefetch(std::integral_constant<int, c + 1>{});
            constexpr int pb = (c & 1) * NA;  // double-buffered plane set
            static_for<0, NA>([&](auto UU) {
                constexpr int u = decltype(UU)::value, a = c * NA + u;
                if constexpr (a < Q) {
                    if constexpr (ALLQ) pl[pb + u][base + p] = fq[a];
                    else if constexpr (c & 1) pl[pb + u][base + p] = roB[u];
                    else pl[pb + u][base + p] = roA[u];
                }
            });
            __syncthreads();
            static_for<0, NA>([&](auto UU) {
                constexpr int u = decltype(UU)::value, a = c * NA + u;
                if constexpr (a < Q) {
                    T v, f0v;
                    if constexpr (ALLQ) v = fq[a];
                    else if constexpr (c & 1) v = roB[u];
                    else v = roA[u];
                    if constexpr (MODE == M_STAGE1) f0v = v;
                    else if constexpr (c & 1) f0v = r0B[u];
                    else f0v = r0A[u];
                    velocity(std::integral_constant<int, a>{}, pl[pb + u], v, f0v);
                }
            });
        });
    }
}

// -------------------------------------------------- boundary-node assembly --
// Direct stiffness summation at shared nodes (continuous Galerkin): the
// element contributions of a node group are summed in ascending member order,
// scaled by the assembled inverse mass, F* is added and the Runge-Kutta
// combination written once for the group. One thread per group, all
// velocities; the member list is read once.
template <typename T>
struct GroupArgs {
    const T *rtb, *f0, *fk, *rhoc, *invMb;
    T *out;
    const int32_t *goff, *hidx;
    int64_t ngrp, Gi, QGi, plane, ngp, nmp;
    T ca, cb, cc;
    int incr;  // ca + cb = 1 (time steps): FP32 increment form
    T fsc[kMaxQ];
    // discontinuous coupling (k_group_split with DGN = N): interface table, face
    // tags, node index of each boundary slot and the metric
    const int32_t *nbr, *ftag, *bpos;
    const T *Gm;
};

// Shared-node assembly (one group per node id on element boundaries): the
// member contributions summed in ascending member order (rank r wrote plane r
// for r < 2 at g, extra plane r - 2 at hidx[g]), times the assembled inverse
// mass, plus F*, then the RK combination. DGN = 0: continuous coupling.
// DGN = N: discontinuous coupling at order N, where every group is one
// element-boundary node (group id e * NB + b) and the upwind flux of its
// interface faces (with the stage value fk across each face) is added to its
// contribution before the mass.
// The velocities of each group are split between two wavefronts: waves 2k
// and 2k + 1 of a workgroup take the lower and upper velocities of the same
// 64 groups (uniform in each wavefront), so a thread holds half the values
// and twice the groups are in flight per CU; the arithmetic of a velocity
// does not depend on the split.
template <int A0, int A1, int Q, typename T, int DGN>
__device__ __forceinline__ void group_range(const GroupArgs<T> &A, int64_t g, int nm, int64_t h, T invM, T rho,
                                            SIdx si)
{
    // every load of the group is issued before its first store (the output
    // may alias the inputs as far as the compiler knows, which would
    // otherwise put one memory latency per velocity on the critical path);
    // read once per stage, so non-temporally
    T sum[A1 - A0], v0[A1 - A0], vk[A1 - A0];
    static_for<A0, A1>([&](auto AA) {
        constexpr int a = decltype(AA)::value, u = a - A0;
        const T *r = A.rtb + (int64_t)a * A.plane;
        const int64_t ix = si.base + (int64_t)a * si.stride;
        // the rest velocity neither streams nor meets a wall flux: its
        // contributions are zero and are not stored by the element kernels
        if constexpr (a == 0) {
            sum[u] = T(0);
        } else {
            sum[u] = __builtin_nontemporal_load(r + g);
            if (nm > 1) sum[u] += __builtin_nontemporal_load(r + A.ngp + g);
        }
        v0[u] = __builtin_nontemporal_load(A.f0 + ix);
        // the discontinuous coupling's stage values are read again by the
        // interface flux of the node across each face: cached loads there
        if constexpr (DGN > 0) vk[u] = A.fk[ix];
        else vk[u] = __builtin_nontemporal_load(A.fk + ix);
    });
    for (int t = 2; t < nm; ++t) {
        const int64_t o = 2 * A.ngp + (t - 2) * A.nmp + h;
        static_for<A0, A1>([&](auto AA) {
            constexpr int a = decltype(AA)::value, u = a - A0;
            if constexpr (a != 0) sum[u] += A.rtb[(int64_t)a * A.plane + o];
        });
    }
    if constexpr (DGN > 0) {
        // upwind interface flux of the discontinuous coupling on the faces
        // of the node that are not walls (every node is a group of one)
        constexpr int DIM = (Q == 9) ? 2 : 3;
        constexpr int n1 = DGN + 1, NP = ipow_c(n1, DIM), NB = NP - ipow_c(DGN - 1, DIM);
        constexpr int nfn = (DIM == 2) ? n1 : n1 * n1;
        const int64_t e = g / NB;
        const int p = A.bpos[g - e * NB];
        const int i = p % n1, j = (p / n1) % n1, k = (DIM == 3) ? p / (n1 * n1) : 0;
        uint32_t icode = 0;
        int32_t gnb[DIM] = {};
        T Gr[DIM][DIM] = {};
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            const int idx = (m == 0) ? i : (m == 1) ? j : k;
            if (idx == 0 || idx == DGN) {
                const int fc = 2 * m + (idx == DGN ? 1 : 0);
                if (A.ftag[e * 2 * DIM + fc] == 0) {
                    const int t0 = (m == 0) ? j : i;
                    const int t1 = (DIM == 2) ? 0 : (m == 2) ? j : k;
                    gnb[m] = A.nbr[(e * 2 * DIM + fc) * nfn + t0 + n1 * t1];
                    icode |= (1u | (idx == DGN ? 2u : 0u)) << (2 * m);
#pragma unroll
                    for (int q = 0; q < DIM; ++q) Gr[m][q] = A.Gm[(e * DIM * DIM + m * DIM + q) * NP + p];
                }
            }
        }
        // face by face: every velocity across the face is loaded before the
        // first is used (the upwind test only selects), so a face costs one
        // memory round trip; per velocity the faces add in the order of m
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            if ((icode >> (2 * m)) & 1u) {
                const SIdx so = sidx_group(gnb[m], Q, A.QGi);
                T vn[A1 - A0];
                static_for<A0, A1>([&](auto AA) {
                    constexpr int a = decltype(AA)::value, u = a - A0;
                    vn[u] = A.fk[so.base + (int64_t)a * so.stride];
                });
                const T sc = (((icode >> (2 * m + 1)) & 1u) ? T(1) : T(-1)) * T(DGN * (DGN + 1)) / T(2);
                static_for<A0, A1>([&](auto AA) {
                    constexpr int a = decltype(AA)::value, u = a - A0;
                    constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
                    T ne = T(ex) * Gr[m][0] + T(ey) * Gr[m][1];
                    if constexpr (DIM == 3) ne += T(ez) * Gr[m][2];
                    ne *= sc;
                    if (ne < T(0)) sum[u] += ne * (vk[u] - vn[u]);
                });
            }
        }
    }
    static_for<A0, A1>([&](auto AA) {
        constexpr int a = decltype(AA)::value, u = a - A0;
        const int64_t ix = si.base + (int64_t)a * si.stride;
        const T L = sum[u] * invM + A.fsc[a] * rho;
        A.out[ix] = rk_combine(A.ca, A.cb, A.cc, v0[u], vk[u], L, A.incr);
    });
}

template <int Q, typename T, int DGN = 0>
__global__ void __launch_bounds__(256) k_group_split(GroupArgs<T> A)
{
    const int w = threadIdx.x >> 6;
    // blocks of 128 groups, a contiguous range of them per XCD: groups are
    // ordered by owner element, so each XCD assembles the groups of the
    // elements it streams, and the next stage finds them in its own L2
    const int64_t nb = (A.ngrp + 127) / 128;
    const int64_t gb = xcd_block(nb);
    if (gb >= nb) return;  // whole workgroup
    const int64_t g = gb * 128 + (w >> 1) * 64 + (threadIdx.x & 63);
    if (g >= A.ngrp) return;
    const int nm = A.goff[g + 1] - A.goff[g];
    const int64_t h = (nm > 2) ? (int64_t)A.hidx[g] : 0;
    const T invM = A.invMb[g];
    const T rho = A.rhoc[A.Gi + g];
    const SIdx si = sidx_group(g, Q, A.QGi);
    constexpr int HQ = (Q + 1) / 2;
    if (w & 1) group_range<HQ, Q, Q, T, DGN>(A, g, nm, h, invM, rho, si);
    else group_range<0, HQ, Q, T, DGN>(A, g, nm, h, invM, rho, si);
}

// ------------------------------------------------------ closure features --
// Per element node (learned closure; the method itself has none): velocity
// u = sum e f / rho, its element-local gradient A_ck = du_c/dx_k (D-hat along
// reference lines and the metric dr/dx = G / wJ), S and W the symmetric and
// skew parts, Pi = sum_a e e (f_a - f^eq_a), lam = nu / c_s^2, and
//   x = [lam^2 S:S, lam^2 W:W, lam^3 tr S^3, lam^3 tr S W W,
//        Pi:Pi / (rho c_s^2)^2, lam Pi:S / (rho c_s^2)]  (raw, not normalised).
// owner_out: one row per node id (owning copy); else one row per element node.
template <typename T>
struct FeatArgs {
    const T *f, *Gm, *D, *F;
    const double *wJ;
    const int32_t *pcode, *bmap;
    const uint8_t *bown;
    float *X;
    int64_t E, nblk, Gi, QGi;
    T rho0, lam;
    int owner_out;
    int filter;  // features of the filtered state (the filter is linear, so the moment fields are filtered)
    double *grad;  // when set: row grad_row of the velocity gradient, du_c/dx_q [E][np][dim] (FP64), no features
    int grad_row;
};

// GRAD: write one row of the velocity gradient instead of the features (a
// separate instantiation, so the feature kernel carries none of it)
template <int DIM, int N, int Q, typename T, bool DEV, bool GRAD = false>
__global__ void __launch_bounds__((Geo<DIM, N>::BLOCK)) k_features(FeatArgs<T> A)
{
    using GG = Geo<DIM, N>;
    constexpr int n1 = GG::n1, NP = GG::NP, NI = GG::NI, NB = GG::NB, EPB = GG::EPB;
    constexpr int NM = 1 + DIM + DIM * (DIM + 1) / 2;  // m0, j, sum e e f
    constexpr bool DIF = std::is_same<T, float>::value;
    __shared__ T pl[NM][EPB * NP];
    __shared__ T sF[n1 * n1];
    const int tid = threadIdx.x;
    const int le = tid / NP;
    const int p = tid - le * NP;
    const int64_t eb = blockIdx.x;
    if (eb >= A.nblk) return;
    const int64_t e = eb * EPB + le;
    const bool valid = e < A.E;
    if (A.filter)
        for (int q = tid; q < n1 * n1; q += GG::BLOCK) sF[q] = A.F[q];
    const int i = p % n1, j = (p / n1) % n1, k = (DIM == 3) ? p / (n1 * n1) : 0;
    const int pc = A.pcode[p];
    const bool inner = pc >= 0;
    const int bsl = inner ? 0 : -pc - 1;
    int64_t gix = 0;
    bool own = false;
    SIdx si{0, 0};
    if (valid) {
        if (inner) {
            gix = e * NI + pc;
            own = true;
            si = sidx_interior(e, pc, Q, NI);
        } else {
            const int64_t g = A.bmap[e * NB + bsl];
            gix = A.Gi + g;
            own = A.bown[e * NB + bsl] != 0;
            si = sidx_group(g, Q, A.QGi);
        }
    }
    const int base = le * NP;
    const int rowr = base + n1 * j + n1 * n1 * k;
    const int rows = base + i + n1 * n1 * k;
    const int rowt = base + i + n1 * j;
    // moment fields of the node: m0 = sum f (deviation sum when DEV), j = sum e f,
    // P = sum e e f (deviation part when DEV: the full value adds rho0 cs^2 I)
    T M[NM] = {};
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        constexpr int ev[3] = {lat_e<DIM, Q>(a, 0), lat_e<DIM, Q>(a, 1), lat_e<DIM, Q>(a, 2)};
        const T v = valid ? A.f[si.base + (int64_t)a * si.stride] : T(0);
        M[0] += v;
        int q = 1 + DIM;
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            if (ev[r] != 0) M[1 + r] += T(ev[r]) * v;
#pragma unroll
            for (int c = r; c < DIM; ++c) {
                if (ev[r] != 0 && ev[c] != 0) M[q] += T(ev[r] * ev[c]) * v;
                ++q;
            }
        }
    });
    if (A.filter) {
        // explicit modal filter (Sec. 2.2.3) of the moment fields, one direction per pass
#pragma unroll
        for (int c = 0; c < NM; ++c) pl[c][base + p] = M[c];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            const int row = (m == 0) ? rowr : (m == 1) ? rows : rowt;
            const int st = (m == 0) ? 1 : (m == 1) ? n1 : n1 * n1;
            const int ir = (m == 0) ? i : (m == 1) ? j : k;
#pragma unroll
            for (int c = 0; c < NM; ++c) {
                const T x = M[c];
                T t = 0;
#pragma unroll
                for (int q = 0; q < n1; ++q) {
                    if constexpr (DIF) t += sF[ir * n1 + q] * (pl[c][row + st * q] - x);
                    else t += sF[ir * n1 + q] * pl[c][row + st * q];
                }
                M[c] = DIF ? t + x : t;
            }
            __syncthreads();
            if (m + 1 < DIM) {
#pragma unroll
                for (int c = 0; c < NM; ++c) pl[c][base + p] = M[c];
                __syncthreads();
            }
        }
    }
    const T rho = valid ? (DEV ? A.rho0 + M[0] : M[0]) : T(1);
    T u[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < DIM; ++c) u[c] = M[1 + c] / rho;
    // non-equilibrium second moment: Pi = sum e e f - rho cs^2 I - rho u u
    // (the second moment of the lattice equilibrium is exactly rho cs^2 I + rho u u)
    T Pi[3][3] = {};
    {
        int q = 1 + DIM;
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = r; c < DIM; ++c) {
                T v = M[q++] - rho * u[r] * u[c];
                if (r == c) v -= (DEV ? M[0] : rho) * T(1.0 / 3.0);
                Pi[r][c] = Pi[c][r] = v;
            }
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) pl[c][base + p] = u[c];
    __syncthreads();
    if (!valid) return;
    const int idx[3] = {i, j, k};
    const int str[3] = {1, n1, n1 * n1};
    T du[3][3] = {};  // du[c][m] = du_c / dr_m
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        const int b0 = base + p - idx[m] * str[m];
#pragma unroll
        for (int q = 0; q < n1; ++q) {
            const T dq = A.D[idx[m] * n1 + q];
#pragma unroll
            for (int c = 0; c < DIM; ++c) du[c][m] += dq * pl[c][b0 + q * str[m]];
        }
    }
    const T iwj = T(1.0 / A.wJ[e * NP + p]);
    T Am[3][3] = {};  // Am[c][q] = du_c / dx_q
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
            const T drdx = A.Gm[(e * DIM * DIM + m * DIM + q) * NP + p] * iwj;
#pragma unroll
            for (int c = 0; c < DIM; ++c) Am[c][q] += du[c][m] * drdx;
        }
    if constexpr (GRAD) {
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
            T v = 0;
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                if (c == A.grad_row) v = Am[c][q];
            A.grad[(e * NP + p) * DIM + q] = double(v);
        }
        return;
    }
    T S[3][3], W[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            S[r][c] = T(0.5) * (Am[r][c] + Am[c][r]);
            W[r][c] = T(0.5) * (Am[r][c] - Am[c][r]);
        }
    T ss = 0, ww = 0, s3 = 0, sww = 0, pp = 0, ps = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ss += S[r][c] * S[r][c];
            ww += W[r][c] * W[r][c];
            pp += Pi[r][c] * Pi[r][c];
            ps += Pi[r][c] * S[r][c];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                s3 += S[r][c] * S[c][q] * S[q][r];
                sww += S[r][c] * W[c][q] * W[q][r];
            }
        }
    const T lam = A.lam, rc = rho * T(1.0 / 3.0);
    const float x[6] = {float(lam * lam * ss), float(lam * lam * ww), float(lam * lam * lam * s3),
                        float(lam * lam * lam * sww), float(pp / (rc * rc)), float(lam * ps / rc)};
    if (A.owner_out) {
        if (own)
#pragma unroll
            for (int q = 0; q < 6; ++q) A.X[gix * 6 + q] = x[q];
    } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) A.X[(e * NP + p) * 6 + q] = x[q];
    }
}

// ---------------------------------------------------------------- geometry --
// Isoparametric geometry in FP64 (Sec. 2.2): dx/dr by D-hat on the node
// coordinates, J = det, grad r_m = (a_{m+1} x a_{m+2}) / J with a_m = dx/dr_m
// (2D: rotated tangents), wJ = w w w J, G_mk = wJ dr_m/dx_k. Node p of
// element e; coordinate q of element node c is sx[q * ld + off + c].
template <int DIM, int N, typename T>
__device__ __forceinline__ void geom_node(const double *sx, int ld, int off, int p, int64_t e, const double *D,
                                          const double *w, double *wJ, double *Jo, T *Gm, int32_t *flag)
{
    constexpr int n1 = N + 1, NP = ipow_c(n1, DIM);
    const int idx[3] = {p % n1, (p / n1) % n1, DIM == 3 ? p / (n1 * n1) : 0};
    const int str[3] = {1, n1, n1 * n1};
    double a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // a[m][q] = dx_q / dr_m
    for (int m = 0; m < DIM; ++m) {
        const int b0 = p - idx[m] * str[m];
        for (int c = 0; c < n1; ++c) {
            const double d = D[idx[m] * n1 + c];
            for (int q = 0; q < DIM; ++q) a[m][q] += d * sx[q * ld + off + b0 + c * str[m]];
        }
    }
    double J, gr[3][3];  // gr[m][q] = dr_m / dx_q
    if (DIM == 2) {
        J = a[0][0] * a[1][1] - a[0][1] * a[1][0];
        gr[0][0] = a[1][1] / J;
        gr[0][1] = -a[1][0] / J;
        gr[1][0] = -a[0][1] / J;
        gr[1][1] = a[0][0] / J;
    } else {
        double cx[3][3];
        for (int m = 0; m < 3; ++m) {
            const double *u = a[(m + 1) % 3], *v = a[(m + 2) % 3];
            cx[m][0] = u[1] * v[2] - u[2] * v[1];
            cx[m][1] = u[2] * v[0] - u[0] * v[2];
            cx[m][2] = u[0] * v[1] - u[1] * v[0];
        }
        J = a[0][0] * cx[0][0] + a[0][1] * cx[0][1] + a[0][2] * cx[0][2];
        for (int m = 0; m < 3; ++m)
            for (int q = 0; q < 3; ++q) gr[m][q] = cx[m][q] / J;
    }
    double wp = w[idx[0]] * w[idx[1]];
    if (DIM == 3) wp *= w[idx[2]];
    const double wj = wp * J;
    wJ[e * NP + p] = wj;
    Jo[e * NP + p] = J;
    for (int m = 0; m < DIM; ++m)
        for (int q = 0; q < DIM; ++q) Gm[(e * DIM * DIM + m * DIM + q) * NP + p] = T(wj * gr[m][q]);
    if (!(J > 0.0)) atomicOr(flag, 1);
}

template <int DIM, int N, typename T>
__global__ void __launch_bounds__((Geo<DIM, N>::BLOCK))
    k_geom(const double *xyz, const double *D, const double *w, double *wJ, double *Jo, T *Gm, int32_t *flag,
           int64_t E, int64_t nblk)
{
    using GG = Geo<DIM, N>;
    constexpr int NP = GG::NP, EPB = GG::EPB;
    __shared__ double sx[DIM][EPB * NP];
    const int tid = threadIdx.x;
    const int le = tid / NP, p = tid - le * NP;
    const int64_t eb = blockIdx.x;
    if (eb >= nblk) return;
    const int64_t e = eb * EPB + le;
    const bool valid = e < E;
#pragma unroll
    for (int q = 0; q < DIM; ++q) sx[q][le * NP + p] = valid ? xyz[(e * NP + p) * DIM + q] : 0.0;
    __syncthreads();
    if (!valid) return;
    geom_node<DIM, N, T>(&sx[0][0], EPB * NP, le * NP, p, e, D, w, wJ, Jo, Gm, flag);
}

// inverse lumped mass: interior nodes 1/wJ, boundary groups 1/sum of member wJ
template <typename T>
__global__ void k_mass_int(const double *wJ, const int32_t *pcode, T *invw, int64_t E, int NP, int NI)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= E * NP) return;
    const int64_t e = q / NP;
    const int p = (int)(q - e * NP);
    const int pc = pcode[p];
    if (pc >= 0) invw[e * NI + pc] = T(1.0 / wJ[q]);
}
template <typename T>
__global__ void k_mass_grp(const double *wJ, const int32_t *bpos, const int32_t *goff, const int32_t *gmem,
                           T *invMb, int64_t ngrp, int NP, int NB)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngrp) return;
    double s = 0.0;
    for (int q = goff[g]; q < goff[g + 1]; ++q) {
        const int64_t lb = gmem[q];
        const int64_t e = lb / NB;
        const int b = (int)(lb - e * NB);
        s += wJ[e * NP + bpos[b]];
    }
    invMb[g] = T(1.0 / s);
}

// per-node helpers over local (element) nodes
struct NodeMap {
    const int32_t *pcode, *bmap;
    const uint8_t *bown;
    int64_t E, Gi, QGi;
    int NP, NI, NB, Q;
    // state index of element node (e, p); own = this copy writes shared nodes
    __device__ __forceinline__ SIdx sidx(int64_t e, int p, bool &own) const
    {
        const int pc = pcode[p];
        if (pc >= 0) {
            own = true;
            return sidx_interior(e, pc, Q, NI);
        }
        const int b = -pc - 1;
        own = bown[e * NB + b] != 0;
        return sidx_group(bmap[e * NB + b], Q, QGi);
    }
};

// f-bar = f^eq(rho, u) - dt F** / 2 (Sec. 2.1 with f = f^eq), computed in FP64
template <int DIM, int Q, typename T, bool DEV>
__global__ void k_init(NodeMap M, const double *rho, const double *u, T *f, double rho0, double dt,
                       double g0, double g1, double g2)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M.E * M.NP) return;
    const int64_t e = q / M.NP;
    const int p = (int)(q - e * M.NP);
    bool own;
    const SIdx si = M.sidx(e, p, own);
    if (!own) return;
    const double r = rho[q];
    double uu[3] = {0, 0, 0};
    for (int c = 0; c < DIM; ++c) uu[c] = u[q * DIM + c];
    const double F[3] = {r * g0, r * g1, r * g2};
    const double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
    const double uF = uu[0] * F[0] + uu[1] * F[1] + uu[2] * F[2];
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        const double ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
        const double t = lat_t<DIM, Q>(a);
        const double eu = ex * uu[0] + ey * uu[1] + ez * uu[2];
        const double eF = ex * F[0] + ey * F[1] + ez * F[2];
        const double feq = t * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2);
        const double fss = t * (9.0 * eu * eF - 3.0 * uF);
        double v = feq - 0.5 * dt * fss;
        if (DEV) v -= t * rho0;
        f[si.base + (int64_t)a * si.stride] = T(v);
    });
}

// one velocity plane between the state and an FP64 element-node array
template <typename T>
__global__ void k_scatter_plane(NodeMap M, const double *src, T *dst, int a, double off)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M.E * M.NP) return;
    const int64_t e = q / M.NP;
    const int p = (int)(q - e * M.NP);
    bool own;
    const SIdx si = M.sidx(e, p, own);
    if (own) dst[si.base + (int64_t)a * si.stride] = T(src[q] - off);
}
template <typename T>
__global__ void k_gather_plane(NodeMap M, const T *src, double *dst, int a, double off)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M.E * M.NP) return;
    const int64_t e = q / M.NP;
    const int p = (int)(q - e * M.NP);
    bool own;
    const SIdx si = M.sidx(e, p, own);
    dst[q] = double(src[si.base + (int64_t)a * si.stride]) + off;
}

// ------------------------------------------------------ per-node force --
// A force density per node F_n is added to rho g (Sec. 2.1; F = rho g + F_n,
// taken at the collision and frozen for the stages). Both force terms are
// linear in F, so the per-node part is applied by two passes over the node
// ids beside the kernels of the body force: F** after the collision, F*
// after each stage's assembly.

// state index of node id q (interior ids first, then the groups)
__device__ __forceinline__ SIdx sidx_node(int64_t q, int64_t Gi, int NI, int Q, int64_t QGi)
{
    if (q < Gi) {
        const int64_t e = q / NI;
        return sidx_interior(e, (int)(q - e * NI), Q, NI);
    }
    return sidx_group(q - Gi, Q, QGi);
}

// F [E][np][dim] (FP64) -> Fn [Gtot][3] by node id, from the owning copies
template <typename T>
__global__ void k_force_set(NodeMap M, const double *F, int dim, T *Fn)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M.E * M.NP) return;
    const int64_t e = q / M.NP;
    const int p = (int)(q - e * M.NP);
    const int pc = M.pcode[p];
    int64_t id;
    if (pc >= 0) {
        id = e * M.NI + pc;
    } else {
        const int b = -pc - 1;
        if (!M.bown[e * M.NB + b]) return;
        id = M.Gi + M.bmap[e * M.NB + b];
    }
    for (int k = 0; k < 3; ++k) Fn[id * 3 + k] = k < dim ? T(F[q * dim + k]) : T(0);
}

// after the collision: f*_a += (1 - omega/2) dt F**_a(u, F_n), with
// F**_a = t_a ((e.u)(e.F)/cs4 - (u.F)/cs2) and u = j / rho of the
// post-collision state (the collision and F** of rho g leave j unchanged)
template <int DIM, int Q, typename T, bool DEV>
__global__ void k_force_collide(T *f, const T *Fn, const float *dtau, int64_t Gtot, int64_t Gi, int NI,
                                int64_t QGi, T tau, T dt, T rho0)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Gtot) return;
    const SIdx si = sidx_node(q, Gi, NI, Q, QGi);
    T v[Q];
    T m0 = 0, j0 = 0, j1 = 0, j2 = 0;
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        v[a] = f[si.base + (int64_t)a * si.stride];
        m0 += v[a];
        if constexpr (lat_e<DIM, Q>(a, 0) != 0) j0 += T(lat_e<DIM, Q>(a, 0)) * v[a];
        if constexpr (lat_e<DIM, Q>(a, 1) != 0) j1 += T(lat_e<DIM, Q>(a, 1)) * v[a];
        if constexpr (lat_e<DIM, Q>(a, 2) != 0) j2 += T(lat_e<DIM, Q>(a, 2)) * v[a];
    });
    const T rho = DEV ? rho0 + m0 : m0;
    const T u0 = j0 / rho, u1 = j1 / rho, u2 = j2 / rho;
    const T F0 = Fn[q * 3], F1 = Fn[q * 3 + 1], F2 = Fn[q * 3 + 2];
    const T uF = u0 * F0 + u1 * F1 + u2 * F2;
    const T omega = T(1) / (tau + (dtau ? T(dtau[q]) : T(0)) + T(0.5));
    const T coef = (T(1) - T(0.5) * omega) * dt;
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
        const T t = T(lat_t<DIM, Q>(a));
        const T eu = T(ex) * u0 + T(ey) * u1 + T(ez) * u2;
        const T eF = T(ex) * F0 + T(ey) * F1 + T(ez) * F2;
        f[si.base + (int64_t)a * si.stride] = v[a] + coef * (t * (T(9) * eu * eF - T(3) * uF));
    });
}

// after a stage out = ca f0 + cb fk + cc L(fk): out_a += cc F*_a(F_n),
// F*_a = t_a (e_a . F) / cs2
template <int DIM, int Q, typename T>
__global__ void k_force_stage(T *out, const T *Fn, int64_t Gtot, int64_t Gi, int NI, int64_t QGi, T cc)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Gtot) return;
    const SIdx si = sidx_node(q, Gi, NI, Q, QGi);
    const T F0 = Fn[q * 3], F1 = Fn[q * 3 + 1], F2 = Fn[q * 3 + 2];
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
        if constexpr (ex != 0 || ey != 0 || ez != 0) {
            const T t = T(lat_t<DIM, Q>(a));
            out[si.base + (int64_t)a * si.stride] += cc * (t * T(3) * (T(ex) * F0 + T(ey) * F1 + T(ez) * F2));
        }
    });
}

// moments (Eqs. pressure, momentum) in FP64 at every element node
template <int DIM, int Q, typename T, bool DEV>
__global__ void k_moments(NodeMap M, const T *f, double rho0, double *rho, double *u)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M.E * M.NP) return;
    const int64_t e = q / M.NP;
    const int p = (int)(q - e * M.NP);
    bool own;
    const SIdx si = M.sidx(e, p, own);
    double m = 0, j[3] = {0, 0, 0};
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        const double v = double(f[si.base + (int64_t)a * si.stride]);
        m += v;
        if constexpr (lat_e<DIM, Q>(a, 0) != 0) j[0] += lat_e<DIM, Q>(a, 0) * v;
        if constexpr (lat_e<DIM, Q>(a, 1) != 0) j[1] += lat_e<DIM, Q>(a, 1) * v;
        if constexpr (lat_e<DIM, Q>(a, 2) != 0) j[2] += lat_e<DIM, Q>(a, 2) * v;
    });
    const double r = DEV ? rho0 + m : m;
    rho[q] = r;
    for (int c = 0; c < DIM; ++c) u[q * DIM + c] = j[c] / r;
}

// per element node: wJ (u . n) and wJ (u = sum e f / rho, Eq. momentum) for
// the radial profile diagnostic, FP64 [2][E][np]
template <int DIM, int Q, typename T, bool DEV>
__global__ void k_axial_terms(NodeMap M, const T *f, const double *wJ, double rho0, double n0, double n1,
                              double n2, double *out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nl = M.E * M.NP;
    if (q >= nl) return;
    const int64_t e = q / M.NP;
    const int p = (int)(q - e * M.NP);
    bool own;
    const SIdx si = M.sidx(e, p, own);
    double m = 0, j[3] = {0, 0, 0};
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        const double v = double(f[si.base + (int64_t)a * si.stride]);
        m += v;
        if constexpr (lat_e<DIM, Q>(a, 0) != 0) j[0] += lat_e<DIM, Q>(a, 0) * v;
        if constexpr (lat_e<DIM, Q>(a, 1) != 0) j[1] += lat_e<DIM, Q>(a, 1) * v;
        if constexpr (lat_e<DIM, Q>(a, 2) != 0) j[2] += lat_e<DIM, Q>(a, 2) * v;
    });
    const double r = DEV ? rho0 + m : m;
    const double un = (j[0] * n0 + j[1] * n1 + j[2] * n2) / r;
    out[q] = wJ[q] * un;
    out[nl + q] = wJ[q];
}

// FP64 integrals with the lumped mass and a non-finite count; per-block
// partial sums in fixed order, summed by k_reduce_final.
template <int DIM, int Q, typename T, bool DEV>
__global__ void __launch_bounds__(256) k_reduce(NodeMap M, const T *f, int64_t nstate, const double *wJ,
                                                double rho0, double *part)
{
    __shared__ double sh[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t nl = M.E * M.NP;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nl; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = q / M.NP;
        const int p = (int)(q - e * M.NP);
        bool own;
        const SIdx si = M.sidx(e, p, own);
        double m = 0, j[3] = {0, 0, 0};
        static_for<0, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            const double v = double(f[si.base + (int64_t)a * si.stride]);
            m += v;
            if constexpr (lat_e<DIM, Q>(a, 0) != 0) j[0] += lat_e<DIM, Q>(a, 0) * v;
            if constexpr (lat_e<DIM, Q>(a, 1) != 0) j[1] += lat_e<DIM, Q>(a, 1) * v;
            if constexpr (lat_e<DIM, Q>(a, 2) != 0) j[2] += lat_e<DIM, Q>(a, 2) * v;
        });
        const double r = DEV ? rho0 + m : m;
        const double wj = wJ[q];
        acc[0] += wj * r;
        double u2 = 0;
        for (int c = 0; c < DIM; ++c) {
            acc[1 + c] += wj * j[c];
            u2 += (j[c] / r) * (j[c] / r);
        }
        acc[4] += wj * 0.5 * rho0 * u2;
    }
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nstate; q += (int64_t)gridDim.x * blockDim.x) {
        const T v = f[q];
        if (!(v == v) || v - v != T(0)) acc[5] += 1.0;
    }
    for (int c = 0; c < 8; ++c) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 8; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 8; ++c) part[blockIdx.x * 8 + c] = sh[c][0];
}

template <typename T>
__global__ void k_reduce_final(const double *part, int nblk, double *out)
{
    if (threadIdx.x >= 8) return;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += part[b * 8 + threadIdx.x];
    out[threadIdx.x] = s;
}

}  // namespace sel
