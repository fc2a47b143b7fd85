// Element kernels for 3D orders whose (N + 1)^3 element nodes exceed one
// workgroup (N >= 10; the paper's Taylor-Green runs reach N = 12, Sec. 3.4).
// One workgroup per element as in k_stage, but each thread takes R nodes
// (node p = tid + r BLOCK) and the velocities pass through LDS one plane at a
// time. The arithmetic per node and velocity is that of k_stage (the same
// collision, streaming, wall-flux and Runge-Kutta helpers); this path serves
// the high orders, the N = 7 throughput path is k_stage / k_stage23_mf.
#pragma once

#include "kernels_impl.h"

namespace sel {

template <int N>
struct BigGeo {
    static constexpr int n1 = N + 1;
    static constexpr int NP = n1 * n1 * n1;
    static constexpr int NI = (N - 1) * (N - 1) * (N - 1);
    static constexpr int NB = NP - NI;
    static constexpr int R = (NP + 1023) / 1024;                          // nodes per thread
    static constexpr int BLOCK = ((NP + R - 1) / R + 63) / 64 * 64;       // whole wavefronts
    static_assert(R * BLOCK >= NP && BLOCK <= 1024, "every node has a thread");
};

// One pass of the modal filter (Sec. 2.2.3) along reference direction m at
// node p of plane P: sum_q F[i_m][q] P(line q). FP32 (DIF) takes it around
// the node's own value, as k_stage does.
template <int N, int m, bool DIF, typename T>
__device__ __forceinline__ T filter_line(const T *P, const T *sF, int p, int i, int j, int k)
{
    constexpr int n1 = N + 1;
    constexpr int st = (m == 0) ? 1 : (m == 1) ? n1 : n1 * n1;
    const int ir = (m == 0) ? i : (m == 1) ? j : k;
    const int row = p - ir * st;
    const T x = P[p];
    T t = 0;
#pragma unroll
    for (int q = 0; q < n1; ++q) {
        if constexpr (DIF) t += sF[ir * n1 + q] * (P[row + st * q] - x);
        else t += sF[ir * n1 + q] * P[row + st * q];
    }
    if constexpr (DIF) t += x;
    return t;
}

template <int N, int Q, typename T, bool DEV, int MODE>
__global__ void __launch_bounds__(BigGeo<N>::BLOCK) k_stage_big(StageArgs<T> A)
{
    using BG = BigGeo<N>;
    constexpr int DIM = 3, n1 = BG::n1, NP = BG::NP, NI = BG::NI, NB = BG::NB, R = BG::R, BLOCK = BG::BLOCK;
    constexpr bool DIF = std::is_same<T, float>::value;
    constexpr bool S1 = MODE == M_STAGE1;
    __shared__ T pl[2][NP];  // a velocity's plane and the filter's second buffer
    __shared__ T sD[n1 * n1], sF[n1 * n1];

    const int tid = threadIdx.x;
    const int64_t e = xcd_block(A.nblk);  // one element per workgroup
    if (e >= A.E) return;                 // whole workgroup
    const bool filt = (MODE == M_FILTER) || (S1 && A.filter);
    for (int q = tid; q < n1 * n1; q += BLOCK) {
        sD[q] = A.D[q];
        if (filt) sF[q] = A.F[q];
    }

    // the thread's nodes: index, state location, owner flag, contribution
    // slot and wall faces (flux bounce-back, as in k_stage)
    int pn[R], ii[R], jj[R], kk[R], pcv[R];
    bool ok[R];
    SIdx si[R];
    int64_t gix[R];
    bool own[R];
    int32_t slot[R];
    uint32_t wcode[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = tid + r * BLOCK;
        ok[r] = p < NP;
        pn[r] = ok[r] ? p : 0;
        ii[r] = pn[r] % n1;
        jj[r] = (pn[r] / n1) % n1;
        kk[r] = pn[r] / (n1 * n1);
        pcv[r] = A.pcode[pn[r]];
        si[r] = {0, 0};
        gix[r] = 0;
        own[r] = false;
        slot[r] = 0;
        wcode[r] = 0;
        if (!ok[r]) continue;
        if (pcv[r] >= 0) {
            gix[r] = e * NI + pcv[r];
            own[r] = true;
            si[r] = sidx_interior(e, pcv[r], Q, NI);
        } else {
            const int bsl = -pcv[r] - 1;
            const int64_t g = A.bmap[e * NB + bsl];
            gix[r] = A.Gi + g;
            own[r] = A.bown[e * NB + bsl] != 0;
            si[r] = sidx_group(g, Q, A.QGi);
            if constexpr (S1 || MODE == M_STAGE23) slot[r] = A.posmap[e * NB + bsl];
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
                const int idx = (m == 0) ? ii[r] : (m == 1) ? jj[r] : kk[r];
                if (idx == 0 || idx == N) {
                    const int fc = 2 * m + (idx == N ? 1 : 0);
                    const uint32_t tag = (uint32_t)A.ftag[e * 2 * DIM + fc];
                    if (tag > 0) wcode[r] |= (tag | (idx == N ? 0x80u : 0u)) << (8 * m);
                }
            }
        }
    }

    // first stage: all velocities of the thread's nodes in registers
    T fq[S1 ? R : 1][S1 ? Q : 1];
    if constexpr (S1 || MODE == M_FILTER) {
        static_for<0, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            if (filt) {
                // explicit modal filter (Sec. 2.2.3): F x F x F on the
                // element's copy of plane a, one direction per pass
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (ok[r]) pl[0][pn[r]] = A.op[si[r].base + (int64_t)a * si[r].stride];
                __syncthreads();  // plane (and the tables) visible
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (ok[r]) pl[1][pn[r]] = filter_line<N, 0, DIF>(pl[0], sF, pn[r], ii[r], jj[r], kk[r]);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (ok[r]) pl[0][pn[r]] = filter_line<N, 1, DIF>(pl[1], sF, pn[r], ii[r], jj[r], kk[r]);
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (!ok[r]) continue;
                    const T y = filter_line<N, 2, DIF>(pl[0], sF, pn[r], ii[r], jj[r], kk[r]);
                    if constexpr (MODE == M_FILTER) {
                        if (own[r]) A.out[si[r].base + (int64_t)a * si[r].stride] = y;
                    } else {
                        fq[r][a] = y;
                    }
                }
                __syncthreads();  // every read of the plane done
            } else if constexpr (S1) {
#pragma unroll
                for (int r = 0; r < R; ++r) fq[r][a] = ok[r] ? A.op[si[r].base + (int64_t)a * si[r].stride] : T(0);
            }
        });
        if constexpr (MODE == M_FILTER) return;
    }
    if (!filt) __syncthreads();  // the tables visible

    T rho[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rho[r] = T(0);
    if constexpr (S1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            T om = A.omega;
            if (A.dtau) om = T(1) / (A.tau + T(A.dtau[gix[r]]) + T(0.5));
            collide_node<DIM, Q, T, DEV>(fq[r], A.rho0, om, A.dt, A.g, rho[r]);
            if (own[r]) {
                static_for<0, Q>([&](auto AA) {
                    constexpr int a = decltype(AA)::value;
                    A.f0out[si[r].base + (int64_t)a * si[r].stride] = fq[r][a];
                });
                A.rhoc[gix[r]] = rho[r];
            }
        }
        if (A.collide_only) return;  // whole workgroup
    } else if constexpr (MODE == M_STAGE23) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (ok[r] && pcv[r] >= 0) rho[r] = A.rhoc[gix[r]];
    }
    T invw[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        invw[r] = (MODE != M_LOCAL && ok[r] && pcv[r] >= 0) ? A.invw[e * NI + pcv[r]] : T(0);

    // FP32: the metric terms of the thread's nodes are read once, and the next
    // velocity's operand and f* are loaded while this one streams (in FP64
    // both made the compiler spill the values it holds: slower)
    constexpr bool PF = DIF;
    T Gk[PF ? R : 1][DIM][DIM];
    T vn[PF ? R : 1], f0n[PF ? R : 1];
    auto fetch = [&](auto BB) {
        constexpr int b = decltype(BB)::value;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (S1) vn[r] = fq[r][b];
            else vn[r] = ok[r] ? A.op[si[r].base + (int64_t)b * si[r].stride] : T(0);
            if constexpr (MODE == M_STAGE23)
                f0n[r] = (ok[r] && pcv[r] >= 0) ? A.f0in[si[r].base + (int64_t)b * si[r].stride] : T(0);
            else f0n[r] = vn[r];
        }
    };
    if constexpr (PF) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int m = 0; m < DIM; ++m)
#pragma unroll
                for (int q = 0; q < DIM; ++q)
                    Gk[r][m][q] = ok[r] ? A.Gm[(e * DIM * DIM + m * DIM + q) * NP + pn[r]] : T(0);
        fetch(std::integral_constant<int, 0>{});
    }

    // streaming operator (Sec. 2.2), one velocity plane at a time
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        constexpr bool rest = lat_e<DIM, Q>(a, 0) == 0 && lat_e<DIM, Q>(a, 1) == 0 && lat_e<DIM, Q>(a, 2) == 0;
        T v[R], f0[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (PF) {
                v[r] = vn[r];
                f0[r] = f0n[r];
            } else if constexpr (S1) {
                v[r] = fq[r][a];
            } else {
                v[r] = ok[r] ? A.op[si[r].base + (int64_t)a * si[r].stride] : T(0);
            }
        }
        if constexpr (PF && a + 1 < Q) fetch(std::integral_constant<int, a + 1>{});
        // the rest velocity does not stream: no plane
        if constexpr (!rest) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (ok[r]) pl[0][pn[r]] = v[r];
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ok[r]) continue;
            const int p = pn[r], i = ii[r], j = jj[r], k = kk[r];
            T rt = T(0);
            if constexpr (!rest) {
                T Di[n1], Dj[n1], Dk[n1];
#pragma unroll
                for (int c = 0; c < n1; ++c) {
                    Di[c] = sD[i * n1 + c];
                    Dj[c] = sD[j * n1 + c];
                    Dk[c] = sD[k * n1 + c];
                }
                T Gr[DIM][DIM];
#pragma unroll
                for (int m = 0; m < DIM; ++m)
#pragma unroll
                    for (int q = 0; q < DIM; ++q) {
                        if constexpr (PF) Gr[m][q] = Gk[r][m][q];
                        else Gr[m][q] = A.Gm[(e * DIM * DIM + m * DIM + q) * NP + p];
                    }
                rt = stream_volume<DIM, N, Q, a, DIF>(pl[0], v[r], Di, Dj, Dk, Gr, n1 * j + n1 * n1 * k,
                                                      i + n1 * n1 * k, i + n1 * j);
                if (wcode[r]) {
                    constexpr int b = lat_opp<DIM, Q>(a);
                    T vb;
                    if constexpr (S1) vb = fq[r][b];
                    else vb = A.op[si[r].base + (int64_t)b * si[r].stride];
                    wall_flux<DIM, N, Q, a>(rt, v[r], vb, Gr, wcode[r], A.wallu, A.rho0);
                }
            }
            if constexpr (MODE == M_LOCAL) {
                A.local[((int64_t)a * A.E + e) * NP + p] = rt;
            } else if (pcv[r] >= 0) {
                T f0v;
                if constexpr (S1) f0v = v[r];
                else if constexpr (PF) f0v = f0[r];
                else f0v = A.f0in[si[r].base + (int64_t)a * si[r].stride];
                const T L = rt * invw[r] + A.fsc[a] * rho[r];
                A.out[si[r].base + (int64_t)a * si[r].stride] = rk_combine(A.ca, A.cb, A.cc, f0v, v[r], L, A.incr);
            } else if constexpr (!rest) {
                // the assembly takes the rest velocity's contributions as zero
                A.rtb[(int64_t)a * A.plane + slot[r]] = rt;
            }
        }
        if constexpr (!rest) __syncthreads();  // every read of the plane done
    });
}

// Isoparametric geometry (as k_geom) at the large orders: R nodes per thread.
template <int N, typename T>
__global__ void __launch_bounds__(BigGeo<N>::BLOCK)
    k_geom_big(const double *xyz, const double *D, const double *w, double *wJ, double *Jo, T *Gm, int32_t *flag,
               int64_t E)
{
    using BG = BigGeo<N>;
    constexpr int NP = BG::NP;
    __shared__ double sx[3][NP];
    const int64_t e = blockIdx.x;
    if (e >= E) return;  // whole workgroup
    for (int p = threadIdx.x; p < NP; p += BG::BLOCK)
#pragma unroll
        for (int q = 0; q < 3; ++q) sx[q][p] = xyz[(e * NP + p) * 3 + q];
    __syncthreads();
    for (int p = threadIdx.x; p < NP; p += BG::BLOCK) geom_node<3, N, T>(&sx[0][0], NP, 0, p, e, D, w, wJ, Jo, Gm, flag);
}

}  // namespace sel
