// FP32 element kernel of the later SSPRK stages (Sec. 2.2.2) for 3D
// elements of order 7 (8 x 8 x 8 nodes, one workgroup of 512 threads per
// element): the streaming operator (Sec. 2.2) with the flux bounce-back term
// (Sec. 2.2.1), the interior Runge-Kutta update and the boundary-node element
// contributions, with two of the three line contractions on the matrix cores.
//
// Memory: the interior block [Q][NI] of the operand and of the post-collision
// state are read as 16-byte vectors (kept in registers for the update); the
// planes of the moving velocities are filled one slot per thread (threads
// 0 .. NB-1 the boundary slots, through the slot's node group; the others
// the interior slots), so that a slot's addresses are computed once (the
// rest velocity neither streams nor meets the wall flux). Results go through
// LDS in slot order: the interior update as 16-byte vectors, the boundary
// contributions one slot per thread.
//
// Contractions: wavefront w holds the k-slice k = w of the element. For each
// velocity, the slice's 8 r-lines and 8 s-lines are one v_mfma_f32_16x16x4f32
// tile pair (K = 8 as two steps of 4): A = D-hat (rows = output position i,
// rows 8..15 zero), B = the 16 lines' values (columns = lines), C[i][line].
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// C[4 (l / 16) + v][l % 16], v < 4; the K index of step s is q = 2 (l / 16) + s.
// The outputs reach the lanes of their nodes through a buffer private to the
// wavefront (wavefront barriers only). The t-lines cross all slices, so the
// t-derivative is taken node by node from the plane.
//
// FP32 without drift: the tile lines are taken relative to their own first
// value r, sum_q D_iq (P_q - r), and the t-lines relative to the node's own
// value; both are exact for constant lines whatever the rounding of D-hat
// (whose rows sum to 0 only in exact arithmetic) and round at the size of the
// variation along the line, not at the level of the populations.
#pragma once

#include "kernels_impl.h"

namespace sel {

typedef float mf4 __attribute__((ext_vector_type(4)));

namespace mfk {

constexpr int n1 = 8, NP = 512, NI = 216, NB = 296;

// node index of interior slot s (interior nodes in lexicographic order)
__device__ __forceinline__ int interior_node(int s)
{
    const int a = s % 6, b = (s / 6) % 6, c = s / 36;
    return (a + 1) + 8 * (b + 1) + 64 * (c + 1);
}

}  // namespace mfk

template <int Q>
__global__ void __launch_bounds__(512, 4) k_stage23_mf(StageArgs<float> A)
{
    using namespace mfk;
    constexpr int DIM = 3;
    // planes of the moving velocities: velocity a in plane a - PO
    constexpr int PO = 1;
    constexpr int NPL = Q - PO;
    constexpr int QM = Q - 1;
    constexpr int STG = QM * NP;  // staging [Q-1][NP] in slot order
    constexpr int PLN = (NPL * NP > STG) ? NPL * NP : STG;
    constexpr int NQ4 = Q * NI / 4;           // float4 of the interior block
    static_assert(NB + NI == NP, "one slot per thread");
    constexpr int NPAIR = (QM + 1) / 2;
    __shared__ __attribute__((aligned(16))) float pl[PLN];
    __shared__ float xb[8][2][128];  // per wavefront: r- and s-derivatives of a velocity pair
    __shared__ float sfs[Q];  // F* per unit density of each velocity

    const int tid = threadIdx.x;
    const int64_t e = xcd_block(A.nblk);
    if (e >= A.nblk) return;  // whole workgroup
    const int p = tid;
    const int i = p & 7, j = (p >> 3) & 7;
    const int k = __builtin_amdgcn_readfirstlane(p >> 6);
    const int pc = A.pcode[p];
    const bool inner = pc >= 0;
    const int bsl = inner ? 0 : -pc - 1;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, li = l & 15, lk = l >> 4;
    const int64_t ib = e * (int64_t)Q * NI;
    static_for<0, Q>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        if (tid == a) sfs[a] = A.fsc[a];
    });

    // ------------------------------------------------------------ loads --
    mf4 fkv[3], f0v[3];
    {
        const mf4 *op4 = reinterpret_cast<const mf4 *>(A.op + ib);
        const mf4 *z4 = reinterpret_cast<const mf4 *>(A.f0in + ib);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int q = tid + 512 * r;
            const bool ok = q < NQ4;
            fkv[r] = ok ? op4[q] : mf4{0.f, 0.f, 0.f, 0.f};
            // read once per stage: non-temporal, like the metric
            f0v[r] = ok ? __builtin_nontemporal_load(z4 + q) : mf4{0.f, 0.f, 0.f, 0.f};
        }
    }
    // boundary slots one per thread (threads 0 .. NB-1): the slot's group is
    // looked up once, then its value of every moving velocity is loaded
    float bv[NPL];
    int bnode = 0;
    if (tid < NB) {
        const int64_t g = A.bmap[e * NB + tid];
        const float *src = A.op + A.QGi + (g / kTile) * (int64_t)Q * kTile + (g % kTile);
        bnode = A.bpos[tid];
        static_for<PO, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            bv[a - PO] = src[a * kTile];
        });
    } else if (tid < NB + NI) {
        // interior slots one per thread as well (the 16-byte vectors above
        // serve the update)
        const int s = tid - NB;
        const float *src = A.op + ib + s;
        bnode = interior_node(s);
        static_for<PO, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            bv[a - PO] = src[a * NI];
        });
    }
    float Gr[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int q = 0; q < 3; ++q) Gr[m][q] = __builtin_nontemporal_load(A.Gm + (e * 9 + m * 3 + q) * NP + p);
    // wall faces through this node (flux bounce-back, Sec. 2.2.1): 8 bits per
    // reference direction, the wall tag and bit 7 for the face r_m = +1
    uint32_t wcode = 0;
    if (!inner) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int idx = (m == 0) ? i : (m == 1) ? j : k;
            if (idx == 0 || idx == 7) {
                const uint32_t tag = (uint32_t)A.ftag[e * 6 + 2 * m + (idx == 7 ? 1 : 0)];
                if (tag > 0) wcode |= (tag | (idx == 7 ? 0x80u : 0u)) << (8 * m);
            }
        }
    }
    // planes
    if (tid < NB + NI) {
        static_for<PO, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            pl[(a - PO) * NP + bnode] = bv[a - PO];
        });
    }
    __syncthreads();

    // --------------------------------------------------- streaming --
    // rt = -wJ e_a . grad f_a = -sum_m c_m d f_a / d r_m (Sec. 2.2) plus the
    // wall flux (Sec. 2.2.1), velocities 1 .. Q-1 in pairs
    float res[QM];
    {
        const float dw0 = li < 8 ? A.D[li * 8 + 2 * lk] : 0.f;
        const float dw1 = li < 8 ? A.D[li * 8 + 2 * lk + 1] : 0.f;
        float Dk[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) Dk[c] = A.D[k * 8 + c];
        const int lbase = (li < 8) ? 8 * li + 64 * k : (li - 8) + 64 * k;
        const int lst = (li < 8) ? 1 : 8;
        const int rowt = i + 8 * j;
        float *X = &xb[w][0][0];
        static_for<0, NPAIR>([&](auto CC) {
            constexpr int c = decltype(CC)::value;
            float tdv[2];
            static_for<0, 2>([&](auto VV) {
                constexpr int v = decltype(VV)::value;
                constexpr int a = 1 + 2 * c + v;
                if constexpr (a < Q) {
                    const float *P = pl + (a - PO) * NP;
                    const float r = P[lbase];
                    const float b0 = P[lbase + lst * (2 * lk)] - r;
                    const float b1 = P[lbase + lst * (2 * lk + 1)] - r;
                    mf4 cv = {0.f, 0.f, 0.f, 0.f};
                    cv = __builtin_amdgcn_mfma_f32_16x16x4f32(dw0, b0, cv, 0, 0, 0);
                    cv = __builtin_amdgcn_mfma_f32_16x16x4f32(dw1, b1, cv, 0, 0, 0);
                    const float x = P[p];
                    float d3 = 0.f;
#pragma unroll
                    for (int q = 0; q < 8; ++q) d3 += Dk[q] * (P[rowt + 64 * q] - x);
                    tdv[v] = d3;
                    if (lk < 2) {
                        if (li < 8) {
#pragma unroll
                            for (int vv = 0; vv < 4; ++vv) X[v * 128 + 4 * lk + vv + 8 * li] = cv[vv];
                        } else {
#pragma unroll
                            for (int vv = 0; vv < 4; ++vv) X[v * 128 + 64 + (li - 8) + 8 * (4 * lk + vv)] = cv[vv];
                        }
                    }
                }
            });
            __builtin_amdgcn_wave_barrier();
            static_for<0, 2>([&](auto VV) {
                constexpr int v = decltype(VV)::value;
                constexpr int a = 1 + 2 * c + v;
                if constexpr (a < Q) {
                    constexpr int ex = lat_e<DIM, Q>(a, 0), ey = lat_e<DIM, Q>(a, 1), ez = lat_e<DIM, Q>(a, 2);
                    const float dr = X[v * 128 + l], ds = X[v * 128 + 64 + l], dt = tdv[v];
                    float cr = 0.f, cs = 0.f, ct = 0.f;
                    if constexpr (ex != 0) {
                        cr += float(ex) * Gr[0][0];
                        cs += float(ex) * Gr[1][0];
                        ct += float(ex) * Gr[2][0];
                    }
                    if constexpr (ey != 0) {
                        cr += float(ey) * Gr[0][1];
                        cs += float(ey) * Gr[1][1];
                        ct += float(ey) * Gr[2][1];
                    }
                    if constexpr (ez != 0) {
                        cr += float(ez) * Gr[0][2];
                        cs += float(ez) * Gr[1][2];
                        ct += float(ez) * Gr[2][2];
                    }
                    float rt = -(cr * dr + cs * ds + ct * dt);
                    if (wcode) {
                        constexpr int b = lat_opp<DIM, Q>(a);
                        wall_flux<DIM, 7, Q, a>(rt, pl[(a - PO) * NP + p], pl[(b - PO) * NP + p], Gr, wcode,
                                                A.wallu, A.rho0);
                    }
                    res[a - 1] = rt;
                }
            });
            __builtin_amdgcn_wave_barrier();
        });
    }

    // ------------------------------------------------------- stores --
    __syncthreads();  // every plane read done: the planes become the staging area
    // staging [Q-1][NP] in slot order (interior slots, then boundary slots):
    // one store per velocity for every node, whichever kind it is
    {
        const int slot = inner ? pc : NI + bsl;
        static_for<1, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            pl[(a - 1) * NP + slot] = res[a - 1];
        });
    }
    __syncthreads();
    // interior: Runge-Kutta update ca f0 + cb fk + cc L, L = rt / wJ + F*
    {
        mf4 *o4 = reinterpret_cast<mf4 *>(A.out + ib);
        const mf4 *rho4 = reinterpret_cast<const mf4 *>(A.rhoc + e * NI);
        const mf4 *iw4 = reinterpret_cast<const mf4 *>(A.invw + e * NI);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int q = tid + 512 * r;
            if (q < NQ4) {
                const int a = (4 * q) / NI, s0 = 4 * q - a * NI;
                const mf4 rh = rho4[s0 / 4];
                const float fs = sfs[a];
                mf4 L;
                if (a == 0) {
                    L = fs * rh;
                } else {
                    const mf4 rt = *reinterpret_cast<const mf4 *>(pl + (a - 1) * NP + s0);
                    L = rt * iw4[s0 / 4] + fs * rh;
                }
                const mf4 fk = fkv[r];
                const mf4 f0 = f0v[r];
                mf4 o;
                if (A.incr) {
                    o = fk + (A.ca * (f0 - fk) + A.cc * L);
                } else {
                    o = A.ca * f0 + A.cb * fk + A.cc * L;
                }
                __builtin_nontemporal_store(o, o4 + q);
            }
        }
    }
    // boundary contributions one slot per thread: the slot's position in the
    // rank planes is read once
    if (tid < NB) {
        float *dst = A.rtb + A.posmap[e * NB + tid];
        static_for<1, Q>([&](auto AA) {
            constexpr int a = decltype(AA)::value;
            dst[(int64_t)a * A.plane] = pl[(a - 1) * NP + NI + tid];
        });
    }
}

}  // namespace sel
