// Launch sequences of the SELBM kernels for one (dim, N, Q, storage) choice.
#pragma once

#include "kernels_big.h"
#include "kernels_impl.h"
#include "kernels_mfma.h"
#include "ops.h"

namespace sel {

#define SEL_LAUNCH_CHECK()                                                                  \
    do {                                                                                    \
        hipError_t err_ = hipGetLastError();                                                \
        if (err_ != hipSuccess) {                                                           \
            set_error(std::string("kernel launch failed: ") + hipGetErrorString(err_));    \
            return SEL_EDEVICE;                                                             \
        }                                                                                   \
    } while (0)

template <int DIM, int N, int Q, typename T, bool DEV>
struct Impl {
    using GG = Geo<DIM, N>;
    static constexpr int NP = GG::NP, NI = GG::NI, NB = GG::NB, EPB = GG::EPB;
    // later-stage element kernel with matrix-core contractions (kernels_mfma.h)
    static constexpr bool kMfma = std::is_same<T, float>::value && DEV && DIM == 3 && N == 7;
    // 3D orders whose element has more nodes than a workgroup has threads
    // (kernels_big.h): several nodes per thread
    static constexpr bool kBig = DIM == 3 && NP > 1024;

    static T *st(sel_sim *s, int i) { return static_cast<T *>(s->f[i]); }
    static int64_t nblk(sel_sim *s) { return (s->E + EPB - 1) / EPB; }

    static NodeMap nodemap(sel_sim *s)
    {
        NodeMap M;
        M.pcode = s->pcode;
        M.bmap = s->bmap;
        M.bown = s->bown;
        M.E = s->E;
        M.Gi = s->Gi;
        M.QGi = (int64_t)Q * s->Gi;
        M.NP = NP;
        M.NI = NI;
        M.NB = NB;
        M.Q = Q;
        return M;
    }

    static StageArgs<T> stage_args(sel_sim *s)
    {
        StageArgs<T> A{};
        A.Gm = static_cast<const T *>(s->Gm);
        A.invw = static_cast<const T *>(s->invw);
        A.D = static_cast<const T *>(s->tabD);
        A.F = static_cast<const T *>(s->tabF);
        A.pcode = s->pcode;
        A.bmap = s->bmap;
        A.bpos = s->bpos;
        A.ftag = s->ftag;
        A.bown = s->bown;
        A.wallu = static_cast<const T *>(s->wallu);
        A.nbr = s->nbr;
        A.E = s->E;
        A.nblk = nblk(s);
        A.Gi = s->Gi;
        A.QGi = (int64_t)Q * s->Gi;
        A.dt = T(s->p.dt);
        A.omega = T(s->omega);
        A.rho0 = T(s->p.rho0);
        for (int q = 0; q < 3; ++q) A.g[q] = T(q < DIM ? s->p.accel[q] : 0.0);
        for (int a = 0; a < Q; ++a) A.fsc[a] = T(s->fsc[a]);
        A.rtb = static_cast<T *>(s->rtb);
        A.posmap = s->posmap;
        A.plane = s->plane;
        A.rhoc = static_cast<T *>(s->rhoc);
        A.tau = T(s->tau);
        A.dtau = nullptr;
        return A;
    }

    static GroupArgs<T> group_args(sel_sim *s)
    {
        GroupArgs<T> B{};
        B.rtb = static_cast<const T *>(s->rtb);
        B.rhoc = static_cast<const T *>(s->rhoc);
        B.invMb = static_cast<const T *>(s->invMb);
        B.goff = s->goff;
        B.hidx = s->hidx;
        B.ngrp = s->ngrp;
        B.Gi = s->Gi;
        B.QGi = (int64_t)Q * s->Gi;
        B.plane = s->plane;
        B.ngp = s->ngp;
        B.nmp = s->nmp;
        for (int a = 0; a < Q; ++a) B.fsc[a] = T(s->fsc[a]);
        B.nbr = s->nbr;
        B.ftag = s->ftag;
        B.bpos = s->bpos;
        B.Gm = static_cast<const T *>(s->Gm);
        return B;
    }

    // events around a launch when sel_step_timed asked for them
    static int tic(sel_sim *s, int kind, hipEvent_t &b)
    {
        if (!s->timing) return SEL_OK;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SEL_EDEVICE;
        s->timing->push_back({kind, {e0, e1}});
        b = e1;
        return hipEventRecord(e0, s->stream) == hipSuccess ? SEL_OK : SEL_EDEVICE;
    }
    static int toc(sel_sim *s, hipEvent_t b)
    {
        if (!s->timing) return SEL_OK;
        return hipEventRecord(b, s->stream) == hipSuccess ? SEL_OK : SEL_EDEVICE;
    }

    template <int MODE>
    static int launch_stage(sel_sim *s, const StageArgs<T> &A)
    {
        dim3 grid((unsigned)xcd_grid(A.nblk)), block(GG::BLOCK);
        hipEvent_t ev = nullptr;
        const int kind = (MODE == M_STAGE1) ? 0 : (MODE == M_STAGE23) ? 1 : 3;
        if constexpr (kBig) {
            if (A.nbr) {
                set_error("the discontinuous coupling takes one thread per element node: 3D orders with at most 1024 nodes (N <= 9)");
                return SEL_EUNSUPPORTED;
            }
            if (int rc = tic(s, kind, ev)) return rc;
            hipLaunchKernelGGL((k_stage_big<N, Q, T, DEV, MODE>), grid, dim3(BigGeo<N>::BLOCK), 0, s->stream, A);
        } else {
            if (int rc = tic(s, kind, ev)) return rc;
            // element contributions under the discontinuous coupling carry the
            // interface flux themselves; in the stages it is added by the
            // assembly (k_group_split), where every element-boundary node is a group
            bool dg = false;
            if constexpr (MODE == M_LOCAL) {
                dg = A.nbr != nullptr;
                if (dg) {
                    hipLaunchKernelGGL((k_stage<DIM, N, Q, T, DEV, MODE, true>), grid, block, 0, s->stream, A);
                }
            }
            if (!dg) {
                // FP32 3D order 7, later stages: vector loads and matrix-core contractions
                if constexpr (kMfma && MODE == M_STAGE23) {
                    hipLaunchKernelGGL((k_stage23_mf<Q>), grid, block, 0, s->stream, A);
                } else {
                    hipLaunchKernelGGL((k_stage<DIM, N, Q, T, DEV, MODE>), grid, block, 0, s->stream, A);
                }
            }
        }
        SEL_LAUNCH_CHECK();
        return toc(s, ev);
    }

    static int launch_group(sel_sim *s, const GroupArgs<T> &B)
    {
        if (s->ngrp == 0) return SEL_OK;
        dim3 block(256);
        hipEvent_t ev = nullptr;
        if (int rc = tic(s, 2, ev)) return rc;
        // the discontinuous coupling adds its interface flux here
        // 128 groups per workgroup, two wavefronts per group
        dim3 grid2((unsigned)xcd_grid((s->ngrp + 127) / 128));
        if (B.nbr) {
            hipLaunchKernelGGL((k_group_split<Q, T, N>), grid2, block, 0, s->stream, B);
        } else {
            hipLaunchKernelGGL((k_group_split<Q, T>), grid2, block, 0, s->stream, B);
        }
        SEL_LAUNCH_CHECK();
        return toc(s, ev);
    }

    static int geometry(sel_sim *s)
    {
        const int64_t nb = nblk(s);
        if constexpr (kBig) {
            hipLaunchKernelGGL((k_geom_big<N, T>), dim3((unsigned)nb), dim3(BigGeo<N>::BLOCK), 0, s->stream, s->xyz,
                               s->geoD, s->geoW, s->wJ, s->J, static_cast<T *>(s->Gm), s->flag, s->E);
        } else {
            hipLaunchKernelGGL((k_geom<DIM, N, T>), dim3((unsigned)nb), dim3(GG::BLOCK), 0, s->stream, s->xyz,
                               s->geoD, s->geoW, s->wJ, s->J, static_cast<T *>(s->Gm), s->flag, s->E, nb);
        }
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    static int mass(sel_sim *s)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_mass_int<T>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s->stream, s->wJ,
                           s->pcode, static_cast<T *>(s->invw), s->E, NP, NI);
        SEL_LAUNCH_CHECK();
        if (s->ngrp > 0) {
            hipLaunchKernelGGL((k_mass_grp<T>), dim3((unsigned)((s->ngrp + 255) / 256)), dim3(256), 0, s->stream,
                               s->wJ, s->bpos, s->goff, s->gmem, static_cast<T *>(s->invMb), s->ngrp, NP, NB);
            SEL_LAUNCH_CHECK();
        }
        return SEL_OK;
    }

    static int init(sel_sim *s, const double *d_rho, const double *d_u)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_init<DIM, Q, T, DEV>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s->stream,
                           nodemap(s), d_rho, d_u, st(s, s->cur), s->p.rho0, s->p.dt, s->p.accel[0],
                           s->p.accel[1], DIM == 3 ? s->p.accel[2] : 0.0);
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    // one time step: collide (and filter the previous step's result) ->
    // SSPRK3 streaming with F* and the wall flux; the filter of this step is
    // applied by the next step's first stage, or at the end of the call.
    // per-node force density (added to rho g): fill from FP64 [E][np][dim]
    static int set_force(sel_sim *s, const double *d_F)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_force_set<T>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s->stream, nodemap(s),
                           d_F, DIM, static_cast<T *>(s->Fn));
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    // its F** part on the post-collision state f
    static int force_collide(sel_sim *s, T *f, const float *dtau)
    {
        hipLaunchKernelGGL((k_force_collide<DIM, Q, T, DEV>), dim3((unsigned)((s->Gtot + 255) / 256)), dim3(256), 0,
                           s->stream, f, static_cast<const T *>(s->Fn), dtau, s->Gtot, s->Gi, NI, (int64_t)Q * s->Gi,
                           T(s->tau), T(s->p.dt), T(s->p.rho0));
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    // its F* part of a stage: out += cc F*(F_n)
    static int force_stage(sel_sim *s, T *out, double cc)
    {
        hipLaunchKernelGGL((k_force_stage<DIM, Q, T>), dim3((unsigned)((s->Gtot + 255) / 256)), dim3(256), 0,
                           s->stream, out, static_cast<const T *>(s->Fn), s->Gtot, s->Gi, NI, (int64_t)Q * s->Gi,
                           T(cc));
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    // One element pass and its assembly: out = ca f0 + cb fk + cc L(fk).
    static int stage_pass(sel_sim *s, StageArgs<T> &A, GroupArgs<T> &B, const T *fk, const T *f0, T *out,
                          double ca, double cb, double cc)
    {
        A.op = fk;
        A.f0in = f0;
        A.out = out;
        A.ca = T(ca);
        A.cb = T(cb);
        A.cc = T(cc);
        if (int rc = launch_stage<M_STAGE23>(s, A)) return rc;
        B.f0 = f0;
        B.fk = fk;
        B.out = out;
        B.ca = T(ca);
        B.cb = T(cb);
        B.cc = T(cc);
        if (int rc = launch_group(s, B)) return rc;
        return s->force_on ? force_stage(s, out, cc) : SEL_OK;
    }

    // First stage: filter (when pending) and collide the state S into the
    // post-collision state y = F0, then FA = y + cc L(y). The continuous
    // coupling streams in the same kernel (a shared node's post-collision
    // value is the same in every element); the discontinuous coupling needs
    // the post-collision values across faces, and a per-node force adds its
    // F** part to y first, so both stream in a second pass.
    static int stage_one(sel_sim *s, StageArgs<T> &A, GroupArgs<T> &B, const T *S, T *F0, T *FA, double cc,
                         bool pending)
    {
        A.op = S;
        A.f0out = F0;
        A.out = FA;
        A.ca = T(0);
        A.cb = T(1);
        A.cc = T(cc);
        A.filter = pending ? 1 : 0;
        if (s->nbr || s->force_on) {
            A.collide_only = 1;
            const int rc = launch_stage<M_STAGE1>(s, A);
            A.collide_only = 0;
            if (rc) return rc;
            if (s->force_on) {
                if (int rc2 = force_collide(s, F0, A.dtau)) return rc2;
            }
            return stage_pass(s, A, B, F0, F0, FA, 0.0, 1.0, cc);
        }
        if (int rc = launch_stage<M_STAGE1>(s, A)) return rc;
        B.f0 = F0;
        B.fk = F0;
        B.out = FA;
        B.ca = T(0);
        B.cb = T(1);
        B.cc = T(cc);
        return launch_group(s, B);
    }

    // The four printed stage formulas of Sec. 2.2.2 with L applied linearly
    // to their combinations (stage values w1..w3, y the post-collision state):
    //   w1 = y + dt/3 L(y)
    //   w2 = w1 - 3dt/4 (L(y) - L(w1))
    //   w3 = w2 + 2dt/3 (L(y) - L(w1) + L(w2))
    //   y' = w3 - dt/4 (L(y) - L(w1) + L(w2) - L(w3)).
    // Each earlier L is eliminated through the stage that defines it, so every
    // stage is a two-state combination ca f0 + cb fk + cc L(fk) with
    // ca + cb = 1 (exact in exact arithmetic, also for an affine L):
    //   w2 = 9/4 y - 5/4 w1 + 3dt/4 L(w1)
    //   w3 = 8/9 w1 + 1/9 w2 + 2dt/3 L(w2)
    //   y' = 3/8 w2 + 5/8 w3 + dt/4 L(w3).
    // Arrays: S holds the state and then y'; F0 holds y and then w3; FA w1;
    // FB w2.
    static int printed4(sel_sim *s, StageArgs<T> &A, GroupArgs<T> &B, T *S, T *FB, T *F0, T *FA, bool pending)
    {
        const double dt = s->p.dt;
        if (int rc = stage_one(s, A, B, S, F0, FA, dt / 3.0, pending)) return rc;
        if (int rc = stage_pass(s, A, B, FA, F0, FB, 9.0 / 4.0, -5.0 / 4.0, 0.75 * dt)) return rc;
        if (int rc = stage_pass(s, A, B, FB, FA, F0, 8.0 / 9.0, 1.0 / 9.0, 2.0 / 3.0 * dt)) return rc;
        return stage_pass(s, A, B, F0, FB, S, 3.0 / 8.0, 5.0 / 8.0, 0.25 * dt);
    }

    static int step(sel_sim *s, int64_t nsteps)
    {
        if (nsteps <= 0) return SEL_OK;
        const double dt = s->p.dt;
        const bool filt = s->p.filter_type != SEL_FILTER_NONE;
        StageArgs<T> A = stage_args(s);
        GroupArgs<T> B = group_args(s);
        A.incr = 1;  // SSPRK weights sum to one
        B.incr = 1;
        T *F0 = st(s, 2), *FA = st(s, 3);
        bool pending = false;
        for (int64_t n = 0; n < nsteps; ++n) {
            if (s->closure_on) {
                // the closure reads the filtered state: its features come from
                // the filtered moment fields (the filter itself stays fused
                // into the first stage); then the network infers the
                // per-node relaxation-time increments
                hipEvent_t ev = nullptr;
                if (int rc = tic(s, 4, ev)) return rc;
                if (int rc = features(s, s->cl_X, 1, pending ? 1 : 0)) return rc;
                if (int rc = toc(s, ev)) return rc;
                if (int rc = tic(s, 5, ev)) return rc;
                if (int rc = launch_mlp_infer(s)) return rc;
                if (int rc = toc(s, ev)) return rc;
                A.dtau = s->cl_dtau;
            } else {
                A.dtau = nullptr;
            }
            T *S = st(s, s->cur), *FB = st(s, s->cur ^ 1);
            if (s->p.rk == SEL_RK_PRINTED4) {
                if (int rc = printed4(s, A, B, S, FB, F0, FA, pending)) return rc;
                pending = filt;
                s->time += dt;
                s->nstep += 1;
                continue;
            }
            // stage 1: f1 = f0 + dt L(f0), f0 = collide(filter(f3_prev) or f-bar)
            if (int rc = stage_one(s, A, B, S, F0, FA, dt, pending)) return rc;
            // stage 2: f2 = 3/4 f0 + 1/4 (f1 + dt L(f1))
            if (int rc = stage_pass(s, A, B, FA, F0, FB, 0.75, 0.25, 0.25 * dt)) return rc;
            // stage 3: f3 = 1/3 f0 + 2/3 (f2 + dt L(f2)), written over the state
            if (int rc = stage_pass(s, A, B, FB, F0, S, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt)) return rc;
            pending = filt;
            s->time += dt;
            s->nstep += 1;
        }
        if (pending) {
            A.op = st(s, s->cur);
            A.out = st(s, s->cur ^ 1);
            if (int rc = launch_stage<M_FILTER>(s, A)) return rc;
            s->cur ^= 1;
        }
        return SEL_OK;
    }

    static int moments(sel_sim *s, double *d_rho, double *d_u)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_moments<DIM, Q, T, DEV>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s->stream,
                           nodemap(s), st(s, s->cur), s->p.rho0, d_rho, d_u);
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    static int reduce(sel_sim *s)
    {
        hipLaunchKernelGGL((k_reduce<DIM, Q, T, DEV>), dim3(s->nred), dim3(256), 0, s->stream, nodemap(s),
                           st(s, s->cur), s->nstate, s->wJ, s->p.rho0, s->red);
        SEL_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_reduce_final<T>), dim3(1), dim3(64), 0, s->stream, s->red, s->nred, s->red + 8 * s->nred);
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    static int scatter(sel_sim *s, int a, const double *d_plane, void *dst, bool sub)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_scatter_plane<T>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s->stream,
                           nodemap(s), d_plane, static_cast<T *>(dst), a, sub ? s->toff[a] : 0.0);
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    static int gather(sel_sim *s, int a, const void *src, double *d_plane, bool add)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_gather_plane<T>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s->stream,
                           nodemap(s), static_cast<const T *>(src), d_plane, a, add ? s->toff[a] : 0.0);
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    // operator pieces on a state in src (scratch arrays only)
    static int apply(sel_sim *s, int op, void *src_v, void *dst_v, void *local_v)
    {
        T *src = static_cast<T *>(src_v), *dst = static_cast<T *>(dst_v);
        StageArgs<T> A = stage_args(s);
        A.op = src;
        if (op == SEL_OP_RHS || op == SEL_OP_RHS_LOCAL) {
            for (int a = 0; a < Q; ++a) A.fsc[a] = T(0);
            if (hipMemsetAsync(s->rhoc, 0, sizeof(T) * s->Gtot, s->stream) != hipSuccess) return SEL_EDEVICE;
            if (op == SEL_OP_RHS_LOCAL) {
                A.local = static_cast<T *>(local_v);
                return launch_stage<M_LOCAL>(s, A);
            }
            A.f0in = src;
            A.out = dst;
            A.ca = T(0);
            A.cb = T(0);
            A.cc = T(1);
            if (int rc = launch_stage<M_STAGE23>(s, A)) return rc;
            GroupArgs<T> B = group_args(s);
            for (int a = 0; a < Q; ++a) B.fsc[a] = T(0);
            B.f0 = src;
            B.fk = src;
            B.out = dst;
            B.ca = T(0);
            B.cb = T(0);
            B.cc = T(1);
            return launch_group(s, B);
        }
        if (op == SEL_OP_COLLIDE) {
            A.f0out = dst;
            A.out = st(s, s->cur ^ 1);
            A.filter = 0;
            A.ca = A.cb = A.cc = T(0);
            return launch_stage<M_STAGE1>(s, A);
        }
        if (op == SEL_OP_FILTER) {
            A.out = dst;
            return launch_stage<M_FILTER>(s, A);
        }
        return SEL_EINVAL;
    }

    // closure features of the current state: one row per node id
    // (owner_out = 1) or per element node
    static int features(sel_sim *s, float *X, int owner_out, int filter) { return feat(s, X, owner_out, filter, nullptr, 0); }

    // row c of the velocity gradient of the current state, du_c/dx_q per
    // element node [E][np][dim] (FP64, device)
    static int grad_row(sel_sim *s, int c, double *d_out) { return feat(s, nullptr, 0, 0, d_out, c); }

    static int feat(sel_sim *s, float *X, int owner_out, int filter, double *grad, int row)
    {
        if constexpr (kBig) {
            set_error("closure features and velocity gradients take one thread per element node: 3D orders with at most 1024 nodes (N <= 9)");
            return SEL_EUNSUPPORTED;
        } else {
            return feat_launch(s, X, owner_out, filter, grad, row);
        }
    }

    static int feat_launch(sel_sim *s, float *X, int owner_out, int filter, double *grad, int row)
    {
        FeatArgs<T> F{};
        F.grad = grad;
        F.grad_row = row;
        F.f = st(s, s->cur);
        F.F = static_cast<const T *>(s->tabF);
        F.filter = filter;
        F.Gm = static_cast<const T *>(s->Gm);
        F.D = static_cast<const T *>(s->tabD);
        F.wJ = s->wJ;
        F.pcode = s->pcode;
        F.bmap = s->bmap;
        F.bown = s->bown;
        F.X = X;
        F.E = s->E;
        F.nblk = nblk(s);
        F.Gi = s->Gi;
        F.QGi = (int64_t)Q * s->Gi;
        F.rho0 = T(s->p.rho0);
        F.lam = T(s->p.nu * 3.0);
        F.owner_out = owner_out;
        if (grad) {
            hipLaunchKernelGGL((k_features<DIM, N, Q, T, DEV, true>), dim3((unsigned)F.nblk), dim3(GG::BLOCK), 0,
                               s->stream, F);
        } else {
            hipLaunchKernelGGL((k_features<DIM, N, Q, T, DEV>), dim3((unsigned)F.nblk), dim3(GG::BLOCK), 0, s->stream,
                               F);
        }
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    // wJ (u . n) and wJ at every element node, FP64 [2][E][np] (device)
    static int axial_terms(sel_sim *s, const double *n, double *d_out)
    {
        const int64_t nl = s->E * NP;
        hipLaunchKernelGGL((k_axial_terms<DIM, Q, T, DEV>), dim3((unsigned)((nl + 255) / 256)), dim3(256), 0,
                           s->stream, nodemap(s), st(s, s->cur), s->wJ, s->p.rho0, n[0], n[1], DIM == 3 ? n[2] : 0.0,
                           d_out);
        SEL_LAUNCH_CHECK();
        return SEL_OK;
    }

    static const Ops *ops()
    {
        static const Ops o = {geometry, mass, init,    step,     moments,  reduce,   scatter,
                              gather,   apply, features, set_force, grad_row, axial_terms};
        return &o;
    }
};

}  // namespace sel
