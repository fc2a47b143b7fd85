// Per-configuration launch table of the SELBM kernels.
#pragma once

#include "sel_internal.h"

namespace sel {

struct Ops {
    int (*geometry)(sel_sim *);
    int (*mass)(sel_sim *);
    int (*init)(sel_sim *, const double *, const double *);
    int (*step)(sel_sim *, int64_t);
    int (*moments)(sel_sim *, double *, double *);
    int (*reduce)(sel_sim *);
    int (*scatter)(sel_sim *, int, const double *, void *, bool);
    int (*gather)(sel_sim *, int, const void *, double *, bool);
    int (*apply)(sel_sim *, int, void *, void *, void *);
    int (*features)(sel_sim *, float *, int owner_out, int filter);
    int (*set_force)(sel_sim *, const double *d_F);  // d_F: device FP64 [E][np][dim]
    int (*grad_row)(sel_sim *, int c, double *d_out);  // du_c/dx_q, FP64 [E][np][dim]
    int (*axial_terms)(sel_sim *, const double *n, double *d_out);  // wJ u.n and wJ, FP64 [2][E][np]
};

// learned-closure inference on the simulation's feature rows (closure.hip)
int launch_mlp_infer(sel_sim *s);

// one table per compiled (dim, N, Q, storage); nullptr if not compiled
const Ops *ops_d2_fp64(int N);
const Ops *ops_d2_fp32(int N);
const Ops *ops_d3q27_fp64(int N);
const Ops *ops_d3q27_fp32(int N);
const Ops *ops_d3q19_fp64(int N);
const Ops *ops_d3q19_fp32(int N);

inline const Ops *find_ops(int dim, int N, int Q, int prec)
{
    const bool f32 = prec == SEL_FP32_DEV;
    if (dim == 2 && Q == 9) return f32 ? ops_d2_fp32(N) : ops_d2_fp64(N);
    if (dim == 3 && Q == 27) return f32 ? ops_d3q27_fp32(N) : ops_d3q27_fp64(N);
    if (dim == 3 && Q == 19) return f32 ? ops_d3q19_fp32(N) : ops_d3q19_fp64(N);
    return nullptr;
}

}  // namespace sel
