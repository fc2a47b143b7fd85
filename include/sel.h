/*
 * sel.h -- C interface of the MI355X (gfx950) filtered spectral-element
 * lattice Boltzmann (SELBM) library with flux bounce-back walls
 * (Zhao, Patel, Lin, Min & Lee, arXiv:2509.19171).
 *
 * One call of sel_step advances the discrete Boltzmann equation (Sec. 2.1,
 * Eq. dbe_m) by whole time steps in the order of the scheme summary at the
 * end of Sec. 2.2: BGK collision with the higher-order force F** (Sec. 2.1),
 * streaming as a Galerkin spectral-element advection solved by SSP
 * Runge-Kutta with the leading-order force F* and the flux bounce-back wall
 * flux (Sec. 2.2, 2.2.1, 2.2.2), then the explicit modal filter (Sec. 2.2.3).
 *
 * Conventions (all arrays row-major, host memory unless stated):
 *   dim 2 or 3; order N; np = (N+1)^dim nodes per element; node index
 *   p = i + (N+1) j + (N+1)^2 k with the first reference direction r fastest
 *   (Sec. 2.2, lumped mass index).
 *   xyz  [E][np][dim]  GLL node coordinates of the isoparametric map.
 *   gid  [E][np]       global node id in [0, E*np); every copy of a node shared
 *                      by several elements (periodic copies included) has the
 *                      same id. Only nodes on element faces may be shared.
 *   face_tag [E][2*dim] faces ordered (r-, r+, s-, s+, t-, t+): 0 = interior or
 *                      periodic, k >= 1 = wall k with velocity wall_u[k-1].
 *   wall_u [ntags][dim] wall velocities u_b of the bounce-back jump.
 *   rho [E][np], u [E][np][dim], f [E][Q][np]: FP64, full distribution f
 *                      (the FP32 deviation form converts inside).
 *   Velocities: a = a0 + 3 a1 (+ 9 a2) with component values {0, +1, -1}[a_i];
 *   D2Q9 (dim 2), D3Q27 and D3Q19 (the D3Q27 entries with |e|^2 <= 2, same
 *   order). Lattice units: particle speed 1, c_s^2 = 1/3.
 *
 * Errors: every call returns SEL_OK (0) or a negative SEL_E* code and never
 * aborts; out-parameters are written only on success; sel_last_error() gives
 * a thread-local message for the last failing call of the thread.
 * Device work is enqueued on the caller's HIP stream; device faults and
 * non-finite states surface at the next synchronising call.
 */
#ifndef SEL_H
#define SEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEL_OK 0
#define SEL_EINVAL (-1)      /* invalid argument, mesh or parameter */
#define SEL_ENOMEM (-2)      /* host or device allocation failed, workspace too small */
#define SEL_EDEVICE (-3)     /* HIP runtime or kernel launch error */
#define SEL_ENONFINITE (-4)  /* the state holds NaN or Inf */
#define SEL_ESTATE (-5)      /* call not valid in the current state */
#define SEL_EUNSUPPORTED (-6) /* valid but not built (order, lattice, form) */

/* storage and arithmetic of the distribution */
#define SEL_FP64 0      /* f in FP64 */
#define SEL_FP32_DEV 1  /* g = f - t_a rho0 stored and streamed in FP32; geometry set up in FP64 */

/* filter transfer functions (Sec. 2.2.3) */
#define SEL_FILTER_NONE 0
#define SEL_FILTER_QUAD 1 /* sigma_k = 1 - amp ((k - kc)/(N - kc))^2, k > kc */
#define SEL_FILTER_EXP 2  /* sigma_k = exp(-amp ((k - kc)/(N - kc))^order), k > kc */

/* time marching (Sec. 2.2.2) */
#define SEL_RK_SSP3 0     /* Shu-Osher SSPRK3 */
#define SEL_RK_PRINTED4 1 /* the four printed stage formulas, L applied linearly */

typedef struct sel_mesh sel_mesh;
typedef struct sel_sim sel_sim;

/* Physical and numerical parameters.
 *   nu = lambda c_s^2 and tau = lambda / dt (Sec. 2.1); dt is stored as given.
 *   accel: body acceleration g, force density F = rho g (Sec. 2.1, Eqs. body
 *   and f_c; Sec. 3.5 drives the pipe with (0, 0, rho g)).
 *   closure / closure_len: host pointer to the FP32 parameter blob of the
 *   learned relaxation-time closure (layout below, closure_len must equal
 *   sel_closure_len()) or NULL. With a blob, every step first evaluates the
 *   closure on the current state and relaxes each node with
 *   omega = 1 / (tau + dtau + 1/2). */
typedef struct sel_params {
    int32_t Q;           /* 9 (dim 2), 19 or 27 (dim 3) */
    int32_t precision;   /* SEL_FP64 or SEL_FP32_DEV */
    int32_t rk;          /* SEL_RK_* */
    int32_t filter_type; /* SEL_FILTER_* */
    int32_t filter_kc;   /* cut-off mode k_c, 0 <= kc < N */
    int32_t reserved0;
    double filter_amp;   /* gamma (quadratic) or alpha (exponential) */
    double filter_order; /* exponent of the exponential filter */
    double rho0;         /* reference density of the wall term and the deviation form */
    double nu;           /* kinematic viscosity > 0 */
    double dt;           /* time step > 0 */
    double accel[3];     /* body acceleration g (entries beyond dim ignored) */
    const float *closure;
    int64_t closure_len;
} sel_params;

/* Mesh ingest: the unstructured quadrilateral/hexahedral mesh of order N of
 * Sec. 2.2 (isoparametric elements, GLL nodes, lumped mass) with the wall
 * faces of the flux bounce-back condition (Sec. 2.2.1). Copies every array
 * (the caller keeps ownership) and checks: dim in {2,3}; supported N; E >= 1;
 * gid in [0, E*np); nodes off the element faces are not shared; face_tag in
 * [0, ntags]; 0 <= ntags <= 127; wall_u given when ntags > 0; and the
 * geometric consistency of the numbering:
 *   - a wall face shares none of its nodes off its edges (it lies on the
 *     domain boundary);
 *   - the nodes of any other face off its edges are either all unshared or
 *     all shared with exactly one other copy, in one element, displaced by
 *     one constant vector (zero, or a periodic translation);
 *   - every copy of a shared node coincides with its first copy up to a sum
 *     of at most dim of those translations (periodic edges and corners);
 *   distances below 1e-9 of the mesh extent count as zero.
 * Element geometry (Jacobian > 0) is checked by sel_init on the device.
 * Returns SEL_EINVAL (with a message naming the failed check),
 * SEL_EUNSUPPORTED or SEL_ENOMEM on failure. */
int sel_mesh_create(int32_t dim, int32_t N, int64_t E, const double *xyz, const int64_t *gid,
                    const int32_t *face_tag, int32_t ntags, const double *wall_u, sel_mesh **out);

/* Discontinuous-Galerkin coupling of the elements (the alternative to the
 * continuous method that the paper's introduction discusses): same
 * arguments and checks as sel_mesh_create, but no node is shared. Every
 * element keeps its own copy of its face nodes with its own lumped mass wJ,
 * gid only identifies the coincident node across each face, and every face
 * that is not a wall adds the upwind flux of the velocities entering the
 * element, (n.e_a) w_s J_s (f_a - f_a^across) for n.e_a < 0 (wall faces keep
 * the FBB term of Sec. 2.2.1). Initial rho and u may differ between copies.
 * Extra errors (SEL_EINVAL): a face that is not a wall must share its set of
 * node ids with exactly one other face, and no face may repeat a node id
 * (one element along a periodic direction). */
int sel_mesh_create_dg(int32_t dim, int32_t N, int64_t E, const double *xyz, const int64_t *gid,
                       const int32_t *face_tag, int32_t ntags, const double *wall_u, sel_mesh **out);
int sel_mesh_destroy(sel_mesh *mesh);

/* info[0..7] = dim, N, E, np, unique nodes, shared-node groups on element
 * boundaries, element-boundary nodes per element, wall faces. */
int sel_mesh_info(const sel_mesh *mesh, int64_t *info);

/* Bytes of device workspace sel_init needs for this mesh and parameters. */
int sel_workspace_bytes(const sel_mesh *mesh, const sel_params *p, size_t *bytes);

/* Create a simulation and set f-bar = f^eq(rho, u) - dt F** / 2 (Sec. 2.1
 * with f = f^eq). rho [E][np] and u [E][np][dim] are FP64 host arrays (shared
 * copies must carry equal values). dev_ws is device memory of at least
 * sel_workspace_bytes bytes owned by the caller, who keeps it alive until
 * sel_destroy; NULL makes the library allocate it. hip_stream is a
 * hipStream_t (NULL = default stream). The mesh may be destroyed after this
 * call. Errors: SEL_EINVAL (bad parameter or non-positive Jacobian),
 * SEL_ENOMEM, SEL_EDEVICE, SEL_EUNSUPPORTED (an order, lattice or storage
 * form not built: D2Q9 N 2..10; D3Q19 and D3Q27 N 2..8; D3Q19 N 12, the
 * highest Taylor-Green order of Sec. 3.4, which runs the continuous coupling
 * without the closure and without sel_velocity_gradient). */
int sel_init(const sel_mesh *mesh, const sel_params *p, const double *rho, const double *u,
             void *dev_ws, size_t ws_bytes, void *hip_stream, sel_sim **out);

/* Enqueue nsteps >= 0 whole time steps on the simulation's stream
 * (asynchronous). One step, in the order of the scheme summary at the end of
 * Sec. 2.2: BGK collision with F** (Sec. 2.1, Eqs. perfect1-perfect2), the
 * streaming operator with F* and the wall flux integrated over dt by the
 * chosen Runge-Kutta form (Sec. 2.2, 2.2.1, 2.2.2), then the modal filter
 * (Sec. 2.2.3; applied lazily: fused into the next step's first stage, or
 * run at the end of the call, so the state seen after the call is filtered).
 * Errors: SEL_EINVAL (null sim or nsteps < 0), SEL_EDEVICE (launch failure);
 * device faults and non-finite states surface at the next synchronising call. */
int sel_step(sel_sim *sim, int64_t nsteps);

/* Same as sel_step, with HIP events recorded on the stream around every
 * kernel launch. On return (it synchronises) ms[k] holds the summed device
 * time and launches[k] the number of launches of kernel kind k:
 *   0 first-stage element kernel (filter of the previous step, collision,
 *     streaming operator), 1 later-stage element kernel (streaming operator),
 *   2 shared-node assembly, 3 end-of-call filter, 4 closure features,
 *   5 closure network (both only with a closure attached). ms and launches
 *   hold SEL_NKIND entries. */
#define SEL_NKIND 6
int sel_step_timed(sel_sim *sim, int64_t nsteps, double *ms, int64_t *launches);

/* Synchronise the stream; SEL_ENONFINITE if the state holds NaN or Inf. */
int sel_sync(sel_sim *sim);

/* Density and velocity of the current f-bar (Eqs. pressure, momentum):
 * rho [E][np], u [E][np][dim], FP64 host arrays. Synchronises. */
int sel_moments(sel_sim *sim, double *rho, double *u);

/* Same on device: d_rho [E][np], d_u [E][np][dim] FP64 device arrays,
 * enqueued on the stream, no synchronisation. */
int sel_moments_device(sel_sim *sim, double *d_rho, double *d_u);

/* FP64 integrals with the lumped mass: out[0] = sum wJ rho,
 * out[1..dim] = sum wJ rho u, out[dim+1] = sum wJ rho0 |u|^2 / 2 (kinetic
 * energy as in Sec. 3.4), out[dim+2] = number of non-finite f entries.
 * Synchronises. */
int sel_reduce(sel_sim *sim, double *out);

/* Checkpoint access: f [E][Q][np] FP64 full distribution (host). set_f takes
 * the value of the lowest-numbered copy of each shared node. Synchronise. */
int sel_get_f(sel_sim *sim, double *f);
int sel_set_f(sel_sim *sim, const double *f);

/* Force density per node added to the body force: F = rho g + F_n (Sec. 2.1;
 * the pipe case of Sec. 3.5 adds a perturbation force of this kind). F is a
 * host array [E][np][dim] (FP64); the copies of a shared node must carry
 * equal values under the continuous coupling (the owning copy is used).
 * Like rho g it is taken at the collision of every following step and frozen
 * for its stages; the current state is not changed, and a time-dependent
 * force is set again between calls of sel_step. NULL removes it. Errors:
 * SEL_EINVAL (null sim or a non-finite entry). Synchronises. */
int sel_set_force(sel_sim *sim, const double *F);

/* Velocity gradient of the current state at every element node:
 * grad [E][np][dim][dim] (FP64 host), grad[..][c][q] = du_c/dx_q, from the
 * element-local derivative with the metric of Sec. 2.2 (u = sum e f / rho,
 * Eq. momentum). Gives the wall shear stress of Sec. 3.5 and the dissipation
 * rate of Sec. 3.4. Synchronises. */
int sel_velocity_gradient(sel_sim *sim, double *grad);

/* Radial profile of the velocity along an axis (the averaged streamwise
 * profile u_z(r) of the pipe case, Sec. 3.5): with the unit axis n through
 * origin (both [dim], FP64 host; axis need not be normalised) and the radial
 * distance r of an element node from that line, the element nodes with
 * r < rmax fall into nbins equal bins of [0, rmax). out [2 nbins] (FP64 host)
 * receives per bin sum wJ (u . n) in out[b] and sum wJ in out[nbins + b]
 * (lumped-mass integrals over the bin's nodes, u = sum e f / rho of
 * Eq. momentum), so out[b] / out[nbins + b] is the bin's space-averaged axial
 * velocity (time averages are sums of calls). In 2D the line is the line
 * through origin along axis (a channel profile). Deterministic: each bin is
 * summed in ascending node order. The first call for a binning allocates its
 * node lists on the device (kept until the binning changes or sel_destroy).
 * Errors: SEL_EINVAL (bad argument, 1 <= nbins <= 4096, rmax > 0),
 * SEL_ENOMEM, SEL_EDEVICE. Synchronises. */
int sel_radial_profile(sel_sim *sim, const double *origin, const double *axis, double rmax, int32_t nbins,
                       double *out);

/* Simulated time and step count. */
int sel_get_time(const sel_sim *sim, double *t, int64_t *nstep);

/* Operator pieces on a host state f [E][Q][np] (FP64 in and out), for
 * checking the kernels one by one. Synchronises.
 *   SEL_OP_RHS:       M^-1 (R(n.j) - C_a f) after assembly (Sec. 2.2, 2.2.1), no F*
 *   SEL_OP_RHS_LOCAL: element contributions R(n.j) - C_a f before assembly
 *   SEL_OP_COLLIDE:   post-collision f* (Sec. 2.1)
 *   SEL_OP_FILTER:    filtered f (Sec. 2.2.3) */
#define SEL_OP_RHS 0
#define SEL_OP_RHS_LOCAL 1
#define SEL_OP_COLLIDE 2
#define SEL_OP_FILTER 3
int sel_apply(sel_sim *sim, int32_t op, const double *fin, double *fout);

/* Geometry computed on the device: wJ [E][np], J [E][np] (FP64 host). */
int sel_geometry(sel_sim *sim, double *wJ, double *J);

/* The hipStream_t the simulation enqueues its work on. */
void *sel_stream(const sel_sim *sim);

int sel_destroy(sel_sim *sim);

/* ---- learned relaxation-time closure ----------------------------------
 * Not part of the paper's method (it has none): a per-node MLP that maps
 * local invariants of the state to an increment dtau >= 0 of the BGK
 * relaxation time (Sec. 2.1) for under-resolved runs.
 *
 * Features per node (FP32), from f-bar of Sec. 2.1 with u = sum e f / rho,
 * A = grad u from the element-local derivative (Sec. 2.2), S and W its
 * symmetric and antisymmetric parts, Pi = sum_a e e (f_a - f_a^eq),
 * lam = nu / c_s^2:
 *   x = [lam^2 S:S, lam^2 W:W, lam^3 tr(S^3), lam^3 tr(S W W),
 *        Pi:Pi / (rho c_s^2)^2, lam Pi:S / (rho c_s^2)].
 * Network: x' = (x - mean) / std, h1 = tanh(W1 x' + b1), h2 = tanh(W2 h1 + b2),
 * h3 = tanh(W3 h2 + b3), z = w4 . h3 + b4 (6 -> 64 -> 64 -> 64 -> 1),
 * dtau = tau softplus(z); a non-finite value, a negative one or one above
 * dtau_max * tau is replaced by 0 (the plain method).
 * Blob (FP32, this order): mean[6], std[6], W1[64][6], b1[64], W2[64][64],
 * b2[64], W3[64][64], b3[64], w4[64], b4, dtau_max. The trainable
 * parameters are the contiguous range W1 .. b4 (8833 values) starting at
 * float offset 12. */

/* Number of floats in the blob (8846). */
int64_t sel_closure_len(void);

/* Replace the blob of a simulation created with one (host pointer, len =
 * sel_closure_len()); NULL switches the closure off (plain method) until the
 * next call with a blob. Synchronises. SEL_ESTATE if the simulation was
 * created without a blob. */
int sel_closure_set(sel_sim *sim, const float *params, int64_t len);

/* Features of the current state, d_X [E][np][6] FP32 device array (every
 * element copy of a node), enqueued on the stream. */
int sel_closure_features(sel_sim *sim, float *d_X);

/* Increments the next step would use, d_dtau [number of unique nodes] FP32
 * device array in the library's node-id order (diagnostics). */
int sel_closure_dtau(sel_sim *sim, float *d_dtau);

/* Coarse graining of a fine simulation onto a coarse one over the same
 * elements (same dim, lattice, storage, E; coarse N <= fine N): each
 * distribution is projected element by element onto the modes k <= N_c of the
 * basis phi_0 = L_0, phi_1 = L_1, phi_k = L_k - L_{k-2} (the filter basis of
 * Sec. 2.2.3) and evaluated at the coarse GLL nodes; shared coarse nodes take
 * the lowest-numbered element's value. Overwrites the coarse state (time and
 * step count unchanged). Synchronises both streams. */
int sel_coarse_grain(const sel_sim *fine, sel_sim *coarse);

/* Training targets, d_y [E][np_coarse] FP32 device array (the element's
 * value on each of its nodes, row-aligned with sel_closure_features):
 * u-bar = P(u), tau_sgs = P(u u) - u-bar u-bar with P the projection above,
 * S-bar the strain rate of u-bar on the coarse element,
 * nu_t = max(0, -<dev tau_sgs : S-bar> / <2 S-bar : S-bar>) with wJ-weighted
 * element sums, dtau* = nu_t / (c_s^2 dt_coarse) and y = dtau* / tau_coarse
 * (the target of softplus(z)). Synchronises. */
int sel_closure_targets(const sel_sim *fine, sel_sim *coarse, float *d_y);

/* Inference on n feature rows d_X [n][6] (device): z [n] and dtau [n] (either
 * may be NULL) for relaxation time tau. Enqueued on stream (hipStream_t). */
int sel_mlp_forward(const float *d_params, const float *d_X, int64_t n, double tau, float *d_z,
                    float *d_dtau, void *stream);

/* Floats of device work memory sel_mlp_train_step / sel_mlp_gradient need
 * for n rows. */
int64_t sel_mlp_work_floats(int64_t n);

/* Loss L = mean_i (softplus(z_i) - y_i)^2 over n rows (targets y = dtau/tau)
 * and its gradient with respect to the trainable range, d_grad [8833].
 * Row i is row d_idx[i] of d_X [.][6] and d_y (d_idx: device int32 [n], or
 * NULL for rows 0..n-1; the caller keeps indices in range). The gradient
 * is summed over fixed chunks of consecutive rows (their size depends on n
 * only), then over the chunks in order, with no atomics: the same inputs give
 * the same result bit for bit. loss (host, may be NULL) synchronises. */
int sel_mlp_gradient(const float *d_params, const float *d_X, const float *d_y, const int32_t *d_idx, int64_t n,
                     float *d_work, float *d_grad, double *loss, void *stream);

/* One Adam step (Kingma and Ba, bias-corrected, step t >= 1) on the
 * trainable range of d_params with moment buffers d_m, d_v [8833]; loss as
 * for sel_mlp_gradient, evaluated before the update. */
int sel_mlp_train_step(float *d_params, float *d_m, float *d_v, const float *d_X, const float *d_y,
                       const int32_t *d_idx, int64_t n, int64_t t, double lr, double b1, double b2, double eps, float *d_work, double *loss,
                       void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * Adam step as sel_mlp_train_step, computed by the same kernels and with the
 * same result bit for bit, but its training work memory is a fixed device
 * array inside the library (8.75 MB per GPU, held until the process ends)
 * instead of a d_work argument. It allocates nothing. n is limited to 4096
 * rows (one minibatch of the training recipe); larger n returns SEL_EINVAL.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one
 * GPU (other streams or host threads) race and must be serialised by the
 * caller. Each call writes every work value it reads, so no clearing is
 * needed between calls. SEL_EDEVICE if the current device cannot be used. */
int sel_mlp_train_step_noalloc(float *d_params, float *d_m, float *d_v, const float *d_X, const float *d_y,
                               const int32_t *d_idx, int64_t n, int64_t t, double lr, double b1, double b2, double eps,
                               double *loss, void *stream);

/* Thread-local message of the last failing call ("" if none). */
const char *sel_last_error(void);

/* Library build string (target, compiled orders). */
const char *sel_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SEL_H */
