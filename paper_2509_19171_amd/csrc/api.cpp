// C interface of the SELBM library: workspace layout, set-up and the calls
// declared in sel.h. Every kernel launch goes through the per-configuration
// table of ops.h.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ops.h"

namespace sel {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

}  // namespace sel

using sel::set_error;

extern "C" const char *sel_last_error(void) { return sel::g_err.c_str(); }

extern "C" const char *sel_version(void)
{
    return "sel gfx950: dim 2 (D2Q9) N 2..10, dim 3 (D3Q27, D3Q19) N 2..8 and D3Q19 N 12; FP64 and FP32 deviation "
           "storage";
}

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
            return SEL_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

namespace {

constexpr size_t kAlign = 256;

struct Plan {
    size_t total = 0;
    size_t tabD, tabF, tabW, geoD, geoW, pcode, bpos, xyz, wJ, J, Gm, invw, invMb, bmap, bown, goff, gmem, ftag,
        wallu, f[4], rtb, rhoc, Fn, io, red, flag, posmap, hidx, nbr = 0, cl_params = 0, cl_X = 0, cl_dtau = 0;
    int nred = 0;
    bool closure = false;
};

size_t carve(size_t &cur, size_t bytes)
{
    cur = (cur + kAlign - 1) / kAlign * kAlign;
    size_t o = cur;
    cur += bytes;
    return o;
}

int check_params(const sel_mesh *m, const sel_params *p)
{
    if (!m || !p) {
        set_error("null mesh or params");
        return SEL_EINVAL;
    }
    if (!((m->dim == 2 && p->Q == 9) || (m->dim == 3 && (p->Q == 19 || p->Q == 27)))) {
        set_error("Q must be 9 in 2D, 19 or 27 in 3D");
        return SEL_EINVAL;
    }
    if (p->precision != SEL_FP64 && p->precision != SEL_FP32_DEV) {
        set_error("precision must be SEL_FP64 or SEL_FP32_DEV");
        return SEL_EINVAL;
    }
    if (!(p->nu > 0.0) || !(p->dt > 0.0) || !(p->rho0 > 0.0) || !std::isfinite(p->nu) || !std::isfinite(p->dt)) {
        set_error("nu, dt and rho0 must be positive and finite");
        return SEL_EINVAL;
    }
    if (p->filter_type < SEL_FILTER_NONE || p->filter_type > SEL_FILTER_EXP) {
        set_error("unknown filter type");
        return SEL_EINVAL;
    }
    if (p->filter_type != SEL_FILTER_NONE && (p->filter_kc < 0 || p->filter_kc >= m->N)) {
        set_error("filter_kc must be in [0, N)");
        return SEL_EINVAL;
    }
    if (p->rk != SEL_RK_SSP3 && p->rk != SEL_RK_PRINTED4) {
        set_error("unknown rk");
        return SEL_EINVAL;
    }
    if (p->closure != nullptr && p->closure_len != sel_closure_len()) {
        set_error("closure_len must equal sel_closure_len()");
        return SEL_EINVAL;
    }
    if (!sel::find_ops(m->dim, m->N, p->Q, p->precision)) {
        set_error("order N not compiled for this dim/Q/precision");
        return SEL_EUNSUPPORTED;
    }
    // elements with more nodes than a workgroup has threads (3D, N >= 10) run
    // the continuous coupling without the learned closure
    if (m->np > 1024 && (m->dg || p->closure != nullptr)) {
        set_error("the closure and the discontinuous coupling take one thread per element node: 3D orders with at most 1024 nodes (N <= 9)");
        return SEL_EUNSUPPORTED;
    }
    return SEL_OK;
}

Plan make_plan(const sel_mesh *m, const sel_params *p)
{
    Plan L;
    const size_t ts = (p->precision == SEL_FP32_DEV) ? 4 : 8;
    const int64_t E = m->E, np = m->np, n1 = m->n1;
    const int64_t Gtot = E * (int64_t)m->nint + m->ngrp;
    size_t c = 0;
    L.tabD = carve(c, ts * n1 * n1);
    L.tabF = carve(c, ts * n1 * n1);
    L.tabW = carve(c, ts * n1);
    L.geoD = carve(c, 8 * n1 * n1);
    L.geoW = carve(c, 8 * n1);
    L.pcode = carve(c, 4 * np);
    L.bpos = carve(c, 4 * (size_t)m->nbe);
    L.xyz = carve(c, 8 * (size_t)(E * np * m->dim));
    L.wJ = carve(c, 8 * (size_t)(E * np));
    L.J = carve(c, 8 * (size_t)(E * np));
    L.Gm = carve(c, ts * (size_t)(E * m->dim * m->dim * np));
    L.invw = carve(c, ts * (size_t)(E * m->nint + 1));
    L.invMb = carve(c, ts * (size_t)(m->ngrp + 1));
    L.bmap = carve(c, 4 * (size_t)(E * m->nbe));
    L.bown = carve(c, (size_t)(E * m->nbe));
    L.goff = carve(c, 4 * (size_t)(m->ngrp + 1));
    L.gmem = carve(c, 4 * (size_t)(E * m->nbe));
    L.ftag = carve(c, 4 * (size_t)(E * 2 * m->dim));
    L.wallu = carve(c, ts * 3 * (size_t)(m->ntags + 1));
    const int64_t nstate = (int64_t)p->Q * (E * m->nint + (m->ngrp + 63) / 64 * 64);
    for (int i = 0; i < 4; ++i) L.f[i] = carve(c, ts * (size_t)nstate);
    L.rtb = carve(c, ts * (size_t)p->Q * (size_t)m->plane);
    L.posmap = carve(c, 4 * (size_t)(E * m->nbe));
    if (m->dg) L.nbr = carve(c, 4 * m->nbr.size());
    L.hidx = carve(c, 4 * (size_t)(m->ngrp + 1));
    L.rhoc = carve(c, ts * (size_t)Gtot);
    L.Fn = carve(c, ts * 3 * (size_t)Gtot);
    L.io = carve(c, 8 * (size_t)(E * np * (m->dim + 1)));
    int64_t nred = (E * np + 255) / 256;
    if (nred > 1024) nred = 1024;
    L.nred = (int)nred;
    L.red = carve(c, 8 * (size_t)(8 * nred + 8));
    L.flag = carve(c, 16);
    if (p->closure != nullptr) {
        L.closure = true;
        L.cl_params = carve(c, 4 * (size_t)sel_closure_len());
        L.cl_X = carve(c, 4 * 6 * (size_t)Gtot);
        L.cl_dtau = carve(c, 4 * (size_t)Gtot);
    }
    L.total = (c + kAlign - 1) / kAlign * kAlign;
    return L;
}

template <typename T>
std::vector<T> conv(const double *src, size_t n)
{
    std::vector<T> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = T(src[i]);
    return v;
}

template <typename T>
int upload_tables(sel_sim *s, const sel::Tables &t, const sel_mesh *m, std::vector<std::vector<char>> &keep)
{
    const int n1 = m->n1;
    std::vector<double> D(n1 * n1), F(n1 * n1), W(n1);
    for (int i = 0; i < n1; ++i) {
        W[i] = t.w[i];
        for (int j = 0; j < n1; ++j) {
            D[i * n1 + j] = t.D[i * n1 + j];
            F[i * n1 + j] = t.F[i * n1 + j];
        }
    }
    auto put = [&](void *dst, const void *src, size_t bytes) -> int {
        keep.emplace_back((const char *)src, (const char *)src + bytes);
        HIP_OK(hipMemcpyAsync(dst, keep.back().data(), bytes, hipMemcpyHostToDevice, s->stream));
        return SEL_OK;
    };
    std::vector<T> Dt = conv<T>(D.data(), D.size()), Ft = conv<T>(F.data(), F.size()), Wt = conv<T>(W.data(), W.size());
    if (put(s->tabD, Dt.data(), sizeof(T) * Dt.size())) return SEL_EDEVICE;
    if (put(s->tabF, Ft.data(), sizeof(T) * Ft.size())) return SEL_EDEVICE;
    if (put(s->tabW, Wt.data(), sizeof(T) * Wt.size())) return SEL_EDEVICE;
    if (put(s->geoD, D.data(), 8 * D.size())) return SEL_EDEVICE;
    if (put(s->geoW, W.data(), 8 * W.size())) return SEL_EDEVICE;
    std::vector<T> wu = conv<T>(m->wall_u.data(), m->wall_u.size());
    if (put(s->wallu, wu.data(), sizeof(T) * wu.size())) return SEL_EDEVICE;
    return SEL_OK;
}

int sync_check(sel_sim *s)
{
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        set_error(std::string("device error: ") + hipGetErrorString(e));
        return SEL_EDEVICE;
    }
    return SEL_OK;
}

}  // namespace

extern "C" int sel_workspace_bytes(const sel_mesh *m, const sel_params *p, size_t *bytes)
{
    if (!bytes) {
        set_error("sel_workspace_bytes: null out pointer");
        return SEL_EINVAL;
    }
    if (int rc = check_params(m, p)) return rc;
    *bytes = make_plan(m, p).total;
    return SEL_OK;
}

// sums of the two per-node terms over the element nodes of each bin, in
// the order of the bin's node list (one workgroup per bin, fixed reduction
// tree: the result does not depend on the launch)
static __global__ void __launch_bounds__(256) k_bin_sums(const double *terms, int64_t nl, const int32_t *nodes,
                                                  const int32_t *off, int nbins, double *out)
{
    __shared__ double sh[2][256];
    const int b = blockIdx.x;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t k = off[b] + threadIdx.x; k < off[b + 1]; k += 256) {
        const int64_t q = nodes[k];
        a0 += terms[q];
        a1 += terms[nl + q];
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[b] = sh[0][0];
        out[nbins + b] = sh[1][0];
    }
}

static void free_profile(sel_sim *s)
{
    // cleanup: a failing free cannot be acted on
    if (s->prof_nodes) (void)hipFree(s->prof_nodes);
    if (s->prof_off) (void)hipFree(s->prof_off);
    if (s->prof_out) (void)hipFree(s->prof_out);
    s->prof_nodes = nullptr;
    s->prof_off = nullptr;
    s->prof_out = nullptr;
    s->prof_nbins = 0;
}

extern "C" int sel_destroy(sel_sim *s)
{
    if (!s) return SEL_OK;
    free_profile(s);
    if (s->owns_ws && s->ws) (void)hipFree(s->ws);  // the handle is released whatever the free returns
    delete s;
    return SEL_OK;
}

extern "C" int sel_init(const sel_mesh *m, const sel_params *p, const double *rho, const double *u, void *dev_ws,
                        size_t ws_bytes, void *hip_stream, sel_sim **out)
{
    if (!out || !rho || !u) {
        set_error("sel_init: null pointer argument");
        return SEL_EINVAL;
    }
    if (int rc = check_params(m, p)) return rc;
    const sel::Ops *ops = sel::find_ops(m->dim, m->N, p->Q, p->precision);
    sel::Tables tab;
    if (sel::build_gll(m->N, tab) || sel::build_filter(m->N, p->filter_type, p->filter_kc, p->filter_amp,
                                                       p->filter_order, tab)) {
        set_error("sel_init: table construction failed");
        return SEL_EINVAL;
    }
    sel::HostLattice lat;
    if (sel::build_lattice(m->dim, p->Q, lat)) {
        set_error("sel_init: lattice");
        return SEL_EINVAL;
    }
    Plan L = make_plan(m, p);
    sel_sim *s = new (std::nothrow) sel_sim();
    if (!s) {
        set_error("sel_init: out of host memory");
        return SEL_ENOMEM;
    }
    s->dim = m->dim;
    s->N = m->N;
    s->n1 = m->n1;
    s->np = m->np;
    s->nint = m->nint;
    s->nbe = m->nbe;
    s->Q = p->Q;
    s->E = m->E;
    s->ngrp = m->ngrp;
    s->Gi = m->E * (int64_t)m->nint;
    s->Gtot = s->Gi + m->ngrp;
    s->nstate = (int64_t)p->Q * (s->Gi + (m->ngrp + 63) / 64 * 64);
    s->nwall = m->nwall;
    s->p = *p;
    s->prec = p->precision;
    s->tsize = (p->precision == SEL_FP32_DEV) ? 4 : 8;
    const double cs2 = 1.0 / 3.0;
    s->tau = (p->nu / cs2) / p->dt;  // nu = lambda cs^2, tau = lambda / dt (Sec. 2.1)
    s->omega = 1.0 / (s->tau + 0.5);
    for (int a = 0; a < p->Q; ++a) {
        double eg = 0.0;
        for (int k = 0; k < m->dim; ++k) eg += lat.e[a][k] * p->accel[k];
        s->fsc[a] = lat.t[a] * eg / cs2;
        s->toff[a] = (p->precision == SEL_FP32_DEV) ? lat.t[a] * p->rho0 : 0.0;
    }
    s->stream = static_cast<hipStream_t>(hip_stream);
    if (dev_ws) {
        if (ws_bytes < L.total) {
            set_error("sel_init: workspace smaller than sel_workspace_bytes");
            delete s;
            return SEL_ENOMEM;
        }
        s->ws = dev_ws;
        s->ws_bytes = ws_bytes;
    } else {
        if (hipMalloc(&s->ws, L.total) != hipSuccess) {
            set_error("sel_init: hipMalloc of the workspace failed");
            delete s;
            return SEL_ENOMEM;
        }
        s->owns_ws = true;
        s->ws_bytes = L.total;
    }
    char *b = static_cast<char *>(s->ws);
    s->tabD = b + L.tabD;
    s->tabF = b + L.tabF;
    s->tabW = b + L.tabW;
    s->geoD = reinterpret_cast<double *>(b + L.geoD);
    s->geoW = reinterpret_cast<double *>(b + L.geoW);
    s->pcode = reinterpret_cast<int32_t *>(b + L.pcode);
    s->bpos = reinterpret_cast<int32_t *>(b + L.bpos);
    s->xyz = reinterpret_cast<double *>(b + L.xyz);
    s->wJ = reinterpret_cast<double *>(b + L.wJ);
    s->J = reinterpret_cast<double *>(b + L.J);
    s->Gm = b + L.Gm;
    s->invw = b + L.invw;
    s->invMb = b + L.invMb;
    s->bmap = reinterpret_cast<int32_t *>(b + L.bmap);
    s->bown = reinterpret_cast<uint8_t *>(b + L.bown);
    s->goff = reinterpret_cast<int32_t *>(b + L.goff);
    s->gmem = reinterpret_cast<int32_t *>(b + L.gmem);
    s->ftag = reinterpret_cast<int32_t *>(b + L.ftag);
    s->wallu = b + L.wallu;
    for (int i = 0; i < 4; ++i) s->f[i] = b + L.f[i];
    s->rtb = b + L.rtb;
    s->posmap = reinterpret_cast<int32_t *>(b + L.posmap);
    if (m->dg) {
        s->nbr = reinterpret_cast<int32_t *>(b + L.nbr);
        s->nfn = m->nfn;
    }
    s->hidx = reinterpret_cast<int32_t *>(b + L.hidx);
    s->plane = m->plane;
    s->ngp = m->ngp;
    s->nmp = m->nmp;
    s->rhoc = b + L.rhoc;
    s->Fn = b + L.Fn;
    s->io = reinterpret_cast<double *>(b + L.io);
    s->red = reinterpret_cast<double *>(b + L.red);
    s->nred = L.nred;
    s->flag = reinterpret_cast<int32_t *>(b + L.flag);
    s->cur = 0;
    if (L.closure) {
        s->closure_space = true;
        s->cl_params = reinterpret_cast<float *>(b + L.cl_params);
        s->cl_X = reinterpret_cast<float *>(b + L.cl_X);
        s->cl_dtau = reinterpret_cast<float *>(b + L.cl_dtau);
    }

    auto fail = [&](int rc) {
        (void)hipStreamSynchronize(s->stream);  // drain before freeing; rc already holds the error
        sel_destroy(s);
        return rc;
    };
    std::vector<std::vector<char>> keep;
    int rc = (s->prec == SEL_FP32_DEV) ? upload_tables<float>(s, tab, m, keep) : upload_tables<double>(s, tab, m, keep);
    if (rc) return fail(rc);
    const int64_t nl = m->E * (int64_t)m->np;
#define UP(dst, src, bytes)                                                                               \
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream) != hipSuccess) {                \
        set_error("sel_init: upload failed");                                                             \
        return fail(SEL_EDEVICE);                                                                         \
    }
    UP(s->pcode, m->pcode.data(), 4 * m->np);
    UP(s->bpos, m->bpos.data(), 4 * m->nbe);
    UP(s->xyz, m->xyz.data(), 8 * nl * m->dim);
    UP(s->bmap, m->bmap.data(), 4 * m->bmap.size());
    UP(s->bown, m->bown.data(), m->bown.size());
    UP(s->goff, m->goff.data(), 4 * m->goff.size());
    UP(s->gmem, m->gmem.data(), 4 * m->gmem.size());
    UP(s->ftag, m->ftag.data(), 4 * m->ftag.size());
    UP(s->posmap, m->posmap.data(), 4 * m->posmap.size());
    if (m->dg) UP(s->nbr, m->nbr.data(), 4 * m->nbr.size());
    UP(s->hidx, m->hidx.data(), 4 * m->hidx.size());
    UP(s->io, rho, 8 * nl);
    UP(s->io + nl, u, 8 * nl * m->dim);
#undef UP
    if (hipMemsetAsync(s->flag, 0, 16, s->stream) != hipSuccess) return fail(SEL_EDEVICE);
    for (int i = 0; i < 4; ++i)
        if (hipMemsetAsync(s->f[i], 0, s->tsize * s->nstate, s->stream) != hipSuccess) return fail(SEL_EDEVICE);
    if (hipMemsetAsync(s->rhoc, 0, s->tsize * s->Gtot, s->stream) != hipSuccess) return fail(SEL_EDEVICE);
    if (L.closure) {
        if (hipMemsetAsync(s->cl_X, 0, 4 * 6 * s->Gtot, s->stream) != hipSuccess ||
            hipMemsetAsync(s->cl_dtau, 0, 4 * s->Gtot, s->stream) != hipSuccess ||
            hipMemcpyAsync(s->cl_params, p->closure, 4 * p->closure_len, hipMemcpyHostToDevice, s->stream) !=
                hipSuccess)
            return fail(SEL_EDEVICE);
        s->closure_on = true;
    }
    if ((rc = ops->geometry(s))) return fail(rc);
    if ((rc = ops->mass(s))) return fail(rc);
    if ((rc = ops->init(s, s->io, s->io + nl))) return fail(rc);
    int32_t flag[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(flag, s->flag, 16, hipMemcpyDeviceToHost, s->stream) != hipSuccess) return fail(SEL_EDEVICE);
    if ((rc = sync_check(s))) return fail(rc);
    if (flag[0]) {
        set_error("sel_init: non-positive Jacobian in some element");
        return fail(SEL_EINVAL);
    }
    *out = s;
    return SEL_OK;
}

static const sel::Ops *ops_of(const sel_sim *s) { return sel::find_ops(s->dim, s->N, s->Q, s->prec); }

extern "C" int sel_step(sel_sim *s, int64_t nsteps)
{
    if (!s) {
        set_error("sel_step: null sim");
        return SEL_EINVAL;
    }
    if (nsteps < 0) {
        set_error("sel_step: nsteps < 0");
        return SEL_EINVAL;
    }
    return ops_of(s)->step(s, nsteps);
}

extern "C" int sel_step_timed(sel_sim *s, int64_t nsteps, double *ms, int64_t *launches)
{
    if (!s || !ms || !launches) {
        set_error("sel_step_timed: null argument");
        return SEL_EINVAL;
    }
    if (nsteps < 0) {
        set_error("sel_step_timed: nsteps < 0");
        return SEL_EINVAL;
    }
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
    ev.reserve(8 * (size_t)nsteps + 8);
    s->timing = &ev;
    int rc = ops_of(s)->step(s, nsteps);
    s->timing = nullptr;
    if (!rc) rc = sync_check(s);
    double acc[SEL_NKIND] = {};
    int64_t cnt[SEL_NKIND] = {};
    for (auto &x : ev) {
        float t = 0.f;
        if (!rc && hipEventElapsedTime(&t, x.second.first, x.second.second) != hipSuccess) rc = SEL_EDEVICE;
        acc[x.first] += t;
        cnt[x.first] += 1;
        (void)hipEventDestroy(x.second.first);
        (void)hipEventDestroy(x.second.second);
    }
    if (rc) return rc;
    for (int k = 0; k < SEL_NKIND; ++k) {
        ms[k] = acc[k];
        launches[k] = cnt[k];
    }
    return SEL_OK;
}

static int reduce_to_host(sel_sim *s, double *out8)
{
    if (int rc = ops_of(s)->reduce(s)) return rc;
    HIP_OK(hipMemcpyAsync(out8, s->red + 8 * s->nred, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    return sync_check(s);
}

extern "C" int sel_sync(sel_sim *s)
{
    if (!s) {
        set_error("sel_sync: null sim");
        return SEL_EINVAL;
    }
    if (int rc = sync_check(s)) return rc;
    double r[8];
    if (int rc = reduce_to_host(s, r)) return rc;
    if (r[5] != 0.0) {
        set_error("sel_sync: the state holds non-finite values");
        return SEL_ENONFINITE;
    }
    return SEL_OK;
}

extern "C" int sel_reduce(sel_sim *s, double *out)
{
    if (!s || !out) {
        set_error("sel_reduce: null argument");
        return SEL_EINVAL;
    }
    double r[8];
    if (int rc = reduce_to_host(s, r)) return rc;
    out[0] = r[0];
    for (int k = 0; k < s->dim; ++k) out[1 + k] = r[1 + k];
    out[1 + s->dim] = r[4];
    out[2 + s->dim] = r[5];
    return SEL_OK;
}

extern "C" int sel_moments_device(sel_sim *s, double *d_rho, double *d_u)
{
    if (!s || !d_rho || !d_u) {
        set_error("sel_moments_device: null argument");
        return SEL_EINVAL;
    }
    return ops_of(s)->moments(s, d_rho, d_u);
}

extern "C" int sel_moments(sel_sim *s, double *rho, double *u)
{
    if (!s || !rho || !u) {
        set_error("sel_moments: null argument");
        return SEL_EINVAL;
    }
    const int64_t nl = s->E * (int64_t)s->np;
    if (int rc = ops_of(s)->moments(s, s->io, s->io + nl)) return rc;
    HIP_OK(hipMemcpyAsync(rho, s->io, 8 * nl, hipMemcpyDeviceToHost, s->stream));
    HIP_OK(hipMemcpyAsync(u, s->io + nl, 8 * nl * s->dim, hipMemcpyDeviceToHost, s->stream));
    if (int rc = sync_check(s)) return rc;
    for (int64_t i = 0; i < nl; ++i)
        if (!std::isfinite(rho[i])) {
            set_error("sel_moments: non-finite density");
            return SEL_ENONFINITE;
        }
    return SEL_OK;
}

extern "C" int sel_get_f(sel_sim *s, double *f)
{
    if (!s || !f) {
        set_error("sel_get_f: null argument");
        return SEL_EINVAL;
    }
    const int64_t nl = s->E * (int64_t)s->np;
    const sel::Ops *ops = ops_of(s);
    for (int a = 0; a < s->Q; ++a) {
        if (int rc = ops->gather(s, a, s->f[s->cur], s->io, true)) return rc;
        HIP_OK(hipMemcpy2DAsync(f + (int64_t)a * s->np, 8 * (size_t)s->Q * s->np, s->io, 8 * (size_t)s->np,
                                8 * (size_t)s->np, (size_t)s->E, hipMemcpyDeviceToHost, s->stream));
    }
    (void)nl;
    return sync_check(s);
}

extern "C" int sel_set_f(sel_sim *s, const double *f)
{
    if (!s || !f) {
        set_error("sel_set_f: null argument");
        return SEL_EINVAL;
    }
    const sel::Ops *ops = ops_of(s);
    for (int a = 0; a < s->Q; ++a) {
        HIP_OK(hipMemcpy2DAsync(s->io, 8 * (size_t)s->np, f + (int64_t)a * s->np, 8 * (size_t)s->Q * s->np,
                                8 * (size_t)s->np, (size_t)s->E, hipMemcpyHostToDevice, s->stream));
        if (int rc = ops->scatter(s, a, s->io, s->f[s->cur], true)) return rc;
    }
    return sync_check(s);
}

extern "C" int sel_set_force(sel_sim *s, const double *F)
{
    if (!s) {
        set_error("sel_set_force: null sim");
        return SEL_EINVAL;
    }
    if (!F) {
        s->force_on = false;
        return SEL_OK;
    }
    for (int64_t i = 0; i < s->E * (int64_t)s->np * s->dim; ++i)
        if (!std::isfinite(F[i])) {
            set_error("sel_set_force: non-finite force");
            return SEL_EINVAL;
        }
    HIP_OK(hipMemcpyAsync(s->io, F, 8 * (size_t)s->E * s->np * s->dim, hipMemcpyHostToDevice, s->stream));
    if (int rc = ops_of(s)->set_force(s, s->io)) return rc;
    s->force_on = true;
    return sync_check(s);
}

extern "C" int sel_velocity_gradient(sel_sim *s, double *grad)
{
    if (!s || !grad) {
        set_error("sel_velocity_gradient: null argument");
        return SEL_EINVAL;
    }
    const int64_t nl = s->E * (int64_t)s->np;
    const int d = s->dim;
    std::vector<double> row((size_t)nl * d);
    for (int c = 0; c < d; ++c) {
        if (int rc = ops_of(s)->grad_row(s, c, s->io)) return rc;
        HIP_OK(hipMemcpyAsync(row.data(), s->io, 8 * row.size(), hipMemcpyDeviceToHost, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));
        for (int64_t l = 0; l < nl; ++l)
            for (int q = 0; q < d; ++q) grad[(l * d + c) * d + q] = row[l * d + q];
    }
    return sync_check(s);
}

extern "C" int sel_radial_profile(sel_sim *s, const double *origin, const double *axis, double rmax, int32_t nbins,
                                  double *out)
{
    if (!s || !origin || !axis || !out) {
        set_error("sel_radial_profile: null argument");
        return SEL_EINVAL;
    }
    if (nbins < 1 || nbins > 4096 || !(rmax > 0.0) || !std::isfinite(rmax)) {
        set_error("sel_radial_profile: need 1 <= nbins <= 4096 and rmax > 0");
        return SEL_EINVAL;
    }
    const int d = s->dim;
    double n[3] = {0, 0, 0}, o[3] = {0, 0, 0}, nn = 0.0;
    for (int k = 0; k < d; ++k) {
        n[k] = axis[k];
        o[k] = origin[k];
        nn += n[k] * n[k];
    }
    if (!(nn > 0.0) || !std::isfinite(nn)) {
        set_error("sel_radial_profile: axis must be a non-zero finite vector");
        return SEL_EINVAL;
    }
    for (int k = 0; k < d; ++k) n[k] /= std::sqrt(nn);
    const int64_t nl = s->E * (int64_t)s->np;
    const double key[7] = {o[0], o[1], o[2], n[0], n[1], n[2], rmax};
    bool same = s->prof_nbins == nbins;
    for (int k = 0; k < 7; ++k) same = same && key[k] == s->prof_key[k];
    if (!same) {
        // node lists per bin from the node coordinates (ascending node order)
        free_profile(s);
        std::vector<double> x((size_t)nl * d);
        HIP_OK(hipMemcpyAsync(x.data(), s->xyz, 8 * x.size(), hipMemcpyDeviceToHost, s->stream));
        if (int rc = sync_check(s)) return rc;
        std::vector<int32_t> bin((size_t)nl), off((size_t)nbins + 1, 0);
        for (int64_t q = 0; q < nl; ++q) {
            double v[3] = {0, 0, 0}, vn = 0.0;
            for (int k = 0; k < d; ++k) {
                v[k] = x[q * d + k] - o[k];
                vn += v[k] * n[k];
            }
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) r2 += (v[k] - vn * n[k]) * (v[k] - vn * n[k]);
            const double rb = std::sqrt(r2) / rmax * nbins;
            bin[q] = (rb < nbins) ? (int32_t)rb : -1;
            if (bin[q] >= 0) off[bin[q] + 1]++;
        }
        for (int b = 0; b < nbins; ++b) off[b + 1] += off[b];
        std::vector<int32_t> nodes((size_t)off[nbins] + 1), pos(off.begin(), off.end() - 1);
        for (int64_t q = 0; q < nl; ++q)
            if (bin[q] >= 0) nodes[pos[bin[q]]++] = (int32_t)q;
        if (hipMalloc(&s->prof_nodes, 4 * nodes.size()) != hipSuccess ||
            hipMalloc(&s->prof_off, 4 * off.size()) != hipSuccess ||
            hipMalloc(&s->prof_out, 8 * (size_t)(2 * nbins)) != hipSuccess) {
            free_profile(s);
            set_error("sel_radial_profile: allocation of the bin lists failed");
            return SEL_ENOMEM;
        }
        if (hipMemcpyAsync(s->prof_nodes, nodes.data(), 4 * nodes.size(), hipMemcpyHostToDevice, s->stream) !=
                hipSuccess ||
            hipMemcpyAsync(s->prof_off, off.data(), 4 * off.size(), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
            sync_check(s) != SEL_OK) {
            free_profile(s);
            set_error("sel_radial_profile: upload of the bin lists failed");
            return SEL_EDEVICE;
        }
        s->prof_nbins = nbins;
        for (int k = 0; k < 7; ++k) s->prof_key[k] = key[k];
    }
    if (int rc = ops_of(s)->axial_terms(s, n, s->io)) return rc;
    hipLaunchKernelGGL(k_bin_sums, dim3((unsigned)nbins), dim3(256), 0, s->stream, s->io, nl, s->prof_nodes,
                       s->prof_off, nbins, s->prof_out);
    if (hipGetLastError() != hipSuccess) {
        set_error("sel_radial_profile: launch failed");
        return SEL_EDEVICE;
    }
    HIP_OK(hipMemcpyAsync(out, s->prof_out, 8 * (size_t)(2 * nbins), hipMemcpyDeviceToHost, s->stream));
    return sync_check(s);
}

extern "C" int sel_get_time(const sel_sim *s, double *t, int64_t *nstep)
{
    if (!s) {
        set_error("sel_get_time: null sim");
        return SEL_EINVAL;
    }
    if (t) *t = s->time;
    if (nstep) *nstep = s->nstep;
    return SEL_OK;
}

extern "C" int sel_apply(sel_sim *s, int32_t op, const double *fin, double *fout)
{
    if (!s || !fin || !fout) {
        set_error("sel_apply: null argument");
        return SEL_EINVAL;
    }
    if (op < SEL_OP_RHS || op > SEL_OP_FILTER) {
        set_error("sel_apply: unknown op");
        return SEL_EINVAL;
    }
    const sel::Ops *ops = ops_of(s);
    void *src = s->f[3], *dst = s->f[2];
    for (int a = 0; a < s->Q; ++a) {
        HIP_OK(hipMemcpy2DAsync(s->io, 8 * (size_t)s->np, fin + (int64_t)a * s->np, 8 * (size_t)s->Q * s->np,
                                8 * (size_t)s->np, (size_t)s->E, hipMemcpyHostToDevice, s->stream));
        if (int rc = ops->scatter(s, a, s->io, src, true)) return rc;
    }
    if (op == SEL_OP_RHS_LOCAL) {
        const size_t n = (size_t)s->Q * s->E * s->np;
        void *loc = nullptr;
        HIP_OK(hipMalloc(&loc, s->tsize * n));
        int rc = ops->apply(s, op, src, dst, loc);
        std::vector<char> h(s->tsize * n);
        if (!rc && hipMemcpyAsync(h.data(), loc, s->tsize * n, hipMemcpyDeviceToHost, s->stream) != hipSuccess)
            rc = SEL_EDEVICE;
        if (!rc) rc = sync_check(s);
        (void)hipFree(loc);  // cleanup: the result code is already decided
        if (rc) return rc;
        // [Q][E][np] (storage type) -> [E][Q][np] FP64
        for (int a = 0; a < s->Q; ++a)
            for (int64_t e = 0; e < s->E; ++e)
                for (int q = 0; q < s->np; ++q) {
                    const size_t si = ((size_t)a * s->E + e) * s->np + q;
                    const double v = (s->tsize == 4) ? (double)reinterpret_cast<float *>(h.data())[si]
                                                     : reinterpret_cast<double *>(h.data())[si];
                    fout[(e * s->Q + a) * s->np + q] = v;
                }
        return SEL_OK;
    }
    if (int rc = ops->apply(s, op, src, dst, nullptr)) return rc;
    const bool add = (op == SEL_OP_COLLIDE || op == SEL_OP_FILTER);
    for (int a = 0; a < s->Q; ++a) {
        if (int rc = ops->gather(s, a, dst, s->io, add)) return rc;
        HIP_OK(hipMemcpy2DAsync(fout + (int64_t)a * s->np, 8 * (size_t)s->Q * s->np, s->io, 8 * (size_t)s->np,
                                8 * (size_t)s->np, (size_t)s->E, hipMemcpyDeviceToHost, s->stream));
    }
    return sync_check(s);
}

extern "C" int sel_geometry(sel_sim *s, double *wJ, double *J)
{
    if (!s) {
        set_error("sel_geometry: null sim");
        return SEL_EINVAL;
    }
    const int64_t nl = s->E * (int64_t)s->np;
    if (wJ) HIP_OK(hipMemcpyAsync(wJ, s->wJ, 8 * nl, hipMemcpyDeviceToHost, s->stream));
    if (J) HIP_OK(hipMemcpyAsync(J, s->J, 8 * nl, hipMemcpyDeviceToHost, s->stream));
    return sync_check(s);
}

extern "C" void *sel_stream(const sel_sim *s) { return s ? (void *)s->stream : nullptr; }
