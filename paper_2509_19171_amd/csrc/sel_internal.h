// Internal declarations of the HIP library (host setup, kernels, C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sel.h"

namespace sel {

constexpr int kMaxN1 = 16;  // host tables up to N = 15
constexpr int kMaxQ = 27;

// Host-side tables of the spectral element (built in tables.cpp).
struct Tables {
    int N = 0;
    double xi[kMaxN1] = {};
    double w[kMaxN1] = {};
    double D[kMaxN1 * kMaxN1] = {};   // D[i][c] = l_c'(xi_i)
    double F[kMaxN1 * kMaxN1] = {};   // filter matrix (identity if no filter)
};
int build_gll(int N, Tables &t);
int build_filter(int N, int type, int kc, double amp, double order, Tables &t);
int build_projection(int Nf, int Nc, double *Pm);

// Lattice (host copy for the few host computations).
struct HostLattice {
    int Q = 0;
    int e[kMaxQ][3] = {};
    double t[kMaxQ] = {};
    int opp[kMaxQ] = {};
};
int build_lattice(int dim, int Q, HostLattice &L);

}  // namespace sel

// Mesh after ingest: copies of the caller's arrays plus the node classes and
// the shared-node groups used by the assembly.
struct sel_mesh {
    int dim = 0, N = 0, n1 = 0, np = 0, nint = 0, nbe = 0, nface = 0;
    int64_t E = 0;
    std::vector<double> xyz;       // [E][np][dim]
    std::vector<int64_t> gid;      // [E][np]
    std::vector<int32_t> ftag;     // [E][2 dim]
    int ntags = 0;
    std::vector<double> wall_u;    // [ntags][3]
    // structural node classes (same for every element)
    std::vector<int32_t> pcode;    // [np]: interior slot s >= 0, or -(b + 1) for boundary slot b
    std::vector<int32_t> bpos;     // [nbe] node index of boundary slot b
    // shared-node groups over element-boundary nodes, ordered by first member
    int64_t ngrp = 0;
    std::vector<int32_t> bmap;     // [E][nbe] group of each element-boundary node
    std::vector<uint8_t> bown;     // [E][nbe] 1 for the first (owning) member
    std::vector<int32_t> goff;     // [ngrp + 1]
    std::vector<int32_t> gmem;     // members as e * nbe + b, ascending
    int64_t nwall = 0;
    int64_t unique_nodes = 0;
    // element-contribution slots: member rank r of group g writes plane r
    // (r < 2) at index g, or extra plane r - 2 at the group's index among the
    // groups with more than two members (hidx)
    int64_t ngp = 0, nmp = 0, plane = 0;  // padded group / multi-group counts, floats per velocity
    int maxm = 0;
    std::vector<int32_t> posmap;  // [E][nbe] slot of each element-boundary node
    std::vector<int32_t> hidx;    // [ngrp] index among groups with > 2 members, or -1
    // discontinuous coupling: no node is shared (one group per element-
    // boundary node); nbr holds, for every face node of every face that is
    // not a wall, the group of the coincident node in the element across it
    int dg = 0;
    int nfn = 0;                  // nodes per face, (N+1)^(dim-1)
    std::vector<int32_t> nbr;     // [E][2 dim][nfn], face nodes in increasing node index; -1 on walls
};

// Device arrays of a simulation, all carved out of one workspace.
struct sel_sim {
    // copy of mesh scalars
    int dim = 0, N = 0, n1 = 0, np = 0, nint = 0, nbe = 0, Q = 0;
    int64_t E = 0, ngrp = 0, Gi = 0, Gtot = 0, nwall = 0;
    int64_t nstate = 0;        // entries of one state array (Q per node, groups padded to tiles of 64)
    sel_params p{};
    int prec = SEL_FP64;
    size_t tsize = 8;
    double tau = 0, omega = 0;
    double fsc[sel::kMaxQ] = {};   // F* per unit density: t_a (e_a . g) / c_s^2
    double toff[sel::kMaxQ] = {};  // t_a rho0 (deviation offset)
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool owns_ws = false;
    double time = 0.0;
    int64_t nstep = 0;
    // device pointers (typed views of the workspace)
    void *tabD = nullptr, *tabF = nullptr, *tabW = nullptr;  // T tables [n1*n1], [n1*n1], [n1]
    double *geoD = nullptr, *geoW = nullptr;                  // FP64 D-hat and GLL weights
    int32_t *pcode = nullptr, *bpos = nullptr;
    double *xyz = nullptr;     // [E][np][dim]
    double *wJ = nullptr;      // [E][np]
    double *J = nullptr;       // [E][np]
    void *Gm = nullptr;        // T [E][dim*dim][np]
    void *invw = nullptr;      // T [E][nint]
    void *invMb = nullptr;     // T [ngrp]
    int32_t *bmap = nullptr;   // [E][nbe]
    uint8_t *bown = nullptr;   // [E][nbe]
    int32_t *goff = nullptr;   // [ngrp+1]
    int32_t *gmem = nullptr;   // [E*nbe]
    int32_t *ftag = nullptr;   // [E][2 dim]
    int32_t *posmap = nullptr; // [E][nbe] contribution slot
    int32_t *hidx = nullptr;   // [ngrp]
    int32_t *nbr = nullptr;    // discontinuous coupling: [E][2 dim][nfn] group across each face, or nullptr
    void *Fn = nullptr;        // T [Gtot][3] force density per node id (added to rho g)
    bool force_on = false;
    int nfn = 0;
    int64_t plane = 0, ngp = 0, nmp = 0;
    void *wallu = nullptr;     // T [ntags+1][3], row 0 = zero
    void *f[4] = {};           // T [nstate]: state, f0, stage a, stage b
    void *rtb = nullptr;       // T [Q][plane] element contributions of boundary nodes
    void *rhoc = nullptr;      // T [Gtot]
    double *io = nullptr;      // FP64 [E][np][dim+1] (moments / per-velocity transfers)
    double *red = nullptr;     // FP64 [nred][8] partial sums
    int nred = 0;
    int32_t *flag = nullptr;   // [4] device flags (0: bad Jacobian)
    int cur = 0;               // index of the state array in f[]
    // learned relaxation-time closure (buffers exist when sel_init got a blob)
    bool closure_space = false;
    bool closure_on = false;
    float *cl_params = nullptr; // [closure blob]
    float *cl_X = nullptr;      // [Gtot][6] features per node id
    float *cl_dtau = nullptr;   // [Gtot]
    // radial profile diagnostic (sel_radial_profile): element nodes grouped by
    // radial bin in ascending order (CSR), built on the first call for a
    // binning and kept until the binning changes or the simulation ends
    int32_t *prof_nodes = nullptr;  // [entries] local node indices e * np + p
    int32_t *prof_off = nullptr;    // [nbins + 1]
    double *prof_out = nullptr;     // [2 nbins] per-bin sums
    int prof_nbins = 0;
    double prof_key[7] = {};        // origin, unit axis, rmax of the current binning
    // optional per-launch timing (sel_step_timed)
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> *timing = nullptr;
};

namespace sel {

void set_error(const std::string &msg);

}  // namespace sel
