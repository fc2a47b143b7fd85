// Mesh ingest: validation, structural node classes and the shared-node
// groups of the continuous-Galerkin assembly.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>

#include "sel_internal.h"

using sel::set_error;

static int ipow(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

static int build_interfaces(sel_mesh *m);

// Geometric consistency of the node numbering (the continuous element
// coupling of Sec. 2.2 identifies the copies of a node; the wall flux of
// Sec. 2.2.1 acts on the domain boundary only):
//  - a wall face is on the domain boundary: none of its face-interior nodes
//    (off the face's edges) is shared;
//  - the face-interior nodes of any other face are either all unshared or all
//    shared with exactly one copy, in one element, displaced by one constant
//    vector: zero for an interface, a translation for a periodic pair;
//  - every copy of every shared node coincides with the node's first copy up
//    to a sum of at most dim such translations (edges and corners of periodic
//    boxes are displaced along several directions at once).
// Distances below 1e-9 of the mesh extent count as zero.
static int check_copies(const sel_mesh *m, const std::vector<int32_t> &cnt)
{
    const int d = m->dim, n1 = m->n1, np = m->np, N = m->N;
    const int64_t E = m->E, nl = E * (int64_t)np;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) lo[k] = hi[k] = m->xyz[k];
    for (int64_t q = 0; q < nl; ++q)
        for (int k = 0; k < d; ++k) {
            lo[k] = std::min(lo[k], m->xyz[q * d + k]);
            hi[k] = std::max(hi[k], m->xyz[q * d + k]);
        }
    double ext = 0.0;
    for (int k = 0; k < d; ++k) ext = std::max(ext, hi[k] - lo[k]);
    const double tol = 1e-9 * (ext > 0.0 ? ext : 1.0);
    auto dist = [&](const double *a, const double *b) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s = std::max(s, std::fabs(a[k] - b[k]));
        return s;
    };
    // copies of every node id (CSR over the local nodes, ascending)
    std::vector<int64_t> first((size_t)nl + 1, 0), ord((size_t)nl);
    for (int64_t q = 0; q < nl; ++q) first[m->gid[q] + 1]++;
    for (int64_t g = 0; g < nl; ++g) first[g + 1] += first[g];
    {
        std::vector<int64_t> pos(first.begin(), first.end() - 1);
        for (int64_t q = 0; q < nl; ++q) ord[pos[m->gid[q]]++] = q;
    }
    // face-interior nodes of each face
    std::vector<std::vector<int>> fint(2 * d);
    for (int p = 0; p < np; ++p) {
        const int ijk[3] = {p % n1, (p / n1) % n1, p / (n1 * n1)};
        for (int a = 0; a < d; ++a) {
            if (ijk[a] != 0 && ijk[a] != N) continue;
            bool inner = true;
            for (int b = 0; b < d; ++b)
                if (b != a && (ijk[b] == 0 || ijk[b] == N)) inner = false;
            if (inner) fint[2 * a + (ijk[a] == N ? 1 : 0)].push_back(p);
        }
    }
    std::vector<std::array<double, 3>> tr;  // distinct non-zero face translations
    for (int64_t e = 0; e < E; ++e)
        for (int fc = 0; fc < 2 * d; ++fc) {
            const bool wall = m->ftag[e * 2 * d + fc] > 0;
            int nshared = 0;
            int64_t e2 = -1;
            double d0[3] = {0, 0, 0};
            for (size_t k = 0; k < fint[fc].size(); ++k) {
                const int64_t q = e * np + fint[fc][k];
                const int64_t g = m->gid[q];
                if (cnt[g] == 1) continue;
                if (wall) {
                    set_error("sel_mesh_create: a wall face shares a node off its edges with another face");
                    return SEL_EINVAL;
                }
                if (cnt[g] != 2) {
                    set_error("sel_mesh_create: a node inside a face has more than two copies");
                    return SEL_EINVAL;
                }
                const int64_t q2 = (ord[first[g]] == q) ? ord[first[g] + 1] : ord[first[g]];
                double dv[3] = {0, 0, 0};
                for (int c = 0; c < d; ++c) dv[c] = m->xyz[q2 * d + c] - m->xyz[q * d + c];
                if (nshared == 0) {
                    e2 = q2 / np;
                    for (int c = 0; c < 3; ++c) d0[c] = dv[c];
                } else if (q2 / np != e2 || dist(dv, d0) > tol) {
                    set_error("sel_mesh_create: the copies across a face are not one element's face displaced by "
                              "one vector (inconsistent node ids or coordinates)");
                    return SEL_EINVAL;
                }
                ++nshared;
            }
            if (nshared != 0 && nshared != (int)fint[fc].size()) {
                set_error("sel_mesh_create: a face is only partly shared");
                return SEL_EINVAL;
            }
            const double zero[3] = {0, 0, 0};
            if (nshared && dist(d0, zero) > tol) {
                bool seen = false;
                for (auto &t : tr)
                    if (dist(t.data(), d0) <= tol) seen = true;
                if (!seen) {
                    if (tr.size() >= 64) {
                        set_error("sel_mesh_create: more than 64 distinct periodic translations");
                        return SEL_EINVAL;
                    }
                    tr.push_back({d0[0], d0[1], d0[2]});
                }
            }
        }
    // sums of at most dim translations (each face translation appears with both signs)
    std::vector<std::array<double, 3>> sums{{0.0, 0.0, 0.0}};
    for (int r = 0; r < d; ++r) {
        const size_t n0 = sums.size();
        for (size_t i = 0; i < n0; ++i)
            for (auto &t : tr) {
                std::array<double, 3> s = sums[i];
                for (int c = 0; c < 3; ++c) s[c] += t[c];
                bool seen = false;
                for (auto &u : sums)
                    if (dist(u.data(), s.data()) <= tol) seen = true;
                if (!seen) sums.push_back(s);
                if (sums.size() > 4096) {
                    set_error("sel_mesh_create: too many combinations of periodic translations");
                    return SEL_EINVAL;
                }
            }
    }
    for (int64_t g = 0; g < nl; ++g) {
        if (first[g + 1] - first[g] < 2) continue;
        const double *x0 = m->xyz.data() + ord[first[g]] * d;
        for (int64_t i = first[g] + 1; i < first[g + 1]; ++i) {
            const double *x1 = m->xyz.data() + ord[i] * d;
            if (dist(x0, x1) <= tol) continue;
            double dv[3] = {0, 0, 0};
            for (int c = 0; c < d; ++c) dv[c] = x1[c] - x0[c];
            bool ok = false;
            for (auto &s : sums)
                if (dist(s.data(), dv) <= tol) {
                    ok = true;
                    break;
                }
            if (!ok) {
                set_error("sel_mesh_create: copies of node id " + std::to_string(g) +
                          " do not coincide (nor differ by the mesh's periodic translations)");
                return SEL_EINVAL;
            }
        }
    }
    return SEL_OK;
}

static int mesh_create(int32_t dim, int32_t N, int64_t E, const double *xyz, const int64_t *gid,
                       const int32_t *face_tag, int32_t ntags, const double *wall_u, int dg, sel_mesh **out)
{
    if (!out || !xyz || !gid) {
        set_error("sel_mesh_create: null pointer argument");
        return SEL_EINVAL;
    }
    if (dim != 2 && dim != 3) {
        set_error("sel_mesh_create: dim must be 2 or 3");
        return SEL_EINVAL;
    }
    if (N < 2 || N + 1 > sel::kMaxN1) {
        set_error("sel_mesh_create: order N must be in [2, 15]");
        return SEL_EUNSUPPORTED;
    }
    if (E < 1) {
        set_error("sel_mesh_create: E must be >= 1");
        return SEL_EINVAL;
    }
    if (ntags < 0 || (ntags > 0 && !wall_u)) {
        set_error("sel_mesh_create: ntags < 0 or wall_u missing");
        return SEL_EINVAL;
    }
    if (ntags > 127) {
        set_error("sel_mesh_create: at most 127 wall tags");
        return SEL_EUNSUPPORTED;
    }
    sel_mesh *m = new (std::nothrow) sel_mesh();
    if (!m) {
        set_error("sel_mesh_create: out of host memory");
        return SEL_ENOMEM;
    }
    try {
        m->dim = dim;
        m->N = N;
        m->n1 = N + 1;
        m->np = ipow(N + 1, dim);
        m->nint = ipow(N - 1, dim);
        m->nbe = m->np - m->nint;
        m->nface = 2 * dim;
        m->E = E;
        const int64_t nl = E * (int64_t)m->np;
        if (E * (int64_t)m->nbe > INT32_MAX || nl > INT32_MAX) {
            set_error("sel_mesh_create: mesh too large for 32-bit node indices");
            delete m;
            return SEL_EUNSUPPORTED;
        }
        m->xyz.assign(xyz, xyz + nl * dim);
        m->gid.assign(gid, gid + nl);
        m->ftag.assign((size_t)E * m->nface, 0);
        if (face_tag)
            for (int64_t i = 0; i < E * m->nface; ++i) {
                if (face_tag[i] < 0 || face_tag[i] > ntags) {
                    set_error("sel_mesh_create: face_tag out of [0, ntags]");
                    delete m;
                    return SEL_EINVAL;
                }
                m->ftag[i] = face_tag[i];
            }
        m->ntags = ntags;
        m->wall_u.assign((size_t)(ntags + 1) * 3, 0.0);
        for (int t = 0; t < ntags; ++t)
            for (int k = 0; k < dim; ++k) m->wall_u[3 * (t + 1) + k] = wall_u[t * dim + k];
        m->nwall = 0;
        for (int32_t v : m->ftag) m->nwall += (v > 0);

        // structural classes: interior nodes (no index at 0 or N) and boundary
        // slots. Boundary slots are numbered face by face (face interiors in
        // face order, then edges, then corners), so that the nodes of one
        // shared face are a contiguous slot range in both elements.
        m->pcode.resize(m->np);
        m->bpos.resize(m->nbe);
        std::vector<std::pair<int64_t, int>> bkey;
        int ns = 0;
        for (int p = 0; p < m->np; ++p) {
            int ijk[3] = {p % m->n1, (p / m->n1) % m->n1, dim == 3 ? p / (m->n1 * m->n1) : 1};
            int nbd = 0, cls = 0;
            for (int d = 0; d < dim; ++d)
                if (ijk[d] == 0 || ijk[d] == N) {
                    ++nbd;
                    cls = cls * 8 + 2 * d + (ijk[d] == N ? 1 : 0) + 1;
                }
            if (nbd == 0) {
                m->pcode[p] = ns++;
            } else {
                bkey.push_back({((int64_t)nbd << 40) | ((int64_t)cls << 20) | p, p});
            }
        }
        std::sort(bkey.begin(), bkey.end());
        for (int b = 0; b < (int)bkey.size(); ++b) {
            m->bpos[b] = bkey[b].second;
            m->pcode[bkey[b].second] = -(b + 1);
        }

        // global ids: range check and no sharing of interior nodes
        std::vector<int32_t> cnt((size_t)nl, 0);
        for (int64_t i = 0; i < nl; ++i) {
            if (gid[i] < 0 || gid[i] >= nl) {
                set_error("sel_mesh_create: gid out of [0, E*np)");
                delete m;
                return SEL_EINVAL;
            }
            cnt[gid[i]]++;
        }
        for (int64_t e = 0; e < E; ++e)
            for (int p = 0; p < m->np; ++p)
                if (m->pcode[p] >= 0 && cnt[gid[e * m->np + p]] != 1) {
                    set_error("sel_mesh_create: a node off the element faces is shared");
                    delete m;
                    return SEL_EINVAL;
                }
        if (int rc = check_copies(m, cnt)) {
            delete m;
            return rc;
        }

        // shared-node groups over element-boundary nodes, members ascending,
        // groups ordered by their first member (the owner)
        const int64_t nlb = E * (int64_t)m->nbe;
        std::vector<std::pair<int64_t, int32_t>> key((size_t)nlb);
        for (int64_t e = 0; e < E; ++e)
            for (int b = 0; b < m->nbe; ++b) {
                int64_t lb = e * m->nbe + b;
                // the discontinuous coupling shares no node: one group each
                key[lb] = {dg ? lb : gid[e * m->np + m->bpos[b]], (int32_t)lb};
            }
        std::sort(key.begin(), key.end());
        std::vector<int64_t> run_start;
        for (int64_t i = 0; i < nlb; ++i)
            if (i == 0 || key[i].first != key[i - 1].first) run_start.push_back(i);
        run_start.push_back(nlb);
        const int64_t ngrp = (int64_t)run_start.size() - 1;
        std::vector<int64_t> order((size_t)ngrp);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
            return key[run_start[a]].second < key[run_start[b]].second;
        });
        m->ngrp = ngrp;
        m->goff.resize(ngrp + 1);
        m->gmem.resize(nlb);
        m->bmap.resize(nlb);
        m->bown.assign(nlb, 0);
        int64_t pos = 0;
        for (int64_t g = 0; g < ngrp; ++g) {
            int64_t r = order[g];
            m->goff[g] = (int32_t)pos;
            for (int64_t i = run_start[r]; i < run_start[r + 1]; ++i) {
                int32_t lb = key[i].second;
                m->gmem[pos++] = lb;
                m->bmap[lb] = (int32_t)g;
            }
            m->bown[m->gmem[m->goff[g]]] = 1;
        }
        m->goff[ngrp] = (int32_t)pos;
        m->unique_nodes = E * (int64_t)m->nint + ngrp;

        // contribution slots (rank planes): the assembly reads consecutive
        // groups from consecutive addresses
        m->ngp = (ngrp + 63) / 64 * 64;
        m->hidx.assign((size_t)ngrp, -1);
        int64_t nmulti = 0;
        int maxm = 0;
        for (int64_t g = 0; g < ngrp; ++g) {
            const int c = m->goff[g + 1] - m->goff[g];
            maxm = std::max(maxm, c);
            if (c > 2) m->hidx[g] = (int32_t)nmulti++;
        }
        m->nmp = (nmulti + 63) / 64 * 64;
        m->maxm = maxm;
        m->plane = 2 * m->ngp + (maxm > 2 ? (int64_t)(maxm - 2) * m->nmp : 0);
        if (m->plane > INT32_MAX) {
            set_error("sel_mesh_create: mesh too large for 32-bit contribution slots");
            delete m;
            return SEL_EUNSUPPORTED;
        }
        m->posmap.resize(nlb);
        for (int64_t g = 0; g < ngrp; ++g)
            for (int r = 0; r < m->goff[g + 1] - m->goff[g]; ++r) {
                const int32_t lb = m->gmem[m->goff[g] + r];
                m->posmap[lb] = (int32_t)(r < 2 ? r * m->ngp + g : 2 * m->ngp + (r - 2) * m->nmp + m->hidx[g]);
            }
        {  // every slot in range and written by one element-boundary node only
            std::vector<uint8_t> used((size_t)m->plane, 0);
            for (int64_t lb = 0; lb < nlb; ++lb) {
                const int32_t q = m->posmap[lb];
                if (q < 0 || q >= m->plane || used[q]) {
                    set_error("sel_mesh_create: internal error in contribution slots");
                    delete m;
                    return SEL_EINVAL;
                }
                used[q] = 1;
            }
        }
        m->dg = dg;
        if (dg) {
            if (int rc = build_interfaces(m)) {
                delete m;
                return rc;
            }
        }
    } catch (const std::bad_alloc &) {
        set_error("sel_mesh_create: out of host memory");
        delete m;
        return SEL_ENOMEM;
    }
    *out = m;
    return SEL_OK;
}

// Interfaces of the discontinuous coupling: every face that is not a wall is
// paired with the one other face carrying the same set of node ids, and each
// of its nodes with the node of equal id there.
static int build_interfaces(sel_mesh *m)
{
    const int n1 = m->n1, np = m->np, nface = m->nface, N = m->N;
    const int nfn = m->dim == 2 ? n1 : n1 * n1;
    const int64_t nf = m->E * nface;
    m->nfn = nfn;
    std::vector<std::vector<int>> fnode(nface);
    for (int p = 0; p < np; ++p) {
        const int ijk[3] = {p % n1, (p / n1) % n1, p / (n1 * n1)};
        for (int d = 0; d < m->dim; ++d) {
            if (ijk[d] == 0) fnode[2 * d].push_back(p);
            if (ijk[d] == N) fnode[2 * d + 1].push_back(p);
        }
    }
    std::vector<int64_t> ids((size_t)nf * nfn);
    std::vector<int64_t> faces;
    for (int64_t f = 0; f < nf; ++f) {
        if (m->ftag[f] > 0) continue;
        const int64_t e = f / nface;
        const int fc = (int)(f % nface);
        int64_t *v = ids.data() + f * nfn;
        for (int k = 0; k < nfn; ++k) v[k] = m->gid[e * np + fnode[fc][k]];
        std::sort(v, v + nfn);
        if (std::adjacent_find(v, v + nfn) != v + nfn) {
            set_error("sel_mesh_create_dg: a face repeats a node id (one element along a periodic direction)");
            return SEL_EINVAL;
        }
        faces.push_back(f);
    }
    auto less = [&](int64_t a, int64_t b) {
        return std::lexicographical_compare(ids.begin() + a * nfn, ids.begin() + (a + 1) * nfn, ids.begin() + b * nfn,
                                            ids.begin() + (b + 1) * nfn);
    };
    auto same = [&](int64_t a, int64_t b) { return std::equal(ids.begin() + a * nfn, ids.begin() + (a + 1) * nfn,
                                                              ids.begin() + b * nfn); };
    std::sort(faces.begin(), faces.end(), less);
    m->nbr.assign((size_t)nf * nfn, -1);
    for (size_t i = 0; i < faces.size(); i += 2) {
        if (i + 1 >= faces.size() || !same(faces[i], faces[i + 1]) ||
            (i + 2 < faces.size() && same(faces[i], faces[i + 2]))) {
            set_error("sel_mesh_create_dg: a face that is not a wall has no single partner face");
            return SEL_EINVAL;
        }
        for (int side = 0; side < 2; ++side) {
            const int64_t fa = faces[i + side], fb = faces[i + 1 - side];
            const int64_t ea = fa / nface, eb = fb / nface;
            const int fca = (int)(fa % nface), fcb = (int)(fb % nface);
            for (int k = 0; k < nfn; ++k) {
                const int64_t g = m->gid[ea * np + fnode[fca][k]];
                int pb = -1;
                for (int q : fnode[fcb])
                    if (m->gid[eb * np + q] == g) pb = q;
                if (pb < 0) {
                    set_error("sel_mesh_create_dg: internal error in the face matching");
                    return SEL_EINVAL;
                }
                const int bsl = -m->pcode[pb] - 1;
                m->nbr[fa * nfn + k] = m->bmap[eb * m->nbe + bsl];
            }
        }
    }
    return SEL_OK;
}

extern "C" int sel_mesh_create(int32_t dim, int32_t N, int64_t E, const double *xyz, const int64_t *gid,
                               const int32_t *face_tag, int32_t ntags, const double *wall_u, sel_mesh **out)
{
    return mesh_create(dim, N, E, xyz, gid, face_tag, ntags, wall_u, 0, out);
}

extern "C" int sel_mesh_create_dg(int32_t dim, int32_t N, int64_t E, const double *xyz, const int64_t *gid,
                                  const int32_t *face_tag, int32_t ntags, const double *wall_u, sel_mesh **out)
{
    return mesh_create(dim, N, E, xyz, gid, face_tag, ntags, wall_u, 1, out);
}

extern "C" int sel_mesh_destroy(sel_mesh *mesh)
{
    delete mesh;
    return SEL_OK;
}

extern "C" int sel_mesh_info(const sel_mesh *m, int64_t *info)
{
    if (!m || !info) {
        set_error("sel_mesh_info: null pointer argument");
        return SEL_EINVAL;
    }
    info[0] = m->dim;
    info[1] = m->N;
    info[2] = m->E;
    info[3] = m->np;
    info[4] = m->unique_nodes;
    info[5] = m->ngrp;
    info[6] = m->nbe;
    info[7] = m->nwall;
    return SEL_OK;
}
