// Host-only driver of the library's mesh ingest and table construction, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by the CPU test suite
// (no device code is compiled or run). Usage:
//   ingest_main <mesh file> <expected return code> <dg 0|1>
// The mesh file holds int64 dim, N, E, ntags, then xyz [E][np][dim] (FP64),
// gid [E][np] (int64), face_tag [E][2 dim] (int32), wall_u [ntags][dim] (FP64).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "sel_internal.h"

namespace sel {
static std::string g_msg;
void set_error(const std::string &msg) { g_msg = msg; }
}  // namespace sel

template <typename T>
static bool rd(FILE *f, std::vector<T> &v, size_t n)
{
    v.resize(n);
    return fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char **argv)
{
    if (argc != 4) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<int64_t> hdr;
    if (!rd(f, hdr, 4)) return 2;
    const int dim = (int)hdr[0], N = (int)hdr[1], ntags = (int)hdr[3];
    const int64_t E = hdr[2];
    int64_t np = 1;
    for (int k = 0; k < dim; ++k) np *= N + 1;
    std::vector<double> xyz, wu;
    std::vector<int64_t> gid;
    std::vector<int32_t> ft;
    if (!rd(f, xyz, (size_t)(E * np * dim)) || !rd(f, gid, (size_t)(E * np)) || !rd(f, ft, (size_t)(E * 2 * dim)) ||
        !rd(f, wu, (size_t)ntags * dim))
        return 2;
    fclose(f);
    const int expect = atoi(argv[2]);
    sel_mesh *m = nullptr;
    const int rc = atoi(argv[3]) ? sel_mesh_create_dg(dim, N, E, xyz.data(), gid.data(), ft.data(), ntags,
                                                      ntags ? wu.data() : nullptr, &m)
                                 : sel_mesh_create(dim, N, E, xyz.data(), gid.data(), ft.data(), ntags,
                                                   ntags ? wu.data() : nullptr, &m);
    if (rc != expect) {
        fprintf(stderr, "rc %d expected %d: %s\n", rc, expect, sel::g_msg.c_str());
        return 1;
    }
    if (rc == SEL_OK) {
        int64_t info[8];
        if (sel_mesh_info(m, info) != SEL_OK || info[2] != E) return 1;
        sel_mesh_destroy(m);
    }
    // the element tables at every order the mesh ingest accepts
    for (int n = 2; n + 1 <= sel::kMaxN1; ++n) {
        sel::Tables t;
        if (sel::build_gll(n, t)) return 1;
        if (sel::build_filter(n, SEL_FILTER_QUAD, 2 < n ? 2 : n - 1, 0.1, 2.0, t)) return 1;
        if (sel::build_filter(n, SEL_FILTER_EXP, (2 * n) / 3, 36.0, 16.0, t)) return 1;
        std::vector<double> P((size_t)(n + 1) * (n + 1));
        for (int nc = 1; nc <= n; ++nc)
            if (sel::build_projection(n, nc, P.data())) return 1;
    }
    sel::HostLattice L;
    if (sel::build_lattice(2, 9, L) || sel::build_lattice(3, 19, L) || sel::build_lattice(3, 27, L)) return 1;
    printf("ok\n");
    return 0;
}
