/* Driver of the FP64 oracle built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by the CPU test suite. Usage:
 *   oracle_main <case file> <steps>
 * The case file holds int64 dim, N, E, Q, ntags, filter type, kc, rk,
 * coupling, then FP64 rho0, nu, dt, g[3], famp, forder, then xyz [E][np][dim]
 * (FP64), gid [E][np] (int64), face_tag [E][2 dim] (int32), wall_u
 * [max(ntags,1)][dim] (FP64), rho [E][np], u [E][np][dim] (FP64). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_sim oracle_sim;
oracle_sim *oracle_create(int dim, int N, int64_t E, const double *xyz, const int64_t *gid, const int32_t *face_tag,
                          int ntags, const double *wall_u, int Q, double rho0, double nu, double dt, const double *g,
                          int filter_type, int kc, double famp, double forder, int rk, int coupling);
void oracle_destroy(oracle_sim *s);
int oracle_init(oracle_sim *s, const double *rho, const double *u);
int oracle_step(oracle_sim *s, int64_t nsteps);
int oracle_advect(oracle_sim *s, int64_t nsteps);
int oracle_moments(const oracle_sim *s, double *rho, double *u);
int oracle_reduce(const oracle_sim *s, double *out);
int oracle_get_f(const oracle_sim *s, double *f);
int oracle_rhs(oracle_sim *s, const double *f, double *r);
int oracle_rhs_local(oracle_sim *s, const double *f, double *rt);
int oracle_collide(oracle_sim *s, const double *f, double *fs);
int oracle_filter(oracle_sim *s, const double *f, double *out);
int oracle_set_force(oracle_sim *s, const double *F);
void oracle_set_threads(int n);

static void *rd(FILE *f, size_t size, size_t n)
{
    void *p = malloc(size * (n ? n : 1));
    if (!p || fread(p, size, n, f) != n) exit(2);
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t *h = rd(f, 8, 9);
    double *pr = rd(f, 8, 8);
    const int dim = (int)h[0], N = (int)h[1], Q = (int)h[3], ntags = (int)h[4];
    const int64_t E = h[2];
    int64_t np = 1;
    for (int k = 0; k < dim; ++k) np *= N + 1;
    double *xyz = rd(f, 8, (size_t)(E * np * dim));
    int64_t *gid = rd(f, 8, (size_t)(E * np));
    int32_t *ft = rd(f, 4, (size_t)(E * 2 * dim));
    double *wu = rd(f, 8, (size_t)((ntags ? ntags : 1) * dim));
    double *rho = rd(f, 8, (size_t)(E * np));
    double *u = rd(f, 8, (size_t)(E * np * dim));
    fclose(f);
    oracle_set_threads(1);
    oracle_sim *s = oracle_create(dim, N, E, xyz, gid, ft, ntags, wu, Q, pr[0], pr[1], pr[2], pr + 3, (int)h[5],
                                  (int)h[6], pr[6], pr[7], (int)h[7], (int)h[8]);
    if (!s) return 1;
    oracle_init(s, rho, u);
    const size_t nv = (size_t)(E * Q * np);
    double *fa = malloc(8 * nv), *fb = malloc(8 * nv), *F = malloc(8 * (size_t)(E * np * dim));
    double red[8];
    for (size_t i = 0; i < (size_t)(E * np * dim); ++i) F[i] = 1e-4 * (double)(i % 7);
    oracle_step(s, atoi(argv[2]));
    oracle_set_force(s, F);
    oracle_step(s, 2);
    oracle_set_force(s, NULL);
    oracle_advect(s, 1);
    oracle_moments(s, rho, u);
    oracle_reduce(s, red);
    oracle_get_f(s, fa);
    oracle_rhs(s, fa, fb);
    oracle_rhs_local(s, fa, fb);
    oracle_collide(s, fa, fb);
    oracle_filter(s, fa, fb);
    oracle_destroy(s);
    printf("ok %.17g\n", red[0]);
    free(h), free(pr), free(xyz), free(gid), free(ft), free(wu), free(rho), free(u), free(fa), free(fb), free(F);
    return 0;
}
