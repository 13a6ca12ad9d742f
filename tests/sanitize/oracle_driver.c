/*
 * Driver for the sanitizer build of the oracle (address + undefined-behaviour
 * checks, CPU only).  Runs every exported oracle routine on small seeded
 * problems, including the degenerate ones (a single node, 1 x n strips,
 * every node a source, barriers walling sources in, duplicate sources,
 * per-axis spacing), and checks the cheap consistency facts that tie them
 * together (fast marching = fast sweeping = the serial Algorithm 2
 * emulation at the fixed point, in float64).  Exit status 0 = clean; the
 * sanitizers abort on the first finding.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double eo_godunov(int m, const double* a, double H);
float eo_godunov_f(int m, const float* a, float H);
double eo_godunov_bisect(int m, const double* a, double H);
double eo_godunov_aniso(int m, const double* a, const double* H);
int eo_apply_local(int ndim, const int64_t* dims, double h, const double* F, const double* phi, double* out);
int eo_apply_local_f(int ndim, const int64_t* dims, double h, const float* F, const float* phi, float* out);
int eo_apply_local_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F,
                     const double* phi, double* out);
int eo_fmm(int ndim, const int64_t* dims, double h, const double* F, const int64_t* src, const double* val,
           int64_t nsrc, double* phi, int64_t* accept_order, int64_t* n_accepted);
int eo_fmm_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F, const int64_t* src,
             const double* val, int64_t nsrc, double* phi, int64_t* accept_order, int64_t* n_accepted);
int eo_fsm(int ndim, const int64_t* dims, double h, const double* F, const int64_t* src, const double* val,
           int64_t nsrc, double* phi, int use_bisect, int64_t max_passes, int64_t* passes_out);
int eo_ifim(int ndim, const int64_t* dims, double h, const double* F, const int64_t* src, const double* sval,
            int64_t nsrc, double eps, int skip_remedy, int64_t max_iters, double* phi, int64_t* stats);
int eo_ifim_f(int ndim, const int64_t* dims, double h, const double* F, const int64_t* src, const double* sval,
              int64_t nsrc, double eps, int skip_remedy, int64_t max_iters, float* phi, int64_t* stats);
int eo_fim(int ndim, const int64_t* dims, double h, const double* F, const int64_t* src, const double* sval,
           int64_t nsrc, double eps, int64_t max_iters, double* phi, int64_t* stats);
int eo_adjoint(int ndim, const int64_t* dims, double h, const double* F, const int64_t* src, int64_t nsrc,
               const double* phi, const double* dL_dphi, double* dL_dF, double* lambda_out);
int eo_adjoint_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F, const int64_t* src,
                 int64_t nsrc, const double* phi, const double* dL_dphi, double* dL_dF, double* lambda_out);

static uint64_t rng_state = 2106;
static double urand(void) { /* splitmix64 -> [0, 1) */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                     \
            ++failures;                                \
        }                                              \
    } while (0)

static int same(double a, double b) { return a == b || (isinf(a) && isinf(b)) || fabs(a - b) <= 1e-13 * fabs(b); }

static void run_case(int nd, const int64_t* dims, double zero_frac, int nsrc, int all_sources) {
    int64_t n = 1;
    for (int k = 0; k < nd; ++k) n *= dims[k];
    double* F = malloc((size_t)n * sizeof(double));
    float* F32 = malloc((size_t)n * sizeof(float));
    double *p1 = malloc((size_t)n * 8), *p2 = malloc((size_t)n * 8), *p3 = malloc((size_t)n * 8);
    double *p4 = malloc((size_t)n * 8), *g = malloc((size_t)n * 8), *d = malloc((size_t)n * 8);
    double* lam = malloc((size_t)n * 8);
    float* p32 = malloc((size_t)n * 4);
    float* o32 = malloc((size_t)n * 4);
    int64_t* order = malloc((size_t)n * sizeof(int64_t));
    if (all_sources) nsrc = (int)n;
    int64_t* src = malloc((size_t)(nsrc + 1) * sizeof(int64_t));
    double* val = malloc((size_t)(nsrc + 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        F[i] = exp(log(1e-3) + urand() * (log(1e3) - log(1e-3)));
        if (urand() < zero_frac) F[i] = 0.0;
        F32[i] = (float)F[i];
        F[i] = (double)F32[i];
        g[i] = urand() < 0.2 ? urand() : 0.0;
    }
    for (int k = 0; k < nsrc; ++k) {
        src[k] = all_sources ? k : (int64_t)(urand() * (double)n);
        val[k] = urand() < 0.5 ? 0.0 : urand();
    }
    /* a duplicate source with another value: the minimum wins */
    src[nsrc] = src[0];
    val[nsrc] = val[0] + 1.0;
    const double h = 0.5 + urand();
    int64_t nacc = 0, passes = 0, st[7], fst[4];

    CHECK(eo_fmm(nd, dims, h, F, src, val, nsrc + 1, p1, order, &nacc) == 0, "fmm");
    CHECK(nacc <= n, "fmm accepted %lld of %lld", (long long)nacc, (long long)n);
    CHECK(eo_fsm(nd, dims, h, F, src, val, nsrc + 1, p2, 0, 100000, &passes) == 0, "fsm");
    CHECK(eo_ifim(nd, dims, h, F, src, val, nsrc + 1, 0.0, 0, 4 * n + 64, p3, st) == 0, "ifim");
    CHECK(eo_fim(nd, dims, h, F, src, val, nsrc + 1, 0.0, 4 * n + 64, p4, fst) == 0, "fim");
    for (int64_t i = 0; i < n; ++i) {
        CHECK(same(p1[i], p2[i]), "fmm vs fsm at %lld: %.17g %.17g", (long long)i, p1[i], p2[i]);
        CHECK(same(p1[i], p3[i]), "fmm vs ifim at %lld", (long long)i);
        CHECK(same(p1[i], p4[i]), "fmm vs fim at %lld", (long long)i);
    }
    CHECK(eo_ifim(nd, dims, h, F, src, val, nsrc + 1, 0.0, 1, 4 * n + 64, p3, st) == 0, "ifim skip");
    CHECK(eo_ifim_f(nd, dims, h, F, src, val, nsrc + 1, 0.0, 0, 4 * n + 64, p32, st) == 0, "ifim_f");
    CHECK(eo_apply_local(nd, dims, h, F, p1, p2) == 0, "apply_local");
    for (int64_t i = 0; i < n; ++i) p32[i] = (float)p1[i];
    CHECK(eo_apply_local_f(nd, dims, h, F32, p32, o32) == 0, "apply_local_f");
    (void)eo_fsm(nd, dims, h, F, src, val, nsrc + 1, p2, 1, 100000, &passes); /* bisection: exercised only */
    CHECK(eo_adjoint(nd, dims, h, F, src, nsrc + 1, p1, g, d, lam) == 0, "adjoint");
    CHECK(eo_adjoint(nd, dims, h, F, src, nsrc + 1, p1, g, d, NULL) == 0, "adjoint without lambda");
    double dsp[3] = {0.7, 1.3, 0.9};
    CHECK(eo_fmm_a(nd, dims, 1.0, dsp, F, src, val, nsrc + 1, p1, NULL, NULL) == 0, "fmm aniso");
    CHECK(eo_apply_local_a(nd, dims, 1.0, dsp, F, p1, p2) == 0, "apply_local aniso");
    CHECK(eo_adjoint_a(nd, dims, 1.0, dsp, F, src, nsrc + 1, p1, g, d, NULL) == 0, "adjoint aniso");
    /* the iteration caps are reported, not overrun */
    if (n > 4 && !all_sources) {
        int rc = eo_ifim(nd, dims, h, F, src, val, nsrc + 1, 0.0, 0, 1, p3, st);
        CHECK(rc == 0 || rc == 2, "ifim capped rc %d", rc);
        rc = eo_fsm(nd, dims, h, F, src, val, nsrc + 1, p2, 0, 1, &passes);
        CHECK(rc == 0 || rc == 2, "fsm capped rc %d", rc);
    }
    free(F); free(F32); free(p1); free(p2); free(p3); free(p4); free(g); free(d); free(lam);
    free(p32); free(o32); free(order); free(src); free(val);
}

int main(void) {
    /* local solvers on edge inputs */
    const double inf = INFINITY;
    double a3[3] = {0.0, inf, inf}, a2[2] = {inf, inf}, H3[3] = {1.0, 2.0, 0.5};
    CHECK(eo_godunov(3, a3, 1.0) == 1.0, "godunov one-sided");
    CHECK(isinf(eo_godunov(2, a2, 1.0)), "godunov all infinite");
    CHECK(isinf(eo_godunov(2, a3, inf)), "godunov barrier");
    float f3[3] = {0.f, 0.f, 0.5f};
    CHECK(fabsf(eo_godunov_f(3, f3, 1.f) - 0.69371294f) < 1e-6f, "godunov_f");
    CHECK(fabs(eo_godunov_bisect(3, a3, 1.0) - 1.0) < 1e-12, "bisect");
    CHECK(eo_godunov_aniso(3, a3, H3) == 1.0, "aniso one-sided");

    /* invalid shapes are rejected, not read */
    int64_t bad[3] = {0, 4, 4};
    double one = 1.0, out = 0.0;
    int64_t s0 = 0, s_out = 99;
    CHECK(eo_apply_local(2, bad, 1.0, &one, &one, &out) != 0, "zero dim rejected");
    CHECK(eo_apply_local(4, bad + 1, 1.0, &one, &one, &out) != 0, "ndim 4 rejected");
    int64_t d11[2] = {1, 1};
    CHECK(eo_fmm(2, d11, 1.0, &one, &s_out, NULL, 1, &out, NULL, NULL) != 0, "source out of range rejected");
    CHECK(eo_fmm(2, d11, 1.0, &one, &s0, NULL, 0, &out, NULL, NULL) != 0, "no source rejected");
    CHECK(eo_fmm(2, d11, 0.0, &one, &s0, NULL, 1, &out, NULL, NULL) != 0, "h = 0 rejected");

    /* degenerate and random grids */
    int64_t dims[3];
    dims[0] = 1; dims[1] = 1;
    run_case(2, dims, 0.0, 1, 0);
    dims[0] = 1; dims[1] = 37;
    run_case(2, dims, 0.0, 2, 0);
    dims[0] = 29; dims[1] = 1;
    run_case(2, dims, 0.1, 1, 0);
    dims[0] = 3; dims[1] = 4;
    run_case(2, dims, 0.0, 0, 1);
    dims[0] = 1; dims[1] = 1; dims[2] = 9;
    run_case(3, dims, 0.0, 1, 0);
    dims[0] = 2; dims[1] = 2; dims[2] = 2;
    run_case(3, dims, 0.0, 0, 1);
    for (int s = 0; s < 12; ++s) {
        dims[0] = 1 + (int64_t)(urand() * 24);
        dims[1] = 1 + (int64_t)(urand() * 24);
        run_case(2, dims, s % 3 == 0 ? 0.2 : 0.0, 1 + (int)(urand() * 8), 0);
    }
    for (int s = 0; s < 8; ++s) {
        dims[0] = 1 + (int64_t)(urand() * 9);
        dims[1] = 1 + (int64_t)(urand() * 9);
        dims[2] = 1 + (int64_t)(urand() * 9);
        run_case(3, dims, s % 2 == 0 ? 0.25 : 0.0, 1 + (int)(urand() * 8), 0);
    }
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: clean\n");
    return 0;
}
