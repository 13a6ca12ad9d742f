/*
 * eik_oracle.c -- plain, slow FP64 reference solvers for the discrete eikonal
 * system.  TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU baseline.  It shares no code with the GPU library.
 *
 * The problem (Eq 3): ||grad phi|| = 1/F on a uniform grid of spacing h.
 * The discrete system is the first-order Godunov upwind scheme (Eq 4 in 2D,
 * Eq 6 in 3D): for every node that is not a source,
 *
 *     sum_k [ (phi_i - a_k)^+ / h ]^2 = 1 / F_i^2,
 *     a_k = min(phi[i - e_k], phi[i + e_k])   (out-of-grid neighbour = +inf),
 *
 * and phi_s = v_s on sources.  The system has a unique solution for F > 0;
 * F = 0 marks a barrier cell (Example 4, Eq 8) whose value is +inf.
 *
 * Contents
 *   eo_godunov / eo_godunov_f : exact local solver of the equation above
 *       (the quantity Algorithms 1.1 and 1.3 compute), written in the shifted
 *       form b_k = a_k - a_1 to avoid cancellation.  Branch rule: add the m-th
 *       smallest a while the running root still exceeds it.
 *   eo_godunov_bisect         : the same root by bisection on the monotone
 *       residual -- an independent check of the closed form.
 *   eo_fmm   : fast marching (Section 2.1): heap-ordered acceptance, each
 *       tentative value computed from accepted neighbours only.  This is the
 *       plain definition of the result: the unique fixed point.
 *   eo_fsm   : fast sweeping (Section 2.2): Gauss-Seidel with the 2^d
 *       alternating orderings, repeated until a full pass changes nothing.
 *   eo_ifim  : the improved fast iterative method (Algorithm 2) emulated
 *       serially with synchronous (Jacobi) reads per iteration, in float64 or
 *       float32 arithmetic, with per-phase counters.
 *   eo_fim   : the fast iterative method the paper improves on (Section
 *       2.3), emulated serially: each iteration updates the active list with
 *       synchronous reads; a node whose value no longer changes leaves the
 *       list and each of its neighbours that is not active is evaluated at
 *       once -- if its value drops it takes the new value and (re)joins the
 *       active list.  Counters: iterations, active evaluations, neighbour-check
 *       evaluations, peak list length.
 *   *_a variants (eo_fmm_a, eo_fsm_a, eo_fim_a, eo_apply_local_a,
 *       eo_adjoint_a) take a per-axis spacing (Eq 5 with dx != dy, Algorithm
 *       1.2, and its 3D analogue), solved by eo_godunov_aniso.
 *   eo_adjoint : reverse sweep in fast-marching acceptance order giving
 *       dL/dF for a loss L(phi) (the linearised upwind system, transposed).
 *
 * Readings of the paper used here (the paper's text is the authority):
 *   - Algorithm 1.1/1.3 branch thresholds are replaced by the exact Godunov
 *     validity rule (the printed thresholds do not solve Eq 4 / Eq 6).
 *   - The "phi~ = phi" convergence test of Algorithm 2 is phi - phi~ <= eps.
 *   - "else phi = phi~" is phi = min(phi, phi~).
 *   - Remedy next set = changed nodes and their neighbours (the prose rule of
 *     Section 3.1.2), minus sources.
 *   - An active node whose update is +inf is not converged; it returns to FAR.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EO_OK 0
#define EO_BAD 1
#define EO_NOCONV 2
#define EO_NOMEM 3

typedef struct {
    int nd;
    int64_t d[3];
    int64_t s[3]; /* strides */
    int64_t n;
} grid_t;

static int grid_init(grid_t* g, int ndim, const int64_t* dims) {
    if (ndim < 1 || ndim > 3) return EO_BAD;
    g->nd = ndim;
    g->n = 1;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] < 1) return EO_BAD;
        g->d[k] = dims[k];
        g->n *= dims[k];
    }
    int64_t st = 1;
    for (int k = ndim - 1; k >= 0; --k) {
        g->s[k] = st;
        st *= g->d[k];
    }
    return EO_OK;
}

/* coordinate of flat index i along axis k */
static int64_t coord(const grid_t* g, int64_t i, int k) { return (i / g->s[k]) % g->d[k]; }

/* neighbours of i: writes up to 2*nd indices, returns count */
static int neighbours(const grid_t* g, int64_t i, int64_t* out) {
    int c = 0;
    for (int k = 0; k < g->nd; ++k) {
        int64_t x = coord(g, i, k);
        if (x > 0) out[c++] = i - g->s[k];
        if (x + 1 < g->d[k]) out[c++] = i + g->s[k];
    }
    return c;
}

/* ------------------------------------------------------------------------- */
/* Local solver                                                              */
/* ------------------------------------------------------------------------- */

double eo_godunov(int m, const double* a_in, double H) {
    double a[3];
    for (int k = 0; k < m; ++k) a[k] = a_in[k];
    /* insertion sort, ascending */
    for (int k = 1; k < m; ++k) {
        double v = a[k];
        int j = k - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
    if (!(H < INFINITY) || !(a[0] < INFINITY)) return INFINITY;
    double phi = a[0] + H;
    double S = 0.0, Q = 0.0;
    for (int k = 1; k < m; ++k) {
        if (!(phi > a[k])) break; /* a[k] not upwind: stop (also for a[k] = inf) */
        double b = a[k] - a[0];
        S += b;
        Q += b * b;
        double mm = (double)(k + 1);
        double disc = S * S - mm * (Q - H * H);
        if (disc < 0.0) disc = 0.0;
        phi = a[0] + (S + sqrt(disc)) / mm;
    }
    return phi;
}

float eo_godunov_f(int m, const float* a_in, float H) {
    float a[3];
    for (int k = 0; k < m; ++k) a[k] = a_in[k];
    for (int k = 1; k < m; ++k) {
        float v = a[k];
        int j = k - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
    if (!(H < INFINITY) || !(a[0] < INFINITY)) return INFINITY;
    float phi = a[0] + H;
    float S = 0.0f, Q = 0.0f;
    for (int k = 1; k < m; ++k) {
        if (!(phi > a[k])) break;
        float b = a[k] - a[0];
        S += b;
        Q += b * b;
        float mm = (float)(k + 1);
        float disc = S * S - mm * (Q - H * H);
        if (disc < 0.0f) disc = 0.0f;
        phi = a[0] + (S + sqrtf(disc)) / mm;
    }
    return phi;
}

/*
 * Anisotropic local solve (Eq 5 with dx != dy, the equation Algorithm 1.2
 * solves, and its 3D analogue): the root of
 *     sum_k ((phi - a_k)^+ / H_k)^2 = 1,   H_k = (spacing along axis k) / F,
 * by the same progressive rule on the a_k sorted ascending (each H_k travels
 * with its a_k), in shifted form: with t = phi - a_1, b_k = a_k - a_1 and
 * w_k = 1 / H_k^2 the active axes give A t^2 - 2 B t + C = 0,
 * A = sum w_k, B = sum w_k b_k, C = sum w_k b_k^2 - 1.
 */
double eo_godunov_aniso(int m, const double* a_in, const double* H_in) {
    double a[3], H[3];
    for (int k = 0; k < m; ++k) { a[k] = a_in[k]; H[k] = H_in[k]; }
    for (int k = 1; k < m; ++k) {
        double v = a[k], hv = H[k];
        int j = k - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; H[j + 1] = H[j]; --j; }
        a[j + 1] = v;
        H[j + 1] = hv;
    }
    if (!(a[0] < INFINITY) || !(H[0] < INFINITY)) return INFINITY;
    double phi = a[0] + H[0];
    double A = 1.0 / (H[0] * H[0]), B = 0.0, C = -1.0;
    for (int k = 1; k < m; ++k) {
        if (!(phi > a[k])) break;
        double b = a[k] - a[0];
        double w = 1.0 / (H[k] * H[k]);
        A += w;
        B += w * b;
        C += w * b * b;
        double disc = B * B - A * C;
        if (disc < 0.0) disc = 0.0;
        phi = a[0] + (B + sqrt(disc)) / A;
    }
    return phi;
}

float eo_godunov_aniso_f(int m, const float* a_in, const float* H_in) {
    float a[3], H[3];
    for (int k = 0; k < m; ++k) { a[k] = a_in[k]; H[k] = H_in[k]; }
    for (int k = 1; k < m; ++k) {
        float v = a[k], hv = H[k];
        int j = k - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; H[j + 1] = H[j]; --j; }
        a[j + 1] = v;
        H[j + 1] = hv;
    }
    if (!(a[0] < INFINITY) || !(H[0] < INFINITY)) return INFINITY;
    float phi = a[0] + H[0];
    float A = 1.0f / (H[0] * H[0]), B = 0.0f, C = -1.0f;
    for (int k = 1; k < m; ++k) {
        if (!(phi > a[k])) break;
        float b = a[k] - a[0];
        float w = 1.0f / (H[k] * H[k]);
        A += w;
        B += w * b;
        C += w * b * b;
        float disc = B * B - A * C;
        if (disc < 0.0f) disc = 0.0f;
        phi = a[0] + (B + sqrtf(disc)) / A;
    }
    return phi;
}

/* residual r(phi) = sum_k ((phi - a_k)^+)^2 - H^2, increasing in phi */
static double godunov_residual(int m, const double* a, double H, double phi) {
    double r = -H * H;
    for (int k = 0; k < m; ++k) {
        if (a[k] < phi) {
            double t = phi - a[k];
            r += t * t;
        }
    }
    return r;
}

double eo_godunov_bisect(int m, const double* a, double H) {
    double amin = INFINITY;
    for (int k = 0; k < m; ++k) if (a[k] < amin) amin = a[k];
    if (!(H < INFINITY) || !(amin < INFINITY)) return INFINITY;
    double lo = amin, hi = amin + H; /* r(lo) = -H^2 < 0, r(hi) >= 0 */
    for (int it = 0; it < 4000; ++it) {
        double mid = lo + 0.5 * (hi - lo);
        if (mid <= lo || mid >= hi) break;
        if (godunov_residual(m, a, H, mid) < 0.0) lo = mid; else hi = mid;
    }
    return hi;
}

/* gather a_k = min over each axis of the two neighbour values */
static void axis_mins(const grid_t* g, const double* phi, int64_t i, double* a) {
    for (int k = 0; k < g->nd; ++k) {
        int64_t x = coord(g, i, k);
        double v = INFINITY;
        if (x > 0 && phi[i - g->s[k]] < v) v = phi[i - g->s[k]];
        if (x + 1 < g->d[k] && phi[i + g->s[k]] < v) v = phi[i + g->s[k]];
        a[k] = v;
    }
}

static void axis_mins_f(const grid_t* g, const float* phi, int64_t i, float* a) {
    for (int k = 0; k < g->nd; ++k) {
        int64_t x = coord(g, i, k);
        float v = INFINITY;
        if (x > 0 && phi[i - g->s[k]] < v) v = phi[i - g->s[k]];
        if (x + 1 < g->d[k] && phi[i + g->s[k]] < v) v = phi[i + g->s[k]];
        a[k] = v;
    }
}

static double node_H(double h, double F) { return F > 0.0 ? h / F : INFINITY; }

/* G_i from the axis minima: isotropic spacing h, or per-axis spacing dsp
 * (axis order of dims) when dsp is not NULL */
static double local_solve(int nd, const double* a, double F, double h, const double* dsp) {
    if (!dsp) return eo_godunov(nd, a, node_H(h, F));
    if (!(F > 0.0)) return INFINITY;
    double Hk[3];
    for (int k = 0; k < nd; ++k) Hk[k] = dsp[k] / F;
    return eo_godunov_aniso(nd, a, Hk);
}

/* G_i(phi) for every node (sources included), FP64; dsp as local_solve */
int eo_apply_local_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F,
                     const double* phi, double* out) {
    grid_t g;
    if (grid_init(&g, ndim, dims)) return EO_BAD;
    double a[3];
    for (int64_t i = 0; i < g.n; ++i) {
        axis_mins(&g, phi, i, a);
        out[i] = local_solve(g.nd, a, F[i], h, dsp);
    }
    return EO_OK;
}

int eo_apply_local(int ndim, const int64_t* dims, double h, const double* F,
                   const double* phi, double* out) {
    return eo_apply_local_a(ndim, dims, h, NULL, F, phi, out);
}

/* ------------------------------------------------------------------------- */
/* Sources                                                                   */
/* ------------------------------------------------------------------------- */

/* phi <- +inf; sources get min of their given values; is_src marks them */
static int seed_sources(const grid_t* g, const int64_t* src, const double* val,
                        int64_t nsrc, double* phi, unsigned char* is_src) {
    for (int64_t i = 0; i < g->n; ++i) { phi[i] = INFINITY; is_src[i] = 0; }
    for (int64_t k = 0; k < nsrc; ++k) {
        int64_t s = src[k];
        if (s < 0 || s >= g->n) return EO_BAD;
        double v = val ? val[k] : 0.0;
        if (!is_src[s] || v < phi[s]) phi[s] = v;
        is_src[s] = 1;
    }
    return EO_OK;
}

/* ------------------------------------------------------------------------- */
/* Fast marching (binary min-heap with lazy deletion)                         */
/* ------------------------------------------------------------------------- */

typedef struct { double key; int64_t idx; } hnode;
typedef struct { hnode* a; int64_t n, cap; } heap_t;

static int heap_push(heap_t* h, double key, int64_t idx) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hnode* na = (hnode*)realloc(h->a, (size_t)nc * sizeof(hnode));
        if (!na) return EO_NOMEM;
        h->a = na;
        h->cap = nc;
    }
    int64_t c = h->n++;
    while (c > 0) {
        int64_t p = (c - 1) / 2;
        if (h->a[p].key <= key) break;
        h->a[c] = h->a[p];
        c = p;
    }
    h->a[c].key = key;
    h->a[c].idx = idx;
    return EO_OK;
}

static hnode heap_pop(heap_t* h) {
    hnode top = h->a[0];
    hnode last = h->a[--h->n];
    int64_t c = 0;
    for (;;) {
        int64_t l = 2 * c + 1;
        if (l >= h->n) break;
        int64_t r = l + 1;
        int64_t m = (r < h->n && h->a[r].key < h->a[l].key) ? r : l;
        if (h->a[m].key >= last.key) break;
        h->a[c] = h->a[m];
        c = m;
    }
    if (h->n > 0) h->a[c] = last;
    return top;
}

/* tentative value of i from ACCEPTED neighbours only */
static double tentative(const grid_t* g, const double* phi, const unsigned char* acc,
                        int64_t i, double F, double h, const double* dsp) {
    double a[3];
    for (int k = 0; k < g->nd; ++k) {
        int64_t x = coord(g, i, k);
        double v = INFINITY;
        if (x > 0 && acc[i - g->s[k]] && phi[i - g->s[k]] < v) v = phi[i - g->s[k]];
        if (x + 1 < g->d[k] && acc[i + g->s[k]] && phi[i + g->s[k]] < v) v = phi[i + g->s[k]];
        a[k] = v;
    }
    return local_solve(g->nd, a, F, h, dsp);
}

/*
 * eo_fmm: phi (length N) receives the solution; +inf where unreachable.
 * accept_order (nullable, length N) receives the flat indices in acceptance
 * order (sources first, in index order); *n_accepted its length.
 */
int eo_fmm_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F,
             const int64_t* src, const double* val, int64_t nsrc, double* phi,
             int64_t* accept_order, int64_t* n_accepted) {
    grid_t g;
    if (grid_init(&g, ndim, dims) || nsrc < 1 || !(h > 0.0)) return EO_BAD;
    unsigned char* acc = (unsigned char*)malloc((size_t)g.n);
    if (!acc) return EO_NOMEM;
    int rc = seed_sources(&g, src, val, nsrc, phi, acc);
    if (rc) { free(acc); return rc; }
    int64_t na = 0;
    if (accept_order)
        for (int64_t i = 0; i < g.n; ++i) if (acc[i]) accept_order[na++] = i;
    if (!accept_order) for (int64_t i = 0; i < g.n; ++i) na += acc[i];

    heap_t hp = {0, 0, 0};
    int64_t nb[6];
    for (int64_t i = 0; i < g.n && rc == EO_OK; ++i) {
        if (!acc[i]) continue;
        int c = neighbours(&g, i, nb);
        for (int t = 0; t < c; ++t) {
            int64_t j = nb[t];
            if (acc[j]) continue;
            double v = tentative(&g, phi, acc, j, F[j], h, dsp);
            if (v < phi[j]) {
                phi[j] = v;
                rc = heap_push(&hp, v, j);
            }
        }
    }
    while (hp.n > 0 && rc == EO_OK) {
        hnode top = heap_pop(&hp);
        int64_t i = top.idx;
        if (acc[i] || top.key != phi[i]) continue; /* stale entry */
        acc[i] = 1;
        if (accept_order) accept_order[na] = i;
        ++na;
        int c = neighbours(&g, i, nb);
        for (int t = 0; t < c; ++t) {
            int64_t j = nb[t];
            if (acc[j]) continue;
            double v = tentative(&g, phi, acc, j, F[j], h, dsp);
            if (v < phi[j]) {
                phi[j] = v;
                rc = heap_push(&hp, v, j);
            }
        }
    }
    free(hp.a);
    free(acc);
    if (n_accepted) *n_accepted = na;
    return rc;
}

int eo_fmm(int ndim, const int64_t* dims, double h, const double* F,
           const int64_t* src, const double* val, int64_t nsrc, double* phi,
           int64_t* accept_order, int64_t* n_accepted) {
    return eo_fmm_a(ndim, dims, h, NULL, F, src, val, nsrc, phi, accept_order, n_accepted);
}

/* ------------------------------------------------------------------------- */
/* Fast sweeping (Gauss-Seidel, 2^d alternating orderings)                    */
/* ------------------------------------------------------------------------- */

int eo_fsm_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F,
             const int64_t* src, const double* val, int64_t nsrc, double* phi,
             int use_bisect, int64_t max_passes, int64_t* passes_out) {
    grid_t g;
    if (grid_init(&g, ndim, dims) || nsrc < 1 || !(h > 0.0)) return EO_BAD;
    unsigned char* fixed = (unsigned char*)malloc((size_t)g.n);
    if (!fixed) return EO_NOMEM;
    int rc = seed_sources(&g, src, val, nsrc, phi, fixed);
    if (rc) { free(fixed); return rc; }
    int nord = 1 << g.nd;
    int64_t pass = 0;
    int changed = 1;
    double a[3];
    while (changed && pass < max_passes) {
        changed = 0;
        ++pass;
        for (int o = 0; o < nord; ++o) {
            /* ordering o: bit k set -> axis k runs backwards */
            for (int64_t t = 0; t < g.n; ++t) {
                int64_t i = 0, rem = t;
                for (int k = g.nd - 1; k >= 0; --k) {
                    int64_t x = rem % g.d[k];
                    rem /= g.d[k];
                    if (o & (1 << k)) x = g.d[k] - 1 - x;
                    i += x * g.s[k];
                }
                if (fixed[i]) continue;
                axis_mins(&g, phi, i, a);
                double v = (use_bisect && !dsp) ? eo_godunov_bisect(g.nd, a, node_H(h, F[i]))
                                                : local_solve(g.nd, a, F[i], h, dsp);
                if (v < phi[i]) { phi[i] = v; changed = 1; }
            }
        }
    }
    free(fixed);
    if (passes_out) *passes_out = pass;
    return changed ? EO_NOCONV : EO_OK;
}

int eo_fsm(int ndim, const int64_t* dims, double h, const double* F,
           const int64_t* src, const double* val, int64_t nsrc, double* phi,
           int use_bisect, int64_t max_passes, int64_t* passes_out) {
    return eo_fsm_a(ndim, dims, h, NULL, F, src, val, nsrc, phi, use_bisect, max_passes, passes_out);
}

/* ------------------------------------------------------------------------- */
/* IFIM (Algorithm 2) serial emulation, synchronous reads per iteration       */
/* ------------------------------------------------------------------------- */

enum { L_FAR = 0, L_ACTIVE = 1, L_CONV = 2, L_FIXED = 3 };

/* stats layout: [0] step2 iterations, [1] remedy iterations, [2] step2
 * evaluations, [3] detection evaluations, [4] remedy evaluations, [5] initial
 * remedy size, [6] peak active size */
#define EO_NSTATS 7

#define IFIM_BODY(T, GODUNOV, AXIS_MINS)                                           \
    grid_t g;                                                                      \
    if (grid_init(&g, ndim, dims) || nsrc < 1 || !(h > 0.0)) return EO_BAD;        \
    int64_t N = g.n;                                                               \
    unsigned char* lab = (unsigned char*)calloc((size_t)N, 1);                     \
    int64_t* A = (int64_t*)malloc((size_t)N * sizeof(int64_t));                    \
    int64_t* B = (int64_t*)malloc((size_t)N * sizeof(int64_t));                    \
    T* val = (T*)malloc((size_t)N * sizeof(T));                                    \
    int64_t* stamp = (int64_t*)malloc((size_t)N * sizeof(int64_t));                \
    double* tmp = (double*)malloc((size_t)N * sizeof(double));                     \
    if (!lab || !A || !B || !val || !stamp || !tmp) {                              \
        free(lab); free(A); free(B); free(val); free(stamp); free(tmp);            \
        return EO_NOMEM;                                                           \
    }                                                                              \
    for (int64_t k = 0; k < EO_NSTATS; ++k) stats[k] = 0;                           \
    int rc = seed_sources(&g, src, sval, nsrc, tmp, lab);                          \
    if (rc) goto done;                                                             \
    for (int64_t i = 0; i < N; ++i) {                                              \
        phi[i] = (T)tmp[i];                                                        \
        lab[i] = lab[i] ? L_FIXED : L_FAR;                                         \
        stamp[i] = -1;                                                             \
    }                                                                              \
    const T hT = (T)h;                                                             \
    const T epsT = (T)eps;                                                         \
    int64_t na = 0, nb_ = 0;                                                       \
    int64_t nbr[6];                                                                \
    T a[3];                                                                        \
    /* STEP 1: active set = FAR neighbours (F > 0) of the sources */               \
    for (int64_t i = 0; i < N; ++i) {                                              \
        if (lab[i] != L_FIXED) continue;                                           \
        int c = neighbours(&g, i, nbr);                                            \
        for (int t = 0; t < c; ++t) {                                              \
            int64_t j = nbr[t];                                                    \
            if (lab[j] == L_FAR && F[j] > 0.0) { lab[j] = L_ACTIVE; A[na++] = j; } \
        }                                                                          \
    }                                                                              \
    /* STEP 2: update without the neighbour convergence check */                  \
    while (na > 0) {                                                               \
        if (stats[0] >= max_iters) { rc = EO_NOCONV; goto done; }                  \
        stats[0] += 1;                                                             \
        stats[2] += na;                                                            \
        if (na > stats[6]) stats[6] = na;                                          \
        for (int64_t k = 0; k < na; ++k) {                                         \
            int64_t i = A[k];                                                      \
            AXIS_MINS(&g, phi, i, a);                                              \
            T Hi = F[i] > 0.0 ? hT / (T)F[i] : (T)INFINITY;                        \
            val[k] = GODUNOV(g.nd, a, Hi);                                         \
        }                                                                          \
        nb_ = 0;                                                                   \
        for (int64_t k = 0; k < na; ++k) {                                         \
            int64_t i = A[k];                                                      \
            T pt = val[k];                                                         \
            if (pt < (T)INFINITY && phi[i] - pt <= epsT) {                         \
                lab[i] = L_CONV;                                                   \
                int c = neighbours(&g, i, nbr);                                    \
                for (int t = 0; t < c; ++t) {                                      \
                    int64_t j = nbr[t];                                            \
                    if (lab[j] == L_FAR && F[j] > 0.0) {                           \
                        lab[j] = L_ACTIVE;                                         \
                        B[nb_++] = j;                                              \
                    }                                                              \
                }                                                                  \
            } else if (!(pt < (T)INFINITY)) {                                      \
                lab[i] = L_FAR;                                                    \
            } else {                                                               \
                if (pt < phi[i]) phi[i] = pt;                                      \
                B[nb_++] = i;                                                      \
            }                                                                      \
        }                                                                          \
        { int64_t* t_ = A; A = B; B = t_; na = nb_; }                              \
    }                                                                              \
    if (skip_remedy) goto done;                                                    \
    /* STEP 3a: recompute every non-source node, collect those that drop */        \
    na = 0;                                                                        \
    for (int64_t i = 0; i < N; ++i) {                                              \
        if (lab[i] == L_FIXED) continue;                                           \
        stats[3] += 1;                                                             \
        AXIS_MINS(&g, phi, i, a);                                                  \
        T Hi = F[i] > 0.0 ? hT / (T)F[i] : (T)INFINITY;                            \
        T pt = GODUNOV(g.nd, a, Hi);                                               \
        if (pt < phi[i] - epsT) A[na++] = i;                                       \
    }                                                                              \
    stats[5] = na;                                                                 \
    /* STEP 3b: remedy loop; next = changed nodes and their neighbours */          \
    {                                                                              \
        int64_t it = 0;                                                            \
        while (na > 0) {                                                           \
            if (stats[1] >= max_iters) { rc = EO_NOCONV; goto done; }              \
            stats[1] += 1;                                                         \
            stats[4] += na;                                                        \
            for (int64_t k = 0; k < na; ++k) {                                     \
                int64_t i = A[k];                                                  \
                AXIS_MINS(&g, phi, i, a);                                          \
                T Hi = F[i] > 0.0 ? hT / (T)F[i] : (T)INFINITY;                    \
                val[k] = GODUNOV(g.nd, a, Hi);                                     \
            }                                                                      \
            nb_ = 0;                                                               \
            for (int64_t k = 0; k < na; ++k) {                                     \
                int64_t i = A[k];                                                  \
                T pt = val[k];                                                     \
                if (pt < phi[i] - epsT) {                                          \
                    phi[i] = pt;                                                   \
                    if (stamp[i] != it) { stamp[i] = it; B[nb_++] = i; }           \
                    int c = neighbours(&g, i, nbr);                                \
                    for (int t = 0; t < c; ++t) {                                  \
                        int64_t j = nbr[t];                                        \
                        if (lab[j] != L_FIXED && stamp[j] != it) {                 \
                            stamp[j] = it;                                         \
                            B[nb_++] = j;                                          \
                        }                                                          \
                    }                                                              \
                }                                                                  \
            }                                                                      \
            { int64_t* t_ = A; A = B; B = t_; na = nb_; }                          \
            ++it;                                                                  \
        }                                                                          \
    }                                                                              \
done:                                                                              \
    free(lab); free(A); free(B); free(val); free(stamp); free(tmp);                \
    return rc;

int eo_ifim(int ndim, const int64_t* dims, double h, const double* F,
            const int64_t* src, const double* sval, int64_t nsrc, double eps,
            int skip_remedy, int64_t max_iters, double* phi, int64_t* stats) {
    IFIM_BODY(double, eo_godunov, axis_mins)
}

int eo_ifim_f(int ndim, const int64_t* dims, double h, const double* F,
              const int64_t* src, const double* sval, int64_t nsrc, double eps,
              int skip_remedy, int64_t max_iters, float* phi, int64_t* stats) {
    IFIM_BODY(float, eo_godunov_f, axis_mins_f)
}

/* ------------------------------------------------------------------------- */
/* Fast iterative method (Section 2.3)                                        */
/* ------------------------------------------------------------------------- */
int eo_fim_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F,
             const int64_t* src, const double* sval, int64_t nsrc, double eps,
             int64_t max_iters, double* phi, int64_t* stats) {
    grid_t g;
    if (grid_init(&g, ndim, dims) || nsrc < 1 || !(h > 0.0)) return EO_BAD;
    int64_t N = g.n;
    unsigned char* lab = (unsigned char*)calloc((size_t)N, 1);
    int64_t* A = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    int64_t* B = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    int64_t* C = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    double* val = (double*)malloc((size_t)N * sizeof(double));
    if (!lab || !A || !B || !C || !val) {
        free(lab); free(A); free(B); free(C); free(val);
        return EO_NOMEM;
    }
    for (int k = 0; k < 4; ++k) stats[k] = 0;
    int rc = seed_sources(&g, src, sval, nsrc, phi, lab);
    if (rc) goto done;
    for (int64_t i = 0; i < N; ++i) lab[i] = lab[i] ? L_FIXED : L_FAR;
    int64_t na = 0, nb = 0, nc = 0, nbr[6];
    double a[3];
    /* initialisation: the neighbours (F > 0) of the sources are active */
    for (int64_t i = 0; i < N; ++i) {
        if (lab[i] != L_FIXED) continue;
        int c = neighbours(&g, i, nbr);
        for (int t = 0; t < c; ++t) {
            int64_t j = nbr[t];
            if (lab[j] == L_FAR && F[j] > 0.0) { lab[j] = L_ACTIVE; A[na++] = j; }
        }
    }
    while (na > 0) {
        if (stats[0] >= max_iters) { rc = EO_NOCONV; goto done; }
        stats[0] += 1;
        stats[1] += na;
        if (na > stats[3]) stats[3] = na;
        /* update every active node from the values at the start of the iteration */
        for (int64_t k = 0; k < na; ++k) {
            int64_t i = A[k];
            axis_mins(&g, phi, i, a);
            val[k] = local_solve(g.nd, a, F[i], h, dsp);
        }
        nb = nc = 0;
        for (int64_t k = 0; k < na; ++k) {
            int64_t i = A[k];
            double pt = val[k];
            if (pt < INFINITY && phi[i] - pt <= eps) {
                lab[i] = L_CONV;          /* converged: leaves the active list */
                C[nc++] = i;
            } else if (!(pt < INFINITY)) {
                lab[i] = L_FAR;
            } else {
                if (pt < phi[i]) phi[i] = pt;
                B[nb++] = i;
            }
        }
        /* neighbour check of the converged nodes, after the update */
        for (int64_t k = 0; k < nc; ++k) {
            int c = neighbours(&g, C[k], nbr);
            for (int t = 0; t < c; ++t) {
                int64_t j = nbr[t];
                if (lab[j] == L_ACTIVE || lab[j] == L_FIXED || !(F[j] > 0.0)) continue;
                stats[2] += 1;
                axis_mins(&g, phi, j, a);
                double q = local_solve(g.nd, a, F[j], h, dsp);
                if (q < phi[j] - eps) {
                    phi[j] = q;
                    lab[j] = L_ACTIVE;
                    B[nb++] = j;
                }
            }
        }
        { int64_t* t_ = A; A = B; B = t_; na = nb; }
    }
done:
    free(lab); free(A); free(B); free(C); free(val);
    return rc;
}

int eo_fim(int ndim, const int64_t* dims, double h, const double* F,
           const int64_t* src, const double* sval, int64_t nsrc, double eps,
           int64_t max_iters, double* phi, int64_t* stats) {
    return eo_fim_a(ndim, dims, h, NULL, F, src, sval, nsrc, eps, max_iters, phi, stats);
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the converged discrete system                                   */
/* ------------------------------------------------------------------------- */
/*
 * At the solution, every reached non-source node i with F_i > 0 satisfies
 *   sum_{k in U_i} w_ik^2 = H_i^2,   w_ik = phi_i - phi_{j_k},  H_i = h / F_i,
 * where U_i are the upwind axes (a_k < phi_i) and j_k the neighbour attaining
 * a_k (lower flat index on a tie).  Differentiating:
 *   dphi_i = sum_k (w_ik / W_i) dphi_{j_k} - H_i^2 / (F_i W_i) dF_i,
 *   W_i = sum_k w_ik.
 * With dphi = M dphi + D dF (M strictly upwind), dL/dF = D lambda where
 * lambda = g + M^T lambda is solved downwind-to-upwind (decreasing phi).
 */

/* qsort's comparator reads the values through this pointer; one per thread,
 * so that callers may run the adjoint of different grids concurrently. */
static _Thread_local const double* g_sort_key;
static int cmp_desc(const void* x, const void* y) {
    double a = g_sort_key[*(const int64_t*)x], b = g_sort_key[*(const int64_t*)y];
    if (a > b) return -1;
    if (a < b) return 1;
    int64_t i = *(const int64_t*)x, j = *(const int64_t*)y;
    return (i < j) ? -1 : (i > j);
}

int eo_adjoint_a(int ndim, const int64_t* dims, double h, const double* dsp, const double* F,
                 const int64_t* src, int64_t nsrc, const double* phi,
                 const double* dL_dphi, double* dL_dF, double* lambda_out) {
    grid_t g;
    if (grid_init(&g, ndim, dims) || nsrc < 1 || !(h > 0.0)) return EO_BAD;
    int64_t N = g.n;
    unsigned char* is_src = (unsigned char*)calloc((size_t)N, 1);
    int64_t* ord = (int64_t*)malloc((size_t)N * sizeof(int64_t));
    double* lam = lambda_out ? lambda_out : (double*)malloc((size_t)N * sizeof(double));
    if (!is_src || !ord || !lam) {
        free(is_src); free(ord); if (!lambda_out) free(lam);
        return EO_NOMEM;
    }
    for (int64_t k = 0; k < nsrc; ++k) {
        if (src[k] < 0 || src[k] >= N) { free(is_src); free(ord); if (!lambda_out) free(lam); return EO_BAD; }
        is_src[src[k]] = 1;
    }
    int64_t m = 0;
    for (int64_t i = 0; i < N; ++i) {
        lam[i] = dL_dphi[i];
        dL_dF[i] = 0.0;
        if (!is_src[i] && phi[i] < INFINITY && F[i] > 0.0) ord[m++] = i;
    }
    g_sort_key = phi;
    qsort(ord, (size_t)m, sizeof(int64_t), cmp_desc);
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = ord[t];
        double pi = phi[i];
        int64_t jk[3];
        double wk[3];
        int nu = 0;
        double W = 0.0;
        for (int k = 0; k < g.nd; ++k) {
            int64_t x = coord(&g, i, k);
            int64_t best = -1;
            double v = INFINITY;
            if (x > 0 && phi[i - g.s[k]] < v) { v = phi[i - g.s[k]]; best = i - g.s[k]; }
            if (x + 1 < g.d[k] && phi[i + g.s[k]] < v) { v = phi[i + g.s[k]]; best = i + g.s[k]; }
            if (best >= 0 && v < pi) {
                /* per-axis spacing: the equation weighs axis k by 1/dsp_k^2 */
                jk[nu] = best;
                wk[nu] = dsp ? (pi - v) / (dsp[k] * dsp[k]) : pi - v;
                W += wk[nu];
                ++nu;
            }
        }
        if (nu == 0 || !(W > 0.0)) continue;
        double li = lam[i];
        if (dsp) {
            dL_dF[i] = -li / (F[i] * F[i] * F[i] * W);
        } else {
            double H = h / F[i];
            dL_dF[i] = -li * H * H / (F[i] * W);
        }
        for (int u = 0; u < nu; ++u) lam[jk[u]] += (wk[u] / W) * li;
    }
    free(is_src);
    free(ord);
    if (!lambda_out) free(lam);
    return EO_OK;
}

int eo_adjoint(int ndim, const int64_t* dims, double h, const double* F,
               const int64_t* src, int64_t nsrc, const double* phi,
               const double* dL_dphi, double* dL_dF, double* lambda_out) {
    return eo_adjoint_a(ndim, dims, h, NULL, F, src, nsrc, phi, dL_dphi, dL_dF, lambda_out);
}

/* G_i(phi) with per-axis spacing in float32 arithmetic */
int eo_apply_local_af(int ndim, const int64_t* dims, const double* dsp, const float* F,
                      const float* phi, float* out) {
    grid_t g;
    if (grid_init(&g, ndim, dims)) return EO_BAD;
    float a[3], Hk[3];
    for (int64_t i = 0; i < g.n; ++i) {
        axis_mins_f(&g, phi, i, a);
        if (F[i] > 0.0f) {
            for (int k = 0; k < g.nd; ++k) Hk[k] = (float)dsp[k] / F[i];
            out[i] = eo_godunov_aniso_f(g.nd, a, Hk);
        } else {
            out[i] = INFINITY;
        }
    }
    return EO_OK;
}

/* G_i(phi) for every node in float32 arithmetic (phi, F float32 values) */
int eo_apply_local_f(int ndim, const int64_t* dims, double h, const float* F,
                     const float* phi, float* out) {
    grid_t g;
    if (grid_init(&g, ndim, dims)) return EO_BAD;
    float a[3];
    const float hf = (float)h;
    for (int64_t i = 0; i < g.n; ++i) {
        axis_mins_f(&g, phi, i, a);
        float Hi = F[i] > 0.0f ? hf / F[i] : INFINITY;
        out[i] = eo_godunov_f(g.nd, a, Hi);
    }
    return EO_OK;
}
