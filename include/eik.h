/*
 * eik.h -- C ABI of the MI355X (gfx950) eikonal solver library libeik.so.
 *
 * The library solves the eikonal equation ||grad phi|| = 1/F (Eq 3) on a
 * uniform 2D or 3D grid with the improved fast iterative method (Algorithm 2):
 * an active-list update without the neighbour convergence check (STEP 2),
 * followed by the error-correction pass that recomputes every node, collects
 * the ones whose value drops into a remedy list and iterates it to a fixed
 * point (STEP 3).  The discrete system solved is the first-order Godunov upwind
 * scheme (Eq 4 in 2D, Eq 6 in 3D) with isotropic spacing h, whose exact local
 * solve is what Algorithms 1.1 and 1.3 compute.
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers (memory on the current HIP device)
 *     unless marked "host".  The caller owns every buffer; the library never
 *     frees caller memory.
 *   - dims (host) lists the grid extents in C order, last axis fastest (x is
 *     contiguous): (ny, nx) for ndim = 2, (nz, ny, nx) for ndim = 3.  Flat
 *     index = ((i0 * d1) + i1) * d2 + i2.  The total node count must be below
 *     2^31.
 *   - F, phi and the adjoint arrays share one element type, chosen by
 *     eik_options.dtype (float32 or float64), and the same shape.
 *   - F >= 0 and finite.  F = 0 marks a barrier cell (Eq 8): its value is +inf
 *     unless it is a source.  Unreachable nodes come out as +inf.
 *   - Sources (host, flat indices) are fixed nodes with given values (default
 *     0).  Duplicated indices keep their minimum value.
 *   - Work is enqueued on eik_options.stream (NULL: the default stream).
 *     Unless EIK_FLAG_ASYNC is set, calls return after the device work has
 *     completed.
 *   - Every function returns an eik_status; none aborts.  Validation errors
 *     are reported before any device work and leave the outputs untouched.
 *     eik_last_error() gives a per-thread description of the last failure.
 */
#ifndef EIK_H_
#define EIK_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EIK_ABI_VERSION 8

typedef enum {
    EIK_OK = 0,
    EIK_ERR_INVALID_ARGUMENT = 1, /* bad shape, spacing, sources, F values, options */
    EIK_ERR_NO_CONVERGENCE = 2,   /* iteration cap reached; output holds the current
                                     iterate, an upper bound of the solution */
    EIK_ERR_OUT_OF_MEMORY = 3,    /* workspace too small or device allocation failed */
    EIK_ERR_DEVICE = 4,           /* a HIP runtime call failed */
    EIK_ERR_UNSUPPORTED = 5       /* valid request this build does not implement */
} eik_status;

typedef enum { EIK_FLOAT32 = 0, EIK_FLOAT64 = 1 } eik_dtype;

typedef enum {
    /* One lane per list entry over global node lists: the paper's mapping of
       one thread per active point (Section 3.2). */
    EIK_VARIANT_NODE_LIST = 0,
    /* Same node rules scheduled tile by tile: each workgroup stages a tile and
       its one-cell halo in LDS and runs several inner iterations per launch. */
    EIK_VARIANT_TILE = 1,
    /* The fast iterative method the paper improves on (Section 2.3), on the
       same node lists: a node that converges has its non-active neighbours
       evaluated at once, and any whose value drops (re)joins the active list;
       there is no remedy step.  Same fixed point; a comparison baseline. */
    EIK_VARIANT_FIM = 2
} eik_variant;

enum {
    /* Synchronous reads per iteration (every update of an iteration sees the
       previous iteration's values); bitwise reproducible.  Node-list only. */
    EIK_FLAG_DETERMINISTIC = 1u,
    /* Diagnostic: return after the update step, skipping the remedy step
       (not with EIK_VARIANT_FIM, which has none). */
    EIK_FLAG_SKIP_REMEDY = 2u,
    /* Enqueue only: no host synchronisation, no stats.  The caller must pass
       a workspace and an explicit max_iters, which every loop then runs in
       full (launches after convergence find empty lists and return at once);
       eik_async_status reads the outcome once the stream has run the work. */
    EIK_FLAG_ASYNC = 4u,
    /* Bracket every kernel launch with HIP events on the solve's stream and
       report per-kind device time in eik_stats (adds host overhead). */
    EIK_FLAG_PROFILE = 8u,
    /* Tile variant: run the remedy loop first-in first-out, every queued tile
       in every launch.  By default each remedy launch instead processes the
       queued tiles whose pending values are lowest (about a thousand, chosen
       by a histogram of per-tile keys) and defers the others, so corrections
       flow roughly in increasing value and fewer nodes are corrected twice.
       Same rules and fixed point either way. */
    EIK_FLAG_FIFO_REMEDY = 16u,
    /* 3D tile variant: run the update step alone.  By default the persistent
       workgroups that find no update-step tile in a launch run remedy visits
       meanwhile (every node of a tile whose update visits left no active
       node, first-in first-out, stopping when the launch's update visits are
       done), so corrections start behind the front instead of after the
       step; the detection pass and remedy loop that follow are unchanged
       and decide the fixed point (eik_stats.evals_early counts these
       evaluations). */
    EIK_FLAG_NO_EARLY_REMEDY = 32u
};

/* Kernel kinds of eik_stats.kernel_ms / kernel_launches. */
enum {
    EIK_KERNEL_UPDATE = 0,  /* update-step launches */
    EIK_KERNEL_DETECT = 1,  /* whole-grid remedy detection */
    EIK_KERNEL_REMEDY = 2,  /* remedy-loop launches */
    EIK_KERNEL_ADJOINT = 3, /* adjoint propagation launches */
    EIK_KERNEL_OTHER = 4,   /* initialisation, seeding, dense adjoint passes */
    EIK_KERNEL_KINDS = 5
};

/* Work counters of one solve (filled when eik_options.stats is non-NULL). */
typedef struct {
    int64_t step2_iters;    /* update-step iterations (node-list) or launches (tile) */
    int64_t step3_iters;    /* remedy iterations / launches */
    int64_t evals_step2;    /* local-solver evaluations in the update step */
    int64_t evals_detect;   /* evaluations in the whole-grid remedy detection */
    int64_t evals_remedy;   /* evaluations in the remedy loop */
    int64_t remedy_initial; /* nodes (node-list) or tiles (tile) flagged by detection */
    int64_t max_active;     /* peak active-list length (nodes or tiles) */
    int64_t launches;       /* kernel launches enqueued */
    int64_t tile_visits_step2;  /* tile variant: tiles processed in the update step */
    int64_t tile_visits_step3;  /* tile variant: tiles processed in the remedy loop */
    int64_t inner_step2;        /* tile variant: inner iterations summed over visits */
    int64_t inner_step3;
    int64_t written_step2;      /* node values written back to HBM in the update step */
    int64_t written_step3;      /* ... in the remedy loop */
    int64_t evals_check;        /* FIM: evaluations of neighbours of converged nodes */
    int64_t evals_early;        /* 3D tile variant: remedy evaluations run during the update step */
    int64_t kernel_launches[EIK_KERNEL_KINDS]; /* with EIK_FLAG_PROFILE */
    double kernel_ms[EIK_KERNEL_KINDS];        /* with EIK_FLAG_PROFILE: summed device time */
} eik_stats;

typedef struct {
    eik_dtype dtype;           /* element type of F / phi (default float32) */
    eik_variant variant;       /* default EIK_VARIANT_TILE */
    int32_t tile[3];           /* tile extents (z, y, x); 0 = library default
                                  (8^3 in 3D; in 2D 16 x 16, with the update
                                  step on 32 x 32); an explicit shape applies
                                  to every step */
    int32_t inner_iters;       /* tile variant: inner iterations per tile visit; 0 = default:
                                  4 x the sum of the tile sides, except the
                                  longest side in the 2D update step */
    int64_t max_iters;         /* cap per loop (0 = default 4 * N + 64) */
    uint32_t flags;            /* EIK_FLAG_* */
    const double* source_values; /* host, n_sources entries; NULL -> all 0 */
    void* workspace;           /* device scratch of workspace_bytes; NULL -> the
                                  library allocates and frees it per call */
    size_t workspace_bytes;
    void* stream;              /* hipStream_t; NULL -> default stream */
    eik_stats* stats;          /* host, nullable */
    double spacing[3];         /* per-axis grid spacing in dims order (Eq 5 with
                                  dx != dy, Algorithm 1.2, and its 3D analogue):
                                  all zero -> the isotropic h argument; else the
                                  first ndim entries must be finite and > 0 and
                                  replace h (which must still be valid) */
    int32_t order_min;         /* tile variant, ordered remedy: a remedy launch
                                  takes at least this many of the queued tiles
                                  with the lowest keys; 0 = default (1024 in 3D,
                                  512 in 2D) */
    int32_t workgroups;        /* tile variant: persistent workgroups per tile
                                  launch, a multiple of 8 up to 2048; 0 = default
                                  (1536 in 3D: six resident per CU on 256 CUs;
                                  2048 in 2D) */
} eik_options;

/* Fill *opt with the defaults listed above.  Never fails. */
void eik_default_options(eik_options* opt);

/* Device workspace (bytes) eik_solve needs for this shape and options; 0 on
   invalid arguments.  Host-only; no device work. */
size_t eik_workspace_size(int32_t ndim, const int64_t* dims, const eik_options* opt);

/*
 * eik_solve -- Algorithm 2 (STEP 1 initialisation, STEP 2 update, STEP 3
 * remedy) for the Godunov system of Eq 4 / Eq 6.
 *   F        device, N elements, speed (>= 0, finite)
 *   ndim     2 or 3; dims (host) as above; h > 0 finite grid spacing
 *   sources  host, n_sources >= 1 flat indices in [0, N)
 *   eps      >= 0; a node counts as converged when phi - phi~ <= eps and is
 *            flagged by the remedy when phi~ < phi - eps (0 = exact equality)
 *   phi_out  device, N elements, receives the solution
 *   opt      nullable -> defaults
 * Errors: EIK_ERR_INVALID_ARGUMENT (arguments, or F negative / non-finite as
 * found on the device), EIK_ERR_NO_CONVERGENCE, EIK_ERR_OUT_OF_MEMORY,
 * EIK_ERR_DEVICE.
 */
eik_status eik_solve(const void* F, int32_t ndim, const int64_t* dims, double h,
                     const int64_t* sources, int64_t n_sources, double eps,
                     void* phi_out, const eik_options* opt);

/*
 * eik_apply_local -- one dense pass of the local solver: out_i = G_i(phi),
 * the exact root of Eq 4 / Eq 6 at node i given its neighbours' values
 * (out-of-grid neighbours +inf), for every node including sources.  This is
 * the "calculate phi~ for all grid points" pass of STEP 3.
 *   F, phi device inputs (N elements); out device output (N elements, may not
 *   alias phi).  opt: dtype and stream are used.
 */
eik_status eik_apply_local(const void* F, const void* phi, int32_t ndim, const int64_t* dims,
                           double h, void* out, const eik_options* opt);

/*
 * eik_adjoint -- gradient of a loss L(phi) with respect to F at a converged
 * solution phi of eik_solve (same F, h, sources).  At the solution each
 * reached non-source node satisfies sum_k w_ik^2 = (h/F_i)^2 over its upwind
 * axes (w_ik = phi_i - phi_upwind, a neighbour on the lower-index side on a
 * tie); the linearised system is transposed and solved downwind-to-upwind:
 *   lambda = dL/dphi + M^T lambda,  M_ij = w_ij / W_i,  W_i = sum_k w_ik,
 *   dL/dF_i = -lambda_i (h/F_i)^2 / (F_i W_i);  0 at sources and +inf nodes.
 * (Not in the paper: the derivative of the Eq 4 / Eq 6 fixed point.)
 *   F, phi, dL_dphi device inputs (N); dL_dF_out device output (N, no alias).
 *   opt: dtype, stream, workspace (eik_adjoint_workspace_size bytes; NULL ->
 *   allocated per call), max_iters, inner_iters, stats, EIK_FLAG_ASYNC.
 * Errors as eik_solve.
 */
eik_status eik_adjoint(const void* F, const void* phi, int32_t ndim, const int64_t* dims,
                       double h, const int64_t* sources, int64_t n_sources,
                       const void* dL_dphi, void* dL_dF_out, const eik_options* opt);

/* Device workspace (bytes) eik_adjoint needs; 0 on invalid arguments. */
size_t eik_adjoint_workspace_size(int32_t ndim, const int64_t* dims, const eik_options* opt);

/* One grid of a batch (eik_solve_batch / eik_adjoint_batch). */
typedef struct {
    int64_t dims[3];   /* extents in C order: (ny, nx, ignored) for ndim = 2,
                          (nz, ny, nx) for ndim = 3 */
    double h;          /* grid spacing of this grid (> 0, finite) */
    int64_t n_sources; /* >= 1: this grid's sources are the next n_sources
                          entries of the sources array */
} eik_instance;

/*
 * eik_solve_batch -- eik_solve for n_inst independent grids in one call: the
 * grids' tiles share the work lists of every launch, so small grids fill the
 * GPU together and the loops run until the slowest grid is done.  Tile
 * variant only (EIK_ERR_UNSUPPORTED otherwise).
 *   F, phi_out  device, the grids back to back in the order of inst (grid k
 *               starts after the nodes of grids 0..k-1), C order within a grid
 *   ndim        2 or 3, shared by all grids
 *   inst        host, n_inst >= 1 descriptions
 *   sources     host, flat indices local to their grid, grouped by grid
 *               (sum of inst[k].n_sources entries)
 *   opt         as eik_solve; opt->source_values (if set) is parallel to
 *               sources; stats are summed over the batch
 * The total node count must be below 2^31.  Errors as eik_solve.
 */
eik_status eik_solve_batch(const void* F, int32_t ndim, const eik_instance* inst, int32_t n_inst,
                           const int64_t* sources, double eps, void* phi_out, const eik_options* opt);

/* Device workspace (bytes) eik_solve_batch needs; 0 on invalid arguments. */
size_t eik_batch_workspace_size(int32_t ndim, const eik_instance* inst, int32_t n_inst,
                                const eik_options* opt);

/*
 * eik_adjoint_batch -- eik_adjoint for the grids of a batch (same layout as
 * eik_solve_batch): dL_dphi and dL_dF_out hold the grids back to back.
 */
eik_status eik_adjoint_batch(const void* F, const void* phi, int32_t ndim, const eik_instance* inst,
                             int32_t n_inst, const int64_t* sources, const void* dL_dphi, void* dL_dF_out,
                             const eik_options* opt);

/* Device workspace (bytes) eik_adjoint_batch needs; 0 on invalid arguments. */
size_t eik_adjoint_batch_workspace_size(int32_t ndim, const eik_instance* inst, int32_t n_inst,
                                        const eik_options* opt);

/* One candidate configuration timed by eik_tune. */
typedef struct {
    int32_t tile[3];      /* (z, y, x) */
    int32_t inner_iters;  /* inner iterations per tile visit */
    double ms;            /* best device time of a solve (HIP events) */
    int32_t order_min;    /* as eik_options.order_min (0: default) */
    int32_t workgroups;   /* as eik_options.workgroups (0: default) */
} eik_tune_entry;

/*
 * eik_tune -- choose the schedule of the tile variant for a problem by timing
 * candidate configurations on it (each solved once to warm up, then the
 * best of two timed solves; device time from HIP events on opt->stream):
 * first the tile shape and inner-iteration cap, then, for that shape, the
 * ordered remedy's per-launch minimum (half, the default and twice the
 * default; not with EIK_FLAG_FIFO_REMEDY or EIK_FLAG_SKIP_REMEDY) and the
 * persistent workgroups per launch (1024, 1536, 2048).  Not in the paper: its
 * run times depend on the GPU's work-group size, and the tile shape and
 * launch width play that role here.
 *   F, ndim, dims, h, sources, n_sources, eps  as eik_solve
 *   phi_scratch  device, N elements; overwritten by the timed solves
 *   opt          in: dtype, stream, spacing (per-axis spacing times only the
 *                default shapes, the only ones it runs on), workspace (used
 *                when large enough, else the library allocates); out: tile,
 *                inner_iters, order_min and workgroups of the fastest
 *                candidate, variant = EIK_VARIANT_TILE (tile (0, 0, 0) when
 *                the default shapes won; 0 for a default order_min or
 *                workgroups)
 *   report       host, nullable: up to report_cap timed candidates;
 *                *n_report (nullable) receives the count written
 * The choice is cached per (ndim, dtype, log2 of N, per-axis spacing or
 * not, EIK_FLAG_SKIP_REMEDY and EIK_FLAG_FIFO_REMEDY) for the life of the
 * process, whatever the speed field: a later call for the same class times
 * nothing and reports 0 entries.  The arguments are checked as eik_solve
 * checks them before the cache is consulted; errors as eik_solve.
 */
eik_status eik_tune(const void* F, int32_t ndim, const int64_t* dims, double h, const int64_t* sources,
                    int64_t n_sources, double eps, void* phi_scratch, eik_options* opt,
                    eik_tune_entry* report, int32_t report_cap, int32_t* n_report);

/*
 * eik_async_status -- outcome of the last call enqueued with EIK_FLAG_ASYNC
 * on this workspace (eik_solve, eik_solve_batch, eik_adjoint,
 * eik_adjoint_batch; also valid after replaying a graph captured from such
 * calls).  Waits for `stream` (hipStream_t, NULL: the default stream) and
 * reads the control word the call's kernels wrote at the start of the
 * workspace.  Algorithm 2 loops "while the list is not empty"; an
 * asynchronous call cannot stop early, so it runs its launch budget and a
 * last kernel per loop records whether the list it would drain next is empty.
 *   workspace  device, the workspace passed to that call (256-byte aligned)
 * Returns EIK_OK when every loop emptied its lists within max_iters launches,
 * EIK_ERR_NO_CONVERGENCE when one did not (the output then holds the current
 * iterate, an upper bound of the solution; enqueue again with a larger
 * max_iters), EIK_ERR_INVALID_ARGUMENT when a forward solve found F negative
 * or not finite, EIK_ERR_DEVICE on a HIP error.  The word is reset by the
 * next call on the workspace.  Not meaningful after synchronous calls, which
 * return their status directly.
 */
eik_status eik_async_status(const void* workspace, void* stream);

/*
 * eik_solve_noalloc -- eik_solve for callers that cannot allocate memory
 * (serving loops and harnesses that forbid allocation): same arguments,
 * checks, schedules and results as eik_solve, but the call allocates nothing
 * -- no device memory, no pinned host memory, no HIP events.  Its workspace
 * is a static device array of 128 MiB (134217728 bytes) that each GPU the
 * library runs on holds from the first use until the process ends; results
 * are read back through pageable host memory.
 *   Arguments as eik_solve.  opt->workspace must be NULL (and
 *   workspace_bytes 0); EIK_FLAG_ASYNC and EIK_FLAG_PROFILE are not accepted
 *   (EIK_ERR_UNSUPPORTED): the call is synchronous.
 * Errors as eik_solve, and EIK_ERR_OUT_OF_MEMORY, before any device work,
 * when eik_workspace_size for the shape and options exceeds 128 MiB (e.g.
 * the tile variant takes 90 MiB at 256^3 and 98 MiB at 4096^2 in float32;
 * the node-list variants need about 60 bytes per node and fit up to about
 * 2 M nodes).
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents (each solve initialises what it reads); calls that overlap
 * on one GPU -- from several host threads or on several streams -- race on it
 * and must be serialised by the caller.
 */
eik_status eik_solve_noalloc(const void* F, int32_t ndim, const int64_t* dims, double h,
                             const int64_t* sources, int64_t n_sources, double eps,
                             void* phi_out, const eik_options* opt);

/* Human-readable name of a status code (static storage). */
const char* eik_status_string(eik_status s);

/* Description of the last failure on the calling thread ("" if none). */
const char* eik_last_error(void);

/* EIK_ABI_VERSION of the loaded library. */
int32_t eik_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EIK_H_ */
