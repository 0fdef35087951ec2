/*
 * dpc.h - C ABI of the MI355X exact density-peaks clustering library (libdpc.so).
 *
 * The operations are those of Amagata and Hara, "Fast Density-Peaks Clustering:
 * Multicore-based Parallelization Approach", Section 2.1 (Definitions 1-6):
 *
 *   local density     rho_i   = #{ j : dist(p_i, p_j) < d_cut }, p_i itself included (Def. 1, Eq. 1)
 *   dependent point   q_i     = nearest point of higher density (Def. 2)
 *   dependent dist.   delta_i = dist(p_i, q_i), +inf for the densest point (Def. 3)
 *   noise             rho_i < rho_min (Def. 4)
 *   cluster center    non-noise with delta_i >= delta_min, delta_min > d_cut (Def. 5)
 *   cluster           non-noise points reachable from a center by dependent links (Def. 6)
 *
 * Exact semantics fixed by this library where the paper leaves a choice:
 *   - points are int32 coordinates in [0, 2^17); distances are compared exactly
 *     on integer squared distances: dist < d_cut <=> D2 < ceil(d_cut^2);
 *   - "higher density" is the strict total order (rho descending, id ascending)
 *     (the paper breaks rho ties arbitrarily / by a random addend, Section 3);
 *   - among equidistant higher points the smaller id is the dependent point;
 *   - delta is the correctly rounded FP64 square root of the exact D2;
 *   - labels are center ids; noise gets -1.
 *
 * Conventions for every call:
 *   - array arguments are DEVICE pointers, allocated and owned by the caller;
 *     the library never allocates device memory;
 *   - `ws` is a caller-owned device workspace of at least the size returned by
 *     the matching *_workspace_bytes call; its contents between calls belong to
 *     the library (dpc_dependent may reuse the grid left by dpc_density);
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream); calls
 *     only enqueue work and return without synchronising;
 *   - errors found on the host are returned at once, with nothing enqueued and
 *     the outputs untouched; errors found on the device (coordinates out of
 *     range, inconsistent inputs) are recorded in `ws` and returned by
 *     dpc_sync_status; every call is memory-safe whatever the input values;
 *   - calls on distinct workspaces may run concurrently from several threads.
 */
#ifndef DPC_H
#define DPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dpc_status;

#define DPC_OK 0
#define DPC_EINVAL (-1)     /* bad argument: null pointer, n < 1 or n >= 2^27, d not in [1, 8],
                               d_cut not finite or <= 0, rho_min < 0, delta_min NaN or <= d_cut */
#define DPC_ERANGE (-2)     /* a coordinate outside [0, 2^17) (device-detected, see dpc_sync_status);
                               such coordinates are clamped into range and the results are those of
                               the clamped points */
#define DPC_EWORKSPACE (-3) /* ws_bytes smaller than the required workspace */
#define DPC_EDEVICE (-4)    /* HIP runtime error; dpc_last_error() gives the message */

/* Flag for dpc_dependent: `ws` still holds the grid that dpc_density built for the same
 * pts, n, d and d_cut, so it is not rebuilt.  The grid carries a stamp of the inputs it
 * was built for, checked on the device: if it does not match (no dpc_density call on this
 * workspace, or one with other inputs), nothing is computed, the outputs are left as they
 * were and dpc_sync_status reports DPC_EINVAL.  A reused grid keeps its build's status
 * (DPC_ERANGE when a coordinate was clamped). */
#define DPC_REUSE_GRID 1u

/* Largest number of points per call (ids must fit 27 bits of a packed (D2, id) key). */
#define DPC_MAX_POINTS ((int64_t)1 << 27)
/* Coordinates must lie in [0, DPC_COORD_LIMIT). */
#define DPC_COORD_LIMIT 131072
#define DPC_MAX_DIM 8

/* Bytes of workspace needed by dpc_density, dpc_dependent, dpc_label and dpc_run for
 * these sizes (0 if the arguments are invalid). */
size_t dpc_workspace_bytes(int64_t n, int32_t d, double d_cut);

/*
 * Local density (Def. 1, Eq. 1).
 *   pts  [n][d] int32, row-major, point i at pts + i*d (read only)
 *   rho  [n] int32 output, rho[i] >= 1
 */
dpc_status dpc_density(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t *rho,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * Dependent point and dependent distance (Defs. 2-3) given the densities `rho`
 * (normally dpc_density's output).
 *   dep    [n] int32 output: id of the dependent point, -1 for the densest point
 *   delta  [n] double output: dist(p_i, p_dep_i), +inf for the densest point
 *   flags  0 or DPC_REUSE_GRID
 */
dpc_status dpc_dependent(const int32_t *pts, int64_t n, int32_t d, double d_cut, const int32_t *rho,
                         int32_t *dep, double *delta, uint32_t flags, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Noise, centers and cluster labels (Defs. 4-6) from (rho, dep, delta) alone, so
 * that new thresholds chosen on the decision graph (Section 2.1) only rerun this.
 *   label     [n] int32 output: id of the point's cluster center, -1 for noise
 *   ncenters  device int64 output: number of cluster centers
 * A center's own dependent point is taken to be itself (Section 2.1, after Def. 5).
 */
dpc_status dpc_label(int64_t n, const int32_t *rho, const int32_t *dep, const double *delta,
                     int32_t rho_min, double delta_min, int32_t *label, int64_t *ncenters,
                     void *ws, size_t ws_bytes, void *stream);

/* dpc_density, dpc_dependent (reusing the grid) and dpc_label in one call. */
dpc_status dpc_run(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                   double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                   int64_t *ncenters, void *ws, size_t ws_bytes, void *stream);

/*
 * Approx-DPC (Section 4): the same exact local densities, approximate dependent
 * points where Section 4.3's rules find a denser point close by, exact ones
 * (Defs. 2-3) elsewhere, then labels (Defs. 4-6) as dpc_label computes them.
 * Cells of a second grid (Section 4.1) have side La = 1 + floor(sqrt((R - 1) / d)),
 * R = ceil(d_cut^2): the largest integer side that keeps two points of one cell
 * strictly within d_cut; a point's cell is (x_1 / La, ..., x_d / La), and its
 * cell's densest point p*(c) ranks first by (rho descending, id ascending).
 *   - a point other than p*(c) gets dep = p*(c), delta = d_cut;
 *   - p*(c) gets dep = p*(c') and delta = d_cut for the cell c' with the smallest
 *     coordinates (first dimension most significant) among the cells that hold a
 *     point strictly within d_cut of it and whose points all have a higher rho;
 *   - any other point gets its exact dependent point and distance.
 * With delta_min > d_cut (required, as for dpc_run) the centers and the noise
 * equal dpc_run's (Section 4.4, the cluster center guarantee).
 *   rho, dep, delta, label, ncenters  as for dpc_run (device)
 *   approx  optional [n] uint8 output (NULL: not written): 1 where dep and delta
 *           come from the approximation rules, else 0
 *   ws      device workspace of at least dpc_approx_workspace_bytes(n, d, d_cut)
 *           bytes (more than dpc_run's: a hash table of the occupied cells)
 * Errors: those of dpc_run; DPC_EWORKSPACE when ws_bytes is too small.  Device-
 * detected problems are read with dpc_sync_status, as for dpc_run.
 */
size_t dpc_approx_workspace_bytes(int64_t n, int32_t d, double d_cut);
dpc_status dpc_approx_run(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                          double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                          int64_t *ncenters, uint8_t *approx, void *ws, size_t ws_bytes, void *stream);

/*
 * S-Approx-DPC (Section 5): one picked point per cell of a grid G' stands for the
 * cell.  Cells have side Le = 1 + floor(sqrt((Re - 1) / d)), Re = ceil(e^2) for the
 * double e = eps * d_cut (so a cell's points lie strictly within e of each other);
 * a cell's pick is its smallest id.
 *   - a pick gets its exact local density (Def. 1, against all points);
 *   - a point that was not picked gets dep = its pick, delta = the distance to it,
 *     and rho = the pick's density (it follows its pick into clusters and noise);
 *   - first phase: a pick takes the nearest higher-ranked pick among the picks of
 *     the cells holding a point strictly within d_cut of it (delta <= (1 + eps) d_cut);
 *   - second phase: a pick with none takes its nearest higher-ranked pick of all
 *     (+inf and -1 for the top pick).
 * Ranks are (rho descending, id ascending) over the picks; delta is the correctly
 * rounded distance.
 *   eps     (0, 1]
 *   picked  optional [n] uint8 output (NULL: not written): 1 for the picks
 *   ws      at least dpc_sapprox_workspace_bytes(n, d, d_cut, eps) bytes (0 if invalid)
 * Other arguments, outputs and errors as for dpc_run (DPC_EINVAL also for eps out of range).
 */
size_t dpc_sapprox_workspace_bytes(int64_t n, int32_t d, double d_cut, double eps);
dpc_status dpc_sapprox_run(const int32_t *pts, int64_t n, int32_t d, double d_cut, double eps, int32_t rho_min,
                           double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                           int64_t *ncenters, uint8_t *picked, void *ws, size_t ws_bytes, void *stream);

/*
 * Decision graph (Section 2.1): summaries of the <rho_i, delta_i> pairs from which a
 * user picks rho_min and delta_min, computed on the device from resident outputs of
 * dpc_run / dpc_approx_run (rho [n] int32, delta [n] double, device).
 *
 * dpc_decision_top: the min(k, m) points of largest delta among the m points with
 * rho >= rho_min, ordered by delta descending, then id ascending.
 *   k       1 .. DPC_DECISION_TOP_MAX
 *   ids     [k] int32 output (device); deltas [k] double output; rhos [k] int32 output
 *           or NULL; count  device int64 output: the number of entries written
 *   ws      device workspace of at least DPC_DECISION_WS_BYTES bytes
 * Errors: DPC_EINVAL (null pointer, n < 1, k out of range), DPC_EWORKSPACE.
 */
#define DPC_DECISION_TOP_MAX 4096
#define DPC_DECISION_WS_BYTES ((size_t)128 << 10)
dpc_status dpc_decision_top(int64_t n, const int32_t *rho, const double *delta, int32_t rho_min, int32_t k,
                            int32_t *ids, double *deltas, int32_t *rhos, int64_t *count, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * dpc_decision_histogram: counts[i * n_delta_bins + j] (device int64 output, written
 * whole) = number of points with rho in bin i of rho_edges and delta in bin j of
 * delta_edges.  Edges are device double arrays of n_bins + 1 increasing values; bins
 * are half-open [e_k, e_k+1) except the last, which holds its right edge too (an edge
 * of +inf takes infinite deltas); points outside every bin are not counted.
 * Errors: DPC_EINVAL (null pointer, n < 1, bins < 1, or more than 2^24 bins in all).
 */
dpc_status dpc_decision_histogram(int64_t n, const int32_t *rho, const double *delta, const double *rho_edges,
                                  int32_t n_rho_bins, const double *delta_edges, int32_t n_delta_bins,
                                  int64_t *counts, void *stream);

/*
 * dpc_decision_suggest: a delta_min read off the top list of dpc_decision_top (its
 * deltas and count, device): among consecutive entries (delta_j, delta_j+1) with
 * delta_j finite and > d_cut, the pair of largest ratio delta_j / delta_j+1 (a zero
 * delta_j+1 counts as an infinite ratio; ties: the first pair); delta_min = delta_j,
 * so that the points singled out by a much longer dependent distance become centers
 * (Section 2.1, after Def. 5).
 *   delta_min  device double output: the suggestion, NaN if no pair qualifies
 *   centers    device int64 output: entries of the list with delta >= delta_min (0 if none)
 * Errors: DPC_EINVAL (null pointer, d_cut not finite and > 0).
 */
dpc_status dpc_decision_suggest(const double *top_deltas, const int64_t *count, double d_cut, double *delta_min,
                                int64_t *centers, void *stream);

/*
 * dpc_run for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs as dpc_run, with the scratch space in a static device
 * array of DPC_STATIC_SCRATCH_BYTES that each GPU holds from the first call on it
 * until the process ends.  It calls no allocating routine.
 *   status  optional device uint32 output (NULL: not written): the device-detected
 *           status of this call, bit 0 a coordinate out of range (clamped), bit 1
 *           inconsistent input (as reported by dpc_sync_status for dpc_run)
 * Errors: those of dpc_run, and DPC_EWORKSPACE when dpc_workspace_bytes(n, d, d_cut)
 * exceeds DPC_STATIC_SCRATCH_BYTES (nothing is enqueued).  The stream must belong to
 * the current device.  Every call on one GPU uses that GPU's one array and clears
 * what it needs itself: calls on one GPU must not overlap (their kernels would race
 * on the array), so issue them on one stream or synchronise between them.
 */
#define DPC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
dpc_status dpc_run_static(const int32_t *pts, int64_t n, int32_t d, double d_cut, int32_t rho_min,
                          double delta_min, int32_t *rho, int32_t *dep, double *delta, int32_t *label,
                          int64_t *ncenters, uint32_t *status, void *stream);

/* Minimum workspace of dpc_label called on its own (the device status header). */
#define DPC_LABEL_WS_BYTES 256

/* ceil(d_cut^2) as the library computes it (exactly, by an error-free product), clamped to
 * 2^38 (beyond every squared distance of in-range points); -1 if d_cut is not finite or <= 0.
 * dist < d_cut <=> D2 < this value for integer squared distances D2 (Def. 1). Host only. */
int64_t dpc_cutoff_square(double d_cut);

/* The grid a call would use for these sizes, for diagnostics (host only, nothing enqueued). */
typedef struct {
  int64_t R;             /* ceil(d_cut^2) */
  int64_t cell_side;     /* L: cell side of the grid */
  int64_t cells_per_dim;
  int64_t cells;         /* cells_per_dim^d, the dense cell table */
  int64_t strip_cells;   /* cells per strip along the last dimension */
  int64_t strips;
  int64_t max_tasks;
  int64_t mode;          /* density kernel: 0 packed 16-bit distance path, 1 exact int64 path */
  int64_t workspace_bytes;
  int64_t window_radius; /* K0 cells: K0 * L >= floor(sqrt(R - 1)), so (2 K0 + 1)^d cells hold a d_cut-ball */
  int64_t stages;        /* dependent-search stages */
  int64_t grid_dims;     /* coordinates the cells index (the first grid_dims of d) */
  int64_t lanes;         /* kernel form: 0 tasks of 64 queries sharing windows, 1 one query per lane */
  int64_t open_radius;   /* lane form: radius of the optional second window stage over the
                            points the first leaves open (0: none) */
} dpc_plan_info;
dpc_status dpc_plan(int64_t n, int32_t d, double d_cut, dpc_plan_info *out);

/* Kernel timing for diagnostics.  Level 1: every call records HIP events on its stream
 * around each kernel group (grid_build, density, rank_keys, rank_sort, search, ringk, peaks,
 * finish, label).  Level 2 also synchronises after each dependent search and keeps its work
 * counters (tasks, points left open by the search stages, points sent to the prefix scan,
 * candidates those scans cover).  Level 0 turns it off.  dpc_profile_report waits for the
 * events, writes {"group": [launches, total_ms], ..., "work": {...}} as JSON into buf (up to
 * len bytes, NUL-terminated), returns the full length, and clears the records. */
void dpc_profile_enable(int32_t level);
int32_t dpc_profile_report(char *buf, size_t len);

/* Synchronises `stream` and returns the device-detected status of the most recent call on
 * this workspace: DPC_OK, DPC_ERANGE (coordinates out of range, clamped), DPC_EINVAL (rho or
 * dep inputs not produced by this library: densities outside [1, n] were clamped, dependent
 * links that do not rank higher were cut) or DPC_EDEVICE.  Each call starts with a clear
 * status; this call clears it too. */
dpc_status dpc_sync_status(void *ws, void *stream);

/* Plan options of one problem (0 in any field: the library's default).  Plans change only
 * through these options (dpc_plan_tuned, dpc_batch_plan); every option gives the same
 * results, bit for bit. */
typedef struct {
  int32_t subdiv;          /* cells per cut-off distance along each axis (1..16) */
  int32_t strip_cells;     /* narrower task strips (cells along the last axis) */
  int32_t nstages;         /* dependent-search window stages (1..4), radii and groups below */
  int32_t stage_radius[4]; /* window radius of each stage in cells (1..64); 0: the density
                              window clipped to the cut-off ball (final when closer than d_cut).
                              Lane form runs only the first stage (a block of that radius,
                              or the ball), then the ring search */
  int32_t stage_group[4];  /* tasks whose open points one wave gathers (1..64) */
  int32_t ring_cap;        /* most ring-search steps per point before the prefix scan */
  int32_t grid_dims;       /* coordinates the cells index (default d up to 4, else 3; d if
                              larger): the windows cover those, distances always use all d */
  int32_t lanes;           /* 1: tasks of 64 queries of one strip share each window's candidates
                              (dense data); 2: one query per lane with its own window (sparse
                              data, where a strip holds a few points); 0: the default (lanes for
                              4-D points) */
  int32_t open_radius;     /* lane form after a block stage of radius K: a second window stage of
                              this radius (K+1..16) over the points the first leaves open, before
                              the ring search; 0: none (the default) */
} dpc_tuning;

/* dpc_plan with explicit options (tuning may be NULL). */
dpc_status dpc_plan_tuned(int64_t n, int32_t d, double d_cut, const dpc_tuning *tuning, dpc_plan_info *out);

/*
 * Many problems in one launch per phase (Definitions 1-6 for each job, as dpc_run).
 *
 * A job names its own points, thresholds and outputs (device pointers, caller-owned,
 * as for dpc_run; distinct jobs must not share output arrays).  dpc_batch_plan checks
 * every job as dpc_run would (the first bad job's index is in dpc_last_error), plans
 * each one (`tuning`: NULL or one entry per job), orders the jobs by dimension and then
 * by size, largest first, and returns a host handle and the workspace size.
 * dpc_batch_bind writes the device job table into `ws` (a synchronous copy, so not
 * inside graph capture).  dpc_batch_run then enqueues every phase for all jobs on
 * `stream`, one launch per phase and dimension (no allocation, no host synchronisation:
 * it can be captured in a HIP graph and replayed); it may run any number of times on
 * the bound workspace.  Each job's results are those dpc_run gives for it alone.
 */
typedef struct {
  const int32_t *pts; /* [n][d] int32, device */
  int64_t n;
  int32_t d;
  double d_cut;
  int32_t rho_min;
  double delta_min;
  int32_t *rho, *dep; /* [n] int32 outputs, device */
  double *delta;      /* [n] double output, device */
  int32_t *label;     /* [n] int32 output, device */
  int64_t *ncenters;  /* device int64 output */
} dpc_job;

typedef struct dpc_batch dpc_batch; /* host-side plan of a batch */

dpc_status dpc_batch_plan(const dpc_job *jobs, int32_t njobs, const dpc_tuning *tuning, dpc_batch **out,
                          size_t *ws_bytes);
dpc_status dpc_batch_bind(dpc_batch *batch, void *ws, size_t ws_bytes);
dpc_status dpc_batch_run(const dpc_batch *batch, void *ws, void *stream);
/* Synchronises and ORs the device status of every job (as dpc_sync_status); *first_bad
 * (may be NULL) gets the caller's index of the first job with a non-zero status, or -1. */
dpc_status dpc_batch_sync_status(const dpc_batch *batch, void *ws, void *stream, int32_t *first_bad);
/* Plan of job i (the caller's index) of the batch. */
dpc_status dpc_batch_job_plan(const dpc_batch *batch, int32_t i, dpc_plan_info *out);
void dpc_batch_free(dpc_batch *batch);

/* Message of the last error on the calling thread ("" if none). */
const char *dpc_last_error(void);

/* ABI version (major * 100 + minor). */
int32_t dpc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DPC_H */
