/*
 * nncp.h -- C ABI of the MI355X (gfx950) nonnegative CP decomposition library.
 *
 * The problem (Eq. (1) of Ballard, Hayashi, Kannan, "Parallel Nonnegative CP
 * Decomposition of Dense Tensors"): given a dense tensor X of shape
 * I_1 x ... x I_N and a rank R, find nonnegative factor matrices H^(n)
 * (I_n x R) and weights lambda (R) that minimise
 * || X - sum_r lambda_r H^(1)(:,r) o ... o H^(N)(:,r) ||.  The method is block
 * coordinate descent over the factor matrices (Algorithm 1) with the
 * dimension-tree MTTKRP (Section IV-A), HALS or multiplicative updates
 * (Section II-B), column normalisation and the relative-error identity of
 * Section IV-B / the appendix algorithm.
 *
 * Conventions shared by every entry point:
 *  - Tensors are dense and stored with mode 1 fastest (the generalised
 *    column-major order of Section IV-C): entry (i_1..i_N), 0-based, lives at
 *    i_1 + I_1*(i_2 + I_2*(i_3 + ...)).
 *  - Factor matrices are I_n x R, column-major, float32, leading dimension I_n.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary CPU memory. The library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Work is enqueued on it; calls that return host results synchronise it.
 *  - Every function returns an nncp_status (0 = success). No C++ exception
 *    crosses this boundary. Invalid arguments are rejected before any work is
 *    enqueued; a HIP runtime failure returns NNCP_EDEVICE.
 *  - Tensor values are not scanned: nonnegative data is the intended input
 *    (Eq. (1)), but any finite values are accepted.
 */
#ifndef NNCP_H
#define NNCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NNCP_OK = 0,
  NNCP_EINVAL = -1,    /* bad argument (shape, rank, pointer, enum, buffer size) */
  NNCP_ENOMEM = -2,    /* device memory could not be allocated / job exceeds the HBM budget */
  NNCP_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed */
  NNCP_EBUSY = -4,     /* serving: job not finished yet */
  NNCP_ENOTFOUND = -5, /* serving: unknown job id */
  NNCP_ECANCELED = -6  /* serving: job was cancelled or failed */
} nncp_status;

typedef enum { NNCP_HALS = 0, NNCP_MU = 1 } nncp_update;
typedef enum { NNCP_F32 = 0, NNCP_BF16 = 1, NNCP_F16 = 2 } nncp_dtype;

#define NNCP_MAX_MODES 8
#define NNCP_MAX_RANK 128
#define NNCP_MAX_SWEEPS 100000

/* Options; zero-initialised means: automatic split, record every fit, use a
 * HIP graph per outer iteration, no early stop. */
typedef struct nncp_options {
  int split;          /* root split s (modes 1..s | s+1..N), 1 <= s <= N-1; <= 0: minimise I_L + I_R */
  int no_record_fit;  /* nonzero: fit[] receives only the final value */
  int no_graph;       /* nonzero: launch kernels one by one instead of replaying a HIP graph */
  int phase_timers;   /* nonzero: time each phase with HIP events (implies no_graph) */
  double tol;         /* > 0: stop when |fit_k - fit_{k-1}| < tol (host check each iteration) */
  int pm_wg_kib;      /* partial MTTKRP: aim for at least this many KiB of the tensor per work-group
                         (at most one work-group per CU); <= 0: 256. Depends only on the job, never on
                         what else runs, so a job computes the same sums alone and in a batch. */
  int no_tree;         /* nonzero: compute every mode's MTTKRP directly from the tensor (one partial
                          MTTKRP + multi-TTVs per mode, N passes over X per iteration) instead of
                          through the dimension tree (two passes): the tree-less baseline */
  int inner_sweeps;   /* update sweeps per block update, 1..NNCP_MAX_SWEEPS (<= 0: 1). HALS: that many
                         Gauss-Seidel passes over the columns, each an exact coordinate minimisation,
                         so the sweeps converge to the exact NNLS solution of the block subproblem
                         (Section II-B); MU: that many multiplicative steps. EINVAL above the maximum. */
  int reserved0;
  double inner_tol;   /* > 0: the sweeps of a block update stop early, row by row (each row of a factor
                         is its own NNLS problem): once a sweep changes no entry of the row by more than
                         inner_tol x the row's largest entry. With a small inner_tol and a large
                         inner_sweeps every block update is solved exactly (to that tolerance), the
                         faithful block coordinate descent of Section II-B. 0: always inner_sweeps
                         sweeps. EINVAL if negative or not finite. */
  unsigned long long tree_peel; /* shape of the dimension tree below the root split (Section IV-A allows
                         any binary tree over contiguous mode ranges): an internal node {a..b} (0-based
                         modes) splits as {a} | {a+1..b} (the paper's N = 5 example), or as
                         {a..b-1} | {b} if bit a*8+b is set. Bits of nodes the tree does not contain are
                         ignored. Every shape computes the same MTTKRPs; they differ in the sizes of
                         the temporaries and the multi-TTVs. */
} nncp_options;

/* The most recent HIP runtime failure the library saw (in any thread): its
 * hipError_t in *hip_error and a source location code in *where (for bug
 * reports; either pointer may be NULL). Returns NNCP_EDEVICE if a failure was
 * recorded since the library was loaded, NNCP_OK (both outputs 0) if none. Meant
 * for diagnosing a call that returned NNCP_EDEVICE; the record is not cleared. */
int nncp_last_device_error(int* hip_error, int* where);

/* Human-readable text for a status code (static storage). */
const char* nncp_strerror(int status);

/* Library version as major*10000 + minor*100 + patch. */
int nncp_version(void);

/* Bytes of scratch the nncp() driver needs for this problem (>= 256-byte aligned
 * internally). Returns 0 for invalid arguments. */
size_t nncp_workspace_bytes(int N, const int64_t* dims, int R, int dtype,
                            const nncp_options* opt);

/*
 * nncp: `iters` outer iterations of alternating-update NNCP (Algorithm 1;
 * normalisation and error as in the appendix algorithm).
 *
 *  X          device, the tensor in `dtype` storage (F32, BF16 or F16), I entries.
 *  dims       host, N extents, N in [2, NNCP_MAX_MODES], each >= 1.
 *  R          rank, 1 <= R <= NNCP_MAX_RANK.
 *  update     NNCP_HALS (column-wise HALS sweep) or NNCP_MU (multiplicative).
 *  H          host array of N device pointers, H[n] is I_n x R float32.
 *             In: starting factors (any nonnegative scaling). Out: factors with
 *             unit 2-norm columns (a column that became zero stays zero).
 *  lambda     host, R doubles. In: weights of the starting model (pass ones for
 *             fresh factors). Out: the weights lambda of the final model.
 *  fit        host, `iters` doubles (or 1 if opt->no_record_fit): fit = 1 - eps
 *             after each outer iteration, eps = ||X - model|| / ||X|| from
 *             ||X||^2 - 2<X,model> + ||model||^2 accumulated in float64.
 *  iters_done host, optional: iterations actually run (fewer if tol stopped early).
 *  workspace  device scratch of ws_bytes >= nncp_workspace_bytes(...), or NULL to
 *             let the library allocate (and free before returning).
 * Synchronises `stream` before returning.
 */
int nncp(const void* X, int dtype, int N, const int64_t* dims, int R, int iters, int update,
         float* const* H, double* lambda, double* fit, int* iters_done,
         void* workspace, size_t ws_bytes, const nncp_options* opt, void* stream);

/* ---- Persistent plan: the same driver, split so a caller can time or resume ---- */
typedef struct nncp_plan nncp_plan;

/* Validates, lays out the workspace, computes alpha = ||X||^2 (float64), the
 * starting Gram matrices and lambda (appendix algorithm, initialisation).
 * X, H, workspace stay owned by the caller and must outlive the plan.
 * lambda_in: host R doubles or NULL for ones. */
int nncp_plan_create(nncp_plan** plan, const void* X, int dtype, int N, const int64_t* dims,
                     int R, int update, float* const* H, const double* lambda_in,
                     void* workspace, size_t ws_bytes, const nncp_options* opt, void* stream);
/* Runs `iters` more outer iterations from the current state; fit (host, may be
 * NULL) receives one value per iteration. Synchronises. */
int nncp_plan_run(nncp_plan* plan, int iters, double* fit, int* iters_done);
/* Writes unit-column factors into H (in place) and lambda (host, R). The plan
 * stays valid: a later run continues from this normalised state. */
int nncp_plan_finish(nncp_plan* plan, double* lambda);
/* Milliseconds per phase accumulated by runs with phase_timers set, in the
 * order pm, mttv, nls, gram, err, total. ms must hold 6 doubles. */
int nncp_plan_phase_ms(const nncp_plan* plan, double* ms);
/* Re-runs the tree-node kernel of `mode` (the node op computed just before that
 * mode's update: a root partial MTTKRP for mode 1 and mode s+1, a multi-TTV
 * otherwise) `reps` times back to back on the plan's stream and returns the
 * average milliseconds per launch from HIP events. Reads the current factors;
 * it rewrites only that node's temporary, which the next iteration recomputes. */
int nncp_plan_time_node(nncp_plan* plan, int mode, int reps, double* ms_avg);
/* Re-runs the whole dimension-tree MTTKRP of one outer iteration (every mode's
 * node op and leaf multi-TTV, with the current factors; no update) `reps`
 * times back to back and returns the average milliseconds per tree from HIP
 * events. Rewrites only the tree temporaries and M. */
int nncp_plan_time_mttkrp(nncp_plan* plan, int reps, double* ms_avg);
int nncp_plan_destroy(nncp_plan* plan);
/* Moves the plan to another stream: later calls on it (run, finish, fits, the
 * timing calls) enqueue on `stream`. The caller orders the switch (the plan's
 * earlier work must be complete or ordered before work on the new stream). */
int nncp_plan_set_stream(nncp_plan* plan, void* stream);

/* Root-split autotuning (Section IV-A leaves the root split of the dimension
 * tree free; the cost model picks the split with the smallest node
 * temporaries, which is not always the fastest on the device). For every
 * split s = 1..N-1 this builds a plan with the given options (split
 * overridden), times one dimension-tree MTTKRP sweep of all N modes
 * (nncp_plan_time_mttkrp: one warm-up sweep, then the average of `reps`),
 * and returns the fastest in *best_split. X and H (device) are only read.
 * ms (host, optional) receives N-1 values: ms[s-1] for split s. Each
 * candidate allocates its own workspace for the call; a split whose
 * workspace cannot be allocated gets ms = -1 and is skipped (NNCP_ENOMEM if
 * none fits). Same argument rules as nncp_plan_create; reps >= 1. */
int nncp_autotune_split(const void* X, int dtype, int N, const int64_t* dims, int R, float* const* H,
                        const nncp_options* opt, int reps, int* best_split, double* ms, void* stream);

/* Tree-shape autotuning: times the dimension-tree MTTKRP sweep (as
 * nncp_autotune_split does) for every tree of every root split, each internal
 * node of three or more modes split either way (nncp_options.tree_peel), up to
 * `cap` trees in the order: root split 1..N-1, then the left half's shapes,
 * then the right half's. The paper's memory criterion (Section IV-C) picks the
 * tree with the smallest temporaries; this measures time instead. Candidate k
 * gets splits[k], peels[k] and ms[k] (host arrays of cap entries); *count
 * receives the number timed and *best the index of the fastest. Trees whose
 * workspace cannot be allocated are skipped (NNCP_ENOMEM if none fits). X and
 * H (device) are only read. */
int nncp_autotune_tree(const void* X, int dtype, int N, const int64_t* dims, int R, float* const* H,
                       const nncp_options* opt, int reps, int cap, int* splits, unsigned long long* peels,
                       double* ms, int* count, int* best, void* stream);

/* Host copy of the fits recorded since the plan was created (or since the last
 * nncp_plan_run, which restarts the record): *count = outer iterations
 * completed; fit (host) receives min(*count, cap, 1024) values. */
int nncp_plan_fits(nncp_plan* plan, double* fit, int cap, int* count);

/* ---- Batched plans: many independent decompositions advanced together ----
 * A batch holds caller-created plans (rank <= 64). nncp_batch_run(b, k) runs
 * k outer iterations of every member. One iteration of all members is one
 * HIP graph: for each step of the iteration (per mode: partial MTTKRP or
 * multi-TTV node, split-K reduction, leaf multi-TTV, update, Gram/finalize)
 * one persistent kernel per kernel family walks a device list of (member
 * kernel, tile) items. Each member keeps the kernels, tiles and summation
 * order of its stand-alone run, so its results are bitwise those of
 * nncp_plan_run on the same state, whatever else is in the batch (this is how
 * jobs are batched without coupling: not in the paper, which runs one
 * decomposition at a time). Members stay owned by the caller; removing or
 * adding a member rewrites the device work lists at the next run, without
 * capturing the graph again unless a new kind of launch is needed.
 * Fits are read per member with nncp_plan_fits. */
typedef struct nncp_batch nncp_batch;
int nncp_batch_create(nncp_batch** batch, void* stream);
int nncp_batch_add(nncp_batch* batch, nncp_plan* plan);      /* EINVAL: rank > 64, or already a member */
int nncp_batch_remove(nncp_batch* batch, nncp_plan* plan);   /* ENOTFOUND: not a member */
int nncp_batch_size(const nncp_batch* batch);
/* Runs `ticks` outer iterations of every member; synchronises the stream. */
int nncp_batch_run(nncp_batch* batch, int ticks);
/* Launches per tick and work items per tick of the current work lists. */
int nncp_batch_stats(const nncp_batch* batch, int* launches, int64_t* items);
/* How often the tick's graph was captured and how often the device work lists
 * were rewritten since the batch was created. A membership change rewrites the
 * lists in place; the graph is captured again only when a member needs a
 * launch (a step of its iteration on a kernel variant) that the captured graph
 * does not have, or a list outgrows its device buffer. Either output may be NULL. */
int nncp_batch_captures(const nncp_batch* batch, int64_t* captures, int64_t* list_updates);
/* Host seconds spent between ticks since the batch was created: rewriting the
 * work lists after membership changes (re-recording every member's iteration
 * and uploading the lists; the graph builds included) and building the tick's
 * graph. Either output may be NULL. */
int nncp_batch_build_time(const nncp_batch* batch, double* rebuild_s, double* graph_s);
int nncp_batch_destroy(nncp_batch* batch);   /* does not destroy the member plans */

/* ---- Serving: continuous batching of jobs that arrive over time ----
 * A loader thread admits submitted jobs in arrival order while fewer than
 * max_active are admitted and their device footprint (tensor + factors +
 * workspace) fits in hbm_budget_bytes next to the others; a job that can never
 * fit is rejected with NNCP_ENOMEM. It uploads the job and sets up its plan on
 * a stream of its own while the running jobs compute. A worker thread advances
 * every running job one outer iteration per tick through one batch, lets
 * uploaded jobs join between ticks, and retires a job after its `iters`
 * iterations (results copied to host, device memory freed in stream order).
 * Each job's result is that of its stand-alone plan (see nncp_batch). Times
 * are seconds on the server's clock. */
typedef struct nncp_server nncp_server;
#define NNCP_SERVER_SIMULATE 1  /* flag: run the scheduler without a GPU (ticks sleep); for host tests */
typedef struct nncp_job_request {
  const void* X;            /* host tensor in `dtype` storage, mode 1 fastest; must stay valid until the
                               job is done (it is read when the job is admitted) */
  int dtype, N;
  const int64_t* dims;      /* host, N extents (copied) */
  int R;                    /* 1..64 */
  int update, iters, split; /* split <= 0: automatic */
  const float* const* H0;   /* host, N starting factors I_n x R column-major (copied at submit) */
} nncp_job_request;
typedef struct nncp_job_result {
  int status;               /* NNCP_EBUSY while queued or running, then NNCP_OK or the error */
  int iters_done;
  double submit_s;          /* submitted */
  double admit_s;           /* admitted: memory reserved, upload begins (queue wait = admit_s - submit_s) */
  double start_s;           /* uploaded and set up, joined the running batch (0 if it never did) */
  double done_s;            /* finished: results on the host */
  size_t footprint_bytes;
} nncp_job_result;
typedef struct nncp_server_stats {
  int queued, active, peak_active;   /* active: jobs in the running batch */
  int64_t ticks, completed, rejected;
  size_t bytes_in_use, peak_bytes, budget_bytes;
  double busy_s, now_s;     /* time spent in ticks; server clock now */
  int64_t graph_captures;   /* captures of the batch's tick graph (see nncp_batch_captures) */
  int64_t list_updates;     /* rewrites of its device work lists (membership changes) */
  double rebuild_s, graph_s; /* host time in those rewrites and graph builds (nncp_batch_build_time) */
} nncp_server_stats;
int nncp_server_create(nncp_server** server, size_t hbm_budget_bytes, int max_active, int flags);
int nncp_server_submit(nncp_server* server, const nncp_job_request* req, uint64_t* id);
/* NNCP_EBUSY while the job is queued or running, NNCP_OK when done (res->status
 * says how), NNCP_ENOTFOUND for an unknown or already fetched id. */
int nncp_server_poll(nncp_server* server, uint64_t id, nncp_job_result* res);
/* Blocks until the job is done (timeout_s < 0: no limit); NNCP_EBUSY on timeout. */
int nncp_server_wait(nncp_server* server, uint64_t id, double timeout_s);
/* Copies a finished job's normalised factors (H[n]: host I_n x R floats), lambda
 * (host R) and fits (host, up to fit_cap) and forgets the job. Any output may be
 * NULL. Returns the job's status. */
int nncp_server_fetch(nncp_server* server, uint64_t id, float* const* H, double* lambda, double* fit,
                      int fit_cap, int* fit_count);
int nncp_server_get_stats(nncp_server* server, nncp_server_stats* stats);
/* Cancels queued jobs, lets running ones finish, stops the worker. */
int nncp_server_destroy(nncp_server* server);

/* ---- Steps of the hot path (each is the kernel the driver runs) ---- */

/* Round float32 to bfloat16 / float16 (round to nearest even), n entries, device. */
int nncp_quantize(const float* src, void* dst, int dtype, int64_t n, void* stream);

/* out_dev[0] = sum x^2 over n entries accumulated in float64 (the ||A||^2 of
 * the appendix algorithm's initialisation). out_dev: device double. */
int nncp_norm_sq(const void* X, int dtype, int64_t n, double* out_dev, void* stream);

/*
 * nncp_norm_sq without any device allocation, for callers that cannot allocate
 * (code recorded under HIP graph capture, serving loops that must not touch the
 * allocator). Same result as nncp_norm_sq, bit for bit: the same kernel, grid
 * and summation order. It only enqueues work on `stream` (no synchronisation);
 * out_dev is written when the stream reaches it.
 * Scratch: the FP64 block partials and the arrival counter live in a static
 * device array of 8.2 KB per GPU (1024 partials), held until the process ends;
 * the grid never exceeds 1024 work-groups, so every n >= 1 fits, and a grid that
 * would need more partials is rejected with NNCP_EINVAL. The counter is cleared
 * by a kernel at the start of each call. All calls on one GPU share that array:
 * calls that overlap on one GPU (concurrent streams or threads) race, so
 * serialise them (one stream, or an event between calls).
 * Errors: NNCP_EINVAL for a NULL pointer, n < 1 or an unknown dtype;
 * NNCP_EDEVICE if the scratch address cannot be obtained or a launch fails.
 */
int nncp_norm_sq_noalloc(const void* X, int dtype, int64_t n, double* out_dev, void* stream);

/*
 * Partial MTTKRP for a root branch of the dimension tree (Section IV-A, Fig. 2a):
 * with I_L = I_1*...*I_s and I_R = I_{s+1}*...*I_N, view X as the column-major
 * I_L x I_R matrix X_[L].
 *   side 0 (left node {1..s}):   T = X_[L] * (H^(N) (.) ... (.) H^(s+1)),   T is I_L x R
 *   side 1 (right node {s+1..N}): T = X_[L]^T * (H^(s) (.) ... (.) H^(1)),  T is I_R x R
 * (.) is the Khatri-Rao product with the lowest mode's row index fastest.
 * H: host array of N device factor pointers (only the contracted modes are read).
 * T: device float64, column-major with leading dimension I_L or I_R. Products are
 * formed on FP32 MFMA and summed in FP64 after every 16 or 32 terms.
 */
int nncp_partial_mttkrp(const void* X, int dtype, int N, const int64_t* dims, int s, int side,
                        float* const* H, int R, double* T, void* stream);

/*
 * Multi-TTV (Section IV-A, Fig. 2b) on a tree node {a..b} whose temporary T has
 * shape I_a x ... x I_b x R (column-major, R slowest, float64). `node_dims` are the
 * nm = b-a+1 extents. Sums are accumulated in float64; out is float64.
 *   kind 0 (leaf {a}):  out(i,r) = sum_j T(i, j, r) K(j, r), K = H^(b) (.) ... (.) H^(a+1);
 *                       out is I_a x R. Hf[0..nm-2] are the factors of modes a+1..b.
 *   kind 1 (node {a+1..b}): out(j, r) = sum_i T(i, j, r) H^(a)(i, r); out has shape
 *                       I_{a+1} x ... x I_b x R. Hf[0] is the factor of mode a.
 */
int nncp_mttv(const double* T, int nm, const int64_t* node_dims, int kind, float* const* Hf,
              int R, double* out, void* stream);

/* Full dimension-tree MTTKRP for mode n (0-based) with the given factors: the root
 * PM on n's side of split s, then the chain of multi-TTVs down to leaf n. M: device
 * float64 I_n x R. Uses an internal workspace allocated for the call. */
int nncp_mttkrp(const void* X, int dtype, int N, const int64_t* dims, int s, int n,
                float* const* H, int R, double* M, void* stream);

/* G = H^T H (R x R, float64, device) for a device float32 I x R factor. */
int nncp_gram(const float* H, int64_t I, int R, double* G, void* stream);

/*
 * One NLS-Update of a factor (Section II-B) followed by column normalisation:
 *   W = H diag(lambda) (the block's current value in the model [[lambda; H]]),
 *   HALS: for r = 1..R: W(:,r) = max(0, W(:,r) + (M(:,r) - (W S)(:,r)) / S(r,r));
 *   MU:   W = W * M / max(W S, 1e-16);
 *   lambda = column norms of W, H = W diag(1/lambda), G = H^T H.
 * M: device float64 I x R; H: device float32 I x R; S: device float64 R x R
 * (symmetric); lambda: device float64 R (in/out); G: device float64 R x R (out).
 * The update arithmetic is float64; H is stored as float32.
 */
int nncp_nls_update(const double* M, float* H, int64_t I, int R, const double* S,
                    double* lambda, int update, double* G, void* stream);

/*
 * The block subproblem of Section II-B solved by repeated update sweeps: the
 * same as nncp_nls_update, but each row of W (an independent NNLS problem
 * min_{w >= 0} 1/2 w^T S w - m^T w) gets up to max_sweeps sweeps (HALS: exact
 * coordinate minimisations, so the row converges to the exact NNLS solution;
 * MU: multiplicative steps), stopping once a sweep changes no entry of the row
 * by more than tol x the row's largest entry (tol = 0: always max_sweeps).
 * W_out: device float64 I x R (column-major) or NULL; receives the solution W
 * before normalisation and before H is rounded to float32.
 * max_sweeps in 1..NNCP_MAX_SWEEPS, tol >= 0 and finite, else NNCP_EINVAL.
 */
int nncp_nls_solve(const double* M, float* H, int64_t I, int R, const double* S, double* lambda,
                   int update, int max_sweeps, double tol, double* W_out, double* G, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NNCP_H */
