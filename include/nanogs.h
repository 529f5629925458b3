/*
 * nanogs.h -- C ABI of the MI355X (gfx950) splat-simplification library.
 *
 * The library implements the data-parallel hot path of NanoGS (Xiong et al.,
 * "NanoGS: Training-Free Gaussian Splat Simplification", arXiv 2603.16103):
 * rounds of  kNN merge graph (Sec. 3.1)  ->  merge cost per edge (Sec. 3.2,
 * Eq. cost, Appendix A)  ->  greedy disjoint low-cost pairs (Sec. 3.4,
 * Algorithm 1)  ->  mass-preserved moment-matching merge and compaction
 * (Sec. 3.3), repeated until a target splat count (Algorithm 1).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers owned by the caller unless a
 *    comment says "host".  The library never frees caller memory and never
 *    keeps a pointer after a call returns.
 *  - Arrays are row-major per splat: pos[n][3], sh[n][48], ...; float arrays
 *    must be 4-byte aligned, sh / rot / quat 16-byte aligned, and every
 *    workspace (ws) 256-byte aligned.
 *  - Every call returns a nanogs_status; on failure nanogs_last_error()
 *    (thread-local) describes it.  Argument checks happen before any launch,
 *    so a failed check leaves every output untouched.
 *  - Stage calls are asynchronous on `stream` (0 = the null stream).
 *    nanogs_simplify synchronises `stream` and returns a host count.
 *  - Workspace: each call that needs scratch takes (ws, ws_bytes); the size
 *    comes from the matching *_workspace_bytes query.  A smaller workspace
 *    gives NANOGS_EWORKSPACE.  Workspace contents are not preserved.
 *  - Index limits: n * k < 2^31; the whole loop and the batch (which keep
 *    two adjacency entries per edge) need 2 * n * k < 2^31.
 */
#ifndef NANOGS_H
#define NANOGS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NANOGS_OK = 0,
  NANOGS_EINVAL = 1,      /* bad argument (null pointer, size or alignment) */
  NANOGS_EWORKSPACE = 2,  /* workspace smaller than the size query asked for */
  NANOGS_ENONFINITE = 3,  /* an input value is NaN or infinite */
  NANOGS_EHIP = 4,        /* a HIP runtime call failed */
  NANOGS_ENOTREADY = 5,   /* the library found no usable HIP device */
  NANOGS_ENOMEM = 6,      /* out of device or host memory */
  NANOGS_ECANCELLED = 7   /* the job was cancelled (nanogs_batch_cancel) */
} nanogs_status;

#define NANOGS_SH_COEFFS 48   /* degree-3 spherical harmonics per splat */
#define NANOGS_MAX_K 32       /* largest supported kNN size */
#define NANOGS_MAX_S 16       /* largest supported Monte Carlo draw count */
#define NANOGS_MAX_ROUNDS 64  /* per-round statistics kept in nanogs_stats */

/* Stored 3DGS form: what a trained splat PLY holds (Sec. 1, Algorithm 1
 * input/output).  pos[n][3] centre; log_scale[n][3] per-axis log standard
 * deviation; rot[n][4] quaternion (w,x,y,z), not necessarily unit; opacity[n]
 * logit; sh[n][48] f_dc_0..2 then f_rest_0..44. */
typedef struct {
  float* pos;
  float* log_scale;
  float* rot;
  float* opacity;
  float* sh;
} nanogs_gaussians;

/* Activated form used by the stage calls: mu[n][3] centre; scale[n][3]
 * standard deviations (> 0); quat[n][4] unit quaternion (w,x,y,z);
 * alpha[n] opacity in [0,1]; sh[n][48] appearance feature f (Sec. 3.2);
 * origin[n] provenance (nullable). */
typedef struct {
  float* mu;
  float* scale;
  float* quat;
  float* alpha;
  float* sh;
  int32_t* origin;
} nanogs_splats;

#define NANOGS_PREC_FP32 0  /* FP32 costs, FP64 for ill-conditioned pairs */
#define NANOGS_PREC_FP64 1  /* every edge cost in FP64 */

/* kNN graph of each pass (options.refresh).  FULL rebuilds it every pass.
 * LOCAL (the local neighbourhood refresh of Sec. 3.4) rebuilds it in the
 * first pass; later passes query only the splats a merge formed and those
 * whose previous list named a splat that merged, and every other splat keeps
 * its previous list carried to the new indices (its neighbours did not move;
 * a merged splat that came closer is only seen from its own side, through
 * the union of the lists).  Results differ from FULL by design. */
#define NANOGS_REFRESH_FULL 0
#define NANOGS_REFRESH_LOCAL 1

/* Geometric term D_geo of the edge cost (options.cost_mode). */
#define NANOGS_COST_MC 0     /* Appendix A's Monte Carlo estimate of KL(p || q_m):
                                per draw the component is picked by u < pi */
#define NANOGS_COST_STRAT 1  /* same expectation, component-stratified: each
                                draw's z is used in both components, weighted
                                pi and 1 - pi (no component draw) */
#define NANOGS_COST_BOUND 2  /* pi KL(N_i || q_m) + (1 - pi) KL(N_j || q_m)
                                with the closed-form Gaussian KL of Appendix
                                A: an upper bound of the mixture's
                                divergence (joint convexity), no draws */

typedef struct {
  int32_t S;          /* Monte Carlo draws per edge, 1..NANOGS_MAX_S (1) */
  int32_t app_dims;   /* SH coefficients in the appearance term, 1..48 (48) */
  int32_t precision;  /* NANOGS_PREC_FP32 (default) or NANOGS_PREC_FP64 */
  float fb_ratio;     /* FP64 fallback when a Cholesky factor's smallest
                         diagonal is below fb_ratio times its largest
                         (1/256) */
  uint64_t seed;      /* key of the shared Monte Carlo draws (0) */
  int32_t max_rounds; /* stop after this many passes; 0 = no limit */
  int32_t* d_trace;   /* nullable device [n][2]: provenance pairs merged, in
                         pass order, each row (smaller origin, larger) */
  int32_t* d_origin;  /* nullable device [n]: provenance of each output
                         splat (smallest input index it absorbed) */
  int32_t timing;     /* 1: time each stage with HIP events on the call's
                         stream into nanogs_stats.stage_ms;
                         NANOGS_TIME_SOME | (1 << stage) | ...: only the
                         stages whose bit is set (each event record costs a
                         few microseconds of stream time); 0: off (0) */
  float tau;          /* opacity pre-filter of nanogs_simplify (Algorithm
                         1, before the loop): keep the splats with alpha >=
                         min(tau, median alpha); < 0 turns it off (-1) */
  int32_t cost_mode;  /* NANOGS_COST_MC (default), NANOGS_COST_STRAT or
                         NANOGS_COST_BOUND */
  int32_t refresh;    /* NANOGS_REFRESH_FULL (default) or NANOGS_REFRESH_LOCAL
                         (nanogs_simplify only) */
  float pass_frac;    /* progressive collapses (Sec. 3.4): a pass takes at
                         most max(1, floor(pass_frac * N)) pairs (the
                         product in double); 0 = no cap (P = N - N_tgt) */
} nanogs_options;

/* Stages timed into nanogs_stats.stage_ms when options.timing is set. */
#define NANOGS_T_PRECOMPUTE 0 /* per-splat Cholesky factors and weights */
#define NANOGS_T_KNN_TREE 1   /* cell table of the Morton-sorted centres */
#define NANOGS_T_KNN_QUERY 2  /* kNN block gather kernel (level, histogram,
                                 buffered rows) */
#define NANOGS_T_EDGES 3      /* union edges (flags, scan, emit) */
#define NANOGS_T_COST 4       /* FP32 edge-cost kernel */
#define NANOGS_T_COST_FP64 5  /* FP64 recomputation of flagged edges */
#define NANOGS_T_SELECT 6     /* matching iterations and budget */
#define NANOGS_T_MERGE 7      /* merge and compaction */
#define NANOGS_T_SETUP 8      /* spatial order and activation */
#define NANOGS_T_OUTPUT 9     /* deactivation into the caller's order */
#define NANOGS_T_KNN_EXACT 10 /* kNN exact keys of the buffered rows */
#define NANOGS_T_KNN_WAVE 11  /* kNN queries finished one wave each */
#define NANOGS_NTIMED 12
#define NANOGS_TIME_SOME 0x40000000 /* options.timing: the low NANOGS_NTIMED
                                       bits select the stages timed */

typedef struct {
  int32_t rounds;                          /* passes that merged >= 1 pair */
  int32_t early_exit;                      /* 1 if a pass found no pair */
  int64_t n_out;
  int64_t n_per_round[NANOGS_MAX_ROUNDS];  /* N at the start of pass r */
  int64_t edges_per_round[NANOGS_MAX_ROUNDS];
  int64_t pairs_per_round[NANOGS_MAX_ROUNDS];
  int64_t fallback_per_round[NANOGS_MAX_ROUNDS]; /* edges costed in FP64 */
  int32_t ld_iters_per_round[NANOGS_MAX_ROUNDS]; /* matching iterations */
  int64_t knn_retry_per_round[NANOGS_MAX_ROUNDS]; /* kNN queries finished by
                                                     the wave search */
  int64_t knn_screens_per_round[NANOGS_MAX_ROUNDS]; /* float distance screens
                                                       of the block gather */
  double stage_ms[NANOGS_NTIMED];      /* summed over passes (stages timed) */
  int32_t stage_launches[NANOGS_NTIMED];
  int64_t n_kept;  /* splats the opacity pre-filter kept (n when it is off) */
  int64_t requery_per_round[NANOGS_MAX_ROUNDS]; /* rows whose kNN list was
                                                   queried (N unless the local
                                                   refresh kept some) */
} nanogs_stats;

/* Fills *opt with the defaults listed above. */
void nanogs_default_options(nanogs_options* opt);

/* Thread-local description of the last failure ("" after success). */
const char* nanogs_last_error(void);

/* The shared Monte Carlo draws of pass `round` (Appendix A: common random
 * numbers across candidate pairs; the paper names no generator): S rows of
 * (u, z0, z1, z2), u ~ U[0,1) and z ~ N(0, I3), written to HOST out[S][4].
 * Definition: h = SplitMix64 output for a given state;
 * U(s,c) = (h(h(h(seed) ^ round) ^ (8s+c)) >> 11) * 2^-53;
 * u = U(s,0); (z0, z1) = Box-Muller on (U(s,1), U(s,2));
 * z2 = cosine branch of Box-Muller on (U(s,3), U(s,4)), with ln(1-U);
 * computed in double and rounded to float.  Host-only, no device work. */
void nanogs_crn(uint64_t seed, int32_t round, int32_t S, float* out);

/* ---- whole loop (Algorithm 1) ------------------------------------------- */

size_t nanogs_simplify_workspace_bytes(int64_t n, int32_t k,
                                       const nanogs_options* opt);

/* Simplify n splats to target_n (Algorithm 1: while N > N_tgt: kNN graph
 * with k_eff = min(max(1,k), N-1), union edges, edge costs, at most
 * P = N - N_tgt greedy disjoint pairs, stop if none, merge).  in and out are
 * stored-form arrays of capacity n (they may not alias); on success
 * out[0, *n_out) holds the result in the standard 3DGS form with alpha
 * clipped to [0,1].  Output order: splats keep the relative order of the
 * lowest input index they absorbed.  target_n >= n (or n <= 1) copies the
 * input through activation and back.  opt and stats are nullable (host).
 * With options.tau >= 0 the opacity pre-filter (see nanogs_prune) runs
 * first on the activated opacities and the loop runs on its survivors;
 * provenance (d_origin, d_trace) still names input indices.  The workspace
 * query must then see the same options.
 * Errors: EINVAL (n < 1, target_n < 1, k < 1 or > NANOGS_MAX_K, 2*n*k too
 * large, bad options), EWORKSPACE, ENONFINITE (checked before any merge),
 * EHIP.  Synchronises `stream`. */
nanogs_status nanogs_simplify(const nanogs_gaussians* in, int64_t n,
                              int64_t target_n, int32_t k,
                              const nanogs_options* opt, nanogs_gaussians* out,
                              int64_t* n_out, nanogs_stats* stats, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/* Coarse-to-fine hierarchy (Sec. 3.4: every pass leaves a valid coarser
 * representation): nanogs_simplify that also writes the set at the start of
 * every pass.  Level r (r < *lod_levels) occupies rows
 * [lod_offsets[r], lod_offsets[r+1]) of lod (device, stored form, capacity
 * lod_capacity rows), in the order of that pass (level 0 is the input, or
 * the opacity filter's survivors); lod_parent[row] (device, capacity
 * lod_capacity) is the index, within level r+1, of the splat it becomes:
 * both ends of a merged pair name the merged splat.  Level *lod_levels is
 * out[0, *n_out).  A level that would not fit in lod_capacity rows ends the
 * hierarchy there (the loop still finishes); sum_r N_r <= 2 n rows always
 * suffice when every pass halves the set.  lod_offsets (host, at least
 * NANOGS_MAX_ROUNDS + 1 entries) and lod_levels (host) are written.  Other
 * arguments and errors as nanogs_simplify. */
nanogs_status nanogs_simplify_lod(const nanogs_gaussians* in, int64_t n,
                                  int64_t target_n, int32_t k,
                                  const nanogs_options* opt, nanogs_gaussians* out,
                                  int64_t* n_out, nanogs_gaussians* lod,
                                  int32_t* lod_parent, int64_t lod_capacity,
                                  int64_t* lod_offsets, int32_t* lod_levels,
                                  nanogs_stats* stats, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* ---- boundary conversions ---------------------------------------------- */

/* Stored -> activated: scale = exp(log_scale), alpha = sigmoid(opacity),
 * quat = rot/|rot| (zero -> identity); mu and sh copied.  Computed in double,
 * rounded to float.  If d_nonfinite (device int32, nullable) is non-null, a
 * non-finite input value sets it to 1 (it is never cleared). */
nanogs_status nanogs_activate(const nanogs_gaussians* g, int64_t n,
                              nanogs_splats* s, int32_t* d_nonfinite,
                              hipStream_t stream);

/* Activated -> stored: log_scale = log(scale), opacity =
 * logit(clamp(alpha, 2^-24, 1-2^-24)) (alpha clipped to [0,1] first, the
 * final step of Algorithm 1), rot = quat with w >= 0; mu and sh copied. */
nanogs_status nanogs_deactivate(const nanogs_splats* s, int64_t n,
                                nanogs_gaussians* g, hipStream_t stream);

/* ---- opacity pre-filter (Algorithm 1, before the loop) ------------------ */

/* Robust opacity filter: with tau' = min(tau, median of alpha) (the mean of
 * the two middle values for an even n), out receives the splats of `in`
 * whose alpha >= tau', in their input order (origin carried when both in and
 * out give one).  The median and the comparison are taken in double from the
 * float opacities.  out must hold n splats and may not alias in; the count
 * goes to device int64 *d_nout.  Errors: EINVAL (tau not finite, bad
 * pointers), EWORKSPACE. */
size_t nanogs_prune_workspace_bytes(int64_t n);
nanogs_status nanogs_prune(const nanogs_splats* in, int64_t n, float tau,
                           nanogs_splats* out, int64_t* d_nout, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* ---- stage 1: kNN merge graph (Sec. 3.1) -------------------------------- */

size_t nanogs_knn_workspace_bytes(int64_t n, int32_t k);

/* Directed k nearest neighbours of every centre: nbr[i][t] for
 * t < k_eff = min(k, n-1) is the t-th element of {j != i} ordered by the key
 * (d2, j), d2 = ((dx*dx + dy*dy) + dz*dz) in double from the float centres,
 * no fused multiply-add; entries t >= k_eff are -1.  Exact (not
 * approximate).  mu[n][3] float, nbr[n][k] int32.  Reads nothing back and
 * does not synchronise (capturable into a HIP graph). */
nanogs_status nanogs_knn(const float* mu, int64_t n, int32_t k, int32_t* nbr,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* Undirected union of the lists (Algorithm 1 UndirectedUnionEdges): every
 * unordered pair {i,j} with j in nbr(i) or i in nbr(j) exactly once, as
 * ei[e] < ej[e], in lexicographic (ei, ej) order (so an edge's position is
 * its rank in that order).  ei/ej capacity n*k; the edge count goes to the
 * device int64 *d_m (no host read: the call does not synchronise).  Entries
 * < 0 are skipped. */
size_t nanogs_edges_workspace_bytes(int64_t n, int32_t k);
nanogs_status nanogs_edges(const int32_t* nbr, int64_t n, int32_t k,
                           int32_t* ei, int32_t* ej, int64_t* d_m, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* ---- stage 2: merge cost (Eq. cost = D_geo + D_app) --------------------- */

/* cost[e] = D_geo + D_app of edge (ei[e], ej[e]) over the activated splats:
 * D_geo is the Monte Carlo KL estimate of Appendix A with the S shared draws
 * crn (HOST [S][4], see nanogs_crn): the draw picks splat ei[e] when
 * u < pi = w_i / (w_i + w_j) (Eq. norm_mixture), pi taken in double from
 * the float alpha and scales (w = ((alpha*s0)*s1)*s2; the common
 * (2 pi)^{3/2} cancels), and samples x = mu_c + chol(Sigma_c) z; D_app =
 * ||f_i - f_j||^2 over the first opt->app_dims SH coefficients.  dgeo
 * (nullable) receives D_geo alone.  Accuracy (FP32 mode): |dC| <= 1e-4|C|
 * + 1e-5 against a float64 evaluation.  opt nullable (defaults). */
size_t nanogs_edge_cost_workspace_bytes(int64_t n, int64_t m);
nanogs_status nanogs_edge_cost(const nanogs_splats* s, int64_t n,
                               const int32_t* ei, const int32_t* ej, int64_t m,
                               const float* crn, const nanogs_options* opt,
                               float* cost, float* dgeo, void* ws,
                               size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as nanogs_edge_cost, bit for bit, with no workspace argument.
 * Its scratch (packed splats, per-splat factors, the FP64-fallback list,
 * counters and draws) is a fixed 32 MiB array in the library's code object,
 * one per GPU, held until the process ends; the call allocates nothing.
 * Limits: n <= NANOGS_NOALLOC_MAX_N and m <= NANOGS_NOALLOC_MAX_M, else
 * EINVAL before any launch.  Every call on one GPU uses that GPU's single
 * array: calls that overlap on one GPU (other streams or host threads) race
 * and give undefined results; calls in one stream order are safe. */
#define NANOGS_NOALLOC_MAX_N 131072
#define NANOGS_NOALLOC_MAX_M 2097152
nanogs_status nanogs_edge_cost_noalloc(const nanogs_splats* s, int64_t n,
                                       const int32_t* ei, const int32_t* ej,
                                       int64_t m, const float* crn,
                                       const nanogs_options* opt, float* cost,
                                       float* dgeo, hipStream_t stream);

/* ---- stage 3: greedy disjoint pairs (Algorithm 1 GreedyDisjointPairs) --- */

/* partner[n] receives the result of scanning the edges in increasing
 * (cost, min(i,j), max(i,j)) order and taking an edge whenever both ends are
 * free, stopping after max_pairs: partner[i] = j and partner[j] = i for each
 * taken pair, -1 elsewhere.  Edges with a non-finite cost are never taken;
 * -0 equals +0.  Computed by iterated locally-dominant matching, which yields
 * exactly that scan's result.  The pair count goes to device int64
 * *d_npairs. */
size_t nanogs_select_workspace_bytes(int64_t n, int64_t m);
nanogs_status nanogs_select(const int32_t* ei, const int32_t* ej,
                            const float* cost, int64_t m, int64_t n,
                            int64_t max_pairs, int32_t* partner,
                            int64_t* d_npairs, void* ws, size_t ws_bytes,
                            hipStream_t stream);

/* Device-count forms of stages 2 and 3 (the three-stage decomposition of
 * Sec. 3 chained on the device): the edge count is the device int64 *d_m
 * (as nanogs_edges writes it), m_cap (host) bounds it and sizes the launches
 * and the workspace (the _workspace_bytes queries above with m = m_cap);
 * nanogs_select_dev's budget is the device int64 *d_max_pairs.  The draws
 * d_crn are a DEVICE [S][4] array (options.S rows).  These calls neither
 * read device memory back nor synchronise: a chain knn -> edges ->
 * edge_cost_dev -> select_dev -> merge can be enqueued, or captured into a
 * HIP graph, without the host seeing a count.  Results are those of
 * nanogs_edge_cost / nanogs_select with m = *d_m, max_pairs = *d_max_pairs.
 * Errors: as the host-count forms (checked on the host-side arguments only;
 * *d_m is clamped to [0, m_cap], a negative budget keeps no pair). */
nanogs_status nanogs_edge_cost_dev(const nanogs_splats* s, int64_t n,
                                   const int32_t* ei, const int32_t* ej,
                                   const int64_t* d_m, int64_t m_cap,
                                   const float* d_crn, const nanogs_options* opt,
                                   float* cost, float* dgeo, void* ws,
                                   size_t ws_bytes, hipStream_t stream);
nanogs_status nanogs_select_dev(const int32_t* ei, const int32_t* ej,
                                const float* cost, const int64_t* d_m,
                                int64_t m_cap, int64_t n,
                                const int64_t* d_max_pairs, int32_t* partner,
                                int64_t* d_npairs, void* ws, size_t ws_bytes,
                                hipStream_t stream);

/* ---- stage 4: merge + compaction (Sec. 3.3, Algorithm 1 MergePairs) ---- */

/* Mass-preserved moment matching of every pair in partner (Eq. vm_weights,
 * vm_cov, vm_alpha): the merged splat takes the lower index's place, the
 * higher index is removed, survivors keep their relative order; (scale,
 * quat) of the merged covariance from its eigen-decomposition (eigenvalues
 * decreasing, signs fixed so the largest component of the first two axes is
 * positive, w >= 0).  Centre, covariance, opacity and the eigen-
 * decomposition are computed in double from the float inputs; f_m is formed
 * in float with the mixture weights rounded to float.  out must hold n
 * splats and must not alias in; the new count goes to device int64 *d_nout
 * (nothing is read back: the call does not synchronise and can be captured
 * into a HIP graph; rows past the count are left as they were).  origin, when
 * both in and out give one, becomes the smaller origin of a pair. */
size_t nanogs_merge_workspace_bytes(int64_t n);
nanogs_status nanogs_merge(const nanogs_splats* in, int64_t n,
                           const int32_t* partner, nanogs_splats* out,
                           int64_t* d_nout, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/* ---- launch shapes (autotuned) ------------------------------------------ */

/* Launch parameters of the stage kernels.  Every choice gives bit-identical
 * results (the arithmetic of each output does not depend on it); only the
 * speed changes.  Values apply per size bucket of the pass's splat count N:
 * bucket 0: N < 65536, 1: N < 524288, 2: larger. */
typedef struct {
  int32_t cost_block;     /* threads per workgroup, edge-cost kernel: 64, 128
                             or 256 (256) */
  int32_t knn_block;      /* threads per workgroup of the kNN block search
                             (four lanes per query): 64, 128 or 256 (128) */
  int32_t knn_wave_grid;  /* workgroups striding over the kNN queries that the
                             wave search finishes (one wave each):
                             256..65536 (16384) */
  int32_t knn_level_bias; /* finest cell-table level relative to the default
                             (one above the smallest L with 8^L >= N, at most
                             8): -2..1, positive values add nothing (0) */
  int32_t select_check;   /* matching iterations launched over the whole
                             grid before one workgroup finishes the
                             matching on the device: 1..16 (4) */
  int32_t knn_block_min;  /* rows the 3x3x3 block of cells around a query
                             must hold for the block search to use that
                             cell level: 17..1024 (32) */
  int32_t knn_lane_rows;  /* largest block the block search takes; larger
                             ones go to the wave search: 64..4096 (256) */
} nanogs_tuning;

#define NANOGS_TUNE_BUCKETS 3

/* Sets (or reads) the launch parameters of one bucket; bucket -1 sets all.
 * Process-wide; not thread-safe with concurrent calls.  Errors: EINVAL for a
 * bad bucket or value. */
nanogs_status nanogs_set_tuning(int32_t bucket, const nanogs_tuning* t);
nanogs_status nanogs_get_tuning(int32_t bucket, nanogs_tuning* t);

/* ---- batched and served form: many scenes per pass ---------------------- */

/* A batch keeps several simplification jobs (scenes) in one working set and
 * runs one pass of Algorithm 1 for all of them with one launch per stage;
 * every job gets the same result as nanogs_simplify with the same options
 * and seed (its draws are keyed by its own seed and pass).  Jobs join at pass
 * boundaries as rows free up and leave when they reach their target, so a
 * serving loop can keep the device busy with requests that arrive at any
 * time.  A batch is a host object bound to one stream; it is not
 * thread-safe. */
typedef struct nanogs_batch nanogs_batch;

/* Workspace of a batch holding at most max_rows splats of at most max_jobs
 * jobs at a time, with kNN sizes up to max_k (1..NANOGS_MAX_K). */
size_t nanogs_batch_workspace_bytes(int64_t max_rows, int32_t max_k,
                                    int32_t max_jobs);

/* Creates a batch over the caller's device workspace ws (ws_bytes from
 * nanogs_batch_workspace_bytes, 256-byte aligned), which must outlive it.
 * opt (nullable) applies to every job except its seed, which is per job.
 * Errors: EINVAL, EWORKSPACE. */
nanogs_status nanogs_batch_create(int64_t max_rows, int32_t max_k,
                                  int32_t max_jobs, const nanogs_options* opt,
                                  void* ws, size_t ws_bytes, hipStream_t stream,
                                  nanogs_batch** out);
void nanogs_batch_destroy(nanogs_batch* b);

/* Queues a job: simplify the n splats of `in` (device, stored form) to
 * target_n with kNN size k and draw seed `seed`, writing the result to
 * `out` (device, capacity n) and, if d_origin is non-null, each output
 * splat's provenance (smallest input index it absorbed) to d_origin[n].  The
 * buffers must stay valid until the job is done; `in` is read when the job
 * joins a pass.  *job_id (host) receives the job's handle.  Errors: EINVAL
 * (n < 1, n > max_rows, target_n < 1, k outside 1..max_k). */
nanogs_status nanogs_batch_submit(nanogs_batch* b, const nanogs_gaussians* in,
                                  int64_t n, int64_t target_n, int32_t k,
                                  uint64_t seed, nanogs_gaussians* out,
                                  int32_t* d_origin, int32_t* job_id);

/* Cancels a queued or running job: its state becomes -NANOGS_ECANCELLED at
 * once, its output buffers are not written (those it was given may be
 * released after the next nanogs_batch_step), and a running job's rows
 * leave the working set at the next pass.  Cancelling a job that has
 * finished, failed or been cancelled has no effect.  Errors: EINVAL (bad
 * batch or job id). */
nanogs_status nanogs_batch_cancel(nanogs_batch* b, int32_t job_id);

/* One pass for every job in the working set; queued jobs join first, in
 * submission order, while their rows fit.  *n_done (nullable) receives the
 * number of jobs that completed (or failed) in this call.  Synchronises the
 * stream. */
nanogs_status nanogs_batch_step(nanogs_batch* b, int32_t* n_done);

/* Steps until every submitted job is done. */
nanogs_status nanogs_batch_run(nanogs_batch* b);

/* Job state: 0 queued, 1 running, 2 done (output written), or minus the
 * nanogs_status it failed with.  n_out and stats are nullable (host). */
nanogs_status nanogs_batch_job(const nanogs_batch* b, int32_t job_id,
                               int32_t* state, int64_t* n_out,
                               nanogs_stats* stats);

/* Splats currently held in the working set (admission control). */
int64_t nanogs_batch_rows_in_use(const nanogs_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* NANOGS_H */
