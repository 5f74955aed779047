/*
 * esom.h -- C ABI of libesom, EmbedSOM projection on AMD MI355X (gfx950).
 *
 * EmbedSOM (paper: "Scalable semi-supervised dimensionality reduction with
 * GPU-accelerated EmbedSOM", Section "Landmark-directed dimensionality
 * reduction") maps every high-dimensional point X_i (n x d) to a 2-D point
 * x_i (n x 2) using g landmarks with high-dimensional positions L (g x d) and
 * 2-D positions l (g x 2):
 *   1. find the k nearest landmarks of X_i (3 <= k <= g, Euclidean);
 *   2. give them smooth rank-ordered scores s (highest for the closest, zero
 *      for the k-th when k < g);
 *   3. for every pair (u,v) of neighbours, project X_i on the line through
 *      L_u (coordinate 0) and L_v (coordinate 1), giving D_uv;
 *   4. x_i = argmin_p sum s_u s_v (D_uv - d_uv(p))^2, where d_uv is the same
 *      affine coordinate in 2-D; a 2x2 linear system solved by Cramer's rule
 *      (Section "Projection step").
 *
 * Conventions for every call:
 *   - Array arguments are caller-owned.  Calls marked "device" take device
 *     pointers (e.g. from a torch tensor's data_ptr()); the library never
 *     frees them and keeps no reference after the work it enqueued finishes.
 *   - Device work is enqueued on `stream` (a hipStream_t; NULL = the default
 *     stream) and the call returns before it completes, unless stated.
 *   - Return value: ESOM_OK (0) or a negative ESOM_E* code.  Argument errors
 *     are detected synchronously and enqueue nothing.  esom_last_error()
 *     returns a thread-local message for the last failing call on the calling
 *     thread (valid until that thread's next call).
 *   - Inputs must be finite; NaN/Inf point values are not checked and give
 *     unspecified (but memory-safe) results for those points.
 *   - One context may be used from several host threads only if its calls
 *     are serialised by the caller; calls on one context share its scratch
 *     memory, so two esom_embed calls on one context must not run
 *     concurrently on different streams.  The serving API below manages its
 *     own per-slot scratch and may be used concurrently.
 */
#ifndef ESOM_H
#define ESOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ESOM_OK 0
#define ESOM_EINVAL (-1)    /* invalid argument (shape, parameter, pointer) */
#define ESOM_ENOMEM (-2)    /* device memory: allocation failed or over budget */
#define ESOM_EDEVICE (-3)   /* a HIP runtime call failed */
#define ESOM_EBUSY (-4)     /* serving queue full */
#define ESOM_ETIMEOUT (-5)  /* wait timed out; the request is still pending */
#define ESOM_ENOTFOUND (-6) /* unknown dataset or request id */

/* Limits of the library. */
#define ESOM_MAX_D 256   /* high-dimensional point dimension */
#define ESOM_MAX_K 64    /* neighbours */
#define ESOM_MAX_G 8192  /* landmarks */

typedef struct esom_ctx esom_ctx;

/* Distance pass precision.  Both modes return the exact k-nearest sets (ties
 * broken by landmark index) and the same projection; they differ in how the
 * candidate landmarks are screened:
 *   FP32:          BF16 MFMA threshold pass, FP32 MFMA candidate pass, exact
 *                  FP32 rescore of the candidates;
 *   BF16_RESCORE:  BF16 MFMA threshold pass, BF16 MFMA candidate pass on split
 *                  operands (high and low BF16 parts, three products per
 *                  element, FP32 accumulate), exact FP32 rescore of the
 *                  candidates.
 * In both modes every point is certified against a rigorous bound of the
 * screen's rounding error; uncertified points are recomputed exactly. */
typedef enum { ESOM_MODE_FP32 = 0, ESOM_MODE_BF16_RESCORE = 1 } esom_mode;

typedef struct {
    int32_t k;          /* neighbours, 3 <= k <= g and k <= ESOM_MAX_K */
    float boost;        /* score sharpness beta > 0 ("smoothing"; default 1) */
    float adjust;       /* pair weight exponent a: pair (u,v) is weighted
                           s_u s_v |l_v - l_u|^(2-2a); a = 1 (default) is the
                           paper's objective */
    float cutoff;       /* steepness A > 0 of the factor 1-exp(A(delta/delta_k-1))
                           that zeroes the k-th score when k < g (default 10) */
    float gravity;      /* eps >= 0: adds eps*sum_i s_i|p-l_{n_i}|^2 so the 2x2
                           system is never singular (default 1e-5) */
    int32_t mode;       /* esom_mode */
    int32_t candidates; /* screen target C: every point rescores at least
                           min(C, g) candidates; values below k act as k;
                           0 = default (k) */
} esom_params;

/* Counters accumulated by a context since creation or the last reset. */
typedef struct {
    int64_t n_points;      /* points embedded */
    int64_t n_fallback;    /* points recomputed by the exact FP64 path */
    int64_t n_uncertified; /* ...because the screen certificate failed */
    int64_t n_near_tie;    /* ...because the k-th and (k+1)-th distances are
                              closer than FP32 can order */
    int64_t n_illcond;     /* ...because the 2x2 system is ill-conditioned or a
                              landmark pair is nearly duplicate */
    int64_t n_degenerate;  /* ...because all k distances are equal or all scores
                              vanish (centroid of the neighbours' 2-D positions) */
    int64_t n_candidates;  /* total screened candidates rescored */
    int64_t n_slowpath;    /* points sent whole to the exact path because the
                              shape is outside the fast kernels (k > 32, d above
                              the mode's fast limit, or g > 4096) */
    int64_t n_timed;       /* embed calls timed (see esom_set_timing) */
    double ms_prep;        /* summed device time of landmark preparation (and of
                              the points' locality order where it outlasts it) */
    double ms_main;        /* summed device time of the fused embed kernel */
    double ms_exact;       /* summed device time of the exact FP64 path */
} esom_stats;

/* Fills *p with the defaults (k = 16, boost 1, adjust 1, cutoff 10,
 * gravity 1e-5, FP32 mode, default candidates). */
void esom_default_params(esom_params *p);

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context may hold (0 = no bound besides the device).
 * The context owns one extra HIP stream (default priority) and two events:
 * for 512 or more landmarks and 65536 or more points, esom_embed orders the
 * points for locality on that stream while the landmark preparation runs on
 * the caller's stream, and joins it before the main kernel (all after the
 * caller's earlier work on its stream; on the caller's stream itself while
 * that stream is being captured into a graph). */
int esom_create(int device, size_t hbm_budget_bytes, esom_ctx **out);

/* Waits for the context's outstanding work and frees everything it owns. */
void esom_destroy(esom_ctx *ctx);

/* Thread-local description of the last error on this thread ("" if none). */
const char *esom_last_error(void);

/* EmbedSOM projection (the four steps above) of n points.
 *   X        device, n rows of d floats, row stride ldx >= d floats, 4-byte aligned
 *   L_hd     device, g x d floats, row-major, contiguous
 *   L_2d     device, g x 2 floats, row-major, contiguous
 *   out      device, n x 2 floats (written)
 *   knn_idx  device, n x k int32 or NULL: the k nearest landmark indices, sorted
 *            by (exact distance, index): entries closer than FP32 rescoring can
 *            order are ranked again in FP64; -1 for a point without k finite
 *            distances (non-finite input), whose output is then NaN
 *   knn_dist2 device, n x k floats or NULL: their squared distances (FP32)
 * n == 0 is a no-op.  Errors: ESOM_EINVAL for k < 3, k > g, k > ESOM_MAX_K,
 * d < 1 or > ESOM_MAX_D, g > ESOM_MAX_G, n < 0, ldx < d, NULL or misaligned
 * pointers, boost <= 0, boost*sqrt(H_k) >= 80 (H_k the k-th harmonic number:
 * the largest score exponent), cutoff <= 0, gravity < 0, non-finite adjust,
 * unknown mode, candidates outside [0, g]; ESOM_ENOMEM if the scratch memory
 * does not fit the budget; ESOM_EDEVICE if a launch fails. */
int esom_embed(esom_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
               const float *L_hd, const float *L_2d, int32_t g, const esom_params *params,
               float *out, int32_t *knn_idx, float *knn_dist2, void *stream);

/* Allocation-free variant of esom_embed, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  It computes exactly what esom_embed
 * computes for the same arguments, with the same kernels, but needs no
 * context: its scratch (landmark preparation, the g x g pair table, the
 * exact-path list and counters) is one fixed device array of
 * ESOM_NOALLOC_SCRATCH_BYTES per GPU, part of the library's code object
 * (held by each GPU the library runs on until the process ends).  Points go
 * through in chunks sized to the array's room (more than a million points per
 * chunk at the largest landmark set), so n is not limited.  The first call on
 * a device resolves the array's address on that device; no call allocates.
 * Runs on the calling thread's current device.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from several host threads without ordering) race
 * and give undefined results; calls ordered on one stream are safe.
 * Arguments, outputs and errors as for esom_embed, plus ESOM_EINVAL for
 * g > ESOM_NOALLOC_MAX_G or d > ESOM_NOALLOC_MAX_D. */
#define ESOM_NOALLOC_SCRATCH_BYTES ((size_t)24 << 20)
#define ESOM_NOALLOC_MAX_G 1024
#define ESOM_NOALLOC_MAX_D 128
int esom_embed_noalloc(const float *X, int64_t n, int32_t d, int64_t ldx, const float *L_hd,
                       const float *L_2d, int32_t g, const esom_params *params, float *out,
                       int32_t *knn_idx, float *knn_dist2, void *stream);

/* One semi-supervised landmark step (Section "User supervision and model
 * interaction": an interactive k-means with a low learning rate in graph
 * mode, a SOM trained on the user's 2-D topology in SOM mode), batch form:
 *   b(i) = nearest landmark of X_i; S_j, c_j = sum and count of the points
 *   with b(i) = j;
 *   kind 0 (k-means): L_j += alpha (S_j / c_j - L_j) if c_j > 0;
 *   kind 1 (SOM):     L_j += alpha (sum_b h_jb S_b / sum_b h_jb c_b - L_j) if
 *                     the denominator is positive, h_jb = exp(-|l_j-l_b|^2 /
 *                     (2 sigma^2)) (sigma = 0: h_jb = [j == b]).
 *   L_hd     device, g x d floats, updated in place (stream-ordered)
 *   L_2d     device, g x 2 floats (read; may be NULL for kind 0)
 *   nearest  device, n int32 at stride nearest_ld >= 1 (elements), or NULL:
 *            b(i) from a previous esom_embed, e.g. its knn_idx with
 *            nearest_ld = k (the first column); NULL = computed here exactly.
 *            Entries outside [0, g) are ignored (the point counts nowhere).
 *   counts   device, g int32 or NULL: receives c_j
 * Sums and counts are accumulated in FP64, so the result does not depend on
 * the order in which points are visited beyond the final FP32 rounding.
 * Errors: ESOM_EINVAL for kind not 0/1, alpha not in [0,1], sigma < 0,
 * n < 0, d/g out of range, ldx < d, nearest_ld < 1 with nearest given, NULL
 * required pointers. */
int esom_landmark_update(esom_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx,
                         float *L_hd, const float *L_2d, int32_t g, int32_t kind, float alpha,
                         float sigma, const int32_t *nearest, int64_t nearest_ld, int32_t *counts,
                         void *stream);

/* Online SOM training (Section "Supervised training of self-organizing maps":
 * the user's 2-D landmarks are the map topology, the high-dimensional
 * landmarks are trained as its neuron weights, and the user sweeps the
 * neighbourhood size sigma and learning rate alpha, pausing or fixing parts
 * of the map at will).  Kohonen's online rule moves every landmark towards a
 * presented point x by alpha h(j, b) (x - L_j), with b the point's nearest
 * landmark (ties to the lower index) and h(j, b) = exp(-|l_j - l_b|^2 /
 * (2 sigma^2)) (h = [j == b] for sigma = 0).  Step t presents the `batch`
 * points X[batch_idx[t * batch + i]], finds their nearest landmarks against
 * the step's landmarks, and applies the average of their single-point updates:
 *   L_j += (alpha[t] / batch) sum_i h(j, b_i) (x_i - L_j)
 * (batch = 1 is the serial online rule).  Landmarks with frozen[j] != 0 keep
 * their position.  Batch entries outside [0, n) present no point but count
 * in `batch`.  The sums run in FP64; L_hd is rounded to FP32 after each step.
 *   X          device, n rows of d floats, row stride ldx
 *   L_hd       device, g x d floats, trained in place (stream-ordered)
 *   L_2d       device, g x 2 floats (the topology)
 *   batch_idx  device, steps x batch int32 point indices (the caller draws them)
 *   sigma, alpha  host, `steps` floats each: the schedule (sigma >= 0 finite,
 *              alpha in [0, 1]); read during the call
 *   frozen     device, g bytes, or NULL (none frozen)
 * steps == 0 is a no-op.  Errors: ESOM_EINVAL for batch < 1, steps < 0, bad
 * shapes (as esom_landmark_update), NULL arrays, schedule entries out of
 * range; ESOM_ENOMEM for scratch beyond the context budget. */
int esom_som_train(esom_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx, float *L_hd,
                   const float *L_2d, int32_t g, const int32_t *batch_idx, int32_t batch,
                   int32_t steps, const float *sigma, const float *alpha, const uint8_t *frozen,
                   void *stream);

/* High-dimensional positions of landmarks added to the map at 2-D positions
 * p_2d (Section "Supervised training of self-organizing maps": the initial
 * coordinates of a new landmark are fitted from the landmarks close to it in
 * 2-D).  For each new position p: its min(kfit, g) nearest 2-D landmarks (ties
 * to the lower index) get weights exp(-|l_j - p|^2 / (2 sigma^2)); an affine
 * map from 2-D to the d-dimensional space is fitted to them by weighted least
 * squares and evaluated at p (FP64).  When the neighbours determine no affine
 * map (fewer than three, or collinear in 2-D), their weighted mean is used.
 *   L_hd (g x d), L_2d (g x 2), p_2d (m x 2): device floats; L_new: device,
 *   m x d floats (written).  No context: runs on the current device.
 * Errors: ESOM_EINVAL for g, d out of range, m < 0, kfit outside [1, 64],
 * sigma not finite and > 0, NULL or misaligned arrays (m > 0). */
int esom_fit_landmarks(const float *L_hd, const float *L_2d, int32_t g, int32_t d, const float *p_2d,
                       int32_t m, int32_t kfit, float sigma, float *L_new, void *stream);

/* EmbedSOM projection into 3-D.  The paper states the method in 2-D for
 * brevity (Section "Landmark-directed dimensionality reduction"); with 3-D
 * landmark positions the same four steps give a 3 x 3 linear system per point
 * (normal equations of sum_{u<v} s_u s_v |h|^(2-2a) (D_uv - d_uv(p))^2 plus
 * gravity, h = l_v - l_u in 3-D), solved by Cramer's rule in FP64; a
 * degenerate neighbourhood or a numerically singular system (det <= 1e-9
 * (trace/3)^3) gives the centroid of the neighbours' 3-D positions.  The k
 * nearest landmarks are found exactly as by esom_embed (same screen, exact
 * selection and exact path); scores and pairs are then evaluated in FP64.
 *   L_3d     device, g x 3 floats
 *   out      device, n x 3 floats (written; NaN for a point without k finite distances)
 *   knn_idx  device, n x k int32 or NULL: the k nearest, as esom_embed returns them
 * Other arguments, limits and errors as for esom_embed. */
int esom_embed3(esom_ctx *ctx, const float *X, int64_t n, int32_t d, int64_t ldx, const float *L_hd,
                const float *L_3d, int32_t g, const esom_params *params, float *out, int32_t *knn_idx,
                void *stream);

/* ---------------------------------------------------------------- graph mode
 * Section "Semi-supervised structure reconstruction": the high-dimensional
 * landmarks follow an interactive k-means (esom_landmark_update, kind 0), their
 * 2-D positions a force-based layout of a neighbourhood graph of the
 * landmarks, which the user steers by dragging (fixing) nodes; landmarks are
 * added by duplicating one in both spaces, and removed. */
#define ESOM_GRAPH_MAX_K 32

/* Neighbourhood graph: for every landmark u its kg nearest other landmarks by
 * (squared distance, index), u excluded, distances as FP64 sums.
 *   L_hd  device, g x d floats;  nbr: device, g x kg int32 (written)
 *   dist2 device, g x kg floats or NULL: their squared distances
 * No context: runs on the current device.  Errors: ESOM_EINVAL for g outside
 * [2, ESOM_MAX_G], d out of range, kg outside [1, min(g - 1, ESOM_GRAPH_MAX_K)],
 * NULL or misaligned arrays. */
int esom_landmark_graph(const float *L_hd, int32_t g, int32_t d, int32_t kg, int32_t *nbr,
                        float *dist2, void *stream);

/* Force law of the layout (reading of the paper's "simple force-based graph
 * layout"): on every undirected edge u-v of the graph (v in u's list or u in
 * v's) a spring of rest length scale * |L_u - L_v|, force (r - rest) along the
 * edge (r the 2-D distance; none while r = 0); between all pairs a softened
 * repulsion of repulsion * (l_u - l_v) / (|l_u - l_v|^2 + softening^2).  Each
 * synchronous step moves every free node by step * force, shortened to
 * max_move.  Sums in FP64, positions stored as floats after every step. */
typedef struct {
    float scale;      /* 2-D length per unit of high-dimensional distance (>= 0) */
    float repulsion;  /* >= 0 */
    float softening;  /* > 0 */
    float step;       /* >= 0 */
    float max_move;   /* >= 0: longest move of a node per step */
} esom_layout_params;

/* Defaults: scale 1, repulsion 0.05, softening 0.5, step 0.1, max_move 0.5. */
void esom_default_layout_params(esom_layout_params *p);

/* Runs `steps` layout steps on L_2d (device, g x 2 floats, 8-byte aligned,
 * updated in place).  nbr: the graph (device, g x kg int32; -1 entries are
 * ignored).  fixed: device, g bytes or NULL; nodes with fixed[u] != 0 keep
 * their position (dragged by the user).  The context provides a g x 2 buffer
 * for the steps.  Errors: ESOM_EINVAL for shapes as esom_landmark_graph,
 * steps < 0, parameters not finite or negative (softening <= 0), NULL or
 * misaligned arrays; ESOM_ENOMEM for the buffer beyond the context budget. */
int esom_graph_layout(esom_ctx *ctx, const float *L_hd, int32_t g, int32_t d, const int32_t *nbr,
                      int32_t kg, float *L_2d, const uint8_t *fixed, int32_t steps,
                      const esom_layout_params *params, void *stream);

/* Adds landmark g as a duplicate of landmark j: row g of L_hd := row j, and
 * L_2d[g] := L_2d[j] + (dx, dy).  Both device arrays must hold g + 1 rows.
 * Errors: ESOM_EINVAL for g outside [1, ESOM_MAX_G), j outside [0, g),
 * non-finite offsets, NULL or misaligned arrays. */
int esom_landmark_duplicate(float *L_hd, float *L_2d, int32_t g, int32_t d, int32_t j, float dx,
                            float dy, void *stream);

/* Removes landmark j of g: the last landmark (g - 1) moves into slot j in both
 * arrays, leaving g - 1 landmarks (the caller's count).  Errors: ESOM_EINVAL for
 * g outside [2, ESOM_MAX_G], j outside [0, g), NULL or misaligned arrays. */
int esom_landmark_remove(float *L_hd, float *L_2d, int32_t g, int32_t d, int32_t j, void *stream);

/* ---------------------------------------------------------------- ablations
 * The paper's kernel families (Sections "k-NN step" and "Projection step"),
 * rebuilt for gfx950 in plain FP32 with the paper's work division and
 * caching, for measuring their relative merits against the fused kernel.
 * They have no screen, certificate or FP64 solve: results carry FP32
 * rounding (neighbour order among distances closer than FP32 resolves;
 * coordinates of ill-conditioned systems).
 * X is n x d row-major (contiguous), L_hd g x d, L_2d g x 2 (8-byte aligned).
 * ESOM_ABL_* select the algorithm; d <= 128, k <= 64. */
#define ESOM_ABL_KNN_BASE 0        /* one thread per point, global memory */
#define ESOM_ABL_KNN_SHARED 1      /* landmarks staged in LDS */
#define ESOM_ABL_KNN_GRIDINSERT 2  /* h points x w landmarks per block epoch */
#define ESOM_ABL_KNN_BITONIC 3     /* k threads per point, bitonic merges */
#define ESOM_ABL_PROJ_BASE 0       /* one thread per point */
#define ESOM_ABL_PROJ_SHARED 1     /* a block per point, neighbours in LDS */
#define ESOM_ABL_PROJ_ALIGNED 2    /* Shared with padded rows and float4 */
#define ESOM_ABL_PROJ_REGISTERS 3  /* Aligned with 2 x 2 pair groups per thread */

/* The k nearest landmarks of every point by FP32 distance (ties to the lower
 * index): knn_idx, knn_dist2 device n x k, sorted.  Errors: ESOM_EINVAL for an
 * unknown algo, d outside [1, 128], k outside [1, min(g, 64)], n out of range,
 * NULL or misaligned arrays. */
int esom_ablation_knn(int32_t algo, const float *X, int64_t n, int32_t d, const float *L_hd, int32_t g,
                      int32_t k, int32_t *knn_idx, float *knn_dist2, void *stream);

/* The projection (scores, segment projections, 2x2 Cramer, FP32) of every
 * point from its k sorted neighbours (knn_idx, knn_dist2 as esom_ablation_knn
 * returns them; indices must lie in [0, g), others are clamped into it);
 * out device n x 2.  Parameters as esom_embed (k = params->k,
 * mode ignored); degenerate neighbourhoods map to the neighbours' centroid.
 * Errors: as esom_ablation_knn plus the esom_embed parameter rules. */
int esom_ablation_project(int32_t algo, const float *X, int64_t n, int32_t d, const float *L_hd,
                          const float *L_2d, int32_t g, const esom_params *params, const int32_t *knn_idx,
                          const float *knn_dist2, float *out, void *stream);

/* Waits for the work enqueued on `stream`; ESOM_EDEVICE reports a device fault. */
int esom_sync(esom_ctx *ctx, void *stream);

/* Synchronises `stream`, then copies the context's counters into *stats
 * (host pointer); if reset != 0 the counters restart from zero. */
int esom_get_stats(esom_ctx *ctx, void *stream, esom_stats *stats, int32_t reset);

/* Diagnostics: the points that the last esom_embed (or landmark update
 * computing its own nearest landmarks) on this context handed from the fast
 * kernels to the exact FP64 path, in no particular order, with their reasons
 * as bit flags (1: screen certificate failed, 2: near tie of distances FP32
 * cannot order, 4: ill-conditioned system or nearly duplicate landmark pair,
 * 8: degenerate neighbourhood).  Synchronises `stream` first.  Copies at most
 * cap entries into the host arrays points / reasons (either may be NULL) and
 * stores the full count in *count.  Shapes outside the fast kernels send every
 * point to the exact path and list none (see n_slowpath).
 * Errors: ESOM_EINVAL for NULL ctx or count, cap < 0. */
int esom_get_fallback(esom_ctx *ctx, void *stream, int32_t *points, uint8_t *reasons, int64_t cap,
                      int64_t *count);

/* enable != 0: every following esom_embed on this context records HIP events
 * on its stream around the landmark preparation, the fused kernel and the
 * exact path; esom_get_stats adds their elapsed times to ms_prep / ms_main /
 * ms_exact.  Timing serialises nothing but costs four or five event records
 * per call. */
int esom_set_timing(esom_ctx *ctx, int32_t enable);

/* ---------------------------------------------------------------- serving
 * Continuous batching of embed requests on one GPU (the interactive loop in
 * which the paper re-projects all points every frame while the user edits
 * landmarks; Sections "User supervision and model interaction" and
 * "Accelerated EmbedSOM performance").  Requests with uneven n, d, g and k are
 * queued in arrival order and admitted as soon as one of the server's slots
 * is free and the request's device-memory footprint fits the budget beside
 * the resident datasets and the memory the other slots hold; admitted
 * requests run concurrently on separate HIP streams.  Each request computes
 * exactly what esom_embed computes for the same inputs (results do not depend
 * on what else runs).  Resident datasets cache their last k-nearest result:
 * a request that changes only 2-D landmarks reuses it and skips the distance
 * screen.  A frame on a resident dataset that repeats on a slot (same
 * dataset, shapes, parameters and cache use) is captured into a hipGraph the
 * second time and replayed after that; requests on a resident dataset go to a
 * free slot holding a graph of it when there is one.  All host pointers below are host memory; the server owns its
 * device and pinned staging memory.  Every submitted request must be waited
 * for (esom_serve_wait) to release its bookkeeping. */
typedef struct esom_server esom_server;

typedef struct {
    double submit_ms;      /* host steady-clock times, ms since esom_serve_create */
    double start_ms;       /* admitted to a slot */
    double done_ms;        /* result copied to out_host */
    int64_t n;             /* points */
    int32_t cache_hit;     /* 1: projected from the dataset's cached k nearest */
    int32_t graph_replay;  /* 1: replayed a captured frame */
    int32_t status;        /* ESOM_OK or the error of the device path */
    int32_t reserved;
} esom_request_info;

typedef struct {
    int64_t completed, failed, rejected, points, cache_hits, graph_replays;
    int64_t queued, in_flight, slots;
    int64_t budget_bytes, resident_bytes, held_bytes, peak_bytes;
    int64_t admission_waits; /* requests that waited at the head of the queue
                                for device memory (the budget) */
    int64_t max_queued;      /* deepest queue seen at submission */
    double now_ms;
} esom_serve_stats;

/* Creates a server on `device` with `n_slots` (1..16) concurrent request
 * slots; hbm_budget_bytes bounds datasets + caches + slot memory (0 = none). */
int esom_serve_create(int device, size_t hbm_budget_bytes, int32_t n_slots, esom_server **out);

/* Finishes every queued and running request, then frees everything. */
void esom_serve_destroy(esom_server *srv);

/* Copies n x d host floats (row-major) into a resident device dataset
 * (synchronous).  ESOM_ENOMEM if it does not fit the budget. */
int esom_serve_dataset_put(esom_server *srv, const float *X_host, int64_t n, int32_t d,
                           uint64_t *dataset_id);

/* Drops a resident dataset; its memory is freed once the requests that use it
 * have finished.  ESOM_ENOTFOUND for an unknown id. */
int esom_serve_dataset_drop(esom_server *srv, uint64_t dataset_id);

/* Queues one embed request and returns at once.
 *   dataset_id != 0: embed that resident dataset (X_host must be NULL; n, d ignored);
 *   dataset_id == 0: X_host (n x d host floats, pinned for best latency, valid
 *                    until the request completes) is uploaded with the request.
 *   L_hd_host (g x d) and L_2d_host (g x 2) are copied before the call returns.
 *   out_host (n x 2 floats) is written before esom_serve_wait reports success.
 * Errors: ESOM_EINVAL (arguments, as for esom_embed), ESOM_ENOTFOUND (dataset),
 * ESOM_ENOMEM (the footprint can never fit the budget beside the residents). */
int esom_serve_submit(esom_server *srv, uint64_t dataset_id, const float *X_host, int64_t n,
                      int32_t d, const float *L_hd_host, const float *L_2d_host, int32_t g,
                      const esom_params *params, float *out_host, uint64_t *request_id);

/* Waits up to timeout_ms (< 0: forever) for a request.  ESOM_OK: out_host holds
 * the result and *info (may be NULL) its timing; the id is then forgotten.
 * ESOM_ETIMEOUT: still pending.  ESOM_ENOTFOUND: unknown id.  Other codes: the
 * request failed on the device path (the id is forgotten). */
int esom_serve_wait(esom_server *srv, uint64_t request_id, int32_t timeout_ms,
                    esom_request_info *info);

/* Snapshot of the server's counters. */
int esom_serve_get_stats(esom_server *srv, esom_serve_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* ESOM_H */
