// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esom.h"

namespace esom {

// Screen tiles: 32 landmarks x 32 points per MFMA (v_mfma_f32_32x32x*).
constexpr int TILE = 32;
// Landmark count is padded to a multiple of 64 so tiles come in pairs.
constexpr int TILE_PAIR = 64;
// Fast-path limits (larger shapes go through the exact FP64 path).
constexpr int FAST_MAX_KP = 32;
constexpr int FAST_MAX_DC_BF16 = 8;  // d <= 128
constexpr int FAST_MAX_DC_FP32 = 4;  // d <= 64
constexpr int FAST_MAX_G = 4096;

// Counter slots (uint64) in the context's device counter array.
enum Counter {
    C_FB_LEN = 0,    // length of this call's fallback list (reset per call)
    C_POINTS = 1,
    C_FALLBACK = 2,
    C_UNCERT = 3,
    C_NEARTIE = 4,
    C_ILLCOND = 5,
    C_DEGEN = 6,
    C_CAND = 7,
    C_SLOW = 8,
    C_COUNT = 16,
};

// Fallback reasons (bit flags; a point may carry several).
enum Reason { R_UNCERT = 1, R_NEARTIE = 2, R_ILLCOND = 4, R_DEGEN = 8 };

// Prepared landmark set (device buffers owned by a scratch set).
struct Prep {
    int g = 0, d = 0, dp = 0, dc = 0, ntiles = 0, npairs = 0;
    int mode = 0;
    int need_pairs = 1;      // 0: the pair table is neither allocated nor filled
    float *cent = nullptr;   // dp      centroid of L (FP32 of an FP64 mean)
    void *A = nullptr;       // MFMA landmark operand a = -2 (L - c), tile layout: FP32 (FP32 mode) or
                             // its high BF16 parts ah = bf16(a) (BF16 mode)
    void *A16 = nullptr;     // FP32 mode: bf16(a) (threshold pass); BF16 mode: the low parts bf16(a - ah)
    float *norms = nullptr;  // ntiles * 32: |L_j - c|^2 in MFMA row order
    float *Lpad = nullptr;   // g * dp:  L rows padded with zeros to dp
    float *pairs = nullptr;  // g * g (when need_pairs): 1 / (2 |L_u - L_v|^2), 0 for coincident landmarks
    float *lmax = nullptr;   // 4:       max_j |L_j - c|, max_j |bf16(a_j) - a_j|, and of the split
                             //          a = ah + al + ra (BF16 mode): max_j |al_j|, max_j |ra_j|
    // Landmark order of the screen tiles, rows and pair table: position ->
    // landmark (perm) and landmark -> position (ipos).  Landmarks that are
    // close in the input space get nearby positions (see prep_order).
    int32_t *perm = nullptr;  // g
    int32_t *ipos = nullptr;  // g
    int32_t *pcl = nullptr;   // g: nearest ordering pivot (preparation scratch)
    float *pdist = nullptr;   // g: squared distance to it (preparation scratch)
    float *ppiv = nullptr;    // 64 x 64: pivot-to-pivot squared distances (scratch)
};

// Scratch memory for one in-flight embed (grows on demand).
struct Scratch {
    size_t cap_bytes = 0;
    void *base = nullptr;
    int64_t cap_n = 0;
    int32_t *fb_list = nullptr;     // fallback point list (cap_n)
    uint8_t *fb_reason = nullptr;   // per listed point reason flags (cap_n)
    float *fb_thresh = nullptr;     // per listed point: bound of its k-th distance^2 (cap_n)
    // materialised-distance path, for one chunk of mat_cap points
    int64_t mat_cap = 0;
    float *mat_keys = nullptr;      // mat_cap x gpad
    int32_t *mat_idx = nullptr;     // mat_cap x k
    float *mat_d2 = nullptr;        // mat_cap x k
    uint8_t *mat_mark = nullptr;    // mat_cap
    // locality order of the points (esom_bin.hip), for cap_n points
    uint8_t *pt_cell = nullptr;     // nearest pivot's place per point
    int32_t *pt_order = nullptr;    // processing order: slot -> point
    unsigned *bin_hist = nullptr;   // 2 x 64: points per pivot, then placement cursors
    // the locality order runs on a second stream beside the landmark
    // preparation when the context has one (none: on the call's stream)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    unsigned long long *counters = nullptr;  // C_COUNT
    Prep prep;
};

struct EmbedArgs {
    const float *X;
    int64_t n, ldx;
    int d, dp, g, ntiles, npair_tiles;
    const void *A;    // screen operand of the candidate pass (BF16 or FP32 by mode)
    const void *A16;  // FP32 mode: BF16 operand of the threshold pass; BF16 mode: low BF16 parts
    const float *norms, *cent, *Lpad, *l2d, *lmax;
    const float *pairs;
    const int32_t *perm, *ipos;  // position -> landmark, landmark -> position
    int k, kact, jsel;  // kact: neighbours with non-zero score; jsel: the screen's order statistic
    int pair_select;    // 1: jsel-th of a lane pair's 64 group minima; 0: per lane, larger of the two
    int use_cutoff;
    float boost, cutoff, gravity, adjust, Wk;
    float *out;
    int32_t *knn_idx;
    float *knn_d2;
    int32_t *fb_list;
    uint8_t *fb_reason;
    // Per listed point, an upper bound of the exact k-th nearest squared
    // distance (from the fast kernel's rescored k-th, widened by its rounding
    // bound), or +inf: the exact path only sorts landmarks within it.
    float *fb_thresh;
    unsigned long long *counters;
    int knn_only;  // 1: only write knn outputs (no projection)
    int lds_rows;  // 1: the block stages Lpad in LDS (row stride dp + 4 floats)
    int lds_tiles; // 1: the block stages the screen operands (A tiles, norms) in LDS
    int x_vec4;    // 1: d == dp, X 16-byte aligned and ldx % 4 == 0 (rows load as float4)
    // Optional per-point mark beside knn outputs (serving cache): 1 when the
    // point's neighbours came from the exact path because of the screen
    // (uncertified or near tie); a projection from cached neighbours sends
    // such points to the exact path again.
    uint8_t *knn_mark;
    // 1: adjacent neighbours FP32 cannot order go to the exact path, so that
    // knn_idx is sorted by exact distance (public calls that return the list)
    int knn_exact_order;
    // Optional processing order (slot -> point index, a permutation of 0..n-1):
    // the fused kernel's 64-point tiles take the points of consecutive slots.
    const int32_t *pt_order;
};

// Locality order of the points (esom_bin.hip): each point's nearest of the
// 64 ordering pivots (landmarks j g / 64, BF16 MFMA keys centred on landmark
// 0), then a counting sort by pivot.  Needs nothing from the landmark
// preparation, so it can run beside it.  Used for large landmark sets
// (g >= BIN_MIN_G) and calls of at least BIN_MIN_N points.
constexpr int BIN_MIN_G = 512;
constexpr int64_t BIN_MIN_N = 65536;
struct BinArgs {
    const float *X;
    int64_t n, ldx;
    int d, dp, g;
    const float *L;
    unsigned *hist;        // 2 x 64 (zeroed by launch_bin)
    uint8_t *cell;         // n
    int32_t *order;        // n
    int x_vec4;            // 1: d == dp, X 16-byte aligned, ldx % 4 == 0
};
hipError_t launch_bin(const BinArgs &b, int num_cus, hipStream_t s);

// Launchers (esom_core.hip).
hipError_t launch_prep(const Prep &P, const float *L, int mode, unsigned long long *counters,
                       long long n_points, hipStream_t s);
hipError_t launch_embed(const EmbedArgs &a, int mode, int kp, int num_cus, size_t lds_per_block,
                        hipStream_t s);
hipError_t launch_fallback(const EmbedArgs &a, int num_cus, size_t lds_per_block, hipStream_t s);
hipError_t launch_project(const EmbedArgs &a, int kp, int num_cus, hipStream_t s);
hipError_t launch_all_to_fallback(const EmbedArgs &a, int num_cus, size_t lds_per_block, hipStream_t s);
// Resets the fallback-list length (counters[C_FB_LEN]) with a one-thread kernel.
hipError_t launch_reset_fallback(unsigned long long *counters, hipStream_t s);

// Landmark update (esom_update.hip).
struct UpdateArgs {
    const float *X;
    int64_t n, ldx;
    int d, g, kind;
    float alpha, sigma;
    float *L;
    const float *l2d;
    const int32_t *nearest;
    int64_t nearest_ld;  // element stride of nearest
    int32_t *counts;
    const uint8_t *frozen = nullptr;  // kind 2: landmarks that keep their position
    int64_t batch = 1;                // kind 2: batch size of the averaged online step
};
size_t update_workspace_bytes(int64_t n, int g, int d);
hipError_t launch_update(const UpdateArgs &u, void *ws, int num_cus, hipStream_t s);

// The materialised-distance path (esom_materialise.hip): keys of a chunk of
// points in device memory, then selection, exact rescoring and certificate.
constexpr int MAT_MAX_C = 40;                    // candidates per point (k + 2, k <= 32)
constexpr size_t MAT_KEY_BYTES = (size_t)256 << 20;  // keys of one chunk at most
struct MatArgs {
    const float *X;      // the chunk's rows (stride ldx)
    int64_t n, ldx;      // points in the chunk
    int d, dp, g, gpad, ntiles, k, C, exact_order;
    const void *A;       // FP32 MFMA operand of the preparation (tile layout)
    const float *norms, *cent, *Lpad, *lmax;
    const int32_t *perm; // position -> landmark
    float *keys;         // n x gpad
    int32_t *knn_idx;    // n x k
    float *knn_d2;       // n x k
    uint8_t *knn_mark;   // n: 1 = the exact path decides this point
};
hipError_t launch_materialise(const MatArgs &m, int num_cus, hipStream_t s);

// Projection into 3-D from given k nearest landmarks (esom_embed3.hip).
struct Embed3Args {
    const float *X;
    int64_t n, ldx;
    int d, g, k, use_cutoff;
    const float *L, *l3;       // g x d, g x 3
    const int32_t *knn_idx;    // n x k (any order; entries outside [0, g): NaN output)
    double Wk;                 // the k-th harmonic number
    double boost, cutoff, gravity, adjust;
    float *out;                // n x 3
};
hipError_t launch_embed3(const Embed3Args &e, int num_cus, hipStream_t s);

// The paper's kernel families as ablations (esom_ablation.hip).
constexpr int ABL_MAX_K = 64;
constexpr int ABL_MAX_D = 128;
constexpr int ABL_LDS_FLOATS = 8192;  // landmark tile of the Shared k-NN kernel (32 KB)
struct AbProjArgs {
    const float *X, *L, *l2d;
    const int32_t *idx;
    const float *d2;
    int64_t n;
    int d, g, k;
    float boost, cutoff, gravity, adjust, Wk;
    float *out;
};
hipError_t launch_ablation_knn(int algo, const float *X, int64_t n, int d, const float *L, int g, int k,
                               int32_t *idx, float *d2, hipStream_t s);
hipError_t launch_ablation_project(int algo, const AbProjArgs &p, int num_cus, hipStream_t s);

// Graph-mode supervision (esom_graph.hip).
constexpr int GRAPH_MAX_K = 32;  // neighbours per landmark in the landmark graph
hipError_t launch_landmark_graph(const float *L, int g, int d, int kg, int32_t *nbr, float *dist2,
                                 hipStream_t s);
hipError_t launch_layout_step(const float *L, int g, int d, const int32_t *nbr, int kg, const float *lin,
                              float *lout, const uint8_t *fixed, double scale, double repulsion,
                              double soft, double step, double max_move, hipStream_t s);
hipError_t launch_duplicate(float *L, float *l2d, int g, int d, int j, float dx, float dy, hipStream_t s);
hipError_t launch_remove(float *L, float *l2d, int g, int d, int j, hipStream_t s);

// Online SOM training and the fit of added landmarks (esom_som.hip).
hipError_t launch_som_gather(const float *X, int64_t n, int64_t ldx, int d, const int32_t *rows, int B,
                             float *Xb, hipStream_t s);
hipError_t launch_som_mask(const int32_t *rows, int B, int64_t n, int32_t *nearest, hipStream_t s);
hipError_t launch_fit_landmarks(const float *L, const float *l2d, int g, int d, const float *p, int m,
                                int kfit, float sigma, float *out, hipStream_t s);

// Context-level helpers shared with the serving runtime (esom_api.cpp).
enum EmbedWhat { EMBED_FULL = 0, EMBED_KNN_ONLY = 1, EMBED_PROJECT = 2 };
int run_embed(esom_ctx *c, const float *X, int64_t n, int d, int64_t ldx, const float *L,
              const float *l2d, int g, const esom_params &P, float *out, int32_t *knn_idx,
              float *knn_d2, int what, hipStream_t s, uint8_t *knn_mark = nullptr,
              int exact_order = 0);
// The launch sequence of one embed on the given scratch (laid out by carve for
// at least min(n, chunk) points) and counters: landmark preparation, then per
// chunk of at most `chunk` points (chunk <= 0: all) the fast kernel and the
// exact path.  ev: 4 events recorded around the phases, or NULL.  Allocates nothing.
int enqueue_embed(Scratch &sc, unsigned long long *counters, int num_cus, size_t lds_per_block,
                  const float *X, int64_t n, int d, int64_t ldx, const float *L, const float *l2d,
                  int g, const esom_params &P, float *out, int32_t *knn_idx, float *knn_d2,
                  int what, hipStream_t s, uint8_t *knn_mark, hipEvent_t *ev, int64_t chunk,
                  int exact_order);
// Whether an embed of this shape reads the g x g pair table.
bool embed_needs_pairs(int d, int g, const esom_params &P, int what);
// Lays out an embed scratch at base (NULL: only sizes it) for n points, g
// landmarks, padded dimension dp and a pg x pg pair table; returns its bytes.
size_t carve(Scratch &sc, void *base, int64_t n, int g, int dp, int pg, int64_t mat_n = 0, int mat_k = 0);
// Points per chunk of the materialised-distance path for this shape, or 0 when
// the fused kernel (or the exact path) serves it.
int64_t mat_chunk(int64_t n, int d, int g, const esom_params &P, int what);
size_t ctx_held_bytes(const esom_ctx *c);
// Device address of the context's embed scratch (changes when it grows).
const void *ctx_arena(const esom_ctx *c);
void ctx_trim(esom_ctx *c);
// Bytes of an embed scratch for n points (with params: including the
// materialised-distance path's buffers when that shape takes it).
size_t embed_scratch_bytes(int64_t n, int g, int d, const esom_params *P = nullptr);
int fail_msg(int code, const char *msg);
// Checks the parameters of an embed over g landmarks (the esom_embed rules).
int validate_params(const esom_params &P, int g);
// Checks every esom_embed argument (shapes, parameters, pointers, alignment).
int validate_embed(const float *X, int64_t n, int d, int64_t ldx, const float *L_hd,
                   const float *L_2d, int g, const esom_params &P, const float *out,
                   const int32_t *knn_idx, const float *knn_dist2);

}  // namespace esom
