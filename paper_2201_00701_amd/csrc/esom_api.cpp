// C ABI of libesom: argument validation, context and scratch management, and
// the launch sequence of each entry point (see include/esom.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "esom_internal.h"

using namespace esom;

struct esom_ctx {
    int device = 0;
    int num_cus = 0;
    size_t lds_per_block = 65536;
    size_t budget = 0;  // 0 = unbounded
    size_t held = 0;    // bytes currently allocated
    unsigned long long *counters = nullptr;
    // embed scratch arena
    void *arena = nullptr;
    size_t arena_bytes = 0;
    int64_t cap_n = 0;
    int cap_g = 0, cap_dp = 0, cap_pg = 0;
    int64_t cap_mat = 0;
    int cap_mat_k = 0;
    Scratch sc;
    // landmark-update workspace
    void *uws = nullptr;
    size_t uws_bytes = 0;
    // online SOM training: the gathered batch
    float *som_xb = nullptr;
    size_t som_xb_bytes = 0;
    int32_t *nearest = nullptr;
    int64_t nearest_cap = 0;
    // 3-D projection: neighbour lists when the caller asks for none
    int32_t *k3idx = nullptr;
    size_t k3idx_bytes = 0;
    // graph layout: the other position buffer of the synchronous steps
    float *lay = nullptr;
    size_t lay_bytes = 0;
    // optional per-kernel timing: pending event quadruples (prep, main, exact, end)
    bool timing = false;
    std::vector<hipEvent_t> pending;
    int64_t n_timed = 0;
    double ms_prep = 0.0, ms_main = 0.0, ms_exact = 0.0;
};

namespace {

thread_local std::string t_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(ESOM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

int dev_alloc(esom_ctx *c, void **p, size_t bytes) {
    if (c->budget && c->held + bytes > c->budget)
        return fail(ESOM_ENOMEM, "scratch of %zu bytes exceeds the context budget (%zu held of %zu)",
                    bytes, c->held, c->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(ESOM_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    c->held += bytes;
    return ESOM_OK;
}

void dev_free(esom_ctx *c, void *&p, size_t bytes) {
    if (p) {
        (void)hipFree(p);
        c->held -= bytes;
        p = nullptr;
    }
}

}  // namespace

namespace esom {
// Lays the embed scratch out for (n, g, dp) capacities; the pair table holds
// pg x pg entries (0 when no call so far needed it).
size_t carve(Scratch &sc, void *base, int64_t n, int g, int dp, int pg, int64_t mat_n, int mat_k) {
    const int ntiles = ((g + TILE_PAIR - 1) / TILE_PAIR) * 2;
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *r = base ? p + off : nullptr;
        off += align256(bytes);
        return r;
    };
    sc.prep.cent = static_cast<float *>(take(sizeof(float) * dp));
    sc.prep.A = take(sizeof(float) * (size_t)ntiles * TILE * dp);
    sc.prep.A16 = take(sizeof(uint16_t) * (size_t)ntiles * TILE * dp);
    sc.prep.norms = static_cast<float *>(take(sizeof(float) * (size_t)ntiles * TILE));
    sc.prep.Lpad = static_cast<float *>(take(sizeof(float) * (size_t)g * dp));
    sc.prep.pairs = pg > 0 ? static_cast<float *>(take(sizeof(float) * (size_t)pg * pg)) : nullptr;
    sc.prep.lmax = static_cast<float *>(take(4 * sizeof(float)));
    sc.prep.perm = static_cast<int32_t *>(take(sizeof(int32_t) * (size_t)g));
    sc.prep.ipos = static_cast<int32_t *>(take(sizeof(int32_t) * (size_t)g));
    sc.prep.pcl = static_cast<int32_t *>(take(sizeof(int32_t) * (size_t)g));
    sc.prep.pdist = static_cast<float *>(take(sizeof(float) * (size_t)g));
    sc.prep.ppiv = static_cast<float *>(take(sizeof(float) * 64 * 64));
    sc.fb_list = static_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
    sc.fb_reason = static_cast<uint8_t *>(take((size_t)(n > 0 ? n : 1)));
    sc.fb_thresh = static_cast<float *>(take(sizeof(float) * (size_t)(n > 0 ? n : 1)));
    sc.pt_cell = static_cast<uint8_t *>(take((size_t)(n > 0 ? n : 1)));
    sc.pt_order = static_cast<int32_t *>(take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)));
    sc.bin_hist = static_cast<unsigned *>(take(sizeof(unsigned) * 128));
    sc.mat_cap = mat_n;
    if (mat_n > 0) {
        sc.mat_keys = static_cast<float *>(take(sizeof(float) * (size_t)mat_n * ntiles * TILE));
        sc.mat_idx = static_cast<int32_t *>(take(sizeof(int32_t) * (size_t)mat_n * mat_k));
        sc.mat_d2 = static_cast<float *>(take(sizeof(float) * (size_t)mat_n * mat_k));
        sc.mat_mark = static_cast<uint8_t *>(take((size_t)mat_n));
    } else {
        sc.mat_keys = nullptr;
        sc.mat_idx = nullptr;
        sc.mat_d2 = nullptr;
        sc.mat_mark = nullptr;
    }
    return off;
}
}  // namespace esom

namespace {

int ensure_scratch(esom_ctx *c, int64_t n, int g, int dp, int pg, hipStream_t s, int64_t mat_n = 0,
                   int mat_k = 0) {
    if (c->arena && n <= c->cap_n && g <= c->cap_g && dp <= c->cap_dp && pg <= c->cap_pg &&
        (mat_n == 0 || (mat_n <= c->cap_mat && mat_k <= c->cap_mat_k)))
        return ESOM_OK;
    int64_t nn = n > c->cap_n ? n + n / 4 : c->cap_n;
    int gg = g > c->cap_g ? g : c->cap_g;
    int dd = dp > c->cap_dp ? dp : c->cap_dp;
    int pp = pg > c->cap_pg ? pg : c->cap_pg;
    int64_t mm = mat_n > c->cap_mat ? mat_n : c->cap_mat;
    int mk = mat_k > c->cap_mat_k ? mat_k : c->cap_mat_k;
    const size_t bytes = carve(c->sc, nullptr, nn, gg, dd, pp, mm, mk);
    if (c->arena) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        dev_free(c, c->arena, c->arena_bytes);
        c->arena_bytes = 0;
    }
    int st = dev_alloc(c, &c->arena, bytes);
    if (st != ESOM_OK) {
        c->cap_n = c->cap_g = c->cap_dp = c->cap_pg = 0;
        c->cap_mat = 0;
        c->cap_mat_k = 0;
        return st;
    }
    c->arena_bytes = bytes;
    carve(c->sc, c->arena, nn, gg, dd, pp, mm, mk);
    c->cap_n = nn;
    c->cap_g = gg;
    c->cap_dp = dd;
    c->cap_pg = pp;
    c->cap_mat = mm;
    c->cap_mat_k = mk;
    return ESOM_OK;
}

double harmonic(int k) {
    double h = 0.0;
    for (int i = 1; i <= k; ++i) h += 1.0 / i;
    return h;
}

int validate_common(const float *X, int64_t n, int32_t d, int64_t ldx, const float *L, int32_t g) {
    if (n < 0) return fail(ESOM_EINVAL, "n = %lld < 0", (long long)n);
    if (d < 1 || d > ESOM_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ESOM_MAX_D);
    if (g < 1 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [1, %d]", g, ESOM_MAX_G);
    if (ldx < d) return fail(ESOM_EINVAL, "ldx = %lld < d = %d", (long long)ldx, d);
    if (!L || !aligned4(L)) return fail(ESOM_EINVAL, "L_hd is NULL or not 4-byte aligned");
    if (n > 0 && (!X || !aligned4(X))) return fail(ESOM_EINVAL, "X is NULL or not 4-byte aligned");
    if (n > (int64_t)INT32_MAX) return fail(ESOM_EINVAL, "n = %lld exceeds 2^31 - 1", (long long)n);
    return ESOM_OK;
}

struct Plan {
    int dp, dc, kp, C, jsel, pair_select;
    bool fast;
    bool mat;  // the materialised-distance path (d beyond the fused kernel's budget)
};

Plan make_plan(int d, int g, int k, int mode, int candidates) {
    Plan p;
    p.dp = 16 * ((d + 15) / 16);
    p.dc = p.dp / 16;
    p.kp = k <= 8 ? 8 : k <= 16 ? 16 : k <= 20 ? 20 : k <= 24 ? 24 : k <= 32 ? 32 : 0;
    const int maxdc = mode == 1 ? FAST_MAX_DC_BF16 : FAST_MAX_DC_FP32;
    p.fast = p.kp != 0 && p.dc <= maxdc && g <= FAST_MAX_G;
    p.mat = !p.fast && p.kp != 0 && g <= FAST_MAX_G && p.dp <= ESOM_MAX_D;
    int C = candidates > 0 ? candidates : k;
    if (C < k) C = k;
    p.C = C;
    // C <= 32: the C-th of a lane pair's 64 group minima; beyond, each lane's
    // ceil(C / 2)-th (at most 32), the larger of the two
    p.pair_select = C <= 32 ? 1 : 0;
    p.jsel = p.pair_select ? C : (C + 1) / 2;
    if (p.jsel > 32) p.jsel = 32;
    if (p.jsel < 1) p.jsel = 1;
    return p;
}

}  // namespace

namespace esom {
// Enqueues preparation + fast kernel + exact path.  what: EMBED_FULL,
// EMBED_KNN_ONLY (k nearest only) or EMBED_PROJECT (scores/pairs/solve from
// the given knn_idx / knn_d2).
bool embed_needs_pairs(int d, int g, const esom_params &P, int what) {
    const Plan pl = make_plan(d, g, P.k, P.mode, P.candidates);
    // the pair table is read only by the fast kernels' projection
    return what != EMBED_KNN_ONLY && pl.kp != 0 && (what == EMBED_PROJECT || pl.fast || pl.mat);
}

int64_t mat_chunk(int64_t n, int d, int g, const esom_params &P, int what) {
    const Plan pl = make_plan(d, g, P.k, P.mode, P.candidates);
    if (!pl.mat || what != EMBED_FULL) return 0;
    const int64_t gpad = ((g + TILE_PAIR - 1) / TILE_PAIR) * TILE_PAIR;
    int64_t m = (int64_t)(MAT_KEY_BYTES / (sizeof(float) * (size_t)gpad));
    m &= ~(int64_t)63;
    if (m < 64) m = 64;
    return n < m ? n : m;
}

int enqueue_embed(Scratch &sc, unsigned long long *counters, int num_cus, size_t lds_per_block,
                  const float *X, int64_t n, int d, int64_t ldx, const float *L, const float *l2d,
                  int g, const esom_params &P, float *out, int32_t *knn_idx, float *knn_d2,
                  int what, hipStream_t s, uint8_t *knn_mark, hipEvent_t *ev, int64_t chunk,
                  int exact_order) {
    const int knn_only = what == EMBED_KNN_ONLY;
    const Plan pl = make_plan(d, g, P.k, P.mode, P.candidates);
    const bool need_pairs = embed_needs_pairs(d, g, P, what);
    // shapes beyond the fused kernel's register budget take the
    // materialised-distance path when the scratch holds its buffers (the
    // allocation-free entry point sends them to the exact path instead)
    const bool use_mat = pl.mat && what == EMBED_FULL && sc.mat_cap > 0;
    const int prep_mode = use_mat ? ESOM_MODE_FP32 : P.mode;  // FP32 keys on that path
    Prep &pr = sc.prep;
    pr.g = g;
    pr.d = d;
    pr.dp = pl.dp;
    pr.dc = pl.dc;
    pr.ntiles = ((g + TILE_PAIR - 1) / TILE_PAIR) * 2;
    pr.npairs = pr.ntiles / 2;
    pr.mode = prep_mode;
    pr.need_pairs = need_pairs ? 1 : 0;
    if (chunk <= 0 || chunk > n) chunk = n;
    if (use_mat && chunk > sc.mat_cap) chunk = sc.mat_cap;
    // Large landmark sets: the points go through the fused kernel in locality
    // order (nearest ordering pivot), so that a wavefront's points share
    // pair-table lines, landmark rows and candidate words; no result changes.
    // With a second stream and the whole call in one chunk (and no graph
    // capture on the call's stream) the order is built beside the landmark
    // preparation; otherwise per chunk on the call's stream.
    const bool bin_all = pl.fast && what == EMBED_FULL && g >= BIN_MIN_G && n >= BIN_MIN_N;
    auto bin_args = [&](const float *Xc, int64_t m) {
        BinArgs bb;
        bb.X = Xc;
        bb.n = m;
        bb.ldx = ldx;
        bb.d = d;
        bb.dp = pl.dp;
        bb.g = g;
        bb.L = L;
        bb.hist = sc.bin_hist;
        bb.cell = sc.pt_cell;
        bb.order = sc.pt_order;
        bb.x_vec4 = (d == pl.dp && ldx % 4 == 0 && ((uintptr_t)Xc & 15) == 0) ? 1 : 0;
        return bb;
    };
    bool bin_side = false;
    if (bin_all && sc.side && chunk >= n) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const hipError_t qe = hipStreamIsCapturing(s, &cs);
        if (qe != hipSuccess) (void)hipGetLastError();  // unknown: build the order on the call's stream
        if (qe == hipSuccess && cs == hipStreamCaptureStatusNone) {
            hipError_t e = hipEventRecord(sc.fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(sc.side, sc.fork, 0);
            if (e == hipSuccess) e = launch_bin(bin_args(X, n), num_cus, sc.side);
            if (e == hipSuccess) e = hipEventRecord(sc.join, sc.side);
            if (e != hipSuccess) return hip_fail(e, "point binning launch");
            bin_side = true;
        }
    }
    if (ev) (void)hipEventRecord(ev[0], s);
    hipError_t e = launch_prep(pr, L, prep_mode, counters, knn_only ? 0 : (long long)n, s);
    if (e != hipSuccess) return hip_fail(e, "landmark preparation launch");
    if (ev) (void)hipEventRecord(ev[1], s);

    EmbedArgs a;
    memset(&a, 0, sizeof a);
    a.ldx = ldx;
    a.d = d;
    a.dp = pl.dp;
    a.g = g;
    a.ntiles = pr.ntiles;
    a.npair_tiles = pr.npairs;
    a.A = pr.A;
    a.A16 = pr.A16;
    a.norms = pr.norms;
    a.cent = pr.cent;
    a.Lpad = pr.Lpad;
    a.l2d = l2d;
    a.pairs = pr.pairs;
    a.lmax = pr.lmax;
    a.perm = pr.perm;
    a.ipos = pr.ipos;
    a.k = P.k;
    a.kact = P.k < g ? P.k - 1 : P.k;
    a.jsel = pl.jsel;
    a.pair_select = pl.pair_select;
    a.use_cutoff = P.k < g ? 1 : 0;
    a.boost = P.boost;
    a.cutoff = P.cutoff;
    a.gravity = P.gravity;
    a.adjust = P.adjust;
    a.Wk = (float)harmonic(P.k);
    a.fb_list = sc.fb_list;
    a.fb_reason = sc.fb_reason;
    a.fb_thresh = sc.fb_thresh;
    a.counters = counters;
    a.knn_only = knn_only;
    a.knn_exact_order = (exact_order && knn_idx) ? 1 : 0;
    // Points go in chunks of at most `chunk` (the fallback list's capacity):
    // each chunk is screened, then its listed points are recomputed, before
    // the next chunk reuses the list.
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int64_t m = n - c0 < chunk ? n - c0 : chunk;
        if (c0 > 0) {
            e = launch_reset_fallback(counters, s);
            if (e != hipSuccess) return hip_fail(e, "counter reset launch");
        }
        a.X = X + c0 * ldx;
        a.n = m;
        a.out = out ? out + 2 * c0 : nullptr;
        a.knn_idx = knn_idx ? knn_idx + c0 * P.k : nullptr;
        a.knn_d2 = knn_d2 ? knn_d2 + c0 * P.k : nullptr;
        a.knn_mark = knn_mark ? knn_mark + c0 : nullptr;
        a.x_vec4 = (d == pl.dp && ldx % 4 == 0 && ((uintptr_t)a.X & 15) == 0 &&
                    ((uintptr_t)pr.cent & 15) == 0) ? 1 : 0;
        const bool last = c0 + m >= n;
        if (what == EMBED_PROJECT && pl.kp != 0) {
            e = launch_project(a, pl.kp, num_cus, s);
            if (e != hipSuccess) return hip_fail(e, "projection kernel launch");
            if (ev && last) (void)hipEventRecord(ev[2], s);
            e = launch_fallback(a, num_cus, lds_per_block, s);
            if (e != hipSuccess) return hip_fail(e, "exact-path launch");
        } else if (use_mat) {
            MatArgs mm;
            mm.X = a.X;
            mm.n = m;
            mm.ldx = ldx;
            mm.d = d;
            mm.dp = pl.dp;
            mm.g = g;
            mm.ntiles = pr.ntiles;
            mm.gpad = pr.ntiles * TILE;
            mm.k = P.k;
            mm.C = P.k + 2 < g ? P.k + 2 : g;
            mm.exact_order = a.knn_exact_order;
            mm.A = pr.A;
            mm.norms = pr.norms;
            mm.cent = pr.cent;
            mm.Lpad = pr.Lpad;
            mm.lmax = pr.lmax;
            mm.perm = pr.perm;
            mm.keys = sc.mat_keys;
            mm.knn_idx = a.knn_idx ? a.knn_idx : sc.mat_idx;
            mm.knn_d2 = a.knn_d2 ? a.knn_d2 : sc.mat_d2;
            mm.knn_mark = a.knn_mark ? a.knn_mark : sc.mat_mark;
            e = launch_materialise(mm, num_cus, s);
            if (e != hipSuccess) return hip_fail(e, "materialised-distance launch");
            // the projection from those neighbours; marked points go to the exact path
            EmbedArgs ap = a;
            ap.knn_idx = mm.knn_idx;
            ap.knn_d2 = mm.knn_d2;
            ap.knn_mark = mm.knn_mark;
            e = launch_project(ap, pl.kp, num_cus, s);
            if (e != hipSuccess) return hip_fail(e, "projection kernel launch");
            if (ev && last) (void)hipEventRecord(ev[2], s);
            e = launch_fallback(ap, num_cus, lds_per_block, s);
            if (e != hipSuccess) return hip_fail(e, "exact-path launch");
        } else if (pl.fast) {
            a.pt_order = nullptr;
            if (bin_side) {
                e = hipStreamWaitEvent(s, sc.join, 0);
                if (e != hipSuccess) return hip_fail(e, "point binning join");
                a.pt_order = sc.pt_order;
                // the fused kernel's timing starts after the join: whatever of
                // the locality order outlasts the landmark preparation counts
                // as preparation
                if (ev) (void)hipEventRecord(ev[1], s);
            } else if (bin_all && m >= BIN_MIN_N) {
                e = launch_bin(bin_args(a.X, m), num_cus, s);
                if (e != hipSuccess) return hip_fail(e, "point binning launch");
                a.pt_order = sc.pt_order;
            }
            e = launch_embed(a, P.mode, pl.kp, num_cus, lds_per_block, s);
            if (e != hipSuccess) return hip_fail(e, "embed kernel launch");
            if (ev && last) (void)hipEventRecord(ev[2], s);
            e = launch_fallback(a, num_cus, lds_per_block, s);
            if (e != hipSuccess) return hip_fail(e, "exact-path launch");
        } else {
            if (ev && last) (void)hipEventRecord(ev[2], s);
            e = launch_all_to_fallback(a, num_cus, lds_per_block, s);
            if (e != hipSuccess) return hip_fail(e, "exact-path launch");
        }
    }
    if (ev) (void)hipEventRecord(ev[3], s);
    return ESOM_OK;
}

int run_embed(esom_ctx *c, const float *X, int64_t n, int d, int64_t ldx, const float *L,
              const float *l2d, int g, const esom_params &P, float *out, int32_t *knn_idx,
              float *knn_d2, int what, hipStream_t s, uint8_t *knn_mark, int exact_order) {
    const Plan pl = make_plan(d, g, P.k, P.mode, P.candidates);
    const int64_t mat_n = mat_chunk(n, d, g, P, what);
    int st = ensure_scratch(c, n, g, pl.dp, embed_needs_pairs(d, g, P, what) ? g : 0, s, mat_n,
                            mat_n ? P.k : 0);
    if (st != ESOM_OK) return st;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timed = c->timing && what != EMBED_KNN_ONLY;
    if (timed) {
        for (int i = 0; i < 4; ++i) {
            hipError_t ee = hipEventCreate(&ev[i]);
            if (ee != hipSuccess) return hip_fail(ee, "hipEventCreate");
        }
    }
    st = enqueue_embed(c->sc, c->counters, c->num_cus, c->lds_per_block, X, n, d, ldx, L, l2d, g, P,
                       out, knn_idx, knn_d2, what, s, knn_mark, timed ? ev : nullptr, n, exact_order);
    if (timed) {
        if (st == ESOM_OK) {
            for (int i = 0; i < 4; ++i) c->pending.push_back(ev[i]);
        } else {
            for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
        }
    }
    return st;
}

size_t ctx_held_bytes(const esom_ctx *c) { return c->held; }

const void *ctx_arena(const esom_ctx *c) { return c->arena; }

void ctx_trim(esom_ctx *c) {
    dev_free(c, c->arena, c->arena_bytes);
    c->arena_bytes = 0;
    c->cap_n = c->cap_g = c->cap_dp = c->cap_pg = 0;
    c->cap_mat = 0;
    c->cap_mat_k = 0;
}

size_t embed_scratch_bytes(int64_t n, int g, int d, const esom_params *P) {
    Scratch sc;
    const int64_t mat_n = P ? mat_chunk(n, d, g, *P, EMBED_FULL) : 0;
    return carve(sc, nullptr, n, g, 16 * ((d + 15) / 16), g, mat_n, mat_n ? P->k : 0);
}

int fail_msg(int code, const char *msg) { return fail(code, "%s", msg); }

int validate_embed(const float *X, int64_t n, int d, int64_t ldx, const float *L_hd,
                   const float *L_2d, int g, const esom_params &P, const float *out,
                   const int32_t *knn_idx, const float *knn_dist2) {
    int st = validate_common(X, n, d, ldx, L_hd, g);
    if (st != ESOM_OK) return st;
    st = validate_params(P, g);
    if (st != ESOM_OK) return st;
    if (!L_2d || !aligned4(L_2d)) return fail(ESOM_EINVAL, "L_2d is NULL or not 4-byte aligned");
    if (n > 0 && (!out || ((uintptr_t)out & 7u)))
        return fail(ESOM_EINVAL, "out is NULL or not 8-byte aligned");
    if ((knn_idx && !aligned4(knn_idx)) || (knn_dist2 && !aligned4(knn_dist2)))
        return fail(ESOM_EINVAL, "knn outputs must be 4-byte aligned");
    if (((uintptr_t)L_2d & 7u)) return fail(ESOM_EINVAL, "L_2d must be 8-byte aligned");
    return ESOM_OK;
}

int validate_params(const esom_params &P, int g) {
    if (g < 3 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [3, %d]", g, ESOM_MAX_G);
    if (P.k < 3 || P.k > g || P.k > ESOM_MAX_K)
        return fail(ESOM_EINVAL, "k = %d outside [3, min(g = %d, %d)]", P.k, g, ESOM_MAX_K);
    if (!(P.boost > 0.f) || !(P.boost * sqrt(harmonic(P.k)) < 80.0))
        return fail(ESOM_EINVAL, "boost = %g must be > 0 with boost*sqrt(H_k) < 80", (double)P.boost);
    if (!(P.cutoff > 0.f) || !isfinite(P.cutoff))
        return fail(ESOM_EINVAL, "cutoff = %g must be finite and > 0", (double)P.cutoff);
    if (!(P.gravity >= 0.f) || !isfinite(P.gravity))
        return fail(ESOM_EINVAL, "gravity = %g must be finite and >= 0", (double)P.gravity);
    if (!isfinite(P.adjust)) return fail(ESOM_EINVAL, "adjust must be finite");
    if (P.mode != ESOM_MODE_FP32 && P.mode != ESOM_MODE_BF16_RESCORE)
        return fail(ESOM_EINVAL, "unknown mode %d", P.mode);
    if (P.candidates < 0 || P.candidates > g)
        return fail(ESOM_EINVAL, "candidates = %d outside [0, g]", P.candidates);
    return ESOM_OK;
}

}  // namespace esom

// ---------------------------------------------------------------- allocation-free embed
// One fixed device array per GPU holds everything an embed needs beyond its
// inputs and outputs: the counters (first 256 bytes), then one embed scratch
// (landmark preparation, pair table, exact-path list of one chunk of points).
// In host code `scratch` names a host-side stand-in; its device address on
// each GPU comes from hipGetSymbolAddress, resolved once per device.
static __device__ __align__(256) unsigned char scratch[ESOM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr size_t NOALLOC_COUNTER_BYTES = 256;
static_assert(sizeof(unsigned long long) * C_COUNT <= NOALLOC_COUNTER_BYTES, "counter slots");

struct NoallocDevice {
    std::once_flag once;
    hipError_t err = hipSuccess;
    unsigned char *ptr = nullptr;  // device address of `scratch` on this device
    int num_cus = 0;
    size_t lds_per_block = 0;
};
NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// Resolves the array's address and the launch attributes of the current
// device (once per device).
void noalloc_setup(NoallocDevice &nd) {
    nd.err = hipGetSymbolAddress(reinterpret_cast<void **>(&nd.ptr), HIP_SYMBOL(scratch));
    if (nd.err != hipSuccess) return;
    int dev = 0, cus = 0, lds = 0;
    nd.err = hipGetDevice(&dev);
    if (nd.err == hipSuccess) nd.err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (nd.err == hipSuccess)
        nd.err = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    nd.num_cus = cus;
    nd.lds_per_block = (size_t)lds;
}

}  // namespace

extern "C" {

void esom_default_params(esom_params *p) {
    if (!p) return;
    p->k = 16;
    p->boost = 1.0f;
    p->adjust = 1.0f;
    p->cutoff = 10.0f;
    p->gravity = 1e-5f;
    p->mode = ESOM_MODE_FP32;
    p->candidates = 0;
}

const char *esom_last_error(void) { return t_err.c_str(); }

int esom_create(int device, size_t hbm_budget_bytes, esom_ctx **out) {
    t_err.clear();
    if (!out) return fail(ESOM_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev)
        return fail(ESOM_EINVAL, "device %d outside [0, %d)", device, ndev);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    esom_ctx *c = new esom_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    c->num_cus = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    int st = dev_alloc(c, reinterpret_cast<void **>(&c->counters),
                       sizeof(unsigned long long) * C_COUNT);
    if (st != ESOM_OK) {
        delete c;
        return st;
    }
    e = hipMemset(c->counters, 0, sizeof(unsigned long long) * C_COUNT);
    if (e != hipSuccess) {
        dev_free(c, reinterpret_cast<void *&>(c->counters), sizeof(unsigned long long) * C_COUNT);
        delete c;
        return hip_fail(e, "hipMemset");
    }
    // second stream for the locality order (default priority); without it
    // the order runs on the call's stream
    if (hipStreamCreateWithFlags(&c->sc.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->sc.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->sc.join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (c->sc.fork) (void)hipEventDestroy(c->sc.fork);
        if (c->sc.side) (void)hipStreamDestroy(c->sc.side);
        c->sc.side = nullptr;
        c->sc.fork = c->sc.join = nullptr;
    }
    *out = c;
    return ESOM_OK;
}

int esom_get_fallback(esom_ctx *c, void *stream, int32_t *points, uint8_t *reasons, int64_t cap,
                      int64_t *count) {
    t_err.clear();
    if (!c || !count) return fail(ESOM_EINVAL, "ctx or count is NULL");
    if (cap < 0) return fail(ESOM_EINVAL, "cap = %lld < 0", (long long)cap);
    int st = esom_sync(c, stream);
    if (st != ESOM_OK) return st;
    unsigned long long len = 0;
    hipError_t e = hipMemcpy(&len, c->counters + C_FB_LEN, sizeof len, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    if (!c->arena) len = 0;
    if (len > (unsigned long long)c->cap_n) len = (unsigned long long)c->cap_n;
    *count = (int64_t)len;
    const size_t m = (size_t)((int64_t)len < cap ? (int64_t)len : cap);
    if (m && points) {
        e = hipMemcpy(points, c->sc.fb_list, m * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    if (m && reasons) {
        e = hipMemcpy(reasons, c->sc.fb_reason, m, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    return ESOM_OK;
}

int esom_set_timing(esom_ctx *c, int32_t enable) {
    t_err.clear();
    if (!c) return fail(ESOM_EINVAL, "ctx is NULL");
    c->timing = enable != 0;
    return ESOM_OK;
}

void esom_destroy(esom_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t ev : c->pending) (void)hipEventDestroy(ev);
    c->pending.clear();
    dev_free(c, c->arena, c->arena_bytes);
    dev_free(c, c->uws, c->uws_bytes);
    dev_free(c, reinterpret_cast<void *&>(c->som_xb), c->som_xb_bytes);
    dev_free(c, reinterpret_cast<void *&>(c->nearest), sizeof(int32_t) * (size_t)c->nearest_cap);
    dev_free(c, reinterpret_cast<void *&>(c->k3idx), c->k3idx_bytes);
    dev_free(c, reinterpret_cast<void *&>(c->lay), c->lay_bytes);
    dev_free(c, reinterpret_cast<void *&>(c->counters), sizeof(unsigned long long) * C_COUNT);
    if (c->sc.join) (void)hipEventDestroy(c->sc.join);
    if (c->sc.fork) (void)hipEventDestroy(c->sc.fork);
    if (c->sc.side) (void)hipStreamDestroy(c->sc.side);
    delete c;
}

int esom_embed(esom_ctx *c, const float *X, int64_t n, int32_t d, int64_t ldx, const float *L_hd,
               const float *L_2d, int32_t g, const esom_params *params, float *out,
               int32_t *knn_idx, float *knn_dist2, void *stream) {
    t_err.clear();
    if (!c) return fail(ESOM_EINVAL, "ctx is NULL");
    if (!params) return fail(ESOM_EINVAL, "params is NULL");
    int st;
    const esom_params &P = *params;
    st = validate_embed(X, n, d, ldx, L_hd, L_2d, g, P, out, knn_idx, knn_dist2);
    if (st != ESOM_OK) return st;
    if (n == 0) return ESOM_OK;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return run_embed(c, X, n, d, ldx, L_hd, L_2d, g, P, out, knn_idx, knn_dist2, EMBED_FULL,
                     static_cast<hipStream_t>(stream), nullptr, 1);
}

int esom_embed_noalloc(const float *X, int64_t n, int32_t d, int64_t ldx, const float *L_hd,
                       const float *L_2d, int32_t g, const esom_params *params, float *out,
                       int32_t *knn_idx, float *knn_dist2, void *stream) {
    t_err.clear();
    if (!params) return fail(ESOM_EINVAL, "params is NULL");
    const esom_params &P = *params;
    int st = validate_embed(X, n, d, ldx, L_hd, L_2d, g, P, out, knn_idx, knn_dist2);
    if (st != ESOM_OK) return st;
    if (g > ESOM_NOALLOC_MAX_G)
        return fail(ESOM_EINVAL, "g = %d exceeds the allocation-free limit %d", g, ESOM_NOALLOC_MAX_G);
    if (d > ESOM_NOALLOC_MAX_D)
        return fail(ESOM_EINVAL, "d = %d exceeds the allocation-free limit %d", d, ESOM_NOALLOC_MAX_D);
    if (n == 0) return ESOM_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(ESOM_EINVAL, "device %d beyond the allocation-free limit %d", dev, NOALLOC_MAX_DEVICES);
    NoallocDevice &nd = g_noalloc[dev];
    std::call_once(nd.once, noalloc_setup, std::ref(nd));
    if (nd.err != hipSuccess) return hip_fail(nd.err, "allocation-free scratch set-up");
    // Layout: counters, then the embed scratch for `chunk` points.  Every
    // chunk point adds 4 + 1 + 4 bytes to the exact-path list and 1 + 4 to
    // the locality order; with chunk a multiple of 256 those five arrays need
    // no alignment padding beyond what carve reserves for one point each.
    const Plan pl = make_plan(d, g, P.k, P.mode, P.candidates);
    const int pg = embed_needs_pairs(d, g, P, EMBED_FULL) ? g : 0;
    const size_t room = ESOM_NOALLOC_SCRATCH_BYTES - NOALLOC_COUNTER_BYTES;
    Scratch sc;
    const size_t fixed = carve(sc, nullptr, 1, g, pl.dp, pg);
    if (fixed + 14 * 256 > room) return fail(ESOM_EINVAL, "landmark set too large for the allocation-free scratch");
    int64_t chunk = (int64_t)((room - fixed) / 14) & ~(int64_t)255;
    if (chunk > n) chunk = n;
    if (carve(sc, nullptr, chunk, g, pl.dp, pg) > room)
        return fail(ESOM_EINVAL, "internal: allocation-free scratch layout overflow");
    carve(sc, nd.ptr + NOALLOC_COUNTER_BYTES, chunk, g, pl.dp, pg);
    unsigned long long *counters = reinterpret_cast<unsigned long long *>(nd.ptr);
    return enqueue_embed(sc, counters, nd.num_cus, nd.lds_per_block, X, n, d, ldx, L_hd, L_2d, g, P,
                         out, knn_idx, knn_dist2, EMBED_FULL, static_cast<hipStream_t>(stream), nullptr,
                         nullptr, chunk, 1);
}

namespace {

int grow_nearest(esom_ctx *c, int64_t n, hipStream_t s) {
    if (n <= c->nearest_cap) return ESOM_OK;
    if (c->nearest) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        dev_free(c, reinterpret_cast<void *&>(c->nearest), sizeof(int32_t) * (size_t)c->nearest_cap);
    }
    int st = dev_alloc(c, reinterpret_cast<void **>(&c->nearest), sizeof(int32_t) * (size_t)n);
    c->nearest_cap = st == ESOM_OK ? n : 0;
    return st;
}

int grow_update_ws(esom_ctx *c, int64_t n, int g, int d, hipStream_t s) {
    const size_t need = update_workspace_bytes(n, g, d);
    if (need <= c->uws_bytes) return ESOM_OK;
    if (c->uws) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        dev_free(c, c->uws, c->uws_bytes);
        c->uws_bytes = 0;
    }
    int st = dev_alloc(c, &c->uws, need);
    if (st == ESOM_OK) c->uws_bytes = need;
    return st;
}

}  // namespace

int esom_som_train(esom_ctx *c, const float *X, int64_t n, int32_t d, int64_t ldx, float *L_hd,
                   const float *L_2d, int32_t g, const int32_t *batch_idx, int32_t batch,
                   int32_t steps, const float *sigma, const float *alpha, const uint8_t *frozen,
                   void *stream) {
    t_err.clear();
    if (!c) return fail(ESOM_EINVAL, "ctx is NULL");
    if (steps < 0) return fail(ESOM_EINVAL, "steps = %d < 0", steps);
    if (batch < 1) return fail(ESOM_EINVAL, "batch = %d < 1", batch);
    int st = validate_common(X, n, d, ldx, L_hd, g);
    if (st != ESOM_OK) return st;
    if (!L_2d || !aligned4(L_2d)) return fail(ESOM_EINVAL, "L_2d is NULL or not 4-byte aligned");
    if (!batch_idx || !aligned4(batch_idx)) return fail(ESOM_EINVAL, "batch_idx is NULL or not 4-byte aligned");
    if (steps > 0 && (!sigma || !alpha)) return fail(ESOM_EINVAL, "sigma and alpha are required");
    for (int t = 0; t < steps; ++t) {
        if (!(sigma[t] >= 0.f) || !isfinite(sigma[t]))
            return fail(ESOM_EINVAL, "sigma[%d] = %g must be finite and >= 0", t, (double)sigma[t]);
        if (!(alpha[t] >= 0.f && alpha[t] <= 1.f))
            return fail(ESOM_EINVAL, "alpha[%d] = %g outside [0, 1]", t, (double)alpha[t]);
    }
    if (steps == 0) return ESOM_OK;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t xb = sizeof(float) * (size_t)batch * d;
    if (xb > c->som_xb_bytes) {
        if (c->som_xb) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            dev_free(c, reinterpret_cast<void *&>(c->som_xb), c->som_xb_bytes);
            c->som_xb_bytes = 0;
        }
        st = dev_alloc(c, reinterpret_cast<void **>(&c->som_xb), xb);
        if (st != ESOM_OK) return st;
        c->som_xb_bytes = xb;
    }
    if ((st = grow_nearest(c, batch, s)) != ESOM_OK) return st;
    if ((st = grow_update_ws(c, batch, g, d, s)) != ESOM_OK) return st;
    esom_params P;
    esom_default_params(&P);
    P.k = 1;
    P.mode = ESOM_MODE_FP32;
    for (int t = 0; t < steps; ++t) {
        const int32_t *rows = batch_idx + (size_t)t * batch;
        e = launch_som_gather(X, n, ldx, d, rows, batch, c->som_xb, s);
        if (e != hipSuccess) return hip_fail(e, "batch gather launch");
        // best-matching landmarks of the batch against this step's landmarks
        st = run_embed(c, c->som_xb, batch, d, d, L_hd, L_2d, g, P, nullptr, c->nearest, nullptr,
                       EMBED_KNN_ONLY, s);
        if (st != ESOM_OK) return st;
        e = launch_som_mask(rows, batch, n, c->nearest, s);
        if (e != hipSuccess) return hip_fail(e, "batch mask launch");
        UpdateArgs u;
        u.X = c->som_xb;
        u.n = batch;
        u.ldx = d;
        u.d = d;
        u.g = g;
        u.kind = 2;
        u.alpha = alpha[t];
        u.sigma = sigma[t];
        u.L = L_hd;
        u.l2d = L_2d;
        u.nearest = c->nearest;
        u.nearest_ld = 1;
        u.counts = nullptr;
        u.frozen = frozen;
        u.batch = batch;
        e = launch_update(u, c->uws, c->num_cus, s);
        if (e != hipSuccess) return hip_fail(e, "online SOM update launch");
    }
    return ESOM_OK;
}

int esom_fit_landmarks(const float *L_hd, const float *L_2d, int32_t g, int32_t d, const float *p_2d,
                       int32_t m, int32_t kfit, float sigma, float *L_new, void *stream) {
    t_err.clear();
    if (g < 1 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [1, %d]", g, ESOM_MAX_G);
    if (d < 1 || d > ESOM_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ESOM_MAX_D);
    if (m < 0) return fail(ESOM_EINVAL, "m = %d < 0", m);
    if (kfit < 1 || kfit > 64) return fail(ESOM_EINVAL, "kfit = %d outside [1, 64]", kfit);
    if (!(sigma > 0.f) || !isfinite(sigma)) return fail(ESOM_EINVAL, "sigma = %g must be finite and > 0", (double)sigma);
    if (m == 0) return ESOM_OK;
    if (!L_hd || !L_2d || !p_2d || !L_new || !aligned4(L_hd) || !aligned4(L_2d) || !aligned4(p_2d) ||
        !aligned4(L_new))
        return fail(ESOM_EINVAL, "NULL or misaligned array");
    hipError_t e = launch_fit_landmarks(L_hd, L_2d, g, d, p_2d, m, kfit < g ? kfit : g, sigma, L_new,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "landmark fit launch");
    return ESOM_OK;
}

int esom_landmark_update(esom_ctx *c, const float *X, int64_t n, int32_t d, int64_t ldx,
                         float *L_hd, const float *L_2d, int32_t g, int32_t kind, float alpha,
                         float sigma, const int32_t *nearest, int64_t nearest_ld, int32_t *counts,
                         void *stream) {
    t_err.clear();
    if (!c) return fail(ESOM_EINVAL, "ctx is NULL");
    int st = validate_common(X, n, d, ldx, L_hd, g);
    if (st != ESOM_OK) return st;
    if (kind != 0 && kind != 1) return fail(ESOM_EINVAL, "kind = %d must be 0 or 1", kind);
    if (!(alpha >= 0.f && alpha <= 1.f)) return fail(ESOM_EINVAL, "alpha = %g outside [0, 1]", (double)alpha);
    if (!(sigma >= 0.f) || !isfinite(sigma)) return fail(ESOM_EINVAL, "sigma = %g must be >= 0", (double)sigma);
    if (kind == 1 && (!L_2d || ((uintptr_t)L_2d & 3u)))
        return fail(ESOM_EINVAL, "L_2d is required (4-byte aligned) for the SOM update");
    if ((nearest && !aligned4(nearest)) || (counts && !aligned4(counts)))
        return fail(ESOM_EINVAL, "nearest/counts must be 4-byte aligned");
    if (nearest && nearest_ld < 1) return fail(ESOM_EINVAL, "nearest_ld = %lld < 1", (long long)nearest_ld);
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t *near = nearest;
    int64_t near_ld = nearest ? nearest_ld : 1;
    if (!near && n > 0) {
        if (n > c->nearest_cap) {
            if (c->nearest) {
                e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
                dev_free(c, reinterpret_cast<void *&>(c->nearest), sizeof(int32_t) * (size_t)c->nearest_cap);
            }
            st = dev_alloc(c, reinterpret_cast<void **>(&c->nearest), sizeof(int32_t) * (size_t)n);
            if (st != ESOM_OK) {
                c->nearest_cap = 0;
                return st;
            }
            c->nearest_cap = n;
        }
        esom_params P;
        esom_default_params(&P);
        P.k = 1;
        P.mode = ESOM_MODE_FP32;
        st = run_embed(c, X, n, d, ldx, L_hd, L_2d, g, P, nullptr, c->nearest, nullptr, EMBED_KNN_ONLY, s);
        if (st != ESOM_OK) return st;
        near = c->nearest;
    }
    const size_t need = update_workspace_bytes(n, g, d);
    if (need > c->uws_bytes) {
        if (c->uws) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            dev_free(c, c->uws, c->uws_bytes);
            c->uws_bytes = 0;
        }
        st = dev_alloc(c, &c->uws, need);
        if (st != ESOM_OK) return st;
        c->uws_bytes = need;
    }
    UpdateArgs u;
    u.X = X;
    u.n = n;
    u.ldx = ldx;
    u.d = d;
    u.g = g;
    u.kind = kind;
    u.alpha = alpha;
    u.sigma = sigma;
    u.L = L_hd;
    u.l2d = L_2d;
    u.nearest = near;
    u.nearest_ld = near_ld;
    u.counts = counts;
    e = launch_update(u, c->uws, c->num_cus, s);
    if (e != hipSuccess) return hip_fail(e, "landmark update launch");
    return ESOM_OK;
}

int esom_embed3(esom_ctx *c, const float *X, int64_t n, int32_t d, int64_t ldx, const float *L_hd,
                const float *L_3d, int32_t g, const esom_params *params, float *out, int32_t *knn_idx,
                void *stream) {
    t_err.clear();
    if (!c) return fail(ESOM_EINVAL, "ctx is NULL");
    if (!params) return fail(ESOM_EINVAL, "params is NULL");
    const esom_params &P = *params;
    int st = validate_common(X, n, d, ldx, L_hd, g);
    if (st != ESOM_OK) return st;
    st = validate_params(P, g);
    if (st != ESOM_OK) return st;
    if (!L_3d || !aligned4(L_3d)) return fail(ESOM_EINVAL, "L_3d is NULL or not 4-byte aligned");
    if (n > 0 && (!out || !aligned4(out))) return fail(ESOM_EINVAL, "out is NULL or not 4-byte aligned");
    if (knn_idx && !aligned4(knn_idx)) return fail(ESOM_EINVAL, "knn_idx must be 4-byte aligned");
    if (n == 0) return ESOM_OK;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *kidx = knn_idx;
    if (!kidx) {
        const size_t need = sizeof(int32_t) * (size_t)n * P.k;
        if (need > c->k3idx_bytes) {
            if (c->k3idx) {
                e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
                dev_free(c, reinterpret_cast<void *&>(c->k3idx), c->k3idx_bytes);
                c->k3idx_bytes = 0;
            }
            st = dev_alloc(c, reinterpret_cast<void **>(&c->k3idx), need);
            if (st != ESOM_OK) return st;
            c->k3idx_bytes = need;
        }
        kidx = c->k3idx;
    }
    // the k nearest landmarks (screen, exact selection, exact path)
    st = run_embed(c, X, n, d, ldx, L_hd, nullptr, g, P, nullptr, kidx, nullptr, EMBED_KNN_ONLY, s,
                   nullptr, knn_idx ? 1 : 0);
    if (st != ESOM_OK) return st;
    Embed3Args a;
    a.X = X;
    a.n = n;
    a.ldx = ldx;
    a.d = d;
    a.g = g;
    a.k = P.k;
    a.use_cutoff = P.k < g ? 1 : 0;
    a.L = L_hd;
    a.l3 = L_3d;
    a.knn_idx = kidx;
    a.Wk = harmonic(P.k);
    a.boost = P.boost;
    a.cutoff = P.cutoff;
    a.gravity = P.gravity;
    a.adjust = P.adjust;
    a.out = out;
    e = launch_embed3(a, c->num_cus, s);
    if (e != hipSuccess) return hip_fail(e, "3-D projection launch");
    return ESOM_OK;
}

int esom_landmark_graph(const float *L_hd, int32_t g, int32_t d, int32_t kg, int32_t *nbr,
                        float *dist2, void *stream) {
    t_err.clear();
    if (g < 2 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [2, %d]", g, ESOM_MAX_G);
    if (d < 1 || d > ESOM_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ESOM_MAX_D);
    if (kg < 1 || kg > ESOM_GRAPH_MAX_K || kg > g - 1)
        return fail(ESOM_EINVAL, "kg = %d outside [1, min(g - 1, %d)]", kg, ESOM_GRAPH_MAX_K);
    if (!L_hd || !nbr || !aligned4(L_hd) || !aligned4(nbr) || (dist2 && !aligned4(dist2)))
        return fail(ESOM_EINVAL, "NULL or misaligned array");
    hipError_t e = launch_landmark_graph(L_hd, g, d, kg, nbr, dist2, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "landmark graph launch");
    return ESOM_OK;
}

void esom_default_layout_params(esom_layout_params *p) {
    if (!p) return;
    p->scale = 1.0f;
    p->repulsion = 0.05f;
    p->softening = 0.5f;
    p->step = 0.1f;
    p->max_move = 0.5f;
}

int esom_graph_layout(esom_ctx *c, const float *L_hd, int32_t g, int32_t d, const int32_t *nbr, int32_t kg,
                      float *L_2d, const uint8_t *fixed, int32_t steps, const esom_layout_params *lp,
                      void *stream) {
    t_err.clear();
    if (!c || !lp) return fail(ESOM_EINVAL, "ctx or params is NULL");
    if (g < 2 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [2, %d]", g, ESOM_MAX_G);
    if (d < 1 || d > ESOM_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ESOM_MAX_D);
    if (kg < 1 || kg > ESOM_GRAPH_MAX_K) return fail(ESOM_EINVAL, "kg = %d outside [1, %d]", kg, ESOM_GRAPH_MAX_K);
    if (steps < 0) return fail(ESOM_EINVAL, "steps = %d < 0", steps);
    if (!L_hd || !nbr || !L_2d || !aligned4(L_hd) || !aligned4(nbr) || ((uintptr_t)L_2d & 7u))
        return fail(ESOM_EINVAL, "NULL or misaligned array (L_2d needs 8-byte alignment)");
    const bool ok = isfinite(lp->scale) && lp->scale >= 0.f && isfinite(lp->repulsion) && lp->repulsion >= 0.f &&
                    isfinite(lp->softening) && lp->softening > 0.f && isfinite(lp->step) && lp->step >= 0.f &&
                    isfinite(lp->max_move) && lp->max_move >= 0.f;
    if (!ok) return fail(ESOM_EINVAL, "layout parameters must be finite and >= 0 (softening > 0)");
    if (steps == 0) return ESOM_OK;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t need = sizeof(float) * 2 * (size_t)g;
    if (need > c->lay_bytes) {
        if (c->lay) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            dev_free(c, reinterpret_cast<void *&>(c->lay), c->lay_bytes);
            c->lay_bytes = 0;
        }
        int st = dev_alloc(c, reinterpret_cast<void **>(&c->lay), need);
        if (st != ESOM_OK) return st;
        c->lay_bytes = need;
    }
    // synchronous steps alternate between L_2d and the context's buffer; an
    // odd count ends in the buffer and is copied back
    float *bufs[2] = {L_2d, c->lay};
    for (int t = 0; t < steps; ++t) {
        e = launch_layout_step(L_hd, g, d, nbr, kg, bufs[t & 1], bufs[(t + 1) & 1], fixed, lp->scale,
                               lp->repulsion, lp->softening, lp->step, lp->max_move, s);
        if (e != hipSuccess) return hip_fail(e, "layout step launch");
    }
    if (steps & 1) {
        e = hipMemcpyAsync(L_2d, c->lay, need, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return ESOM_OK;
}

int esom_landmark_duplicate(float *L_hd, float *L_2d, int32_t g, int32_t d, int32_t j, float dx, float dy,
                            void *stream) {
    t_err.clear();
    if (g < 1 || g >= ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [1, %d)", g, ESOM_MAX_G);
    if (d < 1 || d > ESOM_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ESOM_MAX_D);
    if (j < 0 || j >= g) return fail(ESOM_EINVAL, "j = %d outside [0, g)", j);
    if (!isfinite(dx) || !isfinite(dy)) return fail(ESOM_EINVAL, "offset must be finite");
    if (!L_hd || !L_2d || !aligned4(L_hd) || !aligned4(L_2d)) return fail(ESOM_EINVAL, "NULL or misaligned array");
    hipError_t e = launch_duplicate(L_hd, L_2d, g, d, j, dx, dy, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "duplicate launch");
    return ESOM_OK;
}

int esom_landmark_remove(float *L_hd, float *L_2d, int32_t g, int32_t d, int32_t j, void *stream) {
    t_err.clear();
    if (g < 2 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [2, %d]", g, ESOM_MAX_G);
    if (d < 1 || d > ESOM_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ESOM_MAX_D);
    if (j < 0 || j >= g) return fail(ESOM_EINVAL, "j = %d outside [0, g)", j);
    if (!L_hd || !L_2d || !aligned4(L_hd) || !aligned4(L_2d)) return fail(ESOM_EINVAL, "NULL or misaligned array");
    if (j == g - 1) return ESOM_OK;
    hipError_t e = launch_remove(L_hd, L_2d, g, d, j, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "remove launch");
    return ESOM_OK;
}

int esom_ablation_knn(int32_t algo, const float *X, int64_t n, int32_t d, const float *L_hd, int32_t g,
                      int32_t k, int32_t *knn_idx, float *knn_dist2, void *stream) {
    t_err.clear();
    if (algo < 0 || algo > 3) return fail(ESOM_EINVAL, "algo = %d outside [0, 3]", algo);
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(ESOM_EINVAL, "n = %lld out of range", (long long)n);
    if (d < 1 || d > ABL_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ABL_MAX_D);
    if (g < 1 || g > ESOM_MAX_G) return fail(ESOM_EINVAL, "g = %d outside [1, %d]", g, ESOM_MAX_G);
    if (k < 1 || k > ABL_MAX_K || k > g) return fail(ESOM_EINVAL, "k = %d outside [1, min(g, %d)]", k, ABL_MAX_K);
    if (n == 0) return ESOM_OK;
    if (!X || !L_hd || !knn_idx || !knn_dist2 || !aligned4(X) || !aligned4(L_hd) || !aligned4(knn_idx) ||
        !aligned4(knn_dist2))
        return fail(ESOM_EINVAL, "NULL or misaligned array");
    hipError_t e = launch_ablation_knn(algo, X, n, d, L_hd, g, k, knn_idx, knn_dist2,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "ablation k-NN launch");
    return ESOM_OK;
}

int esom_ablation_project(int32_t algo, const float *X, int64_t n, int32_t d, const float *L_hd,
                          const float *L_2d, int32_t g, const esom_params *params, const int32_t *knn_idx,
                          const float *knn_dist2, float *out, void *stream) {
    t_err.clear();
    if (!params) return fail(ESOM_EINVAL, "params is NULL");
    const esom_params &P = *params;
    if (algo < 0 || algo > 3) return fail(ESOM_EINVAL, "algo = %d outside [0, 3]", algo);
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(ESOM_EINVAL, "n = %lld out of range", (long long)n);
    if (d < 1 || d > ABL_MAX_D) return fail(ESOM_EINVAL, "d = %d outside [1, %d]", d, ABL_MAX_D);
    int st = validate_params(P, g);
    if (st != ESOM_OK) return st;
    if (P.k > ABL_MAX_K) return fail(ESOM_EINVAL, "k = %d above %d", P.k, ABL_MAX_K);
    if (n == 0) return ESOM_OK;
    if (!X || !L_hd || !L_2d || !knn_idx || !knn_dist2 || !out || !aligned4(X) || !aligned4(L_hd) ||
        ((uintptr_t)L_2d & 7u) || !aligned4(knn_idx) || !aligned4(knn_dist2) || ((uintptr_t)out & 7u))
        return fail(ESOM_EINVAL, "NULL or misaligned array");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    AbProjArgs a;
    a.X = X;
    a.L = L_hd;
    a.l2d = L_2d;
    a.idx = knn_idx;
    a.d2 = knn_dist2;
    a.n = n;
    a.d = d;
    a.g = g;
    a.k = P.k;
    a.boost = P.boost;
    a.cutoff = P.cutoff;
    a.gravity = P.gravity;
    a.adjust = P.adjust;
    a.Wk = (float)harmonic(P.k);
    a.out = out;
    e = launch_ablation_project(algo, a, cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "ablation projection launch");
    return ESOM_OK;
}

int esom_sync(esom_ctx *c, void *stream) {
    t_err.clear();
    if (!c) return fail(ESOM_EINVAL, "ctx is NULL");
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ESOM_OK;
}

int esom_get_stats(esom_ctx *c, void *stream, esom_stats *stats, int32_t reset) {
    t_err.clear();
    if (!c || !stats) return fail(ESOM_EINVAL, "ctx or stats is NULL");
    int st = esom_sync(c, stream);
    if (st != ESOM_OK) return st;
    unsigned long long h[C_COUNT];
    hipError_t e = hipMemcpy(h, c->counters, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    stats->n_points = (int64_t)h[C_POINTS];
    stats->n_fallback = (int64_t)h[C_FALLBACK];
    stats->n_uncertified = (int64_t)h[C_UNCERT];
    stats->n_near_tie = (int64_t)h[C_NEARTIE];
    stats->n_illcond = (int64_t)h[C_ILLCOND];
    stats->n_degenerate = (int64_t)h[C_DEGEN];
    stats->n_candidates = (int64_t)h[C_CAND];
    stats->n_slowpath = (int64_t)h[C_SLOW];
    for (size_t i = 0; i + 3 < c->pending.size(); i += 4) {
        float t01 = 0.f, t12 = 0.f, t23 = 0.f;
        (void)hipEventSynchronize(c->pending[i + 3]);
        (void)hipEventElapsedTime(&t01, c->pending[i], c->pending[i + 1]);
        (void)hipEventElapsedTime(&t12, c->pending[i + 1], c->pending[i + 2]);
        (void)hipEventElapsedTime(&t23, c->pending[i + 2], c->pending[i + 3]);
        c->ms_prep += t01;
        c->ms_main += t12;
        c->ms_exact += t23;
        c->n_timed += 1;
    }
    for (hipEvent_t ev : c->pending) (void)hipEventDestroy(ev);
    c->pending.clear();
    stats->n_timed = c->n_timed;
    stats->ms_prep = c->ms_prep;
    stats->ms_main = c->ms_main;
    stats->ms_exact = c->ms_exact;
    if (reset) {
        c->n_timed = 0;
        c->ms_prep = c->ms_main = c->ms_exact = 0.0;
        // all but the last call's fallback-list length (esom_get_fallback reads it)
        e = hipMemset(c->counters + C_POINTS, 0, sizeof h - C_POINTS * sizeof(unsigned long long));
        if (e != hipSuccess) return hip_fail(e, "hipMemset");
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    }
    return ESOM_OK;
}

}  // extern "C"
