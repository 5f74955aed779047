// Serving runtime: continuous batching of EmbedSOM requests on one GPU.
//
// Requests (uneven n, d, g, k) queue in arrival order.  A scheduler thread
// admits the head of the queue as soon as a slot is free and the request's
// device-memory footprint fits the budget beside the resident datasets and
// the memory other slots hold; admitted requests run concurrently, each on
// its own slot (own HIP stream, own scratch context, own landmark and output
// buffers), so the device overlaps them.  A host function enqueued after the
// output copy wakes the scheduler, which copies the result to the caller's
// buffer, frees the slot and admits more work.
//
// Resident datasets keep their points on the device.  For each dataset the
// last k nearest landmarks (indices and squared distances) are cached with a
// key of the high-dimensional landmarks and the selection parameters: a
// request that only moved 2-D landmarks (the interactive edit of the paper's
// supervision loop) skips the distance screen and runs the projection from
// the cache.  Frames on a resident dataset are captured into a hipGraph the
// second time the same frame (dataset, shapes, parameters, cache use, slot
// buffers) runs on a slot, and replayed from then on; each slot keeps the
// graphs of its last few distinct frames, and the scheduler routes a request
// on a resident dataset to a free slot that already holds a graph of that
// dataset, so the interactive edits of several datasets keep replaying.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "esom_internal.h"

using namespace esom;

namespace {

double now_ms(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Dataset {
    uint64_t id = 0;
    float *X = nullptr;
    int64_t n = 0;
    int d = 0;
    size_t bytes = 0;
    int refs = 0;
    bool dropped = false;
    // k-nearest cache
    int32_t *kidx = nullptr;
    float *kd2 = nullptr;
    uint8_t *kmark = nullptr;
    size_t cache_bytes = 0;
    bool cache_valid = false;
    bool cache_busy = false;
    uint64_t cache_key = 0;
};

struct Request {
    uint64_t id = 0;
    uint64_t dataset = 0;
    const float *Xh = nullptr;
    int64_t n = 0;
    int d = 0;
    int g = 0;
    std::vector<float> Lhd, l2d;
    esom_params P;
    float *out_host = nullptr;
    double t_submit = 0, t_start = 0, t_done = 0;
    int status = ESOM_OK;
    bool done = false;
    bool cache_hit = false;
    bool graph_replay = false;
    bool waited_memory = false;  // admission held back by the memory budget
    uint64_t hd_key = 0;
};

struct Slot {
    esom_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    // device buffers (grow on demand)
    float *dL = nullptr, *dl = nullptr, *dout = nullptr, *dX = nullptr;
    int32_t *dkidx = nullptr;
    float *dkd2 = nullptr;
    size_t capL = 0, capl = 0, capout = 0, capX = 0, capk = 0;
    // pinned staging
    float *hL = nullptr, *hl = nullptr, *hout = nullptr;
    size_t caphL = 0, caphl = 0, caphout = 0;
    Request *cur = nullptr;
    std::atomic<bool> finished{false};
    bool cache_writer = false;
    // captured frames: frame key -> graph (null until the frame is seen twice)
    struct Frame {
        hipGraphExec_t exec = nullptr;
        uint64_t dataset = 0;
        uint64_t last_use = 0;
    };
    std::map<uint64_t, Frame> frames;
    uint64_t use_clock = 0;
};

// Distinct frames a slot keeps graphs for (least recently used evicted).
constexpr size_t SLOT_FRAMES = 8;

}  // namespace

struct esom_server {
    int device = 0;
    size_t budget = 0;
    size_t resident = 0;  // datasets + caches
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;                 // all state below; may be held across HIP calls
    std::condition_variable cv_done;
    // Wake-ups for the scheduler.  note_mu is never held across a HIP call, so
    // the stream host functions that take it can never block device progress.
    std::mutex note_mu;
    std::condition_variable cv_note;
    bool note_pending = false;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> requests;
    std::map<uint64_t, std::unique_ptr<Dataset>> datasets;
    std::vector<std::unique_ptr<Slot>> slots;
    std::thread sched;
    bool stop = false;
    uint64_t next_id = 1;
    esom_serve_stats st{};
    std::string sched_error;
};

namespace {

size_t slot_held(esom_server *S) {
    size_t b = 0;
    for (auto &sl : S->slots) {
        b += ctx_held_bytes(sl->ctx);
        b += (sl->capL + sl->capl + sl->capout + sl->capX) * sizeof(float) +
             sl->capk * (sizeof(int32_t) + sizeof(float));
    }
    return b;
}

// Device bytes a request needs in a slot (beyond the resident datasets),
// including the growth headroom the slot buffers are allocated with.
size_t footprint(const Request &r) {
    size_t b = embed_scratch_bytes(r.n + r.n / 4, r.g, r.d, &r.P);
    size_t buf = sizeof(float) * ((size_t)r.g * r.d + 2 * (size_t)r.g + 2 * (size_t)r.n);
    if (!r.dataset) buf += sizeof(float) * (size_t)r.n * r.d;
    return b + buf + buf / 8 + 4096;
}

template <class T>
int grow_dev(T *&p, size_t &cap, size_t need) {
    if (need <= cap) return ESOM_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    const size_t n = need + need / 8;
    if (hipMalloc(reinterpret_cast<void **>(&p), n * sizeof(T)) != hipSuccess)
        return fail_msg(ESOM_ENOMEM, "serving: device allocation failed");
    cap = n;
    return ESOM_OK;
}

int grow_pinned(float *&p, size_t &cap, size_t need) {
    if (need <= cap) return ESOM_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t n = need + need / 8;
    if (hipHostMalloc(reinterpret_cast<void **>(&p), n * sizeof(float), hipHostMallocDefault) != hipSuccess)
        return fail_msg(ESOM_ENOMEM, "serving: pinned allocation failed");
    cap = n;
    return ESOM_OK;
}

void slot_drop_frames(Slot &sl) {
    for (auto &kv : sl.frames)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    sl.frames.clear();
}

bool slot_has_dataset_frame(const Slot &sl, uint64_t dataset) {
    for (auto &kv : sl.frames)
        if (kv.second.dataset == dataset) return true;
    return false;
}

void slot_free_buffers(Slot &sl) {
    slot_drop_frames(sl);
    auto f = [](auto *&p, size_t &cap) {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    };
    f(sl.dL, sl.capL);
    f(sl.dl, sl.capl);
    f(sl.dout, sl.capout);
    f(sl.dX, sl.capX);
    size_t ck = sl.capk;
    f(sl.dkidx, ck);
    ck = sl.capk;
    f(sl.dkd2, ck);
    sl.capk = 0;
    ctx_trim(sl.ctx);
}

void wake(esom_server *S) {
    {
        std::lock_guard<std::mutex> lk(S->note_mu);
        S->note_pending = true;
    }
    S->cv_note.notify_all();
}

void host_done(void *arg) {
    // Runs on a HIP runtime thread: no HIP calls and not the state mutex here.
    auto *pair = static_cast<std::pair<esom_server *, Slot *> *>(arg);
    pair->second->finished.store(true);
    wake(pair->first);
    delete pair;
}

// Enqueues the request's device work on the slot's stream (lock held).
int launch_request(esom_server *S, Slot &sl, Request &r) {
    hipStream_t s = sl.stream;
    Dataset *ds = nullptr;
    if (r.dataset) {
        auto it = S->datasets.find(r.dataset);
        ds = it->second.get();
    }
    int st = ESOM_OK;
    const size_t nL = (size_t)r.g * r.d, nl = 2 * (size_t)r.g, nout = 2 * (size_t)r.n;
    if ((st = grow_dev(sl.dL, sl.capL, nL)) || (st = grow_dev(sl.dl, sl.capl, nl)) ||
        (st = grow_dev(sl.dout, sl.capout, nout)) || (st = grow_pinned(sl.hL, sl.caphL, nL)) ||
        (st = grow_pinned(sl.hl, sl.caphl, nl)) || (st = grow_pinned(sl.hout, sl.caphout, nout)))
        return st;
    const float *X = nullptr;
    if (ds) {
        X = ds->X;
    } else {
        if ((st = grow_dev(sl.dX, sl.capX, (size_t)r.n * r.d))) return st;
        X = sl.dX;
    }
    memcpy(sl.hL, r.Lhd.data(), nL * sizeof(float));
    memcpy(sl.hl, r.l2d.data(), nl * sizeof(float));

    // k-nearest cache of the dataset (one writer at a time)
    int what = EMBED_FULL;
    int32_t *kidx = nullptr;
    float *kd2 = nullptr;
    uint8_t *kmark = nullptr;
    sl.cache_writer = false;
    if (ds && !ds->cache_busy && r.P.k <= 32) {
        if (ds->cache_valid && ds->cache_key == r.hd_key) {
            what = EMBED_PROJECT;
            r.cache_hit = true;
        } else {
            const size_t need = (size_t)ds->n * r.P.k;
            const size_t bytes = need * (sizeof(int32_t) + sizeof(float)) + (size_t)ds->n;
            if (bytes > ds->cache_bytes) {
                const size_t have = S->resident + slot_held(S) - ds->cache_bytes;
                if (have + bytes <= S->budget || S->budget == 0) {
                    if (ds->kidx) (void)hipFree(ds->kidx);
                    if (ds->kd2) (void)hipFree(ds->kd2);
                    if (ds->kmark) (void)hipFree(ds->kmark);
                    S->resident -= ds->cache_bytes;
                    ds->kidx = nullptr;
                    ds->kd2 = nullptr;
                    ds->kmark = nullptr;
                    ds->cache_bytes = 0;
                    if (hipMalloc(reinterpret_cast<void **>(&ds->kidx), need * sizeof(int32_t)) ==
                            hipSuccess &&
                        hipMalloc(reinterpret_cast<void **>(&ds->kd2), need * sizeof(float)) ==
                            hipSuccess &&
                        hipMalloc(reinterpret_cast<void **>(&ds->kmark), (size_t)ds->n) == hipSuccess) {
                        ds->cache_bytes = bytes;
                        S->resident += bytes;
                    }
                }
            }
            if (ds->cache_bytes >= bytes) {
                ds->cache_valid = false;
                sl.cache_writer = true;
            }
        }
        if (r.cache_hit || sl.cache_writer) {
            ds->cache_busy = true;
            kidx = ds->kidx;
            kd2 = ds->kd2;
            kmark = ds->kmark;
        }
    }

    // frame key: replay a captured graph for an identical repeated frame
    uint64_t key = 0;
    if (ds) {
        uint64_t v[12] = {r.dataset, (uint64_t)r.n, (uint64_t)r.d, (uint64_t)r.g,
                          (uint64_t)what, (uint64_t)(uintptr_t)kidx, (uint64_t)(uintptr_t)sl.dL,
                          (uint64_t)(uintptr_t)sl.dout, (uint64_t)(uintptr_t)sl.hL,
                          (uint64_t)(uintptr_t)sl.hout, (uint64_t)ctx_held_bytes(sl.ctx),
                          (uint64_t)(uintptr_t)ctx_arena(sl.ctx)};
        key = fnv1a(v, sizeof v, fnv1a(&r.P, sizeof r.P));
    }
    auto enqueue = [&]() -> int {
        if (hipMemcpyAsync(sl.dL, sl.hL, nL * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(sl.dl, sl.hl, nl * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail_msg(ESOM_EDEVICE, "serving: landmark upload failed");
        if (!ds && hipMemcpyAsync(sl.dX, r.Xh, (size_t)r.n * r.d * sizeof(float),
                                  hipMemcpyHostToDevice, s) != hipSuccess)
            return fail_msg(ESOM_EDEVICE, "serving: point upload failed");
        int e = run_embed(sl.ctx, X, r.n, r.d, r.d, sl.dL, sl.dl, r.g, r.P, sl.dout, kidx, kd2, what, s,
                          kmark);
        if (e != ESOM_OK) return e;
        if (hipMemcpyAsync(sl.hout, sl.dout, nout * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess)
            return fail_msg(ESOM_EDEVICE, "serving: result download failed");
        return ESOM_OK;
    };
    auto fit = ds ? sl.frames.find(key) : sl.frames.end();
    if (fit != sl.frames.end() && fit->second.exec) {
        if (hipGraphLaunch(fit->second.exec, s) != hipSuccess) return fail_msg(ESOM_EDEVICE, "graph launch failed");
        fit->second.last_use = ++sl.use_clock;
        r.graph_replay = true;
        S->st.graph_replays++;
    } else if (fit != sl.frames.end()) {
        // second identical frame on this slot: capture it (scratch and buffers
        // are already sized, so the capture records no allocation)
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail_msg(ESOM_EDEVICE, "stream capture failed");
        int e = enqueue();
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (e != ESOM_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return e;
        }
        if (ce != hipSuccess) return fail_msg(ESOM_EDEVICE, "stream capture failed");
        hipGraphExec_t exec = nullptr;
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) return fail_msg(ESOM_EDEVICE, "graph instantiation failed");
        fit->second.exec = exec;
        fit->second.last_use = ++sl.use_clock;
        if (hipGraphLaunch(exec, s) != hipSuccess) return fail_msg(ESOM_EDEVICE, "graph launch failed");
    } else {
        int e = enqueue();
        if (e != ESOM_OK) return e;
        if (ds) {
            if (sl.frames.size() >= SLOT_FRAMES) {
                auto lru = sl.frames.begin();
                for (auto it = sl.frames.begin(); it != sl.frames.end(); ++it)
                    if (it->second.last_use < lru->second.last_use) lru = it;
                if (lru->second.exec) (void)hipGraphExecDestroy(lru->second.exec);
                sl.frames.erase(lru);
            }
            Slot::Frame f;
            f.dataset = r.dataset;
            f.last_use = ++sl.use_clock;
            sl.frames[key] = f;
        }
    }
    auto *arg = new std::pair<esom_server *, Slot *>(S, &sl);
    if (hipLaunchHostFunc(s, host_done, arg) != hipSuccess) {
        delete arg;
        return fail_msg(ESOM_EDEVICE, "serving: host callback enqueue failed");
    }
    return ESOM_OK;
}

void finish_request(esom_server *S, Slot &sl) {
    Request &r = *sl.cur;
    if (r.status == ESOM_OK) memcpy(r.out_host, sl.hout, 2 * (size_t)r.n * sizeof(float));
    if (r.dataset) {
        auto it = S->datasets.find(r.dataset);
        if (it != S->datasets.end()) {
            Dataset &ds = *it->second;
            if (sl.cache_writer) {
                ds.cache_valid = r.status == ESOM_OK;
                ds.cache_key = r.hd_key;
            }
            if (sl.cache_writer || r.cache_hit) ds.cache_busy = false;
            if (--ds.refs == 0 && ds.dropped) {
                (void)hipFree(ds.X);
                if (ds.kidx) (void)hipFree(ds.kidx);
                if (ds.kd2) (void)hipFree(ds.kd2);
                if (ds.kmark) (void)hipFree(ds.kmark);
                S->resident -= ds.bytes + ds.cache_bytes;
                S->datasets.erase(it);
            }
        }
    }
    r.t_done = now_ms(S->t0);
    r.done = true;
    S->st.completed++;
    S->st.points += r.n;
    if (r.cache_hit) S->st.cache_hits++;
    sl.cur = nullptr;
    sl.cache_writer = false;
    sl.finished.store(false);
}

void scheduler(esom_server *S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::unique_lock<std::mutex> lk(S->mu);
        bool progressed = false;
        for (auto &sl : S->slots) {
            if (sl->cur && sl->finished.load()) {
                finish_request(S, *sl);
                progressed = true;
            }
        }
        if (progressed) S->cv_done.notify_all();
        // admit from the head of the queue
        while (!S->queue.empty()) {
            Request *r = S->queue.front();
            // a free slot, preferring one that holds a captured frame of the
            // request's resident dataset
            Slot *free_slot = nullptr;
            for (auto &sl : S->slots)
                if (!sl->cur) {
                    if (!free_slot) free_slot = sl.get();
                    if (r->dataset && slot_has_dataset_frame(*sl, r->dataset)) {
                        free_slot = sl.get();
                        break;
                    }
                }
            if (!free_slot) break;
            const size_t need = footprint(*r);
            size_t used = S->resident + slot_held(S);
            if (S->budget && used + need > S->budget) {
                // release the buffers of idle slots before deciding to wait
                for (auto &sl : S->slots)
                    if (!sl->cur) slot_free_buffers(*sl);
                used = S->resident + slot_held(S);
                if (used + need > S->budget) {
                    // wait for running requests to finish
                    if (!r->waited_memory) {
                        r->waited_memory = true;
                        S->st.admission_waits++;
                    }
                    break;
                }
            }
            S->queue.pop_front();
            r->t_start = now_ms(S->t0);
            free_slot->cur = r;
            free_slot->finished.store(false);
            const int st = launch_request(S, *free_slot, *r);
            if (st != ESOM_OK) {
                r->status = st;
                // drain whatever was enqueued before marking the slot free
                (void)hipStreamSynchronize(free_slot->stream);
                if (r->dataset) {
                    auto it = S->datasets.find(r->dataset);
                    if (it != S->datasets.end()) {
                        if (free_slot->cache_writer || r->cache_hit) it->second->cache_busy = false;
                        it->second->cache_valid = it->second->cache_valid && !free_slot->cache_writer;
                        it->second->refs--;
                    }
                }
                r->t_done = now_ms(S->t0);
                r->done = true;
                free_slot->cur = nullptr;
                free_slot->cache_writer = false;
                S->st.failed++;
                S->cv_done.notify_all();
            }
            const size_t held = S->resident + slot_held(S);
            if (held > (size_t)S->st.peak_bytes) S->st.peak_bytes = (int64_t)held;
        }
        bool inflight = false;
        for (auto &sl : S->slots) inflight |= sl->cur != nullptr;
        if (S->stop && S->queue.empty() && !inflight) break;
        lk.unlock();
        std::unique_lock<std::mutex> nl(S->note_mu);
        S->cv_note.wait_for(nl, std::chrono::milliseconds(50), [&] { return S->note_pending; });
        S->note_pending = false;
    }
}

}  // namespace

extern "C" {

int esom_serve_create(int device, size_t hbm_budget_bytes, int32_t n_slots, esom_server **out) {
    if (!out) return fail_msg(ESOM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_slots < 1 || n_slots > 16) return fail_msg(ESOM_EINVAL, "n_slots must be in [1, 16]");
    auto S = std::make_unique<esom_server>();
    S->device = device;
    S->budget = hbm_budget_bytes;
    S->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < n_slots; ++i) {
        auto sl = std::make_unique<Slot>();
        int st = esom_create(device, 0, &sl->ctx);
        if (st != ESOM_OK) {
            for (auto &s : S->slots) {
                slot_free_buffers(*s);
                (void)hipStreamDestroy(s->stream);
                esom_destroy(s->ctx);
            }
            return st;
        }
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
            esom_destroy(sl->ctx);
            return fail_msg(ESOM_EDEVICE, "hipStreamCreate failed");
        }
        S->slots.push_back(std::move(sl));
    }
    S->st.budget_bytes = (int64_t)hbm_budget_bytes;
    S->st.slots = n_slots;
    esom_server *raw = S.release();
    raw->sched = std::thread(scheduler, raw);
    *out = raw;
    return ESOM_OK;
}

void esom_serve_destroy(esom_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    wake(S);
    if (S->sched.joinable()) S->sched.join();
    (void)hipSetDevice(S->device);
    for (auto &sl : S->slots) {
        (void)hipStreamSynchronize(sl->stream);
        slot_free_buffers(*sl);
        if (sl->hL) (void)hipHostFree(sl->hL);
        if (sl->hl) (void)hipHostFree(sl->hl);
        if (sl->hout) (void)hipHostFree(sl->hout);
        (void)hipStreamDestroy(sl->stream);
        esom_destroy(sl->ctx);
    }
    for (auto &kv : S->datasets) {
        Dataset &ds = *kv.second;
        if (ds.X) (void)hipFree(ds.X);
        if (ds.kidx) (void)hipFree(ds.kidx);
        if (ds.kd2) (void)hipFree(ds.kd2);
        if (ds.kmark) (void)hipFree(ds.kmark);
    }
    delete S;
}

int esom_serve_dataset_put(esom_server *S, const float *X_host, int64_t n, int32_t d,
                           uint64_t *dataset_id) {
    if (!S || !X_host || !dataset_id) return fail_msg(ESOM_EINVAL, "NULL argument");
    if (n < 1 || d < 1 || d > ESOM_MAX_D) return fail_msg(ESOM_EINVAL, "bad dataset shape");
    if (n > (int64_t)INT32_MAX) return fail_msg(ESOM_EINVAL, "n exceeds 2^31 - 1");
    const size_t bytes = (size_t)n * d * sizeof(float);
    // The bytes are reserved under the lock; the allocation and the upload run
    // without it, so admissions and completions of the running slots are not
    // held up by a large upload.
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->budget && S->resident + slot_held(S) + bytes > S->budget)
        return fail_msg(ESOM_ENOMEM, "dataset does not fit the serving budget");
    S->resident += bytes;
    const uint64_t id = S->next_id++;
    lk.unlock();
    auto unreserve = [&](int code, const char *msg) {
        std::lock_guard<std::mutex> g(S->mu);
        S->resident -= bytes;
        return fail_msg(code, msg);
    };
    (void)hipSetDevice(S->device);
    auto ds = std::make_unique<Dataset>();
    if (hipMalloc(reinterpret_cast<void **>(&ds->X), bytes) != hipSuccess)
        return unreserve(ESOM_ENOMEM, "dataset allocation failed");
    if (hipMemcpy(ds->X, X_host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(ds->X);
        return unreserve(ESOM_EDEVICE, "dataset upload failed");
    }
    ds->n = n;
    ds->d = d;
    ds->bytes = bytes;
    ds->id = id;
    lk.lock();
    *dataset_id = id;
    S->datasets[id] = std::move(ds);
    return ESOM_OK;
}

int esom_serve_dataset_drop(esom_server *S, uint64_t dataset_id) {
    if (!S) return fail_msg(ESOM_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->datasets.find(dataset_id);
    if (it == S->datasets.end() || it->second->dropped)
        return fail_msg(ESOM_ENOTFOUND, "unknown dataset");
    Dataset &ds = *it->second;
    ds.dropped = true;
    if (ds.refs == 0) {
        (void)hipSetDevice(S->device);
        (void)hipFree(ds.X);
        if (ds.kidx) (void)hipFree(ds.kidx);
        if (ds.kd2) (void)hipFree(ds.kd2);
        if (ds.kmark) (void)hipFree(ds.kmark);
        S->resident -= ds.bytes + ds.cache_bytes;
        S->datasets.erase(it);
    }
    return ESOM_OK;
}

int esom_serve_submit(esom_server *S, uint64_t dataset_id, const float *X_host, int64_t n,
                      int32_t d, const float *L_hd_host, const float *L_2d_host, int32_t g,
                      const esom_params *params, float *out_host, uint64_t *request_id) {
    if (!S || !params || !L_hd_host || !L_2d_host || !out_host || !request_id)
        return fail_msg(ESOM_EINVAL, "NULL argument");
    const esom_params &P = *params;
    int vst = validate_params(P, g);
    if (vst != ESOM_OK) return vst;
    if (((uintptr_t)L_hd_host & 3u) || ((uintptr_t)L_2d_host & 3u) || ((uintptr_t)out_host & 3u))
        return fail_msg(ESOM_EINVAL, "host arrays must be 4-byte aligned");
    auto r = std::make_unique<Request>();
    std::unique_lock<std::mutex> lk(S->mu);
    if (dataset_id) {
        auto it = S->datasets.find(dataset_id);
        if (it == S->datasets.end() || it->second->dropped)
            return fail_msg(ESOM_ENOTFOUND, "unknown dataset");
        if (X_host) return fail_msg(ESOM_EINVAL, "X_host must be NULL for a resident dataset");
        n = it->second->n;
        d = it->second->d;
        it->second->refs++;
    } else {
        if (!X_host || n < 1 || d < 1 || d > ESOM_MAX_D || n > (int64_t)INT32_MAX)
            return fail_msg(ESOM_EINVAL,
                            "inline request needs X_host, 1 <= n <= 2^31 - 1, 1 <= d <= ESOM_MAX_D");
        if ((uintptr_t)X_host & 3u) return fail_msg(ESOM_EINVAL, "X_host must be 4-byte aligned");
    }
    r->dataset = dataset_id;
    r->Xh = X_host;
    r->n = n;
    r->d = d;
    r->g = g;
    r->P = P;
    r->out_host = out_host;
    r->Lhd.assign(L_hd_host, L_hd_host + (size_t)g * d);
    r->l2d.assign(L_2d_host, L_2d_host + 2 * (size_t)g);
    r->hd_key = fnv1a(r->Lhd.data(), r->Lhd.size() * sizeof(float));
    uint64_t sel[4] = {(uint64_t)g, (uint64_t)d, (uint64_t)P.k,
                       ((uint64_t)P.mode << 32) | (uint64_t)(uint32_t)P.candidates};
    r->hd_key = fnv1a(sel, sizeof sel, r->hd_key);
    const size_t need = footprint(*r);
    if (S->budget && need + (dataset_id ? 0 : 0) > S->budget - std::min(S->budget, S->resident)) {
        if (dataset_id) S->datasets[dataset_id]->refs--;
        S->st.rejected++;
        return fail_msg(ESOM_ENOMEM, "request footprint can never fit the serving budget");
    }
    r->id = S->next_id++;
    r->t_submit = now_ms(S->t0);
    *request_id = r->id;
    S->queue.push_back(r.get());
    if ((int64_t)S->queue.size() > S->st.max_queued) S->st.max_queued = (int64_t)S->queue.size();
    S->requests[r->id] = std::move(r);
    lk.unlock();
    wake(S);
    return ESOM_OK;
}

int esom_serve_wait(esom_server *S, uint64_t request_id, int32_t timeout_ms,
                    esom_request_info *info) {
    if (!S) return fail_msg(ESOM_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->requests.find(request_id);
    if (it == S->requests.end()) return fail_msg(ESOM_ENOTFOUND, "unknown request");
    Request *r = it->second.get();
    auto pred = [&] { return r->done; };
    if (timeout_ms < 0)
        S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
        return fail_msg(ESOM_ETIMEOUT, "request still pending");
    if (info) {
        info->submit_ms = r->t_submit;
        info->start_ms = r->t_start;
        info->done_ms = r->t_done;
        info->cache_hit = r->cache_hit ? 1 : 0;
        info->graph_replay = r->graph_replay ? 1 : 0;
        info->status = r->status;
        info->n = r->n;
    }
    const int st = r->status;
    S->requests.erase(it);
    if (st != ESOM_OK) return fail_msg(st, "request failed on the device path");
    return ESOM_OK;
}

int esom_serve_get_stats(esom_server *S, esom_serve_stats *out) {
    if (!S || !out) return fail_msg(ESOM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->queued = (int64_t)S->queue.size();
    int64_t inflight = 0;
    for (auto &sl : S->slots) inflight += sl->cur != nullptr;
    out->in_flight = inflight;
    out->resident_bytes = (int64_t)S->resident;
    out->held_bytes = (int64_t)(S->resident + slot_held(S));
    out->now_ms = now_ms(S->t0);
    return ESOM_OK;
}

}  // extern "C"
