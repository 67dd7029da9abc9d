// Served form of the pipeline: several UAV streams, frames submitted as they
// arrive, each matched against its stream's previous keyframes (the
// sliding bundle of the online-mapping use; keyframe when the camera moved
// at least min_baseline since the last keyframe), admitted into one of
// n_slots pipeline slots when a slot is free and the device memory the
// slots hold, plus what the chosen slot must grow by for the frame, fits the
// budget, and run concurrently (each slot is a handle with its own HIP
// stream, so frames overlap on the device).
//
// Host code over the library's public C ABI.  A worker thread admits
// queued frames and collects finished ones; submit and result calls only
// touch the queues.  Keyframe images stay on the device (pooled image
// buffers, held by reference counts of the frames that use them and of the
// keyframe list), each with its whole pyramid, built once when the image
// arrives, so the frames that match against it copy its levels instead of
// rebuilding them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fassmvs.h"
#include "handle_internal.hpp"

using fmvs::handle_growth;
using fmvs::handle_held;
using fmvs::handle_reserve;
using fmvs::handle_set_exact_growth;
using fmvs::handle_submit_pyramids;
using fmvs::handle_trim;
using fmvs::pyramid_build;
using fmvs::pyramid_bytes;

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t1) {
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Stream;

// A device copy of one frame's image (uploaded asynchronously through a
// pinned staging buffer on the server's upload stream; `ready` marks the
// end of the upload), returned to its stream's pool when the last user lets
// go.
struct ImageBuf {
    uint8_t *p = nullptr;       // device
    uint8_t *stage = nullptr;   // pinned host staging
    hipEvent_t ready = nullptr;
};
struct MapBuf {
    float *depth = nullptr, *normal = nullptr, *conf = nullptr;
};
// Free buffers of the server, by frame size (pixels): streams of the same
// size share them, and nothing is freed before the server goes (hipFree
// would synchronise the device and stall the frames in flight).
struct Pools {
    std::mutex mu;
    std::map<size_t, std::vector<ImageBuf>> img;
    std::map<size_t, std::vector<MapBuf>> maps;
};
struct DevImage {
    ImageBuf b;
    size_t n = 0;
    Pools *pools = nullptr;
    ~DevImage();
};

struct Stream {
    int id = 0;
    double K[9];
    int w = 0, h = 0;
    std::vector<fassmvs_plane_family> fams;
    // copies of the families' explicit plane lists (fams[f].delta points
    // into them); shared so that a frame being submitted keeps them alive
    std::shared_ptr<const std::vector<std::vector<double>>> lists;
    int max_kf = 4;
    double min_baseline = 1.0;
    // keyframes, most recent first: image and pose
    struct Key {
        std::shared_ptr<DevImage> img;
        double R[9], t[3], C[3];
    };
    std::deque<Key> keys;
    Pools *pools = nullptr;
    bool closed = false;
};

DevImage::~DevImage() {
    if (b.p && pools) {
        std::lock_guard<std::mutex> lk(pools->mu);
        pools->img[n].push_back(b);
    }
}

struct Request {
    uint64_t id = 0;
    int stream = 0;
    Clock::time_point arrival;
    std::shared_ptr<DevImage> img;
    double R[9], t[3];
    std::vector<Stream::Key> views;   // snapshot of the stream's keyframes
    bool keyframe = false;
    uint64_t footprint = 0;
};

struct Result {
    fassmvs_server_result info;
    Pools *pools = nullptr;
    float *depth = nullptr, *normal = nullptr, *conf = nullptr;   // device, from the map pool
};

// Result maps of a frame size from the pool, allocated on first use.
bool take_maps(Stream &st, Result &r) {
    const size_t N = (size_t)st.w * st.h;
    {
        std::lock_guard<std::mutex> lk(st.pools->mu);
        auto &v = st.pools->maps[N];
        if (!v.empty()) {
            MapBuf m = v.back();
            v.pop_back();
            r.depth = m.depth;
            r.normal = m.normal;
            r.conf = m.conf;
            r.pools = st.pools;
            return true;
        }
    }
    float *d = nullptr, *n = nullptr, *c = nullptr;
    if (hipMalloc(&d, N * 4) != hipSuccess || hipMalloc(&n, N * 12) != hipSuccess || hipMalloc(&c, N * 4) != hipSuccess) {
        (void)hipGetLastError();
        if (d) hipFree(d);
        if (n) hipFree(n);
        if (c) hipFree(c);
        return false;
    }
    r.depth = d;
    r.normal = n;
    r.conf = c;
    r.pools = st.pools;
    return true;
}

void give_maps(Result &r) {
    if (!r.pools || !r.depth) return;
    std::lock_guard<std::mutex> lk(r.pools->mu);
    r.pools->maps[(size_t)r.info.width * r.info.height].push_back(MapBuf{r.depth, r.normal, r.conf});
    r.depth = r.normal = r.conf = nullptr;
}

struct Slot {
    fassmvs_handle *h = nullptr;
    hipStream_t stream = nullptr;
    bool busy = false;
    uint64_t ticket = 0;
    Request req;
    Result res;
};

}  // namespace

struct fassmvs_server {
    fassmvs_config cfg;
    uint64_t budget = 0;
    std::vector<Slot> slots;
    std::map<int, std::unique_ptr<Stream>> streams;
    Pools pools;
    std::mutex mu;        // queues, streams, results
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::deque<Result> done;
    std::map<uint64_t, Result> fetched_pending;   // results reported but not yet fetched
    uint64_t next_id = 1;
    int next_stream = 1;
    bool stop = false;
    std::string err;
    std::thread worker;
    size_t in_flight = 0;
    bool reserve_pending = false;   // a stream opened: size the slots for it when the device is idle
    hipStream_t upload = nullptr, fetch = nullptr;   // non-blocking streams for image uploads and result copies
    std::mutex fetch_mu;
};

namespace {

fassmvs_status sfail(fassmvs_server *s, fassmvs_status st, const std::string &m) {
    if (s) s->err = m;
    return st;
}

void camera_centre(const double *R, const double *t, double *C) {
    for (int i = 0; i < 3; ++i) C[i] = -(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
}

// The frame's bundle as the pipeline takes it: the reference image and its
// stream's keyframes (all earlier in the sequence: left side).
int bundle_of(const Request &req, const Stream &st, fassmvs_image &ref, fassmvs_image *views, int8_t *side) {
    std::memset(&ref, 0, sizeof(ref));
    ref.pixels = req.img->b.p;
    ref.width = st.w;
    ref.height = st.h;
    ref.stride = st.w;
    std::memcpy(ref.R, req.R, sizeof(ref.R));
    std::memcpy(ref.t, req.t, sizeof(ref.t));
    const int nv = (int)req.views.size();
    for (int k = 0; k < nv; ++k) {
        std::memset(&views[k], 0, sizeof(views[k]));
        views[k].pixels = req.views[k].img->b.p;
        views[k].width = st.w;
        views[k].height = st.h;
        views[k].stride = st.w;
        std::memcpy(views[k].R, req.views[k].R, sizeof(views[k].R));
        std::memcpy(views[k].t, req.views[k].t, sizeof(views[k].t));
        side[k] = -1;
    }
    return nv;
}

// Admit the head of the queue into a free slot if the device memory allows.
// The account is the memory the slots' pipelines actually hold (their
// buffers only grow, exactly to what a frame needs) plus the growth the
// frame needs on the chosen slot (the free slot that needs the least).  A
// slot grows only while no frame is in flight, so its reallocation never
// waits on other frames; when the budget is short and the device is idle,
// the other idle slots' buffers are released first, then the chosen one's.
// Called by the worker (which alone touches the slots) with lk held; the
// lock is released while the frame is enqueued.  Returns true if a request
// left the queue.
bool admit_one(fassmvs_server *s, std::unique_lock<std::mutex> &lk) {
    if (s->queue.empty()) return false;
    Request &head = s->queue.front();
    Stream &hs = *s->streams.at(head.stream);
    Slot *free_slot = nullptr;
    uint64_t grow = 0;
    if (!head.views.empty()) {
        fassmvs_image ref, views[FASSMVS_MAX_VIEWS];
        int8_t side[FASSMVS_MAX_VIEWS];
        const int nv = bundle_of(head, hs, ref, views, side);
        for (auto &sl : s->slots) {
            if (sl.busy) continue;
            uint64_t g = 0;
            if (handle_growth(sl.h, &ref, views, side, nv, hs.K, hs.fams.data(), (int32_t)hs.fams.size(), &g) !=
                FASSMVS_OK)
                g = 0;   // the submit reports the frame's error
            if (!free_slot || g < grow) {
                free_slot = &sl;
                grow = g;
            }
        }
        if (!free_slot) return false;
        if (grow > 0 && s->in_flight > 0) return false;
        uint64_t held = 0;
        for (auto &sl : s->slots) held += handle_held(sl.h);
        if (held + grow > s->budget) {
            if (s->in_flight > 0) return false;
            for (auto &sl : s->slots)
                if (&sl != free_slot) handle_trim(sl.h);
            held = 0;
            for (auto &sl : s->slots) held += handle_held(sl.h);
            if (held + grow > s->budget) {
                handle_trim(free_slot->h);
                if (handle_growth(free_slot->h, &ref, views, side, nv, hs.K, hs.fams.data(),
                                  (int32_t)hs.fams.size(), &grow) != FASSMVS_OK)
                    grow = 0;
            }
        }
    }
    Request req = std::move(head);
    s->queue.pop_front();
    Stream &st = *s->streams.at(req.stream);
    Result res;
    std::memset(&res.info, 0, sizeof(res.info));
    res.info.request_id = req.id;
    res.info.stream_id = req.stream;
    res.info.width = st.w;
    res.info.height = st.h;
    res.info.keyframe = req.keyframe ? 1 : 0;
    res.info.n_views = (int32_t)req.views.size();
    if (req.views.empty()) {
        // nothing to match against yet (first keyframe of a stream)
        res.info.status = FASSMVS_ENOTFOUND;
        res.info.latency_ms = ms_since(req.arrival, Clock::now());
        s->done.push_back(res);
        s->cv_done.notify_all();
        return true;
    }
    if (!take_maps(st, res)) {
        res.info.status = FASSMVS_ENOMEM;
        s->done.push_back(res);
        s->cv_done.notify_all();
        return true;
    }
    // reserve before enqueueing (the lock is dropped meanwhile)
    free_slot->busy = true;
    s->in_flight++;
    const double K[9] = {st.K[0], st.K[1], st.K[2], st.K[3], st.K[4], st.K[5], st.K[6], st.K[7], st.K[8]};
    const std::vector<fassmvs_plane_family> fams = st.fams;
    const auto lists = st.lists;
    fassmvs_image ref, views[FASSMVS_MAX_VIEWS];
    int8_t side[FASSMVS_MAX_VIEWS];
    const int nv = bundle_of(req, st, ref, views, side);
    lk.unlock();
    // the slot's stream waits (on the device) for the images' uploads
    hipStreamWaitEvent(free_slot->stream, req.img->b.ready, 0);
    for (auto &v : req.views) hipStreamWaitEvent(free_slot->stream, v.img->b.ready, 0);
    uint64_t ticket = 0;
    fassmvs_status rc =
        handle_submit_pyramids(free_slot->h, &ref, views, side, nv, K, fams.data(), (int32_t)fams.size(), &ticket);
    lk.lock();
    if (rc != FASSMVS_OK) {
        give_maps(res);
        res.info.status = rc;
        res.info.latency_ms = ms_since(req.arrival, Clock::now());
        free_slot->busy = false;
        s->in_flight--;
        s->done.push_back(res);
        s->cv_done.notify_all();
        return true;
    }
    free_slot->ticket = ticket;
    free_slot->req = std::move(req);
    free_slot->res = res;
    return true;
}

// Collect finished frames (non-blocking).  lk held on entry and exit; the
// maps' copy out of a finished slot runs without it.
bool collect(fassmvs_server *s, std::unique_lock<std::mutex> &lk) {
    bool any = false;
    for (auto &sl : s->slots) {
        if (!sl.busy || sl.ticket == 0) continue;
        lk.unlock();
        fassmvs_status rc = fassmvs_poll(sl.h, sl.ticket, sl.res.depth, sl.res.normal, sl.res.conf,
                                         FASSMVS_MEM_DEVICE, 0);
        const Clock::time_point now = Clock::now();
        Request finished;
        if (rc != FASSMVS_PENDING) finished = std::move(sl.req);   // drop the image references outside the lock
        lk.lock();
        if (rc == FASSMVS_PENDING) continue;
        Result res = sl.res;
        res.info.status = rc;
        res.info.latency_ms = ms_since(finished.arrival, now);
        if (rc != FASSMVS_OK) give_maps(res);
        s->in_flight--;
        sl.busy = false;
        sl.ticket = 0;
        sl.req = Request();
        s->done.push_back(res);
        any = true;
        lk.unlock();
        finished = Request();
        lk.lock();
    }
    if (any) s->cv_done.notify_all();
    return any;
}

// Grow every slot to hold any frame of every open stream (a bundle of the
// stream's size with its full keyframe count), within the budget, while no
// frame is in flight: afterwards a frame never waits for the device to go
// idle before its slot can grow (growth waits for that, since freeing device
// memory synchronises the device).  lk held.
void reserve_slots(fassmvs_server *s) {
    if (!s->reserve_pending || s->in_flight > 0) return;
    s->reserve_pending = false;
    for (auto &kv : s->streams) {
        const Stream &st = *kv.second;
        if (st.closed) continue;
        for (auto &sl : s->slots) {
            uint64_t g = 0, held = 0;
            if (handle_reserve(sl.h, st.w, st.h, st.max_kf, st.K, st.fams.data(), (int32_t)st.fams.size(), false,
                               &g) != FASSMVS_OK || g == 0)
                continue;
            for (auto &o : s->slots) held += handle_held(o.h);
            if (held + g > s->budget) continue;
            (void)handle_reserve(sl.h, st.w, st.h, st.max_kf, st.K, st.fams.data(), (int32_t)st.fams.size(), true,
                                 &g);
        }
    }
}

void worker_loop(fassmvs_server *s) {
    hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop && s->queue.empty() && s->in_flight == 0) break;
        bool progress = collect(s, lk);
        reserve_slots(s);
        while (admit_one(s, lk)) progress = true;
        if (!progress) {
            if (s->in_flight > 0)
                s->cv_work.wait_for(lk, std::chrono::microseconds(50));
            else
                s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

extern "C" {

fassmvs_status fassmvs_server_create(const fassmvs_config *cfg, int32_t n_slots, uint64_t hbm_budget_bytes,
                                     fassmvs_server **out) {
    if (!out) return FASSMVS_EINVAL;
    *out = nullptr;
    if (!cfg || n_slots < 1 || n_slots > 16) return FASSMVS_EINVAL;
    std::unique_ptr<fassmvs_server> s(new fassmvs_server());
    s->cfg = *cfg;
    if (hipSetDevice(cfg->device) != hipSuccess) return FASSMVS_EDEVICE;
    if (hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return FASSMVS_EDEVICE;
        hbm_budget_bytes = (uint64_t)(fr * 0.8);
    }
    s->budget = hbm_budget_bytes;
    if (hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->fetch, hipStreamNonBlocking) != hipSuccess)
        return FASSMVS_EDEVICE;
    s->slots.resize(n_slots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) return FASSMVS_EDEVICE;
        fassmvs_config c = *cfg;
        c.stream = sl.stream;
        c.keep_levels = 0;
        c.hbm_budget_bytes = hbm_budget_bytes;
        fassmvs_status st = fassmvs_create(&c, &sl.h);
        if (st == FASSMVS_OK) handle_set_exact_growth(sl.h);
        if (st != FASSMVS_OK) {
            for (auto &o : s->slots) {
                if (o.h) fassmvs_destroy(o.h);
                if (o.stream) hipStreamDestroy(o.stream);
            }
            return st;
        }
    }
    s->worker = std::thread(worker_loop, s.get());
    *out = s.release();
    return FASSMVS_OK;
}

fassmvs_status fassmvs_server_open_stream(fassmvs_server *s, const double K[9], int32_t width, int32_t height,
                                          const fassmvs_plane_family *families, int32_t n_families,
                                          int32_t max_keyframes, double min_baseline, int32_t *stream_id) {
    if (!s || !K || !families || !stream_id || width < 8 || height < 8 || n_families < 1 ||
        n_families > FASSMVS_MAX_FAMILIES || max_keyframes < 1 || max_keyframes > FASSMVS_MAX_VIEWS ||
        !(min_baseline >= 0.0))
        return sfail(s, FASSMVS_EINVAL, "bad stream arguments");
    std::unique_ptr<Stream> st(new Stream());
    std::memcpy(st->K, K, sizeof(st->K));
    st->w = width;
    st->h = height;
    st->fams.assign(families, families + n_families);
    auto lists = std::make_shared<std::vector<std::vector<double>>>(n_families);
    for (int f = 0; f < n_families; ++f) {
        if (!families[f].delta) continue;
        if (families[f].count < 2 || families[f].count > FASSMVS_MAX_TOP_PLANES)
            return sfail(s, FASSMVS_EINVAL, "an explicit plane list needs 2..256 distances");
        (*lists)[f].assign(families[f].delta, families[f].delta + families[f].count);
        st->fams[f].delta = (*lists)[f].data();
    }
    st->lists = lists;
    st->max_kf = max_keyframes;
    st->min_baseline = min_baseline;
    st->pools = &s->pools;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        st->id = s->next_stream++;
        *stream_id = st->id;
        s->streams[st->id] = std::move(st);
        s->reserve_pending = true;
    }
    s->cv_work.notify_all();
    return FASSMVS_OK;
}

fassmvs_status fassmvs_server_submit(fassmvs_server *s, int32_t stream_id, const uint8_t *pixels, int32_t stride,
                                     const double R[9], const double t[3], uint64_t *request_id) {
    const Clock::time_point arrival = Clock::now();
    if (!s || !pixels || !R || !t || !request_id) return sfail(s, FASSMVS_EINVAL, "null argument");
    Stream *st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->streams.find(stream_id);
        if (it == s->streams.end() || it->second->closed) return sfail(s, FASSMVS_ENOTFOUND, "unknown stream");
        st = it->second.get();
    }
    if (stride < st->w) return sfail(s, FASSMVS_EINVAL, "stride smaller than the width");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(R[i])) return sfail(s, FASSMVS_EINVAL, "non-finite pose");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(t[i])) return sfail(s, FASSMVS_EINVAL, "non-finite pose");
    // the image goes to the device now (asynchronously): every later frame
    // of the stream that takes it as a keyframe finds it there
    ImageBuf b;
    const size_t N = (size_t)st->w * st->h;
    const size_t NP = pyramid_bytes(st->w, st->h, s->cfg.n_levels);   // the image and its coarser levels
    {
        std::lock_guard<std::mutex> lk(s->pools.mu);
        auto &v = s->pools.img[N];
        if (!v.empty()) {
            b = v.back();
            v.pop_back();
        }
    }
    if (!b.p) {
        if (hipMalloc(&b.p, NP) != hipSuccess || hipHostMalloc(&b.stage, N) != hipSuccess ||
            hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (b.p) hipFree(b.p);
            if (b.stage) hipHostFree(b.stage);
            return sfail(s, FASSMVS_ENOMEM, "image buffer allocation failed");
        }
    } else if (hipEventSynchronize(b.ready) != hipSuccess) {   // staging free again
        return sfail(s, FASSMVS_EDEVICE, "image buffer reuse");
    }
    for (int y = 0; y < st->h; ++y) std::memcpy(b.stage + (size_t)y * st->w, pixels + (size_t)y * stride, st->w);
    auto img = std::make_shared<DevImage>();
    img->b = b;
    img->n = N;
    img->pools = &s->pools;
    if (hipMemcpyAsync(b.p, b.stage, N, hipMemcpyHostToDevice, s->upload) != hipSuccess ||
        pyramid_build(b.p, st->w, st->h, s->cfg.n_levels, s->upload) != hipSuccess ||
        hipEventRecord(b.ready, s->upload) != hipSuccess)
        return sfail(s, FASSMVS_EDEVICE, "image upload failed");
    Request req;
    req.arrival = arrival;
    req.stream = stream_id;
    req.img = img;
    std::memcpy(req.R, R, sizeof(req.R));
    std::memcpy(req.t, t, sizeof(req.t));
    uint64_t fp = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        req.views.assign(st->keys.begin(), st->keys.end());
        if (!req.views.empty() &&
            fassmvs_frame_footprint(&s->cfg, st->w, st->h, (int32_t)req.views.size(), st->fams.data(),
                                    (int32_t)st->fams.size(), &fp) != FASSMVS_OK)
            return sfail(s, FASSMVS_EINVAL, "footprint");
        if (fp > s->budget) return sfail(s, FASSMVS_ENOMEM, "frame footprint exceeds the server's budget");
        req.id = s->next_id++;
        double C[3];
        camera_centre(R, t, C);
        bool key = st->keys.empty();
        if (!key) {
            const double *Cl = st->keys.front().C;
            const double d = std::sqrt((C[0] - Cl[0]) * (C[0] - Cl[0]) + (C[1] - Cl[1]) * (C[1] - Cl[1]) +
                                       (C[2] - Cl[2]) * (C[2] - Cl[2]));
            key = d >= st->min_baseline;
        }
        req.keyframe = key;
        if (key) {
            Stream::Key k;
            k.img = img;
            std::memcpy(k.R, R, sizeof(k.R));
            std::memcpy(k.t, t, sizeof(k.t));
            std::memcpy(k.C, C, sizeof(k.C));
            st->keys.push_front(k);
            while ((int)st->keys.size() > st->max_kf) st->keys.pop_back();
        }
        req.footprint = fp;
        *request_id = req.id;
        s->queue.push_back(std::move(req));
    }
    s->cv_work.notify_all();
    return FASSMVS_OK;
}

fassmvs_status fassmvs_server_next(fassmvs_server *s, int32_t wait_ms, fassmvs_server_result *out) {
    if (!s || !out) return FASSMVS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return !s->done.empty(); };
    if (!ready()) {
        if (wait_ms == 0) return FASSMVS_PENDING;
        if (wait_ms < 0)
            s->cv_done.wait(lk, ready);
        else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready))
            return FASSMVS_PENDING;
    }
    Result r = s->done.front();
    s->done.pop_front();
    *out = r.info;
    if (r.depth) s->fetched_pending[r.info.request_id] = r;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_server_fetch(fassmvs_server *s, uint64_t request_id, float *depth, float *normal,
                                    float *confidence, int32_t mem_kind) {
    if (!s) return FASSMVS_EINVAL;
    if (mem_kind != FASSMVS_MEM_HOST && mem_kind != FASSMVS_MEM_DEVICE) return sfail(s, FASSMVS_EINVAL, "bad mem_kind");
    Result r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->fetched_pending.find(request_id);
        if (it == s->fetched_pending.end()) return sfail(s, FASSMVS_ENOTFOUND, "no maps for this request");
        r = it->second;
        s->fetched_pending.erase(it);
    }
    const size_t N = (size_t)r.info.width * r.info.height;
    const hipMemcpyKind kind = mem_kind == FASSMVS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    // copies on the server's own non-blocking stream: they wait for nothing
    // but themselves, frames in flight keep running
    std::lock_guard<std::mutex> flk(s->fetch_mu);
    hipError_t e = hipSuccess;
    if (depth && e == hipSuccess) e = hipMemcpyAsync(depth, r.depth, N * 4, kind, s->fetch);
    if (normal && e == hipSuccess) e = hipMemcpyAsync(normal, r.normal, N * 12, kind, s->fetch);
    if (confidence && e == hipSuccess) e = hipMemcpyAsync(confidence, r.conf, N * 4, kind, s->fetch);
    if (e == hipSuccess) e = hipStreamSynchronize(s->fetch);
    give_maps(r);
    return e == hipSuccess ? FASSMVS_OK : sfail(s, FASSMVS_EDEVICE, "result copy failed");
}

fassmvs_status fassmvs_server_close_stream(fassmvs_server *s, int32_t stream_id) {
    if (!s) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end()) return sfail(s, FASSMVS_ENOTFOUND, "unknown stream");
    it->second->closed = true;
    it->second->keys.clear();
    return FASSMVS_OK;
}

const char *fassmvs_server_last_error(const fassmvs_server *s) { return s ? s->err.c_str() : ""; }

void fassmvs_server_destroy(fassmvs_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    hipSetDevice(s->cfg.device);
    for (auto &r : s->done) give_maps(r);
    for (auto &kv : s->fetched_pending) give_maps(kv.second);
    for (auto &sl : s->slots) {
        sl.req = Request();
        if (sl.h) fassmvs_destroy(sl.h);
        if (sl.stream) hipStreamDestroy(sl.stream);
    }
    for (auto &kv : s->streams) kv.second->keys.clear();
    for (auto &kv : s->pools.img)
        for (ImageBuf &b : kv.second) {
            hipEventSynchronize(b.ready);
            hipEventDestroy(b.ready);
            hipHostFree(b.stage);
            hipFree(b.p);
        }
    for (auto &kv : s->pools.maps)
        for (MapBuf &m : kv.second) {
            hipFree(m.depth);
            hipFree(m.normal);
            hipFree(m.conf);
        }
    if (s->upload) hipStreamDestroy(s->upload);
    if (s->fetch) hipStreamDestroy(s->fetch);
    delete s;
}

}  // extern "C"
