// Host runtime of the FaSS-MVS library: handle, argument validation,
// per-frame planning (relative poses, level intrinsics, plane lists,
// homographies and the P2 table in double precision), device buffers, the
// coarse-to-fine level loop on one HIP stream, polling, stage timers and the
// stage entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fassmvs.h"
#include "kernels.hpp"
#include "handle_internal.hpp"

using namespace fmvs;

namespace {

enum Stage {
    ST_UPLOAD = 0, ST_PYR, ST_CENSUS, ST_SWEEP, ST_SGM_DIRS, ST_SGM_WTA, ST_REFINE, ST_MEDIAN,
    ST_NORMALS, ST_SEED, ST_OUTPUT, ST_SGM_DEBUG, ST_POST, ST_COUNT
};
static_assert(ST_COUNT == FASSMVS_N_STAGES, "stage count");
const char *kStageNames[ST_COUNT] = {"upload", "pyramid", "census", "sweep", "sgm_dirs", "sgm_wta",
                                     "refine", "median", "normals", "seed", "output", "sgm_debug", "post"};

std::string g_create_error;

// Scratch of the allocation-free DoG filter (fassmvs_filter_dog_noalloc): the
// horizontal Gaussian pass (double) and the two mask images (u8) of at most
// kNoAllocMaxPixels pixels.  Each device holds its own copy from module load
// until the process ends; its address is looked up once per device, with
// that device current, when the first handle on it is created.
constexpr size_t kNoAllocMaxPixels = (size_t)1 << 22;
constexpr size_t kNoAllocBytes = kNoAllocMaxPixels * 10;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be
// current).  Returns nullptr if the lookup fails.
void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

__global__ void k_fill(uint8_t *p, uint8_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Plain device-to-device copy in 16-byte units (grid-stride).  Reads and
// writes every byte exactly once, so its HBM byte counters calibrate the
// profiler's fetch / write counters.
__global__ void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct LevelPlan {
    int w = 0, h = 0;
    double K[9], Kinv[9];
    int F = 0, D = 0, sumG = 0;
    int G[kMaxFam], W[kMaxFam], foff[kMaxFam], goff[kMaxFam];
    double step[kMaxFam];   // inverse-distance step (lists uniform in 1/delta; path-gradient SGM)
    bool windows = false, sn = false;
    size_t h_off = 0;   // offset (doubles) of this level's homographies in the parameter blob
    size_t d_off = 0;   // offset (doubles) of this level's plane lists
    size_t i_off = 0;   // offset (doubles) of their inverse distances
};

struct FramePlan {
    int n_levels = 0, n_views = 0, nL = 0, nR = 0, m = 0;
    int w = 0, h = 0;
    int F = 0;
    double fam_n[kMaxFam][3];
    int p1 = 0;
    int lut[256];
    std::vector<double> blob;   // homographies then plane lists, all levels
    LevelPlan lv[FASSMVS_MAX_LEVELS];
    int side[kMaxViews];
    double work_hyp = 0, work_hyp_views = 0, sgm_bytes = 0;
};

struct TimedEvent {
    int stage, level;
    hipEvent_t a, b;
};

}  // namespace

struct fassmvs_handle {
    fassmvs_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    bool latched = false;
    std::mutex mu;

    // frame state (one slot)
    bool busy = false;
    uint64_t ticket = 0, next_ticket = 1;
    hipEvent_t done = nullptr;
    FramePlan plan;
    int out_w = 0, out_h = 0;

    // device buffers
    size_t held = 0;
    uint64_t gen = 0;   // bumped whenever a device buffer moves (captured graphs then go stale)
    bool exact_growth = false;

    // batched frames (fassmvs_submit_batch): one child handle per frame of
    // the batch (own buffers and plan, this handle's stream)
    std::vector<fassmvs_handle *> children;
    int batch_n = 0;
    bool batch_busy = false;
    uint64_t batch_ticket = 0;
    DevBuf batch_dev;                 // per-round argument blocks of the batched launches
    void *batch_stage = nullptr;      // their pinned host copy
    size_t batch_stage_bytes = 0;
    struct BatchGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<hipGraphExec_t> parts;   // a batch: one graph per frame group
        uint64_t gen = 0;
        uint64_t used = 0;   // last use (the least recently used graph is dropped when the cache is full)
    };
    uint64_t graph_clock = 0;
    std::map<std::string, BatchGraph> graphs;
    std::map<std::string, BatchGraph> frame_graphs;   // single frames (profile off), by plan shape and values
    struct Tuning {
        int rpt = 0, target = 8192, groups = 1;   // rpt 0: each frame level's own tile height
        bool graph = true;
        double ms = 0.0;
    };
    std::vector<hipStream_t> group_streams;   // one per frame group of a batch
    std::vector<hipEvent_t> group_ev;         // fork, then one join per group
    hipEvent_t batch_tev[2] = {nullptr, nullptr};   // tuning timer
    std::map<std::string, Tuning> tuned;
    Tuning last_tuning;
    DevBuf pyr[kMaxViews + 1];       // every level of each image, level 0 first
    DevBuf ct, S, wta, c3, params, work_ctr;
    DevBuf sgmbuf[8];
    DevBuf sbar;
    DevBuf post_tmp, post_m0, post_m1, post_hits;
    struct LevelBufs {
        DevBuf depth_raw, depth, nraw, normal, conf, label, fam, offs, dI, dbar, nbar;
    } lb[FASSMVS_MAX_LEVELS];
    // pinned staging
    void *pin = nullptr;
    size_t pin_bytes = 0;

    // timers
    std::vector<TimedEvent> pending_timers;
    std::vector<hipEvent_t> event_pool;
    double stage_ms[ST_COUNT] = {};
    int32_t stage_n[ST_COUNT] = {};
    double stage_ms_lv[FASSMVS_MAX_LEVELS][ST_COUNT] = {};
    int32_t stage_n_lv[FASSMVS_MAX_LEVELS][ST_COUNT] = {};
    int cur_level = -1;                 // level the timers being enqueued belong to (-1: frame-wide)
    bool prebuilt = false;              // this frame's device images carry their whole pyramids
    DevBuf wtab;                        // normal-smoothing weight table (see weight_table)
    const void *wtab_at = nullptr;      // the allocation the table was last written to
    int wtab_radius = -1;
    double wtab_beta = 0.0;
    hipEvent_t frame_t0 = nullptr;      // the frame's start on the stream (profiling)
    std::vector<fassmvs_timeline_entry> timeline;   // the last polled frame's timed steps
    double last_work[4] = {};
    unsigned long long sweep_work = 0;
    unsigned long long *work_host = nullptr;   // pinned: the counter's copy must not block the submit
};

namespace {

fassmvs_status fail(fassmvs_handle *h, fassmvs_status st, const std::string &msg) {
    if (h) h->err = msg;
    return st;
}

fassmvs_status dev_fail(fassmvs_handle *h, hipError_t e, const char *what) {
    h->latched = true;
    h->err = std::string(what) + ": " + hipGetErrorString(e);
    return FASSMVS_EDEVICE;
}

#define HIPCHK(h, expr, what)                                   \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return dev_fail((h), e_, (what)); \
    } while (0)

fassmvs_status ensure(fassmvs_handle *h, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return FASSMVS_OK;
    // some headroom for the next, larger frame (not for server slots, whose
    // admission counts the exact growth)
    size_t want = h->exact_growth ? bytes : bytes + bytes / 8;
    if (h->cfg.hbm_budget_bytes && h->held - b.bytes + want > h->cfg.hbm_budget_bytes) {
        want = bytes;
        if (h->held - b.bytes + want > h->cfg.hbm_budget_bytes)
            return fail(h, FASSMVS_ENOMEM, "frame exceeds the handle's HBM budget");
    }
    if (b.p) {
        hipFree(b.p);
        h->held -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(h, FASSMVS_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    b.bytes = want;
    h->held += want;
    h->gen++;
    return FASSMVS_OK;
}

void release(DevBuf &b) {
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

hipEvent_t get_event(fassmvs_handle *h) {
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Timer {
    fassmvs_handle *h;
    int stage;
    hipEvent_t a = nullptr;
    Timer(fassmvs_handle *hh, int st) : h(hh), stage(st) {
        if (h->cfg.profile) {
            a = get_event(h);
            if (a) hipEventRecord(a, h->stream);
        }
    }
    ~Timer() {
        if (a) {
            hipEvent_t b = get_event(h);
            if (b) {
                hipEventRecord(b, h->stream);
                h->pending_timers.push_back({stage, h->cur_level, a, b});
            } else {
                h->event_pool.push_back(a);
            }
        }
    }
};

void collect_timers(fassmvs_handle *h) {
    if (h->frame_t0) h->timeline.clear();
    for (auto &t : h->pending_timers) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            h->stage_ms[t.stage] += ms;
            h->stage_n[t.stage] += 1;
            if (t.level >= 0 && t.level < FASSMVS_MAX_LEVELS) {
                h->stage_ms_lv[t.level][t.stage] += ms;
                h->stage_n_lv[t.level][t.stage] += 1;
            }
            float st = 0.0f;
            if (h->frame_t0 && hipEventElapsedTime(&st, h->frame_t0, t.a) == hipSuccess)
                h->timeline.push_back(fassmvs_timeline_entry{t.stage, t.level, (double)st, (double)ms});
        }
        h->event_pool.push_back(t.a);
        h->event_pool.push_back(t.b);
    }
    h->pending_timers.clear();
    if (h->frame_t0) h->event_pool.push_back(h->frame_t0);
    h->frame_t0 = nullptr;
}

// Sweep tuning knob, read at every launch: FASSMVS_SWEEP_ROWS = 4 or 8 rows
// per thread (tile 64x16 or 64x32).  Unset, the launcher picks 8 for census
// and 4 for NCC.  It changes the schedule only, never the result.
int sweep_rows() {
    const char *e = std::getenv("FASSMVS_SWEEP_ROWS");
    const int r = e ? std::atoi(e) : 0;
    return (r == 4 || r == 8) ? r : 0;
}


bool finite_all(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// ------------------------------------------------------------- geometry
// Intrinsics of pyramid level l (focal lengths, skew and principal point
// scaled by 2^-l, exact) and their inverse by back substitution on the
// upper-triangular matrix.
bool kinv_level(const double *K, int level, double *Kl, double *Ki) {
    if (K[3] != 0.0 || K[6] != 0.0 || K[7] != 0.0 || K[8] != 1.0) return false;
    const double sc = std::ldexp(1.0, -level);
    for (int i = 0; i < 9; ++i) Kl[i] = i == 8 ? 1.0 : K[i] * sc;
    if (!(Kl[0] > 0.0) || !(Kl[4] > 0.0)) return false;
    // rows from the bottom: Ki = K^-1 with K = [fx s cx; 0 fy cy; 0 0 1]
    const double ify = 1.0 / Kl[4], ifx = 1.0 / Kl[0];
    Ki[6] = 0.0;
    Ki[7] = 0.0;
    Ki[8] = 1.0;
    Ki[3] = 0.0;
    Ki[4] = ify;
    Ki[5] = -Kl[5] * ify;
    Ki[0] = ifx;
    Ki[1] = -Kl[1] * Ki[4] * ifx;
    Ki[2] = -(Kl[1] * Ki[5] + Kl[2]) * ifx;
    return true;
}

// Pose of view k relative to the reference camera: R = R_k R_ref^T and, with
// the camera centres C = -R^T t of both cameras, t = R_k (C_ref - C_k), so
// that x_k = R x_ref + t.
void relative_pose(const double *Rr, const double *tr, const double *Rk, const double *tk, double *R, double *t) {
    double Cr[3], Ck[3], d[3];
    for (int i = 0; i < 3; ++i) {
        Cr[i] = -(Rr[i] * tr[0] + Rr[3 + i] * tr[1] + Rr[6 + i] * tr[2]);
        Ck[i] = -(Rk[i] * tk[0] + Rk[3 + i] * tk[1] + Rk[6 + i] * tk[2]);
    }
    for (int i = 0; i < 3; ++i) d[i] = Cr[i] - Ck[i];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[r * 3 + c] = Rk[r * 3] * Rr[c * 3] + Rk[r * 3 + 1] * Rr[c * 3 + 1] + Rk[r * 3 + 2] * Rr[c * 3 + 2];
        t[r] = Rk[r * 3] * d[0] + Rk[r * 3 + 1] * d[1] + Rk[r * 3 + 2] * d[2];
    }
}

// Plane-induced homographies of one view at one level (Eq. homography),
// in the form the sweep's plane loop wants: for planes n^T X + delta = 0 of
// one family, H(delta) = A + (1/delta) B with A = K R K^-1 (the homography
// at infinity) and the rank-1 B = -(K t)(K^-T n)^T, since
// K (R - t n^T / delta) K^-1 = K R K^-1 - (K t)(n^T K^-1) / delta.
struct ViewGeom {
    double A[9];    // K R K^-1
    double Kt[3];   // K t
};

void view_geom(const double *K, const double *Ki, const double *R, const double *t, ViewGeom &g) {
    double KR[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) KR[r * 3 + c] = K[r * 3] * R[c] + K[r * 3 + 1] * R[3 + c] + K[r * 3 + 2] * R[6 + c];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            g.A[r * 3 + c] = KR[r * 3] * Ki[c] + KR[r * 3 + 1] * Ki[3 + c] + KR[r * 3 + 2] * Ki[6 + c];
        g.Kt[r] = K[r * 3] * t[0] + K[r * 3 + 1] * t[1] + K[r * 3 + 2] * t[2];
    }
}

// B = -(K t)(n^T K^-1): the part of the homography that scales with 1/delta.
void family_term(const ViewGeom &g, const double *Ki, const double *n, double *B) {
    double nK[3];
    for (int c = 0; c < 3; ++c) nK[c] = n[0] * Ki[c] + n[1] * Ki[3 + c] + n[2] * Ki[6 + c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[r * 3 + c] = -g.Kt[r] * nK[c];
}

// ------------------------------------------------------------- plane lists
// The coarsest list of a family with count planes uniform in inverse
// distance over [lo, hi] (index 0 at the nearest plane).
void uniform_list(double lo, double hi, int count, double *out) {
    const double near_inv = 1.0 / lo;
    const double step = (near_inv - 1.0 / hi) / (double)(count - 1);
    for (int j = 0; j < count; ++j) out[j] = 1.0 / (near_inv - (double)j * step);
}

// A list of G planes from a list top[0..Gt-1] of increasing distances:
// plane j sits at the fractional index j (Gt - 1) / (G - 1) of top; between
// two planes of top the inverse distance runs linearly, and a plane at a
// whole index keeps top's distance.  Finer levels refine the coarsest list
// this way; a list longer than the 256-plane cap is resampled the same way.
void resample_list(const double *top, int Gt, int G, double *out) {
    const long den = G - 1;
    for (int j = 0; j < G; ++j) {
        const long pos = (long)j * (Gt - 1);
        const long k = pos / den, frac = pos % den;
        if (frac == 0) {
            out[j] = top[k];
            continue;
        }
        const double u = (double)frac / (double)den;
        const double i0 = 1.0 / top[k], i1 = 1.0 / top[k + 1];
        out[j] = 1.0 / (i0 + u * (i1 - i0));
    }
}

// Parameters of the DoG texture filter: 7x7 Gaussian with sigma
// 0.3 ((7 - 1) / 2 - 1) + 0.8 = 1.4, taps normalised to sum 1, threshold 0.5
// on the 0..255 scale, speckle sizes 7 (activation) and 21 (deactivation).
PostArgs dog_args() {
    PostArgs a;
    std::memset(&a, 0, sizeof(a));
    a.radius = 3;
    const double sigma = 1.4;
    double sum = 0.0;
    for (int i = -a.radius; i <= a.radius; ++i) {
        a.taps[i + a.radius] = std::exp(-(double)(i * i) / (2.0 * sigma * sigma));
        sum += a.taps[i + a.radius];
    }
    for (int i = 0; i <= 2 * a.radius; ++i) a.taps[i] /= sum;
    a.thresh = 0.5;
    a.min_on = 7;
    a.min_off = 21;
    return a;
}

// Cross-ratio plane list (Alg. 2).  Writes up to cap distances into out
// and returns the list length, or -1 on degenerate geometry.
int cross_ratio_list(const double *K, int w, int h, const double *R, const double *t, const double *n, double dmin,
                     double dmax, int cap, double *out) {
    double Kl[9], Ki[9];
    if (!kinv_level(K, 0, Kl, Ki)) return -1;
    double Ck[3];   // camera centre of view k in reference coordinates
    for (int i = 0; i < 3; ++i) Ck[i] = -(R[0 * 3 + i] * t[0] + R[1 * 3 + i] * t[1] + R[2 * 3 + i] * t[2]);
    if (!(n[0] * Ck[0] + n[1] * Ck[1] + n[2] * Ck[2] + dmin > 0.0)) return -1;
    auto cross_norm = [](const double *a, const double *b) {
        const double c0 = a[1] * b[2] - a[2] * b[1], c1 = a[2] * b[0] - a[0] * b[2], c2 = a[0] * b[1] - a[1] * b[0];
        return std::sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    };
    auto norm = [](const double *a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); };
    auto sin_between = [&](const double *a, const double *b) { return cross_norm(a, b) / (norm(a) * norm(b)); };
    double seg = -1.0, q0[3] = {0, 0, 0}, q1[3] = {0, 0, 0}, i0[2] = {0, 0}, i1[2] = {0, 0};
    for (int c = 0; c < 4; ++c) {
        const double u = (c & 1) ? w - 0.5 : 0.5, v = (c & 2) ? h - 0.5 : 0.5;
        const double r[3] = {Ki[0] * u + Ki[1] * v + Ki[2], Ki[3] * u + Ki[4] * v + Ki[5], Ki[6] * u + Ki[7] * v + Ki[8]};
        const double nr = n[0] * r[0] + n[1] * r[1] + n[2] * r[2];
        if (!(nr < 0.0)) continue;
        double ends[2][3], img[2][2];
        bool ok = true;
        for (int e = 0; e < 2; ++e) {
            const double s = -(e == 0 ? dmin : dmax) / nr;
            const double X[3] = {s * r[0], s * r[1], s * r[2]};
            for (int i = 0; i < 3; ++i) ends[e][i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + t[i];
            if (!(ends[e][2] > 0.0)) { ok = false; break; }
            img[e][0] = (K[0] * ends[e][0] + K[1] * ends[e][1] + K[2] * ends[e][2]) / ends[e][2];
            img[e][1] = (K[3] * ends[e][0] + K[4] * ends[e][1] + K[5] * ends[e][2]) / ends[e][2];
        }
        if (!ok) continue;
        const double L = std::hypot(img[0][0] - img[1][0], img[0][1] - img[1][1]);
        if (L > seg) {
            seg = L;
            std::memcpy(q0, ends[0], sizeof(q0));
            std::memcpy(q1, ends[1], sizeof(q1));
            std::memcpy(i0, img[0], sizeof(i0));
            std::memcpy(i1, img[1], sizeof(i1));
        }
    }
    if (!(seg > 0.0)) return -1;
    const int whole = (int)std::floor(seg);
    const int len = whole + 1 + ((double)whole < seg ? 1 : 0);
    const double dx = (i0[0] - i1[0]) / seg, dy = (i0[1] - i1[1]) / seg;
    const double s01 = sin_between(q0, q1), se1 = sin_between(t, q1);
    for (int i = 0; i < len && i < cap; ++i) {
        double d;
        if (i == 0) {
            d = dmax;
        } else if (i > whole) {
            d = dmin;
        } else {
            const double u = i1[0] + i * dx, v = i1[1] + i * dy;
            const double V[3] = {Ki[0] * u + Ki[1] * v + Ki[2], Ki[3] * u + Ki[4] * v + Ki[5], Ki[6] * u + Ki[7] * v + Ki[8]};
            const double s0i = sin_between(q0, V);
            if (!(s0i > 0.0)) {
                d = dmin;
            } else {
                const double Q = sin_between(t, V) * s01 / (se1 * s0i);
                d = Q * dmax * dmin / (Q * dmax - (dmax - dmin));
            }
        }
        out[i] = d;
    }
    return len;
}

fassmvs_status validate_config(const fassmvs_config *c, std::string &msg) {
    if (c->n_levels < 1 || c->n_levels > FASSMVS_MAX_LEVELS) { msg = "n_levels must be 1..5"; return FASSMVS_EINVAL; }
    if (!(c->census_w & 1) || !(c->census_h & 1) || c->census_w < 3 || c->census_h < 3) {
        msg = "census window must be odd";
        return FASSMVS_EINVAL;
    }
    if (c->cost != 0 && c->cost != 1) { msg = "cost must be 0 (census) or 1 (NCC)"; return FASSMVS_EINVAL; }
    if (c->cost == 0) {
        if (c->census_w * c->census_h - 1 > 64) { msg = "census window exceeds 64 bits"; return FASSMVS_EINVAL; }
        bool ok_cw = (c->census_w == 5 && c->census_h == 5) || (c->census_w == 9 && c->census_h == 7) ||
                     (c->census_w == 7 && c->census_h == 7) || (c->census_w == 3 && c->census_h == 3);
        if (!ok_cw) { msg = "census window not built (3x3, 5x5, 7x7, 9x7)"; return FASSMVS_EUNSUPPORTED; }
    } else {
        bool ok_nw = c->census_w == c->census_h && c->census_w >= 3 && c->census_w <= 9;
        if (!ok_nw) { msg = "NCC window not built (3x3, 5x5, 7x7, 9x9)"; return FASSMVS_EUNSUPPORTED; }
    }
    if (c->n_paths != 4 && c->n_paths != 8) { msg = "n_paths must be 4 or 8"; return FASSMVS_EINVAL; }
    if (c->sgm_variant < 0 || c->sgm_variant > 2) { msg = "sgm_variant must be 0, 1 or 2"; return FASSMVS_EINVAL; }
    if (c->p1 < 0 || c->p1 > 4096) { msg = "p1 out of range"; return FASSMVS_EINVAL; }
    if (c->p2_mode != 0 && c->p2_mode != 1) { msg = "p2_mode must be 0 or 1"; return FASSMVS_EINVAL; }
    if (c->p2_mode == 0 && (c->p2_fixed < c->p1 || c->p2_fixed > 65535)) {
        msg = "fixed P2 must be >= P1";
        return FASSMVS_EINVAL;
    }
    if (c->p2_mode == 1 && (!(c->p2_alpha >= 0.0) || !(c->p2_beta > 0.0) || !std::isfinite(c->p2_alpha))) {
        msg = "adaptive P2 needs alpha >= 0 and beta > 0";
        return FASSMVS_EINVAL;
    }
    if (c->window_labels < 0) { msg = "window_labels must be >= 0"; return FASSMVS_EINVAL; }
    if (c->dog_filter != 0 && c->dog_filter != 1) { msg = "dog_filter must be 0 or 1"; return FASSMVS_EINVAL; }
    if (c->normal_radius < 1 || c->normal_radius > 4) { msg = "normal_radius must be 1..4"; return FASSMVS_EINVAL; }
    if (!(c->normal_beta > 0.0) || !(c->conf_rho_deg > 0.0 && c->conf_rho_deg < 90.0)) {
        msg = "normal_beta > 0 and 0 < rho < 90 required";
        return FASSMVS_EINVAL;
    }
    return FASSMVS_OK;
}

// Validate a frame and build its plan (EINVAL / EUNSUPPORTED on failure).
fassmvs_status make_plan(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views, const int8_t *side,
                         int n_views, const double *K, const fassmvs_plane_family *fam, int F, FramePlan &P) {
    const fassmvs_config &c = h->cfg;
    if (!ref || !views || !side || !K || !fam) return fail(h, FASSMVS_EINVAL, "null argument");
    if (n_views < 1 || n_views > kMaxViews) return fail(h, FASSMVS_EINVAL, "n_views must be 1..8");
    if (F < 1 || F > kMaxFam) return fail(h, FASSMVS_EINVAL, "n_families must be 1..8");
    const int w = ref->width, hh = ref->height;
    if (w <= 0 || hh <= 0 || ref->stride < w || !ref->pixels) return fail(h, FASSMVS_EINVAL, "bad reference image");
    if ((w >> (c.n_levels - 1)) < 8 || (hh >> (c.n_levels - 1)) < 8)
        return fail(h, FASSMVS_EINVAL, "image too small for the pyramid height");
    if ((size_t)w * hh > (size_t)1 << 28) return fail(h, FASSMVS_EINVAL, "image too large");
    if (!finite_all(ref->R, 9) || !finite_all(ref->t, 3)) return fail(h, FASSMVS_EINVAL, "non-finite reference pose");
    P = FramePlan();
    P.n_levels = c.n_levels;
    P.n_views = n_views;
    P.w = w;
    P.h = hh;
    P.F = F;
    for (int k = 0; k < n_views; ++k) {
        const fassmvs_image &v = views[k];
        if (v.width != w || v.height != hh || v.stride < w || !v.pixels)
            return fail(h, FASSMVS_EINVAL, "matching images must have the reference's size");
        if (!finite_all(v.R, 9) || !finite_all(v.t, 3)) return fail(h, FASSMVS_EINVAL, "non-finite view pose");
        if (side[k] == -1) P.nL++;
        else if (side[k] == 1) P.nR++;
        else return fail(h, FASSMVS_EINVAL, "view_side must be -1 or +1");
        P.side[k] = side[k];
    }
    P.m = std::max(P.nL, P.nR);
    // cost bound of S and the penalty scale: the census sum over a subset is
    // scaled to m views; the NCC subset mean stays on one view's 0..255
    const int nbits = c.cost == 0 ? c.census_w * c.census_h - 1 : 255;
    const int mpen = c.cost == 0 ? P.m : 1;
    if (c.cost == 0 && P.m * nbits > 255)
        return fail(h, FASSMVS_EUNSUPPORTED, "matching cost exceeds 8 bits (m * census bits > 255)");
    if (!(std::fabs(K[0]) > 0) || K[3] != 0.0 || K[6] != 0.0 || K[7] != 0.0 || K[8] != 1.0 || !finite_all(K, 9))
        return fail(h, FASSMVS_EINVAL, "K must be upper triangular with K[8] = 1");
    // relative poses and camera centres in reference coordinates
    double Rrel[kMaxViews][9], trel[kMaxViews][3];
    for (int k = 0; k < n_views; ++k) relative_pose(ref->R, ref->t, views[k].R, views[k].t, Rrel[k], trel[k]);
    // coarsest-level plane list of every family, increasing distances
    double Kt[9], Kti[9];
    if (!kinv_level(K, c.n_levels - 1, Kt, Kti)) return fail(h, FASSMVS_EINVAL, "K must have positive focal lengths");
    const int wt = w >> (c.n_levels - 1), ht = hh >> (c.n_levels - 1);
    std::vector<double> top[kMaxFam];
    bool all_uniform = true;
    for (int f = 0; f < F; ++f) {
        const fassmvs_plane_family &pf = fam[f];
        double nn = pf.n[0] * pf.n[0] + pf.n[1] * pf.n[1] + pf.n[2] * pf.n[2];
        if (!finite_all(pf.n, 3) || std::fabs(nn - 1.0) > 1e-6 || !(pf.n[2] < 0.0))
            return fail(h, FASSMVS_EINVAL, "plane normals must be unit vectors facing the camera");
        for (int i = 0; i < 3; ++i) P.fam_n[f][i] = pf.n[i];
        if (pf.delta) {
            if (pf.count < 2 || pf.count > FASSMVS_MAX_TOP_PLANES)
                return fail(h, FASSMVS_EINVAL, "an explicit plane list needs 2..256 distances");
            top[f].assign(pf.delta, pf.delta + pf.count);
            if (top[f].front() > top[f].back()) std::reverse(top[f].begin(), top[f].end());
            for (int j = 0; j < pf.count; ++j)
                if (!std::isfinite(top[f][j]) || !(top[f][j] > 0.0) || (j > 0 && !(top[f][j] > top[f][j - 1])))
                    return fail(h, FASSMVS_EINVAL, "plane distances must be positive and strictly monotone");
            all_uniform = false;
        } else {
            double lo = pf.delta_min, hi = pf.delta_max;
            if (lo == 0.0 && hi == 0.0) {
                // bounding planes of the depth range over the reference frustum
                double bp[2];
                if (fassmvs_bounding_planes(K, w, hh, pf.n, pf.depth_min, pf.depth_max, bp) != FASSMVS_OK)
                    return fail(h, FASSMVS_EINVAL, "a family without distances needs 0 < depth_min < depth_max");
                lo = bp[0];
                hi = bp[1];
            }
            if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi))
                return fail(h, FASSMVS_EINVAL, "plane distances need 0 < delta_min < delta_max");
            if (pf.count != 0) {
                if (pf.count < 2 || pf.count > FASSMVS_MAX_TOP_PLANES)
                    return fail(h, FASSMVS_EINVAL, "plane count at the coarsest level must be 0 or 2..256");
                top[f].resize(pf.count);
                uniform_list(lo, hi, pf.count, top[f].data());
            } else {
                // the cross-ratio list of the view whose list is longest
                all_uniform = false;
                std::vector<double> best;
                for (int k = 0; k < n_views; ++k) {
                    double probe[1];
                    const int len = cross_ratio_list(Kt, wt, ht, Rrel[k], trel[k], pf.n, lo, hi, 0, probe);
                    if (len <= (int)best.size()) continue;
                    std::vector<double> lst(len);
                    cross_ratio_list(Kt, wt, ht, Rrel[k], trel[k], pf.n, lo, hi, len, lst.data());
                    best.swap(lst);
                }
                if (best.size() < 2) return fail(h, FASSMVS_EINVAL, "no cross-ratio plane list for a family with count 0");
                std::reverse(best.begin(), best.end());
                if (best.size() > (size_t)FASSMVS_MAX_TOP_PLANES) {
                    top[f].resize(FASSMVS_MAX_TOP_PLANES);
                    resample_list(best.data(), (int)best.size(), FASSMVS_MAX_TOP_PLANES, top[f].data());
                } else {
                    top[f].swap(best);
                }
            }
        }
        // every camera centre in front of the nearest plane
        for (int k = 0; k < n_views; ++k) {
            double C[3];
            for (int i = 0; i < 3; ++i)
                C[i] = -(Rrel[k][0 * 3 + i] * trel[k][0] + Rrel[k][1 * 3 + i] * trel[k][1] + Rrel[k][2 * 3 + i] * trel[k][2]);
            if (!(pf.n[0] * C[0] + pf.n[1] * C[1] + pf.n[2] * C[2] + top[f].front() > 0.0))
                return fail(h, FASSMVS_EINVAL, "a camera centre lies behind the nearest sweep plane");
        }
    }
    if (c.sgm_variant == 2 && !all_uniform)
        return fail(h, FASSMVS_EUNSUPPORTED, "SGM^Pi-pg needs plane lists uniform in inverse distance");
    // penalties: P1 and P2 scaled like the cost
    P.p1 = mpen * c.p1;
    int p2max = 0;
    for (int i = 0; i < 256; ++i) {
        if (c.p2_mode == 0)
            P.lut[i] = mpen * c.p2_fixed;
        else
            P.lut[i] = (int)std::floor((double)P.p1 * (1.0 + c.p2_alpha * std::exp(-(double)i / c.p2_beta)) + 0.5);
        p2max = std::max(p2max, P.lut[i]);
    }
    if ((long)c.n_paths * ((long)mpen * nbits + p2max) > 65535)
        return fail(h, FASSMVS_EUNSUPPORTED, "aggregated cost could exceed 16 bits; lower P1/P2 or views");
    // levels
    size_t hsz = 0, dsz = 0;
    for (int l = 0; l < c.n_levels; ++l) {
        LevelPlan &L = P.lv[l];
        L.w = l == 0 ? w : P.lv[l - 1].w / 2;
        L.h = l == 0 ? hh : P.lv[l - 1].h / 2;
        if (!kinv_level(K, l, L.K, L.Kinv)) return fail(h, FASSMVS_EINVAL, "K must have positive focal lengths");
        L.F = F;
        const bool coarsest = l == c.n_levels - 1;
        L.windows = !coarsest && c.window_labels > 0;
        L.sn = !coarsest && c.sgm_variant == 1;
        int D = 0, sumG = 0;
        for (int f = 0; f < F; ++f) {
            long G = (long)top[f].size() << (c.n_levels - 1 - l);
            if (G > 65535) return fail(h, FASSMVS_EUNSUPPORTED, "plane list too long");
            L.G[f] = (int)G;
            L.W[f] = L.windows ? std::min(c.window_labels, L.G[f]) : L.G[f];
            L.foff[f] = D;
            L.goff[f] = sumG;
            D += L.W[f];
            sumG += L.G[f];
        }
        if (D > FASSMVS_MAX_LABELS) return fail(h, FASSMVS_EUNSUPPORTED, "more than 512 labels per pixel at a level");
        L.D = D;
        L.sumG = sumG;
        L.h_off = hsz;
        hsz += (size_t)n_views * sumG * 9;
        P.work_hyp += (double)L.w * L.h * D;
        P.work_hyp_views += (double)L.w * L.h * D * n_views;
        // S read once per path, each path's u16 costs written once and read once
        P.sgm_bytes += (double)L.w * L.h * D * (c.n_paths * (1.0 + 2.0 + 2.0));
    }
    for (int l = 0; l < c.n_levels; ++l) {
        P.lv[l].d_off = hsz + dsz;
        P.lv[l].i_off = hsz + dsz + P.lv[l].sumG;
        dsz += 2 * (size_t)P.lv[l].sumG;
    }
    P.blob.assign(hsz + dsz, 0.0);
    for (int l = 0; l < c.n_levels; ++l) {
        LevelPlan &L = P.lv[l];
        double *dl = P.blob.data() + L.d_off;
        for (int f = 0; f < F; ++f) {
            double *lst = dl + L.goff[f];
            const int Gt = (int)top[f].size();
            if (L.G[f] == Gt)
                std::copy(top[f].begin(), top[f].end(), lst);
            else
                resample_list(top[f].data(), Gt, L.G[f], lst);
            for (int j = 1; j < L.G[f]; ++j)
                if (!(lst[j] > lst[j - 1])) return fail(h, FASSMVS_EINVAL, "plane list too dense at a finer level");
            double *inv = P.blob.data() + L.i_off + L.goff[f];
            for (int j = 0; j < L.G[f]; ++j) inv[j] = 1.0 / lst[j];
            // inverse-distance step of a uniform list (path-gradient SGM)
            L.step[f] = (1.0 / lst[0] - 1.0 / lst[L.G[f] - 1]) / (double)(L.G[f] - 1);
        }
        for (int k = 0; k < n_views; ++k) {
            ViewGeom g;
            view_geom(L.K, L.Kinv, Rrel[k], trel[k], g);
            for (int f = 0; f < F; ++f) {
                double B[9];
                family_term(g, L.Kinv, P.fam_n[f], B);
                for (int j = 0; j < L.G[f]; ++j) {
                    double *H = P.blob.data() + L.h_off + ((size_t)k * L.sumG + L.goff[f] + j) * 9;
                    const double iv = 1.0 / dl[L.goff[f] + j];
                    for (int e = 0; e < 9; ++e) H[e] = g.A[e] + iv * B[e];
                    if (!finite_all(H, 9)) return fail(h, FASSMVS_EINVAL, "degenerate homography");
                }
            }
        }
    }
    return FASSMVS_OK;
}

size_t pyr_total(int w, int hh, int levels) {
    size_t s = 0;
    for (int l = 0; l < levels; ++l) {
        s += (size_t)w * hh;
        w /= 2;
        hh /= 2;
    }
    return s;
}

// The normal-smoothing weights of Eq. normal-smooth, g0 exp(-d2 / (2
// sigma^2) - dI / beta) with sigma = radius and g0 = 1 / sqrt(2 pi sigma^2),
// for every squared offset d2 = 0..2 radius^2 and intensity difference
// dI = 0..255, evaluated on the host in double (the expression as written),
// uploaded to the handle's table once per (radius, beta).  Synchronous: call
// outside graph capture.
size_t weight_table_bytes(int radius) { return (size_t)(2 * radius * radius + 1) * 256 * 8; }

fassmvs_status weight_table(fassmvs_handle *h, int radius, double beta) {
    if (h->wtab.p && h->wtab.p == h->wtab_at && h->wtab_radius == radius && h->wtab_beta == beta)
        return FASSMVS_OK;
    const double PI = 3.14159265358979323846;
    const double sigma = (double)radius;
    const double g0 = 1.0 / std::sqrt(2.0 * PI * sigma * sigma);
    const int nd = 2 * radius * radius + 1;
    std::vector<double> t((size_t)nd * 256);
    for (int d2 = 0; d2 < nd; ++d2)
        for (int i = 0; i < 256; ++i) {
            const double dI = (double)i;
            t[(size_t)d2 * 256 + i] = g0 * std::exp(-(double)d2 / (2.0 * sigma * sigma) - dI / beta);
        }
    fassmvs_status st = ensure(h, h->wtab, t.size() * 8);
    if (st != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpy(h->wtab.p, t.data(), t.size() * 8, hipMemcpyHostToDevice), "weight table");
    h->wtab_at = h->wtab.p;
    h->wtab_radius = radius;
    h->wtab_beta = beta;
    return FASSMVS_OK;
}

// Every device buffer a frame needs and its size in bytes.
void frame_buffers(fassmvs_handle *h, const FramePlan &P, std::vector<std::pair<DevBuf *, size_t>> &out) {
    const fassmvs_config &c = h->cfg;
    const size_t N0 = (size_t)P.w * P.h;
    size_t NDmax = 0;
    for (int l = 0; l < P.n_levels; ++l) NDmax = std::max(NDmax, (size_t)P.lv[l].w * P.lv[l].h * P.lv[l].D);
    const size_t pyr = pyr_total(P.w, P.h, P.n_levels);
    out.clear();
    for (int i = 0; i <= P.n_views; ++i) out.emplace_back(&h->pyr[i], pyr);
    out.emplace_back(&h->ct, N0 * 8);
    out.emplace_back(&h->S, NDmax);
    for (int i = 0; i < c.n_paths; ++i) out.emplace_back(&h->sgmbuf[i], NDmax * 2);
    if (c.sgm_debug) out.emplace_back(&h->sbar, NDmax * 2);
    out.emplace_back(&h->wta, N0 * 2);
    if (c.dog_filter) {
        out.emplace_back(&h->post_tmp, N0 * 8);
        out.emplace_back(&h->post_m0, N0);
        out.emplace_back(&h->post_m1, N0);
    }
    out.emplace_back(&h->c3, N0 * 6);
    out.emplace_back(&h->wtab, weight_table_bytes(c.normal_radius));
    out.emplace_back(&h->params, P.blob.size() * 8);
    out.emplace_back(&h->work_ctr, 8);
    for (int l = 0; l < P.n_levels; ++l) {
        const size_t N = (size_t)P.lv[l].w * P.lv[l].h;
        auto &B = h->lb[l];
        out.emplace_back(&B.depth_raw, N * 4);
        out.emplace_back(&B.depth, N * 4);
        out.emplace_back(&B.nraw, N * 12);
        out.emplace_back(&B.normal, N * 12);
        out.emplace_back(&B.conf, N * 4);
        out.emplace_back(&B.label, N * 4);
        out.emplace_back(&B.fam, N * 4);
        out.emplace_back(&B.offs, N * 4 * P.F);
        out.emplace_back(&B.dI, N * 8 * P.F);
        out.emplace_back(&B.dbar, N * 4);
        out.emplace_back(&B.nbar, N * 12);
    }
}

fassmvs_status alloc_frame(fassmvs_handle *h, const FramePlan &P) {
    std::vector<std::pair<DevBuf *, size_t>> bufs;
    frame_buffers(h, P, bufs);
    fassmvs_status st;
    for (auto &b : bufs)
        if ((st = ensure(h, *b.first, b.second)) != FASSMVS_OK) return st;
    size_t pin = pyr_total(P.w, P.h, 1) * (P.n_views + 1) + P.blob.size() * 8 + 64;
    if (h->pin_bytes < pin) {
        if (h->pin) hipHostFree(h->pin);
        h->pin = nullptr;
        h->pin_bytes = 0;
        if (hipHostMalloc(&h->pin, pin) != hipSuccess) {
            (void)hipGetLastError();
            h->pin = nullptr;
            return fail(h, FASSMVS_ENOMEM, "pinned staging allocation failed");
        }
        h->pin_bytes = pin;
    }
    return FASSMVS_OK;
}

// Run the SGM stage of one level: every direction writes its own path-cost
// buffer in one launch (all paths of all directions concurrently), then a
// streaming kernel sums the buffers and takes the argmin.  With Sbar the
// full aggregate is also written (tests).
struct PgGeom {
    const double *delta;   // device plane lists of the level
    const double (*fam_n)[3];
};

fassmvs_status run_sgm(fassmvs_handle *h, const LevelPlan &L, const uint8_t *S, const int32_t *offs,
                       const int8_t *dI, const uint8_t *ref, int p1, const int *lut, int n_paths, uint16_t *const *bufs,
                       uint16_t *Sbar, uint16_t *wta, uint16_t *c3, const PgGeom *pgg = nullptr) {
    SgmArgs a;
    std::memset(&a, 0, sizeof(a));
    if (pgg) {
        if (L.sumG > kMaxPgPlanes) return fail(h, FASSMVS_EUNSUPPORTED, "path-gradient SGM holds at most 2048 planes");
        a.pg = 1;
        a.sumG = L.sumG;
        a.delta = pgg->delta;
        for (int f = 0; f < L.F; ++f) {
            a.goff[f] = L.goff[f];
            a.step[f] = L.step[f];
            for (int i = 0; i < 3; ++i) a.fam_n[f][i] = pgg->fam_n[f][i];
        }
        std::memcpy(a.Kinv, L.Kinv, sizeof(a.Kinv));
    }
    a.w = L.w;
    a.h = L.h;
    a.D = L.D;
    a.n_fam = L.F;
    for (int f = 0; f < L.F; ++f) {
        a.W[f] = L.W[f];
        a.foff[f] = L.foff[f];
    }
    a.S = S;
    a.offs = offs;
    a.dI = dI;
    a.ref = ref;
    a.p1 = p1;
    for (int i = 0; i < 256; ++i) a.lut[i] = lut[i];
    {
        Timer t(h, ST_SGM_DIRS);
        a.n_dirs = n_paths;
        for (int d = 0; d < n_paths; ++d) {
            a.dirs[d] = d;
            a.out[d] = bufs[d];
        }
        HIPCHK(h, launch_sgm(a, h->stream), "sgm launch");
    }
    if (Sbar) {
        Timer t(h, ST_SGM_DEBUG);
        HIPCHK(h, launch_sum_u16(bufs, n_paths, (size_t)L.w * L.h * L.D, Sbar, h->stream), "sum launch");
    }
    if (wta) {
        Timer t(h, ST_SGM_WTA);
        a.n_dirs = 0;
        a.n_in = n_paths;
        for (int b = 0; b < n_paths; ++b) a.in[b] = bufs[b];
        a.final_mode = 1;
        a.wta = wta;
        a.c3 = c3;
        HIPCHK(h, launch_sgm(a, h->stream), "wta launch");
    }
    return FASSMVS_OK;
}

// ---------------------------------------------------------------- the frame's steps
// A frame runs as: pyramid; then per level, coarsest first: reference
// census, sweep, aggregation (all directions), winner-takes-all,
// refinement and the rest (median, normals, DoG mask, seeds of the next
// level).  The single-frame path runs them in order; the batched path runs
// each step for every frame of a round before the next, with the sweeps
// and the aggregations of all frames in one launch each.

size_t level_offset(const FramePlan &P, int l) {
    size_t off = 0;
    for (int i = 0; i < l; ++i) off += (size_t)P.lv[i].w * P.lv[i].h;
    return off;
}

fassmvs_status enqueue_pyramid(fassmvs_handle *h, const FramePlan &P) {
    if (!h->prebuilt) {
        Timer t(h, ST_PYR);
        for (int i = 0; i <= P.n_views; ++i) {
            uint8_t *base = (uint8_t *)h->pyr[i].p;
            size_t off = 0;
            for (int l = 0; l + 1 < P.n_levels; ++l) {
                const LevelPlan &L = P.lv[l];
                HIPCHK(h, launch_pyr_down(base + off, L.w, L.h, L.w, base + off + (size_t)L.w * L.h, h->stream),
                       "pyramid launch");
                off += (size_t)L.w * L.h;
            }
        }
    }
    h->sweep_work = 0;
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, h->stream, (uint8_t *)h->work_ctr.p, (uint8_t)0, (size_t)8);
    HIPCHK(h, hipGetLastError(), "work counter");
    return FASSMVS_OK;
}

const uint8_t *level_ref(fassmvs_handle *h, const FramePlan &P, int l) {
    return (const uint8_t *)h->pyr[0].p + level_offset(P, l);
}

fassmvs_status enqueue_census(fassmvs_handle *h, const FramePlan &P, int l) {
    const fassmvs_config &c = h->cfg;
    if (c.cost != 0) return FASSMVS_OK;
    const LevelPlan &L = P.lv[l];
    Timer t(h, ST_CENSUS);
    HIPCHK(h, launch_census(level_ref(h, P, l), L.w, L.h, c.census_w, c.census_h, (uint64_t *)h->ct.p, h->stream),
           "census");
    return FASSMVS_OK;
}

SweepArgs sweep_args(fassmvs_handle *h, const FramePlan &P, int l) {
    const fassmvs_config &c = h->cfg;
    const LevelPlan &L = P.lv[l];
    const size_t off = level_offset(P, l);
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = L.w;
    a.h = L.h;
    a.cw = c.census_w;
    a.ch = c.census_h;
    a.n_views = P.n_views;
    a.nL = P.nL;
    a.nR = P.nR;
    a.m = P.m;
    for (int k = 0; k < P.n_views; ++k) {
        a.views[k] = (const uint8_t *)h->pyr[k + 1].p + off;
        a.side[k] = P.side[k];
    }
    a.cost = c.cost;
    a.ct_ref = (const uint64_t *)h->ct.p;
    a.ref = level_ref(h, P, l);
    a.n_fam = L.F;
    a.D = L.D;
    a.sumG = L.sumG;
    for (int f = 0; f < L.F; ++f) {
        a.G[f] = L.G[f];
        a.W[f] = L.W[f];
        a.foff[f] = L.foff[f];
        a.goff[f] = L.goff[f];
    }
    a.H = (const double *)h->params.p + L.h_off;
    a.offs = L.windows ? (const int32_t *)h->lb[l].offs.p : nullptr;
    a.S = (uint8_t *)h->S.p;
    a.work = (unsigned long long *)h->work_ctr.p;
    // Tile height for the census cost (FASSMVS_SWEEP_ROWS overrides): 64x16
    // tiles where several plane families share the level (each family's
    // label windows move across a tile, and a shorter tile evaluates a
    // smaller union of them; it also keeps 4 waves per SIMD resident) or
    // where the level is small (more tiles to spread over the CUs); 64x32
    // otherwise (less halo to warp).  The same costs either way.
    int rows = sweep_rows();
    if (rows == 0 && c.cost == 0)
        rows = (L.F > 1 || (double)L.w * L.h * L.D <= 33554432.0) ? 4 : 8;
    a.rows_per_thread = rows;
    return a;
}

// The aggregation's arguments for every direction of the frame's level,
// each into its own path-cost buffer.
SgmArgs sgm_args(fassmvs_handle *h, const FramePlan &P, int l) {
    const LevelPlan &L = P.lv[l];
    SgmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = L.w;
    a.h = L.h;
    a.D = L.D;
    a.n_fam = L.F;
    for (int f = 0; f < L.F; ++f) {
        a.W[f] = L.W[f];
        a.foff[f] = L.foff[f];
    }
    a.S = (const uint8_t *)h->S.p;
    a.offs = L.windows ? (const int32_t *)h->lb[l].offs.p : nullptr;
    a.dI = L.sn ? (const int8_t *)h->lb[l].dI.p : nullptr;
    a.ref = level_ref(h, P, l);
    a.p1 = P.p1;
    for (int i = 0; i < 256; ++i) a.lut[i] = P.lut[i];
    a.n_dirs = h->cfg.n_paths;
    for (int d = 0; d < a.n_dirs; ++d) {
        a.dirs[d] = d;
        a.out[d] = (uint16_t *)h->sgmbuf[d].p;
    }
    return a;
}

// Winner-takes-all over the level's path-cost buffers.
fassmvs_status enqueue_wta(fassmvs_handle *h, const SgmArgs &dirs) {
    Timer t(h, ST_SGM_WTA);
    SgmArgs a = dirs;
    a.n_dirs = 0;
    a.n_in = h->cfg.n_paths;
    for (int b = 0; b < a.n_in; ++b) a.in[b] = (uint16_t *)h->sgmbuf[b].p;
    a.final_mode = 1;
    a.wta = (uint16_t *)h->wta.p;
    a.c3 = (uint16_t *)h->c3.p;
    HIPCHK(h, launch_sgm(a, h->stream), "wta launch");
    return FASSMVS_OK;
}

// Refinement, median, normals with confidence, the DoG mask at level 0, and
// the seeds of the next finer level.
fassmvs_status enqueue_post(fassmvs_handle *h, const FramePlan &P, int l) {
    const fassmvs_config &c = h->cfg;
    double *dblob = (double *)h->params.p;
    const LevelPlan &L = P.lv[l];
    const size_t N = (size_t)L.w * L.h;
    auto &B = h->lb[l];
    const uint8_t *ref = level_ref(h, P, l);
    const int32_t *offs = L.windows ? (const int32_t *)B.offs.p : nullptr;
    {
        Timer t(h, ST_REFINE);
        RefineArgs a;
        std::memset(&a, 0, sizeof(a));
        a.w = L.w;
        a.h = L.h;
        a.n_fam = L.F;
        for (int f = 0; f < L.F; ++f) {
            a.W[f] = L.W[f];
            a.G[f] = L.G[f];
            a.foff[f] = L.foff[f];
            a.goff[f] = L.goff[f];
            for (int i = 0; i < 3; ++i) a.fam_n[f][i] = P.fam_n[f][i];
        }
        std::memcpy(a.Kinv, L.Kinv, sizeof(a.Kinv));
        a.delta = dblob + L.d_off;
        a.offs = offs;
        a.wta = (const uint16_t *)h->wta.p;
        a.c3 = (const uint16_t *)h->c3.p;
        a.label = (int32_t *)B.label.p;
        a.fam = (int32_t *)B.fam.p;
        a.depth = (float *)(c.median ? B.depth_raw.p : B.depth.p);
        HIPCHK(h, launch_refine(a, h->stream), "refine launch");
    }
    if (c.median) {
        Timer t(h, ST_MEDIAN);
        HIPCHK(h, launch_median5((const float *)B.depth_raw.p, L.w, L.h, (float *)B.depth.p, h->stream), "median");
    }
    {
        Timer t(h, ST_NORMALS);
        NormalArgs a;
        std::memset(&a, 0, sizeof(a));
        a.w = L.w;
        a.h = L.h;
        a.radius = c.normal_radius;
        a.beta = c.normal_beta;
        a.wtab = (const double *)h->wtab.p;
        a.cos_rho = std::cos(c.conf_rho_deg * 3.14159265358979323846 / 180.0);
        std::memcpy(a.Kinv, L.Kinv, sizeof(a.Kinv));
        a.n_fam = L.F;
        for (int f = 0; f < L.F; ++f)
            for (int i = 0; i < 3; ++i) a.fam_n[f][i] = P.fam_n[f][i];
        a.depth = (const float *)B.depth.p;
        a.img = ref;
        a.label = (const int32_t *)B.label.p;
        a.fam = (const int32_t *)B.fam.p;
        a.nraw = (float *)B.nraw.p;
        a.normal = (float *)B.normal.p;
        a.conf = (float *)B.conf.p;
        HIPCHK(h, launch_normals(a, h->stream), "normals launch");
    }
    if (l == 0 && c.dog_filter) {
        Timer t(h, ST_POST);
        PostArgs pa = dog_args();
        HIPCHK(h, launch_dog_mask(ref, L.w, L.h, pa, (double *)h->post_tmp.p, (uint8_t *)h->post_m0.p,
                                  (uint8_t *)h->post_m1.p, h->stream),
               "dog filter");
        HIPCHK(h, launch_apply_keep((const uint8_t *)h->post_m1.p, N, (float *)B.depth.p, (float *)B.normal.p,
                                    (float *)B.conf.p, h->stream),
               "dog apply");
    }
    if (l > 0) {
        Timer t(h, ST_SEED);
        const LevelPlan &Lf = P.lv[l - 1];
        auto &Bf = h->lb[l - 1];
        SeedArgs a;
        std::memset(&a, 0, sizeof(a));
        a.cw = L.w;
        a.ch = L.h;
        a.fw = Lf.w;
        a.fh = Lf.h;
        a.n_fam = Lf.F;
        std::memcpy(a.Kinv, Lf.Kinv, sizeof(a.Kinv));
        for (int f = 0; f < Lf.F; ++f) {
            for (int i = 0; i < 3; ++i) a.fam_n[f][i] = P.fam_n[f][i];
            a.goff[f] = Lf.goff[f];
            a.G[f] = Lf.G[f];
            a.W[f] = Lf.W[f];
        }
        a.inv = dblob + Lf.i_off;
        a.depth_c = (const float *)B.depth.p;
        a.normal_c = (const float *)B.normal.p;
        a.dbar = (float *)Bf.dbar.p;
        a.nbar = (float *)Bf.nbar.p;
        a.offs = (int32_t *)Bf.offs.p;
        a.dI = Lf.sn ? (int8_t *)Bf.dI.p : nullptr;
        HIPCHK(h, launch_seed(a, h->stream), "seed launch");
    }
    return FASSMVS_OK;
}

// Images to level 0 of each pyramid and the parameter blob to the device,
// through the handle's pinned staging (host images) or device copies.
fassmvs_status upload_frame(fassmvs_handle *h, const FramePlan &P, const fassmvs_image *ref,
                            const fassmvs_image *views, int mem_kind) {
    fassmvs_status wst = weight_table(h, h->cfg.normal_radius, h->cfg.normal_beta);
    if (wst != FASSMVS_OK) return wst;
    const size_t N0 = (size_t)P.w * P.h;
    Timer t(h, ST_UPLOAD);
    uint8_t *pin = (uint8_t *)h->pin;
    for (int i = 0; i <= P.n_views; ++i) {
        const fassmvs_image &im = i == 0 ? *ref : views[i - 1];
        uint8_t *dst = (uint8_t *)h->pyr[i].p;
        if (mem_kind == FASSMVS_MEM_HOST) {
            uint8_t *stg = pin + N0 * i;
            for (int y = 0; y < P.h; ++y) std::memcpy(stg + (size_t)y * P.w, im.pixels + (size_t)y * im.stride, P.w);
            HIPCHK(h, hipMemcpyAsync(dst, stg, N0, hipMemcpyHostToDevice, h->stream), "image upload");
        } else if (h->prebuilt) {
            HIPCHK(h, hipMemcpyAsync(dst, im.pixels, level_offset(P, P.n_levels), hipMemcpyDeviceToDevice, h->stream),
                   "pyramid copy");
        } else {
            HIPCHK(h, hipMemcpy2DAsync(dst, P.w, im.pixels, im.stride, P.w, P.h, hipMemcpyDeviceToDevice, h->stream),
                   "image copy");
        }
    }
    double *pb = (double *)(pin + N0 * (P.n_views + 1) + 64 - ((uintptr_t)(pin + N0 * (P.n_views + 1)) & 63));
    std::memcpy(pb, P.blob.data(), P.blob.size() * 8);
    HIPCHK(h, hipMemcpyAsync(h->params.p, pb, P.blob.size() * 8, hipMemcpyHostToDevice, h->stream), "params");
    return FASSMVS_OK;
}

fassmvs_status enqueue_frame(fassmvs_handle *h, const FramePlan &P) {
    const fassmvs_config &c = h->cfg;
    fassmvs_status st;
    if ((st = enqueue_pyramid(h, P)) != FASSMVS_OK) return st;
    for (int l = P.n_levels - 1; l >= 0; --l) {
        const LevelPlan &L = P.lv[l];
        h->cur_level = l;
        if ((st = enqueue_census(h, P, l)) != FASSMVS_OK) return st;
        {
            Timer t(h, ST_SWEEP);
            HIPCHK(h, launch_sweep(sweep_args(h, P, l), h->stream), "sweep launch");
        }
        const SgmArgs sa = sgm_args(h, P, l);
        uint16_t *bufs[8];
        for (int i = 0; i < 8; ++i) bufs[i] = (uint16_t *)h->sgmbuf[i].p;
        PgGeom pgg{(const double *)h->params.p + L.d_off, P.fam_n};
        st = run_sgm(h, L, sa.S, sa.offs, sa.dI, sa.ref, P.p1, P.lut, c.n_paths, bufs,
                     c.sgm_debug ? (uint16_t *)h->sbar.p : nullptr, (uint16_t *)h->wta.p, (uint16_t *)h->c3.p,
                     c.sgm_variant == 2 ? &pgg : nullptr);
        if (st != FASSMVS_OK) return st;
        if ((st = enqueue_post(h, P, l)) != FASSMVS_OK) return st;
    }
    h->cur_level = -1;
    return FASSMVS_OK;
}

constexpr size_t kMaxFrameGraphs = 8;   // captured frame graphs kept per handle

void release_graph(fassmvs_handle::BatchGraph &g) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    for (hipGraphExec_t e : g.parts)
        if (e) hipGraphExecDestroy(e);
    g.parts.clear();
}

// The cache entry for key, making room (dropping the least recently used
// graph) when the cache is full; marks it used.
fassmvs_handle::BatchGraph &graph_slot(fassmvs_handle *h, std::map<std::string, fassmvs_handle::BatchGraph> &cache,
                                       const std::string &key, size_t cap) {
    if (cache.size() >= cap && !cache.count(key)) {
        auto lru = cache.begin();
        for (auto it = cache.begin(); it != cache.end(); ++it)
            if (it->second.used < lru->second.used) lru = it;
        release_graph(lru->second);
        cache.erase(lru);
    }
    auto &g = cache[key];
    g.used = ++h->graph_clock;
    return g;
}

// A frame plan's shape and the values its launches take by value (the key
// of a captured frame graph), with the launch-time tuning knobs.
std::string plan_signature(const FramePlan &P) {
    std::string sig;
    auto raw = [&sig](const void *p, size_t b) { sig.append((const char *)p, b); };
    const char *knobs[] = {"FASSMVS_SWEEP_ROWS", "FASSMVS_SWEEP_BLOCKS", "FASSMVS_SGM_UNPACKED"};
    for (const char *k : knobs) {
        const char *e = std::getenv(k);
        sig += std::string(k) + "=" + (e ? e : "") + ";";
    }
    raw(&P.n_levels, sizeof(int));
    raw(&P.n_views, sizeof(int));
    raw(&P.w, sizeof(int));
    raw(&P.h, sizeof(int));
    raw(&P.F, sizeof(int));
    raw(&P.nL, sizeof(int));
    raw(&P.nR, sizeof(int));
    raw(P.side, sizeof(int) * P.n_views);
    raw(P.fam_n, sizeof(double) * 3 * P.F);
    raw(&P.p1, sizeof(int));
    raw(P.lut, sizeof(P.lut));
    for (int l = 0; l < P.n_levels; ++l) {
        const LevelPlan &L = P.lv[l];
        raw(&L.w, sizeof(int));
        raw(&L.h, sizeof(int));
        raw(&L.D, sizeof(int));
        raw(&L.sumG, sizeof(int));
        raw(L.G, sizeof(int) * L.F);
        raw(L.W, sizeof(int) * L.F);
        raw(L.step, sizeof(double) * L.F);
        raw(L.Kinv, sizeof(L.Kinv));
        const char flags[2] = {(char)L.windows, (char)L.sn};
        raw(flags, 2);
        raw(&L.h_off, sizeof(size_t));
        raw(&L.d_off, sizeof(size_t));
        raw(&L.i_off, sizeof(size_t));
    }
    return sig;
}

// Enqueue the frame's launches: replayed from a captured graph when the
// handle does not profile (HIP-event timers cannot sit in a graph) and
// FASSMVS_FRAME_GRAPH is not 0; launch by launch otherwise.
fassmvs_status enqueue_frame_graph(fassmvs_handle *h, const FramePlan &P) {
    const char *e = std::getenv("FASSMVS_FRAME_GRAPH");
    if (h->cfg.profile || (e && std::atoi(e) == 0)) return enqueue_frame(h, P);
    const std::string key = plan_signature(P);
    auto &g = graph_slot(h, h->frame_graphs, key, kMaxFrameGraphs);
    if (!g.exec || g.gen != h->gen) {
        release_graph(g);
        HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed), "frame graph capture");
        fassmvs_status st = enqueue_frame(h, P);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(h->stream, &graph);
        if (st != FASSMVS_OK) {
            if (graph) hipGraphDestroy(graph);
            h->frame_graphs.erase(key);
            return st;
        }
        HIPCHK(h, ee, "frame graph capture");
        ee = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        HIPCHK(h, ee, "frame graph instantiation");
        g.gen = h->gen;
    }
    HIPCHK(h, hipGraphLaunch(g.exec, h->stream), "frame graph launch");
    return FASSMVS_OK;
}

fassmvs_status copy_out(fassmvs_handle *h, void *dst, const void *src, size_t bytes, int mem_kind) {
    if (!dst) return FASSMVS_OK;
    hipMemcpyKind k = mem_kind == FASSMVS_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(h, hipMemcpyAsync(dst, src, bytes, k, h->stream), "output copy");
    return FASSMVS_OK;
}

// ---------------------------------------------------------------- batched frames
// A batch runs as G groups of frames, each group on a stream of its own
// (forked from and joined back into the handle's stream), so the
// instruction-bound sweeps of one group overlap the memory-bound
// aggregations of another.  Inside a group, frames run round by round from
// each frame's coarsest level (frames with fewer levels finish early); a
// round's sweeps are one launch and its aggregations one persistent launch
// per label-pair count.

// One persistent aggregation launch over some frames of a round.
struct SgmLaunch {
    size_t off = 0;
    int n = 0, jobs = 0, kp = 1, nf = 1;
    bool win = false, sn = false;
};

// One sweep launch over some frames of a round (one tile height).
struct SweepLaunch {
    size_t off = 0;
    int rpt = 8, blocks = 0;
    std::vector<int> idx;   // positions in the round's frame list
};

struct BatchRound {
    std::vector<int> frames, levels;   // frames (batch order) and their level in this round
    std::vector<SweepLaunch> sweeps;   // one per tile height among the round's frames
    std::vector<SgmLaunch> sgm;
    std::vector<char> own_sgm;   // per frame of the round: aggregates in launches of its own
};

struct BatchGroup {
    std::vector<int> frames;
    std::vector<BatchRound> rounds;
    size_t counter_off = 0;   // the persistent aggregation's job counter
};

// Sweep rows per thread of a frame level in a batch: the tuned value, or
// with 0 the level's own choice (sweep_args), as a single frame would run.
int batch_rows(fassmvs_handle *c, int l, int tuned) {
    if (tuned == 4 || tuned == 8) return tuned;
    const int r = sweep_args(c, c->plan, l).rows_per_thread;
    return (r == 4 || r == 8) ? r : (c->cfg.cost == 1 ? 4 : 8);
}

constexpr size_t kAlign = 256;
constexpr size_t kMaxBatchGraphs = 8;   // captured batch graphs kept per handle
constexpr int kMaxBatchGroups = 16;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// The batch's shape: sizes, view split, plane counts and windows of every
// frame and level.  With values, also what the per-frame launches take by
// value (intrinsics, plane normals, list steps, penalties), so that a
// captured graph is replayed only for frames that agree in all of it.
std::string batch_signature(fassmvs_handle *h, int n, const fassmvs_handle::Tuning *t, bool values) {
    std::string sig = t ? std::to_string(t->rpt) + "/" + std::to_string(t->target) + "/" + std::to_string(t->groups)
                        : std::string("shape");
    auto raw = [&sig](const void *p, size_t b) { sig.append((const char *)p, b); };
    for (int i = 0; i < n; ++i) {
        const FramePlan &P = h->children[i]->plan;
        sig += "|" + std::to_string(P.w) + "x" + std::to_string(P.h) + "v" + std::to_string(P.nL) + "," +
               std::to_string(P.nR) + "F" + std::to_string(P.F);
        for (int l = 0; l < P.n_levels; ++l) {
            const LevelPlan &L = P.lv[l];
            sig += ":" + std::to_string(L.D) + "/" + std::to_string(L.sumG) + (L.windows ? "w" : "") +
                   (L.sn ? "s" : "");
            if (values) {
                raw(L.Kinv, sizeof(L.Kinv));
                raw(L.step, sizeof(double) * L.F);
                raw(L.G, sizeof(int) * L.F);
                raw(L.W, sizeof(int) * L.F);
            }
        }
        if (values) {
            raw(P.fam_n, sizeof(double) * 3 * P.F);
            raw(&P.p1, sizeof(P.p1));
            raw(P.lut, sizeof(P.lut));
        }
    }
    return sig;
}

// Frames into groups of about equal work (pixels x labels x views over the
// levels), largest first.
std::vector<std::vector<int>> batch_groups(fassmvs_handle *h, int n, int G) {
    std::vector<std::pair<double, int>> work(n);
    for (int i = 0; i < n; ++i) {
        const FramePlan &P = h->children[i]->plan;
        double w = 0.0;
        for (int l = 0; l < P.n_levels; ++l) w += (double)P.lv[l].w * P.lv[l].h * P.lv[l].D * P.n_views;
        work[i] = {w, i};
    }
    std::stable_sort(work.begin(), work.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
        return x.first > y.first;
    });
    G = std::max(1, std::min(G, n));
    std::vector<std::vector<int>> groups(G);
    std::vector<double> load(G, 0.0);
    for (auto &wi : work) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        groups[g].push_back(wi.second);
        load[g] += wi.first;
    }
    for (auto &g : groups) std::sort(g.begin(), g.end());
    return groups;
}

// Every group's and round's argument blocks into the pinned stage (grown as
// needed); *bytes receives their size, the groups' job counters at its end.
fassmvs_status batch_prepare(fassmvs_handle *h, int n, const fassmvs_handle::Tuning &t,
                             std::vector<BatchGroup> &groups, size_t *bytes) {
    const auto assign = batch_groups(h, n, t.groups);
    groups.assign(assign.size(), BatchGroup());
    // the rounds and their frames; label-pair classes decide the layout
    size_t off = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        BatchGroup &g = groups[gi];
        g.frames = assign[gi];
        int R = 0;
        for (int i : g.frames) R = std::max(R, h->children[i]->plan.n_levels);
        g.rounds.assign(R, BatchRound());
        for (int r = 0; r < R; ++r) {
            BatchRound &br = g.rounds[r];
            for (int i : g.frames) {
                const int l = h->children[i]->plan.n_levels - 1 - r;
                if (l < 0) continue;
                br.frames.push_back(i);
                br.levels.push_back(l);
            }
            for (int rpt : {8, 4}) {
                SweepLaunch S;
                S.rpt = rpt;
                for (size_t j = 0; j < br.frames.size(); ++j)
                    if (batch_rows(h->children[br.frames[j]], br.levels[j], t.rpt) == rpt) S.idx.push_back((int)j);
                if (S.idx.empty()) continue;
                S.off = off;
                off = align_up(off + sweep_batch_bytes((int)S.idx.size()));
                br.sweeps.push_back(S);
            }
            int count[5] = {0, 0, 0, 0, 0};
            for (size_t j = 0; j < br.frames.size(); ++j) {
                const int D = h->children[br.frames[j]]->plan.lv[br.levels[j]].D;
                count[std::min(4, (D + 127) / 128)]++;
            }
            for (int kp = 1; kp <= 4; ++kp) {
                if (!count[kp]) continue;
                SgmLaunch L;
                L.off = off;
                L.kp = kp;
                L.n = count[kp];
                br.sgm.push_back(L);
                off = align_up(off + sgm_batch_bytes(count[kp]));
            }
        }
    }
    for (auto &g : groups) {
        g.counter_off = off;
        off += kAlign;
    }
    const size_t total = off;
    if (h->batch_stage_bytes < total) {
        if (h->batch_stage) hipHostFree(h->batch_stage);
        h->batch_stage = nullptr;
        h->batch_stage_bytes = 0;
        if (hipHostMalloc(&h->batch_stage, total) != hipSuccess) {
            (void)hipGetLastError();
            h->batch_stage = nullptr;
            return fail(h, FASSMVS_ENOMEM, "pinned batch staging allocation failed");
        }
        h->batch_stage_bytes = total;
    }
    uint8_t *stage = (uint8_t *)h->batch_stage;
    // the path-gradient form and the debug sums aggregate frame by frame
    const bool shared_sgm = !h->cfg.sgm_debug && h->cfg.sgm_variant != 2;
    for (auto &g : groups)
        for (auto &br : g.rounds) {
            const int m = (int)br.frames.size();
            for (auto &S : br.sweeps) {
                std::vector<SweepArgs> sw;
                for (int j : S.idx) {
                    fassmvs_handle *c = h->children[br.frames[j]];
                    sw.push_back(sweep_args(c, c->plan, br.levels[j]));
                }
                S.blocks = prepare_sweep_batch(sw.data(), (int)sw.size(), S.rpt, t.target, stage + S.off);
                if (S.blocks < 0) return fail(h, FASSMVS_EINVAL, "frames of a batch must share the matching cost");
            }
            br.own_sgm.assign(m, shared_sgm ? 0 : 1);
            for (auto &L : br.sgm) {
                std::vector<SgmArgs> sg;
                std::vector<int> idx;
                for (int j = 0; j < m; ++j) {
                    fassmvs_handle *c = h->children[br.frames[j]];
                    const int D = c->plan.lv[br.levels[j]].D;
                    if (std::min(4, (D + 127) / 128) != L.kp) continue;
                    sg.push_back(sgm_args(c, c->plan, br.levels[j]));
                    idx.push_back(j);
                }
                L.jobs = shared_sgm ? prepare_sgm_batch(sg.data(), (int)sg.size(), stage + L.off, &L.kp, &L.win, &L.sn,
                                                        &L.nf)
                                    : -1;
                if (L.jobs < 0)
                    for (int j : idx) br.own_sgm[j] = 1;
            }
        }
    *bytes = total;
    return FASSMVS_OK;
}

// One group's launches on stream s (kernels only, so the sequence can be
// captured in a graph).
fassmvs_status batch_enqueue_group(fassmvs_handle *h, const BatchGroup &g, hipStream_t s) {
    const fassmvs_config &c = h->cfg;
    fassmvs_status st;
    for (int i : g.frames) {
        h->children[i]->stream = s;
        if ((st = enqueue_pyramid(h->children[i], h->children[i]->plan)) != FASSMVS_OK) return st;
    }
    uint8_t *dev = (uint8_t *)h->batch_dev.p;
    unsigned *counter = (unsigned *)(dev + g.counter_off);
    for (const BatchRound &br : g.rounds) {
        const int m = (int)br.frames.size();
        for (int j = 0; j < m; ++j) {
            fassmvs_handle *ch = h->children[br.frames[j]];
            if ((st = enqueue_census(ch, ch->plan, br.levels[j])) != FASSMVS_OK) return fail(h, st, ch->err);
        }
        for (const SweepLaunch &S : br.sweeps)
            HIPCHK(h,
                   launch_sweep_batch(dev + S.off, (int)S.idx.size(), S.blocks, S.rpt, c.census_w, c.census_h, c.cost,
                                      s),
                   "batched sweep launch");
        for (const SgmLaunch &L : br.sgm)
            if (L.jobs >= 0)
                HIPCHK(h, launch_sgm_batch(dev + L.off, L.n, L.jobs, L.kp, L.win, L.sn, L.nf, counter, s),
                       "batched aggregation launch");
        for (int j = 0; j < m; ++j) {
            fassmvs_handle *ch = h->children[br.frames[j]];
            const FramePlan &P = ch->plan;
            const int l = br.levels[j];
            const SgmArgs sa = sgm_args(ch, P, l);
            if (br.own_sgm[j]) {
                uint16_t *bufs[8];
                for (int i = 0; i < 8; ++i) bufs[i] = (uint16_t *)ch->sgmbuf[i].p;
                PgGeom pgg{(const double *)ch->params.p + P.lv[l].d_off, P.fam_n};
                st = run_sgm(ch, P.lv[l], sa.S, sa.offs, sa.dI, sa.ref, P.p1, P.lut, c.n_paths, bufs,
                             c.sgm_debug ? (uint16_t *)ch->sbar.p : nullptr, (uint16_t *)ch->wta.p,
                             (uint16_t *)ch->c3.p, c.sgm_variant == 2 ? &pgg : nullptr);
                if (st != FASSMVS_OK) return fail(h, st, ch->err);
            } else if ((st = enqueue_wta(ch, sa)) != FASSMVS_OK) {
                return fail(h, st, ch->err);
            }
            if ((st = enqueue_post(ch, P, l)) != FASSMVS_OK) return fail(h, st, ch->err);
        }
    }
    return FASSMVS_OK;
}

// The whole batch on the handle's stream: groups forked onto their own
// streams and joined back.  With ev, ev[0] / ev[1] bracket it.
fassmvs_status batch_enqueue(fassmvs_handle *h, const std::vector<BatchGroup> &groups, hipEvent_t *ev) {
    fassmvs_status st;
    if (ev) HIPCHK(h, hipEventRecord(ev[0], h->stream), "timing event");
    if (groups.size() == 1) {
        if ((st = batch_enqueue_group(h, groups[0], h->stream)) != FASSMVS_OK) return st;
    } else {
        HIPCHK(h, hipEventRecord(h->group_ev[0], h->stream), "batch fork");
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            HIPCHK(h, hipStreamWaitEvent(h->group_streams[gi], h->group_ev[0], 0), "batch fork");
            if ((st = batch_enqueue_group(h, groups[gi], h->group_streams[gi])) != FASSMVS_OK) return st;
            HIPCHK(h, hipEventRecord(h->group_ev[gi + 1], h->group_streams[gi]), "batch join");
            HIPCHK(h, hipStreamWaitEvent(h->stream, h->group_ev[gi + 1], 0), "batch join");
        }
    }
    if (ev) HIPCHK(h, hipEventRecord(ev[1], h->stream), "timing event");
    return FASSMVS_OK;
}

fassmvs_status batch_upload_args(fassmvs_handle *h, size_t bytes) {
    if (h->batch_dev.bytes < bytes) {
        fassmvs_status st = ensure(h, h->batch_dev, bytes);
        if (st != FASSMVS_OK) return st;
    }
    HIPCHK(h, hipMemcpyAsync(h->batch_dev.p, h->batch_stage, bytes, hipMemcpyHostToDevice, h->stream), "batch args");
    return FASSMVS_OK;
}

// Streams and fork / join events for up to kMaxBatchGroups groups.
fassmvs_status batch_streams(fassmvs_handle *h) {
    while ((int)h->group_streams.size() < kMaxBatchGroups) {
        hipStream_t s;
        HIPCHK(h, hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "batch stream");
        h->group_streams.push_back(s);
    }
    while ((int)h->group_ev.size() < kMaxBatchGroups + 1) {
        hipEvent_t e;
        HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "batch event");
        h->group_ev.push_back(e);
    }
    for (auto &e : h->batch_tev)
        if (!e) HIPCHK(h, hipEventCreate(&e), "timing event");
    return FASSMVS_OK;
}

bool env_off(const char *name) {
    const char *e = std::getenv(name);
    return e && std::atoi(e) == 0;
}

}  // namespace

namespace {
fassmvs_status submit_frame_locked(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                   const int8_t *view_side, int32_t n_views, const double K[9],
                                   const fassmvs_plane_family *families, int32_t n_families, int32_t mem_kind,
                                   uint64_t *ticket) {
    if (h->latched) return FASSMVS_EDEVICE;
    if (h->busy || h->batch_busy) return fail(h, FASSMVS_EBUSY, "a frame is in flight; poll it first");
    if (!ticket) return fail(h, FASSMVS_EINVAL, "null ticket");
    if (mem_kind != FASSMVS_MEM_HOST && mem_kind != FASSMVS_MEM_DEVICE) return fail(h, FASSMVS_EINVAL, "bad mem_kind");
    HIPCHK(h, hipSetDevice(h->cfg.device), "hipSetDevice");
    FramePlan &P = h->plan;
    fassmvs_status st = make_plan(h, ref, views, view_side, n_views, K, families, n_families, P);
    if (st != FASSMVS_OK) return st;
    if ((st = alloc_frame(h, P)) != FASSMVS_OK) return st;
    if (h->cfg.profile) {
        if (h->frame_t0) h->event_pool.push_back(h->frame_t0);
        h->frame_t0 = get_event(h);
        if (h->frame_t0) HIPCHK(h, hipEventRecord(h->frame_t0, h->stream), "frame start event");
    }
    h->cur_level = -1;
    if ((st = upload_frame(h, P, ref, views, mem_kind)) != FASSMVS_OK) return st;
    if ((st = enqueue_frame_graph(h, P)) != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->work_host, h->work_ctr.p, 8, hipMemcpyDeviceToHost, h->stream), "work counter");
    HIPCHK(h, hipEventRecord(h->done, h->stream), "event record");
    h->out_w = P.w;
    h->out_h = P.h;
    h->busy = true;
    h->ticket = h->next_ticket++;
    *ticket = h->ticket;
    return FASSMVS_OK;
}
}  // namespace

namespace fmvs {
fassmvs_status handle_submit_pyramids(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                      const int8_t *view_side, int32_t n_views, const double K[9],
                                      const fassmvs_plane_family *families, int32_t n_families, uint64_t *ticket) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (ref && ref->stride != ref->width) return fail(h, FASSMVS_EINVAL, "pyramid images are packed");
    for (int k = 0; views && k < n_views; ++k)
        if (views[k].stride != views[k].width) return fail(h, FASSMVS_EINVAL, "pyramid images are packed");
    h->prebuilt = true;
    fassmvs_status st =
        submit_frame_locked(h, ref, views, view_side, n_views, K, families, n_families, FASSMVS_MEM_DEVICE, ticket);
    h->prebuilt = false;
    return st;
}

size_t pyramid_bytes(int w, int h, int n_levels) {
    size_t b = 0;
    for (int l = 0; l < n_levels; ++l) {
        b += (size_t)w * h;
        w /= 2;
        h /= 2;
    }
    return b;
}

hipError_t pyramid_build(uint8_t *img, int w, int h, int n_levels, hipStream_t s) {
    size_t off = 0;
    for (int l = 0; l + 1 < n_levels; ++l) {
        hipError_t e = launch_pyr_down(img + off, w, h, w, img + off + (size_t)w * h, s);
        if (e != hipSuccess) return e;
        off += (size_t)w * h;
        w /= 2;
        h /= 2;
    }
    return hipSuccess;
}
}  // namespace fmvs

// =================================================================== C ABI

extern "C" {

fassmvs_status fassmvs_frame_footprint(const fassmvs_config *cfg, int32_t w, int32_t hgt, int32_t n_views,
                                       const fassmvs_plane_family *families, int32_t n_families, uint64_t *bytes) {
    if (!cfg || !families || !bytes || w < 1 || hgt < 1 || n_views < 1 || n_views > kMaxViews || n_families < 1 ||
        n_families > kMaxFam || cfg->n_levels < 1 || cfg->n_levels > FASSMVS_MAX_LEVELS)
        return FASSMVS_EINVAL;
    size_t NDmax = 0, maps = 0, params = 0;
    int lw = w, lh = hgt;
    for (int l = 0; l < cfg->n_levels; ++l) {
        if (l > 0) {
            lw /= 2;
            lh /= 2;
        }
        size_t D = 0;
        for (int f = 0; f < n_families; ++f) {
            // an explicit list has count entries; count 0 is counted at the cap
            const size_t count = families[f].count > 0 ? (size_t)families[f].count : (size_t)FASSMVS_MAX_TOP_PLANES;
            const size_t G = count << (cfg->n_levels - 1 - l);
            const bool windows = l < cfg->n_levels - 1 && cfg->window_labels > 0;
            D += windows ? std::min((size_t)cfg->window_labels, G) : G;
            params += G * ((size_t)n_views * 9 + 2) * 8;   // homographies, the plane list and its inverses
        }
        const size_t N = (size_t)lw * lh;
        NDmax = std::max(NDmax, N * D);
        // depth, raw depth, normals (raw, smoothed), confidence, label,
        // family, offsets and surface-normal offsets per family, seeds
        maps += N * (4 + 4 + 12 + 12 + 4 + 4 + 4 + 4 * (size_t)n_families + 8 * (size_t)n_families + 4 + 12);
    }
    const size_t N0 = (size_t)w * hgt;
    size_t total = NDmax * (1 + 2 * (size_t)cfg->n_paths) + maps + pyr_total(w, hgt, cfg->n_levels) * (n_views + 1) +
                   N0 * (8 + 2 + 6) + params + weight_table_bytes(cfg->normal_radius) + 256;
    if (cfg->sgm_debug) total += NDmax * 2;
    if (cfg->dog_filter) total += N0 * 10;
    *bytes = total;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_bounding_planes(const double K[9], int32_t w, int32_t hgt, const double n[3], double d_min,
                                       double d_max, double out[2]) {
    if (!K || !n || !out || w < 1 || hgt < 1 || !(d_min > 0.0) || !(d_max > d_min) || !finite_all(K, 9) ||
        !finite_all(n, 3))
        return FASSMVS_EINVAL;
    double Kl[9], Ki[9];
    if (!kinv_level(K, 0, Kl, Ki)) return FASSMVS_EINVAL;
    double lo = 0.0, hi = 0.0;
    for (int c = 0; c < 4; ++c) {
        const double u = (c & 1) ? (double)w : 0.0, v = (c & 2) ? (double)hgt : 0.0;
        const double r[3] = {Ki[0] * u + Ki[1] * v + Ki[2], Ki[3] * u + Ki[4] * v + Ki[5], Ki[6] * u + Ki[7] * v + Ki[8]};
        const double a = std::fabs(n[0] * r[0] + n[1] * r[1] + n[2] * r[2]);
        lo = c == 0 ? a * d_min : std::min(lo, a * d_min);
        hi = c == 0 ? a * d_max : std::max(hi, a * d_max);
    }
    out[0] = lo;
    out[1] = hi;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_cross_ratio_planes(const double K[9], int32_t w, int32_t hgt, const double R[9],
                                          const double t[3], const double n[3], double delta_min, double delta_max,
                                          int32_t max_planes, double *deltas, int32_t *count) {
    if (count) *count = 0;
    if (!K || !R || !t || !n || !count || w < 1 || hgt < 1 || !(delta_min > 0.0) || !(delta_max > delta_min) ||
        max_planes < 0 || (max_planes > 0 && !deltas) || !finite_all(K, 9) || !finite_all(R, 9) || !finite_all(t, 3) ||
        !finite_all(n, 3))
        return FASSMVS_EINVAL;
    const int len = cross_ratio_list(K, w, hgt, R, t, n, delta_min, delta_max, max_planes, deltas);
    if (len < 0) return FASSMVS_EINVAL;
    *count = len;
    return len > max_planes ? FASSMVS_EUNSUPPORTED : FASSMVS_OK;
}

void fassmvs_config_default(fassmvs_config *c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->n_levels = 3;
    c->census_w = 9;
    c->census_h = 7;
    c->n_paths = 8;
    c->sgm_variant = 0;
    c->p1 = 24;
    c->p2_mode = 1;
    c->p2_fixed = 64;
    c->p2_alpha = 8.0;
    c->p2_beta = 10.0;
    c->window_labels = 128;
    c->median = 1;
    c->normal_radius = 2;
    c->normal_beta = 10.0;
    c->conf_rho_deg = 60.0;
}

fassmvs_status fassmvs_create(const fassmvs_config *cfg, fassmvs_handle **out) {
    if (!out) return FASSMVS_EINVAL;
    *out = nullptr;
    if (!cfg) {
        g_create_error = "null config";
        return FASSMVS_EINVAL;
    }
    std::string msg;
    fassmvs_status st = validate_config(cfg, msg);
    if (st != FASSMVS_OK) {
        g_create_error = msg;
        return st;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        g_create_error = "no HIP device";
        return FASSMVS_EDEVICE;
    }
    if (cfg->device < 0 || cfg->device >= ndev) {
        g_create_error = "device ordinal out of range";
        return FASSMVS_EINVAL;
    }
    if (hipSetDevice(cfg->device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        return FASSMVS_EDEVICE;
    }
    if (!scratch_address(cfg->device)) {
        g_create_error = "scratch symbol lookup failed";
        return FASSMVS_EDEVICE;
    }
    fassmvs_handle *h = new fassmvs_handle();
    h->cfg = *cfg;
    if (cfg->stream) {
        h->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
            delete h;
            g_create_error = "stream creation failed";
            return FASSMVS_EDEVICE;
        }
        h->own_stream = true;
    }
    if (hipEventCreateWithFlags(&h->done, hipEventDisableTiming) != hipSuccess) {
        if (h->own_stream) hipStreamDestroy(h->stream);
        delete h;
        g_create_error = "event creation failed";
        return FASSMVS_EDEVICE;
    }
    if (hipHostMalloc((void **)&h->work_host, 64) != hipSuccess) {
        (void)hipGetLastError();
        hipEventDestroy(h->done);
        if (h->own_stream) hipStreamDestroy(h->stream);
        delete h;
        g_create_error = "pinned counter allocation failed";
        return FASSMVS_ENOMEM;
    }
    *h->work_host = 0;
    *out = h;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_submit_frame(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                    const int8_t *view_side, int32_t n_views, const double K[9],
                                    const fassmvs_plane_family *families, int32_t n_families, int32_t mem_kind,
                                    uint64_t *ticket) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    h->prebuilt = false;
    return submit_frame_locked(h, ref, views, view_side, n_views, K, families, n_families, mem_kind, ticket);
}

fassmvs_status fassmvs_submit_frame_range(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                          const int8_t *view_side, int32_t n_views, const double K[9], double d_min,
                                          double d_max, const fassmvs_plane_family *families, int32_t n_families,
                                          int32_t mem_kind, uint64_t *ticket) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (!(d_min > 0.0) || !(d_max > d_min) || !std::isfinite(d_max))
        return fail(h, FASSMVS_EINVAL, "depth range must satisfy 0 < d_min < d_max");
    if (!families || n_families < 1 || n_families > kMaxFam) return fail(h, FASSMVS_EINVAL, "n_families must be 1..8");
    fassmvs_plane_family fams[kMaxFam];
    for (int f = 0; f < n_families; ++f) {
        fams[f] = families[f];
        if (!fams[f].delta && fams[f].delta_min == 0.0 && fams[f].delta_max == 0.0) {
            fams[f].depth_min = d_min;
            fams[f].depth_max = d_max;
        }
    }
    h->prebuilt = false;
    return submit_frame_locked(h, ref, views, view_side, n_views, K, fams, n_families, mem_kind, ticket);
}

fassmvs_status fassmvs_submit_batch(fassmvs_handle *h, const fassmvs_frame *frames, int32_t n_frames, int32_t mem_kind,
                                    uint64_t *ticket) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->latched) return FASSMVS_EDEVICE;
    if (h->busy || h->batch_busy) return fail(h, FASSMVS_EBUSY, "a frame or batch is in flight; poll it first");
    if (!ticket || !frames || n_frames < 1 || n_frames > FASSMVS_MAX_BATCH)
        return fail(h, FASSMVS_EINVAL, "a batch holds 1..64 frames");
    if (mem_kind != FASSMVS_MEM_HOST && mem_kind != FASSMVS_MEM_DEVICE) return fail(h, FASSMVS_EINVAL, "bad mem_kind");
    HIPCHK(h, hipSetDevice(h->cfg.device), "hipSetDevice");
    // one child handle per frame: its own plan and buffers, this stream
    while ((int)h->children.size() < n_frames) {
        fassmvs_config cc = h->cfg;
        cc.stream = h->stream;
        cc.profile = 0;
        fassmvs_handle *ch = nullptr;
        fassmvs_status st = fassmvs_create(&cc, &ch);
        if (st != FASSMVS_OK) return fail(h, st, "batch slot: " + g_create_error);
        h->children.push_back(ch);
    }
    for (int i = 0; i < n_frames; ++i) {
        const fassmvs_frame &fr = frames[i];
        fassmvs_handle *ch = h->children[i];
        ch->cfg = h->cfg;
        ch->cfg.stream = h->stream;
        ch->cfg.profile = 0;
        if (fr.n_levels != 0) ch->cfg.n_levels = fr.n_levels;
        if (fr.window_labels >= 0) ch->cfg.window_labels = fr.window_labels;
        if (ch->cfg.n_levels < 1 || ch->cfg.n_levels > FASSMVS_MAX_LEVELS)
            return fail(h, FASSMVS_EINVAL, "frame " + std::to_string(i) + ": n_levels must be 1..5");
        fassmvs_status st = make_plan(ch, fr.ref, fr.views, fr.view_side, fr.n_views, fr.K, fr.families,
                                      fr.n_families, ch->plan);
        if (st != FASSMVS_OK) return fail(h, st, "frame " + std::to_string(i) + ": " + ch->err);
        if ((st = alloc_frame(ch, ch->plan)) != FASSMVS_OK) return fail(h, st, "frame " + std::to_string(i) + ": " + ch->err);
    }
    const bool graph_on = !env_off("FASSMVS_BATCH_GRAPH"), tune = !env_off("FASSMVS_BATCH_TUNE");
    fassmvs_status st;
    if ((st = batch_streams(h)) != FASSMVS_OK) return st;
    for (int i = 0; i < n_frames; ++i) {
        const fassmvs_frame &fr = frames[i];
        fassmvs_handle *ch = h->children[i];
        ch->stream = h->stream;
        if ((st = upload_frame(ch, ch->plan, fr.ref, fr.views, mem_kind)) != FASSMVS_OK) return fail(h, st, ch->err);
    }
    // One run of the batch with tuning t, from a captured graph or launch by
    // launch; with ms, timed (HIP events on the handle's stream).
    auto run = [&](const fassmvs_handle::Tuning &t, bool graph, double *ms) -> fassmvs_status {
        std::vector<BatchGroup> groups;
        size_t bytes = 0;
        fassmvs_status s2;
        if ((s2 = batch_prepare(h, n_frames, t, groups, &bytes)) != FASSMVS_OK) return s2;
        if ((s2 = batch_upload_args(h, bytes)) != FASSMVS_OK) return s2;
        hipEvent_t *ev = ms ? h->batch_tev : nullptr;
        if (graph) {
            uint64_t gen = h->gen;
            for (int i = 0; i < n_frames; ++i) gen += h->children[i]->gen;
            const std::string key = batch_signature(h, n_frames, &t, true);
            auto &g = graph_slot(h, h->graphs, key, kMaxBatchGraphs);
            const size_t G = groups.size();
            if (g.parts.size() != G || g.gen != gen) {
                release_graph(g);
                // each group's launches captured once on its stream and
                // replayed while the shape and the buffers stay: the groups'
                // graphs launch one after another, so the first group runs
                // while the host launches the rest
                g.parts.assign(G, nullptr);
                for (size_t gi = 0; gi < G; ++gi) {
                    hipStream_t gs = G == 1 ? h->stream : h->group_streams[gi];
                    HIPCHK(h, hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed), "graph capture");
                    s2 = batch_enqueue_group(h, groups[gi], gs);
                    hipGraph_t graph_ = nullptr;
                    hipError_t e = hipStreamEndCapture(gs, &graph_);
                    if (s2 == FASSMVS_OK && e == hipSuccess)
                        e = hipGraphInstantiate(&g.parts[gi], graph_, nullptr, nullptr, 0);
                    if (graph_) hipGraphDestroy(graph_);
                    if (s2 != FASSMVS_OK || e != hipSuccess) {
                        release_graph(g);
                        h->graphs.erase(key);
                        if (s2 != FASSMVS_OK) return s2;
                        HIPCHK(h, e, "graph capture");
                    }
                }
                g.gen = gen;
            }
            if (ev) HIPCHK(h, hipEventRecord(ev[0], h->stream), "timing event");
            if (G == 1) {
                HIPCHK(h, hipGraphLaunch(g.parts[0], h->stream), "graph launch");
            } else {
                HIPCHK(h, hipEventRecord(h->group_ev[0], h->stream), "batch fork");
                for (size_t gi = 0; gi < G; ++gi) {
                    HIPCHK(h, hipStreamWaitEvent(h->group_streams[gi], h->group_ev[0], 0), "batch fork");
                    HIPCHK(h, hipGraphLaunch(g.parts[gi], h->group_streams[gi]), "graph launch");
                    HIPCHK(h, hipEventRecord(h->group_ev[gi + 1], h->group_streams[gi]), "batch join");
                    HIPCHK(h, hipStreamWaitEvent(h->stream, h->group_ev[gi + 1], 0), "batch join");
                }
            }
            if (ev) HIPCHK(h, hipEventRecord(ev[1], h->stream), "timing event");
        } else if ((s2 = batch_enqueue(h, groups, ev)) != FASSMVS_OK) {
            return s2;
        }
        if (ms) {
            HIPCHK(h, hipEventSynchronize(ev[1]), "batch tuning run");
            float t_ = 0.0f;
            HIPCHK(h, hipEventElapsedTime(&t_, ev[0], ev[1]), "timing");
            *ms = t_;
        }
        return FASSMVS_OK;
    };
    // The sweep's tile height and workgroup target, the number of frame
    // groups and the graph: tuned once per batch shape by timing whole runs
    // (none of them changes a result).
    const std::string shape = batch_signature(h, n_frames, nullptr, false);
    auto tit = h->tuned.find(shape);
    fassmvs_handle::Tuning t;
    {
        // untuned: FASSMVS_BATCH_GROUPS groups (default 2)
        const char *e = std::getenv("FASSMVS_BATCH_GROUPS");
        const int G = e && std::atoi(e) > 0 ? std::atoi(e) : 2;
        t.groups = std::max(1, std::min({G, n_frames, kMaxBatchGroups}));
    }
    t.graph = graph_on;
    if (tit != h->tuned.end()) {
        t = tit->second;
    } else if (tune) {
        // the group count at the default sweep shape, then the sweep shape
        // at that count; graphs timed on their first replay
        fassmvs_handle::Tuning best;
        best.ms = 1e30;
        auto trial = [&](int rpt, int target, int G) -> fassmvs_status {
            fassmvs_handle::Tuning c;
            c.rpt = rpt;
            c.target = target;
            c.groups = G;
            c.graph = graph_on;
            fassmvs_status s2 = FASSMVS_OK;
            if (graph_on) s2 = run(c, true, nullptr);
            if (s2 == FASSMVS_OK) s2 = run(c, graph_on, &c.ms);
            if (s2 == FASSMVS_OK && c.ms < best.ms) best = c;
            return s2;
        };
        for (int G = 1; G <= std::min(n_frames, kMaxBatchGroups); G *= 2)
            if ((st = trial(0, 8192, G)) != FASSMVS_OK) return st;
        const int G = best.groups;
        for (int rpt : {0, 8, 4})
            for (int target : {8192, 16384})
                if (!(rpt == 0 && target == 8192) && (st = trial(rpt, target, G)) != FASSMVS_OK) return st;
        if (graph_on) {
            // launched call by call instead, if that is faster
            double e = 0.0;
            if ((st = run(best, false, &e)) != FASSMVS_OK) return st;
            if (e < best.ms) {
                best.graph = false;
                best.ms = e;
            }
        }
        t = best;
        h->tuned[shape] = t;
    }
    h->last_tuning = t;
    if ((st = run(t, t.graph && graph_on, nullptr)) != FASSMVS_OK) return st;
    HIPCHK(h, hipEventRecord(h->done, h->stream), "event record");
    h->batch_n = n_frames;
    h->batch_busy = true;
    h->batch_ticket = h->next_ticket++;
    *ticket = h->batch_ticket;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_poll_batch(fassmvs_handle *h, uint64_t ticket, int32_t index, float *depth, float *normal,
                                  float *confidence, int32_t mem_kind, int32_t wait_ms) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->latched) return FASSMVS_EDEVICE;
    if (ticket == 0 || ticket != h->batch_ticket) return fail(h, FASSMVS_ENOTFOUND, "unknown batch ticket");
    if (index < 0 || index >= h->batch_n) return fail(h, FASSMVS_EINVAL, "frame index outside the batch");
    if (mem_kind != FASSMVS_MEM_HOST && mem_kind != FASSMVS_MEM_DEVICE) return fail(h, FASSMVS_EINVAL, "bad mem_kind");
    HIPCHK(h, hipSetDevice(h->cfg.device), "hipSetDevice");
    if (h->batch_busy) {
        auto t0 = std::chrono::steady_clock::now();
        for (;;) {
            hipError_t e = hipEventQuery(h->done);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady) return dev_fail(h, e, "batch execution");
            if (wait_ms == 0) return FASSMVS_PENDING;
            if (wait_ms < 0) {
                HIPCHK(h, hipEventSynchronize(h->done), "batch execution");
                break;
            }
            double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (el >= wait_ms) return FASSMVS_PENDING;
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
        h->batch_busy = false;
    }
    fassmvs_handle *ch = h->children[index];
    const size_t N0 = (size_t)ch->plan.w * ch->plan.h;
    auto &B = ch->lb[0];
    fassmvs_status st;
    if ((st = copy_out(h, depth, B.depth.p, N0 * 4, mem_kind)) != FASSMVS_OK) return st;
    if ((st = copy_out(h, normal, B.normal.p, N0 * 12, mem_kind)) != FASSMVS_OK) return st;
    if ((st = copy_out(h, confidence, B.conf.p, N0 * 4, mem_kind)) != FASSMVS_OK) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream), "output copy");
    return FASSMVS_OK;
}

fassmvs_status fassmvs_batch_tuning(fassmvs_handle *h, int32_t *rows_per_thread, int32_t *sweep_blocks,
                                    int32_t *groups, int32_t *graph, double *ms) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (rows_per_thread) *rows_per_thread = h->last_tuning.rpt;
    if (sweep_blocks) *sweep_blocks = h->last_tuning.target;
    if (groups) *groups = h->last_tuning.groups;
    if (graph) *graph = h->last_tuning.graph ? 1 : 0;
    if (ms) *ms = h->last_tuning.ms;
    return FASSMVS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- for the served form
namespace fmvs {

void handle_set_exact_growth(fassmvs_handle *h) {
    std::lock_guard<std::mutex> lk(h->mu);
    h->exact_growth = true;
}

uint64_t handle_held(fassmvs_handle *h) {
    std::lock_guard<std::mutex> lk(h->mu);
    return h->held;
}

fassmvs_status handle_growth(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                             const int8_t *side, int32_t n_views, const double K[9],
                             const fassmvs_plane_family *families, int32_t n_families, uint64_t *grow) {
    std::lock_guard<std::mutex> lk(h->mu);
    FramePlan P;
    fassmvs_status st = make_plan(h, ref, views, side, n_views, K, families, n_families, P);
    if (st != FASSMVS_OK) return st;
    std::vector<std::pair<DevBuf *, size_t>> bufs;
    frame_buffers(h, P, bufs);
    uint64_t g = 0;
    for (auto &b : bufs) {
        const size_t need = b.second == 0 ? 256 : b.second;
        if (b.first->bytes >= need) continue;
        g += (h->exact_growth ? need : need + need / 8) - b.first->bytes;
    }
    *grow = g;
    return FASSMVS_OK;
}

fassmvs_status handle_reserve(fassmvs_handle *h, int w, int hgt, int n_views, const double K[9],
                              const fassmvs_plane_family *families, int n_families, bool apply, uint64_t *grow) {
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->busy || h->batch_busy) return fail(h, FASSMVS_EBUSY, "frame in flight");
    if (n_views < 1 || n_views > kMaxViews) return fail(h, FASSMVS_EINVAL, "n_views must be 1..8");
    // a bundle of that shape: the buffers depend on sizes, views and plane
    // counts, not on the poses (identity poses; pixels are not read)
    static const uint8_t dummy = 0;
    fassmvs_image ims[kMaxViews + 1];
    int8_t side[kMaxViews];
    for (int i = 0; i <= n_views; ++i) {
        std::memset(&ims[i], 0, sizeof(ims[i]));
        ims[i].pixels = &dummy;
        ims[i].width = w;
        ims[i].height = hgt;
        ims[i].stride = w;
        ims[i].R[0] = ims[i].R[4] = ims[i].R[8] = 1.0;
        if (i < n_views) side[i] = -1;
    }
    FramePlan P;
    fassmvs_status st = make_plan(h, &ims[0], &ims[1], side, n_views, K, families, n_families, P);
    if (st != FASSMVS_OK) return st;
    std::vector<std::pair<DevBuf *, size_t>> bufs;
    frame_buffers(h, P, bufs);
    uint64_t g = 0;
    for (auto &b : bufs) {
        const size_t need = b.second == 0 ? 256 : b.second;
        if (b.first->bytes < need) g += (h->exact_growth ? need : need + need / 8) - b.first->bytes;
    }
    if (grow) *grow = g;
    if (apply && g > 0) {
        HIPCHK(h, hipSetDevice(h->cfg.device), "hipSetDevice");
        HIPCHK(h, hipStreamSynchronize(h->stream), "reserve");
        return alloc_frame(h, P);
    }
    return FASSMVS_OK;
}

void handle_trim(fassmvs_handle *h) {
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->busy) return;
    hipSetDevice(h->cfg.device);
    hipStreamSynchronize(h->stream);
    auto drop = [&](DevBuf &b) {
        if (b.p) hipFree(b.p);
        h->held -= b.bytes;
        b = DevBuf();
    };
    h->gen++;
    for (auto &b : h->pyr) drop(b);
    drop(h->ct);
    drop(h->S);
    drop(h->wta);
    drop(h->c3);
    drop(h->params);
    drop(h->work_ctr);
    for (auto &b : h->sgmbuf) drop(b);
    drop(h->sbar);
    drop(h->post_tmp);
    drop(h->post_m0);
    drop(h->post_m1);
    drop(h->post_hits);
    for (auto &L : h->lb) {
        for (DevBuf *b : {&L.depth_raw, &L.depth, &L.nraw, &L.normal, &L.conf, &L.label, &L.fam, &L.offs, &L.dI,
                          &L.dbar, &L.nbar})
            drop(*b);
    }
}

}  // namespace fmvs

extern "C" {

fassmvs_status fassmvs_poll(fassmvs_handle *h, uint64_t ticket, float *depth, float *normal, float *confidence,
                            int32_t mem_kind, int32_t wait_ms) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->latched) return FASSMVS_EDEVICE;
    if (!h->busy || ticket != h->ticket) return fail(h, FASSMVS_ENOTFOUND, "unknown ticket");
    if (mem_kind != FASSMVS_MEM_HOST && mem_kind != FASSMVS_MEM_DEVICE) return fail(h, FASSMVS_EINVAL, "bad mem_kind");
    HIPCHK(h, hipSetDevice(h->cfg.device), "hipSetDevice");
    auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        hipError_t e = hipEventQuery(h->done);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return dev_fail(h, e, "frame execution");
        if (wait_ms == 0) return FASSMVS_PENDING;
        if (wait_ms < 0) {
            HIPCHK(h, hipEventSynchronize(h->done), "frame execution");
            break;
        }
        double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (el >= wait_ms) return FASSMVS_PENDING;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    const size_t N0 = (size_t)h->out_w * h->out_h;
    auto &B = h->lb[0];
    fassmvs_status st;
    {
        Timer t(h, ST_OUTPUT);
        if ((st = copy_out(h, depth, B.depth.p, N0 * 4, mem_kind)) != FASSMVS_OK) return st;
        if ((st = copy_out(h, normal, B.normal.p, N0 * 12, mem_kind)) != FASSMVS_OK) return st;
        if ((st = copy_out(h, confidence, B.conf.p, N0 * 4, mem_kind)) != FASSMVS_OK) return st;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream), "output copy");
    collect_timers(h);
    h->last_work[0] = h->plan.work_hyp;
    h->last_work[1] = h->plan.work_hyp_views;
    h->sweep_work = *h->work_host;
    h->last_work[2] = (double)h->sweep_work;
    h->last_work[3] = h->plan.sgm_bytes;
    h->busy = false;
    return FASSMVS_OK;
}

void fassmvs_destroy(fassmvs_handle *h) {
    if (!h) return;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        hipSetDevice(h->cfg.device);
        hipStreamSynchronize(h->stream);
        // batch slots run on this stream and the group streams: released before them
        for (auto *c : h->children) fassmvs_destroy(c);
        h->children.clear();
        for (auto s_ : h->group_streams) hipStreamDestroy(s_);
        for (auto e : h->group_ev) hipEventDestroy(e);
        for (auto e : h->batch_tev)
            if (e) hipEventDestroy(e);
        for (auto &b : h->pyr) release(b);
        release(h->ct);
        release(h->S);
        release(h->wta);
        release(h->c3);
        release(h->params);
        release(h->work_ctr);
        release(h->sbar);
        release(h->wtab);
        for (auto &b : h->sgmbuf) release(b);
        for (auto &L : h->lb) {
            release(L.depth_raw); release(L.depth); release(L.nraw); release(L.normal); release(L.conf);
            release(L.label); release(L.fam); release(L.offs); release(L.dI); release(L.dbar); release(L.nbar);
        }
        for (auto &g : h->graphs) release_graph(g.second);
        for (auto &g : h->frame_graphs) release_graph(g.second);
        release(h->batch_dev);
        if (h->batch_stage) hipHostFree(h->batch_stage);
        if (h->pin) hipHostFree(h->pin);
        if (h->work_host) hipHostFree(h->work_host);
        for (auto &t : h->pending_timers) {
            hipEventDestroy(t.a);
            hipEventDestroy(t.b);
        }
        for (auto e : h->event_pool) hipEventDestroy(e);
        if (h->frame_t0) hipEventDestroy(h->frame_t0);
        if (h->done) hipEventDestroy(h->done);
        if (h->own_stream) hipStreamDestroy(h->stream);
    }
    delete h;
}

const char *fassmvs_last_error(const fassmvs_handle *h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

fassmvs_status fassmvs_stage_times(fassmvs_handle *h, double *ms, int32_t *counts, int32_t n) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    for (int i = 0; i < n && i < ST_COUNT; ++i) {
        if (ms) ms[i] = h->stage_ms[i];
        if (counts) counts[i] = h->stage_n[i];
    }
    return FASSMVS_OK;
}

fassmvs_status fassmvs_stage_times_level(fassmvs_handle *h, int32_t level, double *ms, int32_t *counts, int32_t n) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    if (level < 0 || level >= FASSMVS_MAX_LEVELS) return fail(h, FASSMVS_EINVAL, "level must be 0..4");
    for (int i = 0; i < n && i < ST_COUNT; ++i) {
        if (ms) ms[i] = h->stage_ms_lv[level][i];
        if (counts) counts[i] = h->stage_n_lv[level][i];
    }
    return FASSMVS_OK;
}

fassmvs_status fassmvs_frame_timeline(fassmvs_handle *h, fassmvs_timeline_entry *out, int32_t max_entries,
                                      int32_t *n_entries) {
    if (!h || !n_entries || max_entries < 0 || (max_entries > 0 && !out)) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    const int n = (int)h->timeline.size();
    for (int i = 0; i < n && i < max_entries; ++i) out[i] = h->timeline[i];
    *n_entries = n;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_reset_stage_times(fassmvs_handle *h) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    for (int i = 0; i < ST_COUNT; ++i) {
        h->stage_ms[i] = 0;
        h->stage_n[i] = 0;
        for (int l = 0; l < FASSMVS_MAX_LEVELS; ++l) {
            h->stage_ms_lv[l][i] = 0;
            h->stage_n_lv[l][i] = 0;
        }
    }
    return FASSMVS_OK;
}

const char *fassmvs_stage_name(int32_t s) { return (s >= 0 && s < ST_COUNT) ? kStageNames[s] : ""; }

fassmvs_status fassmvs_frame_work(fassmvs_handle *h, double *out, int32_t n) {
    if (!h || !out) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    for (int i = 0; i < n && i < 4; ++i) out[i] = h->last_work[i];
    for (int l = 0; l < FASSMVS_MAX_LEVELS && 4 + l < n; ++l)
        out[4 + l] = l < h->plan.n_levels ? (double)h->plan.lv[l].w * h->plan.lv[l].h * h->plan.lv[l].D : 0.0;
    return FASSMVS_OK;
}

fassmvs_status fassmvs_level_map(fassmvs_handle *h, int32_t level, int32_t what, void *dst, size_t dst_bytes) {
    if (!h || !dst) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    const FramePlan &P = h->plan;
    if (level < 0 || level >= P.n_levels) return fail(h, FASSMVS_EINVAL, "no such level");
    if (h->busy) return fail(h, FASSMVS_EBUSY, "frame in flight");
    const LevelPlan &L = P.lv[level];
    const size_t N = (size_t)L.w * L.h;
    if (what == 8) {
        if (dst_bytes < 8) return FASSMVS_EINVAL;
        int32_t *o = (int32_t *)dst;
        o[0] = L.w;
        o[1] = L.h;
        return FASSMVS_OK;
    }
    auto &B = h->lb[level];
    const void *src = nullptr;
    size_t bytes = 0;
    switch (what) {
        case 0: src = B.depth.p; bytes = N * 4; break;
        case 1: src = h->cfg.median ? B.depth_raw.p : B.depth.p; bytes = N * 4; break;
        case 2: src = B.normal.p; bytes = N * 12; break;
        case 3: src = B.conf.p; bytes = N * 4; break;
        case 4: src = B.label.p; bytes = N * 4; break;
        case 5: src = B.fam.p; bytes = N * 4; break;
        case 6: src = B.offs.p; bytes = N * 4 * P.F; break;
        case 7: src = B.dI.p; bytes = N * 8 * P.F; break;
        case 9:
            if (level != 0) return fail(h, FASSMVS_EINVAL, "the cost volume is kept for level 0 only");
            src = h->S.p;
            bytes = N * L.D;
            break;
        case 20:
            if (level != 0) return fail(h, FASSMVS_EINVAL, "the reference census is kept for level 0 only");
            src = h->ct.p;
            bytes = N * 8;
            break;
        default:
            if (what >= 10 && what < 10 + h->cfg.n_paths && level == 0) {
                // path costs of direction r (each direction has its own buffer)
                src = h->sgmbuf[what - 10].p;
                bytes = N * L.D * 2;
                break;
            }
            if (what >= 30 && what <= 30 + P.n_views) {
                size_t off = 0;
                for (int l = 0; l < level; ++l) off += (size_t)P.lv[l].w * P.lv[l].h;
                src = (const uint8_t *)h->pyr[what - 30].p + off;
                bytes = N;
                break;
            }
            return fail(h, FASSMVS_EINVAL, "unknown map");
    }
    if (dst_bytes < bytes) return fail(h, FASSMVS_EINVAL, "destination too small");
    HIPCHK(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, h->stream), "level map copy");
    HIPCHK(h, hipStreamSynchronize(h->stream), "level map copy");
    return FASSMVS_OK;
}

// ---------------------------------------------------------------- plumbing

fassmvs_status fassmvs_device_alloc(fassmvs_handle *h, size_t bytes, void **ptr) {
    if (!h || !ptr) return FASSMVS_EINVAL;
    *ptr = nullptr;
    hipSetDevice(h->cfg.device);
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return fail(h, FASSMVS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return FASSMVS_OK;
}

fassmvs_status fassmvs_device_free(fassmvs_handle *h, void *ptr) {
    if (!h) return FASSMVS_EINVAL;
    if (!ptr) return FASSMVS_OK;
    std::lock_guard<std::mutex> lk(h->mu);
    hipSetDevice(h->cfg.device);
    HIPCHK(h, hipStreamSynchronize(h->stream), "sync before free");
    HIPCHK(h, hipFree(ptr), "hipFree");
    return FASSMVS_OK;
}

fassmvs_status fassmvs_memcpy(fassmvs_handle *h, void *dst, const void *src, size_t bytes, int32_t kind) {
    if (!h || (!dst && bytes) || (!src && bytes)) return FASSMVS_EINVAL;
    if (kind < 0 || kind > 2) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    hipSetDevice(h->cfg.device);
    if (bytes == 0) return FASSMVS_OK;
    const hipMemcpyKind k[3] = {hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice};
    HIPCHK(h, hipStreamSynchronize(h->stream), "sync before copy");
    const bool al16 = ((uintptr_t)dst % 16 == 0) && ((uintptr_t)src % 16 == 0) && bytes % 16 == 0;
    const char *dc = (const char *)dst, *sc = (const char *)src;
    const bool overlap = dc < sc + bytes && sc < dc + bytes;
    if (kind == 2 && al16 && !overlap) {
        hipLaunchKernelGGL(k_copy16, dim3(2048), dim3(256), 0, h->stream, (uint4 *)dst, (const uint4 *)src,
                           bytes / 16);
        HIPCHK(h, hipGetLastError(), "copy launch");
    } else {
        HIPCHK(h, hipMemcpyAsync(dst, src, bytes, k[kind], h->stream), "copy");
    }
    HIPCHK(h, hipStreamSynchronize(h->stream), "copy");
    return FASSMVS_OK;
}

fassmvs_status fassmvs_fill(fassmvs_handle *h, void *dst, uint8_t value, size_t bytes) {
    if (!h || (!dst && bytes)) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    hipSetDevice(h->cfg.device);
    if (bytes == 0) return FASSMVS_OK;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, h->stream, (uint8_t *)dst, value,
                       bytes);
    HIPCHK(h, hipGetLastError(), "fill launch");
    HIPCHK(h, hipStreamSynchronize(h->stream), "fill");
    return FASSMVS_OK;
}

fassmvs_status fassmvs_synchronize(fassmvs_handle *h) {
    if (!h) return FASSMVS_EINVAL;
    std::lock_guard<std::mutex> lk(h->mu);
    hipSetDevice(h->cfg.device);
    HIPCHK(h, hipStreamSynchronize(h->stream), "synchronize");
    return FASSMVS_OK;
}

// ---------------------------------------------------------------- stage entry points

#define STAGE_BEGIN                                  \
    if (!h) return FASSMVS_EINVAL;                   \
    std::lock_guard<std::mutex> lk(h->mu);           \
    if (h->latched) return FASSMVS_EDEVICE;          \
    HIPCHK(h, hipSetDevice(h->cfg.device), "hipSetDevice")

#define STAGE_END                                                     \
    HIPCHK(h, hipStreamSynchronize(h->stream), "stage execution");   \
    return FASSMVS_OK

fassmvs_status fassmvs_stage_pyr_down(fassmvs_handle *h, const uint8_t *src, int32_t w, int32_t hgt, uint8_t *dst) {
    STAGE_BEGIN;
    if (!src || !dst || w < 2 || hgt < 2) return fail(h, FASSMVS_EINVAL, "bad pyramid arguments");
    HIPCHK(h, launch_pyr_down(src, w, hgt, w, dst, h->stream), "pyramid launch");
    STAGE_END;
}

fassmvs_status fassmvs_stage_census(fassmvs_handle *h, const uint8_t *img, int32_t w, int32_t hgt, int32_t cw,
                                    int32_t ch, uint64_t *out) {
    STAGE_BEGIN;
    if (!img || !out || w < 1 || hgt < 1 || !(cw & 1) || !(ch & 1) || cw * ch - 1 > 64)
        return fail(h, FASSMVS_EINVAL, "bad census arguments");
    HIPCHK(h, launch_census(img, w, hgt, cw, ch, out, h->stream), "census launch");
    STAGE_END;
}

fassmvs_status fassmvs_stage_warp(fassmvs_handle *h, const uint8_t *src, int32_t sw, int32_t sh, const double H[9],
                                  int32_t rw, int32_t rh, float *out) {
    STAGE_BEGIN;
    if (!src || !H || !out || sw < 1 || sh < 1 || rw < 1 || rh < 1) return fail(h, FASSMVS_EINVAL, "bad warp arguments");
    if (!finite_all(H, 9)) return fail(h, FASSMVS_EINVAL, "non-finite homography");
    fassmvs_status st = ensure(h, h->params, 9 * 8);
    if (st != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->params.p, H, 72, hipMemcpyHostToDevice, h->stream), "H upload");
    HIPCHK(h, launch_warp(src, sw, sh, (const double *)h->params.p, rw, rh, out, h->stream), "warp launch");
    STAGE_END;
}

namespace {
fassmvs_status stage_cost_any(fassmvs_handle *h, int cost, int32_t w, int32_t hgt, const uint64_t *ct_ref,
                              const uint8_t *ref_img, int32_t n_views, const uint8_t *const *views,
                              const int8_t *view_side, int32_t cw, int32_t ch, int32_t n_fam, const int32_t *G,
                              const int32_t *W, const double *H, const int32_t *offs, const float *warped,
                              uint8_t *S) {
    if ((cost == 0 ? !ct_ref : !ref_img) || !views || !view_side || !G || !W || !H || !S || w < 1 || hgt < 1)
        return fail(h, FASSMVS_EINVAL, "bad cost arguments");
    if (n_views < 1 || n_views > kMaxViews || n_fam < 1 || n_fam > kMaxFam) return fail(h, FASSMVS_EINVAL, "bad counts");
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = w;
    a.h = hgt;
    a.cw = cw;
    a.ch = ch;
    a.cost = cost;
    a.n_views = n_views;
    for (int k = 0; k < n_views; ++k) {
        if (!views[k] && !warped) return fail(h, FASSMVS_EINVAL, "null view");
        if (view_side[k] != -1 && view_side[k] != 1) return fail(h, FASSMVS_EINVAL, "view_side must be -1 or +1");
        a.views[k] = views[k];
        a.side[k] = view_side[k];
        if (view_side[k] < 0) a.nL++; else a.nR++;
    }
    a.m = std::max(a.nL, a.nR);
    if (cost == 0 && a.m * (cw * ch - 1) > 255) return fail(h, FASSMVS_EUNSUPPORTED, "cost exceeds 8 bits");
    a.n_fam = n_fam;
    for (int f = 0; f < n_fam; ++f) {
        if (W[f] < 1 || W[f] > G[f] || (!offs && W[f] != G[f])) return fail(h, FASSMVS_EINVAL, "bad family sizes");
        a.G[f] = G[f];
        a.W[f] = W[f];
        a.foff[f] = a.D;
        a.goff[f] = a.sumG;
        a.D += W[f];
        a.sumG += G[f];
    }
    if (a.D > kMaxLabels) return fail(h, FASSMVS_EUNSUPPORTED, "too many labels");
    fassmvs_status st = ensure(h, h->params, (size_t)n_views * a.sumG * 72);
    if (st != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->params.p, H, (size_t)n_views * a.sumG * 72, hipMemcpyHostToDevice, h->stream),
           "H upload");
    HIPCHK(h, hipStreamSynchronize(h->stream), "H upload");
    a.H = (const double *)h->params.p;
    a.ct_ref = ct_ref;
    a.ref = ref_img;
    a.offs = offs;
    a.warped = warped;
    a.S = S;
    a.rows_per_thread = sweep_rows();
    hipError_t e = launch_sweep(a, h->stream);
    if (e == hipErrorInvalidValue) return fail(h, FASSMVS_EUNSUPPORTED, "matching window not built");
    HIPCHK(h, e, "sweep launch");
    return FASSMVS_OK;
}
}  // namespace

fassmvs_status fassmvs_stage_cost(fassmvs_handle *h, int32_t w, int32_t hgt, const uint64_t *ct_ref, int32_t n_views,
                                  const uint8_t *const *views, const int8_t *view_side, int32_t cw, int32_t ch,
                                  int32_t n_fam, const int32_t *G, const int32_t *W, const double *H,
                                  const int32_t *offs, const float *warped, uint8_t *S) {
    STAGE_BEGIN;
    fassmvs_status st = stage_cost_any(h, 0, w, hgt, ct_ref, nullptr, n_views, views, view_side, cw, ch, n_fam, G, W,
                                       H, offs, warped, S);
    if (st != FASSMVS_OK) return st;
    STAGE_END;
}

fassmvs_status fassmvs_stage_cost_ncc(fassmvs_handle *h, int32_t w, int32_t hgt, const uint8_t *ref_img,
                                      int32_t n_views, const uint8_t *const *views, const int8_t *view_side,
                                      int32_t cw, int32_t ch, int32_t n_fam, const int32_t *G, const int32_t *W,
                                      const double *H, const int32_t *offs, const float *warped, uint8_t *S) {
    STAGE_BEGIN;
    if (cw != ch) return fail(h, FASSMVS_EUNSUPPORTED, "NCC windows are square");
    fassmvs_status st = stage_cost_any(h, 1, w, hgt, nullptr, ref_img, n_views, views, view_side, cw, ch, n_fam, G,
                                       W, H, offs, warped, S);
    if (st != FASSMVS_OK) return st;
    STAGE_END;
}

fassmvs_status fassmvs_filter_dog(fassmvs_handle *h, const uint8_t *img, int32_t w, int32_t hgt, float *depth,
                                  float *normal, float *confidence, uint8_t *mask_out) {
    STAGE_BEGIN;
    if (!img || w < 1 || hgt < 1 || (size_t)w * hgt > ((size_t)1 << 28)) return fail(h, FASSMVS_EINVAL, "bad DoG arguments");
    const size_t N = (size_t)w * hgt;
    fassmvs_status st;
    if ((st = ensure(h, h->post_tmp, N * 8)) || (st = ensure(h, h->post_m0, N)) || (st = ensure(h, h->post_m1, N)))
        return st;
    PostArgs pa = dog_args();
    HIPCHK(h, launch_dog_mask(img, w, hgt, pa, (double *)h->post_tmp.p, (uint8_t *)h->post_m0.p,
                              (uint8_t *)h->post_m1.p, h->stream),
           "dog filter");
    HIPCHK(h, launch_apply_keep((const uint8_t *)h->post_m1.p, N, depth, normal, confidence, h->stream), "dog apply");
    if (mask_out)
        HIPCHK(h, hipMemcpyAsync(mask_out, h->post_m1.p, N, hipMemcpyDeviceToDevice, h->stream), "mask copy");
    STAGE_END;
}

fassmvs_status fassmvs_filter_dog_noalloc(fassmvs_handle *h, const uint8_t *img, int32_t w, int32_t hgt,
                                          float *depth, float *normal, float *confidence, uint8_t *mask_out) {
    STAGE_BEGIN;
    if (!img || w < 1 || hgt < 1) return fail(h, FASSMVS_EINVAL, "bad DoG arguments");
    const size_t N = (size_t)w * hgt;
    if (N > kNoAllocMaxPixels)
        return fail(h, FASSMVS_EINVAL, "image exceeds the allocation-free filter's maximum of 4194304 pixels");
    // the address looked up when the handle was created on this device;
    // never the array's host-side name
    uint8_t *base = (uint8_t *)scratch_address(h->cfg.device);
    if (!base) return fail(h, FASSMVS_EDEVICE, "scratch address missing");
    double *tmp = (double *)base;
    uint8_t *m0 = base + N * 8, *m1 = m0 + N;
    PostArgs pa = dog_args();
    HIPCHK(h, launch_dog_mask(img, w, hgt, pa, tmp, m0, m1, h->stream), "dog filter");
    HIPCHK(h, launch_apply_keep(m1, N, depth, normal, confidence, h->stream), "dog apply");
    if (mask_out) HIPCHK(h, hipMemcpyAsync(mask_out, m1, N, hipMemcpyDeviceToDevice, h->stream), "mask copy");
    STAGE_END;
}

fassmvs_status fassmvs_filter_geometric(fassmvs_handle *h, int32_t w, int32_t hgt, const double K[9], float *depth,
                                        float *normal, float *confidence, int32_t n_nb, const float *const *depth_nb,
                                        const double *R_rel, const double *t_rel, double eta_r, int32_t eta_h,
                                        int32_t *hits_out, uint8_t *keep_out) {
    STAGE_BEGIN;
    if (!K || !depth || w < 1 || hgt < 1 || (size_t)w * hgt > ((size_t)1 << 28) || n_nb < 1 || n_nb > kMaxViews ||
        !depth_nb || !R_rel || !t_rel || !(eta_r > 0.0) || eta_h < 0)
        return fail(h, FASSMVS_EINVAL, "bad geometric filter arguments");
    GeoArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = w;
    a.h = hgt;
    a.depth_ref = depth;
    a.n_nb = n_nb;
    for (int k = 0; k < n_nb; ++k) {
        if (!depth_nb[k]) return fail(h, FASSMVS_EINVAL, "null neighbour map");
        if (!finite_all(R_rel + 9 * k, 9) || !finite_all(t_rel + 3 * k, 3)) return fail(h, FASSMVS_EINVAL, "bad pose");
        a.depth_nb[k] = depth_nb[k];
        std::memcpy(a.R[k], R_rel + 9 * k, sizeof(a.R[k]));
        std::memcpy(a.t[k], t_rel + 3 * k, sizeof(a.t[k]));
    }
    double Kl[9];
    if (!kinv_level(K, 0, Kl, a.Kinv)) return fail(h, FASSMVS_EINVAL, "K must have positive focal lengths");
    std::memcpy(a.K, K, sizeof(a.K));
    a.eta_r = eta_r;
    a.eta_h = eta_h;
    const size_t N = (size_t)w * hgt;
    fassmvs_status st;
    if ((st = ensure(h, h->post_m0, N))) return st;
    uint8_t *keep = (uint8_t *)h->post_m0.p;
    HIPCHK(h, launch_geo(a, hits_out, keep, h->stream), "geometric filter");
    HIPCHK(h, launch_apply_keep(keep, N, depth, normal, confidence, h->stream), "geometric apply");
    if (keep_out) HIPCHK(h, hipMemcpyAsync(keep_out, keep, N, hipMemcpyDeviceToDevice, h->stream), "keep copy");
    STAGE_END;
}

fassmvs_status fassmvs_stage_sgm(fassmvs_handle *h, int32_t w, int32_t hgt, int32_t n_fam, const int32_t *W,
                                 const uint8_t *S, const int32_t *offs, const int8_t *dI, const uint8_t *ref,
                                 int32_t p1, const int32_t *lut, int32_t n_paths, uint16_t *Lr, uint16_t *Sbar,
                                 uint16_t *wta, uint16_t *c3) {
    STAGE_BEGIN;
    if (!W || !S || !ref || !lut || w < 1 || hgt < 1 || n_fam < 1 || n_fam > kMaxFam)
        return fail(h, FASSMVS_EINVAL, "bad sgm arguments");
    if (n_paths != 4 && n_paths != 8) return fail(h, FASSMVS_EINVAL, "n_paths must be 4 or 8");
    if ((wta == nullptr) != (c3 == nullptr)) return fail(h, FASSMVS_EINVAL, "wta and c3 go together");
    LevelPlan L;
    L.w = w;
    L.h = hgt;
    L.F = n_fam;
    L.D = 0;
    for (int f = 0; f < n_fam; ++f) {
        if (W[f] < 1) return fail(h, FASSMVS_EINVAL, "bad window");
        L.W[f] = W[f];
        L.foff[f] = L.D;
        L.D += W[f];
    }
    if (L.D > kMaxLabels) return fail(h, FASSMVS_EUNSUPPORTED, "too many labels");
    for (int i = 0; i < 256; ++i)
        if (lut[i] < p1) return fail(h, FASSMVS_EINVAL, "P2 must be >= P1");
    const size_t ND = (size_t)w * hgt * L.D;
    uint16_t *bufs[8];
    fassmvs_status st;
    if (Lr) {
        for (int d = 0; d < n_paths; ++d) bufs[d] = Lr + (size_t)d * ND;
    } else {
        for (int d = 0; d < n_paths; ++d) {
            if ((st = ensure(h, h->sgmbuf[d], ND * 2)) != FASSMVS_OK) return st;
            bufs[d] = (uint16_t *)h->sgmbuf[d].p;
        }
    }
    st = run_sgm(h, L, S, offs, dI, ref, p1, lut, n_paths, bufs, Sbar, wta, c3);
    if (st != FASSMVS_OK) return st;
    STAGE_END;
}

fassmvs_status fassmvs_stage_sgm_pg(fassmvs_handle *h, int32_t w, int32_t hgt, int32_t n_fam, const int32_t *W,
                                    const int32_t *G, const uint8_t *S, const int32_t *offs, const uint8_t *ref,
                                    int32_t p1, const int32_t *lut, int32_t n_paths, const double *fam_delta,
                                    const double *fam_n, const double *Kinv, const double *step, uint16_t *Lr,
                                    uint16_t *Sbar, uint16_t *wta, uint16_t *c3) {
    STAGE_BEGIN;
    if (!W || !G || !S || !ref || !lut || !fam_delta || !fam_n || !Kinv || !step || w < 1 || hgt < 1 || n_fam < 1 ||
        n_fam > kMaxFam)
        return fail(h, FASSMVS_EINVAL, "bad sgm arguments");
    if (n_paths != 4 && n_paths != 8) return fail(h, FASSMVS_EINVAL, "n_paths must be 4 or 8");
    if ((wta == nullptr) != (c3 == nullptr)) return fail(h, FASSMVS_EINVAL, "wta and c3 go together");
    LevelPlan L;
    L.w = w;
    L.h = hgt;
    L.F = n_fam;
    L.D = 0;
    L.sumG = 0;
    for (int f = 0; f < n_fam; ++f) {
        if (W[f] < 1 || W[f] > G[f] || (!offs && W[f] != G[f])) return fail(h, FASSMVS_EINVAL, "bad family sizes");
        L.W[f] = W[f];
        L.G[f] = G[f];
        L.foff[f] = L.D;
        L.goff[f] = L.sumG;
        L.step[f] = step[f];
        L.D += W[f];
        L.sumG += G[f];
    }
    std::memcpy(L.Kinv, Kinv, 72);
    if (L.D > kMaxLabels) return fail(h, FASSMVS_EUNSUPPORTED, "too many labels");
    for (int i = 0; i < 256; ++i)
        if (lut[i] < p1) return fail(h, FASSMVS_EINVAL, "P2 must be >= P1");
    fassmvs_status st = ensure(h, h->params, (size_t)L.sumG * 8);
    if (st != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->params.p, fam_delta, (size_t)L.sumG * 8, hipMemcpyHostToDevice, h->stream), "delta");
    double fn[kMaxFam][3];
    for (int f = 0; f < n_fam; ++f)
        for (int i = 0; i < 3; ++i) fn[f][i] = fam_n[3 * f + i];
    PgGeom pgg{(const double *)h->params.p, fn};
    const size_t ND = (size_t)w * hgt * L.D;
    uint16_t *bufs[8];
    if (Lr) {
        for (int d = 0; d < n_paths; ++d) bufs[d] = Lr + (size_t)d * ND;
    } else {
        for (int d = 0; d < n_paths; ++d) {
            if ((st = ensure(h, h->sgmbuf[d], ND * 2)) != FASSMVS_OK) return st;
            bufs[d] = (uint16_t *)h->sgmbuf[d].p;
        }
    }
    st = run_sgm(h, L, S, offs, nullptr, ref, p1, lut, n_paths, bufs, Sbar, wta, c3, &pgg);
    if (st != FASSMVS_OK) return st;
    STAGE_END;
}

fassmvs_status fassmvs_stage_refine(fassmvs_handle *h, int32_t w, int32_t hgt, int32_t n_fam, const int32_t *W,
                                    const int32_t *G, const int32_t *offs, const uint16_t *wta, const uint16_t *c3,
                                    const double *fam_n, const double *fam_delta, const double *Kinv, int32_t *label,
                                    int32_t *fam, float *depth) {
    STAGE_BEGIN;
    if (!W || !G || !wta || !c3 || !fam_n || !fam_delta || !Kinv || !label || !fam || !depth || n_fam < 1 ||
        n_fam > kMaxFam)
        return fail(h, FASSMVS_EINVAL, "bad refine arguments");
    RefineArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = w;
    a.h = hgt;
    a.n_fam = n_fam;
    int D = 0, sumG = 0;
    for (int f = 0; f < n_fam; ++f) {
        a.W[f] = W[f];
        a.G[f] = G[f];
        a.foff[f] = D;
        a.goff[f] = sumG;
        D += W[f];
        sumG += G[f];
        for (int i = 0; i < 3; ++i) a.fam_n[f][i] = fam_n[f * 3 + i];
    }
    std::memcpy(a.Kinv, Kinv, 72);
    fassmvs_status st = ensure(h, h->params, (size_t)sumG * 8);
    if (st != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->params.p, fam_delta, (size_t)sumG * 8, hipMemcpyHostToDevice, h->stream), "delta upload");
    HIPCHK(h, hipStreamSynchronize(h->stream), "delta upload");
    a.delta = (const double *)h->params.p;
    a.offs = offs;
    a.wta = wta;
    a.c3 = c3;
    a.label = label;
    a.fam = fam;
    a.depth = depth;
    HIPCHK(h, launch_refine(a, h->stream), "refine launch");
    STAGE_END;
}

fassmvs_status fassmvs_stage_median(fassmvs_handle *h, const float *in, int32_t w, int32_t hgt, float *out) {
    STAGE_BEGIN;
    if (!in || !out || w < 1 || hgt < 1) return fail(h, FASSMVS_EINVAL, "bad median arguments");
    HIPCHK(h, launch_median5(in, w, hgt, out, h->stream), "median launch");
    STAGE_END;
}

fassmvs_status fassmvs_stage_normals(fassmvs_handle *h, const float *depth, const uint8_t *img, int32_t w, int32_t hgt,
                                     const double *Kinv, int32_t radius, double beta, const int32_t *label,
                                     const int32_t *fam, int32_t n_fam, const double *fam_n, double rho_deg,
                                     float *nraw, float *normal, float *conf) {
    STAGE_BEGIN;
    if (!depth || !img || !Kinv || !label || !fam || !fam_n || !normal || !conf || n_fam < 1 || n_fam > kMaxFam ||
        radius < 1 || radius > 4)
        return fail(h, FASSMVS_EINVAL, "bad normals arguments");
    NormalArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = w;
    a.h = hgt;
    fassmvs_status wst = weight_table(h, radius, beta);
    if (wst != FASSMVS_OK) return wst;
    a.radius = radius;
    a.beta = beta;
    a.wtab = (const double *)h->wtab.p;
    a.cos_rho = std::cos(rho_deg * 3.14159265358979323846 / 180.0);
    std::memcpy(a.Kinv, Kinv, 72);
    a.n_fam = n_fam;
    for (int f = 0; f < n_fam; ++f)
        for (int i = 0; i < 3; ++i) a.fam_n[f][i] = fam_n[f * 3 + i];
    a.depth = depth;
    a.img = img;
    a.label = label;
    a.fam = fam;
    DevBuf tmp;
    float *nr = nraw;
    if (!nr) {
        HIPCHK(h, hipMalloc(&tmp.p, (size_t)w * hgt * 12), "temporary normals");
        nr = (float *)tmp.p;
    }
    a.nraw = nr;
    a.normal = normal;
    a.conf = conf;
    hipError_t e = launch_normals(a, h->stream);
    hipError_t e2 = hipStreamSynchronize(h->stream);
    if (tmp.p) hipFree(tmp.p);
    HIPCHK(h, e, "normals launch");
    HIPCHK(h, e2, "normals execution");
    return FASSMVS_OK;
}

fassmvs_status fassmvs_stage_seed(fassmvs_handle *h, const float *depth_c, const float *normal_c, int32_t cw,
                                  int32_t ch, int32_t fw, int32_t fh, const double *Kinv, int32_t n_fam,
                                  const double *fam_n, const double *fam_delta, const int32_t *G, const int32_t *W,
                                  float *dbar, float *nbar, int32_t *offs, int8_t *dI) {
    STAGE_BEGIN;
    if (!depth_c || !normal_c || !Kinv || !fam_n || !fam_delta || !G || !W || !dbar || !nbar || !offs ||
        n_fam < 1 || n_fam > kMaxFam || cw < 1 || ch < 1 || fw < 1 || fh < 1)
        return fail(h, FASSMVS_EINVAL, "bad seed arguments");
    SeedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.cw = cw;
    a.ch = ch;
    a.fw = fw;
    a.fh = fh;
    a.n_fam = n_fam;
    std::memcpy(a.Kinv, Kinv, 72);
    int sumG = 0;
    for (int f = 0; f < n_fam; ++f) {
        if (G[f] < 2 || W[f] < 1 || W[f] > G[f]) return fail(h, FASSMVS_EINVAL, "bad family sizes");
        for (int i = 0; i < 3; ++i) a.fam_n[f][i] = fam_n[f * 3 + i];
        a.goff[f] = sumG;
        a.G[f] = G[f];
        a.W[f] = W[f];
        sumG += G[f];
    }
    std::vector<double> inv(sumG);
    for (int j = 0; j < sumG; ++j) {
        if (!(fam_delta[j] > 0.0) || !std::isfinite(fam_delta[j])) return fail(h, FASSMVS_EINVAL, "bad plane list");
        inv[j] = 1.0 / fam_delta[j];
    }
    for (int f = 0; f < n_fam; ++f)
        for (int j = 1; j < G[f]; ++j)
            if (!(inv[a.goff[f] + j] < inv[a.goff[f] + j - 1]))
                return fail(h, FASSMVS_EINVAL, "plane lists must increase strictly");
    fassmvs_status st = ensure(h, h->params, (size_t)sumG * 8);
    if (st != FASSMVS_OK) return st;
    HIPCHK(h, hipMemcpyAsync(h->params.p, inv.data(), (size_t)sumG * 8, hipMemcpyHostToDevice, h->stream),
           "list upload");
    HIPCHK(h, hipStreamSynchronize(h->stream), "list upload");
    a.inv = (const double *)h->params.p;
    a.depth_c = depth_c;
    a.normal_c = normal_c;
    a.dbar = dbar;
    a.nbar = nbar;
    a.offs = offs;
    a.dI = dI;
    HIPCHK(h, launch_seed(a, h->stream), "seed launch");
    STAGE_END;
}

}  // extern "C"
