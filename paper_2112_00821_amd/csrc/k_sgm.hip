// Semi-global aggregation on gfx950 (Eq. sgm-path / sgm-smooth-fp /
// sgm-smooth-sn / sgm-aggr / sgm-wta of the paper, adaptive P2 of
// Eq. p2-grad).
//
// One wavefront walks one path; label i of the pixel sits in lane i % 64 of
// register i / 64.  The predecessor's path costs live in a per-wave LDS
// buffer with three guard entries on each side of every family segment, so
// the zero-cost transition shifted by the window offsets and the
// surface-normal offset (a per-pixel, per-family shift) is a plain indexed
// LDS read.  The predecessor minimum comes from a DPP reduction.
//
// All directions run in one launch, each writing its own uint16 buffer (no
// read-modify-write of a shared aggregate, so every path of every direction
// proceeds concurrently); a streaming kernel then adds the buffers and takes
// the winner-takes-all argmin, so the aggregate volume is never written.
#include "dev_common.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace fmvs {

namespace {
constexpr uint32_t INF = 0x3FFFFFFFu;
constexpr int WAVES = 4;
constexpr int GUARD = 3;
constexpr int LBUF = kMaxLabels + 2 * GUARD * kMaxFam;

struct PathGeom {
    int sx, sy, dx, dy, len;
};

__device__ __forceinline__ PathGeom path_geom(int dir, int pi, int w, int h) {
    PathGeom g;
    g.dx = dir_dx(dir);
    g.dy = dir_dy(dir);
    if (g.dy == 0) {
        g.sx = g.dx > 0 ? 0 : w - 1;
        g.sy = pi;
        g.len = w;
    } else if (g.dx == 0) {
        g.sx = pi;
        g.sy = g.dy > 0 ? 0 : h - 1;
        g.len = h;
    } else {
        if (pi < w) {
            g.sx = pi;
            g.sy = g.dy > 0 ? 0 : h - 1;
        } else {
            int j = pi - w;
            g.sx = g.dx > 0 ? 0 : w - 1;
            g.sy = g.dy > 0 ? j + 1 : h - 2 - j;
        }
        int lx = g.dx > 0 ? w - g.sx : g.sx + 1;
        int ly = g.dy > 0 ? h - g.sy : g.sy + 1;
        g.len = lx < ly ? lx : ly;
    }
    return g;
}
}  // namespace

int sgm_paths(int dir, int w, int h) {
    int dx = dir_dx(dir), dy = dir_dy(dir);
    if (dy == 0) return h;
    if (dx == 0) return w;
    return w + h - 1;
}

// Path costs of one direction, written to that direction's buffer.  Loads
// run ahead of the recursion: a ring of PF steps holds each lane's cost
// bytes, and the per-step uniform values (reference intensity, window
// offsets, surface-normal offsets) of 64 steps are fetched by one vector
// load per quantity (lane j holds step t0 + j) and read back with readlane.
template <int K, bool WIN, bool SN>
__global__ __launch_bounds__(64 * WAVES) void k_sgm(const SgmArgs a) {
    constexpr int PF = 8;
    __shared__ uint32_t lbuf[WAVES][2][LBUF];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int path = blockIdx.x * WAVES + wid;
    if (path >= a.path_begin[a.n_dirs]) return;
    int slot = 0;
    while (path >= a.path_begin[slot + 1]) ++slot;
    const int dir = a.dirs[slot];
    const PathGeom pg = path_geom(dir, path - a.path_begin[slot], a.w, a.h);
    const size_t N = (size_t)a.w * a.h;
    const int D = a.D;
    const int F = a.n_fam;
    const long pstride = (long)pg.dy * a.w + pg.dx;
    const long p0 = (long)pg.sy * a.w + pg.sx;
    const int len = pg.len;

    int fam[K], li[K], wf[K], seg[K];
    bool lv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = k * 64 + lane;
        lv[k] = i < D;
        int f = 0;
        while (f + 1 < F && i >= a.foff[f + 1]) ++f;
        fam[k] = f;
        li[k] = i - a.foff[f];
        wf[k] = a.W[f];
        int sb = GUARD;
        for (int ff = 0; ff < f; ++ff) sb += a.W[ff] + 2 * GUARD;
        seg[k] = sb;
    }
    uint32_t *buf0 = lbuf[wid][0];
    uint32_t *buf1 = lbuf[wid][1];
    for (int i = lane; i < LBUF; i += 64) {
        buf0[i] = INF;
        buf1[i] = INF;
    }
    __builtin_amdgcn_wave_barrier();

    const uint8_t *__restrict__ S = a.S;
    uint16_t *__restrict__ out = a.out[slot];

    // per-step uniform values, 64 steps per chunk
    auto load_chunk = [&](int t0, int &ref_v, int (&off_v)[kMaxFam], int (&di_v)[kMaxFam]) {
        int t = t0 + lane;
        long p = p0 + (long)(t < len ? t : len - 1) * pstride;
        ref_v = a.ref[p];
#pragma unroll
        for (int f = 0; f < kMaxFam; ++f) {
            off_v[f] = (WIN && f < F) ? a.offs[(size_t)f * N + p] : 0;
            di_v[f] = (SN && f < F) ? (int)a.dI[((size_t)dir * N + p) * F + f] : 0;
        }
    };
    int c_ref, n_ref;
    int c_off[kMaxFam], n_off[kMaxFam], c_di[kMaxFam], n_di[kMaxFam];
    load_chunk(0, c_ref, c_off, c_di);
    if (len > 64) load_chunk(64, n_ref, n_off, n_di);

    // ring of cost bytes, PF steps ahead
    uint32_t ring[PF][K];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        long p = p0 + (long)(u < len ? u : len - 1) * pstride;
#pragma unroll
        for (int k = 0; k < K; ++k) ring[u][k] = lv[k] ? S[(size_t)p * D + k * 64 + lane] : 0u;
    }

    uint32_t L[K];
    uint32_t Mq = 0;
    int Iq = 0;
    int oq[kMaxFam];
#pragma unroll
    for (int f = 0; f < kMaxFam; ++f) oq[f] = 0;

    for (int t0 = 0; t0 < len; t0 += PF) {
        if (t0 > 0 && (t0 & 63) == 0) {
            c_ref = n_ref;
#pragma unroll
            for (int f = 0; f < kMaxFam; ++f) {
                c_off[f] = n_off[f];
                c_di[f] = n_di[f];
            }
            if (t0 + 64 < len) load_chunk(t0 + 64, n_ref, n_off, n_di);
        }
        const int lb = t0 & 63;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = t0 + u;
            if (t >= len) break;
            const long p = p0 + (long)t * pstride;
            uint32_t sv[K];
#pragma unroll
            for (int k = 0; k < K; ++k) sv[k] = ring[u][k];
            if (t + PF < len) {
                const long pn = p + (long)PF * pstride;
#pragma unroll
                for (int k = 0; k < K; ++k) ring[u][k] = lv[k] ? S[(size_t)pn * D + k * 64 + lane] : 0u;
            }
            const int Ip = __builtin_amdgcn_readlane(c_ref, lb + u);
            int op[kMaxFam];
#pragma unroll
            for (int f = 0; f < kMaxFam; ++f) op[f] = WIN ? __builtin_amdgcn_readlane(c_off[f], lb + u) : 0;
            uint32_t *cur = (t & 1) ? buf1 : buf0;
            const uint32_t *prev = (t & 1) ? buf0 : buf1;
            if (t == 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) L[k] = sv[k];
            } else {
                int dI = Ip - Iq;
                const uint32_t P2 = (uint32_t)a.lut[dI < 0 ? -dI : dI];
                const uint32_t P1 = (uint32_t)a.p1;
                int sh[kMaxFam];
#pragma unroll
                for (int f = 0; f < kMaxFam; ++f) {
                    int v = WIN ? op[f] - oq[f] : 0;
                    if (SN) v += __builtin_amdgcn_readlane(c_di[f], lb + u);
                    sh[f] = v;
                }
                const uint32_t floor2 = Mq + P2;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    int sft = sh[0];
#pragma unroll
                    for (int f = 1; f < kMaxFam; ++f)
                        if (fam[k] == f) sft = sh[f];
                    int j = li[k] + sft;
                    j = j < -2 ? -2 : (j > wf[k] + 1 ? wf[k] + 1 : j);
                    const uint32_t *q = prev + seg[k] + j;
                    uint32_t c0 = q[0];
                    uint32_t cm = q[-1];
                    uint32_t cp = q[1];
                    uint32_t c1 = (cm < cp ? cm : cp) + P1;
                    uint32_t best = c0 < c1 ? c0 : c1;
                    best = best < floor2 ? best : floor2;
                    L[k] = sv[k] + best - Mq;
                }
            }
            uint32_t m = INF;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (lv[k]) {
                    cur[seg[k] + li[k]] = L[k];
                    out[(size_t)p * D + k * 64 + lane] = (uint16_t)L[k];
                }
                uint32_t v = lv[k] ? L[k] : INF;
                m = v < m ? v : m;
            }
            __builtin_amdgcn_wave_barrier();
            Mq = wave_min_u32(m);
            Iq = Ip;
#pragma unroll
            for (int f = 0; f < kMaxFam; ++f) oq[f] = op[f];
        }
    }
}

// Winner-takes-all over the summed path costs (Eq. sgm-aggr, sgm-wta): one
// wavefront per pixel, labels across lanes; the packed (cost << 16 | label)
// minimum gives the smallest label on ties.  Also records the aggregate at
// the winner's two neighbours inside its family window for the refinement.
template <int K>
__global__ __launch_bounds__(256) void k_wta(const SgmArgs a) {
    const int lane = threadIdx.x & 63;
    const size_t N = (size_t)a.w * a.h;
    const int D = a.D;
    const size_t waves = (size_t)gridDim.x * 4;
    for (size_t p = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < N; p += waves) {
        uint32_t tot[K];
        uint32_t key = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = k * 64 + lane;
            uint32_t s = 0;
            if (i < D) {
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    if (b < a.n_in) s += a.in[b][p * D + i];
                uint32_t kk = (s << 16) | (uint32_t)i;
                key = kk < key ? kk : key;
            }
            tot[k] = s;
        }
        key = wave_min_u32(key);
        const int best = (int)(key & 0xFFFFu);
        int f = 0;
        while (f + 1 < a.n_fam && best >= a.foff[f + 1]) ++f;
        const int l = best - a.foff[f];
        uint32_t cm = 0xFFFF, cp = 0xFFFF;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = k * 64 + lane;
            if (l >= 1 && i == best - 1) cm = tot[k];
            if (l + 1 < a.W[f] && i == best + 1) cp = tot[k];
        }
        cm = wave_min_u32(cm);
        cp = wave_min_u32(cp);
        if (lane == 0) {
            a.wta[p] = (uint16_t)best;
            a.c3[3 * p] = (uint16_t)cm;
            a.c3[3 * p + 1] = (uint16_t)(key >> 16);
            a.c3[3 * p + 2] = (uint16_t)cp;
        }
    }
}

template <int K>
static void launch_k(const SgmArgs &a, bool win, bool sn, dim3 grid, hipStream_t s) {
    if (a.final_mode) {
        unsigned blocks = (unsigned)std::min<size_t>(((size_t)a.w * a.h + 3) / 4, 65536);
        hipLaunchKernelGGL((k_wta<K>), dim3(blocks), dim3(256), 0, s, a);
        return;
    }
#define FMVS_SGM(W_, S_)                                                             \
    if (win == W_ && sn == S_) {                                                     \
        hipLaunchKernelGGL((k_sgm<K, W_, S_>), grid, dim3(64 * WAVES), 0, s, a);     \
        return;                                                                      \
    }
    FMVS_SGM(false, false)
    FMVS_SGM(true, false)
    FMVS_SGM(false, true)
    FMVS_SGM(true, true)
#undef FMVS_SGM
}

hipError_t launch_sgm(const SgmArgs &a0, hipStream_t s) {
    SgmArgs a = a0;
    a.path_begin[0] = 0;
    for (int i = 0; i < a.n_dirs; ++i) a.path_begin[i + 1] = a.path_begin[i] + sgm_paths(a.dirs[i], a.w, a.h);
    for (int i = a.n_dirs + 1; i < 9; ++i) a.path_begin[i] = a.path_begin[a.n_dirs];
    int paths = a.path_begin[a.n_dirs];
    if (paths == 0 && !a.final_mode) return hipSuccess;
    dim3 grid((unsigned)((paths + WAVES - 1) / WAVES));
    bool win = a.offs != nullptr, sn = a.dI != nullptr;
    int K = (a.D + 63) / 64;
    switch (K) {
        case 1: launch_k<1>(a, win, sn, grid, s); break;
        case 2: launch_k<2>(a, win, sn, grid, s); break;
        case 3: launch_k<3>(a, win, sn, grid, s); break;
        case 4: launch_k<4>(a, win, sn, grid, s); break;
        case 5: launch_k<5>(a, win, sn, grid, s); break;
        case 6: launch_k<6>(a, win, sn, grid, s); break;
        case 7: launch_k<7>(a, win, sn, grid, s); break;
        case 8: launch_k<8>(a, win, sn, grid, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fmvs
