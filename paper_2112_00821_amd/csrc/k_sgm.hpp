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
#pragma once
#include "dev_common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cstdlib>

namespace fmvs {

namespace {
constexpr uint32_t INF = 0x3FFFFFFFu;
constexpr int WAVES = 4;
// cache-policy bit of the buffer intrinsics for non-temporal (streaming)
// accesses on gfx950
constexpr int kNonTemporal = 2;
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
            // longest paths first within each direction (the dispatcher
            // starts workgroups in index order, so short paths fill the tail)
            g.sx = g.dx > 0 ? pi : w - 1 - pi;
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


// Path costs of one direction, written to that direction's buffer.  Loads
// run ahead of the recursion: a ring of PF steps holds each lane's cost
// bytes, and the per-step uniform values (the P2 penalty of the step's
// intensity change, window offsets, surface-normal offsets) of 64 steps are
// fetched by one vector load per quantity (lane j holds step t0 + j) and
// read back with readlane.
// NF bounds the plane families (1, or up to the maximum), which sizes the
// per-family registers.
template <int K, int NF, bool WIN, bool SN, bool PG>
__global__ __launch_bounds__(64 * WAVES) void k_sgm(const SgmArgs a) {
    constexpr int PF = 8;
    __shared__ uint32_t lbuf[WAVES][2][LBUF];
    __shared__ double pdelta[PG ? kMaxPgPlanes : 1];
    if (PG) {
        for (int i = threadIdx.x; i < a.sumG; i += 64 * WAVES) pdelta[i] = a.delta[i];
        __syncthreads();
    }
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
    const int F = NF == 1 ? 1 : a.n_fam;
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
    auto load_chunk = [&](int t0, int &ref_v, int (&off_v)[NF], int (&di_v)[NF]) {
        // ref_v: the penalty P2 of step t = t0 + lane, from the intensity
        // step between its pixel and the previous one on the path
        const int t = t0 + lane < len ? t0 + lane : len - 1;
        const long p = p0 + (long)t * pstride;
        const long pp = p0 + (long)(t > 0 ? t - 1 : 0) * pstride;
        const int di = (int)a.ref[p] - (int)a.ref[pp];
        ref_v = a.lut[di < 0 ? -di : di];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            off_v[f] = (WIN && f < F) ? a.offs[(size_t)f * N + p] : 0;
            di_v[f] = (SN && f < F) ? (int)a.dI[((size_t)dir * N + p) * F + f] : 0;
        }
    };
    int c_ref, n_ref;
    int c_off[NF], n_off[NF], c_di[NF], n_di[NF];
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
    int oq[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) oq[f] = 0;
    // path-gradient state: depths of the last two minimum-cost points
    double dq1 = 0.0, dq2 = 0.0;

    for (int t0 = 0; t0 < len; t0 += PF) {
        if (t0 > 0 && (t0 & 63) == 0) {
            c_ref = n_ref;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                c_off[f] = n_off[f];
                c_di[f] = n_di[f];
            }
            if (t0 + 64 < len) load_chunk(t0 + 64, n_ref, n_off, n_di);
        }
        const int lb = t0 & 63;   // PF divides 64
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
            const uint32_t P2 = (uint32_t)__builtin_amdgcn_readlane(c_ref, lb + u);
            int op[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) op[f] = WIN ? __builtin_amdgcn_readlane(c_off[f], lb + u) : 0;
            uint32_t *cur = (t & 1) ? buf1 : buf0;
            const uint32_t *prev = (t & 1) ? buf0 : buf1;
            if (t == 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) L[k] = sv[k];
            } else {
                const uint32_t P1 = (uint32_t)a.p1;
                int sh[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    int v = WIN ? op[f] - oq[f] : 0;
                    if (SN) v += __builtin_amdgcn_readlane(c_di[f], lb + u);
                    sh[f] = v;
                }
                if (PG && t >= 2 && dq1 > 0.0 && dq2 > 0.0) {
                    // extrapolated inverse depth of the path's minimum-cost
                    // points, as a plane-index jump per family
                    const int px = pg.sx + t * pg.dx, py = pg.sy + t * pg.dy;
                    double rp[3], rq[3];
                    ray_of(a.Kinv, px + 0.5, py + 0.5, rp);
                    ray_of(a.Kinv, (px - pg.dx) + 0.5, (py - pg.dy) + 0.5, rq);
                    const double inv = 2.0 / dq1 - 1.0 / dq2;
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        if (f >= F) break;
                        const double *n = a.fam_n[f];
                        const double cp = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
                        const double cq = -(n[0] * rq[0] + n[1] * rq[1] + n[2] * rq[2]);
                        if (!(cp > 0.0) || !(cq > 0.0)) continue;
                        const double ip = inv / cp;
                        const double iq = 1.0 / (dq1 * cq);
                        double v = (ip - iq) / a.step[f];
                        v = fmin(fmax(v, -7.0), 7.0);
                        sh[f] += (int)round(v);
                    }
                }
                const uint32_t floor2 = Mq + P2;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    int sft = sh[0];
#pragma unroll
                    for (int f = 1; f < NF; ++f)
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
            if (PG) {
                // minimum and its label in one reduction (smallest label on ties)
                uint32_t key = 0xFFFFFFFFu;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t kk = lv[k] ? ((L[k] << 16) | (uint32_t)(k * 64 + lane)) : 0xFFFFFFFFu;
                    key = kk < key ? kk : key;
                }
                key = wave_min_u32(key);
                Mq = key >> 16;
                const int bi = (int)(key & 0xFFFFu);
                int f = 0;
                while (f + 1 < F && bi >= a.foff[f + 1]) ++f;
                const int g = (WIN ? op[f] : 0) + (bi - a.foff[f]);
                const int px = pg.sx + t * pg.dx, py = pg.sy + t * pg.dy;
                double rr[3];
                ray_of(a.Kinv, px + 0.5, py + 0.5, rr);
                const double den = a.fam_n[f][0] * rr[0] + a.fam_n[f][1] * rr[1] + a.fam_n[f][2] * rr[2];
                dq2 = dq1;
                dq1 = den < 0.0 ? -pdelta[a.goff[f] + g] / den : 0.0;
            } else {
                Mq = wave_min_u32(m);
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) oq[f] = op[f];
        }
    }
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// Path costs of one direction with two labels per lane as packed 16-bit
// values (labels 2i, 2i+1 of pair i = 64k + lane in register k).  Same
// recursion and results as k_sgm; every family window must hold an even
// number of labels so no pair straddles two families.  The predecessor
// buffer holds 16-bit costs with six +inf guards around each family
// segment; a pair's three taps (j-1, j), (j, j+1), (j+1, j+2) come from
// three aligned 32-bit LDS reads and byte permutes whose selectors follow
// the parity of the shifted index j.  P1 is added with unsigned saturation
// so the guards stay +inf; every finite sum stays below 2^16 by the
// configuration bound.  Global traffic goes through buffer resources built
// per step on the scalar unit from row pointers that advance by one add
// (row base = pixel of the step): the lane offset is the only vector
// operand, and lanes past the label count read 0 and drop their stores by
// the resource's range check.  With PG the same kernel runs the
// path-gradient variant (Eq. sgm-smooth-pg).
// Wave-uniform copies of values read from an argument block (its arrays
// indexed by a uniform index stay uniform, wherever the block lives).
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T *rflp(T *p) {
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}

constexpr int PK_G2 = 6;
constexpr int PK_LW = (kMaxLabels + 2 * PK_G2 * kMaxFam) / 2 + 1;   // 32-bit words per buffer, last one a sink

// One path of the two-label kernel: path index `path` of the frame a (all
// its directions' paths numbered by a.path_begin), run by one wavefront with
// the P2 table s_lut and (path gradient) the plane lists pdelta in LDS, and
// buf0 / buf1 its two LDS predecessor buffers.
template <int KP, int NF, bool WIN, bool SN, bool PG>
__device__ __forceinline__ void sgm_pk_path(const SgmArgs a, const int path, const int *s_lut,
                                            const double *pdelta, uint32_t *buf0, uint32_t *buf1) {
    constexpr int PF = KP >= 2 ? 8 : 16;   // steps per block (ring depth): fewer registers for many labels
    constexpr int G2 = PK_G2;
    constexpr int LW = PK_LW;
    const int lane = threadIdx.x & 63;
    // the argument block's scalars as wave-uniform locals (the block may sit
    // in registers, private memory or global memory depending on the caller)
    const int aw = rfl(a.w), ah = rfl(a.h);
    const uint8_t *__restrict__ aref = rflp(a.ref);
    const int32_t *__restrict__ aoffs = rflp(a.offs);
    const int8_t *__restrict__ adI = rflp(a.dI);
    int slot = 0;
    while (path >= rfl(a.path_begin[slot + 1])) ++slot;
    const int dir = rfl(a.dirs[slot]);
    const PathGeom pg = path_geom(dir, path - rfl(a.path_begin[slot]), aw, ah);
    const size_t N = (size_t)aw * ah;
    const int D = rfl(a.D);
    const int F = NF == 1 ? 1 : rfl(a.n_fam);
    const long pstride = (long)pg.dy * aw + pg.dx;
    const long p0 = (long)pg.sy * aw + pg.sx;
    const int len = pg.len;
    const bool all_valid = D == 128 * KP;

    int fam[KP], li[KP], jmax[KP], seg[KP], widx[KP];
    uint32_t lo8[KP];   // byte offset of the pair inside a pixel's cost row
    bool lv[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int i = 2 * (k * 64 + lane);   // first label of the pair
        lo8[k] = (uint32_t)i;
        lv[k] = i < D;
        int f = 0;
        while (f + 1 < F && i >= a.foff[f + 1]) ++f;
        fam[k] = f;
        li[k] = i - a.foff[f];
        jmax[k] = a.W[f] + 2;
        int sb = G2;
        for (int ff = 0; ff < f; ++ff) sb += a.W[ff] + 2 * G2;
        seg[k] = sb;
        widx[k] = lv[k] ? (sb + li[k]) >> 1 : LW - 1;
    }
    for (int i = lane; i < LW; i += 64) {
        buf0[i] = 0xFFFFFFFFu;
        buf1[i] = 0xFFFFFFFFu;
    }
    __builtin_amdgcn_wave_barrier();

    const uint8_t *__restrict__ S = rflp(a.S);
    uint16_t *__restrict__ out = rflp(a.out[slot]);

    // Uniform per-step values of one block of PF steps, one vector load per
    // quantity (lane j holds step t0 + j, j < PF): the penalty P2 of the
    // intensity change from the previous pixel, the window offsets and the
    // surface-normal offsets.  The loads of a block are issued one block
    // ahead and finished (the P2 lookup in LDS) when the block starts, so no
    // load is waited for before its use.  The first step of the path gets
    // P2 = 0: with the predecessor minimum at 0 the recursion then reduces
    // to L = S there, so the first step needs no code of its own.
    struct BlockRaw {
        int i0, i1;   // intensities at the step and at its predecessor
        bool first;
        int off[NF], di[NF];
    };
    auto issue_block = [&](int t0, BlockRaw &r) {
        const int tl = t0 + (lane & (PF - 1));
        const int t = tl < len ? tl : len - 1;
        const long p = p0 + (long)t * pstride;
        const long pp = p0 + (long)(t > 0 ? t - 1 : 0) * pstride;
        r.i0 = aref[p];
        r.i1 = aref[pp];
        r.first = t == 0;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            r.off[f] = (WIN && f < F) ? aoffs[(size_t)f * N + p] : 0;
            r.di[f] = (SN && f < F) ? (int)adI[((size_t)dir * N + p) * F + f] : 0;
        }
    };
    int c_ref;
    int c_off[NF], c_di[NF];
    auto finish_block = [&](const BlockRaw &r) {
        const int d = r.i0 - r.i1;
        c_ref = r.first ? 0 : s_lut[d < 0 ? -d : d];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            c_off[f] = r.off[f];
            c_di[f] = r.di[f];
        }
    };
    BlockRaw raw;
    issue_block(0, raw);
    finish_block(raw);

    // ring of cost byte pairs, PF steps ahead (steps past the path's end
    // re-read its last pixel)
    uint16_t ring[PF][KP];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const long p = p0 + (long)(u < len ? u : len - 1) * pstride;
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(S + (size_t)p * D, D);
#pragma unroll
        for (int k = 0; k < KP; ++k) ring[u][k] = __builtin_amdgcn_raw_buffer_load_b16(rs, lo8[k], 0, 0);
    }

    u16x2 L[KP];
    uint32_t Mq = 0;
    int oq[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) oq[f] = 0;
    // path-gradient state: depths of the last two minimum-cost points, 2/d
    // of each, and -n^T K^-1 p of the previous pixel per family.  Values
    // carried from one step to the next are the same doubles the formulas
    // would recompute (the ray and its dot products of a pixel, and
    // 1/d = (2/d) / 2, exact in binary floating point).
    double dq1 = 0.0, dq2 = 0.0, a1 = 0.0, a2 = 0.0;
    double c_prev[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) c_prev[f] = 0.0;

    // Row pointers advance by one path step at a time (two scalar adds)
    // instead of being recomputed from the step index: s_ahead is the cost
    // row the ring loads next (PF steps ahead, held at the path's last
    // pixel), o_cur the output row of the current step.
    const long sstride = pstride * D;
    const uint8_t *s_ahead = S + (size_t)(p0 + (long)(PF < len ? PF : len - 1) * pstride) * D;
    uint16_t *o_cur = out + (size_t)p0 * D;

    // one step of the recursion at path position t (ring slot and block
    // lane u); clamp: the ring row may reach the path's last pixel in this
    // step (else it advances unconditionally)
    auto step = [&](const int t, const int u, const bool clamp) __attribute__((always_inline)) {
        u16x2 sv[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) sv[k] = as_u16x2(__builtin_amdgcn_perm(0u, ring[u][k], 0x0c010c00u));
        {
            // the reload of ring[u] may not move above its use (an empty
            // asm that takes sv and yields the offset), so the slot keeps
            // one register across the loop
            uint32_t off[KP];
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                off[k] = lo8[k];
                asm volatile("" : "+v"(off[k]) : "v"(sv[k]));
            }
            const __amdgpu_buffer_rsrc_t rs = row_rsrc(s_ahead, D);
#pragma unroll
            for (int k = 0; k < KP; ++k) ring[u][k] = __builtin_amdgcn_raw_buffer_load_b16(rs, off[k], 0, 0);
            if (!clamp || t + PF + 1 < len) s_ahead += sstride;
            // one live row pointer (the compiler would otherwise keep a
            // precomputed address per unrolled step in scalar registers)
            asm volatile("" : "+s"(s_ahead));
        }
        const uint32_t P2 = (uint32_t)__builtin_amdgcn_readlane(c_ref, u);
        int op[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) op[f] = WIN ? __builtin_amdgcn_readlane(c_off[f], u) : 0;
        uint32_t *cur = (u & 1) ? buf1 : buf0;
        const uint32_t *prev = (u & 1) ? buf0 : buf1;
        double c_cur[NF];   // path gradient: -n^T K^-1 p of this step's pixel
        {
            // splats of uniform 16-bit values (the packed instructions take
            // them as one scalar operand)
            const uint32_t P1 = (uint32_t)rfl(a.p1);
            const u16x2 p1v = (u16x2)(uint16_t)P1;
            const u16x2 mqv = (u16x2)(uint16_t)Mq;
            const uint16_t fl = (uint16_t)(Mq + P2);
            const u16x2 flv = (u16x2)fl;
            int sh[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                int v = WIN ? op[f] - oq[f] : 0;
                if (SN) v += __builtin_amdgcn_readlane(c_di[f], u);
                sh[f] = v;
            }
            // -n^T K^-1 p of this step's pixel per family (path gradient)
            if (PG) {
                const int px = pg.sx + t * pg.dx, py = pg.sy + t * pg.dy;
                double rp[3];
                ray_of(a.Kinv, px + 0.5, py + 0.5, rp);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const double *n = a.fam_n[f < F ? f : 0];
                    c_cur[f] = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
                }
            }
            if (PG && t >= 2 && dq1 > 0.0 && dq2 > 0.0) {
                // extrapolated inverse depth of the path's minimum-cost
                // points, as a plane-index jump per family:
                // 1/d* = 2/dq1 - 1/dq2
                const double inv = a1 - 0.5 * a2;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    if (f >= F) break;
                    const double cp = c_cur[f], cq = c_prev[f];
                    if (!(cp > 0.0) || !(cq > 0.0)) continue;
                    const double ip = inv / cp;
                    const double iq = 1.0 / (dq1 * cq);
                    double v = (ip - iq) / a.step[f];
                    v = fmin(fmax(v, -7.0), 7.0);
                    sh[f] += (int)round(v);
                }
            }
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                int sft = sh[0];
#pragma unroll
                for (int f = 1; f < NF; ++f)
                    if (fam[k] == f) sft = sh[f];
                const int jm = NF == 1 ? a.W[0] + 2 : jmax[k];
                const int sg = NF == 1 ? G2 : seg[k];
                const int j = min(max(li[k] + sft, -4), jm);
                const int base = sg + j;
                // The taps (j-1, j), (j, j+1), (j+1, j+2) of the pair are the
                // 16-bit entries q .. q+3, q = base - 1, of three aligned
                // words A, B, C; byte permutes pick them whatever the
                // parity of q.  One family: every lane shares that parity
                // (the shift's); where j is clamped the words hold guards
                // only, so the choice does not matter there.
                const int q = base - 1;
                const uint32_t qodd = NF == 1 ? (uint32_t)((sft & 1) ^ 1) : (uint32_t)(q & 1);
                const uint32_t s1 = 0x03020100u + qodd * 0x02020202u;
                const uint32_t s2 = s1 + 0x02020202u;
                const int e0 = q >> 1;
                const uint32_t A = prev[e0], B = prev[e0 + 1], C = prev[e0 + 2];
                const uint32_t wm = __builtin_amdgcn_perm(B, A, s1);
                const uint32_t w0 = __builtin_amdgcn_perm(B, A, s2);
                const uint32_t wp = __builtin_amdgcn_perm(C, B, s1);
                const u16x2 cm = as_u16x2(wm), c0 = as_u16x2(w0), cp = as_u16x2(wp);
                const u16x2 c1 = __builtin_elementwise_add_sat(__builtin_elementwise_min(cm, cp), p1v);
                u16x2 best = __builtin_elementwise_min(c0, c1);
                best = __builtin_elementwise_min(best, flv);
                L[k] = sv[k] + (best - mqv);
            }
        }
        u16x2 m2 = as_u16x2(0xFFFFFFFFu);
        const __amdgpu_buffer_rsrc_t ro = row_rsrc(o_cur, 2 * D);
        o_cur += sstride;
        asm volatile("" : "+s"(o_cur));
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            cur[widx[k]] = as_u32(L[k]);
            // non-temporal: the path costs are read once, by the
            // winner-takes-all pass, long after the caches have turned over
            __builtin_amdgcn_raw_buffer_store_b32(as_u32(L[k]), ro, 2 * lo8[k], 0, kNonTemporal);
            m2 = __builtin_elementwise_min(m2, (all_valid || lv[k]) ? L[k] : as_u16x2(0xFFFFFFFFu));
        }
        __builtin_amdgcn_wave_barrier();
        if (PG) {
            // minimum and its label in one reduction (smallest label on ties)
            uint32_t key = 0xFFFFFFFFu;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const uint32_t lw = as_u32(L[k]);
                const uint32_t i0 = lo8[k];
                const uint32_t k0 = (lw << 16) | i0, k1 = (lw & 0xFFFF0000u) | (i0 + 1);
                const bool ok = all_valid || lv[k];
                key = ok && k0 < key ? k0 : key;
                key = ok && k1 < key ? k1 : key;
            }
            key = wave_min_u32(key);
            Mq = key >> 16;
            const int bi = (int)(key & 0xFFFFu);
            int f = 0;
            while (f + 1 < F && bi >= a.foff[f + 1]) ++f;
            const int g = (WIN ? op[f] : 0) + (bi - a.foff[f]);
            double cf = c_cur[0];
#pragma unroll
            for (int ff = 1; ff < NF; ++ff)
                if (ff == f) cf = c_cur[ff];
            const double den = -cf;   // n^T K^-1 p, exactly
            dq2 = dq1;
            a2 = a1;
            dq1 = den < 0.0 ? -pdelta[a.goff[f] + g] / den : 0.0;
            a1 = dq1 > 0.0 ? 2.0 / dq1 : 0.0;
#pragma unroll
            for (int ff = 0; ff < NF; ++ff) c_prev[ff] = c_cur[ff];
        } else {
            const uint32_t mw = as_u32(m2);
            const uint32_t lo = mw & 0xFFFFu, hi = mw >> 16;
            Mq = wave_min_u32(lo < hi ? lo : hi);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) oq[f] = op[f];
    };

    // Whole blocks of PF steps, then the tail.  The loop body is one
    // straight run of PF steps, so every ring slot and block value keeps its
    // register from one block to the next and no load is waited for before
    // its use PF steps later.
    int t0 = 0;
    for (; t0 + 2 * PF + 1 <= len; t0 += PF) {
        issue_block(t0 + PF, raw);
#pragma unroll
        for (int u = 0; u < PF; ++u) step(t0 + u, u, false);
        finish_block(raw);
    }
    for (; t0 + PF <= len; t0 += PF) {
        issue_block(t0 + PF, raw);
#pragma unroll
        for (int u = 0; u < PF; ++u) step(t0 + u, u, true);
        finish_block(raw);
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        if (t0 + u >= len) break;
        step(t0 + u, u, true);
    }
}

template <int KP, int NF, bool WIN, bool SN, bool PG>
__global__ __launch_bounds__(64 * WAVES) void k_sgm_pk(const SgmArgs a) {
    __shared__ uint32_t lbuf[WAVES][2][PK_LW];
    __shared__ int s_lut[256];   // P2 by intensity change
    __shared__ double pdelta[PG ? kMaxPgPlanes : 1];   // path gradient: the level's plane lists
    for (int i = threadIdx.x; i < 256; i += 64 * WAVES) s_lut[i] = a.lut[i];
    if (PG)
        for (int i = threadIdx.x; i < a.sumG; i += 64 * WAVES) pdelta[i] = a.delta[i];
    __syncthreads();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int path = blockIdx.x * WAVES + wid;
    if (path >= a.path_begin[a.n_dirs]) return;
    sgm_pk_path<KP, NF, WIN, SN, PG>(a, path, s_lut, pdelta, lbuf[wid][0], lbuf[wid][1]);
}

// The fields the aggregation reads of a frame's arguments in device memory,
// as wave-uniform values (the frame index is uniform, so are its fields).
__device__ __forceinline__ SgmArgs uniform_sgm_args(const SgmArgs *__restrict__ p) {
    SgmArgs a;
    a.w = rfl(p->w);
    a.h = rfl(p->h);
    a.D = rfl(p->D);
    a.n_fam = rfl(p->n_fam);
    for (int f = 0; f < kMaxFam; ++f) {
        a.W[f] = rfl(p->W[f]);
        a.foff[f] = rfl(p->foff[f]);
    }
    a.S = rflp(p->S);
    a.offs = rflp(p->offs);
    a.dI = rflp(p->dI);
    a.ref = rflp(p->ref);
    a.p1 = rfl(p->p1);
    a.n_dirs = rfl(p->n_dirs);
    for (int d = 0; d < 8; ++d) {
        a.dirs[d] = rfl(p->dirs[d]);
        a.out[d] = rflp(p->out[d]);
    }
    for (int d = 0; d < 9; ++d) a.path_begin[d] = rfl(p->path_begin[d]);
    a.pg = 0;
    return a;
}

// Persistent form over the paths of several frames: every wavefront takes
// the next job (a path of some frame: jobs prefix[f] .. prefix[f + 1] - 1
// are frame f's) from the counter until none is left, and loads the frame's
// P2 table into its own LDS slice when the frame changes.  The counter
// starts at 0 (the host clears it before the launch).
template <int KP, int NF, bool WIN, bool SN>
__global__ __launch_bounds__(64 * WAVES) void k_sgm_pk_jobs(const SgmArgs *__restrict__ list,
                                                            const int *__restrict__ prefix, int n,
                                                            unsigned *__restrict__ counter) {
    __shared__ uint32_t lbuf[WAVES][2][PK_LW];
    __shared__ int s_lut[WAVES][256];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total = rfl(prefix[n]);
    int cur = -1;
    for (;;) {
        unsigned j = 0;
        if (lane == 0) j = atomicAdd(counter, 1u);
        const int job = __builtin_amdgcn_readfirstlane((int)j);
        if (job >= total) break;
        int f = 0;
        while (f + 1 < n && job >= rfl(prefix[f + 1])) ++f;
        if (f != cur) {
            for (int i = lane; i < 256; i += 64) s_lut[wid][i] = list[f].lut[i];
            __builtin_amdgcn_wave_barrier();
            cur = f;
        }
        sgm_pk_path<KP, NF, WIN, SN, false>(uniform_sgm_args(list + f), job - rfl(prefix[f]), s_lut[wid], nullptr,
                                            lbuf[wid][0], lbuf[wid][1]);
    }
}

// Launch the two-label kernel for KP label pairs per lane (variant chosen
// at run time).  Instantiated once per KP in k_sgm_inst.hip.
template <int KP>
void sgm_launch_pk(const SgmArgs &a, bool win, bool sn, dim3 grid, hipStream_t s) {
#define FMVS_SGMPK(W_, S_, P_)                                                                     \
    if (win == W_ && sn == S_ && (a.pg != 0) == P_) {                                              \
        if (a.n_fam == 1)                                                                          \
            hipLaunchKernelGGL((k_sgm_pk<KP, 1, W_, S_, P_>), grid, dim3(64 * WAVES), 0, s, a);    \
        else if (a.n_fam <= 4)                                                                     \
            hipLaunchKernelGGL((k_sgm_pk<KP, 4, W_, S_, P_>), grid, dim3(64 * WAVES), 0, s, a);    \
        else                                                                                       \
            hipLaunchKernelGGL((k_sgm_pk<KP, kMaxFam, W_, S_, P_>), grid, dim3(64 * WAVES), 0, s, a); \
        return;                                                                                    \
    }
    FMVS_SGMPK(false, false, false)
    FMVS_SGMPK(true, false, false)
    FMVS_SGMPK(false, true, false)
    FMVS_SGMPK(true, true, false)
    FMVS_SGMPK(false, false, true)
    FMVS_SGMPK(true, false, true)
#undef FMVS_SGMPK
}

// The persistent form over several frames (no path gradient): nf_max bounds
// the families of every frame (1 or up to 4).
template <int KP>
hipError_t sgm_launch_pk_jobs(const SgmArgs *list, const int *prefix, int n, unsigned *counter, bool win, bool sn,
                              int nf_max, int blocks, hipStream_t s) {
#define FMVS_SGMJ(W_, S_)                                                                                        \
    if (win == W_ && sn == S_) {                                                                                \
        if (nf_max == 1)                                                                                        \
            hipLaunchKernelGGL((k_sgm_pk_jobs<KP, 1, W_, S_>), dim3(blocks), dim3(64 * WAVES), 0, s, list, prefix, \
                               n, counter);                                                                     \
        else if (nf_max <= 4)                                                                                   \
            hipLaunchKernelGGL((k_sgm_pk_jobs<KP, 4, W_, S_>), dim3(blocks), dim3(64 * WAVES), 0, s, list, prefix, \
                               n, counter);                                                                     \
        else                                                                                                    \
            return hipErrorInvalidValue;                                                                        \
        return hipGetLastError();                                                                               \
    }
    FMVS_SGMJ(false, false)
    FMVS_SGMJ(true, false)
    FMVS_SGMJ(false, true)
    FMVS_SGMJ(true, true)
#undef FMVS_SGMJ
    return hipErrorInvalidValue;
}

}  // namespace fmvs
