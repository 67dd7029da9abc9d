// Fused plane-sweep matching on gfx950 (Alg. 1 of the paper): for a tile of
// reference pixels and each plane label, every matching view is warped onto
// the tile (plus the window halo) into LDS; the matching cost of each pixel
// is taken in LDS -- the census of the warped view and its Hamming distance
// to the reference census (v_bcnt), or the negated, truncated and scaled
// NCC against the reference window -- the per-side sums combined by the
// occlusion-robust minimum, and the cost written to the label-innermost
// uint8 volume S[y][x][label].
//
// Tile 64 x 4*RPT pixels, 256 threads = 4 waves; thread (tx, ty) owns
// column tx and RPT consecutive rows (RPT 8 or 4, the caller's choice per
// level), so every LDS row read serves up to RPT census windows.  The label
// range of a block is the union of its pixels' windows
// (dynamic cost volume); pixels whose window misses a label skip the store.
// Costs leave in 4-byte words per pixel (label-innermost rows are
// contiguous), so the L2 sees whole-word writes rather than single bytes.
// Warped values are double-buffered so one barrier per (label, view) pair
// suffices.  Blocks are remapped so that neighbouring tiles share an XCD's L2.
#pragma once
#include "dev_common.hpp"
#include "kernels.hpp"

#include <climits>

namespace fmvs {

namespace {
constexpr int TW = 64, NT = 256;

__device__ __forceinline__ uint32_t insert_sign(uint32_t acc, float v, float c) {
    // (acc << 1) | [v < c]: the sign of v - c (exact for distinct floats,
    // +0 when equal) shifted in through alignbit
    return __builtin_amdgcn_alignbit(acc, __float_as_uint(v - c), 31);
}

// Subset mean for the NCC cost: min over non-empty X of floor(s^X / |X|).
__device__ __forceinline__ int combine_mean(int sL, int sR, int nL, int nR) {
    int best = INT_MAX;
    if (nL > 0) best = sL / nL;
    if (nR > 0) {
        int v = sR / nR;
        best = v < best ? v : best;
    }
    return best;
}

__device__ __forceinline__ int combine_lr(int sL, int sR, int nL, int nR, int m) {
    if (nL == m && nR == m) return sL < sR ? sL : sR;
    int best = INT_MAX;
    if (nL > 0) best = (sL * m) / nL;
    if (nR > 0) {
        int v = (sR * m) / nR;
        best = v < best ? v : best;
    }
    return best;
}

// Warp the tile region onto the reference grid into LDS.  tq holds the
// (clamped) pixel-centre coordinates of every region sample (exact in
// float), so the halo replicates the image border and a thread's sample i
// is one LDS read at a fixed offset.
// INSIDE: every sample of the region maps inside the view (the same value
// without the border clamps, warp_sample_inside).
template <int NS, bool INSIDE>
__device__ __forceinline__ void warp_region(float *buf, const uint8_t *__restrict__ src, int w, int h,
                                            const float2 *tq, int tid, double h0, double h1, double h2, double h3,
                                            double h4, double h5, double h6, double h7, double h8) {
    constexpr int NFULL = NS / NT;
    auto one = [&](const float2 q) {
        return INSIDE ? warp_sample_inside(src, w, h, h0, h1, h2, h3, h4, h5, h6, h7, h8, (double)q.x, (double)q.y)
                      : warp_sample(src, w, h, h0, h1, h2, h3, h4, h5, h6, h7, h8, (double)q.x, (double)q.y);
    };
#pragma unroll 2
    for (int i = 0; i < NFULL; ++i) buf[tid + i * NT] = one(tq[tid + i * NT]);
    if (NS % NT != 0 && tid + NFULL * NT < NS) buf[tid + NFULL * NT] = one(tq[tid + NFULL * NT]);
}
}  // namespace

// NCC cost of one view at one pixel from its window sums (the oracle's
// definition, the same operations in the same order): sA and vA = n sAA -
// sA^2 are exact integers of the reference window.
__device__ __forceinline__ int ncc_finish(int sA_i, int vA_i, double sB, double sBB, double sAB, double n) {
    const double sA = (double)sA_i;
    const double vA = (double)vA_i;
    const double vB = n * sBB - sB * sB;
    const double cov = n * sAB - sA * sB;
    double rho = 0.0;
    if (vA > 0.0 && vB > 0.0) rho = cov / sqrt(vA * vB);
    rho = fmin(1.0, fmax(-1.0, rho));
    const double c = fmin(1.0, 1.0 - rho);
    return (int)floor(255.0 * c + 0.5);
}

// XCD-aware remap: hardware dispatches workgroup b to XCD b % 8; give each
// XCD a contiguous range of logical work items.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
    const int q = nb >> 3, r8 = nb & 7, xcd = b & 7, slot = b >> 3;
    return xcd * q + min(xcd, r8) + slot;
}

// One workgroup's share of the sweep of one frame: logical = tile *
// n_chunks + chunk.
template <int CW, int CH, int RPT, bool WARPED, int COST>
__device__ __forceinline__ void sweep_block(const SweepArgs &a, const int logical) {
    constexpr int TH = 4 * RPT;
    constexpr int RX = CW / 2, RY = CH / 2;
    constexpr int RW = TW + 2 * RX, RH = TH + 2 * RY;
    constexpr int NB = CW * CH - 1;
    constexpr int NHI = NB > 32 ? NB - 32 : 0;
    constexpr int NS = RW * RH;
    __shared__ float wbuf[2][NS];
    __shared__ double aref[COST == 1 ? NS : 1];   // reference intensities of the region (NCC)
    __shared__ float2 tq[NS];   // sample coordinates of the region
    __shared__ int s_lo[kMaxFam], s_hi[kMaxFam];
    __shared__ int s_inside[2][kMaxViews];   // per plane (double-buffered) and view: region maps inside

    const int chunk = logical % a.n_chunks;
    const int tile = logical / a.n_chunks;
    const int x0 = (tile % a.tiles_x) * TW;
    const int y0 = (tile / a.tiles_x) * TH;

    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int x = x0 + tx;
    const size_t N = (size_t)a.w * a.h;

    if (tid < kMaxFam) {
        s_lo[tid] = INT_MAX;
        s_hi[tid] = INT_MIN;
    }
    for (int s2 = tid; s2 < NS; s2 += NT) {
        const int rx = s2 % RW, ry = s2 / RW;
        tq[s2] = make_float2((float)min(max(x0 - RX + rx, 0), a.w - 1) + 0.5f,
                             (float)min(max(y0 - RY + ry, 0), a.h - 1) + 0.5f);
    }
    // corners of the region's (clamped) sample points
    const double qx_lo = (double)max(x0 - RX, 0) + 0.5, qx_hi = (double)min(x0 - RX + RW - 1, a.w - 1) + 0.5;
    const double qy_lo = (double)max(y0 - RY, 0) + 0.5, qy_hi = (double)min(y0 - RY + RH - 1, a.h - 1) + 0.5;
    __syncthreads();

    uint32_t ref_hi[RPT], ref_lo[RPT];   // census cost: the reference census words
    int refA[RPT], refV[RPT];            // NCC cost: sum and n * sum of squares - sum^2 of the window
    bool valid[RPT];
    uint32_t pix[RPT];
    if (COST == 1) {
        for (int s2 = tid; s2 < NS; s2 += NT) {
            const int rx = s2 % RW, ry = s2 / RW;
            const int qx = min(max(x0 - RX + rx, 0), a.w - 1), qy = min(max(y0 - RY + ry, 0), a.h - 1);
            aref[s2] = (double)a.ref[(size_t)qy * a.w + qx];
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        int y = y0 + ty * RPT + j;
        valid[j] = x < a.w && y < a.h;
        pix[j] = valid[j] ? (uint32_t)(y * a.w + x) : 0u;
        if (COST == 0) {
            uint64_t ct = valid[j] ? a.ct_ref[pix[j]] : 0;
            ref_hi[j] = (uint32_t)(ct >> 32);
            ref_lo[j] = (uint32_t)ct;
        } else {
            int sA = 0, sAA = 0;
#pragma unroll 1
            for (int dy = 0; dy < CH; ++dy)
                for (int dx = 0; dx < CW; ++dx) {
                    const int v = (int)aref[(ty * RPT + j + dy) * RW + tx + dx];
                    sA += v;
                    sAA += v * v;
                }
            refA[j] = sA;
            refV[j] = CW * CH * sAA - sA * sA;
        }
        if (valid[j]) {
            for (int f = 0; f < a.n_fam; ++f) {
                int o = a.offs ? a.offs[(size_t)f * N + pix[j]] : 0;
                atomicMin(&s_lo[f], o);
                atomicMax(&s_hi[f], o + a.W[f]);
            }
        }
    }
    __syncthreads();

    // this block's share of the concatenated union of label ranges
    int total = 0;
    for (int f = 0; f < a.n_fam; ++f) total += s_hi[f] > s_lo[f] ? s_hi[f] - s_lo[f] : 0;
    const int per = (total + a.n_chunks - 1) / a.n_chunks;
    const int pos0 = chunk * per;
    const int pos1 = min(total, pos0 + per);
    if (pos0 >= pos1) return;
    if (a.work && tid == 0) {
        int nv = min(TW, a.w - x0) * min(TH, a.h - y0);
        atomicAdd(a.work, (unsigned long long)(pos1 - pos0) * (unsigned long long)nv);
    }

    int f = 0, fbase = 0;
    while (f < a.n_fam && pos0 >= fbase + (s_hi[f] - s_lo[f])) {
        fbase += s_hi[f] - s_lo[f];
        ++f;
    }
    int g = s_lo[f] + (pos0 - fbase);
    // labels of family f this block evaluates: [g_first, g_last]
    int g_first = g;
    int g_last = s_lo[f] + min(pos1 - fbase, s_hi[f] - s_lo[f]) - 1;
    int off[RPT];   // window offsets of the current family
#pragma unroll
    for (int j = 0; j < RPT; ++j) off[j] = (a.offs && valid[j]) ? a.offs[(size_t)f * N + pix[j]] : 0;
    // Costs are written 4 labels at a time when the label count keeps the
    // pixel rows 4-byte aligned: acc holds the last bytes of the pixel's
    // run, the newest in the top byte.  Byte stores otherwise.
    const bool pack = (a.D & 3) == 0 && ((uintptr_t)a.S & 3) == 0;
    uint32_t acc[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) acc[j] = 0;

    // Whether each view's region maps inside the view for plane (f_, g_),
    // into slot sl, by the first wave: lane 4k + c tests corner c of view k.
    auto mark_inside = [&](int sl, int f_, int g_) {
        if (WARPED || tid >= 64) return;
        const int k = tid >> 2;
        bool in = true;
        if (k < a.n_views)
            in = warp_corner_inside(a.H + ((size_t)k * a.sumG + a.goff[f_] + g_) * 9, tid & 3, qx_lo, qx_hi, qy_lo,
                                    qy_hi, a.w, a.h);
        const unsigned long long all = __ballot(in);
        if (k < a.n_views && (tid & 3) == 0) s_inside[sl][k] = ((all >> (4 * k)) & 0xFull) == 0xFull;
    };
    // the plane after (f_, g_) in this block's order
    auto next_plane = [&](int &f_, int &g_) {
        if (++g_ >= s_hi[f_]) {
            ++f_;
            while (f_ < a.n_fam && s_hi[f_] <= s_lo[f_]) ++f_;
            if (f_ < a.n_fam) g_ = s_lo[f_];
        }
    };
    mark_inside(pos0 & 1, f, g);
    __syncthreads();

    int it = 0;
    for (int pos = pos0; pos < pos1; ++pos) {
        // left-view sums in the low 16 bits, right-view sums in the high 16
        // (at most 8 views of at most 255 each): one shift-add per view and
        // pixel, the subset decided by a uniform shift
        uint32_t sLR[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) sLR[j] = 0;
        const size_t lab = (size_t)a.goff[f] + g;
        for (int k = 0; k < a.n_views; ++k, ++it) {
            float *buf = wbuf[it & 1];
            const size_t hk = (size_t)k * a.sumG + lab;
            if (WARPED) {
                const float *src = a.warped + hk * N;
                for (int s = tid; s < NS; s += NT) {
                    int rx = s % RW, ry = s / RW;
                    int qx = clampi(x0 - RX + rx, 0, a.w - 1), qy = clampi(y0 - RY + ry, 0, a.h - 1);
                    buf[s] = src[(size_t)qy * a.w + qx];
                }
            } else {
                const double *Hm = a.H + hk * 9;
                const double h0 = Hm[0], h1 = Hm[1], h2 = Hm[2], h3 = Hm[3], h4 = Hm[4], h5 = Hm[5], h6 = Hm[6],
                             h7 = Hm[7], h8 = Hm[8];
                // the next plane's flags, while this plane's are read (that
                // slot was last read before the previous barrier)
                if (k == 0 && pos + 1 < pos1) {
                    int fn = f, gn = g;
                    next_plane(fn, gn);
                    mark_inside((pos + 1) & 1, fn, gn);
                }
                const uint8_t *src = a.views[k];
                if (s_inside[pos & 1][k])
                    warp_region<NS, true>(buf, src, a.w, a.h, tq, tid, h0, h1, h2, h3, h4, h5, h6, h7, h8);
                else
                    warp_region<NS, false>(buf, src, a.w, a.h, tq, tid, h0, h1, h2, h3, h4, h5, h6, h7, h8);
            }
            __syncthreads();
            const uint32_t sh = a.side[k] < 0 ? 0u : 16u;
            const float *base = buf + (ty * RPT) * RW + tx;
            if (COST == 0) {
                // census of the warped view for this thread's pixels
                float c[RPT];
#pragma unroll
                for (int j = 0; j < RPT; ++j) c[j] = base[(j + RY) * RW + RX];
                uint32_t hi[RPT], lo[RPT];
#pragma unroll
                for (int j = 0; j < RPT; ++j) hi[j] = lo[j] = 0;
#pragma unroll
                for (int rr = 0; rr < RPT + 2 * RY; ++rr) {
                    float v[CW];
#pragma unroll
                    for (int cx = 0; cx < CW; ++cx) v[cx] = base[rr * RW + cx];
#pragma unroll
                    for (int j = 0; j < RPT; ++j) {
                        const int wy = rr - j;
                        if (wy < 0 || wy >= CH) continue;
#pragma unroll
                        for (int cx = 0; cx < CW; ++cx) {
                            if (wy == RY && cx == RX) continue;
                            const int bpos = wy * CW + cx - ((wy > RY || (wy == RY && cx > RX)) ? 1 : 0);
                            if (bpos < NHI)
                                hi[j] = insert_sign(hi[j], v[cx], c[j]);
                            else
                                lo[j] = insert_sign(lo[j], v[cx], c[j]);
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    const uint32_t cst = __popc(hi[j] ^ ref_hi[j]) + __popc(lo[j] ^ ref_lo[j]);
                    sLR[j] += cst << sh;
                }
            } else {
                // NCC: row sums of the window rows, left to right, then the
                // window sums over the rows top to bottom, in double.  Every
                // term is non-negative, so starting the sums at +0 gives the
                // same values as starting them at the first term.  The row
                // loop stays rolled (its bounds are uniform, the tests on
                // them scalar): unrolled, the hoisted LDS reads exhaust the
                // registers.
                const double *abase = aref + (ty * RPT) * RW + tx;
                double wB[RPT], wBB[RPT], wAB[RPT];
#pragma unroll
                for (int j = 0; j < RPT; ++j) wB[j] = wBB[j] = wAB[j] = 0.0;
#pragma unroll 1
                for (int rr = 0; rr < RPT + 2 * RY; ++rr) {
                    double rB = 0.0, rBB = 0.0, rAB = 0.0;
#pragma unroll
                    for (int cx = 0; cx < CW; ++cx) {
                        const double vb = (double)base[rr * RW + cx];
                        const double va = abase[rr * RW + cx];
                        rB = rB + vb;
                        rBB = __builtin_fma(vb, vb, rBB);
                        rAB = __builtin_fma(va, vb, rAB);
                    }
#pragma unroll
                    for (int j = 0; j < RPT; ++j) {
                        if ((unsigned)(rr - j) < (unsigned)CH) {
                            wB[j] = wB[j] + rB;
                            wBB[j] = wBB[j] + rBB;
                            wAB[j] = wAB[j] + rAB;
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    const uint32_t cst = (uint32_t)ncc_finish(refA[j], refV[j], wB[j], wBB[j], wAB[j], (double)(CW * CH));
                    sLR[j] += cst << sh;
                }
            }
        }
        // store the combined cost where this label lies in the pixel's window
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int o = off[j];
            if (valid[j] && g >= o && g < o + a.W[f]) {
                const int sL = (int)(sLR[j] & 0xFFFFu), sR = (int)(sLR[j] >> 16);
                const uint32_t cst = COST == 0 ? (uint32_t)combine_lr(sL, sR, a.nL, a.nR, a.m)
                                               : (uint32_t)combine_mean(sL, sR, a.nL, a.nR);
                const int idx = a.foff[f] + (g - o);
                uint8_t *dst = a.S + (size_t)pix[j] * a.D + idx;
                if (pack) {
                    acc[j] = (acc[j] >> 8) | (cst << 24);
                    const int run_end = min(o + a.W[f], g_last + 1) - 1;
                    if ((idx & 3) == 3 || g == run_end) {
                        const int n = min((idx & 3) + 1, g - max(o, g_first) + 1);
                        if (n == 4) {
                            *(uint32_t *)(dst - 3) = acc[j];
                        } else {
                            for (int b = 0; b < n; ++b) dst[b - n + 1] = (uint8_t)(acc[j] >> (8 * (4 - n + b)));
                        }
                    }
                } else {
                    *dst = (uint8_t)cst;
                }
            }
        }
        if (++g >= s_hi[f]) {
            fbase += s_hi[f] - s_lo[f];
            ++f;
            while (f < a.n_fam && s_hi[f] <= s_lo[f]) ++f;
            if (f < a.n_fam) {
                g = s_lo[f];
                g_first = g;
                g_last = s_lo[f] + min(pos1 - fbase, s_hi[f] - s_lo[f]) - 1;
#pragma unroll
                for (int j = 0; j < RPT; ++j) off[j] = (a.offs && valid[j]) ? a.offs[(size_t)f * N + pix[j]] : 0;
            }
        }
    }
}

template <int CW, int CH, int RPT, bool WARPED, int COST>
__global__ __launch_bounds__(NT) void k_sweep(const SweepArgs a) {
    sweep_block<CW, CH, RPT, WARPED, COST>(a, xcd_logical(blockIdx.x, gridDim.x));
}

// Several frames in one launch: the workgroups of frame f are the logical
// items prefix[f] .. prefix[f + 1] - 1 (each frame's tiles x chunks), the
// whole grid remapped to XCDs as one.
template <int CW, int CH, int RPT, int COST>
__global__ __launch_bounds__(NT) void k_sweep_batch(const SweepArgs *__restrict__ list,
                                                    const int *__restrict__ prefix, int n) {
    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    int f = 0;
    while (f + 1 < n && logical >= prefix[f + 1]) ++f;
    sweep_block<CW, CH, RPT, false, COST>(list[f], logical - prefix[f]);
}

// Launch one window size and cost: tiles of 64 x 4*rpt pixels (rpt 4 or 8),
// from homographies or from pre-warped views.  Each (window, cost) pair is
// instantiated in a translation unit of its own so the sweep variants
// compile in parallel.
template <int CW, int CH, int COST>
hipError_t sweep_launch_cfg(const SweepArgs &a, dim3 grid, int rpt, hipStream_t s) {
    if (rpt == 4) {
        if (a.warped)
            hipLaunchKernelGGL((k_sweep<CW, CH, 4, true, COST>), grid, dim3(NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_sweep<CW, CH, 4, false, COST>), grid, dim3(NT), 0, s, a);
    } else {
        if (a.warped)
            hipLaunchKernelGGL((k_sweep<CW, CH, 8, true, COST>), grid, dim3(NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_sweep<CW, CH, 8, false, COST>), grid, dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

template <int CW, int CH, int COST>
hipError_t sweep_launch_batch_cfg(const SweepArgs *list, const int *prefix, int n, int blocks, int rpt,
                                  hipStream_t s) {
    if (rpt == 4)
        hipLaunchKernelGGL((k_sweep_batch<CW, CH, 4, COST>), dim3(blocks), dim3(NT), 0, s, list, prefix, n);
    else
        hipLaunchKernelGGL((k_sweep_batch<CW, CH, 8, COST>), dim3(blocks), dim3(NT), 0, s, list, prefix, n);
    return hipGetLastError();
}

}  // namespace fmvs
