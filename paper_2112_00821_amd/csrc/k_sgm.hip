// Host dispatch of the semi-global aggregation and the winner-takes-all
// kernels (Eq. sgm-path, sgm-aggr, sgm-wta of the paper); the aggregation
// kernels themselves are in k_sgm.hpp (the two-label kernel is instantiated
// per label-pair count in k_sgm_inst.hip so the variants compile in
// parallel).
#include "k_sgm.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>

namespace fmvs {

extern template void sgm_launch_pk<1>(const SgmArgs &, bool, bool, dim3, hipStream_t);
extern template void sgm_launch_pk<2>(const SgmArgs &, bool, bool, dim3, hipStream_t);
extern template void sgm_launch_pk<3>(const SgmArgs &, bool, bool, dim3, hipStream_t);
extern template void sgm_launch_pk<4>(const SgmArgs &, bool, bool, dim3, hipStream_t);
extern template hipError_t sgm_launch_pk_jobs<1>(const SgmArgs *, const int *, int, unsigned *, bool, bool, int, int,
                                                 hipStream_t);
extern template hipError_t sgm_launch_pk_jobs<2>(const SgmArgs *, const int *, int, unsigned *, bool, bool, int, int,
                                                 hipStream_t);
extern template hipError_t sgm_launch_pk_jobs<3>(const SgmArgs *, const int *, int, unsigned *, bool, bool, int, int,
                                                 hipStream_t);
extern template hipError_t sgm_launch_pk_jobs<4>(const SgmArgs *, const int *, int, unsigned *, bool, bool, int, int,
                                                 hipStream_t);

int sgm_paths(int dir, int w, int h) {
    int dx = dir_dx(dir), dy = dir_dy(dir);
    if (dy == 0) return h;
    if (dx == 0) return w;
    return w + h - 1;
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

// Row-level (16-lane) minimum: every lane of a DPP row ends with its row's
// minimum.
__device__ __forceinline__ uint32_t row_min_u32(uint32_t v) {
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false);
    v = v < t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false);
    v = v < t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false);
    v = v < t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false);
    return v < t ? v : t;
}

typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));

// Winner-takes-all for label counts that are a multiple of 8: a DPP row of
// 16 lanes owns one pixel (4 pixels per wavefront, contiguous in memory);
// each lane reads 8 labels of every direction buffer with one 16-byte load
// and adds them as packed 16-bit pairs (the aggregate fits 16 bits by the
// configuration's bound); argmin and the neighbours' aggregates come from
// row-level DPP reductions.
template <int NCH>
__global__ __launch_bounds__(256) void k_wta16(const SgmArgs a) {
    const int lane = threadIdx.x & 63;
    const int row = lane >> 4, l16 = lane & 15;
    const size_t N = (size_t)a.w * a.h;
    const int D = a.D;
    const int nch = D >> 3;
    const size_t waves = (size_t)gridDim.x * 4;
    const size_t wid = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const size_t vol_bytes = N * D * 2;
    const bool rsrc_ok = vol_bytes < ((size_t)1 << 32);
    for (size_t pb = wid * 4; pb < N; pb += waves * 4) {
        const size_t p = pb + row;
        const bool pv = p < N;
        uint32_t key = 0xFFFFFFFFu;
        uint32_t acc[NCH][4];
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int c = l16 + 16 * j;
            const bool cv = pv && c < nch;
            ushort2_t s4[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                if (b < a.n_in && cv) {
                    // each path cost is read once: non-temporal load
                    // through a buffer resource over the whole volume
                    // (32-bit byte offsets), else a plain load
                    uint4 v;
                    if (rsrc_ok) {
                        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
                            const_cast<uint16_t *>(a.in[b]), 0, (int)(uint32_t)vol_bytes, 0x00020000);
                        v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                          rb, (uint32_t)((p * D + 8 * c) * 2), 0, kNonTemporal));
                    } else {
                        v = *(const uint4 *)(a.in[b] + p * D + 8 * c);
                    }
                    s4[0] += __builtin_bit_cast(ushort2_t, v.x);
                    s4[1] += __builtin_bit_cast(ushort2_t, v.y);
                    s4[2] += __builtin_bit_cast(ushort2_t, v.z);
                    s4[3] += __builtin_bit_cast(ushort2_t, v.w);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[j][e] = __builtin_bit_cast(uint32_t, s4[e]);
                if (cv) {
                    const uint32_t lo = acc[j][e] & 0xFFFFu, hi = acc[j][e] >> 16;
                    const uint32_t i0 = (uint32_t)(8 * c + 2 * e);
                    const uint32_t k0 = (lo << 16) | i0, k1 = (hi << 16) | (i0 + 1);
                    key = k0 < key ? k0 : key;
                    key = k1 < key ? k1 : key;
                }
            }
        }
        key = row_min_u32(key);
        const int best = (int)(key & 0xFFFFu);
        int f = 0;
        while (f + 1 < a.n_fam && best >= a.foff[f + 1]) ++f;
        const int l = best - a.foff[f];
        const bool has_m = l >= 1, has_p = l + 1 < a.W[f];
        uint32_t cm = 0xFFFFu, cp = 0xFFFFu;
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int c = l16 + 16 * j;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = 8 * c + e;
                const uint32_t v = (e & 1) ? (acc[j][e >> 1] >> 16) : (acc[j][e >> 1] & 0xFFFFu);
                if (has_m && i == best - 1) cm = v;
                if (has_p && i == best + 1) cp = v;
            }
        }
        cm = row_min_u32(cm);
        cp = row_min_u32(cp);
        if (pv && l16 == 0) {
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
        const size_t N = (size_t)a.w * a.h;
        if ((a.D & 7) == 0) {
            unsigned blocks = (unsigned)std::min<size_t>((N + 15) / 16, 65536);
            const int ncb = ((a.D >> 3) + 15) / 16;   // 8-label chunks per lane
            switch (ncb) {
                case 1: hipLaunchKernelGGL((k_wta16<1>), dim3(blocks), dim3(256), 0, s, a); return;
                case 2: hipLaunchKernelGGL((k_wta16<2>), dim3(blocks), dim3(256), 0, s, a); return;
                case 3: hipLaunchKernelGGL((k_wta16<3>), dim3(blocks), dim3(256), 0, s, a); return;
                default: hipLaunchKernelGGL((k_wta16<4>), dim3(blocks), dim3(256), 0, s, a); return;
            }
        }
        unsigned blocks = (unsigned)std::min<size_t>((N + 3) / 4, 65536);
        hipLaunchKernelGGL((k_wta<K>), dim3(blocks), dim3(256), 0, s, a);
        return;
    }
#define FMVS_SGM(W_, S_, P_)                                                                  \
    if (win == W_ && sn == S_ && (a.pg != 0) == P_) {                                         \
        if (a.n_fam == 1)                                                                     \
            hipLaunchKernelGGL((k_sgm<K, 1, W_, S_, P_>), grid, dim3(64 * WAVES), 0, s, a);   \
        else                                                                                  \
            hipLaunchKernelGGL((k_sgm<K, kMaxFam, W_, S_, P_>), grid, dim3(64 * WAVES), 0, s, a); \
        return;                                                                               \
    }
    FMVS_SGM(false, false, false)
    FMVS_SGM(true, false, false)
    FMVS_SGM(false, true, false)
    FMVS_SGM(true, true, false)
    FMVS_SGM(false, false, true)
    FMVS_SGM(true, false, true)
#undef FMVS_SGM
}


// Packed two-label kernel when every family window is even (all variants);
// the one-label kernel otherwise.
__global__ void k_zero_u32(unsigned *p) {
    if (threadIdx.x == 0) *p = 0u;
}

static bool use_packed(const SgmArgs &a) {
    if (a.final_mode || (a.D & 1)) return false;
    for (int f = 0; f < a.n_fam; ++f)
        if (a.W[f] & 1) return false;
    // FASSMVS_SGM_UNPACKED=1 selects the one-label kernel (same results);
    // read per launch so a process can run both
    const char *e = std::getenv("FASSMVS_SGM_UNPACKED");
    return !(e && std::atoi(e) != 0);
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
    if (a.pg && (sn || a.sumG > kMaxPgPlanes || !a.delta)) return hipErrorInvalidValue;
    if (use_packed(a)) {
        switch ((a.D + 127) / 128) {
            case 1: sgm_launch_pk<1>(a, win, sn, grid, s); break;
            case 2: sgm_launch_pk<2>(a, win, sn, grid, s); break;
            case 3: sgm_launch_pk<3>(a, win, sn, grid, s); break;
            case 4: sgm_launch_pk<4>(a, win, sn, grid, s); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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

// Several frames' aggregation in one persistent launch (two steps, as for
// the sweep).  prepare_sgm_batch: host[0..n-1] are the frames' args, each
// with its directions and output buffers set (write mode, no path gradient,
// even label counts and windows so the two-label kernel applies, at most 4
// families, the same windows / surface-normal choice); their path prefix
// per direction is set and they are written with the job prefix (n + 1
// ints) to out (host memory of sgm_batch_bytes(n)).  Returns the job count
// (paths over all frames), or -1 if the frames cannot share a launch; *kp,
// *win, *sn, *nf_max receive the kernel variant.
size_t sgm_batch_bytes(int n) { return sizeof(SgmArgs) * n + sizeof(int) * (n + 1); }

int prepare_sgm_batch(SgmArgs *host, int n, void *out, int *kp, bool *win, bool *sn, int *nf_max) {
    if (n < 1) return -1;
    int *prefix = (int *)((SgmArgs *)out + n);
    prefix[0] = 0;
    *kp = 1;
    *nf_max = 1;
    *win = host[0].offs != nullptr;
    *sn = host[0].dI != nullptr;
    for (int i = 0; i < n; ++i) {
        SgmArgs &a = host[i];
        if (a.pg || a.final_mode || !use_packed(a) || a.n_fam > 4 || (a.offs != nullptr) != *win ||
            (a.dI != nullptr) != *sn)
            return -1;
        a.path_begin[0] = 0;
        for (int d = 0; d < a.n_dirs; ++d) a.path_begin[d + 1] = a.path_begin[d] + sgm_paths(a.dirs[d], a.w, a.h);
        for (int d = a.n_dirs + 1; d < 9; ++d) a.path_begin[d] = a.path_begin[a.n_dirs];
        prefix[i + 1] = prefix[i] + a.path_begin[a.n_dirs];
        *kp = std::max(*kp, (a.D + 127) / 128);
        *nf_max = std::max(*nf_max, a.n_fam);
    }
    if (*kp > 4) return -1;
    std::memcpy(out, host, sizeof(SgmArgs) * n);
    return prefix[n];
}

// launch_sgm_batch: the args block prepared above in device memory at dev;
// counter: a device word the launch takes jobs from, cleared here by a fill
// kernel.  The grid holds up to six workgroups per CU; every wavefront
// leaves when the jobs run out.
hipError_t launch_sgm_batch(const void *dev, int n, int jobs, int kp, bool win, bool sn, int nf_max,
                            unsigned *counter, hipStream_t s) {
    if (jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const SgmArgs *dl = (const SgmArgs *)dev;
    const int *dp = (const int *)((const SgmArgs *)dev + n);
    const int blocks = std::min((jobs + WAVES - 1) / WAVES, 256 * 6);
    switch (kp) {
        case 1: return sgm_launch_pk_jobs<1>(dl, dp, n, counter, win, sn, nf_max, blocks, s);
        case 2: return sgm_launch_pk_jobs<2>(dl, dp, n, counter, win, sn, nf_max, blocks, s);
        case 3: return sgm_launch_pk_jobs<3>(dl, dp, n, counter, win, sn, nf_max, blocks, s);
        case 4: return sgm_launch_pk_jobs<4>(dl, dp, n, counter, win, sn, nf_max, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fmvs
