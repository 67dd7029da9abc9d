// Post-processing filters on gfx950 (Sec. on post-processing and depth map
// filtering): the DoG texture mask of Alg. 3 and the geometric consistency
// check of Alg. 4.  Both are per-pixel stencils over level-0 maps.
//
// The speckle steps of Alg. 3 need the size of a pixel's 4-connected
// component only up to the threshold K (7 or 21): a bounded breadth-first
// search from every pixel stops as soon as K pixels are found, so no global
// labelling is needed and the result is exact.  The visited list lives in
// registers (K entries, filled by a select chain).
#include "dev_common.hpp"
#include "kernels.hpp"

namespace fmvs {

namespace {

__global__ void k_gauss_h(const uint8_t *__restrict__ img, int w, int h, PostArgs a, double *__restrict__ tmp) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= w || y >= h) return;
    const uint8_t *row = img + (size_t)y * w;
    double acc = 0.0;
    for (int i = -a.radius; i <= a.radius; ++i) acc = acc + a.taps[i + a.radius] * (double)row[clampi(x + i, 0, w - 1)];
    tmp[(size_t)y * w + x] = acc;
}

__global__ void k_gauss_v_dog(const uint8_t *__restrict__ img, const double *__restrict__ tmp, int w, int h,
                              PostArgs a, uint8_t *__restrict__ on) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= w || y >= h) return;
    double acc = 0.0;
    for (int j = -a.radius; j <= a.radius; ++j)
        acc = acc + a.taps[j + a.radius] * tmp[(size_t)clampi(y + j, 0, h - 1) * w + x];
    const double dog = (double)img[(size_t)y * w + x] - acc;
    on[(size_t)y * w + x] = fabs(dog) > a.thresh ? 1 : 0;
}

// Pixels equal to v whose 4-connected component has fewer than K pixels
// flip to 1 - v; everything else is copied.
template <int K>
__global__ void k_speckle(const uint8_t *__restrict__ in, int w, int h, int v, uint8_t *__restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= w || y >= h) return;
    const uint8_t c = in[(size_t)y * w + x];
    if (c != v) {
        out[(size_t)y * w + x] = c;
        return;
    }
    int vis[K];   // packed (x, y) of the pixels found so far
#pragma unroll
    for (int i = 0; i < K; ++i) vis[i] = -1;
    vis[0] = (y << 16) | x;
    int count = 1;
#pragma unroll
    for (int qi = 0; qi < K; ++qi) {
        if (qi >= count || count >= K) break;
        const int cx = vis[qi] & 0xFFFF, cy = vis[qi] >> 16;
        const int nx[4] = {cx - 1, cx + 1, cx, cx};
        const int ny[4] = {cy, cy, cy - 1, cy + 1};
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (count >= K) break;
            if (nx[d] < 0 || nx[d] >= w || ny[d] < 0 || ny[d] >= h) continue;
            if (in[(size_t)ny[d] * w + nx[d]] != v) continue;
            const int key = (ny[d] << 16) | nx[d];
            bool seen = false;
#pragma unroll
            for (int j = 0; j < K; ++j) seen |= vis[j] == key;
            if (seen) continue;
#pragma unroll
            for (int j = 0; j < K; ++j) vis[j] = j == count ? key : vis[j];
            ++count;
        }
    }
    out[(size_t)y * w + x] = count < K ? (uint8_t)(1 - v) : (uint8_t)v;
}

__global__ void k_dilate3(const uint8_t *__restrict__ in, int w, int h, uint8_t *__restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= w || y >= h) return;
    uint8_t v = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = x + dx, yy = y + dy;
            if (xx >= 0 && xx < w && yy >= 0 && yy < h && in[(size_t)yy * w + xx]) v = 1;
        }
    out[(size_t)y * w + x] = v;
}

// Zero the maps where keep is 0 (depth, normal xyz, confidence; any NULL).
__global__ void k_apply_keep(const uint8_t *__restrict__ keep, size_t n, float *depth, float *normal, float *conf) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || keep[i]) return;
    if (depth) depth[i] = 0.0f;
    if (normal) {
        normal[3 * i] = 0.0f;
        normal[3 * i + 1] = 0.0f;
        normal[3 * i + 2] = 0.0f;
    }
    if (conf) conf[i] = 0.0f;
}

__global__ void k_geo(GeoArgs a, int32_t *__restrict__ hits, uint8_t *__restrict__ keep) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.w || y >= a.h) return;
    const size_t p = (size_t)y * a.w + x;
    const double d = a.depth_ref[p];
    const double *K = a.K;
    int nh = 0;
    if (d > 0.0) {
        const double u0 = x + 0.5, v0 = y + 0.5;
        double ray[3];
        ray_of(a.Kinv, u0, v0, ray);
        const double X[3] = {d * ray[0], d * ray[1], d * ray[2]};
        for (int k = 0; k < a.n_nb; ++k) {
            const double *Rk = a.R[k];
            const double *tk = a.t[k];
            double Xk[3];
            for (int i = 0; i < 3; ++i) Xk[i] = Rk[3 * i] * X[0] + Rk[3 * i + 1] * X[1] + Rk[3 * i + 2] * X[2] + tk[i];
            if (!(Xk[2] > 0.0)) continue;
            const double uk = (K[0] * Xk[0] + K[1] * Xk[1] + K[2] * Xk[2]) / Xk[2];
            const double vk = (K[3] * Xk[0] + K[4] * Xk[1] + K[5] * Xk[2]) / Xk[2];
            const double fx = floor(uk), fy = floor(vk);
            if (!(fx >= 0.0 && fx < (double)a.w && fy >= 0.0 && fy < (double)a.h)) continue;
            const double dk = a.depth_nb[k][(size_t)fy * a.w + (size_t)fx];
            if (!(dk > 0.0)) continue;
            double rk[3];
            ray_of(a.Kinv, uk, vk, rk);
            const double Y[3] = {dk * rk[0] - tk[0], dk * rk[1] - tk[1], dk * rk[2] - tk[2]};
            double Xb[3];
            for (int i = 0; i < 3; ++i) Xb[i] = Rk[i] * Y[0] + Rk[3 + i] * Y[1] + Rk[6 + i] * Y[2];
            if (!(Xb[2] > 0.0)) continue;
            const double ub = (K[0] * Xb[0] + K[1] * Xb[1] + K[2] * Xb[2]) / Xb[2];
            const double vb = (K[3] * Xb[0] + K[4] * Xb[1] + K[5] * Xb[2]) / Xb[2];
            const double eu = ub - u0, ev = vb - v0;
            if (sqrt(eu * eu + ev * ev) < a.eta_r) ++nh;
        }
    }
    if (hits) hits[p] = nh;
    keep[p] = (d > 0.0 && nh >= a.eta_h) ? 1 : 0;
}

}  // namespace

hipError_t launch_dog_mask(const uint8_t *img, int w, int h, const PostArgs &a, double *tmp, uint8_t *m0, uint8_t *m1,
                           hipStream_t s) {
    const dim3 blk(256), grid((unsigned)((w + 255) / 256), (unsigned)h);
    hipLaunchKernelGGL(k_gauss_h, grid, blk, 0, s, img, w, h, a, tmp);
    hipLaunchKernelGGL(k_gauss_v_dog, grid, blk, 0, s, img, tmp, w, h, a, m0);
    // speckle on the activations, dilation, speckle on the deactivations:
    // m0 -> m1 -> m0 -> m1
    if (a.min_on == 7)
        hipLaunchKernelGGL((k_speckle<7>), grid, blk, 0, s, m0, w, h, 1, m1);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dilate3, grid, blk, 0, s, m1, w, h, m0);
    if (a.min_off == 21)
        hipLaunchKernelGGL((k_speckle<21>), grid, blk, 0, s, m0, w, h, 0, m1);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_apply_keep(const uint8_t *keep, size_t n, float *depth, float *normal, float *conf, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_apply_keep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keep, n, depth, normal, conf);
    return hipGetLastError();
}

hipError_t launch_geo(const GeoArgs &a, int32_t *hits, uint8_t *keep, hipStream_t s) {
    const dim3 blk(256), grid((unsigned)((a.w + 255) / 256), (unsigned)a.h);
    hipLaunchKernelGGL(k_geo, grid, blk, 0, s, a, hits, keep);
    return hipGetLastError();
}

}  // namespace fmvs
