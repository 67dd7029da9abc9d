// Device helpers shared by the gfx950 kernels of the FaSS-MVS library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmvs {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// 1 / z for a positive normal double: the hardware estimate refined by two
// Newton steps (within an ulp of the correctly rounded quotient).
__device__ __forceinline__ double recip(double z) {
    const double r0 = __builtin_amdgcn_rcp(z);
    const double r1 = __builtin_fma(r0, __builtin_fma(-z, r0, 1.0), r0);
    return __builtin_fma(r1, __builtin_fma(-z, r1, 1.0), r1);
}

// Bilinear clamp-to-edge sample of an 8-bit view at the point the
// homography H maps the reference-grid point (qx, qy) to (pixel-centre
// coordinates on both sides).  Every operation is fixed: fused
// multiply-adds for the homography rows, the coordinate shift and the
// interpolation, and one correctly rounded double reciprocal, so the census
// bits that compare these values are reproducible.  Points mapped behind the
// view (hz <= 1e-300) get reciprocal 0 and read the top-left corner.
// Branch-free; result on the 0..255 scale.
__device__ __forceinline__ float warp_sample(const uint8_t *__restrict__ src, int sw, int sh, double h0, double h1,
                                             double h2, double h3, double h4, double h5, double h6, double h7,
                                             double h8, double qx, double qy) {
    const double hx = __builtin_fma(h0, qx, __builtin_fma(h1, qy, h2));
    const double hy = __builtin_fma(h3, qx, __builtin_fma(h4, qy, h5));
    const double hz = __builtin_fma(h6, qx, __builtin_fma(h7, qy, h8));
    const double r = recip(hz);
    const double inv = hz > 1e-300 ? r : 0.0;
    // The coordinate is clamped to [0, size - 1] rather than [-1, size]:
    // outside [0, size - 1] both bilinear neighbours of the clamp-to-edge
    // sample are the same border pixel, so the value is that pixel whatever
    // the fraction, and at the clamped coordinate the fraction is 0 and the
    // left (top) neighbour is that pixel.  With a non-negative coordinate the
    // truncating conversion is the floor.
    double sx = __builtin_fma(hx, inv, -0.5);
    double sy = __builtin_fma(hy, inv, -0.5);
    sx = __builtin_fmin(__builtin_fmax(sx, 0.0), (double)(sw - 1));
    sy = __builtin_fmin(__builtin_fmax(sy, 0.0), (double)(sh - 1));
    const uint32_t xa = (uint32_t)(int)sx, ya = (uint32_t)(int)sy;
    // fraction of a non-negative coordinate: exactly sx - floor(sx) (the
    // fract instruction is correctly rounded and the difference is
    // representable)
    const float ax = (float)__builtin_amdgcn_fract(sx);
    const float ay = (float)__builtin_amdgcn_fract(sy);
    const uint32_t xb = min(xa + 1u, (uint32_t)(sw - 1)), yb = min(ya + 1u, (uint32_t)(sh - 1));
    const uint32_t ra = __umul24(ya, (uint32_t)sw), rb = __umul24(yb, (uint32_t)sw);
    const float i00 = (float)src[ra + xa];
    const float i10 = (float)src[ra + xb];
    const float i01 = (float)src[rb + xa];
    const float i11 = (float)src[rb + xb];
    const float top = __builtin_fmaf(ax, i10 - i00, i00);
    const float bot = __builtin_fmaf(ax, i11 - i01, i01);
    return __builtin_fmaf(ay, bot - top, top);
}

// warp_sample for a reference region whose samples all map in front of the
// view and inside [0, sw - 2] x [0, sh - 2] (warp_region_mode): there the
// reciprocal guard and the border clamps change nothing, so the same
// operations without them give the same value.  The texel offset is clamped
// to the image only as a memory guard.
__device__ __forceinline__ float warp_sample_inside(const uint8_t *__restrict__ src, int sw, int sh, double h0,
                                                    double h1, double h2, double h3, double h4, double h5, double h6,
                                                    double h7, double h8, double qx, double qy) {
    const double hx = __builtin_fma(h0, qx, __builtin_fma(h1, qy, h2));
    const double hy = __builtin_fma(h3, qx, __builtin_fma(h4, qy, h5));
    const double hz = __builtin_fma(h6, qx, __builtin_fma(h7, qy, h8));
    const double r = recip(hz);
    const double sx = __builtin_fma(hx, r, -0.5);
    const double sy = __builtin_fma(hy, r, -0.5);
    const uint32_t xa = (uint32_t)(int)sx, ya = (uint32_t)(int)sy;
    const float ax = (float)__builtin_amdgcn_fract(sx);
    const float ay = (float)__builtin_amdgcn_fract(sy);
    const uint32_t b0 = min(__umul24(ya, (uint32_t)sw) + xa, (uint32_t)(sw * (sh - 1) - 2));
    const uint32_t b1 = b0 + (uint32_t)sw;
    const float i00 = (float)src[b0];
    const float i10 = (float)src[b0 + 1u];
    const float i01 = (float)src[b1];
    const float i11 = (float)src[b1 + 1u];
    const float top = __builtin_fmaf(ax, i10 - i00, i00);
    const float bot = __builtin_fmaf(ax, i11 - i01, i01);
    return __builtin_fmaf(ay, bot - top, top);
}

// Whether every sample of the region with corner sample points (qx_lo..qx_hi)
// x (qy_lo..qy_hi) maps in front of the view and inside [0, sw - 2] x
// [0, sh - 2] (with a 1e-6 px margin for rounding): hz is affine, so a
// region in front of the view maps to the convex quadrilateral of its
// corners' images.  corner selects the corner (bit 0: x, bit 1: y).
__device__ __forceinline__ bool warp_corner_inside(const double *H, int corner, double qx_lo, double qx_hi,
                                                   double qy_lo, double qy_hi, int sw, int sh) {
    const double qx = (corner & 1) ? qx_hi : qx_lo, qy = (corner & 2) ? qy_hi : qy_lo;
    const double hz = H[6] * qx + H[7] * qy + H[8];
    if (!(hz > 1e-200)) return false;
    const double X = (H[0] * qx + H[1] * qy + H[2]) / hz - 0.5;
    const double Y = (H[3] * qx + H[4] * qy + H[5]) / hz - 0.5;
    return X >= 1e-6 && X <= (double)(sw - 2) - 1e-6 && Y >= 1e-6 && Y <= (double)(sh - 2) - 1e-6;
}

// Minimum over the 64 lanes of a wavefront: DPP within each row of 16
// (quad_perm, row_half_mirror, row_mirror), then row_bcast:15 and
// row_bcast:31 carry the row minima up to lane 63, which is read back.
// Every lane must be active.
// Lanes of rows outside ROW_MASK see the identity (all ones), so the
// minimum leaves them unchanged and the move folds into the min as DPP.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_min_step(uint32_t v) {
    const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, CTRL, ROW_MASK, 0xF, false);
    return v < t ? v : t;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = dpp_min_step<0xB1, 0xF>(v);    // quad_perm 1,0,3,2
    v = dpp_min_step<0x4E, 0xF>(v);    // quad_perm 2,3,0,1
    v = dpp_min_step<0x141, 0xF>(v);   // row_half_mirror
    v = dpp_min_step<0x140, 0xF>(v);   // row_mirror: every lane holds its row's minimum
    v = dpp_min_step<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_min_step<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ void ray_of(const double *Ki, double u, double v, double r[3]) {
    r[0] = Ki[0] * u + Ki[1] * v + Ki[2];
    r[1] = Ki[3] * u + Ki[4] * v + Ki[5];
    r[2] = Ki[6] * u + Ki[7] * v + Ki[8];
}

}  // namespace fmvs
