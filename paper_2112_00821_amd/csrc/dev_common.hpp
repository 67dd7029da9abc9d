// Device helpers shared by the gfx950 kernels of the FaSS-MVS library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmvs {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bilinear clamp-to-edge sample of an 8-bit view at the point the
// homography H maps the reference-grid point (qx, qy) to (pixel-centre
// coordinates on both sides).  The projective division runs in double; the
// interpolation in float with a fixed operation order, so the census bits
// that compare these values are reproducible.  Points mapped behind the
// view (hz <= 0) read the top-left corner.  Result on the 0..255 scale.
__device__ __forceinline__ float warp_sample(const uint8_t *__restrict__ src, int sw, int sh, double h0, double h1,
                                             double h2, double h3, double h4, double h5, double h6, double h7,
                                             double h8, double qx, double qy) {
    double hx = h0 * qx + h1 * qy + h2;
    double hy = h3 * qx + h4 * qy + h5;
    double hz = h6 * qx + h7 * qy + h8;
    double sx, sy;
    if (hz > 0.0) {
        double inv = 1.0 / hz;
        sx = hx * inv - 0.5;
        sy = hy * inv - 0.5;
    } else {
        sx = -1.0;
        sy = -1.0;
    }
    sx = fmin(fmax(sx, -1.0), (double)sw);
    sy = fmin(fmax(sy, -1.0), (double)sh);
    double fx0 = floor(sx);
    double fy0 = floor(sy);
    int x0 = (int)fx0, y0 = (int)fy0;
    float ax = (float)(sx - fx0);
    float ay = (float)(sy - fy0);
    int xa = clampi(x0, 0, sw - 1), xb = clampi(x0 + 1, 0, sw - 1);
    int ya = clampi(y0, 0, sh - 1), yb = clampi(y0 + 1, 0, sh - 1);
    const uint8_t *ra = src + (size_t)ya * sw;
    const uint8_t *rb = src + (size_t)yb * sw;
    float i00 = (float)ra[xa];
    float i10 = (float)ra[xb];
    float i01 = (float)rb[xa];
    float i11 = (float)rb[xb];
    float top = i00 + ax * (i10 - i00);
    float bot = i01 + ax * (i11 - i01);
    return top + ay * (bot - top);
}

// Minimum over the 64 lanes of a wavefront: DPP within each row of 16, then
// the four row results through readlane.  Every lane must be active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    v = v < t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    v = v < t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v = v < t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    v = v < t ? v : t;
    uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    a = a < b ? a : b;
    c = c < d ? c : d;
    return a < c ? a : c;
}

__device__ __forceinline__ void ray_of(const double *Ki, double u, double v, double r[3]) {
    r[0] = Ki[0] * u + Ki[1] * v + Ki[2];
    r[1] = Ki[3] * u + Ki[4] * v + Ki[5];
    r[2] = Ki[6] * u + Ki[7] * v + Ki[8];
}

}  // namespace fmvs
