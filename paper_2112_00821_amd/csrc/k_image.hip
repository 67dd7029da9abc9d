// Per-pixel image stages of the FaSS-MVS pipeline on gfx950: pyramid,
// reference census, single-image warp, winner refinement, median, normals
// with appearance-weighted smoothing and confidence, and coarse-to-fine
// seeds.  All are stencils over one level; each thread owns one output pixel.
#include "dev_common.hpp"
#include "kernels.hpp"

namespace fmvs {

// --------------------------------------------------------------- pyramid
// Pipeline overview: 3x3 Gaussian (sigma 1, taps 70/116/70 of 256, rounding
// after each separable pass, replicate border), then the mean of each 2x2
// block -> floor(w/2) x floor(h/2).
__global__ __launch_bounds__(256) void k_pyr_down(const uint8_t *__restrict__ src, int w, int h, int stride,
                                                  uint8_t *__restrict__ dst) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    int w2 = w >> 1, h2 = h >> 1;
    if (x >= w2 || y >= h2) return;
    int cx[4], ry[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        cx[i] = clampi(2 * x - 1 + i, 0, w - 1);
        ry[i] = clampi(2 * y - 1 + i, 0, h - 1);
    }
    int a[4][2];   // horizontal pass at rows 2y-1..2y+2, columns 2x, 2x+1
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint8_t *row = src + (size_t)ry[r] * stride;
        int s0 = row[cx[0]], s1 = row[cx[1]], s2 = row[cx[2]], s3 = row[cx[3]];
        a[r][0] = (70 * s0 + 116 * s1 + 70 * s2 + 128) >> 8;
        a[r][1] = (70 * s1 + 116 * s2 + 70 * s3 + 128) >> 8;
    }
    int s = 0;
#pragma unroll
    for (int r = 1; r <= 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) s += (70 * a[r - 1][c] + 116 * a[r][c] + 70 * a[r + 1][c] + 128) >> 8;
    dst[(size_t)y * w2 + x] = (uint8_t)((s + 2) >> 2);
}

hipError_t launch_pyr_down(const uint8_t *src, int w, int h, int stride, uint8_t *dst, hipStream_t s) {
    dim3 grid(((w >> 1) + 15) / 16, ((h >> 1) + 15) / 16);
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pyr_down, grid, dim3(256), 0, s, src, w, h, stride, dst);
    return hipGetLastError();
}

// --------------------------------------------------------------- census
// Census transform of the reference level (Alg. 1 cost function): bit
// (nbits-1-b) = [I(q_b) < I(p)], q_b the b-th window position in row-major
// order without the centre, replicate border.
__global__ __launch_bounds__(256) void k_census(const uint8_t *__restrict__ img, int w, int h, int cw, int ch,
                                                uint64_t *__restrict__ out) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= w || y >= h) return;
    int rx = cw >> 1, ryy = ch >> 1;
    int c = img[(size_t)y * w + x];
    uint64_t bits = 0;
    for (int dy = -ryy; dy <= ryy; ++dy) {
        const uint8_t *row = img + (size_t)clampi(y + dy, 0, h - 1) * w;
        for (int dx = -rx; dx <= rx; ++dx) {
            if (dx == 0 && dy == 0) continue;
            bits = (bits << 1) | (uint64_t)(row[clampi(x + dx, 0, w - 1)] < c ? 1u : 0u);
        }
    }
    out[(size_t)y * w + x] = bits;
}

hipError_t launch_census(const uint8_t *img, int w, int h, int cw, int ch, uint64_t *out, hipStream_t s) {
    dim3 grid((w + 15) / 16, (h + 15) / 16);
    hipLaunchKernelGGL(k_census, grid, dim3(256), 0, s, img, w, h, cw, ch, out);
    return hipGetLastError();
}

// --------------------------------------------------------------- warp (stage check)
__global__ __launch_bounds__(256) void k_warp(const uint8_t *__restrict__ src, int sw, int sh,
                                              const double *__restrict__ H, int rw, int rh, float *__restrict__ out) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= rw || y >= rh) return;
    out[(size_t)y * rw + x] =
        warp_sample(src, sw, sh, H[0], H[1], H[2], H[3], H[4], H[5], H[6], H[7], H[8], x + 0.5, y + 0.5);
}

hipError_t launch_warp(const uint8_t *src, int sw, int sh, const double *dH, int rw, int rh, float *out,
                       hipStream_t s) {
    dim3 grid((rw + 15) / 16, (rh + 15) / 16);
    hipLaunchKernelGGL(k_warp, grid, dim3(256), 0, s, src, sw, sh, dH, rw, rh, out);
    return hipGetLastError();
}

// --------------------------------------------------------------- refine
// Depth of the winning plane d = -delta / (n^T K^-1 p) (depth extraction for
// SGM^Pi) and parabola through the winner and its neighbours at their
// non-equidistant depths (depth refinement), clamped to the neighbours'
// interval; no refinement at a window end or for a parabola that does not
// open upwards.  Double precision, the same operation order as the
// definition it restates.
__global__ __launch_bounds__(256) void k_refine(const RefineArgs a) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= a.w || y >= a.h) return;
    size_t p = (size_t)y * a.w + x;
    size_t N = (size_t)a.w * a.h;
    int best = a.wta[p];
    const int D = a.foff[a.n_fam - 1] + a.W[a.n_fam - 1];
    if (best >= D) {   // not a label of this level: no depth
        a.fam[p] = 0;
        a.label[p] = -1;
        a.depth[p] = 0.0f;
        return;
    }
    int f = 0;
    while (f + 1 < a.n_fam && best >= a.foff[f + 1]) ++f;
    int li = best - a.foff[f];
    int o = a.offs ? a.offs[(size_t)f * N + p] : 0;
    int g = o + li;
    const double *dl = a.delta + a.goff[f];
    double r[3];
    ray_of(a.Kinv, x + 0.5, y + 0.5, r);
    double den = a.fam_n[f][0] * r[0] + a.fam_n[f][1] * r[1] + a.fam_n[f][2] * r[2];
    a.fam[p] = f;
    if (!(den < 0.0)) {
        a.label[p] = -1;
        a.depth[p] = 0.0f;
        return;
    }
    double d0 = -dl[g] / den;
    a.label[p] = a.goff[f] + g;
    double d = d0;
    if (li >= 1 && li + 1 < a.W[f]) {
        double dm = -dl[g - 1] / den;
        double dp = -dl[g + 1] / den;
        double aa = dm - d0, bb = dp - d0;
        const uint16_t *c = a.c3 + 3 * p;
        double u = (double)c[0] - (double)c[1];
        double v = (double)c[2] - (double)c[1];
        double sa = u / aa, sb = v / bb;
        double alpha = (sa - sb) / (aa - bb);
        if (alpha > 0.0) {
            double beta = sa - alpha * aa;
            double xv = -beta / (2.0 * alpha);
            d = d0 + xv;
            double lo = fmin(dm, dp), hi = fmax(dm, dp);
            d = fmin(fmax(d, lo), hi);
        }
    }
    a.depth[p] = (float)d;
}

hipError_t launch_refine(const RefineArgs &a, hipStream_t s) {
    dim3 grid((a.w + 15) / 16, (a.h + 15) / 16);
    hipLaunchKernelGGL(k_refine, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------- median
// 5x5 median (pipeline overview): replicate border, the 13th smallest of the
// 25 samples, by a bitonic sorting network over 32 registers.
__global__ __launch_bounds__(256) void k_median5(const float *__restrict__ in, int w, int h, float *__restrict__ out) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= w || y >= h) return;
    float v[32];
#pragma unroll
    for (int dy = 0; dy < 5; ++dy) {
        const float *row = in + (size_t)clampi(y + dy - 2, 0, h - 1) * w;
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) v[dy * 5 + dx] = row[clampi(x + dx - 2, 0, w - 1)];
    }
#pragma unroll
    for (int i = 25; i < 32; ++i) v[i] = __int_as_float(0x7f800000);
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                int l = i ^ j;
                if (l > i) {
                    float lo = fminf(v[i], v[l]), hi = fmaxf(v[i], v[l]);
                    if ((i & k) == 0) { v[i] = lo; v[l] = hi; }
                    else { v[i] = hi; v[l] = lo; }
                }
            }
    out[(size_t)y * w + x] = v[12];
}

hipError_t launch_median5(const float *in, int w, int h, float *out, hipStream_t s) {
    dim3 grid((w + 15) / 16, (h + 15) / 16);
    hipLaunchKernelGGL(k_median5, grid, dim3(256), 0, s, in, w, h, out);
    return hipGetLastError();
}

// --------------------------------------------------------------- normals
// Sec. extraction of surface normals: back-projected neighbours, n = h x v
// (central differences, one-sided at the border), oriented toward the
// camera, normalised; zero where a used depth is missing.
__global__ __launch_bounds__(256) void k_normals_raw(const NormalArgs a) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= a.w || y >= a.h) return;
    size_t p = (size_t)y * a.w + x;
    float *o = a.nraw + 3 * p;
    o[0] = o[1] = o[2] = 0.0f;
    auto P = [&](int xx, int yy, double X[3]) {
        double r[3];
        ray_of(a.Kinv, xx + 0.5, yy + 0.5, r);
        double d = a.depth[(size_t)yy * a.w + xx];
        X[0] = d * r[0];
        X[1] = d * r[1];
        X[2] = d * r[2];
        return d > 0.0;
    };
    double Xp[3], A[3], B[3], Cc[3], Dd[3];
    if (a.w < 2 || a.h < 2 || !P(x, y, Xp)) return;
    int xa = x > 0 ? x - 1 : x, xb = x + 1 < a.w ? x + 1 : x;
    int ya = y > 0 ? y - 1 : y, yb = y + 1 < a.h ? y + 1 : y;
    if (!P(xa, y, A) || !P(xb, y, B) || !P(x, ya, Cc) || !P(x, yb, Dd)) return;
    double hv[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double vv[3] = {Dd[0] - Cc[0], Dd[1] - Cc[1], Dd[2] - Cc[2]};
    double n[3] = {hv[1] * vv[2] - hv[2] * vv[1], hv[2] * vv[0] - hv[0] * vv[2], hv[0] * vv[1] - hv[1] * vv[0]};
    if (n[0] * Xp[0] + n[1] * Xp[1] + n[2] * Xp[2] > 0.0) {
        n[0] = -n[0];
        n[1] = -n[1];
        n[2] = -n[2];
    }
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(len > 0.0)) return;
    o[0] = (float)(n[0] / len);
    o[1] = (float)(n[1] / len);
    o[2] = (float)(n[2] / len);
}

// Eq. normal / normal-smooth: n_p plus every valid neighbour q != p of the
// (2r+1)^2 window inside the image, weighted by
// exp(-|q-p|^2/(2 sigma^2) - |I(p)-I(q)|/beta) / sqrt(2 pi sigma^2), sigma = r;
// then Eq. weight-normal for the confidence (both angles within rho).
__global__ __launch_bounds__(256) void k_smooth_conf(const NormalArgs a) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= a.w || y >= a.h) return;
    size_t p = (size_t)y * a.w + x;
    const float *np_ = a.nraw + 3 * p;
    float *o = a.normal + 3 * p;
    o[0] = o[1] = o[2] = 0.0f;
    a.conf[p] = 0.0f;
    if (np_[0] == 0.0f && np_[1] == 0.0f && np_[2] == 0.0f) return;
    double acc[3] = {np_[0], np_[1], np_[2]};
    const int Ip = a.img[p];
    for (int dy = -a.radius; dy <= a.radius; ++dy)
        for (int dx = -a.radius; dx <= a.radius; ++dx) {
            if (dx == 0 && dy == 0) continue;
            int xx = x + dx, yy = y + dy;
            if (xx < 0 || xx >= a.w || yy < 0 || yy >= a.h) continue;
            size_t q = (size_t)yy * a.w + xx;
            const float *nq = a.nraw + 3 * q;
            // the weight of Eq. normal-smooth for this offset and intensity
            // difference, from the table
            const double wq = a.wtab[(dx * dx + dy * dy) * 256 + abs(Ip - (int)a.img[q])];
            acc[0] += wq * nq[0];
            acc[1] += wq * nq[1];
            acc[2] += wq * nq[2];
        }
    double len = sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
    if (!(len > 0.0)) return;
    float n0 = (float)(acc[0] / len), n1 = (float)(acc[1] / len), n2 = (float)(acc[2] / len);
    o[0] = n0;
    o[1] = n1;
    o[2] = n2;
    if (a.label[p] < 0) return;
    const double *m = a.fam_n[a.fam[p]];
    double c1 = (double)n0 * m[0] + (double)n1 * m[1] + (double)n2 * m[2];
    double c2 = -m[2];
    if (!(c1 >= a.cos_rho && c2 >= a.cos_rho)) return;
    double c = (c1 * c2 - a.cos_rho) / (1.0 - a.cos_rho);
    a.conf[p] = (float)fmin(fmax(c, 0.0), 1.0);
}

hipError_t launch_normals(const NormalArgs &a, hipStream_t s) {
    dim3 grid((a.w + 15) / 16, (a.h + 15) / 16);
    hipLaunchKernelGGL(k_normals_raw, grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_conf, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------- seeds
// Continuous index of the inverse distance iv in a plane list of G >= 2
// planes given by their inverse distances inv[0..G-1] (decreasing): the
// interval start i is the last one in [0, G-2] whose plane's inverse
// distance is >= iv (0 if none) -- from a guess by the list's mean spacing
// (rspan = (G - 1) / (inv[0] - inv[G-1])) and the few steps to it -- then
// the linear position inside that interval (end intervals extended beyond
// the list).
__device__ double list_index(const double *__restrict__ inv, int G, double rspan, double iv) {
    const double gd = fmin(fmax((inv[0] - iv) * rspan, 0.0), (double)(G - 2));
    int i = (int)gd;
    while (i < G - 2 && inv[i + 1] >= iv) ++i;
    while (i > 0 && inv[i] < iv) --i;
    const double a = inv[i], b = inv[i + 1];
    return (double)i + (a - iv) / (a - b);
}

// Coarse-to-fine initialisation: nearest-neighbour upsampling of depth and
// normal (fine (x,y) <- coarse (min(x/2, cw-1), min(y/2, ch-1))), the
// per-family sampling windows centred on the plane through the seed depth
// (Eq. sampling_range, dynamic cost volume) -- its rounded continuous index
// in the level's list -- and the surface-normal index offsets of
// Eq. sgm-smooth-sn toward each path predecessor q = p - r, as differences
// of continuous indices.
__global__ __launch_bounds__(256) void k_seed(const SeedArgs a) {
    int x = blockIdx.x * 16 + (threadIdx.x & 15);
    int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= a.fw || y >= a.fh) return;
    size_t p = (size_t)y * a.fw + x;
    size_t N = (size_t)a.fw * a.fh;
    size_t pc = (size_t)min(y >> 1, a.ch - 1) * a.cw + min(x >> 1, a.cw - 1);
    float dbf = a.depth_c[pc];
    float nb0 = a.normal_c[3 * pc], nb1 = a.normal_c[3 * pc + 1], nb2 = a.normal_c[3 * pc + 2];
    a.dbar[p] = dbf;
    a.nbar[3 * p] = nb0;
    a.nbar[3 * p + 1] = nb1;
    a.nbar[3 * p + 2] = nb2;
    double rp[3];
    ray_of(a.Kinv, x + 0.5, y + 0.5, rp);
    double d = dbf;
    double rspan[kMaxFam], jp[kMaxFam];
    for (int f = 0; f < a.n_fam; ++f) {
        const double *inv = a.inv + a.goff[f];
        rspan[f] = (double)(a.G[f] - 1) / (inv[0] - inv[a.G[f] - 1]);
        const double *n = a.fam_n[f];
        double c = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
        int o;
        jp[f] = 0.0;
        if (!(d > 0.0) || !(c > 0.0)) {
            o = (a.G[f] - a.W[f]) / 2;
        } else {
            double delta = d * c;
            double j = list_index(inv, a.G[f], rspan[f], 1.0 / delta);
            j = fmin(fmax(j, -1.0e6), 1.0e6);
            int jr = (int)floor(j + 0.5);
            o = clampi(jr - a.W[f] / 2, 0, a.G[f] - a.W[f]);
        }
        a.offs[(size_t)f * N + p] = o;
    }
    if (!a.dI) return;
    for (int r = 0; r < 8; ++r)
        for (int f = 0; f < a.n_fam; ++f) a.dI[((size_t)r * N + p) * a.n_fam + f] = 0;
    double nb[3] = {nb0, nb1, nb2};
    if (!(d > 0.0) || (nb[0] == 0.0 && nb[1] == 0.0 && nb[2] == 0.0)) return;
    double kP = nb[0] * (d * rp[0]) + nb[1] * (d * rp[1]) + nb[2] * (d * rp[2]);
    // the seed point's continuous index per family (the same for every path)
    for (int f = 0; f < a.n_fam; ++f) {
        const double *n = a.fam_n[f];
        const double cp = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
        if (cp > 0.0) jp[f] = list_index(a.inv + a.goff[f], a.G[f], rspan[f], 1.0 / (d * cp));
    }
    for (int r = 0; r < 8; ++r) {
        double rq[3];
        ray_of(a.Kinv, (x - dir_dx(r)) + 0.5, (y - dir_dy(r)) + 0.5, rq);
        double den = nb[0] * rq[0] + nb[1] * rq[1] + nb[2] * rq[2];
        if (!(fabs(den) > 1e-12)) continue;
        double dT = kP / den;
        if (!(dT > 0.0)) continue;
        for (int f = 0; f < a.n_fam; ++f) {
            const double *n = a.fam_n[f];
            double cp = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
            double cq = -(n[0] * rq[0] + n[1] * rq[1] + n[2] * rq[2]);
            if (!(cp > 0.0) || !(cq > 0.0)) continue;
            double iq = 1.0 / (dT * cq);
            double v = list_index(a.inv + a.goff[f], a.G[f], rspan[f], iq) - jp[f];
            v = fmin(fmax(v, -7.0), 7.0);
            a.dI[((size_t)r * N + p) * a.n_fam + f] = (int8_t)round(v);
        }
    }
}

hipError_t launch_seed(const SeedArgs &a, hipStream_t s) {
    dim3 grid((a.fw + 15) / 16, (a.fh + 15) / 16);
    hipLaunchKernelGGL(k_seed, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------- sum of path costs
__global__ __launch_bounds__(256) void k_sum_u16(const uint16_t *b0, const uint16_t *b1, const uint16_t *b2,
                                                 const uint16_t *b3, const uint16_t *b4, const uint16_t *b5,
                                                 const uint16_t *b6, const uint16_t *b7, int n, size_t count,
                                                 uint16_t *out) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const uint16_t *b[8] = {b0, b1, b2, b3, b4, b5, b6, b7};
    uint32_t s = 0;
    for (int k = 0; k < n; ++k) s += b[k][i];
    out[i] = (uint16_t)s;
}

hipError_t launch_sum_u16(const uint16_t *const *bufs, int n, size_t count, uint16_t *out, hipStream_t s) {
    const uint16_t *b[8] = {};
    for (int i = 0; i < n && i < 8; ++i) b[i] = bufs[i];
    size_t blocks = (count + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_u16, dim3((unsigned)blocks), dim3(256), 0, s, b[0], b[1], b[2], b[3], b[4], b[5], b[6],
                       b[7], n, count, out);
    return hipGetLastError();
}

}  // namespace fmvs
