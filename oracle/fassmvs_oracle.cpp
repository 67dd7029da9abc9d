// FaSS-MVS CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded C++ restatement of the FaSS-MVS hot path
// (Ruf, Weinmann, Hinz: "FaSS-MVS -- Fast Multi-View Stereo with
// Surface-Aware Semi-Global Matching from UAV-borne Monocular Imagery").
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may
// load it.  It shares no code, header or table with the GPU library.
//
// Precision: geometry in double.  Where a floating-point value decides an
// integer result (the census bits decided by warped intensities) the value
// is computed in the same precision the GPU kernel uses: sample coordinates
// in double, bilinear interpolation in float, every operation spelled out
// (explicit fused multiply-adds through std::fma where the definition has
// them).  Built with -ffp-contract=off so that the compiler fuses nothing
// else.
//
// Conventions (readings of passages the paper leaves open):
//  * pixel (x, y) has its centre at (x+0.5, y+0.5) in the coordinates K maps
//    camera rays to; level l uses K with fx, skew, cx, fy, cy scaled by 2^-l.
//  * plane (n, delta): { X : n^T X + delta = 0 } in reference-camera
//    coordinates, n unit and facing the camera.
//  * [R|t] maps reference-camera coordinates to view-k camera coordinates.
//  * census bit order: the b-th window position in row-major order (centre
//    skipped) lands in bit (nbits-1-b); bit = [W(q) < W(p)] (strict).
//
// Parity status: every function here is pinned by the CPU test-suite
// (closed forms, brute force, library routines on special cases,
// invariants, ground-truth recovery); the normal smoothing through its
// fixed points, a two-pixel weight ratio and, on flat intensity, a Gaussian
// correlation; the confidence through closed forms.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------------------
// Warped sample (Alg. 1, patch warping by the plane-induced homography).
// The reference-grid point (qx, qy) (pixel-centre coordinates) maps through H
// to (hx/hz, hy/hz) in the view's pixel-centre coordinates; the view is
// sampled bilinearly with clamp-to-edge addressing.  The paper fixes no
// rounding; this definition fixes every operation (fused multiply-adds for
// the homography rows, the coordinate shift and the interpolation, one
// correctly rounded reciprocal) so that a census bit taken from the sample
// is reproducible.  Points that map behind (or onto the focal plane of) the
// view camera, hz <= 1e-300, get reciprocal 0, which lands them on the
// top-left corner; the threshold keeps the reciprocal finite.  Clamping the
// coordinate to [-1, size] leaves the clamp-to-edge bilinear value unchanged
// and keeps every index finite.  Intensities stay on the 0..255 scale.
// ---------------------------------------------------------------------------
float warp_sample(const uint8_t* src, int sw, int sh, const double* H, double qx, double qy) {
    double hx = std::fma(H[0], qx, std::fma(H[1], qy, H[2]));
    double hy = std::fma(H[3], qx, std::fma(H[4], qy, H[5]));
    double hz = std::fma(H[6], qx, std::fma(H[7], qy, H[8]));
    double inv = hz > 1e-300 ? 1.0 / hz : 0.0;
    double sx = std::fma(hx, inv, -0.5);
    double sy = std::fma(hy, inv, -0.5);
    sx = std::min(std::max(sx, -1.0), (double)sw);
    sy = std::min(std::max(sy, -1.0), (double)sh);
    double fx0 = std::floor(sx);
    double fy0 = std::floor(sy);
    int x0 = (int)fx0, y0 = (int)fy0;
    float ax = (float)(sx - fx0);
    float ay = (float)(sy - fy0);
    int xa = clampi(x0, 0, sw - 1), xb = clampi(x0 + 1, 0, sw - 1);
    int ya = clampi(y0, 0, sh - 1), yb = clampi(y0 + 1, 0, sh - 1);
    float i00 = (float)src[(size_t)ya * sw + xa];
    float i10 = (float)src[(size_t)ya * sw + xb];
    float i01 = (float)src[(size_t)yb * sw + xa];
    float i11 = (float)src[(size_t)yb * sw + xb];
    float top = std::fma(ax, i10 - i00, i00);
    float bot = std::fma(ax, i11 - i01, i01);
    return std::fma(ay, bot - top, top);
}

// census word of a float image at (x, y), window cw x ch (odd), replicate border
uint64_t census_at(const float* img, int w, int h, int x, int y, int cw, int ch) {
    int rx = cw / 2, ry = ch / 2;
    float c = img[(size_t)y * w + x];
    uint64_t bits = 0;
    for (int dy = -ry; dy <= ry; ++dy)
        for (int dx = -rx; dx <= rx; ++dx) {
            if (dx == 0 && dy == 0) continue;
            int xx = clampi(x + dx, 0, w - 1), yy = clampi(y + dy, 0, h - 1);
            bits = (bits << 1) | (uint64_t)(img[(size_t)yy * w + xx] < c ? 1 : 0);
        }
    return bits;
}

inline int popcount64(uint64_t v) {
    int n = 0;
    while (v) { v &= v - 1; ++n; }
    return n;
}

// S = min over the non-empty subsets X in {L, R} of floor(s^X * m / |X|),
// m = max(|L|, |R|) (Alg. 1, occlusion-robust minimum of the left/right sums;
// equals min(s^L, s^R) for equal subset sizes).
inline int combine_lr(long sL, long sR, int nL, int nR) {
    int m = std::max(nL, nR);
    long best = -1;
    if (nL > 0) best = (sL * m) / nL;
    if (nR > 0) {
        long v = (sR * m) / nR;
        best = best < 0 ? v : std::min(best, v);
    }
    return (int)best;
}

// S for the NCC cost: min over the non-empty subsets X of floor(s^X / |X|),
// the mean cost of a subset, which stays on the 0..255 scale of one view
// (the paper normalises the NCC cost's maximum to 255).
inline int combine_mean(long sL, long sR, int nL, int nR) {
    long best = -1;
    if (nL > 0) best = sL / nL;
    if (nR > 0) {
        long v = sR / nR;
        best = best < 0 ? v : std::min(best, v);
    }
    return (int)best;
}

// Negated, truncated and scaled normalised cross-correlation of two cw x ch
// windows a (reference, integer intensities) and b (warped view), both
// row-major (matching cost of Alg. 1 with the NCC similarity).  Sums run
// along each row left to right, then over the rows top to bottom, in
// double; products are fused multiply-adds:
//   n = cw*ch, vA = n*sAA - sA*sA, vB = n*sBB - sB*sB, cov = n*sAB - sA*sB,
//   rho = cov / sqrt(vA * vB)  (0 when vA or vB is not positive),
//   clamped to [-1, 1];  C = floor(255 * min(1, 1 - rho) + 0.5).
// A flat window therefore costs 255, and anti-correlation is truncated at
// the same maximum.
inline int ncc_cost(const uint8_t* a, const float* b, int cw, int ch) {
    double sA = 0, sAA = 0, sB = 0, sBB = 0, sAB = 0;
    for (int y = 0; y < ch; ++y) {
        double rA = 0, rAA = 0, rB = 0, rBB = 0, rAB = 0;
        for (int x = 0; x < cw; ++x) {
            const double va = a[y * cw + x];
            const double vb = b[y * cw + x];
            if (x == 0) {
                rA = va; rAA = va * va; rB = vb; rBB = vb * vb; rAB = va * vb;
            } else {
                rA = rA + va; rAA = std::fma(va, va, rAA);
                rB = rB + vb; rBB = std::fma(vb, vb, rBB); rAB = std::fma(va, vb, rAB);
            }
        }
        if (y == 0) {
            sA = rA; sAA = rAA; sB = rB; sBB = rBB; sAB = rAB;
        } else {
            sA = sA + rA; sAA = sAA + rAA; sB = sB + rB; sBB = sBB + rBB; sAB = sAB + rAB;
        }
    }
    const double n = (double)(cw * ch);
    const double vA = n * sAA - sA * sA;
    const double vB = n * sBB - sB * sB;
    const double cov = n * sAB - sA * sB;
    double rho = 0.0;
    if (vA > 0.0 && vB > 0.0) rho = cov / std::sqrt(vA * vB);
    rho = std::min(1.0, std::max(-1.0, rho));
    const double c = std::min(1.0, 1.0 - rho);
    return (int)std::floor(255.0 * c + 0.5);
}

inline void ray_of(const double* Ki, double u, double v, double r[3]) {
    r[0] = Ki[0] * u + Ki[1] * v + Ki[2];
    r[1] = Ki[3] * u + Ki[4] * v + Ki[5];
    r[2] = Ki[6] * u + Ki[7] * v + Ki[8];
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Setup geometry (Sec. "Materials and Methods", processing pipeline and
// plane-sweep subsections).
// ---------------------------------------------------------------------------

// Inverse of the upper-triangular intrinsic matrix at pyramid level l, whose
// focal lengths, skew and principal point are scaled by 2^-l (pipeline
// overview: the calibration is halved per level).  Closed form of the inverse.
int or_kinv_level(const double* K, int level, double* Kinv, double* Kl) {
    if (K[3] != 0.0 || K[6] != 0.0 || K[7] != 0.0 || K[8] != 1.0) return -1;
    double sc = std::ldexp(1.0, -level);
    double fx = K[0] * sc, s = K[1] * sc, cx = K[2] * sc, fy = K[4] * sc, cy = K[5] * sc;
    if (!(fx != 0.0) || !(fy != 0.0)) return -1;
    Kinv[0] = 1.0 / fx;
    Kinv[1] = -s / (fx * fy);
    Kinv[2] = (s * cy - cx * fy) / (fx * fy);
    Kinv[3] = 0.0;
    Kinv[4] = 1.0 / fy;
    Kinv[5] = -cy / fy;
    Kinv[6] = 0.0;
    Kinv[7] = 0.0;
    Kinv[8] = 1.0;
    if (Kl) {
        Kl[0] = fx; Kl[1] = s; Kl[2] = cx;
        Kl[3] = 0.0; Kl[4] = fy; Kl[5] = cy;
        Kl[6] = 0.0; Kl[7] = 0.0; Kl[8] = 1.0;
    }
    return 0;
}

// Relative transformation of view k with respect to the reference camera:
// R = R_k R_ref^T, t = t_k - R t_ref, mapping reference-camera coordinates to
// view-k camera coordinates (Eq. homography; poses P = K[R|t]).
void or_relative_pose(const double* Rref, const double* tref, const double* Rk, const double* tk,
                      double* R, double* t) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Rk[i * 3 + k] * Rref[j * 3 + k];
            R[i * 3 + j] = s;
        }
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) s += R[i * 3 + j] * tref[j];
        t[i] = tk[i] - s;
    }
}

// Plane-induced homography H = K (R - t n^T / delta) K^-1 for the plane
// n^T X + delta = 0 (Eq. homography; reading of the garbled fraction).
void or_homography(const double* K, const double* Kinv, const double* R, const double* t,
                   const double* n, double delta, double* H) {
    double M[9], A[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i * 3 + j] = R[i * 3 + j] - t[i] * n[j] / delta;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += K[i * 3 + k] * M[k * 3 + j];
            A[i * 3 + j] = s;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * Kinv[k * 3 + j];
            H[i * 3 + j] = s;
        }
}

// Plane distances of one family at one level: G planes uniform in inverse
// distance between delta_min (index 0) and delta_max (index G-1).  Finer
// levels use more planes over the same range (reading of the per-level plane
// list with a per-pixel sampling range).
void or_plane_list(double delta_min, double delta_max, int G, double* delta) {
    double a = 1.0 / delta_min;
    double step = G > 1 ? (a - 1.0 / delta_max) / (double)(G - 1) : 0.0;
    for (int j = 0; j < G; ++j) delta[j] = 1.0 / (a - (double)j * step);
}

// Plane list of a finer level from the coarsest level's list top[0..Gt-1]
// (increasing distances): Gl planes at the fractional indices
// u_j = j (Gt - 1) / (Gl - 1) of the coarsest list, the inverse distance
// interpolated linearly between the two neighbouring coarsest planes (a
// plane at a whole index keeps its distance).  A list uniform in inverse
// distance stays uniform; any other list keeps its spacing profile with
// Gl / Gt times as many planes (reading of the per-level plane list with a
// per-pixel sampling range, extended to the paper's lists of varying
// distances).  Gl < Gt resamples a list down.  Returns -1 on bad sizes.
int or_level_list(const double* top, int Gt, int Gl, double* out) {
    if (Gt < 2 || Gl < 2) return -1;
    for (int j = 0; j < Gl; ++j) {
        long num = (long)j * (Gt - 1);
        long i = num / (Gl - 1);
        long rem = num - i * (Gl - 1);
        if (rem == 0) {
            out[j] = top[i];
        } else {
            double f = (double)rem / (double)(Gl - 1);
            double a = 1.0 / top[i], b = 1.0 / top[i + 1];
            out[j] = 1.0 / (a + f * (b - a));
        }
    }
    return 0;
}

// Continuous index of the inverse distance iv in a plane list delta[0..G-1]
// (increasing distances, so decreasing inverse distances): on the interval
// between planes i and i+1 whose inverse distances enclose iv,
// j = i + (1/delta_i - iv) / (1/delta_i - 1/delta_{i+1}); beyond the ends the
// end interval is extended.  For a list uniform in inverse distance this is
// (1/delta_0 - iv) / step.  The interval is found by a plain scan.
double or_list_index(const double* delta, int G, double iv) {
    int i = 0;
    while (i + 2 < G && 1.0 / delta[i + 1] >= iv) ++i;
    double a = 1.0 / delta[i], b = 1.0 / delta[i + 1];
    return (double)i + (a - iv) / (a - b);
}

// Depth of pixel (x, y) on plane (n, delta): d = -delta / (n^T K^-1 p)
// (depth extraction for SGM^Pi).  Returns 0 when the ray does not meet the
// plane in front of the camera.
double or_depth_on_plane(const double* Kinv, const double* n, double delta, int x, int y) {
    double r[3];
    ray_of(Kinv, x + 0.5, y + 0.5, r);
    double den = n[0] * r[0] + n[1] * r[1] + n[2] * r[2];
    if (!(den < 0.0)) return 0.0;
    return -delta / den;
}

// Adaptive second penalty P2 = P1 (1 + alpha exp(-dI / beta)) tabulated for
// dI = 0..255, rounded half up (Eq. p2-grad); mode 0 gives a constant P2.
void or_p2_lut(int p1, int mode, int p2_fixed, double alpha, double beta, int32_t* lut) {
    for (int i = 0; i < 256; ++i) {
        if (mode == 0)
            lut[i] = p2_fixed;
        else
            lut[i] = (int32_t)std::floor((double)p1 * (1.0 + alpha * std::exp(-(double)i / beta)) + 0.5);
    }
}

// ---------------------------------------------------------------------------
// Gaussian pyramid (pipeline overview: 3x3 Gaussian with sigma = 1, then
// scaling by 0.5).  Reading: separable taps (70,116,70)/256 with replicate
// border and rounding after each pass, then the mean of each 2x2 block, so
// that the halved calibration matches the pixel-centre convention exactly.
// ---------------------------------------------------------------------------
int or_pyr_down(const uint8_t* src, int w, int h, uint8_t* dst) {
    if (w < 2 || h < 2) return -1;
    std::vector<int> a((size_t)w * h), b((size_t)w * h);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int s = 70 * src[(size_t)y * w + clampi(x - 1, 0, w - 1)] + 116 * src[(size_t)y * w + x] +
                    70 * src[(size_t)y * w + clampi(x + 1, 0, w - 1)];
            a[(size_t)y * w + x] = (s + 128) >> 8;
        }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int s = 70 * a[(size_t)clampi(y - 1, 0, h - 1) * w + x] + 116 * a[(size_t)y * w + x] +
                    70 * a[(size_t)clampi(y + 1, 0, h - 1) * w + x];
            b[(size_t)y * w + x] = (s + 128) >> 8;
        }
    int w2 = w / 2, h2 = h / 2;
    for (int y = 0; y < h2; ++y)
        for (int x = 0; x < w2; ++x) {
            int s = b[(size_t)(2 * y) * w + 2 * x] + b[(size_t)(2 * y) * w + 2 * x + 1] +
                    b[(size_t)(2 * y + 1) * w + 2 * x] + b[(size_t)(2 * y + 1) * w + 2 * x + 1];
            dst[(size_t)y * w2 + x] = (uint8_t)((s + 2) >> 2);
        }
    return 0;
}

// ---------------------------------------------------------------------------
// Warping (Alg. 1): the view warped onto the reference grid for one plane.
// ---------------------------------------------------------------------------
void or_warp(const uint8_t* src, int sw, int sh, const double* H, int rw, int rh, float* dst) {
    for (int y = 0; y < rh; ++y)
        for (int x = 0; x < rw; ++x) dst[(size_t)y * rw + x] = warp_sample(src, sw, sh, H, x + 0.5, y + 0.5);
}

// Census transform (Zabih-Woodfill) of a float image; cw x ch window.
int or_census(const float* img, int w, int h, int cw, int ch, uint64_t* out) {
    if ((cw & 1) == 0 || (ch & 1) == 0 || cw * ch - 1 > 64) return -1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) out[(size_t)y * w + x] = census_at(img, w, h, x, y, cw, ch);
    return 0;
}

int or_census_u8(const uint8_t* img, int w, int h, int cw, int ch, uint64_t* out) {
    std::vector<float> f((size_t)w * h);
    for (size_t i = 0; i < f.size(); ++i) f[i] = (float)img[i];
    return or_census(f.data(), w, h, cw, ch, out);
}

// ---------------------------------------------------------------------------
// Cost volume (Alg. 1): for each reference pixel p and plane label, the
// Hamming distance between the reference census and the census of every
// warped view, summed over the left and right subsets, then the
// occlusion-robust minimum.  Labels are the concatenation of the plane
// families; family f contributes W[f] labels per pixel starting at global
// plane index offs[f][p] (the per-pixel sampling window of the dynamic cost
// volume) or all of its G[f] planes when offs is NULL.
//   H: [n_views][sum_f G[f]][9] homographies, family-major global labels.
//   S: [h][w][sum_f W[f]] uint8.
// Returns 0, or -2 if a cost does not fit in 8 bits.
// ---------------------------------------------------------------------------
int or_cost_volume(int w, int h, const uint64_t* ct_ref, int n_views, const uint8_t* const* views,
                   const int8_t* side, int cw, int ch, int n_fam, const int* G, const int* W,
                   const double* H, const int32_t* offs, uint8_t* S) {
    int D = 0, sumG = 0;
    std::vector<int> foff(n_fam), goff(n_fam);
    for (int f = 0; f < n_fam; ++f) {
        foff[f] = D; goff[f] = sumG;
        D += W[f]; sumG += G[f];
        if (!offs && W[f] != G[f]) return -1;
    }
    int nL = 0, nR = 0;
    for (int k = 0; k < n_views; ++k) (side[k] < 0 ? nL : nR)++;
    size_t N = (size_t)w * h;
    std::vector<int32_t> sL(N * D, 0), sR(N * D, 0);
    std::vector<float> warped(N);
    std::vector<uint64_t> ct(N);
    for (int k = 0; k < n_views; ++k)
        for (int f = 0; f < n_fam; ++f)
            for (int g = 0; g < G[f]; ++g) {
                bool needed = false;
                for (size_t p = 0; p < N && !needed; ++p) {
                    int o = offs ? offs[(size_t)f * N + p] : 0;
                    needed = g >= o && g < o + W[f];
                }
                if (!needed) continue;
                const double* Hk = H + ((size_t)k * sumG + goff[f] + g) * 9;
                or_warp(views[k], w, h, Hk, w, h, warped.data());
                or_census(warped.data(), w, h, cw, ch, ct.data());
                for (size_t p = 0; p < N; ++p) {
                    int o = offs ? offs[(size_t)f * N + p] : 0;
                    if (g < o || g >= o + W[f]) continue;
                    int c = popcount64(ct_ref[p] ^ ct[p]);
                    size_t idx = p * D + foff[f] + (g - o);
                    if (side[k] < 0) sL[idx] += c; else sR[idx] += c;
                }
            }
    for (size_t i = 0; i < N * (size_t)D; ++i) {
        int v = combine_lr(sL[i], sR[i], nL, nR);
        if (v > 255) return -2;
        S[i] = (uint8_t)v;
    }
    return 0;
}

// One entry of the cost volume, computed on its own: the census windows of
// the warped views are sampled directly at pixel (x, y) for global plane g
// of family f.  Same definition as or_cost_volume.
int or_cost_sample(int w, int h, const uint64_t* ct_ref, int n_views, const uint8_t* const* views,
                   const int8_t* side, int cw, int ch, int n_fam, const int* G, const double* H,
                   int f, int g, int x, int y) {
    int sumG = 0, gbase = 0;
    for (int i = 0; i < n_fam; ++i) { if (i == f) gbase = sumG; sumG += G[i]; }
    int nL = 0, nR = 0;
    for (int k = 0; k < n_views; ++k) (side[k] < 0 ? nL : nR)++;
    int rx = cw / 2, ry = ch / 2;
    long sL = 0, sR = 0;
    std::vector<float> win((size_t)cw * ch);
    for (int k = 0; k < n_views; ++k) {
        const double* Hk = H + ((size_t)k * sumG + gbase + g) * 9;
        for (int dy = -ry; dy <= ry; ++dy)
            for (int dx = -rx; dx <= rx; ++dx) {
                int xx = clampi(x + dx, 0, w - 1), yy = clampi(y + dy, 0, h - 1);
                win[(size_t)(dy + ry) * cw + (dx + rx)] = warp_sample(views[k], w, h, Hk, xx + 0.5, yy + 0.5);
            }
        uint64_t ct = census_at(win.data(), cw, ch, rx, ry, cw, ch);
        int c = popcount64(ct_ref[(size_t)y * w + x] ^ ct);
        if (side[k] < 0) sL += c; else sR += c;
    }
    return combine_lr(sL, sR, nL, nR);
}

// The cost vectors of a list of pixels (same definition as or_cost_volume,
// evaluated pixel by pixel through or_cost_sample): out[i][label] for pixel
// (xy[2i], xy[2i+1]) with the pixel's window offsets (offs NULL: full lists).
int or_cost_pixels(int w, int h, const uint64_t* ct_ref, int n_views, const uint8_t* const* views,
                   const int8_t* side, int cw, int ch, int n_fam, const int* G, const int* W,
                   const double* H, const int32_t* offs, int n_pix, const int32_t* xy, uint8_t* out) {
    int D = 0;
    for (int f = 0; f < n_fam; ++f) D += W[f];
    size_t N = (size_t)w * h;
    for (int i = 0; i < n_pix; ++i) {
        int x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || x >= w || y < 0 || y >= h) return -1;
        int l = 0;
        for (int f = 0; f < n_fam; ++f) {
            int o = offs ? offs[(size_t)f * N + (size_t)y * w + x] : 0;
            for (int j = 0; j < W[f]; ++j, ++l) {
                int c = or_cost_sample(w, h, ct_ref, n_views, views, side, cw, ch, n_fam, G, H, f, o + j, x, y);
                if (c > 255) return -2;
                out[(size_t)i * D + l] = (uint8_t)c;
            }
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------
// NCC cost volume (Alg. 1 with the negated, truncated and scaled NCC as the
// matching cost, Sec. on the similarity measures): for every pixel, label and
// view, the cw x ch window of the reference (replicate border) against the
// same window of the warped view; S = combine_mean of the left and right
// sums.  Arguments as or_cost_volume with the reference image in place of its
// census.
// ---------------------------------------------------------------------------
int or_ncc_cost_volume(int w, int h, const uint8_t* ref, int n_views, const uint8_t* const* views,
                       const int8_t* side, int cw, int ch, int n_fam, const int* G, const int* W,
                       const double* H, const int32_t* offs, uint8_t* S) {
    int D = 0, sumG = 0;
    std::vector<int> foff(n_fam), goff(n_fam);
    for (int f = 0; f < n_fam; ++f) {
        foff[f] = D; goff[f] = sumG;
        D += W[f]; sumG += G[f];
        if (!offs && W[f] != G[f]) return -1;
    }
    int nL = 0, nR = 0;
    for (int k = 0; k < n_views; ++k) (side[k] < 0 ? nL : nR)++;
    const int rx = cw / 2, ry = ch / 2;
    size_t N = (size_t)w * h;
    std::vector<int32_t> sL(N * D, 0), sR(N * D, 0);
    std::vector<float> warped(N), wb((size_t)cw * ch);
    std::vector<uint8_t> wa((size_t)cw * ch);
    for (int k = 0; k < n_views; ++k)
        for (int f = 0; f < n_fam; ++f)
            for (int g = 0; g < G[f]; ++g) {
                bool needed = false;
                for (size_t p = 0; p < N && !needed; ++p) {
                    int o = offs ? offs[(size_t)f * N + p] : 0;
                    needed = g >= o && g < o + W[f];
                }
                if (!needed) continue;
                const double* Hk = H + ((size_t)k * sumG + goff[f] + g) * 9;
                or_warp(views[k], w, h, Hk, w, h, warped.data());
                for (int y = 0; y < h; ++y)
                    for (int x = 0; x < w; ++x) {
                        size_t p = (size_t)y * w + x;
                        int o = offs ? offs[(size_t)f * N + p] : 0;
                        if (g < o || g >= o + W[f]) continue;
                        for (int dy = -ry; dy <= ry; ++dy)
                            for (int dx = -rx; dx <= rx; ++dx) {
                                int xx = clampi(x + dx, 0, w - 1), yy = clampi(y + dy, 0, h - 1);
                                wa[(size_t)(dy + ry) * cw + dx + rx] = ref[(size_t)yy * w + xx];
                                wb[(size_t)(dy + ry) * cw + dx + rx] = warped[(size_t)yy * w + xx];
                            }
                        int c = ncc_cost(wa.data(), wb.data(), cw, ch);
                        size_t idx = p * D + foff[f] + (g - o);
                        if (side[k] < 0) sL[idx] += c; else sR[idx] += c;
                    }
            }
    for (size_t i = 0; i < N * (size_t)D; ++i) S[i] = (uint8_t)combine_mean(sL[i], sR[i], nL, nR);
    return 0;
}

// The NCC cost vectors of a list of pixels, each entry computed on its own
// from warped samples of the window (same definition as or_ncc_cost_volume).
int or_ncc_cost_pixels(int w, int h, const uint8_t* ref, int n_views, const uint8_t* const* views,
                       const int8_t* side, int cw, int ch, int n_fam, const int* G, const int* W,
                       const double* H, const int32_t* offs, int n_pix, const int32_t* xy, uint8_t* out) {
    int D = 0, sumG = 0;
    std::vector<int> goff(n_fam);
    for (int f = 0; f < n_fam; ++f) { goff[f] = sumG; D += W[f]; sumG += G[f]; }
    int nL = 0, nR = 0;
    for (int k = 0; k < n_views; ++k) (side[k] < 0 ? nL : nR)++;
    const int rx = cw / 2, ry = ch / 2;
    size_t N = (size_t)w * h;
    std::vector<float> wb((size_t)cw * ch);
    std::vector<uint8_t> wa((size_t)cw * ch);
    for (int i = 0; i < n_pix; ++i) {
        int x = xy[2 * i], y = xy[2 * i + 1];
        if (x < 0 || x >= w || y < 0 || y >= h) return -1;
        for (int dy = -ry; dy <= ry; ++dy)
            for (int dx = -rx; dx <= rx; ++dx)
                wa[(size_t)(dy + ry) * cw + dx + rx] =
                    ref[(size_t)clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1)];
        int l = 0;
        for (int f = 0; f < n_fam; ++f) {
            int o = offs ? offs[(size_t)f * N + (size_t)y * w + x] : 0;
            for (int j = 0; j < W[f]; ++j, ++l) {
                long sl = 0, sr = 0;
                for (int k = 0; k < n_views; ++k) {
                    const double* Hk = H + ((size_t)k * sumG + goff[f] + o + j) * 9;
                    for (int dy = -ry; dy <= ry; ++dy)
                        for (int dx = -rx; dx <= rx; ++dx) {
                            int xx = clampi(x + dx, 0, w - 1), yy = clampi(y + dy, 0, h - 1);
                            wb[(size_t)(dy + ry) * cw + dx + rx] = warp_sample(views[k], w, h, Hk, xx + 0.5, yy + 0.5);
                        }
                    int c = ncc_cost(wa.data(), wb.data(), cw, ch);
                    if (side[k] < 0) sl += c; else sr += c;
                }
                out[(size_t)i * D + l] = (uint8_t)combine_mean(sl, sr, nL, nR);
            }
        }
    }
    return 0;
}

// NCC cost of one pair of windows (the definition above), for the pins.
int or_ncc_window(const uint8_t* a, const float* b, int cw, int ch) { return ncc_cost(a, b, cw, ch); }

// ---------------------------------------------------------------------------
// Semi-global aggregation (Eq. sgm-path, sgm-smooth, sgm-aggr for SGM^Pi in
// Eq. xsgm / sgm-smooth-fp and the surface-normal offset of
// Eq. sgm-smooth-sn, adaptive P2 of Eq. p2-grad).
//   L_r(p, u) = S(p, u) + min_u' ( L_r(p - r, u') + V(u + di, u') ) - min_u' L_r(p - r, u')
// with V = 0 / P1 / P2 by plane-index difference 0 / 1 / >1 within a family
// and P2 across families.  The subtraction of the predecessor minimum is the
// customary normalisation; it shifts S-bar(p, .) by a per-pixel constant only.
// Direction order r: (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (1,-1) (-1,1);
// four paths use the first four.  The first pixel of each path takes L = S.
//   dI: [8][h][w][n_fam] int8 or NULL (all zero).  P2 = lut[|I(p) - I(q)|].
// Returns 0, or -2 if an aggregate exceeds 16 bits.
// ---------------------------------------------------------------------------
int or_sgm_pg(int w, int h, int n_fam, const int* W, const int32_t* offs, const uint8_t* S,
              const int8_t* dI, int p1, const int32_t* lut, const uint8_t* ref, int n_paths,
              uint16_t* Sbar, uint16_t* Lr_out, int pg, const int* goff, const double* fam_delta,
              const double* fam_n, const double* Kinv, const double* step);

int or_sgm(int w, int h, int n_fam, const int* W, const int32_t* offs, const uint8_t* S,
           const int8_t* dI, int p1, const int32_t* lut, const uint8_t* ref, int n_paths,
           uint16_t* Sbar, uint16_t* Lr_out) {
    return or_sgm_pg(w, h, n_fam, W, offs, S, dI, p1, lut, ref, n_paths, Sbar, Lr_out, 0, nullptr, nullptr,
                     nullptr, nullptr, nullptr);
}

// Path-gradient variant (Eq. sgm-smooth-pg), reading of the unspecified
// index jump: along a path, the minimum-cost planes of the two previous
// pixels q = p - r and q2 = q - r give depths d_q and d_q2; continuing the
// path's scene-space gradient (for a planar surface inverse depth is affine
// in the pixel, so the extrapolated inverse depth 1/d* = 2/d_q - 1/d_q2 is
// exact) gives the expected point on p's ray; di_pg(p, r, f) =
// round-half-away((1/delta_p - 1/delta_q)/step_f) with 1/delta_q of q's point
// and 1/delta_p = (1/d*) / c_p of the expected point in family f (the plane
// index is affine in inverse distance, so this holds beyond infinite depth
// too), clamped to [-7, 7] -- the same form as the surface-normal offset.
// Zero on the first two pixels of a path and where a depth is missing.
// pg = 1 adds it to the shift; the geometry arguments may then not be NULL.
int or_sgm_pg(int w, int h, int n_fam, const int* W, const int32_t* offs, const uint8_t* S,
              const int8_t* dI, int p1, const int32_t* lut, const uint8_t* ref, int n_paths,
              uint16_t* Sbar, uint16_t* Lr_out, int pg, const int* goff, const double* fam_delta,
              const double* fam_n, const double* Kinv, const double* step) {
    static const int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    static const int DY[8] = {0, 0, 1, -1, 1, -1, -1, 1};
    int D = 0;
    std::vector<int> foff(n_fam);
    for (int f = 0; f < n_fam; ++f) { foff[f] = D; D += W[f]; }
    size_t N = (size_t)w * h;
    std::vector<int64_t> acc(N * D, 0), L(N * D, 0);
    std::vector<double> dhat(pg ? N : 0, 0.0);   // depth of each pixel's minimum-cost plane on this path
    for (int r = 0; r < n_paths; ++r) {
        int dx = DX[r], dy = DY[r];
        for (int yi = 0; yi < h; ++yi) {
            int y = dy >= 0 ? yi : h - 1 - yi;
            for (int xi = 0; xi < w; ++xi) {
                int x = dx >= 0 ? xi : w - 1 - xi;
                size_t p = (size_t)y * w + x;
                int qx = x - dx, qy = y - dy;
                if (qx < 0 || qx >= w || qy < 0 || qy >= h) {
                    for (int i = 0; i < D; ++i) L[p * D + i] = S[p * D + i];
                } else {
                    size_t q = (size_t)qy * w + qx;
                    int64_t Mq = L[q * D];
                    for (int i = 1; i < D; ++i) Mq = std::min(Mq, L[q * D + i]);
                    int dint = std::abs((int)ref[p] - (int)ref[q]);
                    int64_t P2 = lut[dint];
                    // path-gradient offsets from the two previous minimum-cost points
                    int pgdi[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    int q2x = qx - dx, q2y = qy - dy;
                    if (pg && q2x >= 0 && q2x < w && q2y >= 0 && q2y < h) {
                        double d1 = dhat[q], d2 = dhat[(size_t)q2y * w + q2x];
                        if (d1 > 0.0 && d2 > 0.0) {
                            double inv = 2.0 / d1 - 1.0 / d2;   // extrapolated inverse depth
                            double rp[3], rq[3];
                            rp[0] = Kinv[0] * (x + 0.5) + Kinv[1] * (y + 0.5) + Kinv[2];
                            rp[1] = Kinv[3] * (x + 0.5) + Kinv[4] * (y + 0.5) + Kinv[5];
                            rp[2] = Kinv[6] * (x + 0.5) + Kinv[7] * (y + 0.5) + Kinv[8];
                            rq[0] = Kinv[0] * (qx + 0.5) + Kinv[1] * (qy + 0.5) + Kinv[2];
                            rq[1] = Kinv[3] * (qx + 0.5) + Kinv[4] * (qy + 0.5) + Kinv[5];
                            rq[2] = Kinv[6] * (qx + 0.5) + Kinv[7] * (qy + 0.5) + Kinv[8];
                            for (int f = 0; f < n_fam; ++f) {
                                const double* n = fam_n + 3 * f;
                                double cp = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
                                double cq = -(n[0] * rq[0] + n[1] * rq[1] + n[2] * rq[2]);
                                if (!(cp > 0.0) || !(cq > 0.0)) continue;
                                double ip = inv / cp;
                                double iq = 1.0 / (d1 * cq);
                                double v = (ip - iq) / step[f];
                                v = std::min(std::max(v, -7.0), 7.0);
                                pgdi[f] = (int)std::round(v);
                            }
                        }
                    }
                    for (int f = 0; f < n_fam; ++f) {
                        int op = offs ? offs[(size_t)f * N + p] : 0;
                        int oq = offs ? offs[(size_t)f * N + q] : 0;
                        int di = (dI ? dI[(((size_t)r * N) + p) * n_fam + f] : 0) + pgdi[f];
                        for (int i = 0; i < W[f]; ++i) {
                            int target = op + i + di;       // global index of the zero-cost predecessor
                            int64_t best = Mq + P2;
                            for (int e = -1; e <= 1; ++e) {
                                int j = target + e - oq;    // local index in q's window
                                if (j < 0 || j >= W[f]) continue;
                                int64_t c = L[q * D + foff[f] + j] + (e == 0 ? 0 : p1);
                                best = std::min(best, c);
                            }
                            L[p * D + foff[f] + i] = (int64_t)S[p * D + foff[f] + i] + best - Mq;
                        }
                    }
                }
                if (pg) {
                    // depth of this pixel's minimum-cost plane (smallest label on ties)
                    int bi = 0;
                    for (int i = 1; i < D; ++i)
                        if (L[p * D + i] < L[p * D + bi]) bi = i;
                    int f = 0;
                    while (f + 1 < n_fam && bi >= foff[f + 1]) ++f;
                    int g = (offs ? offs[(size_t)f * N + p] : 0) + (bi - foff[f]);
                    const double* n = fam_n + 3 * f;
                    double rr[3];
                    rr[0] = Kinv[0] * (x + 0.5) + Kinv[1] * (y + 0.5) + Kinv[2];
                    rr[1] = Kinv[3] * (x + 0.5) + Kinv[4] * (y + 0.5) + Kinv[5];
                    rr[2] = Kinv[6] * (x + 0.5) + Kinv[7] * (y + 0.5) + Kinv[8];
                    double den = n[0] * rr[0] + n[1] * rr[1] + n[2] * rr[2];
                    dhat[p] = (den < 0.0) ? -fam_delta[goff[f] + g] / den : 0.0;
                }
            }
        }
        for (size_t i = 0; i < N * (size_t)D; ++i) {
            acc[i] += L[i];
            if (Lr_out) {
                if (L[i] > 65535) return -2;
                Lr_out[(size_t)r * N * D + i] = (uint16_t)L[i];
            }
        }
    }
    if (Sbar)
        for (size_t i = 0; i < N * (size_t)D; ++i) {
            if (acc[i] > 65535) return -2;
            Sbar[i] = (uint16_t)acc[i];
        }
    return 0;
}

// ---------------------------------------------------------------------------
// Winner-takes-all (Eq. sgm-wta, smallest label on ties), depth of the
// winning plane (depth extraction for SGM^Pi) and sub-plane refinement by a
// parabola through the winner and its two neighbours at their non-equidistant
// depths (depth refinement subsection).  No refinement at the ends of the
// window or when the parabola does not open upwards; the vertex is clamped to
// the neighbours' depth interval.
//   fam_delta: concatenated plane lists of all families at this level.
//   label: global label (family-major index into fam_delta), -1 if invalid.
// ---------------------------------------------------------------------------
void or_wta_refine(int w, int h, int n_fam, const int* W, const int* G, const int32_t* offs,
                   const uint16_t* Sbar, const double* fam_n, const double* fam_delta, const double* Kinv,
                   int32_t* label, int32_t* fam_out, float* depth) {
    int D = 0;
    std::vector<int> foff(n_fam), goff(n_fam);
    int sumG = 0;
    for (int f = 0; f < n_fam; ++f) { foff[f] = D; D += W[f]; goff[f] = sumG; sumG += G[f]; }
    size_t N = (size_t)w * h;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            size_t p = (size_t)y * w + x;
            const uint16_t* c = Sbar + p * D;
            int best = 0;
            for (int i = 1; i < D; ++i)
                if (c[i] < c[best]) best = i;
            int f = 0;
            while (f + 1 < n_fam && best >= foff[f + 1]) ++f;
            int li = best - foff[f];
            int o = offs ? offs[(size_t)f * N + p] : 0;
            int g = o + li;
            const double* n = fam_n + 3 * f;
            const double* dl = fam_delta + goff[f];
            double d0 = or_depth_on_plane(Kinv, n, dl[g], x, y);
            fam_out[p] = f;
            if (!(d0 > 0.0)) {
                label[p] = -1;
                depth[p] = 0.0f;
                continue;
            }
            label[p] = goff[f] + g;
            double d = d0;
            if (li >= 1 && li + 1 < W[f]) {
                double dm = or_depth_on_plane(Kinv, n, dl[g - 1], x, y);
                double dp = or_depth_on_plane(Kinv, n, dl[g + 1], x, y);
                double a = dm - d0, b = dp - d0;
                double u = (double)c[best - 1] - (double)c[best];
                double v = (double)c[best + 1] - (double)c[best];
                double sa = u / a, sb = v / b;
                double alpha = (sa - sb) / (a - b);
                if (alpha > 0.0) {
                    double beta = sa - alpha * a;
                    double xv = -beta / (2.0 * alpha);
                    d = d0 + xv;
                    double lo = std::min(dm, dp), hi = std::max(dm, dp);
                    d = std::min(std::max(d, lo), hi);
                }
            }
            depth[p] = (float)d;
        }
}

// 5x5 median of the depth map, replicate border, all 25 samples (invalid
// zeros included): the 13th smallest (pipeline overview: median filter).
void or_median5(const float* in, int w, int h, float* out) {
    float v[25];
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int n = 0;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx)
                    v[n++] = in[(size_t)clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1)];
            std::sort(v, v + 25);
            out[(size_t)y * w + x] = v[12];
        }
}

// ---------------------------------------------------------------------------
// Normals (Sec. extraction of surface normals): back-project the depth map,
// n = h x v with h, v the central differences of the horizontal and vertical
// neighbours' points (one-sided at the border), oriented toward the camera
// and normalised.  Invalid (zero) where the pixel or a used neighbour has no
// depth.  Output [h][w][3].
// ---------------------------------------------------------------------------
void or_normals(const float* depth, int w, int h, const double* Kinv, float* nrm) {
    auto P = [&](int x, int y, double X[3]) {
        double r[3];
        ray_of(Kinv, x + 0.5, y + 0.5, r);
        double d = depth[(size_t)y * w + x];
        X[0] = d * r[0]; X[1] = d * r[1]; X[2] = d * r[2];
        return d > 0.0;
    };
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            float* o = nrm + 3 * ((size_t)y * w + x);
            o[0] = o[1] = o[2] = 0.0f;
            double Xp[3], A[3], B[3], Cc[3], Dd[3];
            if (w < 2 || h < 2 || !P(x, y, Xp)) continue;
            int xa = x > 0 ? x - 1 : x, xb = x + 1 < w ? x + 1 : x;
            int ya = y > 0 ? y - 1 : y, yb = y + 1 < h ? y + 1 : y;
            if (!P(xa, y, A) || !P(xb, y, B) || !P(x, ya, Cc) || !P(x, yb, Dd)) continue;
            double hv[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
            double vv[3] = {Dd[0] - Cc[0], Dd[1] - Cc[1], Dd[2] - Cc[2]};
            double n[3] = {hv[1] * vv[2] - hv[2] * vv[1], hv[2] * vv[0] - hv[0] * vv[2],
                           hv[0] * vv[1] - hv[1] * vv[0]};
            if (n[0] * Xp[0] + n[1] * Xp[1] + n[2] * Xp[2] > 0.0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
            double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            if (!(len > 0.0)) continue;
            o[0] = (float)(n[0] / len); o[1] = (float)(n[1] / len); o[2] = (float)(n[2] / len);
        }
}

// Appearance-weighted Gaussian smoothing of the normal map (Eq. normal,
// normal-smooth): n_p plus the neighbours q != p of the (2r+1)^2 window inside
// the image, each weighted by exp(-|q-p|^2 / (2 sigma^2) - |I(p)-I(q)| / beta)
// / sqrt(2 pi sigma^2) with sigma = r, then normalised.  Pixels without a
// normal stay zero.
void or_normal_smooth(const float* nin, const uint8_t* img, int w, int h, int radius, double beta,
                      float* nout) {
    const double PI = 3.14159265358979323846;
    double sigma = (double)radius;
    double g0 = 1.0 / std::sqrt(2.0 * PI * sigma * sigma);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            size_t p = (size_t)y * w + x;
            const float* np_ = nin + 3 * p;
            float* o = nout + 3 * p;
            o[0] = o[1] = o[2] = 0.0f;
            if (np_[0] == 0.0f && np_[1] == 0.0f && np_[2] == 0.0f) continue;
            double a[3] = {np_[0], np_[1], np_[2]};
            for (int dy = -radius; dy <= radius; ++dy)
                for (int dx = -radius; dx <= radius; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int xx = x + dx, yy = y + dy;
                    if (xx < 0 || xx >= w || yy < 0 || yy >= h) continue;
                    size_t q = (size_t)yy * w + xx;
                    const float* nq = nin + 3 * q;
                    double dI = std::fabs((double)img[p] - (double)img[q]);
                    double wq = g0 * std::exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma) - dI / beta);
                    a[0] += wq * nq[0]; a[1] += wq * nq[1]; a[2] += wq * nq[2];
                }
            double len = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            if (!(len > 0.0)) continue;
            o[0] = (float)(a[0] / len); o[1] = (float)(a[1] / len); o[2] = (float)(a[2] / len);
        }
}

// Geometric confidence (Eq. weight-normal): with n_p the normal, n_Pi the
// normal of the winning plane family and v = (0,0,-1),
// C = (<n_p,n_Pi><n_Pi,v> - cos rho) / (1 - cos rho) when both enclosed angles
// are at most rho, else 0; clamped to [0, 1].  fam: winning family per pixel,
// label < 0 marks pixels without depth.
void or_confidence(const float* nrm, const int32_t* label, const int32_t* fam, const double* fam_n,
                   int w, int h, double rho_deg, float* conf) {
    const double PI = 3.14159265358979323846;
    double cr = std::cos(rho_deg * PI / 180.0);
    for (size_t p = 0; p < (size_t)w * h; ++p) {
        conf[p] = 0.0f;
        const float* n = nrm + 3 * p;
        if (label[p] < 0 || (n[0] == 0.0f && n[1] == 0.0f && n[2] == 0.0f)) continue;
        const double* m = fam_n + 3 * fam[p];
        double c1 = (double)n[0] * m[0] + (double)n[1] * m[1] + (double)n[2] * m[2];
        double c2 = -m[2];
        if (!(c1 >= cr && c2 >= cr)) continue;
        double c = (c1 * c2 - cr) / (1.0 - cr);
        conf[p] = (float)std::min(std::max(c, 0.0), 1.0);
    }
}

// ---------------------------------------------------------------------------
// Coarse-to-fine seeding (pipeline overview, Eq. sampling_range; dynamic cost
// volume; Eq. sgm-smooth-sn).
// ---------------------------------------------------------------------------

// Nearest-neighbour upscaling to the next finer level: fine (x, y) takes
// coarse (min(x/2, sw-1), min(y/2, sh-1)); ch channels per pixel.
void or_upsample_nn(const float* src, int sw, int sh, int ch, int dw, int dh, float* dst) {
    for (int y = 0; y < dh; ++y)
        for (int x = 0; x < dw; ++x) {
            int sx = std::min(x / 2, sw - 1), sy = std::min(y / 2, sh - 1);
            for (int c = 0; c < ch; ++c) dst[((size_t)y * dw + x) * ch + c] = src[((size_t)sy * sw + sx) * ch + c];
        }
}

// Per-pixel sampling window: W consecutive planes of the level's list
// (index 0 at the nearest plane) centred on the plane through the seed depth
// along the pixel's ray -- the rounded continuous index of that plane in the
// list (or_list_index) -- clamped to the list.  A pixel without a seed (or
// whose ray misses the family's planes) gets the centre of the list.
//   fam_delta: the level's lists of all families, concatenated; offs:
//   [n_fam][h][w].
void or_window_offsets(const float* dbar, int w, int h, const double* Kinv, int n_fam, const double* fam_n,
                       const double* fam_delta, const int* G, const int* W, int32_t* offs) {
    size_t N = (size_t)w * h;
    int g0 = 0;
    for (int f = 0; f < n_fam; ++f) {
        const double* n = fam_n + 3 * f;
        const double* list = fam_delta + g0;
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                size_t p = (size_t)y * w + x;
                double r[3];
                ray_of(Kinv, x + 0.5, y + 0.5, r);
                double c = -(n[0] * r[0] + n[1] * r[1] + n[2] * r[2]);
                double d = dbar[p];
                int o;
                if (!(d > 0.0) || !(c > 0.0)) {
                    o = (G[f] - W[f]) / 2;
                } else {
                    double delta = d * c;
                    double j = or_list_index(list, G[f], 1.0 / delta);
                    j = std::min(std::max(j, -1.0e6), 1.0e6);
                    int jr = (int)std::floor(j + 0.5);
                    o = clampi(jr - W[f] / 2, 0, G[f] - W[f]);
                }
                offs[(size_t)f * N + p] = o;
            }
        g0 += G[f];
    }
}

// Surface-normal index offset (Eq. sgm-smooth-sn): the tangent plane of the
// seed point P = dbar K^-1 p with seed normal nbar meets the ray of the
// predecessor q = p - r at depth d_T; di(p, r, f) is the plane-index
// difference, in family f's list, between the point on q's ray and P
// (continuous indices of their inverse distances, or_list_index), rounded
// half away from zero and clamped to [-7, 7].  Zero where the seed is
// missing or the construction degenerates.  fam_delta: the level's lists,
// concatenated; dI: [8][h][w][n_fam].
void or_delta_i(const float* dbar, const float* nbar, int w, int h, const double* Kinv, int n_fam,
                const double* fam_n, const double* fam_delta, const int* G, int8_t* dI) {
    static const int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    static const int DY[8] = {0, 0, 1, -1, 1, -1, -1, 1};
    size_t N = (size_t)w * h;
    std::memset(dI, 0, 8 * N * n_fam);
    std::vector<int> g0(n_fam, 0);
    for (int f = 1; f < n_fam; ++f) g0[f] = g0[f - 1] + G[f - 1];
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            size_t p = (size_t)y * w + x;
            double d = dbar[p];
            double nb[3] = {nbar[3 * p], nbar[3 * p + 1], nbar[3 * p + 2]};
            if (!(d > 0.0) || (nb[0] == 0.0 && nb[1] == 0.0 && nb[2] == 0.0)) continue;
            double rp[3];
            ray_of(Kinv, x + 0.5, y + 0.5, rp);
            double kP = nb[0] * (d * rp[0]) + nb[1] * (d * rp[1]) + nb[2] * (d * rp[2]);
            for (int r = 0; r < 8; ++r) {
                double rq[3];
                ray_of(Kinv, (x - DX[r]) + 0.5, (y - DY[r]) + 0.5, rq);
                double den = nb[0] * rq[0] + nb[1] * rq[1] + nb[2] * rq[2];
                if (!(std::fabs(den) > 1e-12)) continue;
                double dT = kP / den;
                if (!(dT > 0.0)) continue;
                for (int f = 0; f < n_fam; ++f) {
                    const double* n = fam_n + 3 * f;
                    double cp = -(n[0] * rp[0] + n[1] * rp[1] + n[2] * rp[2]);
                    double cq = -(n[0] * rq[0] + n[1] * rq[1] + n[2] * rq[2]);
                    if (!(cp > 0.0) || !(cq > 0.0)) continue;
                    double ip = 1.0 / (d * cp);
                    double iq = 1.0 / (dT * cq);
                    const double* list = fam_delta + g0[f];
                    double v = or_list_index(list, G[f], iq) - or_list_index(list, G[f], ip);
                    v = std::min(std::max(v, -7.0), 7.0);
                    dI[((size_t)r * N + p) * n_fam + f] = (int8_t)std::round(v);
                }
            }
        }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Post-processing (Sec. on post-processing and depth map filtering).
//
// DoG texture mask (Alg. 3), with the readings: the 7x7 Gaussian has
// sigma = 0.3 ((7 - 1)/2 - 1) + 0.8 = 1.4 (the usual rule for a kernel size
// without a given sigma), taps exp(-i^2 / (2 sigma^2)) normalised to sum 1,
// separable, replicate border, horizontal pass then vertical, each sum
// accumulated from the first tap in double; DoG = I - I_smooth on the 0..255
// scale; a pixel is active when |DoG| > 0.5; activation areas (4-connected)
// of fewer than min_on pixels are cleared, the mask is dilated with a 3x3
// square, deactivation areas of fewer than min_off pixels are filled.  The
// result marks textured pixels (1); estimates where it is 0 (weakly
// textured) are invalidated -- the stated purpose of the filter, where the
// printed algorithm writes the opposite value.
// ---------------------------------------------------------------------------
namespace {
// 4-connected components of the pixels equal to v; those with fewer than
// min_size pixels flip to 1 - v.  Plain breadth-first search.
void speckle(std::vector<uint8_t>& m, int w, int h, uint8_t v, int min_size) {
    std::vector<int> comp((size_t)w * h, -1);
    std::vector<int> queue;
    for (int s = 0; s < w * h; ++s) {
        if (m[s] != v || comp[s] >= 0) continue;
        queue.clear();
        queue.push_back(s);
        comp[s] = s;
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            int c = queue[qi], x = c % w, y = c / w;
            const int nx[4] = {x - 1, x + 1, x, x};
            const int ny[4] = {y, y, y - 1, y + 1};
            for (int d = 0; d < 4; ++d) {
                if (nx[d] < 0 || nx[d] >= w || ny[d] < 0 || ny[d] >= h) continue;
                int n = ny[d] * w + nx[d];
                if (m[n] == v && comp[n] < 0) {
                    comp[n] = s;
                    queue.push_back(n);
                }
            }
        }
        if ((int)queue.size() < min_size)
            for (int c : queue) m[c] = (uint8_t)(1 - v);
    }
}
}  // namespace

extern "C" {

void or_gauss_taps(double sigma, int radius, double* taps) {
    double sum = 0.0;
    for (int i = -radius; i <= radius; ++i) {
        taps[i + radius] = std::exp(-(double)(i * i) / (2.0 * sigma * sigma));
        sum += taps[i + radius];
    }
    for (int i = 0; i <= 2 * radius; ++i) taps[i] /= sum;
}

// DoG of the reference image (double, [h][w]) with the separable Gaussian.
void or_dog(const uint8_t* img, int w, int h, double sigma, int radius, double* dog) {
    std::vector<double> g(2 * radius + 1), tmp((size_t)w * h);
    or_gauss_taps(sigma, radius, g.data());
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            double acc = 0.0;
            for (int i = -radius; i <= radius; ++i)
                acc = acc + g[i + radius] * (double)img[(size_t)y * w + clampi(x + i, 0, w - 1)];
            tmp[(size_t)y * w + x] = acc;
        }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            double acc = 0.0;
            for (int j = -radius; j <= radius; ++j)
                acc = acc + g[j + radius] * tmp[(size_t)clampi(y + j, 0, h - 1) * w + x];
            dog[(size_t)y * w + x] = (double)img[(size_t)y * w + x] - acc;
        }
}

void or_dog_mask(const uint8_t* img, int w, int h, double sigma, int radius, double thresh, int min_on,
                 int min_off, uint8_t* mask) {
    std::vector<double> dog((size_t)w * h);
    or_dog(img, w, h, sigma, radius, dog.data());
    std::vector<uint8_t> m((size_t)w * h);
    for (size_t i = 0; i < m.size(); ++i) m[i] = std::fabs(dog[i]) > thresh ? 1 : 0;
    speckle(m, w, h, 1, min_on);
    std::vector<uint8_t> d((size_t)w * h, 0);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            uint8_t v = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int xx = x + dx, yy = y + dy;
                    if (xx >= 0 && xx < w && yy >= 0 && yy < h && m[(size_t)yy * w + xx]) v = 1;
                }
            d[(size_t)y * w + x] = v;
        }
    speckle(d, w, h, 0, min_off);
    std::memcpy(mask, d.data(), d.size());
}

// Components of the value v with fewer than min_size pixels flip (the
// speckle step alone, for the pins).
void or_speckle(uint8_t* m, int w, int h, int v, int min_size) {
    std::vector<uint8_t> t(m, m + (size_t)w * h);
    speckle(t, w, h, (uint8_t)v, min_size);
    std::memcpy(m, t.data(), t.size());
}

// ---------------------------------------------------------------------------
// Geometric consistency by mutual reprojection (Alg. 4): for each pixel p of
// the reference map with depth d > 0 and each neighbouring map k, the point
// X = d K^-1 p~ goes to view k (X_k = R_k X + t_k, R_k|t_k reference to view
// k), is projected to the continuous point p_k, takes the depth d_k of the
// pixel containing p_k (a miss outside the image, behind a camera or where
// d_k = 0), is lifted with d_k K^-1 p_k~ and mapped back to the reference,
// where its projection p' gives the reprojection error ||p - p'||.  hits
// counts the maps with error < eta_r; keep = hits >= eta_h.  Double
// precision; pixel centres at (x + 0.5, y + 0.5).
// ---------------------------------------------------------------------------
void or_geo_consistency(int w, int h, const double* K, const float* depth_ref, int n_nb,
                        const float* const* depth_nb, const double* R, const double* t, double eta_r, int eta_h,
                        int32_t* hits, uint8_t* keep) {
    double Ki[9], Kl[9];
    or_kinv_level(K, 0, Ki, Kl);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const size_t p = (size_t)y * w + x;
            const double d = depth_ref[p];
            int nh = 0;
            if (d > 0.0) {
                const double u0 = x + 0.5, v0 = y + 0.5;
                double ray[3];
                ray_of(Ki, u0, v0, ray);
                const double X[3] = {d * ray[0], d * ray[1], d * ray[2]};
                for (int k = 0; k < n_nb; ++k) {
                    const double* Rk = R + 9 * k;
                    const double* tk = t + 3 * k;
                    double Xk[3];
                    for (int i = 0; i < 3; ++i) Xk[i] = Rk[3 * i] * X[0] + Rk[3 * i + 1] * X[1] + Rk[3 * i + 2] * X[2] + tk[i];
                    if (!(Xk[2] > 0.0)) continue;
                    const double uk = (K[0] * Xk[0] + K[1] * Xk[1] + K[2] * Xk[2]) / Xk[2];
                    const double vk = (K[3] * Xk[0] + K[4] * Xk[1] + K[5] * Xk[2]) / Xk[2];
                    const double fx = std::floor(uk), fy = std::floor(vk);
                    if (!(fx >= 0.0 && fx < (double)w && fy >= 0.0 && fy < (double)h)) continue;
                    const double dk = depth_nb[k][(size_t)fy * w + (size_t)fx];
                    if (!(dk > 0.0)) continue;
                    double rk[3];
                    ray_of(Ki, uk, vk, rk);
                    const double Y[3] = {dk * rk[0] - tk[0], dk * rk[1] - tk[1], dk * rk[2] - tk[2]};
                    double Xb[3];
                    for (int i = 0; i < 3; ++i) Xb[i] = Rk[i] * Y[0] + Rk[3 + i] * Y[1] + Rk[6 + i] * Y[2];
                    if (!(Xb[2] > 0.0)) continue;
                    const double ub = (K[0] * Xb[0] + K[1] * Xb[1] + K[2] * Xb[2]) / Xb[2];
                    const double vb = (K[3] * Xb[0] + K[4] * Xb[1] + K[5] * Xb[2]) / Xb[2];
                    const double eu = ub - u0, ev = vb - v0;
                    if (std::sqrt(eu * eu + ev * ev) < eta_r) ++nh;
                }
            }
            if (hits) hits[p] = nh;
            keep[p] = (d > 0.0 && nh >= eta_h) ? 1 : 0;
        }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Plane set (Sec. on bounding planes and on the cross-ratio sampling steps).
// ---------------------------------------------------------------------------
namespace {
double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
double sin_angle(const double* a, const double* b) {
    const double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    return std::sqrt(dot3(c, c)) / (std::sqrt(dot3(a, a)) * std::sqrt(dot3(b, b)));
}
}  // namespace

extern "C" {

// Bounding plane distances of a family with normal n for the depth range
// [d_min, d_max]: the reference frustum's corner rays (image corners
// (0,0), (w,0), (0,h), (w,h)) meet the near plane z = d_min and the far
// plane z = d_max; delta_min is the least |n^T X| over the near corners and
// delta_max the largest over the far corners (the printed second formula
// repeats the minimum; the maximum keeps the whole far face inside the
// sweep).  Returns -1 on bad input.
int or_bounding_planes(const double* K, int w, int h, const double* n, double d_min, double d_max, double* out) {
    if (!(d_min > 0.0) || !(d_max > d_min) || w < 1 || h < 1) return -1;
    double Ki[9], Kl[9];
    or_kinv_level(K, 0, Ki, Kl);
    const double cu[4] = {0.0, (double)w, 0.0, (double)w};
    const double cv[4] = {0.0, 0.0, (double)h, (double)h};
    double lo = 1e300, hi = 0.0;
    for (int i = 0; i < 4; ++i) {
        double r[3];
        ray_of(Ki, cu[i], cv[i], r);
        const double a = std::fabs(dot3(n, r));
        lo = std::min(lo, a * d_min);
        hi = std::max(hi, a * d_max);
    }
    out[0] = lo;
    out[1] = hi;
    return 0;
}

// Plane distances by the cross-ratio (Alg. 2): among the four corner pixel
// centres of the reference image, p is the one whose images in view k on
// the bounding planes lie farthest apart; its ray meets the bounding planes
// at P_min and P_max, seen from view k at p_min and p_max on the epipolar
// line.  Stepping from p_max towards p_min one pixel at a time, the points
// p_i give the cross-ratio Q of the view-k rays to the epipole, p_min, p_i
// and p_max (sines of the enclosed angles), and the distance of the plane
// through the corresponding point of p's ray follows from
//   delta (d_max - d_min) / (d_max (delta - d_min)) = Q,
// i.e. delta = Q d_max d_min / (Q d_max - (d_max - d_min)).  The list runs
// from delta_max to delta_min (appended when the segment length is not a
// whole number of pixels), consecutive planes moving p's image by one
// pixel.  R, t map reference to view-k coordinates.  *count receives the
// length; the list is written when it fits in max_planes (return 0), else
// -2; -1 on bad input (camera centre of view k not in front of the nearest
// plane, degenerate segment).
int or_cross_ratio_planes(const double* K, int w, int h, const double* R, const double* t, const double* n,
                          double dmin, double dmax, int max_planes, double* out, int* count) {
    *count = 0;
    if (!(dmin > 0.0) || !(dmax > dmin) || w < 1 || h < 1) return -1;
    double Ki[9], Kl[9];
    or_kinv_level(K, 0, Ki, Kl);
    // view-k camera centre in reference coordinates: C = -R^T t
    double C[3];
    for (int i = 0; i < 3; ++i) C[i] = -(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
    if (!(dot3(n, C) + dmin > 0.0)) return -1;
    auto to_view = [&](const double* X, double* Y) {
        for (int i = 0; i < 3; ++i) Y[i] = R[3 * i] * X[0] + R[3 * i + 1] * X[1] + R[3 * i + 2] * X[2] + t[i];
    };
    auto project = [&](const double* Y, double* uv) {
        uv[0] = (K[0] * Y[0] + K[1] * Y[1] + K[2] * Y[2]) / Y[2];
        uv[1] = (K[3] * Y[0] + K[4] * Y[1] + K[5] * Y[2]) / Y[2];
    };
    const double cu[4] = {0.5, w - 0.5, 0.5, w - 0.5};
    const double cv[4] = {0.5, 0.5, h - 0.5, h - 0.5};
    double best = -1.0, Ymin[3] = {0, 0, 0}, Ymax[3] = {0, 0, 0}, pmin[2] = {0, 0}, pmax[2] = {0, 0};
    for (int c = 0; c < 4; ++c) {
        double r[3];
        ray_of(Ki, cu[c], cv[c], r);
        const double nr = dot3(n, r);
        if (!(nr < 0.0)) continue;   // the corner ray does not meet the planes in front
        const double Pmin[3] = {-dmin / nr * r[0], -dmin / nr * r[1], -dmin / nr * r[2]};
        const double Pmax[3] = {-dmax / nr * r[0], -dmax / nr * r[1], -dmax / nr * r[2]};
        double Y0[3], Y1[3], a[2], b[2];
        to_view(Pmin, Y0);
        to_view(Pmax, Y1);
        if (!(Y0[2] > 0.0) || !(Y1[2] > 0.0)) continue;
        project(Y0, a);
        project(Y1, b);
        const double L = std::hypot(a[0] - b[0], a[1] - b[1]);
        if (L > best) {
            best = L;
            std::memcpy(Ymin, Y0, sizeof(Y0));
            std::memcpy(Ymax, Y1, sizeof(Y1));
            std::memcpy(pmin, a, sizeof(a));
            std::memcpy(pmax, b, sizeof(b));
        }
    }
    if (!(best > 0.0)) return -1;
    const double kx = (pmin[0] - pmax[0]) / best, ky = (pmin[1] - pmax[1]) / best;
    // rays of view k (camera coordinates): to the epipole (the reference
    // camera centre, at t), to P_min and to P_max
    const double* Ve = t;
    const double s_mm = sin_angle(Ymin, Ymax), s_ex = sin_angle(Ve, Ymax);
    const int steps = (int)std::floor(best);
    const bool tail = (double)steps < best;
    const int total = steps + 1 + (tail ? 1 : 0);
    *count = total;
    if (total > max_planes) return -2;
    int j = 0;
    for (int i = 0; i <= steps; ++i) {
        if (i == 0) {
            out[j++] = dmax;
            continue;
        }
        const double u = pmax[0] + i * kx, v = pmax[1] + i * ky;
        double Vi[3];
        ray_of(Ki, u, v, Vi);
        const double sin_mi = sin_angle(Ymin, Vi);
        if (!(sin_mi > 0.0)) { out[j++] = dmin; continue; }
        const double Q = sin_angle(Ve, Vi) * s_mm / (s_ex * sin_mi);
        out[j++] = Q * dmax * dmin / (Q * dmax - (dmax - dmin));
    }
    if (tail) out[j++] = dmin;
    return 0;
}

}  // extern "C"
