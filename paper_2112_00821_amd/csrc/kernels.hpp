// Internal interface between the FaSS-MVS host runtime and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmvs {

constexpr int kMaxViews = 8;
constexpr int kMaxFam = 8;
constexpr int kMaxLabels = 512;
constexpr int kNumDirs = 8;
constexpr int kMaxPgPlanes = 2048;   // plane-list entries held in LDS by the path-gradient SGM

// Path directions r (step p -> p + r): (1,0) (-1,0) (0,1) (0,-1) (1,1)
// (-1,-1) (1,-1) (-1,1); four-path SGM uses the first four.
__host__ __device__ inline int dir_dx(int r) {
    const int t[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    return t[r];
}
__host__ __device__ inline int dir_dy(int r) {
    const int t[8] = {0, 0, 1, -1, 1, -1, -1, 1};
    return t[r];
}

// ---------------------------------------------------------------- sweep
struct SweepArgs {
    int w, h;                 // reference level size (views have the same size)
    int cw, ch;               // census window
    int n_views, nL, nR, m;
    const uint8_t *views[kMaxViews];
    int side[kMaxViews];
    int cost;                 // 0: census-Hamming, 1: NCC
    const uint64_t *ct_ref;   // [h][w] reference census (census cost)
    const uint8_t *ref;       // [h][w] reference image (NCC cost)
    int n_fam, D, sumG;
    int G[kMaxFam], W[kMaxFam], foff[kMaxFam], goff[kMaxFam];
    const double *H;          // [n_views][sumG][9]
    const int32_t *offs;      // [n_fam][h][w] or nullptr (full lists)
    const float *warped;      // [n_views][sumG][h][w] or nullptr
    uint8_t *S;               // [h][w][D]
    int tiles_x, tiles_y, n_chunks;
    int rows_per_thread;      // 4 (tile 64x16), 8 (tile 64x32), 0 = by cost
    unsigned long long *work; // optional counter of evaluated (pixel, label) pairs
};
hipError_t launch_sweep(const SweepArgs &a, hipStream_t s);
// several frames in one launch (see k_sweep.hip)
size_t sweep_batch_bytes(int n);
int prepare_sweep_batch(SweepArgs *host, int n, int rpt, int target, void *out);
hipError_t launch_sweep_batch(const void *dev, int n, int blocks, int rpt, int cw, int ch, int cost, hipStream_t s);

// ---------------------------------------------------------------- sgm
struct SgmArgs {
    int w, h, D;
    int n_fam;
    int W[kMaxFam], foff[kMaxFam];
    const uint8_t *S;         // [h][w][D]
    const int32_t *offs;      // [n_fam][h][w] or nullptr
    const int8_t *dI;         // [8][h][w][n_fam] or nullptr
    const uint8_t *ref;       // [h][w]
    int p1;
    int lut[256];
    // directions run by this launch and where each writes its path costs
    int n_dirs;
    int dirs[8];
    uint16_t *out[8];         // [h][w][D] per launched direction (write mode)
    int path_begin[9];        // prefix sum of path counts over the launched directions
    // path-gradient offsets (SGM^Pi-pg): level plane lists and geometry
    int pg;
    int sumG;
    int goff[kMaxFam];
    const double *delta;      // device, concatenated plane lists (sumG)
    double fam_n[kMaxFam][3];
    double Kinv[9];
    double step[kMaxFam];
    // final mode: sum the finished directions' buffers, take the argmin
    int final_mode;
    int n_in;
    const uint16_t *in[8];
    uint16_t *wta;            // [h][w]
    uint16_t *c3;             // [h][w][3]
};
int sgm_paths(int dir, int w, int h);
hipError_t launch_sgm(const SgmArgs &a, hipStream_t s);
// several frames' aggregation in one persistent launch (see k_sgm.hip)
size_t sgm_batch_bytes(int n);
int prepare_sgm_batch(SgmArgs *host, int n, void *out, int *kp, bool *win, bool *sn, int *nf_max);
hipError_t launch_sgm_batch(const void *dev, int n, int jobs, int kp, bool win, bool sn, int nf_max,
                            unsigned *counter, hipStream_t s);
hipError_t launch_sum_u16(const uint16_t *const *bufs, int n, size_t count, uint16_t *out, hipStream_t s);

// ---------------------------------------------------------------- image stages
hipError_t launch_pyr_down(const uint8_t *src, int w, int h, int stride, uint8_t *dst, hipStream_t s);
hipError_t launch_census(const uint8_t *img, int w, int h, int cw, int ch, uint64_t *out, hipStream_t s);
hipError_t launch_warp(const uint8_t *src, int sw, int sh, const double *dH, int rw, int rh, float *out,
                       hipStream_t s);

struct RefineArgs {
    int w, h, n_fam;
    int W[kMaxFam], G[kMaxFam], foff[kMaxFam], goff[kMaxFam];
    double fam_n[kMaxFam][3];
    double Kinv[9];
    const double *delta;      // device, concatenated lists (sumG)
    const int32_t *offs;
    const uint16_t *wta, *c3;
    int32_t *label, *fam;
    float *depth;
};
hipError_t launch_refine(const RefineArgs &a, hipStream_t s);
hipError_t launch_median5(const float *in, int w, int h, float *out, hipStream_t s);

struct NormalArgs {
    int w, h, radius;
    double beta, cos_rho;
    // smoothing weights g0 exp(-d2 / (2 sigma^2) - dI / beta) by squared
    // offset d2 (0..2 radius^2) and intensity difference dI (0..255):
    // [d2][256], computed on the host (device memory)
    const double *wtab;
    double Kinv[9];
    int n_fam;
    double fam_n[kMaxFam][3];
    const float *depth;
    const uint8_t *img;
    const int32_t *label, *fam;
    float *nraw, *normal, *conf;
};
hipError_t launch_normals(const NormalArgs &a, hipStream_t s);

struct SeedArgs {
    int cw, ch, fw, fh, n_fam;
    double Kinv[9];
    double fam_n[kMaxFam][3];
    const double *inv;        // the fine level's plane lists as inverse distances 1/delta, concatenated (device)
    int goff[kMaxFam];        // first plane of each family in inv
    int G[kMaxFam], W[kMaxFam];
    const float *depth_c, *normal_c;
    float *dbar, *nbar;
    int32_t *offs;
    int8_t *dI;
};
hipError_t launch_seed(const SeedArgs &a, hipStream_t s);

// ---------------------------------------------------------------- post filters
struct PostArgs {
    int radius;               // Gaussian radius (3 for the 7x7 kernel)
    double taps[15];          // normalised taps, radius*2+1 used
    double thresh;            // |DoG| threshold (0..255 scale)
    int min_on, min_off;      // speckle sizes for activation / deactivation areas
};
hipError_t launch_dog_mask(const uint8_t *img, int w, int h, const PostArgs &a, double *tmp, uint8_t *m0, uint8_t *m1,
                           hipStream_t s);
hipError_t launch_apply_keep(const uint8_t *keep, size_t n, float *depth, float *normal, float *conf, hipStream_t s);

struct GeoArgs {
    int w, h;
    const float *depth_ref;
    int n_nb;
    const float *depth_nb[kMaxViews];
    double R[kMaxViews][9], t[kMaxViews][3];   // reference -> neighbour
    double K[9], Kinv[9];
    double eta_r;
    int eta_h;
};
hipError_t launch_geo(const GeoArgs &a, int32_t *hits, uint8_t *keep, hipStream_t s);


}  // namespace fmvs
