// Host dispatch of the fused plane-sweep kernel (Alg. 1 of the paper): grid
// size, tile height and the (window, cost) variant.  The kernel itself is in
// k_sweep.hpp; k_sweep_inst.hip instantiates one variant per translation
// unit.
#include "kernels.hpp"

#include <cstdlib>
#include <cstring>

namespace fmvs {

constexpr int kSweepTileW = 64;

template <int CW, int CH, int COST>
hipError_t sweep_launch_cfg(const SweepArgs &a, dim3 grid, int rpt, hipStream_t s);
template <int CW, int CH, int COST>
hipError_t sweep_launch_batch_cfg(const SweepArgs *list, const int *prefix, int n, int blocks, int rpt,
                                  hipStream_t s);

// Rows per thread (tile height / 4): 8 halves the halo and the LDS reads per
// pixel, 4 keeps more waves resident (the NCC's double-precision window
// sums take many registers: 4 unless asked otherwise).
int sweep_rpt(const SweepArgs &a) {
    return a.rows_per_thread == 4 ? 4 : (a.rows_per_thread == 8 ? 8 : (a.cost == 1 ? 4 : 8));
}

// Tile grid of one frame for rpt rows per thread; returns the tile count.
int sweep_tiles(SweepArgs &a, int rpt) {
    a.tiles_x = (a.w + kSweepTileW - 1) / kSweepTileW;
    a.tiles_y = (a.h + 4 * rpt - 1) / (4 * rpt);
    return a.tiles_x * a.tiles_y;
}

// Split each tile's label range into chunks until there are about `target`
// workgroups: a tile's whole label loop is long (hundreds of labels x
// views), so with few workgroups the last round leaves CUs idle.
int sweep_chunks(const SweepArgs &a, int tiles, int target) {
    int want = (target + tiles - 1) / tiles;
    int maxc = (a.D + 7) / 8;
    return want < 1 ? 1 : (want > maxc ? maxc : want);
}

hipError_t launch_sweep(const SweepArgs &a0, hipStream_t s) {
    SweepArgs a = a0;
    const int rpt = sweep_rpt(a);
    const int tiles = sweep_tiles(a, rpt);
    if (tiles == 0) return hipSuccess;
    if (a.n_chunks <= 0) {
        // about 8192 workgroups (32 per CU) measured best at 1080p x 128
        // labels and 2704x1520 x 384 labels (2048: 2 % / 28 % slower); more
        // chunks repeat the per-workgroup setup.  FASSMVS_SWEEP_BLOCKS
        // overrides the target.
        const char *e = std::getenv("FASSMVS_SWEEP_BLOCKS");
        const int target = e && std::atoi(e) > 0 ? std::atoi(e) : 8192;
        a.n_chunks = sweep_chunks(a, tiles, target);
    }
    dim3 grid((unsigned)(tiles * a.n_chunks));
    // (window, cost) pairs the sweep is built for
#define FMVS_SWEEP(CWv, CHv, C) \
    if (a.cost == C && a.cw == CWv && a.ch == CHv) return sweep_launch_cfg<CWv, CHv, C>(a, grid, rpt, s);
    FMVS_SWEEP(5, 5, 0)
    FMVS_SWEEP(9, 7, 0)
    FMVS_SWEEP(7, 7, 0)
    FMVS_SWEEP(3, 3, 0)
    FMVS_SWEEP(5, 5, 1)
    FMVS_SWEEP(9, 9, 1)
    FMVS_SWEEP(7, 7, 1)
    FMVS_SWEEP(3, 3, 1)
#undef FMVS_SWEEP
    return hipErrorInvalidValue;
}

// Several frames' sweeps in one launch, in two steps so the launch can be
// captured in a graph apart from the argument upload.
// prepare_sweep_batch: host[0..n-1] are the frames' args (same window and
// cost, no pre-warped input); their tile grids and chunk counts are set
// (about `target` workgroups over all frames, each frame's share by its
// pixels x labels) and they are written with the workgroup prefix (n + 1
// ints) to out (host memory of sweep_batch_bytes(n)).  Returns the
// workgroup count, or -1 if the frames cannot share a launch.
size_t sweep_batch_bytes(int n) { return sizeof(SweepArgs) * n + sizeof(int) * (n + 1); }

int prepare_sweep_batch(SweepArgs *host, int n, int rpt, int target, void *out) {
    if (n < 1) return -1;
    double work = 0.0;
    for (int i = 0; i < n; ++i) work += (double)host[i].w * host[i].h * host[i].D;
    int *prefix = (int *)((SweepArgs *)out + n);
    prefix[0] = 0;
    for (int i = 0; i < n; ++i) {
        SweepArgs &a = host[i];
        if (a.cw != host[0].cw || a.ch != host[0].ch || a.cost != host[0].cost || a.warped) return -1;
        a.rows_per_thread = rpt;
        const int tiles = sweep_tiles(a, rpt);
        const double share = work > 0.0 ? (double)a.w * a.h * a.D / work : 1.0;
        a.n_chunks = sweep_chunks(a, tiles, (int)(target * share + 0.5));
        prefix[i + 1] = prefix[i] + tiles * a.n_chunks;
    }
    std::memcpy(out, host, sizeof(SweepArgs) * n);
    return prefix[n];
}

// launch_sweep_batch: the args block prepared above, in device memory at
// dev, for `blocks` workgroups.
hipError_t launch_sweep_batch(const void *dev, int n, int blocks, int rpt, int cw, int ch, int cost, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const SweepArgs *dl = (const SweepArgs *)dev;
    const int *dp = (const int *)((const SweepArgs *)dev + n);
#define FMVS_SWEEPB(CWv, CHv, C) \
    if (cost == C && cw == CWv && ch == CHv) return sweep_launch_batch_cfg<CWv, CHv, C>(dl, dp, n, blocks, rpt, s);
    FMVS_SWEEPB(5, 5, 0)
    FMVS_SWEEPB(9, 7, 0)
    FMVS_SWEEPB(7, 7, 0)
    FMVS_SWEEPB(3, 3, 0)
    FMVS_SWEEPB(5, 5, 1)
    FMVS_SWEEPB(9, 9, 1)
    FMVS_SWEEPB(7, 7, 1)
    FMVS_SWEEPB(3, 3, 1)
#undef FMVS_SWEEPB
    return hipErrorInvalidValue;
}

}  // namespace fmvs
