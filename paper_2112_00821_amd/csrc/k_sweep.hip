// Host dispatch of the fused plane-sweep kernel (Alg. 1 of the paper): grid
// size, tile height and the (window, cost) variant.  The kernel itself is in
// k_sweep.hpp; k_sweep_inst.hip instantiates one variant per translation
// unit.
#include "kernels.hpp"

#include <cstdlib>

namespace fmvs {

constexpr int kSweepTileW = 64;

template <int CW, int CH, int COST>
hipError_t sweep_launch_cfg(const SweepArgs &a, dim3 grid, int rpt, hipStream_t s);

hipError_t launch_sweep(const SweepArgs &a0, hipStream_t s) {
    SweepArgs a = a0;
    // rows per thread (tile height / 4): 8 halves the halo and the LDS reads
    // per pixel, 4 keeps more waves resident (the NCC's double-precision
    // window sums take many registers: 4 unless asked otherwise)
    int rpt = a.rows_per_thread == 4 ? 4 : (a.rows_per_thread == 8 ? 8 : (a.cost == 1 ? 4 : 8));
    const int th = 4 * rpt;
    a.tiles_x = (a.w + kSweepTileW - 1) / kSweepTileW;
    a.tiles_y = (a.h + th - 1) / th;
    int tiles = a.tiles_x * a.tiles_y;
    if (tiles == 0) return hipSuccess;
    if (a.n_chunks <= 0) {
        // Split each tile's label range into chunks until there are about
        // 8192 workgroups (32 per CU): a tile's whole label loop is long
        // (hundreds of labels x views), so with few workgroups the last
        // round leaves CUs idle.  8192 measured best at 1080p x 128 labels
        // and 2704x1520 x 384 labels (2048: 2 % / 28 % slower); more
        // chunks repeat the per-workgroup setup.  FASSMVS_SWEEP_BLOCKS
        // overrides the target.
        const char *e = std::getenv("FASSMVS_SWEEP_BLOCKS");
        const int target = e && std::atoi(e) > 0 ? std::atoi(e) : 8192;
        int want = (target + tiles - 1) / tiles;
        int maxc = (a.D + 7) / 8;
        a.n_chunks = want < 1 ? 1 : (want > maxc ? maxc : want);
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

}  // namespace fmvs
