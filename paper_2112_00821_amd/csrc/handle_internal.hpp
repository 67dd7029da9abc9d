// Handle internals the served form uses to admit frames against the device
// memory its slots actually hold (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fassmvs.h"

namespace fmvs {
// Buffers grow to exactly what a frame needs (no headroom for larger frames).
void handle_set_exact_growth(fassmvs_handle *h);
// Device bytes the handle holds.
uint64_t handle_held(fassmvs_handle *h);
// Bytes the handle's buffers would grow by to run this frame (validates and
// plans the frame, allocates nothing).
fassmvs_status handle_growth(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                             const int8_t *side, int32_t n_views, const double K[9],
                             const fassmvs_plane_family *families, int32_t n_families, uint64_t *grow);
// Free every device buffer of a handle with no frame in flight.
void handle_trim(fassmvs_handle *h);
// Bytes the handle would grow by to hold any frame of a stream (w x hgt
// images, n_views views on one side, these intrinsics and families), and
// growing it to that (apply); a handle with no frame in flight.
fassmvs_status handle_reserve(fassmvs_handle *h, int w, int hgt, int n_views, const double K[9],
                              const fassmvs_plane_family *families, int n_families, bool apply, uint64_t *grow);
// Bytes of an image's whole pyramid (levels halved with integer division,
// level 0 first, each level's rows packed) for n_levels levels.
size_t pyramid_bytes(int w, int h, int n_levels);
// Enqueue the pyramid levels 1..n_levels-1 of the level-0 image at img (the
// layout above) on stream s.
hipError_t pyramid_build(uint8_t *img, int w, int h, int n_levels, hipStream_t s);
// fassmvs_submit_frame with device images that already carry their whole
// pyramid (the layout above, stride = width): the pipeline copies the
// levels instead of rebuilding them.
fassmvs_status handle_submit_pyramids(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                      const int8_t *view_side, int32_t n_views, const double K[9],
                                      const fassmvs_plane_family *families, int32_t n_families, uint64_t *ticket);
}  // namespace fmvs
