// Handle internals the served form uses to admit frames against the device
// memory its slots actually hold (not part of the public C ABI).
#pragma once
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
}  // namespace fmvs
