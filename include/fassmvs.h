/*
 * fassmvs.h -- C ABI of the MI355X (gfx950) implementation of the FaSS-MVS
 * hot path: hierarchical plane-sweep multi-image matching with a
 * census-Hamming or NCC cost (Alg. 1 of the paper; Eq. homography) followed
 * by surface-aware semi-global matching (Eq. sgm-path ... sgm-smooth-sn,
 * sgm-smooth-pg, Eq. p2-grad), winner-takes-all plane selection with
 * sub-plane depth refinement, normal map (Eq. normal, normal-smooth) and
 * geometric confidence (Eq. weight-normal), run coarse-to-fine over a
 * Gaussian pyramid (pipeline overview; Eq. sampling_range).  Around it: the
 * plane-set generator (bounding planes, cross-ratio steps of Alg. 2), the
 * post-filters (DoG texture mask, Alg. 3; geometric consistency, Alg. 4),
 * per-stage entry points on caller-owned device buffers, and a served form
 * for several concurrent UAV streams.
 *
 * The library is self-contained: plain C types, no exceptions cross the
 * boundary, every call returns a status.  Device memory is owned by the
 * handle unless a pointer is documented as caller-owned device memory.
 *
 * Coordinate conventions shared by every call:
 *  - images are row-major 8-bit grayscale; pixel (x, y) has its centre at
 *    (x + 0.5, y + 0.5) in the coordinates K maps camera rays to;
 *  - poses: x_cam = R x_world + t (R row-major), one intrinsic matrix K for
 *    all images (upper triangular, K[8] == 1);
 *  - a plane (n, delta) is { X : n^T X + delta = 0 } in reference-camera
 *    coordinates, n a unit vector facing the camera (n[2] < 0);
 *  - depth is the z coordinate in the reference camera; maps have the
 *    reference image's size; normals are unit vectors in reference-camera
 *    coordinates, xyz interleaved; invalid pixels get depth 0, normal 0 and
 *    confidence 0.
 */
#ifndef FASSMVS_H
#define FASSMVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fassmvs_handle fassmvs_handle;
typedef int32_t fassmvs_status;

#define FASSMVS_OK 0
#define FASSMVS_PENDING 1          /* frame still running on the device */
#define FASSMVS_EINVAL (-1)        /* bad argument (sizes, poses, plane behind a camera, > 256 planes) */
#define FASSMVS_EUNSUPPORTED (-2)  /* valid but not supported (census size, 8/16-bit cost bounds) */
#define FASSMVS_ENOMEM (-3)        /* device allocation failed or frame exceeds the HBM budget */
#define FASSMVS_EBUSY (-4)         /* a frame is already in flight on this handle; poll first */
#define FASSMVS_EDEVICE (-5)       /* HIP runtime error; the handle is latched, see fassmvs_last_error */
#define FASSMVS_ENOTFOUND (-6)     /* unknown or already consumed ticket */

#define FASSMVS_MEM_HOST 0
#define FASSMVS_MEM_DEVICE 1

#define FASSMVS_MAX_VIEWS 8        /* matching images per bundle */
#define FASSMVS_MAX_FAMILIES 8     /* plane orientations per frame */
#define FASSMVS_MAX_LABELS 512     /* labels per pixel at one level (sum of family windows) */
#define FASSMVS_MAX_TOP_PLANES 256 /* planes per family at the coarsest level (paper's cap) */
#define FASSMVS_MAX_LEVELS 5

/* Number of per-stage timers reported by fassmvs_stage_times. */
#define FASSMVS_N_STAGES 13

typedef struct {
    int32_t n_levels;          /* pyramid height n, 1..5 (pipeline overview) */
    int32_t census_w;          /* matching window width: census 3, 5, 7, 9; NCC 3, 5, 7, 9
                                  (similarity-measure experiment) */
    int32_t census_h;          /* matching window height: census 3, 5, 7 (with width 3, 5, 7, 9);
                                  NCC equal to the width */
    int32_t n_paths;           /* 8, or 4 (diagonals dropped) */
    int32_t sgm_variant;       /* 0: SGM^Pi; 1: SGM^Pi-sn below the coarsest level; 2: SGM^Pi-pg */
    int32_t p1;                /* P1 per matching image; census: scaled by m = max(|L|,|R|) */
    int32_t p2_mode;           /* 0: fixed P2; 1: adaptive P2 (Eq. p2-grad) */
    int32_t p2_fixed;          /* P2 per matching image in fixed mode (>= p1) */
    double p2_alpha;           /* alpha of Eq. p2-grad (paper: 8) */
    double p2_beta;            /* beta of Eq. p2-grad (paper: 10) */
    int32_t window_labels;     /* labels per family and pixel below the coarsest level; 0: whole list */
    int32_t median;            /* 1: 5x5 median on the depth map */
    int32_t normal_radius;     /* smoothing window radius r (sigma = r), 1..4 */
    double normal_beta;        /* beta of Eq. normal-smooth (paper: 10) */
    double conf_rho_deg;       /* critical angle of Eq. weight-normal (paper: 60) */
    int32_t device;            /* HIP device ordinal */
    void *stream;              /* hipStream_t to run on; NULL: the handle creates its own */
    uint64_t hbm_budget_bytes; /* device memory the handle may hold; 0: no limit */
    int32_t profile;           /* 1: time every stage with HIP events */
    int32_t keep_levels;       /* 1: keep per-level maps of the last frame (fassmvs_level_map) */
    int32_t sgm_debug;         /* 1: write every path's costs and the full aggregate (tests) */
    int32_t cost;              /* matching cost of Alg. 1 (Sec. on the similarity measures):
                                  0 census-Hamming, S = min over non-empty subsets X of
                                  floor(s^X m / |X|), P1 and fixed P2 scaled by m;
                                  1 negated, truncated and scaled NCC (0..255 per view),
                                  S = min over X of floor(s^X / |X|), penalties unscaled */
    int32_t dog_filter;        /* 1: apply the DoG texture filter (Alg. 3, see fassmvs_filter_dog)
                                  to the level-0 maps before they are returned */
} fassmvs_config;

typedef struct {
    const uint8_t *pixels;     /* host or device memory, see mem_kind */
    int32_t width, height;
    int32_t stride;            /* bytes between rows, >= width */
    double R[9];               /* row-major rotation, x_cam = R x_world + t */
    double t[3];
} fassmvs_image;

typedef struct {
    double n[3];               /* unit normal in reference-camera coordinates, n[2] < 0 */
    double delta_min;          /* nearest plane distance, > 0; with delta_max 0 and delta NULL:
                                  taken from the depth range (see depth_min) */
    double delta_max;          /* farthest plane distance, > delta_min */
    int32_t count;             /* planes at the coarsest level (2..256), uniform in 1/delta over
                                  [delta_min, delta_max]; with delta != NULL the length of that
                                  list.  0 (and delta NULL): the cross-ratio list (Alg. 2,
                                  fassmvs_cross_ratio_planes) at the coarsest level for the view
                                  with the longest epipolar segment, resampled to 256 planes
                                  when longer */
    const double *delta;       /* NULL, or the coarsest level's plane distances (host memory,
                                  count entries, > 0, strictly increasing or strictly decreasing;
                                  copied before the call returns): the paper's set of planes
                                  with varying distances (Alg. 1) */
    double depth_min;          /* depth range [depth_min, depth_max] of the reference view; when */
    double depth_max;          /* delta_min = delta_max = 0 and delta is NULL, the family's
                                  bounding planes (fassmvs_bounding_planes) give its range */
    /* Level l uses count * 2^(n-1-l) planes: the inverse distance is
     * interpolated linearly at the fractional indices j (count - 1) /
     * (G_l - 1) of the coarsest list (a list uniform in 1/delta stays
     * uniform).  The coarse-to-fine windows and the surface-normal offsets
     * index the level's list by the continuous index of an inverse distance
     * (piecewise linear between planes).  SGM^Pi-pg needs uniform lists. */
} fassmvs_plane_family;

/* Paper defaults: 8 paths, SGM^Pi, census 9x7, P1 24 (census 9x7 setting of
 * the similarity-measure experiment), adaptive P2 with alpha 8 and beta 10,
 * 5x5 median, normal radius 2, beta 10, rho 60 deg, 3 levels, window 128. */
void fassmvs_config_default(fassmvs_config *cfg);

/* Create a handle on cfg->device.  Validates the configuration (EINVAL /
 * EUNSUPPORTED) and creates the stream when cfg->stream is NULL.  Device
 * buffers are allocated lazily by the first frame and grow with the frame
 * size.  *out receives the handle (NULL on failure). */
fassmvs_status fassmvs_create(const fassmvs_config *cfg, fassmvs_handle **out);

/* Enqueue one frame (the problem statement of the pipeline overview: a
 * bundle of images with poses in, depth / normal / confidence maps of the
 * reference image out).
 *   ref, views: reference and n_views matching images, all of the
 *     reference's size; pixel memory is host memory (copied before return)
 *     or, with mem_kind FASSMVS_MEM_DEVICE, device memory read on the
 *     handle's stream (the caller keeps it valid until poll returns OK).
 *   view_side: per view -1 (before the reference in the sequence, left
 *     subset) or +1 (after it, right subset) for the occlusion-robust
 *     minimum of Alg. 1.
 *   K: intrinsics of level 0 (row-major).
 *   families, n_families: plane orientations and distance ranges.
 *   ticket: receives the frame's ticket.
 * One frame may be in flight per handle (EBUSY otherwise).  Errors:
 * EINVAL (sizes, non-finite pose, plane list, a camera centre behind the
 * nearest plane), EUNSUPPORTED (cost or aggregate overflow bounds),
 * ENOMEM, EDEVICE. */
fassmvs_status fassmvs_submit_frame(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                    const int8_t *view_side, int32_t n_views, const double K[9],
                                    const fassmvs_plane_family *families, int32_t n_families,
                                    int32_t mem_kind, uint64_t *ticket);

/* fassmvs_submit_frame with the reference view's depth range [d_min, d_max]
 * given once for the bundle (the problem statement's depth range): every
 * family with no explicit list and delta_min = delta_max = 0 takes its
 * distance range from the bounding planes of that depth range (Sec. on
 * bounding planes; as depth_min / depth_max of the family).  EINVAL when
 * 0 < d_min < d_max does not hold.  Per-stream state (keyframes, their
 * pyramids) belongs to the served form, whose calls take a stream id. */
fassmvs_status fassmvs_submit_frame_range(fassmvs_handle *h, const fassmvs_image *ref, const fassmvs_image *views,
                                          const int8_t *view_side, int32_t n_views, const double K[9], double d_min,
                                          double d_max, const fassmvs_plane_family *families, int32_t n_families,
                                          int32_t mem_kind, uint64_t *ticket);

/* Collect a frame's maps.  depth: W*H floats; normal: W*H*3 floats; confidence:
 * W*H floats in [0, 1]; any may be NULL.  mem_kind says whether the output
 * pointers are host or device memory.  wait_ms: 0 non-blocking, -1 blocking,
 * else a bound in milliseconds.  Returns PENDING while the frame runs, OK
 * once the maps are written (the ticket is then consumed), ENOTFOUND for an
 * unknown ticket. */
fassmvs_status fassmvs_poll(fassmvs_handle *h, uint64_t ticket, float *depth, float *normal, float *confidence,
                            int32_t mem_kind, int32_t wait_ms);

/* ---------------------------------------------------------------------
 * Batched frames: several bundles of uneven size, views, plane count and
 * pyramid height in one submission.  The frames are split into groups of
 * about equal work, each group on a stream of its own forked from and
 * joined back into the handle's stream.  A group runs level round by level
 * round (every frame's coarsest level first); in each round the sweeps of
 * its frames are one launch per tile height and their aggregations one
 * persistent launch per label-pair count over the paths of every frame and
 * direction.  Each group's launches can be captured in a HIP graph once per
 * batch shape and replayed while the shape and the buffers stay; the
 * sweep's tile height and workgroup count, the number of groups (up to 16)
 * and the graph are tuned once per shape by timing the candidates (none of
 * them changes a result).
 * Each frame's maps are those fassmvs_submit_frame gives for the same
 * bundle.
 * --------------------------------------------------------------------- */
#define FASSMVS_MAX_BATCH 64

typedef struct {
    const fassmvs_image *ref;        /* as fassmvs_submit_frame */
    const fassmvs_image *views;
    const int8_t *view_side;
    int32_t n_views;
    const double *K;                 /* 9 values, row-major */
    const fassmvs_plane_family *families;
    int32_t n_families;
    int32_t n_levels;                /* pyramid height of this frame; 0: the handle's */
    int32_t window_labels;           /* labels per family below the coarsest level; -1: the handle's */
} fassmvs_frame;

/* Enqueue n_frames (1..64) frames as one batch on the handle's stream.
 * Pixels as in fassmvs_submit_frame (host memory copied before return, or
 * device memory read on the stream).  The handle holds no other frame while
 * the batch runs (EBUSY).  Errors as fassmvs_submit_frame, naming the frame. */
fassmvs_status fassmvs_submit_batch(fassmvs_handle *h, const fassmvs_frame *frames, int32_t n_frames, int32_t mem_kind,
                                    uint64_t *ticket);

/* Maps of frame `index` of a batch (as fassmvs_poll); PENDING while the batch
 * runs.  The maps stay available until the next submission. */
fassmvs_status fassmvs_poll_batch(fassmvs_handle *h, uint64_t ticket, int32_t index, float *depth, float *normal,
                                  float *confidence, int32_t mem_kind, int32_t wait_ms);

/* What the batch tuner chose for the last batch shape: sweep rows per
 * thread (tile height / 4; 0: each frame level's own choice, as a single
 * frame would take it), sweep workgroup target, number of frame groups
 * (each on a stream of its own), whether the batch replays a captured graph
 * (1) or is launched call by call (0), and the measured time of one batch
 * in ms.  Any output may be NULL. */
fassmvs_status fassmvs_batch_tuning(fassmvs_handle *h, int32_t *rows_per_thread, int32_t *sweep_blocks, int32_t *groups,
                                    int32_t *graph, double *ms);

/* Wait for any frame in flight and release every resource of the handle. */
void fassmvs_destroy(fassmvs_handle *h);

/* Last error message of the handle (owned by the handle, valid until the
 * next call on it); "" if none.  h may be NULL (then: the last create error). */
const char *fassmvs_last_error(const fassmvs_handle *h);

/* Accumulated device time per stage in milliseconds and the number of
 * timed launches (cfg.profile = 1), for stage ids 0..n-1 (see
 * fassmvs_stage_name); reset with fassmvs_reset_stage_times. */
fassmvs_status fassmvs_stage_times(fassmvs_handle *h, double *ms, int32_t *counts, int32_t n);
fassmvs_status fassmvs_reset_stage_times(fassmvs_handle *h);
const char *fassmvs_stage_name(int32_t stage);

/* The same per-stage times for the steps of one pyramid level (0 = full
 * resolution); frame-wide steps (upload, pyramid, output) belong to no
 * level. */
fassmvs_status fassmvs_stage_times_level(fassmvs_handle *h, int32_t level, double *ms, int32_t *counts, int32_t n);

/* One timed step of a frame: stage id, pyramid level (-1: frame-wide),
 * start on the stream relative to the frame's submission, and duration. */
typedef struct {
    int32_t stage;
    int32_t level;
    double start_ms;
    double ms;
} fassmvs_timeline_entry;

/* The timeline of the last polled frame (cfg.profile = 1), in enqueue
 * order: up to max_entries entries into out, *n_entries the full count. */
fassmvs_status fassmvs_frame_timeline(fassmvs_handle *h, fassmvs_timeline_entry *out, int32_t max_entries,
                                      int32_t *n_entries);

/* Work units of the last frame, for throughput and roofline figures:
 * out[0] = sum over levels of pixels x labels (pixel-hypotheses),
 * out[1] = pixel-hypotheses x matching views, out[2] = labels actually
 * evaluated by the sweep (pixel-hypotheses including tile-union work),
 * out[3] = bytes the SGM stage moves by design, out[4 + l] = pixels x
 * labels of level l (0 for levels the frame does not have; n up to 9). */
fassmvs_status fassmvs_frame_work(fassmvs_handle *h, double *out, int32_t n);

/* Copy a per-level map of the last completed frame (cfg.keep_levels = 1)
 * into caller-owned device memory dst of dst_bytes.  what: 0 depth (float
 * W*H, after the median), 1 raw depth (before the median), 2 normal (float
 * W*H*3), 3 confidence, 4 global plane label (int32, -1 invalid), 5 family
 * (int32), 6 window offsets ([F][H][W] int32, levels below the coarsest),
 * 7 surface-normal offsets ([8][H][W][F] int8), 8 level width/height
 * (2 x int32 written to dst as host memory), 9 cost volume S of level 0
 * ([H][W][D] uint8), 10+r path costs of direction r at level 0 ([H][W][D]
 * uint16),
 * 20 reference census of level 0 ([H][W] uint64), 30+i pyramid image i of
 * the level (0 reference, 1.. views; [H][W] uint8). */
fassmvs_status fassmvs_level_map(fassmvs_handle *h, int32_t level, int32_t what, void *dst, size_t dst_bytes);

/* ---------------------------------------------------------------------
 * Plane set (host only, no handle): bounding planes and the cross-ratio
 * sampling steps.
 * --------------------------------------------------------------------- */

/* Bounding plane distances for plane normal n (unit, facing the camera) and
 * the depth range [d_min, d_max] (Sec. on bounding planes): the reference
 * frustum's corner rays through the image corners (0,0), (w,0), (0,h), (w,h)
 * meet the near plane z = d_min and the far plane z = d_max; out[0] = the
 * least |n^T X| over the near corners, out[1] = the largest over the far
 * corners.  EINVAL on bad input. */
fassmvs_status fassmvs_bounding_planes(const double K[9], int32_t w, int32_t hgt, const double n[3], double d_min,
                                       double d_max, double out[2]);

/* Plane distances whose images move by one pixel (Alg. 2, cross-ratio):
 * for the image corner (pixel centre) whose images in view k on the two
 * bounding planes lie farthest apart, points stepped one pixel apart along
 * that epipolar segment are mapped to plane distances through the
 * cross-ratio of the view-k rays to the epipole, the two segment ends and
 * the point.  R, t: reference -> view k (x_k = R x_ref + t).  The list runs
 * from delta_max down to delta_min (appended when the segment is not a
 * whole number of pixels).  *count receives its length; deltas (host,
 * max_planes entries) is written when it fits, else EUNSUPPORTED.  EINVAL
 * when the camera centre of view k is not in front of the nearest plane or
 * no corner ray meets both planes. */
fassmvs_status fassmvs_cross_ratio_planes(const double K[9], int32_t w, int32_t hgt, const double R[9],
                                          const double t[3], const double n[3], double delta_min, double delta_max,
                                          int32_t max_planes, double *deltas, int32_t *count);

/* ---------------------------------------------------------------------
 * Post-processing (Sec. on post-processing and depth map filtering).
 * Synchronous; maps are caller-owned device memory of one W x H frame.
 * --------------------------------------------------------------------- */

/* DoG texture filter (Alg. 3): the reference image img ([H][W] uint8) is
 * smoothed with a 7x7 Gaussian (sigma 1.4, replicate border, double), a
 * pixel is active where |I - I_smooth| > 0.5, activation areas of fewer than
 * 7 pixels (4-connected) are dropped, the mask is dilated by 3x3 and
 * deactivation areas of fewer than 21 pixels are filled.  Where the mask is
 * 0 (weak texture) depth, normal (xyz) and confidence are set to 0; any map
 * may be NULL.  mask_out (NULL or [H][W] uint8) receives the mask (1 kept). */
fassmvs_status fassmvs_filter_dog(fassmvs_handle *h, const uint8_t *img, int32_t w, int32_t hgt, float *depth,
                                  float *normal, float *confidence, uint8_t *mask_out);

/* Allocation-free DoG texture filter, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same filter and results as
 * fassmvs_filter_dog, with its scratch (a double image and two u8 masks,
 * 10 bytes per pixel) in a static device array of 40 MiB that each device
 * holds from module load until the process ends.  Calls no allocating
 * routine.  Images of more than 4194304 pixels (2^22) are rejected with
 * EINVAL.  Every call on one device shares that device's array, so calls
 * that overlap on one device (several handles or threads) race; serialise
 * them.  Synchronous on the handle's stream like fassmvs_filter_dog. */
fassmvs_status fassmvs_filter_dog_noalloc(fassmvs_handle *h, const uint8_t *img, int32_t w, int32_t hgt,
                                          float *depth, float *normal, float *confidence, uint8_t *mask_out);

/* Geometric consistency by mutual reprojection (Alg. 4) of a reference depth
 * map against n_nb (1..8) neighbouring depth maps of the same size:
 * depth_nb[k] device pointers, R_rel / t_rel host arrays (n_nb x 9, n_nb x 3,
 * row-major) of the relative poses reference -> neighbour (x_k = R x_ref + t),
 * K the shared intrinsics.  A pixel with depth d > 0 counts a hit for map k
 * when its point d K^-1 p, seen in k, lands on a pixel with depth d_k > 0
 * whose point maps back within eta_r pixels of p (misses outside the image
 * or behind a camera); pixels with fewer than eta_h hits get depth, normal
 * and confidence 0.  hits_out / keep_out: NULL or [H][W] int32 / uint8. */
fassmvs_status fassmvs_filter_geometric(fassmvs_handle *h, int32_t w, int32_t hgt, const double K[9], float *depth,
                                        float *normal, float *confidence, int32_t n_nb, const float *const *depth_nb,
                                        const double *R_rel, const double *t_rel, double eta_r, int32_t eta_h,
                                        int32_t *hits_out, uint8_t *keep_out);

/* ---------------------------------------------------------------------
 * Served form (online mapping from several UAV streams).
 *
 * The online use the paper discusses with its run-times (Sec. on the
 * discussion of run-time and online processing): one moving camera per
 * sequence, frames used only with an appropriate baseline between them,
 * and a new estimate for every new usable frame that reuses the images of
 * the previous bundle.  Here the bundle is the frame and its stream's
 * previous keyframes (a one-sided bundle; the paper takes the middle image
 * of a bundle as reference, which would delay every estimate by half a
 * bundle).
 *
 * Frames of several streams are submitted as they arrive; each is matched
 * against its stream's previous keyframes (up to max_keyframes, all before
 * it in the sequence: a one-sided bundle, m = number of keyframes; a frame
 * becomes a keyframe when its camera centre moved at least min_baseline
 * since the last keyframe, the first frame always does), so the stream's
 * keyframe images stay on the device.  A worker thread admits queued frames
 * in arrival order into n_slots pipeline slots (each a handle with its own
 * HIP stream, so admitted frames run concurrently) while the device memory
 * the slots hold plus the growth the frame needs on its slot stays within
 * the budget (a slot's buffers grow only while no frame is in flight; idle
 * slots release theirs when the budget is short), and collects finished
 * frames into result maps on the device.
 * Results are the same as the plain pipeline's on the same bundle.
 * --------------------------------------------------------------------- */
typedef struct fassmvs_server fassmvs_server;

typedef struct {
    uint64_t request_id;
    int32_t stream_id;
    int32_t status;            /* OK, ENOTFOUND (no keyframe to match against yet), or the frame's error */
    int32_t width, height;
    int32_t keyframe;          /* 1 if the frame became a keyframe */
    int32_t n_views;           /* keyframes it was matched against */
    double latency_ms;         /* submit call to maps ready on the device */
} fassmvs_server_result;

/* Device bytes one frame holds while it runs (cost volume, path-cost
 * buffers, pyramids, per-level maps); families with count 0 are counted
 * at the 256-plane cap. */
fassmvs_status fassmvs_frame_footprint(const fassmvs_config *cfg, int32_t w, int32_t hgt, int32_t n_views,
                                       const fassmvs_plane_family *families, int32_t n_families, uint64_t *bytes);

/* Create a server with n_slots (1..16) concurrent pipeline slots, all with
 * cfg (cfg->stream is ignored: every slot creates its own).  hbm_budget_bytes
 * 0: 80 % of the device memory free at creation. */
fassmvs_status fassmvs_server_create(const fassmvs_config *cfg, int32_t n_slots, uint64_t hbm_budget_bytes,
                                     fassmvs_server **out);

/* Open a stream of width x height frames with intrinsics K and plane
 * families; *stream_id receives its id. */
fassmvs_status fassmvs_server_open_stream(fassmvs_server *s, const double K[9], int32_t width, int32_t height,
                                          const fassmvs_plane_family *families, int32_t n_families,
                                          int32_t max_keyframes, double min_baseline, int32_t *stream_id);

/* Submit the next frame of a stream (host pixels, copied to the device before
 * return; pose x_cam = R x_world + t).  The arrival time for the latency is
 * the moment of the call.  ENOMEM if the frame's footprint exceeds the whole
 * budget. */
fassmvs_status fassmvs_server_submit(fassmvs_server *s, int32_t stream_id, const uint8_t *pixels, int32_t stride,
                                     const double R[9], const double t[3], uint64_t *request_id);

/* Next finished request in completion order: wait_ms 0 non-blocking, -1
 * blocking, else a bound; PENDING if none.  Its maps (status OK) stay on
 * the device until fetched. */
fassmvs_status fassmvs_server_next(fassmvs_server *s, int32_t wait_ms, fassmvs_server_result *out);

/* Copy a finished request's maps (depth W*H, normal W*H*3, confidence W*H
 * floats; any NULL) to host or device memory and release them; ENOTFOUND
 * if the request has no maps or was fetched already. */
fassmvs_status fassmvs_server_fetch(fassmvs_server *s, uint64_t request_id, float *depth, float *normal,
                                    float *confidence, int32_t mem_kind);

/* Stop taking frames of a stream and drop its keyframes. */
fassmvs_status fassmvs_server_close_stream(fassmvs_server *s, int32_t stream_id);

const char *fassmvs_server_last_error(const fassmvs_server *s);

/* Finish every queued and running frame, then release everything. */
void fassmvs_server_destroy(fassmvs_server *s);

/* ---------------------------------------------------------------------
 * Device-memory plumbing for callers without their own HIP allocator
 * (tests, benchmark).  All run on the handle's device and stream.
 * --------------------------------------------------------------------- */

/* Allocate / free device memory (hipMalloc / hipFree). */
fassmvs_status fassmvs_device_alloc(fassmvs_handle *h, size_t bytes, void **ptr);
fassmvs_status fassmvs_device_free(fassmvs_handle *h, void *ptr);

/* Copy bytes; kind 0 host->device, 1 device->host, 2 device->device.
 * Returns when the copy has completed (the handle's stream is drained first).
 * A device->device copy of non-overlapping, 16-byte aligned buffers whose size
 * is a multiple of 16 runs the library's own plain copy kernel (k_copy16),
 * which touches every byte once; other copies use hipMemcpyAsync.  Ranges
 * that overlap are copied by hipMemcpyAsync with its semantics. */
fassmvs_status fassmvs_memcpy(fassmvs_handle *h, void *dst, const void *src, size_t bytes, int32_t kind);

/* Fill device memory with a byte value (a fill kernel, not a memset node). */
fassmvs_status fassmvs_fill(fassmvs_handle *h, void *dst, uint8_t value, size_t bytes);

/* Wait until everything enqueued on the handle's stream has completed. */
fassmvs_status fassmvs_synchronize(fassmvs_handle *h);

/* ---------------------------------------------------------------------
 * Stage entry points.  Each runs one kernel of the frame pipeline on
 * caller-owned device buffers (dense, row-major, no padding) and returns
 * when it has completed.  They exist so that every stage can be checked on
 * its own inputs; the frame pipeline uses the same kernels.
 * --------------------------------------------------------------------- */

/* Gaussian pyramid step (pipeline overview): 3x3 blur with taps
 * (70,116,70)/256, replicate border, rounding after each pass, then the mean
 * of each 2x2 block.  src w*h, dst (w/2)*(h/2). */
fassmvs_status fassmvs_stage_pyr_down(fassmvs_handle *h, const uint8_t *src, int32_t w, int32_t hgt, uint8_t *dst);

/* Census transform of an 8-bit image (Alg. 1 cost): bit (nbits-1-b) of the
 * result is [I(q_b) < I(p)] for the b-th window position q_b in row-major
 * order, centre skipped, replicate border.  cw x ch odd, cw*ch-1 <= 64. */
fassmvs_status fassmvs_stage_census(fassmvs_handle *h, const uint8_t *img, int32_t w, int32_t hgt, int32_t cw,
                                    int32_t ch, uint64_t *out);

/* Warp one matching image onto the reference grid (Alg. 1): the value at
 * reference pixel q is the bilinear, clamp-to-edge sample of src at
 * H (q + 0.5) - 0.5 on the 0..255 scale (float).  H row-major (host). */
fassmvs_status fassmvs_stage_warp(fassmvs_handle *h, const uint8_t *src, int32_t sw, int32_t sh, const double H[9],
                                  int32_t rw, int32_t rh, float *out);

/* Cost volume (Alg. 1): S[y][x][l] (uint8) for every reference pixel and
 * label l of the concatenated families, each family f contributing W[f]
 * labels from global index offs[f][y][x] (or all of its G[f] planes when
 * offs is NULL).  views: n_views device pointers (host array) to w*h
 * matching images; H: host array [n_views][sum G][9]; ct_ref from
 * fassmvs_stage_census.  With warped != NULL the warp is skipped and the
 * pre-warped float images [n_views][sum G][h][w] are read instead. */
fassmvs_status fassmvs_stage_cost(fassmvs_handle *h, int32_t w, int32_t hgt, const uint64_t *ct_ref,
                                  int32_t n_views, const uint8_t *const *views, const int8_t *view_side,
                                  int32_t cw, int32_t ch, int32_t n_fam, const int32_t *G, const int32_t *W,
                                  const double *H, const int32_t *offs, const float *warped, uint8_t *S);

/* The NCC cost volume (Alg. 1 with the negated, truncated and scaled NCC of
 * the similarity-measure section): for every pixel, label and view the
 * cw x ch window of the reference image ref_img (caller-owned device
 * memory, [h][w] uint8, replicate border) against the same window of the
 * warped view; per view C = floor(255 min(1, 1 - rho) + 0.5) with rho the
 * correlation coefficient (sums in double, 0 for a flat window); S = min
 * over the non-empty subsets of the subset's mean cost.  Other arguments
 * and errors as fassmvs_stage_cost; window sizes 3x3, 5x5, 7x7, 9x9. */
fassmvs_status fassmvs_stage_cost_ncc(fassmvs_handle *h, int32_t w, int32_t hgt, const uint8_t *ref_img,
                                      int32_t n_views, const uint8_t *const *views, const int8_t *view_side,
                                      int32_t cw, int32_t ch, int32_t n_fam, const int32_t *G, const int32_t *W,
                                      const double *H, const int32_t *offs, const float *warped, uint8_t *S);

/* Semi-global aggregation and winner-takes-all (Eq. sgm-path, sgm-aggr,
 * sgm-wta with the smoothness terms of Eq. sgm-smooth-fp / sgm-smooth-sn).
 *   S [h][w][D] uint8, D = sum W; offs [F][h][w] int32 or NULL; dI
 *   [8][h][w][F] int8 or NULL; ref [h][w] level image for P2 = lut[|dI|];
 *   lut: host int32[256]; p1: effective P1.
 * Outputs (any may be NULL): Lr [n_paths][h][w][D] uint16 per-path costs;
 * Sbar [h][w][D] uint16 aggregate; wta [h][w] uint16 winning label (local,
 * smallest on ties); c3 [h][w][3] uint16 aggregate at winner-1, winner,
 * winner+1 (0xFFFF where the neighbour is outside the family's window). */
fassmvs_status fassmvs_stage_sgm(fassmvs_handle *h, int32_t w, int32_t hgt, int32_t n_fam, const int32_t *W,
                                 const uint8_t *S, const int32_t *offs, const int8_t *dI, const uint8_t *ref,
                                 int32_t p1, const int32_t *lut, int32_t n_paths, uint16_t *Lr, uint16_t *Sbar,
                                 uint16_t *wta, uint16_t *c3);

/* SGM^Pi-pg (Eq. sgm-smooth-pg): as fassmvs_stage_sgm, with the zero-cost
 * transition shifted by the path-gradient offset -- the inverse depth of the
 * path's two previous minimum-cost points, extrapolated to the pixel and
 * expressed as a plane-index jump per family (rounded, clamped to +-7).
 * Host arrays: G [F] list sizes, fam_delta (concatenated lists, sum G <= 2048),
 * fam_n [F][3], Kinv [9] of the level, step [F] (inverse-distance step). */
fassmvs_status fassmvs_stage_sgm_pg(fassmvs_handle *h, int32_t w, int32_t hgt, int32_t n_fam, const int32_t *W,
                                    const int32_t *G, const uint8_t *S, const int32_t *offs, const uint8_t *ref,
                                    int32_t p1, const int32_t *lut, int32_t n_paths, const double *fam_delta,
                                    const double *fam_n, const double *Kinv, const double *step, uint16_t *Lr,
                                    uint16_t *Sbar, uint16_t *wta, uint16_t *c3);

/* Depth of the winning plane and parabola refinement (depth extraction for
 * SGM^Pi; depth refinement): from wta and c3 of fassmvs_stage_sgm.  Host
 * arrays: fam_n [F][3], fam_delta (concatenated level plane lists, sum G),
 * Kinv [9] of the level.  Outputs label (global, -1 invalid), fam, depth. */
fassmvs_status fassmvs_stage_refine(fassmvs_handle *h, int32_t w, int32_t hgt, int32_t n_fam, const int32_t *W,
                                    const int32_t *G, const int32_t *offs, const uint16_t *wta, const uint16_t *c3,
                                    const double *fam_n, const double *fam_delta, const double *Kinv,
                                    int32_t *label, int32_t *fam, float *depth);

/* 5x5 median (pipeline overview), replicate border, 13th of 25. */
fassmvs_status fassmvs_stage_median(fassmvs_handle *h, const float *in, int32_t w, int32_t hgt, float *out);

/* Normals (Sec. extraction of surface normals), then appearance-weighted
 * smoothing (Eq. normal, normal-smooth) and confidence (Eq. weight-normal).
 * depth [h][w]; img [h][w] level reference image; label/fam from
 * fassmvs_stage_refine; Kinv, fam_n host arrays.  Outputs nraw (may be NULL),
 * normal [h][w][3], conf [h][w]. */
fassmvs_status fassmvs_stage_normals(fassmvs_handle *h, const float *depth, const uint8_t *img, int32_t w,
                                     int32_t hgt, const double *Kinv, int32_t radius, double beta,
                                     const int32_t *label, const int32_t *fam, int32_t n_fam,
                                     const double *fam_n, double rho_deg, float *nraw, float *normal,
                                     float *conf);

/* Coarse-to-fine seeds (pipeline overview; dynamic cost volume;
 * Eq. sgm-smooth-sn): nearest-neighbour upsampling of the coarse depth and
 * normal (cw x ch) to the fine level (fw x fh), the per-family sampling
 * windows (W[f] planes centred on the rounded continuous index of the seed
 * point's inverse distance in the family's list of the fine level) and,
 * when dI != NULL, the surface-normal index offsets for the 8 path
 * directions (difference of continuous indices, rounded half away from
 * zero, clamped to +-7).  Kinv: fine level; host arrays fam_n [F][3],
 * fam_delta (the fine level's lists of every family, concatenated,
 * increasing distances), G, W per family. */
fassmvs_status fassmvs_stage_seed(fassmvs_handle *h, const float *depth_c, const float *normal_c, int32_t cw,
                                  int32_t ch, int32_t fw, int32_t fh, const double *Kinv, int32_t n_fam,
                                  const double *fam_n, const double *fam_delta, const int32_t *G, const int32_t *W,
                                  float *dbar, float *nbar, int32_t *offs, int8_t *dI);

#ifdef __cplusplus
}
#endif

#endif /* FASSMVS_H */
