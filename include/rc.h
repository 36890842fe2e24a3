/*
 * rc.h -- C ABI of librc: occlusion-aware second-order radiance-cache records
 * in a homogeneous isotropic participating medium, computed on AMD Instinct
 * MI355X (gfx950).
 *
 * Method: Marco, Jarabo, Jarosz, Gutierrez, "Second-Order Occlusion-Aware
 * Volumetric Radiance Caching", ACM TOG 37(2), 2018.  Section and equation
 * names below refer to that paper.
 *
 * Conventions for every entry point
 *   - Pointers documented "device" must point to GPU memory of the current HIP
 *     device; pointers documented "host" to ordinary host memory.  The caller
 *     owns every buffer.  The library owns only the opaque scene handle.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls that take a stream only enqueue work; outputs are valid after the
 *     stream is synchronised.
 *   - Return value: RC_OK or a negative error code.  Arguments are validated
 *     on the host before anything is enqueued; on error nothing is enqueued
 *     and no output is written.  rc_last_error() returns a thread-local text
 *     describing the last failure of the calling thread.
 *   - Values that live only on the device (positions, sample counts) cannot
 *     be validated on the host; records whose device inputs are invalid
 *     (position outside the medium box or not finite, n_theta < 2,
 *     n_phi < 5 or n_phi > params.max_n_phi) are written as NaN and counted
 *     in the workspace's error counter (rc_workspace_errors).
 */
#ifndef RC_H_
#define RC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RC_OK 0
#define RC_EINVAL (-1)   /* invalid argument */
#define RC_ENOMEM (-2)   /* host or device allocation failed */
#define RC_EDEVICE (-3)  /* HIP runtime error (text in rc_last_error) */
#define RC_ENODEV (-4)   /* no usable gfx950 device */
#define RC_ETIMEOUT (-5) /* rc_records_wait: no record finished within the time limit */

#define RC_MAX_LIGHTS 16
#define RC_MAX_RINGS 64
#define RC_MAX_NPHI 256
#define RC_NOALLOC_MAX_RECORDS 4096 /* largest batch of rc_records_noalloc */
#define RC_MARCH_MAX_POINTS_PER_RAY 1048576 /* bound on medium box diagonal / march step */
/* int32 words of the placement state (5 counters + 4096 batch status words) */
#define RC_PLACE_STATE_INTS 4101

typedef struct rc_scene rc_scene;

/* Homogeneous isotropic medium (Table notation; Sec. 4 restricts the method
 * to isotropic homogeneous media).  mu_t = sigma_s + sigma_a. */
typedef struct {
  float sigma_s;
  float sigma_a;
} rc_medium;

/* Point light (Sec. 6, Implementation: point lights are handled separately
 * with shadow rays).  Radiant intensity `intensity` (W/sr). */
typedef struct {
  float pos[3];
  float intensity;
} rc_point_light;

/* Record parameters.
 *   ring_step : spacing of the concentric medium rings (Sec. 6: uniform
 *               ray marching of the medium around x); ring i lies at
 *               (i + xi) * ring_step with one jitter xi per record.
 *   max_rings : rings considered per direction (1..RC_MAX_RINGS); rings past
 *               max_rings * ring_step are ignored.  ceil(box diagonal /
 *               ring_step) + 1 never truncates.
 *   max_n_phi : upper bound of n_phi over the call (5..RC_MAX_NPHI); sizes
 *               the on-chip row buffers.
 *   seed      : seed of the counter-based generator (splitmix64).
 *   rec_base  : record id of pos[0]; record i draws its random numbers with
 *               id rec_base + i (so a subset of a large batch can be
 *               recomputed exactly).
 *   common_random : 0 (default) as above; 1 = every record of the call uses
 *               id rec_base, i.e. the same directions and ring jitter at
 *               every point (common random numbers: records then differ
 *               only through the scene, which makes a cache's interpolation
 *               error measurable apart from Monte Carlo noise).
 *   splits    : wavefronts per record, 0 = automatic (batches of up to 16384
 *               records split each record's strata rows over 1..8
 *               wavefronts, each recomputing one boundary row, as a model of
 *               the launch's makespan suggests: small batches finish sooner);
 *               1..8 forces a count (more than 1 needs P <= 16384).  Parts
 *               leave FP64 partial sums that the last one adds in part order,
 *               so results are deterministic for a given count and differ
 *               from an unsplit record only in FP64 rounding.
 *   precision : 0 = FP32 terms with the two quantities that cancel for
 *               near-degenerate (thin) triangles -- the direction
 *               determinant and grad A -- in FP64, compensated FP32 sums,
 *               FP64 final reduction (default); 1 = every triangle term in
 *               FP64 (study mode).
 *   counters  : device uint64_t[12] or NULL.  If set, the launch also
 *               counts (atomically added): rays traced, BVH nodes visited,
 *               ray/triangle tests, triangle terms evaluated, the shader
 *               clocks each wavefront spent in primary rays, shadow rays, the
 *               Monte Carlo value and the triangle terms (summed over
 *               wavefronts), then for the shadow-ray loop: iterations
 *               (per wavefront), busy lanes summed over iterations, refill
 *               events and lanes refilled.  With light bins, "BVH nodes
 *               visited" counts bin lists opened and "ray/triangle tests"
 *               the entries read.
 *   shadow_bvh : 0 (default) = shadow segments from the per-light triangle
 *               bins (built and cached on the scene at the first call with
 *               a new set of light positions, see rc_light_bins_build);
 *               1 = BVH traversal.  Both give the answer of testing every
 *               triangle, so records are identical.
 *   max_n_theta : largest n_theta of the call, or 0 (unknown).  With a
 *               bound, rc_records_batched traces every primary ray of the
 *               batch first, in a separate launch where each wavefront
 *               takes one stratum of 64 consecutive queued records (nearby
 *               points, nearly parallel rays), into a buffer the scene holds
 *               (8 B per ray: ceil(P / 64) * 64 * (max_n_theta * max_n_phi
 *               + 2) rays); the record kernel then reads the hits.  The hits
 *               are those of the record kernel's own traversal, so records
 *               are identical.  Records with n_theta above the bound are
 *               invalid (NaN, counted).  Not with counters.
 *   shadow_pass : 1 = with the hits pass and light bins, the same pass also
 *               walks the shadow segments of every vertex of its rays (the
 *               surface vertex and the ring vertices, each light) and stores
 *               their visibility bits (ceil((max_rings + 1) / (32 / B))
 *               words per ray, B = the smallest power of two >= n_lights,
 *               at most 4 words, else off); the record kernel reads them.
 *               Same segments, same bits.  0 = the record kernel walks
 *               them (spread over all the vertices of a row, it keeps its
 *               lanes busier: measured faster on the 200k- and 1M-triangle
 *               scenes, 385 vs 433 ms and 3.46 vs 3.87 s; slower on the
 *               10k-triangle one, 13.5 vs 12.9 ms). */
typedef struct {
  float ring_step;
  int32_t max_rings;
  int32_t max_n_phi;
  int32_t precision;
  int32_t common_random;
  int32_t splits;
  uint64_t seed;
  int64_t rec_base;
  uint64_t* counters;
  int32_t shadow_bvh;
  int32_t max_n_theta;
  int32_t shadow_pass;
} rc_params;

/* Scene statistics reported by rc_scene_info. */
typedef struct {
  int64_t n_tri;
  int64_t n_nodes;
  int32_t depth;
  int32_t leaf_max;
  int64_t node_bytes;
  int64_t tri_bytes;
  float pad;
  int64_t device_bytes;      /* device memory of the scene: nodes, the three
                                triangle copies, shading, FP64 planes, emission */
  int64_t light_bin_bytes;   /* device memory of the light bins of the last
                                light set (0 until a launch or
                                rc_light_bins_build made them) */
  int64_t light_bin_entries; /* (triangle, bin) entries in those bins */
} rc_scene_stats;

/* ------------------------------------------------------------------ */
/* Scenes                                                               */
/* ------------------------------------------------------------------ */

/* Build the traversal structure of a triangle scene on the host and upload
 * it to the current device.
 *   tri      : host float[T][9], vertices (v0, v1, v2) of each triangle.
 *   albedo   : host float[T], Lambertian reflectance of each triangle
 *              (two-sided, Sec. 4 restricts to Lambertian surfaces).
 *   emission : host float[T] emitted radiance per triangle, or NULL (none).
 *              Emitters are area lights sampled through the strata (Sec. 6).
 *   box_lo/hi: host float[3], the medium's axis-aligned extent.  Every
 *              triangle must lie inside it (within 1e-4 of its size).
 * On success *out receives a handle; free it with rc_scene_destroy.
 * Errors: RC_EINVAL (T < 0, null pointers, non-finite data, empty box,
 * triangle outside the box), RC_ENOMEM, RC_EDEVICE. */
int rc_scene_create(const float* tri, const float* albedo, const float* emission, int64_t T,
                    const float box_lo[3], const float box_hi[3], rc_scene** out);
int rc_scene_destroy(rc_scene* scene);
int rc_scene_info(const rc_scene* scene, rc_scene_stats* out);

/* Build only the host traversal structure (no device), for inspection.
 * nodes: host float[max_nodes][16] or NULL, tris: host float[T][12] or NULL.
 * Returns the number of nodes (>= 1) or a negative error code. */
int64_t rc_bvh_build_host(const float* tri, int64_t T, const float box_lo[3], const float box_hi[3],
                          float* nodes, int64_t max_nodes, float* tris, rc_scene_stats* stats);

/* ------------------------------------------------------------------ */
/* Workspace                                                            */
/* ------------------------------------------------------------------ */
/* Every launch needs a device workspace owned by the caller (queue
 * counters, error counter, the device-built queue, and for batches of up to
 * 16384 records the per-record part counters and FP64 partial sums of split
 * records).  Size in bytes for up to P records: */
size_t rc_workspace_size(int64_t P);
/* Copy the workspace's invalid-record counter to the host (synchronises
 * `stream`).  Returns the count (>= 0) or a negative error code. */
int64_t rc_workspace_errors(const void* workspace, void* stream);

/* ------------------------------------------------------------------ */
/* Records (Sec. 4; Sec. 6 Implementation)                              */
/* ------------------------------------------------------------------ */
/* Compute one radiance-cache record per cache point.
 *   lights  : host rc_point_light[n_lights], 0 <= n_lights <= RC_MAX_LIGHTS.
 *   pos     : device float[P][3], cache points inside the medium box.
 *   n_theta : device int32[P], strata rows in z   (equal-solid-angle strata,
 *   n_phi   : device int32[P], strata columns in phi  Sec. 6 Implementation).
 *   value   : device double[P][2]  channel 0 = surface (single scattering from
 *             the first surface along each direction), channel 1 = medium
 *             (light in-scattered by the medium rings).  Unbiased Monte Carlo
 *             estimate of Eq. outLF divided by sigma_s(x): the integral of
 *             f_s L_i over the sphere with f_s = 1/(4 pi).
 *   grad    : device double[P][2][3], triangulated gradient
 *             (Eq. SegmentRadianceGradient with Eq. SSSegALGradientSimp).
 *   hess    : device double[P][2][6], triangulated Hessian (xx, xy, xz, yy,
 *             yz, zz) (Eq. SegmentRadianceHessian with SSSegALHessianSimp;
 *             form factor derivatives of App. C, transmittance of App. A).
 *   workspace: device, at least rc_workspace_size(P) bytes.
 * The launch is one persistent kernel: each wavefront pops a record (or one
 * part of a split record, see rc_params.splits) from a queue in `workspace`
 * and computes it on chip. */
int rc_records(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
               const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
               const rc_params* params, double* value, double* grad, double* hess,
               void* workspace, void* stream);

/* rc_records without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as rc_records (the same
 * kernels, bit for bit) without the workspace: the queue, error counter and
 * split-record partial sums live in a workspace of rc_workspace_size(4096)
 * bytes (5.3 MiB) that the library holds in device memory on each device
 * it runs on until the process ends.
 *   P       : 0 <= P <= RC_NOALLOC_MAX_RECORDS, else RC_EINVAL.
 *   The current device must be the scene's device (else RC_EINVAL).
 * Shadow segments come from the scene's light bins if it already holds them
 * for these lights (an earlier rc_records call or rc_light_bins_build with the
 * same positions), else from the BVH, which gives the same segments; no bins
 * are built.  Calls no hipMalloc, hipFree or allocating library routine.
 * All calls on one device share its workspace, which keeps the last call's
 * contents: calls that overlap on one device (two streams, or two threads)
 * race, and so does a call that overlaps one that changes the scene's light
 * set.  The invalid-record count of the last call is read with
 * rc_records_noalloc_errors. */
int rc_records_noalloc(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights,
                       int n_lights, const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                       const rc_params* params, double* value, double* grad, double* hess, void* stream);
/* Invalid records of the last rc_records_noalloc call on the current device
 * (synchronises `stream`).  Returns the count (>= 0) or a negative error. */
int64_t rc_records_noalloc_errors(void* stream);

/* Same records, scheduled from a caller-supplied queue.
 *   order     : device int32[P] permutation of 0..P-1, the order in which
 *               records are popped (e.g. most expensive first), or NULL to
 *               build one on the device: records grouped by n_phi class
 *               (<= 16, 32, 64, 128, 256; widest first), then by octave of
 *               n_theta * n_phi (largest first), then by cell of an 8x8x8
 *               grid over the medium box in Morton order (records in flight
 *               together lie close together and share the caches).  With the
 *               device-built queue, batches of more than 16384 records are
 *               launched once per class, each launch sized (LDS, occupancy)
 *               for its class.
 *   use_graph : nonzero = capture the queue reset and the persistent
 *               launch(es) in a hipGraph on first use for these arguments and
 *               replay it afterwards (the graph is cached in the scene
 *               handle).
 *   tile      : launch configuration index from rc_autotune, or -1 = default.
 * Outputs are identical (bitwise) to rc_records for the same inputs and
 * params (the same number of parts per record is chosen for both). */
int rc_records_batched(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights,
                       int n_lights, const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                       const rc_params* params, const int32_t* order, int use_graph, int tile,
                       double* value, double* grad, double* hess, void* workspace, void* stream);

/* Watchdog for a record call on `stream` (rc_records or
 * rc_records_batched with this workspace): waits until the stream has
 * finished the work queued on it so far; returns RC_ETIMEOUT if it has not
 * and no record (or record part) has finished for timeout_ms milliseconds.
 * The record kernel counts finished records in the workspace, and this call
 * reads that count through a copy on a stream of its own, so it sees
 * progress while the kernel runs.  A timeout does not stop the kernel: the
 * caller decides what to do (the stream stays busy).  Errors: EINVAL,
 * EDEVICE. */
int rc_records_wait(const void* workspace, int timeout_ms, void* stream);

/* Time every launch configuration on the given inputs (synchronises
 * `stream`) and return the fastest configuration index in *best_tile; the
 * per-configuration milliseconds (mean of two runs after a warm-up run) go
 * to ms_out[n_tiles] if non-NULL (n_tiles <= 16).  A configuration sets the
 * persistent grid (a multiple of the resident wavefronts), the idle-lane
 * threshold that refills the BVH shadow loop, the waiting-lane threshold of
 * a triangle step, and the resident wavefronts per SIMD the LDS row width
 * is sized for (4, 3 or 2: wider rows need fewer column sectors but hide
 * less latency).  The result is remembered in the on-disk cache
 * `cache_path` (a text file; NULL = no cache) keyed by device name, scene
 * size and workload shape. */
int rc_autotune(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
                const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                const rc_params* params, double* value, double* grad, double* hess, void* workspace,
                const char* cache_path, int* best_tile, float* ms_out, int* n_tiles, void* stream);
/* The settings of launch configuration `tile` (0 <= tile < n_tiles of
 * rc_autotune): grid multiple, refill threshold, triangle-step threshold, LDS
 * wavefronts per SIMD.  Host only.  Errors: EINVAL (tile out of range or a
 * NULL output). */
int rc_tile_info(int tile, float* grid, int* refill_min, int* leaf_batch, int* lds_waves);

/* ------------------------------------------------------------------ */
/* Validity radius (Sec. 5, Eq. radiusAniso3D; supplement Eq. S.13)     */
/* ------------------------------------------------------------------ */
/* L = value[i][0] + value[i][1], H = hess[i][0] + hess[i][1].
 * R_k = (15 L eps / (4 pi |lambda_k|))^(1/5) for each eigenvalue lambda_k of
 * H, clamped to [r_min, r_max]; lambda_k = 0 gives r_max, L <= 0 gives
 * r_min.  R[i] = min_k R_k (isotropic point with the smallest principal
 * axis, Sec. 6).  axes: device float[P][12] or NULL: (R_1, R_2, R_3, then the
 * three unit eigenvectors, row-major) for anisotropic points.
 * value/hess device double, R device float[P]. */
int rc_radius(const double* value, const double* hess, int64_t P, float eps, float r_min, float r_max,
              float* R, float* axes, void* stream);

/* ------------------------------------------------------------------ */
/* Ray queries (the traversal the record kernel uses, one ray per lane)  */
/* ------------------------------------------------------------------ */
/* Closest hit of rays o + t d, t > 0 (watertight ray/triangle test of Woop,
 * Benthin and Wald 2013: FP32 projection along the ray, edge functions with
 * exact signs, t rounded once to FP32; every ray that meets a closed mesh
 * hits it, at any angle; ties to the lowest triangle index).  orig/dir device float[n][3]; hit_id device int32[n] (triangle
 * index or -1), t device float[n] (hit distance, or the exit distance from
 * the medium box when nothing is hit), front device int32[n] (1 if the ray
 * travels against the triangle normal (v1-v0) x (v2-v0)). */
int rc_trace_rays(const rc_scene* scene, const float* orig, const float* dir, int64_t n, int32_t* hit_id, float* t,
                  int32_t* front, void* stream);
/* Shadow segments o -> o + seg: occ[i] = 1 if a triangle other than skip[i]
 * is hit with 1e-4 < t < 1.  skip device int32[n] or NULL (none). */
int rc_occluded_rays(const rc_scene* scene, const float* orig, const float* seg, const int32_t* skip, int64_t n,
                     int32_t* occ, void* stream);

/* ------------------------------------------------------------------ */
/* Per-light triangle bins (the shadow-segment structure of the record   */
/* kernel; point lights with shadow rays, Sec. 6)                       */
/* ------------------------------------------------------------------ */
/* Seen from a point light, the directions are split into the six faces of a
 * cube and each face into bins at up to 4 levels (B / 4^k per side); each
 * triangle is listed, with its distance from the light, in the bins its
 * padded direction region covers, at the finest level where that is at most
 * 32 x 32 bins.  A segment y -> light then tests only the triangles of its
 * bins that are closer to the light than y, in order of distance.  The
 * padding covers the hit test's FP32 error, so the answers equal those of
 * testing every triangle.
 *
 * Build (host) and upload the bins of these lights, replacing any earlier
 * set; rc_records* do this themselves at the first call with a new set of
 * positions.  Allocates device memory (about 50 B per entry; entries per
 * triangle fall with its size and distance).  B = 0: chosen from the triangle
 * count.  Errors: EINVAL (bad lights or B), ENOMEM, EDEVICE. */
int rc_light_bins_build(rc_scene* scene, const rc_point_light* lights, int n_lights, int B);
/* Segments p_i -> light `light` (index into the last built set) answered from
 * the bins, one per lane: occ[i] = 1 if a triangle other than skip[i] is hit
 * with 1e-4 < t < 1 on o = p_i, d = light - p_i.  pts device float[n][3],
 * skip device int32[n] or NULL, occ device int32[n].  Errors: EINVAL (no
 * bins built, light out of range). */
int rc_light_occluded(const rc_scene* scene, int light, const float* pts, const int32_t* skip, int64_t n,
                      int32_t* occ, void* stream);
/* The bins of one light as the kernels read them, built on the host (no
 * device needed).  B: finest bins per face side (a power of two >= 2, or 0 =
 * chosen from T).  Outputs: *B_out, *levels, level_off[4] (start of each
 * level within offs), offs int32[n_offs] (per level 6 B_k^2 bin starts and a
 * sentinel; absolute entry indices), entries float[n_entries][12] (vertices
 * permuted for the face's axis, id bits in word 3, distance from the light
 * minus the hit-test error in word 7).  Returns the entry count, or a
 * negative error; with offs or entries NULL (or their capacities too small)
 * only the counts are written. */
int64_t rc_light_bins_host(const float* tri, int64_t T, const float box_lo[3], const float box_hi[3],
                           const float light[3], int B, int* B_out, int* levels, int64_t* level_off, int32_t* offs,
                           int64_t cap_offs, int64_t* n_offs, float* entries, int64_t cap_entries);

/* ------------------------------------------------------------------ */
/* Learned placement (project-defined; predicts the validity radius of  */
/* Sec. 5, Eq. radiusAniso3D, from a cheap probe)                       */
/* ------------------------------------------------------------------ */
/* 64-ray probe of candidate points: a 4 x 16 jittered strata grid (same
 * sampler as the records, record id = id_base + i, or id_base for every
 * candidate if common_random = 1; `seed`), closest hits,
 * Lambertian shading of the hits with shadow rays, attenuation to x, and the
 * visibility of the first four lights from x; reduced to 32 features per
 * candidate:
 *   0-3  min, mean, std, max of log hit distance      4 escaped fraction
 *   5    log mean inverse distance   6 log mean radiance   7 radiance CV
 *   8    log max radiance            9-12 light visible from x (lights 0-3)
 *   13-16 log unshadowed irradiance from lights 0-3
 *   17-19 radiance-weighted mean direction  20-22 inverse-distance-weighted
 *   23-26 mean log distance per strata row  27-30 mean log radiance per row
 *   31   neighbour contrast of radiance along phi.
 * cand device float[C][3]; feat32 device float[C][32] and/or feat_bf16 device
 * bfloat16[C][32] (either may be NULL, not both). */
int rc_probe(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
             const float* cand, int64_t C, uint64_t seed, int64_t id_base, int common_random, float* feat32,
             uint16_t* feat_bf16, void* stream);

/* MLP 32 -> 128 -> 128 -> 1 with tanh-GELU, predicting log R.  Parameter
 * block (device, rc_mlp_param_bytes() bytes): float shift[32], scale[32]
 * (feature standardisation x' = (x - shift) * scale), b1[128], b2[128],
 * w3[128], b3, padding to 464 floats; then bfloat16 W1[128][32],
 * W2[128][128], W2^T[128][128].  Training state (device float,
 * 3 * rc_mlp_n_params()): FP32 master parameters, Adam first and second
 * moments, each laid out as W1[128][32], b1[128], W2[128][128], b2[128],
 * w3[128], b3, loss slot. */
size_t rc_mlp_param_bytes(void);
int64_t rc_mlp_n_params(void);
/* Every MLP call below takes at most 2^30 samples (RC_EINVAL beyond). */
/* Glorot-uniform initialisation from the counter-based generator. */
int rc_mlp_init(void* params, float* state, uint64_t seed, void* stream);
/* Rebuild the parameter block's FP32/BF16 copies from master parameters. */
int rc_mlp_load(void* params, const float* state, void* stream);
/* Set the feature standardisation from n samples X (device float[n][32]);
 * workspace device, >= 256 * 64 floats. */
int rc_mlp_fit_features(void* params, const float* X, int64_t n, void* workspace, void* stream);
/* out[i] = MLP(X[i]) (device float[n]); BF16 MFMA (16x16x32), FP32
 * accumulation; layer-1 activations rounded to BF16, layer 2 output FP32. */
int rc_mlp_forward(const void* params, const float* X, int64_t n, float* out, void* stream);
/* Predicted validity radius: R[i] = clamp(safety * exp(MLP(X[i])), r_min,
 * r_max) (device float[n]); safety > 0, 0 < r_min <= r_max. */
int rc_mlp_radius(const void* params, const float* X, int64_t n, float safety, float r_min, float r_max, float* R,
                  void* stream);
/* One Adam step (lr, bias correction for `step` >= 1, betas 0.9/0.999,
 * eps 1e-8) on the mean squared error over the n samples (X, target device
 * float[n]).  workspace: rc_mlp_train_workspace_bytes(n) bytes.  loss (device
 * float[1], sum of squared errors) and grad (device float[n_params], the
 * gradient) are optional outputs. */
size_t rc_mlp_train_workspace_bytes(int64_t n);
int rc_mlp_train_step(void* params, float* state, const float* X, const float* target, int64_t n, float lr,
                      int64_t step, void* workspace, float* loss, float* grad, void* stream);

/* Greedy cover placement over candidates cand device float[C][3], exactly the
 * sequential rule "visit the candidates in order and accept one unless an
 * accepted point lies closer than that point's radius", run in rounds (Sec. 6
 * inserts a cache point where no cached point is valid).  The distance test is
 * ((dx*dx + dy*dy) + dz*dz) < R*R in FP32, dx = candidate - accepted point.
 * order device int32[C] (a permutation: the visiting order) or NULL (index
 * order).  state device int32[RC_PLACE_STATE_INTS] (zero to start): cursor,
 * accepted count, first/count accepted in the last round, gathered batch
 * size, then one status word per gathered candidate.  covered
 * device uint8[C] (zero to start; 1 = decided or covered).
 *   gather: the next `batch` (1..4096) undecided candidates after the cursor
 *           in visiting order: indices batch_idx, positions batch_pos
 *           (device float[batch][3]), and radii batch_R from `radius`
 *           (device float[C]) if given; state[4] = how many were gathered;
 *   accept: decide the gathered batch in order with radii batch_R (all
 *           members become decided); append the accepted ones' indices and
 *           radii to accepted / accepted_R (device, capacity >= C), their
 *           positions to accepted_pos (device float[.][3]) if not NULL, and,
 *           if batch_value/batch_grad (records of the batch slots, device
 *           double [batch][2], [batch][2][3]) are given, copy those records
 *           to cache_value / cache_grad at the appended positions;
 *   cover : mark candidates within the radius of accepted[first ..
 *           first+count) (or of the last round's points if first < 0) as
 *           covered, testing every candidate;
 *   cover_grid : the same for grid candidates, visiting only nearby cells.
 *           Candidate (ix, iy, iz) (index (ix * dims[1] + iy) * dims[2] + iz)
 *           must lie in cell lo + [i, i+1) * cell (host float[3] each) up to
 *           rounding; dims host int32[3], product < 2^31; cand and covered
 *           hold exactly dims[0] * dims[1] * dims[2] candidates.
 * Anisotropic points (Sec. 5, Eq. radiusAniso3D: the valid region is an
 * ellipsoid along the Hessian's eigenvectors): with batch_form (device
 * float[batch][6], from rc_ellipsoid_form) accept tests the ellipsoids of
 * the batch and appends them to accepted_form (device float[.][6]); cover
 * and cover_grid test accepted_form if it is not NULL.  The test is
 * d^T M d < 1 with d = candidate - point, evaluated in FP32 as
 * ((m00 dx^2 + m11 dy^2) + m22 dz^2) + 2 ((m01 dx dy + m02 dx dz) + m12 dy dz);
 * batch_R / accepted_R then hold the ellipsoid's largest radius (the grid
 * search bound).  NULL forms: balls, as above.
 * Errors: EINVAL for NULL pointers, sizes out of range, a bad batch size or a
 * bad grid; the kernels themselves only read indices the state holds. */
int rc_place_gather(const float* cand, const float* radius, const int32_t* order, int64_t C, const uint8_t* covered,
                    int32_t* state, int32_t* batch_idx, float* batch_pos, float* batch_R, int batch, void* stream);
int rc_place_accept(const float* cand, const int32_t* batch_idx, const float* batch_R, uint8_t* covered,
                    int32_t* state, int32_t* accepted, float* accepted_R, float* accepted_pos,
                    const double* batch_value, const double* batch_grad, double* cache_value, double* cache_grad,
                    const float* batch_form, float* accepted_form, void* stream);
int rc_place_cover(const float* cand, int64_t C, uint8_t* covered, const int32_t* state, const int32_t* accepted,
                   const float* accepted_R, int64_t first, int64_t count, const float* accepted_form, void* stream);
int rc_place_cover_grid(const float* cand, const int32_t dims[3], const float lo[3], const float cell[3],
                        uint8_t* covered, const int32_t* state, const int32_t* accepted, const float* accepted_R,
                        int64_t first, int64_t count, const float* accepted_form, void* stream);

/* The ellipsoid of anisotropic points (Sec. 5, Eq. radiusAniso3D) from the
 * axes rc_radius writes (device float[K][12]): form[k] = (m00, m01, m02, m11,
 * m12, m22) of M = sum_i v_i v_i^T / R_i^2 (each entry formed in FP64, terms
 * in axis order, rounded once to FP32), device float[K][6]; r_max (device
 * float[K] or NULL) = the largest R_i. */
int rc_ellipsoid_form(const float* axes, int64_t K, float* form, float* r_max, void* stream);

/* Radiance from a cache (Sec. 5, Eq. radianceTaylor): weighted first-order
 * Taylor expansions of every cache point whose radius contains the query,
 * cubic kernel w = 3d^2 - 2d^3, d = 1 - |x' - x_k|/R_k, FP64.  cache_value
 * [K][2] and cache_grad [K][2][3] are records (channels summed).  out device
 * double[Q] (0 where uncovered), hits device int32[Q] or NULL.  With
 * ref_value (device double[Q][2]) each block of 256 queries writes the sums
 * of (out - ref)^2 and ref^2 over its covered queries to err_partial[2b..].
 * cache_form (device float[K][6] or NULL): anisotropic points, membership by
 * the FP32 ellipsoid test of rc_place_accept and d = 1 - sqrt(e) with e the
 * FP64 value of d^T M d (cache_R is then not read). */
int rc_interp(const float* cache_pos, const double* cache_value, const double* cache_grad, const float* cache_R,
              int64_t K, const float* query, int64_t Q, double* out, int32_t* hits, const double* ref_value,
              double* err_partial, const float* cache_form, void* stream);

/* ------------------------------------------------------------------ */
/* Render pass (Sec. 6 "Implementation"; Results in 3D: uniform ray      */
/* marching with step 0.1): the consumer of the cache                   */
/* ------------------------------------------------------------------ */
/* Camera rays marched through the medium.  Ray r (orig/dir device
 * float[n][3], origin inside the scene's medium box) ends at t_end[r]: its
 * closest triangle hit, or where it leaves the box (the traversal of
 * rc_trace_rays); its march points lie at t_k = (k + xi[r]) * step for
 * k = 0, 1, ... while t_k < t_end[r] (xi device float[n], the ray's offset in
 * [0, 1); k + xi exact in FP64, the product rounded once).  Writes t_end
 * (device float[n]) and offsets (device int64[n + 1]): offsets[0] = 0 and
 * offsets[r + 1] = number of points of rays 0..r, so offsets[n] is the total
 * the caller sizes rc_march_emit's outputs with.  Directions must be nonzero.
 * RC_EINVAL unless step > 0 and box diagonal / step <=
 * RC_MARCH_MAX_POINTS_PER_RAY. */
int rc_march_count(const rc_scene* scene, const float* orig, const float* dir, const float* xi, int64_t n,
                   double step, float* t_end, int64_t* offsets, void* stream);
/* The march points of rc_march_count's rays (same orig, dir, xi, step and its
 * offsets): point offsets[r] + k is at o + t_k d, formed in FP64 and rounded
 * once to FP32 (points device float[offsets[n]][3]), with quadrature weight
 * step * sigma_s * exp(-sigma_t t_k) (weight device double[offsets[n]]): the
 * in-scattering integral of the ray by the march points, attenuated by the
 * transmittance from the eye (sigma_t = sigma_s + sigma_a). */
int rc_march_emit(const float* orig, const float* dir, const float* xi, int64_t n, double step, double sigma_s,
                  double sigma_t, const int64_t* offsets, float* points, double* weight, void* stream);
/* Pixel estimates: pixel p (device double[n_rays / spp]) is the mean over
 * rays p * spp .. p * spp + spp - 1 of the sum of weight * L over the ray's
 * points (L device double[offsets[n_rays]]: in-scattered radiance at each
 * point, e.g. from rc_interp), FP64, points taken in ray order.  weight and L
 * hold offsets[n_rays] entries each (they may be NULL only when that total is
 * 0: the host does not read device offsets).  RC_EINVAL unless spp >= 1
 * divides n_rays. */
int rc_composite(const int64_t* offsets, int64_t n_rays, int32_t spp, const double* weight, const double* L,
                 double* pixel, void* stream);

/* ------------------------------------------------------------------ */
/* The comparison method's records (Jarosz et al. 2008 as summarised in */
/* Sec. 3; supplement Eqs. S.3-S.4; Eq. jaroszRadius)                  */
/* ------------------------------------------------------------------ */
/* From the same samples as rc_records' values (directions, hits, shading,
 * medium rings, params->seed / rec_base / common_random / ring_step /
 * max_rings as there; params' other fields are not read): value [P][2]
 * (SS, MS Monte Carlo values), grad [P][2][3] occlusion-unaware gradients
 * (single scattering: each direction's hit point held fixed, the sample's
 * gradient = sample (grad ln T + grad ln G), T = exp(-mu r), G = (yx . n) /
 * r^3, yx = x - y; multiple scattering: the path x -> ring vertex -> light
 * moved rigidly, visibility held), moments [P][2] = the means over the
 * directions of the per-direction sample L_k (channels summed) and of
 * |grad L_k|, and R [P] = eps * sum L_k / sum |grad L_k| clamped to
 * [r_min, r_max] (r_max when every gradient is zero).  All device FP64
 * except R (FP32).  Records with n_theta < 2, n_phi outside [5, RC_MAX_NPHI]
 * get NaN outputs.  Shadow segments from the scene's light bins of these
 * lights (built on the first call). */
/* The comparison method's extrapolation from a cache (Eq. jaroszExtrapolation):
 * L(x') = exp( sum_k [ln L_k + (grad L_k / L_k) . (x' - x_k)] w_k / sum_k w_k )
 * over the cache points whose radius contains x' (the FP32 ball test and the
 * cubic weights of rc_interp), channels summed; points with L_k <= 0 take no
 * part.  out device double[Q] (0 where uncovered), hits device int32[Q] or
 * NULL. */
int rc_interp_log(const float* cache_pos, const double* cache_value, const double* cache_grad, const float* cache_R,
                  int64_t K, const float* query, int64_t Q, double* out, int32_t* hits, void* stream);
int rc_j08_records(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
                   const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                   const rc_params* params, float eps, float r_min, float r_max, double* value, double* grad,
                   double* moments, float* R, void* stream);

/* ------------------------------------------------------------------ */
/* Diagnostics                                                          */
/* ------------------------------------------------------------------ */
const char* rc_last_error(void);
const char* rc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RC_H_ */
