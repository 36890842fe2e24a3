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

#define RC_MAX_LIGHTS 16
#define RC_MAX_RINGS 64
#define RC_MAX_NPHI 256

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
 *   precision : 0 = FP32 terms, compensated FP32 sums, FP64 for
 *               near-degenerate triangle terms and the final reduction
 *               (default); 1 = every triangle term in FP64 (study mode).
 *   counters  : device uint64_t[8] or NULL.  If set, the launch also counts
 *               (atomically added): rays traced, BVH nodes visited,
 *               ray/triangle tests, triangle terms evaluated, and the shader
 *               clocks each wavefront spent in primary rays, shadow rays, the
 *               Monte Carlo value and the triangle terms (summed over
 *               wavefronts). */
typedef struct {
  float ring_step;
  int32_t max_rings;
  int32_t max_n_phi;
  int32_t precision;
  uint64_t seed;
  int64_t rec_base;
  uint64_t* counters;
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
 * counters, error counter).  Size in bytes for up to P records: */
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
 * The launch is one persistent kernel: each wavefront pops records from a
 * queue in `workspace` and computes its whole record on chip. */
int rc_records(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
               const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
               const rc_params* params, double* value, double* grad, double* hess,
               void* workspace, void* stream);

/* Same records, scheduled from a caller-supplied queue.
 *   order     : device int32[P] permutation of 0..P-1, the order in which
 *               records are popped (e.g. most expensive first), or NULL to
 *               build one on the device (records sorted by n_theta * n_phi,
 *               largest first).
 *   use_graph : nonzero = capture the queue reset and the persistent launch in
 *               a hipGraph on first use for this (scene, P, tile) and replay
 *               it afterwards (the graph is cached in the scene handle).
 *   tile      : launch configuration index from rc_autotune, or -1 = default.
 * Outputs are identical (bitwise) to rc_records for the same inputs. */
int rc_records_batched(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights,
                       int n_lights, const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                       const rc_params* params, const int32_t* order, int use_graph, int tile,
                       double* value, double* grad, double* hess, void* workspace, void* stream);

/* Time every launch configuration on the given inputs (synchronises
 * `stream`) and return the fastest configuration index in *best_tile; the
 * per-configuration milliseconds go to ms_out[n_tiles] if non-NULL.  The
 * result is remembered in the on-disk cache `cache_path` (a text file; NULL
 * = no cache) keyed by device name, scene size and workload shape. */
int rc_autotune(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
                const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                const rc_params* params, double* value, double* grad, double* hess, void* workspace,
                const char* cache_path, int* best_tile, float* ms_out, int* n_tiles, void* stream);

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
/* Closest hit of rays o + t d, t > 0 (Moller-Trumbore in FP32, rays within
 * ~0.6 degrees of a triangle plane rejected, ties to the lowest triangle
 * index).  orig/dir device float[n][3]; hit_id device int32[n] (triangle
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
/* Diagnostics                                                          */
/* ------------------------------------------------------------------ */
const char* rc_last_error(void);
const char* rc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RC_H_ */
