/* ppt.h -- C ABI of the MI355X (gfx950) differentiable polarized path tracer.
 *
 * The library renders Stokes images with Monte Carlo path tracing in Mueller-Stokes
 * calculus and computes reverse-mode gradients of them with path replay backpropagation
 * using cached suffix radiance, so no Mueller matrix is ever inverted (paper: Sec. 3.1
 * problem statement and Eq. 1-2; Sec. 3.2 path replay; Sec. 3.3 Mueller-Stokes calculus;
 * Sec. 4.3 and Fig. 2 cached suffix replay).  All arithmetic runs in hand-written HIP
 * kernels for gfx950 in FP32 (gradients are accumulated in FP64).
 *
 * Conventions for every entry point
 *   - Return value: PPT_OK (0) or a negative PPT_E* code; ppt_last_error() then holds a
 *     message (thread-local).  Nothing aborts and no C++ exception crosses the ABI.
 *   - "device" pointers are HIP device memory owned by the caller (e.g. torch tensors);
 *     "host" pointers are ordinary host memory owned by the caller and only read during
 *     the call.  Objects created by the library (scene, plan) own their device memory
 *     until destroyed.
 *   - `stream` is a hipStream_t passed as void*; work is enqueued on it and no call
 *     synchronizes the host except where stated.  Entry points that enqueue work contain
 *     only kernel launches, so they can be captured in a HIP graph.
 *   - A scene and a plan may be used concurrently on different streams provided each call
 *     gets its own workspace.
 */
#ifndef PPT_H
#define PPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PPT_OK 0
#define PPT_EINVAL (-1)       /* invalid argument, size or layout */
#define PPT_ENOMEM (-2)       /* device allocation failed */
#define PPT_EDEVICE (-3)      /* HIP runtime or launch error */
#define PPT_EUNSUPPORTED (-4) /* valid request outside the compiled limits */

/* flags of ppt_plan_create */
#define PPT_FLAG_NO_NEE 1u    /* pure BSDF sampling: every emitter hit counts, no light sampling */

/* sensor types of ppt_view.sensor */
#define PPT_SENSOR_NONE 0      /* full Stokes vector in the sensor frame */
#define PPT_SENSOR_POLARIZER 1 /* ideal linear polarizer at angle theta (a parameter, radians) */
#define PPT_SENSOR_ANALYZER4 2 /* polarizers at 0, 45, 90 degrees and QWP(0) followed by 45 degrees */
#define PPT_SENSOR_LIGHTSTAGE4 3 /* polarizers at 0, 45, 90 degrees and QWP(0) followed by -45 degrees
                                    (a left-circular analyzer: it passes s3 < 0) */

/* One camera view (88 bytes, host memory).  The image is width x height pixels; only the
 * window [crop_x0, crop_x0 + crop_w) x [crop_y0, crop_y0 + crop_h) is rendered.  The
 * random stream of a path is keyed by (pixel index in the full image, sample, view_id),
 * so a window or a batch renders exactly the same paths as the full single view.
 * The sensor frame for light arriving along k = -ray has x = right vector projected
 * perpendicular to k and y = k x x; polarizer angles are measured from x toward y. */
typedef struct ppt_view {
    int32_t world;                       /* world index inside the scene */
    int32_t width, height, spp;          /* image size and samples per pixel (>= 1) */
    int32_t crop_x0, crop_y0, crop_w, crop_h;
    float origin[3], target[3], up[3];   /* pinhole camera */
    float fov_y_deg;                     /* vertical field of view */
    int32_t sensor;                      /* PPT_SENSOR_* */
    int32_t theta_slot, theta_off;       /* parameter element holding theta (POLARIZER only) */
    uint32_t view_id;                    /* random-stream index of the view (< 2^24) */
} ppt_view;

typedef struct ppt_plan_opts {
    int64_t chunk_paths;          /* paths in flight per chunk (path-state capacity); 0 = min(all, 16M) */
    int64_t checkpoint_interval;  /* backward replay (Sec. 4.4): 0 = cached suffix replay, every vertex
                                   * keeps W_b, E_b and its suffix (128 B); k >= 1 = hybrid cached
                                   * replay, only a 16-byte hit record per vertex, the suffix every k
                                   * vertices, and the vertices in between recomputed from it (exact;
                                   * less workspace for deep paths, more arithmetic).  k <= 128. */
    int32_t hybrid_rule;          /* hybrid replay only.  0: a suffix inside a block is recovered by
                                   * recomputing the block from its checkpoint.  1: Eq. 3's decision
                                   * rule (Sec. 4.4): the replay tracks the detached block throughput
                                   * beta since the block's checkpoint and the radiance its vertices
                                   * have not yet emitted, and recovers a suffix by the scalar PRB
                                   * update (intensity only) when the depolarization index of beta
                                   * (Gil-Bernabeu) is below hybrid_gamma, by inverting beta when
                                   * |det beta| > hybrid_eps beta_00^4, else by recomputing the rest
                                   * of the block.  The scalar update is exact where the suffix's
                                   * polarization is not needed (depolarizing blocks) and an
                                   * approximation elsewhere; inversion is exact up to rounding, which
                                   * it amplifies by the condition number of beta. */
    float hybrid_gamma;           /* >= 0; 0 disables the scalar update */
    float hybrid_eps;             /* >= 0 (infinity disables inversion) */
    int32_t adjoint;              /* PPT_ADJOINT_CACHED (0): the method above.  PPT_ADJOINT_PPRB: the
                                   * comparator of Sec. 4.2, polarized PRB with noise regularisation:
                                   * every sampled weight becomes W_b + u_b I with u_b ~ N(0, pprb_sigma)
                                   * drawn per vertex from the path's counters (Box-Muller of two
                                   * uniforms of counter call 2), the same in the primal and the
                                   * adjoint, and the replay recovers each suffix by inverting it.  An
                                   * unbiased but noisier estimator of the gradient; pprb_sigma = 0
                                   * inverts rank-deficient weights and gives non-finite gradients.
                                   * Requires checkpoint_interval = 0.
                                   * PPT_ADJOINT_TAPE: the conventional-AD baseline ("Conv. AD", Sec. 5.1,
                                   * 5.4): the forward pass stores every vertex's loop state (prefix
                                   * throughput, weight, emission, hit, incoming ray: 240 B per vertex of
                                   * max_depth per path of the chunk) and a reverse sweep walks each path
                                   * from its last vertex back, carrying the throughput's adjoint as a
                                   * full 4x4 matrix per channel.  Same gradient as the cached replay; no
                                   * normal/specular maps or circular emitters; no checkpoints.
                                   * PPT_ADJOINT_PRB: the comparator of Sec. 5.1, polarized radiative
                                   * backpropagation: the replay reads, for each vertex b, an independent
                                   * estimate of the suffix beyond it, a new path traced from the ray
                                   * leaving b under the key seed + (b + 1) * 0x9E3779B97F4A7C15 (its
                                   * vertices keep their numbers b + 1, b + 2, ... in the counters); one
                                   * sub-path pass per vertex index.  Unbiased, with the variance of that
                                   * estimate; no light-stage features; no checkpoints; 337 more bytes of
                                   * workspace per path of the chunk. */
    float pprb_sigma;             /* >= 0, finite */
} ppt_plan_opts;
#define PPT_ADJOINT_CACHED 0
#define PPT_ADJOINT_PPRB 1
#define PPT_ADJOINT_TAPE 2
#define PPT_ADJOINT_PRB 3

typedef struct ppt_scene ppt_scene;
typedef struct ppt_plan ppt_plan;

/* Scene blob (little-endian, 32-bit words unless stated):
 *   header     magic 0x31545050 ('PPT1'), version 2, n_slots (<= 64), n_worlds
 *   slots      n_slots element counts (the float32 parameter tensors of every call)
 *   per world  n_tris, n_spheres, n_materials, n_lights, then
 *              triangles: n_tris x 9 floats (v0, v1, v2), n_tris x 6 floats (uv0, uv1, uv2),
 *                         n_tris material indices;
 *              spheres:   n_spheres x 4 floats (centre, signed radius: < 0 = inward normal),
 *                         n_spheres material indices;
 *              materials: 128-byte records {type; albedo slot, offset, texture width, height;
 *                         roughness slot, offset, width, height; eta slot, offset; kappa slot,
 *                         offset; emission slot, offset; sheet axis[3]; blend; emission circ;
 *                         specular-map slot, offset, width, height; normal-map slot, offset,
 *                         width, height; 4 reserved}
 *                         (slot -1 = absent, width 0 = constant, texture layout [h][w][ch]);
 *              lights:    48-byte records {p0[3], eu[3], ev[3]; radiance slot, offset; circ},
 *                         one-sided rectangles emitting along eu x ev (their geometry is also
 *                         present as two triangles with an emitter material).
 *   Emission: an emitter radiates the Stokes vector Le (1, 0, 0, circ) per RGB channel, circ in
 *   [-1, 1] the degree of circular polarization (right-circular = s3 > 0 in this library's
 *   Stokes convention; circular polarization needs no transverse frame).  A light record and
 *   the emitter material of its geometry should carry the same circ.
 *   Specular map (GGX types and the blend): a 1-channel scale of the GGX lobe (absent = 1).
 *   Normal map (every scattering type; triangles only, spheres keep their geometric normal):
 *   3 channels (t, b, n) give the outward shading normal normalize(t T + b B + n N), with N the
 *   geometric normal, T the unit tangent along increasing u (dP/du made perpendicular to N; the
 *   canonical basis of N for a degenerate uv map) and B = N x T.  A vertex seen from behind its
 *   shading normal is black (its emission still counts); a light sample or a sampled direction
 *   on the wrong side of the geometric surface is discarded.  The shading normal is
 *   differentiated, including the s/p frames of the smooth dielectric.
 *   Material types: 0 Lambertian, 1 smooth dielectric, 2 GGX dielectric (reflection),
 *   3 GGX conductor (complex IOR eta + i kappa), 4 linear polarizer sheet, 5 emitter,
 *   6 Lambertian/GGX-dielectric blend (lobe probability = blend).
 * ppt_scene_create parses and validates a blob, builds one SAH bounding volume hierarchy per
 * world on the host and uploads everything to the current device.
 * blob/nbytes: host memory.  *out receives a library-owned handle.
 * Errors: PPT_EINVAL for a malformed blob (truncated, bad magic, indices out of range),
 * PPT_ENOMEM / PPT_EDEVICE for device failures. */
int ppt_scene_create(const void* blob, size_t nbytes, ppt_scene** out);
void ppt_scene_destroy(ppt_scene* scene);

/* Number of parameter slots; if numel_out is not NULL it receives min(cap, n) element counts. */
int ppt_scene_slots(const ppt_scene* scene, int32_t* n_slots, int64_t* numel_out, int32_t cap);

/* Fix the views, the maximum path depth (1..128 surface interactions) and the flags of a
 * family of calls.  All paths of all views form one index space that is processed in chunks
 * of chunk_paths paths (one launch sequence covers the whole batch of views, also views of
 * different worlds, resolutions and sample counts).  views: host array of n_views records.
 * Errors: PPT_EINVAL for an invalid view or option, PPT_EUNSUPPORTED for a depth outside
 * 1..128, 2^19 or more views, or a view with 2^31 or more paths (crop pixels x spp). */
int ppt_plan_create(const ppt_scene* scene, const ppt_view* views, int32_t n_views, int32_t max_depth,
                    uint32_t flags, const ppt_plan_opts* opts, ppt_plan** out);
void ppt_plan_destroy(ppt_plan* plan);

/* Output layout: the concatenation over views of [A][crop_h][crop_w][3][4] float32 (A = 4 for
 * PPT_SENSOR_ANALYZER4, else 1; 3 RGB channels; Stokes s0..s3).  Paths are numbered
 * (view, crop row, crop column, sample). */
int64_t ppt_plan_image_numel(const ppt_plan* plan);
int64_t ppt_plan_num_paths(const ppt_plan* plan);

/* Device workspace bytes needed by ppt_render (op = 0) or ppt_backward (op = 1): the
 * per-path records of one chunk of paths (for the backward pass including the per-vertex cache
 * of max_depth 128-byte records per path of the chunk, or the tape of the conventional-AD
 * baseline), independent of the total number of paths, and the FP64 gradient accumulators. */
size_t ppt_plan_workspace_bytes(const ppt_plan* plan, int32_t op);

/* Optional per-path mask (device, one byte per path, NULL = all paths).  A path whose byte is
 * zero contributes nothing to images or gradients.  The buffer must outlive its use. */
int ppt_plan_set_path_mask(ppt_plan* plan, const uint8_t* mask);

/* Render (Sec. 3.1, Eq. 2): every pixel is the mean over its samples of S(theta) sum_b beta_b E_b
 * in Mueller-Stokes calculus.  params: host array of n_params device pointers, one per scene
 * slot, each float32 with the slot's element count.  stokes_out: device, image_numel floats,
 * overwritten.  ws: device workspace of at least ppt_plan_workspace_bytes(plan, 0) bytes. */
int ppt_render(const ppt_plan* plan, const float* const* params, int32_t n_params, uint64_t seed,
               float* stokes_out, void* ws, size_t ws_bytes, void* stream);

/* Reverse-mode gradient by path replay with cached suffix radiance (Sec. 3.2, 4.3, Fig. 2):
 * grads[k] = d(sum d_stokes . I) / d params[k] for the estimator I of ppt_render with the same
 * seed (a different seed gives the decorrelated replay of Sec. 3.2).  Sampling is detached:
 * positions, directions, lobe choices and pdfs are constants; Mueller/BSDF values, emission
 * and the sensor Mueller matrix are differentiated.  d_stokes: device, image layout.
 * grads: host array of n_params device pointers (float32, slot sizes); NULL entries are
 * skipped, the others are overwritten.  ws: at least ppt_plan_workspace_bytes(plan, 1). */
int ppt_backward(const ppt_plan* plan, const float* const* params, int32_t n_params, uint64_t seed,
                 const float* d_stokes, float* const* grads, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of ppt_backward, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  It returns the
 * same gradients as ppt_backward (same arguments, minus the workspace) and allocates nothing
 * (no hipMalloc, hipFree or allocating library call): the per-path records of one chunk and the
 * FP64 gradient accumulators live in a fixed device array of PPT_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held until the process ends; the first call on a device looks up that
 * device's array.  Paths run in chunks of at most the plan's chunk size, cut down to what the array
 * holds (results do not depend on the chunking; a deep path needs 128 bytes per vertex of max_depth).
 * Every call on one GPU uses the same array, which keeps the previous call's contents (each call
 * clears what it needs): calls that overlap on one GPU, from other streams or threads, race and must
 * be serialized by the caller.  Work counters are not collected and per-kernel timing is not
 * recorded.  Errors: as ppt_backward; PPT_EUNSUPPORTED when the gradient accumulators (8 bytes per
 * parameter element) and the records of one 64-path chunk do not fit in the array. */
#define PPT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ppt_backward_noalloc(const ppt_plan* plan, const float* const* params, int32_t n_params, uint64_t seed,
                         const float* d_stokes, float* const* grads, void* stream);

/* Per-path 64-bit signatures (FNV-1a over primitive id, light-sample state and lobe of every
 * vertex, the lobe word of a sampled direction also holding the branch of its sampling frame, the
 * sign of the shading normal's z in the Duff et al. basis) used to detect paths whose discrete decisions differ
 * from another implementation.
 * sig_out: device, num_paths uint64.  ws as for ppt_render. */
int ppt_signatures(const ppt_plan* plan, const float* const* params, int32_t n_params, uint64_t seed,
                   uint64_t* sig_out, void* ws, size_t ws_bytes, void* stream);

/* Work counters of the last render/backward call made with a workspace: out[0] path vertices,
 * [1] paths, [2] BVH nodes visited by closest-hit rays, [3] their primitive tests, [4] shadow
 * (next-event) rays, [5] closest-hit rays, [6] BVH nodes visited by shadow rays, [7] their
 * primitive tests.  Collected while the plan's counters are enabled (the default;
 * ppt_plan_set_stats), else left at zero.  Synchronizes the stream.  ws: device workspace;
 * out: host, 8 entries. */
int ppt_plan_set_stats(ppt_plan* plan, int32_t enabled);
int ppt_read_stats(const void* ws, int64_t* out, void* stream);

/* Branch counts of the hybrid replay's decision rule in the last backward call made with workspace
 * ws while the plan's counters were enabled: out[0] suffixes recovered by the scalar update,
 * out[1] by inversion, out[2] by recomputation (a recomputation covers the rest of its block).
 * Synchronizes the stream.  out: host, 3 entries. */
int ppt_read_hybrid_stats(const void* ws, int64_t* out, void* stream);

/* Per-kernel event timing (diagnostics).  While enabled, every render/backward call on the plan
 * records a HIP event on its stream before each kernel launch and one after its last launch.
 * ppt_plan_kernel_times waits for the most recent such call of `op` (0 render, 1 backward) and
 * writes, for kernel family k < n, the summed time between an event and the next (ms[k], in
 * milliseconds) and the number of launches (launches[k]).  Families: 0 camera rays launched
 * alone (none at present: the first traversal launch generates them), 1 traversal (closest hits
 * of a bounce's rays, from the second bounce on in the same launch as the shadow rays of the
 * previous bounce), 2 shading, 3 shadow rays launched alone (none at
 * present), 4 pixel reduction, 5 suffix fold, 6 adjoint replay, 7 setup / clearing /
 * finalization, 8 hit compaction.  Enabling or disabling clears the
 * records.  Not for use under stream capture; calls on one plan must not overlap while
 * enabled.  Errors: PPT_EINVAL when no timed call of `op` was made, PPT_EDEVICE on HIP errors. */
int ppt_plan_set_timing(ppt_plan* plan, int32_t enabled);
int ppt_plan_kernel_times(const ppt_plan* plan, int32_t op, double* ms, int32_t* launches, int32_t n);

/* Philox4x32-10 (Salmon et al. 2011) on n counters: ctr and out are device arrays of n x 4
 * uint32; key = (seed low 32 bits, seed high 32 bits). */
int ppt_debug_rng(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n, void* stream);

/* Chunking of the plan: paths per chunk, number of chunks, traversal stack entries per thread. */
int ppt_plan_launch_info(const ppt_plan* plan, int64_t* chunk_paths, int32_t* n_chunks, int32_t* stack_entries);

const char* ppt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PPT_H */
