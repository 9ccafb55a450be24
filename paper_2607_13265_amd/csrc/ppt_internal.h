// ppt_internal.h -- device-side data layout shared by the host plan builder and the HIP kernels.
// Not part of the public ABI (see include/ppt.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ppt {

constexpr int MAX_SLOTS = 64;   // parameter tensors per scene
constexpr int WAVE = 64;
constexpr int BLOCK = 256;      // 4 wavefronts per workgroup
constexpr int MAX_DEPTH = 128;
constexpr int STACK = 64;       // BVH traversal stack entries per lane

// Per-path records in the workspace (one record per slot, 16-byte vectors; a path touches only
// its own cache lines even when the ray queues have scattered the live slots).  The shading
// kernel writes cache and shadow records whole, unused words included: records written in part
// measured slower even where whole ones move more bytes.
//   ray record, RAY_F4 = 4 vectors (64 B):
//     [0] ro.x ro.y ro.z rd.x   [1] rd.y rd.z Cs Ss   [2] t u v prim   [3] info pix smp view-id
//     (Cs, Ss: sensor rotation of the camera ray; view-id: the view's sampling identity; the hit is
//     one aligned vector, written by traversal in one 16-byte store)
//   shadow record, SHD_F4 = 8 vectors (128 B):
//     [0] so.x so.y so.z tmax   [1] sd.x sd.y sd.z info (of the vertex whose light sample it is)
//     [2..4] 12 Stokes words: the pending next-event contribution   [5..7] the backward's E_b (restored
//     into the cache record for an occluded sample), or zeros.  After the fold (backward): [0] the
//     camera ray's direction, info   [1] pix smp - -   [2..4] the replay's adjoint rows
//   accumulator record (render), ACC_F4 = 8 vectors (128 B):
//     [0..3] prefix Mueller product beta (16)   [4] beta RGB scales (3)   [5..7] radiance Lo (12)
//   rank-one render record (every view a linear polarizer), R1_F4 = 4 vectors (64 B, two to a cache
//   line): [0] rho = q^T R_s beta   [1] RGB scales   [2] y_c = q^T R_s Lo_c (3), with a pending
//   next-event part included as if visible   [3] y without that part (restored for an occluded
//   sample); the shadow ray in a dense 32-byte record behind the chunk's rank-one records, [0] origin,
//   tmax   [1] direction, info; no shadow record
//   cache record (backward), one per (vertex b, slot), CACHE_F4 = 8 vectors (128 B):
//     [0] rgb0 rgb1 rgb2 A   [1] B C D Cin   [2] Sin Cout Sout hitword   [3] u-or-t v - -
//     [4..6] E_b (12 words; with the next-event part as if visible when a light sample is pending, set
//     back to E_b by the shadow-ray traversal if occluded), overwritten by the fold with the suffix radiance beyond the vertex,
//     L[b+1], which is what the replay of vertex b reads (not stored for a path's last vertex)
//     [7] x: the next-event visibility (written as visible by shading for a pending light sample,
//     rewritten with E_b's words by the shadow-ray traversal when it is occluded)
//   hitword = prim | next-event state << 26 | weight kind << 29 (the state as sampled: pending for a
//   light sample; its visibility goes to [7])
//   hybrid replay (checkpoint interval k): per vertex a hit record [hitword, u-or-t, v, -] (16 B);
//   per block of k vertices a checkpoint record, CKPT_F4 = 5 vectors (80 B):
//     [0] o.x o.y o.z prev-delta   [1] d.x d.y d.z -   (the ray into the block's first vertex)
//     [2..4] suffix radiance beyond the block's last vertex (written by the fold);
//   and k cache records of scratch for the block being re-evaluated.
//   tape record (conventional-AD baseline), one per (vertex b, slot), TAPE_F4 = 15 vectors (240 B):
//     [0..7] as the cache record (E_b stays: the reverse sweep reads it)   [8..11] the prefix
//     throughput beta_b (shared 4x4)   [12] its RGB scales, previous vertex delta   [13..14] the ray into
//     the vertex (o, d)
constexpr int RAY_F4 = 4, SHD_F4 = 8, ACC_F4 = 8, R1_F4 = 4, CACHE_F4 = 8, CKPT_F4 = 5, TAPE_F4 = 15;

enum MatType : int32_t { MAT_LAMBERT = 0, MAT_DIELECTRIC = 1, MAT_GGX_DIELECTRIC = 2, MAT_GGX_CONDUCTOR = 3,
                         MAT_SHEET = 4, MAT_EMITTER = 5, MAT_BLEND = 6 };
enum SensorType : int32_t { SENSOR_NONE = 0, SENSOR_POLARIZER = 1, SENSOR_ANALYZER4 = 2, SENSOR_LIGHTSTAGE4 = 3 };
enum Lobe : int32_t { LOBE_NONE = 0, LOBE_REFLECT = 1, LOBE_TRANSMIT = 2, LOBE_DIFFUSE = 3, LOBE_GLOSSY = 4,
                      LOBE_SHEET = 5, LOBE_INVALID = 6 };

struct DevMaterial {
    int32_t type;
    int32_t alb_slot, alb_off, alb_tw, alb_th;
    int32_t alpha_slot, alpha_off, alpha_tw, alpha_th;
    int32_t eta_slot, eta_off;
    int32_t kap_slot, kap_off;
    int32_t emit_slot, emit_off;
    float axis[3];
    float blend;
    float emit_circ;                                // emitted Stokes Le (1, 0, 0, emit_circ)
    int32_t spec_slot, spec_off, spec_tw, spec_th;  // specular map (scale of the GGX lobe); slot -1 = none
    int32_t nrm_slot, nrm_off, nrm_tw, nrm_th;      // tangent-space normal map (3 channels); slot -1 = none
};

struct DevLight {
    float p0[3], eu[3], ev[3], n[3];
    float area;
    int32_t le_slot, le_off;
    float circ;  // emitted Stokes Le (1, 0, 0, circ)
};

// BVH2 node: both children's boxes in one 32-byte record (the two-box layout of Aila & Laine 2009
// with the box bounds as IEEE half floats, lo rounded down and hi rounded up, so that each stored
// box contains the exact one).  Words, each a pair of halves (first, second) or an int:
//   q0 = ((L.lo.x, L.hi.x), (L.lo.y, L.hi.y), (R.lo.x, R.hi.x), (R.lo.y, R.hi.y)),
//   q1 = ((L.lo.z, L.hi.z), (R.lo.z, R.hi.z), ref L, ref R).
// A reference >= 0 is an inner node; < 0 is a leaf: ~ref = first << 3 | (count - 1).
// Primitive records (3 x float4, BVH order): triangle (v0, orig), (e1, mat), (e2, 0);
// sphere (c, orig), (r, 0, 0, mat), (0, 0, 0, 1); orig (original primitive id), mat (material) and
// the last word (0: a triangle, 1: a sphere) as int bits.
struct DevWorld {
    const float4* nodes;
    const float4* prims;
    const float* tri_uv;         // 6 per original triangle
    const DevMaterial* mats;
    const DevLight* lights;
    int32_t n_tris, n_prims, n_lights, root;  // root: node reference (may be a leaf reference)
};

struct DevView {
    int32_t world, width, height, spp;
    int32_t crop_x0, crop_y0, crop_w, crop_h;
    float o[3], f[3], r[3], u[3];
    float tan_h, aspect;
    int32_t sensor, theta_slot, theta_off, n_analyzers;
    uint32_t view_id, pad;
    int64_t out_off;             // float offset of this view in the output image
    int64_t path_off;            // index of its first path (view, crop row, crop column, sample)
};

// Per-call device table written by the setup kernel (kernel arguments cannot be indexed
// per lane without spilling): parameter pointers and gradient accumulator offsets.
struct CallTable {
    const float* p[MAX_SLOTS];
    int64_t goff[MAX_SLOTS];     // element offset into the FP64 gradient accumulator, -1 = not requested
    float* gout[MAX_SLOTS];      // user gradient tensors (finalize kernel)
    int64_t numel[MAX_SLOTS];
    int32_t lds_d[MAX_SLOTS];    // offset in the workgroup FP64 gradient accumulator, -1 = none
    int32_t lds_f[MAX_SLOTS];    // offset in the workgroup FP32 gradient accumulator, -1 = none
};

constexpr int LDS_GRAD_D = 1024;    // FP64 entries of the workgroup gradient accumulator (small slots)
constexpr int LDS_GRAD_F = 12800;   // FP32 entries (textures)

// Work counters, accumulated by every launch while enabled (64-bit).  nodes/prims count the
// closest-hit traversals, shadow_nodes/shadow_prims the next-event (any-hit) traversals.
enum { ST_VERTICES, ST_PATHS, ST_NODES, ST_PRIMS, ST_SHADOW_RAYS, ST_RAYS, ST_SHADOW_NODES, ST_SHADOW_PRIMS, ST_COUNT };
struct Stats {
    unsigned long long c[ST_COUNT];
    unsigned long long hyb[3];  // hybrid replay decision rule: suffixes by scalar update, inversion, recomputation
};

// Kernel families for the optional per-launch event timing.
enum { KF_GEN, KF_EXTEND, KF_SHADE, KF_SHADOW, KF_ACCUM, KF_FOLD, KF_REPLAY, KF_OTHER, KF_COMPACT, KF_COUNT };
// Called before every launch with the family of the kernel about to be launched (may be NULL).
struct LaunchMarker {
    void (*fn)(void* ctx, int family, hipStream_t s);
    void* ctx;
    void operator()(int family, hipStream_t s) const { if (fn) fn(ctx, family, s); }
};

// State of the paths of one chunk (capacity Q slots) in the workspace, as per-slot records.
struct PathState {
    float4* ray;    // [Q][RAY_F4]
    float4* shd;    // [Q][SHD_F4]
    float4* acc;    // [Q][ACC_F4] (render)
    uint8_t* nv;    // [Q] vertices of the path: the first traversal writes 0 or 1, the backward's shading
                    // kernels the count; read by the rank-one pixel reduction (has the path a radiance
                    // record) and by the fold, so that neither reads a ray record (NULL: not kept)
    float4* cache;  // [max_depth or k][Q][CACHE_F4] (backward; per block scratch in the hybrid replay)
    float4* hits;   // [max_depth][Q] hit records (hybrid replay)
    float4* ckpt;   // [ceil(max_depth / k)][Q][CKPT_F4] checkpoint records (hybrid replay)
    int* queue0;    // ray queues (alternating per bounce; queue0 is the replay queue after the fold)
    int* queue1;
    int* squeue;    // shadow-ray queue
    int* hqueue;    // queue of the rays of this bounce that hit a surface (input of the shading kernel)
    uint8_t* hflag; // [Q] outcome of the slot's last closest-hit ray: 0 miss, 1 hit, 2 no ray (masked path)
    int* counts;    // 8 ints: [0], [1] sizes of queue0, queue1; [2] size of the shadow queue; [3] size of
                    // the replay queue; [4], [5] work counters of the replay and traversal kernels; [6]
                    // unused; [7] size of the hit queue
};

struct WArgs {
    const DevWorld* worlds;
    const DevView* views;
    int32_t n_views;
    int32_t max_depth;
    uint32_t flags;
    int32_t stack_cap;      // traversal stack entries per thread (LDS)
    uint64_t seed;
    CallTable* table;
    Stats* stats;           // NULL: no counters
    PathState S;
    int32_t Q;              // slots per chunk
    int32_t n_chunk;        // paths in this chunk
    int64_t g0;             // global index of the chunk's first path
    int32_t qin;            // ray queue read in this bounce (0/1)
    int32_t first;          // first bounce: the queue is the identity over the chunk's slots
    int32_t lds_nd, lds_nf;  // used entries of the workgroup gradient accumulators
    int32_t ckpt;           // hybrid replay checkpoint interval k, 0 = cached suffix replay
    int32_t hyb_rule;       // hybrid replay: Eq. 3's decision rule (else recomputation only)
    float hyb_gamma;        // scalar PRB update below this depolarization index
    float hyb_eps;          // inversion above this determinant of the normalised block throughput
    unsigned long long* hyb_stats;  // NULL or 3 counters of the rule's branches
    int32_t tape;           // backward by the conventional-AD baseline (stored tape, reverse sweep)
    int32_t prb;            // backward by the P-RB comparator (independent suffix estimates)
    PathState S2;           // P-RB: state of the sub-paths
    int32_t pprb;           // backward by the noise-regularised P-PRB comparator (Sec. 4.2)
    float pprb_sigma;       // its noise deviation
    int32_t ext;            // the scene uses normal maps, specular maps or circular emitters
    int32_t r1;             // render by the rank-one record (every view has a linear-polarizer sensor, no ext)
    int32_t r1adj;          // cached backward of such a batch: the replay start record's rank-one form
    float* out;             // render output
    const float* dout;      // backward: dL/dStokes
    double* gacc;           // backward: FP64 gradient accumulators
    uint64_t* sig;          // optional per-path signatures (global path index)
    const uint8_t* mask;    // optional per-path mask (global path index)
    int32_t one_world;      // the scene has one world, world0 (read from the arguments, not per lane)
    DevWorld world0;
};

// workgroups per kernel family (extend_st: traversal with work counters); compute units
struct LaunchGrid { int extend, shade, adjoint, other, cu, extend_st; };

constexpr uint32_t FLAG_NO_NEE = 1u;

// Size of the fixed device scratch of the allocation-free backward entry point (per GPU).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;

}  // namespace ppt
