// ppt_kernels.hip -- wavefront kernels of the differentiable polarized path tracer (gfx950).
//
// Paths are processed in chunks of a flat index space that spans every view of a plan (the
// batch): path g = (view, crop pixel, sample), samples fastest.  Per chunk and bounce:
//   k_extend   closest-hit traversal of the queued rays (lean kernel, LDS traversal stack),
//              from the second bounce on together with the any-hit traversal of the previous
//              bounce's next-event rays,
//   k_compact  from the one-byte outcome that traversal leaves per slot: misses end their path,
//              hits go to the shading queue,
//   k_shade    vertex sampling and Mueller weights; appends continuing paths to the next ray
//              queue and next-event rays to the shadow queue (workgroup-staged queues, one
//              global atomic per flush).
// Render (Sec. 3.1, Eq. 2): the state carries the prefix Mueller product beta and the radiance
// sum; k_accum reduces the samples of each pixel.  Backward (Sec. 3.2, 4.3, Fig. 2): the primal
// pass caches, per vertex, the weight W_b, the emission + next-event Stokes E_b and a hit record;
// k_fold folds the cache into suffix radiance L[b] = E_b + W_b L[b+1] and queues the paths;
// k_replay replays them forward from the hit records (no second traversal), differentiating each
// vertex against the cached L[b+1].  No Mueller matrix is inverted.
#include "ppt_device.h"

#include <mutex>

namespace ppt {

// ============================================================================ wave helpers
// Workgroup-aggregated counters: one global atomic per workgroup and nonzero counter.  Every
// thread of the workgroup must call it (it synchronizes the workgroup).
struct Count {
    uint32_t c[ST_COUNT];
    DEV Count() {
#pragma unroll
        for (int k = 0; k < ST_COUNT; ++k) c[k] = 0u;
    }
};
DEV void flush_stats(Stats* st, const Count& n) {
    if (!st) return;
    __shared__ uint32_t part[ST_COUNT];
    if (threadIdx.x < ST_COUNT) part[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) {
        uint32_t v = wave_sum_u(n.c[k]);
        if (lane_id() == 0 && v) atomicAdd(&part[k], v);
    }
    __syncthreads();
    if (threadIdx.x < ST_COUNT && part[threadIdx.x]) atomicAdd(&st->c[threadIdx.x], (unsigned long long)part[threadIdx.x]);
}

// Workgroup queue in LDS: lanes append with one LDS atomic per wavefront; the buffer is copied
// to the global queue (one global atomic per flush) when another workgroup iteration might not
// fit, and at the end.
constexpr int QBUF = 2048;
struct BlockQueue {
    int n, base;
    int buf[QBUF];
};
DEV void bq_push(BlockQueue& q, bool pred, int slot) {
    unsigned long long m = __ballot(pred);
    int wb = 0;
    if (lane_id() == 0 && m) wb = atomicAdd(&q.n, (int)__popcll(m));
    wb = __shfl(wb, 0, WAVE);
    if (pred) q.buf[wb + (int)__popcll(m & ((1ull << lane_id()) - 1ull))] = slot;
}
// all threads of the workgroup call it after the pushes of an iteration
DEV void bq_flush(BlockQueue& q, int* gcount, int* gqueue, bool force) {
    __syncthreads();
    int n = q.n;
    if (n > 0 && (force || n > QBUF - BLOCK)) {
        if (threadIdx.x == 0) q.base = atomicAdd(gcount, n);
        __syncthreads();
        int b = q.base;
        for (int k = threadIdx.x; k < n; k += BLOCK) gqueue[b + k] = q.buf[k];
        __syncthreads();
        if (threadIdx.x == 0) q.n = 0;
        __syncthreads();
    }
}
DEV void sig_add(uint64_t& h, uint32_t x) {
#pragma unroll
    for (int i = 0; i < 4; ++i) { h ^= (x >> (8 * i)) & 0xffu; h *= 1099511628211ull; }
}

// Work distribution of the persistent kernels.  Only the first ceil(n / BLOCK) workgroups take
// part (fetch_active; the others leave at once).  Active wavefront w first takes the static batch
// [w * s, (w + 1) * s) with s = n / active wavefronts rounded up and kept in [FETCH_MIN,
// FETCH_BATCH]; positions beyond all static batches are handed out in batches of FETCH_BATCH
// through one atomic on a counter that the previous kernel cleared.  A queue of up to FETCH_BATCH
// positions per wavefront is thus covered by the static batches alone, with no atomic (rounding s
// down to whole wavefronts left up to half of a mid-sized queue to the atomic batches, whose
// early round ends for refill made such launches slower).  A wavefront gives its positions, in
// order, to its lanes that have no work; every lane of the wavefront must call take().
constexpr int FETCH_MIN = WAVE, FETCH_BATCH = 4 * WAVE;
DEV int fetch_blocks(int n) { return max(1, min((int)gridDim.x, (n + BLOCK - 1) / BLOCK)); }
DEV bool fetch_active(int n) { return (int)blockIdx.x < fetch_blocks(n); }
struct WaveFetch {
    int c, cend;    // the wavefront's current batch [c, cend)
    int stat;       // positions covered by the static batches
    bool exhausted;
    DEV explicit WaveFetch(int n) {
        const int waves = fetch_blocks(n) * (BLOCK / WAVE);
        const int w = blockIdx.x * (BLOCK / WAVE) + (int)(threadIdx.x / WAVE);
        int sb = (n + waves - 1) / waves;
        sb = sb < FETCH_MIN ? FETCH_MIN : (sb > FETCH_BATCH ? FETCH_BATCH : sb);
        stat = waves * sb;
        c = min(w * sb, n);
        cend = min(c + sb, n);
        exhausted = n <= stat;
    }
    DEV int take(bool need, int n, int* grab) {
        const unsigned long long m = __ballot(need);
        const int k = (int)__popcll(m), rank = (int)__popcll(m & ((1ull << lane_id()) - 1ull));
        const int rem = cend - c;
        int nb = -1;
        if (k > rem && !exhausted) {
            int base = 0;
            if (lane_id() == 0) base = atomicAdd(grab, FETCH_BATCH);
            nb = stat + __builtin_amdgcn_readfirstlane(__shfl(base, 0, WAVE));
        }
        int idx = -1;
        if (need) {
            if (rank < rem) idx = c + rank;
            else if (nb >= 0 && nb + (rank - rem) < min(nb + FETCH_BATCH, n)) idx = nb + (rank - rem);
        }
        if (nb >= 0) {
            if (nb >= n) { exhausted = true; c = cend = 0; }
            else { cend = min(nb + FETCH_BATCH, n); c = min(nb + (k - rem), cend); }
        } else {
            c = min(c + k, cend);
        }
        return idx;
    }
    DEV bool more() const { return !exhausted || c < cend; }  // wave-uniform
};

// view of a global path index (binary search over the views' first path indices)
DEV int find_view(const DevView* views, int n_views, int64_t g) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (gval(views, (size_t)mid).path_off <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}
// Path keys of a global path index.  The lanes of a wavefront mostly hold consecutive paths, so
// the view of a wave-uniform first index g_first is looked up once and a lane searches only when
// its path lies outside [g_first, end of that view).  The index within a view fits 32 bits (checked
// when the plan is made).
struct PathId { int v, px, py, lx, ly; uint32_t smp, pix, view_id; };
DEV void path_keys(const DevView& V, int64_t g, PathId& r) {
    const uint32_t local = (uint32_t)(g - V.path_off);
    const uint32_t spp = (uint32_t)V.spp, cw = (uint32_t)V.crop_w;
    const uint32_t pl = local / spp;
    r.smp = local - pl * spp;
    r.ly = (int)(pl / cw);
    r.lx = (int)(pl - (uint32_t)r.ly * cw);
    r.px = V.crop_x0 + r.lx;
    r.py = V.crop_y0 + r.ly;
    r.pix = (uint32_t)(r.py * V.width + r.px);
    r.view_id = V.view_id;
}
DEV PathId path_id(const DevView* views, int n_views, int64_t g, int64_t g_first) {
    PathId r;
    const int v0 = __builtin_amdgcn_readfirstlane(find_view(views, n_views, g_first));
    r.v = v0;
    const int64_t end0 = v0 + 1 < n_views ? gval(views, (size_t)(v0 + 1)).path_off : INT64_MAX;
    if (g >= end0 || g < g_first) r.v = find_view(views, n_views, g);
    const DevView V = gval(views, (size_t)r.v);
    path_keys(V, g, r);
    return r;
}

// The call table (parameter pointers, gradient routing) is read for every parameter access; a
// copy in LDS turns those dependent global loads into LDS reads.  All threads call it, followed by
// a workgroup barrier before first use.
DEV void table_to_lds(CallTable* dst, const CallTable* src) {
    const int n = (int)(sizeof(CallTable) / sizeof(int));
    for (int k = threadIdx.x; k < n; k += BLOCK) ((int*)dst)[k] = ((const int*)src)[k];
}

// Record accessors (layouts in ppt_internal.h).
DEV float4* ray_rec(const PathState& S, int i) { return S.ray + (size_t)i * RAY_F4; }
DEV float4* shd_rec(const PathState& S, int i) { return S.shd + (size_t)i * SHD_F4; }
DEV float4* acc_rec(const PathState& S, int i) { return S.acc + (size_t)i * ACC_F4; }
DEV float4* r1_rec(const PathState& S, int i) { return S.acc + (size_t)i * R1_F4; }  // (rank-one render)
// the rank-one render's shadow rays: a dense 32-byte record per slot behind the rank-one records
DEV float4* r1_shd(const PathState& S, int Q, int i) { return S.acc + (size_t)Q * R1_F4 + (size_t)i * 2; }
static_assert(R1_F4 + 2 <= ACC_F4, "the rank-one records and their shadow rays fit in the accumulator array");
// The cached replay's start record in its rank-one form (every view a linear-polarizer sensor): the
// adjoint rows are s_c r with one row r shared by the channels, so the record is 64 bytes, two to a
// line, in the shadow-record array: [0] camera-ray direction, info  [1] pix, smp, r1, r2  [2] s_c
// (r0 = 1, r3 = 0).
DEV float4* rst_rec(const PathState& S, int i) { return S.shd + (size_t)i * 4; }
static_assert(2 + 3 <= SHD_F4 && 4 <= SHD_F4,
              "the dense shadow rays, emitting E_b and rank-one start records fit in the shadow-record array");
// The cached backward's bounces use the shadow-record array as two dense arrays (the fold later
// writes whole 128-byte records there): a 32-byte shadow ray per slot, four to a cache line, and
// the 48-byte E_b of an emitting vertex behind them.
DEV float4* shd1_rec(const PathState& S, int i) { return S.shd + (size_t)i * 2; }
DEV float4* emit1_rec(const PathState& S, int Q, int i) { return S.shd + (size_t)Q * 2 + (size_t)i * 3; }
DEV float4* cache_rec(const PathState& S, int Q, int b0, int i) {  // b0: 0-based vertex index
    return S.cache + ((size_t)b0 * Q + i) * CACHE_F4;
}
DEV float4* hit_rec(const PathState& S, int Q, int b0, int i) { return S.hits + ((size_t)b0 * Q + i); }
DEV float4* tape_rec(const PathState& S, int Q, int b0, int i) {  // (the tape occupies the cache region)
    return S.cache + ((size_t)b0 * Q + i) * TAPE_F4;
}
DEV float4* ckpt_rec(const PathState& S, int Q, int blk, int i) { return S.ckpt + ((size_t)blk * Q + i) * CKPT_F4; }
DEV float4 f4(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
DEV void ld12(const float4* r, float* v) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { float4 t = r[k]; v[4 * k] = t.x; v[4 * k + 1] = t.y; v[4 * k + 2] = t.z; v[4 * k + 3] = t.w; }
}
DEV void st12(float4* r, const float* v) {
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = f4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}
// ray record: origin and direction ([0], [1].xy); keys in [3]
DEV void ray_od(const float4* R, v3& o, v3& d) {
    float4 a = R[0], b = R[1];
    o = mk(a.x, a.y, a.z);
    d = mk(a.w, b.x, b.y);
}
DEV void ray_set(float4* R, v3 o, v3 d, float Cs = 0.0f, float Ss = 0.0f) {
    R[0] = f4(o.x, o.y, o.z, d.x);
    R[1] = f4(d.y, d.z, Cs, Ss);
}

constexpr int INFO_DEAD = 1 << 9;
constexpr int INFO_EMIT = 1 << 10;  // (a cached-backward shadow ray's vertex emits: its E_b is kept)
DEV int info_make(int nverts, bool prev_delta, int view) { return nverts | (prev_delta ? 256 : 0) | (view << 12); }

// World of a view: in a scene of one world it comes from the launch arguments (wave-uniform
// scalar loads), otherwise from the world table through the view.
DEV DevWorld world_of(const WArgs& A, int view) {
    if (A.one_world) return A.world0;
    return gval(A.worlds, (size_t)gval(A.views, (size_t)view).world);
}
DEV DevWorld world_of(const WArgs& A, const DevView& V) { return A.one_world ? A.world0 : gval(A.worlds, (size_t)V.world); }

// ============================================================================ chunk start
#ifndef PPT_EXT_TU  // (non-template kernels: in the main compilation unit only)
__global__ void k_reset_counts(int* counts) {
    if (threadIdx.x < 8) counts[threadIdx.x] = 0;
}

#endif  // PPT_EXT_TU

// Closest hits of the rays of one bounce: a persistent kernel in which a lane takes the next queued
// ray as soon as its own is finished.  SMODE >= 0: the same launch resolves the shadow rays of the
// previous bounce (positions [0, n_s) of one work list, any hit; SMODE is that bounce's mode: 0
// render, 1 backward, 2 hybrid replay), so the two kinds of rays share one launch and its tail.
// SMODE 4: the render's mode for a linear-polarizer sensor (shadow rays and pending radiance in the
// rank-one record of k_shade<4>).
// SMODE -1: the first bounce of rays whose records are written (P-RB sub-paths); SMODE -2: the
// first bounce of a chunk's camera paths, each lane generating the camera ray of the path it takes
// (no separate ray-generation pass writing records that this launch would read back).
// STATS: the launch adds to the work counters (A.stats set); without them a lane holds no counter
// registers.
template <int SMODE, bool STATS>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(STATS ? 1 : 8, 8))) k_extend(WArgs A) {
    extern __shared__ int lds_stack[];
    int* stack = lds_stack + threadIdx.x;
    trav_stack_init(stack);
    PathState& S = A.S;
    const int Q = A.Q;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the queues the following kernels append to
        S.counts[1 - A.qin] = 0;
        S.counts[7] = 0;
        if (SMODE < 0) S.counts[2] = 0;  // (a launch with shadow rays reads it: compaction clears it)
    }
    const int* q = A.qin ? S.queue1 : S.queue0;
    const int ne = A.first ? A.n_chunk : S.counts[A.qin];
    const int ns = SMODE >= 0 ? S.counts[2] : 0;
    const int n = ns + ne;
    if (!fetch_active(n)) return;
    Count cnt;
    WaveFetch F(n);
    Trav T;
    bool alive = false, any = false;
    int slot = -1, info = 0;
    while (true) {
        const int idx = F.take(!alive, n, &S.counts[5]);
        if (idx >= 0) {
            any = idx < ns;
            if (SMODE >= 0 && any) {
                slot = S.squeue[idx];
                // the shadow ray and its vertex's info word in one record (no read of the ray
                // record, whose line would be fetched for its 16-byte key word)
                const float4* H = SMODE == 4 ? r1_shd(S, Q, slot) : SMODE == 1 ? shd1_rec(S, slot) : shd_rec(S, slot);
                const float4 s0 = H[0], s1 = H[1];
                info = __float_as_int(s1.w);
                trav_begin(T, world_of(A, info >> 12),
                           mk(s0.x, s0.y, s0.z), mk(s1.x, s1.y, s1.z), s0.w);
                alive = true;
                ++cnt.c[ST_SHADOW_RAYS];
            } else if (SMODE == -2) {
                // the camera ray of path slot, generated here (its record is written when the ray
                // is finished; a masked path's keys at once, and it is not traversed)
                slot = idx;
                const int64_t g = A.g0 + idx;
                const int64_t g_first = A.g0 + __builtin_amdgcn_readfirstlane(idx);
                const PathId id = path_id(A.views, A.n_views, g, g_first);
                const DevView V = gval(A.views, (size_t)id.v);
                const bool live = !(A.mask && !A.mask[g]);
                v3 o, d;
                camera_ray(V, id.px, id.py, id.smp, A.seed, o, d);
                info = info_make(0, false, id.v) | (live ? 0 : INFO_DEAD);
                trav_begin(T, world_of(A, V), o, d, 3.0e38f);
                alive = live;
                if (A.sig) A.sig[g] = live ? 1469598103934665603ull : 0ull;
                if (live) {
                    ++cnt.c[ST_PATHS];
                    ++cnt.c[ST_RAYS];
                } else {
                    ray_rec(S, slot)[3] = f4(__int_as_float(info), __uint_as_float(id.pix), __uint_as_float(id.smp),
                                             __uint_as_float(V.view_id));
                    S.hflag[slot] = 2;
                    if (S.nv) S.nv[slot] = 0;  // (no vertex)
                }
            } else {
                slot = A.first ? idx : q[idx - ns];
                const float4* R = ray_rec(S, slot);
                // the ray and its info word in one round trip (a dead ray's record is set up
                // and not traversed); a queued continuing ray is live, so in a scene of one world
                // its info word is not needed
                v3 o, d;
                ray_od(R, o, d);
                const bool need_info = A.first || !A.one_world;
                info = need_info ? __float_as_int(R[3].x) : 0;
                trav_begin(T, world_of(A, info >> 12), o, d, 3.0e38f);
                alive = !(info & INFO_DEAD);
                if (alive) ++cnt.c[ST_RAYS];
            }
        }
        if (!__any(alive) && !F.more()) break;
        const bool refill = F.more();
        uint32_t nn = 0, np = 0;
        const bool done = alive && trav_round<STATS>(T, SMODE >= 0 && any, nn, np, stack, refill);
        if (STATS) {
            if (SMODE >= 0 && any) {
                cnt.c[ST_SHADOW_NODES] += nn; cnt.c[ST_SHADOW_PRIMS] += np;
            } else {
                cnt.c[ST_NODES] += nn; cnt.c[ST_PRIMS] += np;
            }
        }
        if (done) {
            alive = false;
            if (SMODE == 4 && any) {
                // rank-one render: the path's radiance words already hold the next-event part
                // (k_shade<4>); an occluded light sample restores them from word 3
                if (T.h.prim >= 0) {
                    float4* AC = r1_rec(S, slot);
                    AC[2] = AC[3];
                }
                if (A.sig) sig_add(A.sig[A.g0 + slot], (uint32_t)(T.h.prim >= 0 ? NEE_OCCLUDED : NEE_VISIBLE));
            } else if (SMODE >= 0 && any) {
                const bool occ = T.h.prim >= 0;
                const float4* H = shd_rec(S, slot);
                if (SMODE == 1) {
                    // the cache record holds E_b plus the next-event part and a visible sample
                    // (k_shade<1>); an occluded light sample sets the E words back to E_b (zero unless
                    // the vertex emits, when it was kept beside the shadow rays) and its visibility word
                    // (two whole 32-byte sectors); a visible one writes nothing
                    if (occ) {
                        float4* dst = cache_rec(S, Q, (info & 255) - 1, slot) + 4;
                        if (info & INFO_EMIT) {
                            const float4* Eb = emit1_rec(S, Q, slot);
#pragma unroll
                            for (int k = 0; k < 3; ++k) dst[k] = Eb[k];
                        } else {  // (E_b is zero)
#pragma unroll
                            for (int k = 0; k < 3; ++k) dst[k] = f4(0.0f, 0.0f, 0.0f, 0.0f);
                        }
                        dst[3] = f4(__int_as_float(NEE_OCCLUDED), 0.0f, 0.0f, 0.0f);
                    }
                } else if (SMODE != 2) {  // the hybrid replay recomputes the next-event part from the visibility bit
                    // (the tape forward adds it to both the radiance and the vertex's E_b)
                    float4* dst = acc_rec(S, slot) + 5;
                    if (!occ)
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            float4 a = dst[k], p = H[2 + k];
                            dst[k] = f4(a.x + p.x, a.y + p.y, a.z + p.z, a.w + p.w);
                        }
                    if (SMODE == 3 && !occ) {
                        float4* te = tape_rec(S, Q, (info & 255) - 1, slot) + 4;
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            float4 a = te[k], p = H[5 + k];
                            te[k] = f4(a.x + p.x, a.y + p.y, a.z + p.z, a.w + p.w);
                        }
                    }
                }
                if (SMODE != 0 && SMODE != 1) {  // in the hit word of the vertex whose light sample this is
                    float* hwp = SMODE == 3 ? &tape_rec(S, Q, (info & 255) - 1, slot)[2].w
                                            : &hit_rec(S, Q, (info & 255) - 1, slot)->x;
                    uint32_t hw = (uint32_t)__float_as_int(*hwp);
                    hw = (hw & ~(7u << 26)) | ((uint32_t)(occ ? NEE_OCCLUDED : NEE_VISIBLE) << 26);
                    *hwp = __int_as_float((int)hw);
                }
                if (A.sig) sig_add(A.sig[A.g0 + slot], (uint32_t)(occ ? NEE_OCCLUDED : NEE_VISIBLE));
            } else if (SMODE == -2) {
                // the camera ray's record: the whole record for a hit (ray, sensor rotation, hit,
                // keys), the keys alone for a ray that escaped (nothing else of it is read); the
                // keys again from the slot and the view in the info word
                float4* R = ray_rec(S, slot);
                const DevView V = gval(A.views, (size_t)(info >> 12));
                PathId id;
                path_keys(V, A.g0 + slot, id);
                if (T.h.prim >= 0) {
                    // rotation from the canonical frame of the light arriving along -d to the
                    // sensor frame, kept in the record's spare words for the pixel reduction
                    const v3 kc = -T.d;
                    float Cs, Ss;
                    rot_cs(kc, canon_x(kc), normalize(ld3(V.r) - kc * dot(ld3(V.r), kc)), Cs, Ss);
                    ray_set(R, T.o, T.d, Cs, Ss);
                    R[2] = f4(T.tb, T.h.u, T.h.v, __int_as_float(T.h.prim));
                }
                R[3] = f4(__int_as_float(info), __uint_as_float(id.pix), __uint_as_float(id.smp),
                          __uint_as_float(V.view_id));
                S.hflag[slot] = T.h.prim >= 0 ? 1 : 0;
                // whether the path has a vertex (the shading kernels of the backward then count them)
                if (S.nv) S.nv[slot] = T.h.prim >= 0 ? 1 : 0;
            } else {
                float4* R = ray_rec(S, slot);
                // the hit in one aligned 16-byte store (a hit's distance is the final tb); a miss
                // writes only its outcome byte (its path ends: nothing reads the hit words)
                if (T.h.prim >= 0) R[2] = f4(T.tb, T.h.u, T.h.v, __int_as_float(T.h.prim));
                S.hflag[slot] = T.h.prim >= 0 ? 1 : 0;
            }
        }
    }
    if (STATS) flush_stats(A.stats, cnt);
}

// ============================================================================ hit compaction
// Splits the rays of this bounce by the outcome byte traversal wrote for each slot: misses end their
// path here (signature; a camera ray that escapes keeps a vertex count of 0, which the pixel
// reduction reads as no radiance), hits go, in queue order, to the hit queue that the shading kernel
// reads, so its lanes all hold a vertex.
template <int MODE>
__global__ void __launch_bounds__(BLOCK) k_compact(WArgs A) {
    PathState& S = A.S;
    const int* qin = A.qin ? S.queue1 : S.queue0;
    const int n = A.first ? A.n_chunk : S.counts[A.qin];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        S.counts[2] = 0;  // the shadow queue the shading kernel appends to (the traversal read it)
        S.counts[5] = 0;  // the work counter of the next traversal launch
    }
    __shared__ BlockQueue qh;
    if (threadIdx.x == 0) qh.n = 0;
    __syncthreads();
    for (int bb = blockIdx.x * BLOCK; bb < n; bb += gridDim.x * BLOCK) {
        const int i = bb + threadIdx.x;
        bool hit = false;
        int slot = 0;
        if (i < n) {
            slot = A.first ? i : qin[i];
            const int f = S.hflag[slot];  // (a byte per ray instead of the hit words of its record)
            hit = f == 1;
            if (f == 0 && A.sig) sig_add(A.sig[A.g0 + slot], 0xffffffffu);
        }
        bq_push(qh, hit, slot);
        bq_flush(qh, &S.counts[7], S.hqueue, false);
    }
    bq_flush(qh, &S.counts[7], S.hqueue, true);
}

// ============================================================================ shading
template <int MODE, bool EXT>
// (four waves per SIMD where the registers then fit without spills)
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MODE == 1 && EXT ? 1 : 4, 8))) k_shade(WArgs A) {
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, nullptr};
    int* qout = A.qin ? S.queue0 : S.queue1;
    const int n = S.counts[7];
    __shared__ BlockQueue qn, qs;
    __shared__ CallTable tab;
    table_to_lds(&tab, A.table);
    K.tab = &tab;
    if (threadIdx.x == 0) { qn.n = 0; qs.n = 0; }
    __syncthreads();
    Count cnt;
    for (int bb = blockIdx.x * BLOCK; bb < n; bb += gridDim.x * BLOCK) {
        int i = bb + threadIdx.x;
        bool cont = false, shadow = false;
        int slot = 0;
        if (i < n) slot = S.hqueue[i];
        const float4* R = ray_rec(S, slot);
        if (i < n) {  // a queued ray is a live path's hit (a dead slot's outcome is never a hit)
            const float4 r3 = R[3], r0 = R[0], r1 = R[1], r2 = R[2];  // one round trip
            const int info = __float_as_int(r3.x);
            int nb = info & 255, v = info >> 12;
            bool prev_delta = (info >> 8) & 1;
            int64_t g = A.g0 + slot;
            const uint32_t pix = __float_as_uint(r3.y), smp = __float_as_uint(r3.z);
            const DevWorld W = world_of(A, v);
            Hit h;
            h.prim = __float_as_int(r2.w);
            h.t = r2.x; h.u = r2.y; h.v = r2.z;
            v3 o = mk(r0.x, r0.y, r0.z), d = mk(r0.w, r1.x, r1.y);
            {  // every queued ray hit a surface
                int b = nb + 1;
                ++cnt.c[ST_VERTICES];
                if (MODE == 1 || MODE == 2 || MODE == 3) S.nv[slot] = (uint8_t)b;  // (the fold reads these)
                Vtx x;
                surface(W, h, o, d, x);
                v3 so, sd;
                float stmax = 0.0f;
                vertex_setup<EXT>(W, K, __float_as_uint(r3.w), A.seed, pix, smp, b, A.max_depth, A.flags, prev_delta, d, x,
                                  so, sd, stmax);
                if (A.sig) {
                    uint64_t sg = A.sig[g];
                    sig_add(sg, (uint32_t)x.orig);
                    // (a sampled direction's lobe word also carries the branch of the sampling frame,
                    // the sign of ns.z in the Duff et al. basis, which rounding can flip for a normal
                    // with z near 0)
                    const bool framed = x.lobe == LOBE_DIFFUSE || x.lobe == LOBE_GLOSSY;
                    sig_add(sg, (uint32_t)x.lobe | (framed && signbit(x.ns.z) ? 16u : 0u));
                    if (x.nee != NEE_PENDING) sig_add(sg, (uint32_t)x.nee);
                    A.sig[g] = sg;
                }
                WC w;
                w.kind = 0;
                float Ee[12], En[12];
                if (MODE != 2) eval_vertex<false, EXT>(W, K, x, w, Ee, En, nullptr, nullptr);
                cont = x.lobe != LOBE_NONE && x.lobe != LOBE_INVALID;
                shadow = x.nee == NEE_PENDING;
                float4* H = shd_rec(S, slot);
                // the vertex's info word carried by its shadow ray's record (vertex count and view;
                // the delta bit is the continuing ray's and is not read for a shadow ray)
                const int info_shd = info_make(b, false, v);
                if (MODE == 2) {
                    // hybrid replay: the hit record, and at a block start the ray into this vertex
                    const bool sphere = !x.tri;
                    *hit_rec(S, A.Q, b - 1, slot) = f4(__int_as_float(h.prim | (x.nee << 26)), sphere ? h.t : h.u, h.v, 0.0f);
                    if ((b - 1) % A.ckpt == 0) {
                        float4* CK = ckpt_rec(S, A.Q, (b - 1) / A.ckpt, slot);
                        CK[0] = f4(o.x, o.y, o.z, prev_delta ? 1.0f : 0.0f);
                        CK[1] = f4(d.x, d.y, d.z, 0.0f);
                    }
                } else if (MODE == 4) {
                    // render with a linear-polarizer sensor: its analyzer is rank one, so the image
                    // needs per channel only the scalar y_c = q^T R_s Lo_c (q: the analyzer's row, R_s:
                    // the sensor rotation).  The path carries the row rho = q^T R_s beta (shared by
                    // the channels, beside beta's RGB scales) instead of beta, and y instead of Lo:
                    // one 64-byte record [rho | rgb | y | y before the next-event part], the shadow ray
                    // in a dense record of its own
                    float4* AC = r1_rec(S, slot);
                    float rho[4], brgb[3], y[3];
                    if (nb == 0) {
                        const DevView V = gval(A.views, (size_t)v);
                        const float th = K.p(V.theta_slot, V.theta_off);
                        const float C2 = cosf(2.0f * th), S2 = sinf(2.0f * th);
                        const float Cs = r1.z, Ss = r1.w;  // sensor rotation of the camera ray
                        rho[0] = 0.5f;
                        rho[1] = 0.5f * (C2 * Cs - S2 * Ss);
                        rho[2] = 0.5f * (C2 * Ss + S2 * Cs);
                        rho[3] = 0.0f;
#pragma unroll
                        for (int c = 0; c < 3; ++c) { brgb[c] = 1.0f; y[c] = 0.0f; }
                    } else {
                        const float4 a0 = AC[0], a1 = AC[1], a4 = AC[2];
                        rho[0] = a0.x; rho[1] = a0.y; rho[2] = a0.z; rho[3] = a0.w;
                        brgb[0] = a1.x; brgb[1] = a1.y; brgb[2] = a1.z;
                        y[0] = a4.x; y[1] = a4.y; y[2] = a4.z;
                    }
                    float pn[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        y[c] += brgb[c] * (rho[0] * Ee[4 * c] + rho[1] * Ee[4 * c + 1] + rho[2] * Ee[4 * c + 2] +
                                           rho[3] * Ee[4 * c + 3]);
                        pn[c] = brgb[c] * (rho[0] * En[4 * c] + rho[1] * En[4 * c + 1] + rho[2] * En[4 * c + 2] +
                                           rho[3] * En[4 * c + 3]);
                    }
                    if (cont) {
                        if (w.kind == 1) {
                            rho[1] = rho[2] = rho[3] = 0.0f;
                        } else {
                            WC ws = w;
                            ws.rgb[0] = 1.0f;
                            float o4[4];
                            w_row(ws, 0, rho, o4);
                            rho[0] = o4[0]; rho[1] = o4[1]; rho[2] = o4[2]; rho[3] = o4[3];
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) brgb[c] *= w.rgb[c];
                    }
                    // the whole record (partial records measured slower)
                    AC[0] = f4(rho[0], rho[1], rho[2], rho[3]);
                    AC[1] = f4(brgb[0], brgb[1], brgb[2], 0.0f);
                    // y with the next-event part as if its light sample were visible (traversal then
                    // writes nothing for a visible one, and restores y from word 3 for an occluded one)
                    if (shadow)
                        AC[2] = f4(y[0] + pn[0], y[1] + pn[1], y[2] + pn[2], 0.0f);
                    else
                        AC[2] = f4(y[0], y[1], y[2], 0.0f);
                    AC[3] = f4(y[0], y[1], y[2], 0.0f);
                    if (shadow) {  // the shadow ray in its dense 32-byte record
                        float4* H4 = r1_shd(S, A.Q, slot);
                        H4[0] = f4(so.x, so.y, so.z, stmax);
                        H4[1] = f4(sd.x, sd.y, sd.z, __int_as_float(info_shd));
                    }
                } else if (MODE == 0 || MODE == 3) {
                    float4* AC = acc_rec(S, slot);
                    float beta[16], brgb[3], Lo[12];
                    if (nb == 0) {  // first vertex: beta = I, no radiance yet
#pragma unroll
                        for (int k = 0; k < 16; ++k) beta[k] = (k % 5 == 0) ? 1.0f : 0.0f;
#pragma unroll
                        for (int c = 0; c < 3; ++c) brgb[c] = 1.0f;
#pragma unroll
                        for (int k = 0; k < 12; ++k) Lo[k] = 0.0f;
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            float4 t = AC[k];
                            beta[4 * k] = t.x; beta[4 * k + 1] = t.y; beta[4 * k + 2] = t.z; beta[4 * k + 3] = t.w;
                        }
                        float4 t = AC[4];
                        brgb[0] = t.x; brgb[1] = t.y; brgb[2] = t.z;
                        ld12(AC + 5, Lo);
                    }
                    // Lo_c += brgb_c beta Ee_c; the pending next-event part likewise
                    float pn[12];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float se = beta[4 * r] * Ee[4 * c] + beta[4 * r + 1] * Ee[4 * c + 1] +
                                       beta[4 * r + 2] * Ee[4 * c + 2] + beta[4 * r + 3] * Ee[4 * c + 3];
                            Lo[4 * c + r] += brgb[c] * se;
                            float sn = beta[4 * r] * En[4 * c] + beta[4 * r + 1] * En[4 * c + 1] +
                                       beta[4 * r + 2] * En[4 * c + 2] + beta[4 * r + 3] * En[4 * c + 3];
                            pn[4 * c + r] = brgb[c] * sn;
                        }
                    }
                    if (shadow) st12(H + 2, pn);
                    st12(AC + 5, Lo);
                    if (MODE == 3) {
                        // the tape record of this vertex: weight, hit, emission (its next-event part is
                        // added when the shadow ray is resolved), the prefix throughput before the
                        // vertex, and the ray into it
                        float4* T = tape_rec(S, A.Q, b - 1, slot);
                        const bool sphere = !x.tri;
                        T[0] = f4(w.rgb[0], w.rgb[1], w.rgb[2], w.A);
                        T[1] = f4(w.B, w.C, w.D, w.ci);
                        T[2] = f4(w.si, w.co, w.so, __int_as_float(h.prim | (x.nee << 26) | (w.kind << 29)));
                        T[3] = f4(sphere ? h.t : h.u, h.v, 0.0f, 0.0f);
                        st12(T + 4, Ee);
                        T[7] = f4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                        for (int k = 0; k < 4; ++k) T[8 + k] = f4(beta[4 * k], beta[4 * k + 1], beta[4 * k + 2], beta[4 * k + 3]);
                        T[12] = f4(brgb[0], brgb[1], brgb[2], prev_delta ? 1.0f : 0.0f);
                        T[13] = f4(o.x, o.y, o.z, d.x);
                        T[14] = f4(d.y, d.z, 0.0f, 0.0f);
                    }
                    if (cont) {
                        if (w.kind == 1) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) { beta[4 * r + 1] = beta[4 * r + 2] = beta[4 * r + 3] = 0.0f; }
                        } else {
                            WC ws = w;
                            ws.rgb[0] = 1.0f;
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                float row[4] = {beta[4 * r], beta[4 * r + 1], beta[4 * r + 2], beta[4 * r + 3]}, o4[4];
                                w_row(ws, 0, row, o4);
                                beta[4 * r] = o4[0]; beta[4 * r + 1] = o4[1]; beta[4 * r + 2] = o4[2]; beta[4 * r + 3] = o4[3];
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k) AC[k] = f4(beta[4 * k], beta[4 * k + 1], beta[4 * k + 2], beta[4 * k + 3]);
                        AC[4] = f4(brgb[0] * w.rgb[0], brgb[1] * w.rgb[1], brgb[2] * w.rgb[2], 0.0f);
                    }
                } else {  // MODE 1
                    float4* C = cache_rec(S, A.Q, b - 1, slot);
                    const bool sphere = !x.tri;
                    C[0] = f4(w.rgb[0], w.rgb[1], w.rgb[2], w.A);
                    C[1] = f4(w.B, w.C, w.D, w.ci);
                    C[2] = f4(w.si, w.co, w.so, __int_as_float(h.prim | (x.nee << 26) | (w.kind << 29)));
                    C[3] = f4(sphere ? h.t : h.u, h.v, 0.0f, 0.0f);
                    // E_b with the next-event part as if its light sample were visible, so that traversal
                    // writes nothing here for a visible one (an occluded one restores E_b from the
                    // shadow record's words 5..7)
                    if (shadow) {
                        float EN[12];
#pragma unroll
                        for (int k = 0; k < 12; ++k) EN[k] = Ee[k] + En[k];
                        st12(C + 4, EN);
                        // the shadow ray in its dense 32-byte record, and E_b where the vertex emits (an
                        // occluded sample restores it; a non-emitting vertex's E_b is zero)
                        float4* H1 = shd1_rec(S, slot);
                        H1[0] = f4(so.x, so.y, so.z, stmax);
                        H1[1] = f4(sd.x, sd.y, sd.z, __int_as_float(info_shd | (x.emit ? INFO_EMIT : 0)));
                        if (x.emit) st12(emit1_rec(S, A.Q, slot), Ee);
                    } else {
                        st12(C + 4, Ee);
                    }
                    // a whole 128-byte record is written; a pending light sample's visibility as if
                    // visible (traversal rewrites it for an occluded one)
                    C[7] = f4(__int_as_float(shadow ? NEE_VISIBLE : 0), 0.0f, 0.0f, 0.0f);
                }
                if (MODE != 4 && MODE != 1 && shadow) {  // a whole record (the Stokes words are [2..4]; partial ones measured slower)
                    H[0] = f4(so.x, so.y, so.z, stmax);
                    H[1] = f4(sd.x, sd.y, sd.z, __int_as_float(info_shd));
                    if (MODE == 3) st12(H + 5, En);  // (the tape's E_b takes the unweighted part)
                    else H[5] = H[6] = H[7] = f4(0.0f, 0.0f, 0.0f, 0.0f);
                }
                float4* Rw = ray_rec(S, slot);
                if (cont) ray_set(Rw, spawn(x.p, x.ng, x.wi), x.wi, r1.z, r1.w);  // (keeps the sensor rotation)
                Rw[3].x = __int_as_float(info_make(b, is_delta(gval(W.mats, (size_t)x.mat).type), v));
            }
        }
        bq_push(qn, cont, slot);
        bq_push(qs, shadow, slot);
        bq_flush(qn, &S.counts[1 - A.qin], qout, false);
        bq_flush(qs, &S.counts[2], S.squeue, false);
    }
    bq_flush(qn, &S.counts[1 - A.qin], qout, true);
    bq_flush(qs, &S.counts[2], S.squeue, true);
    flush_stats(A.stats, cnt);
}

#ifndef PPT_EXT_TU  // (in the main compilation unit only)
// ============================================================================ render: pixel reduction
// Every lane rotates its path's radiance into the sensor frame; the lanes of one pixel (adjacent,
// samples fastest) are summed by a segmented wavefront scan, and the last lane of each segment
// applies the analyzers and adds the mean to the image.  A pixel whose samples span two
// wavefronts or chunks receives several additions.
// R1: the rank-one render of a linear-polarizer sensor, whose paths carry y_c = q^T R_s Lo_c (rotation
// and analyzer row already applied): the scan sums three scalars and the output is (1, C, S, 0) y_c,
// C = cos 2 theta, S = sin 2 theta (the polarizer's Mueller matrix is q' q'^T / 2 with q' = (1, C, S, 0)).
template <bool R1>
__global__ void __launch_bounds__(BLOCK) k_accum(WArgs A) {
    if (!A.out) return;  // signature-only runs produce no image
    constexpr int NA = R1 ? 3 : 12;
    PathState& S = A.S;
    Call K{A.table, nullptr};
    const int lane = lane_id();
    for (int base = blockIdx.x * BLOCK + (threadIdx.x & ~(WAVE - 1)); base < A.n_chunk; base += gridDim.x * BLOCK) {
        int i = base + lane;
        bool valid = i < A.n_chunk;
        int64_t key = -1 - lane;  // distinct per invalid lane
        float acc[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] = 0.0f;
        int v = 0, lx = 0, ly = 0;
        if (R1 && valid) {
            // the keys from the path's index (the wavefront holds consecutive paths), and y from the
            // path's record when the path has a vertex (one byte per path says so): no ray record
            // is read, and no record of a path without radiance
            const PathId id = path_id(A.views, A.n_views, A.g0 + i, A.g0 + base);
            v = id.v; lx = id.lx; ly = id.ly;
            key = ((int64_t)v << 32) | (int64_t)id.pix;
            if (S.nv[i]) {
                const float4 y = r1_rec(S, i)[2];
                acc[0] = y.x; acc[1] = y.y; acc[2] = y.z;
            }
        } else if (valid) {
            // pixel of the path from its stored keys; the segment key is (view, pixel)
            const float4* R = ray_rec(S, i);
            const float4 r3 = R[3];
            const int info = __float_as_int(r3.x);
            v = info >> 12;
            const DevView V = gval(A.views, (size_t)v);
            const uint32_t pix = __float_as_uint(r3.y);
            const int py = (int)(pix / (uint32_t)V.width), px = (int)(pix - (uint32_t)py * (uint32_t)V.width);
            lx = px - V.crop_x0; ly = py - V.crop_y0;
            key = ((int64_t)v << 32) | (int64_t)pix;
            if (!(info & INFO_DEAD) && (info & 255) != 0) {  // a camera ray that escaped has no radiance
                if constexpr (!R1) {
                    const float4 r1 = R[1];
                    const float Cs = r1.z, Ss = r1.w;  // sensor rotation of the camera ray
                    float Lo[12];
                    ld12(acc_rec(S, i) + 5, Lo);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float l1 = Lo[4 * c + 1], l2 = Lo[4 * c + 2];
                        acc[4 * c] = Lo[4 * c];
                        acc[4 * c + 1] = Cs * l1 + Ss * l2;
                        acc[4 * c + 2] = -Ss * l1 + Cs * l2;
                        acc[4 * c + 3] = Lo[4 * c + 3];
                    }
                }
            }
        }
        // inclusive segmented scan toward higher lanes
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            int64_t kup = __shfl_up(key, off, WAVE);
            bool take = lane >= off && kup == key;
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                float t = __shfl_up(acc[k], off, WAVE);
                if (take) acc[k] += t;
            }
        }
        int64_t knext = __shfl_down(key, 1, WAVE);
        bool tail = valid && (lane == WAVE - 1 || knext != key);
        if (tail) {
            const DevView V = gval(A.views, (size_t)v);
            float theta = V.sensor == SENSOR_POLARIZER ? K.p(V.theta_slot, V.theta_off) : 0.0f;
            float inv = 1.0f / (float)V.spp;
            int64_t ob = V.out_off + ((int64_t)ly * V.crop_w + lx) * 12;
            if constexpr (R1) {
                const float C2 = cosf(2.0f * theta), S2 = sinf(2.0f * theta);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float o4[3] = {acc[c], C2 * acc[c], S2 * acc[c]};
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        if (o4[k] != 0.0f) atomicAdd(A.out + ob + 4 * c + k, o4[k] * inv);
                }
            } else {
                int64_t astride = (int64_t)V.crop_w * V.crop_h * 12;
                for (int a = 0; a < V.n_analyzers; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float o4[4];
                        analyzer_apply(V.sensor, theta, a, acc + 4 * c, o4);
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (o4[k] != 0.0f) atomicAdd(A.out + ob + a * astride + 4 * c + k, o4[k] * inv);
                    }
            }
        }
    }
}

#endif  // PPT_EXT_TU

// W_c applied to a Stokes vector without branches on the weight's kind (the loads of a record
// stay together ahead of the arithmetic): the Fresnel form is evaluated and then selected.
// Entries of kind-0 records are not read into the result.
DEV void w_apply_select(const WC& w, int c, const float* in, float* out) {
    float v1 = w.ci * in[1] + w.si * in[2], v2 = -w.si * in[1] + w.ci * in[2];
    float f0 = w.A * in[0] + w.B * v1, f1 = w.B * in[0] + w.A * v1;
    float f2 = w.C * v2 + w.D * in[3], f3 = -w.D * v2 + w.C * in[3];
    const float s = w.rgb[c];
    const bool fr = w.kind == 2, df = w.kind == 1;
    out[0] = fr ? s * f0 : (df ? s * in[0] : 0.0f);
    out[1] = fr ? s * (w.co * f1 + w.so * f2) : 0.0f;
    out[2] = fr ? s * (-w.so * f1 + w.co * f2) : 0.0f;
    out[3] = fr ? s * f3 : 0.0f;
}

// ============================================================================ hybrid replay blocks
// Hybrid cached replay (Sec. 4.4): the primal pass keeps a hit record per vertex and, every k
// vertices, the ray into the block's first vertex; suffix values are kept only at block ends.
// block_eval re-evaluates vertices [s, e) of the path in `slot` from the ray (o, d) into vertex s,
// with each vertex's recorded next-event visibility, into the scratch cache records rec0 ..
// rec0 + e-s-1 (W_b and E_b); block_fold then folds records rec0 .. rec0 + n-1 back from the
// suffix L beyond the last of them, leaving in L the suffix at the first one's vertex (with
// store_suffix, each record's E words receive the suffix beyond its vertex, which the replay reads).
template <bool EXT>
DEV void block_eval(const WArgs& A, const Call& K, const DevView& V, const DevWorld& W, int slot, uint32_t pix,
                    uint32_t smp, int s, int e, v3 o, v3 d, bool prev_delta, int rec0 = 0) {
    const PathState& S = A.S;
    const int Q = A.Q;
    for (int v = s; v < e; ++v) {
        const float4 hr = *hit_rec(S, Q, v, slot);
        const uint32_t hw = __float_as_uint(hr.x);
        Hit h;
        h.prim = (int)(hw & ((1u << 26) - 1));
        h.u = hr.y; h.t = hr.y; h.v = hr.z;
        Vtx x;
        surface(W, h, o, d, x);
        v3 so, sd;
        float stmax;
        vertex_setup<EXT>(W, K, V.view_id, A.seed, pix, smp, v + 1, A.max_depth, A.flags, prev_delta, d, x, so, sd, stmax);
        if (x.nee == NEE_PENDING) x.nee = (int)((hw >> 26) & 7);
        WC w;
        float Ee[12], En[12];
        eval_vertex<false, EXT>(W, K, x, w, Ee, En, nullptr, nullptr);
        float4* C = cache_rec(S, Q, rec0 + v - s, slot);
        C[0] = f4(w.rgb[0], w.rgb[1], w.rgb[2], w.A);
        C[1] = f4(w.B, w.C, w.D, w.ci);
        C[2] = f4(w.si, w.co, w.so, __int_as_float(w.kind << 29));
#pragma unroll
        for (int q = 0; q < 12; ++q) Ee[q] += En[q];
        st12(C + 4, Ee);
        prev_delta = is_delta(gval(W.mats, (size_t)x.mat).type);
        o = spawn(x.p, x.ng, x.wi);
        d = x.wi;
    }
}
DEV void block_fold(const PathState& S, int Q, int slot, int n, float* L, bool store_suffix, int rec0 = 0) {
    for (int u = rec0 + n - 1; u >= rec0; --u) {
        float4* C = cache_rec(S, Q, u, slot);
        const float4 c0 = C[0], c1 = C[1], c2 = C[2];
        float e[12];
        ld12(C + 4, e);
        if (store_suffix) st12(C + 4, L);
        WC w;
        w.rgb[0] = c0.x; w.rgb[1] = c0.y; w.rgb[2] = c0.z;
        w.A = c0.w; w.B = c1.x; w.C = c1.y; w.D = c1.z;
        w.ci = c1.w; w.si = c2.x; w.co = c2.y; w.so = c2.z;
        w.kind = (__float_as_int(c2.w) >> 29) & 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float o4[4];
            w_apply_select(w, c, L + 4 * c, o4);
#pragma unroll
            for (int k = 0; k < 4; ++k) L[4 * c + k] = e[4 * c + k] + o4[k];
        }
    }
}

// ============================================================================ P-PRB comparator
// Regularisation noise of the noise-regularised polarized PRB (Sec. 4.2): one normal variate
// u ~ N(0, sigma) per path vertex (1-based index vtx) from two uniforms of the vertex's counter
// (call 2) by the Box-Muller transform; the fold and the replay draw the same value.
DEV float pprb_noise(const WArgs& A, uint32_t pix, uint32_t smp, uint32_t view_id, int vtx) {
    float u[4];
    uniforms(A.seed, pix, smp, view_id, (uint32_t)vtx, 2, u);
    return A.pprb_sigma * sqrtf(-2.0f * logf(1.0f - u[0])) * cosf(6.28318530717958648f * u[1]);
}
// W_c of a compact weight as a row-major 4x4 (column j = W_c e_j)
DEV void w_matrix(const WC& w, int c, float* m) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float e[4] = {j == 0 ? 1.0f : 0.0f, j == 1 ? 1.0f : 0.0f, j == 2 ? 1.0f : 0.0f, j == 3 ? 1.0f : 0.0f}, o[4];
        w_apply(w, c, e, o);
#pragma unroll
        for (int r = 0; r < 4; ++r) m[4 * r + j] = o[r];
    }
}

// ============================================================================ backward: fold

// Per path with at least one vertex: folds the cache into the suffix radiance
// L[b] = E_b + W_b L[b+1] (L[b+1] written over E_b), adds the polarizer-angle term
// delta^T (dP/dtheta) R_s L[1],
// and sets up the replay: the adjoint rows a_c = (delta^T A / spp) R_s, the camera ray's direction,
// the path's keys and vertex count (all in the shadow record's words 0..4) and an entry of the replay queue (queue0, size counts[3]).  Each workgroup folds one
// contiguous range of slots, so its lanes mostly see a single view and keep the angle term in a
// register until the view changes.
// PPRB (the noise-regularised comparator of Sec. 4.2): the fold uses W_b + u_b I, keeps the records'
// E words (the replay inverts the weights instead of reading suffixes) and stores the path's
// regularised radiance L'[1] in the shadow record's words 5..7.
// TAPE (the conventional-AD baseline): no fold; the path's radiance comes from the forward
// accumulator, for the polarizer-angle term and the adjoint rows.
template <bool HYB, bool EXT, bool PPRB = false, bool TAPE = false>
// (six waves per SIMD for the cached fold: its registers then fit without spills, measured faster)
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(HYB ? 1 : 6, 8))) k_fold(WArgs A) {
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, A.gacc};
    __shared__ BlockQueue rq;
    if (threadIdx.x == 0) rq.n = 0;
    __syncthreads();
    const int r0 = (int)((int64_t)A.n_chunk * blockIdx.x / gridDim.x);
    const int r1 = (int)((int64_t)A.n_chunk * (blockIdx.x + 1) / gridDim.x);
    float gtheta = 0.0f;
    int tkey = -1;
    for (int base = r0; base < r1; base += BLOCK) {
        const int i = base + threadIdx.x;
        bool push = false;
        // the path's vertex count from the dense byte array and its keys from its index (no read of
        // its ray record, which would cost a 128-byte line for 16 bytes)
        const int B = i < r1 ? (int)S.nv[i] : 0;
        float gt = 0.0f;
        if (B > 0) {
            push = true;
            // (keys before the fold only where the fold needs them: fewer registers live across it)
            const int64_t gw = A.g0 + base + (int)(threadIdx.x & ~(WAVE - 1));
            PathId id{};
            if (HYB || PPRB) id = path_id(A.views, A.n_views, A.g0 + i, gw);
            // fold over records B-1 .. 0 (record r holds vertex r+1): the record's E words receive
            // the suffix beyond its vertex, L[r+2], so the replay of a vertex reads one record (the
            // last vertex's suffix is zero and is not stored)
            float L[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) L[k] = 0.0f;
            if (HYB) {
                // blocks from the last to the first: re-evaluate from the block's checkpoint ray,
                // store the suffix beyond the block, fold back to the block's first vertex
                const DevView Vh = gval(A.views, (size_t)id.v);
                const DevWorld Wh = world_of(A, Vh);
                const int kc = A.ckpt;
                for (int j = (B + kc - 1) / kc - 1; j >= 0; --j) {
                    const int s0 = j * kc, e0 = min(B, s0 + kc);
                    float4* CK = ckpt_rec(S, Q, j, i);
                    const float4 k0 = CK[0], k1 = CK[1];
                    block_eval<EXT>(A, K, Vh, Wh, i, id.pix, id.smp, s0, e0, mk(k0.x, k0.y, k0.z), mk(k1.x, k1.y, k1.z),
                               k0.w != 0.0f);
                    st12(CK + 2, L);
                    block_fold(S, Q, i, e0 - s0, L, false);
                }
                // the suffix at the first vertex, the decision rule's remaining radiance of block 0
                if (A.hyb_rule) st12(shd_rec(S, i) + 5, L);
            }
            if (TAPE) ld12(acc_rec(S, i) + 5, L);
            for (int b = HYB || TAPE ? -1 : B - 1; b >= 0; --b) {
                float4* C = cache_rec(S, Q, b, i);
                const float4 c0 = C[0], c1 = C[1], c2 = C[2];
                float e[12];
                ld12(C + 4, e);
                if (!PPRB && b < B - 1) st12(C + 4, L);
                const float u = PPRB ? pprb_noise(A, id.pix, id.smp, id.view_id, b + 1) : 0.0f;
                WC w;
                w.rgb[0] = c0.x; w.rgb[1] = c0.y; w.rgb[2] = c0.z;
                w.A = c0.w; w.B = c1.x; w.C = c1.y; w.D = c1.z;
                w.ci = c1.w; w.si = c2.x; w.co = c2.y; w.so = c2.z;
                w.kind = (__float_as_int(c2.w) >> 29) & 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float o4[4];
                    w_apply_select(w, c, L + 4 * c, o4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) L[4 * c + k] = e[4 * c + k] + o4[k] + (PPRB ? u * L[4 * c + k] : 0.0f);
                }
            }
            if (PPRB) st12(shd_rec(S, i) + 5, L);
            if (!(HYB || PPRB)) id = path_id(A.views, A.n_views, A.g0 + i, gw);
            const int v = id.v;
            const uint32_t pix = id.pix, smp = id.smp;
            const DevView V = gval(A.views, (size_t)v);
            const int py = (int)(pix / (uint32_t)V.width), px = (int)(pix - (uint32_t)py * (uint32_t)V.width);
            const int lx = px - V.crop_x0, ly = py - V.crop_y0;
            v3 o, d;
            camera_ray(V, px, py, smp, A.seed, o, d);
            v3 kc = -d;
            float Cs, Ss;
            rot_cs(kc, canon_x(kc), normalize(ld3(V.r) - kc * dot(ld3(V.r), kc)), Cs, Ss);
            const bool pol = V.sensor == SENSOR_POLARIZER;
            float theta = pol ? K.p(V.theta_slot, V.theta_off) : 0.0f;
            // adjoint of the pixel mean in the sensor frame: a_sens_c = sum_a delta_a,c^T A_a / spp;
            // the polarizer-angle term (one analyzer) is delta^T (dP/dtheta) R_s L[1]
            const float inv = 1.0f / (float)V.spp;
            const int64_t astride = (int64_t)V.crop_w * V.crop_h * 12;
            const float* dp = A.dout + V.out_off + ((int64_t)ly * V.crop_w + lx) * 12;
            float asens[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) asens[k] = 0.0f;
            for (int a = 0; a < V.n_analyzers; ++a) {
                float dl[12];
#pragma unroll
                for (int k = 0; k < 12; ++k) dl[k] = dp[a * astride + k] * inv;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float r4[4];
                    analyzer_row(V.sensor, theta, a, dl + 4 * c, r4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) asens[4 * c + k] += r4[k];
                    if (pol && a == 0) {
                        float l1 = L[4 * c + 1], l2 = L[4 * c + 2];
                        float ls[4] = {L[4 * c], Cs * l1 + Ss * l2, -Ss * l1 + Cs * l2, L[4 * c + 3]};
                        gt += polarizer_dtheta(theta, dl + 4 * c, ls);
                    }
                }
            }
            float av[12];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float a1 = asens[4 * c + 1], a2 = asens[4 * c + 2];
                av[4 * c] = asens[4 * c];
                av[4 * c + 1] = Cs * a1 - Ss * a2;
                av[4 * c + 2] = Ss * a1 + Cs * a2;
                av[4 * c + 3] = asens[4 * c + 3];
            }
            // the replay's start in one record: the camera ray's direction (its origin is the view's),
            // the info word (vertex count, view), the keys and the adjoint rows
            const int info_rs = info_make((int)S.nv[i], false, v);  // (B read again: fewer live registers)
            if (!HYB && !PPRB && !TAPE && A.r1adj) {
                // rank-one form: a linear polarizer's analyzer row is q' = (1, C, S, 0) and a_c = s_c q'^T
                // rotated by R_s, with s_c = asens_c0
                const float C2 = cosf(2.0f * theta), S2 = sinf(2.0f * theta);
                float4* Hr = rst_rec(S, i);
                Hr[0] = f4(d.x, d.y, d.z, __int_as_float(info_rs));
                Hr[1] = f4(__uint_as_float(pix), __uint_as_float(smp), Cs * C2 - Ss * S2, Ss * C2 + Cs * S2);
                Hr[2] = f4(asens[0], asens[4], asens[8], 0.0f);
                Hr[3] = f4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                float4* Hs = shd_rec(S, i);
                Hs[0] = f4(d.x, d.y, d.z, __int_as_float(info_rs));
                Hs[1] = f4(__uint_as_float(pix), __uint_as_float(smp), 0.0f, 0.0f);
                st12(Hs + 2, av);
                // the rest of the 128-byte record where nothing else fills it (a line written in part
                // is the slower path)
                if (!PPRB && !(HYB && A.hyb_rule)) Hs[5] = Hs[6] = Hs[7] = f4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            if (pol) {
                if (tkey != v) {
                    if (tkey >= 0) K.g(A.views[tkey].theta_slot, A.views[tkey].theta_off, gtheta);
                    gtheta = 0.0f;
                    tkey = v;
                }
                gtheta += gt;
            }
        }
        bq_push(rq, push, i);
        bq_flush(rq, &S.counts[3], S.queue0, false);
    }
    bq_flush(rq, &S.counts[3], S.queue0, true);
    // polarizer angles: one atomic per distinct view among the wavefront's running sums
    bool pending = tkey >= 0;
    while (__ballot(pending)) {
        unsigned long long m = __ballot(pending);
        int leader = __ffsll((long long)m) - 1;
        int key = __shfl(tkey, leader, WAVE);
        bool mine = pending && tkey == key;
        float s = wave_sum(mine ? gtheta : 0.0f);
        if (lane_id() == leader) K.g(A.views[key].theta_slot, A.views[key].theta_off, s);
        pending = pending && !mine;
    }
}

// ============================================================================ gradient accumulators
// Adds a workgroup's LDS gradient accumulators into the global FP64 accumulator (every thread calls
// it after a workgroup barrier).
DEV void flush_lds_grads(const WArgs& A, const Call& K) {
    __syncthreads();
    const CallTable* T = A.table;
    for (int s = 0; s < MAX_SLOTS; ++s) {
        int od = T->lds_d[s], of = T->lds_f[s];
        if (od < 0 && of < 0) continue;
        int64_t go = T->goff[s], nn = T->numel[s];
        for (int64_t q = threadIdx.x; q < nn; q += BLOCK) {
            double val = od >= 0 ? K.lds_d[od + q] : (double)K.lds_f[of + q];
            if (val != 0.0) unsafeAtomicAdd(A.gacc + go + q, val);
        }
    }
}

// ============================================================================ hybrid replay: decision rule
// 4x4 inverse by Laplace expansion along the first two rows: returns det m and writes its adjugate
// (row-major; inverse = adj / det).
DEV float adjugate4(const float* m, float* adj) {
    const float a0 = m[0], a1 = m[1], a2 = m[2], a3 = m[3], b0 = m[4], b1 = m[5], b2 = m[6], b3 = m[7];
    const float c0 = m[8], c1 = m[9], c2 = m[10], c3 = m[11], d0 = m[12], d1 = m[13], d2 = m[14], d3 = m[15];
    const float s0 = a0 * b1 - a1 * b0, s1 = a0 * b2 - a2 * b0, s2 = a0 * b3 - a3 * b0;
    const float s3 = a1 * b2 - a2 * b1, s4 = a1 * b3 - a3 * b1, s5 = a2 * b3 - a3 * b2;
    const float t0 = c0 * d1 - c1 * d0, t1 = c0 * d2 - c2 * d0, t2 = c0 * d3 - c3 * d0;
    const float t3 = c1 * d2 - c2 * d1, t4 = c1 * d3 - c3 * d1, t5 = c2 * d3 - c3 * d2;
    adj[0] = b1 * t5 - b2 * t4 + b3 * t3;   adj[1] = -a1 * t5 + a2 * t4 - a3 * t3;
    adj[2] = d1 * s5 - d2 * s4 + d3 * s3;   adj[3] = -c1 * s5 + c2 * s4 - c3 * s3;
    adj[4] = -b0 * t5 + b2 * t2 - b3 * t1;  adj[5] = a0 * t5 - a2 * t2 + a3 * t1;
    adj[6] = -d0 * s5 + d2 * s2 - d3 * s1;  adj[7] = c0 * s5 - c2 * s2 + c3 * s1;
    adj[8] = b0 * t4 - b1 * t2 + b3 * t0;   adj[9] = -a0 * t4 + a1 * t2 - a3 * t0;
    adj[10] = d0 * s4 - d1 * s2 + d3 * s0;  adj[11] = -c0 * s4 + c1 * s2 - c3 * s0;
    adj[12] = -b0 * t3 + b1 * t1 - b2 * t0; adj[13] = a0 * t3 - a1 * t1 + a2 * t0;
    adj[14] = -d0 * s3 + d1 * s1 - d2 * s0; adj[15] = c0 * s3 - c1 * s1 + c2 * s0;
    return s0 * t5 - s1 * t4 + s2 * t3 + s3 * t2 - s4 * t1 + s5 * t0;
}

// Eq. 3 at vertex v0 of the block [s0, e0) (v0 + 1 < e0): adds the vertex's detached weight and
// emission to the block throughput (Mb, bs) and the remaining radiance, then recovers the suffix
// L[v0+1] into Ln by the scalar PRB update, the inverse, or recomputation of vertices v0+1 .. e0-1
// into the scratch records (rec_from = v0 + 1 afterwards).  One decision serves the three channels:
// their throughputs differ by a scale, which neither test sees.
template <bool EXT>
DEV void suffix_by_rule(const WArgs& A, const Call& K, const DevView& V, const DevWorld& W, const Vtx& x, int slot,
                        uint32_t pix, uint32_t smp, int v0, int s0, int e0, float* Mb, float* bs, float* Lrem,
                        float* Ln, int& rec_from, uint32_t* n_br) {
    WC wf;
    float Ef[12], Enf[12];
    eval_vertex<false, EXT>(W, K, x, wf, Ef, Enf, nullptr, nullptr);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float se = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) se += Mb[4 * r + j] * (Ef[4 * c + j] + Enf[4 * c + j]);
            Lrem[4 * c + r] -= bs[c] * se;
        }
    if (wf.kind == 2) {
        WC ws = wf;
        ws.rgb[0] = 1.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float row[4] = {Mb[4 * r], Mb[4 * r + 1], Mb[4 * r + 2], Mb[4 * r + 3]}, o4[4];
            w_row(ws, 0, row, o4);
            Mb[4 * r] = o4[0]; Mb[4 * r + 1] = o4[1]; Mb[4 * r + 2] = o4[2]; Mb[4 * r + 3] = o4[3];
        }
    } else {  // diffuse: only the first column survives; no weight: nothing does
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (wf.kind == 0) Mb[4 * r] = 0.0f;
            Mb[4 * r + 1] = Mb[4 * r + 2] = Mb[4 * r + 3] = 0.0f;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) bs[c] *= wf.kind == 0 ? 0.0f : wf.rgb[c];
    const float m00 = Mb[0];
    const bool live = m00 > 0.0f && bs[0] > 0.0f && bs[1] > 0.0f && bs[2] > 0.0f;
    int br = 2;
    float adj[16], det = 0.0f;
    if (live) {
        const float im = 1.0f / m00;
        float ss = 0.0f, Mn[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) { Mn[k] = Mb[k] * im; ss += Mn[k] * Mn[k]; }
        const float di = sqrtf(fmaxf(0.0f, ss - 1.0f)) * 0.57735026918962576f;  // (normalised: M00 = 1)
        if (di < A.hyb_gamma) {
            br = 0;
        } else {
            det = adjugate4(Mn, adj);
            if (fabsf(det) > A.hyb_eps) br = 1;
        }
    }
    n_br[0] += br == 0 ? 1u : 0u;  // (constant indices: the counters stay in registers)
    n_br[1] += br == 1 ? 1u : 0u;
    n_br[2] += br == 2 ? 1u : 0u;
    if (br == 0) {  // treated as depolarizing: the suffix's intensity only
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Ln[4 * c] = Lrem[4 * c] / (m00 * bs[c]);
            Ln[4 * c + 1] = Ln[4 * c + 2] = Ln[4 * c + 3] = 0.0f;
        }
    } else if (br == 1) {  // beta^-1 Lrem = (Mn^-1 Lrem) / (m00 bs_c)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float f = 1.0f / (det * m00 * bs[c]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Ln[4 * c + r] = f * (adj[4 * r] * Lrem[4 * c] + adj[4 * r + 1] * Lrem[4 * c + 1] +
                                     adj[4 * r + 2] * Lrem[4 * c + 2] + adj[4 * r + 3] * Lrem[4 * c + 3]);
        }
    } else {  // recompute the rest of the block from the ray leaving this vertex
        const PathState& S = A.S;
        const int rec0 = v0 + 1 - s0;
        block_eval<EXT>(A, K, V, W, slot, pix, smp, v0 + 1, e0, spawn(x.p, x.ng, x.wi), x.wi,
                        is_delta(gval(W.mats, (size_t)x.mat).type), rec0);
        ld12(ckpt_rec(S, A.Q, s0 / A.ckpt, slot) + 2, Ln);
        block_fold(S, A.Q, slot, e0 - v0 - 1, Ln, true, rec0);
        rec_from = v0 + 1;
    }
}

// ============================================================================ backward: replay
// Persistent replay of the queued paths from their hit records (no second traversal): every lane
// replays one vertex per iteration and takes the next queued path as soon as its own ends, so
// short and long paths share a wavefront without idling.  At vertex b the lane differentiates
// E_b + W_b L[b+1] against its adjoint rows, then advances them, a <- a W_b.  Gradients go to
// workgroup LDS accumulators, flushed at the end.
//
// Hybrid replay (HYB): the suffix beyond a vertex comes from the scratch records of its block.
// Without RULE the whole block is recomputed from its checkpoint ray when the replay enters it.
// With RULE (Sec. 4.4, Eq. 3) the lane instead carries the detached block throughput beta (the
// product of the block's weights so far: a shared 4x4 and RGB scales) and the radiance of the
// block's checkpoint that its vertices have not yet emitted, Lrem = beta L[b+1], and recovers a
// suffix by the scalar PRB update (Lrem_0 / beta_00, unpolarized) when the depolarization index
// of beta is below gamma, by beta^-1 Lrem when |det beta| > eps beta_00^4, and otherwise by
// recomputing the rest of the block into the scratch records, which the block's later vertices
// then read.  The block's last suffix is the next checkpoint's.
//
// PPRB (the comparator of Sec. 4.2): no cached suffix; the lane carries the regularised radiance
// L'_b still to be explained and recovers the suffix as (W_b + u_b I)^-1 (L'_b - E_b) from the
// primal's weight and emission records, advancing its adjoint rows by W_b + u_b I.
template <bool HYB, bool EXT, bool RULE = false, bool PPRB = false>
__global__ void __launch_bounds__(BLOCK) k_replay(WArgs A) {
    extern __shared__ double lds_grad[];
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, A.gacc};
    __shared__ CallTable tab;
    table_to_lds(&tab, A.table);
    K.tab = &tab;
    K.lds_d = lds_grad;
    K.lds_f = (float*)(lds_grad + A.lds_nd);
    for (int k = threadIdx.x; k < A.lds_nd; k += BLOCK) K.lds_d[k] = 0.0;
    for (int k = threadIdx.x; k < A.lds_nf; k += BLOCK) K.lds_f[k] = 0.0f;
    __syncthreads();
    const int n = S.counts[3];
    WaveFetch F(n);
    int slot = -1, b = 0, B = 0, v = 0;
    uint32_t pix = 0, smp = 0;
    bool prev_delta = false;
    float av[12];
    v3 o = mk(0.0f, 0.0f, 0.0f), d = o;
#pragma unroll
    for (int k = 0; k < 12; ++k) av[k] = 0.0f;
    // decision-rule state (RULE): block throughput (shared part and RGB scales), remaining radiance,
    // first vertex of the block whose suffix sits in the scratch records, and branch counts
    float Mb[RULE ? 16 : 1], bs[RULE ? 3 : 1], Lrem[RULE ? 12 : 1];
    float Lcur[PPRB ? 12 : 1];  // PPRB: the regularised suffix at the current vertex
    int rec_from = 0;
    uint32_t n_br[3] = {0u, 0u, 0u};
    while (true) {
        // hand queue entries to the lanes without a path
        const int idx = F.take(slot < 0, n, &S.counts[4]);
        if (idx >= 0) {
            slot = S.queue0[idx];
            // the path's start as the fold left it in the shadow-record array (one record per path)
            const bool r1s = !HYB && !PPRB && A.r1adj;  // (the 64-byte rank-one form)
            const float4* H = r1s ? rst_rec(S, slot) : shd_rec(S, slot);
            const float4 h0 = H[0], h1 = H[1];
            const int info = __float_as_int(h0.w);
            B = info & 255;
            v = info >> 12;
            b = 1;
            prev_delta = false;
            pix = __float_as_uint(h1.x);
            smp = __float_as_uint(h1.y);
            if (r1s) {
                const float4 h2 = H[2];
                const float sc[3] = {h2.x, h2.y, h2.z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    av[4 * c] = sc[c]; av[4 * c + 1] = sc[c] * h1.z; av[4 * c + 2] = sc[c] * h1.w; av[4 * c + 3] = 0.0f;
                }
            } else {
                ld12(H + 2, av);
            }
            if (PPRB) ld12(H + 5, Lcur);
            d = mk(h0.x, h0.y, h0.z);
            o = ld3(gval(A.views, (size_t)v).o);  // (a pinhole camera's rays leave the view's origin)
        }
        if (!__any(slot >= 0)) break;
        if (slot >= 0) {
            const DevView V = gval(A.views, (size_t)v);
            const DevWorld W = world_of(A, V);
            uint32_t hw;
            float hu, hv;
            const float4* C;  // the record whose E words hold the suffix beyond this vertex
            const int v0 = b - 1;
            const int s0 = HYB ? v0 - v0 % A.ckpt : 0, e0 = HYB ? min(B, s0 + A.ckpt) : 0;
            if (HYB) {
                if (!RULE && v0 == s0) {  // block start: recompute the block's suffix values
                    block_eval<EXT>(A, K, V, W, slot, pix, smp, v0, e0, o, d, prev_delta);
                    float Lb[12];
                    ld12(ckpt_rec(S, Q, v0 / A.ckpt, slot) + 2, Lb);
                    block_fold(S, Q, slot, e0 - v0, Lb, true);
                }
                if constexpr (RULE) {
                    if (v0 == s0) {  // block start: beta = I, Lrem = the suffix at the block's first vertex
#pragma unroll
                        for (int k = 0; k < 16; ++k) Mb[k] = (k % 5 == 0) ? 1.0f : 0.0f;
                        bs[0] = bs[1] = bs[2] = 1.0f;
                        ld12(s0 == 0 ? shd_rec(S, slot) + 5 : ckpt_rec(S, Q, s0 / A.ckpt - 1, slot) + 2, Lrem);
                        rec_from = 0x7fffffff;
                    }
                }
                const float4 hr = *hit_rec(S, Q, v0, slot);
                hw = __float_as_uint(hr.x); hu = hr.y; hv = hr.z;
                C = cache_rec(S, Q, v0 - s0, slot);
            } else {
                C = cache_rec(S, Q, b - 1, slot);
                const float4 c2 = C[2], c3 = C[3];
                hw = __float_as_uint(c2.w); hu = c3.x; hv = c3.y;
            }
            Hit h;
            h.prim = (int)(hw & ((1u << 26) - 1));
            // the next-event visibility: in the hit record's word (hybrid), in the cache record's
            // last vector (cached)
            const int rec_nee = HYB ? (int)((hw >> 26) & 7) : __float_as_int(C[7].x);
            h.u = hu; h.t = hu; h.v = hv;
            Vtx x;
            surface(W, h, o, d, x);
            v3 so, sd;
            float stmax;
            vertex_setup<EXT>(W, K, V.view_id, A.seed, pix, smp, b, A.max_depth, A.flags, prev_delta, d, x, so, sd, stmax);
            if (x.nee == NEE_PENDING) x.nee = rec_nee;
            float Ln[12];  // L[b+1], stored in this vertex's record by the fold (zero after the last)
            if (b >= B) {
#pragma unroll
                for (int q = 0; q < 12; ++q) Ln[q] = 0.0f;
            } else if (PPRB) {
                // (W_b + u I)^-1 (L'_b - E_b) per channel, from the primal's records
                const float4 c0 = C[0], c1 = C[1], c2 = C[2];
                WC wr;
                wr.rgb[0] = c0.x; wr.rgb[1] = c0.y; wr.rgb[2] = c0.z;
                wr.A = c0.w; wr.B = c1.x; wr.C = c1.y; wr.D = c1.z;
                wr.ci = c1.w; wr.si = c2.x; wr.co = c2.y; wr.so = c2.z;
                wr.kind = (__float_as_int(c2.w) >> 29) & 3;
                float e[12];
                ld12(C + 4, e);
                const float u = pprb_noise(A, pix, smp, V.view_id, b);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float m[16], adj[16];
                    w_matrix(wr, c, m);
                    m[0] += u; m[5] += u; m[10] += u; m[15] += u;
                    const float idet = 1.0f / adjugate4(m, adj);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float t = 0.0f;
#pragma unroll
                        for (int j = 0; j < 4; ++j) t += adj[4 * r + j] * (Lcur[4 * c + j] - e[4 * c + j]);
                        Ln[4 * c + r] = t * idet;
                    }
                }
            } else if (!RULE) {
                ld12(C + 4, Ln);
            } else if (v0 + 1 == e0) {  // the block's last suffix: the next checkpoint's
                ld12(ckpt_rec(S, Q, s0 / A.ckpt, slot) + 2, Ln);
            } else if (v0 >= rec_from) {  // recomputed earlier in this block
                ld12(C + 4, Ln);
            } else {
                suffix_by_rule<EXT>(A, K, V, W, x, slot, pix, smp, v0, s0, e0, Mb, bs, Lrem, Ln, rec_from, n_br);
            }
            WC w;
            float Ee[12], En[12];
            K.coherent = b == 1;
            eval_vertex<true, EXT>(W, K, x, w, Ee, En, av, Ln);
            if (b >= B || x.lobe == LOBE_NONE || x.lobe == LOBE_INVALID) {
                slot = -1;
            } else {
                const float un = PPRB ? pprb_noise(A, pix, smp, V.view_id, b) : 0.0f;
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    float o4[4];
                    w_row(w, cc, av + 4 * cc, o4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) av[4 * cc + q] = o4[q] + (PPRB ? un * av[4 * cc + q] : 0.0f);
                }
                if (PPRB)
#pragma unroll
                    for (int q = 0; q < 12; ++q) Lcur[q] = Ln[q];
                prev_delta = is_delta(gval(W.mats, (size_t)x.mat).type);
                o = spawn(x.p, x.ng, x.wi);
                d = x.wi;
                ++b;
            }
        }
    }
    // flush the workgroup accumulators into the global FP64 accumulator
    __syncthreads();
    if (RULE && A.hyb_stats) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t t = wave_sum_u(n_br[k]);
            if (lane_id() == 0 && t) atomicAdd(&A.hyb_stats[k], (unsigned long long)t);
        }
    }
    flush_lds_grads(A, K);
}

#ifndef PPT_EXT_TU  // (non-template kernels and the host side: in the main compilation unit only)
// ============================================================================ P-RB comparator
// Polarized radiative backpropagation (the comparator of Sec. 5.1): the replay reads, for each vertex
// b1, an independent estimate of the suffix beyond it instead of the cached one.  Pass b1 traces,
// for every path with more than b1 vertices, a new path from the ray leaving vertex b1 (state S2,
// key prb_seed(seed, b1 + 1), vertex numbers continuing at b1 + 1) through the usual bounce kernels,
// and stores its radiance over the cached suffix in the vertex's record.
DEV uint64_t prb_seed(uint64_t seed, uint32_t v_first) { return seed + (uint64_t)v_first * 0x9E3779B97F4A7C15ull; }

// The ray leaving vertex b1 of each path: its prefix is replayed from the camera ray (its direction
// written by the fold) and the hit records, with the path's own key; the sub-path starts there with an identity
// throughput and no radiance.  Paths with b1 or fewer vertices start nothing.
__global__ void __launch_bounds__(BLOCK) k_prb_start(WArgs A, PathState S2, int b1) {
    const PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, nullptr};
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < A.n_chunk; i += gridDim.x * BLOCK) {
        const float4* R = ray_rec(S, i);
        const float4 r3 = R[3];
        const int info = __float_as_int(r3.x);
        const int B = (info & INFO_DEAD) ? 0 : (info & 255);
        const int view = info >> 12;
        float4* R2 = ray_rec(S2, i);
        if (B <= b1) {
            R2[3] = f4(__int_as_float(info_make(b1, false, view) | INFO_DEAD), r3.y, r3.z, r3.w);
            S2.hflag[i] = 2;
            continue;
        }
        const DevView V = gval(A.views, (size_t)view);
        const DevWorld W = world_of(A, V);
        const uint32_t pix = __float_as_uint(r3.y), smp = __float_as_uint(r3.z);
        // the camera ray: the view's origin and the direction the fold stored in the shadow record
        const float4 h0 = shd_rec(S, i)[0];
        v3 o = ld3(V.o), d = mk(h0.x, h0.y, h0.z);
        bool prev_delta = false;
        for (int b = 1; b <= b1; ++b) {
            const float4* C = cache_rec(S, Q, b - 1, i);
            const float4 c2 = C[2], c3 = C[3];
            const uint32_t hw = __float_as_uint(c2.w);
            Hit h;
            h.prim = (int)(hw & ((1u << 26) - 1));
            h.u = c3.x; h.t = c3.x; h.v = c3.y;
            Vtx x;
            surface(W, h, o, d, x);
            v3 so, sd;
            float stmax;
            vertex_setup<false>(W, K, V.view_id, A.seed, pix, smp, b, A.max_depth, A.flags, prev_delta, d, x, so, sd, stmax);
            prev_delta = is_delta(gval(W.mats, (size_t)x.mat).type);
            o = spawn(x.p, x.ng, x.wi);
            d = x.wi;
        }
        ray_set(R2, o, d);
        R2[2] = f4(0.0f, 0.0f, 0.0f, 0.0f);
        R2[3] = f4(__int_as_float(info_make(b1, prev_delta, view)), r3.y, r3.z, r3.w);
        float4* AC = acc_rec(S2, i);
        AC[0] = f4(1.0f, 0.0f, 0.0f, 0.0f); AC[1] = f4(0.0f, 1.0f, 0.0f, 0.0f);
        AC[2] = f4(0.0f, 0.0f, 1.0f, 0.0f); AC[3] = f4(0.0f, 0.0f, 0.0f, 1.0f);
        AC[4] = f4(1.0f, 1.0f, 1.0f, 0.0f);
        AC[5] = AC[6] = AC[7] = f4(0.0f, 0.0f, 0.0f, 0.0f);
        S2.hflag[i] = 0;
    }
}
// The sub-path radiance of pass b1 over the cached suffix beyond vertex b1.
__global__ void __launch_bounds__(BLOCK) k_prb_store(WArgs A, PathState S2, int b1) {
    const PathState& S = A.S;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < A.n_chunk; i += gridDim.x * BLOCK) {
        const int info = __float_as_int(ray_rec(S, i)[3].x);
        const int B = (info & INFO_DEAD) ? 0 : (info & 255);
        if (B <= b1) continue;
        float Lo[12];
        ld12(acc_rec(S2, i) + 5, Lo);
        st12(cache_rec(S, A.Q, b1 - 1, i) + 4, Lo);
    }
}

// ============================================================================ tape AD baseline: reverse sweep
// Conventional reverse-mode AD of the path loop (the "Conv. AD" the paper compares against, Sec. 5.1,
// 5.4): the forward pass stored every vertex's loop state on the tape (prefix throughput beta_b,
// weight W_b, emission E_b, hit and incoming ray); this kernel walks each path from its last vertex
// to its first, carrying the adjoint of the throughput as a full 4x4 matrix per channel, as a
// generic reverse sweep does (it does not know that the adjoint is an outer product):
//   Ebar_b = beta_b^T a0,   Wbar_b = beta_b^T betabar_{b+1},   betabar_b = a0 E_b^T + betabar_{b+1} W_b^T,
// with a0 the adjoint of the path's radiance at the sensor; each vertex's parameter derivatives
// come from its re-evaluated interaction with (Ebar_b, Wbar_b).  Scenes without the light-stage
// features only.
__global__ void __launch_bounds__(BLOCK) k_tape_reverse(WArgs A) {
    extern __shared__ double lds_grad[];
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, A.gacc};
    __shared__ CallTable tab;
    table_to_lds(&tab, A.table);
    K.tab = &tab;
    K.lds_d = lds_grad;
    K.lds_f = (float*)(lds_grad + A.lds_nd);
    for (int k = threadIdx.x; k < A.lds_nd; k += BLOCK) K.lds_d[k] = 0.0;
    for (int k = threadIdx.x; k < A.lds_nf; k += BLOCK) K.lds_f[k] = 0.0f;
    __syncthreads();
    const int n = S.counts[3];
    WaveFetch F(n);
    int slot = -1, b = 0, v = 0;
    uint32_t pix = 0, smp = 0;
    float a0[12], bbar[48];  // adjoint at the sensor; adjoint of beta_{b+1} per channel (4x4, row-major)
#pragma unroll
    for (int k = 0; k < 12; ++k) a0[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 48; ++k) bbar[k] = 0.0f;
    while (true) {
        const int idx = F.take(slot < 0, n, &S.counts[4]);
        if (idx >= 0) {
            slot = S.queue0[idx];
            const float4 r3 = ray_rec(S, slot)[3];
            const int info = __float_as_int(r3.x);
            b = info & 255;
            v = info >> 12;
            pix = __float_as_uint(r3.y);
            smp = __float_as_uint(r3.z);
            ld12(shd_rec(S, slot) + 2, a0);
#pragma unroll
            for (int k = 0; k < 48; ++k) bbar[k] = 0.0f;
        }
        if (!__any(slot >= 0)) break;
        if (slot >= 0) {
            const DevView V = gval(A.views, (size_t)v);
            const DevWorld W = world_of(A, V);
            const float4* T = tape_rec(S, Q, b - 1, slot);
            const float4 t0 = T[0], t1 = T[1], t2 = T[2], t3 = T[3], t12 = T[12], t13 = T[13], t14 = T[14];
            WC wt;
            wt.rgb[0] = t0.x; wt.rgb[1] = t0.y; wt.rgb[2] = t0.z;
            wt.A = t0.w; wt.B = t1.x; wt.C = t1.y; wt.D = t1.z;
            wt.ci = t1.w; wt.si = t2.x; wt.co = t2.y; wt.so = t2.z;
            const uint32_t hw = __float_as_uint(t2.w);
            wt.kind = (int)((hw >> 29) & 3);
            float E[12], M[16];
            ld12(T + 4, E);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 q = T[8 + k];
                M[4 * k] = q.x; M[4 * k + 1] = q.y; M[4 * k + 2] = q.z; M[4 * k + 3] = q.w;
            }
            const float brgb[3] = {t12.x, t12.y, t12.z};
            // Ebar_b = beta_b^T a0 and Wbar_b = beta_b^T betabar_{b+1}, per channel (beta_c = brgb_c M)
            float Eb[12], Wb[48];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float t = 0.0f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) t += M[4 * i + j] * a0[4 * c + i];
                    Eb[4 * c + j] = brgb[c] * t;
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        float u = 0.0f;
#pragma unroll
                        for (int i = 0; i < 4; ++i) u += M[4 * i + j] * bbar[16 * c + 4 * i + l];
                        Wb[16 * c + 4 * j + l] = brgb[c] * u;
                    }
                }
            // the interaction again, from the stored ray and hit
            Hit h;
            h.prim = (int)(hw & ((1u << 26) - 1));
            h.u = t3.x; h.t = t3.x; h.v = t3.y;
            const v3 o = mk(t13.x, t13.y, t13.z), d = mk(t13.w, t14.x, t14.y);
            Vtx x;
            surface(W, h, o, d, x);
            v3 so, sd;
            float stmax;
            vertex_setup<false>(W, K, V.view_id, A.seed, pix, smp, b, A.max_depth, A.flags, t12.w != 0.0f, d, x,
                                so, sd, stmax);
            if (x.nee == NEE_PENDING) x.nee = (int)((hw >> 26) & 7);
            WC w;
            float Ee[12], En[12];
            K.coherent = b == 1;
            eval_vertex<true, false, true>(W, K, x, w, Ee, En, Eb, Wb);
            // betabar_b = a0 E_b^T + betabar_{b+1} W_b^T (the stored weight)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float Wm[16];
                w_matrix(wt, c, Wm);
                float nb_[16];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float t = a0[4 * c + i] * E[4 * c + j];
#pragma unroll
                        for (int k = 0; k < 4; ++k) t += bbar[16 * c + 4 * i + k] * Wm[4 * j + k];
                        nb_[4 * i + j] = t;
                    }
#pragma unroll
                for (int k = 0; k < 16; ++k) bbar[16 * c + k] = nb_[k];
            }
            if (--b == 0) slot = -1;
        }
    }
    flush_lds_grads(A, K);
}

// ============================================================================ small kernels
__global__ void k_setup(CallTable tab, CallTable* dst, Stats* stats, int reset_stats) {
    int i = threadIdx.x;
    if (i < MAX_SLOTS) {
        dst->p[i] = tab.p[i];
        dst->goff[i] = tab.goff[i];
        dst->gout[i] = tab.gout[i];
        dst->numel[i] = tab.numel[i];
        dst->lds_d[i] = tab.lds_d[i];
        dst->lds_f[i] = tab.lds_f[i];
    }
    if (i < ST_COUNT && reset_stats) stats->c[i] = 0ull;
    if (i < 3 && reset_stats) stats->hyb[i] = 0ull;
}
__global__ void k_fill_f32(float* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}
__global__ void k_fill_f64(double* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
__global__ void k_finalize(const CallTable* tab, const double* gacc, int n_slots) {
    for (int s = 0; s < n_slots; ++s) {
        float* out = tab->gout[s];
        int64_t off = tab->goff[s], n = tab->numel[s];
        if (!out || off < 0) continue;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            out[i] = (float)gacc[off + i];
    }
}
__global__ void k_rng(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
    philox(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * i] = c0; out[4 * i + 1] = c1; out[4 * i + 2] = c2; out[4 * i + 3] = c3;
}

// ============================================================================ fixed scratch
// Device memory of the allocation-free backward entry point: the per-path records of one chunk and
// the FP64 gradient accumulators live here instead of in a caller workspace.  Each GPU the library
// runs on holds its own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device array: its device address is looked up once per device
// (hipGetSymbolAddress with that device current) and only that address is used afterwards.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** ptr) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidValue;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// ============================================================================ launchers
static uint64_t prb_seed_host(uint64_t seed, uint32_t v_first) { return seed + (uint64_t)v_first * 0x9E3779B97F4A7C15ull; }
static int blocks_for(int64_t n, int cap) {
    int64_t b = (n + BLOCK - 1) / BLOCK;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_setup(const CallTable& tab, CallTable* dst, Stats* stats, bool reset_stats, hipStream_t s) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(MAX_SLOTS), 0, s, tab, dst, stats, reset_stats ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n, 4096)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n, 4096)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_finalize(const CallTable* tab, const double* gacc, int n_slots, int64_t max_numel, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(max_numel, 2048)), dim3(BLOCK), 0, s, tab, gacc, n_slots);
    return hipGetLastError();
}
hipError_t launch_rng(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rng, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, ctr, out, n);
    return hipGetLastError();
}

// Workgroups of a grid-filling launch of kernel fn: as many per compute unit as its registers and
// its LDS (static + lds bytes) allow, and no more than the items need.
static int resident_grid(const void* fn, size_t lds, int64_t n, const LaunchGrid& G) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLOCK, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    return blocks_for(n, per_cu * G.cu);
}

// The variants for scenes with the light-stage features are compiled in their own unit
// (ppt_kernels_ext.hip) with FP32 division and square root correctly rounded: they differentiate
// the shading normal through the smooth dielectric's s/p rotators, which amplify rounding.
extern template __global__ void k_shade<0, true>(WArgs);
extern template __global__ void k_shade<1, true>(WArgs);
extern template __global__ void k_shade<2, true>(WArgs);
extern template __global__ void k_fold<true, true, false, false>(WArgs);
extern template __global__ void k_replay<false, true, false, false>(WArgs);
extern template __global__ void k_replay<true, true, false, false>(WArgs);
extern template __global__ void k_replay<true, true, true, false>(WArgs);
extern template __global__ void k_replay<false, true, false, true>(WArgs);

// A traversal launch, with or without the work counters.
template <int SMODE>
static void launch_extend(const WArgs& a, int grid, size_t lds, hipStream_t s) {
    if (a.stats) hipLaunchKernelGGL((k_extend<SMODE, true>), dim3(grid), dim3(BLOCK), lds, s, a);
    else hipLaunchKernelGGL((k_extend<SMODE, false>), dim3(grid), dim3(BLOCK), lds, s, a);
}

// One chunk of paths through every bounce.  mode 0: render, 1: backward.  M is told the family
// of every kernel before its launch (event timing).
hipError_t launch_chunk(WArgs a, int mode, const LaunchGrid& G, hipStream_t s, const LaunchMarker& M) {
    // the backward's rank-one replay start (cached replay; the comparators and the hybrid keep the
    // general record)
    a.r1adj = mode == 1 && a.r1 && a.ckpt == 0 && !a.pprb && !a.tape && !a.prb ? 1 : 0;
    if (mode != 0 || !a.S.nv) a.r1 = 0;  // (the rank-one record is the render's, with its vertex flags)
    size_t lds = (size_t)a.stack_cap * BLOCK * sizeof(int);
    M(KF_OTHER, s);
    hipLaunchKernelGGL(k_reset_counts, dim3(1), dim3(64), 0, s, a.S.counts);
    int gb = blocks_for(a.n_chunk, G.other);
    const int xg = blocks_for(a.n_chunk, a.stats ? G.extend_st : G.extend);
    a.qin = 0;
    a.first = 1;
    M(KF_EXTEND, s);
    launch_extend<-2>(a, xg, lds, s);  // (camera rays generated in the launch)
    for (int b = 1; b <= a.max_depth; ++b) {
        a.qin = (b - 1) & 1;
        a.first = b == 1;
        M(KF_COMPACT, s);
        if (mode == 0) hipLaunchKernelGGL(k_compact<0>, dim3(gb), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL(k_compact<1>, dim3(gb), dim3(BLOCK), 0, s, a);
        M(KF_SHADE, s);
        // (a grid sized to each variant's own occupancy measured slower for the render variant)
        const int sg = blocks_for(a.n_chunk, G.shade);
        if (mode == 0 && a.r1) {
            hipLaunchKernelGGL((k_shade<4, false>), dim3(sg), dim3(BLOCK), 0, s, a);
        } else if (mode == 1 && a.tape) {
            hipLaunchKernelGGL((k_shade<3, false>), dim3(sg), dim3(BLOCK), 0, s, a);
        } else if (a.ext) {
            if (mode == 0) hipLaunchKernelGGL((k_shade<0, true>), dim3(sg), dim3(BLOCK), 0, s, a);
            else if (a.ckpt > 0) hipLaunchKernelGGL((k_shade<2, true>), dim3(sg), dim3(BLOCK), 0, s, a);
            else hipLaunchKernelGGL((k_shade<1, true>), dim3(sg), dim3(BLOCK), 0, s, a);
        } else {
            if (mode == 0) hipLaunchKernelGGL((k_shade<0, false>), dim3(sg), dim3(BLOCK), 0, s, a);
            else if (a.ckpt > 0) hipLaunchKernelGGL((k_shade<2, false>), dim3(sg), dim3(BLOCK), 0, s, a);
            else hipLaunchKernelGGL((k_shade<1, false>), dim3(sg), dim3(BLOCK), 0, s, a);
        }
        // the rays of bounce b + 1 and the shadow rays of bounce b in one traversal launch (a
        // vertex at the maximum depth starts neither, so nothing follows the last bounce)
        if (b < a.max_depth) {
            a.qin = b & 1;
            a.first = 0;
            M(KF_EXTEND, s);
            if (mode == 0 && a.r1) launch_extend<4>(a, xg, lds, s);
            else if (mode == 0) launch_extend<0>(a, xg, lds, s);
            else if (a.tape) launch_extend<3>(a, xg, lds, s);
            else if (a.ckpt > 0) launch_extend<2>(a, xg, lds, s);
            else launch_extend<1>(a, xg, lds, s);
        }
    }
    if (mode == 0) {
        if (a.out) {
            M(KF_ACCUM, s);
            if (a.r1) hipLaunchKernelGGL(k_accum<true>, dim3(gb), dim3(BLOCK), 0, s, a);
            else hipLaunchKernelGGL(k_accum<false>, dim3(gb), dim3(BLOCK), 0, s, a);
        }
    } else {
        size_t glds = (size_t)a.lds_nd * sizeof(double) + (size_t)a.lds_nf * sizeof(float);
        M(KF_FOLD, s);
        // each fold workgroup takes one contiguous slice of the chunk, so the grid is the resident
        // one (a second, partial round of workgroups would leave most of the GPU idle)
        const void* fold_fn = a.ckpt > 0 ? (a.ext ? (const void*)k_fold<true, true> : (const void*)k_fold<true, false>)
                              : a.tape ? (const void*)k_fold<false, false, false, true>
                              : a.pprb ? (const void*)k_fold<false, false, true> : (const void*)k_fold<false, false>;
        const int fg = resident_grid(fold_fn, 0, a.n_chunk, G);
        if (a.tape) hipLaunchKernelGGL((k_fold<false, false, false, true>), dim3(fg), dim3(BLOCK), 0, s, a);
        else if (a.ckpt > 0 && a.ext) hipLaunchKernelGGL((k_fold<true, true>), dim3(fg), dim3(BLOCK), 0, s, a);
        else if (a.ckpt > 0) hipLaunchKernelGGL((k_fold<true, false>), dim3(fg), dim3(BLOCK), 0, s, a);
        else if (a.pprb) hipLaunchKernelGGL((k_fold<false, false, true>), dim3(fg), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL((k_fold<false, false>), dim3(fg), dim3(BLOCK), 0, s, a);
        if (a.prb) {  // P-RB: independent suffix estimates, one sub-path pass per vertex index
            WArgs b2 = a;
            b2.S = a.S2;
            b2.stats = nullptr;
            b2.sig = nullptr;
            b2.mask = nullptr;
            b2.out = nullptr;
            for (int b1 = 1; b1 < a.max_depth; ++b1) {
                M(KF_OTHER, s);
                hipLaunchKernelGGL(k_reset_counts, dim3(1), dim3(64), 0, s, b2.S.counts);
                hipLaunchKernelGGL(k_prb_start, dim3(gb), dim3(BLOCK), 0, s, a, a.S2, b1);
                b2.seed = prb_seed_host(a.seed, (uint32_t)(b1 + 1));
                b2.qin = 0;
                b2.first = 1;
                M(KF_EXTEND, s);
                launch_extend<-1>(b2, xg, lds, s);
                for (int bb = b1 + 1; bb <= a.max_depth; ++bb) {
                    const int it = bb - b1;
                    b2.qin = (it - 1) & 1;
                    b2.first = it == 1;
                    M(KF_COMPACT, s);
                    hipLaunchKernelGGL(k_compact<0>, dim3(gb), dim3(BLOCK), 0, s, b2);
                    M(KF_SHADE, s);
                    hipLaunchKernelGGL((k_shade<0, false>), dim3(blocks_for(a.n_chunk, G.shade)), dim3(BLOCK), 0, s, b2);
                    if (bb < a.max_depth) {
                        b2.qin = it & 1;
                        b2.first = 0;
                        M(KF_EXTEND, s);
                        launch_extend<0>(b2, xg, lds, s);
                    }
                }
                M(KF_OTHER, s);
                hipLaunchKernelGGL(k_prb_store, dim3(gb), dim3(BLOCK), 0, s, a, a.S2, b1);
            }
        }
        M(KF_REPLAY, s);
        // the persistent replay grid: as many workgroups per compute unit as this call's
        // accumulator size and the variant's registers allow
        if (a.tape) {  // the reverse sweep of the stored tape
            const int tg = resident_grid((const void*)k_tape_reverse, glds, a.n_chunk, G);
            hipLaunchKernelGGL(k_tape_reverse, dim3(tg), dim3(BLOCK), glds, s, a);
            return hipGetLastError();
        }
        const bool rule = a.ckpt > 0 && a.hyb_rule;
        const bool pprb = a.ckpt == 0 && a.pprb;
        const void* fn = a.ext ? (rule ? (const void*)k_replay<true, true, true>
                                       : pprb ? (const void*)k_replay<false, true, false, true>
                                       : a.ckpt > 0 ? (const void*)k_replay<true, true> : (const void*)k_replay<false, true>)
                               : (rule ? (const void*)k_replay<true, false, true>
                                       : pprb ? (const void*)k_replay<false, false, false, true>
                                       : a.ckpt > 0 ? (const void*)k_replay<true, false> : (const void*)k_replay<false, false>);
        const int rg = resident_grid(fn, glds, a.n_chunk, G);
        if (pprb) {
            if (a.ext) hipLaunchKernelGGL((k_replay<false, true, false, true>), dim3(rg), dim3(BLOCK), glds, s, a);
            else hipLaunchKernelGGL((k_replay<false, false, false, true>), dim3(rg), dim3(BLOCK), glds, s, a);
        } else if (a.ext) {
            if (rule) hipLaunchKernelGGL((k_replay<true, true, true>), dim3(rg), dim3(BLOCK), glds, s, a);
            else if (a.ckpt > 0) hipLaunchKernelGGL((k_replay<true, true>), dim3(rg), dim3(BLOCK), glds, s, a);
            else hipLaunchKernelGGL((k_replay<false, true>), dim3(rg), dim3(BLOCK), glds, s, a);
        } else {
            if (rule) hipLaunchKernelGGL((k_replay<true, false, true>), dim3(rg), dim3(BLOCK), glds, s, a);
            else if (a.ckpt > 0) hipLaunchKernelGGL((k_replay<true, false>), dim3(rg), dim3(BLOCK), glds, s, a);
            else hipLaunchKernelGGL((k_replay<false, false>), dim3(rg), dim3(BLOCK), glds, s, a);
        }
    }
    return hipGetLastError();
}

hipError_t occupancy_grid(int cu, int stack_cap, LaunchGrid* G) {
    int e = 0, sh = 0, ad = 0, ot = 0;
    size_t lds = (size_t)stack_cap * BLOCK * sizeof(int);
    hipError_t r;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&e, k_extend<1, false>, BLOCK, lds)) != hipSuccess) return r;
    int es = 0;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&es, k_extend<1, true>, BLOCK, lds)) != hipSuccess) return r;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&sh, k_shade<1, false>, BLOCK, 0)) != hipSuccess) return r;
    size_t glds = (size_t)LDS_GRAD_D * sizeof(double) + (size_t)LDS_GRAD_F * sizeof(float);
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ad, k_replay<false, false>, BLOCK, glds)) != hipSuccess) return r;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ot, k_compact<0>, BLOCK, 0)) != hipSuccess) return r;
    G->extend = (e > 0 ? e : 1) * cu;
    G->extend_st = (es > 0 ? es : 1) * cu;
    G->shade = (sh > 0 ? sh : 1) * cu;
    G->adjoint = (ad > 0 ? ad : 1) * cu;
    G->cu = cu;
    G->other = (ot > 0 ? ot : 1) * cu;
    return hipSuccess;
}

#endif  // PPT_EXT_TU
}  // namespace ppt
