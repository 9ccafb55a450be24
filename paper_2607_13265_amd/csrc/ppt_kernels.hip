// ppt_kernels.hip -- wavefront kernels of the differentiable polarized path tracer (gfx950).
//
// Paths are processed in chunks of a flat index space that spans every view of a plan (the
// batch): path g = (view, crop pixel, sample), samples fastest.  Per chunk and bounce:
//   k_extend   closest-hit traversal of the queued rays (lean kernel, LDS traversal stack),
//   k_shade    vertex sampling and Mueller weights; appends continuing paths to the next ray
//              queue and next-event rays to the shadow queue (wave-aggregated atomics),
//   k_shadow   any-hit traversal of the next-event rays.
// Render (Sec. 3.1, Eq. 2): the state carries the prefix Mueller product beta and the radiance
// sum; k_accum reduces the samples of each pixel.  Backward (Sec. 3.2, 4.3, Fig. 2): the primal
// pass caches, per vertex, the weight W_b, the emission + next-event Stokes E_b and a hit record;
// k_adjoint folds the cache into suffix radiance L[b] = E_b + W_b L[b+1] and replays the path
// forward from the hit records (no second traversal), differentiating each vertex against the
// cached L[b+1].  No Mueller matrix is inverted.
#include "ppt_device.h"

namespace ppt {

// ============================================================================ wave helpers
// Workgroup-aggregated counters: one global atomic per workgroup and counter.  Every thread of
// the workgroup must call it (it synchronizes the workgroup).
DEV void flush_stats(Stats* st, uint32_t nodes, uint32_t prims, uint32_t shadow, uint32_t verts, uint32_t paths) {
    if (!st) return;
    __shared__ uint32_t part[5];
    if (threadIdx.x < 5) part[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t v[5] = {wave_sum_u(nodes), wave_sum_u(prims), wave_sum_u(shadow), wave_sum_u(verts), wave_sum_u(paths)};
    if (lane_id() == 0)
        for (int k = 0; k < 5; ++k)
            if (v[k]) atomicAdd(&part[k], v[k]);
    __syncthreads();
    if (threadIdx.x < 5 && part[threadIdx.x]) {
        unsigned long long* dst[5] = {&st->nodes, &st->prims, &st->shadow_rays, &st->vertices, &st->paths};
        atomicAdd(dst[threadIdx.x], (unsigned long long)part[threadIdx.x]);
    }
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

// view of a global path index (views are few; binary search over their path offsets)
DEV int find_view(const DevView* views, int n_views, int64_t g) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].path_off <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}
struct PathId { int v, px, py, lx, ly; uint32_t smp, pix; };
DEV PathId path_id(const DevView* views, int n_views, int64_t g) {
    PathId r;
    r.v = find_view(views, n_views, g);
    const DevView& V = views[r.v];
    int64_t local = g - V.path_off;
    int64_t pl = local / V.spp;
    r.smp = (uint32_t)(local - pl * V.spp);
    r.lx = (int)(pl % V.crop_w);
    r.ly = (int)(pl / V.crop_w);
    r.px = V.crop_x0 + r.lx;
    r.py = V.crop_y0 + r.ly;
    r.pix = (uint32_t)(r.py * V.width + r.px);
    return r;
}

// SoA accessors
DEV v3 ld_v3(const float* a, int Q, int i) { return mk(a[i], a[Q + i], a[2 * Q + i]); }
DEV void st_v3(float* a, int Q, int i, v3 v) { a[i] = v.x; a[Q + i] = v.y; a[2 * Q + i] = v.z; }

constexpr int INFO_DEAD = 1 << 9;
DEV int info_make(int nverts, bool prev_delta, int view) { return nverts | (prev_delta ? 256 : 0) | (view << 12); }

// ============================================================================ chunk start
__global__ void k_reset_counts(int* counts) {
    if (threadIdx.x < 4) counts[threadIdx.x] = 0;
}

// Camera rays of the chunk's paths (masked paths are marked and skipped by the first bounce).
__global__ void __launch_bounds__(BLOCK) k_gen(WArgs A) {
    PathState& S = A.S;
    const int Q = A.Q;
    uint32_t npaths = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < A.n_chunk; i += gridDim.x * BLOCK) {
        int64_t g = A.g0 + i;
        PathId id = path_id(A.views, A.n_views, g);
        const DevView& V = A.views[id.v];
        bool live = !(A.mask && !A.mask[g]);
        v3 o, d;
        camera_ray(V, id.px, id.py, id.smp, A.seed, o, d);
        st_v3(S.ro, Q, i, o);
        st_v3(S.rd, Q, i, d);
        S.info[i] = info_make(0, false, id.v) | (live ? 0 : INFO_DEAD);
        S.pix[i] = id.pix;
        S.smp[i] = id.smp;
        if (A.sig) A.sig[g] = live ? 1469598103934665603ull : 0ull;
        if (live) ++npaths;
    }
    flush_stats(A.stats, 0, 0, 0, 0, npaths);
}

// ============================================================================ traversal kernels
__global__ void __launch_bounds__(BLOCK) k_extend(WArgs A) {
    extern __shared__ int lds_stack[];
    int* stack = lds_stack + threadIdx.x;
    PathState& S = A.S;
    const int Q = A.Q;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the queues the following shade kernel appends to
        S.counts[1 - A.qin] = 0;
        S.counts[2] = 0;
    }
    const int* q = A.qin ? S.queue1 : S.queue0;
    const int n = A.first ? A.n_chunk : S.counts[A.qin];
    uint32_t nodes = 0, prims = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        int slot = A.first ? i : q[i];
        int info = S.info[slot];
        if (info & INFO_DEAD) continue;
        int v = info >> 12;
        const DevWorld& W = A.worlds[A.views[v].world];
        Hit h;
        trace<false>(W, ld_v3(S.ro, Q, slot), ld_v3(S.rd, Q, slot), 3.0e38f, h, nodes, prims, stack);
        S.hprim[slot] = h.prim;
        S.ht[slot] = h.t; S.hu[slot] = h.u; S.hv[slot] = h.v;
    }
    flush_stats(A.stats, nodes, prims, 0, 0, 0);
}

template <int MODE>
__global__ void __launch_bounds__(BLOCK) k_shadow(WArgs A) {
    extern __shared__ int lds_stack[];
    int* stack = lds_stack + threadIdx.x;
    PathState& S = A.S;
    const int Q = A.Q;
    const int n = S.counts[2];
    uint32_t nodes = 0, prims = 0, rays = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        int slot = S.squeue[i];
        int info = S.info[slot];
        const DevWorld& W = A.worlds[A.views[info >> 12].world];
        Hit h;
        ++rays;
        bool occ = trace<true>(W, ld_v3(S.so, Q, slot), ld_v3(S.sd, Q, slot), S.stmax[slot], h, nodes, prims, stack);
        if (MODE == 0) {
            if (!occ)
#pragma unroll
                for (int k = 0; k < 12; ++k) S.Lo[k * Q + slot] += S.pend[k * Q + slot];
        } else {
            int b = (info & 255) - 1;  // the vertex whose light sample this is
            float* C = S.cache + (size_t)b * CACHE_WORDS * Q;
            if (!occ)
#pragma unroll
                for (int k = 0; k < 12; ++k) C[(CW_E + k) * Q + slot] += S.pend[k * Q + slot];
            uint32_t hw = (uint32_t)__float_as_int(C[CW_HIT * Q + slot]);
            hw = (hw & ~(7u << 26)) | ((uint32_t)(occ ? NEE_OCCLUDED : NEE_VISIBLE) << 26);
            C[CW_HIT * Q + slot] = __int_as_float((int)hw);
        }
        if (A.sig) sig_add(A.sig[A.g0 + slot], (uint32_t)(occ ? NEE_OCCLUDED : NEE_VISIBLE));
    }
    flush_stats(A.stats, nodes, prims, rays, 0, 0);
}

// ============================================================================ shading
template <int MODE>
__global__ void __launch_bounds__(BLOCK) k_shade(WArgs A) {
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, nullptr};
    const int* qin = A.qin ? S.queue1 : S.queue0;
    int* qout = A.qin ? S.queue0 : S.queue1;
    const int n = A.first ? A.n_chunk : S.counts[A.qin];
    __shared__ BlockQueue qn, qs;
    if (threadIdx.x == 0) { qn.n = 0; qs.n = 0; }
    __syncthreads();
    uint32_t nverts = 0;
    for (int bb = blockIdx.x * BLOCK; bb < n; bb += gridDim.x * BLOCK) {
        int i = bb + threadIdx.x;
        bool cont = false, shadow = false;
        int slot = 0;
        if (i < n) slot = A.first ? i : qin[i];
        if (i < n && !(S.info[slot] & INFO_DEAD)) {
            int info = S.info[slot];
            int nb = info & 255, v = info >> 12;
            bool prev_delta = (info >> 8) & 1;
            int64_t g = A.g0 + slot;
            const uint32_t pix = S.pix[slot], smp = S.smp[slot];
            const DevView& V = A.views[v];
            const DevWorld& W = A.worlds[V.world];
            Hit h;
            h.prim = S.hprim[slot];
            h.t = S.ht[slot]; h.u = S.hu[slot]; h.v = S.hv[slot];
            v3 o = ld_v3(S.ro, Q, slot), d = ld_v3(S.rd, Q, slot);
            if (h.prim < 0) {
                if (A.sig) sig_add(A.sig[g], 0xffffffffu);
                if (MODE == 0 && nb == 0)
#pragma unroll
                    for (int k = 0; k < 12; ++k) S.Lo[k * Q + slot] = 0.0f;
            } else {
                int b = nb + 1;
                ++nverts;
                Vtx x;
                surface(W, h, o, d, x);
                v3 so, sd;
                float stmax = 0.0f;
                vertex_setup(W, K, V, A.seed, pix, smp, b, A.max_depth, A.flags, prev_delta, d, x, so, sd, stmax);
                if (A.sig) {
                    uint64_t sg = A.sig[g];
                    sig_add(sg, (uint32_t)x.orig);
                    sig_add(sg, (uint32_t)x.lobe);
                    if (x.nee != NEE_PENDING) sig_add(sg, (uint32_t)x.nee);
                    A.sig[g] = sg;
                }
                WC w;
                float Ee[12], En[12];
                eval_vertex<false>(W, K, x, w, Ee, En, nullptr, nullptr);
                cont = x.lobe != LOBE_NONE && x.lobe != LOBE_INVALID;
                shadow = x.nee == NEE_PENDING;
                if (MODE == 0) {
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
                        for (int k = 0; k < 16; ++k) beta[k] = S.beta[k * Q + slot];
#pragma unroll
                        for (int c = 0; c < 3; ++c) brgb[c] = S.beta[(16 + c) * Q + slot];
#pragma unroll
                        for (int k = 0; k < 12; ++k) Lo[k] = S.Lo[k * Q + slot];
                    }
                    // Lo_c += brgb_c beta Ee_c; the pending next-event part likewise
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float se = beta[4 * r] * Ee[4 * c] + beta[4 * r + 1] * Ee[4 * c + 1] +
                                       beta[4 * r + 2] * Ee[4 * c + 2] + beta[4 * r + 3] * Ee[4 * c + 3];
                            Lo[4 * c + r] += brgb[c] * se;
                            if (shadow) {
                                float sn = beta[4 * r] * En[4 * c] + beta[4 * r + 1] * En[4 * c + 1] +
                                           beta[4 * r + 2] * En[4 * c + 2] + beta[4 * r + 3] * En[4 * c + 3];
                                S.pend[(4 * c + r) * Q + slot] = brgb[c] * sn;
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 12; ++k) S.Lo[k * Q + slot] = Lo[k];
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
                        for (int k = 0; k < 16; ++k) S.beta[k * Q + slot] = beta[k];
#pragma unroll
                        for (int c = 0; c < 3; ++c) S.beta[(16 + c) * Q + slot] = brgb[c] * w.rgb[c];
                    }
                } else {
                    float* C = S.cache + (size_t)(b - 1) * CACHE_WORDS * Q;
                    C[0 * Q + slot] = w.rgb[0]; C[1 * Q + slot] = w.rgb[1]; C[2 * Q + slot] = w.rgb[2];
                    C[3 * Q + slot] = w.A; C[4 * Q + slot] = w.B; C[5 * Q + slot] = w.C; C[6 * Q + slot] = w.D;
                    C[7 * Q + slot] = w.ci; C[8 * Q + slot] = w.si; C[9 * Q + slot] = w.co; C[10 * Q + slot] = w.so;
#pragma unroll
                    for (int k = 0; k < 12; ++k) C[(CW_E + k) * Q + slot] = Ee[k];
                    if (shadow)
#pragma unroll
                        for (int k = 0; k < 12; ++k) S.pend[k * Q + slot] = En[k];
                    bool sphere = __float_as_int(W.prims[3 * h.prim + 1].w) != 0;
                    C[CW_HIT * Q + slot] = __int_as_float(h.prim | (x.nee << 26) | (w.kind << 29));
                    C[(CW_HIT + 1) * Q + slot] = sphere ? h.t : h.u;
                    C[(CW_HIT + 2) * Q + slot] = h.v;
                }
                if (shadow) {
                    st_v3(S.so, Q, slot, so);
                    st_v3(S.sd, Q, slot, sd);
                    S.stmax[slot] = stmax;
                }
                if (cont) {
                    st_v3(S.ro, Q, slot, spawn(x.p, x.ng, x.wi));
                    st_v3(S.rd, Q, slot, x.wi);
                }
                S.info[slot] = info_make(b, is_delta(W.mats[x.mat].type), v);
            }
        }
        bq_push(qn, cont, slot);
        bq_push(qs, shadow, slot);
        bq_flush(qn, &S.counts[1 - A.qin], qout, false);
        bq_flush(qs, &S.counts[2], S.squeue, false);
    }
    bq_flush(qn, &S.counts[1 - A.qin], qout, true);
    bq_flush(qs, &S.counts[2], S.squeue, true);
    flush_stats(A.stats, 0, 0, 0, nverts, 0);
}

// ============================================================================ render: pixel reduction
// Every lane rotates its path's radiance into the sensor frame; the lanes of one pixel (adjacent,
// samples fastest) are summed by a segmented wavefront scan, and the last lane of each segment
// applies the analyzers and adds the mean to the image.  A pixel whose samples span two
// wavefronts or chunks receives several additions.
__global__ void __launch_bounds__(BLOCK) k_accum(WArgs A) {
    if (!A.out) return;  // signature-only runs produce no image
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, nullptr};
    const int lane = lane_id();
    for (int base = blockIdx.x * BLOCK + (threadIdx.x & ~(WAVE - 1)); base < A.n_chunk; base += gridDim.x * BLOCK) {
        int i = base + lane;
        bool valid = i < A.n_chunk;
        int64_t key = -1 - lane;  // distinct per invalid lane
        float acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = 0.0f;
        PathId id{};
        if (valid) {
            int64_t g = A.g0 + i;
            id = path_id(A.views, A.n_views, g);
            key = g - id.smp;
            if (!(S.info[i] & INFO_DEAD)) {
                const DevView& V = A.views[id.v];
                v3 o, d;
                camera_ray(V, id.px, id.py, id.smp, A.seed, o, d);
                v3 kc = -d;
                float Cs, Ss;
                rot_cs(kc, canon_x(kc), normalize(ld3(V.r) - kc * dot(ld3(V.r), kc)), Cs, Ss);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float l1 = S.Lo[(4 * c + 1) * Q + i], l2 = S.Lo[(4 * c + 2) * Q + i];
                    acc[4 * c] = S.Lo[(4 * c) * Q + i];
                    acc[4 * c + 1] = Cs * l1 + Ss * l2;
                    acc[4 * c + 2] = -Ss * l1 + Cs * l2;
                    acc[4 * c + 3] = S.Lo[(4 * c + 3) * Q + i];
                }
            }
        }
        // inclusive segmented scan toward higher lanes
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            int64_t kup = __shfl_up(key, off, WAVE);
            bool take = lane >= off && kup == key;
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                float v = __shfl_up(acc[k], off, WAVE);
                if (take) acc[k] += v;
            }
        }
        int64_t knext = __shfl_down(key, 1, WAVE);
        bool tail = valid && (lane == WAVE - 1 || knext != key);
        if (tail) {
            const DevView& V = A.views[id.v];
            float theta = V.sensor == SENSOR_POLARIZER ? K.p(V.theta_slot, V.theta_off) : 0.0f;
            float inv = 1.0f / (float)V.spp;
            int64_t astride = (int64_t)V.crop_w * V.crop_h * 12;
            int64_t ob = V.out_off + ((int64_t)id.ly * V.crop_w + id.lx) * 12;
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

// ============================================================================ backward: fold + replay
__global__ void __launch_bounds__(BLOCK) k_adjoint(WArgs A) {
    extern __shared__ double lds_grad[];
    PathState& S = A.S;
    const int Q = A.Q;
    Call K{A.table, A.gacc};
    K.lds_d = lds_grad;
    K.lds_f = (float*)(lds_grad + A.lds_nd);
    for (int k = threadIdx.x; k < A.lds_nd; k += BLOCK) K.lds_d[k] = 0.0;
    for (int k = threadIdx.x; k < A.lds_nf; k += BLOCK) K.lds_f[k] = 0.0f;
    __syncthreads();
    for (int base = blockIdx.x * BLOCK + (threadIdx.x & ~(WAVE - 1)); base < A.n_chunk; base += gridDim.x * BLOCK) {
        int i = base + lane_id();
        float gtheta = 0.0f;
        int tkey = -1;
        if (i < A.n_chunk && !(S.info[i] & INFO_DEAD)) {
            int64_t g = A.g0 + i;
            PathId id = path_id(A.views, A.n_views, g);
            const DevView& V = A.views[id.v];
            const DevWorld& W = A.worlds[V.world];
            const int B = S.info[i] & 255;
            float theta = V.sensor == SENSOR_POLARIZER ? K.p(V.theta_slot, V.theta_off) : 0.0f;
            // adjoint of the pixel mean in the sensor frame: a_sens_c = sum_a delta_a,c^T A_a / spp
            float asens[12], dl[12];
            float inv = 1.0f / (float)V.spp;
            int64_t astride = (int64_t)V.crop_w * V.crop_h * 12;
            int64_t ob = V.out_off + ((int64_t)id.ly * V.crop_w + id.lx) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) asens[k] = 0.0f;
            for (int a = 0; a < V.n_analyzers; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float d4[4], r4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) d4[k] = A.dout[ob + a * astride + 4 * c + k] * inv;
                    if (a == 0) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) dl[4 * c + k] = d4[k];
                    }
                    analyzer_row(V.sensor, theta, a, d4, r4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) asens[4 * c + k] += r4[k];
                }
            v3 o, d;
            camera_ray(V, id.px, id.py, id.smp, A.seed, o, d);
            v3 kc = -d;
            float Cs, Ss;
            rot_cs(kc, canon_x(kc), normalize(ld3(V.r) - kc * dot(ld3(V.r), kc)), Cs, Ss);
            // ---- backward fold over the cache: L[b] = E_b + W_b L[b+1], written over E_b
            float L[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) L[k] = 0.0f;
            for (int b = B - 1; b >= 0; --b) {
                float* C = S.cache + (size_t)b * CACHE_WORDS * Q;
                WC w;
                w.rgb[0] = C[0 * Q + i]; w.rgb[1] = C[1 * Q + i]; w.rgb[2] = C[2 * Q + i];
                w.A = C[3 * Q + i]; w.B = C[4 * Q + i]; w.C = C[5 * Q + i]; w.D = C[6 * Q + i];
                w.ci = C[7 * Q + i]; w.si = C[8 * Q + i]; w.co = C[9 * Q + i]; w.so = C[10 * Q + i];
                w.kind = (__float_as_int(C[CW_HIT * Q + i]) >> 29) & 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float o4[4];
                    w_apply(w, c, L + 4 * c, o4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        L[4 * c + k] = C[(CW_E + 4 * c + k) * Q + i] + o4[k];
                        C[(CW_E + 4 * c + k) * Q + i] = L[4 * c + k];
                    }
                }
            }
            // polarizer-angle term: delta^T (dP/dtheta) R_s L[1]
            if (V.sensor == SENSOR_POLARIZER) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float l1 = L[4 * c + 1], l2 = L[4 * c + 2];
                    float ls[4] = {L[4 * c], Cs * l1 + Ss * l2, -Ss * l1 + Cs * l2, L[4 * c + 3]};
                    gtheta += polarizer_dtheta(theta, dl + 4 * c, ls);
                }
                tkey = id.v;
            }
            // ---- replay from the hit records: a_c = a_sens_c R_s, then vertex by vertex
            float av[12];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float a1 = asens[4 * c + 1], a2 = asens[4 * c + 2];
                av[4 * c] = asens[4 * c];
                av[4 * c + 1] = Cs * a1 - Ss * a2;
                av[4 * c + 2] = Ss * a1 + Cs * a2;
                av[4 * c + 3] = asens[4 * c + 3];
            }
            bool prev_delta = false;
            for (int b = 1; b <= B; ++b) {
                const float* C = S.cache + (size_t)(b - 1) * CACHE_WORDS * Q;
                uint32_t hw = (uint32_t)__float_as_int(C[CW_HIT * Q + i]);
                Hit h;
                h.prim = (int)(hw & ((1u << 26) - 1));
                int rec_nee = (int)((hw >> 26) & 7);
                float hu = C[(CW_HIT + 1) * Q + i];
                h.u = hu; h.t = hu; h.v = C[(CW_HIT + 2) * Q + i];
                Vtx x;
                surface(W, h, o, d, x);
                v3 so, sd;
                float stmax;
                vertex_setup(W, K, V, A.seed, id.pix, id.smp, b, A.max_depth, A.flags, prev_delta, d, x, so, sd, stmax);
                if (x.nee == NEE_PENDING) x.nee = rec_nee;
                float Ln[12];
                if (b < B) {
                    const float* Cn = S.cache + (size_t)b * CACHE_WORDS * Q;
#pragma unroll
                    for (int k = 0; k < 12; ++k) Ln[k] = Cn[(CW_E + k) * Q + i];
                } else {
#pragma unroll
                    for (int k = 0; k < 12; ++k) Ln[k] = 0.0f;
                }
                WC w;
                float Ee[12], En[12];
                eval_vertex<true>(W, K, x, w, Ee, En, av, Ln);
                if (x.lobe == LOBE_NONE || x.lobe == LOBE_INVALID) break;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float o4[4];
                    w_row(w, c, av + 4 * c, o4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) av[4 * c + k] = o4[k];
                }
                prev_delta = is_delta(W.mats[x.mat].type);
                o = spawn(x.p, x.ng, x.wi);
                d = x.wi;
            }
        }
        // polarizer angles: one atomic per distinct view in the wavefront
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
    // flush the workgroup accumulators into the global FP64 accumulator
    __syncthreads();
    const CallTable* T = A.table;
    for (int s = 0; s < MAX_SLOTS; ++s) {
        int od = T->lds_d[s], of = T->lds_f[s];
        if (od < 0 && of < 0) continue;
        int64_t go = T->goff[s], n = T->numel[s];
        for (int64_t k = threadIdx.x; k < n; k += BLOCK) {
            double v = od >= 0 ? K.lds_d[od + k] : (double)K.lds_f[of + k];
            if (v != 0.0) unsafeAtomicAdd(A.gacc + go + k, v);
        }
    }
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
    if (i == 0 && reset_stats) stats->vertices = stats->paths = stats->nodes = stats->prims = stats->shadow_rays = 0ull;
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

// ============================================================================ launchers
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

// One chunk of paths through every bounce.  mode 0: render, 1: backward.
hipError_t launch_chunk(WArgs a, int mode, const LaunchGrid& G, hipStream_t s) {
    size_t lds = (size_t)a.stack_cap * BLOCK * sizeof(int);
    hipLaunchKernelGGL(k_reset_counts, dim3(1), dim3(64), 0, s, a.S.counts);
    int gb = blocks_for(a.n_chunk, G.other);
    hipLaunchKernelGGL(k_gen, dim3(gb), dim3(BLOCK), 0, s, a);
    for (int b = 1; b <= a.max_depth; ++b) {
        a.qin = (b - 1) & 1;
        a.first = b == 1;
        hipLaunchKernelGGL(k_extend, dim3(blocks_for(a.n_chunk, G.extend)), dim3(BLOCK), lds, s, a);
        if (mode == 0) {
            hipLaunchKernelGGL(k_shade<0>, dim3(blocks_for(a.n_chunk, G.shade)), dim3(BLOCK), 0, s, a);
            hipLaunchKernelGGL(k_shadow<0>, dim3(blocks_for(a.n_chunk, G.extend)), dim3(BLOCK), lds, s, a);
        } else {
            hipLaunchKernelGGL(k_shade<1>, dim3(blocks_for(a.n_chunk, G.shade)), dim3(BLOCK), 0, s, a);
            hipLaunchKernelGGL(k_shadow<1>, dim3(blocks_for(a.n_chunk, G.extend)), dim3(BLOCK), lds, s, a);
        }
    }
    if (mode == 0) {
        if (a.out) hipLaunchKernelGGL(k_accum, dim3(gb), dim3(BLOCK), 0, s, a);
    } else {
        size_t glds = (size_t)a.lds_nd * sizeof(double) + (size_t)a.lds_nf * sizeof(float);
        hipLaunchKernelGGL(k_adjoint, dim3(blocks_for(a.n_chunk, G.adjoint)), dim3(BLOCK), glds, s, a);
    }
    return hipGetLastError();
}

hipError_t occupancy_grid(int cu, int stack_cap, LaunchGrid* G) {
    int e = 0, sh = 0, ad = 0, ot = 0;
    size_t lds = (size_t)stack_cap * BLOCK * sizeof(int);
    hipError_t r;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&e, k_extend, BLOCK, lds)) != hipSuccess) return r;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&sh, k_shade<1>, BLOCK, 0)) != hipSuccess) return r;
    size_t glds = (size_t)LDS_GRAD_D * sizeof(double) + (size_t)LDS_GRAD_F * sizeof(float);
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ad, k_adjoint, BLOCK, glds)) != hipSuccess) return r;
    if ((r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ot, k_gen, BLOCK, 0)) != hipSuccess) return r;
    G->extend = (e > 0 ? e : 1) * cu;
    G->shade = (sh > 0 ? sh : 1) * cu;
    G->adjoint = (ad > 0 ? ad : 1) * cu;
    G->other = (ot > 0 ? ot : 1) * cu;
    return hipSuccess;
}

}  // namespace ppt
