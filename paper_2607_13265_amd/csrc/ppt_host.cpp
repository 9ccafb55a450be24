// ppt_host.cpp -- host side of the C ABI: scene blob parsing and validation, binned-SAH BVH
// construction (flattened to the two-box node layout the traversal kernel reads), plan
// creation (views and chunking of the path index space), workspace layout and the launch sequence.
#include "ppt_internal.h"
#include "ppt_half.h"
#include "../../include/ppt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace ppt {
hipError_t launch_setup(const CallTable& tab, CallTable* dst, Stats* stats, bool reset_stats, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s);
hipError_t launch_finalize(const CallTable* tab, const double* gacc, int n_slots, int64_t max_numel, hipStream_t s);
hipError_t launch_rng(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_chunk(WArgs a, int mode, const LaunchGrid& G, hipStream_t s, const LaunchMarker& M);
hipError_t occupancy_grid(int cu, int stack_cap, LaunchGrid* G);
hipError_t noalloc_scratch(void** ptr);
}  // namespace ppt

using namespace ppt;

// ============================================================================ errors
static thread_local std::string g_err;
static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
#define HIP_TRY(expr, what)                                                                          \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(PPT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ============================================================================ device buffers
struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    ~DevBuf() { if (p) (void)hipFree(p); }
    int upload(const void* src, size_t bytes, const char* what) {
        n = bytes;
        if (bytes == 0) return PPT_OK;
        if (hipMalloc(&p, bytes) != hipSuccess) { p = nullptr; return fail(PPT_ENOMEM, std::string("hipMalloc ") + what); }
        HIP_TRY(hipMemcpy(p, src, bytes, hipMemcpyHostToDevice), what);
        return PPT_OK;
    }
};

// ============================================================================ blob records
struct BlobMaterial {
    uint32_t type;
    int32_t alb_slot; uint32_t alb_off, alb_tw, alb_th;
    int32_t alpha_slot; uint32_t alpha_off, alpha_tw, alpha_th;
    int32_t eta_slot; uint32_t eta_off;
    int32_t kap_slot; uint32_t kap_off;
    int32_t emit_slot; uint32_t emit_off;
    float axis[3]; float blend;
    float emit_circ;
    int32_t spec_slot; uint32_t spec_off, spec_tw, spec_th;
    int32_t nrm_slot; uint32_t nrm_off, nrm_tw, nrm_th;
    uint32_t reserved[4];
};
static_assert(sizeof(BlobMaterial) == 128, "material record");
struct BlobLight { float p0[3], eu[3], ev[3]; int32_t le_slot; uint32_t le_off; float circ; };
static_assert(sizeof(BlobLight) == 48, "light record");
static_assert(sizeof(ppt_view) == 88, "view record");

// ============================================================================ BVH (binned SAH)
// Box bounds as IEEE half floats rounded outward (ppt_half.h).
static float half_pair(float lo, float hi) {   // (rounded-down lo, rounded-up hi) in one word
    const uint32_t w = (uint32_t)half_down(lo) | ((uint32_t)half_up(hi) << 16);
    float f;
    std::memcpy(&f, &w, 4);
    return f;
}
struct BPrim { float lo[3], hi[3], c[3]; };
struct BNode { float lo[3], hi[3]; int left, right, first, count; };

struct Builder {
    static constexpr int NB = 32;          // SAH bins per axis (16 measured 1% more node visits)
    static constexpr float C_TRAV = 0.5f;  // cost of a node visit relative to a primitive test
    static constexpr int MAX_LEAF = 8;     // primitives per leaf (the leaf reference holds count - 1 in 3 bits)
    static constexpr int SWEEP_MAX = 512;  // nodes up to this size: exact SAH sweep instead of bins
    std::vector<BPrim> prims;
    std::vector<int> idx;
    std::vector<BNode> nodes;
    int max_depth = 0;

    static float area(const float lo[3], const float hi[3]) {
        float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        if (dx < 0 || dy < 0 || dz < 0) return 0.0f;
        return 2.0f * (dx * dy + dy * dz + dz * dx);
    }
    int build(int first, int count, int depth) {
        max_depth = std::max(max_depth, depth);
        BNode n;
        float clo[3] = {1e30f, 1e30f, 1e30f}, chi[3] = {-1e30f, -1e30f, -1e30f};
        for (int a = 0; a < 3; ++a) { n.lo[a] = 1e30f; n.hi[a] = -1e30f; }
        for (int i = first; i < first + count; ++i) {
            const BPrim& p = prims[idx[i]];
            for (int a = 0; a < 3; ++a) {
                n.lo[a] = std::min(n.lo[a], p.lo[a]); n.hi[a] = std::max(n.hi[a], p.hi[a]);
                clo[a] = std::min(clo[a], p.c[a]); chi[a] = std::max(chi[a], p.c[a]);
            }
        }
        int id = (int)nodes.size();
        nodes.push_back(n);
        nodes[id].left = nodes[id].right = -1;
        nodes[id].first = first; nodes[id].count = count;
        if (count <= 2) return id;
        float leaf_cost0 = area(n.lo, n.hi) * count;
        if (count <= SWEEP_MAX) {  // small nodes: every split of the centroid order on each axis
            float bc_cost = 1e30f;
            int bc_axis = -1, bc_at = -1;
            std::vector<int> ord(idx.begin() + first, idx.begin() + first + count);
            std::vector<float> racc((size_t)count);
            for (int a = 0; a < 3; ++a) {
                std::sort(ord.begin(), ord.end(), [&](int p, int q) {
                    return prims[p].c[a] < prims[q].c[a] || (prims[p].c[a] == prims[q].c[a] && p < q);
                });
                float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
                for (int i = count - 1; i >= 1; --i) {
                    const BPrim& p = prims[ord[i]];
                    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p.lo[k]); hi[k] = std::max(hi[k], p.hi[k]); }
                    racc[i] = area(lo, hi) * (count - i);
                }
                for (int k = 0; k < 3; ++k) { lo[k] = 1e30f; hi[k] = -1e30f; }
                for (int i = 0; i < count - 1; ++i) {
                    const BPrim& p = prims[ord[i]];
                    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p.lo[k]); hi[k] = std::max(hi[k], p.hi[k]); }
                    const float cost = area(lo, hi) * (i + 1) + racc[i + 1];
                    if (cost < bc_cost) { bc_cost = cost; bc_axis = a; bc_at = i + 1; }
                }
            }
            const float split_cost0 = bc_axis >= 0 ? C_TRAV * area(n.lo, n.hi) + bc_cost : 1e30f;
            if (count <= MAX_LEAF && leaf_cost0 <= split_cost0) return id;
            if (bc_axis >= 0) {
                const int a = bc_axis;
                std::sort(idx.begin() + first, idx.begin() + first + count, [&](int p, int q) {
                    return prims[p].c[a] < prims[q].c[a] || (prims[p].c[a] == prims[q].c[a] && p < q);
                });
                const int mid = first + bc_at;
                int l = build(first, mid - first, depth + 1);
                int r = build(mid, first + count - mid, depth + 1);
                nodes[id].left = l; nodes[id].right = r; nodes[id].count = 0;
                return id;
            }
        }
        // binned SAH over the three axes
        float best_cost = 1e30f;
        int best_axis = -1, best_bin = -1;
        for (int a = 0; a < 3; ++a) {
            float ext = chi[a] - clo[a];
            if (!(ext > 0.0f)) continue;
            float blo[NB][3], bhi[NB][3];
            int bc[NB] = {0};
            for (int b = 0; b < NB; ++b)
                for (int k = 0; k < 3; ++k) { blo[b][k] = 1e30f; bhi[b][k] = -1e30f; }
            float sc = NB / ext;
            for (int i = first; i < first + count; ++i) {
                const BPrim& p = prims[idx[i]];
                int b = std::min(NB - 1, (int)((p.c[a] - clo[a]) * sc));
                bc[b]++;
                for (int k = 0; k < 3; ++k) { blo[b][k] = std::min(blo[b][k], p.lo[k]); bhi[b][k] = std::max(bhi[b][k], p.hi[k]); }
            }
            float rlo[NB][3], rhi[NB][3];
            int rc[NB];
            float alo[3] = {1e30f, 1e30f, 1e30f}, ahi[3] = {-1e30f, -1e30f, -1e30f};
            int acount = 0;
            for (int b = NB - 1; b >= 1; --b) {
                for (int k = 0; k < 3; ++k) { alo[k] = std::min(alo[k], blo[b][k]); ahi[k] = std::max(ahi[k], bhi[b][k]); }
                acount += bc[b];
                for (int k = 0; k < 3; ++k) { rlo[b][k] = alo[k]; rhi[b][k] = ahi[k]; }
                rc[b] = acount;
            }
            float llo[3] = {1e30f, 1e30f, 1e30f}, lhi[3] = {-1e30f, -1e30f, -1e30f};
            int lcount = 0;
            for (int b = 0; b < NB - 1; ++b) {
                for (int k = 0; k < 3; ++k) { llo[k] = std::min(llo[k], blo[b][k]); lhi[k] = std::max(lhi[k], bhi[b][k]); }
                lcount += bc[b];
                int rcount = rc[b + 1];
                if (lcount == 0 || rcount == 0) continue;
                float cost = area(llo, lhi) * lcount + area(rlo[b + 1], rhi[b + 1]) * rcount;
                if (cost < best_cost) { best_cost = cost; best_axis = a; best_bin = b; }
            }
        }
        float leaf_cost = area(n.lo, n.hi) * count;
        float split_cost = best_axis >= 0 ? C_TRAV * area(n.lo, n.hi) + best_cost : 1e30f;
        if (count <= MAX_LEAF && leaf_cost <= split_cost) return id;
        int mid;
        if (best_axis < 0) {
            mid = first + count / 2;  // all centroids coincide: split the list in half
        } else {
            float ext = chi[best_axis] - clo[best_axis];
            float sc = NB / ext;
            int a = best_axis, bb = best_bin;
            float c0 = clo[a];
            auto it = std::partition(idx.begin() + first, idx.begin() + first + count, [&](int q) {
                return std::min(NB - 1, (int)((prims[q].c[a] - c0) * sc)) <= bb;
            });
            mid = (int)(it - idx.begin());
            if (mid == first || mid == first + count) mid = first + count / 2;
        }
        int l = build(first, mid - first, depth + 1);
        int r = build(mid, first + count - mid, depth + 1);
        nodes[id].left = l; nodes[id].right = r; nodes[id].count = 0;
        return id;
    }
};

// ============================================================================ scene / plan objects
struct WorldHost {
    DevBuf nodes, prims, tri_uv, mats, lights;
    DevWorld dev;
    int bvh_depth = 0;
};

struct ppt_scene {
    int device = 0;
    std::vector<int64_t> slot_numel;
    std::vector<WorldHost*> worlds;
    DevBuf dev_worlds;
    int cu_count = 256;
    int stack_cap = 2;     // traversal stack entries: deepest BVH + 2
    bool has_ext = false;  // normal maps, specular maps or circularly polarized emitters
    ~ppt_scene() { for (auto* w : worlds) delete w; }
};

// Optional event timing of the launches of one call (diagnostics): an event before every kernel
// launch and one after the last, with the family of the kernel each interval belongs to.
struct KTimer {
    std::vector<hipEvent_t> ev;  // pool, grown on demand
    std::vector<int> fam;
    size_t n = 0;
    bool failed = false;
    ~KTimer() { for (hipEvent_t e : ev) (void)hipEventDestroy(e); }
    void begin() { n = 0; fam.clear(); failed = false; }
    void mark(int family, hipStream_t s) {
        if (failed) return;
        if (n == ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { failed = true; return; }
            ev.push_back(e);
        }
        if (hipEventRecord(ev[n], s) != hipSuccess) { failed = true; return; }
        fam.push_back(family);
        ++n;
    }
    static void mark_fn(void* ctx, int family, hipStream_t s) { ((KTimer*)ctx)->mark(family, s); }
};

struct ppt_plan {
    const ppt_scene* scene = nullptr;
    std::vector<ppt_view> views;
    std::vector<DevView> dviews;
    DevBuf dev_views;
    int32_t max_depth = 1;
    uint32_t flags = 0;
    int64_t image_numel = 0, num_paths = 0;
    int32_t Q = 64;             // paths per chunk (slots of the path state)
    int32_t n_chunks = 1;
    LaunchGrid grid{1, 1, 1, 1, 0, 1};
    const uint8_t* mask = nullptr;
    bool stats = true;
    bool timing = false;
    int32_t ckpt = 0;           // hybrid replay checkpoint interval, 0 = cached
    int32_t hyb_rule = 0;       // hybrid replay decision rule (Eq. 3) and its thresholds
    float hyb_gamma = 0.0f, hyb_eps = 0.0f;
    int32_t adjoint = 0;        // PPT_ADJOINT_*
    bool all_polarizer = false;  // every view has a linear-polarizer sensor (the render's rank-one record)
    float pprb_sigma = 0.0f;
    mutable KTimer timer[2];  // most recent render / backward call while timing is enabled
};

static bool slot_ok(const ppt_scene* s, int32_t slot, int64_t off, int64_t n) {
    return slot >= 0 && slot < (int32_t)s->slot_numel.size() && off >= 0 && n >= 0 && off + n <= s->slot_numel[slot];
}

// Parse and validate one world; unless dry, build its BVH and upload it.
static int convert_world(ppt_scene* sc, const uint8_t*& p, const uint8_t* end, WorldHost& wh, int wi, bool dry) {
    auto need = [&](size_t k) { return (size_t)(end - p) >= k; };
    if (!need(16)) return fail(PPT_EINVAL, "blob truncated (world header)");
    uint32_t cnt[4];
    std::memcpy(cnt, p, 16); p += 16;
    uint64_t nt = cnt[0], ns = cnt[1], nm = cnt[2], nl = cnt[3];
    if (nt + ns >= (1ull << 26)) return fail(PPT_EUNSUPPORTED, "more than 2^26 primitives in a world");
    size_t bytes = nt * 36 + nt * 24 + nt * 4 + ns * 16 + ns * 4 + nm * sizeof(BlobMaterial) + nl * sizeof(BlobLight);
    if (!need(bytes)) return fail(PPT_EINVAL, "blob truncated (world data)");
    const float* tv = (const float*)p; p += nt * 36;
    const float* tuv = (const float*)p; p += nt * 24;
    const uint32_t* tm = (const uint32_t*)p; p += nt * 4;
    const float* sp = (const float*)p; p += ns * 16;
    const uint32_t* sm = (const uint32_t*)p; p += ns * 4;
    const BlobMaterial* bm = (const BlobMaterial*)p; p += nm * sizeof(BlobMaterial);
    const BlobLight* bl = (const BlobLight*)p; p += nl * sizeof(BlobLight);

    // materials
    std::vector<DevMaterial> mats(nm);
    for (uint64_t i = 0; i < nm; ++i) {
        BlobMaterial b;
        std::memcpy(&b, bm + i, sizeof(b));
        DevMaterial& m = mats[i];
        m.type = (int32_t)b.type;
        m.alb_slot = b.alb_slot; m.alb_off = (int32_t)b.alb_off; m.alb_tw = (int32_t)b.alb_tw; m.alb_th = (int32_t)b.alb_th;
        m.alpha_slot = b.alpha_slot; m.alpha_off = (int32_t)b.alpha_off; m.alpha_tw = (int32_t)b.alpha_tw; m.alpha_th = (int32_t)b.alpha_th;
        m.eta_slot = b.eta_slot; m.eta_off = (int32_t)b.eta_off;
        m.kap_slot = b.kap_slot; m.kap_off = (int32_t)b.kap_off;
        m.emit_slot = b.emit_slot; m.emit_off = (int32_t)b.emit_off;
        for (int k = 0; k < 3; ++k) m.axis[k] = b.axis[k];
        m.blend = b.blend;
        m.emit_circ = b.emit_circ;
        m.spec_slot = b.spec_slot; m.spec_off = (int32_t)b.spec_off; m.spec_tw = (int32_t)b.spec_tw; m.spec_th = (int32_t)b.spec_th;
        m.nrm_slot = b.nrm_slot; m.nrm_off = (int32_t)b.nrm_off; m.nrm_tw = (int32_t)b.nrm_tw; m.nrm_th = (int32_t)b.nrm_th;
        char msg[160];
        std::snprintf(msg, sizeof msg, "world %d material %llu: invalid parameter reference", wi, (unsigned long long)i);
        bool ok = b.type <= MAT_BLEND;
        bool tex_a = b.alb_tw > 0, tex_r = b.alpha_tw > 0;
        if (tex_a && (b.alb_th == 0 || (uint64_t)b.alb_tw * b.alb_th > (1ull << 30))) ok = false;
        if (tex_r && (b.alpha_th == 0 || (uint64_t)b.alpha_tw * b.alpha_th > (1ull << 30))) ok = false;
        auto alb_ok = [&] { return slot_ok(sc, b.alb_slot, b.alb_off, tex_a ? (int64_t)b.alb_tw * b.alb_th * 3 : 3); };
        auto alpha_ok = [&] { return slot_ok(sc, b.alpha_slot, b.alpha_off, tex_r ? (int64_t)b.alpha_tw * b.alpha_th : 1); };
        if (ok) switch (b.type) {
            case MAT_LAMBERT: ok = alb_ok(); break;
            case MAT_DIELECTRIC: ok = slot_ok(sc, b.eta_slot, b.eta_off, 1); break;
            case MAT_GGX_DIELECTRIC: ok = alpha_ok() && slot_ok(sc, b.eta_slot, b.eta_off, 1); break;
            case MAT_GGX_CONDUCTOR:
                ok = alpha_ok() && slot_ok(sc, b.eta_slot, b.eta_off, 1) && slot_ok(sc, b.kap_slot, b.kap_off, 1);
                break;
            case MAT_SHEET: {
                float l = b.axis[0] * b.axis[0] + b.axis[1] * b.axis[1] + b.axis[2] * b.axis[2];
                ok = l > 1e-12f;
                break;
            }
            case MAT_EMITTER: ok = true; break;
            case MAT_BLEND:
                ok = alb_ok() && alpha_ok() && slot_ok(sc, b.eta_slot, b.eta_off, 1) && b.blend >= 0.0f && b.blend <= 1.0f;
                break;
        }
        if (ok && b.emit_slot >= 0) ok = slot_ok(sc, b.emit_slot, b.emit_off, 3) && std::fabs(b.emit_circ) <= 1.0f;
        // optional maps: specular scale (1 channel) and tangent-space normal (3 channels)
        auto map_ok = [&](int32_t slot, uint32_t off, uint32_t tw, uint32_t th, int ch) {
            if (slot < 0) return true;
            if (tw > 0 && (th == 0 || (uint64_t)tw * th > (1ull << 30))) return false;
            return slot_ok(sc, slot, off, tw > 0 ? (int64_t)tw * th * ch : ch);
        };
        if (ok) ok = map_ok(b.spec_slot, b.spec_off, b.spec_tw, b.spec_th, 1) &&
                     map_ok(b.nrm_slot, b.nrm_off, b.nrm_tw, b.nrm_th, 3);
        if (ok && b.spec_slot >= 0 && !(b.type == MAT_GGX_DIELECTRIC || b.type == MAT_GGX_CONDUCTOR || b.type == MAT_BLEND))
            ok = false;
        if (ok && b.nrm_slot >= 0 && !(b.type == MAT_LAMBERT || b.type == MAT_DIELECTRIC || b.type == MAT_GGX_DIELECTRIC ||
                                       b.type == MAT_GGX_CONDUCTOR || b.type == MAT_BLEND))
            ok = false;
        if (ok && b.type == MAT_EMITTER && b.emit_slot < 0) ok = false;
        if (!ok) return fail(PPT_EINVAL, msg);
        if (b.type != MAT_GGX_CONDUCTOR) m.kap_slot = -1;
        if (b.nrm_slot >= 0 || b.spec_slot >= 0 || b.emit_circ != 0.0f) sc->has_ext = true;
    }
    // lights
    std::vector<DevLight> lights(nl);
    for (uint64_t i = 0; i < nl; ++i) {
        BlobLight b;
        std::memcpy(&b, bl + i, sizeof(b));
        if (!slot_ok(sc, b.le_slot, b.le_off, 3)) return fail(PPT_EINVAL, "light radiance reference out of range");
        if (!(std::fabs(b.circ) <= 1.0f)) return fail(PPT_EINVAL, "light circular polarization outside [-1, 1]");
        DevLight& L = lights[i];
        double eu[3] = {b.eu[0], b.eu[1], b.eu[2]}, ev[3] = {b.ev[0], b.ev[1], b.ev[2]};
        double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        double a = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(a > 0.0)) return fail(PPT_EINVAL, "degenerate light");
        for (int k = 0; k < 3; ++k) {
            L.p0[k] = b.p0[k]; L.eu[k] = b.eu[k]; L.ev[k] = b.ev[k]; L.n[k] = (float)(n[k] / a);
        }
        L.area = (float)a;
        L.le_slot = b.le_slot; L.le_off = (int32_t)b.le_off;
        L.circ = b.circ;
        if (b.circ != 0.0f) sc->has_ext = true;
    }
    // primitives
    uint64_t np = nt + ns;
    std::vector<int32_t> pmat(np);
    for (uint64_t i = 0; i < nt; ++i) {
        if (tm[i] >= nm) return fail(PPT_EINVAL, "triangle material out of range");
        pmat[i] = (int32_t)tm[i];
    }
    for (uint64_t j = 0; j < ns; ++j) {
        if (sm[j] >= nm) return fail(PPT_EINVAL, "sphere material out of range");
        pmat[nt + j] = (int32_t)sm[j];
    }
    Builder B;
    B.prims.resize(np);
    B.idx.resize(np);
    for (uint64_t i = 0; i < np; ++i) {
        BPrim& q = B.prims[i];
        B.idx[i] = (int)i;
        if (i < nt) {
            const float* v = tv + 9 * i;
            for (int k = 0; k < 9; ++k)
                if (!std::isfinite(v[k])) return fail(PPT_EINVAL, "non-finite geometry");
            for (int a = 0; a < 3; ++a) {
                q.lo[a] = std::min({v[a], v[3 + a], v[6 + a]});
                q.hi[a] = std::max({v[a], v[3 + a], v[6 + a]});
            }
        } else {
            const float* s = sp + 4 * (i - nt);
            for (int k = 0; k < 4; ++k)
                if (!std::isfinite(s[k])) return fail(PPT_EINVAL, "non-finite geometry");
            float r = std::fabs(s[3]);
            for (int a = 0; a < 3; ++a) { q.lo[a] = s[a] - r; q.hi[a] = s[a] + r; }
        }
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(q.lo[a]) || !std::isfinite(q.hi[a])) return fail(PPT_EINVAL, "non-finite geometry");
            q.c[a] = 0.5f * (q.lo[a] + q.hi[a]);
        }
    }
    if (dry) return PPT_OK;
    int root_ref = 0;
    std::vector<float4> nodes, prims;
    if (np > 0) {
        B.build(0, (int)np, 0);
        if (B.max_depth >= STACK - 1) return fail(PPT_EUNSUPPORTED, "BVH deeper than the traversal stack");
        wh.bvh_depth = B.max_depth;
        // leaf references / inner node renumbering (inner nodes only, preorder)
        std::vector<int> inner_id(B.nodes.size(), -1);
        int n_inner = 0;
        for (size_t i = 0; i < B.nodes.size(); ++i)
            if (B.nodes[i].left >= 0) inner_id[i] = n_inner++;
        auto ref_of = [&](int i) -> int {
            const BNode& n = B.nodes[i];
            if (n.left >= 0) return inner_id[i];
            int first = n.first, cnt = n.count;
            return ~((first << 3) | (cnt - 1));
        };
        bool ok_leaves = true;
        for (const BNode& n : B.nodes)
            if (n.left < 0 && (n.count < 1 || n.count > 8)) ok_leaves = false;
        if (!ok_leaves) return fail(PPT_EDEVICE, "internal error: leaf size");
        nodes.resize((size_t)std::max(n_inner, 1) * 2);
        std::memset(nodes.data(), 0, nodes.size() * sizeof(float4));
        for (size_t i = 0; i < B.nodes.size(); ++i) {
            const BNode& n = B.nodes[i];
            if (n.left < 0) continue;
            const BNode& L = B.nodes[n.left];
            const BNode& R = B.nodes[n.right];
            float4* q = &nodes[2 * (size_t)inner_id[i]];
            int rl = ref_of(n.left), rr = ref_of(n.right);
            float fl, fr;
            std::memcpy(&fl, &rl, 4); std::memcpy(&fr, &rr, 4);
            q[0] = make_float4(half_pair(L.lo[0], L.hi[0]), half_pair(L.lo[1], L.hi[1]),
                               half_pair(R.lo[0], R.hi[0]), half_pair(R.lo[1], R.hi[1]));
            q[1] = make_float4(half_pair(L.lo[2], L.hi[2]), half_pair(R.lo[2], R.hi[2]), fl, fr);
        }
        root_ref = ref_of(0);
        prims.resize(np * 3);
        for (uint64_t k = 0; k < np; ++k) {
            int i = B.idx[k];
            float forig, fmat;
            int32_t orig = i;
            std::memcpy(&forig, &orig, 4);
            std::memcpy(&fmat, &pmat[i], 4);
            if ((uint64_t)i < nt) {
                const float* v = tv + 9 * (size_t)i;
                float e1[3], e2[3];
                for (int a = 0; a < 3; ++a) {
                    e1[a] = (float)((double)v[3 + a] - (double)v[a]);
                    e2[a] = (float)((double)v[6 + a] - (double)v[a]);
                }
                prims[3 * k] = make_float4(v[0], v[1], v[2], forig);
                prims[3 * k + 1] = make_float4(e1[0], e1[1], e1[2], fmat);
                prims[3 * k + 2] = make_float4(e2[0], e2[1], e2[2], 0.0f);
            } else {
                const float* s = sp + 4 * ((size_t)i - nt);
                int32_t one = 1;
                float fone;
                std::memcpy(&fone, &one, 4);
                prims[3 * k] = make_float4(s[0], s[1], s[2], forig);
                prims[3 * k + 1] = make_float4(s[3], 0.0f, 0.0f, fmat);
                prims[3 * k + 2] = make_float4(0.0f, 0.0f, 0.0f, fone);
            }
        }
    }
    int rc;
    if ((rc = wh.nodes.upload(nodes.data(), nodes.size() * sizeof(float4), "bvh nodes"))) return rc;
    if ((rc = wh.prims.upload(prims.data(), prims.size() * sizeof(float4), "primitives"))) return rc;
    if ((rc = wh.tri_uv.upload(tuv, nt * 24, "uv"))) return rc;
    if ((rc = wh.mats.upload(mats.data(), mats.size() * sizeof(DevMaterial), "materials"))) return rc;
    if ((rc = wh.lights.upload(lights.data(), lights.size() * sizeof(DevLight), "lights"))) return rc;
    wh.dev.nodes = (const float4*)wh.nodes.p;
    wh.dev.prims = (const float4*)wh.prims.p;
    wh.dev.tri_uv = (const float*)wh.tri_uv.p;
    wh.dev.mats = (const DevMaterial*)wh.mats.p;
    wh.dev.lights = (const DevLight*)wh.lights.p;
    wh.dev.n_tris = (int32_t)nt;
    wh.dev.n_prims = (int32_t)np;
    wh.dev.n_lights = (int32_t)nl;
    wh.dev.root = root_ref;
    return PPT_OK;
}

// ============================================================================ workspace layout
// [call table][stats][queue counts][path state of one chunk (SoA)][FP64 gradient accumulators]
struct WsLayout {
    size_t table, stats, counts, gacc, total;
    int lds_nd = 0, lds_nf = 0;
    size_t ray, shd, acc, cache, hits, ckpt, q0, q1, sq, hq, hf, nv, nv_bytes;
    size_t ray2, shd2, acc2, q0_2, q1_2, sq2, hq2, hf2, counts2;  // P-RB sub-path state
    int64_t gacc_n;
};
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
// Q: path-state slots of one chunk (the plan's chunk size, or less for the fixed scratch)
// The render keeps each path's state in the rank-one record (no shadow record) when every view has a
// linear-polarizer sensor and the scene has none of the light-stage features.
static bool rank_one(const ppt_plan* p) { return p->all_polarizer && !p->scene->has_ext; }

static WsLayout ws_layout(const ppt_plan* p, int op, int32_t Qslots) {
    WsLayout L{};
    const size_t Q = (size_t)Qslots;
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t r = at; at = align256(at + bytes); return r; };
    L.table = take(sizeof(CallTable));
    L.stats = take(sizeof(Stats));
    L.counts = take(32);
    L.ray = take(RAY_F4 * 16 * Q);
    L.shd = take(op == 0 && rank_one(p) ? 0 : SHD_F4 * 16 * Q);
    const bool tape = op == 1 && p->adjoint == PPT_ADJOINT_TAPE;  // (forward accumulator + per-vertex tape)
    L.acc = take(op == 0 || tape ? ACC_F4 * 16 * Q : 0);
    L.nv_bytes = (op == 0 && rank_one(p)) || op == 1 ? Q : 0;  // vertex counts (rank-one render, backward)
    L.nv = take(L.nv_bytes);
    const bool hybrid = op == 1 && p->ckpt > 0;
    const size_t records = hybrid ? (size_t)std::min(p->ckpt, p->max_depth) : (size_t)p->max_depth;
    L.cache = take(op == 1 ? records * (tape ? TAPE_F4 : CACHE_F4) * 16 * Q : 0);
    L.hits = take(hybrid ? (size_t)p->max_depth * 16 * Q : 0);
    L.ckpt = take(hybrid ? (size_t)((p->max_depth + p->ckpt - 1) / p->ckpt) * CKPT_F4 * 16 * Q : 0);
    L.q0 = take(4 * Q); L.q1 = take(4 * Q); L.sq = take(4 * Q); L.hq = take(4 * Q); L.hf = take(Q);
    const bool prb = op == 1 && p->adjoint == PPT_ADJOINT_PRB;
    const size_t Q2 = prb ? Q : 0;
    L.counts2 = take(prb ? 32 : 0);
    L.ray2 = take(RAY_F4 * 16 * Q2); L.shd2 = take(SHD_F4 * 16 * Q2); L.acc2 = take(ACC_F4 * 16 * Q2);
    L.q0_2 = take(4 * Q2); L.q1_2 = take(4 * Q2); L.sq2 = take(4 * Q2); L.hq2 = take(4 * Q2); L.hf2 = take(Q2);
    L.gacc_n = 0;
    if (op == 1)
        for (int64_t n : p->scene->slot_numel) L.gacc_n += n;
    L.gacc = take((size_t)L.gacc_n * 8);
    L.total = at;
    return L;
}
static PathState path_state2(void* ws, const WsLayout& L) {
    char* w = (char*)ws;
    PathState S{};
    S.ray = (float4*)(w + L.ray2);
    S.shd = (float4*)(w + L.shd2);
    S.acc = (float4*)(w + L.acc2);
    S.queue0 = (int*)(w + L.q0_2); S.queue1 = (int*)(w + L.q1_2); S.squeue = (int*)(w + L.sq2); S.hqueue = (int*)(w + L.hq2);
    S.hflag = (uint8_t*)(w + L.hf2);
    S.counts = (int*)(w + L.counts2);
    return S;
}
static PathState path_state(void* ws, const WsLayout& L) {
    char* w = (char*)ws;
    PathState S;
    S.ray = (float4*)(w + L.ray);
    S.shd = (float4*)(w + L.shd);
    S.acc = (float4*)(w + L.acc);
    S.nv = L.nv_bytes ? (uint8_t*)(w + L.nv) : nullptr;
    S.cache = (float4*)(w + L.cache);
    S.hits = (float4*)(w + L.hits);
    S.ckpt = (float4*)(w + L.ckpt);
    S.queue0 = (int*)(w + L.q0); S.queue1 = (int*)(w + L.q1); S.squeue = (int*)(w + L.sq); S.hqueue = (int*)(w + L.hq);
    S.hflag = (uint8_t*)(w + L.hf);
    S.counts = (int*)(w + L.counts);
    return S;
}

// ============================================================================ C ABI
extern "C" {

const char* ppt_last_error(void) { return g_err.c_str(); }

int ppt_scene_create(const void* blob, size_t nbytes, ppt_scene** out) {
    if (!blob || !out) return fail(PPT_EINVAL, "null argument");
    *out = nullptr;
    const uint8_t* p = (const uint8_t*)blob;
    const uint8_t* end = p + nbytes;
    if (nbytes < 16) return fail(PPT_EINVAL, "blob truncated (header)");
    uint32_t hdr[4];
    std::memcpy(hdr, p, 16); p += 16;
    if (hdr[0] != 0x31545050u || hdr[1] != 2u) return fail(PPT_EINVAL, "bad blob magic or version");
    if (hdr[2] > (uint32_t)MAX_SLOTS) return fail(PPT_EUNSUPPORTED, "too many parameter slots");
    if (hdr[3] == 0 || hdr[3] > 4096) return fail(PPT_EINVAL, "bad world count");
    if ((size_t)(end - p) < 4ull * hdr[2]) return fail(PPT_EINVAL, "blob truncated (slots)");
    ppt_scene* sc = new ppt_scene();
    for (uint32_t i = 0; i < hdr[2]; ++i) {
        uint32_t n;
        std::memcpy(&n, p, 4); p += 4;
        sc->slot_numel.push_back(n);
    }
    // validate every world on the host before any device work
    const uint8_t* body = p;
    for (uint32_t w = 0; w < hdr[3]; ++w) {
        WorldHost tmp;
        int rc = convert_world(sc, p, end, tmp, (int)w, true);
        if (rc) { delete sc; return rc; }
    }
    if (p != end) { delete sc; return fail(PPT_EINVAL, "trailing bytes after the last world"); }
    p = body;
    if (hipGetDevice(&sc->device) != hipSuccess) { delete sc; return fail(PPT_EDEVICE, "no HIP device"); }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, sc->device) != hipSuccess) { delete sc; return fail(PPT_EDEVICE, "device properties"); }
    sc->cu_count = prop.multiProcessorCount;
    std::vector<DevWorld> dw;
    for (uint32_t w = 0; w < hdr[3]; ++w) {
        WorldHost* wh = new WorldHost();
        sc->worlds.push_back(wh);
        int rc = convert_world(sc, p, end, *wh, (int)w, false);
        if (rc) { delete sc; return rc; }
        dw.push_back(wh->dev);
        sc->stack_cap = std::max(sc->stack_cap, wh->bvh_depth + 2);
    }
    int rc = sc->dev_worlds.upload(dw.data(), dw.size() * sizeof(DevWorld), "world table");
    if (rc) { delete sc; return rc; }
    *out = sc;
    return PPT_OK;
}

void ppt_scene_destroy(ppt_scene* s) { delete s; }

int ppt_scene_slots(const ppt_scene* s, int32_t* n_slots, int64_t* numel_out, int32_t cap) {
    if (!s) return fail(PPT_EINVAL, "null scene");
    if (n_slots) *n_slots = (int32_t)s->slot_numel.size();
    if (numel_out)
        for (int32_t i = 0; i < cap && i < (int32_t)s->slot_numel.size(); ++i) numel_out[i] = s->slot_numel[i];
    return PPT_OK;
}

int ppt_plan_create(const ppt_scene* sc, const ppt_view* views, int32_t n_views, int32_t max_depth, uint32_t flags,
                    const ppt_plan_opts* opts, ppt_plan** out) {
    if (!sc || !views || !out || n_views < 1) return fail(PPT_EINVAL, "null argument or no views");
    *out = nullptr;
    if (max_depth < 1 || max_depth > MAX_DEPTH) return fail(PPT_EUNSUPPORTED, "max_depth must be in [1, 128]");
    if (flags & ~PPT_FLAG_NO_NEE) return fail(PPT_EINVAL, "unknown flags");
    ppt_plan* P = new ppt_plan();
    P->scene = sc;
    P->max_depth = max_depth;
    P->flags = flags;
    P->views.assign(views, views + n_views);
    int64_t out_off = 0, path_off = 0;
    if (n_views >= (1 << 19)) { delete P; return fail(PPT_EUNSUPPORTED, "too many views"); }
    for (int32_t v = 0; v < n_views; ++v) {
        const ppt_view& V = views[v];
        bool ok = V.world >= 0 && V.world < (int32_t)sc->worlds.size() && V.width >= 1 && V.height >= 1 &&
                  V.spp >= 1 && V.crop_x0 >= 0 && V.crop_y0 >= 0 && V.crop_w >= 0 && V.crop_h >= 0 &&
                  (int64_t)V.crop_x0 + V.crop_w <= V.width && (int64_t)V.crop_y0 + V.crop_h <= V.height &&
                  (int64_t)V.width * V.height <= (1ll << 31) && V.view_id < (1u << 24) &&
                  V.sensor >= PPT_SENSOR_NONE && V.sensor <= PPT_SENSOR_LIGHTSTAGE4 && V.fov_y_deg > 0.0f &&
                  V.fov_y_deg < 180.0f;
        if (ok && V.sensor == PPT_SENSOR_POLARIZER) ok = slot_ok(sc, V.theta_slot, V.theta_off, 1);
        if (ok && (int64_t)V.crop_w * V.crop_h * V.spp >= (1ll << 31)) {
            delete P;
            return fail(PPT_EUNSUPPORTED, "a view has 2^31 or more paths");
        }
        double o[3] = {V.origin[0], V.origin[1], V.origin[2]}, t[3] = {V.target[0], V.target[1], V.target[2]};
        double up[3] = {V.up[0], V.up[1], V.up[2]};
        double f[3] = {t[0] - o[0], t[1] - o[1], t[2] - o[2]};
        double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        double r[3] = {0, 0, 0}, u[3];
        double rl = 0;
        if (fl > 0) {
            for (double& x : f) x /= fl;
            r[0] = f[1] * up[2] - f[2] * up[1]; r[1] = f[2] * up[0] - f[0] * up[2]; r[2] = f[0] * up[1] - f[1] * up[0];
            rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        }
        if (!(fl > 0 && rl > 0)) ok = false;
        if (!ok) {
            delete P;
            char msg[96];
            std::snprintf(msg, sizeof msg, "invalid view %d", v);
            return fail(PPT_EINVAL, msg);
        }
        for (double& x : r) x /= rl;
        u[0] = r[1] * f[2] - r[2] * f[1]; u[1] = r[2] * f[0] - r[0] * f[2]; u[2] = r[0] * f[1] - r[1] * f[0];
        DevView D{};
        D.world = V.world; D.width = V.width; D.height = V.height; D.spp = V.spp;
        D.crop_x0 = V.crop_x0; D.crop_y0 = V.crop_y0; D.crop_w = V.crop_w; D.crop_h = V.crop_h;
        for (int k = 0; k < 3; ++k) { D.o[k] = V.origin[k]; D.f[k] = (float)f[k]; D.r[k] = (float)r[k]; D.u[k] = (float)u[k]; }
        D.tan_h = (float)std::tan(0.5 * (double)V.fov_y_deg * M_PI / 180.0);
        D.aspect = (float)((double)V.width / (double)V.height);
        D.sensor = V.sensor; D.theta_slot = V.theta_slot; D.theta_off = V.theta_off;
        D.n_analyzers = (V.sensor == PPT_SENSOR_ANALYZER4 || V.sensor == PPT_SENSOR_LIGHTSTAGE4) ? 4 : 1;
        D.view_id = V.view_id;
        D.out_off = out_off;
        D.path_off = path_off;
        out_off += (int64_t)D.n_analyzers * V.crop_w * V.crop_h * 12;
        path_off += (int64_t)V.crop_w * V.crop_h * V.spp;
        P->dviews.push_back(D);
    }
    P->image_numel = out_off;
    P->num_paths = path_off;
    P->all_polarizer = n_views > 0;
    for (int32_t v = 0; v < n_views; ++v) P->all_polarizer = P->all_polarizer && views[v].sensor == PPT_SENSOR_POLARIZER;
    // chunk of paths in flight: all paths up to 16M by default, a multiple of the wavefront size
    if (opts && (opts->checkpoint_interval < 0 || opts->checkpoint_interval > MAX_DEPTH)) {
        delete P;
        return fail(PPT_EINVAL, "checkpoint_interval must be in [0, 128]");
    }
    P->ckpt = opts ? (int32_t)opts->checkpoint_interval : 0;
    if (opts && opts->hybrid_rule) {
        if (opts->hybrid_rule != 1 || P->ckpt < 1 || !(opts->hybrid_gamma >= 0.0f) || !(opts->hybrid_eps >= 0.0f)) {
            delete P;
            return fail(PPT_EINVAL, "hybrid_rule needs checkpoint_interval >= 1, hybrid_gamma >= 0 and hybrid_eps >= 0");
        }
        P->hyb_rule = 1;
        P->hyb_gamma = opts->hybrid_gamma;
        P->hyb_eps = opts->hybrid_eps;
    }
    if (opts && opts->adjoint) {
        const bool ok_pprb = opts->adjoint == PPT_ADJOINT_PPRB && opts->pprb_sigma >= 0.0f && std::isfinite(opts->pprb_sigma);
        const bool ok_tape = opts->adjoint == PPT_ADJOINT_TAPE;
        const bool ok_prb = opts->adjoint == PPT_ADJOINT_PRB;
        if (!(ok_pprb || ok_tape || ok_prb) || P->ckpt != 0) {
            delete P;
            return fail(PPT_EINVAL, "adjoint must be PPT_ADJOINT_CACHED, PPT_ADJOINT_PPRB (finite pprb_sigma >= 0), "
                                    "PPT_ADJOINT_TAPE or PPT_ADJOINT_PRB, the last three without checkpoints");
        }
        if (ok_prb && sc->has_ext) {
            delete P;
            return fail(PPT_EUNSUPPORTED, "the P-RB comparator does not support normal maps, specular maps or "
                                          "circularly polarized emitters");
        }
        if (ok_tape && sc->has_ext) {
            delete P;
            return fail(PPT_EUNSUPPORTED, "the tape baseline does not support normal maps, specular maps or "
                                          "circularly polarized emitters");
        }
        P->adjoint = opts->adjoint;
        P->pprb_sigma = ok_pprb ? opts->pprb_sigma : 0.0f;
    }
    int64_t q = opts && opts->chunk_paths > 0 ? opts->chunk_paths : (int64_t)1 << 24;
    q = std::min<int64_t>(q, std::max<int64_t>(path_off, 1));
    q = ((q + WAVE - 1) / WAVE) * WAVE;
    if (q > ((int64_t)1 << 28)) { delete P; return fail(PPT_EUNSUPPORTED, "chunk too large"); }
    P->Q = (int32_t)q;
    P->n_chunks = (int32_t)std::max<int64_t>(1, (path_off + q - 1) / q);
    if (occupancy_grid(sc->cu_count, sc->stack_cap, &P->grid) != hipSuccess) {
        delete P;
        return fail(PPT_EDEVICE, "occupancy query failed");
    }
    int rc = P->dev_views.upload(P->dviews.data(), P->dviews.size() * sizeof(DevView), "views");
    if (rc) { delete P; return rc; }
    *out = P;
    return PPT_OK;
}

void ppt_plan_destroy(ppt_plan* p) { delete p; }
int64_t ppt_plan_image_numel(const ppt_plan* p) { return p ? p->image_numel : -1; }
int64_t ppt_plan_num_paths(const ppt_plan* p) { return p ? p->num_paths : -1; }
size_t ppt_plan_workspace_bytes(const ppt_plan* p, int32_t op) {
    if (!p || op < 0 || op > 1) return 0;
    return ws_layout(p, op, p->Q).total;
}
int ppt_plan_set_stats(ppt_plan* p, int32_t enabled) {
    if (!p) return fail(PPT_EINVAL, "null plan");
    p->stats = enabled != 0;
    return PPT_OK;
}
int ppt_plan_set_path_mask(ppt_plan* p, const uint8_t* mask) {
    if (!p) return fail(PPT_EINVAL, "null plan");
    p->mask = mask;
    return PPT_OK;
}
int ppt_plan_launch_info(const ppt_plan* p, int64_t* chunk_paths, int32_t* n_chunks, int32_t* stack_entries) {
    if (!p) return fail(PPT_EINVAL, "null plan");
    if (chunk_paths) *chunk_paths = p->Q;
    if (n_chunks) *n_chunks = p->n_chunks;
    if (stack_entries) *stack_entries = p->scene->stack_cap;
    return PPT_OK;
}

static int fill_table(const ppt_plan* p, const float* const* params, int32_t n_params, float* const* grads,
                      WsLayout& L, CallTable& t, int64_t* max_numel) {
    const ppt_scene* sc = p->scene;
    if (!params || n_params != (int32_t)sc->slot_numel.size()) return fail(PPT_EINVAL, "parameter count mismatch");
    std::memset(&t, 0, sizeof t);
    int64_t off = 0, mx = 1;
    for (int i = 0; i < MAX_SLOTS; ++i) { t.goff[i] = -1; t.lds_d[i] = -1; t.lds_f[i] = -1; }
    for (int32_t i = 0; i < n_params; ++i) {
        if (!params[i] && sc->slot_numel[i] > 0) return fail(PPT_EINVAL, "null parameter pointer");
        t.p[i] = params[i];
        t.numel[i] = sc->slot_numel[i];
        if (grads && grads[i]) { t.goff[i] = off; t.gout[i] = grads[i]; }
        off += sc->slot_numel[i];
        mx = std::max(mx, sc->slot_numel[i]);
    }
    if (max_numel) *max_numel = mx;
    // workgroup gradient accumulators: small slots in FP64, then textures in FP32 while they fit
    int nd = 0, nf = 0;
    for (int32_t i = 0; i < n_params; ++i) {
        if (t.goff[i] < 0) continue;
        int64_t n = sc->slot_numel[i];
        if (n <= 64 && nd + n <= LDS_GRAD_D) { t.lds_d[i] = nd; nd += (int)n; }
        else if (nf + n <= LDS_GRAD_F) { t.lds_f[i] = nf; nf += (int)n; }
    }
    L.lds_nd = nd; L.lds_nf = nf;
    return PPT_OK;
}

static WArgs make_args(const ppt_plan* p, uint64_t seed, void* ws, const WsLayout& L, int32_t Q) {
    WArgs a{};
    char* w = (char*)ws;
    a.worlds = (const DevWorld*)p->scene->dev_worlds.p;
    a.views = (const DevView*)p->dev_views.p;
    a.n_views = (int32_t)p->dviews.size();
    a.max_depth = p->max_depth;
    a.flags = p->flags;
    a.stack_cap = p->scene->stack_cap;
    a.seed = seed;
    a.table = (CallTable*)(w + L.table);
    a.stats = p->stats ? (Stats*)(w + L.stats) : nullptr;
    a.S = path_state(ws, L);
    a.Q = Q;
    a.mask = p->mask;
    a.ext = p->scene->has_ext ? 1 : 0;  // kernels with normal/specular maps and circular emitters
    a.r1 = rank_one(p) ? 1 : 0;
    if (p->scene->worlds.size() == 1) {
        a.one_world = 1;
        a.world0 = p->scene->worlds[0]->dev;
    }
    return a;
}

static int check_ws(const ppt_plan* p, void* ws, size_t ws_bytes, int op, WsLayout& L) {
    if (!p) return fail(PPT_EINVAL, "null plan");
    L = ws_layout(p, op, p->Q);
    if (!ws || ws_bytes < L.total) return fail(PPT_EINVAL, "workspace too small");
    if (((uintptr_t)ws & 255) != 0) return fail(PPT_EINVAL, "workspace must be 256-byte aligned");
    return PPT_OK;
}

static LaunchMarker marker(const ppt_plan* p, int op) {
    return p->timing ? LaunchMarker{&KTimer::mark_fn, &p->timer[op]} : LaunchMarker{nullptr, nullptr};
}

// every chunk of a.Q paths (the plan's chunk size unless the caller's memory holds less)
static int run_chunks(const ppt_plan* p, WArgs a, int mode, hipStream_t s, const LaunchMarker& M) {
    const int64_t n_chunks = std::max<int64_t>(1, (p->num_paths + a.Q - 1) / a.Q);
    for (int64_t c = 0; c < n_chunks; ++c) {
        a.g0 = c * a.Q;
        a.n_chunk = (int32_t)std::min<int64_t>(a.Q, p->num_paths - a.g0);
        if (a.n_chunk <= 0) break;
        HIP_TRY(launch_chunk(a, mode, p->grid, s, M), mode == 0 ? "render launch" : "backward launch");
    }
    return PPT_OK;
}

static int render_impl(const ppt_plan* p, const float* const* params, int32_t n_params, uint64_t seed,
                       float* out, uint64_t* sig, void* ws, size_t ws_bytes, void* stream) {
    WsLayout L;
    int rc = check_ws(p, ws, ws_bytes, 0, L);
    if (rc) return rc;
    if (!out && !sig) return fail(PPT_EINVAL, "null output");
    CallTable t;
    if ((rc = fill_table(p, params, n_params, nullptr, L, t, nullptr))) return rc;
    hipStream_t s = (hipStream_t)stream;
    WArgs a = make_args(p, seed, ws, L, p->Q);
    a.out = out;
    a.sig = sig;
    const LaunchMarker M = marker(p, 0);
    if (p->timing) p->timer[0].begin();
    M(KF_OTHER, s);
    HIP_TRY(launch_setup(t, a.table, (Stats*)((char*)ws + L.stats), p->stats, s), "setup launch");
    if (out) HIP_TRY(launch_fill_f32(out, p->image_numel, s), "clear launch");
    if ((rc = run_chunks(p, a, 0, s, M))) return rc;
    M(-1, s);
    return PPT_OK;
}

int ppt_render(const ppt_plan* p, const float* const* params, int32_t n_params, uint64_t seed, float* out, void* ws,
               size_t ws_bytes, void* stream) {
    if (!out) return fail(PPT_EINVAL, "null output");
    return render_impl(p, params, n_params, seed, out, nullptr, ws, ws_bytes, stream);
}

int ppt_signatures(const ppt_plan* p, const float* const* params, int32_t n_params, uint64_t seed, uint64_t* sig,
                   void* ws, size_t ws_bytes, void* stream) {
    if (!sig) return fail(PPT_EINVAL, "null signature output");
    return render_impl(p, params, n_params, seed, nullptr, sig, ws, ws_bytes, stream);
}

// The backward pass over workspace ws laid out by L for chunks of Q paths; M times the launches.
static int backward_impl(const ppt_plan* p, const float* const* params, int32_t n_params, uint64_t seed,
                         const float* d_stokes, float* const* grads, void* ws, WsLayout& L, int32_t Q, bool stats,
                         int op_timer, void* stream) {
    if (!d_stokes) return fail(PPT_EINVAL, "null d_stokes");
    if (!grads) return fail(PPT_EINVAL, "null gradient table");
    CallTable t;
    int64_t mx = 1;
    int rc;
    if ((rc = fill_table(p, params, n_params, grads, L, t, &mx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    WArgs a = make_args(p, seed, ws, L, Q);
    if (!stats) a.stats = nullptr;
    a.dout = d_stokes;
    a.gacc = (double*)((char*)ws + L.gacc);
    a.lds_nd = L.lds_nd;
    a.lds_nf = L.lds_nf;
    a.ckpt = p->ckpt;
    a.hyb_rule = p->hyb_rule;
    a.hyb_gamma = p->hyb_gamma;
    a.hyb_eps = p->hyb_eps;
    a.hyb_stats = a.stats ? ((Stats*)((char*)ws + L.stats))->hyb : nullptr;
    a.pprb = p->adjoint == PPT_ADJOINT_PPRB;
    a.tape = p->adjoint == PPT_ADJOINT_TAPE;
    a.prb = p->adjoint == PPT_ADJOINT_PRB;
    if (a.prb) a.S2 = path_state2(ws, L);
    a.pprb_sigma = p->pprb_sigma;
    const LaunchMarker M = op_timer >= 0 ? marker(p, op_timer) : LaunchMarker{nullptr, nullptr};
    if (op_timer >= 0 && p->timing) p->timer[op_timer].begin();
    M(KF_OTHER, s);
    HIP_TRY(launch_setup(t, a.table, (Stats*)((char*)ws + L.stats), stats, s), "setup launch");
    HIP_TRY(launch_fill_f64(a.gacc, L.gacc_n, s), "clear launch");
    if ((rc = run_chunks(p, a, 1, s, M))) return rc;
    M(KF_OTHER, s);
    HIP_TRY(launch_finalize(a.table, a.gacc, n_params, mx, s), "finalize launch");
    M(-1, s);
    return PPT_OK;
}

int ppt_backward(const ppt_plan* p, const float* const* params, int32_t n_params, uint64_t seed,
                 const float* d_stokes, float* const* grads, void* ws, size_t ws_bytes, void* stream) {
    WsLayout L;
    int rc = check_ws(p, ws, ws_bytes, 1, L);
    if (rc) return rc;
    return backward_impl(p, params, n_params, seed, d_stokes, grads, ws, L, p->Q, p->stats, 1, stream);
}

int ppt_backward_noalloc(const ppt_plan* p, const float* const* params, int32_t n_params, uint64_t seed,
                         const float* d_stokes, float* const* grads, void* stream) {
    if (!p) return fail(PPT_EINVAL, "null plan");
    // the largest chunk (a multiple of the wavefront size, at most the plan's) whose records and
    // the gradient accumulators fit in the fixed scratch
    const size_t cap = NOALLOC_SCRATCH_BYTES;
    if (ws_layout(p, 1, WAVE).total > cap) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "the fixed scratch (%zu bytes) cannot hold the gradient accumulators and one %d-path chunk "
                      "at depth %d (%zu bytes needed)", cap, WAVE, p->max_depth, ws_layout(p, 1, WAVE).total);
        return fail(PPT_EUNSUPPORTED, msg);
    }
    int64_t lo = 1, hi = std::max<int64_t>(1, p->Q / WAVE);  // in wavefronts
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (ws_layout(p, 1, (int32_t)(mid * WAVE)).total <= cap) lo = mid; else hi = mid - 1;
    }
    const int32_t Q = (int32_t)(lo * WAVE);
    void* ws = nullptr;
    HIP_TRY(noalloc_scratch(&ws), "scratch address lookup");
    WsLayout L = ws_layout(p, 1, Q);
    return backward_impl(p, params, n_params, seed, d_stokes, grads, ws, L, Q, false, -1, stream);
}

int ppt_plan_set_timing(ppt_plan* p, int32_t enabled) {
    if (!p) return fail(PPT_EINVAL, "null plan");
    p->timing = enabled != 0;
    p->timer[0].begin();
    p->timer[1].begin();
    return PPT_OK;
}

int ppt_plan_kernel_times(const ppt_plan* p, int32_t op, double* ms, int32_t* launches, int32_t n) {
    if (!p || !ms || !launches || n < 0) return fail(PPT_EINVAL, "bad argument");
    if (op < 0 || op > 1) return fail(PPT_EINVAL, "op must be 0 (render) or 1 (backward)");
    const KTimer& T = p->timer[op];
    if (T.failed) return fail(PPT_EDEVICE, "event recording failed");
    if (T.n < 2 || T.fam[T.n - 1] != -1) return fail(PPT_EINVAL, "no timed call of this op recorded");
    for (int32_t k = 0; k < n; ++k) { ms[k] = 0.0; launches[k] = 0; }
    HIP_TRY(hipEventSynchronize(T.ev[T.n - 1]), "event sync");
    for (size_t j = 0; j + 1 < T.n; ++j) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, T.ev[j], T.ev[j + 1]), "event time");
        int f = T.fam[j];
        if (f >= 0 && f < n) { ms[f] += t; launches[f] += 1; }
    }
    return PPT_OK;
}

int ppt_read_stats(const void* ws, int64_t* out, void* stream) {
    if (!ws || !out) return fail(PPT_EINVAL, "null argument");
    // the stats block sits at a fixed offset, right after the call table
    size_t off = align256(sizeof(CallTable));
    Stats st;
    HIP_TRY(hipMemcpyAsync(&st, (const char*)ws + off, sizeof st, hipMemcpyDeviceToHost, (hipStream_t)stream), "stats copy");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "stats sync");
    for (int k = 0; k < ST_COUNT; ++k) out[k] = (int64_t)st.c[k];
    return PPT_OK;
}

int ppt_read_hybrid_stats(const void* ws, int64_t* out, void* stream) {
    if (!ws || !out) return fail(PPT_EINVAL, "null argument");
    size_t off = align256(sizeof(CallTable));
    Stats st;
    HIP_TRY(hipMemcpyAsync(&st, (const char*)ws + off, sizeof st, hipMemcpyDeviceToHost, (hipStream_t)stream), "stats copy");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "stats sync");
    for (int k = 0; k < 3; ++k) out[k] = (int64_t)st.hyb[k];
    return PPT_OK;
}

int ppt_debug_rng(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n, void* stream) {
    if (!ctr || !out || n < 0) return fail(PPT_EINVAL, "bad argument");
    HIP_TRY(launch_rng(seed, ctr, out, n, (hipStream_t)stream), "rng launch");
    return PPT_OK;
}

}  // extern "C"
