// ppt_device.h -- device-side library of the polarized path tracer (gfx950): vector and
// complex arithmetic, Philox RNG, Stokes frames, Fresnel amplitudes and their adjoints,
// GGX microfacet terms, parameter/texture access, BVH traversal, path-vertex sampling and the
// per-vertex Mueller weights with their vector-Jacobian products.
#pragma once
#include "ppt_internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ppt {

#define DEV __device__ __forceinline__

constexpr float PI_F = 3.14159265358979323846f;

// ============================================================================ vectors
struct v3 { float x, y, z; };
DEV v3 mk(float x, float y, float z) { return {x, y, z}; }
DEV v3 operator+(v3 a, v3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
DEV v3 operator-(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
DEV v3 operator-(v3 a) { return {-a.x, -a.y, -a.z}; }
DEV v3 operator*(v3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
DEV float dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DEV v3 cross(v3 a, v3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
DEV v3 normalize(v3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
DEV v3 ld3(const float* p) { return {p[0], p[1], p[2]}; }

// ============================================================================ complex
struct cf { float re, im; };
DEV cf cadd(cf a, cf b) { return {a.re + b.re, a.im + b.im}; }
DEV cf csub(cf a, cf b) { return {a.re - b.re, a.im - b.im}; }
DEV cf cmul(cf a, cf b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
DEV cf cscale(cf a, float s) { return {a.re * s, a.im * s}; }
DEV cf cconj(cf a) { return {a.re, -a.im}; }
DEV float cabs2(cf a) { return a.re * a.re + a.im * a.im; }
DEV cf cdiv(cf a, cf b) {
    float d = 1.0f / cabs2(b);
    return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}
// principal square root; a zero imaginary part counts as +0
DEV cf csqrt(cf z) {
    float r = hypotf(z.re, z.im);
    if (r == 0.0f) return {0.0f, 0.0f};
    if (z.re >= 0.0f) {
        float t = sqrtf(0.5f * (r + z.re));
        return {t, z.im / (2.0f * t)};
    }
    float t = sqrtf(0.5f * (r - z.re));
    return {fabsf(z.im) / (2.0f * t), z.im < 0.0f ? -t : t};
}

// ============================================================================ RNG
// Philox4x32-10 (Salmon et al., SC'11).  Counter (pixel, sample, view << 8 | bounce, call).
DEV void philox(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
}
DEV float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }  // exact: 24 bits / 2^24
DEV void uniforms(uint64_t seed, uint32_t pix, uint32_t smp, uint32_t view, uint32_t bounce, uint32_t call,
                  float u[4]) {
    uint32_t c0 = pix, c1 = smp, c2 = (view << 8) | (bounce & 0xffu), c3 = call;
    philox(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    u[0] = u01(c0); u[1] = u01(c1); u[2] = u01(c2); u[3] = u01(c3);
}

// ============================================================================ wave helpers
DEV int lane_id() { return threadIdx.x & (WAVE - 1); }
DEV float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
DEV uint32_t wave_sum_u(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
// Sums of N values over the active lanes of the wavefront (act: their mask, taken where the caller
// runs), returned to every active lane; usable under divergence.  Butterfly over aligned blocks: a
// lane adds the partial sum of the block next to its own, read from that block's lowest active lane
// (every active lane of a block holds the block's sum), and nothing for a block without active lanes.
template <int N>
DEV void wave_sum_active(float* v, uint64_t act) {
    const unsigned lane = (unsigned)lane_id();
#pragma unroll 1
    for (int d = 1; d < WAVE; d <<= 1) {
        const unsigned base = (lane ^ (unsigned)d) & ~(unsigned)(d - 1);
        const uint64_t in = act & (((1ull << d) - 1ull) << base);
        const int q = in ? __ffsll((long long)in) - 1 : (int)lane;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const float t = __shfl(v[j], q, WAVE);
            v[j] += in ? t : 0.0f;
        }
    }
}
// maximum over the wavefront, returned wave-uniform (every lane must be active)
DEV int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    return __builtin_amdgcn_readfirstlane(v);
}

// ============================================================================ frames
// Orthonormal basis (x, y, n) of Duff et al. 2017.
DEV void onb(v3 n, v3& x, v3& y) {
    float sg = copysignf(1.0f, n.z);
    float a = -1.0f / (sg + n.z);
    float b = n.x * n.y * a;
    x = mk(1.0f + sg * n.x * n.x * a, sg * b, -sg * n.x);
    y = mk(b, sg + n.y * n.y * a, -n.y);
}
// canonical transverse basis vector of the Stokes frame of light travelling along k
DEV v3 canon_x(v3 k) {
    v3 x, y;
    onb(k, x, y);
    return x;
}
// Stokes rotator between transverse bases x_from -> x_to about k: (cos 2phi, sin 2phi)
DEV void rot_cs(v3 k, v3 x_from, v3 x_to, float& C, float& S) {
    float c = dot(x_from, x_to), s = dot(cross(k, x_from), x_to);
    C = c * c - s * s;
    S = 2.0f * c * s;
}
// s-axis of a specular event for incident propagation k_in and normal n_inc on the incident side
DEV v3 s_axis(v3 k_in, v3 n_inc) {
    v3 s = cross(k_in, n_inc);
    float l2 = dot(s, s);
    if (l2 < 1e-16f) return canon_x(k_in);
    return s * (1.0f / sqrtf(l2));
}

// ============================================================================ Fresnel
struct Fres { cf rs, rp, ts, tp, ct; float kappa, st2r; };
// Born & Wolf amplitudes for incidence cosine ci and relative index m = n2 / n1.
DEV void fresnel_amp(float ci, cf m, Fres& F, bool trans) {
    cf m2 = cmul(m, m);
    cf st2 = cdiv(cf{1.0f - ci * ci, 0.0f}, m2);
    F.ct = csqrt(csub(cf{1.0f, 0.0f}, st2));
    cf mct = cmul(m, F.ct), mci = cscale(m, ci);
    cf c{ci, 0.0f};
    F.rs = cdiv(csub(c, mct), cadd(c, mct));
    F.rp = cdiv(csub(mci, F.ct), cadd(mci, F.ct));
    if (trans) {
        F.ts = cdiv(cf{2.0f * ci, 0.0f}, cadd(c, mct));
        F.tp = cdiv(cf{2.0f * ci, 0.0f}, cadd(mci, F.ct));
        F.kappa = mct.re / ci;
    }
}
// Mueller entries (a, b, c, d) of a Jones matrix diag(as, ap)
DEV void jones_abcd(cf as, cf ap, float& a, float& b, float& c, float& d) {
    float A = cabs2(as), B = cabs2(ap);
    cf z = cmul(as, cconj(ap));
    a = 0.5f * (A + B); b = 0.5f * (A - B); c = z.re; d = z.im;
}
DEV void fresnel_R(float ci, cf m, float& a, float& b, float& c, float& d) {
    Fres F;
    fresnel_amp(ci, m, F, false);
    jones_abcd(F.rs, F.rp, a, b, c, d);
}
DEV void fresnel_T(float ci, cf m, float& a, float& b, float& c, float& d) {
    Fres F;
    fresnel_amp(ci, m, F, true);
    jones_abcd(F.ts, F.tp, a, b, c, d);
    a *= F.kappa; b *= F.kappa; c *= F.kappa; d *= F.kappa;
}
// Adjoint of jones_abcd: gradients (conjugate convention d/dRe + i d/dIm) of the amplitudes.
DEV void jones_abcd_vjp(cf as, cf ap, float ga, float gb, float gc, float gd, cf& g_as, cf& g_ap) {
    float gA = 0.5f * (ga + gb), gB = 0.5f * (ga - gb);
    cf gz{gc, gd}, gzc{gc, -gd};
    g_as = cadd(cscale(as, 2.0f * gA), cmul(gz, ap));
    g_ap = cadd(cscale(ap, 2.0f * gB), cmul(gzc, as));
}
// d(loss)/dm (conjugate convention) of the reflection entries; the amplitudes are holomorphic
// in m with d(m ct)/dm = 1/ct and d ct/dm = st2 / (m ct).
DEV cf fresnel_R_vjp(float ci, cf m, float ga, float gb, float gc, float gd) {
    Fres F;
    fresnel_amp(ci, m, F, false);
    cf g_rs, g_rp;
    jones_abcd_vjp(F.rs, F.rp, ga, gb, gc, gd, g_rs, g_rp);
    cf m2 = cmul(m, m);
    cf st2 = cdiv(cf{1.0f - ci * ci, 0.0f}, m2);
    cf u = cmul(m, F.ct), v = cscale(m, ci);
    cf cu = cadd(cf{ci, 0.0f}, u), cv = cadd(v, F.ct);
    cf drs = cdiv(cf{-2.0f * ci, 0.0f}, cmul(cmul(cu, cu), F.ct));
    cf drp = cdiv(cscale(csub(cmul(F.ct, F.ct), st2), 2.0f * ci), cmul(F.ct, cmul(cv, cv)));
    return cadd(cmul(g_rs, cconj(drs)), cmul(g_rp, cconj(drp)));
}
DEV cf fresnel_T_vjp(float ci, cf m, float ga, float gb, float gc, float gd) {
    Fres F;
    fresnel_amp(ci, m, F, true);
    float a, b, c, d;
    jones_abcd(F.ts, F.tp, a, b, c, d);
    float gk = ga * a + gb * b + gc * c + gd * d;
    cf g_ts, g_tp;
    jones_abcd_vjp(F.ts, F.tp, F.kappa * ga, F.kappa * gb, F.kappa * gc, F.kappa * gd, g_ts, g_tp);
    cf m2 = cmul(m, m);
    cf st2 = cdiv(cf{1.0f - ci * ci, 0.0f}, m2);
    cf u = cmul(m, F.ct), v = cscale(m, ci);
    cf cu = cadd(cf{ci, 0.0f}, u), cv = cadd(v, F.ct);
    cf dts = cdiv(cf{-2.0f * ci, 0.0f}, cmul(cmul(cu, cu), F.ct));
    cf dct = cdiv(st2, cmul(m, F.ct));
    cf dtp = cdiv(cscale(cadd(cf{ci, 0.0f}, dct), -2.0f * ci), cmul(cv, cv));
    cf du = cdiv(cf{1.0f, 0.0f}, F.ct);
    cf g = cadd(cmul(g_ts, cconj(dts)), cmul(g_tp, cconj(dtp)));
    return cadd(g, cscale(cconj(du), gk / ci));
}

// d(loss)/d ci of the reflection entries (a moving shading normal changes the incidence cosine):
// d ct/d ci = ci / (m^2 ct), drs/d ci = 2 (u - ci u') / (ci + u)^2 with u = m ct,
// drp/d ci = 2 m (ct - ci ct') / (m ci + ct)^2.
DEV float fresnel_R_dci(float ci, cf m, float ga, float gb, float gc, float gd) {
    Fres F;
    fresnel_amp(ci, m, F, false);
    cf g_rs, g_rp;
    jones_abcd_vjp(F.rs, F.rp, ga, gb, gc, gd, g_rs, g_rp);
    cf dct = cdiv(cf{ci, 0.0f}, cmul(cmul(m, m), F.ct));
    cf u = cmul(m, F.ct), du = cmul(m, dct);
    cf cu = cadd(cf{ci, 0.0f}, u), cv = cadd(cscale(m, ci), F.ct);
    cf drs = cdiv(cscale(csub(u, cscale(du, ci)), 2.0f), cmul(cu, cu));
    cf drp = cdiv(cmul(cscale(m, 2.0f), csub(F.ct, cscale(dct, ci))), cmul(cv, cv));
    return cmul(g_rs, cconj(drs)).re + cmul(g_rp, cconj(drp)).re;
}
// the same for the flux-form transmission entries kappa (a, b, c, d)(ts, tp), kappa = Re(m ct)/ci
DEV float fresnel_T_dci(float ci, cf m, float ga, float gb, float gc, float gd) {
    Fres F;
    fresnel_amp(ci, m, F, true);
    float a, b, c, d;
    jones_abcd(F.ts, F.tp, a, b, c, d);
    float gk = ga * a + gb * b + gc * c + gd * d;
    cf g_ts, g_tp;
    jones_abcd_vjp(F.ts, F.tp, F.kappa * ga, F.kappa * gb, F.kappa * gc, F.kappa * gd, g_ts, g_tp);
    cf dct = cdiv(cf{ci, 0.0f}, cmul(cmul(m, m), F.ct));
    cf u = cmul(m, F.ct), du = cmul(m, dct);
    cf cu = cadd(cf{ci, 0.0f}, u), cv = cadd(cscale(m, ci), F.ct);
    cf dts = cdiv(cscale(csub(u, cscale(du, ci)), 2.0f), cmul(cu, cu));
    cf dtp = cdiv(cscale(csub(F.ct, cscale(dct, ci)), 2.0f), cmul(cv, cv));
    float dkap = du.re / ci - u.re / (ci * ci);
    return cmul(g_ts, cconj(dts)).re + cmul(g_tp, cconj(dtp)).re + gk * dkap;
}

// ============================================================================ GGX
DEV float ggx_D(float ch, float a) {
    if (ch <= 0.0f) return 0.0f;
    float a2 = a * a, d = (a2 - 1.0f) * ch * ch + 1.0f;
    return a2 / (PI_F * d * d);
}
DEV float ggx_dlnD(float ch, float a) {
    float a2 = a * a, d = (a2 - 1.0f) * ch * ch + 1.0f;
    return 2.0f / a - 4.0f * a * ch * ch / d;
}
DEV float smith_G1(float cw, float a) {
    if (cw <= 0.0f) return 0.0f;
    float t2 = (1.0f - cw * cw) / (cw * cw);
    float s = sqrtf(1.0f + a * a * t2);
    return 1.0f / (1.0f + 0.5f * (s - 1.0f));
}
DEV float smith_dlnG1(float cw, float a) {
    float t2 = (1.0f - cw * cw) / (cw * cw);
    float s = sqrtf(1.0f + a * a * t2);
    float lam = 0.5f * (s - 1.0f);
    return -(a * t2 / (2.0f * s)) / (1.0f + lam);
}
// d ln D / d cos_h and d ln G1 / d cos_w (derivatives along a moving shading normal)
DEV float ggx_dlnD_dc(float ch, float a) {
    float a2 = a * a, d = (a2 - 1.0f) * ch * ch + 1.0f;
    return -4.0f * ch * (a2 - 1.0f) / d;
}
DEV float smith_dlnG1_dc(float cw, float a) {
    float t2 = (1.0f - cw * cw) / (cw * cw);
    float s = sqrtf(1.0f + a * a * t2);
    float lam = 0.5f * (s - 1.0f);
    return a * a / (2.0f * s * cw * cw * cw * (1.0f + lam));
}

// ============================================================================ scene access
// Parameter reads and gradient writes of one call.  Gradients go to a workgroup-local LDS
// accumulator when the slot has one (FP64 for small slots, FP32 for textures), else to the
// global FP64 accumulator.
// Reads of device global memory through global-address-space pointers: the loads are global
// (not flat) loads, whose completion the compiler does not have to wait for together with LDS.
#define PPT_GLOBAL __attribute__((address_space(1)))
template <class T>
DEV T gval(const T* p, size_t i) {
    static_assert(sizeof(T) % 4 == 0, "records of 32-bit words");
    T r;
    const PPT_GLOBAL uint32_t* src = (const PPT_GLOBAL uint32_t*)(p + i);
    uint32_t* dst = (uint32_t*)&r;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
    return r;
}

// the four texels of a bilinear lookup (element offsets) and their weights
struct Bilin { int i[4]; float w[4]; };

struct Call {
    const CallTable* tab;
    double* gacc;
    double* lds_d = nullptr;
    float* lds_f = nullptr;
    bool coherent = false;  // this lane's vertex is its path's first (texture scatters group such lanes)
    DEV float p(int slot, int idx) const { return gval(tab->p[slot], (size_t)idx); }
    // Bilinear scatter of CH channels: g[c] w_k to element off + B.i[k] + c of a slot.
    template <int CH>
    DEV void gb(int slot, int off, const Bilin& B, const float* g) const;
    DEV void g(int slot, int idx, float v) const {
        if (v == 0.0f) return;
        if (lds_d) {
            int o = tab->lds_d[slot];
            if (o >= 0) { atomicAdd(lds_d + o + idx, (double)v); return; }
            o = tab->lds_f[slot];
            if (o >= 0) { atomicAdd(lds_f + o + idx, v); return; }
        }
        int64_t o = tab->goff[slot];
        if (o >= 0) global_add(gacc + o + idx, v);
    }
    // FP64 global accumulation.  Lanes of the wavefront that add to the address of the first
    // active lane (neighbouring samples landing on the same texel) are summed through readlane
    // and added by one atomic; the other lanes add their own values.
    DEV static void global_add(double* a, float v) {
        const uint64_t ad = (uint64_t)a;
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)ad);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(ad >> 32));
        const bool lead = (uint32_t)ad == lo && (uint32_t)(ad >> 32) == hi;
        unsigned long long same = __ballot(lead);
        if (__popcll(same) < 4) { unsafeAtomicAdd(a, (double)v); return; }
        if (lead) {
            const int first = __ffsll((long long)same) - 1;
            float sum = 0.0f;
            while (same) {
                const int l = __ffsll((long long)same) - 1;
                sum += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
                same &= same - 1ull;
            }
            if ((int)lane_id() == first) unsafeAtomicAdd(a, (double)sum);
        } else {
            unsafeAtomicAdd(a, (double)v);
        }
    }
};

// Grouped bilinear scatter into the global accumulator: adds g[c] w_k to texel k, channel c, through
// add(k, c, value).  Among
// the lanes that flag themselves coherent (a path's first vertex: the samples of one pixel land in
// one or two texel cells), lanes whose four texels are the same (key: texel 0's address and the
// offsets of texels 1 and 3, which fix texel 2 = 0 + 3 - 1) are found group by group from the first
// pending lane; a group of at least GROUP_MIN lanes has its 4 CH values summed and added by one lane.
// Every other lane adds its own values.  (Textures in the workgroup accumulators keep per-lane LDS
// atomics: grouping there measured slower, the replay of the 128-view batch 6.3 -> 7.0 ms.)
constexpr int GROUP_MIN = 2, GROUP_ROUNDS = 8;
template <int CH, class Add>
DEV void bilin_grouped(uint64_t key, const Bilin& B, const float* g, bool coherent, Add add) {
    const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
    const int d1 = B.i[1] - B.i[0], d3 = B.i[3] - B.i[0];
    const uint64_t act = __ballot(1);
    bool pending = coherent, done = false;
#pragma unroll 1
    for (int r = 0; r < GROUP_ROUNDS; ++r) {
        const uint64_t pend = __ballot(pending);
        if (__popcll(pend) < GROUP_MIN) break;
        const int lead = __ffsll((long long)pend) - 1;
        const bool match = pending && klo == (uint32_t)__builtin_amdgcn_readlane((int)klo, lead) &&
                           khi == (uint32_t)__builtin_amdgcn_readlane((int)khi, lead) &&
                           d1 == __builtin_amdgcn_readlane(d1, lead) && d3 == __builtin_amdgcn_readlane(d3, lead);
        pending = pending && !match;
        if (__popcll(__ballot(match)) < GROUP_MIN) continue;
        done = done || match;
        // one channel at a time (four sums in flight keep the register count down)
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            float t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) t[k] = match ? g[c] * B.w[k] : 0.0f;
            wave_sum_active<4>(t, act);
            if ((int)lane_id() == lead) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (t[k] != 0.0f) add(k, c, t[k]);
            }
        }
    }
    if (!done) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const float v = g[c] * B.w[k];
                if (v != 0.0f) add(k, c, v);
            }
    }
}
template <int CH>
DEV void Call::gb(int slot, int off, const Bilin& B, const float* g) const {
    if (lds_d) {
        int o = tab->lds_d[slot];
        if (o >= 0) {
            double* a = lds_d + o + off;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const float v = g[c] * B.w[k];
                    if (v != 0.0f) atomicAdd(a + B.i[k] + c, (double)v);
                }
            return;
        }
        o = tab->lds_f[slot];
        if (o >= 0) {
            float* a = lds_f + o + off;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const float v = g[c] * B.w[k];
                    if (v != 0.0f) atomicAdd(a + B.i[k] + c, v);
                }
            return;
        }
    }
    const int64_t o = tab->goff[slot];
    if (o >= 0) {
        double* a = gacc + o + off;
        bilin_grouped<CH>((uint64_t)(a + B.i[0]), B, g, coherent,
                          [&](int k, int c, float v) { unsafeAtomicAdd(a + B.i[k] + c, (double)v); });
    }
}

// Per-vertex gradient of the parameters a vertex reads, combined over its next-event and
// continuation terms before it is scattered (one bilinear scatter per texture).
struct GradVtx {
    float rho[3], alpha, eta, kap, le[3], emit[3], ks;
    v3 gns;  // d(loss)/d(shading normal) of a normal-mapped vertex
    DEV void zero() {
        rho[0] = rho[1] = rho[2] = 0.0f; alpha = eta = kap = ks = 0.0f;
        le[0] = le[1] = le[2] = 0.0f; emit[0] = emit[1] = emit[2] = 0.0f;
        gns = mk(0.0f, 0.0f, 0.0f);
    }
};

// bilinear, clamp to edge, texel centres at (i + 1/2)/N, layout [th][tw][ch]
DEV void bilin(float u, float v, int tw, int th, int ch, Bilin& B) {
    float x = u * (float)tw - 0.5f, y = v * (float)th - 0.5f;
    float x0f = floorf(x), y0f = floorf(y);
    float fx = x - x0f, fy = y - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    int xa = min(max(x0, 0), tw - 1), xb = min(max(x0 + 1, 0), tw - 1);
    int ya = min(max(y0, 0), th - 1), yb = min(max(y0 + 1, 0), th - 1);
    B.i[0] = (ya * tw + xa) * ch; B.w[0] = (1.0f - fx) * (1.0f - fy);
    B.i[1] = (ya * tw + xb) * ch; B.w[1] = fx * (1.0f - fy);
    B.i[2] = (yb * tw + xa) * ch; B.w[2] = (1.0f - fx) * fy;
    B.i[3] = (yb * tw + xb) * ch; B.w[3] = fx * fy;
}
// The CH channels of the four texels of a bilinear lookup: every load is issued before any is used
// (one round trip; left to itself the register allocator chained them, one texel at a time), then
// out[c] = sum_k w_k t_kc in tap order.
template <int CH>
DEV void bilin_fetch(const Call& K, int slot, int off, const Bilin& B, float* out) {
    float t[4 * CH];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < CH; ++c) t[CH * k + c] = K.p(slot, off + B.i[k] + c);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        float r = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) r += t[CH * k + c] * B.w[k];
        out[c] = r;
    }
}
// the CH channels of a constant (tw = 0) or bilinear texture
template <int CH>
DEV void tex_read(const Call& K, int slot, int off, int tw, int th, float u, float v, float* out) {
    if (tw == 0) {
#pragma unroll
        for (int c = 0; c < CH; ++c) out[c] = K.p(slot, off + c);
        return;
    }
    Bilin B;
    bilin(u, v, tw, th, CH, B);
    bilin_fetch<CH>(K, slot, off, B, out);
}
DEV void albedo3(const Call& K, const DevMaterial& m, float u, float v, float* rho) {
    tex_read<3>(K, m.alb_slot, m.alb_off, m.alb_tw, m.alb_th, u, v, rho);
}
DEV void albedo_scatter(const Call& K, const DevMaterial& m, float u, float v, const float* g) {
    if (g[0] == 0.0f && g[1] == 0.0f && g[2] == 0.0f) return;
    if (m.alb_tw == 0) {
        for (int c = 0; c < 3; ++c) K.g(m.alb_slot, m.alb_off + c, g[c]);
        return;
    }
    Bilin B;
    bilin(u, v, m.alb_tw, m.alb_th, 3, B);
    K.gb<3>(m.alb_slot, m.alb_off, B, g);
}
// roughness, clamped to [1e-3, 1]; *inside tells whether the clamp is inactive
DEV float rough(const Call& K, const DevMaterial& m, float u, float v, bool* inside) {
    float a;
    tex_read<1>(K, m.alpha_slot, m.alpha_off, m.alpha_tw, m.alpha_th, u, v, &a);
    bool in = a >= 1e-3f && a <= 1.0f;
    if (inside) *inside = in;
    return fminf(fmaxf(a, 1e-3f), 1.0f);
}
DEV void rough_scatter(const Call& K, const DevMaterial& m, float u, float v, float g) {
    if (g == 0.0f) return;
    if (m.alpha_tw == 0) { K.g(m.alpha_slot, m.alpha_off, g); return; }
    Bilin B;
    bilin(u, v, m.alpha_tw, m.alpha_th, 1, B);
    K.gb<1>(m.alpha_slot, m.alpha_off, B, &g);
}
// the scatter of a constant or bilinear texture's gradient
template <int CH>
DEV void tex_scatter(const Call& K, int slot, int off, int tw, int th, float u, float v, const float* g) {
    if (tw == 0) {
#pragma unroll
        for (int c = 0; c < CH; ++c) K.g(slot, off + c, g[c]);
        return;
    }
    Bilin B;
    bilin(u, v, tw, th, CH, B);
    K.gb<CH>(slot, off, B, g);
}
// specular map: scale of the GGX lobe (1 without a map)
DEV float spec_scale(const Call& K, const DevMaterial& m, float u, float v) {
    if (m.spec_slot < 0) return 1.0f;
    float k;
    tex_read<1>(K, m.spec_slot, m.spec_off, m.spec_tw, m.spec_th, u, v, &k);
    return k;
}
DEV cf ior(const Call& K, const DevMaterial& m) {
    return cf{K.p(m.eta_slot, m.eta_off), m.kap_slot >= 0 ? K.p(m.kap_slot, m.kap_off) : 0.0f};
}

// ============================================================================ traversal
struct Hit { int prim; float t, u, v; };

// Scene arrays live in device global memory: reading them through global-address-space pointers
// gives global (not flat) loads, whose completion is not tied to the LDS traversal stack.
typedef float f32x4 __attribute__((ext_vector_type(4)));
DEV float4 ldg4(const float4* p, int i) {
    f32x4 v = ((const __attribute__((address_space(1))) f32x4*)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// The two halves of a word of a BVH node, widened to float.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
DEV float half_lo(float w) { return (float)__builtin_bit_cast(f16x2, w).x; }
DEV float half_hi(float w) { return (float)__builtin_bit_cast(f16x2, w).y; }

// Reciprocal direction for the slab tests, by the hardware reciprocal (1 ulp): the node boxes are
// rounded outward to half floats, a margin far wider than the reciprocal's error.
DEV v3 safe_inv(v3 d) {
    const float e = 1e-20f;
    return mk(__builtin_amdgcn_rcpf(fabsf(d.x) > e ? d.x : copysignf(e, d.x)),
              __builtin_amdgcn_rcpf(fabsf(d.y) > e ? d.y : copysignf(e, d.y)),
              __builtin_amdgcn_rcpf(fabsf(d.z) > e ? d.z : copysignf(e, d.z)));
}

// Intersection of primitive i (triangle or sphere) with the ray; accepted when 0 < t < tb, which
// then shrinks to t.
DEV bool hit_prim(const float4* prims, int i, v3 o, v3 d, float& tb, Hit& h) {
    const float4* pr = prims + 3 * i;
    // the kind is read from the third word, so all three are loaded at once (one round trip)
    const float4 A = ldg4(pr, 0), B = ldg4(pr, 1), C = ldg4(pr, 2);
    if (__float_as_int(C.w) == 0) {
        v3 v0 = mk(A.x, A.y, A.z), e1 = mk(B.x, B.y, B.z), e2 = mk(C.x, C.y, C.z);
        // every quantity is computed and one predicate decides (the same tests as early
        // rejections, without their branches)
        v3 p = cross(d, e2);
        float det = dot(e1, p);
        float inv = 1.0f / det;
        v3 s = o - v0;
        float uu = dot(s, p) * inv;
        v3 q = cross(s, e1);
        float vv = dot(d, q) * inv;
        float t = dot(e2, q) * inv;
        const bool ok = det != 0.0f && !(uu < 0.0f || uu > 1.0f) && !(vv < 0.0f || uu + vv > 1.0f) && t > 0.0f && t < tb;
        if (!ok) return false;
        tb = t; h.prim = i; h.t = t; h.u = uu; h.v = vv;
        return true;
    }
    v3 oc = o - mk(A.x, A.y, A.z);
    float r = B.x;
    float bb = dot(d, oc), cc = dot(oc, oc) - r * r;
    float disc = bb * bb - cc;
    if (disc < 0.0f) return false;
    float sq = sqrtf(disc);
    float t = -bb - sq;
    if (!(t > 0.0f)) t = -bb + sq;
    if (!(t > 0.0f && t < tb)) return false;
    tb = t; h.prim = i; h.t = t; h.u = 0.0f; h.v = 0.0f;
    return true;
}

// Resumable traversal state of one ray.  The stack lives in LDS, entry k at stack[(k + 2) * BLOCK]:
// two entries of padding below the bottom let the node step read the two top entries and write the
// next one at fixed offsets from one address.  The padding holds TRAV_DONE (trav_stack_init, once
// per lane; nothing writes it afterwards), so a pop below the bottom reads the end of traversal.
constexpr int TRAV_DONE = 0x7fffffff;
DEV void trav_stack_init(int* stack) { stack[0] = TRAV_DONE; stack[BLOCK] = TRAV_DONE; }
struct Trav {
    v3 o, d, id, ood;
    float tb;
    int ref;   // >= 0 inner node, < 0 leaf, TRAV_DONE when the stack is exhausted
    int leaf;  // parked leaf (< 0) or none
    int sp;
    Hit h;
    const float4* nodes;
    const float4* prims;
};
DEV void trav_begin(Trav& T, const DevWorld& W, v3 o, v3 d, float tmax) {
    T.o = o; T.d = d;
    T.id = safe_inv(d);
    T.ood = mk(o.x * T.id.x, o.y * T.id.y, o.z * T.id.z);
    T.tb = tmax;
    T.sp = 0;
    T.h.prim = -1; T.h.t = 0.0f; T.h.u = 0.0f; T.h.v = 0.0f;
    T.nodes = W.nodes;
    T.prims = W.prims;
    T.leaf = 0;
    T.ref = W.n_prims == 0 ? TRAV_DONE : W.root;
    if (T.ref < 0) { T.leaf = T.ref; T.ref = TRAV_DONE; }
}
// One round of while-while traversal with speculative leaf postponement (Aila & Laine 2009):
// the lanes of the wavefront in this call descend, a lane that reaches a leaf parks it and keeps
// descending until every such lane holds a leaf (or, with refill, until fewer than a quarter of
// the wavefront's lanes still descend), then the parked leaves are tested.  Returns true
// when the ray is finished: closest hit in T.h (any = false), or the first hit (any = true).
// CNT: count node visits and primitive tests into n_nodes, n_prims (their registers cost the
// kernel a wavefront per SIMD, so launches without work counters leave them out).
template <bool CNT>
DEV bool trav_round(Trav& T, bool any, uint32_t& n_nodes, uint32_t& n_prims, int* stack, bool refill) {
    while (T.ref != TRAV_DONE && T.ref >= 0) {
        if (CNT) ++n_nodes;
        // the two top stack entries, read while the node is in flight (below the bottom of the
        // stack the padding is read and not used)
        const int sp = T.sp;
        int* const sb = stack + sp * BLOCK;
        const int top1 = sb[BLOCK], top2 = sb[0];
        __builtin_amdgcn_sched_barrier(0);
        const float4* nd = T.nodes + 2 * T.ref;
        const float4 q0 = ldg4(nd, 0), q1 = ldg4(nd, 1);
        __builtin_amdgcn_sched_barrier(0);  // (keeps the stack reads ahead of the wait for the node)
        const v3 id = T.id, ood = T.ood;
        float a0 = fmaf(half_lo(q0.x), id.x, -ood.x), a1 = fmaf(half_hi(q0.x), id.x, -ood.x);
        float b0 = fmaf(half_lo(q0.y), id.y, -ood.y), b1 = fmaf(half_hi(q0.y), id.y, -ood.y);
        float c0 = fmaf(half_lo(q1.x), id.z, -ood.z), c1 = fmaf(half_hi(q1.x), id.z, -ood.z);
        float tnL = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), 0.0f));
        float txL = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), T.tb));
        float e0 = fmaf(half_lo(q0.z), id.x, -ood.x), e1 = fmaf(half_hi(q0.z), id.x, -ood.x);
        float f0 = fmaf(half_lo(q0.w), id.y, -ood.y), f1 = fmaf(half_hi(q0.w), id.y, -ood.y);
        float g0 = fmaf(half_lo(q1.y), id.z, -ood.z), g1 = fmaf(half_hi(q1.y), id.z, -ood.z);
        float tnR = fmaxf(fmaxf(fminf(e0, e1), fminf(f0, f1)), fmaxf(fminf(g0, g1), 0.0f));
        float txR = fminf(fminf(fmaxf(e0, e1), fmaxf(f0, f1)), fminf(fmaxf(g0, g1), T.tb));
        const bool hL = tnL <= txL, hR = tnR <= txR;
        const int rL = __float_as_int(q1.z), rR = __float_as_int(q1.w);
        // next reference, by selects: the nearer hit child (the farther one is pushed), else the
        // top of the stack; a leaf is parked (when none is) and the descent goes on past it.  The
        // two pops this can need were read above (pushing and at once popping the farther child
        // of a parked nearer leaf is skipped).
        const bool goR = hR & (!hL | (tnR < tnL));  // (bitwise: no branch)
        const int near = goR ? rR : rL, far = goR ? rL : rR;
        const bool both = hL && hR, none = !hL && !hR, free_slot = T.leaf == 0;
        const int pop1 = top1, pop2 = top2;  // (below the bottom: the padding, which holds TRAV_DONE)
        const bool park_near = !none && near < 0 && free_slot;
        const bool park_pop = none && pop1 < 0 && free_slot;
        const bool push = both && !park_near;
        // written whether or not it is pushed: entry sp is above the top unless this pushes, and it
        // is in the stack (at an inner node of depth d at most d entries are held, d < BVH depth,
        // and the capacity is the BVH depth + 2 entries, padding included)
        sb[2 * BLOCK] = far;
        int ref = park_near ? (both ? far : pop1) : near;
        ref = none ? (park_pop ? pop2 : pop1) : ref;
        T.ref = ref;
        T.leaf = park_near ? near : (park_pop ? pop1 : T.leaf);
        const int npop = none ? (park_pop ? 2 : 1) : (park_near && !both ? 1 : 0);
        T.sp = push ? sp + 1 : max(sp - npop, 0);
        // the round ends when every lane in this loop holds a leaf, or, while queued rays remain
        // (refill, wave-uniform), when fewer than a quarter of the wavefront's lanes still descend,
        // so that the finished lanes take new rays (thresholds of 1/8, 1/2 and 3/4, and no early
        // end, measured slower); one wave-uniform test
        const unsigned long long looping = __ballot(true), unparked = __ballot(T.leaf == 0);
        if (unparked == 0ull || (refill && (int)__builtin_popcountll(looping) < WAVE / 4)) break;
    }
    while (T.leaf < 0) {
        int enc = ~T.leaf;
        int first = enc >> 3, cnt = (enc & 7) + 1;
        for (int k = 0; k < cnt; ++k) {
            if (CNT) ++n_prims;
            if (hit_prim(T.prims, first + k, T.o, T.d, T.tb, T.h) && any) {
                T.leaf = 0;
                T.ref = TRAV_DONE;
                return true;
            }
        }
        T.leaf = 0;
        if (T.ref < 0) {  // the node loop stopped on a second leaf
            T.leaf = T.ref;
            T.ref = T.sp ? stack[(--T.sp + 2) * BLOCK] : TRAV_DONE;
        }
    }
    return T.ref == TRAV_DONE;
}

DEV float offset_eps(v3 p) { return 1e-4f * (1.0f + fmaxf(fmaxf(fabsf(p.x), fabsf(p.y)), fabsf(p.z))); }
DEV v3 spawn(v3 p, v3 ng, v3 dir) {
    float e = offset_eps(p);
    return p + ng * (dot(dir, ng) > 0.0f ? e : -e);
}

// ============================================================================ path vertices
struct Vtx {
    v3 p, ng, ns, wo, wi, wl;
    float u, v;
    int mat, orig, prim;  // prim: primitive record index (BVH order)
    bool tri, nmap;       // a triangle; its material has a normal map (ns comes from it)
    bool front, emit;
    int lobe, nee, light;
    float prob, pdf, nee_geom;
};

struct Sig {
    uint64_t h;
    DEV void add(uint32_t x) {
#pragma unroll
        for (int i = 0; i < 4; ++i) { h ^= (x >> (8 * i)) & 0xffu; h *= 1099511628211ull; }
    }
};

struct Counters { uint32_t nodes, prims, shadow, verts; };

DEV bool is_delta(int t) { return t == MAT_DIELECTRIC || t == MAT_SHEET; }

// Surface data of a hit (identical whether the hit comes from traversal or from a record).
DEV void surface(const DevWorld& W, const Hit& h, v3 o, v3 d, Vtx& x) {
    const float4* pr = W.prims + 3 * h.prim;
    // the kind is in the third word and the material in the second: one round trip for the record
    const float4 A = ldg4(pr, 0), B = ldg4(pr, 1), C = ldg4(pr, 2);
    x.orig = __float_as_int(A.w);
    x.prim = h.prim;
    x.mat = __float_as_int(B.w);
    x.tri = __float_as_int(C.w) == 0;
    if (x.tri) {
        v3 e1 = mk(B.x, B.y, B.z), e2 = mk(C.x, C.y, C.z);
        x.p = mk(A.x, A.y, A.z) + e1 * h.u + e2 * h.v;
        x.ng = normalize(cross(e1, e2));
        const float* t = W.tri_uv + 6 * (size_t)x.orig;
        float b0 = 1.0f - h.u - h.v;
        x.u = b0 * gval(t, 0) + h.u * gval(t, 2) + h.v * gval(t, 4);
        x.v = b0 * gval(t, 1) + h.u * gval(t, 3) + h.v * gval(t, 5);
    } else {
        x.p = o + d * h.t;
        v3 nout = normalize(x.p - mk(A.x, A.y, A.z));
        x.ng = B.x < 0.0f ? -nout : nout;
        x.u = 0.5f + atan2f(nout.z, nout.x) * (0.5f / PI_F);
        x.v = acosf(fminf(fmaxf(nout.y, -1.0f), 1.0f)) * (1.0f / PI_F);
    }
}

// Tangent frame of a triangle hit at its outward geometric normal ng: the tangent follows
// increasing u (dP/du of the triangle's uv map, made perpendicular to ng; the canonical basis of
// ng for a degenerate uv map), the bitangent is ng x tangent.
DEV void tangent_frame(const DevWorld& W, const Vtx& x, v3& tg, v3& bt) {
    const float4* pr = W.prims + 3 * x.prim;
    float4 Bq = ldg4(pr, 1), Cq = ldg4(pr, 2);
    v3 e1 = mk(Bq.x, Bq.y, Bq.z), e2 = mk(Cq.x, Cq.y, Cq.z);
    const float* t = W.tri_uv + 6 * (size_t)x.orig;
    float u0 = gval(t, 0), v0 = gval(t, 1);
    float du1 = gval(t, 2) - u0, dv1 = gval(t, 3) - v0, du2 = gval(t, 4) - u0, dv2 = gval(t, 5) - v0;
    float det = du1 * dv2 - du2 * dv1;
    v3 dpdu = (e1 * dv2 - e2 * dv1) * (det < 0.0f ? -1.0f : 1.0f);
    v3 tp = dpdu - x.ng * dot(dpdu, x.ng);
    float l = sqrtf(dot(tp, tp));
    if (det == 0.0f || !(l > 1e-6f * (sqrtf(dot(e1, e1)) + sqrtf(dot(e2, e2))))) {
        v3 yy;
        onb(x.ng, tg, yy);
    } else {
        tg = tp * (1.0f / l);
    }
    bt = cross(x.ng, tg);
}
// Normal-mapped shading normal toward the viewer side: the map's tangent-space components
// (t, b, n) give the outward normal normalize(t T + b B + n N).  il = +-1 / |t T + b B + n N|.
DEV v3 mapped_normal(const DevWorld& W, const Call& K, const DevMaterial& m, const Vtx& x, v3& tg, v3& bt, float& il) {
    tangent_frame(W, x, tg, bt);
    float c[3];
    tex_read<3>(K, m.nrm_slot, m.nrm_off, m.nrm_tw, m.nrm_th, x.u, x.v, c);
    v3 n = mk(c[0] * tg.x + c[1] * bt.x + c[2] * x.ng.x, c[0] * tg.y + c[1] * bt.y + c[2] * x.ng.y,
              c[0] * tg.z + c[1] * bt.z + c[2] * x.ng.z);
    il = 1.0f / sqrtf(dot(n, n));
    if (!x.front) il = -il;
    return n * il;
}

DEV int sample_glossy(v3 ns, v3 wo, float alpha, float u1, float u2, v3& wi, float& pdf) {
    float tan2 = alpha * alpha * u1 / (1.0f - u1);
    float ch = 1.0f / sqrtf(1.0f + tan2);
    float sh = sqrtf(fmaxf(0.0f, 1.0f - ch * ch));
    float ph = 2.0f * PI_F * u2;
    v3 tx, ty;
    onb(ns, tx, ty);
    v3 h = tx * (sh * cosf(ph)) + ty * (sh * sinf(ph)) + ns * ch;
    float woh = dot(wo, h);
    if (!(woh > 0.0f)) return LOBE_INVALID;
    wi = h * (2.0f * woh) - wo;
    if (!(dot(ns, wi) > 0.0f)) return LOBE_INVALID;
    pdf = ggx_D(ch, alpha) * ch / (4.0f * woh);
    return LOBE_GLOSSY;
}
DEV int sample_diffuse(v3 ns, float u1, float u2, v3& wi, float& pdf) {
    v3 tx, ty;
    onb(ns, tx, ty);
    float r = sqrtf(u1), ph = 2.0f * PI_F * u2;
    wi = tx * (r * cosf(ph)) + ty * (r * sinf(ph)) + ns * sqrtf(fmaxf(0.0f, 1.0f - u1));
    pdf = dot(ns, wi) * (1.0f / PI_F);
    return LOBE_DIFFUSE;
}

// Camera ray of (pixel, sample): jitter from bounce 0, call 0.
DEV void camera_ray(const DevView& V, int px, int py, uint32_t smp, uint64_t seed, v3& o, v3& d) {
    float u[4];
    uniforms(seed, (uint32_t)(py * V.width + px), smp, V.view_id, 0, 0, u);
    float sx = (2.0f * ((float)px + u[0]) / (float)V.width - 1.0f) * V.tan_h * V.aspect;
    float sy = (1.0f - 2.0f * ((float)py + u[1]) / (float)V.height) * V.tan_h;
    o = ld3(V.o);
    d = normalize(ld3(V.f) + ld3(V.r) * sx + ld3(V.u) * sy);
}

constexpr int NEE_NONE = 0, NEE_VISIBLE = 1, NEE_OCCLUDED = 2, NEE_ZERO = 3, NEE_PENDING = 4;

// Everything detached about vertex b (1-based) given the ray direction d that reached it:
// emission rule, the next-event light sample, the lobe choice and continuation direction.
// When the light sample needs a visibility test, x.nee = NEE_PENDING and (so, sd, stmax)
// describe the shadow ray; the caller resolves it (a shadow-ray kernel, or a recorded flag).
// EXT: the extended material features (normal maps, specular maps, circularly polarized
// emitters) are compiled in; kernels of scenes without them skip that code.
template <bool EXT>
DEV void vertex_setup(const DevWorld& W, const Call& K, uint32_t view_id, uint64_t seed, uint32_t pix, uint32_t smp,
                      int b, int max_depth, uint32_t flags, bool prev_delta, v3 d, Vtx& x, v3& so, v3& sd,
                      float& stmax) {
    const DevMaterial m = gval(W.mats, (size_t)x.mat);
    x.wo = -d;
    x.front = dot(x.ng, x.wo) > 0.0f;
    x.ns = x.front ? x.ng : -x.ng;
    const v3 ngf = x.ns;  // geometric normal on the viewer side
    x.nmap = EXT && m.nrm_slot >= 0 && x.tri;
    if (x.nmap) {
        v3 tg, bt;
        float il;
        x.ns = mapped_normal(W, K, m, x, tg, bt, il);
    }
    x.emit = m.emit_slot >= 0 && x.front && (b == 1 || prev_delta || (flags & FLAG_NO_NEE));
    x.lobe = LOBE_NONE;
    x.nee = NEE_NONE;
    x.prob = 1.0f; x.pdf = 1.0f; x.nee_geom = 0.0f; x.light = 0;
    if (m.type == MAT_EMITTER || b == max_depth) return;
    // a normal-mapped vertex seen from behind its shading normal neither scatters nor samples a light
    if (x.nmap && !(dot(x.ns, x.wo) > 0.0f)) {
        x.nee = NEE_ZERO;
        x.lobe = LOBE_INVALID;
        return;
    }
    float ua[4], ub[4];
    uniforms(seed, pix, smp, view_id, (uint32_t)b, 0, ua);
    uniforms(seed, pix, smp, view_id, (uint32_t)b, 1, ub);
    if (!is_delta(m.type) && !(flags & FLAG_NO_NEE) && W.n_lights > 0) {
        int nl = W.n_lights;
        int li = min((int)(ua[3] * (float)nl), nl - 1);
        const DevLight L = gval(W.lights, (size_t)li);
        v3 y = ld3(L.p0) + ld3(L.eu) * ub[0] + ld3(L.ev) * ub[1];
        v3 dv = y - x.p;
        float dist2 = dot(dv, dv), dist = sqrtf(dist2);
        x.wl = dv * (1.0f / dist);
        x.light = li;
        float cos_y = -dot(ld3(L.n), x.wl), cos_x = dot(x.ns, x.wl);
        // with a normal map the light must also lie above the geometric surface
        if (!(cos_y > 0.0f) || !(cos_x > 0.0f) || (x.nmap && !(dot(ngf, x.wl) > 0.0f))) {
            x.nee = NEE_ZERO;
        } else {
            so = spawn(x.p, x.ng, x.wl);
            v3 sv = y - so;
            float sl = sqrtf(dot(sv, sv));
            sd = sv * (1.0f / sl);
            stmax = sl - offset_eps(y);
            x.nee = NEE_PENDING;
            x.nee_geom = cos_y * L.area * (float)nl / dist2;
        }
    }
    switch (m.type) {
        case MAT_LAMBERT:
            x.lobe = sample_diffuse(x.ns, ua[1], ua[2], x.wi, x.pdf);
            break;
        case MAT_GGX_DIELECTRIC:
        case MAT_GGX_CONDUCTOR:
            x.lobe = sample_glossy(x.ns, x.wo, rough(K, m, x.u, x.v, nullptr), ua[1], ua[2], x.wi, x.pdf);
            break;
        case MAT_BLEND:
            if (ua[0] < m.blend) {
                x.lobe = sample_diffuse(x.ns, ua[1], ua[2], x.wi, x.pdf);
                x.prob = m.blend;
            } else {
                x.lobe = sample_glossy(x.ns, x.wo, rough(K, m, x.u, x.v, nullptr), ua[1], ua[2], x.wi, x.pdf);
                x.prob = 1.0f - m.blend;
            }
            break;
        case MAT_DIELECTRIC: {
            float eta = K.p(m.eta_slot, m.eta_off);
            float ecam = x.front ? 1.0f : eta, efar = x.front ? eta : 1.0f;
            float mr = efar / ecam;
            float co = dot(x.ns, x.wo);
            float st2 = (1.0f - co * co) / (mr * mr);
            float PR = 1.0f;
            if (st2 < 1.0f) {
                float a, bb, c, dd;
                fresnel_R(co, cf{mr, 0.0f}, a, bb, c, dd);
                PR = a;
            }
            if (ua[0] < PR) {
                x.wi = x.ns * (2.0f * co) - x.wo;
                x.prob = PR;
                x.lobe = LOBE_REFLECT;
            } else {
                float ct = sqrtf(1.0f - st2);
                x.wi = normalize((-x.wo) * (1.0f / mr) + x.ns * (co / mr - ct));
                x.prob = 1.0f - PR;
                x.lobe = LOBE_TRANSMIT;
            }
            break;
        }
        case MAT_SHEET:
            x.wi = -x.wo;
            x.lobe = LOBE_SHEET;
            break;
        default:
            x.lobe = LOBE_INVALID;
    }
    // with a normal map, a reflected direction must leave above the geometric surface and a
    // transmitted one below it
    if (x.nmap && x.lobe != LOBE_INVALID && x.lobe != LOBE_SHEET) {
        float side = dot(ngf, x.wi);
        if (x.lobe == LOBE_TRANSMIT ? !(side < 0.0f) : !(side > 0.0f)) x.lobe = LOBE_INVALID;
    }
}

// ============================================================================ Mueller weights
// Compact sample weight: W_c = rgb_c * (kind 1: E00 | kind 2: Rout * F(A,B,C,D) * Rin),
// F = [[A,B,0,0],[B,A,0,0],[0,0,C,D],[0,0,-D,C]], R = rotator (cos 2phi, sin 2phi).
struct WC {
    float rgb[3];
    float A, B, C, D;
    float ci, si, co, so;
    int kind;  // 0 zero, 1 diffuse, 2 Fresnel form
};
DEV void w_apply(const WC& w, int c, const float* in, float* out) {
    if (w.kind == 0) { out[0] = out[1] = out[2] = out[3] = 0.0f; return; }
    if (w.kind == 1) { out[0] = w.rgb[c] * in[0]; out[1] = out[2] = out[3] = 0.0f; return; }
    float v1 = w.ci * in[1] + w.si * in[2], v2 = -w.si * in[1] + w.ci * in[2];
    float f0 = w.A * in[0] + w.B * v1, f1 = w.B * in[0] + w.A * v1;
    float f2 = w.C * v2 + w.D * in[3], f3 = -w.D * v2 + w.C * in[3];
    float s = w.rgb[c];
    out[0] = s * f0;
    out[1] = s * (w.co * f1 + w.so * f2);
    out[2] = s * (-w.so * f1 + w.co * f2);
    out[3] = s * f3;
}
DEV void w_row(const WC& w, int c, const float* a, float* out) {
    if (w.kind == 0) { out[0] = out[1] = out[2] = out[3] = 0.0f; return; }
    if (w.kind == 1) { out[0] = w.rgb[c] * a[0]; out[1] = out[2] = out[3] = 0.0f; return; }
    float r1 = w.co * a[1] - w.so * a[2], r2 = w.so * a[1] + w.co * a[2];
    float g0 = w.A * a[0] + w.B * r1, g1 = w.B * a[0] + w.A * r1;
    float g2 = w.C * r2 - w.D * a[3], g3 = w.D * r2 + w.C * a[3];
    float s = w.rgb[c];
    out[0] = s * g0;
    out[1] = s * (w.ci * g1 - w.si * g2);
    out[2] = s * (w.si * g1 + w.ci * g2);
    out[3] = s * g3;
}
// Local-frame adjoint of the Fresnel-form entries: gA..gD = sum_c of a_c^T (dW) L_c terms.
DEV void w_local_grad(const WC& w, const float* a, const float* L, float& gA, float& gB, float& gC, float& gD) {
    gA = gB = gC = gD = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float* ac = a + 4 * c;
        const float* Lc = L + 4 * c;
        float r1 = w.co * ac[1] - w.so * ac[2], r2 = w.so * ac[1] + w.co * ac[2];  // a R_out
        float l1 = w.ci * Lc[1] + w.si * Lc[2], l2 = -w.si * Lc[1] + w.ci * Lc[2];  // R_in L
        float s = w.rgb[c];
        gA += s * (ac[0] * Lc[0] + r1 * l1);
        gB += s * (ac[0] * l1 + r1 * Lc[0]);
        gC += s * (r2 * l2 + ac[3] * Lc[3]);
        gD += s * (r2 * Lc[3] - ac[3] * l2);
    }
}
// The same for a general adjoint W̄_c of every channel's weight (Wbar: 3 row-major 4x4 blocks, the
// adjoint a conventional reverse sweep carries): gA..gD = sum_c s_c of the entries of
// G_c = R_out^T Wbar_c R_in^T that multiply A, B, C, D in F.
DEV void w_local_grad_full(const WC& w, const float* Wbar, float& gA, float& gB, float& gC, float& gD) {
    gA = gB = gC = gD = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float* M = Wbar + 16 * c;
        // rows 1, 2 mixed by R_out^T, then columns 1, 2 by R_in^T
        float T[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T[j] = M[j];
            T[4 + j] = w.co * M[4 + j] - w.so * M[8 + j];
            T[8 + j] = w.so * M[4 + j] + w.co * M[8 + j];
            T[12 + j] = M[12 + j];
        }
        float G[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            G[4 * i] = T[4 * i];
            G[4 * i + 1] = w.ci * T[4 * i + 1] + w.si * T[4 * i + 2];
            G[4 * i + 2] = -w.si * T[4 * i + 1] + w.ci * T[4 * i + 2];
            G[4 * i + 3] = T[4 * i + 3];
        }
        const float s = w.rgb[c];
        gA += s * (G[0] + G[5]);
        gB += s * (G[1] + G[4]);
        gC += s * (G[10] + G[15]);
        gD += s * (G[11] - G[14]);
    }
}

// frames of a specular event with incident propagation k_in, incident-side normal n_inc, output k_out
DEV void spec_frames(v3 k_in, v3 n_inc, v3 k_out, WC& w) {
    v3 s = s_axis(k_in, n_inc);
    rot_cs(k_in, canon_x(k_in), s, w.ci, w.si);
    rot_cs(k_out, s, canon_x(k_out), w.co, w.so);
}

// GGX microfacet pBRDF for light arriving along -wi and leaving along wo: frames, local
// Fresnel entries (unscaled) and kappa = D G / (4 cos_i cos_o).
struct GGXv { WC w; float a, b, c, d, kappa, ih, ci, co, ch, alpha; bool in; };
DEV void ggx_eval(const Call& K, const DevMaterial& m, const Vtx& x, v3 wi, cf eta, GGXv& g) {
    v3 h = normalize(wi + x.wo);
    g.ci = dot(x.ns, wi); g.co = dot(x.ns, x.wo); g.ch = dot(x.ns, h);
    g.ih = fabsf(dot(wi, h));
    g.alpha = rough(K, m, x.u, x.v, &g.in);
    float D = ggx_D(g.ch, g.alpha);
    float G = smith_G1(g.ci, g.alpha) * smith_G1(g.co, g.alpha);
    g.kappa = D * G / (4.0f * g.ci * g.co);
    fresnel_R(g.ih, eta, g.a, g.b, g.c, g.d);
    spec_frames(-wi, h, x.wo, g.w);
    g.w.rgb[0] = g.w.rgb[1] = g.w.rgb[2] = 1.0f;
    g.w.kind = 2;
}
// Gradient of a GGX lobe with entries s ks kappa (a, b, c, d) whose local adjoints are gA..gD
// (ks the specular-map scale).  Returns d(loss)/d ln kappa for the shading-normal chain.
DEV float ggx_backprop(const Vtx& x, cf eta, const GGXv& g, float s, float ks, float gA, float gB, float gC, float gD,
                       GradVtx& gv) {
    float q = s * (g.a * gA + g.b * gB + g.c * gC + g.d * gD);  // d/d(ks kappa)
    float jk = q * ks * g.kappa;
    gv.ks += q * g.kappa;
    if (g.in && g.kappa != 0.0f) {
        float dln = ggx_dlnD(g.ch, g.alpha) + smith_dlnG1(g.ci, g.alpha) + smith_dlnG1(g.co, g.alpha);
        gv.alpha += jk * dln;
    }
    float sk = s * ks * g.kappa;
    cf gm = fresnel_R_vjp(g.ih, eta, sk * gA, sk * gB, sk * gC, sk * gD);
    gv.eta += gm.re;
    gv.kap += gm.im;
    return jk;
}
// d ln(kappa cos_i) / d ns of a GGX lobe for light arriving along -wi (the 1/cos_i inside kappa
// cancels the cosine factor of the weight): D through cos_h, G1 through cos_i and cos_o, 1/cos_o
DEV v3 ggx_dln_dns(const GGXv& g, v3 wi, v3 wo) {
    v3 h = normalize(wi + wo);
    return h * ggx_dlnD_dc(g.ch, g.alpha) + wi * smith_dlnG1_dc(g.ci, g.alpha) +
           wo * (smith_dlnG1_dc(g.co, g.alpha) - 1.0f / g.co);
}
// d(loss)/d of the rotator entries (ci, si, co, so) of a Fresnel-form weight: sum_c a_c^T W_c L_c
DEV void w_frame_grad(const WC& w, const float* a, const float* L, float& gci, float& gsi, float& gco, float& gso) {
    gci = gsi = gco = gso = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float* ac = a + 4 * c;
        const float* Lc = L + 4 * c;
        float s = w.rgb[c];
        float v1 = w.ci * Lc[1] + w.si * Lc[2], v2 = -w.si * Lc[1] + w.ci * Lc[2];
        float f1 = w.B * Lc[0] + w.A * v1, f2 = w.C * v2 + w.D * Lc[3];
        float r1 = w.co * ac[1] - w.so * ac[2], r2 = w.so * ac[1] + w.co * ac[2];
        gco += s * (ac[1] * f1 + ac[2] * f2);
        gso += s * (ac[1] * f2 - ac[2] * f1);
        float d1 = s * (ac[0] * w.B + r1 * w.A), d2 = s * (r2 * w.C - ac[3] * w.D);
        gci += d1 * Lc[1] + d2 * Lc[2];
        gsi += d1 * Lc[2] - d2 * Lc[1];
    }
}
// d(loss)/d n_inc through the two rotators of a specular event (spec_frames), given the adjoints
// of their entries: c = x_from . s, sn = (k x x_from) . s, (C, S) = (c^2 - sn^2, 2 c sn), and
// s = normalize(k_in x n_inc)
DEV v3 spec_frames_grad(v3 k_in, v3 n_inc, v3 k_out, float gci, float gsi, float gco, float gso) {
    v3 sr = cross(k_in, n_inc);
    float l2 = dot(sr, sr);
    if (l2 < 1e-16f) return mk(0.0f, 0.0f, 0.0f);  // normal incidence: the axis is fixed
    float il = 1.0f / sqrtf(l2);
    v3 s = sr * il;
    v3 xi = canon_x(k_in), yi = cross(k_in, xi);
    float c1 = dot(xi, s), s1 = dot(yi, s);
    v3 gs = xi * (2.0f * (c1 * gci + s1 * gsi)) + yi * (2.0f * (c1 * gsi - s1 * gci));
    v3 xo = canon_x(k_out), yo = cross(xo, k_out);
    float c2 = dot(s, xo), s2 = dot(s, yo);
    gs = gs + xo * (2.0f * (c2 * gco + s2 * gso)) + yo * (2.0f * (c2 * gso - s2 * gco));
    v3 gsr = (gs - s * dot(s, gs)) * il;
    return cross(gsr, k_in);
}

// W_b and E_b of a vertex (values), and with GRAD their vector-Jacobian products against the
// adjoint rows a (3 x 4, canonical frame of wo) and the cached suffix Ln (3 x 4, frame of -wi):
// d(sum_c a_c . (E_c + W_c Ln_c)) / d params, accumulated through Call.
// Eemit receives the emission of the vertex and Enee the next-event part (computed when the
// light sample is visible or still pending).  Emitters radiate Le (1, 0, 0, circ).  With a
// normal map the shading normal x.ns is differentiated too: every cosine, the GGX D and G
// terms, the dielectric's Fresnel incidence cosine and its s/p frames.  EXT: the extended
// material features are compiled in (without them: no circular emission, no maps).
// FULL (conventional reverse sweep, scenes without the light-stage features): Ln is the general
// adjoint of the weight, 3 row-major 4x4 blocks, instead of the suffix whose outer product with a
// gives it.
template <bool GRAD, bool EXT, bool FULL = false>
DEV void eval_vertex(const DevWorld& W, const Call& K, const Vtx& x, WC& w, float* Eemit, float* Enee, const float* a,
                     const float* Ln) {
    static_assert(!(FULL && EXT), "the general weight adjoint is not implemented with the light-stage features");
    const DevMaterial m = gval(W.mats, (size_t)x.mat);
    const bool nm = EXT && x.nmap;
#pragma unroll
    for (int i = 0; i < 12; ++i) { Eemit[i] = 0.0f; Enee[i] = 0.0f; }
    GradVtx gv;
    if (GRAD) gv.zero();
    w.kind = 0;
    if (x.emit) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float le = K.p(m.emit_slot, m.emit_off + c);
            Eemit[4 * c] = le;
            if (EXT) Eemit[4 * c + 3] = le * m.emit_circ;
            if (GRAD) gv.emit[c] += EXT ? a[4 * c] + m.emit_circ * a[4 * c + 3] : a[4 * c];
        }
    }
    // next-event estimation: E_c += f_c (e0 + circ e3) * cos_x * geom * Le_c
    if (x.nee == NEE_VISIBLE || x.nee == NEE_PENDING) {
        const DevLight L = gval(W.lights, (size_t)x.light);
        float cx = dot(x.ns, x.wl);
        float gs = cx * x.nee_geom;
        float le[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) le[c] = K.p(L.le_slot, L.le_off + c);
        float wd = 0.0f, wg = 0.0f;
        if (m.type == MAT_LAMBERT) wd = 1.0f;
        else if (m.type == MAT_BLEND) { wd = m.blend; wg = 1.0f - m.blend; }
        else if (m.type == MAT_GGX_DIELECTRIC || m.type == MAT_GGX_CONDUCTOR) wg = 1.0f;
        if (wd != 0.0f) {
            float jl = 0.0f;  // this term's share of the loss (linear in cos_x)
            float rho3[3];
            albedo3(K, m, x.u, x.v, rho3);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float rho = rho3[c];
                Enee[4 * c] += wd * rho * (1.0f / PI_F) * gs * le[c];
                if (GRAD) {
                    gv.rho[c] += a[4 * c] * wd * gs * le[c] * (1.0f / PI_F);
                    gv.le[c] += a[4 * c] * wd * rho * gs * (1.0f / PI_F);
                    jl += a[4 * c] * wd * rho * gs * le[c] * (1.0f / PI_F);
                }
            }
            if (GRAD && nm) gv.gns = gv.gns + x.wl * (jl / cx);
        }
        if (wg != 0.0f) {
            bool real_ior = m.type != MAT_GGX_CONDUCTOR;
            cf eta = real_ior ? cf{K.p(m.eta_slot, m.eta_off), 0.0f} : ior(K, m);
            GGXv g;
            ggx_eval(K, m, x, x.wl, eta, g);
            const float ks = EXT ? spec_scale(K, m, x.u, x.v) : 1.0f, kk = g.kappa * ks;
            const float circ = EXT ? L.circ : 0.0f;
            // columns 0 and 3 of Rout F Rin: kappa (a, Cout b, -Sout b, 0) and kappa (0, Sout d, Cout d, c)
            float col[4] = {kk * g.a, kk * g.w.co * g.b, -kk * g.w.so * g.b, 0.0f};
            if (EXT) {
                col[1] += kk * circ * g.w.so * g.d;
                col[2] += kk * circ * g.w.co * g.d;
                col[3] = kk * circ * g.c;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float s = wg * gs * le[c];
                Enee[4 * c] += s * col[0]; Enee[4 * c + 1] += s * col[1]; Enee[4 * c + 2] += s * col[2];
                if (EXT) Enee[4 * c + 3] += s * col[3];
            }
            if (GRAD && !EXT) {
                float qa = 0.0f, qb = 0.0f;  // sum_c s_c (a_c0) and sum_c s_c (a_c1 Cout - a_c2 Sout)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float q = a[4 * c], r = a[4 * c + 1] * g.w.co - a[4 * c + 2] * g.w.so;
                    float s = wg * gs * le[c];
                    qa += s * q; qb += s * r;
                    gv.le[c] += wg * gs * g.kappa * (q * g.a + r * g.b);
                }
                ggx_backprop(x, eta, g, 1.0f, 1.0f, qa, qb, 0.0f, 0.0f, gv);
            }
            if (GRAD && EXT) {
                float Lv[12];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float s = wg * gs * le[c];
                    Lv[4 * c] = s; Lv[4 * c + 1] = 0.0f; Lv[4 * c + 2] = 0.0f; Lv[4 * c + 3] = circ * s;
                    gv.le[c] += wg * gs * (a[4 * c] * col[0] + a[4 * c + 1] * col[1] + a[4 * c + 2] * col[2] +
                                           a[4 * c + 3] * col[3]);
                }
                float gA, gB, gC, gD;
                w_local_grad(g.w, a, Lv, gA, gB, gC, gD);
                float jk = ggx_backprop(x, eta, g, 1.0f, ks, gA, gB, gC, gD, gv);
                if (nm && jk != 0.0f) gv.gns = gv.gns + ggx_dln_dns(g, x.wl, x.wo) * jk;
            }
        }
    }
    // continuation weight W = f cos / (pdf * lobe probability), both detached
    switch (x.lobe) {
        case LOBE_DIFFUSE: {
            w.kind = 1;
            float jw = 0.0f;
            albedo3(K, m, x.u, x.v, w.rgb);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (GRAD && FULL) gv.rho[c] += Ln[16 * c];
                if (GRAD && !FULL) {
                    gv.rho[c] += a[4 * c] * Ln[4 * c];
                    jw += a[4 * c] * w.rgb[c] * Ln[4 * c];
                }
            }
            // the weight is rho cos_i / (pi pdf) with the pdf detached: linear in cos_i
            if (GRAD && nm) gv.gns = gv.gns + x.wi * (jw / dot(x.ns, x.wi));
            w.A = w.B = w.C = w.D = 0.0f; w.ci = w.co = 1.0f; w.si = w.so = 0.0f;
            break;
        }
        case LOBE_GLOSSY: {
            bool real_ior = m.type != MAT_GGX_CONDUCTOR;
            cf eta = real_ior ? cf{K.p(m.eta_slot, m.eta_off), 0.0f} : ior(K, m);
            GGXv g;
            ggx_eval(K, m, x, x.wi, eta, g);
            const float ks = EXT ? spec_scale(K, m, x.u, x.v) : 1.0f;
            float s = g.ci / x.pdf;  // f cos / pdf; the selected lobe's weight equals its probability
            float k = g.kappa * s * ks;
            w = g.w;
            w.A = k * g.a; w.B = k * g.b; w.C = k * g.c; w.D = k * g.d;
            if (GRAD) {
                float gA, gB, gC, gD;
                if (FULL) w_local_grad_full(w, Ln, gA, gB, gC, gD);
                else w_local_grad(w, a, Ln, gA, gB, gC, gD);
                float jk = ggx_backprop(x, eta, g, s, ks, gA, gB, gC, gD, gv);
                if (nm && jk != 0.0f) gv.gns = gv.gns + ggx_dln_dns(g, x.wi, x.wo) * jk;
            }
            break;
        }
        case LOBE_REFLECT:
        case LOBE_TRANSMIT: {
            float eta = K.p(m.eta_slot, m.eta_off);
            float ecam = x.front ? 1.0f : eta, efar = x.front ? eta : 1.0f;
            float a0, b0, c0, d0, ci;
            cf mm;
            const bool refl = x.lobe == LOBE_REFLECT;
            const v3 n_inc = refl ? x.ns : -x.ns;
            if (refl) {
                ci = dot(x.ns, x.wo);
                mm = cf{efar / ecam, 0.0f};
                fresnel_R(ci, mm, a0, b0, c0, d0);
            } else {
                ci = fabsf(dot(x.wi, x.ns));
                mm = cf{ecam / efar, 0.0f};
                fresnel_T(ci, mm, a0, b0, c0, d0);
            }
            spec_frames(-x.wi, n_inc, x.wo, w);
            float ip = 1.0f / x.prob;
            w.kind = 2;
            w.rgb[0] = w.rgb[1] = w.rgb[2] = 1.0f;
            w.A = a0 * ip; w.B = b0 * ip; w.C = c0 * ip; w.D = d0 * ip;
            if (GRAD) {
                float gA, gB, gC, gD;
                if (FULL) w_local_grad_full(w, Ln, gA, gB, gC, gD);
                else w_local_grad(w, a, Ln, gA, gB, gC, gD);
                cf gm = refl ? fresnel_R_vjp(ci, mm, gA * ip, gB * ip, gC * ip, gD * ip)
                             : fresnel_T_vjp(ci, mm, gA * ip, gB * ip, gC * ip, gD * ip);
                // m = eta (camera outside, reflection) or 1/eta, and the reverse for transmission
                bool m_is_eta = refl == x.front;
                gv.eta += m_is_eta ? gm.re : -gm.re / (eta * eta);
                if (nm) {
                    // incidence cosine: wo . ns (reflection) or |wi . ns| (transmission)
                    float gci = refl ? fresnel_R_dci(ci, mm, gA * ip, gB * ip, gC * ip, gD * ip)
                                     : fresnel_T_dci(ci, mm, gA * ip, gB * ip, gC * ip, gD * ip);
                    v3 dci = refl ? x.wo : (dot(x.wi, x.ns) < 0.0f ? -x.wi : x.wi);
                    float g1, g2, g3, g4;
                    w_frame_grad(w, a, Ln, g1, g2, g3, g4);
                    v3 gn = spec_frames_grad(-x.wi, n_inc, x.wo, g1, g2, g3, g4);
                    gv.gns = gv.gns + dci * gci + (refl ? gn : -gn);
                }
            }
            break;
        }
        case LOBE_SHEET: {
            v3 k = x.wo;
            v3 t = mk(m.axis[0], m.axis[1], m.axis[2]);
            v3 xt = normalize(t - k * dot(t, k));
            rot_cs(k, canon_x(k), xt, w.ci, w.si);
            rot_cs(k, xt, canon_x(k), w.co, w.so);
            w.kind = 2;
            w.rgb[0] = w.rgb[1] = w.rgb[2] = 1.0f;
            w.A = w.B = 0.5f; w.C = w.D = 0.0f;
            break;
        }
        default:
            break;
    }
    if (GRAD) {
        // one scatter per parameter the vertex read (the single values first, so that fewer
        // values stay live across the texture scatters)
        if (m.eta_slot >= 0) K.g(m.eta_slot, m.eta_off, gv.eta);
        if (m.kap_slot >= 0) K.g(m.kap_slot, m.kap_off, gv.kap);
        if (x.nee == NEE_VISIBLE || x.nee == NEE_PENDING) {
            const DevLight L = gval(W.lights, (size_t)x.light);
            for (int c = 0; c < 3; ++c) K.g(L.le_slot, L.le_off + c, gv.le[c]);
        }
        if (m.emit_slot >= 0)
            for (int c = 0; c < 3; ++c) K.g(m.emit_slot, m.emit_off + c, gv.emit[c]);
        albedo_scatter(K, m, x.u, x.v, gv.rho);
        if (m.alpha_slot >= 0) rough_scatter(K, m, x.u, x.v, gv.alpha);
        if (EXT && m.spec_slot >= 0 && gv.ks != 0.0f)
            tex_scatter<1>(K, m.spec_slot, m.spec_off, m.spec_tw, m.spec_th, x.u, x.v, &gv.ks);
        if (nm) {
            // ns = il (t T + b B + n N): d/d(t, b, n) = (T, B, N) . il (I - ns ns^T) g
            v3 tg, bt;
            float il;
            mapped_normal(W, K, m, x, tg, bt, il);
            v3 gr = (gv.gns - x.ns * dot(x.ns, gv.gns)) * il;
            float gt[3] = {dot(tg, gr), dot(bt, gr), dot(x.ng, gr)};
            if (gt[0] != 0.0f || gt[1] != 0.0f || gt[2] != 0.0f)
                tex_scatter<3>(K, m.nrm_slot, m.nrm_off, m.nrm_tw, m.nrm_th, x.u, x.v, gt);
        }
    }
}

// ============================================================================ sensor
// analyzer a applied to a sensor-frame Stokes vector
DEV void analyzer_apply(int sensor, float theta, int a, const float* v, float* o) {
    if (sensor == SENSOR_NONE) { o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3]; return; }
    float C, S, q;
    if (sensor == SENSOR_POLARIZER) {
        C = cosf(2.0f * theta); S = sinf(2.0f * theta);
        q = 0.5f * (v[0] + C * v[1] + S * v[2]);
    } else if (a == 0) { C = 1.0f; S = 0.0f; q = 0.5f * (v[0] + v[1]); }
    else if (a == 1) { C = 0.0f; S = 1.0f; q = 0.5f * (v[0] + v[2]); }
    else if (a == 2) { C = -1.0f; S = 0.0f; q = 0.5f * (v[0] - v[1]); }
    else if (sensor == SENSOR_ANALYZER4) { C = 0.0f; S = 1.0f; q = 0.5f * (v[0] + v[3]); }  // QWP(0), polarizer at 45 deg
    else { C = 0.0f; S = -1.0f; q = 0.5f * (v[0] - v[3]); }  // QWP(0), polarizer at -45 deg: left-circular
    o[0] = q; o[1] = C * q; o[2] = S * q; o[3] = 0.0f;
}
// row delta^T A_a
DEV void analyzer_row(int sensor, float theta, int a, const float* dl, float* r) {
    if (sensor == SENSOR_NONE) { r[0] = dl[0]; r[1] = dl[1]; r[2] = dl[2]; r[3] = dl[3]; return; }
    float C, S;
    int kind = 0;
    if (sensor == SENSOR_POLARIZER) { C = cosf(2.0f * theta); S = sinf(2.0f * theta); }
    else if (a == 0) { C = 1.0f; S = 0.0f; }
    else if (a == 1) { C = 0.0f; S = 1.0f; }
    else if (a == 2) { C = -1.0f; S = 0.0f; }
    else { C = 0.0f; S = sensor == SENSOR_ANALYZER4 ? 1.0f : -1.0f; kind = 1; }
    float q = 0.5f * (dl[0] + C * dl[1] + S * dl[2]);  // output = w q(v), w = (1, C, S, 0)
    if (kind == 0) { r[0] = q; r[1] = C * q; r[2] = S * q; r[3] = 0.0f; }
    else { r[0] = q; r[1] = 0.0f; r[2] = 0.0f; r[3] = S * q; }  // circular analyzers: q(v) = (v0 + S v3) / 2
}
// delta^T (dP(theta)/dtheta) v
DEV float polarizer_dtheta(float theta, const float* dl, const float* v) {
    float C = cosf(2.0f * theta), S = sinf(2.0f * theta);
    float r0 = -S * dl[1] + C * dl[2];
    float r1 = -S * dl[0] - 2.0f * C * S * dl[1] + (C * C - S * S) * dl[2];
    float r2 = C * dl[0] + (C * C - S * S) * dl[1] + 2.0f * C * S * dl[2];
    return r0 * v[0] + r1 * v[1] + r2 * v[2];
}


}  // namespace ppt
