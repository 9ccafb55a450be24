// ppt_oracle.cpp -- plain, slow FP64 CPU oracle for differentiable polarized path tracing.
//
// TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the smoke check
// and by the CPU-baseline leg of the benchmark; the GPU library never links, loads or calls
// it, and it shares no code with the GPU path.  Everything is double precision.
//
// What it computes (paper, Sec. 3-4):
//   * the Monte Carlo image of Sec. 3.1 (rendering equation, Eq. 2) in Mueller-Stokes
//     calculus (Sec. 3.3): per path, per RGB channel c,
//        C = S(theta) * sum_b beta_b E_b,   beta_1 = I, beta_{b+1} = beta_b W_b,
//     W_b the 4x4 Mueller sample weight at vertex b and E_b the emitted + next-event Stokes
//     vector leaving vertex b; the pixel is the mean over its samples;
//   * the reverse-mode gradient of that estimator with the sampled path frozen (detached
//     sampling: positions, directions, lobe choices, pdfs and probabilities are constants;
//     only Mueller/BSDF values, emission and the sensor Mueller are differentiated, as in
//     the PRB adjoint of Sec. 3.2) in three independent ways:
//       mode 1  conventional AD: one stored tape over the whole path (the "Conv. AD"
//               reference of Sec. 5.1);
//       mode 2  cached suffix replay (Sec. 4.3, Fig. 2): primal records per-vertex W_b and
//               E_b, a backward fold builds the suffix radiance L[b] = E_b + W_b L[b+1], and
//               the adjoint replay differentiates each vertex locally against the cached
//               L[b+1] -- automatic differentiation only inside the loop body (Sec. 3.2);
//       mode 3  basic polarized PRB (Sec. 4.1, Alg. 2): the suffix is recovered by inverting
//               the sampled Mueller weight; the negative control the paper describes for
//               rank-deficient operators, and with sigma > 0 the noise-regularised P-PRB
//               comparator (Sec. 4.2): every weight becomes W_b + u_b I, u_b ~ N(0, sigma) drawn
//               per vertex from the path's counters, in the primal fold, the inversion and the
//               adjoint (an unbiased estimator of the same gradient, with its own variance);
//       mode 5  polarized radiative backpropagation (P-RB), the other comparator of Sec. 5.1:
//               the replay's suffix beyond each vertex is an independent estimate, a new path
//               traced from the ray leaving the vertex under a key of its own (unbiased, with the
//               variance of that estimate and the cost of one more path per vertex);
//       mode 4  hybrid cached replay (Sec. 4.4, Eq. 3) with checkpoint interval k: only the
//               suffix values at vertices 0, k, 2k, ... are kept.  Inside a block the replay
//               tracks the detached block throughput beta (the product of the weights since the
//               block's checkpoint) and the radiance the block has not yet emitted; any other
//               suffix is recovered by Eq. 3's rule: the scalar PRB update when the
//               depolarization index DI(beta) is below gamma, the inverse of beta applied to the
//               remaining radiance when |det beta| > eps beta_00^4, else recomputation of the
//               vertices up to the next checkpoint and a fold back from it (the rest of that
//               block then reads the recomputed values).  gamma = 0 and eps = infinity give
//               recomputation only.
//
// Conventions that the paper delegates to its renderer (Sec. 3.3) are fixed here as
// plain textbook definitions (Stokes frames, rotators, Fresnel amplitudes in the Born &
// Wolf form, Smith-GGX with Walter et al. 2007 sampling, Philox4x32-10 of Salmon et al.
// 2011); the rendering description and the binary scene format are documented with the
// GPU library's public header, which this file does not include.
//
// Pins (tests that tie this oracle to something other than itself): Philox known-answer
// vectors; closed forms for Fresnel (normal incidence, Brewster, R+T=1, TIR, conductors),
// polarizer/rotator/retarder identities; halving and Malus's law through polarizers; a
// chain of polarizer sheets; a closed-sphere furnace with value and gradient in closed
// form; frame-gauge invariance; Stokes validity; the fold identity; agreement of modes
// 1 and 2; detached and full central finite differences; the closed-form polarizer-angle
// derivative; linearity in the light radiance; BVH against brute force.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <unordered_map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace ora {

// ============================================================================ RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter c[4], key k[2].
static inline void philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
static inline double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

// Uniforms of one (pixel, sample, view, bounce, call) counter.
static inline void uniforms(uint64_t seed, uint32_t pix, uint32_t smp, uint32_t view, uint32_t bounce,
                            uint32_t call, double u[4]) {
    uint32_t c[4] = {pix, smp, (view << 8) | (bounce & 0xffu), call}, o[4];
    philox(c, seed, o);
    for (int i = 0; i < 4; ++i) u[i] = u01(o[i]);
}

// Regularisation noise of the noise-regularised polarized PRB (Sec. 4.2): one normal variate
// u ~ N(0, sigma) per path vertex (1-based vertex index vtx), from two uniforms of the vertex's counter
// (call 2) by the Box-Muller transform, so that the primal and the adjoint phase see the same noise.
static inline double pprb_noise(uint64_t seed, uint32_t pix, uint32_t smp, uint32_t view, uint32_t vtx, double sigma) {
    double u[4];
    uniforms(seed, pix, smp, view, vtx, 2, u);
    return sigma * std::sqrt(-2.0 * std::log(1.0 - u[0])) * std::cos(2.0 * M_PI * u[1]);
}

// Key of the independent suffix estimate of polarized radiative backpropagation (P-RB): the sub-path
// whose first vertex is vertex v_first of the path draws its random numbers from the usual counters
// under this key instead of the path's own.
static inline uint64_t prb_seed(uint64_t seed, uint32_t v_first) { return seed + (uint64_t)v_first * 0x9E3779B97F4A7C15ull; }

// ============================================================================ tape AD
struct Tape {
    std::vector<int> pa, pb;
    std::vector<double> ga, gb;
    int push(int a, double da, int b, double db) {
        pa.push_back(a); ga.push_back(da); pb.push_back(b); gb.push_back(db);
        return (int)pa.size() - 1;
    }
    void clear() { pa.clear(); pb.clear(); ga.clear(); gb.clear(); }
    // reverse sweep from a seeded adjoint vector
    void backward(std::vector<double>& adj) const {
        for (int i = (int)pa.size() - 1; i >= 0; --i) {
            double g = adj[i];
            if (g == 0.0) continue;
            if (pa[i] >= 0) adj[pa[i]] += ga[i] * g;
            if (pb[i] >= 0) adj[pb[i]] += gb[i] * g;
        }
    }
};
static thread_local Tape* g_tape = nullptr;

struct Var {
    double v;
    int i;
    Var() : v(0.0), i(-1) {}
    Var(double x) : v(x), i(-1) {}
    Var(double x, int id) : v(x), i(id) {}
};
static inline Var mk(double v, int a, double da, int b, double db) {
    if (a < 0 && b < 0) return Var(v);
    return Var(v, g_tape->push(a, da, b, db));
}
static inline Var leaf(double v) { return Var(v, g_tape->push(-1, 0.0, -1, 0.0)); }
static inline Var operator+(Var a, Var b) { return mk(a.v + b.v, a.i, 1.0, b.i, 1.0); }
static inline Var operator-(Var a, Var b) { return mk(a.v - b.v, a.i, 1.0, b.i, -1.0); }
static inline Var operator*(Var a, Var b) { return mk(a.v * b.v, a.i, b.v, b.i, a.v); }
static inline Var operator/(Var a, Var b) {
    double r = a.v / b.v;
    return mk(r, a.i, 1.0 / b.v, b.i, -r / b.v);
}
static inline Var operator-(Var a) { return mk(-a.v, a.i, -1.0, -1, 0.0); }
static inline Var& operator+=(Var& a, Var b) { a = a + b; return a; }
static inline Var sqrt(Var a) {
    double r = std::sqrt(a.v);
    return mk(r, a.i, 0.5 / r, -1, 0.0);
}
static inline Var sin(Var a) { return mk(std::sin(a.v), a.i, std::cos(a.v), -1, 0.0); }
static inline Var cos(Var a) { return mk(std::cos(a.v), a.i, -std::sin(a.v), -1, 0.0); }
static inline double val(double x) { return x; }
static inline double val(Var x) { return x.v; }
using std::sqrt; using std::sin; using std::cos;

// ============================================================================ small math
struct V3 { double x, y, z; };
static inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
static inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
static inline V3 operator-(V3 a) { return {-a.x, -a.y, -a.z}; }
static inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
static inline double len(V3 a) { return std::sqrt(dot(a, a)); }
static inline V3 normalize(V3 a) { return a * (1.0 / len(a)); }

// Vectors whose entries may be tape variables (the shading normal of a normal-mapped surface).
template <class T> struct VT { T x, y, z; };
template <class T> static inline VT<T> lift(V3 a) { return {T(a.x), T(a.y), T(a.z)}; }
template <class T> static inline T dot(const VT<T>& a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> static inline T dot(const VT<T>& a, const VT<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> static inline VT<T> cross(V3 a, const VT<T>& b) {
    return {b.z * a.y - b.y * a.z, b.x * a.z - b.z * a.x, b.y * a.x - b.x * a.y};
}
template <class T> static inline VT<T> vscale(const VT<T>& a, T s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> static inline VT<T> vneg(const VT<T>& a) { return {-a.x, -a.y, -a.z}; }

template <class T> struct Cx { T re, im; };
template <class T> static inline Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> static inline Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> static inline Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> static inline Cx<T> cdiv(Cx<T> a, Cx<T> b) {
    T d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
template <class T> static inline Cx<T> cscale(Cx<T> a, double s) { return {a.re * s, a.im * s}; }
template <class T> static inline T cabs2(Cx<T> a) { return a.re * a.re + a.im * a.im; }
// principal square root; a zero imaginary part counts as +0 (so sqrt(-x) = +i sqrt(x))
static inline void csqrt_d(double x, double y, double& wr, double& wi) {
    double r = std::hypot(x, y);
    if (r == 0.0) { wr = 0.0; wi = 0.0; return; }
    if (x >= 0.0) {
        double t = std::sqrt(0.5 * (r + x));
        wr = t; wi = y / (2.0 * t);
    } else {
        double t = std::sqrt(0.5 * (r - x));
        wr = std::fabs(y) / (2.0 * t); wi = (y < 0.0) ? -t : t;
    }
}
static inline Cx<double> csqrt(Cx<double> z) {
    Cx<double> w; csqrt_d(z.re, z.im, w.re, w.im); return w;
}
static inline Cx<Var> csqrt(Cx<Var> z) {
    double wr, wi; csqrt_d(z.re.v, z.im.v, wr, wi);
    // holomorphic: dw/dz = 1/(2w) = p + i q; Cauchy-Riemann gives the real partials
    double d = 2.0 * (wr * wr + wi * wi);
    double p = wr / d, q = -wi / d;
    Var r = mk(wr, z.re.i, p, z.im.i, -q);
    Var im = mk(wi, z.re.i, q, z.im.i, p);
    return {r, im};
}

template <class T> struct M4 { T m[4][4]; };
template <class T> struct S4 { T s[4]; };
template <class T> static inline M4<T> mzero() { M4<T> r; for (auto& row : r.m) for (auto& e : row) e = T(0.0); return r; }
template <class T> static inline M4<T> meye() { M4<T> r = mzero<T>(); for (int i = 0; i < 4; ++i) r.m[i][i] = T(1.0); return r; }
template <class T> static inline S4<T> szero() { S4<T> r; for (auto& e : r.s) e = T(0.0); return r; }
template <class A, class B>
static inline auto mmul(const M4<A>& a, const M4<B>& b) -> M4<decltype(A() * B())> {
    using R = decltype(A() * B());
    M4<R> r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            R acc = a.m[i][0] * b.m[0][j];
            for (int k = 1; k < 4; ++k) acc = acc + a.m[i][k] * b.m[k][j];
            r.m[i][j] = acc;
        }
    return r;
}
template <class A, class B>
static inline auto mvec(const M4<A>& a, const S4<B>& v) -> S4<decltype(A() * B())> {
    using R = decltype(A() * B());
    S4<R> r;
    for (int i = 0; i < 4; ++i) {
        R acc = a.m[i][0] * v.s[0];
        for (int k = 1; k < 4; ++k) acc = acc + a.m[i][k] * v.s[k];
        r.s[i] = acc;
    }
    return r;
}
template <class T> static inline M4<T> mscale(const M4<T>& a, T s) {
    M4<T> r; for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) r.m[i][j] = a.m[i][j] * s; return r;
}
template <class T> static inline M4<T> madd(const M4<T>& a, const M4<T>& b) {
    M4<T> r; for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) r.m[i][j] = a.m[i][j] + b.m[i][j]; return r;
}
template <class T> static inline S4<T> sadd(const S4<T>& a, const S4<T>& b) {
    S4<T> r; for (int i = 0; i < 4; ++i) r.s[i] = a.s[i] + b.s[i]; return r;
}
template <class T> static inline S4<T> sscale(const S4<T>& a, T s) {
    S4<T> r; for (int i = 0; i < 4; ++i) r.s[i] = a.s[i] * s; return r;
}
static M4<double> mconst(const M4<Var>& a) {
    M4<double> r; for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) r.m[i][j] = a.m[i][j].v; return r;
}

// ============================================================================ Stokes frames
static int g_gauge = 0;  // when set, every canonical frame is rotated by a smooth function of k

// Orthonormal basis (x, y, n) around unit n, Duff et al. 2017; y = n x x.
static void onb(V3 n, V3& x, V3& y) {
    double sg = std::copysign(1.0, n.z);
    double a = -1.0 / (sg + n.z);
    double b = n.x * n.y * a;
    x = {1.0 + sg * n.x * n.x * a, sg * b, -sg * n.x};
    y = {b, sg + n.y * n.y * a, -n.y};
}

// Canonical transverse basis vector x(k) for light propagating along unit k: the first
// tangent of the Duff et al. basis; y(k) = k x x(k).  (The gauge test rotates it.)
static V3 canon_x(V3 k) {
    V3 x, yy;
    onb(k, x, yy);
    if (g_gauge) {
        V3 y = cross(k, x);
        double phi = 3.0 * k.x - 5.0 * k.y + 7.0 * k.z + 0.3;
        x = x * std::cos(phi) + y * std::sin(phi);
    }
    return x;
}

// Rotator taking Stokes components in transverse basis x_from to basis x_to (both unit and
// perpendicular to the propagation direction k): with c = cos and s = sin of the angle
// from x_from to x_to, s1' = cos2 s1 + sin2 s2, s2' = -sin2 s1 + cos2 s2.
static M4<double> rotator(V3 k, V3 x_from, V3 x_to) {
    double c = dot(x_from, x_to), s = dot(cross(k, x_from), x_to);
    double c2 = c * c - s * s, s2 = 2.0 * c * s;
    M4<double> r = meye<double>();
    r.m[1][1] = c2; r.m[1][2] = s2; r.m[2][1] = -s2; r.m[2][2] = c2;
    return r;
}
static V3 transverse(V3 v, V3 k) { return normalize(v - k * dot(v, k)); }

// Ideal linear polarizer, transmission axis at angle th from x toward y.
template <class T> static M4<T> polarizer(T th) {
    T C = cos(th * 2.0), S = sin(th * 2.0);
    M4<T> r = mzero<T>();
    r.m[0][0] = T(0.5); r.m[0][1] = C * 0.5; r.m[0][2] = S * 0.5;
    r.m[1][0] = C * 0.5; r.m[1][1] = C * C * 0.5; r.m[1][2] = C * S * 0.5;
    r.m[2][0] = S * 0.5; r.m[2][1] = C * S * 0.5; r.m[2][2] = S * S * 0.5;
    return r;
}
// Linear retarder with its axis along x and retardance delta.
static M4<double> retarder(double delta) {
    M4<double> r = meye<double>();
    r.m[2][2] = std::cos(delta); r.m[2][3] = std::sin(delta);
    r.m[3][2] = -std::sin(delta); r.m[3][3] = std::cos(delta);
    return r;
}

// Mueller matrix of a Jones matrix diag(as, ap) in the (s, p) basis.
template <class T> static M4<T> jones_diag_mueller(Cx<T> as, Cx<T> ap) {
    T A = cabs2(as), B = cabs2(ap);
    Cx<T> z = cmul(as, Cx<T>{ap.re, -ap.im});
    M4<T> r = mzero<T>();
    r.m[0][0] = (A + B) * 0.5; r.m[0][1] = (A - B) * 0.5;
    r.m[1][0] = (A - B) * 0.5; r.m[1][1] = (A + B) * 0.5;
    r.m[2][2] = z.re; r.m[2][3] = z.im;
    r.m[3][2] = -z.im; r.m[3][3] = z.re;
    return r;
}

// Fresnel reflection and (flux-form) transmission Mueller matrices, Born & Wolf amplitudes,
// for incidence cosine ci and complex relative index m = n2/n1.  Bases: s perpendicular to
// the plane of incidence, p = k x s for each wave.
template <class T> static void fresnel(T ci, Cx<T> m, M4<T>* MR, M4<T>* MT) {
    Cx<T> m2 = cmul(m, m);
    Cx<T> one{T(1.0), T(0.0)};
    Cx<T> st2 = cdiv(Cx<T>{T(1.0) - ci * ci, T(0.0)}, m2);
    Cx<T> ct = csqrt(csub(one, st2));
    Cx<T> cI{ci, T(0.0)};
    Cx<T> mct = cmul(m, ct), mci = cmul(m, cI);
    Cx<T> rs = cdiv(csub(cI, mct), cadd(cI, mct));
    Cx<T> rp = cdiv(csub(mci, ct), cadd(mci, ct));
    if (MR) *MR = jones_diag_mueller(rs, rp);
    if (MT) {
        Cx<T> ts = cdiv(cscale(cI, 2.0), cadd(cI, mct));
        Cx<T> tp = cdiv(cscale(cI, 2.0), cadd(mci, ct));
        T kappa = mct.re / ci;
        *MT = mscale(jones_diag_mueller(ts, tp), kappa);
    }
}

// ============================================================================ GGX
template <class T> static T ggx_D(T cos_h, T a) {
    if (val(cos_h) <= 0.0) return T(0.0);
    T a2 = a * a;
    T d = (a2 - 1.0) * (cos_h * cos_h) + 1.0;
    return a2 / (d * d * M_PI);
}
template <class T> static T smith_G1(T cos_w, T a) {
    if (val(cos_w) <= 0.0) return T(0.0);
    T tan2 = (T(1.0) - cos_w * cos_w) / (cos_w * cos_w);
    T lam = (sqrt(a * a * tan2 + 1.0) - 1.0) * 0.5;
    return T(1.0) / (lam + 1.0);
}

// ============================================================================ scene
enum { MAT_LAMBERT = 0, MAT_DIELECTRIC = 1, MAT_GGX_DIELECTRIC = 2, MAT_GGX_CONDUCTOR = 3, MAT_SHEET = 4,
       MAT_EMITTER = 5, MAT_BLEND = 6 };
enum { SENSOR_NONE = 0, SENSOR_POLARIZER = 1, SENSOR_ANALYZER4 = 2, SENSOR_LIGHTSTAGE4 = 3 };
enum { FLAG_NO_NEE = 1, FLAG_GAUGE = 1 << 16 };
enum { LOBE_NONE = 0, LOBE_REFLECT = 1, LOBE_TRANSMIT = 2, LOBE_DIFFUSE = 3, LOBE_GLOSSY = 4, LOBE_SHEET = 5,
       LOBE_INVALID = 6 };

struct Material {
    uint32_t type;
    int32_t alb_slot; uint32_t alb_off, alb_tw, alb_th;
    int32_t alpha_slot; uint32_t alpha_off, alpha_tw, alpha_th;
    int32_t eta_slot; uint32_t eta_off;
    int32_t kap_slot; uint32_t kap_off;
    int32_t emit_slot; uint32_t emit_off;
    float axis[3]; float blend;
    float emit_circ;                                        // emitted Stokes: Le (1, 0, 0, emit_circ)
    int32_t spec_slot; uint32_t spec_off, spec_tw, spec_th;  // specular map: scale of the GGX lobe
    int32_t nrm_slot; uint32_t nrm_off, nrm_tw, nrm_th;      // tangent-space normal map (3 channels)
    uint32_t reserved[4];
};
static_assert(sizeof(Material) == 128, "material record");
// circ: the light emits Le (1, 0, 0, circ) (circular polarization is frame-independent)
struct LightRec { float p0[3], eu[3], ev[3]; int32_t le_slot; uint32_t le_off; float circ; };
static_assert(sizeof(LightRec) == 48, "light record");

struct View {
    int32_t world, width, height, spp, crop_x0, crop_y0, crop_w, crop_h;
    float origin[3], target[3], up[3], fov_y_deg;
    int32_t sensor, theta_slot, theta_off;
    uint32_t view_id;
};
static_assert(sizeof(View) == 88, "view record");

struct BNode { double lo[3], hi[3]; int left, right, first, count; };

struct World {
    std::vector<V3> v0, v1, v2;
    std::vector<double> uv;      // 6 per triangle
    std::vector<uint32_t> tmat;
    std::vector<V3> sc; std::vector<double> sr; std::vector<uint32_t> smat;
    std::vector<Material> mats;
    std::vector<LightRec> lights;
    std::vector<BNode> nodes;
    std::vector<int> order;
    int nprim() const { return (int)v0.size() + (int)sc.size(); }
};
struct Scene {
    std::vector<uint32_t> slot_numel;
    std::vector<World> worlds;
};

static V3 f3(const float* p) { return {p[0], p[1], p[2]}; }

static void prim_bounds(const World& w, int p, double lo[3], double hi[3]) {
    int nt = (int)w.v0.size();
    if (p < nt) {
        V3 a = w.v0[p], b = w.v1[p], c = w.v2[p];
        lo[0] = std::min({a.x, b.x, c.x}); lo[1] = std::min({a.y, b.y, c.y}); lo[2] = std::min({a.z, b.z, c.z});
        hi[0] = std::max({a.x, b.x, c.x}); hi[1] = std::max({a.y, b.y, c.y}); hi[2] = std::max({a.z, b.z, c.z});
    } else {
        V3 c = w.sc[p - nt]; double r = std::fabs(w.sr[p - nt]);
        lo[0] = c.x - r; lo[1] = c.y - r; lo[2] = c.z - r; hi[0] = c.x + r; hi[1] = c.y + r; hi[2] = c.z + r;
    }
}

// Median-split bounding volume hierarchy (plain object-median build, up to 4 primitives per leaf).
static int build_node(World& w, int first, int count, std::vector<double>& cen) {
    BNode n;
    for (int a = 0; a < 3; ++a) { n.lo[a] = 1e300; n.hi[a] = -1e300; }
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    for (int i = first; i < first + count; ++i) {
        double lo[3], hi[3]; prim_bounds(w, w.order[i], lo, hi);
        for (int a = 0; a < 3; ++a) {
            n.lo[a] = std::min(n.lo[a], lo[a]); n.hi[a] = std::max(n.hi[a], hi[a]);
            double c = cen[3 * w.order[i] + a];
            clo[a] = std::min(clo[a], c); chi[a] = std::max(chi[a], c);
        }
    }
    int id = (int)w.nodes.size();
    w.nodes.push_back(n);
    if (count <= 4) {
        w.nodes[id].left = w.nodes[id].right = -1; w.nodes[id].first = first; w.nodes[id].count = count;
        return id;
    }
    int ax = 0;
    for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[ax] - clo[ax]) ax = a;
    int mid = first + count / 2;
    std::nth_element(w.order.begin() + first, w.order.begin() + mid, w.order.begin() + first + count,
                     [&](int p, int q) { return cen[3 * p + ax] < cen[3 * q + ax]; });
    int l = build_node(w, first, mid - first, cen);
    int r = build_node(w, mid, first + count - mid, cen);
    w.nodes[id].left = l; w.nodes[id].right = r; w.nodes[id].first = 0; w.nodes[id].count = 0;
    return id;
}
static void build_bvh(World& w) {
    int n = w.nprim();
    w.order.resize(n);
    std::vector<double> cen(3 * (size_t)std::max(n, 1));
    for (int i = 0; i < n; ++i) {
        w.order[i] = i;
        double lo[3], hi[3]; prim_bounds(w, i, lo, hi);
        for (int a = 0; a < 3; ++a) cen[3 * i + a] = 0.5 * (lo[a] + hi[a]);
    }
    w.nodes.clear();
    if (n > 0) build_node(w, 0, n, cen);
}

// ============================================================================ ray queries
struct Hit { int prim = -1; double t = 0, bu = 0, bv = 0; };

// Moller-Trumbore 1997.
static bool hit_tri(const World& w, int i, V3 o, V3 d, double tmax, Hit& h) {
    V3 e1 = w.v1[i] - w.v0[i], e2 = w.v2[i] - w.v0[i];
    V3 p = cross(d, e2);
    double det = dot(e1, p);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    V3 s = o - w.v0[i];
    double u = dot(s, p) * inv;
    if (u < 0.0 || u > 1.0) return false;
    V3 q = cross(s, e1);
    double v = dot(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return false;
    double t = dot(e2, q) * inv;
    if (!(t > 0.0 && t < tmax)) return false;
    h.prim = i; h.t = t; h.bu = u; h.bv = v;
    return true;
}
static bool hit_sphere(const World& w, int j, V3 o, V3 d, double tmax, Hit& h) {
    V3 oc = o - w.sc[j];
    double r = w.sr[j];
    double b = dot(d, oc), c = dot(oc, oc) - r * r;
    double disc = b * b - c;
    if (disc < 0.0) return false;
    double sq = std::sqrt(disc);
    double t = -b - sq;
    if (!(t > 0.0)) t = -b + sq;
    if (!(t > 0.0 && t < tmax)) return false;
    h.prim = (int)w.v0.size() + j; h.t = t; h.bu = 0; h.bv = 0;
    return true;
}
static bool hit_prim(const World& w, int p, V3 o, V3 d, double tmax, Hit& h) {
    int nt = (int)w.v0.size();
    return p < nt ? hit_tri(w, p, o, d, tmax, h) : hit_sphere(w, p - nt, o, d, tmax, h);
}
static bool box_hit(const BNode& n, V3 o, V3 d, double tmax) {
    double t0 = 0.0, t1 = tmax;
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    for (int a = 0; a < 3; ++a) {
        if (dd[a] == 0.0) {
            if (oo[a] < n.lo[a] || oo[a] > n.hi[a]) return false;
            continue;
        }
        double ta = (n.lo[a] - oo[a]) / dd[a], tb = (n.hi[a] - oo[a]) / dd[a];
        if (ta > tb) std::swap(ta, tb);
        t0 = std::max(t0, ta); t1 = std::min(t1, tb);
        if (t0 > t1) return false;
    }
    return true;
}
// closest hit (any_hit = false) or any hit (any_hit = true) with 0 < t < tmax
static bool trace(const World& w, V3 o, V3 d, double tmax, bool any_hit, bool brute, Hit& best) {
    best.prim = -1;
    double tb = tmax;
    if (brute || w.nodes.empty()) {
        for (int p = 0; p < w.nprim(); ++p) {
            Hit h;
            if (hit_prim(w, p, o, d, tb, h)) { best = h; tb = h.t; if (any_hit) return true; }
        }
        return best.prim >= 0;
    }
    int stack[128]; int sp = 0; stack[sp++] = 0;
    while (sp) {
        const BNode& n = w.nodes[stack[--sp]];
        if (!box_hit(n, o, d, tb)) continue;
        if (n.left < 0) {
            for (int i = n.first; i < n.first + n.count; ++i) {
                Hit h;
                if (hit_prim(w, w.order[i], o, d, tb, h)) { best = h; tb = h.t; if (any_hit) return true; }
            }
        } else {
            stack[sp++] = n.left; stack[sp++] = n.right;
        }
    }
    return best.prim >= 0;
}

static double offset_eps(V3 p) {
    return 1e-4 * (1.0 + std::max({std::fabs(p.x), std::fabs(p.y), std::fabs(p.z)}));
}
// ray origin leaving surface point p (geometric normal ng) toward direction dir
static V3 spawn(V3 p, V3 ng, V3 dir) {
    double e = offset_eps(p);
    return p + ng * (dot(dir, ng) > 0.0 ? e : -e);
}

// ============================================================================ parameters
// Read access to the parameter tensors.  For the AD modes every element that is read
// becomes a tape leaf the first time it is touched.
template <class T> struct PAcc;
template <> struct PAcc<double> {
    const double* const* p;
    double get(int s, uint32_t i) const { return p[s][i]; }
};
template <> struct PAcc<Var> {
    const double* const* p;
    mutable std::unordered_map<int64_t, Var> leaves;
    Var get(int s, uint32_t i) const {
        int64_t key = ((int64_t)s << 40) | i;
        auto it = leaves.find(key);
        if (it != leaves.end()) return it->second;
        Var v = leaf(p[s][i]);
        leaves.emplace(key, v);
        return v;
    }
};

// Bilinear lookup, clamp-to-edge, texel centres at (i + 1/2) / N; texel layout [th][tw][ch].
template <class T>
static T tex_lookup(const PAcc<T>& P, int slot, uint32_t off, uint32_t tw, uint32_t th, int ch, int c, double u,
                    double v) {
    double x = u * tw - 0.5, y = v * th - 0.5;
    double x0f = std::floor(x), y0f = std::floor(y);
    double fx = x - x0f, fy = y - y0f;
    long x0 = (long)x0f, y0 = (long)y0f;
    auto cl = [](long a, long n) { return a < 0 ? 0 : (a >= n ? n - 1 : a); };
    long xa = cl(x0, tw), xb = cl(x0 + 1, tw), ya = cl(y0, th), yb = cl(y0 + 1, th);
    auto at = [&](long xx, long yy) { return P.get(slot, off + (uint32_t)((yy * tw + xx) * ch + c)); };
    return at(xa, ya) * ((1 - fx) * (1 - fy)) + at(xb, ya) * (fx * (1 - fy)) + at(xa, yb) * ((1 - fx) * fy) +
           at(xb, yb) * (fx * fy);
}
template <class T> static T mat_albedo(const PAcc<T>& P, const Material& m, int c, double u, double v) {
    if (m.alb_tw == 0) return P.get(m.alb_slot, m.alb_off + c);
    return tex_lookup(P, m.alb_slot, m.alb_off, m.alb_tw, m.alb_th, 3, c, u, v);
}
template <class T> static T mat_alpha(const PAcc<T>& P, const Material& m, double u, double v) {
    T a = (m.alpha_tw == 0) ? P.get(m.alpha_slot, m.alpha_off)
                            : tex_lookup(P, m.alpha_slot, m.alpha_off, m.alpha_tw, m.alpha_th, 1, 0, u, v);
    if (val(a) < 1e-3) return T(1e-3);  // roughness is clamped to [1e-3, 1]
    if (val(a) > 1.0) return T(1.0);
    return a;
}
// Specular map: scale of the GGX lobe (1 when the material has none).
template <class T> static T mat_spec(const PAcc<T>& P, const Material& m, double u, double v) {
    if (m.spec_slot < 0) return T(1.0);
    if (m.spec_tw == 0) return P.get(m.spec_slot, m.spec_off);
    return tex_lookup(P, m.spec_slot, m.spec_off, m.spec_tw, m.spec_th, 1, 0, u, v);
}
template <class T> static Cx<T> mat_ior(const PAcc<T>& P, const Material& m) {
    T n = P.get(m.eta_slot, m.eta_off);
    T k = (m.kap_slot >= 0) ? P.get(m.kap_slot, m.kap_off) : T(0.0);
    return {n, k};
}

// ============================================================================ path geometry
// Everything about one path vertex that is *not* differentiated.
struct Vtx {
    int prim, mat;
    V3 p, ng, ns, wo;          // position, geometric normal, shading normal (toward wo), toward previous vertex
    double u, v;               // texture coordinates
    bool front;                // wo on the side the geometric normal points to
    bool emit;                 // emission of this vertex is counted
    int lobe;                  // continuation lobe
    V3 wi;                     // continuation direction (away from the vertex)
    double prob;               // discrete selection probability of the lobe (detached)
    double pdf;                // solid-angle pdf of wi for the glossy lobe (detached)
    double eta_cam, eta_far;   // real IORs on the wo side and the other side (dielectric only)
    int nee;                   // 0 none, 1 visible, 2 occluded, 3 zero (back-facing)
    V3 wl;                     // direction to the light sample
    double nee_geom;           // cos_light * area * n_lights / dist^2
    int light;
    bool nmap;                 // the material has a normal map: ns comes from it
    V3 tg, bt;                 // tangent frame (u direction, ng x tangent) of a normal-mapped triangle
};

static bool is_delta(uint32_t t) { return t == MAT_DIELECTRIC || t == MAT_SHEET; }

struct Sig {
    uint64_t h = 1469598103934665603ull;
    void add(uint32_t x) {
        for (int i = 0; i < 4; ++i) { h ^= (x >> (8 * i)) & 0xffu; h *= 1099511628211ull; }
    }
};

struct Camera { V3 o, f, r, u; double tanh_, aspect; };
static Camera make_camera(const View& v) {
    Camera c;
    c.o = f3(v.origin);
    c.f = normalize(f3(v.target) - c.o);
    c.r = normalize(cross(c.f, f3(v.up)));
    c.u = cross(c.r, c.f);
    c.tanh_ = std::tan(0.5 * v.fov_y_deg * M_PI / 180.0);
    c.aspect = (double)v.width / (double)v.height;
    return c;
}


// ============================================================================ shading normal
// Tangent frame of triangle p at its outward geometric normal N: the tangent follows increasing
// u (dP/du from the triangle's uv parameterisation, made perpendicular to N), the bitangent is
// N x tangent.  A triangle with a degenerate uv map takes the canonical basis of N instead.
static void tangent_frame(const World& w, int p, V3 N, V3& tg, V3& bt) {
    V3 e1 = w.v1[p] - w.v0[p], e2 = w.v2[p] - w.v0[p];
    const double* t = &w.uv[6 * (size_t)p];
    double du1 = t[2] - t[0], dv1 = t[3] - t[1], du2 = t[4] - t[0], dv2 = t[5] - t[1];
    double det = du1 * dv2 - du2 * dv1;
    V3 dpdu = (e1 * dv2 - e2 * dv1) * (det < 0.0 ? -1.0 : 1.0);
    V3 tp = dpdu - N * dot(dpdu, N);
    double l = len(tp);
    if (det == 0.0 || !(l > 1e-6 * (len(e1) + len(e2)))) {
        V3 yy;
        onb(N, tg, yy);
    } else {
        tg = tp * (1.0 / l);
    }
    bt = cross(N, tg);
}
// Shading normal toward the viewer side: the normal map's tangent-space components (t, b, n)
// give the outward normal normalize(t T + b B + n N); on the back side it is negated.
template <class T> static VT<T> shading_normal(const PAcc<T>& P, const Material& m, const Vtx& x) {
    if (!x.nmap) return lift<T>(x.ns);
    T c[3];
    for (int k = 0; k < 3; ++k)
        c[k] = (m.nrm_tw == 0) ? P.get(m.nrm_slot, m.nrm_off + k)
                               : tex_lookup(P, m.nrm_slot, m.nrm_off, m.nrm_tw, m.nrm_th, 3, k, x.u, x.v);
    VT<T> n{c[0] * x.tg.x + c[1] * x.bt.x + c[2] * x.ng.x, c[0] * x.tg.y + c[1] * x.bt.y + c[2] * x.ng.y,
            c[0] * x.tg.z + c[1] * x.bt.z + c[2] * x.ng.z};
    T il = T(1.0) / sqrt(dot(n, n));
    if (!x.front) il = -il;
    return vscale(n, il);
}

// ============================================================================ path tracing (detached part)
static V3 onb_x(V3 n) { V3 x, y; onb(n, x, y); return x; }

template <class T> static T mat_ggx_alpha_path(const PAcc<T>& P, const Material& m, double u, double v) {
    return mat_alpha(P, m, u, v);
}

// Walter et al. 2007 half-vector sampling of the GGX distribution around ns, mirrored about h.
static int sample_glossy(V3 ns, V3 wo, double alpha, double u1, double u2, V3& wi, double& pdf) {
    double tan2 = alpha * alpha * u1 / (1.0 - u1);
    double ch = 1.0 / std::sqrt(1.0 + tan2);
    double sh = std::sqrt(std::max(0.0, 1.0 - ch * ch));
    double ph = 2.0 * M_PI * u2;
    V3 tx, ty; onb(ns, tx, ty);
    V3 h = tx * (sh * std::cos(ph)) + ty * (sh * std::sin(ph)) + ns * ch;
    double woh = dot(wo, h);
    if (!(woh > 0.0)) return LOBE_INVALID;
    wi = h * (2.0 * woh) - wo;
    if (!(dot(ns, wi) > 0.0)) return LOBE_INVALID;
    pdf = ggx_D(ch, alpha) * ch / (4.0 * woh);
    return LOBE_GLOSSY;
}
static int sample_diffuse(V3 ns, double u1, double u2, V3& wi, double& pdf) {
    V3 tx, ty; onb(ns, tx, ty);
    double r = std::sqrt(u1), ph = 2.0 * M_PI * u2;
    wi = tx * (r * std::cos(ph)) + ty * (r * std::sin(ph)) + ns * std::sqrt(std::max(0.0, 1.0 - u1));
    pdf = dot(ns, wi) / M_PI;
    return LOBE_DIFFUSE;
}

struct PathGeom {
    std::vector<Vtx> v;
    V3 k_cam, x_sensor;
    uint64_t sig;
};

static void trace_from(const World& w, const View& vw, uint32_t pix, int smp, uint64_t seed, int max_depth,
                       uint32_t flags, const PAcc<double>& P, V3 o, V3 d, int b_start, bool prev_delta, PathGeom& g,
                       Sig& sig);

// Trace one camera path: RNG counter (pixel, sample, view<<8 | bounce, call).  Sampling
// decisions read the parameters through P (the "path" parameters).
static void trace_path(const World& w, const View& vw, int px, int py, int smp, uint64_t seed, int max_depth,
                       uint32_t flags, const PAcc<double>& P, PathGeom& g) {
    g.v.clear();
    Camera cam = make_camera(vw);
    uint32_t pix = (uint32_t)(py * vw.width + px);
    double u[4];
    uniforms(seed, pix, (uint32_t)smp, vw.view_id, 0, 0, u);
    double sx = (2.0 * (px + u[0]) / vw.width - 1.0) * cam.tanh_ * cam.aspect;
    double sy = (1.0 - 2.0 * (py + u[1]) / vw.height) * cam.tanh_;
    V3 d = normalize(cam.f + cam.r * sx + cam.u * sy);
    V3 o = cam.o;
    g.k_cam = -d;
    g.x_sensor = transverse(cam.r, g.k_cam);
    Sig sig;
    trace_from(w, vw, pix, smp, seed, max_depth, flags, P, o, d, 1, false, g, sig);
    g.sig = sig.h;
}

// The vertices b_start, b_start + 1, ... (1-based vertex numbers, which key the random numbers) of a
// path entering along the ray (o, d), appended to g.v; prev_delta: the vertex before b_start was a
// delta vertex (it decides whether an emitter hit at b_start counts).
static void trace_from(const World& w, const View& vw, uint32_t pix, int smp, uint64_t seed, int max_depth,
                       uint32_t flags, const PAcc<double>& P, V3 o, V3 d, int b_start, bool prev_delta, PathGeom& g,
                       Sig& sig) {
    int nt = (int)w.v0.size();
    for (int b = b_start; b <= max_depth; ++b) {
        Hit h;
        if (!trace(w, o, d, 1e30, false, false, h)) { sig.add(0xffffffffu); break; }
        Vtx x{};
        x.prim = h.prim;
        if (h.prim < nt) {
            int p = h.prim;
            V3 e1 = w.v1[p] - w.v0[p], e2 = w.v2[p] - w.v0[p];
            x.p = w.v0[p] + e1 * h.bu + e2 * h.bv;
            x.ng = normalize(cross(e1, e2));
            const double* t = &w.uv[6 * (size_t)p];
            double b0 = 1.0 - h.bu - h.bv;
            x.u = b0 * t[0] + h.bu * t[2] + h.bv * t[4];
            x.v = b0 * t[1] + h.bu * t[3] + h.bv * t[5];
            x.mat = (int)w.tmat[p];
        } else {
            int j = h.prim - nt;
            x.p = o + d * h.t;
            V3 nout = normalize(x.p - w.sc[j]);
            x.ng = w.sr[j] < 0 ? -nout : nout;
            x.u = 0.5 + std::atan2(nout.z, nout.x) / (2.0 * M_PI);
            x.v = std::acos(std::max(-1.0, std::min(1.0, nout.y))) / M_PI;
            x.mat = (int)w.smat[j];
        }
        const Material& m = w.mats[x.mat];
        x.wo = -d;
        x.front = dot(x.ng, x.wo) > 0.0;
        x.ns = x.front ? x.ng : -x.ng;
        const V3 ngf = x.ns;  // geometric normal on the viewer side
        x.nmap = m.nrm_slot >= 0 && h.prim < nt;
        if (x.nmap) {
            tangent_frame(w, h.prim, x.ng, x.tg, x.bt);
            VT<double> n = shading_normal(P, m, x);
            x.ns = V3{n.x, n.y, n.z};
        }
        x.emit = m.emit_slot >= 0 && x.front && (b == 1 || prev_delta || (flags & FLAG_NO_NEE));
        x.lobe = LOBE_NONE;
        x.nee = 0;
        // a normal-mapped vertex seen from behind its shading normal neither scatters nor samples
        // a light (its emission still counts)
        const bool dark = x.nmap && !(dot(x.ns, x.wo) > 0.0);
        if (dark && !(m.type == MAT_EMITTER || b == max_depth)) {
            x.nee = 3;
            x.lobe = LOBE_INVALID;
            sig.add((uint32_t)x.prim); sig.add((uint32_t)x.lobe); sig.add((uint32_t)x.nee);
            g.v.push_back(x);
            break;
        }
        if (m.type == MAT_EMITTER || b == max_depth) {
            sig.add((uint32_t)x.prim); sig.add(0); sig.add(0);
            g.v.push_back(x);
            break;
        }
        double ua[4], ub[4];
        uniforms(seed, pix, (uint32_t)smp, vw.view_id, (uint32_t)b, 0, ua);
        uniforms(seed, pix, (uint32_t)smp, vw.view_id, (uint32_t)b, 1, ub);
        // next-event estimation: one uniformly chosen light, a uniform point on it
        if (!is_delta(m.type) && !(flags & FLAG_NO_NEE) && !w.lights.empty()) {
            int nl = (int)w.lights.size();
            int li = std::min((int)(ua[3] * nl), nl - 1);
            const LightRec& L = w.lights[li];
            V3 eu = f3(L.eu), ev = f3(L.ev);
            V3 y = f3(L.p0) + eu * ub[0] + ev * ub[1];
            V3 nraw = cross(eu, ev);
            double area = len(nraw);
            V3 nl_ = nraw * (1.0 / area);
            V3 dv = y - x.p;
            double dist2 = dot(dv, dv), dist = std::sqrt(dist2);
            x.wl = dv * (1.0 / dist);
            x.light = li;
            double cos_y = -dot(nl_, x.wl), cos_x = dot(x.ns, x.wl);
            // with a normal map the light must also lie above the geometric surface
            if (!(cos_y > 0.0) || !(cos_x > 0.0) || (x.nmap && !(dot(ngf, x.wl) > 0.0))) {
                x.nee = 3;
            } else {
                V3 so = spawn(x.p, x.ng, x.wl);
                V3 sd = y - so;
                double sl = len(sd);
                sd = sd * (1.0 / sl);
                Hit hh;
                bool occ = trace(w, so, sd, sl - offset_eps(y), true, false, hh);
                x.nee = occ ? 2 : 1;
                x.nee_geom = cos_y * area * nl / dist2;
            }
        }
        // continuation
        switch (m.type) {
            case MAT_LAMBERT:
                x.lobe = sample_diffuse(x.ns, ua[1], ua[2], x.wi, x.pdf);
                x.prob = 1.0;
                break;
            case MAT_GGX_DIELECTRIC:
            case MAT_GGX_CONDUCTOR:
                x.lobe = sample_glossy(x.ns, x.wo, mat_alpha(P, m, x.u, x.v), ua[1], ua[2], x.wi, x.pdf);
                x.prob = 1.0;
                break;
            case MAT_BLEND:
                if (ua[0] < m.blend) {
                    x.lobe = sample_diffuse(x.ns, ua[1], ua[2], x.wi, x.pdf);
                    x.prob = m.blend;
                } else {
                    x.lobe = sample_glossy(x.ns, x.wo, mat_alpha(P, m, x.u, x.v), ua[1], ua[2], x.wi, x.pdf);
                    x.prob = 1.0 - m.blend;
                }
                break;
            case MAT_DIELECTRIC: {
                double eta = P.get(m.eta_slot, m.eta_off);
                x.eta_cam = x.front ? 1.0 : eta;
                x.eta_far = x.front ? eta : 1.0;
                double mr = x.eta_far / x.eta_cam;
                double co = dot(x.ns, x.wo);
                double st2 = (1.0 - co * co) / (mr * mr);
                double PR = 1.0;
                if (st2 < 1.0) {
                    M4<double> MR;
                    fresnel<double>(co, Cx<double>{mr, 0.0}, &MR, nullptr);
                    PR = MR.m[0][0];
                }
                if (ua[0] < PR) {
                    x.wi = x.ns * (2.0 * co) - x.wo;
                    x.prob = PR;
                    x.lobe = LOBE_REFLECT;
                } else {
                    double ct = std::sqrt(1.0 - st2);
                    x.wi = normalize((-x.wo) * (1.0 / mr) + x.ns * (co / mr - ct));
                    x.prob = 1.0 - PR;
                    x.lobe = LOBE_TRANSMIT;
                }
                break;
            }
            case MAT_SHEET:
                x.wi = -x.wo;
                x.prob = 1.0;
                x.lobe = LOBE_SHEET;
                break;
            default:
                x.lobe = LOBE_INVALID;
        }
        // with a normal map, a reflected direction must leave above the geometric surface and a
        // transmitted one below it
        if (x.nmap && x.lobe != LOBE_INVALID && x.lobe != LOBE_SHEET) {
            double side = dot(ngf, x.wi);
            if (x.lobe == LOBE_TRANSMIT ? !(side < 0.0) : !(side > 0.0)) x.lobe = LOBE_INVALID;
        }
        // (parity signature: the lobe word of a sampled direction also carries the branch of the
        // sampling frame, the sign of ns.z in the Duff et al. basis, which rounding can flip for a
        // normal with z near 0)
        const bool framed = x.lobe == LOBE_DIFFUSE || x.lobe == LOBE_GLOSSY;
        sig.add((uint32_t)x.prim);
        sig.add((uint32_t)x.lobe | (framed && std::signbit(x.ns.z) ? 16u : 0u));
        sig.add((uint32_t)x.nee);
        g.v.push_back(x);
        if (x.lobe == LOBE_INVALID) break;
        prev_delta = is_delta(m.type);
        o = spawn(x.p, x.ng, x.wi);
        d = x.wi;
    }
}

// ============================================================================ differentiated values
// Express a local Mueller matrix (input basis x_in about k_in, output basis x_out about
// k_out) in the canonical frames of the two propagation directions.
template <class T> static M4<T> to_canon(const M4<T>& Ml, V3 k_in, V3 x_in, V3 k_out, V3 x_out) {
    M4<double> Rin = rotator(k_in, canon_x(k_in), x_in);
    M4<double> Rout = rotator(k_out, x_out, canon_x(k_out));
    return mmul(mmul(Rout, Ml), Rin);
}
// A specular (Fresnel) event: s = k_in x n_inc (n_inc the normal on the incident side).
template <class T> static M4<T> specular_canon(const M4<T>& Ml, V3 k_in, V3 n_inc, V3 k_out) {
    V3 s = cross(k_in, n_inc);
    double l = len(s);
    V3 sx = (l > 1e-12) ? s * (1.0 / l) : onb_x(k_in);
    return to_canon(Ml, k_in, sx, k_out, sx);
}
// The same with a differentiated normal (a normal-mapped shading normal): the s axis, and with
// it both rotators, move with the normal.
template <class T> static M4<T> rotator_t(V3 k, const VT<T>& x_from, const VT<T>& x_to) {
    T c = dot(x_from, x_to), s = dot(cross(k, x_from), x_to);
    T c2 = c * c - s * s, s2 = c * s * 2.0;
    M4<T> r = meye<T>();
    r.m[1][1] = c2; r.m[1][2] = s2; r.m[2][1] = -s2; r.m[2][2] = c2;
    return r;
}
template <class T> static M4<T> specular_canon(const M4<T>& Ml, V3 k_in, const VT<T>& n_inc, V3 k_out) {
    VT<T> s = cross(k_in, n_inc);
    T l = sqrt(dot(s, s));
    VT<T> sx = (val(l) > 1e-12) ? vscale(s, T(1.0) / l) : lift<T>(onb_x(k_in));
    M4<T> Rin = rotator_t(k_in, lift<T>(canon_x(k_in)), sx);
    M4<T> Rout = rotator_t(k_out, sx, lift<T>(canon_x(k_out)));
    return mmul(mmul(Rout, Ml), Rin);
}

// GGX microfacet pBRDF value f(wi -> wo) in canonical frames (without the cosine), for the
// (possibly differentiated) shading normal ns.
template <class T> static M4<T> ggx_f(const VT<T>& ns, V3 wi, V3 wo, T alpha, Cx<T> m) {
    V3 h = normalize(wi + wo);
    T ci = dot(ns, wi), co = dot(ns, wo), chh = dot(ns, h);
    double ih = std::fabs(dot(wi, h));
    T D = ggx_D(chh, alpha);
    T G = smith_G1(ci, alpha) * smith_G1(co, alpha);
    M4<T> MR;
    fresnel(T(ih), m, &MR, (M4<T>*)nullptr);
    M4<T> Ml = mscale(MR, D * G / (ci * co * 4.0));
    return specular_canon(Ml, -wi, h, wo);
}
template <class T> static M4<T> diffuse_f(T rho) {
    M4<T> r = mzero<T>();
    r.m[0][0] = rho / M_PI;
    return r;
}

// BSDF value (per channel) for light arriving along -wi and leaving along x.wo, canonical frames.
template <class T>
static void bsdf_eval(const Material& m, const Vtx& x, const VT<T>& ns, V3 wi, const PAcc<T>& P, M4<T> f[3]) {
    if (m.type == MAT_LAMBERT) {
        for (int c = 0; c < 3; ++c) f[c] = to_canon(diffuse_f(mat_albedo(P, m, c, x.u, x.v)), -wi, canon_x(-wi), x.wo, canon_x(x.wo));
    } else if (m.type == MAT_GGX_DIELECTRIC || m.type == MAT_GGX_CONDUCTOR) {
        M4<T> g = mscale(ggx_f(ns, wi, x.wo, mat_alpha(P, m, x.u, x.v), mat_ior(P, m)), mat_spec(P, m, x.u, x.v));
        for (int c = 0; c < 3; ++c) f[c] = g;
    } else if (m.type == MAT_BLEND) {
        Cx<T> eta{P.get(m.eta_slot, m.eta_off), T(0.0)};
        M4<T> g = mscale(ggx_f(ns, wi, x.wo, mat_alpha(P, m, x.u, x.v), eta), mat_spec(P, m, x.u, x.v));
        for (int c = 0; c < 3; ++c) {
            M4<T> dl = to_canon(diffuse_f(mat_albedo(P, m, c, x.u, x.v)), -wi, canon_x(-wi), x.wo, canon_x(x.wo));
            f[c] = madd(mscale(dl, T((double)m.blend)), mscale(g, T(1.0 - (double)m.blend)));
        }
    } else {
        for (int c = 0; c < 3; ++c) f[c] = mzero<T>();
    }
}

template <class T> struct VEval { M4<T> W[3]; S4<T> E[3]; };

// Differentiated per-vertex quantities: the Mueller sample weight W_b (f cos / pdf over the
// discrete lobe probability, the latter two detached) and the emitted + NEE Stokes vector E_b.
template <class T>
static void eval_vertex(const World& w, const Vtx& x, const PAcc<T>& P, VEval<T>& out) {
    const Material& m = w.mats[x.mat];
    for (int c = 0; c < 3; ++c) { out.E[c] = szero<T>(); out.W[c] = mzero<T>(); }
    // the shading normal is a differentiated quantity when it comes from a normal map
    const VT<T> ns = shading_normal(P, m, x);
    if (x.emit)
        for (int c = 0; c < 3; ++c) {
            T le = P.get(m.emit_slot, m.emit_off + c);
            out.E[c].s[0] = le;
            out.E[c].s[3] = le * (double)m.emit_circ;
        }
    if (x.nee == 1) {
        // light Stokes Le (1, 0, 0, circ): columns 0 and 3 of the BSDF Mueller matrix
        const LightRec& L = w.lights[x.light];
        M4<T> f[3];
        bsdf_eval(m, x, ns, x.wl, P, f);
        T cx = dot(ns, x.wl);
        for (int c = 0; c < 3; ++c) {
            T s = P.get(L.le_slot, L.le_off + c) * (cx * x.nee_geom);
            for (int i = 0; i < 4; ++i)
                out.E[c].s[i] = out.E[c].s[i] + f[c].m[i][0] * s + f[c].m[i][3] * (s * (double)L.circ);
        }
    }
    switch (x.lobe) {
        case LOBE_DIFFUSE:
        case LOBE_GLOSSY: {
            // the selected lobe's own value: weight and selection probability are equal (blend)
            T ci = dot(ns, x.wi);
            for (int c = 0; c < 3; ++c) {
                M4<T> f;
                if (x.lobe == LOBE_DIFFUSE)
                    f = to_canon(diffuse_f(mat_albedo(P, m, c, x.u, x.v)), -x.wi, canon_x(-x.wi), x.wo, canon_x(x.wo));
                else {
                    Cx<T> eta = (m.type == MAT_BLEND) ? Cx<T>{P.get(m.eta_slot, m.eta_off), T(0.0)} : mat_ior(P, m);
                    f = mscale(ggx_f(ns, x.wi, x.wo, mat_alpha(P, m, x.u, x.v), eta), mat_spec(P, m, x.u, x.v));
                }
                out.W[c] = mscale(f, ci / x.pdf);
            }
            break;
        }
        case LOBE_REFLECT:
        case LOBE_TRANSMIT: {
            T eta = P.get(m.eta_slot, m.eta_off);
            T ecam = x.front ? T(1.0) : eta, efar = x.front ? eta : T(1.0);
            M4<T> M;
            if (x.lobe == LOBE_REFLECT) {
                fresnel(dot(ns, x.wo), Cx<T>{efar / ecam, T(0.0)}, &M, (M4<T>*)nullptr);
                M = x.nmap ? specular_canon(M, -x.wi, ns, x.wo) : specular_canon(M, -x.wi, x.ns, x.wo);
            } else {
                // light crosses from the far side: incidence cosine |wi.n|, relative index ecam/efar
                T cw = dot(ns, x.wi);
                fresnel(val(cw) < 0.0 ? -cw : cw, Cx<T>{ecam / efar, T(0.0)}, (M4<T>*)nullptr, &M);
                M = x.nmap ? specular_canon(M, -x.wi, vneg(ns), x.wo) : specular_canon(M, -x.wi, -x.ns, x.wo);
            }
            M = mscale(M, T(1.0 / x.prob));
            for (int c = 0; c < 3; ++c) out.W[c] = M;
            break;
        }
        case LOBE_SHEET: {
            V3 k = x.wo;
            V3 xt = transverse(V3{m.axis[0], m.axis[1], m.axis[2]}, k);
            M4<double> M = to_canon(polarizer<double>(0.0), k, xt, k, xt);
            for (int c = 0; c < 3; ++c)
                for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) out.W[c].m[i][j] = T(M.m[i][j]);
            break;
        }
        default:
            break;
    }
}

// Sensor Mueller matrices (one per analyzer) for light arriving along k_cam.
template <class T>
static int sensor(const View& vw, V3 k_cam, V3 x_sensor, const PAcc<T>& P, M4<T> S[4]) {
    M4<double> R = rotator(k_cam, canon_x(k_cam), x_sensor);
    M4<T> RT;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) RT.m[i][j] = T(R.m[i][j]);
    if (vw.sensor == SENSOR_POLARIZER) {
        S[0] = mmul(polarizer<T>(P.get(vw.theta_slot, vw.theta_off)), R);
        return 1;
    }
    if (vw.sensor == SENSOR_ANALYZER4 || vw.sensor == SENSOR_LIGHTSTAGE4) {
        S[0] = mmul(polarizer<double>(0.0), RT);
        S[1] = mmul(polarizer<double>(M_PI / 4), RT);
        S[2] = mmul(polarizer<double>(M_PI / 2), RT);
        // circular analyzers: a quarter-wave plate at 0 then a polarizer at +45 degrees (passes
        // s3 > 0, right-circular here) or at -45 degrees (passes s3 < 0, left-circular)
        double a3 = vw.sensor == SENSOR_ANALYZER4 ? M_PI / 4 : -M_PI / 4;
        S[3] = mmul(mmul(polarizer<double>(a3), retarder(M_PI / 2)), RT);
        return 4;
    }
    S[0] = RT;
    return 1;
}

// Gauss-Jordan inverse with partial pivoting (the inversion of the basic polarized PRB).
static M4<double> inverse4(const M4<double>& a) {
    double m[4][8];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? a.m[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int c = 0; c < 4; ++c) {
        int p = c;
        for (int r = c + 1; r < 4; ++r) if (std::fabs(m[r][c]) > std::fabs(m[p][c])) p = r;
        if (p != c) for (int j = 0; j < 8; ++j) std::swap(m[p][j], m[c][j]);
        double piv = m[c][c];
        for (int j = 0; j < 8; ++j) m[c][j] /= piv;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            double f = m[r][c];
            for (int j = 0; j < 8; ++j) m[r][j] -= f * m[c][j];
        }
    }
    M4<double> r;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) r.m[i][j] = m[i][j + 4];
    return r;
}

// Determinant by Gaussian elimination with partial pivoting.
static double det4(const M4<double>& a) {
    double m[4][4];
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) m[i][j] = a.m[i][j];
    double det = 1.0;
    for (int c = 0; c < 4; ++c) {
        int p = c;
        for (int r = c + 1; r < 4; ++r) if (std::fabs(m[r][c]) > std::fabs(m[p][c])) p = r;
        if (m[p][c] == 0.0) return 0.0;
        if (p != c) { for (int j = 0; j < 4; ++j) std::swap(m[p][j], m[c][j]); det = -det; }
        det *= m[c][c];
        for (int r = c + 1; r < 4; ++r) {
            double f = m[r][c] / m[c][c];
            for (int j = c; j < 4; ++j) m[r][j] -= f * m[c][j];
        }
    }
    return det;
}

// Depolarization index of Gil & Bernabeu (1985): sqrt(sum_ij M_ij^2 - M_00^2) / (sqrt(3) M_00); 1 for a
// non-depolarizing Mueller matrix, 0 for an ideal depolarizer (Sec. 4.4, the test of Eq. 3).
static double depol_index(const M4<double>& a) {
    double s = 0.0;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) s += a.m[i][j] * a.m[i][j];
    return std::sqrt(std::max(0.0, s - a.m[0][0] * a.m[0][0])) / (std::sqrt(3.0) * a.m[0][0]);
}

// ============================================================================ drivers
struct RunArgs {
    const Scene* sc;
    const double* const* pp;  // parameters read by sampling decisions (detached)
    const double* const* pv;  // parameters read by differentiated values
    const View* views;
    int n_views, max_depth;
    uint32_t flags;
    uint64_t seed;
    int mode;
    int ckpt;                 // hybrid replay (mode 4): checkpoint interval k >= 1
    double gamma, eps;        // hybrid replay decision rule (Eq. 3): DI threshold, determinant threshold
    double sigma;             // mode 3: standard deviation of the regularisation noise u I (Sec. 4.2)
    const double* d_image;
    double* image;
    uint64_t* sig;
    const uint8_t* mask;
};

struct ThreadAcc {
    std::vector<std::vector<double>> g;
    int64_t n_vert = 0, n_path = 0;
    int64_t n_branch[3] = {0, 0, 0};  // hybrid replay (mode 4): decisions for the scalar update, inversion and
                                      // recomputation (one recomputation covers the rest of its block)
    int pix_slot = -1;              // slot whose per-pixel gradient image is requested
    std::vector<double> pix_g;      // that slot's gradient (every element) from the current pixel
};

static void collect(const PAcc<Var>& PV, const std::vector<double>& adj, ThreadAcc& acc) {
    for (auto& kv : PV.leaves) {
        int s = (int)(kv.first >> 40);
        uint32_t i = (uint32_t)(kv.first & ((1ll << 40) - 1));
        if (!acc.g[s].empty()) acc.g[s][i] += adj[kv.second.i];
        if (s == acc.pix_slot) acc.pix_g[i] += adj[kv.second.i];
    }
}

// One path: returns its contribution C[a][c][k] (sensor output, before the 1/spp mean)
// and, for the gradient modes, accumulates d(sum_a,c,k dC[a][c][k] C[a][c][k]) / d params.
static void run_path(const RunArgs& A, const View& vw, int px, int py, int s, const double* dC, double C[4][3][4],
                     uint64_t* sig_out, ThreadAcc& acc, Tape& tape, std::vector<double>& adj) {
    const World& w = A.sc->worlds[vw.world];
    PAcc<double> PP{A.pp};
    PAcc<double> PVd{A.pv};
    PathGeom g;
    trace_path(w, vw, px, py, s, A.seed, A.max_depth, A.flags, PP, g);
    if (sig_out) *sig_out = g.sig;
    acc.n_vert += (int64_t)g.v.size();
    acc.n_path += 1;
    const int B = (int)g.v.size();
    std::memset(C, 0, sizeof(double) * 48);

    if (A.mode == 0 || A.mode == 2 || A.mode == 3 || A.mode == 4 || A.mode == 5) {
        // primal: per-vertex W_b, E_b; forward sum and backward fold
        std::vector<VEval<double>> ev(B);
        for (int b = 0; b < B; ++b) eval_vertex(w, g.v[b], PVd, ev[b]);
        // mode 3 with noise (Sec. 4.2): every weight becomes W_b + u_b I, in the fold, the inversion
        // and the adjoint alike (the same noise in the primal and the adjoint phase)
        std::vector<double> nz(B, 0.0);
        if (A.mode == 3 && A.sigma > 0.0) {
            const uint32_t pix = (uint32_t)(py * vw.width + px);
            for (int b = 0; b < B; ++b) {
                nz[b] = pprb_noise(A.seed, pix, (uint32_t)s, vw.view_id, (uint32_t)(b + 1), A.sigma);
                for (int c = 0; c < 3; ++c)
                    for (int i = 0; i < 4; ++i) ev[b].W[c].m[i][i] += nz[b];
            }
        }
        M4<double> S[4];
        int na = sensor(vw, g.k_cam, g.x_sensor, PVd, S);
        std::vector<std::array<S4<double>, 3>> L(B + 1);
        for (int c = 0; c < 3; ++c) L[B][c] = szero<double>();
        for (int b = B - 1; b >= 0; --b)
            for (int c = 0; c < 3; ++c) L[b][c] = sadd(ev[b].E[c], mvec(ev[b].W[c], L[b + 1][c]));
        for (int a = 0; a < na; ++a)
            for (int c = 0; c < 3; ++c) {
                S4<double> o = mvec(S[a], L[0][c]);
                for (int k = 0; k < 4; ++k) C[a][c][k] = o.s[k];
            }
        if (A.mode == 0) return;

        // sensor term: local AD of the sensor Mueller matrices against the cached L[1]
        g_tape = &tape;
        tape.clear();
        {
            PAcc<Var> PV{A.pv, {}};
            M4<Var> SV[4];
            sensor(vw, g.k_cam, g.x_sensor, PV, SV);
            Var J(0.0);
            for (int a = 0; a < na; ++a)
                for (int c = 0; c < 3; ++c) {
                    S4<Var> o = mvec(SV[a], L[0][c]);
                    for (int k = 0; k < 4; ++k) J = J + o.s[k] * dC[(a * 3 + c) * 4 + k];
                }
            if (J.i >= 0) {
                adj.assign(tape.pa.size(), 0.0); adj[J.i] = 1.0;
                tape.backward(adj);
                collect(PV, adj, acc);
            }
        }
        // adjoint row vectors a_c = sum_a dC[a][c]^T S_a
        double av[3][4] = {};
        for (int a = 0; a < na; ++a)
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < 4; ++j)
                    for (int i = 0; i < 4; ++i) av[c][j] += dC[(a * 3 + c) * 4 + i] * S[a].m[i][j];

        // hybrid cached replay (Sec. 4.4): only the suffix values at the checkpoints b = 0, k, 2k, ...
        // are kept from the fold; the full fold is dropped before the replay
        const int K = A.ckpt > 0 ? A.ckpt : 1;
        std::vector<std::array<S4<double>, 3>> Lck;
        if (A.mode == 4) {
            for (int b = 0; b < B; b += K) Lck.push_back(L[b]);
            L.clear();
        }

        // replay: the same RNG stream re-traces the same path
        PathGeom g2;
        trace_path(w, vw, px, py, s, A.seed, A.max_depth, A.flags, PP, g2);
        const int B2 = (int)g2.v.size();
        // suffix source: cached fold (mode 2), inversion of the sampled weight (mode 3), or, in
        // mode 4, Eq. 3's rule inside each block of k vertices
        std::array<S4<double>, 3> Lcur;
        for (int ch = 0; ch < 3; ++ch) Lcur[ch] = A.mode == 4 ? szero<double>() : L[0][ch];
        std::array<M4<double>, 3> bt;   // mode 4: detached block throughput W_s .. W_b
        std::array<S4<double>, 3> Lrem; // mode 4: L[s] minus what vertices s .. b emit toward the block start
        bool recomputed = false;        // mode 4: this block's suffixes were recomputed
        for (int b = 0; b < B2; ++b) {
            std::array<S4<double>, 3> Lnext;
            if (A.mode == 2) {
                Lnext = L[b + 1];
            } else if (A.mode == 5) {
                // P-RB: an independent estimate of the suffix beyond vertex b, a new path from the ray
                // leaving it under its own key (the vertices keep their numbers)
                for (int ch = 0; ch < 3; ++ch) Lnext[ch] = szero<double>();
                if (b + 1 < B2) {
                    const Vtx& xb = g2.v[b];
                    PathGeom gs;
                    Sig ss;
                    trace_from(w, vw, (uint32_t)(py * vw.width + px), s, prb_seed(A.seed, (uint32_t)(b + 2)),
                               A.max_depth, A.flags, PP, spawn(xb.p, xb.ng, xb.wi), xb.wi, b + 2,
                               is_delta(w.mats[xb.mat].type), gs, ss);
                    for (int v = (int)gs.v.size() - 1; v >= 0; --v) {
                        VEval<double> es;
                        eval_vertex(w, gs.v[v], PVd, es);
                        for (int ch = 0; ch < 3; ++ch) Lnext[ch] = sadd(es.E[ch], mvec(es.W[ch], Lnext[ch]));
                    }
                }
            } else if (A.mode == 4) {
                const int nb = b + 1;
                if (b % K == 0) {  // block start: its checkpoint holds the suffix L[s]
                    for (int ch = 0; ch < 3; ++ch) { bt[ch] = meye<double>(); Lrem[ch] = Lck[b / K][ch]; }
                    recomputed = false;
                }
                // the detached weight and emission of vertex b extend the block throughput and use
                // up part of the remaining radiance: Lrem = bt L[b+1] afterwards
                VEval<double> evb;
                eval_vertex(w, g2.v[b], PVd, evb);
                for (int ch = 0; ch < 3; ++ch) {
                    S4<double> e = mvec(bt[ch], evb.E[ch]);
                    for (int q = 0; q < 4; ++q) Lrem[ch].s[q] -= e.s[q];
                    bt[ch] = mmul(bt[ch], evb.W[ch]);
                }
                const int c = ((nb + K - 1) / K) * K;  // the next checkpoint
                enum { CACHED, SCALAR, INVERT, RECOMPUTE } br = RECOMPUTE;
                bool decided = false;
                if (nb >= B2 || nb == c) {
                    br = CACHED;
                } else if (!recomputed) {
                    decided = true;
                    // one decision for the three channels, on the channel of largest throughput
                    // (the weights of a vertex differ between channels by a scale, which neither
                    // test sees); a channel without throughput leaves only recomputation
                    int cm = 0;
                    double mmin = bt[0].m[0][0];
                    for (int ch = 1; ch < 3; ++ch) {
                        if (bt[ch].m[0][0] > bt[cm].m[0][0]) cm = ch;
                        mmin = std::min(mmin, bt[ch].m[0][0]);
                    }
                    const double m00 = bt[cm].m[0][0];
                    if (mmin > 0.0 && depol_index(bt[cm]) < A.gamma) br = SCALAR;
                    else if (mmin > 0.0 && std::fabs(det4(bt[cm])) > A.eps * m00 * m00 * m00 * m00) br = INVERT;
                }
                if (br == RECOMPUTE) recomputed = true;
                if (decided) ++acc.n_branch[br == SCALAR ? 0 : br == INVERT ? 1 : 2];
                if (br == CACHED) {
                    for (int ch = 0; ch < 3; ++ch) Lnext[ch] = nb >= B2 ? szero<double>() : Lck[c / K][ch];
                } else if (br == SCALAR) {  // treated as depolarizing: intensity only
                    for (int ch = 0; ch < 3; ++ch) {
                        Lnext[ch] = szero<double>();
                        Lnext[ch].s[0] = Lrem[ch].s[0] / bt[ch].m[0][0];
                    }
                } else if (br == INVERT) {
                    for (int ch = 0; ch < 3; ++ch) Lnext[ch] = mvec(inverse4(bt[ch]), Lrem[ch]);
                } else {
                    // recompute L[v] = E_v + W_v L[v+1] for v = c-1 .. b+1 from the next checkpoint
                    Lnext = c >= B2 ? std::array<S4<double>, 3>{szero<double>(), szero<double>(), szero<double>()}
                                    : Lck[c / K];
                    for (int v = std::min(c, B2) - 1; v >= nb; --v) {
                        VEval<double> ev2;
                        eval_vertex(w, g2.v[v], PVd, ev2);
                        for (int ch = 0; ch < 3; ++ch) Lnext[ch] = sadd(ev2.E[ch], mvec(ev2.W[ch], Lnext[ch]));
                    }
                }
            } else {
                bool cont = g2.v[b].lobe != LOBE_NONE && g2.v[b].lobe != LOBE_INVALID;
                for (int c = 0; c < 3; ++c) {
                    if (!cont) { Lnext[c] = szero<double>(); continue; }
                    S4<double> r;
                    for (int k = 0; k < 4; ++k) r.s[k] = Lcur[c].s[k] - ev[b].E[c].s[k];
                    Lnext[c] = mvec(inverse4(ev[b].W[c]), r);
                }
            }
            tape.clear();
            PAcc<Var> PV{A.pv, {}};
            VEval<Var> e;
            eval_vertex(w, g2.v[b], PV, e);
            Var J(0.0);
            for (int c = 0; c < 3; ++c) {
                S4<Var> wl = mvec(e.W[c], Lnext[c]);
                for (int k = 0; k < 4; ++k) J = J + (e.E[c].s[k] + wl.s[k]) * av[c][k];
            }
            if (J.i >= 0) {
                adj.assign(tape.pa.size(), 0.0); adj[J.i] = 1.0;
                tape.backward(adj);
                collect(PV, adj, acc);
            }
            // a <- a W_b (detached; with the regularisation noise in mode 3)
            for (int c = 0; c < 3; ++c) {
                double na_[4] = {};
                for (int j = 0; j < 4; ++j) {
                    for (int i = 0; i < 4; ++i) na_[j] += av[c][i] * e.W[c].m[i][j].v;
                    if (A.mode == 3) na_[j] += av[c][j] * nz[b];
                }
                for (int j = 0; j < 4; ++j) av[c][j] = na_[j];
            }
            Lcur = Lnext;
        }
        return;
    }

    // mode 1: conventional reverse-mode AD, one tape over the whole path
    g_tape = &tape;
    tape.clear();
    PAcc<Var> PV{A.pv, {}};
    M4<Var> S[4];
    int na = sensor(vw, g.k_cam, g.x_sensor, PV, S);
    M4<Var> beta[3] = {meye<Var>(), meye<Var>(), meye<Var>()};
    S4<Var> Lo[3] = {szero<Var>(), szero<Var>(), szero<Var>()};
    for (int b = 0; b < B; ++b) {
        VEval<Var> ev;
        eval_vertex(w, g.v[b], PV, ev);
        for (int c = 0; c < 3; ++c) {
            Lo[c] = sadd(Lo[c], mvec(beta[c], ev.E[c]));
            if (b + 1 < B) beta[c] = mmul(beta[c], ev.W[c]);
        }
    }
    Var J(0.0);
    for (int a = 0; a < na; ++a)
        for (int c = 0; c < 3; ++c) {
            S4<Var> o = mvec(S[a], Lo[c]);
            for (int k = 0; k < 4; ++k) {
                C[a][c][k] = o.s[k].v;
                J = J + o.s[k] * dC[(a * 3 + c) * 4 + k];
            }
        }
    if (J.i >= 0) {
        adj.assign(tape.pa.size(), 0.0); adj[J.i] = 1.0;
        tape.backward(adj);
        collect(PV, adj, acc);
    }
}

static int n_analyzers(const View& v) {
    return (v.sensor == SENSOR_ANALYZER4 || v.sensor == SENSOR_LIGHTSTAGE4) ? 4 : 1;
}

}  // namespace ora

// ============================================================================ C API
using namespace ora;

static void set_err(char* err, int n, const char* msg) {
    if (err && n > 0) { std::snprintf(err, (size_t)n, "%s", msg); }
}

struct Reader {
    const uint8_t* p; size_t n, at = 0;
    bool get(void* dst, size_t k) {
        if (at + k > n) return false;
        if (k) std::memcpy(dst, p + at, k);  // (an empty array may have no storage: no copy at all)
        at += k;
        return true;
    }
};

extern "C" {

void* ppto_scene_load(const void* blob, size_t nbytes, char* err, int errlen) {
    Reader r{(const uint8_t*)blob, nbytes};
    uint32_t hdr[4];
    if (!r.get(hdr, 16) || hdr[0] != 0x31545050u || hdr[1] != 2u) { set_err(err, errlen, "bad header"); return nullptr; }
    Scene* sc = new Scene();
    sc->slot_numel.resize(hdr[2]);
    if (hdr[2] && !r.get(sc->slot_numel.data(), 4ull * hdr[2])) { delete sc; set_err(err, errlen, "truncated slots"); return nullptr; }
    sc->worlds.resize(hdr[3]);
    for (uint32_t wi = 0; wi < hdr[3]; ++wi) {
        World& w = sc->worlds[wi];
        uint32_t cnt[4];
        if (!r.get(cnt, 16)) { delete sc; set_err(err, errlen, "truncated world header"); return nullptr; }
        std::vector<float> tv(9ull * cnt[0]), tuv(6ull * cnt[0]), sph(4ull * cnt[1]);
        w.tmat.resize(cnt[0]); w.smat.resize(cnt[1]); w.mats.resize(cnt[2]); w.lights.resize(cnt[3]);
        bool ok = r.get(tv.data(), 4 * tv.size()) && r.get(tuv.data(), 4 * tuv.size()) &&
                  r.get(w.tmat.data(), 4ull * cnt[0]) && r.get(sph.data(), 4 * sph.size()) &&
                  r.get(w.smat.data(), 4ull * cnt[1]) && r.get(w.mats.data(), sizeof(Material) * cnt[2]) &&
                  r.get(w.lights.data(), sizeof(LightRec) * cnt[3]);
        if (!ok) { delete sc; set_err(err, errlen, "truncated world data"); return nullptr; }
        for (uint32_t i = 0; i < cnt[0]; ++i) {
            w.v0.push_back(f3(&tv[9 * i])); w.v1.push_back(f3(&tv[9 * i + 3])); w.v2.push_back(f3(&tv[9 * i + 6]));
            if (w.tmat[i] >= cnt[2]) { delete sc; set_err(err, errlen, "triangle material out of range"); return nullptr; }
        }
        w.uv.assign(tuv.begin(), tuv.end());
        for (uint32_t i = 0; i < cnt[1]; ++i) {
            w.sc.push_back(f3(&sph[4 * i])); w.sr.push_back(sph[4 * i + 3]);
            if (w.smat[i] >= cnt[2]) { delete sc; set_err(err, errlen, "sphere material out of range"); return nullptr; }
        }
        build_bvh(w);
    }
    if (r.at != r.n) { delete sc; set_err(err, errlen, "trailing bytes"); return nullptr; }
    return sc;
}

void ppto_scene_free(void* s) { delete (Scene*)s; }

int ppto_scene_counts(void* s, int world, int* out4) {
    Scene* sc = (Scene*)s;
    if (world < 0 || world >= (int)sc->worlds.size()) return -1;
    const World& w = sc->worlds[world];
    out4[0] = (int)w.v0.size(); out4[1] = (int)w.sc.size(); out4[2] = (int)w.mats.size(); out4[3] = (int)w.lights.size();
    return 0;
}

// mode 0: render; 1: conventional tape AD; 2: cached suffix replay; 3: basic polarized PRB (inversion).
// Image layout [V][A][crop_h][crop_w][3][4]; paths ordered (view, crop row, crop column, sample).
// Gradients are *added* into grads_out[slot] (NULL entries are skipped).
int ppto_run(void* scene, const double* const* params_path, const double* const* params_val, int n_slots,
             const void* views_, int n_views, int max_depth, uint32_t flags, uint64_t seed, int mode,
             const double* d_image, double* image_out, double* const* grads_out, uint64_t* sig_out,
             const uint8_t* path_mask, int64_t* stats, int nthreads, char* err, int errlen, int pix_slot,
             double* pix_grad, int ckpt_interval, double hybrid_gamma, double hybrid_eps, double pprb_sigma) {
    Scene* sc = (Scene*)scene;
    const View* views = (const View*)views_;
    if (!sc || n_slots != (int)sc->slot_numel.size()) { set_err(err, errlen, "slot count mismatch"); return -1; }
    if (max_depth < 1 || max_depth > 200) { set_err(err, errlen, "max_depth out of range"); return -1; }
    if (mode < 0 || mode > 5 || (mode > 0 && !d_image)) { set_err(err, errlen, "bad mode"); return -1; }
    if (mode == 4 && ckpt_interval < 1) { set_err(err, errlen, "checkpoint interval must be >= 1"); return -1; }
    std::vector<int64_t> img_off(n_views + 1, 0), path_off(n_views + 1, 0);
    for (int v = 0; v < n_views; ++v) {
        const View& vw = views[v];
        if (vw.world < 0 || vw.world >= (int)sc->worlds.size() || vw.spp < 1 || vw.width < 1 || vw.height < 1 ||
            vw.crop_x0 < 0 || vw.crop_y0 < 0 || vw.crop_w < 0 || vw.crop_h < 0 ||
            vw.crop_x0 + vw.crop_w > vw.width || vw.crop_y0 + vw.crop_h > vw.height) {
            set_err(err, errlen, "bad view"); return -1;
        }
        if (vw.sensor == SENSOR_POLARIZER &&
            (vw.theta_slot < 0 || vw.theta_slot >= n_slots || vw.theta_off < 0 ||
             (uint32_t)vw.theta_off >= sc->slot_numel[vw.theta_slot])) {
            set_err(err, errlen, "bad theta slot"); return -1;
        }
        img_off[v + 1] = img_off[v] + (int64_t)n_analyzers(vw) * vw.crop_w * vw.crop_h * 12;
        path_off[v + 1] = path_off[v] + (int64_t)vw.crop_w * vw.crop_h * vw.spp;
    }
    g_gauge = (flags & FLAG_GAUGE) ? 1 : 0;
    RunArgs A{sc, params_path, params_val ? params_val : params_path, views, n_views, max_depth, flags, seed, mode,
              ckpt_interval, hybrid_gamma, hybrid_eps, pprb_sigma, d_image, image_out, sig_out, path_mask};
    // per-pixel index (view, crop row, crop column) for the gradient-image output
    std::vector<int64_t> pix_off(n_views + 1, 0);
    for (int v = 0; v < n_views; ++v) pix_off[v + 1] = pix_off[v] + (int64_t)views[v].crop_w * views[v].crop_h;
    auto pix_index = [&](int v, int lx, int ly) { return pix_off[v] + (int64_t)ly * views[v].crop_w + lx; };
    // work items: (view, crop row)
    std::vector<std::pair<int, int>> items;
    for (int v = 0; v < n_views; ++v)
        for (int y = 0; y < views[v].crop_h; ++y) items.push_back({v, y});
    int nt = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
    int maxt = omp_get_max_threads();
    if (nthreads <= 0) nt = maxt;
#endif
    std::vector<ThreadAcc> accs(nt);
    for (auto& a : accs) {
        a.pix_slot = pix_grad ? pix_slot : -1;
        if (a.pix_slot >= 0) a.pix_g.assign(sc->slot_numel[pix_slot], 0.0);
        a.g.resize(n_slots);
        if (mode > 0)
            for (int s = 0; s < n_slots; ++s)
                if (grads_out && grads_out[s]) a.g[s].assign(sc->slot_numel[s], 0.0);
    }
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        ThreadAcc& acc = accs[tid];
        Tape tape;
        std::vector<double> adj;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (long it = 0; it < (long)items.size(); ++it) {
            int v = items[it].first, ly = items[it].second;
            const View& vw = views[v];
            int na = n_analyzers(vw);
            for (int lx = 0; lx < vw.crop_w; ++lx) {
                int px = vw.crop_x0 + lx, py = vw.crop_y0 + ly;
                int64_t pix_img = img_off[v] + ((int64_t)ly * vw.crop_w + lx) * 12;
                int64_t a_stride = (int64_t)vw.crop_w * vw.crop_h * 12;
                double dC[48] = {};
                if (mode > 0)
                    for (int a = 0; a < na; ++a)
                        for (int k = 0; k < 12; ++k) dC[a * 12 + k] = d_image[pix_img + a * a_stride + k] / vw.spp;
                double sum[4][3][4] = {};
                std::fill(acc.pix_g.begin(), acc.pix_g.end(), 0.0);
                for (int s = 0; s < vw.spp; ++s) {
                    int64_t pidx = path_off[v] + ((int64_t)ly * vw.crop_w + lx) * vw.spp + s;
                    if (path_mask && !path_mask[pidx]) { if (sig_out) sig_out[pidx] = 0; continue; }
                    double C[4][3][4];
                    run_path(A, vw, px, py, s, dC, C, sig_out ? &sig_out[pidx] : nullptr, acc, tape, adj);
                    for (int a = 0; a < na; ++a)
                        for (int c = 0; c < 3; ++c)
                            for (int k = 0; k < 4; ++k) sum[a][c][k] += C[a][c][k];
                }
                if (pix_grad && mode > 0)
                    for (size_t i = 0; i < acc.pix_g.size(); ++i)
                        pix_grad[pix_index(v, lx, ly) * (int64_t)acc.pix_g.size() + (int64_t)i] = acc.pix_g[i];
                if (image_out)
                    for (int a = 0; a < na; ++a)
                        for (int c = 0; c < 3; ++c)
                            for (int k = 0; k < 4; ++k)
                                image_out[pix_img + a * a_stride + c * 4 + k] = sum[a][c][k] / vw.spp;
            }
        }
    }
    int64_t nv = 0, np = 0, nbr[3] = {0, 0, 0};
    for (auto& a : accs) {
        nv += a.n_vert; np += a.n_path;
        for (int k = 0; k < 3; ++k) nbr[k] += a.n_branch[k];
        if (mode > 0)
            for (int s = 0; s < n_slots; ++s)
                if (grads_out && grads_out[s])
                    for (size_t i = 0; i < a.g[s].size(); ++i) grads_out[s][i] += a.g[s][i];
    }
    if (stats) {
        stats[0] = nv; stats[1] = np;
        for (int k = 0; k < 3; ++k) stats[2 + k] = nbr[k];
    }
    g_gauge = 0;
    return 0;
}

// ---- unit-level entry points used by the pin tests
void ppto_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out) { philox(ctr, seed, out); }
void ppto_fresnel(double ci, double m_re, double m_im, double* MR, double* MT) {
    M4<double> R, T;
    fresnel<double>(ci, Cx<double>{m_re, m_im}, &R, &T);
    for (int i = 0; i < 16; ++i) { MR[i] = R.m[i / 4][i % 4]; MT[i] = T.m[i / 4][i % 4]; }
}
void ppto_polarizer(double th, double* M) {
    M4<double> P = polarizer<double>(th);
    for (int i = 0; i < 16; ++i) M[i] = P.m[i / 4][i % 4];
}
void ppto_retarder(double delta, double* M) {
    M4<double> P = retarder(delta);
    for (int i = 0; i < 16; ++i) M[i] = P.m[i / 4][i % 4];
}
void ppto_rotator(const double* k, const double* xf, const double* xt, double* M) {
    M4<double> P = rotator(V3{k[0], k[1], k[2]}, V3{xf[0], xf[1], xf[2]}, V3{xt[0], xt[1], xt[2]});
    for (int i = 0; i < 16; ++i) M[i] = P.m[i / 4][i % 4];
}
void ppto_canon_x(const double* k, double* x) {
    V3 r = canon_x(V3{k[0], k[1], k[2]});
    x[0] = r.x; x[1] = r.y; x[2] = r.z;
}
// GGX pBRDF value f (16, canonical frames) and the scalars D and G for a conductor/dielectric.
void ppto_ggx_eval(const double* ns, const double* wi, const double* wo, double alpha, double m_re, double m_im,
                   double* f16) {
    M4<double> f = ggx_f<double>(VT<double>{ns[0], ns[1], ns[2]}, V3{wi[0], wi[1], wi[2]}, V3{wo[0], wo[1], wo[2]},
                                 alpha, Cx<double>{m_re, m_im});
    for (int i = 0; i < 16; ++i) f16[i] = f.m[i / 4][i % 4];
}
// The microfacet distribution D(cos_h), the Smith masking term G1(cos_w) and one Walter et al.
// half-vector sample (returns the lobe; wi and pdf are written for a valid sample).
double ppto_ggx_D(double cos_h, double alpha) { return ggx_D<double>(cos_h, alpha); }
double ppto_smith_G1(double cos_w, double alpha) { return smith_G1<double>(cos_w, alpha); }
int ppto_sample_glossy(const double* ns, const double* wo, double alpha, double u1, double u2, double* wi,
                       double* pdf) {
    V3 w{0.0, 0.0, 0.0};
    double p = 0.0;
    int lobe = sample_glossy(V3{ns[0], ns[1], ns[2]}, V3{wo[0], wo[1], wo[2]}, alpha, u1, u2, w, p);
    wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
    *pdf = p;
    return lobe;
}
int ppto_trace(void* scene, int world, const double* o, const double* d, double tmax, int any_hit, int brute,
               double* t_out) {
    Scene* sc = (Scene*)scene;
    Hit h;
    bool ok = trace(sc->worlds[world], V3{o[0], o[1], o[2]}, V3{d[0], d[1], d[2]}, tmax, any_hit != 0, brute != 0, h);
    if (t_out) *t_out = ok ? h.t : -1.0;
    return ok ? h.prim : -1;
}

}  // extern "C"

extern "C" void ppto_philox_n(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) ora::philox(ctr + 4 * i, seed, out + 4 * i);
}
