"""Pins of the oracle's estimator pieces that the closed-form scenes of the other pin files do not
reach: the absolute scale of next-event estimation (the Lambertian value rho/pi, the light's area,
both cosines, the squared distance and the uniform choice among the lights), the GGX
microfacet functions (normalisation of D, Smith masking, and the density of Walter et al.'s
half-vector sampling), and the lobe weights of the smooth dielectric (reflection and
transmission divided by their selection probabilities).

Each pin compares with something the oracle does not compute: a closed form, a quadrature of the
defining integral, or an independent estimator of the same expectation (a mean within four
standard errors).  Each test names the factor whose omission it catches.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import scenegen as sg


# ----------------------------------------------------------------------------- next-event scale
def _rot(v, axis, ang):
    """Rodrigues rotation of v about the unit axis by ang."""
    v, k = np.asarray(v, np.float64), np.asarray(axis, np.float64)
    k = k / np.linalg.norm(k)
    return v * np.cos(ang) + np.cross(k, v) * np.sin(ang) + k * np.dot(k, v) * (1 - np.cos(ang))


def _tiny_light(w, centre, tilt_axis, tilt, size, s_le):
    """A size x size light at centre whose normal is the direction to the origin turned by tilt
    about tilt_axis; returns its (float32-rounded) corner, edges and normal."""
    c = np.asarray(centre, np.float64)
    n = _rot(-c / np.linalg.norm(c), tilt_axis, tilt)
    a = np.cross(n, [0.0, 0.0, 1.0]) if abs(n[2]) < 0.9 else np.cross(n, [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    eu, ev = a * size, b * size          # eu x ev = size^2 n: one-sided toward the origin
    p0 = c - 0.5 * (eu + ev)
    w.add_light(p0, eu, ev, s_le)
    r = lambda x: np.asarray(x, np.float32).astype(np.float64)
    return r(p0), r(eu), r(ev)


def _nee_closed_form(albedo, le, p0, eu, ev, x=np.zeros(3), n=np.array([0.0, 1.0, 0.0])):
    """rho/pi Le A cos_x cos_y / r^2 for a point x on a Lambertian surface with normal n and a light
    small enough that the integrand is constant over it (evaluated at the light's centre)."""
    y = p0 + 0.5 * (eu + ev)
    nl = np.cross(eu, ev)
    area = np.linalg.norm(nl)
    nl /= area
    d = y - x
    r2 = float(d @ d)
    wl = d / np.sqrt(r2)
    cos_x, cos_y = float(n @ wl), float(-nl @ wl)
    return np.asarray(albedo) / np.pi * le * area * cos_x * cos_y / r2, cos_x, cos_y


def _plane_with_lights(lights, albedo=(0.6, 0.5, 0.4), le=5.0, size=1e-4):
    sc = sg.Scene()
    s_alb = sc.add_slot("albedo", list(albedo))
    s_le = sc.add_slot("light_Le", [le, le, le])
    w = sc.add_world()
    m = w.add_material(type=sg.MAT_LAMBERT, albedo_slot=s_alb)
    w.add_quad((-50.0, 0.0, 50.0), (100.0, 0.0, 0.0), (0.0, 0.0, -100.0), m)  # y = 0, normal +y
    geo = [_tiny_light(w, c, ax, t, size, s_le) for c, ax, t in lights]
    return sc, geo


def _render_plane(sc, spp=4):
    # straight down at the origin through a 0.005-degree field: every path's vertex lies within
    # 2e-4 of the origin, and one bounce (depth 2) makes the image the next-event term alone
    v = np.asarray([sg.make_view(0, 4, 4, spp, (0.0, 4.0, 0.0), (0, 0, 0), (0, 0, -1), 0.005, sg.SENSOR_NONE)],
                   sg.VIEW_DTYPE)
    img = oracle.OracleScene.from_scene(sc).run(sc.params(), v, 2, 11)["image"]
    return img.reshape(-1, 3, 4)


def test_nee_absolute_scale_one_light(oracle_lib):
    # light 20 away, 0.5 rad off the surface normal, its own normal turned 0.3 rad away from the
    # point: s0 = rho/pi Le A cos_x cos_y / r^2 per channel.  Dropping pi (x3.14), the area (x1e8),
    # cos_x (x1.14), cos_y (x1.05) or r^2 fails; the image is unpolarized.
    c = 20.0 * np.array([np.sin(0.5), np.cos(0.5), 0.0])
    sc, geo = _plane_with_lights([(c, (0.0, 0.0, 1.0), 0.3)])
    img = _render_plane(sc)
    expect, cos_x, cos_y = _nee_closed_form((0.6, 0.5, 0.4), 5.0, *geo[0])
    assert abs(cos_x - np.cos(0.5)) < 1e-6 and abs(cos_y - np.cos(0.3)) < 1e-6
    assert np.allclose(img[..., 0], expect[None, :], rtol=2e-5, atol=0.0), (img[..., 0].mean(0), expect)
    assert np.allclose(img[..., 1:], 0.0, atol=1e-12 * expect.max())


def test_nee_absolute_scale_two_lights(oracle_lib):
    # two lights at the same distance and angles (mirror images about the normal's plane): the
    # estimator picks one uniformly and weights it by the number of lights, so every sample reads
    # the sum of both; a missing light count halves the image
    c1 = 20.0 * np.array([np.sin(0.5), np.cos(0.5), 0.0])
    c2 = 20.0 * np.array([0.0, np.cos(0.5), np.sin(0.5)])
    sc, geo = _plane_with_lights([(c1, (0.0, 0.0, 1.0), 0.3), (c2, (-1.0, 0.0, 0.0), 0.3)])
    img = _render_plane(sc)
    e1 = _nee_closed_form((0.6, 0.5, 0.4), 5.0, *geo[0])[0]
    e2 = _nee_closed_form((0.6, 0.5, 0.4), 5.0, *geo[1])[0]
    assert np.allclose(e1, e2, rtol=1e-6)
    assert np.allclose(img[..., 0], (e1 + e2)[None, :], rtol=2e-5, atol=0.0), (img[..., 0].mean(0), e1 + e2)


def _z_score(a, b):
    """Mean of the per-pixel differences over its standard error (pixels are independent)."""
    d = (np.asarray(a) - np.asarray(b)).ravel()
    se = d.std(ddof=1) / np.sqrt(d.size)
    return float(d.mean() / se), float(se)


def test_nee_on_equals_bsdf_sampling_in_expectation(oracle_lib):
    # two unbiased estimators of the same image: next-event estimation (emitter hits count only
    # after the camera or a delta vertex) and pure BSDF sampling (every emitter hit counts).  The
    # per-pixel s0 difference averages to zero within four standard errors; the standard error is
    # below 1% of the image, so a next-event term off by the area (x4), pi or the light count fails.
    wl = sg.config1()
    v = wl.views.copy()
    v["spp"] = 512
    v["sensor"] = sg.SENSOR_NONE
    osc = oracle.OracleScene.from_scene(wl.scene)
    p = wl.scene.params()
    a = osc.run(p, v, wl.max_depth, 21)["image"].reshape(-1, 3, 4)[..., 0]
    b = osc.run(p, v, wl.max_depth, 21, flags=sg.FLAG_NO_NEE)["image"].reshape(-1, 3, 4)[..., 0]
    z, se = _z_score(a, b)
    print(f"NEE vs BSDF sampling: z {z:.2f}, standard error {se / a.mean():.2e} of the mean")
    assert abs(z) < 4.0
    assert se < 0.01 * a.mean()


# ----------------------------------------------------------------------------- GGX
ALPHAS = (0.05, 0.2, 0.5, 1.0)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_ggx_distribution_is_normalised(oracle_lib, alpha):
    # the projected microfacet area integrates to one: 2 pi int_0^1 D(mu) mu dmu = 1.  A D without
    # its 1/pi, or with alpha in place of alpha^2, fails.
    val, err = integrate.quad(lambda mu: oracle.ggx_D(mu, alpha) * mu, 0.0, 1.0, points=[1.0 - alpha * alpha],
                              epsabs=1e-13, epsrel=1e-12, limit=400)
    assert abs(2.0 * np.pi * val - 1.0) < 1e-9, 2.0 * np.pi * val


def _phi_integral(sin_o, cos_o, mu):
    """int_0^2pi max(0, wo . h) dphi for h at polar cosine mu (wo at polar sine/cosine sin_o, cos_o)."""
    A, B = sin_o * np.sqrt(max(0.0, 1.0 - mu * mu)), cos_o * mu
    if B >= A:
        return 2.0 * np.pi * B
    if B <= -A:
        return 0.0
    return 2.0 * (B * np.arccos(-B / A) + np.sqrt(A * A - B * B))


@pytest.mark.parametrize("alpha", (0.1, 0.3, 0.7))
@pytest.mark.parametrize("theta_o", (0.2, 0.7, 1.2, 1.45))
def test_smith_masking_projected_area(oracle_lib, alpha, theta_o):
    # Heitz 2014: the visible projected microfacet area equals the projected macro-surface,
    # G1(wo) int max(0, wo . h) D(h) dw_h = cos theta_o.  A wrong Lambda (the 1/2, the square root,
    # tan^2 against tan) fails.
    so, co = np.sin(theta_o), np.cos(theta_o)
    val, _ = integrate.quad(lambda mu: oracle.ggx_D(mu, alpha) * _phi_integral(so, co, mu), 0.0, 1.0,
                            points=[1.0 - alpha * alpha], epsabs=1e-13, epsrel=1e-11, limit=400)
    assert abs(oracle.smith_G1(co, alpha) * val / co - 1.0) < 1e-8


def _albedo_quadrature(wo, alpha, m, n_t=96, n_p=192):
    """int f00(wi, wo) cos theta_i dw_i over the upper hemisphere (Gauss-Legendre in cos theta and phi)."""
    xt, wt = np.polynomial.legendre.leggauss(n_t)
    xp, wp = np.polynomial.legendre.leggauss(n_p)
    mu, wmu = 0.5 * (xt + 1.0), 0.5 * wt
    ph, wph = np.pi * (xp + 1.0), np.pi * wp
    ns = np.array([0.0, 0.0, 1.0])
    tot = 0.0
    for m_i, w_i in zip(mu, wmu):
        s = np.sqrt(1.0 - m_i * m_i)
        for p_j, w_j in zip(ph, wph):
            wi = np.array([s * np.cos(p_j), s * np.sin(p_j), m_i])
            tot += w_i * w_j * oracle.ggx_eval(ns, wi, wo, alpha, m)[0, 0] * m_i
    return tot


def _albedo_sampled(wo, alpha, m, n=128):
    """Mean of f00 cos / pdf over a stratified n x n grid of the sampler's two uniforms (rejected
    samples count zero)."""
    ns = np.array([0.0, 0.0, 1.0])
    tot = 0.0
    for i in range(n):
        for j in range(n):
            lobe, wi, pdf = oracle.sample_glossy(ns, wo, alpha, (i + 0.5) / n, (j + 0.5) / n)
            if lobe != oracle.LOBE_GLOSSY:
                continue
            tot += oracle.ggx_eval(ns, wi, wo, alpha, m)[0, 0] * wi[2] / pdf
    return tot / (n * n)


@pytest.mark.parametrize("m", (1.5, 0.5 + 3.0j))
@pytest.mark.parametrize("alpha,theta_o", ((0.3, 0.4), (0.6, 1.0)))
def test_ggx_sampling_density(oracle_lib, m, alpha, theta_o):
    # the estimator E[f cos / pdf] of Walter et al.'s sampling equals the quadrature of
    # int f cos dw_i (the directional albedo): a pdf without the 1/(4 |wo.h|) Jacobian or the
    # cos(theta_h) factor fails
    wo = np.array([np.sin(theta_o), 0.0, np.cos(theta_o)])
    q = _albedo_quadrature(wo, alpha, m)
    s = _albedo_sampled(wo, alpha, m)
    print(f"GGX albedo m={m} alpha={alpha} theta_o={theta_o}: quadrature {q:.6f}, sampled {s:.6f}")
    assert 0.01 < q < 1.0
    assert abs(s / q - 1.0) < 2e-3


# ----------------------------------------------------------------------------- smooth dielectric
def _glass_in_furnace():
    """A glass sphere and a tilted glass cube (IOR 1.5) inside a closed, uniformly emitting sphere."""
    sc = sg.Scene()
    s_ior = sc.add_slot("ior", [1.5])
    s_le = sc.add_slot("emission", [2.0, 2.0, 2.0])
    w = sc.add_world()
    m_glass = w.add_material(type=sg.MAT_DIELECTRIC, eta_slot=s_ior)
    m_emit = w.add_material(type=sg.MAT_EMITTER, emit_slot=s_le)
    w.add_sphere((0.0, 0.0, 0.0), -10.0, m_emit)  # inward normals: emits into the enclosure
    w.add_sphere((-0.8, 0.0, 0.0), 0.7, m_glass)
    # unit cube, rotated, outward-facing quads
    R = np.eye(3)
    for ax, ang in (((1, 0, 0), 0.5), ((0, 1, 0), 0.7)):
        R = np.stack([_rot(R[:, k], ax, ang) for k in range(3)], 1)
    ctr = np.array([0.9, 0.0, 0.0])
    for k in range(3):
        for sgn in (-1.0, 1.0):
            n = np.zeros(3); n[k] = sgn
            u = np.zeros(3); u[(k + 1) % 3] = 1.0
            v = np.cross(n, u)
            p0 = ctr + R @ (0.35 * n - 0.35 * u - 0.35 * v)
            w.add_quad(p0, R @ (0.7 * u), R @ (0.7 * v), m_glass)
    return sc


def test_dielectric_lobe_weights_furnace(oracle_lib):
    # inside a uniform unpolarized enclosure a lossless dielectric is invisible: every pixel's
    # expected Stokes vector is (Le, 0, 0, 0).  Reflection and transmission are chosen with
    # probability P_R = F and weighted M_R / P_R and M_T / (1 - P_R); a weight without its
    # probability, a P_R from another cosine, or a transmission without the flux factor fails.
    # The tilted cube adds total internal reflection.
    sc = _glass_in_furnace()
    v = np.asarray([sg.make_view(0, 24, 24, 16, (0.0, 0.3, 4.0), (0.05, 0.0, 0.0), (0, 1, 0), 38.0,
                                 sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    img = oracle.OracleScene.from_scene(sc).run(sc.params(), v, 48, 5, flags=sg.FLAG_NO_NEE)["image"]
    img = img.reshape(-1, 3, 4)
    le = 2.0
    z0, se0 = _z_score(img[..., 0], np.full(img[..., 0].shape, le))
    print(f"dielectric furnace: s0 mean {img[..., 0].mean():.6f} (z {z0:.2f}, se {se0:.1e})")
    assert abs(z0) < 4.0 and se0 < 2e-3 * le
    for k in (1, 2, 3):
        zk, sek = _z_score(img[..., k], np.zeros(img[..., k].shape))
        print(f"  s{k} mean {img[..., k].mean():.2e} (z {zk:.2f})")
        assert abs(zk) < 4.0
    # many pixels see glass (the expected value alone would hold for empty pixels too)
    assert np.mean(np.abs(img[..., 0] - le) > 1e-9) > 0.3
