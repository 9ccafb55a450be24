"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the fact it checks: published known-answer vectors, closed forms of optics
(Malus's law, halving through a polarizer, Fresnel special cases), identities of Mueller
calculus, a furnace scene with a closed-form value and gradient, invariance under the
(arbitrary) choice of Stokes frames, and finite differences of the estimator.
"""
import os

import numpy as np
import pytest

import oracle
import scenegen as sg

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------- RNG
def test_philox_known_answers(oracle_lib):
    n = 0
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = oracle.philox(w[4] | (w[5] << 32), w[:4])
        assert [int(x) for x in out] == w[6:]
        n += 1
    assert n == 3


def test_philox_uniformity_chi2(oracle_lib):
    rng = np.random.default_rng(0)
    seed = int(rng.integers(0, 2**63))
    vals = []
    for i in range(4000):
        vals.extend(oracle.philox(seed, [i, 7, (3 << 8) | 1, 0]))
    u = (np.asarray(vals, np.uint64) >> 8).astype(np.float64) / 2**24
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    exp = len(u) / 64
    chi2 = np.sum((hist - exp) ** 2 / exp)
    assert chi2 < 120  # 63 dof, p ~ 1e-5
    assert u.min() >= 0 and u.max() < 1


# ----------------------------------------------------------------------------- Mueller identities
def test_polarizer_rank_idempotent_halving(oracle_lib):
    for th in np.linspace(0, np.pi, 7):
        P = oracle.polarizer(th)
        assert np.linalg.matrix_rank(P, tol=1e-12) == 1  # rank-deficient (Sec. 4.1)
        assert np.allclose(P @ P, P, atol=1e-14)
        out = P @ np.array([1.0, 0, 0, 0])
        assert np.allclose(out, 0.5 * np.array([1, np.cos(2 * th), np.sin(2 * th), 0]), atol=1e-14)


def test_malus_between_polarizers(oracle_lib):
    for a, b in [(0.1, 0.9), (0.3, 0.3), (1.0, 2.5)]:
        s = oracle.polarizer(b) @ oracle.polarizer(a) @ np.array([1.0, 0, 0, 0])
        assert np.isclose(s[0], 0.5 * np.cos(a - b) ** 2, atol=1e-14)


def _basis(k, ang):
    x0 = oracle.canon_x(k)
    y0 = np.cross(k, x0)
    return np.cos(ang) * x0 + np.sin(ang) * y0


def test_rotator_group_laws(oracle_lib):
    rng = np.random.default_rng(1)
    k = rng.normal(size=3); k /= np.linalg.norm(k)
    a, b = 0.37, -1.21
    xa, xab, x0 = _basis(k, a), _basis(k, a + b), _basis(k, 0.0)
    Ra = oracle.rotator(k, x0, xa)
    Rb = oracle.rotator(k, xa, xab)
    Rab = oracle.rotator(k, x0, xab)
    assert np.allclose(Rb @ Ra, Rab, atol=1e-13)
    assert np.allclose(oracle.rotator(k, x0, -x0), np.eye(4), atol=1e-13)  # R(pi) = I
    # a polarizer expressed in a rotated basis is the polarizer at the shifted angle
    th = 0.8
    assert np.allclose(Ra @ oracle.polarizer(th) @ Ra.T, oracle.polarizer(th - a), atol=1e-13)


def test_retarder_invertible_qwp(oracle_lib):
    Q = oracle.retarder(np.pi / 2)
    assert np.isclose(np.linalg.det(Q), 1.0, atol=1e-14)  # invertible (Sec. 4.1)
    # two quarter-wave plates make a half-wave plate, which mirrors +45 deg light to -45 deg
    assert np.allclose(Q @ Q @ np.array([1, 0, 1.0, 0]), [1, 0, -1.0, 0], atol=1e-14)
    # a QWP at 0 turns +45 deg linear light into fully circular light
    s = Q @ np.array([1, 0, 1.0, 0])
    assert np.isclose(abs(s[3]), 1.0, atol=1e-14)


def test_ggx_pbrdf_is_non_depolarizing(oracle_lib):
    # a microfacet pBRDF is a scalar times a Fresnel Mueller matrix in rotated frames, hence
    # non-depolarizing (sum M_ij^2 = 4 M00^2) and, away from Brewster/TIR, of full rank
    # (the depolarizing Lambertian case is pinned by the furnace test: s1 = s2 = s3 = 0)
    ns = np.array([0, 0, 1.0])
    wi = np.array([0.3, 0.1, 0.9]); wi /= np.linalg.norm(wi)
    wo = np.array([-0.2, 0.4, 0.8]); wo /= np.linalg.norm(wo)
    for m in (1.5, complex(0.4, 3.0)):
        f = oracle.ggx_eval(ns, wi, wo, 0.3, m)
        assert np.linalg.matrix_rank(f, tol=1e-12) == 4
        assert np.isclose(np.sum(f ** 2), 4 * f[0, 0] ** 2, rtol=1e-12)


# ----------------------------------------------------------------------------- Fresnel closed forms
@pytest.mark.parametrize("eta", [1.33, 1.5, 2.4])
def test_fresnel_normal_incidence_and_energy(oracle_lib, eta):
    R, T = oracle.fresnel(1.0, eta)
    assert np.isclose(R[0, 0], ((eta - 1) / (eta + 1)) ** 2, rtol=1e-13)
    for ci in [1.0, 0.8, 0.5, 0.2, 0.05]:
        R, T = oracle.fresnel(ci, eta)
        # energy conservation separately for s- and p-polarized light
        for s in ([1, 1, 0, 0.0], [1, -1, 0, 0.0], [1, 0, 0, 0.0]):
            assert np.isclose((R @ s)[0] + (T @ s)[0], s[0], rtol=1e-13)
        # a Jones-derived (non-depolarizing) Mueller matrix: sum M_ij^2 = 4 M00^2
        for M in (R, T):
            assert np.isclose(np.sum(M ** 2), 4 * M[0, 0] ** 2, rtol=1e-12)


def test_fresnel_brewster(oracle_lib):
    eta = 1.5
    th = np.arctan(eta)
    R, _ = oracle.fresnel(np.cos(th), eta)
    # Rp = 0 at Brewster's angle: a = b, so reflected light is fully s-polarized
    assert np.isclose(R[0, 0], R[0, 1], atol=1e-15)
    out = R @ np.array([1.0, 0, 0, 0])
    assert np.isclose(out[1] / out[0], 1.0, atol=1e-12)  # DoLP = 1 along s
    rs = (np.cos(th) - eta * np.sqrt(1 - np.sin(th) ** 2 / eta ** 2)) / (np.cos(th) + eta * np.sqrt(1 - np.sin(th) ** 2 / eta ** 2))
    assert np.isclose(R[0, 0], rs ** 2 / 2, rtol=1e-12)


def test_fresnel_total_internal_reflection(oracle_lib):
    m = 1 / 1.5  # from glass into air
    crit = np.arcsin(m)
    for th in [crit + 0.05, crit + 0.3, 1.4]:
        R, T = oracle.fresnel(np.cos(th), m)
        assert np.isclose(R[0, 0], 1.0, atol=1e-14) and abs(R[0, 1]) < 1e-14
        assert np.allclose(T, 0, atol=1e-14)
        # pure retarder: the (s2, s3) block is a rotation
        assert np.isclose(R[2, 2] ** 2 + R[2, 3] ** 2, 1.0, atol=1e-13)


@pytest.mark.parametrize("n,k", [(0.2, 3.0), (1.5, 2.0), (0.5, 5.0)])
def test_conductor_normal_incidence(oracle_lib, n, k):
    R, T = oracle.fresnel(1.0, complex(n, k))
    assert np.isclose(R[0, 0], ((n - 1) ** 2 + k ** 2) / ((n + 1) ** 2 + k ** 2), rtol=1e-13)
    R2, _ = oracle.fresnel(0.4, complex(n, k))
    assert np.isclose(np.sum(R2 ** 2), 4 * R2[0, 0] ** 2, rtol=1e-12)


# ----------------------------------------------------------------------------- closed-form scenes
def _render(scene, views, depth, seed=7, flags=0, params=None, sensor=None):
    osc = oracle.OracleScene.from_scene(scene)
    p = scene.params() if params is None else params
    return osc.run(p, views, depth, seed, flags=flags)


def test_halving_and_unpolarized_wall(oracle_lib):
    sc, s_th = sg.emitter_wall_scene(le=10.0)
    for th in [0.0, 0.4, 1.3]:
        p = sc.params(); p[s_th][0] = th
        v = np.asarray([sg.make_view(0, 8, 8, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 30.0, sg.SENSOR_POLARIZER, s_th)], sg.VIEW_DTYPE)
        img = _render(sc, v, 3, params=p)["image"].reshape(-1, 3, 4)
        assert np.allclose(img[..., 0], 5.0, rtol=1e-14)  # half of the unpolarized radiance
    v = np.asarray([sg.make_view(0, 8, 8, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 30.0, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    img = _render(sc, v, 3)["image"].reshape(-1, 3, 4)
    assert np.allclose(img[..., 0], 10.0) and np.allclose(img[..., 1:], 0.0, atol=1e-13)


@pytest.mark.parametrize("theta,alpha", [(0.0, 0.0), (0.3, 1.1), (2.0, 0.4), (0.7, 0.7 + np.pi / 2)])
def test_malus_through_sheet(oracle_lib, theta, alpha):
    sc, s_th = sg.emitter_wall_scene(le=10.0, sheets=(alpha,))
    p = sc.params(); p[s_th][0] = theta
    # near-paraxial camera so the sheet axis projects onto itself
    v = np.asarray([sg.make_view(0, 4, 4, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 0.01, sg.SENSOR_POLARIZER, s_th)], sg.VIEW_DTYPE)
    img = _render(sc, v, 4, params=p)["image"].reshape(-1, 3, 4)
    assert np.allclose(img[..., 0], 5.0 * np.cos(theta - alpha) ** 2, atol=1e-7)


@pytest.mark.parametrize("n", [1, 3, 8])
def test_polarizer_chain(oracle_lib, n):
    # light -> sheet at 0 -> sheets at k pi / 2n (k = 1..n) -> camera without filter
    angles_light_first = [0.0] + [k * np.pi / (2 * n) for k in range(1, n + 1)]
    sc, _ = sg.emitter_wall_scene(le=10.0, sheets=tuple(reversed(angles_light_first)), z_light=-(n + 6.0))
    v = np.asarray([sg.make_view(0, 4, 4, 1, (0, 0, 0), (0, 0, -1), (0, 1, 0), 0.01, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    img = _render(sc, v, n + 3)["image"].reshape(-1, 3, 4)
    expect = 5.0 * np.cos(np.pi / (2 * n)) ** (2 * n)
    assert np.allclose(img[..., 0], expect, rtol=1e-6)
    assert np.allclose(img[..., 1], -expect, rtol=1e-6)  # polarized along the last axis (pi/2)
    # one bounce too few: the emitter is never reached
    img2 = _render(sc, v, n + 1)["image"]
    assert np.allclose(img2, 0.0)


@pytest.mark.parametrize("depth", [1, 2, 5])
def test_furnace_value_and_gradient(oracle_lib, depth):
    sc, s_th = sg.furnace_scene(rho=0.6, le=1.5)
    rho, le = float(sc.slot_values[sc.slot("albedo")][0]), float(sc.slot_values[sc.slot("emission")][0])
    v = np.asarray([sg.make_view(0, 6, 5, 3, (0.1, 0.2, 0.3), (1, 0, 0), (0, 1, 0), 60.0, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    osc = oracle.OracleScene.from_scene(sc)
    r = osc.run(sc.params(), v, depth, 11, flags=oracle.FLAG_NO_NEE)
    img = r["image"].reshape(-1, 3, 4)
    expect = le * sum(rho ** k for k in range(depth))
    assert np.allclose(img[..., 0], expect, rtol=1e-13) and np.allclose(img[..., 1:], 0, atol=1e-13)
    dI = np.zeros_like(r["image"]).reshape(-1, 3, 4); dI[..., 0] = 1.0
    g_expect = le * sum(k * rho ** (k - 1) for k in range(1, depth)) * dI.shape[0]
    for mode in (oracle.MODE_TAPE_AD, oracle.MODE_CACHED_PRB):
        g = osc.run(sc.params(), v, depth, 11, flags=oracle.FLAG_NO_NEE, mode=mode, d_image=dI.ravel())["grads"]
        assert np.allclose(g[sc.slot("albedo")], g_expect, rtol=1e-12, atol=1e-12)
        assert np.allclose(g[sc.slot("emission")], expect / le * dI.shape[0], rtol=1e-12)


# ----------------------------------------------------------------------------- estimator-level pins
def _c1():
    wl = sg.config1()
    osc = oracle.OracleScene.from_scene(wl.scene)
    return wl, osc


def test_gauge_invariance(oracle_lib):
    wl, osc = _c1()
    p = wl.scene.params()
    a = osc.run(p, wl.views, wl.max_depth, wl.seed)
    b = osc.run(p, wl.views, wl.max_depth, wl.seed, flags=oracle.FLAG_GAUGE)
    assert np.allclose(a["image"], b["image"], rtol=0, atol=1e-12 * np.abs(a["image"]).max())
    d = np.random.default_rng(3).normal(size=a["image"].size)
    ga = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    gb = osc.run(p, wl.views, wl.max_depth, wl.seed, flags=oracle.FLAG_GAUGE, mode=oracle.MODE_CACHED_PRB, d_image=d)["grads"]
    for x, y in zip(ga, gb):
        assert np.allclose(x, y, rtol=1e-10, atol=1e-12 * np.abs(x).max())


def test_stokes_validity(oracle_lib):
    wl, osc = _c1()
    for sensor in (sg.SENSOR_POLARIZER, sg.SENSOR_NONE):
        v = wl.views.copy(); v["sensor"] = sensor
        img = osc.run(wl.scene.params(), v, wl.max_depth, wl.seed)["image"].reshape(-1, 3, 4)
        assert np.all(img[..., 0] >= np.linalg.norm(img[..., 1:], axis=-1) - 1e-12)


def test_fold_equals_forward_sum(oracle_lib):
    # mode 0 builds the image from the backward fold L[1]; mode 1 from sum_b beta_b E_b
    wl, osc = _c1()
    p = wl.scene.params()
    a = osc.run(p, wl.views, wl.max_depth, wl.seed)["image"]
    d = np.ones_like(a)
    b = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)
    assert np.allclose(a, b["image"], rtol=0, atol=1e-12 * np.abs(a).max())
    assert b["n_vertices"] > 0


def _loss_grad_modes(wl, osc, d, slots=None):
    p = wl.scene.params()
    out = {}
    for mode in (oracle.MODE_TAPE_AD, oracle.MODE_CACHED_PRB):
        out[mode] = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=mode, d_image=d, grad_slots=slots)["grads"]
    return out


def test_cached_replay_equals_tape_ad_c1(oracle_lib):
    wl, osc = _c1()
    d = np.random.default_rng(5).normal(size=sg.image_numel(wl.views))
    g = _loss_grad_modes(wl, osc, d)
    for a, b in zip(g[oracle.MODE_TAPE_AD], g[oracle.MODE_CACHED_PRB]):
        assert np.allclose(a, b, rtol=1e-10, atol=1e-12 * max(np.abs(a).max(), 1e-30))
    assert np.abs(g[oracle.MODE_TAPE_AD][wl.scene.slot("theta")]).max() > 0


def test_cached_replay_equals_tape_ad_c2_crop(oracle_lib):
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 120, 150, 6, 5)
    wl.views["spp"] = 8
    osc = oracle.OracleScene.from_scene(wl.scene)
    d = np.random.default_rng(6).normal(size=sg.image_numel(wl.views))
    g = _loss_grad_modes(wl, osc, d)
    nz = 0
    for a, b in zip(g[oracle.MODE_TAPE_AD], g[oracle.MODE_CACHED_PRB]):
        scale = max(np.abs(a).max(), 1e-30)
        assert np.allclose(a, b, rtol=1e-9, atol=1e-11 * scale)
        nz += np.count_nonzero(a)
    assert nz > 10


def _fd_check(wl, osc, d, slot, idx, h, detached=True, rtol=1e-6):
    p0 = wl.scene.params()
    g = osc.run(p0, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d, grad_slots=[slot])["grads"][slot]
    vals = []
    for sgn in (+1, -1):
        pv = [x.astype(np.float64) for x in p0]
        pv[slot][idx] += sgn * h
        if detached:
            img = osc.run(p0, wl.views, wl.max_depth, wl.seed, params_val=pv)["image"]
        else:
            img = osc.run(pv, wl.views, wl.max_depth, wl.seed)["image"]
        vals.append(np.dot(d, img))
    fd = (vals[0] - vals[1]) / (2 * h)
    assert np.isclose(g[idx], fd, rtol=rtol, atol=1e-9 * (abs(fd) + 1e-3)), (slot, idx, g[idx], fd)
    return g[idx], fd


def test_detached_finite_differences_c1(oracle_lib):
    wl, osc = _c1()
    d = np.random.default_rng(8).normal(size=sg.image_numel(wl.views))
    s = wl.scene.slot
    for slot, idx in [(s("theta"), 0), (s("albedo"), 0), (s("albedo"), 2), (s("ior"), 0), (s("light_Le"), 1)]:
        _fd_check(wl, osc, d, slot, idx, 1e-5, detached=True)


def test_full_finite_differences_path_independent_params(oracle_lib):
    # theta, albedo and Le do not steer sampling: the full derivative equals the detached one
    wl, osc = _c1()
    d = np.random.default_rng(9).normal(size=sg.image_numel(wl.views))
    s = wl.scene.slot
    for slot, idx in [(s("theta"), 0), (s("albedo"), 1), (s("light_Le"), 0)]:
        _fd_check(wl, osc, d, slot, idx, 1e-5, detached=False)


def test_detached_fd_c2_texture_and_roughness(oracle_lib):
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 100, 140, 5, 4)
    wl.views["spp"] = 4
    osc = oracle.OracleScene.from_scene(wl.scene)
    d = np.random.default_rng(10).normal(size=sg.image_numel(wl.views))
    p0 = wl.scene.params()
    s = wl.scene.slot
    g = osc.run(p0, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    checks = [(s("roughness"), int(np.argmax(np.abs(g[s("roughness")])))),
              (s("albedo_tex"), int(np.argmax(np.abs(g[s("albedo_tex")])))),
              (s("ior"), int(np.argmax(np.abs(g[s("ior")])))),
              (s("cond_k"), int(np.argmax(np.abs(g[s("cond_k")])))),
              (s("theta"), 0)]
    for slot, idx in checks:
        if g[slot][idx] != 0:
            _fd_check(wl, osc, d, slot, idx, 1e-5, detached=True, rtol=2e-6)


def test_theta_closed_form(oracle_lib):
    # with the unfiltered Stokes s in the sensor frame, I0 = (s0 + s1 cos2t + s2 sin2t)/2 and
    # dI0/dt = -s1 sin2t + s2 cos2t
    wl, osc = _c1()
    p = wl.scene.params()
    th = float(p[wl.scene.slot("theta")][0])
    vn = wl.views.copy(); vn["sensor"] = sg.SENSOR_NONE
    s = osc.run(p, vn, wl.max_depth, wl.seed)["image"].reshape(-1, 3, 4)
    ip = osc.run(p, wl.views, wl.max_depth, wl.seed)["image"].reshape(-1, 3, 4)
    I0 = 0.5 * (s[..., 0] + s[..., 1] * np.cos(2 * th) + s[..., 2] * np.sin(2 * th))
    assert np.allclose(ip[..., 0], I0, rtol=1e-12, atol=1e-14)
    d = np.zeros_like(ip); d[..., 0] = 1.0
    g = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=d.ravel())["grads"]
    dI0 = np.sum(-s[..., 1] * np.sin(2 * th) + s[..., 2] * np.cos(2 * th))
    assert np.isclose(g[wl.scene.slot("theta")][0], dI0, rtol=1e-11)


def test_light_linearity(oracle_lib):
    wl, osc = _c1()
    p = wl.scene.params()
    s_le = wl.scene.slot("light_Le")
    I = osc.run(p, wl.views, wl.max_depth, wl.seed)["image"]
    p2 = [x.copy() for x in p]; p2[s_le] = p2[s_le] * 2
    I2 = osc.run(p2, wl.views, wl.max_depth, wl.seed)["image"]
    assert np.allclose(I2, 2 * I, rtol=1e-13, atol=1e-15)
    d = np.random.default_rng(4).normal(size=I.size)
    g = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"][s_le]
    Ic = I.reshape(-1, 3, 4); dc = d.reshape(-1, 3, 4)
    for c in range(3):
        assert np.isclose(g[c], np.sum(dc[:, c] * Ic[:, c]) / p[s_le][c], rtol=1e-11)


def test_bvh_matches_brute_force(oracle_lib):
    sc, _ = sg.scene2(2)
    osc = oracle.OracleScene.from_scene(sc)
    rng = np.random.default_rng(12)
    nhit = 0
    for _ in range(400):
        o = rng.uniform(-4, 4, 3) + np.array([0, 1.0, 0])
        d = rng.normal(size=3); d /= np.linalg.norm(d)
        a = oracle.trace(osc, o, d)
        b = oracle.trace(osc, o, d, brute=True)
        assert a[0] == b[0] and np.isclose(a[1], b[1], rtol=1e-14)
        if a[0] >= 0:
            nhit += 1
            assert oracle.trace(osc, o, d, any_hit=True)[0] >= 0
            assert oracle.trace(osc, o, d, tmax=a[1] * 0.999, any_hit=True)[0] < 0
    assert nhit > 100


def test_basic_polarized_prb_breaks_down(oracle_lib):
    # negative control: inverting rank-deficient Mueller weights (Sec. 4.1, Sec. 5.1)
    wl, osc = _c1()
    d = np.random.default_rng(13).normal(size=sg.image_numel(wl.views))
    p = wl.scene.params()
    with np.errstate(all="ignore"):
        g = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_BASIC_PRB, d_image=d)["grads"]
    ref = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    s = wl.scene.slot
    bad = [not np.all(np.isfinite(g[s(n)])) or not np.allclose(g[s(n)], ref[s(n)], rtol=1e-3)
           for n in ("theta", "albedo")]
    assert any(bad)


# ----------------------------------------------------------------------------- hybrid cached replay
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_hybrid_replay_equals_cached_and_tape_c2_crop(oracle_lib, k):
    # Sec. 4.4 with the recomputation branch of Eq. 3: keeping suffix values only every k vertices
    # and recomputing the ones in between gives the cached method's gradient exactly (the same
    # floating-point recursion from a stored checkpoint) and hence conventional AD's
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 120, 150, 6, 5)
    wl.views["spp"] = 8
    osc = oracle.OracleScene.from_scene(wl.scene)
    d = np.random.default_rng(6).normal(size=sg.image_numel(wl.views))
    p = wl.scene.params()
    # one thread: the per-thread gradient sums are then added in a fixed order
    gc = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=d, nthreads=1)["grads"]
    gh = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_HYBRID, d_image=d, ckpt=k, nthreads=1)["grads"]
    gt = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    for a, b, t in zip(gc, gh, gt):
        assert np.array_equal(a, b)
        scale = max(np.abs(t).max(), 1e-30)
        assert np.allclose(b, t, rtol=1e-9, atol=1e-11 * scale)


def test_hybrid_replay_deep_polarizer_stack(oracle_lib):
    # 85 delta vertices before the first diffuse one: checkpoints every 16 vertices (the deep-path
    # case the variant is for) still give the cached gradient of the floor albedo exactly
    wl = sg.polarizer_stack(width=32, height=18, spp=2)
    v = sg.crop_views(wl.views, 12, 6, 6, 6)
    osc = oracle.OracleScene.from_scene(wl.scene)
    d = np.random.default_rng(9).normal(size=sg.image_numel(v))
    p = wl.scene.params()
    r = osc.run(p, v, 128, wl.seed)
    assert r["n_vertices"] > 80 * r["n_paths"]
    gc = osc.run(p, v, 128, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=d, nthreads=1)["grads"]
    for k in (16, 200):
        gh = osc.run(p, v, 128, wl.seed, mode=oracle.MODE_HYBRID, d_image=d, ckpt=k, nthreads=1)["grads"]
        for a, b in zip(gc, gh):
            assert np.array_equal(a, b)
    assert np.abs(gc[wl.scene.slot("floor_albedo")]).max() > 0


def test_hybrid_replay_rejects_zero_interval(oracle_lib):
    wl, osc = _c1()
    d = np.zeros(sg.image_numel(wl.views))
    with pytest.raises(ValueError, match="checkpoint"):
        osc.run(wl.scene.params(), wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_HYBRID, d_image=d, ckpt=0)
