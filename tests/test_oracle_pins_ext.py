"""Pins of the oracle's light-stage features against facts that do not come from the oracle:
circularly polarized emission seen through the four analyzers (closed forms), Lambertian
depolarization of circular light, Lambert's cosine law about a normal-mapped shading normal,
the specular map as an exact scale of the GGX lobe, and finite differences of the estimator
with respect to normal and specular maps (these parameters move the shading frame)."""
import numpy as np
import pytest

import oracle
import scenegen as sg


def _wall(circ, sensor):
    sc, _ = sg.emitter_wall_scene(le=10.0, circ=circ)
    v = np.asarray([sg.make_view(0, 4, 4, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 30.0, sensor)], sg.VIEW_DTYPE)
    img = oracle.OracleScene.from_scene(sc).run(sc.params(), v, 3, 7)["image"]
    return img.reshape(sg.analyzer_count(sensor), -1, 3, 4)


@pytest.mark.parametrize("circ", [1.0, -1.0, 0.5, 0.0])
def test_circular_emitter_through_analyzers(oracle_lib, circ):
    # the emitter radiates Le (1, 0, 0, circ); s3 needs no frame, so the sensor sees it unchanged
    full = _wall(circ, sg.SENSOR_NONE)
    assert np.allclose(full[..., 0], 10.0, rtol=1e-14) and np.allclose(full[..., 3], 10.0 * circ, rtol=1e-14)
    assert np.allclose(full[..., 1:3], 0.0, atol=1e-13)
    # linear analyzers pass half of the intensity whatever the circular part
    ls = _wall(circ, sg.SENSOR_LIGHTSTAGE4)
    assert np.allclose(ls[:3, ..., 0], 5.0, rtol=1e-14)
    # left-circular analyzer (QWP at 0, polarizer at -45 deg): (s0 - s3) / 2, leaving along -45 deg
    q = 5.0 * (1.0 - circ)
    assert np.allclose(ls[3, ..., 0], q, rtol=1e-14, atol=1e-13)
    assert np.allclose(ls[3, ..., 2], -q, rtol=1e-14, atol=1e-13)
    assert np.allclose(ls[3, ..., 1], 0.0, atol=1e-13) and np.allclose(ls[3, ..., 3], 0.0, atol=1e-13)
    # right-circular analyzer (polarizer at +45 deg): (s0 + s3) / 2
    a4 = _wall(circ, sg.SENSOR_ANALYZER4)
    assert np.allclose(a4[3, ..., 0], 5.0 * (1.0 + circ), rtol=1e-14, atol=1e-13)


def _plane(phi=0.0, mat=sg.MAT_LAMBERT, nm=True, spec=None, depth=2, circ=0.0, sensor=sg.SENSOR_NONE, params=None):
    sc = sg.tilted_plane_scene(phi, 0.5, mat, spec=spec, normal_map_on=nm)
    if circ:
        w = sc.worlds[0]
        for rec in w.lights:
            rec["circ"] = circ
    v = np.asarray([sg.make_view(0, 4, 4, 2, (0.0, 4.0, 0.0), (0, 0, 0), (0, 0, -1), 0.05, sensor)], sg.VIEW_DTYPE)
    osc = oracle.OracleScene.from_scene(sc)
    p = sc.params() if params is None else params(sc)
    return osc.run(p, v, depth, 7)["image"].reshape(sg.analyzer_count(sensor), -1, 3, 4)


@pytest.mark.parametrize("phi", [0.3, -0.4, 0.6])
def test_normal_map_lambert_cosine_law(oracle_lib, phi):
    # one Lambertian bounce lit by a tiny light 0.5 rad from the geometric normal: the next-event
    # term follows the cosine to the mapped normal, tilted by phi toward the light (+x, the
    # direction of increasing u).  A tilt about the wrong axis or with the wrong sign fails.
    r = _plane(phi)[..., 0] / _plane(0.0)[..., 0]
    assert np.allclose(r, np.cos(0.5 - phi) / np.cos(0.5), rtol=2e-4)


def test_flat_normal_map_is_the_geometric_normal(oracle_lib):
    # (t, b, n) = (0, 0, 1) reproduces the unmapped surface for every scattering type
    for mat in (sg.MAT_LAMBERT, sg.MAT_GGX_DIELECTRIC, sg.MAT_DIELECTRIC, sg.MAT_BLEND):
        a = _plane(0.0, mat, nm=True, depth=4)
        b = _plane(0.0, mat, nm=False, depth=4)
        assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max()), mat


def test_lambert_depolarizes_circular_light(oracle_lib):
    # a Lambertian BSDF has only M00: a circularly polarized light gives the same image
    a = _plane(0.2, circ=0.0, sensor=sg.SENSOR_LIGHTSTAGE4)
    b = _plane(0.2, circ=1.0, sensor=sg.SENSOR_LIGHTSTAGE4)
    assert np.array_equal(a, b)
    # a GGX reflection keeps part of it: the left- and right-circular analyzers then differ,
    # and the image is affine in the degree of circular polarization
    g0 = _plane(0.2, sg.MAT_GGX_DIELECTRIC, circ=0.0, sensor=sg.SENSOR_LIGHTSTAGE4)
    g1 = _plane(0.2, sg.MAT_GGX_DIELECTRIC, circ=1.0, sensor=sg.SENSOR_LIGHTSTAGE4)
    gh = _plane(0.2, sg.MAT_GGX_DIELECTRIC, circ=0.5, sensor=sg.SENSOR_LIGHTSTAGE4)
    assert np.abs(g1[3] - g0[3]).max() > 1e-3 * np.abs(g0).max()
    assert np.allclose(gh, 0.5 * (g0 + g1), rtol=0, atol=1e-12 * np.abs(g1).max())


def test_specular_map_scales_the_ggx_lobe(oracle_lib):
    # a unit map changes nothing; with one scattering vertex the image is linear in the scale
    one = _plane(0.1, sg.MAT_GGX_DIELECTRIC, spec=1.0)
    none = _plane(0.1, sg.MAT_GGX_DIELECTRIC, spec=None)
    assert np.array_equal(one, none)
    zero = _plane(0.1, sg.MAT_GGX_DIELECTRIC, spec=0.0)
    two = _plane(0.1, sg.MAT_GGX_DIELECTRIC, spec=2.0)
    assert np.abs(one).max() > 0 and np.allclose(zero, 0.0)
    assert np.allclose(two - zero, 2.0 * (one - zero), rtol=1e-13, atol=1e-13 * np.abs(two).max())


def _lightstage_crop():
    wl = sg.lightstage(res=64, spp=4, n_views=2, max_depth=5)
    wl.views = sg.crop_views(wl.views, 24, 26, 6, 5)
    return wl, oracle.OracleScene.from_scene(wl.scene)


def test_lightstage_cached_and_hybrid_replay_equal_tape_ad(oracle_lib):
    wl, osc = _lightstage_crop()
    p = wl.scene.params()
    d = np.random.default_rng(3).normal(size=sg.image_numel(wl.views))
    ga = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    gb = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=d)["grads"]
    gc = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_HYBRID, d_image=d, ckpt=2)["grads"]
    for name, a, b, c in zip(wl.scene.slot_names, ga, gb, gc):
        scale = max(np.abs(a).max(), 1e-30)
        assert np.allclose(a, b, rtol=1e-10, atol=1e-12 * scale), name
        assert np.allclose(a, c, rtol=1e-10, atol=1e-12 * scale), name
    for name in ("ground_normal", "object_normal", "glass_normal", "metal_normal", "ground_specular"):
        assert np.count_nonzero(ga[wl.scene.slot(name)]) > 0, name


def test_lightstage_detached_finite_differences(oracle_lib):
    # path frozen, values re-evaluated at +-h: normal maps of the blend, the smooth dielectric
    # (its s/p frames move with the normal) and the conductor, and the specular maps
    wl, osc = _lightstage_crop()
    p0 = wl.scene.params()
    d = np.random.default_rng(4).normal(size=sg.image_numel(wl.views))
    g = osc.run(p0, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    for name in ("ground_normal", "object_normal", "glass_normal", "metal_normal", "ground_specular",
                 "object_specular", "metal_specular"):
        s = wl.scene.slot(name)
        idx = int(np.argmax(np.abs(g[s])))
        vals = []
        for sgn in (+1, -1):
            pv = [x.astype(np.float64) for x in p0]
            pv[s][idx] += sgn * 1e-5
            vals.append(np.dot(d, osc.run(p0, wl.views, wl.max_depth, wl.seed, params_val=pv)["image"]))
        fd = (vals[0] - vals[1]) / 2e-5
        assert g[s][idx] != 0.0 and np.isclose(g[s][idx], fd, rtol=1e-6, atol=1e-9 * abs(fd)), (name, g[s][idx], fd)
