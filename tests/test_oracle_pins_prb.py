"""Pins of the oracle's polarized radiative backpropagation comparator (P-RB, Sec. 5.1): the replay
replaces each cached suffix by an independent estimate, a new path traced from the ray leaving the
vertex under a key of its own.

Pins: where every suffix is deterministic (a closed Lambertian furnace with pure BSDF sampling:
every path from a vertex reads the same radiance), P-RB equals conventional AD to rounding;
parameters whose derivative does not involve the suffix (the sensor angle, the light radiance)
equal conventional AD's on any scene; elsewhere the estimate is unbiased (a z-test of the
gradient images against conventional AD) but differs per sample by far more than rounding.
"""
import numpy as np

import oracle
import scenegen as sg


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_prb_equals_tape_ad_with_deterministic_suffixes(oracle_lib):
    sc, _ = sg.furnace_scene(rho=0.6, le=1.5)
    v = np.asarray([sg.make_view(0, 8, 8, 4, (0.1, 0.2, 0.3), (1, 0, 0), (0, 1, 0), 60.0, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    osc = oracle.OracleScene.from_scene(sc)
    d = np.random.default_rng(41).normal(size=sg.image_numel(v))
    for depth in (2, 5):
        gt = osc.run(sc.params(), v, depth, 3, flags=sg.FLAG_NO_NEE, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
        gr = osc.run(sc.params(), v, depth, 3, flags=sg.FLAG_NO_NEE, mode=oracle.MODE_PRB_INDEPENDENT, d_image=d)["grads"]
        for a, b in zip(gr, gt):
            assert _rel(a, b) < 1e-12


def test_prb_suffix_free_parameters_and_unbiasedness(oracle_lib):
    wl = sg.config1()
    wl.views["spp"] = 16
    osc = oracle.OracleScene.from_scene(wl.scene)
    p = wl.scene.params()
    d = np.random.default_rng(42).normal(size=sg.image_numel(wl.views))
    s = wl.scene.slot
    gt = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d)["grads"]
    gr = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_PRB_INDEPENDENT, d_image=d)["grads"]
    for name in ("theta", "light_Le"):  # their derivatives need no suffix
        assert _rel(gr[s(name)], gt[s(name)]) < 1e-12
    assert _rel(gr[s("albedo")], gt[s("albedo")]) > 1e-3
    kw = dict(grad_slots=[s("albedo")], pixel_grad_slot=s("albedo"), want_image=False, d_image=d)
    ip = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_PRB_INDEPENDENT, **kw)["pixel_grad"]
    it = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, **kw)["pixel_grad"]
    diff = (ip - it).ravel()
    z = diff.mean() / (diff.std(ddof=1) / np.sqrt(diff.size))
    print("P-RB albedo gradient images: z", z)
    assert abs(z) < 4.0
