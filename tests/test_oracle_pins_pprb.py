"""Pins of the oracle's noise-regularised polarized PRB (P-PRB, Sec. 4.2), the comparator of the
paper's gradient analysis: every sampled weight becomes W_b + u_b I with u_b ~ N(0, sigma) drawn
per vertex from the path's own counters, the same in the primal fold and the adjoint replay.

Pins: the regularised image is unbiased and its spread scales with sigma (a standard deviation);
the P-PRB gradient is the exact derivative of the regularised estimator (central finite
differences of the regularised image, path frozen); that estimator is unbiased, so over many
independent pixels its gradient images average to conventional AD's (a z-test), while per sample
it differs from conventional AD by far more than rounding, and without noise the inversion of
rank-deficient weights breaks down (the negative control in test_oracle_pins.py).
"""
import numpy as np

import oracle
import scenegen as sg

SIGMA = 0.3


def _c1(spp=4):
    wl = sg.config1()
    wl.views["spp"] = spp
    return wl, oracle.OracleScene.from_scene(wl.scene)


def test_regularised_image_is_unbiased(oracle_lib):
    # E_u[prod (W_b + u_b I)] = prod W_b for independent zero-mean u: the regularised image (the
    # P-PRB primal) averages to the unregularised one
    wl, osc = _c1(spp=64)
    p = wl.scene.params()
    d = np.zeros(sg.image_numel(wl.views))
    reg = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_BASIC_PRB, d_image=d,
                  pprb_sigma=SIGMA, grad_slots=[])["image"]
    ref = osc.run(p, wl.views, wl.max_depth, wl.seed)["image"]
    diff = (reg - ref).reshape(-1, 12)[:, [0, 4, 8]].ravel()  # s0 of every pixel and channel
    z = diff.mean() / (diff.std(ddof=1) / np.sqrt(diff.size))
    print("regularised image: z", z, "relative spread", diff.std() / np.abs(ref).mean())
    assert abs(z) < 4.0
    assert np.abs(reg - ref).max() > 1e-3 * np.abs(ref).max()  # the noise is really there


def test_pprb_gradient_is_the_derivative_of_the_regularised_estimator(oracle_lib):
    # detached central differences of the regularised image (mode 3 renders it) against the P-PRB
    # gradient; the noise depends only on the path's counters, not on the parameters
    wl, osc = _c1()
    d = np.random.default_rng(31).normal(size=sg.image_numel(wl.views))
    p = [x.astype(np.float64) for x in wl.scene.params()]
    g = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_BASIC_PRB, d_image=d,
                pprb_sigma=SIGMA)["grads"]
    s = wl.scene.slot
    for slot, idx in [(s("theta"), 0), (s("albedo"), 0), (s("albedo"), 2), (s("ior"), 0), (s("light_Le"), 1)]:
        h = 1e-5 * max(1.0, abs(p[slot][idx]))
        vals = []
        for sgn in (1.0, -1.0):
            pv = [x.copy() for x in p]
            pv[slot][idx] += sgn * h
            img = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_BASIC_PRB, d_image=d,
                          params_val=pv, pprb_sigma=SIGMA, grad_slots=[])["image"]
            vals.append(np.dot(d, img))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert np.isclose(g[slot][idx], fd, rtol=1e-5, atol=1e-9 * (abs(fd) + 1e-3)), (slot, idx, g[slot][idx], fd)


def test_pprb_unbiased_but_noisy_against_conventional_ad(oracle_lib):
    # per pixel the regularised gradient differs from conventional AD's; over many pixels the
    # differences average to zero (z-test on the albedo and polarizer-angle gradient images)
    wl, osc = _c1(spp=4)
    p = wl.scene.params()
    d = np.random.default_rng(32).normal(size=sg.image_numel(wl.views))
    s = wl.scene.slot
    for name in ("albedo", "theta"):
        gp = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_BASIC_PRB, d_image=d, pprb_sigma=SIGMA,
                     grad_slots=[s(name)], pixel_grad_slot=s(name), want_image=False)["pixel_grad"]
        gt = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d,
                     grad_slots=[s(name)], pixel_grad_slot=s(name), want_image=False)["pixel_grad"]
        diff = (gp - gt).ravel()
        z = diff.mean() / (diff.std(ddof=1) / np.sqrt(diff.size))
        re = np.linalg.norm(gp.sum(0) - gt.sum(0)) / np.linalg.norm(gt.sum(0))
        print(name, "z", z, "relative error of the gradient", re)
        assert abs(z) < 4.0
        assert re > 1e-3  # noise, not rounding


def test_regularisation_noise_scales_with_sigma(oracle_lib):
    # to first order the regularised image moves by sum_b u_b (prefix) (suffix) with u_b = sigma n_b:
    # halving sigma halves the spread of the image change (sigma is a standard deviation)
    wl, osc = _c1(spp=16)
    p = wl.scene.params()
    d = np.zeros(sg.image_numel(wl.views))
    ref = osc.run(p, wl.views, wl.max_depth, wl.seed)["image"]
    spread = []
    for sig in (0.02, 0.01):
        reg = osc.run(p, wl.views, wl.max_depth, wl.seed, mode=oracle.MODE_BASIC_PRB, d_image=d, pprb_sigma=sig,
                      grad_slots=[])["image"]
        spread.append(np.std(reg - ref))
    assert abs(spread[0] / spread[1] - 2.0) < 0.02, spread
