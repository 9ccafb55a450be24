"""Pins of the hybrid cached replay's decision rule (Sec. 4.4, Eq. 3) in the oracle.

Inside a block of k vertices the replay recovers a suffix by the scalar PRB update when the block
throughput's depolarization index is below gamma, by inverting the block throughput when its
normalised determinant exceeds eps, and otherwise by recomputing up to the next checkpoint.  The
pins: with the rule switched off (gamma = 0, eps = infinity) the result is that of recomputation
bit for bit; the inversion branch is exact (to FP64 rounding) on blocks of invertible operators
(microfacet Fresnel reflections); the scalar branch is exact where only the intensity of the
suffix matters, on blocks of ideal depolarizers (Sec. 4.1, case ii: Lambertian surfaces), and an
approximation after polarizing vertices; every branch taken together on a mixed scene still gives
the conventional-AD gradient.
"""
import numpy as np

import oracle
import scenegen as sg


def _grads(wl, mode, d, **kw):
    osc = oracle.OracleScene.from_scene(wl.scene)
    r = osc.run(wl.scene.params(), wl.views, wl.max_depth, wl.seed, flags=wl.flags, mode=mode, d_image=d,
                want_image=False, nthreads=1, **kw)
    return r["grads"], r["hybrid_branches"]


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def _delta(wl, seed):
    return np.random.default_rng(seed).normal(size=sg.image_numel(wl.views))


def test_rule_off_is_recomputation_bit_for_bit(oracle_lib):
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    d = _delta(wl, 1)
    g0, b0 = _grads(wl, oracle.MODE_HYBRID, d, ckpt=3)
    g1, b1 = _grads(wl, oracle.MODE_HYBRID, d, ckpt=3, hybrid_gamma=0.0, hybrid_eps=np.inf)
    gc, _ = _grads(wl, oracle.MODE_CACHED_PRB, d)
    assert b0["scalar"] == b0["invert"] == 0 and b0["recompute"] > 0
    for a, b, c in zip(g0, g1, gc):
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_inversion_branch_exact_on_invertible_blocks(oracle_lib):
    # microfacet-only scene: the block throughputs are products of rotated Fresnel reflections,
    # invertible away from Brewster-like configurations, which eps sends to recomputation
    wl = sg.glossy_scene()
    d = _delta(wl, 2)
    gc, _ = _grads(wl, oracle.MODE_CACHED_PRB, d)
    gh, br = _grads(wl, oracle.MODE_HYBRID, d, ckpt=4, hybrid_eps=1e-3)
    assert br["invert"] > 10 * br["recompute"] and br["scalar"] == 0
    for name, a, b in zip(wl.scene.slot_names, gh, gc):
        assert _rel(a, b) <= 1e-10, (name, _rel(a, b))


def test_scalar_branch_exact_on_depolarizing_blocks(oracle_lib):
    # Lambertian floor and wall under an area light: every block throughput is a multiple of
    # e0 e0^T (depolarization index 0) and every vertex's derivative needs only the suffix's intensity
    wl = sg.polarizer_stack(n_sheets=0, width=32, height=18, spp=4, max_depth=8)
    d = _delta(wl, 3)
    gc, _ = _grads(wl, oracle.MODE_CACHED_PRB, d)
    gh, br = _grads(wl, oracle.MODE_HYBRID, d, ckpt=4, hybrid_gamma=0.5)
    assert br["scalar"] > 0 and br["invert"] == br["recompute"] == 0
    for name, a, b in zip(wl.scene.slot_names, gh, gc):
        assert _rel(a, b) <= 1e-12, (name, _rel(a, b))


def test_scalar_branch_approximates_after_polarizing_vertices(oracle_lib):
    # forcing the scalar update everywhere (gamma above any index) drops the polarization of the
    # suffix at microfacet vertices: the gradients of their parameters move by far more than rounding
    wl = sg.glossy_scene()
    d = _delta(wl, 2)
    gc, _ = _grads(wl, oracle.MODE_CACHED_PRB, d)
    gh, br = _grads(wl, oracle.MODE_HYBRID, d, ckpt=4, hybrid_gamma=1.01)
    assert br["scalar"] > 0 and br["invert"] == br["recompute"] == 0
    errs = {n: _rel(a, b) for n, a, b in zip(wl.scene.slot_names, gh, gc)}
    print("scalar update everywhere:", errs)
    assert max(errs["roughness"], errs["eta"], errs["kappa"]) > 1e-3


def test_all_branches_on_a_mixed_scene_match_tape_ad(oracle_lib):
    # the config-2 crop (Lambertian, GGX dielectric and conductor materials): each branch is taken
    # where its test admits it, and the gradient is still conventional AD's
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    d = _delta(wl, 4)
    gt, _ = _grads(wl, oracle.MODE_TAPE_AD, d)
    gh, br = _grads(wl, oracle.MODE_HYBRID, d, ckpt=3, hybrid_gamma=0.5, hybrid_eps=1e-3)
    print("branches:", br)
    assert br["scalar"] > 0 and br["invert"] > 0
    for name, a, b in zip(wl.scene.slot_names, gh, gt):
        assert _rel(a, b) <= 1e-9, (name, _rel(a, b))
