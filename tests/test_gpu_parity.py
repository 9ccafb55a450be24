"""GPU (HIP, gfx950) against the FP64 oracle, through the C ABI.

Tolerances (written here, derived in the design notes): Stokes images relative L2 <= 1e-4,
gradients relative L2 <= 1e-3 per parameter group, on the paths whose discrete decisions
agree (divergent paths are masked on both sides and counted).
"""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity import GRAD_TOL, IMG_TOL, check_image, describe, loss_delta_c1, run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_13265_amd as ppt
    ppt.lib()


def test_rng_bitwise_equal_to_oracle():
    import paper_2607_13265_amd as ppt
    rng = np.random.default_rng(0)
    n = 1 << 20
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    seed = int(rng.integers(0, 2**63))
    g = ppt.debug_rng(seed, torch.from_numpy(ctr.view(np.int32)).cuda()).cpu().numpy().view(np.uint32)
    o = oracle.philox_n(seed, ctr)
    assert np.array_equal(g, o)


def _check(res, gate_groups=None, max_div_frac=0.01):
    """Gate: image; the listed aggregate gradient groups (all when None); every gradient image."""
    print(describe(res))
    assert res["divergent"] <= max_div_frac * res["n_paths"]
    check_image(res)
    for k, v in res.get("grad_rel", {}).items():
        if gate_groups is None or k in gate_groups:
            assert v <= GRAD_TOL, (k, v)
    for k, v in res.get("pixel_grad_rel", {}).items():
        assert v <= GRAD_TOL, ("gradient image", k, v)


def test_c1_tiny_parity_config_loss():
    # the config-1 workload: L2 loss to a target rendered at 45 degrees
    wl = sg.config1()
    res = run(wl, d=loss_delta_c1(wl))
    _check(res)
    assert res["stats_render"]["vertices"] == res["n_vertices_ref"]


@pytest.mark.parametrize("seed", [1, 77])
def test_c1_parity_random_delta_gradient_images(seed):
    # random dL/dI: scalar groups are compared as per-pixel gradient images, texture-free
    wl = sg.config1()
    res = run(wl, seed=seed, pixel_grad_slots=("theta", "ior", "albedo"))
    _check(res, gate_groups=("albedo", "light_Le"))


def test_c1_parity_cached_replay_reference():
    # the GPU gradient also matches the oracle's own cached-suffix replay
    wl = sg.config1()
    _check(run(wl, oracle_mode=oracle.MODE_CACHED_PRB, seed=5, d=loss_delta_c1(wl)))


def test_c2_crop_parity_full_spp_depth():
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)  # ragged: 2 x 2 tiles, partially filled
    res = run(wl, pixel_grad_slots=("theta", "roughness", "ior", "cond_n", "cond_k"))
    _check(res, gate_groups=("albedo_tex", "light_Le"))


def test_c5_uneven_multiworld_crops():
    # eight seeded worlds (terrain of 1e5..1e6 triangles + icospheres), four analyzers, depth 12,
    # uneven resolutions and spp; the central 32x32 crop of every view in one batched plan.
    # dL/dI weights the analyzer intensities (s0 of every analyzer output) positively, so each
    # aggregate gradient group sums contributions without sign cancellation.
    wl = sg.config5(crop=(32, 32))
    n = sg.image_numel(wl.views)
    w = np.random.default_rng(505).uniform(0.5, 1.5, n).astype(np.float32)
    d = np.where(np.arange(n) % 4 == 0, w, 0.0).astype(np.float32)
    res = run(wl, d=d, oracle_mode=oracle.MODE_CACHED_PRB)
    _check(res)
    assert len(res["grad_rel"]) == len(wl.scene.slot_names)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_hybrid_replay_parity_c2_crop(k):
    # hybrid cached replay (checkpoint interval k): same gradient as the oracle's cached replay
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    res = run(wl, oracle_mode=oracle.MODE_CACHED_PRB, plan_kw={"checkpoint_interval": k})
    _check(res, gate_groups=("albedo_tex", "roughness", "cond_n", "cond_k", "light_Le"))


def test_hybrid_replay_parity_c1_config_loss():
    wl = sg.config1()
    _check(run(wl, d=loss_delta_c1(wl), oracle_mode=oracle.MODE_HYBRID, plan_kw={"checkpoint_interval": 2}))


# the light stage: right-circular lights, analyzers at 0, 45, 90 degrees and left-circular,
# normal maps (blend, smooth dielectric, conductor), specular and roughness maps, depth 6
LIGHTSTAGE_TEX = ("ground_albedo", "ground_roughness", "ground_specular", "ground_normal", "object_albedo",
                  "object_roughness", "object_specular", "object_normal", "glass_normal", "metal_normal")


def _lightstage_crops():
    wl = sg.lightstage(res=128, spp=8)
    wl.views = sg.crop_views(wl.views[[0, 3, 5]], 44, 52, 13, 11)
    return wl


def test_lightstage_crop_parity():
    wl = _lightstage_crops()
    res = run(wl, oracle_mode=oracle.MODE_CACHED_PRB, pixel_grad_slots=("ior", "metal_specular", "light_Le"),
              max_pixels=48)
    _check(res, gate_groups=LIGHTSTAGE_TEX)


def test_lightstage_hybrid_replay_parity():
    wl = _lightstage_crops()
    res = run(wl, oracle_mode=oracle.MODE_HYBRID, plan_kw={"checkpoint_interval": 2})
    _check(res, gate_groups=LIGHTSTAGE_TEX)


def test_circular_emitter_analyzers_closed_form():
    # GPU images of a right/left/partially circular emitter against the closed forms:
    # left-circular analyzer (s0 - s3)/2, right-circular (s0 + s3)/2, linear ones s0/2
    import paper_2607_13265_amd as ppt
    for circ in (1.0, -1.0, 0.5):
        sc, _ = sg.emitter_wall_scene(le=10.0, circ=circ)
        for sensor, expect3 in ((sg.SENSOR_LIGHTSTAGE4, 5.0 * (1 - circ)), (sg.SENSOR_ANALYZER4, 5.0 * (1 + circ))):
            v = np.asarray([sg.make_view(0, 16, 8, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 30.0, sensor)], sg.VIEW_DTYPE)
            plan = ppt.Plan(ppt.Scene(sc.to_blob()), v, 3)
            img = plan.render([torch.from_numpy(p).cuda() for p in sc.params()], 7).cpu().numpy().reshape(4, -1, 3, 4)
            assert np.allclose(img[:3, ..., 0], 5.0, rtol=1e-6)
            assert np.allclose(img[3, ..., 0], expect3, rtol=1e-6, atol=1e-5)


def _far_scene(offset, scale):
    """A Lambertian icosphere (1280 triangles), a dielectric sphere, a ground quad and a light, moved
    to offset + scale * p.  The BVH's half-float box bounds are rounded outward: far from the
    origin they widen (by ~2 units at 3e3) or, beyond the half range (6.55e4), become infinite;
    either way no hit may be lost."""
    off = np.asarray(offset, np.float64)
    sc = sg.Scene()
    s_alb = sc.add_slot("albedo", [0.6, 0.5, 0.4])
    s_ior = sc.add_slot("ior", [1.5])
    s_le = sc.add_slot("light_Le", [10.0, 10.0, 10.0])
    w = sc.add_world()
    m_lam = w.add_material(type=sg.MAT_LAMBERT, albedo_slot=s_alb)
    m_die = w.add_material(type=sg.MAT_DIELECTRIC, eta_slot=s_ior)
    P = lambda p: off + scale * np.asarray(p, np.float64)
    w.add_quad(P((-10, -1.5, -10)), scale * np.array([0, 0, 20.0]), scale * np.array([20.0, 0, 0]), m_lam)
    w.add_tris(P(0.8 * sg.icosphere(3) + np.array([-0.6, -0.4, 0.0])), None, m_lam)
    w.add_sphere(P((0.9, -0.8, 0.5)), 0.5 * scale, m_die)
    w.add_light(P((-1, 3, -1)), scale * np.array([2.0, 0, 0]), scale * np.array([0, 0, 2.0]), s_le)
    views = np.asarray([sg.make_view(0, 32, 32, 4, P((0, 1, 6)), P((0, -0.5, 0)), (0, 1, 0), 40.0,
                                     sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    return sg.Workload("far", sc, views, max_depth=3, seed=5)


@pytest.mark.parametrize("offset,scale", [((0, 0, 0), 1.0), ((3000, 0, 0), 30.0),
                                          ((1.2e5, -5.0e4, 8.0e4), 1000.0)])
def test_far_geometry_no_lost_hits(offset, scale):
    # same paths as the oracle (float64 boxes, its traversal pinned to brute force) wherever the
    # scene sits; the scale keeps the float32 precision of the geometry relative to its size as at
    # the origin
    res = run(_far_scene(offset, scale), with_grads=False)
    print(describe(res))
    assert res["divergent"] <= 0.01 * res["n_paths"]
    # away from the origin the float32 coordinates resolve hit points and normals more coarsely
    # (3e3 units: 2.4e-4 steps for 30-unit features), which perturbs every Stokes component by an
    # amount of the intensity's order: the components are gated against the intensity norm
    check_image(res, components_vs_intensity=tuple(offset) != (0, 0, 0))


# the deep polarizer stack (85 sheets 1 degree apart in front of a Lambertian floor and wall under an
# area light, 1280x720): every camera path through the stack crosses 85 delta vertices before its
# first diffuse one.  Windows at full resolution, 4 spp; dL/dI weights the intensities positively
# and the polarization components with small random weights, so the aggregate gradient of each
# albedo and the light sums contributions mostly of one sign.
def _stack_delta(n, seed):
    rng = np.random.default_rng(seed)
    idx = np.arange(n)
    return np.where(idx % 4 == 0, rng.uniform(0.5, 1.5, n), 0.2 * rng.normal(size=n)).astype(np.float32)


# (depth 87: the first diffuse vertex is the 86th and is the last that samples a light; at depth 86
# the window is black)
@pytest.mark.parametrize("depth", [87, 128])
@pytest.mark.parametrize("k", [0, 16])
def test_polarizer_stack_window_parity(depth, k):
    wl = sg.polarizer_stack(spp=4, max_depth=depth)
    wl.views = sg.crop_views(wl.views, 632, 352, 16, 12)
    d = _stack_delta(sg.image_numel(wl.views), 86)
    res = run(wl, d=d, oracle_mode=oracle.MODE_CACHED_PRB, plan_kw={"checkpoint_interval": k},
              pixel_grad_slots=("floor_albedo",), max_pixels=48)
    assert res["n_vertices_ref"] > 85 * res["n_paths"]  # the window sees through the whole stack
    _check(res)


def test_polarizer_stack_tape_ad_parity():
    # the same deep paths against the oracle's conventional stored-tape AD (a smaller window)
    wl = sg.polarizer_stack(spp=4, max_depth=128)
    wl.views = sg.crop_views(wl.views, 636, 356, 6, 5)
    d = _stack_delta(sg.image_numel(wl.views), 87)
    _check(run(wl, d=d, oracle_mode=oracle.MODE_TAPE_AD, plan_kw={"checkpoint_interval": 16}))


# the hybrid replay's decision rule (Sec. 4.4, Eq. 3) on the GPU against the oracle's
def _rule_run(wl, k, gamma, eps, d=None, **kw):
    res = run(wl, d=d, oracle_mode=oracle.MODE_HYBRID,
              plan_kw={"checkpoint_interval": k, "hybrid_rule": (gamma, eps)},
              oracle_kw={"ckpt": k, "hybrid_gamma": gamma, "hybrid_eps": eps}, **kw)
    res["gpu_branches"] = res["plan"].hybrid_stats()
    print("branches: gpu", res["gpu_branches"], "oracle", res["oracle_branches"])
    return res


def _same_branches(res, tol=0.02):
    g, o = res["gpu_branches"], res["oracle_branches"]
    for key in ("scalar", "invert", "recompute"):
        assert abs(g[key] - o[key]) <= tol * max(1, sum(o.values())), (key, g, o)


def test_hybrid_rule_off_thresholds_recompute_only():
    # gamma = 0 and eps = inf: every suffix inside a block is recomputed, as without the rule
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    res = _rule_run(wl, 3, 0.0, float("inf"))
    _check(res, gate_groups=("albedo_tex", "roughness", "cond_n", "cond_k", "light_Le"))
    assert res["gpu_branches"]["scalar"] == res["gpu_branches"]["invert"] == 0
    assert res["gpu_branches"]["recompute"] > 0
    _same_branches(res, 0.0)


def test_hybrid_rule_inversion_on_microfacet_blocks():
    # GGX-only scene: most suffixes recovered by inverting the block throughput
    wl = sg.glossy_scene(width=48, height=32, spp=8)
    res = _rule_run(wl, 4, 0.0, 1e-3)
    _check(res)
    assert res["gpu_branches"]["invert"] > 10 * res["gpu_branches"]["recompute"]
    _same_branches(res)


def test_hybrid_rule_scalar_update_on_depolarizing_blocks():
    # Lambertian floor and wall: every block is an ideal depolarizer, the scalar update is exact
    wl = sg.polarizer_stack(n_sheets=0, width=64, height=36, spp=4, max_depth=8)
    res = _rule_run(wl, 4, 0.5, float("inf"))
    _check(res)
    assert res["gpu_branches"]["scalar"] > 0 and res["gpu_branches"]["invert"] == 0
    assert res["gpu_branches"]["recompute"] == 0
    _same_branches(res, 0.0)


def test_hybrid_rule_all_branches_c2_crop():
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    res = _rule_run(wl, 3, 0.5, 1e-3, pixel_grad_slots=("roughness", "ior"), max_pixels=32)
    _check(res, gate_groups=("albedo_tex", "roughness", "cond_n", "cond_k", "light_Le"))
    b = res["gpu_branches"]
    assert b["scalar"] > 0 and b["invert"] > 0
    _same_branches(res)


# the noise-regularised P-PRB comparator (Sec. 4.2) on the GPU against the oracle's
@pytest.mark.parametrize("sigma", [0.3, 1.0])
def test_pprb_comparator_parity_c1(sigma):
    wl = sg.config1()
    res = run(wl, d=loss_delta_c1(wl), oracle_mode=oracle.MODE_BASIC_PRB, plan_kw={"pprb_sigma": sigma},
              oracle_kw={"pprb_sigma": sigma})
    _check(res)


def test_pprb_comparator_parity_c2_crop():
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    res = run(wl, oracle_mode=oracle.MODE_BASIC_PRB, plan_kw={"pprb_sigma": 0.3}, oracle_kw={"pprb_sigma": 0.3})
    _check(res, gate_groups=("albedo_tex", "light_Le"))


# the conventional-AD baseline (stored tape of every vertex's loop state, reverse sweep with full
# 4x4 adjoints) on the GPU against the oracle's stored-tape AD
def test_tape_ad_baseline_parity_c1():
    wl = sg.config1()
    res = run(wl, d=loss_delta_c1(wl), oracle_mode=oracle.MODE_TAPE_AD, plan_kw={"tape": True})
    _check(res)


def test_tape_ad_baseline_parity_c2_crop():
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    res = run(wl, oracle_mode=oracle.MODE_TAPE_AD, plan_kw={"tape": True},
              pixel_grad_slots=("roughness", "ior", "cond_k"), max_pixels=32)
    _check(res, gate_groups=("albedo_tex", "light_Le"))


def test_tape_ad_baseline_equals_cached_replay_and_needs_more_memory():
    import paper_2607_13265_amd as ppt
    wl = sg.config3(n_angles=2, n_poses=2)
    scene = ppt.Scene(wl.scene.to_blob())
    params = [torch.from_numpy(p).cuda() for p in wl.scene.params()]
    cached = ppt.Plan(scene, wl.views, wl.max_depth)
    tape = ppt.Plan(scene, wl.views, wl.max_depth, tape=True)
    d = torch.randn(cached.image_numel, device="cuda")
    gc, gt = cached.backward(params, 3, d), tape.backward(params, 3, d)
    for name, a, b in zip(wl.scene.slot_names, gc, gt):
        na = float(a.double().norm())
        assert float((a.double() - b.double()).norm()) <= 1e-4 * max(na, 1e-12), name
    assert tape.workspace_bytes(1) > 1.8 * cached.workspace_bytes(1)
    # normal maps and circular emitters are outside the baseline
    ls = sg.lightstage(res=16, spp=1)
    with pytest.raises(ppt.PPTError, match="EUNSUPPORTED"):
        ppt.Plan(ppt.Scene(ls.scene.to_blob()), ls.views, ls.max_depth, tape=True)


# the P-RB comparator (independent suffix estimates, one sub-path pass per vertex index) against the
# oracle's; the sub-paths draw from their own keys, identically on both sides
def test_prb_comparator_parity_c1():
    wl = sg.config1()
    _check(run(wl, d=loss_delta_c1(wl), oracle_mode=oracle.MODE_PRB_INDEPENDENT, plan_kw={"prb": True}))


def test_prb_comparator_parity_c2_crop():
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
    res = run(wl, oracle_mode=oracle.MODE_PRB_INDEPENDENT, plan_kw={"prb": True},
              pixel_grad_slots=("roughness", "ior"), max_pixels=32)
    _check(res, gate_groups=("albedo_tex", "light_Le"))
