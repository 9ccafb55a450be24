"""GPU system tests through the C ABI: closed forms on the device, batching, chunking, graph
replay, edge cases, plan-level errors, the autograd wrapper and full-size sampled parity."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from parity import GRAD_TOL, IMG_TOL, check_image, describe, image_metrics, pixel_slices, rel, run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ppt():
    import paper_2607_13265_amd as ppt
    return ppt


def _params(scene):
    return [torch.from_numpy(p).cuda() for p in scene.params()]


# ----------------------------------------------------------------------------- closed forms on the GPU
def test_gpu_halving_malus_chain():
    ppt = _ppt()
    for sheets, theta, expect in [((), 0.7, 5.0), ((1.1,), 0.3, 5.0 * np.cos(0.3 - 1.1) ** 2)]:
        sc, s_th = sg.emitter_wall_scene(le=10.0, sheets=sheets)
        p = sc.params(); p[s_th][0] = theta
        v = np.asarray([sg.make_view(0, 8, 8, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 0.01, sg.SENSOR_POLARIZER, s_th)],
                       sg.VIEW_DTYPE)
        plan = ppt.Plan(ppt.Scene(sc.to_blob()), v, 4)
        img = plan.render([torch.from_numpy(x).cuda() for x in p], 3).cpu().numpy().reshape(-1, 3, 4)
        assert np.allclose(img[..., 0], expect, rtol=2e-5)
    n = 8
    angles = [0.0] + [k * np.pi / (2 * n) for k in range(1, n + 1)]
    sc, _ = sg.emitter_wall_scene(le=10.0, sheets=tuple(reversed(angles)), z_light=-(n + 6.0))
    v = np.asarray([sg.make_view(0, 4, 4, 1, (0, 0, 0), (0, 0, -1), (0, 1, 0), 0.01, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    plan = ppt.Plan(ppt.Scene(sc.to_blob()), v, n + 3)
    img = plan.render(_params(sc), 3).cpu().numpy().reshape(-1, 3, 4)
    e = 5.0 * np.cos(np.pi / (2 * n)) ** (2 * n)
    assert np.allclose(img[..., 0], e, rtol=2e-5) and np.allclose(img[..., 1], -e, rtol=2e-5)


@pytest.mark.parametrize("depth", [1, 4])
def test_gpu_furnace_value_and_gradient(depth):
    ppt = _ppt()
    sc, _ = sg.furnace_scene(rho=0.6, le=1.5)
    rho = float(sc.slot_values[sc.slot("albedo")][0]); le = float(sc.slot_values[sc.slot("emission")][0])
    v = np.asarray([sg.make_view(0, 16, 8, 4, (0.1, 0.2, 0.3), (1, 0, 0), (0, 1, 0), 60.0, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    plan = ppt.Plan(ppt.Scene(sc.to_blob()), v, depth, ppt.FLAG_NO_NEE)
    params = _params(sc)
    img = plan.render(params, 9).cpu().numpy().reshape(-1, 3, 4)
    expect = le * sum(rho ** k for k in range(depth))
    assert np.allclose(img[..., 0], expect, rtol=1e-5) and np.allclose(img[..., 1:], 0, atol=1e-5)
    d = np.zeros((img.shape[0], 3, 4), np.float32); d[..., 0] = 1
    g = plan.backward(params, 9, torch.from_numpy(d.ravel()).cuda())
    g_expect = le * sum(k * rho ** (k - 1) for k in range(1, depth)) * img.shape[0]
    assert np.allclose(g[sc.slot("albedo")].cpu().numpy(), g_expect, rtol=1e-5, atol=1e-6)


# ----------------------------------------------------------------------------- batching / chunking / graphs
def _small_batch(n_views=6, res=24, spp=4):
    wl = sg.config3(res=res, spp=spp, n_angles=3, n_poses=2)
    wl.views = wl.views[:n_views]
    return wl


def test_launches_without_work_counters_match():
    """With the work counters off, traversal runs its counter-free variants (fewer registers, one
    more wavefront per SIMD): image and gradients equal those of the counting launches up to the
    order of the atomic additions, and the counters are left untouched."""
    ppt = _ppt()
    wl = _small_batch()
    scene = ppt.Scene(wl.scene.to_blob())
    params = _params(wl.scene)
    plan = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=4096)
    d = torch.randn(plan.image_numel, device="cuda")
    img_a = plan.render(params, 13)
    g_a = plan.backward(params, 13, d)
    st_a = plan.stats(0)
    plan.set_stats(False)
    img_b = plan.render(params, 13)
    g_b = plan.backward(params, 13, d)
    plan.set_stats(True)
    assert float((img_a - img_b).norm()) <= 1e-6 * float(img_a.norm())
    for a, b in zip(g_a, g_b):
        if a is not None:
            assert float((a.double() - b.double()).norm()) <= 1e-6 * max(float(a.double().norm()), 1e-30)
    assert st_a["nodes"] > 0 and st_a["vertices"] > 0


def test_rank_one_render_equals_full_render():
    """A plan whose views all have a linear-polarizer sensor renders with the rank-one record (the
    row q^T R_s beta and three scalars per path); one more view with no sensor makes the same
    plan render with the full 4x4 throughput.  The polarizer views' paths are the same in both, so
    their images agree to FP32 rounding of the reassociated products, in every Stokes component."""
    ppt = _ppt()
    wl = _small_batch(n_views=4, res=24, spp=4)
    scene = ppt.Scene(wl.scene.to_blob())
    params = _params(wl.scene)
    extra = wl.views[:1].copy()
    extra["sensor"] = sg.SENSOR_NONE
    extra["view_id"] = 999
    both = np.concatenate([wl.views, extra])
    a = ppt.Plan(scene, wl.views, wl.max_depth).render(params, 21).double().cpu().numpy()
    b = ppt.Plan(scene, both, wl.max_depth).render(params, 21).double().cpu().numpy()[:a.size]
    a4, b4 = a.reshape(-1, 4), b.reshape(-1, 4)
    assert np.abs(b4).max() > 0
    for k in range(3):  # s3 is zero behind a linear polarizer
        nb = np.linalg.norm(b4[:, k])
        assert np.linalg.norm(a4[:, k] - b4[:, k]) <= 1e-5 * nb, k
    assert np.abs(a4[:, 3]).max() == 0.0 and np.abs(b4[:, 3]).max() == 0.0


def test_batched_equals_per_view_and_chunk_invariance():
    ppt = _ppt()
    wl = _small_batch()
    scene = ppt.Scene(wl.scene.to_blob())
    params = _params(wl.scene)
    plan = ppt.Plan(scene, wl.views, wl.max_depth)
    img = plan.render(params, 11)
    d = torch.randn(plan.image_numel, device="cuda")
    g = plan.backward(params, 11, d)
    offs = sg.view_offsets(wl.views)
    gsum = [torch.zeros_like(p) for p in params]
    for v in range(len(wl.views)):
        pv = ppt.Plan(scene, wl.views[v:v + 1], wl.max_depth)
        o = int(offs[v])
        iv = pv.render(params, 11)
        assert torch.equal(iv, img[o:o + pv.image_numel])
        gv = pv.backward(params, 11, d[o:o + pv.image_numel].contiguous())
        for a, b in zip(gsum, gv):
            a += b
    for a, b in zip(gsum, g):
        assert rel(a.cpu().numpy(), b.cpu().numpy(), floor=1e-12) < 1e-5
    # a chunk size that splits pixels between chunks gives the same image and gradients
    pc = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=1000)
    assert pc.launch_info()["n_chunks"] > 1
    assert rel(pc.render(params, 11).cpu().numpy(), img.cpu().numpy()) < 1e-6
    for a, b in zip(pc.backward(params, 11, d), g):
        assert rel(a.cpu().numpy(), b.cpu().numpy(), floor=1e-12) < 1e-5


def test_graph_replay_matches_eager():
    ppt = _ppt()
    wl = _small_batch()
    plan = ppt.Plan(ppt.Scene(wl.scene.to_blob()), wl.views, wl.max_depth)
    params = _params(wl.scene)
    d = torch.randn(plan.image_numel, device="cuda")
    out = torch.empty(plan.image_numel, device="cuda")
    grads = [torch.empty_like(p) for p in params]
    ws0, ws1 = plan.workspace(0), plan.workspace(1)

    def step():
        plan.render(params, 5, out=out, ws=ws0)
        plan.backward(params, 5, d, grads=grads, ws=ws1)

    step()
    torch.cuda.synchronize()
    ref_img = out.clone()
    ref_g = [x.clone() for x in grads]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for r in range(3):
        out.zero_()
        for x in grads:
            x.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_img), r
        for a, b in zip(grads, ref_g):
            assert rel(a.cpu().numpy(), b.cpu().numpy(), floor=1e-12) < 1e-6
        _ = plan.render(params, 6)  # eager work between replays
        torch.cuda.synchronize()


# ----------------------------------------------------------------------------- edge cases (parity)
def _check(res, gate=None):
    print(describe(res))
    assert res["divergent"] <= 0.01 * res["n_paths"]
    check_image(res)
    for k, v in res.get("grad_rel", {}).items():
        if gate is None or k in gate:
            assert v <= GRAD_TOL, (k, v)
    for k, v in res.get("pixel_grad_rel", {}).items():
        assert v <= GRAD_TOL, (k, v)


def test_edge_ragged_spp1_depth1_empty_view():
    wl = sg.config2()
    v0 = sg.crop_views(wl.views, 70, 90, 13, 7)
    v0["spp"] = 1
    v1 = sg.crop_views(wl.views, 10, 10, 0, 5)  # empty window
    v1["view_id"] = 1
    v2 = sg.crop_views(wl.views, 120, 100, 9, 9)
    v2["spp"] = 3; v2["view_id"] = 2
    wl.views = np.concatenate([v0, v1, v2])
    _check(run(wl, pixel_grad_slots=("theta",)), gate=("albedo_tex", "light_Le"))
    wl.max_depth = 1
    _check(run(wl), gate=("albedo_tex", "light_Le", "theta"))


def test_edge_no_nee_and_sensor_modes():
    wl = sg.config1()
    wl.flags = sg.FLAG_NO_NEE
    wl.views["spp"] = 16
    _check(run(wl, pixel_grad_slots=("theta", "ior")), gate=("albedo", "light_Le"))
    wl = sg.config2()
    wl.views = sg.crop_views(wl.views, 100, 120, 10, 10)
    wl.views["sensor"] = sg.SENSOR_ANALYZER4
    wl.views["spp"] = 16
    _check(run(wl, pixel_grad_slots=("roughness",)), gate=("albedo_tex", "light_Le"))
    wl.views["sensor"] = sg.SENSOR_NONE
    _check(run(wl, pixel_grad_slots=("cond_k",)), gate=("albedo_tex", "light_Le"))


# ----------------------------------------------------------------------------- errors
def test_plan_and_call_errors():
    ppt = _ppt()
    wl = sg.config1()
    scene = ppt.Scene(wl.scene.to_blob())
    bad = wl.views.copy(); bad["crop_w"] = 40  # window outside the image
    with pytest.raises(ppt.PPTError, match="EINVAL"):
        ppt.Plan(scene, bad, 3)
    bad = wl.views.copy(); bad["theta_slot"] = 9
    with pytest.raises(ppt.PPTError, match="EINVAL"):
        ppt.Plan(scene, bad, 3)
    for depth in (0, 129):
        with pytest.raises(ppt.PPTError, match="EUNSUPPORTED"):
            ppt.Plan(scene, wl.views, depth)
    plan = ppt.Plan(scene, wl.views, 3)
    params = _params(wl.scene)
    with pytest.raises(ppt.PPTError):
        plan.render(params[:-1], 1)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ppt.PPTError, match="workspace"):
        plan.render(params, 1, ws=small)


# ----------------------------------------------------------------------------- counters and timing
def test_counters_and_kernel_timing():
    ppt = _ppt()
    wl = _small_batch()
    scene = ppt.Scene(wl.scene.to_blob())
    params = _params(wl.scene)
    plan = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=2048)
    n_chunks = plan.launch_info()["n_chunks"]
    with pytest.raises(ppt.PPTError, match="EINVAL"):
        plan.kernel_times(0)  # nothing timed yet
    plan.set_timing(True)
    plan.render(params, 5)
    d = torch.randn(plan.image_numel, device="cuda")
    plan.backward(params, 5, d)
    tr, tb = plan.kernel_times(0), plan.kernel_times(1)
    st_r, st_b = plan.stats(0), plan.stats(1)
    plan.set_timing(False)
    # launches per family: one per chunk and bounce for the bounce kernels (the shadow rays of a bounce
    # are traversed in the same launch as the rays of the next one)
    assert tr["extend"][1] == tr["compact"][1] == tr["shade"][1] == n_chunks * wl.max_depth
    assert tr["shadow"][1] == 0
    # (the first traversal launch of a chunk generates its camera rays: no launch of their own)
    assert tr["camera"][1] == tb["camera"][1] == 0
    assert tr["accum"][1] == n_chunks and tr["fold"][1] == tr["replay"][1] == 0
    assert tb["fold"][1] == tb["replay"][1] == n_chunks and tb["accum"][1] == 0
    for t in (tr, tb):
        assert all(ms >= 0.0 for ms, _ in t.values()) and sum(ms for ms, _ in t.values()) > 0.0
    # the backward's primal pass retraces exactly the render's paths (same seed); node and
    # primitive counts depend on which rays share a wavefront (speculative leaf postponement),
    # and the queues of later bounces are filled in a different order, so they only agree closely
    for k in ("vertices", "paths", "rays", "shadow_rays"):
        assert st_r[k] == st_b[k], k
    for k in ("nodes", "prim_tests", "shadow_nodes", "shadow_prim_tests"):
        assert abs(st_r[k] - st_b[k]) <= 0.05 * st_r[k], k
    assert st_r["paths"] == plan.num_paths
    assert st_r["vertices"] <= st_r["rays"] <= st_r["paths"] * wl.max_depth
    assert 0 < st_r["shadow_rays"] <= st_r["vertices"]
    assert st_r["nodes"] >= st_r["rays"] and st_r["shadow_nodes"] >= st_r["shadow_rays"]


# ----------------------------------------------------------------------------- autograd
def test_autograd_function_matches_backward():
    ppt = _ppt()
    wl = sg.config1()
    plan = ppt.Plan(ppt.Scene(wl.scene.to_blob()), wl.views, wl.max_depth)
    params = [p.clone().requires_grad_(True) for p in _params(wl.scene)]
    target = plan.render([p.detach() for p in params], 1234)
    img = ppt.render(plan, params, wl.seed)
    loss = ((img - target) ** 2).sum()
    loss.backward()
    d = (2 * (img.detach() - target)).contiguous()
    ref = plan.backward([p.detach() for p in params], wl.seed, d)
    for p, r in zip(params, ref):
        assert torch.allclose(p.grad, r, rtol=1e-5, atol=1e-7)


# ----------------------------------------------------------------------------- full size, sampled
# the benchmark's timed configuration: the whole 67.1M-path batch as one chunk
BENCH_CHUNK = 1 << 26


def test_full_size_batched_sampled_parity():
    """The 128-view configuration at full size in the launch configuration the benchmark times (one
    2^26-path chunk), checked on sampled 8x8 pixel windows of twelve views (the oracle computes
    them one by one; dL/dI is zero outside the windows, so the gradient is exactly theirs), for the
    three gradient groups the benchmark's backward computes: the albedo texture, the per-material
    roughness and the per-view polarizer angles, all compared element by element."""
    ppt = _ppt()
    wl = sg.config3()
    scene = ppt.Scene(wl.scene.to_blob())
    plan = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=BENCH_CHUNK)
    assert plan.launch_info()["n_chunks"] == 1
    params = _params(wl.scene)
    rng = np.random.default_rng(2024)
    views_pick = np.sort(rng.choice(len(wl.views), 12, replace=False))
    picks = [(int(v), int(rng.integers(16, 104)), int(rng.integers(16, 104))) for v in views_pick]
    B = 8
    osc = oracle.OracleScene.from_scene(wl.scene)
    p64 = [p.astype(np.float64) for p in wl.scene.params()]
    sub = np.concatenate([sg.crop_views(wl.views[v:v + 1], x0, y0, B, B) for v, x0, y0 in picks])
    sig_o = osc.run(p64, sub, wl.max_depth, wl.seed, want_sig=True, want_image=False)["sig"]
    # signatures of the same paths from the full launch
    sig_full = plan.signatures(params, wl.seed).cpu().numpy().view(np.uint64)
    spp = int(wl.views["spp"][0]); W = int(wl.views["width"][0])
    idx = []
    for v, x0, y0 in picks:
        base = v * W * W * spp
        for y in range(y0, y0 + B):
            for x in range(x0, x0 + B):
                idx.extend(base + (y * W + x) * spp + np.arange(spp))
    idx = np.asarray(idx)
    agree = sig_full[idx] == sig_o
    mask_full = np.ones(plan.num_paths, np.uint8)
    mask_full[idx[~agree]] = 0
    plan.set_path_mask(torch.from_numpy(mask_full).cuda())
    img = plan.render(params, wl.seed).cpu().numpy()
    ref = osc.run(p64, sub, wl.max_depth, wl.seed, mask=agree.astype(np.uint8))
    offs = sg.view_offsets(wl.views)
    got = []
    for v, x0, y0 in picks:
        blk = img[int(offs[v]):int(offs[v]) + W * W * 12].reshape(W, W, 12)
        got.append(blk[y0:y0 + B, x0:x0 + B].ravel())
    got = np.concatenate(got)
    m = image_metrics(got, ref["image"], sub)
    print("divergent", int((~agree).sum()), "of", agree.size, "image", m)
    assert (~agree).sum() <= 0.01 * agree.size
    check_image(m)
    # gradients of the windows only
    d_sub = rng.normal(size=ref["image"].size).astype(np.float32)
    d_full = np.zeros(plan.image_numel, np.float32)
    k = 0
    for v, x0, y0 in picks:
        blk = d_full[int(offs[v]):int(offs[v]) + W * W * 12].reshape(W, W, 12)
        blk[y0:y0 + B, x0:x0 + B] = d_sub[k:k + B * B * 12].reshape(B, B, 12)
        k += B * B * 12
    want = [n in wl.grad_slots for n in wl.scene.slot_names]
    g = plan.backward(params, wl.seed, torch.from_numpy(d_full).cuda(), want=want)
    s = wl.scene.slot
    gr = osc.run(p64, sub, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d_sub.astype(np.float64),
                 mask=agree.astype(np.uint8), grad_slots=[s(n) for n in wl.grad_slots])["grads"]
    assert set(wl.grad_slots) == {"albedo_tex", "roughness", "theta_views"}
    for name in wl.grad_slots:
        r = rel(g[s(name)].cpu().numpy(), gr[s(name)], floor=1e-12)
        print(name, r, "nonzero entries", int(np.count_nonzero(gr[s(name)])))
        assert np.count_nonzero(gr[s(name)]) > 0
        assert r <= GRAD_TOL, (name, r)


def test_deep_polarizer_stack_closed_form():
    # 85 sheets whose axes turn by 1 degree each, in front of an unpolarized emitter wall: the
    # camera sees Le/2 prod cos^2(1 deg) (Malus along the chain), fully linearly polarized along
    # the first sheet's axis; 86 vertices per path, past the 64 of the default plans.  The
    # gradient of the image sum with respect to Le is the image sum over Le.
    ppt = _ppt()
    n = 85
    step = np.deg2rad(1.0)
    angles = [k * step for k in range(n)]
    sc, _ = sg.emitter_wall_scene(le=10.0, sheets=tuple(angles), z_light=-(n * 0.05 + 4.0))
    v = np.asarray([sg.make_view(0, 8, 8, 2, (0, 0, 0), (0, 0, -1), (0, 1, 0), 0.01, sg.SENSOR_NONE)], sg.VIEW_DTYPE)
    for depth in (n + 1, 128):
        plan = ppt.Plan(ppt.Scene(sc.to_blob()), v, depth)
        params = _params(sc)
        img = plan.render(params, 3).cpu().numpy().reshape(-1, 3, 4)
        e = 5.0 * np.cos(step) ** (2 * (n - 1))
        assert np.allclose(img[..., 0], e, rtol=2e-5)
        assert np.allclose(np.hypot(img[..., 1], img[..., 2]), e, rtol=2e-5)
        assert np.allclose(img[..., 3], 0.0, atol=1e-6)
        d = torch.zeros(plan.image_numel, device="cuda")
        d[0::4] = 1.0
        g = plan.backward(params, 3, d)[sc.slot("light_Le")].double().sum().item()
        assert abs(g - img[..., 0].sum() / 10.0) <= 2e-5 * abs(g)
    plan = ppt.Plan(ppt.Scene(sc.to_blob()), v, n)  # one vertex short of the emitter: black
    assert float(plan.render(_params(sc), 3).abs().max()) == 0.0


def test_adam_through_autograd_reduces_loss():
    # inverse rendering in miniature: recover the config-1 albedo from a target rendered with the
    # true albedo, through PolarizedRender with a decorrelated backward seed every step
    ppt = _ppt()
    wl = sg.config1()
    plan = ppt.Plan(ppt.Scene(wl.scene.to_blob()), wl.views, wl.max_depth)
    truth = _params(wl.scene)
    target = sum(plan.render(truth, 100 + k) for k in range(8)) / 8.0
    si = wl.scene.slot("albedo")
    params = [p.clone() for p in truth]
    params[si] = torch.full_like(truth[si], 0.5).requires_grad_(True)
    opt = torch.optim.Adam([params[si]], lr=0.05)
    losses = []
    for it in range(40):
        opt.zero_grad()
        img = ppt.render(plan, params, 1 + it, backward_seed=10_000 + it)
        loss = (img - target).pow(2).mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            params[si].clamp_(0.0, 1.0)
        losses.append(float(loss.detach()))
    err0 = float((torch.full_like(truth[si], 0.5) - truth[si]).abs().max())
    err1 = float((params[si].detach() - truth[si]).abs().max())
    assert np.mean(losses[-5:]) < np.mean(losses[:5])
    assert err1 < 0.5 * err0


def test_workspace_depends_on_chunk_and_depth_only():
    # the backward workspace holds one chunk of paths with D cache records each: it grows with
    # the chunk and the depth, not with the number of views or paths
    ppt = _ppt()
    wl = _small_batch(n_views=6)
    scene = ppt.Scene(wl.scene.to_blob())
    q = 4096
    ws = {}
    for nv in (2, 6):
        for D in (2, 6):
            plan = ppt.Plan(scene, wl.views[:nv], D, chunk_paths=q)
            assert plan.num_paths > q
            ws[(nv, D)] = plan.workspace_bytes(1)
    assert ws[(2, 2)] == ws[(6, 2)] and ws[(2, 6)] == ws[(6, 6)]
    assert abs((ws[(6, 6)] - ws[(6, 2)]) - 4 * q * 128) <= 256


def test_plain_c_caller_matches_binding(tmp_path):
    # a C program (tests/c/abi_render.c) drives scene creation, render and backward through the
    # C ABI with its own hipMalloc'ed buffers; its image and gradients equal the binding's
    import subprocess

    from test_abi import build_c_program
    ppt = _ppt()
    exe = build_c_program(tmp_path)
    wl = sg.config1()
    blob = wl.scene.to_blob()
    (tmp_path / "scene.blob").write_bytes(blob)
    (tmp_path / "views.bin").write_bytes(np.ascontiguousarray(wl.views).tobytes())
    params = wl.scene.params()
    (tmp_path / "params.bin").write_bytes(b"".join(np.ascontiguousarray(p, np.float32).tobytes() for p in params))
    out = tmp_path / "out.bin"
    r = subprocess.run([exe, str(tmp_path / "scene.blob"), str(tmp_path / "views.bin"), str(tmp_path / "params.bin"),
                        str(wl.seed), str(wl.max_depth), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    got = np.fromfile(str(out), np.float32)
    plan = ppt.Plan(ppt.Scene(blob), wl.views, wl.max_depth)
    tp = _params(wl.scene)
    img = plan.render(tp, wl.seed).cpu().numpy()
    grads = plan.backward(tp, wl.seed, torch.ones(plan.image_numel, device="cuda"))
    ref = np.concatenate([img] + [g.cpu().numpy() for g in grads])
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-6)


def test_hybrid_replay_matches_cached_and_saves_workspace():
    # deep paths (85 polarizer sheets, depth 128): the hybrid replay gives the cached gradient
    # with a fraction of the backward workspace; batches and chunking as for the cached replay
    ppt = _ppt()
    wl = sg.polarizer_stack(width=64, height=36, spp=2)
    scene = ppt.Scene(wl.scene.to_blob())
    params = _params(wl.scene)
    cached = ppt.Plan(scene, wl.views, 128)
    d = torch.randn(cached.image_numel, device="cuda")
    gc = cached.backward(params, 4, d)
    for k in (1, 8, 16, 200 // 2):
        hyb = ppt.Plan(scene, wl.views, 128, checkpoint_interval=k)
        gh = hyb.backward(params, 4, d)
        for a, b in zip(gc, gh):
            assert rel(b.cpu().numpy(), a.cpu().numpy(), floor=1e-12) < 1e-5
        if k in (8, 16):  # hit records + a suffix every k vertices + k records of block scratch
            assert hyb.workspace_bytes(1) < 0.4 * cached.workspace_bytes(1)
    hc = ppt.Plan(scene, wl.views, 128, chunk_paths=1000, checkpoint_interval=16)
    for a, b in zip(gc, hc.backward(params, 4, d)):
        assert rel(b.cpu().numpy(), a.cpu().numpy(), floor=1e-12) < 1e-5
    for bad in (-1, 129):
        with pytest.raises(ppt.PPTError, match="EINVAL"):
            ppt.Plan(scene, wl.views, 128, checkpoint_interval=bad)
