"""GPU-vs-oracle parity harness (used by the gpu-marked tests, smoke and bench).

Protocol: both sides export a 64-bit signature per path (primitive ids, light-sample
states and lobes of its vertices).  Paths whose signatures differ took different discrete
decisions in FP32 and FP64 (grazing hits, lobe choices at u ~ F); they are masked out on
both sides, counted, and reported.  On the remaining paths the image must agree to
relative L2 <= 1e-4 and every requested gradient group to relative L2 <= 1e-3.
"""
from __future__ import annotations

import numpy as np

import oracle
import scenegen as sg

IMG_TOL = 1e-4
GRAD_TOL = 1e-3


def rel(a, b, floor=0.0):
    a = np.asarray(a, np.float64).ravel(); b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / max(nb, floor)) if max(nb, floor) > 0 else float(np.linalg.norm(a))


def pixel_slices(views):
    """For every (view, crop pixel): the list of its entries in the image vector."""
    offs = sg.view_offsets(views)
    out = []
    for v, vw in enumerate(views):
        a = sg.analyzer_count(int(vw["sensor"]))
        w, h = int(vw["crop_w"]), int(vw["crop_h"])
        for p in range(w * h):
            out.append([int(offs[v]) + ai * w * h * 12 + p * 12 for ai in range(a)])
    return out


def loss_delta_c1(wl, params=None):
    """dL/dI of the config-1 loss L = sum (I - T)^2, T rendered at theta = 45 deg with seed + 1000
    (both renders by the oracle, so the GPU and the oracle receive the same float32 delta)."""
    params = wl.scene.params() if params is None else params
    osc = oracle.OracleScene.from_scene(wl.scene)
    p64 = [p.astype(np.float64) for p in params]
    pt = [p.copy() for p in p64]
    pt[wl.scene.slot("theta")][0] = np.deg2rad(wl.meta["target_theta_deg"])
    T = osc.run(pt, wl.views, wl.max_depth, wl.meta["target_seed"])["image"]
    I = osc.run(p64, wl.views, wl.max_depth, wl.seed)["image"]
    return (2.0 * (I - T)).astype(np.float32)


def run(wl, params=None, seed=None, d=None, grad_slots=None, with_grads=True, oracle_mode=oracle.MODE_TAPE_AD,
        device="cuda", plan_kw=None, pixel_grad_slots=(), max_pixels=None):
    """Render (+ backward) on the GPU and with the oracle on the same seeded inputs.

    ``pixel_grad_slots``: slots whose gradient is also compared split by pixel (the gradient
    images of Sec. 5.1), which isolates FP32 rounding from the cancellation of a scalar sum."""
    import torch

    import paper_2607_13265_amd as ppt

    seed = wl.seed if seed is None else seed
    params = wl.scene.params() if params is None else [np.asarray(p, np.float32) for p in params]
    scene = ppt.Scene(wl.scene.to_blob())
    plan = ppt.Plan(scene, wl.views, wl.max_depth, wl.flags, **(plan_kw or {}))
    tp = [torch.from_numpy(p).to(device) for p in params]
    osc = oracle.OracleScene.from_scene(wl.scene)
    p64 = [p.astype(np.float64) for p in params]
    sig_o = osc.run(p64, wl.views, wl.max_depth, seed, flags=wl.flags, want_sig=True, want_image=False)["sig"]
    sig_g = plan.signatures(tp, seed).cpu().numpy().view(np.uint64)
    mask = (sig_o == sig_g).astype(np.uint8)
    plan.set_path_mask(torch.from_numpy(mask).to(device))
    img_g = plan.render(tp, seed).cpu().numpy().astype(np.float64)
    out = {"plan": plan, "mask": mask, "divergent": int(mask.size - mask.sum()), "n_paths": int(mask.size)}
    ro = osc.run(p64, wl.views, wl.max_depth, seed, flags=wl.flags, mask=mask)
    out["img_gpu"], out["img_ref"] = img_g, ro["image"]
    out["img_rel"] = rel(img_g, ro["image"])
    out["n_vertices_ref"] = ro["n_vertices"]
    out["stats_render"] = plan.stats(0)
    if with_grads:
        if d is None:
            d = np.random.default_rng(12345).normal(size=plan.image_numel).astype(np.float32)
        d = np.asarray(d, np.float32)
        slots = list(range(len(params))) if grad_slots is None else [wl.scene.slot(s) if isinstance(s, str) else s
                                                                     for s in grad_slots]
        want = [i in slots for i in range(len(params))]
        g = plan.backward(tp, seed, torch.from_numpy(d).to(device), want=want)
        go = osc.run(p64, wl.views, wl.max_depth, seed, flags=wl.flags, mode=oracle_mode,
                     d_image=d.astype(np.float64), grad_slots=slots, mask=mask)["grads"]
        out["grads_gpu"] = {i: g[i].cpu().numpy().astype(np.float64) for i in slots}
        out["grads_ref"] = {i: go[i] for i in slots}
        out["grad_rel"] = {}
        for i in slots:
            ref = go[i]
            scale = np.linalg.norm(ref)
            out["grad_rel"][wl.scene.slot_names[i]] = rel(out["grads_gpu"][i], ref, floor=1e-12) if scale > 0 else \
                float(np.linalg.norm(out["grads_gpu"][i]))
        out["stats_backward"] = plan.stats(1)
        out["pixel_grad_rel"] = {}
        pix = pixel_slices(wl.views)
        sel = np.arange(len(pix))
        if max_pixels is not None and len(pix) > max_pixels:
            sel = np.sort(np.random.default_rng(7).choice(len(pix), max_pixels, replace=False))
        for name in pixel_grad_slots:
            si = wl.scene.slot(name)
            gref = osc.run(p64, wl.views, wl.max_depth, seed, flags=wl.flags, mode=oracle_mode,
                           d_image=d.astype(np.float64), grad_slots=[si], mask=mask, want_image=False,
                           pixel_grad_slot=si)["pixel_grad"][sel]
            ggpu = np.zeros(len(sel))
            want1 = [i == si for i in range(len(params))]
            dt = torch.from_numpy(d).to(device)
            for j, p in enumerate(sel):
                dp = torch.zeros_like(dt)
                for o in pix[p]:
                    dp[o:o + 12] = dt[o:o + 12]
                ggpu[j] = float(plan.backward(tp, seed, dp, want=want1)[si].double().sum().item())
            out["pixel_grad_rel"][name] = rel(ggpu, gref, floor=1e-12)
    return out


def describe(res):
    s = f"img rel {res['img_rel']:.2e}, divergent {res['divergent']}/{res['n_paths']}"
    if "grad_rel" in res:
        s += ", grads " + ", ".join(f"{k} {v:.2e}" for k, v in res["grad_rel"].items())
    if res.get("pixel_grad_rel"):
        s += ", gradient images " + ", ".join(f"{k} {v:.2e}" for k, v in res["pixel_grad_rel"].items())
    return s
