#!/usr/bin/env python3
"""Benchmark: Mpath-vertices/s of forward + PRB adjoint (render + backward) on one MI355X.

Workload (the batched configuration the metric names): the seeded 20.5k-triangle scene of
16 icospheres + ground + one area light, 4 camera poses on a ring x 32 polarizer angles
theta_k = k pi / 32 = 128 views, 128 x 128 pixels, 32 spp, max depth 6, random dL/dStokes
~ N(0, 1).  One step = one batched persistent render launch + one batched persistent
backward launch over all 128 views, replayed from a captured HIP graph.  The plain
per-view form (128 render + 128 backward launches) is timed beside it on identical paths.

A path vertex is one surface interaction of a camera path, counted in-kernel; the value is
vertices / (render + backward time).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpath-vertices/s fwd+PRB adjoint; batched vs per-view launch, grad rel.err≤1e-3"

# Algorithmic FP32 operations (an FMA counts 2) per unit of work, read off the kernel source;
# the design notes itemise them.
FLOP_NODE = 51          # one two-box BVH node test: 12 FMA + 24 min/max + 3 compares
FLOP_PRIM = 52          # one Moller-Trumbore triangle test
FLOP_SHADE = 450        # one vertex in the shading kernel (sampling, Fresnel/GGX weight, next-event setup)
FLOP_REPLAY = 950       # one vertex of the adjoint replay (re-evaluation + vector-Jacobian products)
BYTES_FOLD_VERTEX = 144  # fold: 24 cache words read + 12 written back per vertex
BYTES_FOLD_PATH = 96     # fold: keys read (16), adjoint rows (48) + camera ray (32) written per folded path
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (256 CU x 2.4 GHz x 64 lanes x FMA x packed)
PEAK_HBM_GBS = 8000.0
# files whose content decides whether stored hardware counters still describe the kernels
KERNEL_SOURCES = ("paper_2607_13265_amd/csrc/ppt_kernels.hip", "paper_2607_13265_amd/csrc/ppt_kernels_ext.hip",
                  "paper_2607_13265_amd/csrc/ppt_device.h",
                  "paper_2607_13265_amd/csrc/ppt_internal.h", "paper_2607_13265_amd/csrc/ppt_host.cpp",
                  "paper_2607_13265_amd/csrc/ppt_half.h",  # (the host builds the BVH the kernels traverse)
                  "paper_2607_13265_amd/build.py")  # (and the compiler flags)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_{}.md")
KERNEL_SYMBOL = {"extend": "ppt::k_extend", "shade": "ppt::k_shade", "compact": "ppt::k_compact",
                 "fold": "ppt::k_fold", "replay": "ppt::k_replay", "accum": "ppt::k_accum"}


def one_or_list(xs):
    return xs[0] if len(set(xs)) == 1 else xs


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, kernel: str, chunk: int):
    """HBM bytes per launch of `kernel` from the committed counter summary of the workload, or None
    when there is none for this kernel and chunk size or the kernel sources changed since."""
    path = TRAFFIC_FILE.format(workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if line.startswith("    ") and ":" in line:
                k, v = line.strip().split(":", 1)
                kv.setdefault(k.strip(), []).append(v.strip())
    try:
        if kv["source_digest"][0] != kernel_source_digest() or int(kv["chunk_paths"][0]) != chunk:
            return None
        for name, val in zip(kv["kernel"], kv["traffic_bytes_per_launch"]):
            if name == kernel:
                return float(val)
    except (KeyError, ValueError, IndexError):
        return None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--per-view-steps", type=int, default=2)
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=48, help="full views in the oracle sample (all host threads)")
    ap.add_argument("--cpu-views-1t", type=int, default=2, help="full views in the one-thread oracle sample")
    ap.add_argument("--bounded-chunk", type=int, default=1 << 22,
                    help="chunk size of the memory-bounded measurement (0: skip)")
    ap.add_argument("--timing-steps", type=int, default=3, help="eager steps with per-kernel event timing")
    ap.add_argument("--workload", choices=("batched128", "config2", "uneven8", "lightstage", "optimise", "depth_sweep",
                                           "comparators"),
                    default="batched128",
                    help="batched128: 128 views of one scene (the headline); config2: one 256x256 view at 64 spp, "
                         "depth 8; uneven8: eight worlds of uneven size; "
                         "lightstage: 8 views with circular lights, four analyzers and normal/specular maps; "
                         "optimise: Adam recovery of textures and lights through the autograd wrapper; "
                         "depth_sweep: time and memory against the maximum depth behind an 85-sheet polarizer stack; "
                         "comparators: gradient relative error of every backward method against FP64 conventional AD, "
                         "and their time and memory")
    ap.add_argument("--no-deep", action="store_true",
                    help="skip the deep-path point (85-sheet stack at depth 128) of the headline run")
    ap.add_argument("--opt-steps", type=int, default=200)
    ap.add_argument("--res", type=int, default=128)
    ap.add_argument("--spp", type=int, default=32)
    ap.add_argument("--chunk-paths", type=int, default=0, help="0: autotuned (cached per workload)")
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--json-out", default="")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scales the HBM byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def optimise(args, torch, ppt, sg, dev):
    """Inverse rendering through PolarizedRender: 8 polarizer angles, 512x512, 16 spp, depth 6;
    Adam on the hidden 256x256 albedo and roughness maps and the two lights' RGB intensities,
    with a decorrelated backward seed every step.  Reports the loss curve, the time per step and
    the peak device memory and time of one backward: PRB in chunks, the cached replay with all paths
    in one chunk, and the conventional-AD baseline (a stored tape of every vertex's loop state for
    every path, reverse sweep)."""
    wl = sg.config4(truth=False)
    truth = sg.config4(truth=True)
    scene = ppt.Scene(wl.scene.to_blob())
    names = wl.scene.slot_names
    p_true = [torch.from_numpy(p).to(dev) for p in truth.scene.params()]
    chunk = args.chunk_paths or (1 << 23)
    plan = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=chunk)
    plan.set_stats(False)
    target = plan.render(p_true, 777_777).clone()
    opt_names = ("albedo_tex", "roughness_tex", "light_Le")
    params = [torch.from_numpy(p).to(dev).requires_grad_(n in opt_names) for n, p in zip(names, wl.scene.params())]
    lr = {"albedo_tex": 0.02, "roughness_tex": 0.02, "light_Le": 0.1}
    opt = torch.optim.Adam([{"params": [params[names.index(n)]], "lr": lr[n]} for n in opt_names])
    bounds = {"albedo_tex": (0.0, 1.0), "roughness_tex": (0.01, 1.0), "light_Le": (0.0, 100.0)}

    def errors():
        return {n: float((params[names.index(n)].detach() - p_true[names.index(n)]).pow(2).mean().sqrt())
                for n in opt_names}

    err0 = errors()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    losses, times = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for it in range(args.opt_steps):
        e0.record()
        opt.zero_grad(set_to_none=True)
        img = ppt.render(plan, params, 1 + it, backward_seed=1_000_003 + it)
        loss = (img - target).pow(2).mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            for n in opt_names:
                params[names.index(n)].clamp_(*bounds[n])
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        losses.append(float(loss.detach()))
        if it % 20 == 0 or it == args.opt_steps - 1:
            log(f"[optimise] step {it}: loss {losses[-1]:.6e}, {times[-1]:.1f} ms")
    peak_prb = torch.cuda.max_memory_allocated(dev)
    err1 = errors()
    n_paths = plan.num_paths
    del opt
    torch.cuda.empty_cache()
    d = (2.0 / target.numel()) * (plan.render([p.detach() for p in params], 1) - target)
    want_opt = [n in opt_names for n in names]
    pd = [p.detach() for p in params]

    def one_backward(pl):
        """Peak device memory (GB) and time (ms) of one backward of plan pl, and its gradients."""
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats(dev)
        pl.set_stats(False)
        pl.backward(pd, 1, d, want=want_opt)  # (allocates the workspace)
        torch.cuda.synchronize()
        e0.record()
        g = pl.backward(pd, 1, d, want=want_opt)
        e1.record()
        torch.cuda.synchronize()
        return torch.cuda.max_memory_allocated(dev), e0.elapsed_time(e1), g

    peak_chunk, ms_chunk, g_chunk = one_backward(plan)
    # the cached replay with every path's per-vertex records at once (one chunk)
    store = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=((n_paths + 63) // 64) * 64)
    ws_bytes = store.workspace_bytes(1)
    peak_store, ms_store, _ = one_backward(store)
    del store
    # the conventional-AD baseline: a tape of every vertex's loop state for every path, reverse sweep
    tape = ppt.Plan(scene, wl.views, wl.max_depth, chunk_paths=((n_paths + 63) // 64) * 64, tape=True)
    tape_ws = tape.workspace_bytes(1)
    peak_tape, ms_tape, g_tape = one_backward(tape)
    del tape
    tape_rel = {n: float((a.double() - b.double()).norm() / max(float(b.double().norm()), 1e-30))
                for n, a, b in zip(names, g_tape, g_chunk) if a is not None}
    log(f"[optimise] backward peak GB: PRB chunked {peak_chunk / 1e9:.2f}, one-chunk cached {peak_store / 1e9:.2f}, "
        f"tape AD {peak_tape / 1e9:.2f}; tape vs PRB gradient rel {tape_rel}")
    res = {
        "metric": "inverse rendering: Adam steps through the autograd wrapper (render + PRB backward)",
        "workload": f"{len(wl.views)} polarizer angles, 512x512, 16 spp, depth {wl.max_depth}, 40.96k triangles, "
                    "2 lights; recover 256x256x3 albedo, 256x256 roughness, 6 light intensities",
        "steps": args.opt_steps, "paths_per_step": int(n_paths), "chunk_paths": plan.launch_info()["chunk_paths"],
        "ms_per_step_median": float(np.median(times)), "loss_first": losses[0], "loss_last": losses[-1],
        "loss_curve": [round(x, 9) for x in losses],
        "rmse_to_truth_start": err0, "rmse_to_truth_end": err1,
        "peak_device_memory_gb": {"optimisation_loop_prb_chunked": round(peak_prb / 1e9, 3),
                                  "backward_prb_chunked": round(peak_chunk / 1e9, 3),
                                  "backward_cached_replay_one_chunk": round(peak_store / 1e9, 3),
                                  "backward_tape_ad": round(peak_tape / 1e9, 3)},
        "backward_ms": {"prb_chunked": round(ms_chunk, 2), "cached_replay_one_chunk": round(ms_store, 2),
                        "tape_ad": round(ms_tape, 2)},
        "workspace_gb": {"cached_replay_one_chunk": round(ws_bytes / 1e9, 3), "tape_ad": round(tape_ws / 1e9, 3)},
        "tape_ad_grad_rel_diff_vs_prb": tape_rel,
        "prb_workspace_gb": {"render": round(plan.workspace_bytes(0) / 1e9, 3),
                             "backward": round(plan.workspace_bytes(1) / 1e9, 3)},
    }
    line = json.dumps(res)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def depth_sweep(args, torch, ppt, sg, dev):
    """Render + backward (gradient of the floor albedo) of the 1280x720, 1 spp scene behind 85
    polarizer sheets for maximum depths 1..128: time, vertices, workspace and peak device memory,
    with all paths in one chunk and with 128k-path chunks (cached suffix replay), with all paths in
    one chunk under the hybrid replay with checkpoints every 16 vertices (recomputation only, and
    with Eq. 3's decision rule), and for the conventional-AD baseline (stored tape, all paths)."""
    rows = []
    for D in (1, 2, 4, 8, 16, 32, 48, 64, 86, 96, 112, 128):
        wl = sg.polarizer_stack(max_depth=D)
        scene = ppt.Scene(wl.scene.to_blob())
        params = [torch.from_numpy(p).to(dev) for p in wl.scene.params()]
        want = [n in wl.grad_slots for n in wl.scene.slot_names]
        for chunk, kc, extra in ((0, 0, {}), (1 << 17, 0, {}), (0, 16, {}), (0, 16, {"hybrid_rule": (0.5, 1e-3)}),
                                 (0, 0, {"tape": True})):
            plan = ppt.Plan(scene, wl.views, D, chunk_paths=chunk or wl.n_paths(), checkpoint_interval=kc, **extra)
            d = torch.from_numpy(np.random.default_rng(D).standard_normal(plan.image_numel, dtype=np.float32)).to(dev)
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            torch.cuda.reset_peak_memory_stats(dev)
            base = torch.cuda.memory_allocated(dev)
            plan.render(params, wl.seed)
            plan.backward(params, wl.seed, d, want=want)
            torch.cuda.synchronize()
            st = plan.stats(1)
            plan.set_stats(False)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            tr, tb = [], []
            for _ in range(3):
                e0.record()
                plan.render(params, wl.seed)
                e1.record()
                plan.backward(params, wl.seed, d, want=want)
                e2.record()
                torch.cuda.synchronize()
                tr.append(e0.elapsed_time(e1)); tb.append(e1.elapsed_time(e2))
            label = ("tape AD" if extra.get("tape") else
                     f"hybrid k={kc}" + (" + Eq. 3 rule (gamma 0.5, eps 1e-3)" if extra.get("hybrid_rule") else "")
                     if kc else "cached")
            rows.append({"max_depth": D, "chunk_paths": plan.launch_info()["chunk_paths"],
                         "replay": label,
                         "vertices": st["vertices"], "render_ms": round(float(np.median(tr)), 3),
                         "backward_ms": round(float(np.median(tb)), 3),
                         "workspace_gb": {"render": round(plan.workspace_bytes(0) / 1e9, 4),
                                          "backward": round(plan.workspace_bytes(1) / 1e9, 4)},
                         "peak_gb": round((torch.cuda.max_memory_allocated(dev) - base) / 1e9, 4)})
            log(f"[depth] {rows[-1]}")
            del plan
    res = {"metric": "render + PRB backward time and device memory against the maximum path depth",
           "workload": "1280x720, 1 spp, 85 linear polarizer sheets (axes 1 degree apart) in front of a Lambertian "
                       "floor and wall under an area light; gradient of the floor albedo",
           "rows": rows}
    line = json.dumps(res)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


# the backward methods: the paper's cached suffix replay, its hybrid variant with Eq. 3's rule, and the
# comparators of its evaluation (Sec. 4.2, 5.1): noise-regularised P-PRB, P-RB and conventional AD
METHODS = (("ours (cached suffix replay)", {}),
           ("ours hybrid k=2, Eq. 3 rule (gamma 0.5, eps 1e-3)", {"checkpoint_interval": 2, "hybrid_rule": (0.5, 1e-3)}),
           ("P-PRB sigma 0.01", {"pprb_sigma": 0.01}),
           ("P-PRB sigma 0.1", {"pprb_sigma": 0.1}),
           ("P-PRB sigma 1", {"pprb_sigma": 1.0}),
           ("P-RB", {"prb": True}),
           ("conventional AD (GPU tape)", {"tape": True}))


def comparators(args, torch, ppt, sg, dev):
    """Relative error (RE, ||g - g_ref|| / ||g_ref||, the metric of the paper's gradient analysis) of every
    backward method's gradient per parameter group against the FP64 oracle's conventional AD of the same
    paths, on the config-1 scene (its L2 loss to a target at 45 degrees) and a config-2 window (random
    dL/dI); then the time and peak memory of one backward of each method on the 128-view batch and on
    the 85-sheet stack at depth 128."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import loss_delta_c1
    tables = []
    for name, wl, d in (("config 1 (32x32, 4 spp, depth 3, L2 loss)", sg.config1(), None),
                        ("config 2 window (13x11 of 256x256, 64 spp, depth 8, random dL/dI)", sg.config2(), None)):
        if wl.name == "c1_tiny":
            d = loss_delta_c1(wl)
        else:
            wl.views = sg.crop_views(wl.views, 96, 112, 13, 11)
            d = np.random.default_rng(12345).normal(size=sg.image_numel(wl.views)).astype(np.float32)
        osc = oracle.OracleScene.from_scene(wl.scene)
        p64 = [p.astype(np.float64) for p in wl.scene.params()]
        ref = osc.run(p64, wl.views, wl.max_depth, wl.seed, flags=wl.flags, mode=oracle.MODE_TAPE_AD,
                      d_image=d.astype(np.float64))["grads"]
        scene = ppt.Scene(wl.scene.to_blob())
        params = [torch.from_numpy(p).to(dev) for p in wl.scene.params()]
        dt = torch.from_numpy(d).to(dev)
        rows = {}
        for label, kw in METHODS:
            plan = ppt.Plan(scene, wl.views, wl.max_depth, wl.flags, **kw)
            g = plan.backward(params, wl.seed, dt)
            re = {}
            for i, n in enumerate(wl.scene.slot_names):
                gg = g[i].double().cpu().numpy()
                nr = float(np.linalg.norm(ref[i]))
                if nr > 0:
                    re[n] = float(np.linalg.norm(gg - ref[i]) / nr) if np.all(np.isfinite(gg)) else float("nan")
            rows[label] = re
            log(f"[comparators] {name} / {label}: {re}")
        tables.append({"scene": name, "reference": "FP64 oracle, conventional AD (stored tape), same paths",
                       "relative_error": rows})
    # time and memory of one backward
    perf = []
    for name, wl, chunk in (("128 views, 128x128, 32 spp, depth 6", sg.config3(), 1 << 24),
                            ("85-sheet stack, 1280x720, 1 spp, depth 128", sg.polarizer_stack(max_depth=128), 0)):
        scene = ppt.Scene(wl.scene.to_blob())
        params = [torch.from_numpy(p).to(dev) for p in wl.scene.params()]
        want = [n in wl.grad_slots for n in wl.scene.slot_names]
        n_paths = int(wl.n_paths())
        d = torch.from_numpy(np.random.default_rng(7).standard_normal(sg.image_numel(wl.views), dtype=np.float32)).to(dev)
        for label, kw in METHODS:
            if "P-PRB sigma 0.01" in label or "P-PRB sigma 1" == label:
                continue
            ck = ((n_paths + 63) // 64) * 64 if kw.get("tape") else (chunk or ((n_paths + 63) // 64) * 64)
            try:
                plan = ppt.Plan(scene, wl.views, wl.max_depth, wl.flags, chunk_paths=ck, **kw)
                plan.set_stats(False)
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                torch.cuda.reset_peak_memory_stats(dev)
                base = torch.cuda.memory_allocated(dev)
                plan.backward(params, wl.seed, d, want=want)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ts = []
                for _ in range(3):
                    e0.record()
                    plan.backward(params, wl.seed, d, want=want)
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1))
                row = {"workload": name, "method": label, "chunk_paths": plan.launch_info()["chunk_paths"],
                       "backward_ms": round(float(np.median(ts)), 3),
                       "workspace_gb": round(plan.workspace_bytes(1) / 1e9, 3),
                       "peak_gb": round((torch.cuda.max_memory_allocated(dev) - base) / 1e9, 3)}
                del plan
            except Exception as e:  # noqa: BLE001 (reported: e.g. a workspace beyond the device memory)
                row = {"workload": name, "method": label, "error": str(e)[:200]}
            torch.cuda.empty_cache()
            perf.append(row)
            log(f"[comparators] {row}")
    res = {"metric": "gradient relative error against conventional AD, and backward time and memory, per method",
           "tables": tables, "backward_cost": perf}
    line = json.dumps(res)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2607_13265_amd as ppt
    import scenegen as sg

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration} MiB three times")
        return
    if args.workload == "optimise":
        return optimise(args, torch, ppt, sg, dev)
    if args.workload == "depth_sweep":
        return depth_sweep(args, torch, ppt, sg, dev)
    if args.workload == "comparators":
        return comparators(args, torch, ppt, sg, dev)
    if args.workload == "batched128":
        wl = sg.config3(res=args.res, spp=args.spp)
        desc = (f"batched views: {len(wl.views)} views (4 ring poses x 32 polarizer angles), {args.res}x{args.res}, "
                f"{args.spp} spp, depth {wl.max_depth}, 20.5k-triangle icosphere scene, render + PRB backward, "
                "HIP-graph replay")
    elif args.workload == "config2":
        wl = sg.config2()
        desc = ("config 2 at full size: one view, 256x256, 64 spp, depth 8, polarizer, 20.5k-triangle icosphere "
                "scene (GGX dielectric, conductor, textured Lambertian), render + PRB backward, HIP-graph replay")
    elif args.workload == "lightstage":
        wl = sg.lightstage()
        desc = (f"light stage: {len(wl.views)} views on a ring, {int(wl.views[0]['width'])}^2, "
                f"{int(wl.views[0]['spp'])} spp, depth {wl.max_depth}, 8 right-circular lights, analyzers 0/45/90 "
                "degrees and left-circular, normal/specular/roughness maps (7.7k triangles), render + PRB backward, "
                "HIP-graph replay")
    else:
        wl = sg.config5()
        res_l = [int(v["width"]) for v in wl.views]
        spp_l = [int(v["spp"]) for v in wl.views]
        desc = (f"uneven batch: {len(wl.views)} worlds (Perlin terrain 1e5..1e6 triangles + icospheres), "
                f"resolutions {res_l}, spp {spp_l}, depth {wl.max_depth}, 4 analyzers, render + PRB backward, "
                "HIP-graph replay")
    log(f"[bench] workload {wl.name}: {desc}")
    blob = wl.scene.to_blob()
    scene = ppt.Scene(blob)
    params = [torch.from_numpy(p).to(dev) for p in wl.scene.params()]
    chunk = args.chunk_paths
    tuned = None
    if chunk == 0:
        from paper_2607_13265_amd import autotune
        want0 = [n in wl.grad_slots for n in wl.scene.slot_names]
        chunk, tuned = autotune.tune(scene, blob, wl.views, wl.max_depth, params, want=want0, flags=wl.flags,
                                     force=args.retune, log=log)
        log(f"[bench] autotuned chunk {chunk}: {tuned}")
    plan = ppt.Plan(scene, wl.views, wl.max_depth, wl.flags, chunk_paths=chunk)
    info = plan.launch_info()
    rng = np.random.default_rng(wl.meta.get("delta_seed", 5005))
    d = torch.from_numpy(rng.standard_normal(plan.image_numel, dtype=np.float32)).to(dev)
    want = [n in wl.grad_slots for n in wl.scene.slot_names]
    out = torch.empty(plan.image_numel, dtype=torch.float32, device=dev)
    grads = [torch.empty_like(p) if w else None for p, w in zip(params, want)]
    ws_r, ws_b = plan.workspace(0), plan.workspace(1)

    def step():
        plan.render(params, wl.seed, out=out, ws=ws_r)
        plan.backward(params, wl.seed, d, grads=grads, ws=ws_b)

    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)  # (the autotuner's trial plans are gone)

    # eager warm-up, counters, and per-kernel timing with events on the launch stream
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    st_r, st_b = plan.stats(0), plan.stats(1)
    verts = st_r["vertices"]
    plan.set_stats(False)  # counters are not needed in the timed region
    log(f"[bench] vertices/step {verts}, paths {st_r['paths']}, grid {info}")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_r, t_b = [], []
    for _ in range(max(3, args.steps // 2)):
        ev[0].record()
        plan.render(params, wl.seed, out=out, ws=ws_r)
        ev[1].record()
        plan.backward(params, wl.seed, d, grads=grads, ws=ws_b)
        ev[2].record()
        torch.cuda.synchronize()
        t_r.append(ev[0].elapsed_time(ev[1]))
        t_b.append(ev[1].elapsed_time(ev[2]))
    ms_r, ms_b = float(np.median(t_r)), float(np.median(t_b))
    log(f"[bench] eager: render {ms_r:.2f} ms, backward {ms_b:.2f} ms")

    # batched step captured in a HIP graph
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = verts / (ms_step * 1e-3) / 1e6
    log(f"[bench] graph: {ms_step:.2f} ms/step, {value:.1f} Mpath-vertices/s (wall {wall:.2f} s)")

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpath-vertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc,
                   "views": len(wl.views), "resolution": one_or_list([int(v["width"]) for v in wl.views]),
                   "spp": one_or_list([int(v["spp"]) for v in wl.views]), "max_depth": wl.max_depth,
                   "vertices_per_step": verts, "paths_per_step": st_r["paths"],
                   "chunk_paths": info["chunk_paths"], "chunks": info["n_chunks"],
                   "autotune_ms": tuned},
    }

    peak_timed = torch.cuda.max_memory_allocated(dev)
    result["memory"] = {"render_workspace_gb": round(plan.workspace_bytes(0) / 1e9, 3),
                        "backward_workspace_gb": round(plan.workspace_bytes(1) / 1e9, 3),
                        "peak_allocated_gb": round(peak_timed / 1e9, 3)}

    # the same step with a memory-bounded chunk (the path records of 2^22 paths in flight)
    if args.bounded_chunk and args.bounded_chunk < info["chunk_paths"]:
        pb = ppt.Plan(scene, wl.views, wl.max_depth, wl.flags, chunk_paths=args.bounded_chunk)
        pb.set_stats(False)
        wb_r, wb_b = pb.workspace(0), pb.workspace(1)
        gb_ = [torch.empty_like(p) if w else None for p, w in zip(params, want)]
        for _ in range(2):
            pb.render(params, wl.seed, out=out, ws=wb_r)
            pb.backward(params, wl.seed, d, grads=gb_, ws=wb_b)
        torch.cuda.synchronize()
        nb = max(2, args.steps // 4)
        e0.record()
        for _ in range(nb):
            pb.render(params, wl.seed, out=out, ws=wb_r)
            pb.backward(params, wl.seed, d, grads=gb_, ws=wb_b)
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / nb
        gdiff = max(float((a - b).norm() / max(float(b.norm()), 1e-30)) for a, b in zip(gb_, grads) if a is not None)
        result["memory_bounded"] = {"chunk_paths": pb.launch_info()["chunk_paths"], "chunks": pb.launch_info()["n_chunks"],
                                    "value": round(verts / (ms_b * 1e-3) / 1e6, 2), "ms_per_step": round(ms_b, 3),
                                    "render_workspace_gb": round(pb.workspace_bytes(0) / 1e9, 3),
                                    "backward_workspace_gb": round(pb.workspace_bytes(1) / 1e9, 3),
                                    "grad_rel_diff_vs_timed": gdiff}
        log(f"[bench] memory-bounded chunk {args.bounded_chunk}: {ms_b:.2f} ms/step, "
            f"{result['memory_bounded']['value']} Mpath-vertices/s, backward workspace "
            f"{result['memory_bounded']['backward_workspace_gb']} GB, grad rel diff {gdiff:.2e}")
        del pb, wb_r, wb_b, gb_
        torch.cuda.empty_cache()

    # per-view launches on the same paths (view_id keeps the random streams identical); every view
    # keeps its own gradient tensors, summed afterwards and compared with the batched gradients
    if not args.no_per_view:
        plans = []
        for v in range(len(wl.views)):
            pv = ppt.Plan(scene, wl.views[v:v + 1], wl.max_depth, wl.flags, chunk_paths=chunk)
            plans.append(pv)
        outs = [torch.empty(p.image_numel, dtype=torch.float32, device=dev) for p in plans]
        gviews = [[torch.empty_like(p) if w else None for p, w in zip(params, want)] for _ in plans]
        offs = sg.view_offsets(wl.views)
        ds = [d[int(offs[v]):int(offs[v]) + plans[v].image_numel] for v in range(len(plans))]

        def step_pv():
            for v, pv in enumerate(plans):
                pv.render(params, wl.seed, out=outs[v], ws=ws_r)
                pv.backward(params, wl.seed, ds[v], grads=gviews[v], ws=ws_b)

        step_pv()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.per_view_steps):
            step_pv()
        e1.record()
        torch.cuda.synchronize()
        ms_pv = e0.elapsed_time(e1) / args.per_view_steps
        step()
        torch.cuda.synchronize()
        img_pv = torch.cat(outs)
        img_rel = float((img_pv - out).norm() / out.norm())
        grad_rel = {}
        for i, name in enumerate(wl.scene.slot_names):
            if grads[i] is None:
                continue
            gsum = torch.stack([gv[i].double() for gv in gviews]).sum(0)
            grad_rel[name] = float((gsum - grads[i].double()).norm() / max(float(grads[i].double().norm()), 1e-30))
        result["per_view"] = {"value": round(verts / (ms_pv * 1e-3) / 1e6, 2), "ms_per_step": round(ms_pv, 3),
                              "launches_per_step": 2 * len(plans), "image_rel_diff_vs_batched": img_rel,
                              "grad_rel_diff_vs_batched": grad_rel}
        result["speedup_batched_vs_per_view"] = round(ms_pv / ms_step, 3)
        log(f"[bench] per-view: {ms_pv:.2f} ms/step, image rel diff {img_rel:.2e}, summed gradients rel diff {grad_rel}")
        del plans, outs, gviews

    # per-kernel HIP-event timing on the launch stream (eager steps right after the timed region)
    plan.set_timing(True)
    fam_ms, fam_n = {}, {}
    for _ in range(max(1, args.timing_steps)):
        step()
        for op in (0, 1):
            for f, (ms, n) in plan.kernel_times(op).items():
                fam_ms[f] = fam_ms.get(f, 0.0) + ms
                fam_n[f] = fam_n.get(f, 0) + n
    plan.set_timing(False)
    reps = max(1, args.timing_steps)
    per_step = {f: fam_ms[f] / reps for f in fam_ms if fam_n[f]}
    launches = {f: fam_n[f] // reps for f in fam_ms if fam_n[f]}
    log("[bench] per-kernel ms/step: " + ", ".join(f"{f} {per_step[f]:.2f} ({launches[f]})" for f in per_step))

    # algorithmic work per step of every family, from the in-kernel counters
    st = {k: st_r[k] + st_b[k] for k in st_r}
    work = {
        # one traversal family: closest-hit rays and, in the same launches, the shadow rays
        "extend": ("alu", FLOP_NODE * (st["nodes"] + st["shadow_nodes"])
                   + FLOP_PRIM * (st["prim_tests"] + st["shadow_prim_tests"])),
        "shade": ("alu", FLOP_SHADE * st["vertices"]),
        "replay": ("alu", FLOP_REPLAY * st_b["vertices"]),
        "fold": ("hbm", BYTES_FOLD_VERTEX * st_b["vertices"] + BYTES_FOLD_PATH * st_b["paths"]),
    }
    fams = {}
    for f, (bound, amount) in work.items():
        if f not in per_step:
            continue
        avg_ms = per_step[f] / launches[f]
        per_launch = amount / launches[f]
        if bound == "alu":
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e12, PEAK_FP32_TFLOPS, "TFLOP/s"
        else:
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e9, PEAK_HBM_GBS, "GB/s"
        fams[f] = {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
                   "frac": round(ach / peak, 4), "avg_launch_ms": round(avg_ms, 4), "launches_per_step": launches[f],
                   "ms_per_step": round(per_step[f], 3), "work_per_launch": per_launch}
    dom = max(fams, key=lambda f: fams[f]["ms_per_step"])
    D = fams[dom]
    result["roofline"] = {"bound": D["bound"], "achieved": D["achieved"], "peak": D["peak"], "unit": D["unit"],
                          "frac": D["frac"], "traffic": stored_traffic(args.workload, KERNEL_SYMBOL[dom], info["chunk_paths"]),
                          "kernel": KERNEL_SYMBOL[dom], "avg_launch_ms": D["avg_launch_ms"],
                          "launches_per_step": D["launches_per_step"],
                          "algorithmic_per_launch": D["work_per_launch"],
                          "kernels": {KERNEL_SYMBOL[f]: v for f, v in fams.items()},
                          "counters": {"render": st_r, "backward": st_b}}

    # deep paths: the same step on the 85-sheet stack at depth 128 (a throughput point beside the
    # shallow headline, whose paths average under one vertex)
    if args.workload == "batched128" and not args.no_deep:
        result["deep_stack"] = deep_stack(torch, ppt, sg, dev)

    # CPU baseline and accuracy of the timed configuration: the FP64 oracle (render + cached-suffix
    # replay) on a bounded sample of the workload, whose image and gradients are also the reference
    # for the timed plan's output on the same paths
    if not args.no_cpu:
        result.update(cpu_leg(args, torch, ppt, sg, wl, plan, params, d, out, want))

    line = json.dumps(result)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def deep_stack(torch, ppt, sg, dev, depth=128, steps=3):
    """Render + cached-suffix-replay backward (gradient of the floor albedo) of the 1280x720, 1 spp
    scene behind 85 polarizer sheets at maximum depth 128, all paths in one chunk: throughput in path
    vertices per second, time per step and backward workspace."""
    wl = sg.polarizer_stack(max_depth=depth)
    scene = ppt.Scene(wl.scene.to_blob())
    params = [torch.from_numpy(p).to(dev) for p in wl.scene.params()]
    want = [n in wl.grad_slots for n in wl.scene.slot_names]
    plan = ppt.Plan(scene, wl.views, depth, chunk_paths=wl.n_paths())
    d = torch.from_numpy(np.random.default_rng(depth).standard_normal(plan.image_numel, dtype=np.float32)).to(dev)
    ws_r, ws_b = plan.workspace(0), plan.workspace(1)
    grads = [torch.empty_like(p) if w else None for p, w in zip(params, want)]
    plan.render(params, wl.seed, ws=ws_r)
    plan.backward(params, wl.seed, d, grads=grads, ws=ws_b)
    torch.cuda.synchronize()
    verts = plan.stats(0)["vertices"]
    plan.set_stats(False)

    def step():
        plan.render(params, wl.seed, ws=ws_r)
        plan.backward(params, wl.seed, d, grads=grads, ws=ws_b)

    # the step's launches (about 3 per bounce and pass) captured in a HIP graph, as the headline's
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    res = {"workload": "1280x720, 1 spp, 85 polarizer sheets, depth 128, floor-albedo gradient, cached suffix replay, "
                       "one chunk, HIP-graph replay", "vertices_per_step": verts, "paths_per_step": wl.n_paths(),
           "value": round(verts / (ms * 1e-3) / 1e6, 2), "unit": "Mpath-vertices/s", "ms_per_step": round(ms, 3),
           "backward_workspace_gb": round(plan.workspace_bytes(1) / 1e9, 3)}
    log(f"[bench] deep stack: {res}")
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_leg(args, torch, ppt, sg, wl, plan, params, d, out, want):
    """The oracle timed at all host threads of this GPU's share and at one thread, and the parity of
    the timed configuration: the timed plan's image and gradients on the sampled views (dL/dI zero
    elsewhere; paths whose discrete decisions differ masked on both sides) against the oracle's."""
    import oracle
    # threads: the CPU share of this GPU's job (OMP_NUM_THREADS where the launcher sets it), else
    # every CPU this process may run on
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    if args.workload == "batched128":
        sel = np.arange(max(1, min(args.cpu_views, len(wl.views))))
        sample_views = wl.views[sel]
        sample_desc = f"{len(sel)} of the {len(wl.views)} views, whole {args.res}x{args.res} images"
        crop = None
    else:
        sel = np.arange(len(wl.views))
        sample_views = sg.crop_views(wl.views, 0, 0, 64, 64)
        sample_views["crop_x0"] = (sample_views["width"] - 64) // 2
        sample_views["crop_y0"] = (sample_views["height"] - 64) // 2
        sample_desc = f"the central 64x64 crop of each of the {len(wl.views)} views"
        crop = sample_views
    osc = oracle.OracleScene.from_scene(wl.scene)
    p64 = [p.astype(np.float64) for p in wl.scene.params()]
    # the GPU's per-path index of every sampled path, and the sampled part of the image vector
    offs = sg.view_offsets(wl.views)
    path_off = np.concatenate([[0], np.cumsum(wl.views["crop_w"].astype(np.int64) * wl.views["crop_h"]
                                              * wl.views["spp"])])
    gidx, iidx = [], []
    for j, v in enumerate(sel):
        vw = wl.views[v]
        W, H, spp, A = int(vw["crop_w"]), int(vw["crop_h"]), int(vw["spp"]), sg.analyzer_count(int(vw["sensor"]))
        if crop is None:
            x0, y0, w, h = 0, 0, W, H
        else:
            x0, y0, w, h = int(crop[j]["crop_x0"]), int(crop[j]["crop_y0"]), 64, 64
        ys, xs = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
        pix = (ys * W + xs).ravel()
        gidx.append(path_off[v] + (pix[:, None] * spp + np.arange(spp)[None, :]).ravel())
        ent = (pix[:, None] * 12 + np.arange(12)[None, :]).ravel()
        iidx.append(np.concatenate([int(offs[v]) + a * W * H * 12 + ent for a in range(A)]))
    gidx, iidx = np.concatenate(gidx), np.concatenate(iidx)
    d_all = d.cpu().numpy()
    dd = d_all[iidx].astype(np.float64)
    grad_slots = [i for i, w in enumerate(want) if w]
    # all threads: render (with the per-path signatures) + cached-suffix replay
    t0 = time.perf_counter()
    r = osc.run(p64, sample_views, wl.max_depth, wl.seed, want_sig=True, nthreads=nthreads)
    tr = time.perf_counter() - t0
    r2 = osc.run(p64, sample_views, wl.max_depth, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=dd,
                 want_image=False, grad_slots=grad_slots, nthreads=nthreads)
    tc = time.perf_counter() - t0
    base = {"value": round(r["n_vertices"] / tc / 1e6, 4), "unit": "Mpath-vertices/s", "cores": nthreads,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
            "sample": f"{sample_desc} at full spp, depth {wl.max_depth} ({r['n_paths']} paths, {r['n_vertices']} "
                      f"vertices): FP64 render + cached-suffix replay, {tc:.1f} s on {nthreads} threads",
            "render_only": {"value": round(r["n_vertices"] / tr / 1e6, 4), "cores": nthreads,
                            "sample": f"the same paths, render alone, {tr:.1f} s"}}
    log(f"[bench] cpu oracle ({nthreads} threads): {base['value']} Mpath-vertices/s "
        f"(render alone {base['render_only']['value']})")
    # one thread on a smaller sample
    n1 = max(1, min(args.cpu_views_1t, len(sample_views)))
    v1 = sample_views[:n1]
    d1 = np.random.default_rng(1).standard_normal(sg.image_numel(v1))
    t0 = time.perf_counter()
    q = osc.run(p64, v1, wl.max_depth, wl.seed, nthreads=1)
    osc.run(p64, v1, wl.max_depth, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=d1, want_image=False,
            grad_slots=grad_slots, nthreads=1)
    t1 = time.perf_counter() - t0
    base["one_thread"] = {"value": round(q["n_vertices"] / t1 / 1e6, 4), "cores": 1,
                          "sample": f"{n1} of the sampled views ({q['n_paths']} paths, {q['n_vertices']} vertices), "
                                    f"{t1:.1f} s"}
    log(f"[bench] cpu oracle (1 thread): {base['one_thread']['value']} Mpath-vertices/s")
    # conventional AD (the oracle's stored tape: its own forward pass records every vertex, then the
    # reverse sweep) on that smaller sample, all threads
    t0 = time.perf_counter()
    qt = osc.run(p64, v1, wl.max_depth, wl.seed, mode=oracle.MODE_TAPE_AD, d_image=d1, want_image=False,
                 grad_slots=grad_slots, nthreads=nthreads)
    tt = time.perf_counter() - t0
    base["tape_ad"] = {"value": round(qt["n_vertices"] / tt / 1e6, 4), "cores": nthreads,
                       "sample": f"{n1} of the sampled views ({qt['n_vertices']} vertices): FP64 tape forward + "
                                 f"reverse sweep, {tt:.1f} s"}
    log(f"[bench] cpu oracle, tape AD ({nthreads} threads): {base['tape_ad']['value']} Mpath-vertices/s")
    # parity of the timed plan on the sampled paths
    sig_g = plan.signatures(params, wl.seed).cpu().numpy().view(np.uint64)[gidx]
    agree = sig_g == r["sig"]
    img_ref, grads_ref = r["image"], r2["grads"]
    if not agree.all():  # mask the divergent paths on both sides
        mk = agree.astype(np.uint8)
        img_ref = osc.run(p64, sample_views, wl.max_depth, wl.seed, mask=mk, nthreads=nthreads)["image"]
        grads_ref = osc.run(p64, sample_views, wl.max_depth, wl.seed, mode=oracle.MODE_CACHED_PRB, d_image=dd,
                            want_image=False, grad_slots=grad_slots, mask=mk, nthreads=nthreads)["grads"]
        mask_full = torch.ones(plan.num_paths, dtype=torch.uint8, device=params[0].device)
        mask_full[torch.from_numpy(gidx[~agree]).to(params[0].device)] = 0
        plan.set_path_mask(mask_full)
    plan.render(params, wl.seed, out=out)
    img_g = out.cpu().numpy()[iidx].astype(np.float64)
    d_s = torch.zeros_like(d)
    d_s[torch.from_numpy(iidx).to(d.device)] = d[torch.from_numpy(iidx).to(d.device)]
    g = plan.backward(params, wl.seed, d_s, want=want)
    plan.set_path_mask(None)
    torch.cuda.synchronize()

    def rel(a, b):
        nb = float(np.linalg.norm(b))
        return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))

    par = {"img_rel": rel(img_g, img_ref), "grad_rel": {}, "divergent_paths": int((~agree).sum()),
           "paths_compared": int(agree.size), "reference": "FP64 oracle, cached-suffix replay",
           "gates": {"img_rel": 1e-4, "grad_rel": 1e-3}}
    for i in grad_slots:
        par["grad_rel"][wl.scene.slot_names[i]] = rel(g[i].double().cpu().numpy(), grads_ref[i])
    par["pass"] = bool(par["img_rel"] <= 1e-4 and all(v <= 1e-3 for v in par["grad_rel"].values())
                       and par["divergent_paths"] <= 0.01 * agree.size)
    log(f"[bench] parity of the timed configuration: {par}")
    return {"cpu_baseline": base, "parity": par}


if __name__ == "__main__":
    main()
