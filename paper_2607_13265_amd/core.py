"""Scene / plan objects over the C ABI.  PyTorch provides device memory and streams only:
every step of rendering and differentiation runs in the HIP kernels of libppt.so."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import PlanOpts, PPTError, check, lib, ptr_table

FLAG_NO_NEE = 1

VIEW_DTYPE = np.dtype([
    ("world", "<i4"), ("width", "<i4"), ("height", "<i4"), ("spp", "<i4"),
    ("crop_x0", "<i4"), ("crop_y0", "<i4"), ("crop_w", "<i4"), ("crop_h", "<i4"),
    ("origin", "<f4", 3), ("target", "<f4", 3), ("up", "<f4", 3), ("fov_y_deg", "<f4"),
    ("sensor", "<i4"), ("theta_slot", "<i4"), ("theta_off", "<i4"), ("view_id", "<u4"),
])


# counters of ppt_read_stats and kernel families of ppt_plan_kernel_times, in ABI order
STAT_KEYS = ("vertices", "paths", "nodes", "prim_tests", "shadow_rays", "rays", "shadow_nodes",
             "shadow_prim_tests")
KERNEL_FAMILIES = ("camera", "extend", "shade", "shadow", "accum", "fold", "replay", "other", "compact")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Scene:
    """A parsed scene blob resident on the current device (BVH built on the host)."""

    def __init__(self, blob: bytes):
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().ppt_scene_create(buf, len(blob), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int32()
        check(lib().ppt_scene_slots(h, ctypes.byref(n), None, 0))
        numel = (ctypes.c_int64 * max(n.value, 1))()
        check(lib().ppt_scene_slots(h, None, numel, n.value))
        self.slot_numel = [int(numel[i]) for i in range(n.value)]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().ppt_scene_destroy(h)
            self._h = None


class Plan:
    """Views + max depth + flags; paths of all views are processed in chunks of chunk_paths.
    checkpoint_interval k > 0 selects the hybrid cached replay for the backward pass; with
    hybrid_rule (a (gamma, eps) pair) it recovers suffixes inside a block by Eq. 3's decision rule.
    pprb_sigma selects the noise-regularised P-PRB comparator for the backward pass (Sec. 4.2), tape
    the conventional-AD baseline (stored tape of every vertex's loop state, reverse sweep), prb the P-RB
    comparator (independent suffix estimates, Sec. 5.1)."""

    def __init__(self, scene: Scene, views, max_depth: int, flags: int = 0, chunk_paths: int = 0,
                 checkpoint_interval: int = 0, hybrid_rule=None, pprb_sigma=None, tape=False, prb=False):
        self.scene = scene
        self.views = np.ascontiguousarray(views, VIEW_DTYPE)
        self.max_depth = int(max_depth)
        self.flags = int(flags)
        rule = (0, 0.0, 0.0) if hybrid_rule is None else (1, float(hybrid_rule[0]), float(hybrid_rule[1]))
        adj = (2, 0.0) if tape else (3, 0.0) if prb else (0, 0.0) if pprb_sigma is None else (1, float(pprb_sigma))
        opts = PlanOpts(int(chunk_paths), int(checkpoint_interval), *rule, *adj)
        h = ctypes.c_void_p()
        check(lib().ppt_plan_create(scene.handle, self.views.ctypes.data_as(ctypes.c_void_p), len(self.views),
                                    self.max_depth, self.flags, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.image_numel = int(lib().ppt_plan_image_numel(h))
        self.num_paths = int(lib().ppt_plan_num_paths(h))
        self._ws = {}
        self._mask = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().ppt_plan_destroy(h)
            self._h = None

    def launch_info(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().ppt_plan_launch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"chunk_paths": a.value, "n_chunks": b.value, "stack_entries": c.value}

    def workspace_bytes(self, op: int) -> int:
        return int(lib().ppt_plan_workspace_bytes(self._h, op))

    def workspace(self, op: int, device=None):
        """A cached device workspace for op (0 render, 1 backward)."""
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        key = (op, str(dev))
        ws = self._ws.get(key)
        n = self.workspace_bytes(op)
        if ws is None or ws.numel() < n:
            ws = torch.empty(n + 256, dtype=torch.uint8, device=dev)
            self._ws[key] = ws
        return ws

    @staticmethod
    def _ws_args(ws):
        """(256-byte aligned device pointer, usable bytes) of a uint8 workspace tensor."""
        p = ws.data_ptr()
        pad = (-p) % 256
        return ctypes.c_void_p(p + pad), max(0, ws.numel() * ws.element_size() - pad)

    def set_stats(self, enabled: bool):
        """Enable/disable the in-kernel work counters (on by default)."""
        check(lib().ppt_plan_set_stats(self._h, 1 if enabled else 0))

    def set_timing(self, enabled: bool):
        """Enable/disable per-kernel HIP-event timing of the plan's calls (diagnostics; not under capture)."""
        check(lib().ppt_plan_set_timing(self._h, 1 if enabled else 0))

    def kernel_times(self, op: int):
        """Per kernel family of the most recent timed call of op (0 render, 1 backward):
        {family: (milliseconds, launches)}; waits for that call to finish."""
        ms = (ctypes.c_double * len(KERNEL_FAMILIES))()
        n = (ctypes.c_int32 * len(KERNEL_FAMILIES))()
        check(lib().ppt_plan_kernel_times(self._h, int(op), ms, n, len(KERNEL_FAMILIES)))
        return {f: (float(ms[i]), int(n[i])) for i, f in enumerate(KERNEL_FAMILIES)}

    def set_path_mask(self, mask):
        """Optional per-path mask (uint8 device tensor of num_paths entries) or None."""
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.is_cuda and mask.numel() == self.num_paths
            mask = mask.contiguous()
        self._mask = mask
        check(lib().ppt_plan_set_path_mask(self._h, None if mask is None else ctypes.c_void_p(mask.data_ptr())))

    def _params(self, params):
        if len(params) != len(self.scene.slot_numel):
            raise PPTError(f"expected {len(self.scene.slot_numel)} parameter tensors, got {len(params)}")
        out = []
        for p, n in zip(params, self.scene.slot_numel):
            if p.dtype != torch.float32 or not p.is_cuda or p.numel() != n or not p.is_contiguous():
                raise PPTError("parameters must be contiguous float32 device tensors of the slot sizes")
            out.append(p)
        return out

    def render(self, params, seed: int, out=None, ws=None, stream=None):
        params = self._params(params)
        if out is None:
            out = torch.empty(self.image_numel, dtype=torch.float32, device=params[0].device)
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != self.image_numel or not out.is_contiguous():
            raise PPTError("out must be a contiguous float32 device tensor of image_numel entries")
        ws = self.workspace(0, params[0].device) if ws is None else ws
        pt = ptr_table(params)
        wp, wn = self._ws_args(ws)
        check(lib().ppt_render(self._h, pt, len(params), int(seed) & (2**64 - 1), ctypes.c_void_p(out.data_ptr()),
                               wp, wn, _stream(stream)))
        return out

    def backward(self, params, seed: int, d_stokes, want=None, grads=None, ws=None, stream=None):
        params = self._params(params)
        d_stokes = d_stokes.contiguous()
        if d_stokes.dtype != torch.float32 or d_stokes.numel() != self.image_numel:
            raise PPTError("d_stokes must be float32 with image_numel entries")
        if grads is None:
            want = [True] * len(params) if want is None else list(want)
            grads = [torch.empty_like(p) if w else None for p, w in zip(params, want)]
        if len(grads) != len(params) or any(g is not None and (g.dtype != torch.float32 or not g.is_cuda or
                                                                g.numel() != p.numel() or not g.is_contiguous())
                                            for g, p in zip(grads, params)):
            raise PPTError("grads must match the parameter tensors (float32, contiguous, same sizes)")
        ws = self.workspace(1, params[0].device) if ws is None else ws
        pt, gt = ptr_table(params), ptr_table(grads)
        wp, wn = self._ws_args(ws)
        check(lib().ppt_backward(self._h, pt, len(params), int(seed) & (2**64 - 1),
                                 ctypes.c_void_p(d_stokes.data_ptr()), gt, wp, wn, _stream(stream)))
        return grads

    def backward_noalloc(self, params, seed: int, d_stokes, grads, stream=None):
        """ppt_backward_noalloc: the gradients of backward() computed in the library's fixed device
        scratch (no workspace); ``grads`` are caller-provided tensors (None entries skipped)."""
        params = self._params(params)
        if d_stokes.dtype != torch.float32 or d_stokes.numel() != self.image_numel or not d_stokes.is_contiguous():
            raise PPTError("d_stokes must be contiguous float32 with image_numel entries")
        if len(grads) != len(params) or any(g is not None and (g.dtype != torch.float32 or not g.is_cuda or
                                                                g.numel() != p.numel() or not g.is_contiguous())
                                            for g, p in zip(grads, params)):
            raise PPTError("grads must match the parameter tensors (float32, contiguous, same sizes)")
        check(lib().ppt_backward_noalloc(self._h, ptr_table(params), len(params), int(seed) & (2**64 - 1),
                                         ctypes.c_void_p(d_stokes.data_ptr()), ptr_table(grads), _stream(stream)))
        return grads

    def signatures(self, params, seed: int, ws=None, stream=None):
        params = self._params(params)
        sig = torch.empty(self.num_paths, dtype=torch.int64, device=params[0].device)
        ws = self.workspace(0, params[0].device) if ws is None else ws
        wp, wn = self._ws_args(ws)
        check(lib().ppt_signatures(self._h, ptr_table(params), len(params), int(seed) & (2**64 - 1),
                                   ctypes.c_void_p(sig.data_ptr()), wp, wn, _stream(stream)))
        return sig

    def hybrid_stats(self, stream=None):
        """Branch counts (scalar, invert, recompute) of the decision rule in the last backward call."""
        ws = self._ws[(1, str(torch.device("cuda", torch.cuda.current_device())))]
        out = (ctypes.c_int64 * 3)()
        check(lib().ppt_read_hybrid_stats(self._ws_args(ws)[0], out, _stream(stream)))
        return {"scalar": int(out[0]), "invert": int(out[1]), "recompute": int(out[2])}

    def stats(self, op: int, stream=None):
        ws = self._ws[(op, str(torch.device("cuda", torch.cuda.current_device())))]
        out = (ctypes.c_int64 * len(STAT_KEYS))()
        check(lib().ppt_read_stats(self._ws_args(ws)[0], out, _stream(stream)))
        return {k: int(out[i]) for i, k in enumerate(STAT_KEYS)}


def debug_rng(seed: int, ctr):
    """Philox4x32-10 of the GPU library on a (n, 4) uint32 counter tensor (stored as int32)."""
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    check(lib().ppt_debug_rng(int(seed) & (2**64 - 1), ctypes.c_void_p(ctr.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), ctr.shape[0], _stream()))
    return out
