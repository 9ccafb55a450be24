"""FP64 CPU oracle of differentiable polarized path tracing -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this package.
It wraps ``ppt_oracle.cpp`` (plain C++, double precision, OpenMP over pixel rows), which
shares no code with the GPU library; it never imports the product package.

Modes of :func:`OracleScene.run` (paper Sec. 3.2, 4.1, 4.3, 5.1):
  0 render            Monte Carlo Stokes image (Eq. 2 in Mueller-Stokes calculus)
  1 conventional AD   one stored tape per path with detached sampling ("Conv. AD")
  2 cached replay     per-vertex cache + backward fold + local-AD replay (Sec. 4.3)
  3 basic P-PRB       suffix recovered by Mueller inversion (Alg. 2), negative control; with
                      pprb_sigma > 0 the noise-regularised P-PRB comparator (Sec. 4.2)
  4 hybrid replay     checkpoints every k vertices and Eq. 3's rule in between (Sec. 4.4)
  5 P-RB              radiative backpropagation: each suffix an independent path estimate (Sec. 5.1)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ppt_oracle.cpp")
LIB_PATH = os.path.join(_HERE, "libppt_oracle.so")

MODE_RENDER, MODE_TAPE_AD, MODE_CACHED_PRB, MODE_BASIC_PRB, MODE_HYBRID, MODE_PRB_INDEPENDENT = 0, 1, 2, 3, 4, 5
FLAG_NO_NEE = 1
FLAG_GAUGE = 1 << 16

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP); returns the library path."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-std=c++17", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, c_int, c_u64, c_dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        L.ppto_scene_load.restype = vp
        L.ppto_scene_load.argtypes = [vp, ctypes.c_size_t, ctypes.c_char_p, c_int]
        L.ppto_scene_free.argtypes = [vp]
        L.ppto_scene_counts.argtypes = [vp, c_int, vp]
        L.ppto_run.restype = c_int
        L.ppto_run.argtypes = [vp, vp, vp, c_int, vp, c_int, c_int, ctypes.c_uint32, c_u64, c_int,
                               vp, vp, vp, vp, vp, vp, c_int, ctypes.c_char_p, c_int, c_int, vp, c_int, c_dbl, c_dbl,
                               c_dbl]
        L.ppto_philox.argtypes = [c_u64, vp, vp]
        L.ppto_philox_n.argtypes = [c_u64, vp, vp, ctypes.c_int64]
        L.ppto_fresnel.argtypes = [c_dbl, c_dbl, c_dbl, vp, vp]
        L.ppto_polarizer.argtypes = [c_dbl, vp]
        L.ppto_retarder.argtypes = [c_dbl, vp]
        L.ppto_rotator.argtypes = [vp, vp, vp, vp]
        L.ppto_canon_x.argtypes = [vp, vp]
        L.ppto_ggx_eval.argtypes = [vp, vp, vp, c_dbl, c_dbl, c_dbl, vp]
        L.ppto_ggx_D.restype = c_dbl
        L.ppto_ggx_D.argtypes = [c_dbl, c_dbl]
        L.ppto_smith_G1.restype = c_dbl
        L.ppto_smith_G1.argtypes = [c_dbl, c_dbl]
        L.ppto_sample_glossy.restype = c_int
        L.ppto_sample_glossy.argtypes = [vp, vp, c_dbl, c_dbl, c_dbl, vp, vp]
        L.ppto_trace.restype = c_int
        L.ppto_trace.argtypes = [vp, c_int, vp, vp, c_dbl, c_int, c_int, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ptr_array(arrs):
    """ctypes array of double* (None -> NULL); keeps the arrays referenced by the caller."""
    t = (ctypes.c_void_p * len(arrs))()
    for i, a in enumerate(arrs):
        t[i] = None if a is None else a.ctypes.data
    return t


class OracleScene:
    def __init__(self, blob: bytes, slot_numel):
        self._blob = blob
        self.slot_numel = [int(n) for n in slot_numel]
        err = ctypes.create_string_buffer(256)
        buf = ctypes.create_string_buffer(blob, len(blob))
        self.h = lib().ppto_scene_load(buf, len(blob), err, 256)
        if not self.h:
            raise ValueError("oracle scene load failed: " + err.value.decode())

    @classmethod
    def from_scene(cls, scene):
        return cls(scene.to_blob(), [v.size for v in scene.slot_values])

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ppto_scene_free(self.h)
            self.h = None

    def counts(self, world=0):
        out = np.zeros(4, np.int32)
        lib().ppto_scene_counts(self.h, world, _ptr(out))
        return out

    def run(self, params, views, max_depth, seed, flags=0, mode=MODE_RENDER, d_image=None, params_val=None,
            grad_slots=None, want_image=True, want_sig=False, mask=None, nthreads=0, pixel_grad_slot=None,
            ckpt=1, hybrid_gamma=0.0, hybrid_eps=float("inf"), pprb_sigma=0.0):
        """Run the oracle.  ``params`` (and ``params_val``) are per-slot arrays (converted to float64).

        Returns a dict with ``image`` (float64, [V][A][h][w][3][4] flattened per view),
        ``hybrid_branches`` (mode 4: how often Eq. 3's rule chose each branch; one recomputation
        covers the rest of its block),
        ``grads`` (list per slot, None where not requested), ``sig`` (uint64 per path),
        ``n_vertices`` and ``n_paths``; with ``pixel_grad_slot`` also ``pixel_grad``: that slot's
        gradient split by pixel (the gradient images of Sec. 5.1), shape (pixels, slot elements) with
        the pixels in (view, crop row, crop column) order.
        ``ckpt``: checkpoint interval k of the hybrid replay (``MODE_HYBRID``); ``hybrid_gamma`` and
        ``hybrid_eps``: the thresholds of its decision rule (Eq. 3): the scalar PRB update where the
        block throughput's depolarization index is below gamma, the inverse where |det| > eps
        beta_00^4, else recomputation (gamma = 0 and eps = inf: recomputation only).
        ``pprb_sigma``: mode 3's regularisation noise (Sec. 4.2), 0 for the plain inversion.
        """
        from scenegen import VIEW_DTYPE, image_numel  # input-layout helpers only

        views = np.ascontiguousarray(views, VIEW_DTYPE)
        pp = [np.ascontiguousarray(p, np.float64) for p in params]
        pv = pp if params_val is None else [np.ascontiguousarray(p, np.float64) for p in params_val]
        n_img = image_numel(views)
        n_paths = int(np.sum(views["crop_w"].astype(np.int64) * views["crop_h"] * views["spp"]))
        image = np.zeros(n_img, np.float64) if want_image else None
        grads = [None] * len(pp)
        if mode != MODE_RENDER:
            want = range(len(pp)) if grad_slots is None else grad_slots
            for s in want:
                grads[s] = np.zeros(self.slot_numel[s], np.float64)
            d_image = np.ascontiguousarray(d_image, np.float64)
            assert d_image.size == n_img
        sig = np.zeros(n_paths, np.uint64) if want_sig else None
        mk = None if mask is None else np.ascontiguousarray(mask, np.uint8)
        stats = np.zeros(5, np.int64)
        n_pix = int(np.sum(views["crop_w"].astype(np.int64) * views["crop_h"]))
        pg = np.zeros(n_pix * self.slot_numel[pixel_grad_slot]) if pixel_grad_slot is not None else None
        err = ctypes.create_string_buffer(256)
        ptp, ptv, pgr = _ptr_array(pp), _ptr_array(pv), _ptr_array(grads)
        rc = lib().ppto_run(self.h, ptp, ptv, len(pp), _ptr(views), len(views), int(max_depth), int(flags),
                            int(seed) & (2 ** 64 - 1), int(mode),
                            None if d_image is None else _ptr(d_image),
                            None if image is None else _ptr(image), pgr,
                            None if sig is None else _ptr(sig), None if mk is None else _ptr(mk),
                            _ptr(stats), int(nthreads), err, 256,
                            -1 if pixel_grad_slot is None else int(pixel_grad_slot), None if pg is None else _ptr(pg),
                            int(ckpt), float(hybrid_gamma), float(hybrid_eps), float(pprb_sigma))
        if rc != 0:
            raise ValueError("oracle run failed: " + err.value.decode())
        return {"image": image, "grads": grads, "sig": sig, "n_vertices": int(stats[0]), "n_paths": int(stats[1]),
                "hybrid_branches": {"scalar": int(stats[2]), "invert": int(stats[3]), "recompute": int(stats[4])},
                "pixel_grad": None if pg is None else pg.reshape(n_pix, -1)}


# ---- unit-level helpers for the pin tests
def philox(seed, ctr):
    c = np.asarray(ctr, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().ppto_philox(int(seed), _ptr(c), _ptr(o))
    return o


def philox_n(seed, ctr):
    c = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    o = np.zeros_like(c)
    lib().ppto_philox_n(int(seed), _ptr(c), _ptr(o), c.shape[0])
    return o


def fresnel(cos_i, m):
    m = complex(m)
    R = np.zeros(16); T = np.zeros(16)
    lib().ppto_fresnel(float(cos_i), m.real, m.imag, _ptr(R), _ptr(T))
    return R.reshape(4, 4), T.reshape(4, 4)


def polarizer(theta):
    M = np.zeros(16)
    lib().ppto_polarizer(float(theta), _ptr(M))
    return M.reshape(4, 4)


def retarder(delta):
    M = np.zeros(16)
    lib().ppto_retarder(float(delta), _ptr(M))
    return M.reshape(4, 4)


def rotator(k, x_from, x_to):
    M = np.zeros(16)
    a = [np.ascontiguousarray(v, np.float64) for v in (k, x_from, x_to)]
    lib().ppto_rotator(_ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(M))
    return M.reshape(4, 4)


def canon_x(k):
    k = np.ascontiguousarray(k, np.float64)
    x = np.zeros(3)
    lib().ppto_canon_x(_ptr(k), _ptr(x))
    return x


def ggx_eval(ns, wi, wo, alpha, m):
    m = complex(m)
    f = np.zeros(16)
    a = [np.ascontiguousarray(v, np.float64) for v in (ns, wi, wo)]
    lib().ppto_ggx_eval(_ptr(a[0]), _ptr(a[1]), _ptr(a[2]), float(alpha), m.real, m.imag, _ptr(f))
    return f.reshape(4, 4)


def ggx_D(cos_h, alpha):
    return float(lib().ppto_ggx_D(float(cos_h), float(alpha)))


def smith_G1(cos_w, alpha):
    return float(lib().ppto_smith_G1(float(cos_w), float(alpha)))


LOBE_GLOSSY, LOBE_INVALID = 4, 6


def sample_glossy(ns, wo, alpha, u1, u2):
    """One GGX half-vector sample: (lobe, wi, pdf); lobe is LOBE_INVALID for a rejected sample."""
    a = [np.ascontiguousarray(v, np.float64) for v in (ns, wo)]
    wi = np.zeros(3)
    pdf = np.zeros(1)
    lobe = lib().ppto_sample_glossy(_ptr(a[0]), _ptr(a[1]), float(alpha), float(u1), float(u2), _ptr(wi), _ptr(pdf))
    return int(lobe), wi, float(pdf[0])


def trace(scene: OracleScene, o, d, tmax=1e30, any_hit=False, brute=False, world=0):
    o = np.ascontiguousarray(o, np.float64); d = np.ascontiguousarray(d, np.float64)
    t = np.zeros(1)
    prim = lib().ppto_trace(scene.h, world, _ptr(o), _ptr(d), float(tmax), int(any_hit), int(brute), _ptr(t))
    return prim, float(t[0])
