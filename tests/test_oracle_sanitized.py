"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

A copy of the oracle is built with g++ -fsanitize=address,undefined (no recovery) and loaded in a
child Python process with the sanitizer runtime preloaded; it runs small scenes through every mode
(render with signatures, conventional tape AD, cached suffix replay, P-PRB, hybrid replay with the
decision rule, P-RB), the light-stage features and the deep polarizer stack.  Pass: the child ends
without a sanitizer report and its outputs equal the regular build's (the same FP64 arithmetic).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the cases, as code both processes run: name -> (workload expression, mode, keyword arguments)
CASES = r'''
import numpy as np
import oracle
import scenegen as sg


def _c1():
    wl = sg.config1()
    wl.views["spp"] = 2
    return wl


def _ls():
    wl = sg.lightstage()
    wl.views = sg.crop_views(wl.views[:2], 120, 120, 6, 5)
    wl.views["spp"] = 2
    return wl


def _stack():
    return sg.polarizer_stack(n_sheets=4, width=8, height=6, spp=2, max_depth=10)


CASES = {
    "c1_render": (_c1, oracle.MODE_RENDER, dict(want_sig=True)),
    "c1_tape": (_c1, oracle.MODE_TAPE_AD, {}),
    "c1_cached": (_c1, oracle.MODE_CACHED_PRB, {}),
    "c1_pprb": (_c1, oracle.MODE_BASIC_PRB, dict(pprb_sigma=0.3)),
    "c1_hybrid_rule": (_c1, oracle.MODE_HYBRID, dict(ckpt=2, hybrid_gamma=0.5, hybrid_eps=1e-3)),
    "c1_prb": (_c1, oracle.MODE_PRB_INDEPENDENT, {}),
    "lightstage_cached": (_ls, oracle.MODE_CACHED_PRB, {}),
    "stack_hybrid_rule": (_stack, oracle.MODE_HYBRID, dict(ckpt=3, hybrid_gamma=0.5, hybrid_eps=1e-3)),
}


def run_case(name):
    make, mode, kw = CASES[name]
    wl = make()
    osc = oracle.OracleScene.from_scene(wl.scene)
    d = None if mode == oracle.MODE_RENDER else np.random.default_rng(7).normal(size=sg.image_numel(wl.views))
    r = osc.run(wl.scene.params(), wl.views, wl.max_depth, wl.seed, flags=wl.flags, mode=mode, d_image=d,
                nthreads=2, **kw)
    out = {"image": [] if r["image"] is None else r["image"].tolist(),
           "grads": [[] if g is None else g.tolist() for g in r["grads"]],
           "sig": [] if r["sig"] is None else [int(x) for x in r["sig"]],
           "n_vertices": r["n_vertices"], "branches": r["hybrid_branches"]}
    return out
'''

CHILD = r'''
import json, sys
sys.path.insert(0, sys.argv[1])
import oracle
oracle.LIB_PATH = sys.argv[2]
ns = {}
exec(sys.argv[3], ns)
res = {name: ns["run_case"](name) for name in ns["CASES"]}
print("RESULT " + json.dumps(res))
'''


def _runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.timeout(600)
def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None or _runtime("libubsan.so") is None:
        pytest.skip("g++ sanitizer runtimes not installed")
    so = str(tmp_path / "libppt_oracle_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fopenmp", "-std=c++17", "-shared", "-fPIC",
                           "-o", so, oracle.SRC])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    p = subprocess.run([sys.executable, "-c", CHILD, ROOT, so, CASES], capture_output=True, text=True, env=env,
                       timeout=540)
    tail = (p.stdout[-2000:] if p.stdout else "") + (p.stderr[-4000:] if p.stderr else "")
    assert p.returncode == 0, "sanitized oracle failed:\n" + tail
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error:" not in p.stderr, tail
    line = [ln for ln in p.stdout.splitlines() if ln.startswith("RESULT ")]
    assert line, tail
    got = json.loads(line[-1][len("RESULT "):])

    # the regular build on the same cases
    ns = {}
    exec(CASES, ns)
    for name in ns["CASES"]:
        ref = ns["run_case"](name)
        g = got[name]
        assert g["n_vertices"] == ref["n_vertices"] > 0, name
        assert g["sig"] == ref["sig"], name
        assert g["branches"] == ref["branches"], name
        a, b = np.asarray(g["image"]), np.asarray(ref["image"])
        assert a.shape == b.shape and np.allclose(a, b, rtol=1e-12, atol=1e-14 * (np.abs(b).max() if b.size else 1)), name
        for ga, gb in zip(g["grads"], ref["grads"]):
            ga, gb = np.asarray(ga), np.asarray(gb)
            assert ga.shape == gb.shape, name
            if gb.size:
                assert np.allclose(ga, gb, rtol=1e-10, atol=1e-12 * np.abs(gb).max()), name
