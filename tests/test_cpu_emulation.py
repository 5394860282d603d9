"""The library's kernels and host code run on the CPU through a small HIP
emulation (tests/cpuemu: host threads for the threads of a block, host memory
for device memory) built with AddressSanitizer.  Every kernel launch of
binding, leaf and level operators, V-cycle and CG is checked for
out-of-bounds access and its results against the oracle, without a GPU.

The emulated cases run in parallel subprocesses (libasan preloaded, since
the Python interpreter itself is not instrumented)."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "cpuemu"))

# (case, precision of the multigrid levels)
EMU_CASES = [("fichera-q1", 64), ("cube-q2", 64), ("lshape-q1", 32), ("fichera-q2", 32), ("fichera-q3", 64),
             ("fichera-q4", 32), ("lshape-q4", 32),
             # degenerate: no free DoF, one level only, one family at degree 3
             ("cube-q1-g0", 64), ("fichera-q2-g0", 64), ("cube-q3-g1", 32)]


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def emu_results():
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("AddressSanitizer runtime not available")
    import build_emu
    build_emu.build()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    procs = {}
    for case, prec in EMU_CASES + [("serve", 64)]:
        procs[(case, prec)] = subprocess.Popen(
            [sys.executable, os.path.join(HERE, "cpuemu", "run_emu.py"), case, str(prec)],
            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
    out = {}
    for key, p in procs.items():
        try:
            so, se = p.communicate(timeout=600)
        except subprocess.TimeoutExpired:
            p.kill()
            so, se = p.communicate()
        out[key] = (p.returncode, so, se)
    return out


def test_emulated_serving_batched_matches_solo(emu_results):
    """The serving loop (scheduler and worker threads, batched V-cycles) in
    the emulation: two requests, three CG iterations each, match their solo
    solves (same status and iteration count; rounding-level differences only,
    the emulated LDS additions having no fixed order), and batched V-cycles
    did run."""
    rc, so, se = emu_results[("serve", 64)]
    assert "AddressSanitizer" not in se, se[-6000:]
    assert rc == 0, se[-6000:]
    r = json.loads(so.strip().splitlines()[-1])
    assert r["completed"] == 2 and r["same_its"]
    assert r["rel"] <= 1e-12
    assert r["batched_iterations"] == 6


@pytest.mark.parametrize("case,prec", EMU_CASES)
def test_emulated_kernels_match_oracle(emu_results, case, prec):
    rc, so, se = emu_results[(case, prec)]
    assert "AddressSanitizer" not in se, se[-6000:]
    assert rc == 0, se[-6000:]
    r = json.loads(so.strip().splitlines()[-1])
    assert r["lam_rel"] <= 1e-11
    assert r["leaf_rel"] <= 1e-13 and r["rhs_rel"] <= 1e-13
    if prec == 64:
        assert r["level_rel"] <= 1e-13 and r["edge_rel"] <= 1e-13 and r["vcycle_rel"] <= 1e-11
    else:
        # FP32 level operators and V-cycle: single-precision rounding
        assert r["level_rel"] <= 2e-6 and r["edge_rel"] <= 2e-6 and r["vcycle_rel"] <= 1e-5
    assert r["noalloc_equal"]
    assert r["batch_equal"]
    # error estimator (Sec. 4.3) entry by entry against the largest entry,
    # and the marking of its 14.2 % largest values
    assert r["est_rel"] <= 1e-12 and r["mark_equal"]
    assert r["status"] == 0 and r["its"] == r["its_oracle"]
    assert r["solve_rel"] <= 1e-10
