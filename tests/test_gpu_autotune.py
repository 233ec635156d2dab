"""GPU tests of the smoother autotuner: valid choices on every level, the same
choices for every handle of a problem in a process, FP64 results identical
with and without tuning (the vector variants differ only in how columns are
split between workgroups, not in arithmetic), and the JSON cache file."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(msg):
    print(f"[gpu-tune] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("case", ["square4x4_p4_l4", "cube2x2x2_p3_l4"])
def test_tuned_variants_are_valid_and_shared(torch_cuda, case):
    from paper_1804_02539_amd import igamg
    prob = W.square_4x4_bezier(levels=4) if case.startswith("square") else W.cube_2x2x2_trilinear(levels=4)
    opts = igamg.default_options(precision=igamg.MIXED)
    S1 = igamg.Solver(prob, opts)
    S2 = igamg.Solver(prob, opts)
    for l in range(1, prob.levels):
        v64, v32 = S1.tuning(l, False), S1.tuning(l, True)
        _say(f"{case} level {l}: fp64 {igamg.FD_NAMES[v64]}, fp32 {igamg.FD_NAMES[v32]}")
        assert v64 in (igamg.FD_VEC8, igamg.FD_VEC4)
        assert v32 in (igamg.FD_VEC8, igamg.FD_VEC4, igamg.FD_MFMA, igamg.FD_FUSED)
        if v32 == igamg.FD_FUSED:            # only on levels of 2D tensors
            assert case.startswith("square")
        assert (v64, v32) == (S2.tuning(l, False), S2.tuning(l, True))
    f = W.random_rhs(S1.N, 3)
    u1, i1 = S1.solve(f)
    u2, i2 = S2.solve(f)
    assert i1.iterations == i2.iterations and torch_cuda.equal(u1, u2)


def test_fp64_results_do_not_depend_on_tuning(torch_cuda):
    from paper_1804_02539_amd import igamg
    prob = W.cube_2x2x2_trilinear(levels=4)
    St = igamg.Solver(prob, igamg.default_options(autotune=1))
    S0 = igamg.Solver(prob, igamg.default_options(autotune=0))
    assert all(S0.tuning(l) == igamg.FD_VEC8 for l in range(1, prob.levels))
    r = np.random.default_rng(2).standard_normal(St.N)
    assert torch_cuda.equal(St.vcycle(r), S0.vcycle(r))


def test_tuning_cache_file(torch_cuda, tmp_path):
    path = tmp_path / "tune.json"
    code = ("import sys; sys.path.insert(0, %r); from paper_1804_02539_amd import igamg, workloads as W; "
            "S = igamg.Solver(W.unit_square_2x2(), igamg.default_options(precision=igamg.MIXED)); "
            "print(S.tuning(-1, True))" % ROOT)
    env = dict(os.environ, IGAMG_TUNE_CACHE=str(path))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    cache = json.loads(path.read_text())
    keys = [k for k in cache if "/f32/" in k]
    assert keys and all(v in (0, 1, 2, 3) for v in cache.values())
    # a second process reads the choice back instead of timing again
    out2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert out2.returncode == 0 and out2.stdout.strip() == out.stdout.strip()
