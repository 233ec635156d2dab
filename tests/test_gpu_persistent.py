"""The persistent coarse cycle (options.persistent): the levels below the
finest with at most 65536 local rows run as one launch over a work list of
the cycle's phases.  Each work item runs the same body as the separate
launch, so with the same smoother variant (vector FMAs, 8-column chunks:
autotune off) the results must equal the per-kernel launches bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-persistent] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


CASES = {
    "square4x4_p4_l6": lambda: W.square_4x4_bezier(),
    "square2x2_p2": lambda: W.unit_square_2x2(),
    "cube2x2x2_p3_l5": lambda: W.cube_2x2x2_trilinear(levels=5),
    "fichera7_p2_l4": lambda: W.fichera(2, 4),
    "graded_cube2x2x2_p2_l3": lambda: W.graded_cube_2x2x2(),
    "single_patch_p5_l4": lambda: W.box_grid(2, [1, 1], 5, 2, 4, gdeg=1),
}


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_persistent_cycle_equals_launches(torch_cuda, name, precision):
    from paper_1804_02539_amd import igamg
    prob = CASES[name]()
    base = dict(precision=precision, autotune=0)
    S0 = igamg.Solver(prob, igamg.default_options(**base))
    S1 = igamg.Solver(prob, igamg.default_options(persistent=1, **base))
    r = np.random.default_rng(4).standard_normal(S0.N)
    op = igamg.OP_CYCLE_FP32 if precision else None
    if op is None:
        z0, z1 = S0.vcycle(r), S1.vcycle(r)
    else:
        z0, z1 = S0.operator(op, -1, r), S1.operator(op, -1, r)
    same = bool(torch_cuda.equal(z0, z1))
    diff = float((z0 - z1).abs().max() / z0.abs().max())
    _say(f"{name} precision={precision}: persistent cycle {'equals' if same else 'differs from'} the launches "
         f"(max rel diff {diff:.1e})")
    assert same
    # repeated cycles reuse the counters (reset by a kernel before each launch)
    z2 = S1.vcycle(r) if op is None else S1.operator(op, -1, r)
    assert torch_cuda.equal(z1, z2)
    f = W.random_rhs(S0.N, 6)
    u0, i0 = S0.solve(f)
    u1, i1 = S1.solve(f)
    _say(f"  solves: {i0.iterations} / {i1.iterations} iterations")
    assert i0.iterations == i1.iterations and torch_cuda.equal(u0, u1)


def test_persistent_batch_equals_alone(torch_cuda):
    from paper_1804_02539_amd import igamg
    probs = [CASES["square4x4_p4_l6"](), CASES["cube2x2x2_p3_l5"](), CASES["square2x2_p2"]()]
    solvers = [igamg.Solver(p, igamg.default_options(persistent=1, precision=igamg.MIXED)) for p in probs]
    rhs = [W.random_rhs(S.N, 8 + i) for i, S in enumerate(solvers)]
    alone = [S.solve(f)[0] for S, f in zip(solvers, rhs)]
    us, infos, codes, code = igamg.solve_batch(solvers, rhs)
    assert code == igamg.OK and all(c == igamg.OK for c in codes)
    for a, b in zip(alone, us):
        assert torch_cuda.equal(a, b)
    _say(f"batch of {len(solvers)} mixed solves with persistent cycles equals the solves alone")
