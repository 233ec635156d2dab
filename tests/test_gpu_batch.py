"""GPU tests of the solve driver: HIP-graph replay, batched lockstep solves and
continuous batching.  Every request's result must be the same alone and in
the mix (the kernels are deterministic, so the comparison is exact)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-batch] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _problems():
    # mixed dimensions, degrees, patch counts and sizes
    return [
        ("square2x2_p2", W.unit_square_2x2(), "sine"),
        ("square4x4_p4_l4", W.square_4x4_bezier(levels=4), "random"),
        ("cube2x2x2_p3_l4", W.cube_2x2x2_trilinear(levels=4), "sine"),
        ("fichera7_p3_l3", W.fichera(3, 3), "random"),
        ("box3x1_p5_l3", W.box_grid(2, [3, 1], 5, 2, 3, gdeg=1, dirichlet_sides=[0]), "random"),
    ]


def _rhs(S, prob, kind, seed):
    if kind == "sine":
        return S.load_vector(*prob.meta["source"][1:])
    return W.random_rhs(S.N, seed)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_direct_launches(torch_cuda, precision):
    from paper_1804_02539_amd import igamg
    prec = igamg.MIXED if precision == "mixed" else igamg.FP64
    for name, prob, kind in _problems()[:3]:
        _say(f"graphs vs direct {name} {precision}")
        Sg = igamg.Solver(prob, igamg.default_options(precision=prec, graphs=1))
        Sd = igamg.Solver(prob, igamg.default_options(precision=prec, graphs=0))
        f = _rhs(Sg, prob, kind, 3)
        ug, ig = Sg.solve(f)
        ud, idd = Sd.solve(f)
        assert ig.iterations == idd.iterations and ig.outer_iterations == idd.outer_iterations
        assert torch_cuda.equal(ug, ud)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_individual(torch_cuda, precision):
    from paper_1804_02539_amd import igamg
    prec = igamg.MIXED if precision == "mixed" else igamg.FP64
    probs = _problems()
    solvers = [igamg.Solver(p, igamg.default_options(precision=prec)) for _, p, _ in probs]
    rhss = [_rhs(S, p, k, 10 + i) for i, (S, (_, p, k)) in enumerate(zip(solvers, probs))]
    alone = [S.solve(f) for S, f in zip(solvers, rhss)]
    _say(f"batch of {len(solvers)} ({precision})")
    us, infos, codes, code = igamg.solve_batch(solvers, rhss)
    assert code == igamg.OK and all(c == igamg.OK for c in codes)
    for (u1, i1), u2, i2, (name, _, _) in zip(alone, us, infos, probs):
        _say(f"  {name}: alone {i1.iterations} it, batched {i2.iterations} it")
        assert i1.iterations == i2.iterations
        assert torch_cuda.equal(u1, u2)


def test_continuous_batching_join_and_leave(torch_cuda):
    """Requests join a running batch at different steps and leave when done;
    each result equals the request solved alone."""
    from paper_1804_02539_amd import igamg
    probs = _problems()
    opts = [igamg.default_options(), igamg.default_options(precision=igamg.MIXED)]
    solvers = [igamg.Solver(p, opts[i % 2]) for i, (_, p, _) in enumerate(probs)]
    rhss = [_rhs(S, p, k, 20 + i) for i, (S, (_, p, k)) in enumerate(zip(solvers, probs))]
    alone = [S.solve(f) for S, f in zip(solvers, rhss)]
    B = igamg.Batch()
    pending = list(range(len(solvers)))
    slots = {}
    results = {}
    step = 0
    while pending or slots:
        # admit one new request every second step
        if pending and step % 2 == 0:
            i = pending.pop(0)
            slots[i] = B.add(solvers[i], rhss[i])
        B.step()
        step += 1
        for i, sl in list(slots.items()):
            done, info, code = B.poll(sl)
            if done:
                assert code == igamg.OK
                results[i] = (B.result(sl).clone(), info)
                B.remove(sl)
                del slots[i]
        assert step < 2000
    _say(f"continuous batching finished in {step} steps")
    for i, (u1, i1) in enumerate(alone):
        u2, i2 = results[i]
        assert i1.iterations == i2.iterations
        assert torch_cuda.equal(u1, u2)


def test_batch_reports_nan_request_alone(torch_cuda):
    from paper_1804_02539_amd import igamg
    probs = _problems()[:3]
    solvers = [igamg.Solver(p) for _, p, _ in probs]
    rhss = [_rhs(S, p, k, 30 + i) for i, (S, (_, p, k)) in enumerate(zip(solvers, probs))]
    bad = np.array(rhss[1], dtype=np.float64)
    bad[5] = np.nan
    rhss[1] = bad
    us, infos, codes, code = igamg.solve_batch(solvers, rhss)
    assert codes[1] == igamg.ENAN and code == igamg.ENAN
    assert codes[0] == igamg.OK and codes[2] == igamg.OK
    assert infos[0].converged and infos[2].converged and not infos[1].converged
