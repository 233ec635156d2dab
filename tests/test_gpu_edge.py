"""GPU edge cases of the solver entry points: a zero right-hand side, the
iteration cap, non-finite input in a single solve, argument errors through the
C ABI, removing a running request from a batch, and the largest degree."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-edge] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_rhs_gives_zero_solution(torch_cuda, precision):
    from paper_1804_02539_amd import igamg
    prec = igamg.MIXED if precision == "mixed" else igamg.FP64
    S = igamg.Solver(W.square_4x4_bezier(levels=3), igamg.default_options(precision=prec))
    u, info = S.solve(np.zeros(S.N))
    assert info.converged and info.iterations == 0 and info.rel_residual == 0.0
    assert float(u.abs().max()) == 0.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_iteration_cap_reports_enoconv(torch_cuda, precision):
    from paper_1804_02539_amd import igamg
    prec = igamg.MIXED if precision == "mixed" else igamg.FP64
    S = igamg.Solver(W.square_4x4_bezier(levels=3), igamg.default_options(precision=prec, maxit=3))
    u, info = S.solve(W.random_rhs(S.N, 1), raise_on_error=False)
    _say(f"{precision}: code {S.last_code}, {info.iterations} it, residual {info.rel_residual:.2e}")
    assert S.last_code == igamg.ENOCONV
    assert not info.converged and info.iterations <= 3 + 1 and 0 < info.rel_residual < 1
    # the handle stays usable
    S2 = igamg.Solver(W.square_4x4_bezier(levels=3), igamg.default_options(precision=prec))
    _, ok = S2.solve(W.random_rhs(S2.N, 1))
    assert ok.converged


def test_nonfinite_rhs_reports_enan(torch_cuda):
    from paper_1804_02539_amd import igamg
    S = igamg.Solver(W.unit_square_2x2())
    f = W.random_rhs(S.N, 2)
    f[3] = np.inf
    _, info = S.solve(f, raise_on_error=False)
    assert S.last_code == igamg.ENAN and not info.converged
    # a finite solve on the same handle afterwards is fine
    _, info = S.solve(W.random_rhs(S.N, 2))
    assert info.converged


def test_argument_errors_through_the_abi(torch_cuda):
    import torch
    from paper_1804_02539_amd import igamg
    S = igamg.Solver(W.unit_square_2x2())
    lib = igamg.lib()
    f = torch.zeros(S.N, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(S.N, dtype=torch.float64, device="cuda:0")
    info = igamg.SolveInfo()
    assert lib.igamg_solve(S.h, None, ctypes.c_void_p(f.data_ptr()), 1e-8, ctypes.byref(info), None) == igamg.EINVAL
    assert lib.igamg_solve(S.h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(f.data_ptr()), 1e-8,
                           ctypes.byref(info), None) == igamg.EINVAL          # rhs and u alias
    assert lib.igamg_solve(S.h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()), -1.0,
                           ctypes.byref(info), None) == igamg.EINVAL          # tol must be positive
    assert lib.igamg_operator(S.h, 99, 1, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                              None) == igamg.EINVAL                           # unknown operator
    assert lib.igamg_operator(S.h, igamg.OP_APPLY, 7, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                              None) == igamg.EINVAL                           # level out of range
    assert lib.igamg_vcycle(None, ctypes.c_void_p(8), ctypes.c_void_p(16), None) == igamg.EINVAL
    with pytest.raises(ValueError):
        S.solve(np.zeros(S.N + 1))
    assert igamg.lib().igamg_last_error()


def test_batch_remove_running_request(torch_cuda):
    from paper_1804_02539_amd import igamg
    probs = [W.square_4x4_bezier(levels=3), W.cube_2x2x2_trilinear(levels=3)]
    S = [igamg.Solver(p) for p in probs]
    f = [W.random_rhs(s.N, 4) for s in S]
    alone = [s.solve(x) for s, x in zip(S, f)]
    B = igamg.Batch()
    a = B.add(S[0], f[0])
    b = B.add(S[1], f[1])
    for _ in range(3):
        B.step()
    B.remove(a)                       # abandoned mid-solve
    a2 = B.add(S[0], f[0])            # and restarted from scratch
    for _ in range(500):
        if B.step() == 0:
            break
    for slot, (u1, i1) in ((a2, alone[0]), (b, alone[1])):
        done, info, code = B.poll(slot)
        assert done and code == igamg.OK and info.iterations == i1.iterations
        assert torch_cuda.equal(B.result(slot), u1)


def test_largest_degree_matches_oracle(torch_cuda):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    prob = W.box_grid(2, [2, 1], 8, 1, 3, gdeg=1, dirichlet_sides=[0, 2])
    H = Hierarchy(prob)
    S = igamg.Solver(prob)
    r = np.random.default_rng(8).standard_normal(S.N)
    y = S.operator(igamg.OP_APPLY, -1, r).cpu().numpy()
    assert np.abs(y - H.finest.apply(r)).max() < 1e-12 * np.abs(y).max()
    z = S.vcycle(r).cpu().numpy()
    assert np.abs(z - H.vcycle(r)).max() < 1e-10 * np.abs(z).max()
    f = W.random_rhs(S.N, 8)
    u, info = S.solve(f)
    res = np.linalg.norm(f - H.finest.apply(u.cpu().numpy())) / np.linalg.norm(f)
    _say(f"p=8: {info.iterations} it, residual {res:.2e}")
    assert info.converged and res <= 1.0001e-8


def test_singular_coarse_matrix_on_the_device_reports_enotspd(torch_cuda):
    # no Dirichlet side: the coarse matrix is singular; the device
    # factorization (forced here) reports it
    from paper_1804_02539_amd import igamg
    from paper_1804_02539_amd import workloads as W
    bad = W.box_grid(2, [2, 1], 2, 1, 2, gdeg=1, dirichlet_sides=[])
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(bad, igamg.default_options(coarse_factor=2))
    assert e.value.code == igamg.ENOTSPD
    _say(f"singular coarse matrix on the device: {e.value}")
