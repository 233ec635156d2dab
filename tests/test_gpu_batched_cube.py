"""GPU tests of the 4x4x4-patch p=5 workload (uneven slab element counts,
N = 2.87M at full size) and of the device factorization of the coarse
matrix it needs (30,056 coarse unknowns).

* small cases with the coarse matrix forced onto the device, against the oracle;
* the down-scaled replica (element counts / 4, same topology, degree,
  geometry and coarsest level) against the oracle: apply, coarse solve, cycle,
  and both solvers' residuals by the oracle's operator;
* the full-size problem: the finest apply on two whole patches against the
  oracle's patch operator, FP64 and mixed solves to 1e-8, and the two
  solutions against each other.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-cube64] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("case", ["square", "cube"])
def test_device_coarse_factorization_matches_oracle(torch_cuda, case):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    prob = W.square_4x4_bezier(levels=3) if case == "square" else W.cube_2x2x2_trilinear(levels=3)
    H = Hierarchy(prob)
    S = igamg.Solver(prob, igamg.default_options(coarse_factor=2))
    x = np.random.default_rng(3).standard_normal(H.levels[0].N)
    _say(f"device coarse factorization {case}, N0 = {H.levels[0].N}")
    assert rel(S.operator(igamg.OP_COARSE, 0, x).cpu().numpy(), H.coarse_solve(x)) < 1e-11
    r = np.random.default_rng(4).standard_normal(H.finest.N)
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10


def test_replica_matches_oracle(torch_cuda):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    prob = W.batched_patch_cube(divide=4)
    _say("replica: oracle hierarchy (64 patches, p=5, N0 = 30,056)")
    H = Hierarchy(prob)
    S = igamg.Solver(prob)
    assert S.N == H.finest.N
    N0 = H.levels[0].N
    _say(f"  N = {S.N}, N0 = {N0}")
    r = np.random.default_rng(5).standard_normal(S.N)
    assert rel(S.operator(igamg.OP_APPLY, -1, r).cpu().numpy(), H.finest.apply(r)) < 1e-12
    x0 = np.random.default_rng(6).standard_normal(N0)
    assert rel(S.operator(igamg.OP_COARSE, 0, x0).cpu().numpy(), H.coarse_solve(x0)) < 1e-10
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10
    _say("  apply, coarse solve and cycle match")
    f = W.random_rhs(S.N, 4)
    nf = np.linalg.norm(f)
    u64, i64 = S.solve(f)
    res64 = np.linalg.norm(f - H.finest.apply(u64.cpu().numpy())) / nf
    Sm = igamg.Solver(prob, igamg.default_options(precision=igamg.MIXED))
    um, im = Sm.solve(f)
    resm = np.linalg.norm(f - H.finest.apply(um.cpu().numpy())) / nf
    _say(f"  FP64 {i64.iterations} it, residual {res64:.2e}; mixed {im.iterations} inner it, "
         f"{im.outer_iterations} refinements, residual {resm:.2e}")
    assert i64.converged and res64 <= 1.0001e-8
    assert im.converged and resm <= 1.0001e-8
    # two solutions with residuals <= 1e-8 differ by at most about kappa(A) 2e-8
    # in the worst case; they agree far better than that in practice
    diff = float(np.linalg.norm(um.cpu().numpy() - u64.cpu().numpy()) / np.linalg.norm(u64.cpu().numpy()))
    _say(f"  |u_mixed - u_fp64| / |u_fp64| = {diff:.2e}")
    assert diff < 1e-5
    # both against the oracle's own PCG solution (Sec. 4) of the same system
    uo, ito, _ = H.pcg(f, tol=1e-8)
    no = np.linalg.norm(uo)
    e64 = float(np.linalg.norm(u64.cpu().numpy() - uo) / no)
    em = float(np.linalg.norm(um.cpu().numpy() - uo) / no)
    _say(f"  oracle PCG {ito} it; |u - u_oracle| / |u_oracle|: FP64 {e64:.2e}, mixed {em:.2e}")
    # three solutions with residuals <= 1e-8 of an operator with the
    # replica's conditioning agree to well below 1e-6
    assert e64 < 1e-6 and em < 1e-6


def test_concurrent_setups_factor_correctly(torch_cuda):
    # Two setups in two threads, as the serving loop runs them, each factoring
    # the replica's 30,056-unknown coarse matrix on the device: every setup
    # must succeed and solve exactly as a setup made alone (before device
    # factorizations were serialised, half of such overlapping setups
    # reported a non-positive-definite coarse matrix).
    import concurrent.futures as cf
    from paper_1804_02539_amd import igamg
    prob = W.batched_patch_cube(divide=4)

    def setup_and_solve(i):
        st = torch_cuda.cuda.Stream()
        with torch_cuda.cuda.stream(st):
            S = igamg.Solver(prob, stream=st)
        st.synchronize()
        u, info = S.solve(torch_cuda.as_tensor(W.random_rhs(S.N, 9), device="cuda:0"))
        return u.cpu().numpy(), info.iterations

    ref_u, ref_it = setup_and_solve(-1)
    with cf.ThreadPoolExecutor(2) as ex:
        res = list(ex.map(setup_and_solve, range(4)))
    _say(f"4 concurrent setups: iterations {[r[1] for r in res]} (alone {ref_it})")
    for u, it in res:
        assert it == ref_it and np.array_equal(u, ref_u)


def _patch_check(S, prob, k, rng):
    """Finest apply of the library on a vector living on the strict interior of
    patch k, against the oracle's operator of that patch."""
    from oracle.assembly import PatchOp
    from oracle.topology import DofMap
    from paper_1804_02539_amd import igamg
    L = prob.levels - 1
    dm = DofMap(prob, L)
    gid = dm.patch_gid(k)
    n = dm.n[k]
    idx = np.indices(list(reversed(n))).reshape(3, -1)[::-1]          # (i0, i1, i2), i0 fastest
    interior = np.all([(idx[c] > 0) & (idx[c] < n[c] - 1) for c in range(3)], axis=0)
    assert np.all(gid[interior] >= 0)
    x_loc = np.zeros(dm.size[k])
    x_loc[interior] = rng.standard_normal(int(interior.sum()))
    X = np.zeros(S.N)
    X[gid[interior]] = x_loc[interior]
    Y = S.operator(igamg.OP_APPLY, -1, X).cpu().numpy()
    op = PatchOp(prob.geo_degree[k], prob.geo_ctrl[k], prob.degree, prob.nel(L)[k])
    y_loc = op.apply(x_loc)
    return rel(Y[gid[interior]], y_loc[interior])


def test_full_size_solves(torch_cuda):
    import torch
    from paper_1804_02539_amd import igamg
    prob = W.batched_patch_cube()
    _say("full size: FP64 setup (N = 2.87M, 64 patches, p=5)")
    S = igamg.Solver(prob)
    assert S.N == 2872567
    nel = prob.nel(prob.levels - 1)
    sizes = [int(np.prod(e)) for e in nel]
    small = int(np.argmin(sizes))
    longest = min((k for k in range(prob.npatch) if nel[k].max() == 48), key=lambda k: sizes[k])
    rng = np.random.default_rng(7)
    for k in (small, longest):
        err = _patch_check(S, prob, k, rng)
        _say(f"  patch {k} {nel[k].tolist()}: apply vs oracle patch operator {err:.1e}")
        assert err < 1e-12
    f = torch.as_tensor(W.random_rhs(S.N, 4), device="cuda:0")
    u64, i64 = S.solve(f)
    assert i64.converged and i64.rel_residual <= 1e-8
    _say(f"  FP64: {i64.iterations} it, {i64.solve_ms:.0f} ms")
    Sm = igamg.Solver(prob, igamg.default_options(precision=igamg.MIXED))
    um, im = Sm.solve(f)
    assert im.converged and im.rel_residual <= 1e-8
    _say(f"  mixed: {im.iterations} inner it, {im.outer_iterations} refinements, {im.solve_ms:.0f} ms")
    # both residuals by the FP64 band (checked above against the oracle)
    for u in (u64, um):
        r = f - S.operator(igamg.OP_APPLY, -1, u)
        assert float(torch.linalg.norm(r) / torch.linalg.norm(f)) <= 1.0001e-8
    diff = float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64))
    _say(f"  |u_mixed - u_fp64| / |u_fp64| = {diff:.2e}")
    assert diff < 1e-4
