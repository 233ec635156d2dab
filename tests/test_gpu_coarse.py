"""The exact coarse solve (Sec. 4): A_0^{-1} in packed lower 64 x 64 tiles,
formed on the host (coarse_factor = 1) or by the library's tiled Cholesky
factorization and inversion on the device (coarse_factor = 2), applied by
the two-pass symmetric tile product.  Checked against the oracle's Cholesky
solve of the same coarse matrix, on coarse sizes below one tile, of exactly
one tile, and of many tiles with a ragged last one."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-coarse] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


CASES = {   # name: (problem, free coarse unknowns)
    "n36": (lambda: W.box_grid(2, [1, 1], 2, 6, 2), 36),
    "n64": (lambda: W.box_grid(2, [1, 1], 1, 9, 2), 64),
    "n121": (lambda: W.box_grid(2, [2, 2], 3, 4, 2), 121),
    "n1331_3d": (lambda: W.box_grid(3, [1, 1, 1], 2, 11, 2), 1331),
    "n1681": (lambda: W.box_grid(2, [1, 1], 2, 41, 2), 1681),
}


@pytest.mark.parametrize("where", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_coarse_inverse_matches_oracle(torch_cuda, name, where):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    make, n0 = CASES[name]
    prob = make()
    H = Hierarchy(prob)
    assert H.levels[0].N == n0
    S = igamg.Solver(prob, igamg.default_options(coarse_factor=where, autotune=0))
    A0 = H.levels[0].A.toarray()
    cond = float(np.linalg.cond(A0))
    # a backward-stable Cholesky inverse errs by a modest multiple of
    # cond(A_0) * eps; 64 * cond * eps bounds both sides here
    tol = 64 * cond * 2.0 ** -52
    worst = 0.0
    rng = np.random.default_rng(11)
    for _ in range(3):
        x = rng.standard_normal(n0)
        worst = max(worst, rel(S.operator(igamg.OP_COARSE, 0, x).cpu().numpy(), H.coarse_solve(x)))
    _say(f"{name} on {'host' if where == 1 else 'device'}: N0 = {n0}, cond {cond:.1e}, "
         f"max rel diff {worst:.2e} (bar {tol:.1e})")
    assert worst < tol


def test_device_coarse_inverse_is_deterministic(torch_cuda):
    from paper_1804_02539_amd import igamg
    prob = CASES["n1681"][0]()
    opts = igamg.default_options(coarse_factor=2, autotune=0)
    S1, S2 = igamg.Solver(prob, opts), igamg.Solver(prob, opts)
    x = np.random.default_rng(12).standard_normal(1681)
    y1 = S1.operator(igamg.OP_COARSE, 0, x)
    assert bool(torch_cuda.equal(y1, S2.operator(igamg.OP_COARSE, 0, x)))
    assert bool(torch_cuda.equal(y1, S1.operator(igamg.OP_COARSE, 0, x)))
    _say("two device factorizations give the same coarse solve bit for bit")


def test_coarse_inverse_beyond_32_bit_indexing(torch_cuda):
    """The Fichera corner, K = 448, p = 5, l = 1: N0 = 56,000, so A_0 has more
    than 2^31 entries (the size at which 32-bit dense factorizations fail).
    The device inverse applied to random vectors must give back x under the
    oracle's A_0 (a residual check: the oracle's dense solve at this size is
    too slow for a test), and the solve must converge as in the Fichera table."""
    from oracle.multigrid import Level
    from paper_1804_02539_amd import igamg
    prob = W.fichera(5, 2, split=4)
    S = igamg.Solver(prob)
    L0 = Level(prob, 0)
    assert L0.N == 56000 and L0.N ** 2 > 2 ** 31
    rng = np.random.default_rng(13)
    worst = 0.0
    for _ in range(2):
        x = rng.standard_normal(L0.N)
        y = S.operator(igamg.OP_COARSE, 0, x).cpu().numpy()
        worst = max(worst, float(np.linalg.norm(L0.A @ y - x) / np.linalg.norm(x)))
    u, info = S.solve(S.load_vector(*prob.meta["source"][1:]))
    _say(f"fichera448 p=5 l=1: N0 = {L0.N}, |A0 (A0^-1 x) - x| / |x| = {worst:.2e}; "
         f"solve {info.iterations} iterations, residual {info.rel_residual:.2e}")
    assert worst < 1e-9
    assert info.converged and 20 <= info.iterations <= 28
