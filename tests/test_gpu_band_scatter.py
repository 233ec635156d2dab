"""GPU parity of the scatter form of the symmetric half-band apply: each
stored coefficient fetched once, its mirrored term added through per-tile
windows and a second, fixed-order reduction.  options.band_form = 2 puts it
on every level, so problems the oracle finishes in seconds (2D and 3D,
p = 1..8, several tiles per patch, ragged last tiles, Dirichlet and Neumann
sides, graded and curved patches, tensors wider than one tile's window
reach) cover it; the full-size 3D tests cover its default use on 3D levels
above 65536 rows."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-band-scatter] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need cuda:0"
    return torch


CASES = {
    "square2x2_p2": lambda: W.unit_square_2x2(),
    "square4x4_p4_l4": lambda: W.square_4x4_bezier(levels=4),
    "single_patch_p5_l3": lambda: W.box_grid(2, [1, 1], 5, 2, 3, gdeg=1),
    "box3x1_p1_l4": lambda: W.box_grid(2, [3, 1], 1, 2, 4, gdeg=1, dirichlet_sides=[0]),
    "graded_square3x2_p3_l3": lambda: W.graded_square_3x2(),
    "square_p8_l3": lambda: W.box_grid(2, [2, 2], 8, 2, 3, gdeg=1),
    "cube2x2x2_p3_l4": lambda: W.cube_2x2x2_trilinear(levels=4),
    "cube2x2x2_p2_l3": lambda: W.cube_2x2x2_trilinear(p=2, levels=3),
    "fichera7_p2_l3": lambda: W.fichera(2, 3),
    "cube_p4_l3_neumann": lambda: W.box_grid(3, [2, 1, 1], 4, 1, 3, gdeg=1, dirichlet_sides=[0, 2]),
    "graded_cube2x2x2_p2_l3": lambda: W.graded_cube_2x2x2(),
    "fine_cube_x_p2_m88": lambda: W.box_grid(3, [1, 1, 2], 2, [[11], [2], [2, 2]], 4, gdeg=1,
                                             dirichlet_sides=[0, 2, 4]),
    "box_p1_l4": lambda: W.box_grid(3, [1, 2, 1], 1, 2, 4, gdeg=1, dirichlet_sides=[0]),
    "box_p5_l2": lambda: W.box_grid(3, [1, 1, 1], 5, 2, 2, gdeg=1),
    # the high degrees (each degree and type has its own load-buffer depth)
    "box_p6_l2": lambda: W.box_grid(3, [1, 1, 2], 6, 1, 2, gdeg=1),
    "box_p7_l2": lambda: W.box_grid(3, [2, 1, 1], 7, 1, 2, gdeg=1, dirichlet_sides=[0, 2]),
    "box_p8_l2": lambda: W.box_grid(3, [1, 1, 1], 8, 1, 2, gdeg=1),
    # windows of 6,046 values, 96.7 KB of LDS with u in FP64: the widest that fit
    "wide_x_p5_fits": lambda: W.box_grid(3, [1, 1, 1], 5, [[38], [1], [1]], 2, gdeg=1),
}
# windows of 8,466 values (135 KB): above the LDS limit, so the level keeps the
# gather form even with band_form = 2
WIDE_GATHER = lambda: W.box_grid(3, [1, 1, 1], 5, [[60], [1], [1]], 2, gdeg=1)

_ORACLE = {}
_GPU = {}
_ABS = {}   # |A_k| per (case, level), for the FP32 rounding bound


def oracle_for(name):
    from oracle.multigrid import Hierarchy
    if name not in _ORACLE:
        _ORACLE[name] = Hierarchy(CASES[name]())
    return _ORACLE[name]


def gpu_for(name, **opts):
    from paper_1804_02539_amd import igamg
    key = (name, tuple(sorted(opts.items())))
    if key not in _GPU:
        _GPU[key] = igamg.Solver(CASES[name](), igamg.default_options(**opts))
    return _GPU[key]


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(CASES))
def test_scatter_apply_matches_oracle(torch_cuda, name):
    """y = A_l x on every level, scatter form, against the oracle's apply; the
    same input twice gives the same bits (fixed summation order)."""
    from paper_1804_02539_amd import igamg
    _say(f"apply {name}")
    H = oracle_for(name)
    S = gpu_for(name, band_form=2)
    rng = np.random.default_rng(11)
    for l in range(1, len(H.levels)):
        assert S.band_form(l) == igamg.BAND_SCATTER, l
        x = rng.standard_normal(H.levels[l].N)
        y = S.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        assert rel(y, H.levels[l].apply(x)) < 1e-12, l
        y2 = S.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        assert np.array_equal(y, y2), l


@pytest.mark.parametrize("name", ["square4x4_p4_l4", "square_p8_l3", "cube2x2x2_p3_l4", "fichera7_p2_l3",
                                  "cube_p4_l3_neumann", "box_p5_l2"])
def test_scatter_and_gather_forms_agree(torch_cuda, name):
    """The two forms of the same half band differ by summation order only."""
    from paper_1804_02539_amd import igamg
    _say(f"forms {name}")
    H = oracle_for(name)
    Ss = gpu_for(name, band_form=2)
    Sg = gpu_for(name, band_form=1)
    rng = np.random.default_rng(12)
    for l in range(1, len(H.levels)):
        assert Sg.band_form(l) == igamg.BAND_GATHER, l
        x = rng.standard_normal(H.levels[l].N)
        ys = Ss.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        yg = Sg.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        assert rel(ys, yg) < 1e-13, l


@pytest.mark.parametrize("name", ["square4x4_p4_l4", "graded_square3x2_p3_l3", "cube2x2x2_p3_l4", "fichera7_p2_l3",
                                  "graded_cube2x2x2_p2_l3", "fine_cube_x_p2_m88"])
def test_scatter_cycle_and_solve_match_oracle(torch_cuda, name):
    """A V-cycle and a solve to 1e-8 with the scatter form on every level,
    against the oracle; graph replay and direct launches give the same bits."""
    from paper_1804_02539_amd import igamg
    _say(f"cycle and solve {name}")
    H = oracle_for(name)
    S = gpu_for(name, band_form=2)
    r = np.random.default_rng(13).standard_normal(H.finest.N)
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10
    f = W.random_rhs(H.finest.N, 3)
    u_ref, it_ref, _ = H.pcg(f, tol=1e-8)
    u, info = S.solve(f, tol=1e-8)
    u = u.cpu().numpy()
    assert info.converged and abs(info.iterations - it_ref) <= 1
    assert np.linalg.norm(f - H.finest.apply(u)) <= 1.0001e-8 * np.linalg.norm(f)
    ud, infod = gpu_for(name, band_form=2, graphs=0).solve(f, tol=1e-8)
    assert infod.iterations == info.iterations
    assert np.array_equal(ud.cpu().numpy(), u)


@pytest.mark.parametrize("fd_mfma", [0, 1])
@pytest.mark.parametrize("name", ["square4x4_p4_l4", "cube2x2x2_p3_l4", "fichera7_p2_l3", "cube_p4_l3_neumann",
                                  "box_p1_l4"])
def test_scatter_fp32_cycle_and_mixed_solve(torch_cuda, name, fd_mfma):
    """FP32 half band in scatter form: the FP32 cycle within FP32 rounding of
    the oracle's FP64 cycle, and the mixed solve to the FP64 tolerance."""
    from paper_1804_02539_amd import igamg
    _say(f"fp32 {name} fd_mfma={fd_mfma}")
    H = oracle_for(name)
    S = gpu_for(name, band_form=2, precision=igamg.MIXED, fd_mfma=fd_mfma)
    r = np.random.default_rng(14).standard_normal(H.finest.N)
    z = S.operator(igamg.OP_CYCLE_FP32, -1, r).cpu().numpy()
    err = rel(z, H.vcycle(r))
    _say(f"  fp32 cycle max rel error {err:.2e}")
    assert err < 1e-4
    f = W.random_rhs(H.finest.N, 4)
    u, info = S.solve(f, tol=1e-8)
    res = np.linalg.norm(f - H.finest.apply(u.cpu().numpy())) / np.linalg.norm(f)
    assert info.converged and res <= 1.0001e-8


def test_default_form_by_level_size(torch_cuda):
    """options.band_form = 0: the scatter form on the 3D levels above 65536
    local rows (padded), the gather form below, and on 2D levels up to 2^17
    rows (FP64) or 2^19 (mixed).  The 2x2x2 p=3 cube: 343,000 local rows on the finest level, 55,296
    on the next."""
    from paper_1804_02539_amd import igamg
    S = igamg.Solver(W.cube_2x2x2_trilinear())
    L = S.prob.levels - 1
    assert S.num_dofs(L)[1] == 343000 and S.num_dofs(L - 1)[1] == 54872
    assert S.band_form(L) == igamg.BAND_SCATTER
    assert all(S.band_form(l) == igamg.BAND_GATHER for l in range(1, L))
    S2 = igamg.Solver(W.square_4x4_bezier(levels=4))
    assert all(S2.band_form(l) == igamg.BAND_GATHER for l in range(1, 4))
    # 2D, 282,624 rows on the finest level: above 2^17 (FP64 handles), not
    # above 2^19 (mixed handles)
    S7 = igamg.Solver(W.square_4x4_bezier(levels=7))
    assert S7.band_form(-1) == igamg.BAND_SCATTER and S7.band_form(5) == igamg.BAND_GATHER
    S7m = igamg.Solver(W.square_4x4_bezier(levels=7), igamg.default_options(precision=igamg.MIXED))
    assert S7m.band_form(-1) == igamg.BAND_GATHER


def test_windows_above_lds_limit_keep_gather_form(torch_cuda):
    """A level whose windows and u exceed the LDS limit (p = 5, 125 functions
    along x) keeps the gather form under band_form = 2, and applies A as the
    oracle does."""
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    _say("windows above the LDS limit")
    prob = WIDE_GATHER()
    H = Hierarchy(prob)
    S = igamg.Solver(WIDE_GATHER(), igamg.default_options(band_form=2))
    assert S.band_form(1) == igamg.BAND_GATHER
    x = np.random.default_rng(15).standard_normal(H.levels[1].N)
    assert rel(S.operator(igamg.OP_APPLY, 1, x).cpu().numpy(), H.levels[1].apply(x)) < 1e-12


@pytest.mark.parametrize("form", [2, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_fp32_apply_within_rounding_bound(torch_cuda, name, form):
    """y = A_l x with the FP32 band (IGAMG_OP_APPLY_FP32), both forms, on
    every level: each row within the first-order bound of an FP32 product
    sum, (n + 3) eps_32 sum_k (|A_k| |x_k|)_i over the patch matrices that
    hold row i, n = (2p+1)^d terms per patch row (x and the coefficients
    rounded once each, n additions, the result rounded once).  A wrong
    coefficient or index costs O(1) of that sum."""
    from paper_1804_02539_amd import igamg
    _say(f"fp32 apply {name} band_form={form}")
    H = oracle_for(name)
    S = gpu_for(name, band_form=form, precision=igamg.MIXED)
    prob = CASES[name]()
    n_terms = (2 * prob.degree + 1) ** prob.dim
    eps32 = float(np.finfo(np.float32).eps)
    rng = np.random.default_rng(16)
    for l in range(1, len(H.levels)):
        lev = H.levels[l]
        x = rng.standard_normal(lev.N)
        y = S.operator(igamg.OP_APPLY_FP32, l, x).cpu().numpy()
        key = (name, l)
        if key not in _ABS:
            _ABS[key] = [abs(op.matrix()).tocsr() for op in lev.ops]
        bound = np.zeros(lev.N)
        for Sel, absA in zip(lev.S, _ABS[key]):
            bound += Sel @ (absA @ np.abs(Sel.T @ x))
        excess = np.abs(y - lev.apply(x)) / ((n_terms + 3) * eps32 * bound)
        assert excess.max() <= 1.0, (l, float(excess.max()))
