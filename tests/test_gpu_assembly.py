"""GPU tests of the device assembly of the banded patch matrices (Sec. 4):
Gauss quadrature with p+1 points per element and direction, sum-factorised,
written straight into the tiled band.  The device-assembled operators are
checked against the oracle's, and against the host assembly (options.assembly
= 1); a patch whose det J changes sign only on a fine level is rejected."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-assembly] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = {
    "square4x4_bezier_p4_l4": lambda: W.square_4x4_bezier(levels=4),
    "square4x4_bezier_p3_nel1": lambda: W.square_4x4_bezier(p=3, nel0=1, levels=3, seed=5),
    "cube2x2x2_trilinear_p3_l4": lambda: W.cube_2x2x2_trilinear(levels=4),
    "cube2x2x2_trilinear_p5_l3": lambda: W.cube_2x2x2_trilinear(p=5, levels=3),
    "fichera7_p4_l2": lambda: W.fichera(4, 2),
    "box3x1_p1_l4": lambda: W.box_grid(2, [3, 1], 1, 2, 4, gdeg=1, dirichlet_sides=[0]),
    "box1x2_p8_l3": lambda: W.box_grid(2, [1, 2], 8, 1, 3, gdeg=1),
    "cube_p4_l3_neumann": lambda: W.box_grid(3, [2, 1, 1], 4, 1, 3, gdeg=1, dirichlet_sides=[0, 2]),
    "box3d_p6_l2": lambda: W.box_grid(3, [1, 1, 2], 6, 1, 2, gdeg=1),
}

ORACLE_CASES = ["cube2x2x2_trilinear_p5_l3", "fichera7_p4_l2", "box1x2_p8_l3", "box3d_p6_l2"]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need cuda:0"
    return torch


@pytest.mark.parametrize("name", list(CASES))
def test_device_assembly_equals_host_assembly(torch_cuda, name):
    from paper_1804_02539_amd import igamg
    prob = CASES[name]()
    Sd = igamg.Solver(prob)
    Sh = igamg.Solver(prob, igamg.default_options(assembly=1))
    rng = np.random.default_rng(4)
    worst = 0.0
    for l in range(1, prob.levels):
        x = rng.standard_normal(Sd.num_dofs(l)[0])
        yd = Sd.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        yh = Sh.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        worst = max(worst, rel(yd, yh))
    r = rng.standard_normal(Sd.N)
    vc = rel(Sd.vcycle(r).cpu().numpy(), Sh.vcycle(r).cpu().numpy())
    _say(f"{name}: apply device vs host {worst:.2e}, cycle {vc:.2e}")
    # the cycle to the bound of its parity against the oracle: at p = 8 the
    # smoother turns band differences of 3e-16 into cycle differences of 1e-11
    assert worst < 1e-13 and vc < 1e-10


@pytest.mark.parametrize("name", ORACLE_CASES)
def test_device_assembly_matches_oracle(torch_cuda, name):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    prob = CASES[name]()
    H = Hierarchy(prob)
    S = igamg.Solver(prob)
    rng = np.random.default_rng(5)
    worst = 0.0
    for l in range(1, len(H.levels)):
        x = rng.standard_normal(H.levels[l].N)
        worst = max(worst, rel(S.operator(igamg.OP_APPLY, l, x).cpu().numpy(), H.levels[l].apply(x)))
    _say(f"{name}: device-assembled apply vs oracle {worst:.2e}")
    assert worst < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_device_assembled_solve(torch_cuda, precision):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    prob = CASES["cube2x2x2_trilinear_p3_l4"]()
    H = Hierarchy(prob)
    opts = igamg.default_options(precision=igamg.MIXED if precision == "mixed" else igamg.FP64)
    S = igamg.Solver(prob, opts)
    f = S.load_vector(*prob.meta["source"][1:])
    u, info = S.solve(torch_cuda.as_tensor(f, device="cuda:0"), tol=1e-8)
    res = np.linalg.norm(f - H.finest.apply(u.cpu().numpy())) / np.linalg.norm(f)
    _say(f"{precision}: {info.iterations} iterations, residual by the oracle's operator {res:.2e}")
    assert info.converged and res <= 1.0001e-8


def _folded(levels):
    # x = s, y = t (s + t - 0.1): det J = s + 2t - 0.1 is positive at every
    # Gauss point of levels 0 and 1 (nearest the corner: 0.113 and 0.056) and
    # negative at the level-2 point nearest the corner (0.028, 0.028)
    ctrl = np.array([[0, 0], [1, 0], [0, -0.05], [1, 0.45], [0, 0.9], [1, 1.9]], dtype=float)
    return W.Problem(dim=2, degree=2, levels=levels, nel0=np.array([[1, 1]], np.int32),
                     geo_degree=np.array([[1, 2]], np.int32), geo_ctrl=[ctrl],
                     iface=np.zeros((0, 5), np.int32), bc=np.array([[1, 1, 1, 1]], np.int32), name="folded")


@pytest.mark.parametrize("assembly", [0, 1])
def test_fold_on_a_fine_level_is_rejected(torch_cuda, assembly):
    from paper_1804_02539_amd import igamg
    igamg.Solver(_folded(2), igamg.default_options(assembly=assembly))
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(_folded(3), igamg.default_options(assembly=assembly))
    assert e.value.code == igamg.EGEOM
    _say(f"assembly={assembly}: {e.value}")


def test_setup_time_device_and_host(torch_cuda):
    """Reports both setup times (no assertion on wall-clock time)."""
    from paper_1804_02539_amd import igamg
    prob = W.cube_2x2x2_trilinear(p=4, levels=5)
    igamg.Solver(prob)   # warm-up: the smoother choices are then cached for both timed setups
    times = {}
    for a in (1, 0):
        torch_cuda.cuda.synchronize()
        t0 = time.perf_counter()
        S = igamg.Solver(prob, igamg.default_options(assembly=a))
        torch_cuda.cuda.synchronize()
        times[a] = time.perf_counter() - t0
        del S
    _say(f"cube p=4, 5 levels: setup {times[1]:.2f} s with host assembly, {times[0]:.2f} s with device assembly")
