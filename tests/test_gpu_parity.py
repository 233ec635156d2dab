"""GPU parity: the HIP library against the FP64 oracle, operator by operator,
for one cycle and for full PCG solves.  Runs on cuda:0 through the C-ABI."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need cuda:0"
    return torch


CASES = {
    # name: (problem factory, rhs kind)
    "square2x2_p2": lambda: W.unit_square_2x2(),
    "square4x4_p4_l4": lambda: W.square_4x4_bezier(levels=4),
    "square4x4_p3_l3_nel1": lambda: W.square_4x4_bezier(p=3, nel0=1, levels=3, seed=5),
    "cube2x2x2_p3_l4": lambda: W.cube_2x2x2_trilinear(levels=4),
    "cube2x2x2_p2_l3": lambda: W.cube_2x2x2_trilinear(p=2, levels=3),
    "fichera7_p2_l3": lambda: W.fichera(2, 3),
    "fichera448_p3_l1": lambda: W.fichera(3, 2, split=4),
    "fichera448_p4_l1": lambda: W.fichera(4, 2, split=4),
    "box3x1_p1_l4": lambda: W.box_grid(2, [3, 1], 1, 2, 4, gdeg=1, dirichlet_sides=[0]),
    "single_patch_p5_l3": lambda: W.box_grid(2, [1, 1], 5, 2, 3, gdeg=1),
    "cube_p4_l3_neumann": lambda: W.box_grid(3, [2, 1, 1], 4, 1, 3, gdeg=1, dirichlet_sides=[0, 2]),
    "graded_square3x2_p3_l3": lambda: W.graded_square_3x2(),
    "graded_cube2x2x2_p2_l3": lambda: W.graded_cube_2x2x2(),
    # patches finer than the FD kernels stage in LDS (88 interior functions
    # along a direction on the finest level): the kernels read those
    # tensors' operands from memory
    "fine_square_p2_m88": lambda: W.box_grid(2, [1, 1], 2, 11, 4, gdeg=1),
    "fine_cube_z_p2_m88": lambda: W.box_grid(3, [2, 2, 1], 2, [[2, 2], [2, 2], [11]], 4, gdeg=1),
    "fine_cube_x_p2_m88": lambda: W.box_grid(3, [1, 1, 2], 2, [[11], [2], [2, 2]], 4, gdeg=1,
                                             dirichlet_sides=[0, 2, 4]),
}

_ORACLE = {}
_GPU = {}


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
def test_operators_match_oracle(torch_cuda, name):
    from paper_1804_02539_amd import igamg
    _say(f"operators {name}")
    H = oracle_for(name)
    S = gpu_for(name)
    rng = np.random.default_rng(1)
    for l in range(len(H.levels)):
        lev = H.levels[l]
        x = rng.standard_normal(lev.N)
        if l == 0:
            y = S.operator(igamg.OP_COARSE, 0, x).cpu().numpy()
            assert rel(y, H.coarse_solve(x)) < 1e-11, ("coarse", l)
            continue
        y = S.operator(igamg.OP_APPLY, l, x).cpu().numpy()
        assert rel(y, lev.apply(x)) < 1e-12, ("apply", l)
        y = S.operator(igamg.OP_SMOOTHER, l, x).cpu().numpy()
        assert rel(y, lev.smoother.apply(x)) < 1e-11, ("smoother", l)
        xc = rng.standard_normal(H.levels[l - 1].N)
        y = S.operator(igamg.OP_PROLONG, l, xc).cpu().numpy()
        assert rel(y, H.P[l] @ xc) < 1e-13, ("prolong", l)
        y = S.operator(igamg.OP_RESTRICT, l, x).cpu().numpy()
        assert rel(y, H.P[l].T @ x) < 1e-13, ("restrict", l)


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_matches_oracle(torch_cuda, name):
    _say(f"vcycle {name}")
    H = oracle_for(name)
    S = gpu_for(name)
    r = np.random.default_rng(2).standard_normal(H.finest.N)
    z = S.vcycle(r).cpu().numpy()
    assert rel(z, H.vcycle(r)) < 1e-10


def test_wcycle_matches_oracle(torch_cuda):
    from oracle.multigrid import Hierarchy
    _say("wcycle square4x4_p3_l3_nel1 mu=2 nu=2")
    prob = CASES["square4x4_p3_l3_nel1"]()
    H = Hierarchy(prob, mu=2, nu=2)
    S = gpu_for("square4x4_p3_l3_nel1", mu=2, nu=2)
    r = np.random.default_rng(3).standard_normal(H.finest.N)
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10


SOLVE_CASES = ["square2x2_p2", "square4x4_p4_l4", "cube2x2x2_p3_l4", "fichera7_p2_l3", "fichera448_p3_l1",
               "fichera448_p4_l1", "graded_cube2x2x2_p2_l3"]


def _rhs(name, H, S):
    from oracle.multigrid import load_vector
    prob = CASES[name]()
    if prob.meta["source"][0] == "sine":
        f = load_vector(prob, H.finest)
        fg = S.load_vector(*prob.meta["source"][1:])
        assert rel(fg, f) < 1e-13
        return f
    return W.random_rhs(H.finest.N, prob.meta["source"][1])


def _nrel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


# Two PCG runs (Sec. 4) of exactly k iterations from u = 0 on the same
# operator and preconditioner agree up to rounding.  For most problems the
# library's and the oracle's iterates agree to 1e-10 relative, the bar.  Where
# the PCG amplifies rounding more than that, the bar comes from the oracle
# itself.  The library's cycle and coarse solve are compared with the
# oracle's on random vectors (relative max-norm differences e_cyc and e_crs,
# at least 2^-52).  The oracle's PCG is then rerun with every output of its
# coarse solve and of its cycle perturbed elementwise by relative amounts of
# those sizes (three seeds); ten times the largest move of its iterate (and of
# its residual) is what two correct FP64 runs of the same PCG may differ by.
FIXED_K_TOL = 1e-10


def _perturbed_pcg(H, f, k, seed, e_cyc, e_crs):
    rng = np.random.default_rng(seed)
    cycle, coarse = H.vcycle, H.coarse_solve
    H.coarse_solve = lambda r: (lambda z: z * (1.0 + e_crs * rng.uniform(-1.0, 1.0, z.shape)))(coarse(r))
    H.vcycle = lambda r: (lambda z: z * (1.0 + e_cyc * rng.uniform(-1.0, 1.0, z.shape)))(cycle(r))
    try:
        u, _, hist = H.pcg(f, tol=0.0, maxit=k)
    finally:
        del H.vcycle
        del H.coarse_solve
    return u, hist[-1]


def _bar(H, S, f, k, u_k, res_k, err):
    """(bar for u, bar for the final relative residual, sensitivity or None):
    the fixed bars, or the measured rounding sensitivity of the oracle's PCG
    after k iterations (computed only when err exceeds FIXED_K_TOL)."""
    from paper_1804_02539_amd import igamg
    if err < FIXED_K_TOL:
        return FIXED_K_TOL, 1e-6 * res_k, None
    rng = np.random.default_rng(11)
    r = rng.standard_normal(H.finest.N)
    zc = H.vcycle(r)
    e_cyc = max(2.0 ** -52, float(np.abs(S.vcycle(r).cpu().numpy() - zc).max() / np.abs(zc).max()))
    r0 = rng.standard_normal(H.levels[0].N)
    z0 = H.coarse_solve(r0)
    e_crs = max(2.0 ** -52, float(np.abs(S.operator(igamg.OP_COARSE, 0, r0).cpu().numpy() - z0).max()
                                  / np.abs(z0).max()))
    runs = [_perturbed_pcg(H, f, k, s, e_cyc, e_crs) for s in range(3)]
    sens = max(_nrel(u, u_k) for u, _ in runs)
    sens_r = max(abs(rr - res_k) for _, rr in runs)
    _say(f"  measured differences: cycle {e_cyc:.1e}, coarse solve {e_crs:.1e}; oracle PCG sensitivity "
         f"{sens:.1e} (u), {sens_r:.1e} (residual)")
    return max(FIXED_K_TOL, 10.0 * sens), max(1e-6 * res_k, 10.0 * sens_r), sens


@pytest.mark.parametrize("name", SOLVE_CASES)
def test_solve_matches_oracle(torch_cuda, name):
    _say(f"solve {name}")
    H = oracle_for(name)
    S = gpu_for(name)
    f = _rhs(name, H, S)
    u_ref, it_ref, _ = H.pcg(f, tol=1e-8)
    u, info = S.solve(f, tol=1e-8)
    u = u.cpu().numpy()
    res = np.linalg.norm(f - H.finest.apply(u)) / np.linalg.norm(f)
    assert res <= 1.0001e-8 and info.rel_residual <= 1e-8
    assert abs(res - info.rel_residual) <= 1e-3 * res + 1e-14
    # the GPU solution against the oracle's iterate after the same number of
    # iterations, whether or not the two stopping tests fired on the same one
    u_same, _, hist_same = H.pcg(f, tol=0.0, maxit=info.iterations)
    e_same = _nrel(u, u_same)
    e_conv = _nrel(u, u_ref)
    bar, _, sens = _bar(H, S, f, info.iterations, u_same, hist_same[-1], e_same)
    _say(f"  GPU {info.iterations} it, oracle {it_ref} it; |u - u_oracle(k)|/|u_oracle(k)| = {e_same:.2e} "
         f"(bar {bar:.1e}{'' if sens is None else f', oracle rounding sensitivity {sens:.1e}'}), "
         f"against the oracle's converged u {e_conv:.2e}")
    assert e_same < bar
    assert abs(info.iterations - it_ref) <= 2, (info.iterations, it_ref)


@pytest.mark.parametrize("name", SOLVE_CASES)
def test_solve_fixed_iterations_match_oracle(torch_cuda, name):
    """Both PCGs run exactly k iterations (tolerance 1e-300, cap k); the iterates
    must agree to the bar above at k = 5 and at half the converged count."""
    from paper_1804_02539_amd import igamg
    H = oracle_for(name)
    _, it_ref, _ = H.pcg(_rhs(name, H, gpu_for(name)), tol=1e-8)
    for k in sorted({5, max(1, it_ref // 2)}):
        S = igamg.Solver(CASES[name](), igamg.default_options(maxit=k))
        f = _rhs(name, H, S)
        u, info = S.solve(f, tol=1e-300, raise_on_error=False)
        assert S.last_code == igamg.ENOCONV and info.iterations == k, (S.last_code, info.iterations)
        u_k, _, hist = H.pcg(f, tol=0.0, maxit=k)
        err = _nrel(u.cpu().numpy(), u_k)
        bar, bar_r, sens = _bar(H, S, f, k, u_k, hist[-1], err)
        _say(f"  {name} k={k}: |u - u_oracle|/|u_oracle| = {err:.2e} (bar {bar:.1e}), residual "
             f"{hist[-1]:.3e}, GPU {info.rel_residual:.3e} (bar {bar_r:.1e})")
        assert err < bar
        assert abs(info.rel_residual - hist[-1]) <= bar_r


def test_full_size_square4x4(torch_cuda):
    """The 2D 16-patch p=4 workload at its full size (6 levels, 71,824 dofs)."""
    _say("full-size square4x4_p4 (6 levels)")
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    prob = W.square_4x4_bezier()
    H = Hierarchy(prob)
    S = igamg.Solver(prob)
    assert S.N == H.finest.N == 71824
    rng = np.random.default_rng(4)
    r = rng.standard_normal(S.N)
    assert rel(S.operator(igamg.OP_APPLY, -1, r).cpu().numpy(), H.finest.apply(r)) < 1e-12
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10
    f = W.random_rhs(S.N, 2)
    u_ref, it_ref, _ = H.pcg(f)
    u, info = S.solve(f)
    assert abs(info.iterations - it_ref) <= 1
    assert np.linalg.norm(f - H.finest.apply(u.cpu().numpy())) <= 1.0001e-8 * np.linalg.norm(f)


def test_full_size_cube_sampled(torch_cuda):
    """The 3D 8-patch p=3 workload at full size (32^3 elements per patch, 300,763
    dofs): the finest apply against the oracle's matrix-free apply, a full cycle
    against the oracle's cycle, and the solve residual by the oracle's operator."""
    _say("full-size cube2x2x2_p3 (6 levels)")
    from oracle.multigrid import Hierarchy, load_vector
    from paper_1804_02539_amd import igamg
    prob = W.cube_2x2x2_trilinear()
    H = Hierarchy(prob)
    _say("  oracle hierarchy built")
    S = igamg.Solver(prob)
    assert S.N == H.finest.N == 300763
    r = np.random.default_rng(5).standard_normal(S.N)
    assert rel(S.operator(igamg.OP_APPLY, -1, r).cpu().numpy(), H.finest.apply(r)) < 1e-12
    _say("  apply ok")
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10
    _say("  cycle ok")
    f = load_vector(prob, H.finest)
    u, info = S.solve(f)
    assert info.converged
    assert np.linalg.norm(f - H.finest.apply(u.cpu().numpy())) <= 1.0001e-8 * np.linalg.norm(f)


# --- mixed precision: FP32 inner solves inside FP64 iterative refinement ----

@pytest.mark.parametrize("fd_mfma", [1, 2])
@pytest.mark.parametrize("name", ["square4x4_p4_l4", "cube2x2x2_p3_l4", "fichera7_p2_l3", "cube_p4_l3_neumann",
                                  "single_patch_p5_l3", "fine_square_p2_m88", "fine_cube_z_p2_m88"])
def test_fp32_cycle_close_to_oracle(torch_cuda, name, fd_mfma):
    """The FP32 cycle (FP32 bands, smoothers, transfers; FP32 coarse inverse)
    against the oracle's FP64 cycle: FP32 rounding only.  fd_mfma = 1 runs the
    smoother's mode products on the matrix cores, 2 on vector FMAs."""
    from paper_1804_02539_amd import igamg
    _say(f"fp32 cycle {name} fd_mfma={fd_mfma}")
    H = oracle_for(name)
    S = gpu_for(name, precision=igamg.MIXED, fd_mfma=fd_mfma)
    r = np.random.default_rng(7).standard_normal(H.finest.N)
    z = S.operator(igamg.OP_CYCLE_FP32, -1, r).cpu().numpy()
    err = rel(z, H.vcycle(r))
    _say(f"  fp32 cycle max rel error {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("name,fd_mfma", [("square2x2_p2", 0), ("square4x4_p4_l4", 0), ("cube2x2x2_p3_l4", 0),
                                          ("fichera7_p2_l3", 0), ("square4x4_p4_l4", 1), ("fichera7_p2_l3", 1),
                                          ("cube2x2x2_p3_l4", 2), ("square4x4_p4_l4", 3), ("cube2x2x2_p3_l4", 3),
                                          ("fichera7_p2_l3", 3)])
def test_mixed_solve_reaches_fp64_tolerance(torch_cuda, name, fd_mfma):
    from oracle.multigrid import load_vector
    from paper_1804_02539_amd import igamg
    _say(f"mixed solve {name} fd_mfma={fd_mfma}")
    prob = CASES[name]()
    H = oracle_for(name)
    S = gpu_for(name, precision=igamg.MIXED, fd_mfma=fd_mfma)
    if prob.meta["source"][0] == "sine":
        f = load_vector(prob, H.finest)
    else:
        f = W.random_rhs(H.finest.N, prob.meta["source"][1])
    u_ref, it_ref, _ = H.pcg(f, tol=1e-8)
    u, info = S.solve(f, tol=1e-8)
    u = u.cpu().numpy()
    res = np.linalg.norm(f - H.finest.apply(u)) / np.linalg.norm(f)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    _say(f"  mixed: {info.outer_iterations} refinements, {info.iterations} inner it "
         f"(FP64 PCG {it_ref}); rel residual {res:.2e}; |u - u_oracle|/|u_oracle| {err:.2e}")
    assert info.converged and res <= 1.0001e-8
    assert err < 1e-6
    # the FP64 handle of the same problem still gives the oracle's result
    u64, info64 = gpu_for(name).solve(f, tol=1e-8)
    assert abs(info64.iterations - it_ref) <= 1


# readings of the smoother constants: library option -> oracle reading
READING_OPTS = {
    "omega_mean": ({"geometry_scaling": 1}, {"omega": "mean"}),
    "s1_K": ({"s1_sigma": 0}, {"k1": "K"}),
    "mult": ({"iface_multiplicity": 1}, {"mult": True}),
    "physh": ({"physical_h": 1}, {"h": "physical"}),
    "direct": ({"iface_direct": 1}, {"edges": "direct"}),
    "direct_hostasm": ({"iface_direct": 1, "assembly": 1}, {"edges": "direct"}),
}


@pytest.mark.parametrize("reading", list(READING_OPTS))
@pytest.mark.parametrize("name", ["fichera7_p2_l3", "cube2x2x2_p3_l4", "square4x4_p3_l3_nel1",
                                  "graded_cube2x2x2_p2_l3"])
def test_smoother_readings_match_oracle(torch_cuda, reading, name):
    from oracle.multigrid import Hierarchy
    from paper_1804_02539_amd import igamg
    lib_opts, orc = READING_OPTS[reading]
    _say(f"reading {reading} {name}")
    prob = CASES[name]()
    H = Hierarchy(prob, reading=orc)
    S = igamg.Solver(prob, igamg.default_options(**lib_opts))
    rng = np.random.default_rng(8)
    for l in range(1, len(H.levels)):
        x = rng.standard_normal(H.levels[l].N)
        y = S.operator(igamg.OP_SMOOTHER, l, x).cpu().numpy()
        assert rel(y, H.levels[l].smoother.apply(x)) < 1e-11, l
    r = rng.standard_normal(H.finest.N)
    assert rel(S.vcycle(r).cpu().numpy(), H.vcycle(r)) < 1e-10


@pytest.mark.parametrize("name", ["square4x4_p4_l4", "square2x2_p2", "cube2x2x2_p3_l4", "fichera7_p2_l3",
                                  "single_patch_p5_l3"])
def test_bf16_smoother_cycle_error_stated(torch_cuda, name):
    """The FP32 cycle with the smoother's mode products in bfloat16 (FP32
    accumulation) against the oracle's FP64 cycle: the error is stated; it
    is bfloat16 rounding (2^-9 per operand), nothing larger."""
    from paper_1804_02539_amd import igamg
    H = oracle_for(name)
    S = gpu_for(name, precision=igamg.MIXED, fd_mfma=3)
    r = np.random.default_rng(7).standard_normal(H.finest.N)
    z = S.operator(igamg.OP_CYCLE_FP32, -1, r).cpu().numpy()
    err = rel(z, H.vcycle(r))
    S32 = gpu_for(name, precision=igamg.MIXED, fd_mfma=1)
    e32 = rel(S32.operator(igamg.OP_CYCLE_FP32, -1, r).cpu().numpy(), H.vcycle(r))
    _say(f"bf16 cycle {name}: rel err {err:.2e} against the FP64 oracle (FP32 matrix cores {e32:.2e}); "
         f"finest variant {igamg.FD_NAMES[S.tuning(-1, True)]}")
    assert S.tuning(-1, True) == igamg.FD_MFMA_BF16
    assert err < 3e-2
    # the precision value IGAMG_MIXED_BF16 selects the same kernels
    Sb = gpu_for(name, precision=igamg.MIXED_BF16)
    assert bool(torch_cuda.equal(Sb.operator(igamg.OP_CYCLE_FP32, -1, r), S.operator(igamg.OP_CYCLE_FP32, -1, r)))
