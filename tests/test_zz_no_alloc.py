"""The no-allocation setup (igamg_setup_noalloc) against igamg_setup: the
same problem set up both ways must give the same cycle and the same solve,
on two calls in a row, the second with a smaller problem."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1804_02539_amd import workloads as W  # noqa: E402


def _say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("band_form", [0, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_setup_equals_setup_twice(torch_cuda, precision, band_form):
    """band_form = 2 puts the scatter-form apply, and its windows in the
    caller's workspace, on every level."""
    from paper_1804_02539_amd import igamg
    cases = [("cube2x2x2_p3_l4", lambda: W.cube_2x2x2_trilinear(levels=4)),
             ("square4x4_p3_l3", lambda: W.square_4x4_bezier(p=3, levels=3))]
    for name, make in cases:        # the second problem is the smaller one
        prob = make()
        opts = igamg.default_options(precision=precision, autotune=0, band_form=band_form)
        ref = igamg.Solver(prob, opts)
        na = igamg.Solver(prob, opts, noalloc=True)
        assert na.N == ref.N
        nbytes = na.workspace.numel() - 256
        _say(f"{name} precision={precision} band_form={band_form}: N = {na.N}, no-allocation workspace {nbytes} bytes, "
             f"setup workspace {igamg.workspace_size(prob, opts)} bytes")
        assert nbytes <= igamg.workspace_size(prob, opts)
        r = np.random.default_rng(3).standard_normal(na.N)
        z, zr = na.vcycle(r).cpu().numpy(), ref.vcycle(r).cpu().numpy()
        e = rel(z, zr)
        f = W.random_rhs(na.N, 5)
        u, info = na.solve(f)
        ur, infor = ref.solve(f)
        eu = float(np.linalg.norm(u.cpu().numpy() - ur.cpu().numpy()) / np.linalg.norm(ur.cpu().numpy()))
        _say(f"  cycle rel diff {e:.2e}; solve {info.iterations} it vs {infor.iterations}, u rel diff {eu:.2e}")
        assert e < 1e-10
        assert info.converged and info.iterations == infor.iterations
        assert eu < 1e-10
        del na, ref


def test_noalloc_device_coarse_factorization(torch_cuda):
    # the coarse matrix factored and inverted on the device, in the workspace
    from paper_1804_02539_amd import igamg
    prob = W.square_4x4_bezier(p=3, levels=3)
    opts = igamg.default_options(coarse_factor=2, autotune=0)
    ref = igamg.Solver(prob, opts)
    na = igamg.Solver(prob, opts, noalloc=True)
    r = np.random.default_rng(8).standard_normal(na.N)
    e = rel(na.vcycle(r).cpu().numpy(), ref.vcycle(r).cpu().numpy())
    _say(f"device coarse factorization without allocation: cycle rel diff {e:.2e}")
    assert e == 0.0
