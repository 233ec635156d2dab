"""GPU test of the serving loop: a seeded request mix with Poisson arrivals
under an HBM budget small enough to force evictions.  Every request's
solution must equal the same request solved alone (bit for bit: the kernels
are deterministic and a request's graph branch is independent of the others),
and the device memory the server holds must stay within its budget."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-serve] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_serving_mix_equals_alone_within_budget(precision):
    import torch
    from paper_1804_02539_amd import igamg, serve
    assert torch.cuda.is_available()
    opts = igamg.default_options(precision=igamg.MIXED if precision == "mixed" else igamg.FP64)
    fams, reqs = serve.request_mix(24, seed=11, n_families=6, n_min=3e3, n_max=4e4)
    sizes = sorted(igamg.workspace_size(f, opts) for f in fams)
    budget = sizes[-1] + sizes[-2] + sizes[-3] + 3 * 256    # about three hierarchies at once
    _say(f"{precision}: families {[f.name for f in fams]}, budget {budget / 1e6:.1f} MB")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    S = serve.Server(budget, opts=opts, handles_per_key=2, setup_workers=2)
    arr = [(float(t), r) for t, r in zip(serve.poisson_offsets(len(reqs), 400.0, seed=3), reqs)]
    t = S.run(arrivals=arr, timeout=300)
    S.close()
    st = S.stats(t)
    _say(f"{precision}: {st}")
    assert st["requests"] == len(reqs) and st["rejected"] == 0 and st["failed"] == 0
    assert S.peak_used <= budget
    vec_bytes = sum(2 * 8 * r.n for r in reqs)            # rhs and solution tensors, outside the budget
    assert torch.cuda.max_memory_allocated() - base <= budget + vec_bytes + (64 << 20)
    # each request alone, on a fresh hierarchy of its family
    alone = {}
    for r in reqs:
        if r.key not in alone:
            alone[r.key] = igamg.Solver(r.problem, opts)
        Sa = alone[r.key]
        u, info = Sa.solve(torch.as_tensor(r.rhs_fn(Sa.N), device="cuda:0"))
        assert info.iterations == r.info.iterations, r.problem.name
        assert torch.equal(u, r.result), r.problem.name
    _say(f"{precision}: {len(reqs)} requests equal to their solo solves")
