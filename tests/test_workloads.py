"""CPU checks of the seeded workload generators that the GPU tests and the
benchmark use (sizes, conformity, the coarse level shared by the replica)."""
import numpy as np

from paper_1804_02539_amd import workloads as W


def _free_dofs_formula(slabs, p):
    # per direction: sum of slab element counts + p per slab, minus the 3
    # shared interface functions and the 2 Dirichlet ends (open knots, C0)
    return int(np.prod([sum(s) + 4 * p - 5 for s in slabs]))


def test_batched_patch_cube_sizes_and_levels():
    from oracle.topology import DofMap
    prob = W.batched_patch_cube()
    slabs = prob.meta["slabs"]
    assert prob.npatch == 64 and prob.degree == 5 and prob.levels == 4
    assert all(c in (8, 16, 24, 32, 48) for s in slabs for c in s)
    n = _free_dofs_formula(slabs, 5)
    assert 2e6 <= n <= 4e6
    # every patch's finest counts are 8x its coarsest ones, and neighbours conform
    fine = prob.nel(prob.levels - 1)
    assert np.array_equal(fine, prob.nel0 * 8)
    assert DofMap(prob, prob.levels - 1).N == n
    # seeded
    assert W.batched_patch_cube().meta["slabs"] == slabs


def test_batched_patch_cube_replica_keeps_the_coarse_level():
    from oracle.topology import DofMap
    full = W.batched_patch_cube()
    rep = W.batched_patch_cube(divide=4)
    assert rep.levels == 2 and rep.npatch == 64
    assert np.array_equal(rep.nel0, full.nel0)
    assert np.array_equal(rep.nel(1) * 4, full.nel(3))
    for a, b in zip(rep.geo_ctrl, full.geo_ctrl):
        assert np.array_equal(a, b)
    assert DofMap(rep, 1).N == _free_dofs_formula(rep.meta["slabs"], 5)
    assert DofMap(rep, 0).N == DofMap(full, 0).N


def test_serving_families_are_seeded_and_bounded():
    a = W.serving_families(6, seed=9)
    b = W.serving_families(6, seed=9)
    assert [f.name for f in a] == [f.name for f in b]
    for f in a:
        assert f.dim in (2, 3) and 2 <= f.degree <= 6
