"""Pins of the oracle's global dof numbering and piece splitting (Sec. 2, 3, 5)."""
import json
import os

import numpy as np
import pytest

from oracle.topology import DofMap, pieces
from oracle.multigrid import Level
from paper_1804_02539_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def fichera_cases():
    with open(os.path.join(GOLD, "fichera_dofs.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", [c for c in fichera_cases() if c["split"] <= 4],
                         ids=lambda c: f"K{7 * c['split'] ** 3}-l{c['l']}-p{c['p']}")
def test_fichera_dof_counts_match_paper(case):
    prob = W.fichera(case["p"], case["l"] + 1, split=case["split"])
    assert prob.npatch == 7 * case["split"] ** 3
    assert DofMap(prob, case["l"]).N == case["N"]


def test_config_dof_counts():
    # closed forms: C0 lines of patches, Dirichlet sides removed
    assert DofMap(W.unit_square_2x2(), 3).N == (2 * 17 + 1 - 2) ** 2          # 1089
    assert DofMap(W.square_4x4_bezier(), 5).N == (4 * 67 + 1 - 1) ** 2       # 71824
    dm = DofMap(W.cube_2x2x2_trilinear(levels=4), 3)                          # nel 8, p 3
    assert dm.N == (2 * 10 + 1 - 2) ** 3


def _flip_problem(d, orient):
    """Two patches glued along x; the second has its tangential axes reversed or
    swapped in its own parametrization, which the interface orientation undoes."""
    base = W.box_grid(d, [2] + [1] * (d - 1), 2, 2, 2, gdeg=1, dirichlet_sides=[0])
    ctrl = base.geo_ctrl[1].reshape([2] * d + [d])     # (.., y, x, coord)
    if d == 2:
        if orient & 2:
            ctrl = ctrl[::-1, :, :]                       # reverse y parameter
    else:
        if orient & 1:
            ctrl = np.swapaxes(ctrl, 0, 1)                # swap y and z parameters
        if orient & 2:
            # partner of side-a's t0 (=y) reversed: after a swap that axis is z'
            ax = 0 if orient & 1 else 1
            ctrl = np.flip(ctrl, axis=ax)
        if orient & 4:
            ax = 1 if orient & 1 else 0
            ctrl = np.flip(ctrl, axis=ax)
    base.geo_ctrl[1] = np.ascontiguousarray(ctrl).reshape(-1, d)
    base.iface[0, 4] = orient
    return base


@pytest.mark.parametrize("d,orient", [(2, 2), (3, 1), (3, 2), (3, 4), (3, 7)])
def test_interface_orientation(d, orient):
    # the glued operator must not depend on how patch 2 is parametrised: the
    # sorted spectrum of the global matrix equals the unflipped problem's
    ref = Level(_flip_problem(d, 0), 1, explicit=True)
    got = Level(_flip_problem(d, orient), 1, explicit=True)
    assert ref.N == got.N
    ev_ref = np.linalg.eigvalsh(ref.A.toarray())
    ev_got = np.linalg.eigvalsh(got.A.toarray())
    assert np.allclose(ev_ref, ev_got, atol=1e-12 * ev_ref.max())
    # a globally linear function has the same energy on both
    assert got.A.nnz == ref.A.nnz


def test_pieces_partition_square():
    dm = DofMap(W.unit_square_2x2(), 1)
    pcs = pieces(dm)
    kinds = sorted(pc.kind for pc in pcs)
    # 4 interiors, 4 interface edges (outer boundary is Dirichlet), 1 centre vertex
    assert kinds.count("interior") == 4 and kinds.count("edge") == 4 and kinds.count("vertex") == 1
    alld = np.concatenate([pc.dofs for pc in pcs])
    assert np.array_equal(np.sort(alld), np.arange(dm.N))
    centre = [pc for pc in pcs if pc.kind == "vertex"][0]
    assert len(centre.adjacent) == 4


def test_pieces_partition_cube_neumann():
    prob = W.box_grid(3, [2, 2, 2], 2, 1, 2, gdeg=1, dirichlet_sides=[0])
    dm = DofMap(prob, 1)
    pcs = pieces(dm)
    alld = np.concatenate([pc.dofs for pc in pcs])
    assert np.array_equal(np.sort(alld), np.arange(dm.N))
    kinds = [pc.kind for pc in pcs]
    # Neumann outer faces are pieces too; the x=0 side is eliminated
    assert kinds.count("interior") == 8
    assert kinds.count("vertex") == 27 - 9
    for pc in pcs:
        if pc.kind == "face":
            assert 1 <= len(pc.adjacent) <= 2
        if pc.kind == "edge":
            assert 1 <= len(pc.adjacent) <= 4
