"""Pins of the oracle's smoother (Sec. 3): the fast-diagonalization form of the
subspace-corrected mass smoother against the literal additive sum over the
subspace products, symmetry, basis invariance and the subspace definition."""
import numpy as np
import pytest

from oracle import bspline
from oracle.smoother import (interior_1d, split_basis, literal_interior_inverse,
                             null_space, _modes)

rng = np.random.default_rng(7)


@pytest.mark.parametrize("p,nel", [(2, 8), (3, 2), (3, 8), (4, 4), (5, 2), (5, 16), (6, 3), (6, 8)])
def test_split_basis_orthonormality_and_subspace(p, nel):
    Mi, Ki, C = interior_1d(p, bspline.open_uniform_knots(p, nel))
    sigma = 5.0 * nel * nel
    U, mu, k0, Z = split_basis(Mi, Ki, C, sigma)
    m = Mi.shape[0]
    assert U.shape == (m, m)
    assert np.allclose(U.T @ Mi @ U, np.eye(m), atol=1e-10)
    # first k0 columns lie in S~: every constraint (even derivative at the ends) vanishes
    t = bspline.open_uniform_knots(p, nel)
    for l in range(1, (p + 1) // 2):
        if 2 * l >= p:
            break
        for x in (0.0, 1.0):
            row = bspline.eval_basis(t, p, [x], 2 * l)[0, 1:-1]
            assert np.allclose(row @ U[:, :k0], 0.0, atol=1e-8 * np.abs(row).max())
    # on the complement the columns diagonalise K
    KU = U[:, k0:].T @ Ki @ U[:, k0:]
    assert np.allclose(KU, np.diag(mu[k0:]), atol=1e-8 * max(1.0, np.abs(mu).max()))
    assert np.all(mu[:k0] == sigma)
    # generic dimension count on fine grids: S1 has dim 2*floor((p-1)/2)
    if m >= 2 * p:
        assert m - k0 == 2 * ((p - 1) // 2)


@pytest.mark.parametrize("dims", [[(2, 4), (2, 3)], [(4, 3), (4, 2)], [(3, 2), (3, 2), (3, 3)],
                                  [(5, 2), (5, 4)], [(6, 2), (6, 2), (6, 2)]])
def test_fd_equals_literal_additive_sum(dims):
    Mis, Kis, Cs, sig, Us, mus = [], [], [], [], [], []
    for p, nel in dims:
        Mi, Ki, C = interior_1d(p, bspline.open_uniform_knots(p, nel))
        s = 5.0 * nel * nel
        U, mu, _, _ = split_basis(Mi, Ki, C, s)
        Mis.append(Mi); Kis.append(Ki); Cs.append(C); sig.append(s); Us.append(U); mus.append(mu)
    om = 0.73
    ref = literal_interior_inverse(Mis, Kis, Cs, sig, om)
    d = len(dims)
    D = om * sum(np.meshgrid(*[mu for mu in reversed(mus)], indexing="ij")[d - 1 - c]
                 for c in range(d))
    n = ref.shape[0]
    shape = [U.shape[0] for U in reversed(Us)]
    fd = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        T = _modes(e.reshape(shape), Us, transpose=True) / D
        fd[:, j] = _modes(T, Us, transpose=False).reshape(-1)
    assert np.allclose(fd, ref, atol=1e-10 * np.abs(ref).max())
    assert np.allclose(fd, fd.T, atol=1e-12 * np.abs(fd).max())
    assert np.all(np.linalg.eigvalsh(fd) > 0)


def test_fd_independent_of_basis_within_subspace():
    p, nel = 5, 8
    Mi, Ki, C = interior_1d(p, bspline.open_uniform_knots(p, nel))
    U, mu, k0, _ = split_basis(Mi, Ki, C, 5.0 * nel * nel)
    Q, _ = np.linalg.qr(rng.standard_normal((k0, k0)))
    U2 = U.copy()
    U2[:, :k0] = U[:, :k0] @ Q          # another M-orthonormal basis of S~
    U2[:, k0:] *= -1.0                  # and opposite eigenvector signs
    A = U @ np.diag(1 / mu) @ U.T
    B = U2 @ np.diag(1 / mu) @ U2.T
    assert np.allclose(A, B, atol=1e-12 * np.abs(A).max())


def test_null_space_rank_gap():
    # the subspace dimension decision must be clear-cut for every size used: no
    # relative singular value between 1e-13 and 1e-4, so any threshold in that
    # window (the oracle cuts at 1e-10, a Gram-matrix route needs ~1e-5) agrees
    for p in range(2, 9):
        for nel in [1, 2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48, 64, 96]:
            Mi, Ki, C = interior_1d(p, bspline.open_uniform_knots(p, nel))
            if C.shape[0] == 0:
                continue
            s = np.linalg.svd(C / np.linalg.norm(C, axis=1, keepdims=True), compute_uv=False)
            small = s[s <= 1e-10 * s[0]]
            big = s[s > 1e-10 * s[0]]
            assert small.size == 0 or small.max() < 1e-13 * s[0]
            assert big.min() > 1e-4 * s[0]


@pytest.mark.parametrize("make", [lambda: __import__("paper_1804_02539_amd.workloads", fromlist=["x"]).fichera(2, 3),
                                  lambda: __import__("paper_1804_02539_amd.workloads", fromlist=["x"]).square_4x4_bezier(p=3, levels=3)])
def test_direct_edge_and_vertex_pieces_solve_the_restriction(make):
    # the variant of Sec. 3 (its reference's direct solvers): on an edge or a
    # vertex T the smoother solves A_l[T, T] z_T = r_T exactly.  Checked with
    # the patch-wise matrix-free apply of the level (not the matrix the
    # smoother sliced), on a vector supported on one piece.
    from oracle.multigrid import Hierarchy
    prob = make()
    H = Hierarchy(prob, reading={"edges": "direct"})
    lev = H.finest
    kinds = {"edge": 0, "vertex": 0}
    for pc in lev.pieces:
        if pc.kind not in kinds or kinds[pc.kind] >= 3:
            continue
        kinds[pc.kind] += 1
        r = np.zeros(lev.N)
        r[pc.dofs] = rng.standard_normal(len(pc.dofs))
        z = lev.smoother.apply(r)
        assert np.count_nonzero(z) <= len(pc.dofs)
        Az = np.zeros(lev.N)
        for S, op in zip(lev.S, lev.ops):
            Az += S @ op.apply(S.T @ z)
        assert np.abs(Az[pc.dofs] - r[pc.dofs]).max() <= 1e-10 * np.abs(r).max()
    assert kinds["edge"] > 0 and kinds["vertex"] > 0
