"""Pins of the oracle's patch operators and transfers (Sec. 2, Sec. 3)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bspline, geometry
from oracle.assembly import PatchOp
from oracle.multigrid import Level, prolongation
from paper_1804_02539_amd import workloads as W

rng = np.random.default_rng(5)


def box_ctrl(lo, hi, d):
    return W._grid_ctrl(lo, hi, [1] * d)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_box_patch_is_kronecker_sum_2d(p):
    # an axis-parallel box [0,a]x[0,b]: a(u,v) = (b/a) K(x)M + (a/b) M(x)K in
    # parameter-domain 1D matrices (x direction fastest)
    a, b = 0.7, 1.9
    op = PatchOp([1, 1], box_ctrl([0.2, -1.0], [0.2 + a, -1.0 + b], 2), p, [3, 4])
    A = op.matrix().toarray()
    M0, K0 = bspline.mass_stiffness(op.knots[0], p)
    M1, K1 = bspline.mass_stiffness(op.knots[1], p)
    ref = (b / a) * np.kron(M1, K0) + (a / b) * np.kron(K1, M0)
    assert np.allclose(A, ref, atol=1e-12)


def test_box_patch_is_kronecker_sum_3d():
    a, b, c = 0.5, 1.5, 0.8
    p = 2
    op = PatchOp([1, 1, 1], box_ctrl([0, 0, 0], [a, b, c], 3), p, [2, 3, 2])
    A = op.matrix().toarray()
    Ms, Ks = zip(*[bspline.mass_stiffness(t, p) for t in op.knots])
    ref = (b * c / a) * np.kron(Ms[2], np.kron(Ms[1], Ks[0])) \
        + (a * c / b) * np.kron(Ms[2], np.kron(Ks[1], Ms[0])) \
        + (a * b / c) * np.kron(Ks[2], np.kron(Ms[1], Ms[0]))
    assert np.allclose(A, ref, atol=1e-12)


@pytest.mark.parametrize("p", [2, 4])
def test_symmetry_zero_rowsum_and_linear_energy_2d(p):
    prob = W.square_4x4_bezier(p=p, nel0=2, levels=2, seed=9)
    k = 5
    op = PatchOp(prob.geo_degree[k], prob.geo_ctrl[k], p, [4, 3])
    A = op.matrix().toarray()
    assert np.allclose(A, A.T, atol=1e-13)
    assert np.allclose(A.sum(axis=1), 0.0, atol=1e-12)          # constants in the kernel
    assert np.all(np.linalg.eigvalsh(A)[1:] > 1e-10)            # only constants
    # linear functions u = a.x lie in the isoparametric space; their energy is
    # |a|^2 * area, and the curved patch (straight edges) has the area w^2.
    # This fixes the metric |det J| J^{-1} J^{-T} (the transposed product fails).
    gx = [bspline.greville(t, p) for t in op.knots]
    X, _ = op.geo.eval_grid(gx)
    Bx = [bspline.eval_basis(t, p, g) for t, g in zip(op.knots, gx)]
    coll = np.kron(Bx[1], Bx[0])
    avec = np.array([0.3, -1.2])
    u = np.linalg.solve(coll, (X @ avec).reshape(-1))
    w = 0.25
    assert abs(u @ A @ u - avec @ avec * w * w) < 1e-12


def test_linear_energy_3d_trilinear():
    prob = W.cube_2x2x2_trilinear(p=2, nel0=1, levels=2, seed=3)
    k = 0
    op = PatchOp(prob.geo_degree[k], prob.geo_ctrl[k], 2, [2, 2, 3])
    A = op.matrix().toarray()
    assert np.allclose(A, A.T, atol=1e-13) and np.allclose(A.sum(axis=1), 0, atol=1e-12)
    gx = [bspline.greville(t, 2) for t in op.knots]
    X, _ = op.geo.eval_grid(gx)
    Bx = [bspline.eval_basis(t, 2, g) for t, g in zip(op.knots, gx)]
    coll = np.kron(Bx[2], np.kron(Bx[1], Bx[0]))
    avec = np.array([0.3, -1.2, 0.7])
    u = np.linalg.solve(coll, (X @ avec).reshape(-1))
    # volume of the patch by the divergence theorem is awkward; instead use that
    # the energy of a linear function equals |a|^2 times int det J, and int det J
    # is the load of f = 1 summed over the basis (partition of unity)
    vol = op.load(lambda Y: np.ones(Y.shape[:-1])).sum()
    assert abs(u @ A @ u - avec @ avec * vol) < 1e-12
    # the patch [0,.5]^3 with its corner (.5,.5,.5) moved by delta has volume
    # 1/8 + (delta_x + delta_y + delta_z)/8 * (1/2)^2 ... checked independently:
    # a trilinear hexahedron's volume is the mean of det J over the 2-point rule
    x2, w2 = bspline.gauss_legendre(2)
    _, J = op.geo.eval_grid([x2] * 3)
    vol2 = np.einsum("k,j,i,kji->", w2, w2, w2, np.linalg.det(J))
    assert abs(vol - vol2) < 1e-14


@pytest.mark.parametrize("make", [
    lambda: W.box_grid(2, [2, 3], 2, 1, 3, gdeg=1, dirichlet_sides=[0, 3]),
    lambda: W.box_grid(3, [2, 1, 2], 2, 1, 2, gdeg=1),
    lambda: W.box_grid(2, [2, 2], 4, 2, 2, gdeg=2, dirichlet_sides=[1]),
])
def test_galerkin_identity_affine(make):
    # nested spaces + exact quadrature on affine maps: P^T A_l P = A_{l-1}
    prob = make()
    levs = [Level(prob, l, explicit=True) for l in range(prob.levels)]
    for l in range(1, prob.levels):
        P = prolongation(prob, levs[l - 1], levs[l])
        G = (P.T @ levs[l].A @ P).toarray()
        assert np.allclose(G, levs[l - 1].A.toarray(), atol=1e-12 * abs(G).max())


def test_prolongation_reproduces_coarse_functions():
    # for a curved geometry the embedding is still exact in parameter space:
    # a coarse spline and its prolongation agree at random points of every patch
    prob = W.square_4x4_bezier(p=3, nel0=1, levels=2, seed=4)
    lc, lf = Level(prob, 0, explicit=True), Level(prob, 1, explicit=True)
    P = prolongation(prob, lc, lf)
    uc = rng.standard_normal(lc.N)
    uf = P @ uc
    xs = [rng.random(7), rng.random(5)]
    for k in range(prob.npatch):
        vc = lc.ops[k].eval_field(lc.S[k].T @ uc, xs)
        vf = lf.ops[k].eval_field(lf.S[k].T @ uf, xs)
        assert np.allclose(vc, vf, atol=1e-13)


def test_matrix_free_equals_explicit():
    prob = W.cube_2x2x2_trilinear(p=3, nel0=1, levels=3)
    le = Level(prob, 2, explicit=True)
    lm = Level(prob, 2, explicit=False)
    u = rng.standard_normal(le.N)
    assert np.allclose(le.apply(u), lm.apply(u), atol=1e-12 * np.abs(le.apply(u)).max())


def test_jacobian_convention():
    # G(x, y) = (2x + y, 3y): J = [[2, 1], [0, 3]] with J_ij = dG_i/dxi_j
    ctrl = np.array([[0, 0], [2, 0], [1, 3], [3, 3]], dtype=float)
    geo = geometry.BezierMap([1, 1], ctrl)
    _, J = geo.eval_grid([np.array([0.3]), np.array([0.6])])
    assert np.allclose(J[0, 0], [[2, 1], [0, 3]])
    assert abs(geometry.omega(geo) - 6 * np.trace(np.linalg.inv(J[0, 0]) @ np.linalg.inv(J[0, 0]).T) / 2) < 1e-13


def _plain_patch_matrix(gdeg, ctrl, p, nel):
    """A_k of Sec. 2 (the bilinear form a_k with the metric |det J| J^{-1} J^{-T})
    summed the plain way: element by element, Gauss point by Gauss point, pair
    of basis functions by pair.  Basis values, the geometry map and the Gauss
    rule come from scipy and numpy, not from the oracle's own routines."""
    import itertools
    from scipy.interpolate import BSpline
    d = len(nel)
    knots = [np.r_[np.zeros(p), np.linspace(0.0, 1.0, e + 1), np.ones(p)] for e in nel]
    nfun = [len(t) - p - 1 for t in knots]
    ctrl = np.asarray(ctrl, dtype=float).reshape([g + 1 for g in reversed(gdeg)] + [d])
    gk = [np.r_[np.zeros(g + 1), np.ones(g + 1)] for g in gdeg]

    def basis(c, i, x, nu):
        coef = np.zeros(nfun[c])
        coef[i] = 1.0
        return float(BSpline(knots[c], coef, p)(x, nu=nu))

    def bern(c, a, x, nu):
        coef = np.zeros(gdeg[c] + 1)
        coef[a] = 1.0
        return float(BSpline(gk[c], coef, gdeg[c])(x, nu=nu))

    def jacobian(xi):
        J = np.zeros((d, d))
        for idx in itertools.product(*[range(g + 1) for g in gdeg]):
            cp = ctrl[tuple(reversed(idx))]
            for j in range(d):
                w = 1.0
                for c in range(d):
                    w *= bern(c, idx[c], xi[c], 1 if c == j else 0)
                J[:, j] += cp * w
        return J

    gx, gw = np.polynomial.legendre.leggauss(p + 1)
    n_loc = int(np.prod(nfun))
    A = np.zeros((n_loc, n_loc))
    for el in itertools.product(*[range(e) for e in nel]):
        lo = [el[c] / nel[c] for c in range(d)]
        pts = [lo[c] + 0.5 * (gx + 1.0) / nel[c] for c in range(d)]
        wts = [0.5 * gw / nel[c] for c in range(d)]
        funs = [range(el[c], el[c] + p + 1) for c in range(d)]
        for qi in itertools.product(*[range(p + 1) for _ in range(d)]):
            xi = [pts[c][qi[c]] for c in range(d)]
            w = np.prod([wts[c][qi[c]] for c in range(d)])
            J = jacobian(xi)
            Ji = np.linalg.inv(J)
            G = abs(np.linalg.det(J)) * Ji @ Ji.T
            grads = {}
            for fi in itertools.product(*funs):
                g = np.ones(d)
                for a in range(d):
                    for c in range(d):
                        g[a] *= basis(c, fi[c], xi[c], 1 if c == a else 0)
                row = 0
                for c in reversed(range(d)):
                    row = row * nfun[c] + fi[c]
                grads[row] = g
            for i, gi in grads.items():
                for j, gj in grads.items():
                    A[i, j] += w * gi @ G @ gj
    return A


@pytest.mark.parametrize("case", ["2d_p2", "2d_p3", "3d_p2"])
def test_matrix_equals_plain_quadrature_loop(case):
    # the sum-factorised element contraction of PatchOp.matrix() against the
    # plain quadrature sum, on small curved patches
    if case.startswith("2d"):
        p = int(case[-1])
        prob = W.square_4x4_bezier(p=p, nel0=2, levels=2, seed=11)
        k, nel = 6, [2, 3]
    else:
        p = 2
        prob = W.cube_2x2x2_trilinear(p=p, levels=2, seed=13)
        k, nel = 7, [2, 1, 2]
    op = PatchOp(prob.geo_degree[k], prob.geo_ctrl[k], p, nel)
    ref = _plain_patch_matrix(prob.geo_degree[k], prob.geo_ctrl[k], p, nel)
    A = op.matrix().toarray()
    assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


def test_omega_of_boxes_closed_form():
    """The geometry scale of the alternative smoother reading on axis-aligned
    boxes, worked out by hand: |det J| = prod of the sides, J^{-1} J^{-T} =
    diag(side^-2), so omega = prod(s) * sum(s^-2) / d (the side length for a
    cube in 3D, 1 for any square in 2D)."""
    import itertools
    for sides in ([1.0, 2.0, 4.0], [0.25, 0.25, 0.25], [2.0, 3.0], [0.5, 0.5]):
        d = len(sides)
        corners = [np.array([s * c for s, c in zip(sides, idx[::-1])])
                   for idx in itertools.product([0, 1], repeat=d)]      # x fastest
        geo = geometry.BezierMap([1] * d, np.array(corners))
        expect = np.prod(sides) * sum(1.0 / s ** 2 for s in sides) / d
        assert abs(geometry.omega(geo) - expect) < 1e-13 * expect, (sides, geometry.omega(geo), expect)


def test_axis_lengths_closed_forms():
    """The mean physical length of each parameter direction (the physical-h
    reading): the sides of a box, and on a trapezoid with bottom a and top b,
    G(xi, eta) = (xi (a + (b - a) eta), eta), the x-length (a + b) / 2 and the
    y-length int_0^1 sqrt(1 + c^2 xi^2) dxi = sqrt(1 + c^2) / 2 + asinh(c) / (2 c),
    c = b - a."""
    import itertools
    for sides in ([1.0, 2.0, 4.0], [3.0, 0.5]):
        d = len(sides)
        corners = [np.array([s * c for s, c in zip(sides, idx[::-1])])
                   for idx in itertools.product([0, 1], repeat=d)]
        geo = geometry.BezierMap([1] * d, np.array(corners))
        assert np.allclose(geometry.axis_lengths(geo), sides, rtol=1e-13)
    a, b = 1.0, 2.5
    c = b - a
    geo = geometry.BezierMap([1, 1], np.array([[0.0, 0.0], [a, 0.0], [0.0, 1.0], [b, 1.0]]))
    lx, ly = geometry.axis_lengths(geo)
    assert abs(lx - (a + b) / 2) < 1e-13
    assert abs(ly - (np.sqrt(1 + c * c) / 2 + np.arcsinh(c) / (2 * c))) < 1e-9
