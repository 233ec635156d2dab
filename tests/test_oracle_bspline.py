"""Pins of the oracle's univariate spline machinery against textbook facts."""
from math import comb

import numpy as np
import pytest

from oracle import bspline

rng = np.random.default_rng(11)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("nel", [1, 3, 8])
def test_partition_of_unity_and_derivative_sum(p, nel):
    t = bspline.open_uniform_knots(p, nel)
    x = np.concatenate([rng.random(50), [0.0, 1.0, 0.5]])
    B = bspline.eval_basis(t, p, x)
    assert B.shape == (len(x), nel + p)
    assert np.all(B >= -1e-15)
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-14)
    for r in (1, 2):
        D = bspline.eval_basis(t, p, x, r)
        assert np.allclose(D.sum(axis=1), 0.0, atol=1e-9 * nel ** (r + 1) * p ** (2 * r))


def test_uniform_cubic_values_at_knots():
    # uniform cubic B-spline takes 1/6, 2/3, 1/6 at consecutive knots
    t = bspline.open_uniform_knots(3, 10)
    x = np.array([0.4, 0.5, 0.6])
    B = bspline.eval_basis(t, 3, x)
    centre = [i for i in range(B.shape[1]) if abs(B[1, i] - 2 / 3) < 1e-14]
    assert len(centre) == 1
    i = centre[0]
    assert np.allclose(B[:, i], [1 / 6, 2 / 3, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_bernstein_values_and_second_derivatives(p):
    # single element: the B-splines are the Bernstein polynomials
    t = np.r_[np.zeros(p + 1), np.ones(p + 1)]
    x = rng.random(20)
    for r in range(0, 3):
        B = bspline.eval_basis(t, p, x, r)
        for i in range(p + 1):
            poly = np.polynomial.Polynomial([comb(p, i)]) * \
                np.polynomial.Polynomial([0, 1]) ** i * np.polynomial.Polynomial([1, -1]) ** (p - i)
            assert np.allclose(B[:, i], poly.deriv(r)(x), atol=1e-12)


@pytest.mark.parametrize("nq", [1, 2, 3, 5, 7])
def test_gauss_exactness(nq):
    x, w = bspline.gauss_legendre(nq, 0.0, 2.0)
    for k in range(2 * nq):
        assert abs(np.sum(w * x ** k) - 2.0 ** (k + 1) / (k + 1)) < 1e-12 * 2.0 ** k
    k = 2 * nq
    assert abs(np.sum(w * x ** k) - 2.0 ** (k + 1) / (k + 1)) > 1e-8


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_mass_row_sums_are_integrals(p):
    t = bspline.open_uniform_knots(p, 7)
    M, K = bspline.mass_stiffness(t, p)
    n = M.shape[0]
    integrals = np.array([(t[i + p + 1] - t[i]) / (p + 1) for i in range(n)])
    assert np.allclose(M.sum(axis=1), integrals, atol=1e-15)
    assert np.allclose(K, K.T, atol=1e-12) and np.allclose(M, M.T, atol=1e-15)
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-10)
    assert np.all(np.linalg.eigvalsh(M) > 0)


def test_linear_closed_forms():
    nel = 5
    h = 1.0 / nel
    M, K = bspline.mass_stiffness(bspline.open_uniform_knots(1, nel), 1)
    Mx = np.diag(np.r_[1 / 3, [2 / 3] * (nel - 1), 1 / 3] * h) + np.diag([h / 6] * nel, 1) \
        + np.diag([h / 6] * nel, -1)
    Kx = (np.diag(np.r_[1, [2] * (nel - 1), 1]) - np.diag([1] * nel, 1) - np.diag([1] * nel, -1)) / h
    assert np.allclose(M, Mx, atol=1e-15)
    assert np.allclose(K, Kx, atol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_midpoint_refinement(p):
    assert np.allclose(bspline.insert_midpoints(bspline.open_uniform_knots(p, 3)),
                       bspline.open_uniform_knots(p, 6), rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_embedding(p):
    tc = bspline.open_uniform_knots(p, 4)
    tf = bspline.open_uniform_knots(p, 8)
    P = bspline.embedding(tc, tf, p)
    x = rng.random(40)
    # coarse functions are fine splines: pointwise identity away from the
    # collocation points used to build P
    assert np.allclose(bspline.eval_basis(tf, p, x) @ P, bspline.eval_basis(tc, p, x), atol=1e-13)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-14)
    # dyadic subdivision: an interior coarse function splits with the weights
    # 2^-p C(p+1, j), j = 0..p+1 (Lane-Riesenfeld)
    tc = bspline.open_uniform_knots(p, 8)
    tf = bspline.open_uniform_knots(p, 16)
    P = bspline.embedding(tc, tf, p)
    col = P[:, p]          # support [t_p, t_{2p+1}] = [0, (p+1)/8]: uniform knots
    nz = col[np.abs(col) > 1e-14]
    assert np.allclose(nz, [comb(p + 1, j) / 2 ** p for j in range(p + 2)], atol=1e-14)


def _graded_breaks(nel, seed):
    r = np.random.default_rng(seed)
    b = np.arange(nel + 1, dtype=np.float64) / nel
    b[1:-1] += r.uniform(-0.3, 0.3, size=nel - 1) / nel
    return b


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_nonuniform_knots_partition_integrals_and_embedding(p):
    # explicit coarsest breakpoints (Sec. 2 allows any open knot vector of
    # maximal smoothness): partition of unity, the closed-form integrals
    # int B_i = (t_{i+p+1} - t_i) / (p+1), and the refinement identity
    # B_fine P = B_coarse when every span is halved
    tc = bspline.open_knots(p, _graded_breaks(5, p))
    assert len(tc) == 5 + 1 + 2 * p
    x = np.concatenate([rng.random(60), [0.0, 1.0]])
    B = bspline.eval_basis(tc, p, x)
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-14)
    M, _ = bspline.mass_stiffness(tc, p)
    n = bspline.num_basis(tc, p)
    integrals = np.array([(tc[i + p + 1] - tc[i]) / (p + 1) for i in range(n)])
    assert np.allclose(M.sum(axis=1), integrals, atol=1e-14)
    tf = bspline.insert_midpoints(tc)
    spans_c = np.diff(np.unique(tc))
    spans_f = np.diff(np.unique(tf))
    assert np.allclose(spans_f, np.repeat(spans_c / 2, 2), atol=1e-15)
    P = bspline.embedding(tc, tf, p)
    assert np.allclose(bspline.eval_basis(tf, p, x) @ P, B, atol=1e-12)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
