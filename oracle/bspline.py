"""Univariate spline machinery of the oracle (Sec. 2: the space S_{p,h}(0,1)).

Test infrastructure only (see ``oracle/__init__``).

* open knot vectors of maximal smoothness C^{p-1} (Sec. 2), uniform or with
  given coarsest breakpoints, refined by halving every span (Sec. 3);
* all B-splines and their derivatives by the Cox-de Boor recursion;
* Gauss-Legendre quadrature per knot span;
* univariate mass and stiffness matrices (the M_l, K_l of the edge and face
  smoothers, Sec. 3);
* the canonical embedding between two nested spline spaces (the P_l of Sec. 3),
  obtained by interpolation at the fine Greville abscissae, not by knot
  insertion.

Pins (tests/test_oracle_bspline.py): partition of unity, closed-form cubic
values, integrals of B-splines, p=1 closed forms of M and K, Gauss exactness,
pointwise refinement identity and the dyadic subdivision stencil.
"""
import numpy as np


def open_uniform_knots(p, nel):
    """Open knot vector on [0,1]: p+1 repeated end knots and nel equal spans.

    Uniform grid size h = 1/nel and maximal smoothness C^{p-1} (Sec. 2).
    """
    inner = np.arange(1, nel, dtype=np.float64) / nel
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def open_knots(p, breaks):
    """Open knot vector with the given breakpoints (0 = x_0 < ... < x_nel = 1)
    as simple interior knots: maximal smoothness C^{p-1} (Sec. 2)."""
    b = np.asarray(breaks, dtype=np.float64)
    return np.concatenate([np.full(p, b[0]), b, np.full(p, b[-1])])


def level_knots(prob, level, k, c):
    """Knot vector of patch k in direction c on grid level ``level``: the
    coarsest breakpoints (uniform unless the problem gives them) with every
    span halved once per level (the uniform refinement of Sec. 3)."""
    p = prob.degree
    kn0 = getattr(prob, "knots0", None)
    if kn0 is None:
        return open_uniform_knots(p, int(prob.nel(level)[k][c]))
    t = open_knots(p, kn0[k][c])
    for _ in range(level):
        t = insert_midpoints(t)
    return t


def insert_midpoints(knots):
    """Uniform refinement: insert the midpoint of every non-empty span (Sec. 3)."""
    t = np.asarray(knots, dtype=np.float64)
    out = [t[0]]
    for a, b in zip(t[:-1], t[1:]):
        if b > a:
            out.append(0.5 * (a + b))
        out.append(b)
    return np.array(out)


def num_basis(knots, p):
    return len(knots) - p - 1


def eval_basis(knots, p, x, deriv=0):
    """All B-splines of degree p on ``knots`` (or their ``deriv``-th derivative) at x.

    Returns an array of shape (len(x), n).  Degree 0 functions are indicators
    of [t_i, t_{i+1}); at the right end x = t_last the last non-empty span is
    used, so values there are left limits.  Derivatives use
    B'_{i,p} = p (B_{i,p-1}/(t_{i+p}-t_i) - B_{i+1,p-1}/(t_{i+p+1}-t_{i+1})).
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if deriv > 0:
        if p == 0:
            return np.zeros((len(x), num_basis(t, 0)))
        low = eval_basis(t, p - 1, x, deriv - 1)
        n = num_basis(t, p)
        out = np.zeros((len(x), n))
        for i in range(n):
            d1 = t[i + p] - t[i]
            d2 = t[i + p + 1] - t[i + 1]
            if d1 > 0:
                out[:, i] += p * low[:, i] / d1
            if d2 > 0:
                out[:, i] -= p * low[:, i + 1] / d2
        return out
    m = len(t) - 1
    B = np.zeros((len(x), m))
    nonempty = [i for i in range(m) if t[i + 1] > t[i]]
    for i in nonempty:
        B[:, i] = ((x >= t[i]) & (x < t[i + 1])).astype(np.float64)
    B[x >= t[-1], nonempty[-1]] = 1.0
    for k in range(1, p + 1):
        Bn = np.zeros((len(x), m - k))
        for i in range(m - k):
            v = np.zeros(len(x))
            if t[i + k] > t[i]:
                v += (x - t[i]) / (t[i + k] - t[i]) * B[:, i]
            if t[i + k + 1] > t[i + 1]:
                v += (t[i + k + 1] - x) / (t[i + k + 1] - t[i + 1]) * B[:, i + 1]
            Bn[:, i] = v
        B = Bn
    return B


def gauss_legendre(nq, a=0.0, b=1.0):
    """nq-point Gauss-Legendre rule on [a, b] (exact for degree 2 nq - 1)."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (b - a) * xg + 0.5 * (b + a), 0.5 * (b - a) * wg


def span_quadrature(knots, nq):
    """Tensor of nq-point Gauss rules over every non-empty knot span, in order."""
    t = np.asarray(knots)
    xs, ws = [], []
    for a, b in zip(t[:-1], t[1:]):
        if b > a:
            x, w = gauss_legendre(nq, a, b)
            xs.append(x)
            ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def mass_stiffness(knots, p):
    """Univariate mass M_ij = int B_i B_j and stiffness K_ij = int B_i' B_j' on (0,1).

    (p+1) Gauss points per span integrate the degree-2p integrands exactly.
    """
    x, w = span_quadrature(knots, p + 1)
    B = eval_basis(knots, p, x)
    D = eval_basis(knots, p, x, 1)
    M = B.T @ (w[:, None] * B)
    K = D.T @ (w[:, None] * D)
    return M, K


def greville(knots, p):
    t = np.asarray(knots)
    n = num_basis(t, p)
    if p == 0:
        return 0.5 * (t[:n] + t[1:n + 1])
    return np.array([t[i + 1:i + p + 1].mean() for i in range(n)])


def embedding(knots_coarse, knots_fine, p):
    """Matrix P of the canonical embedding S(coarse) -> S(fine) (Sec. 3, P_l).

    Every coarse B-spline is a fine spline, B_c = B_f P.  P is found by
    interpolation at the fine Greville abscissae, where the fine collocation
    matrix is nonsingular (Schoenberg-Whitney).
    """
    g = greville(knots_fine, p)
    Bf = eval_basis(knots_fine, p, g)
    Bc = eval_basis(knots_coarse, p, g)
    P = np.linalg.solve(Bf, Bc)
    P[np.abs(P) < 1e-14] = 0.0
    return P
