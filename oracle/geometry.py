"""Patch geometry maps G_k : (0,1)^d -> Omega_k of the oracle (Sec. 2).

Test infrastructure only.  Each patch map is one tensor-product Bezier element
of degree g_c in direction c (the Bernstein basis is the B-spline basis on the
knot vector [0]*(g+1) + [1]*(g+1)).  Jacobian convention: J_ij = dG_i/dxi_j.
"""
import numpy as np

from . import bspline


class BezierMap:
    def __init__(self, degrees, ctrl):
        self.deg = [int(g) for g in degrees]
        self.d = len(self.deg)
        self.ctrl = np.asarray(ctrl, dtype=np.float64).reshape(
            [g + 1 for g in reversed(self.deg)] + [self.d])   # (.., y, x, coord)

    def _bern(self, c, x, deriv):
        g = self.deg[c]
        return bspline.eval_basis(np.r_[np.zeros(g + 1), np.ones(g + 1)], g, x, deriv)

    def eval_grid(self, xs):
        """Map and Jacobian on the tensor grid xs[0] x xs[1] (x xs[2]).

        Returns X with shape (Q_{d-1}, .., Q_0, d) and J with shape (.., d, d),
        J[..., i, j] = dG_i/dxi_j, arrays ordered like the x-fastest layout.
        """
        d = self.d
        vals = [self._bern(c, xs[c], 0) for c in range(d)]
        ders = [self._bern(c, xs[c], 1) for c in range(d)]
        if d == 2:
            X = np.einsum("bj,ai,jic->bac", vals[1], vals[0], self.ctrl)
            J = np.empty(X.shape[:2] + (2, 2))
            J[..., :, 0] = np.einsum("bj,ai,jic->bac", vals[1], ders[0], self.ctrl)
            J[..., :, 1] = np.einsum("bj,ai,jic->bac", ders[1], vals[0], self.ctrl)
        else:
            X = np.einsum("ck,bj,ai,kjix->cbax", vals[2], vals[1], vals[0], self.ctrl)
            J = np.empty(X.shape[:3] + (3, 3))
            J[..., :, 0] = np.einsum("ck,bj,ai,kjix->cbax", vals[2], vals[1], ders[0], self.ctrl)
            J[..., :, 1] = np.einsum("ck,bj,ai,kjix->cbax", vals[2], ders[1], vals[0], self.ctrl)
            J[..., :, 2] = np.einsum("ck,bj,ai,kjix->cbax", ders[2], vals[1], vals[0], self.ctrl)
        return X, J


def metric(J):
    """|det J| J^{-1} J^{-T} and det J at every point (eq. of the bilinear form a_k).

    Reading: the paper prints the metric as |det J| J^{-T} J^{-1}; with the
    convention J_ij = dG_i/dxi_j the gradient transforms as grad u = J^{-T}
    grad_xi u, which gives J^{-1} J^{-T}.
    """
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    G = np.abs(det)[..., None, None] * (Jinv @ np.swapaxes(Jinv, -1, -2))
    return G, det


def omega(geo, nq=8):
    """Geometry scale of a patch: the parameter-domain average of
    |det J| tr(J^{-1} J^{-T}) / d with the nq-point Gauss rule per direction.

    Used by the alternative reading (omega = "mean") of Sec. 2's remark that
    the physical and parameter-domain Laplacians agree up to factors that
    depend on the geometry: every piece operator of the smoother is then
    multiplied by this constant (1 for any square in 2D, the side length for a
    cube in 3D).  The default reading takes omega = 1.
    """
    x, w = bspline.gauss_legendre(nq)
    _, J = geo.eval_grid([x] * geo.d)
    G, _ = metric(J)
    tr = np.trace(G, axis1=-2, axis2=-1) / geo.d
    W = w
    for _ in range(geo.d - 1):
        W = np.multiply.outer(w, W)
    return float(np.sum(W * tr))


def axis_lengths(geo, nq=8):
    """Mean physical length of each parameter direction of a patch: the
    parameter-domain average of |dG/dxi_c| (the c-th Jacobian column), with the
    nq-point Gauss rule per direction.  Used by the physical-h reading of the
    smoother (h_c = length_c / nel_c)."""
    x, w = bspline.gauss_legendre(nq)
    _, J = geo.eval_grid([x] * geo.d)
    W = w
    for _ in range(geo.d - 1):
        W = np.multiply.outer(w, W)
    return [float(np.sum(W * np.linalg.norm(J[..., :, c], axis=-1))) for c in range(geo.d)]
