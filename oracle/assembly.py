"""Patch-local Galerkin operators of the oracle (Sec. 2, eq. of a_k, and Sec. 4).

Test infrastructure only.

For patch k the matrix A_k has entries
    A_k[i, j] = sum_q w_q grad B_i(xi_q)^T (|det J| J^{-1} J^{-T})(xi_q) grad B_j(xi_q)
over the tensor Gauss rule with (p+1) points per span and direction (reading:
the paper does not name a rule; p+1 points integrate the affine case exactly).
It is the full patch matrix including the boundary layers, i.e. before any
Dirichlet elimination (the per-patch matrices A_{l,k} of Sec. 4).

Two evaluations of the same sum are provided:
* ``PatchOp.matrix()`` builds A_k explicitly, element by element (sum-factorised
  over the tensor quadrature of each element);
* ``PatchOp.apply(u)`` evaluates A_k u without forming A_k (same quadrature, used
  for sizes whose explicit matrix does not fit).
Pins: symmetry, zero row sums, the Kronecker form K(x)M + M(x)K for identity maps,
the Galerkin identity P^T A_l P = A_{l-1} for affine maps, and agreement of the
two evaluations (tests/test_oracle_assembly.py).
"""
import numpy as np
import scipy.sparse as sp

from . import bspline
from .geometry import BezierMap, metric


class PatchOp:
    def __init__(self, degrees_geo, ctrl, p, nel, nq=None, knots=None):
        self.d = len(nel)
        self.p = p
        self.nel = [int(e) for e in nel]
        self.geo = BezierMap(degrees_geo, ctrl)
        nq = p + 1 if nq is None else nq
        if knots is None:
            knots = [bspline.open_uniform_knots(p, e) for e in self.nel]
        self.knots = [np.asarray(t, dtype=np.float64) for t in knots]
        self.n = [bspline.num_basis(t, p) for t in self.knots]
        self.quad = [bspline.span_quadrature(t, nq) for t in self.knots]
        self.B = [bspline.eval_basis(t, p, q[0]) for t, q in zip(self.knots, self.quad)]
        self.D = [bspline.eval_basis(t, p, q[0], 1) for t, q in zip(self.knots, self.quad)]
        _, J = self.geo.eval_grid([q[0] for q in self.quad])
        G, det = metric(J)
        # G_k is only required to be bijective (Sec. 2): det J may have either
        # sign but must not vanish or change sign; |det J| enters a_k
        if not (np.all(det > 0) or np.all(det < 0)):
            raise ValueError("geometry map is singular or folds (det J changes sign)")
        W = self.quad[0][1]
        for c in range(1, self.d):
            W = np.multiply.outer(self.quad[c][1], W)
        self.W = W                       # quadrature weights on the grid, (.., Q1, Q0)
        self.det = det
        self.G = G * W[..., None, None]  # weighted metric

    @property
    def size(self):
        return int(np.prod(self.n))

    def _factors(self, a):
        """1D factors of the a-th gradient component (derivative in direction a)."""
        return [self.D[c] if c == a else self.B[c] for c in range(self.d)]

    def _element_tables(self, c, deriv):
        """Values (or derivatives) of the p+1 functions living on each span of
        direction c at that span's quadrature points: shape (nel, nq, p+1)."""
        nq = len(self.quad[c][0]) // self.nel[c]
        X = self.D[c] if deriv else self.B[c]
        out = np.empty((self.nel[c], nq, self.p + 1))
        for e in range(self.nel[c]):
            out[e] = X[e * nq:(e + 1) * nq, e:e + self.p + 1]
        return out

    def matrix(self):
        """Explicit sparse A_k (all local functions, boundary layers included),
        summed element by element over the same quadrature.

        The tensor quadrature of each element is contracted one direction at a
        time (direction 0 first), so the element matrices come out with axes
        (E_{d-1}, .., E_0, i_0, j_0, .., i_{d-1}, j_{d-1}).
        """
        d, p = self.d, self.p
        q = p + 1
        nq = len(self.quad[0][0]) // self.nel[0]
        tabs = [[self._element_tables(c, 0), self._element_tables(c, 1)] for c in range(d)]
        shape = []
        for c in reversed(range(d)):
            shape += [self.nel[c], nq]
        E = 0
        for a in range(d):
            for b in range(d):
                T = self.G[..., a, b].reshape(shape)     # (E_{d-1}, q_{d-1}, .., E_0, q_0)
                for c in range(d):
                    Xa = tabs[c][1 if c == a else 0]
                    Xb = tabs[c][1 if c == b else 0]
                    XX = (Xa[:, :, :, None] * Xb[:, :, None, :]).reshape(self.nel[c], nq, q * q)
                    # T axes: (E, q) pairs of directions c..d-1 (slowest first), the
                    # element axes already done, their (i, j) blocks.  Bring E_c to
                    # the front as the batch axis and q_c to the back.
                    ax_e = 2 * (d - 1 - c)
                    ax_q = ax_e + 1
                    rest = [x for x in range(T.ndim) if x not in (ax_e, ax_q)]
                    Tt = np.transpose(T, [ax_e] + rest + [ax_q])
                    rshape = Tt.shape[1:-1]
                    R = np.matmul(Tt.reshape(self.nel[c], -1, nq), XX)
                    R = R.reshape((self.nel[c],) + rshape + (q * q,))
                    # E_c joins the block of processed element axes
                    nd = R.ndim
                    n_front = 2 * (d - 1 - c)          # remaining (E, q) axes
                    order = list(range(1, 1 + n_front)) + [0] + list(range(1 + n_front, nd))
                    T = np.transpose(R, order)
                E = E + T
        n = self.n
        nel = self.nel
        Es = np.meshgrid(*[np.arange(nel[c]) for c in reversed(range(d))], indexing="ij")
        ids = np.meshgrid(*[np.arange(q) for _ in range(2 * d)], indexing="ij")
        # axes of E: (E_{d-1}, .., E_0, i_0, j_0, .., i_{d-1}, j_{d-1})
        ebase = []
        for c in range(d):
            ebase.append(Es[d - 1 - c].reshape(Es[0].shape + (1,) * (2 * d)))
        rows = 0
        cols = 0
        stride = 1
        for c in range(d):
            ic = ids[2 * c].reshape((1,) * d + ids[0].shape)
            jc = ids[2 * c + 1].reshape((1,) * d + ids[0].shape)
            rows = rows + (ebase[c] + ic) * stride
            cols = cols + (ebase[c] + jc) * stride
            stride *= n[c]
        Eflat = E.reshape(tuple(nel[c] for c in reversed(range(d))) + (q,) * (2 * d))
        rows = np.broadcast_to(rows, Eflat.shape).reshape(-1)
        cols = np.broadcast_to(cols, Eflat.shape).reshape(-1)
        N = self.size
        return sp.csr_matrix((Eflat.reshape(-1), (rows, cols)), shape=(N, N))

    def _forward(self, mats, U):
        if self.d == 2:
            return np.einsum("bj,ai,ji->ba", mats[1], mats[0], U, optimize=True)
        return np.einsum("ck,bj,ai,kji->cba", mats[2], mats[1], mats[0], U, optimize=True)

    def _backward(self, mats, V):
        if self.d == 2:
            return np.einsum("bj,ai,ba->ji", mats[1], mats[0], V, optimize=True)
        return np.einsum("ck,bj,ai,cba->kji", mats[2], mats[1], mats[0], V, optimize=True)

    def apply(self, u):
        """A_k u by the same quadrature sum, without forming A_k."""
        d = self.d
        U = np.asarray(u, dtype=np.float64).reshape(list(reversed(self.n)))
        grads = [self._forward(self._factors(b), U) for b in range(d)]
        out = np.zeros_like(U)
        for a in range(d):
            flux = sum(self.G[..., a, b] * grads[b] for b in range(d))
            out += self._backward(self._factors(a), flux)
        return out.reshape(-1)

    def load(self, fun):
        """Load vector f_k[i] = sum_q w_q f(G_k(xi_q)) B_i(xi_q) |det J|."""
        X, _ = self.geo.eval_grid([q[0] for q in self.quad])
        vals = fun(X) * np.abs(self.det) * self.W
        return self._backward(self.B, vals).reshape(-1)

    def eval_field(self, u, xs, deriv=None):
        """Values of the spline with coefficients u at the tensor grid xs
        (or its derivative in direction ``deriv`` in parameter space)."""
        mats = []
        for c in range(self.d):
            mats.append(bspline.eval_basis(self.knots[c], self.p, xs[c],
                                           1 if deriv == c else 0))
        U = np.asarray(u, dtype=np.float64).reshape(list(reversed(self.n)))
        return self._forward(mats, U)


def sine_source(amp, freq):
    """f(x) = amp * prod_c sin(freq * pi * x_c) (the right-hand sides of Sec. 5 and
    of the manufactured-solution workloads)."""
    def f(X):
        out = amp * np.ones(X.shape[:-1])
        for c in range(X.shape[-1]):
            out = out * np.sin(freq * np.pi * X[..., c])
        return out
    return f
