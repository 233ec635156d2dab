"""Multigrid hierarchy, V-cycle and PCG of the oracle (Sec. 3, Sec. 4, Algorithm 1).

Test infrastructure only.  Works on global free-dof vectors; the accumulation
Sigma and the restriction chi of Algorithm 1 are the identity there (they are
the parallel bookkeeping of distributed vectors).

Readings:
* the coarse-grid correction is undamped, as in Algorithm 1 (the prose version
  in Sec. 3 carries a factor tau);
* coarse operators are re-discretised on every level (for affine maps this is
  identical to P^T A P, a pinned test);
* the stopping test of the PCG is ||f - A u||_2 <= tol ||f||_2 on the free dofs,
  starting from u = 0 (Sec. 5 solves to a relative accuracy of 1e-8).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import bspline, geometry
from .assembly import PatchOp, sine_source
from .smoother import Smoother
from .topology import DofMap, pieces


EXPLICIT_LIMIT = 120_000   # local rows up to which a level's matrix is formed


class Level:
    def __init__(self, prob, level, explicit=None, sigma_scale=5.0, reading=None):
        self.level = level
        self.dm = DofMap(prob, level)
        self.N = self.dm.N
        nel = prob.nel(level)
        self.knots = [[bspline.level_knots(prob, level, k, c) for c in range(prob.dim)]
                      for k in range(prob.npatch)]
        self.ops = [PatchOp(prob.geo_degree[k], prob.geo_ctrl[k], prob.degree, nel[k], knots=self.knots[k])
                    for k in range(prob.npatch)]
        self.S = [self.dm.selection(k) for k in range(prob.npatch)]
        if explicit is None:
            explicit = sum(self.dm.size) <= EXPLICIT_LIMIT
        self.A = None
        if explicit:
            A = None
            for S, op in zip(self.S, self.ops):
                t = S @ op.matrix() @ S.T
                A = t if A is None else A + t
            self.A = A.tocsr()
        omegas = [geometry.omega(op.geo) for op in self.ops]
        self.omegas = omegas
        self.lengths = [geometry.axis_lengths(op.geo) for op in self.ops]
        self.pieces = pieces(self.dm)
        self.prob = prob
        self.sigma_scale = sigma_scale
        self.set_reading(reading)

    def set_reading(self, reading):
        """(Re)build the smoother under a reading of its constants (see oracle.smoother)."""
        self.smoother = Smoother(self.prob, self.level, self.dm, self.pieces, self.omegas,
                                 self.sigma_scale, reading=reading, lengths=self.lengths, knots=self.knots,
                                 restrict=self.restricted)

    def restricted(self, dofs):
        """The restriction A_l[dofs, dofs] of the level's matrix to a set of
        free dofs (dense)."""
        dofs = np.asarray(dofs)
        if self.A is not None:
            return self.A[dofs][:, dofs].toarray()
        out = np.zeros((len(dofs), len(dofs)))
        for j, g in enumerate(dofs):
            e = np.zeros(self.N)
            e[g] = 1.0
            out[:, j] = self.apply(e)[dofs]
        return out

    def apply(self, u):
        """A_l u (eq. of the linear system) on free dofs."""
        if self.A is not None:
            return self.A @ u
        out = np.zeros(self.N)
        for S, op in zip(self.S, self.ops):
            out += S @ op.apply(S.T @ u)
        return out

    def load(self, fun):
        out = np.zeros(self.N)
        for S, op in zip(self.S, self.ops):
            out += S @ op.load(fun)
        return out


def prolongation(prob, coarse, fine):
    """Global P_l (N_fine x N_coarse): the canonical embedding V_{l-1} -> V_l of Sec. 3.

    Per patch it is the Kronecker product of the 1D embeddings; the row of a fine
    dof shared by several patches is taken from the first patch holding it (all
    agree, Sec. 4, block-triangular structure of the transfer).
    """
    p = prob.degree
    rows, cols, vals = [], [], []
    done = np.zeros(fine.N, dtype=bool)
    for k in range(prob.npatch):
        Ps = []
        for c in range(prob.dim):
            tc = coarse.knots[k][c]
            tf = fine.knots[k][c]
            Ps.append(sp.csr_matrix(bspline.embedding(tc, tf, p)))
        Pk = Ps[0]
        for Pc in Ps[1:]:
            Pk = sp.kron(Pc, Pk, format="csr")
        gf = fine.dm.patch_gid(k)
        gc = coarse.dm.patch_gid(k)
        Pk = Pk.tocoo()
        take = (gf[Pk.row] >= 0) & (gc[Pk.col] >= 0) & (~done[np.maximum(gf[Pk.row], 0)])
        rows.append(gf[Pk.row[take]])
        cols.append(gc[Pk.col[take]])
        vals.append(Pk.data[take])
        done[gf[gf >= 0]] = True
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.N, coarse.N))
    return P


class Hierarchy:
    def __init__(self, prob, tau=0.25, nu=1, mu=1, sigma_scale=5.0, explicit=None, reading=None):
        self.prob = prob
        self.tau, self.nu, self.mu = tau, nu, mu
        self.levels = [Level(prob, l, explicit=(True if l == 0 else explicit),
                             sigma_scale=sigma_scale, reading=reading)
                       for l in range(prob.levels)]
        self.P = [None] + [prolongation(prob, self.levels[l - 1], self.levels[l])
                           for l in range(1, prob.levels)]
        A0 = self.levels[0].A.toarray()
        self.coarse_factor = sla.cho_factor(A0, lower=True)

    def set_reading(self, reading):
        """Rebuild every level's smoother under another reading of its constants."""
        for lev in self.levels:
            lev.set_reading(reading)

    @property
    def finest(self):
        return self.levels[-1]

    def coarse_solve(self, r):
        """Exact solve with A_0 (Sec. 4, the global direct solver on level 0)."""
        return sla.cho_solve(self.coarse_factor, r)

    def smooth(self, l, u, f):
        """One smoothing step u <- u + tau L^{-1} (f - A u) (eq. of the smoothing step)."""
        lev = self.levels[l]
        return u + self.tau * lev.smoother.apply(f - lev.apply(u))

    def cycle(self, l, u, f):
        """Algorithm 1 on level l >= 1."""
        lev = self.levels[l]
        for _ in range(self.nu):
            u = self.smooth(l, u, f)
        r = self.P[l].T @ (f - lev.apply(u))
        if l == 1:
            pc = self.coarse_solve(r)
        else:
            pc = np.zeros(self.levels[l - 1].N)
            for _ in range(self.mu):
                pc = self.cycle(l - 1, pc, r)
        u = u + self.P[l] @ pc
        for _ in range(self.nu):
            u = self.smooth(l, u, f)
        return u

    def vcycle(self, r):
        """One cycle with zero initial guess on the finest level: the preconditioner."""
        L = len(self.levels) - 1
        return self.cycle(L, np.zeros(self.levels[L].N), r)

    def pcg(self, f, tol=1e-8, maxit=500):
        """Preconditioned CG from u = 0 with one cycle as preconditioner (Sec. 4)."""
        lev = self.finest
        u = np.zeros(lev.N)
        r = f.copy()
        nf = np.linalg.norm(f)
        hist = [1.0]
        if nf == 0:
            return u, 0, hist
        z = self.vcycle(r)
        p = z.copy()
        rho = r @ z
        for it in range(1, maxit + 1):
            q = lev.apply(p)
            alpha = rho / (p @ q)
            u += alpha * p
            r -= alpha * q
            rel = np.linalg.norm(r) / nf
            hist.append(rel)
            if rel <= tol:
                return u, it, hist
            z = self.vcycle(r)
            rho_new = r @ z
            p = z + (rho_new / rho) * p
            rho = rho_new
        return u, maxit, hist


def load_vector(prob, level_obj):
    src = prob.meta.get("source")
    kind = src[0]
    if kind != "sine":
        raise ValueError("load vectors exist for sine sources only")
    return level_obj.load(sine_source(src[1], src[2]))
