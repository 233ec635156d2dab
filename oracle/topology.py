"""Global degrees of freedom and pieces of the oracle (Sec. 2 and Sec. 3).

Test infrastructure only.

* ``DofMap``: the C0 multi-patch space V_l (eq. of V_l): boundary-layer
  functions of two matching sides are one global function; functions on a
  Dirichlet side are eliminated.  Global free numbering: sweep the patches in
  order and their local functions x-fastest; a function gets the next number
  the first time its class is met.
* ``pieces``: the splitting of Sec. 3 into patch interiors, faces (3D), edges
  and vertices, each free degree of freedom in exactly one piece.  A local
  function of patch k belongs to the entity given by the set of directions in
  which its index sits on the patch boundary (none: interior; one: side; ...).

Pins: the DOF counts of the paper's Fichera corner tables (Sec. 5) and the
piece partition invariants (tests/test_oracle_topology.py).
"""
import itertools

import numpy as np


def _side_layer(n, side):
    """Local flat indices of the layer on side ``side`` of a patch with sizes n,
    indexed by the tangential indices: shape (n_t0,) in 2D, (n_t1, n_t0) in 3D
    where t0 < t1 are the tangential directions."""
    d = len(n)
    c, end = divmod(side, 2)
    tang = [a for a in range(d) if a != c]
    fix = 0 if end == 0 else n[c] - 1
    strides = [int(np.prod(n[:a])) for a in range(d)]
    if d == 2:
        t0 = tang[0]
        return np.array([fix * strides[c] + j * strides[t0] for j in range(n[t0])])
    t0, t1 = tang
    out = np.empty((n[t1], n[t0]), dtype=np.int64)
    for j1 in range(n[t1]):
        for j0 in range(n[t0]):
            out[j1, j0] = fix * strides[c] + j0 * strides[t0] + j1 * strides[t1]
    return out


def _oriented(layer_b, orient, d):
    """Re-index side b's layer by side a's tangential indices (see workloads for the
    orientation convention)."""
    if d == 2:
        return layer_b[::-1] if orient & 2 else layer_b
    L = layer_b                        # indexed [u1, u0]
    if orient & 1:
        L = L.T                        # now [u0, u1]: a.t0 pairs u1, a.t1 pairs u0
    # L is indexed [partner of t1, partner of t0]
    if orient & 2:
        L = L[:, ::-1]
    if orient & 4:
        L = L[::-1, :]
    return L


class DofMap:
    def __init__(self, prob, level):
        d = prob.dim
        p = prob.degree
        K = prob.npatch
        self.d, self.K = d, K
        self.n = [[int(e) + p for e in row] for row in prob.nel(level)]
        self.size = [int(np.prod(nk)) for nk in self.n]
        self.off = np.concatenate([[0], np.cumsum(self.size)]).astype(np.int64)
        tot = int(self.off[-1])
        parent = np.arange(tot)

        def find(x):
            r = x
            while parent[r] != r:
                r = parent[r]
            while parent[x] != r:
                parent[x], x = r, parent[x]
            return r

        for a, sa, b, sb, orient in prob.iface:
            la = _side_layer(self.n[a], sa)
            lb = _oriented(_side_layer(self.n[b], sb), orient, d)
            if la.shape != lb.shape:
                raise ValueError("non-matching interface")
            for x, y in zip((la + self.off[a]).ravel(), (lb + self.off[b]).ravel()):
                rx, ry = find(x), find(y)
                if rx != ry:
                    parent[max(rx, ry)] = min(rx, ry)
        roots = np.array([find(x) for x in range(tot)])
        iface_sides = {(int(a), int(sa)) for a, sa, _, _, _ in prob.iface}
        iface_sides |= {(int(b), int(sb)) for _, _, b, sb, _ in prob.iface}
        dirich = np.zeros(tot, dtype=bool)
        for k in range(K):
            for s in range(2 * d):
                if prob.bc[k, s] == 1 and (k, s) not in iface_sides:
                    dirich[_side_layer(self.n[k], s).ravel() + self.off[k]] = True
        dir_root = np.zeros(tot, dtype=bool)
        dir_root[roots[dirich]] = True
        gid = -np.ones(tot, dtype=np.int64)
        number = {}
        for x in range(tot):
            r = roots[x]
            if dir_root[r]:
                continue
            if r not in number:
                number[r] = len(number)
            gid[x] = number[r]
        self.gid = gid                      # flat local (over all patches) -> global free id
        self.N = len(number)
        self.copies = [[] for _ in range(self.N)]
        for x in range(tot):
            if gid[x] >= 0:
                self.copies[gid[x]].append(x)

    def patch_gid(self, k):
        return self.gid[self.off[k]:self.off[k + 1]]

    def local_index(self, x):
        """(patch, tensor index) of a flat local position."""
        k = int(np.searchsorted(self.off, x, side="right") - 1)
        r = int(x - self.off[k])
        idx = []
        for c in range(self.d):
            idx.append(r % self.n[k][c])
            r //= self.n[k][c]
        return k, idx

    def selection(self, k):
        """Sparse S_k (N x n_k) with S_k[g, i] = 1 when local i of patch k is free dof g."""
        import scipy.sparse as sp
        g = self.patch_gid(k)
        cols = np.nonzero(g >= 0)[0]
        return sp.csr_matrix((np.ones(len(cols)), (g[cols], cols)), shape=(self.N, self.size[k]))


class Piece:
    def __init__(self, kind, owner, bdirs, ends, dofs, local):
        self.kind = kind          # 'interior' | 'face' | 'edge' | 'vertex'
        self.owner = owner        # patch whose parametrization orders the piece
        self.bdirs = bdirs        # directions in which the entity sits on the boundary
        self.ends = ends
        self.dofs = dofs          # global free ids, ordered x-fastest in the owner patch
        self.local = local        # owner-local tensor shape of the piece (per free dir)
        self.adjacent = []        # [(patch, boundary dirs in that patch)]


def _entity_kind(d, nb):
    free = d - nb
    if nb == 0:
        return "interior"
    if free == 0:
        return "vertex"
    if free == 1:
        return "edge"
    return "face"


def pieces(dm):
    """Pieces of Sec. 3 (eq. of the additive smoother), each a set of free dofs."""
    d = dm.d
    seen = np.zeros(dm.N, dtype=bool)
    out = []
    for k in range(dm.K):
        n = dm.n[k]
        g = dm.patch_gid(k)
        for nb in range(d + 1):
            for bdirs in itertools.combinations(range(d), nb):
                for ends in itertools.product([0, 1], repeat=nb):
                    ranges = []
                    for c in range(d):
                        if c in bdirs:
                            e = ends[bdirs.index(c)]
                            ranges.append([0 if e == 0 else n[c] - 1])
                        else:
                            ranges.append(list(range(1, n[c] - 1)))
                    if any(len(r) == 0 for r in ranges):
                        continue
                    grids = np.meshgrid(*[np.array(r) for r in reversed(ranges)],
                                        indexing="ij")
                    loc = sum(grids[d - 1 - c] * int(np.prod(n[:c])) for c in range(d))
                    gl = g[loc.ravel()]
                    if np.all(gl < 0):
                        continue
                    if np.any(gl < 0):
                        raise AssertionError("entity with mixed Dirichlet status")
                    if seen[gl[0]]:
                        assert np.all(seen[gl])
                        continue
                    seen[gl] = True
                    shape = [n[c] - 2 for c in range(d) if c not in bdirs]
                    out.append(Piece(_entity_kind(d, nb), k, list(bdirs), list(ends),
                                     gl, shape))
    assert np.all(seen), "every free dof must lie in one piece"
    for pc in out:
        pats = {}
        for x in dm.copies[pc.dofs[0]]:
            kk, idx = dm.local_index(x)
            bd = [c for c in range(d) if idx[c] in (0, dm.n[kk][c] - 1)]
            pats[kk] = bd
        pc.adjacent = sorted(pats.items())
    return out
