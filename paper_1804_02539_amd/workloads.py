"""Seeded synthetic problem descriptions (inputs only, no solver arithmetic).

A problem is the data of the model problem of Sec. 2: a set of patches, each a
single-element Bezier geometry map of (0,1)^d, fully matching interfaces
between patch sides, a boundary-condition flag per free side, the spline
degree, the coarsest element counts and the number of grid levels.  This
module is imported by both the HIP library's callers and the test oracle; it
only lays out coordinates, index tables and seeded random numbers.

Conventions shared by every consumer of a ``Problem``:

* local tensor indices run x fastest (index i1 + n1*(i2 + n2*i3));
* side s of a patch is ``2*dir + end``: the face where parameter ``dir`` is 0
  (end 0) or 1 (end 1);
* an interface row is (patch a, side a, patch b, side b, orient).  The
  tangential parameter axes of side a, in increasing direction order (t0, t1),
  meet those of side b (u0, u1); orient bit 0 swaps the pairing (t0<->u1,
  t1<->u0), bit 1 reverses the axis paired with t0, bit 2 the one paired with
  t1;
* bc[k, s] = 1 marks a homogeneous Dirichlet side, 0 a homogeneous Neumann one
  (ignored on interface sides);
* level l has nel0 * 2**l elements per patch and direction, l = 0..levels-1;
  the coarsest breakpoints are uniform unless ``knots0[k][c]`` gives them
  (nel0[k][c] + 1 increasing values from 0 to 1).
"""
from dataclasses import dataclass, field
import itertools

import numpy as np


@dataclass
class Problem:
    dim: int
    degree: int
    levels: int
    nel0: np.ndarray          # (K, d) int32
    geo_degree: np.ndarray    # (K, d) int32
    geo_ctrl: list            # K arrays of shape (prod(g+1), d), x-fastest
    iface: np.ndarray         # (nif, 5) int32
    bc: np.ndarray            # (K, 2d) int32
    name: str = ""
    meta: dict = field(default_factory=dict)
    knots0: list = None       # None, or K lists of d breakpoint arrays (coarsest level)

    @property
    def npatch(self):
        return int(self.nel0.shape[0])

    def nel(self, level):
        return self.nel0 * (2 ** level)

    def flat_knots0(self):
        """Breakpoints of every patch and direction, concatenated (direction
        fastest), or None for uniform knots."""
        if self.knots0 is None:
            return None
        return np.ascontiguousarray(np.concatenate([np.asarray(b, dtype=np.float64)
                                                    for kk in self.knots0 for b in kk]))

    def flat_ctrl(self):
        return np.ascontiguousarray(np.concatenate([c.reshape(-1) for c in self.geo_ctrl]),
                                    dtype=np.float64)


def _grid_ctrl(lo, hi, gdeg):
    """Control points of the affine map of (0,1)^d onto the box [lo, hi] (degree gdeg)."""
    d = len(lo)
    axes = [np.linspace(lo[c], hi[c], gdeg[c] + 1) for c in range(d)]
    pts = []
    for idx in itertools.product(*[range(g + 1) for g in reversed(gdeg)]):
        idx = idx[::-1]
        pts.append([axes[c][idx[c]] for c in range(d)])
    return np.array(pts, dtype=np.float64)


def box_grid(dim, npp, p, nel0, levels, *, gdeg=1, dirichlet_sides=None,
             extent=None, name=""):
    """Patches of an axis-aligned box split into npp[0] x npp[1] (x npp[2]) equal boxes.

    ``nel0`` is either an int or a per-direction list of per-slab coarse element
    counts (``nel0[c][j]`` for slab j of direction c), so that interfaces conform.
    ``dirichlet_sides`` lists the outer sides (0..2d-1) carrying Dirichlet data;
    default all.
    """
    npp = list(npp)
    if extent is None:
        extent = [1.0] * dim
    if dirichlet_sides is None:
        dirichlet_sides = list(range(2 * dim))
    if isinstance(nel0, (int, np.integer)):
        nel0 = [[int(nel0)] * npp[c] for c in range(dim)]
    gd = [gdeg] * dim if isinstance(gdeg, int) else list(gdeg)
    pid = {}
    ctrl, nels, gdegs, bcs = [], [], [], []
    for idx in itertools.product(*[range(npp[c]) for c in reversed(range(dim))]):
        idx = idx[::-1]
        pid[idx] = len(ctrl)
        lo = [extent[c] * idx[c] / npp[c] for c in range(dim)]
        hi = [extent[c] * (idx[c] + 1) / npp[c] for c in range(dim)]
        ctrl.append(_grid_ctrl(lo, hi, gd))
        nels.append([nel0[c][idx[c]] for c in range(dim)])
        gdegs.append(gd)
        b = np.zeros(2 * dim, dtype=np.int32)
        for c in range(dim):
            if idx[c] == 0 and (2 * c) in dirichlet_sides:
                b[2 * c] = 1
            if idx[c] == npp[c] - 1 and (2 * c + 1) in dirichlet_sides:
                b[2 * c + 1] = 1
        bcs.append(b)
    iface = []
    for idx, k in pid.items():
        for c in range(dim):
            nb = list(idx)
            nb[c] += 1
            nb = tuple(nb)
            if nb in pid:
                iface.append([k, 2 * c + 1, pid[nb], 2 * c, 0])
    return Problem(dim=dim, degree=p, levels=levels,
                   nel0=np.array(nels, dtype=np.int32),
                   geo_degree=np.array(gdegs, dtype=np.int32),
                   geo_ctrl=ctrl,
                   iface=np.array(iface, dtype=np.int32).reshape(-1, 5),
                   bc=np.array(bcs, dtype=np.int32), name=name,
                   meta={"npp": npp, "pid": pid})


def perturb_centres_2d(prob, rel, rng):
    """Biquadratic patches: displace each centre control point by U[-rel*w, rel*w]^2.

    The 8 boundary control points stay on the straight patch edges, so neighbouring
    maps agree on their common edge.
    """
    for k, c in enumerate(prob.geo_ctrl):
        assert list(prob.geo_degree[k]) == [2, 2]
        w = c[2, 0] - c[0, 0]
        c[4] += rng.uniform(-rel * w, rel * w, size=2)
    return prob


def perturb_vertex_3d(prob, vertex, amp, rng):
    """Trilinear patches: move the macro vertex ``vertex`` by U[-amp, amp]^3 in every patch."""
    delta = rng.uniform(-amp, amp, size=3)
    v = np.asarray(vertex, dtype=np.float64)
    for c in prob.geo_ctrl:
        hit = np.all(np.abs(c - v) < 1e-12, axis=1)
        c[hit] += delta
    return prob


def perturb_interior_vertices_3d(prob, rel, rng):
    """Trilinear patches on a grid: move every interior macro vertex by <= rel * width."""
    pts = np.concatenate(prob.geo_ctrl)
    uniq = np.unique(np.round(pts, 12), axis=0)
    moves = {}
    for v in uniq:
        if np.all(v > 1e-12) and np.all(v < 1 - 1e-12):
            moves[tuple(v)] = None
    w = min(float(c[:, 0].max() - c[:, 0].min()) for c in prob.geo_ctrl)
    for v in sorted(moves):
        moves[v] = rng.uniform(-rel * w, rel * w, size=3)
    for c in prob.geo_ctrl:
        for i in range(c.shape[0]):
            key = tuple(np.round(c[i], 12))
            if key in moves:
                c[i] = c[i] + moves[key]
    return prob


def grade_slab_knots(prob, rel, rng):
    """Non-uniform coarsest breakpoints for a ``box_grid`` problem: per
    direction and slab, the interior breakpoints of the uniform grid are moved
    by U[-rel, rel] times the span.  Patches of one slab share the vector, so
    the interfaces stay fully matching."""
    npp, pid = prob.meta["npp"], prob.meta["pid"]
    slab = {}
    for c in range(prob.dim):
        for j in range(npp[c]):
            k0 = next(k for idx, k in pid.items() if idx[c] == j)
            e = int(prob.nel0[k0][c])
            b = np.arange(e + 1, dtype=np.float64) / e
            b[1:-1] += rng.uniform(-rel, rel, size=e - 1) / e
            b[0], b[-1] = 0.0, 1.0
            slab[(c, j)] = b
    prob.knots0 = [[slab[(c, idx[c])] for c in range(prob.dim)]
                   for idx, k in sorted(pid.items(), key=lambda t: t[1])]
    return prob


# --- the workloads ------------------------------------------------------------

def graded_square_3x2(p=3, nel0=3, levels=3, seed=12):
    """2D box (0,1.5)x(0,1) as 3x2 affine patches with seeded non-uniform
    coarsest knot vectors (interior breakpoints moved by up to 30% of a span);
    Dirichlet on x=0 and y=0, Neumann elsewhere; seeded U[-1,1] right-hand side."""
    rng = np.random.default_rng(seed)
    prob = box_grid(2, [3, 2], p, nel0, levels, gdeg=1, dirichlet_sides=[0, 2], extent=[1.5, 1.0],
                    name="graded_square3x2")
    grade_slab_knots(prob, 0.3, rng)
    prob.meta["source"] = ("random", seed)
    return prob


def graded_cube_2x2x2(p=2, nel0=2, levels=3, seed=14):
    """3D unit cube as 2x2x2 trilinear patches (interior vertex moved as in
    the 3D cube workload) with seeded non-uniform coarsest knot vectors (up to
    30% of a span); full Dirichlet; seeded U[-1,1] right-hand side."""
    rng = np.random.default_rng(seed)
    prob = box_grid(3, [2, 2, 2], p, nel0, levels, gdeg=1, name="graded_cube2x2x2")
    perturb_vertex_3d(prob, [0.5, 0.5, 0.5], 0.05, rng)
    grade_slab_knots(prob, 0.3, rng)
    prob.meta["source"] = ("random", seed)
    return prob


def unit_square_2x2(p=2, nel0=2, levels=4):
    """2D unit square as 2x2 identity-scaled patches, full Dirichlet (f = 2 pi^2 sin sin)."""
    prob = box_grid(2, [2, 2], p, nel0, levels, gdeg=1, name="square2x2")
    prob.meta["source"] = ("sine", 2.0 * np.pi ** 2, 1.0)
    return prob


def square_4x4_bezier(p=4, nel0=2, levels=6, seed=2):
    """2D unit square as 4x4 biquadratic patches with seeded interior control points.

    Dirichlet on x=0 and y=0, Neumann elsewhere; right-hand side is a seeded
    U[-1,1] coefficient vector over the free degrees of freedom.
    """
    rng = np.random.default_rng(seed)
    prob = box_grid(2, [4, 4], p, nel0, levels, gdeg=2, dirichlet_sides=[0, 2],
                    name="square4x4")
    perturb_centres_2d(prob, 0.1, rng)
    prob.meta["source"] = ("random", seed)
    return prob


def cube_2x2x2_trilinear(p=3, nel0=1, levels=6, seed=3):
    """3D unit cube as 2x2x2 trilinear patches; the shared centre vertex is moved by
    U[-0.05, 0.05]^3.  Full Dirichlet; f = 3 pi^2 sin sin sin."""
    rng = np.random.default_rng(seed)
    prob = box_grid(3, [2, 2, 2], p, nel0, levels, gdeg=1, name="cube2x2x2")
    perturb_vertex_3d(prob, [0.5, 0.5, 0.5], 0.05, rng)
    prob.meta["source"] = ("sine", 3.0 * np.pi ** 2, 1.0)
    return prob


def fichera(p, levels, split=1):
    """The Fichera corner (0,2)^3 minus [1,2)^3 as 7 unit cubes, each split into
    split^3 patches.  Dirichlet on the planes x=0, y=0, z=0, Neumann elsewhere
    (Sec. 5, the 3D experiment)."""
    npp = [2 * split] * 3
    prob = box_grid(3, npp, p, 1, levels, gdeg=1, dirichlet_sides=[0, 2, 4],
                    extent=[2.0, 2.0, 2.0], name=f"fichera{7 * split ** 3}")
    pid = prob.meta["pid"]
    keep = [idx for idx in pid if not all(i >= split for i in idx)]
    keep.sort(key=lambda idx: pid[idx])
    newid = {idx: j for j, idx in enumerate(keep)}
    old2new = {pid[idx]: newid[idx] for idx in keep}
    ctrl = [prob.geo_ctrl[pid[idx]] for idx in keep]
    nel0 = prob.nel0[[pid[idx] for idx in keep]]
    gdeg = prob.geo_degree[[pid[idx] for idx in keep]]
    bc = prob.bc[[pid[idx] for idx in keep]]
    iface = [[old2new[a], sa, old2new[b], sb, o] for a, sa, b, sb, o in prob.iface
             if a in old2new and b in old2new]
    prob.geo_ctrl, prob.nel0, prob.geo_degree, prob.bc = ctrl, nel0, gdeg, bc
    prob.iface = np.array(iface, dtype=np.int32).reshape(-1, 5)
    prob.meta = {"source": ("sine", 75.0 * np.pi ** 2, 5.0)}
    return prob


def random_rhs(n, seed):
    """Seeded U[-1,1] right-hand-side coefficients for n free degrees of freedom."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


CONFIGS = {
    "square2x2_p2": lambda: unit_square_2x2(),
    "square4x4_p4": lambda: square_4x4_bezier(),
    "cube2x2x2_p3": lambda: cube_2x2x2_trilinear(),
}


def serving_families(n_families, seed=5, n_min=1e4, n_max=3e5, band_bytes_max=1.5e9, n0_max=2500):
    """Seeded problem families for the serving workload.

    Each family draws d in {2, 3} and p in {2..6} uniformly, a patch grid of
    2..4 patches per direction, and a target size N log-uniform in
    [n_min, n_max]; the coarsest element count (1..3 per patch and direction)
    and the level count are the pair whose number of free dofs is closest to
    the target (among the pairs inside [n_min, n_max] when there are any),
    subject to the FP64 band of the finest level staying under band_bytes_max,
    the coarsest level having at most n0_max unknowns (the dense coarse
    inverse is N0^2 / 2 doubles; up to 3,000 unknowns it is factored on the
    host)
    and every patch having at most 84 interior functions per direction (the
    largest tensors the smoother kernels stage whole in LDS).
    2D families are biquadratic grids with seeded interior control points
    (Dirichlet on x=0 and y=0), 3D ones trilinear grids with every interior
    macro vertex moved by up to 10% of the patch width (full Dirichlet).
    """
    rng = np.random.default_rng(seed)
    fams = []
    for j in range(n_families):
        best = None
        while best is None:       # redraw families that no size choice admits
            d = int(rng.integers(2, 4))
            p = int(rng.integers(2, 7))
            npp = [int(rng.integers(2, 5)) for _ in range(d)]
            target = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
            # free dofs exactly: 2D families are Dirichlet on one side per
            # direction, 3D ones on both
            nd = 1 if d == 2 else 2
            for nel0 in (1, 2, 3):
                for levels in range(2, 11):
                    nel = nel0 * 2 ** (levels - 1)
                    rows = int(np.prod([k * (nel + p) for k in npp]))
                    n_free = float(np.prod([k * (nel + p - 1) + 1 - nd for k in npp]))
                    n0 = float(np.prod([k * (nel0 + p - 1) + 1 - nd for k in npp]))
                    if rows * (2 * p + 1) ** d * 8 > band_bytes_max or n0 > n0_max or nel + p - 2 > 84:
                        continue
                    # sizes inside [n_min, n_max] first, then the closest to the target
                    score = (not (n_min <= n_free <= n_max), abs(np.log(n_free / target)))
                    if best is None or score < best[0]:
                        best = (score, nel0, levels)
        _, nel0, levels = best
        name = f"fam{j}_d{d}_p{p}_{'x'.join(map(str, npp))}_e{nel0}_L{levels}"
        if d == 2:
            prob = box_grid(2, npp, p, nel0, levels, gdeg=2, dirichlet_sides=[0, 2], name=name)
            perturb_centres_2d(prob, 0.1, rng)
        else:
            prob = box_grid(3, npp, p, nel0, levels, gdeg=1, name=name)
            perturb_interior_vertices_3d(prob, 0.1, rng)
        prob.meta["target_n"] = target
        fams.append(prob)
    return fams


def batched_patch_cube(seed=4, p=5, divide=1, levels=None, n_range=(2e6, 4e6), counts=(8, 16, 24, 32, 48)):
    """The unit cube as 4x4x4 equal-width patches with uneven element counts.

    Per direction, the 4 slabs draw element counts from ``counts`` (seeded);
    the draw is repeated until the number of free dofs N lies in ``n_range``.
    Every interior macro vertex of the trilinear maps moves by up to 10% of
    the patch width; full Dirichlet; p=5; 4 levels, so the coarsest level has
    count/8 elements per slab; seeded U[-1,1] right-hand side.

    ``divide`` = 4 gives the down-scaled replica: counts/4 at the finest of 2
    levels, the same topology, degree, geometry and coarsest level.
    """
    rng = np.random.default_rng(seed)
    while True:
        slabs = [[int(c) for c in rng.choice(counts, size=4)] for _ in range(3)]
        n = float(np.prod([sum(s) + 4 * p - 5 for s in slabs]))
        if n_range[0] <= n <= n_range[1]:
            break
    if levels is None:
        levels = 4 if divide == 1 else 4 - int(np.log2(divide))
    fine = [[c // divide for c in s] for s in slabs]
    nel0 = [[c // 2 ** (levels - 1) for c in s] for s in fine]
    assert all(c * 2 ** (levels - 1) == f for s0, s1 in zip(nel0, fine) for c, f in zip(s0, s1))
    name = "cube4x4x4_p%d" % p + ("" if divide == 1 else "_div%d" % divide)
    prob = box_grid(3, [4, 4, 4], p, nel0, levels, gdeg=1, name=name)
    perturb_interior_vertices_3d(prob, 0.1, rng)
    prob.meta["source"] = ("random", seed)
    prob.meta["slabs"] = fine
    return prob
