"""CPU tests of the library: the C-ABI loads and exports every declared symbol,
the host setup (assembly, dof maps, knot-insertion transfers, load vectors)
equals the oracle's, and the error codes come back for bad input."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1804_02539_amd import igamg
from paper_1804_02539_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "igamg.h")).read()
    return sorted(set(re.findall(r"\b(igamg_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(igamg.LIB_PATH)
    names = declared_symbols()
    assert "igamg_setup" in names and "igamg_solve" in names and "igamg_vcycle" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(igamg.EXPORTED) == names


@pytest.mark.parametrize("make", [
    lambda: W.unit_square_2x2(levels=3),
    lambda: W.square_4x4_bezier(p=3, levels=3),
    lambda: W.cube_2x2x2_trilinear(levels=3),
    lambda: W.fichera(2, 2),
    lambda: W.box_grid(2, [3, 1], 1, 2, 3, gdeg=1, dirichlet_sides=[0]),
    lambda: W.graded_square_3x2(),
    lambda: W.graded_cube_2x2x2(),
])
def test_host_setup_equals_oracle(make):
    from oracle.multigrid import Hierarchy, load_vector
    prob = make()
    s = igamg.Solver(prob, host_only=True)
    H = Hierarchy(prob)
    for l in range(prob.levels):
        A = s.export(igamg.EXPORT_MATRIX, l)
        Ao = H.levels[l].A.toarray()
        assert A.shape == Ao.shape
        assert np.abs(A - Ao).max() <= 1e-13 * np.abs(Ao).max()
        if l > 0:
            P = s.export(igamg.EXPORT_PROLONG, l)
            assert np.abs(P - H.P[l].toarray()).max() <= 1e-14
    if prob.meta.get("source", ("",))[0] == "sine":
        f = s.load_vector(*prob.meta["source"][1:])
        fo = load_vector(prob, H.finest)
        assert np.abs(f - fo).max() <= 1e-12 * np.abs(fo).max()


@pytest.mark.parametrize("make", [lambda: W.square_4x4_bezier(p=2, levels=2),
                                  lambda: W.fichera(3, 2)])
def test_dof_numbering_equals_oracle(make):
    # the global free numbering is a shared convention: compare the copies of
    # every dof as (patch, local index) pairs
    from oracle.topology import DofMap
    prob = make()
    s = igamg.Solver(prob, host_only=True)
    for l in range(prob.levels):
        dm = DofMap(prob, l)
        ptr, idx = s.dof_map(l)
        assert len(ptr) - 1 == dm.N
        # library patch offsets are 256-aligned: recover (patch, local) by sizes
        sizes = [int(np.prod(n)) for n in dm.n]
        offs = np.cumsum([0] + [(z + 255) // 256 * 256 for z in sizes])
        for g in range(0, dm.N, max(1, dm.N // 500)):
            lib_c = []
            for x in idx[ptr[g]:ptr[g + 1]]:
                k = int(np.searchsorted(offs, x, side="right") - 1)
                lib_c.append((k, int(x - offs[k])))
            orc_c = []
            for x in dm.copies[g]:
                k = int(np.searchsorted(dm.off, x, side="right") - 1)
                orc_c.append((k, int(x - dm.off[k])))
            assert lib_c == orc_c, g


def _expect(code, fn):
    with pytest.raises(igamg.IgamgError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


def test_error_codes():
    bad = W.unit_square_2x2(levels=2)
    bad.degree = 9
    _expect(igamg.EINVAL, lambda: igamg.Solver(bad, host_only=True))
    bad = W.unit_square_2x2(levels=2)
    bad.levels = 1
    _expect(igamg.EINVAL, lambda: igamg.Solver(bad, host_only=True))
    # non-matching interface: element counts differ across the glued side
    bad = W.unit_square_2x2(levels=2)
    bad.nel0 = bad.nel0.copy()
    bad.nel0[1, 1] = 3
    _expect(igamg.ETOPO, lambda: igamg.Solver(bad, host_only=True))
    bad = W.unit_square_2x2(levels=2)
    bad.iface = bad.iface.copy()
    bad.iface[0, 1] = 7
    _expect(igamg.ETOPO, lambda: igamg.Solver(bad, host_only=True))
    # folded geometry: a control point pulled across the patch
    bad = W.unit_square_2x2(levels=2)
    bad.geo_ctrl[0] = bad.geo_ctrl[0].copy()
    bad.geo_ctrl[0][3] = [-0.4, -0.4]
    _expect(igamg.EGEOM, lambda: igamg.Solver(bad, host_only=True))
    # no Dirichlet side: the coarse matrix is singular
    bad = W.box_grid(2, [2, 1], 2, 1, 2, gdeg=1, dirichlet_sides=[])
    _expect(igamg.ENOTSPD, lambda: igamg.Solver(bad, host_only=True))
    # workspace too small is reported before any device access
    prob = W.unit_square_2x2(levels=2)
    cp = igamg._CProblem(prob)
    h = ctypes.c_void_p()
    code = igamg.lib().igamg_setup(ctypes.byref(cp.s), ctypes.byref(igamg.default_options()),
                                   ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert code == igamg.ENOMEM
    # invalid options
    _expect(igamg.EINVAL, lambda: igamg.Solver(prob, igamg.default_options(mu=3), host_only=True))
    # solver entry points refuse a host-only handle
    s = igamg.Solver(prob, host_only=True)
    assert igamg.lib().igamg_vcycle(s.h, ctypes.c_void_p(8), ctypes.c_void_p(16), None) == igamg.EINVAL


def test_workspace_size_matches_setup_plan():
    prob = W.square_4x4_bezier(p=3, levels=3)
    n = igamg.workspace_size(prob)
    # band of the finest level alone: (2p+1)^2 doubles per local row
    assert n > 49 * 8 * 16 * (3 * 2 ** 2 + 3) ** 2
    assert n < 64 * 1024 * 1024


def test_binding_loads_a_single_hip_runtime():
    """The library must bind to the HIP runtime torch loads: importing the
    binding first in a fresh process maps exactly one libamdhip64."""
    import subprocess
    import sys
    code = ("import os, sys; sys.path.insert(0, %r); from paper_1804_02539_amd import igamg; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_piece_wider_than_the_smoother_kernels_is_rejected():
    """Patches with more than 256 interior functions in a direction are
    rejected at setup (the fast-diagonalization kernels give each row of a
    tensor one thread of a 256-thread workgroup); 128 elements per direction
    (the paper's finest per-patch resolution, l = 7) are accepted."""
    ok = W.box_grid(2, [1, 1], 2, 2, 7, gdeg=1)        # 128 elements per direction at the finest level
    assert igamg.Solver(ok, host_only=True).N == 128 * 128
    prob = W.box_grid(2, [1, 1], 2, 2, 9, gdeg=1)      # 512 elements per direction
    _expect(igamg.EINVAL, lambda: igamg.Solver(prob, host_only=True))


def test_knots0_validation():
    prob = W.graded_square_3x2()
    s = igamg.Solver(prob, host_only=True)
    assert s.N > 0
    # breakpoints that do not increase, or do not run from 0 to 1
    bad = W.graded_square_3x2()
    bad.knots0[0][0] = bad.knots0[0][0][::-1].copy()
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(bad, host_only=True)
    assert e.value.code == igamg.EINVAL
    bad = W.graded_square_3x2()
    bad.knots0[0][1] = bad.knots0[0][1] * 0.5
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(bad, host_only=True)
    assert e.value.code == igamg.EINVAL
    # the two sides of an interface with different breakpoints (Sec. 2:
    # fully matching interfaces)
    bad = W.graded_square_3x2()
    b = bad.knots0[0][1].copy()
    b[1] = 0.5 * (b[1] + b[2])
    bad.knots0[0][1] = b
    with pytest.raises(igamg.IgamgError) as e:
        igamg.Solver(bad, host_only=True)
    assert e.value.code == igamg.ETOPO


def test_noalloc_size_query_and_limits():
    # the no-allocation setup answers a size query on the host (workspace
    # NULL): its workspace leaves out the device assembly's setup scratch
    prob = W.cube_2x2x2_trilinear(levels=3)
    opts = igamg.default_options()
    cp = igamg._CProblem(prob)
    need = ctypes.c_size_t()
    lib = igamg.lib()
    assert lib.igamg_setup_noalloc(ctypes.byref(cp.s), ctypes.byref(opts), None, 0, None, None,
                                   ctypes.byref(need)) == igamg.OK
    assert 0 < need.value < igamg.workspace_size(prob, opts)
    # a device factorization of the coarse matrix needs its scratch in the workspace
    dev = igamg.default_options(coarse_factor=2)
    need_dev = ctypes.c_size_t()
    assert lib.igamg_setup_noalloc(ctypes.byref(cp.s), ctypes.byref(dev), None, 0, None, None,
                                   ctypes.byref(need_dev)) == igamg.OK
    assert need_dev.value >= need.value
    # a query needs somewhere to write the size
    assert lib.igamg_setup_noalloc(ctypes.byref(cp.s), ctypes.byref(opts), None, 0, None, None, None) == igamg.EINVAL


def test_bf16_precision_value():
    """IGAMG_MIXED_BF16 is IGAMG_MIXED with the bfloat16 matrix-core smoother
    products (fd_mfma = 3); other precision values and a conflicting fd_mfma
    are rejected."""
    prob = W.square_4x4_bezier(levels=3)
    mixed = igamg.workspace_size(prob, igamg.default_options(precision=igamg.MIXED))
    assert igamg.workspace_size(prob, igamg.default_options(precision=igamg.MIXED_BF16)) == mixed
    assert igamg.workspace_size(prob, igamg.default_options(precision=igamg.MIXED_BF16, fd_mfma=3)) == mixed
    _expect(igamg.EINVAL, lambda: igamg.workspace_size(prob, igamg.default_options(precision=3)))
    _expect(igamg.EINVAL, lambda: igamg.workspace_size(prob, igamg.default_options(precision=igamg.MIXED_BF16,
                                                                                    fd_mfma=1)))


def test_scatter_form_workspace_accounting():
    """The workspace plan of the scatter-form apply, against the layout
    formulas (host only).  The 2x2x2 p=3 cube: its finest level, 8 patches of
    35^3 rows padded to 256 (344,064 rows, 1,344 tiles), is the only one
    above 65,536 rows.  A tile's windows hold (p+1) 256 + (2p+1)(p + p n0)
    = 1,780 values (n0 = 35), kept in FP64: 1,344 * 1,780 * 8 bytes more than
    the gather form.  Mixed precision also stores that level's FP32 band as
    the half band, nbh = 172 planes instead of 343."""
    prob = W.cube_2x2x2_trilinear()
    p, n0, tiles = 3, 35, 8 * ((35 ** 3 + 255) // 256)
    assert tiles == 1344
    ws = (p + 1) * 256 + (2 * p + 1) * (p + p * n0)
    assert ws == 1780
    windows = tiles * ws * 8
    nb, nbh = (2 * p + 1) ** 3, ((2 * p + 1) ** 3 + 1) // 2
    size = lambda **kw: igamg.workspace_size(prob, igamg.default_options(**kw))
    assert size(band_form=0) - size(band_form=1) == windows
    half32 = (nb - nbh) * tiles * 256 * 4
    assert size(band_form=0, precision=igamg.MIXED) - size(band_form=1, precision=igamg.MIXED) == windows - half32
    # 2D: the 4x4 p=4 square keeps the gather form (its finest level has
    # 77,824 rows); one level finer (16 patches of 132^2 rows: 1,104 tiles,
    # 282,624 rows) takes the scatter form in an FP64 handle (above 2^17
    # rows), with windows of 5 * 256 + 9 * 4 = 1,316 values per tile, and
    # the gather form in a mixed one (up to 2^19 rows)
    sq = W.square_4x4_bezier()
    assert igamg.workspace_size(sq, igamg.default_options()) == igamg.workspace_size(sq, igamg.default_options(band_form=1))
    assert igamg.workspace_size(sq, igamg.default_options(band_form=2)) > igamg.workspace_size(sq, igamg.default_options())
    sq7 = W.square_4x4_bezier(levels=7)
    s7 = lambda **kw: igamg.workspace_size(sq7, igamg.default_options(**kw))
    assert s7(band_form=0) - s7(band_form=1) == 1104 * 1316 * 8
    assert s7(band_form=0, precision=igamg.MIXED) == s7(band_form=1, precision=igamg.MIXED)
    with pytest.raises(igamg.IgamgError):
        igamg.workspace_size(prob, igamg.default_options(band_form=3))
