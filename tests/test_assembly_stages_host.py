"""The device-assembly stages (Gauss quadrature sum-factorised over the
tensor rule, Sec. 4) run on the host: their per-entry arithmetic is shared by
the kernels of assemble.hip and this check, which builds it with g++ and
compares the tiled bands with the library's host assembly (itself checked
against the oracle in test_lib_host.py) for every level above the coarsest."""
import ctypes
import os
import subprocess

import pytest

from paper_1804_02539_amd import igamg
from paper_1804_02539_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1804_02539_amd", "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")


@pytest.fixture(scope="module")
def stages(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asm") / "asm_stages_host.so")
    cmd = ["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", "-I", INCLUDE, "-I", CSRC,
           "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-Wno-unknown-pragmas",
           os.path.join(HERE, "asm_stages_host.cpp"), os.path.join(CSRC, "host_setup.cpp"), "-o", out]
    subprocess.check_call(cmd)
    lib = ctypes.CDLL(out)
    lib.asm_stages_vs_host.restype = ctypes.c_int
    lib.coarse_dense_vs_serial.restype = ctypes.c_long
    lib.asm_max_dispatch_items.restype = ctypes.c_longlong
    return lib


CASES = {
    "square4x4_bezier_p4_l3": lambda: W.square_4x4_bezier(levels=3),
    "cube2x2x2_trilinear_p3_l3": lambda: W.cube_2x2x2_trilinear(levels=3),
    "fichera7_p2_l3": lambda: W.fichera(2, 3),
    "cube_p4_neumann_l3": lambda: W.box_grid(3, [2, 1, 1], 4, 1, 3, gdeg=1, dirichlet_sides=[0, 2]),
    "box1x2_p8_l2": lambda: W.box_grid(2, [1, 2], 8, 1, 2, gdeg=1),
    "graded_square3x2_p3_l3": lambda: W.graded_square_3x2(),
    "graded_cube2x2x2_p2_l3": lambda: W.graded_cube_2x2x2(),
}


@pytest.mark.parametrize("name", list(CASES))
def test_stages_equal_host_assembly(stages, name):
    cp = igamg._CProblem(CASES[name]())
    rel, flags = ctypes.c_double(), ctypes.c_int()
    assert stages.asm_stages_vs_host(ctypes.byref(cp.s), ctypes.byref(rel), ctypes.byref(flags)) == 0
    assert rel.value < 1e-14, rel.value
    assert flags.value == 1      # det J > 0 at every Gauss point


@pytest.mark.parametrize("name,prob", [
    ("box3d_p4_4x3x2_e3", lambda: W.box_grid(3, [4, 3, 2], 4, 3, 2, gdeg=1)),
    ("box3d_p5_2x2x4_e3", lambda: W.box_grid(3, [2, 2, 4], 5, 3, 2, gdeg=1)),
    ("box2d_p3_4x4_e16", lambda: W.box_grid(2, [4, 4], 3, 16, 2, gdeg=2, dirichlet_sides=[0, 2])),
])
def test_parallel_coarse_build_equals_serial(stages, name, prob):
    # coarse problems above the host factorization limit are built for the
    # device by blocks of rows in parallel; every entry must match a serial
    # pass bit for bit
    cp = igamg._CProblem(prob())
    assert stages.coarse_dense_vs_serial(ctypes.byref(cp.s)) == 0


def test_assembly_dispatches_stay_below_the_launch_limit(stages):
    """Every per-slab launch of the device assembly stays below the 2^32
    work-items of one dispatch (the launcher also refuses larger ones), for the
    64-patch p=5 workload and for the largest 3D p=6 family the full serving
    recipe can draw (its band capped at 60 GB)."""
    limit = 2 ** 32 - 256

    def items(prob):
        cp = igamg._CProblem(prob)      # keeps the arrays the C struct points to alive
        return stages.asm_max_dispatch_items(ctypes.byref(cp.s))

    c4 = items(W.batched_patch_cube())
    assert 0 < c4 < limit
    fams = W.serving_families(64, 21, n_min=1e4, n_max=4e6, band_bytes_max=60e9, n0_max=8000)
    big = [f for f in fams if f.dim == 3 and f.degree == 6]
    for f in big:
        assert 0 < items(f) < limit
    # the largest 3D patch the smoother takes: 248 elements, p = 8, 254 interior functions
    hw = items(W.box_grid(3, [1, 1, 1], 8, 31, 4, gdeg=1))
    assert 0 < hw < limit, hw
