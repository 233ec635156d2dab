"""Python binding of libigamg.so (ctypes; argument marshalling only).

Every numerical step runs inside the library.  PyTorch supplies device memory
(the workspace and vectors) and the HIP stream.  The library must have been
built in-tree (``paper_1804_02539_amd/build.py``); importing this module
without it raises immediately.
"""
import ctypes
import os

import numpy as np
# torch first: its HIP runtime must be the one the library binds to (the
# library's libamdhip64 dependency then resolves to the copy already loaded;
# two HIP runtimes in one process do not share the device)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigamg.so")

OK, EINVAL, ETOPO, EGEOM, ENOMEM, ENOTSPD, ENOCONV, ENAN, EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, MIXED, MIXED_BF16 = 0, 1, 2
FD_VEC8, FD_VEC4, FD_MFMA, FD_FUSED, FD_MFMA_BF16 = 0, 1, 2, 3, 4
FD_NAMES = {FD_VEC8: "vec8", FD_VEC4: "vec4", FD_MFMA: "mfma", FD_FUSED: "fused", FD_MFMA_BF16: "mfma_bf16"}
OP_APPLY, OP_SMOOTHER, OP_PROLONG, OP_RESTRICT, OP_COARSE, OP_CYCLE_FP32, OP_APPLY_FP32 = 0, 1, 2, 3, 4, 5, 6

ERROR_NAMES = {EINVAL: "EINVAL", ETOPO: "ETOPO", EGEOM: "EGEOM", ENOMEM: "ENOMEM",
               ENOTSPD: "ENOTSPD", ENOCONV: "ENOCONV", ENAN: "ENAN", EDEVICE: "EDEVICE"}


class IgamgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("npatch", ctypes.c_int),
                ("levels", ctypes.c_int), ("nel0", ctypes.POINTER(ctypes.c_int)),
                ("knots0", ctypes.POINTER(ctypes.c_double)),
                ("geo_degree", ctypes.POINTER(ctypes.c_int)),
                ("geo_ctrl", ctypes.POINTER(ctypes.c_double)), ("nif", ctypes.c_int),
                ("iface", ctypes.POINTER(ctypes.c_int)), ("bc", ctypes.POINTER(ctypes.c_int))]


class Options(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("sigma_scale", ctypes.c_double), ("nu", ctypes.c_int),
                ("mu", ctypes.c_int), ("precision", ctypes.c_int), ("maxit", ctypes.c_int),
                ("geometry_scaling", ctypes.c_int), ("inner_maxit", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("graphs", ctypes.c_int), ("fd_mfma", ctypes.c_int),
                ("coarse_factor", ctypes.c_int), ("autotune", ctypes.c_int), ("assembly", ctypes.c_int),
                ("s1_sigma", ctypes.c_int), ("iface_multiplicity", ctypes.c_int), ("physical_h", ctypes.c_int),
                ("iface_direct", ctypes.c_int), ("persistent", ctypes.c_int),
                ("band_form", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("fp64_fallback", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1804_02539_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    P = ctypes.POINTER
    sig = {
        "igamg_default_options": (None, [P(Options)]),
        "igamg_workspace_size": (ctypes.c_int, [P(_Problem), P(Options), P(ctypes.c_size_t)]),
        "igamg_setup": (ctypes.c_int, [P(_Problem), P(Options), vp, ctypes.c_size_t, vp, P(vp)]),
        "igamg_setup_noalloc": (ctypes.c_int, [P(_Problem), P(Options), vp, ctypes.c_size_t, vp, P(vp),
                                                P(ctypes.c_size_t)]),
        "igamg_num_dofs": (ctypes.c_int, [vp, ctypes.c_int, i64p, i64p]),
        "igamg_load_vector": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, P(ctypes.c_double)]),
        "igamg_vcycle": (ctypes.c_int, [vp, vp, vp, vp]),
        "igamg_solve": (ctypes.c_int, [vp, vp, vp, ctypes.c_double, P(SolveInfo), vp]),
        "igamg_operator": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]),
        "igamg_dof_map": (ctypes.c_int, [vp, ctypes.c_int, i64p, i64p, i64p, i64p]),
        "igamg_export": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, P(ctypes.c_double), i64p, i64p]),
        "igamg_profile": (ctypes.c_int, [vp, ctypes.c_int]),
        "igamg_profile_read": (ctypes.c_int, [vp, i64p, P(ctypes.c_double), P(ctypes.c_double)]),
        "igamg_batch_create": (ctypes.c_int, [P(vp)]),
        "igamg_batch_destroy": (ctypes.c_int, [vp]),
        "igamg_batch_add": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_double, vp, P(ctypes.c_int)]),
        "igamg_batch_step": (ctypes.c_int, [vp, vp, P(ctypes.c_int)]),
        "igamg_batch_poll": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_int), P(SolveInfo), P(ctypes.c_int)]),
        "igamg_batch_remove": (ctypes.c_int, [vp, ctypes.c_int]),
        "igamg_solve_batch": (ctypes.c_int, [P(vp), P(vp), P(vp), ctypes.c_int, ctypes.c_double, P(SolveInfo),
                                              P(ctypes.c_int), vp]),
        "igamg_tuning": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, P(ctypes.c_int)]),
        "igamg_band_form": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_int)]),
        "igamg_destroy": (ctypes.c_int, [vp]),
        "igamg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ["igamg_default_options", "igamg_workspace_size", "igamg_setup", "igamg_num_dofs",
            "igamg_load_vector", "igamg_vcycle", "igamg_solve", "igamg_operator", "igamg_dof_map",
            "igamg_export", "igamg_profile", "igamg_profile_read", "igamg_destroy",
            "igamg_last_error", "igamg_batch_create", "igamg_batch_destroy", "igamg_batch_add",
            "igamg_batch_step", "igamg_batch_poll", "igamg_batch_remove", "igamg_solve_batch", "igamg_tuning",
            "igamg_setup_noalloc", "igamg_band_form"]
EXPORT_MATRIX, EXPORT_PROLONG = 0, 1
BAND_GATHER, BAND_SCATTER = 0, 1


def lib():
    return _lib


def _check(code):
    if code != OK:
        raise IgamgError(code, _lib.igamg_last_error().decode())
    return code


def default_options(**kw):
    o = Options()
    _lib.igamg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class _CProblem:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, prob):
        i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))
        self.nel0 = i32(prob.nel0)
        self.gdeg = i32(prob.geo_degree)
        self.ctrl = prob.flat_ctrl()
        self.iface = i32(prob.iface) if len(prob.iface) else np.zeros(5, dtype=np.int32)
        self.bc = i32(prob.bc)
        kn = prob.flat_knots0() if hasattr(prob, "flat_knots0") else None
        self.knots0 = kn
        ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s = _Problem(prob.dim, prob.degree, prob.npatch, prob.levels, ip(self.nel0),
                          dp(kn) if kn is not None else ctypes.POINTER(ctypes.c_double)(),
                          ip(self.gdeg), dp(self.ctrl),
                          int(len(prob.iface)), ip(self.iface), ip(self.bc))


def workspace_size(prob, opts=None):
    cp = _CProblem(prob)
    n = ctypes.c_size_t()
    _check(_lib.igamg_workspace_size(ctypes.byref(cp.s), ctypes.byref(opts or default_options()),
                                     ctypes.byref(n)))
    return int(n.value)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """A multigrid hierarchy resident in a caller-owned device workspace."""

    def __init__(self, prob, opts=None, device="cuda:0", stream=None, host_only=False, noalloc=False):
        import torch
        self.prob = prob
        self.opts = opts or default_options()
        cp = _CProblem(prob)
        h = ctypes.c_void_p()
        if noalloc:
            # igamg_setup_noalloc: size query, then the setup into a workspace
            # of that size (this binding allocates the workspace; the library
            # allocates nothing)
            need = ctypes.c_size_t()
            _check(_lib.igamg_setup_noalloc(ctypes.byref(cp.s), ctypes.byref(self.opts), None, 0, None, None,
                                            ctypes.byref(need)))
            nbytes = int(need.value)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            aligned = (self.workspace.data_ptr() + 255) & ~255
            _check(_lib.igamg_setup_noalloc(ctypes.byref(cp.s), ctypes.byref(self.opts), ctypes.c_void_p(aligned),
                                            nbytes, _stream_ptr(stream), ctypes.byref(h), None))
        elif host_only:
            self.workspace = None
            _check(_lib.igamg_setup(ctypes.byref(cp.s), ctypes.byref(self.opts), None, 0, None,
                                    ctypes.byref(h)))
        else:
            nbytes = workspace_size(prob, self.opts)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            _check(_lib.igamg_setup(ctypes.byref(cp.s), ctypes.byref(self.opts), ctypes.c_void_p(aligned),
                                    nbytes, _stream_ptr(stream), ctypes.byref(h)))
        self.h = h
        self.device = device
        nf, nl = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.igamg_num_dofs(self.h, -1, ctypes.byref(nf), ctypes.byref(nl)))
        self.N, self.N_local = nf.value, nl.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.igamg_destroy(h)
            self.h = None

    def num_dofs(self, level=-1):
        nf, nl = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.igamg_num_dofs(self.h, level, ctypes.byref(nf), ctypes.byref(nl)))
        return nf.value, nl.value

    def dof_map(self, level=-1):
        nf, nc = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.igamg_dof_map(self.h, level, None, None, ctypes.byref(nf), ctypes.byref(nc)))
        ptr = np.zeros(nf.value + 1, dtype=np.int64)
        idx = np.zeros(nc.value, dtype=np.int64)
        i64 = ctypes.POINTER(ctypes.c_int64)
        _check(_lib.igamg_dof_map(self.h, level, ptr.ctypes.data_as(i64), idx.ctypes.data_as(i64),
                                  None, None))
        return ptr, idx

    def export(self, what, level):
        r, c = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.igamg_export(self.h, what, level, None, ctypes.byref(r), ctypes.byref(c)))
        out = np.zeros((r.value, c.value))
        _check(_lib.igamg_export(self.h, what, level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 None, None))
        return out

    def tuning(self, level=-1, fp32=False):
        """Smoother variant (FD_VEC8, FD_VEC4, FD_MFMA) of a level in FP64 or FP32."""
        L = self.prob.levels - 1 if level < 0 else level
        v = ctypes.c_int()
        _check(_lib.igamg_tuning(self.h, L, int(fp32), ctypes.byref(v)))
        return v.value

    def band_form(self, level=-1):
        """BAND_GATHER or BAND_SCATTER: the form of a level's banded apply."""
        L = self.prob.levels - 1 if level < 0 else level
        v = ctypes.c_int()
        _check(_lib.igamg_band_form(self.h, L, ctypes.byref(v)))
        return v.value

    def profile(self, enable):
        _check(_lib.igamg_profile(self.h, int(enable)))

    def profile_read(self):
        """Per-level banded-apply launch counts, ms and bytes: entries [0, levels)
        for FP64 launches, [levels, 2 levels) for FP32 ones."""
        n = 2 * self.prob.levels
        cnt = np.zeros(n, dtype=np.int64)
        ms = np.zeros(n)
        by = np.zeros(n)
        _check(_lib.igamg_profile_read(self.h, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       by.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return cnt, ms, by

    def load_vector(self, amp, freq):
        out = np.zeros(self.N)
        _check(_lib.igamg_load_vector(self.h, amp, freq, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def _vec(self, x, n):
        import torch
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        if x.numel() != n:
            raise ValueError(f"vector of length {x.numel()}, expected {n}")
        return x

    def vcycle(self, r, stream=None):
        import torch
        r = self._vec(r, self.N)
        z = torch.empty_like(r)
        _check(_lib.igamg_vcycle(self.h, _dptr(r), _dptr(z), _stream_ptr(stream)))
        return z

    def operator(self, op, level, x, stream=None):
        import torch
        L = self.prob.levels - 1 if level < 0 else level
        nin = self.num_dofs(L - 1 if op == OP_PROLONG else L)[0]
        nout = self.num_dofs(L - 1 if op == OP_RESTRICT else L)[0]
        x = self._vec(x, nin)
        y = torch.empty(nout, dtype=torch.float64, device=self.device)
        _check(_lib.igamg_operator(self.h, op, L, _dptr(x), _dptr(y), _stream_ptr(stream)))
        return y

    def solve(self, rhs, tol=1e-8, u=None, stream=None, raise_on_error=True):
        import torch
        rhs = self._vec(rhs, self.N)
        if u is None:
            u = torch.empty_like(rhs)
        info = SolveInfo()
        code = _lib.igamg_solve(self.h, _dptr(rhs), _dptr(u), tol, ctypes.byref(info), _stream_ptr(stream))
        if raise_on_error:
            _check(code)
        self.last_code = code
        return u, info


class Batch:
    """Continuous batching of resident solves (igamg_batch_*): requests are
    added and removed between lockstep steps; every step runs one PCG
    iteration of every active request as HIP graphs with one branch each."""

    def __init__(self):
        self.b = ctypes.c_void_p()
        _check(_lib.igamg_batch_create(ctypes.byref(self.b)))
        self._keep = {}

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value and _lib is not None:
            _lib.igamg_batch_destroy(b)
            self.b = None

    def add(self, solver, rhs, u=None, tol=1e-8, stream=None):
        import torch
        rhs = solver._vec(rhs, solver.N)
        if u is None:
            u = torch.empty_like(rhs)
        slot = ctypes.c_int()
        _check(_lib.igamg_batch_add(self.b, solver.h, _dptr(rhs), _dptr(u), tol, _stream_ptr(stream),
                                    ctypes.byref(slot)))
        self._keep[slot.value] = (solver, rhs, u)
        return slot.value

    def step(self, stream=None):
        n = ctypes.c_int()
        _check(_lib.igamg_batch_step(self.b, _stream_ptr(stream), ctypes.byref(n)))
        return n.value

    def poll(self, slot):
        done, code = ctypes.c_int(), ctypes.c_int()
        info = SolveInfo()
        _check(_lib.igamg_batch_poll(self.b, slot, ctypes.byref(done), ctypes.byref(info), ctypes.byref(code)))
        return bool(done.value), info, code.value

    def result(self, slot):
        return self._keep[slot][2]

    def remove(self, slot):
        _check(_lib.igamg_batch_remove(self.b, slot))
        self._keep.pop(slot, None)


def solve_batch(solvers, rhss, tol=1e-8, stream=None):
    """Solve several resident problems to completion in one batch."""
    import torch
    n = len(solvers)
    rh = [s._vec(r, s.N) for s, r in zip(solvers, rhss)]
    us = [torch.empty_like(r) for r in rh]
    H = (ctypes.c_void_p * n)(*[s.h.value for s in solvers])
    R = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rh])
    U = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    infos = (SolveInfo * n)()
    codes = (ctypes.c_int * n)()
    code = _lib.igamg_solve_batch(H, R, U, n, tol, infos, codes, _stream_ptr(stream))
    return us, list(infos), list(codes), code
