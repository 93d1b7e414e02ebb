"""ctypes binding of libpot3d.so (include/pot3d.h).  Argument marshalling only.

Every function keeps the C name and argument order.  Host arrays are numpy
float64 C-contiguous arrays.  Device buffers and streams are passed as
integers: ``tensor.data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``.
There is no CPU fallback.  If the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# POT3D_LIB=checked selects the build whose kernels range-test every index.
LIB_PATH = os.path.join(_HERE, "libpot3d_checked.so" if os.environ.get("POT3D_LIB") == "checked" else "libpot3d.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBREAKDOWN = 0, -1, -2, -3, -4, -5
UPPER_SOURCE_SURFACE, UPPER_CLOSED_WALL = 0, 1
FP64, FP32_REFINED = 0, 1
REFINE_RESTART, REFINE_RELIABLE = 0, 1
ITER_TWO_PASS, ITER_ONE_SWEEP = 0, 1
PC_JACOBI, PC_PHI_LINE = 0, 1
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOCONV: "ENOCONV",
                EBREAKDOWN: "EBREAKDOWN"}

EXPORTED = ("pot3d_create", "pot3d_solve", "pot3d_solve_device", "pot3d_apply_device", "pot3d_rhs_device",
            "pot3d_precondition_device", "pot3d_pole_values", "pot3d_field_device", "pot3d_get_stats", "pot3d_time_kernels", "pot3d_set_refinement",
            "pot3d_set_refinement_mode", "pot3d_set_iteration", "pot3d_set_preconditioner", "pot3d_solve_noalloc",
            "pot3d_destroy",
            "pot3d_last_error", "pot3d_version",
            "pot3d_server_create", "pot3d_server_submit", "pot3d_server_step", "pot3d_server_result",
            "pot3d_server_set_cache_budget", "pot3d_server_get_stats", "pot3d_server_destroy",
            "pot3d_server_last_error")


class pot3d_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("status", ctypes.c_int),
                ("graph_launches", ctypes.c_int), ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("loop_ms", ctypes.c_double), ("bytes_per_iter", ctypes.c_double),
                ("n", ctypes.c_longlong), ("pitch", ctypes.c_int), ("tile_p", ctypes.c_int),
                ("tile_r", ctypes.c_int), ("chunk_p", ctypes.c_int), ("chunk_r", ctypes.c_int),
                ("blocks_p", ctypes.c_int), ("blocks_r", ctypes.c_int), ("iteration", ctypes.c_int),
                ("sweep_rows", ctypes.c_int), ("chunk_s", ctypes.c_int), ("blocks_s", ctypes.c_int),
                ("precond", ctypes.c_int), ("blocks_l", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class pot3d_request_info(ctypes.Structure):
    _fields_ = [("id", ctypes.c_longlong), ("done", ctypes.c_int), ("status", ctypes.c_int),
                ("iters", ctypes.c_int), ("outer", ctypes.c_int), ("nr", ctypes.c_int), ("nt", ctypes.c_int),
                ("np", ctypes.c_int), ("relres_true", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class pot3d_server_stats(ctypes.Structure):
    _fields_ = [("replays", ctypes.c_longlong), ("finished", ctypes.c_longlong), ("active", ctypes.c_int),
                ("queued", ctypes.c_int), ("cached_contexts", ctypes.c_int), ("max_slots", ctypes.c_int),
                ("graph_iters", ctypes.c_int), ("used_bytes", ctypes.c_double), ("budget_bytes", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libpot3d.so.  Raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1709_01126_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    # torch ships its own HIP runtime.  If it is used in this process it must be
    # loaded first, so that the library binds to the same runtime instead of
    # loading a second one (two runtimes in one process do not share devices).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    d = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    i = ctypes.c_int
    lib.pot3d_create.argtypes = [d, i, d, i, d, i, i, i, i, ctypes.POINTER(vp)]
    lib.pot3d_create.restype = i
    lib.pot3d_solve.argtypes = [vp, d, ctypes.c_double, i, d, d, ctypes.POINTER(i), d]
    lib.pot3d_solve.restype = i
    lib.pot3d_solve_device.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, i, ctypes.POINTER(i), d]
    lib.pot3d_solve_device.restype = i
    lib.pot3d_apply_device.argtypes = [vp, vp, vp, vp]
    lib.pot3d_apply_device.restype = i
    lib.pot3d_precondition_device.argtypes = [vp, vp, vp, vp]
    lib.pot3d_precondition_device.restype = i
    lib.pot3d_rhs_device.argtypes = [vp, vp, vp, vp]
    lib.pot3d_rhs_device.restype = i
    lib.pot3d_pole_values.argtypes = [vp, d, d]
    lib.pot3d_pole_values.restype = i
    lib.pot3d_get_stats.argtypes = [vp, ctypes.POINTER(pot3d_stats)]
    lib.pot3d_get_stats.restype = i
    lib.pot3d_time_kernels.argtypes = [vp, i, d, d]
    lib.pot3d_time_kernels.restype = i
    lib.pot3d_set_refinement.argtypes = [vp, ctypes.c_double, i]
    lib.pot3d_set_refinement.restype = i
    lib.pot3d_set_refinement_mode.argtypes = [vp, i]
    lib.pot3d_set_refinement_mode.restype = i
    lib.pot3d_set_iteration.argtypes = [vp, i]
    lib.pot3d_set_iteration.restype = i
    lib.pot3d_set_preconditioner.argtypes = [vp, i]
    lib.pot3d_set_preconditioner.restype = i
    lib.pot3d_solve_noalloc.argtypes = [d, i, d, i, d, i, i, vp, vp, vp, vp, ctypes.c_double, i,
                                        ctypes.POINTER(i), d]
    lib.pot3d_solve_noalloc.restype = i
    lib.pot3d_field_device.argtypes = [vp, vp, vp, vp, vp]
    lib.pot3d_field_device.restype = i
    lib.pot3d_destroy.argtypes = [vp]
    lib.pot3d_destroy.restype = None
    lib.pot3d_last_error.argtypes = [vp]
    lib.pot3d_last_error.restype = ctypes.c_char_p
    lib.pot3d_version.argtypes = []
    lib.pot3d_version.restype = ctypes.c_char_p
    ll = ctypes.c_longlong
    lib.pot3d_server_create.argtypes = [i, i, i, ctypes.c_double, ctypes.POINTER(vp)]
    lib.pot3d_server_create.restype = i
    lib.pot3d_server_submit.argtypes = [vp, d, i, d, i, d, i, d, ctypes.c_double, i, d, ctypes.POINTER(ll)]
    lib.pot3d_server_submit.restype = i
    lib.pot3d_server_step.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(ll)]
    lib.pot3d_server_step.restype = i
    lib.pot3d_server_result.argtypes = [vp, ll, d, ctypes.POINTER(pot3d_request_info)]
    lib.pot3d_server_result.restype = i
    lib.pot3d_server_set_cache_budget.argtypes = [vp, ctypes.c_double]
    lib.pot3d_server_set_cache_budget.restype = i
    lib.pot3d_server_get_stats.argtypes = [vp, ctypes.POINTER(pot3d_server_stats)]
    lib.pot3d_server_get_stats.restype = i
    lib.pot3d_server_destroy.argtypes = [vp]
    lib.pot3d_server_destroy.restype = None
    lib.pot3d_server_last_error.argtypes = [vp]
    lib.pot3d_server_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise ValueError("expected a C-contiguous float64 numpy array")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# Grid shape (nr, nt, np) and device of every live context, so that host
# arrays can be checked against it before the C library reads or writes them.
_CTX_SHAPE = {}


def _host_in(a, n, name):
    """A host input array as C-contiguous float64 of exactly n elements (None stays None)."""
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"{name}: {a.size} elements, the grid needs {n}")
    return a


def _host_out(a, n, name):
    """A caller's output array: must already be C-contiguous float64 with n elements."""
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous and a.flags.writeable):
        raise ValueError(f"{name}: expected a writeable C-contiguous float64 numpy array")
    if a.size != n:
        raise ValueError(f"{name}: {a.size} elements, the grid needs {n}")
    return a


def _dev_tensor(t, n, device, name):
    """A torch tensor handed to the library as a device pointer: float64,
    contiguous, on the context's GPU, with exactly n elements."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name}: tensor on {t.device}, the context is on cuda:{device}")
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.float64")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} elements, expected {n}")
    return t


def _shape(ctx):
    try:
        return _CTX_SHAPE[ctx]
    except KeyError:
        raise ValueError("unknown or destroyed context handle") from None


class Pot3dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def pot3d_version() -> str:
    return load().pot3d_version().decode()


def pot3d_last_error(ctx=None) -> str:
    return load().pot3d_last_error(ctx).decode()


def pot3d_create(r_faces, t_faces, p_faces, upper_bc=UPPER_SOURCE_SURFACE, precision=FP64, device=0):
    """Returns (status, ctx handle or None)."""
    rf, tf, pf = _f64(r_faces), _f64(t_faces), _f64(p_faces)
    out = ctypes.c_void_p(None)
    st = load().pot3d_create(_dp(rf), rf.size - 1, _dp(tf), tf.size - 1, _dp(pf), pf.size - 1,
                             int(upper_bc), int(precision), int(device), ctypes.byref(out))
    if st == OK:
        _CTX_SHAPE[out.value] = (rf.size - 1, tf.size - 1, pf.size - 1, int(device))
    return st, (out.value if st == OK else None)


def pot3d_solve(ctx, br, tol, maxit, phi0, phi_out):
    """Host solve.  phi_out: preallocated float64 array of N.  Returns (status, iters, relres_true).
    Raises ValueError, before any C call, if an array does not have the grid's size."""
    nr, nt, np_, _ = _shape(ctx)
    br = _host_in(br, nt * np_, "br")
    phi0 = _host_in(phi0, nr * nt * np_, "phi0")
    _host_out(phi_out, nr * nt * np_, "phi")
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = load().pot3d_solve(ctx, _dp(br), float(tol), int(maxit), _dp(phi0), _dp(phi_out), ctypes.byref(it),
                            ctypes.byref(rr))
    return st, it.value, rr.value


def pot3d_solve_device(ctx, d_br, d_phi0, d_phi, stream, tol, maxit):
    """Device solve on raw device pointers (ints), as in C: the caller
    guarantees nt*np and N elements (Solver.solve_device checks tensors).
    Returns (status, iters, relres_true)."""
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = load().pot3d_solve_device(ctx, d_br, d_phi0, d_phi, stream, float(tol), int(maxit), ctypes.byref(it),
                                   ctypes.byref(rr))
    return st, it.value, rr.value


def pot3d_apply_device(ctx, d_x, d_y, stream=None):
    return load().pot3d_apply_device(ctx, d_x, d_y, stream)


def pot3d_precondition_device(ctx, d_r, d_z, stream=None):
    return load().pot3d_precondition_device(ctx, d_r, d_z, stream)


def pot3d_rhs_device(ctx, d_br, d_b, stream=None):
    return load().pot3d_rhs_device(ctx, d_br, d_b, stream)


def pot3d_pole_values(ctx, nr):
    if nr != _shape(ctx)[0]:
        raise ValueError(f"nr = {nr}, the context has {_shape(ctx)[0]} radial cells")
    north = np.empty(nr)
    south = np.empty(nr)
    st = load().pot3d_pole_values(ctx, _dp(north), _dp(south))
    return st, north, south


def pot3d_get_stats(ctx):
    s = pot3d_stats()
    st = load().pot3d_get_stats(ctx, ctypes.byref(s))
    return st, s.as_dict()


def pot3d_time_kernels(ctx, reps):
    a = ctypes.c_double(0.0)
    b = ctypes.c_double(0.0)
    st = load().pot3d_time_kernels(ctx, int(reps), ctypes.byref(a), ctypes.byref(b))
    return st, a.value, b.value


def pot3d_set_refinement(ctx, inner_tol, max_outer):
    return load().pot3d_set_refinement(ctx, float(inner_tol), int(max_outer))


def pot3d_set_refinement_mode(ctx, mode):
    return load().pot3d_set_refinement_mode(ctx, int(mode))


def pot3d_set_iteration(ctx, iteration):
    return load().pot3d_set_iteration(ctx, int(iteration))


def pot3d_set_preconditioner(ctx, pc):
    return load().pot3d_set_preconditioner(ctx, int(pc))


def pot3d_solve_noalloc(r_faces, t_faces, p_faces, upper_bc, d_br, d_phi0, d_phi, stream, tol, maxit):
    """The solve that allocates nothing, on raw device pointers (ints) as in
    C: the caller guarantees nt*np and N elements.  Returns (status, iters,
    relres_true)."""
    rf, tf, pf = _f64(r_faces), _f64(t_faces), _f64(p_faces)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = load().pot3d_solve_noalloc(_dp(rf), rf.size - 1, _dp(tf), tf.size - 1, _dp(pf), pf.size - 1, int(upper_bc),
                                    d_br, d_phi0, d_phi, stream, float(tol), int(maxit), ctypes.byref(it),
                                    ctypes.byref(rr))
    return st, it.value, rr.value


def pot3d_field_device(ctx, d_br, d_bt, d_bp, stream=None):
    return load().pot3d_field_device(ctx, d_br, d_bt, d_bp, stream)


def pot3d_destroy(ctx):
    if ctx:
        _CTX_SHAPE.pop(ctx, None)
        load().pot3d_destroy(ctx)


class Solver:
    """Owns one context; raises Pot3dError on EINVAL/ENOMEM/EDEVICE."""

    def __init__(self, r_faces, t_faces, p_faces, upper_bc=UPPER_SOURCE_SURFACE, precision=FP64, device=0,
                 iteration=None):
        st, ctx = pot3d_create(r_faces, t_faces, p_faces, upper_bc, precision, device)
        if st != OK:
            raise Pot3dError(st, pot3d_last_error(None))
        self.ctx = ctx
        self.nr, self.nt, self.np = len(r_faces) - 1, len(t_faces) - 1, len(p_faces) - 1
        self.device = int(device)
        if iteration is not None:
            self.set_iteration(iteration)

    @property
    def shape(self):
        return (self.nr, self.nt, self.np)

    def _check(self, st, allowed=(OK, ENOCONV, EBREAKDOWN)):
        if st not in allowed:
            raise Pot3dError(st, pot3d_last_error(self.ctx))
        return st

    def solve(self, br, tol, maxit, phi0=None):
        """Host arrays in, host Phi out.  Returns (phi, status, iters, relres_true)."""
        phi = np.empty(self.shape)
        st, it, rr = pot3d_solve(self.ctx, br, tol, maxit, phi0, phi)
        self._check(st)
        return phi, st, it, rr

    def solve_device(self, br, phi, tol, maxit, phi0=None, stream=None):
        """torch CUDA float64 tensors in/out on the given (or current) stream."""
        import torch

        n = self.nr * self.nt * self.np
        _dev_tensor(br, self.nt * self.np, self.device, "br")
        _dev_tensor(phi, n, self.device, "phi")
        if phi0 is not None:
            _dev_tensor(phi0, n, self.device, "phi0")
        if stream is None:
            stream = torch.cuda.current_stream(br.device)
        st, it, rr = pot3d_solve_device(self.ctx, br.data_ptr(), phi0.data_ptr() if phi0 is not None else None,
                                        phi.data_ptr(), stream.cuda_stream, tol, maxit)
        self._check(st)
        return st, it, rr

    def apply(self, x, y, stream=None):
        import torch

        n = self.nr * self.nt * self.np
        _dev_tensor(x, n, self.device, "x")
        _dev_tensor(y, n, self.device, "y")
        if x.data_ptr() == y.data_ptr():
            raise ValueError("x and y must be distinct buffers")
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        self._check(pot3d_apply_device(self.ctx, x.data_ptr(), y.data_ptr(), stream.cuda_stream), (OK,))

    def precondition(self, r, z, stream=None):
        """z = M^-1 r with the context's preconditioner (torch CUDA float64 tensors)."""
        import torch

        n = self.nr * self.nt * self.np
        _dev_tensor(r, n, self.device, "r")
        _dev_tensor(z, n, self.device, "z")
        if r.data_ptr() == z.data_ptr():
            raise ValueError("r and z must be distinct buffers")
        if stream is None:
            stream = torch.cuda.current_stream(r.device)
        self._check(pot3d_precondition_device(self.ctx, r.data_ptr(), z.data_ptr(), stream.cuda_stream), (OK,))

    def rhs(self, br, b, stream=None):
        import torch

        _dev_tensor(br, self.nt * self.np, self.device, "br")
        _dev_tensor(b, self.nr * self.nt * self.np, self.device, "b")
        if stream is None:
            stream = torch.cuda.current_stream(br.device)
        self._check(pot3d_rhs_device(self.ctx, br.data_ptr(), b.data_ptr(), stream.cuda_stream), (OK,))

    def pole_values(self):
        st, n, s = pot3d_pole_values(self.ctx, self.nr)
        self._check(st, (OK,))
        return n, s

    def stats(self):
        st, s = pot3d_get_stats(self.ctx)
        self._check(st, (OK,))
        return s

    def time_kernels(self, reps):
        st, a, b = pot3d_time_kernels(self.ctx, reps)
        self._check(st, (OK,))
        return a, b

    def set_refinement(self, inner_tol, max_outer=50):
        self._check(pot3d_set_refinement(self.ctx, inner_tol, max_outer), (OK,))

    def set_refinement_mode(self, mode):
        self._check(pot3d_set_refinement_mode(self.ctx, mode), (OK,))

    def set_iteration(self, iteration):
        self._check(pot3d_set_iteration(self.ctx, iteration), (OK,))

    def set_preconditioner(self, pc):
        self._check(pot3d_set_preconditioner(self.ctx, pc), (OK,))

    def field(self, stream=None):
        """B = -grad Phi of the last solution on the cell faces, as torch CUDA
        tensors (Br (nr+1, nt, np), Btheta (nr, nt+1, np), Bphi (nr, nt, np))."""
        import torch

        nr, nt, np_ = self.shape
        dev = torch.device("cuda", torch.cuda.current_device())
        br = torch.empty((nr + 1, nt, np_), dtype=torch.float64, device=dev)
        bt = torch.empty((nr, nt + 1, np_), dtype=torch.float64, device=dev)
        bp = torch.empty((nr, nt, np_), dtype=torch.float64, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self._check(pot3d_field_device(self.ctx, br.data_ptr(), bt.data_ptr(), bp.data_ptr(), stream.cuda_stream), (OK,))
        return br, bt, bp

    def close(self):
        if self.ctx:
            pot3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def pot3d_server_last_error(sv=None) -> str:
    return load().pot3d_server_last_error(sv).decode()


def pot3d_server_create(device=0, precision=FP64, max_slots=8, hbm_budget_bytes=0.0):
    """Returns (status, server handle or None)."""
    out = ctypes.c_void_p(None)
    st = load().pot3d_server_create(int(device), int(precision), int(max_slots), float(hbm_budget_bytes),
                                    ctypes.byref(out))
    return st, (out.value if st == OK else None)


def pot3d_server_submit(sv, r_faces, t_faces, p_faces, br, tol, maxit, phi_out=None):
    """phi_out: None, or a float64 array of N that receives Phi at retirement
    (keep it alive until the request is done).  Returns (status, request id)."""
    rf, tf, pf = _f64(r_faces), _f64(t_faces), _f64(p_faces)
    nr, nt, np_ = rf.size - 1, tf.size - 1, pf.size - 1
    br = _host_in(br, nt * np_, "br")
    if phi_out is not None:
        _host_out(phi_out, nr * nt * np_, "phi_out")
    rid = ctypes.c_longlong(0)
    st = load().pot3d_server_submit(sv, _dp(rf), rf.size - 1, _dp(tf), tf.size - 1, _dp(pf), pf.size - 1, _dp(br),
                                    float(tol), int(maxit), _dp(phi_out), ctypes.byref(rid))
    return st, rid.value


def pot3d_server_step(sv):
    """Returns (status, active, queued, finished)."""
    a, q, f = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_longlong(0)
    st = load().pot3d_server_step(sv, ctypes.byref(a), ctypes.byref(q), ctypes.byref(f))
    return st, a.value, q.value, f.value


def pot3d_server_result(sv, rid, phi_out=None):
    """phi_out: None (query only) or a float64 array of the request's N.  Returns (status, info dict)."""
    info = pot3d_request_info()
    if phi_out is not None:
        st = load().pot3d_server_result(sv, int(rid), None, ctypes.byref(info))
        if st != OK:
            return st, info.as_dict()
        _host_out(phi_out, info.nr * info.nt * info.np, "phi_out")
    st = load().pot3d_server_result(sv, int(rid), _dp(phi_out), ctypes.byref(info))
    return st, info.as_dict()


def pot3d_server_set_cache_budget(sv, nbytes):
    return load().pot3d_server_set_cache_budget(sv, float(nbytes))


def pot3d_server_get_stats(sv):
    s = pot3d_server_stats()
    st = load().pot3d_server_get_stats(sv, ctypes.byref(s))
    return st, s.as_dict()


def pot3d_server_destroy(sv):
    if sv:
        load().pot3d_server_destroy(sv)


class Server:
    """Owns one continuous-batching server; raises Pot3dError on errors of the calls."""

    def __init__(self, precision=FP64, max_slots=8, hbm_budget_bytes=0.0, device=0):
        st, sv = pot3d_server_create(device, precision, max_slots, hbm_budget_bytes)
        if st != OK:
            raise Pot3dError(st, pot3d_server_last_error(None))
        self.sv = sv
        self.outputs = {}   # request id -> the array Phi is written into

    def _check(self, st):
        if st != OK:
            raise Pot3dError(st, pot3d_server_last_error(self.sv))

    def submit(self, r_faces, t_faces, p_faces, br, tol, maxit):
        """Queue a solve; Phi is written straight into an array the server
        object holds until take()."""
        phi = np.empty((len(r_faces) - 1, len(t_faces) - 1, len(p_faces) - 1))
        st, rid = pot3d_server_submit(self.sv, r_faces, t_faces, p_faces, br, tol, maxit, phi)
        self._check(st)
        self.outputs[rid] = phi
        return rid

    def step(self):
        """One step; returns (active, queued, finished)."""
        st, a, q, f = pot3d_server_step(self.sv)
        self._check(st)
        return a, q, f

    def info(self, rid):
        st, info = pot3d_server_result(self.sv, rid, None)
        self._check(st)
        return info

    def take(self, rid):
        """Phi and info of a finished request (which the server then forgets)."""
        phi = self.outputs[rid]
        st, info = pot3d_server_result(self.sv, rid, phi)
        self._check(st)
        if not info["done"]:
            raise Pot3dError(EINVAL, f"request {rid} is not done")
        del self.outputs[rid]
        return phi, info

    def set_cache_budget(self, nbytes):
        self._check(pot3d_server_set_cache_budget(self.sv, nbytes))

    def stats(self):
        st, s = pot3d_server_get_stats(self.sv)
        self._check(st)
        return s

    def close(self):
        if self.sv:
            pot3d_server_destroy(self.sv)
            self.sv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
