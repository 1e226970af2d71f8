"""Python binding of the C ABI in include/oci.h (argument marshalling only).

Every computation runs in liboci.so on the GPU.  The functions below carry the
ABI's names; ``OciContext`` wraps a context handle.  Device outputs may be
passed as torch CUDA tensors (PyTorch supplies device memory and the HIP
stream); host outputs are numpy arrays.

There is no fallback: if liboci.so is missing or cannot be loaded, importing
this module raises.
"""
import ctypes
import os

import numpy as np

try:  # torch first, so the library binds to the HIP runtime torch already loaded
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the environment
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboci.so")

OCI_OK, OCI_NOT_CONVERGED = 0, 1
OCI_EINVAL, OCI_ENOMEM, OCI_EDEVICE, OCI_ENONFINITE, OCI_ESTATE = -1, -2, -3, -4, -5
OCI_BC_VACUUM, OCI_BC_REFLECT, OCI_BC_INCIDENT = 0, 1, 2
OCI_PREC_FP64 = 0
OCI_PREC_FP32 = 1
OCI_FLAG_STRICT = 1
OCI_FLAG_COMPACT = 2

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class oci_problem(ctypes.Structure):
    _fields_ = [
        ("n_angles", ctypes.c_int32),
        ("mu", _dp), ("w", _dp),
        ("n_regions", ctypes.c_int32),
        ("cells", _ip),
        ("width", _dp), ("sigma_t", _dp), ("sigma_s", _dp), ("source", _dp),
        ("dt", ctypes.c_double), ("speed", ctypes.c_double),
        ("bc_left", ctypes.c_int32), ("bc_right", ctypes.c_int32),
        ("inc_left", _dp), ("inc_right", _dp),
        ("psi0", _dp),
        ("tol", ctypes.c_double),
        ("max_iters", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class oci_step_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("iter_ms", ctypes.c_double), ("launches", ctypes.c_int32),
                ("corrections", ctypes.c_int32), ("err_bound", ctypes.c_double)]

    def as_dict(self):
        return {"iterations": int(self.iterations), "status": int(self.status),
                "residual": float(self.residual), "ms": float(self.ms),
                "iter_ms": float(self.iter_ms), "launches": int(self.launches),
                "err_bound": float(self.err_bound), "corrections": int(self.corrections)}


class OciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_lib.oci_strerror(code).decode(), code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liboci.so not built: run `python -m paper_2305_13555_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    sig = {
        "oci_setup": (ctypes.c_int, [ctypes.POINTER(oci_problem), vp, ctypes.POINTER(vp)]),
        "oci_refactor": (ctypes.c_int, [vp, ctypes.POINTER(oci_problem)]),
        "oci_step": (ctypes.c_int, [vp, ctypes.POINTER(oci_step_info)]),
        "si_step": (ctypes.c_int, [vp, ctypes.POINTER(oci_step_info)]),
        "oci_solve": (ctypes.c_int, [vp, ctypes.c_int32, vp, ctypes.c_int32,
                                     ctypes.POINTER(oci_step_info)]),
        "oci_solve_batch": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(vp), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.POINTER(oci_step_info)),
                                           ctypes.c_int32]),
        "oci_solve_ensemble": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(vp),
                                              ctypes.POINTER(ctypes.POINTER(oci_step_info))]),
        "oci_get_flux": (ctypes.c_int, [vp, vp, ctypes.c_int32]),
        "oci_get_state": (ctypes.c_int, [vp, _dp, ctypes.POINTER(ctypes.c_int64)]),
        "oci_set_state": (ctypes.c_int, [vp, _dp, ctypes.c_int64]),
        "oci_get_quadrature": (ctypes.c_int, [vp, _dp, _dp]),
        "oci_get_sizes": (ctypes.c_int, [vp, _ip, _ip, _ip]),
        "oci_iterates_per_launch": (ctypes.c_int, [vp]),
        "oci_set_iterates_per_launch": (ctypes.c_int, [vp, ctypes.c_int32]),
        "oci_end_fusion": (ctypes.c_int, [vp]),
        "oci_set_end_fusion": (ctypes.c_int, [vp, ctypes.c_int32]),
        "oci_inner_iterations": (ctypes.c_int, [vp]),
        "oci_set_inner_iterations": (ctypes.c_int, [vp, ctypes.c_int32]),
        "oci_get_operator": (ctypes.c_int, [vp, ctypes.c_int32, _dp]),
        "oci_destroy": (None, [vp]),
        "oci_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "oci_last_error": (ctypes.c_char_p, [vp]),
        "oci_gauss_legendre": (ctypes.c_int, [ctypes.c_int32, _dp, _dp]),
        "oci_corrector_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32, vp, ctypes.POINTER(vp)]),
        "oci_corrector_num_weights": (ctypes.c_int64, [vp]),
        "oci_corrector_set_weights": (ctypes.c_int, [vp, _dp]),
        "oci_corrector_get_weights": (ctypes.c_int, [vp, _dp]),
        "oci_corrector_forward": (ctypes.c_int, [vp, vp, ctypes.c_int32, ctypes.c_int32, vp]),
        "oci_corrector_grad": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, _dp,
                                              _dp]),
        "oci_corrector_train_step": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_double, _dp]),
        "oci_corrector_last_error": (ctypes.c_char_p, [vp]),
        "oci_corrector_destroy": (None, [vp]),
        "oci_corrector_forward_noalloc": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp,
                                                         ctypes.c_int32, ctypes.c_int32, vp, vp]),
        "oci_corrector_forward32": (ctypes.c_int, [vp, vp, ctypes.c_int32, ctypes.c_int32, vp]),
        "oci_set_corrector": (ctypes.c_int, [vp, vp, ctypes.c_int32, ctypes.c_int32]),
        "oci_step_history": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp,
                                            ctypes.c_int32, ctypes.POINTER(oci_step_info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _check(code, ctx=None):
    if code < 0:
        raise OciError(code, (_lib.oci_last_error(ctx) or b"").decode())
    return code


def _stream_handle(stream):
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def oci_gauss_legendre(n):
    """The N-point Gauss-Legendre rule computed by the library (host only)."""
    mu = np.zeros(n)
    w = np.zeros(n)
    _check(_lib.oci_gauss_legendre(int(n), _ptr(mu), _ptr(w)))
    return mu, w


def make_problem(prob, tol=None, max_iters=None, strict=None, precision=None, compact=False):
    """Marshal a problem description (attributes as in the workloads module)
    into the C struct.  Returns (struct, keepalive) - keep both alive."""
    keep = {
        "cells": np.ascontiguousarray(prob.cells, dtype=np.int32),
        "width": _f64(prob.width), "sigma_t": _f64(prob.sigma_t),
        "sigma_s": _f64(prob.sigma_s), "source": _f64(prob.source),
        "mu": _f64(getattr(prob, "mu", None)), "w": _f64(getattr(prob, "w", None)),
        "inc_left": _f64(getattr(prob, "inc_left", None)),
        "inc_right": _f64(getattr(prob, "inc_right", None)),
        "psi0": _f64(getattr(prob, "psi0", None)),
    }
    p = oci_problem()
    p.n_angles = int(prob.n_angles)
    p.mu = _ptr(keep["mu"])
    p.w = _ptr(keep["w"])
    p.n_regions = int(len(keep["cells"]))
    p.cells = keep["cells"].ctypes.data_as(_ip)
    p.width = _ptr(keep["width"])
    p.sigma_t = _ptr(keep["sigma_t"])
    p.sigma_s = _ptr(keep["sigma_s"])
    p.source = _ptr(keep["source"])
    p.dt = float(prob.dt)
    p.speed = float(prob.speed)
    p.bc_left = int(prob.bc_left)
    p.bc_right = int(prob.bc_right)
    p.inc_left = _ptr(keep["inc_left"])
    p.inc_right = _ptr(keep["inc_right"])
    p.psi0 = _ptr(keep["psi0"])
    p.tol = float(prob.tol if tol is None else tol)
    p.max_iters = int(prob.max_iters if max_iters is None else max_iters)
    p.precision = int(getattr(prob, "precision", OCI_PREC_FP64) if precision is None
                      else precision)
    st = bool(getattr(prob, "strict", False) if strict is None else strict)
    p.flags = (OCI_FLAG_STRICT if st else 0) | (OCI_FLAG_COMPACT if compact else 0)
    return p, keep


def oci_setup(prob, stream=None, tol=None, max_iters=None, strict=None, precision=None,
              compact=False):
    """Build a context for the problem; returns the raw handle (c_void_p)."""
    p, keep = make_problem(prob, tol, max_iters, strict, precision, compact)
    h = ctypes.c_void_p()
    _check(_lib.oci_setup(ctypes.byref(p), _stream_handle(stream), ctypes.byref(h)))
    del keep
    return h


def oci_refactor(ctx, prob, tol=None, max_iters=None, strict=None, precision=None):
    """Rebuild the operators for new region data of the same shape."""
    p, keep = make_problem(prob, tol, max_iters, strict, precision)
    _check(_lib.oci_refactor(ctx, ctypes.byref(p)), ctx)
    del keep


def oci_step(ctx):
    info = oci_step_info()
    rc = _check(_lib.oci_step(ctx, ctypes.byref(info)), ctx)
    return rc, info.as_dict()


def si_step(ctx):
    info = oci_step_info()
    rc = _check(_lib.si_step(ctx, ctypes.byref(info)), ctx)
    return rc, info.as_dict()


def _out_pointer(out):
    """(pointer, on_device) for a numpy array or a torch CUDA tensor."""
    if out is None:
        return None, 0
    if torch is not None and isinstance(out, torch.Tensor):
        if out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("output tensor must be contiguous float64")
        return ctypes.c_void_p(out.data_ptr()), 1 if out.is_cuda else 0
    if not (isinstance(out, np.ndarray) and out.dtype == np.float64 and out.flags.c_contiguous):
        raise ValueError("output array must be C-contiguous float64")
    return ctypes.c_void_p(out.ctypes.data), 0


def oci_solve(ctx, n_steps, phi_out=None):
    """n_steps OCI steps; phi_out [n_steps][J][4] numpy array or CUDA tensor, or None."""
    ptr, dev = _out_pointer(phi_out)
    infos = (oci_step_info * max(int(n_steps), 1))()
    rc = _check(_lib.oci_solve(ctx, int(n_steps), ptr, dev, infos), ctx)
    return rc, [infos[i].as_dict() for i in range(int(n_steps))]


def oci_solve_batch(ctxs, n_steps, phi_outs=None, n_threads=0):
    """n_steps OCI steps on each context (OciContext or handle), the contexts
    driven concurrently by up to n_threads host threads (0: library default);
    phi_outs: None or one output per context ([n_steps][J][4] numpy array or
    CUDA tensor, or None), all on the host or all on the device.  Returns
    (rc, [infos per context])."""
    n = len(ctxs)
    vp = ctypes.c_void_p
    handles = (vp * n)(*[c.handle if isinstance(c, OciContext) else c for c in ctxs])
    phi_arr, dev = None, 1
    if phi_outs is not None:
        ptrs = [_out_pointer(o) for o in phi_outs]
        devs = {d for p, d in ptrs if p is not None}
        if len(devs) > 1:
            raise ValueError("phi outputs must be all on the host or all on the device")
        dev = devs.pop() if devs else 1
        phi_arr = (vp * n)(*[p for p, _ in ptrs])
    steps = max(int(n_steps), 1)
    arrays = [(oci_step_info * steps)() for _ in range(n)]
    infos = (ctypes.POINTER(oci_step_info) * n)(
        *[ctypes.cast(a, ctypes.POINTER(oci_step_info)) for a in arrays])
    rc = _lib.oci_solve_batch(handles, n, int(n_steps), phi_arr, dev, infos, int(n_threads))
    if rc < 0:
        msgs = [(_lib.oci_last_error(h) or b"").decode() for h in handles]
        raise OciError(rc, "; ".join(m for m in msgs if m) or "batch solve failed")
    return rc, [[a[i].as_dict() for i in range(int(n_steps))] for a in arrays]


def oci_solve_ensemble(ctxs, n_steps, phi_outs=None):
    """n_steps OCI steps of every context (OciContext or handle) advanced together,
    one launch per iteration over all their tiles (work on the first context's
    stream); phi_outs: None or one CUDA tensor [n_steps][J][4] (or None) per
    context.  Returns (rc, [infos per context])."""
    n = len(ctxs)
    vp = ctypes.c_void_p
    handles = (vp * n)(*[c.handle if isinstance(c, OciContext) else c for c in ctxs])
    phi_arr = None
    if phi_outs is not None:
        ptrs = []
        for o in phi_outs:
            p, dev = _out_pointer(o)
            if p is not None and not dev:
                raise ValueError("ensemble outputs must be device tensors")
            ptrs.append(p)
        phi_arr = (vp * n)(*ptrs)
    steps = max(int(n_steps), 1)
    arrays = [(oci_step_info * steps)() for _ in range(n)]
    infos = (ctypes.POINTER(oci_step_info) * n)(
        *[ctypes.cast(a, ctypes.POINTER(oci_step_info)) for a in arrays])
    rc = _lib.oci_solve_ensemble(handles, n, int(n_steps), phi_arr, infos)
    if rc < 0:
        msgs = [(_lib.oci_last_error(h) or b"").decode() for h in handles]
        raise OciError(rc, "; ".join(m for m in msgs if m) or "ensemble solve failed")
    return rc, [[a[i].as_dict() for i in range(int(n_steps))] for a in arrays]


def oci_get_sizes(ctx):
    n, j, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.oci_get_sizes(ctx, ctypes.byref(n), ctypes.byref(j), ctypes.byref(r)), ctx)
    return n.value, j.value, r.value


def oci_iterates_per_launch(ctx):
    return _check(_lib.oci_iterates_per_launch(ctx), ctx)


def oci_set_iterates_per_launch(ctx, k):
    return _check(_lib.oci_set_iterates_per_launch(ctx, int(k)), ctx)


def oci_end_fusion(ctx):
    return _check(_lib.oci_end_fusion(ctx), ctx)


def oci_set_end_fusion(ctx, on):
    return _check(_lib.oci_set_end_fusion(ctx, 1 if on else 0), ctx)


def oci_inner_iterations(ctx):
    return _check(_lib.oci_inner_iterations(ctx), ctx)


def oci_set_inner_iterations(ctx, m):
    return _check(_lib.oci_set_inner_iterations(ctx, int(m)), ctx)


def oci_get_flux(ctx, out=None):
    n, J, _ = oci_get_sizes(ctx)
    if out is None:
        out = np.zeros((J, 4))
    ptr, dev = _out_pointer(out)
    _check(_lib.oci_get_flux(ctx, ptr, dev), ctx)
    return out


def oci_get_state(ctx):
    n, J, _ = oci_get_sizes(ctx)
    psi = np.zeros((J, n, 2))
    step = ctypes.c_int64()
    _check(_lib.oci_get_state(ctx, _ptr(psi), ctypes.byref(step)), ctx)
    return psi, step.value


def oci_set_state(ctx, psi_edge, step=0):
    a = _f64(psi_edge)
    _check(_lib.oci_set_state(ctx, _ptr(a), int(step)), ctx)


def oci_get_quadrature(ctx):
    n, _, _ = oci_get_sizes(ctx)
    mu, w = np.zeros(n), np.zeros(n)
    _check(_lib.oci_get_quadrature(ctx, _ptr(mu), _ptr(w)), ctx)
    return mu, w


def oci_get_operator(ctx, region):
    n, _, _ = oci_get_sizes(ctx)
    op = np.zeros((4 * n + 4, 4 * n + 1))
    _check(_lib.oci_get_operator(ctx, int(region), _ptr(op)), ctx)
    return op


def oci_destroy(ctx):
    _lib.oci_destroy(ctx)


def oci_strerror(code):
    return _lib.oci_strerror(int(code)).decode()


class OciContext:
    """Owning wrapper around a context handle."""

    def __init__(self, prob, stream=None, tol=None, max_iters=None, strict=None,
                 precision=None, compact=False):
        self.precision = precision
        self.handle = oci_setup(prob, stream, tol, max_iters, strict, precision, compact)
        self.n_angles, self.n_cells, self.n_regions = oci_get_sizes(self.handle)
        self.iterates_per_launch = oci_iterates_per_launch(self.handle)

    def set_iterates_per_launch(self, k):
        self.iterates_per_launch = oci_set_iterates_per_launch(self.handle, k)
        return self.iterates_per_launch

    @property
    def end_fusion(self):
        return bool(oci_end_fusion(self.handle))

    def set_end_fusion(self, on):
        return bool(oci_set_end_fusion(self.handle, on))

    @property
    def inner_iterations(self):
        return oci_inner_iterations(self.handle)

    def set_inner_iterations(self, m):
        return oci_set_inner_iterations(self.handle, m)

    def set_corrector(self, corrector, first=3, period=8):
        """Attach a Corrector (or None to detach) for learned corrections
        inside the iteration; the corrector must outlive the attachment."""
        h = corrector._h if corrector is not None else None
        _check(_lib.oci_set_corrector(self.handle, h, int(first), int(period)), self.handle)
        self._corrector = corrector

    def step_history(self, n_hist, first=1, out=None):
        """One plain step that also returns the scalar flux of its iterates
        first .. first + n_hist - 1 ([n_hist][J][4], numpy or CUDA tensor)."""
        if out is None:
            out = np.zeros((int(n_hist), self.n_cells, 4))
        ptr, dev = _out_pointer(out)
        info = oci_step_info()
        rc = _check(_lib.oci_step_history(self.handle, int(first), int(n_hist), ptr, dev,
                                          ctypes.byref(info)), self.handle)
        return rc, info.as_dict(), out

    def refactor(self, prob, tol=None, max_iters=None, strict=None):
        oci_refactor(self.handle, prob, tol, max_iters, strict, self.precision)

    def step(self):
        return oci_step(self.handle)

    def si_step(self):
        return si_step(self.handle)

    def solve(self, n_steps, phi_out=None):
        return oci_solve(self.handle, n_steps, phi_out)

    def flux(self, out=None):
        return oci_get_flux(self.handle, out)

    def state(self):
        return oci_get_state(self.handle)

    def set_state(self, psi_edge, step=0):
        oci_set_state(self.handle, psi_edge, step)

    def quadrature(self):
        return oci_get_quadrature(self.handle)

    def operator(self, region):
        return oci_get_operator(self.handle, region)

    def close(self):
        if self.handle is not None:
            oci_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def oci_corrector_forward_noalloc(w, c_in, c_out, x, out, stream=None):
    """y = f(x) with no allocation inside the library: w (weights), x
    [batch][c_in][cells] and out [batch][c_out][cells] are float64 device
    tensors; enqueued on the stream (default: torch's current stream).
    Returns the library's code (OCI_EINVAL for sizes beyond its limit)."""
    for t in (w, x, out):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("w, x and out must be contiguous float64 device tensors")
    B, J = int(x.shape[0]), int(x.shape[2])
    return _lib.oci_corrector_forward_noalloc(
        ctypes.c_void_p(w.data_ptr()), int(c_in), int(c_out), ctypes.c_void_p(x.data_ptr()), B, J,
        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))


class Corrector:
    """The learned iterate corrector (oci_corrector_* in include/oci.h):
    inputs [batch][c_in][cells], outputs [batch][c_out][cells], FP64 device
    tensors.  Its kernels run on the stream given here (default: torch's
    current stream at creation); tensors passed in must be ready on it."""

    def __init__(self, c_in, c_out, max_batch, max_cells, stream=None):
        h = ctypes.c_void_p()
        code = _lib.oci_corrector_create(int(c_in), int(c_out), int(max_batch), int(max_cells),
                                         _stream_handle(stream), ctypes.byref(h))
        if code < 0:
            raise OciError(code, "oci_corrector_create")
        self._h = h
        self.c_in, self.c_out = int(c_in), int(c_out)

    def _check(self, code):
        if code < 0:
            raise OciError(code, (_lib.oci_corrector_last_error(self._h) or b"").decode())
        return code

    @property
    def num_weights(self):
        return int(_lib.oci_corrector_num_weights(self._h))

    def set_weights(self, w):
        w = _f64(w)
        if w.size != self.num_weights:
            raise ValueError("expected %d weights" % self.num_weights)
        self._check(_lib.oci_corrector_set_weights(self._h, _ptr(w)))

    def weights(self):
        w = np.zeros(self.num_weights)
        self._check(_lib.oci_corrector_get_weights(self._h, _ptr(w)))
        return w

    def _shape(self, x, channels):
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.dim() != 3 \
                or x.shape[1] != channels:
            raise ValueError("expected a contiguous float64 device tensor [batch][%d][cells]"
                             % channels)
        return int(x.shape[0]), int(x.shape[2])

    def forward(self, x, out=None):
        B, J = self._shape(x, self.c_in)
        if out is None:
            out = torch.empty((B, self.c_out, J), dtype=torch.float64, device=x.device)
        self._shape(out, self.c_out)
        self._check(_lib.oci_corrector_forward(self._h, ctypes.c_void_p(x.data_ptr()), B, J,
                                               ctypes.c_void_p(out.data_ptr())))
        return out

    def forward32(self, x, out=None):
        """FP32 inference on the matrix cores: x [batch][c_in][cells] float32
        device tensor."""
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous() or x.dim() != 3 \
                or x.shape[1] != self.c_in:
            raise ValueError("expected a contiguous float32 device tensor [batch][%d][cells]"
                             % self.c_in)
        B, J = int(x.shape[0]), int(x.shape[2])
        if out is None:
            out = torch.empty((B, self.c_out, J), dtype=torch.float32, device=x.device)
        self._check(_lib.oci_corrector_forward32(self._h, ctypes.c_void_p(x.data_ptr()), B, J,
                                                 ctypes.c_void_p(out.data_ptr())))
        return out

    def grad(self, x, target):
        B, J = self._shape(x, self.c_in)
        self._shape(target, self.c_out)
        loss = ctypes.c_double()
        g = np.zeros(self.num_weights)
        self._check(_lib.oci_corrector_grad(self._h, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(target.data_ptr()), B, J,
                                            ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def train_step(self, x, target, lr):
        B, J = self._shape(x, self.c_in)
        self._shape(target, self.c_out)
        loss = ctypes.c_double()
        self._check(_lib.oci_corrector_train_step(self._h, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(target.data_ptr()), B, J,
                                                  float(lr), ctypes.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.oci_corrector_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()
