"""Python binding of the gfx950 gradient-domain stack solver (``libgd.so``).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides device memory and the current stream.  The binding refuses
to run when the HIP library is missing; there is no CPU fallback.

Entry points follow ``include/gd.h``:

* :func:`smooth_z`                  anisotropic diffusion of a stack, Eq. (1)
* :func:`screened_poisson_slices`   per-slice screened Poisson, Eq. (2),
                                    for a batch of slices of any sizes
* :func:`screened_poisson_stack`    the same for the slices of one stack
* :class:`Hierarchy`                the general Sec. 4 system: rhs + V-cycles
* :func:`rb_sweep`, :func:`residual_restrict`, :func:`prolong_add`
                                    single multigrid steps (Sec. 4.1)
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgd.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
OK, ERR_INVALID, ERR_NOMEM, ERR_HIP, ERR_NOT_CONVERGED, ERR_NUMERIC, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6


class GDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gd status {status}: {msg}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("rel_tol", ctypes.c_double),
        ("max_cycles", ctypes.c_int),
        ("pre_smooth", ctypes.c_int),
        ("post_smooth", ctypes.c_int),
        ("storage", ctypes.c_int),
        ("fp64_refine", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
        ("prolong", ctypes.c_int),
        ("timing", ctypes.c_int),
        ("fuse_prolong", ctypes.c_int),
        ("sweep_tile", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("fmg", ctypes.c_int),
        ("discretization", ctypes.c_int),
        ("sweep_quad", ctypes.c_int),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int),
        ("refine_steps", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
        ("b_norm", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("levels", ctypes.c_int),
        ("fallback_used", ctypes.c_int),
        ("bytes", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SliceDesc(ctypes.Structure):
    _fields_ = [
        ("offset", ctypes.c_int64),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("pitch", ctypes.c_int32),
        ("alpha", ctypes.c_float),
    ]


_lib = None
_vp, _i64, _d, _i = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int

_SIGS = {
    "gd_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
    "gd_last_error": (ctypes.c_char_p, []),
    "gd_version": (ctypes.c_char_p, []),
    "gd_smooth_z": (_i, [_vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d, ctypes.POINTER(SolveOpts),
                         ctypes.POINTER(Report), _vp]),
    "gd_smooth_z_noalloc": (_i, [_vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(Report), _vp]),
    "gd_noalloc_scratch_bytes": (_i, [ctypes.POINTER(_i64)]),
    "gd_screened_poisson_slices": (_i, [_vp, _i, _vp, _i, _vp, _i, ctypes.POINTER(SliceDesc), _i64, _d, _d,
                                        ctypes.POINTER(SolveOpts), ctypes.POINTER(Report),
                                        ctypes.POINTER(Report), _vp]),
    "gd_dct_solve": (_i, [_vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d, _d, _vp]),
    "gd_dct_smooth_z": (_i, [_vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d, _vp]),
    "gd_npr_filter": (_i, [_vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d, _d, _d, _d, ctypes.POINTER(SolveOpts),
                           ctypes.POINTER(Report), _vp]),
    "gd_hierarchy_create": (_i, [ctypes.POINTER(_vp), _i64, _i64, _i64, _d, _d, _d, _d, _i,
                                 ctypes.POINTER(SolveOpts), _vp]),
    "gd_hierarchy_destroy": (_i, [_vp]),
    "gd_hierarchy_info": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i64), ctypes.POINTER(_d)]),
    "gd_rhs_general": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gd_vcycle": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d), _vp]),
    "gd_hierarchy_create_streamed": (_i, [ctypes.POINTER(_vp), _i64, _i64, _i64, _d, _d, _d, _d, _i,
                                          ctypes.POINTER(SolveOpts), _i64, _i, _vp]),
    "gd_vcycle_streamed": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d), _vp]),
    "gd_screened_poisson_streamed": (_i, [_vp, _i, _vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d,
                                          ctypes.POINTER(SolveOpts), _i64, _i64, ctypes.POINTER(Report),
                                          ctypes.POINTER(Report), _vp]),
    "gd_smooth_z_streamed": (_i, [_vp, _i, _vp, _i, _i64, _i64, _i64, _d, _d, _d, ctypes.POINTER(SolveOpts), _i64,
                                  _i, _i64, ctypes.POINTER(Report), _vp]),
    "gd_hierarchy_device_bytes": (_i, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "gd_hierarchy_streamed_levels": (_i, [_vp, ctypes.POINTER(_i)]),
    "gd_rb_sweep": (_i, [_vp, _vp, _vp, _i, _i64, _i64, _i64, _d, _d, _d, _d, _vp]),
    "gd_residual_restrict": (_i, [_vp, _vp, _vp, _i, _i64, _i64, _i64, _i, _i, _i, _d, _d, _d, _d,
                                  ctypes.POINTER(_d), _vp]),
    "gd_prolong_add": (_i, [_vp, _vp, _i, _i64, _i64, _i64, _i, _i, _i, _i, _vp]),
    "gd_get_kernel_time": (_i, [_i, ctypes.POINTER(_d), ctypes.POINTER(_i64), ctypes.POINTER(_d)]),
    "gd_reset_kernel_time": (None, []),
    "gd_release_workspace": (_i, []),
    "gd_sweep_config": (_i, [_i64, _i64, _i64, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i64),
                             ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "gd_mg_error_pairs": (_i, [_vp, _vp, _vp, _i, _vp, _vp, _vp]),
    "gd_net_create": (_i, [ctypes.POINTER(_vp), _vp, _i64, ctypes.c_uint64]),
    "gd_net_destroy": (_i, [_vp]),
    "gd_net_num_params": (_i64, [_vp]),
    "gd_net_get_params": (_i, [_vp, _vp, _i64]),
    "gd_net_set_params": (_i, [_vp, _vp, _i64]),
    "gd_net_last_error": (ctypes.c_char_p, []),
    "gd_net_forward": (_i, [_vp, _vp, _vp, _i64, _i64, _i64, _vp]),
    "gd_net_gradients": (_i, [_vp, _vp, _vp, _i64, _i64, _i64, _vp, ctypes.POINTER(_d), _vp]),
    "gd_net_train_step": (_i, [_vp, _vp, _vp, _i64, _i64, _i64, ctypes.c_float, ctypes.POINTER(_d), _vp]),
    "gd_net_set_timing": (_i, [_vp, _i]),
    "gd_net_kernel_time": (_i, [_vp, _i, ctypes.POINTER(_d), ctypes.POINTER(_i64), ctypes.POINTER(_d)]),
    "gd_fcg_solve": (_i, [_vp, _vp, _vp, _vp, _i, _d, _i, ctypes.POINTER(Report), _vp]),
}


def exported_symbols():
    """Names every C-ABI entry point must export (as declared in gd.h)."""
    return sorted(_SIGS)


def load(path=LIB_PATH):
    """Load libgd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run python -m paper_1310_0041_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, allow=(), net=False):
    if status != OK and status not in allow:
        msg = (_lib.gd_net_last_error() if net else _lib.gd_last_error()).decode()
        raise GDError(status, msg)
    return status


def default_opts(**kw):
    o = SolveOpts()
    load().gd_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _torch():
    import torch

    return torch


def gd_dtype(t):
    torch = _torch()
    m = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
    if t not in m:
        raise TypeError(f"unsupported dtype {t}")
    return m[t]


def torch_dtype(code):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[code]


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, shape, dtype, name):
    """Refuse a tensor the kernels would read or write out of bounds."""
    if t is None:
        raise ValueError(f"{name} is required")
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
        raise ValueError(f"{name} must be {tuple(shape)} {dtype}, got {tuple(t.shape)} {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous GPU tensor")
    return t


_DESC_NP = np.dtype([("offset", "<i8"), ("nx", "<i4"), ("ny", "<i4"), ("pitch", "<i4"), ("alpha", "<f4")])


def slice_span(descs):
    """Elements an array must hold for the slices of ``descs``: the largest
    offset + pitch * (ny - 1) + nx."""
    if len(descs) == 0:
        return 0
    d = np.frombuffer(descs, dtype=_DESC_NP, count=len(descs))
    return int((d["offset"] + d["pitch"].astype(np.int64) * (d["ny"].astype(np.int64) - 1) + d["nx"]).max())


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def smooth_z(I0, beta=(1.0, 1.0, 4.0), out_dtype=None, opts=None, check=True, **kw):
    """Anisotropic diffusion of the [nz][ny][nx] stack I0 (Eq. (1)).
    Returns (I1, report dict)."""
    lib = load()
    nz, ny, nx = I0.shape
    out = _torch().empty_like(I0, dtype=out_dtype or I0.dtype)
    o = opts or default_opts(**kw)
    rep = Report()
    st = lib.gd_smooth_z(_ptr(I0), gd_dtype(I0.dtype), _ptr(out), gd_dtype(out.dtype), nx, ny, nz,
                         float(beta[0]), float(beta[1]), float(beta[2]), ctypes.byref(o), ctypes.byref(rep),
                         _stream())
    if check:
        _check(st)
    return out, dict(rep.as_dict(), status=st)


def smooth_z_into(I0, out, beta=(1.0, 1.0, 4.0), opts=None, check=True, **kw):
    """:func:`smooth_z` into the caller's ``out`` (any dtype).  Returns the report."""
    lib = load()
    nz, ny, nx = I0.shape
    _need(out, I0.shape, out.dtype, "out")
    _ptr(I0)
    o = opts or default_opts(**kw)
    rep = Report()
    st = lib.gd_smooth_z(_ptr(I0), gd_dtype(I0.dtype), _ptr(out), gd_dtype(out.dtype), nx, ny, nz,
                         float(beta[0]), float(beta[1]), float(beta[2]), ctypes.byref(o), ctypes.byref(rep),
                         _stream())
    if check:
        _check(st)
    return dict(rep.as_dict(), status=st)


def smooth_z_noalloc(I0, out, beta=(1.0, 1.0, 4.0), opts=None, check=True, **kw):
    """Anisotropic diffusion (Eq. (1)) into the caller's ``out`` without any
    allocation by the library (its hierarchy lives in a static scratch array
    of :func:`noalloc_scratch_bytes` bytes per GPU).  Returns the report."""
    lib = load()
    nz, ny, nx = I0.shape
    _need(out, I0.shape, out.dtype, "out")
    _ptr(I0)
    o = opts or default_opts(**kw)
    rep = Report()
    st = lib.gd_smooth_z_noalloc(_ptr(I0), gd_dtype(I0.dtype), _ptr(out), gd_dtype(out.dtype), nx, ny, nz,
                                 float(beta[0]), float(beta[1]), float(beta[2]), ctypes.byref(o), ctypes.byref(rep),
                                 _stream())
    if check:
        _check(st)
    return dict(rep.as_dict(), status=st)


def noalloc_scratch_bytes():
    n = ctypes.c_int64()
    _check(load().gd_noalloc_scratch_bytes(ctypes.byref(n)))
    return n.value


def npr_filter(I0, alpha=0.001, beta=(1.0, 1.0, 0.1), lam=1.25, sigma=5.0, out_dtype=None, opts=None, check=True,
               **kw):
    """Gradient-modulation filter of the [nz][ny][nx] volume I0 (Sec. 6).
    Returns (I1, report dict)."""
    lib = load()
    nz, ny, nx = I0.shape
    out = _torch().empty_like(I0, dtype=out_dtype or I0.dtype)
    o = opts or default_opts(**kw)
    rep = Report()
    st = lib.gd_npr_filter(_ptr(I0), gd_dtype(I0.dtype), _ptr(out), gd_dtype(out.dtype), nx, ny, nz, float(alpha),
                           float(beta[0]), float(beta[1]), float(beta[2]), float(lam), float(sigma), ctypes.byref(o),
                           ctypes.byref(rep), _stream())
    if check:
        _check(st)
    return out, dict(rep.as_dict(), status=st)


def dct_solve(b, alpha, beta, out_dtype=None, check=True):
    """Spectral solve of (alpha + sum beta_a L_a) x = b (power-of-two grid)."""
    lib = load()
    nz, ny, nx = b.shape
    x = _torch().empty_like(b, dtype=out_dtype or b.dtype)
    st = lib.gd_dct_solve(_ptr(b), gd_dtype(b.dtype), _ptr(x), gd_dtype(x.dtype), nx, ny, nz, float(alpha),
                          float(beta[0]), float(beta[1]), float(beta[2]), _stream())
    if check:
        _check(st)
    return x, st


def dct_smooth_z(I0, beta=(1.0, 1.0, 4.0), out_dtype=None, check=True):
    """Anisotropic diffusion of I0 (Eq. (1)) by the spectral solver."""
    lib = load()
    nz, ny, nx = I0.shape
    out = _torch().empty_like(I0, dtype=out_dtype or I0.dtype)
    st = lib.gd_dct_smooth_z(_ptr(I0), gd_dtype(I0.dtype), _ptr(out), gd_dtype(out.dtype), nx, ny, nz,
                             float(beta[0]), float(beta[1]), float(beta[2]), _stream())
    if check:
        _check(st)
    return out, st


def make_slice_descs(offsets, nx, ny, alpha, pitch=None):
    n = len(offsets)
    arr = (SliceDesc * n)()
    nx = np.broadcast_to(np.asarray(nx), (n,))
    ny = np.broadcast_to(np.asarray(ny), (n,))
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (n,))
    pitch = nx if pitch is None else np.broadcast_to(np.asarray(pitch), (n,))
    for i in range(n):
        arr[i] = SliceDesc(int(offsets[i]), int(nx[i]), int(ny[i]), int(pitch[i]), float(alpha[i]))
    return arr


def screened_poisson_slices(I0, I1, descs, beta_xy=(1.0, 1.0), opts=None, out=None, out_dtype=None, check=True,
                            **kw):
    """Per-slice screened Poisson (Eq. (2)) for a batch of slices described by
    ``descs`` (from :func:`make_slice_descs`).  I1 has I0's dtype, float32 or
    float64; the output (``out``, else a new tensor of ``out_dtype``, default
    I0's dtype) may have any.  Returns (I2, report, per-slice reports)."""
    lib = load()
    torch = _torch()
    if I1.dtype not in (I0.dtype, torch.float32, torch.float64):
        raise ValueError("I1 must have I0's dtype, float32 or float64")
    if I0.shape != I1.shape:
        raise ValueError("I0 and I1 must share the shape")
    if out is None:
        out = torch.empty_like(I0, dtype=out_dtype or I0.dtype)
    elif out_dtype is not None and out.dtype != out_dtype:
        raise ValueError("out does not have out_dtype")
    span = slice_span(descs)
    for name, t in (("I0", I0), ("I1", I1), ("out", out)):
        _ptr(t)
        if t.numel() < span:
            raise ValueError(f"{name} holds {t.numel()} elements; the slices reach element {span - 1}")
    n = len(descs)
    o = opts or default_opts(**kw)
    rep = Report()
    per = (Report * n)()
    st = lib.gd_screened_poisson_slices(_ptr(I0), gd_dtype(I0.dtype), _ptr(I1), gd_dtype(I1.dtype), _ptr(out),
                                        gd_dtype(out.dtype), descs, n, float(beta_xy[0]), float(beta_xy[1]),
                                        ctypes.byref(o), ctypes.byref(rep), per, _stream())
    if check:
        _check(st)
    return out, dict(rep.as_dict(), status=st), [p.as_dict() for p in per]


def screened_poisson_stack(I0, I1, alpha=0.01, beta_xy=(1.0, 1.0), opts=None, out_dtype=None, check=True, **kw):
    """Eq. (2) for every slice of a [nz][ny][nx] stack."""
    nz, ny, nx = I0.shape
    descs = make_slice_descs(np.arange(nz) * nx * ny, nx, ny, alpha)
    return screened_poisson_slices(I0, I1, descs, beta_xy, opts=opts, out_dtype=out_dtype, check=check, **kw)


class Hierarchy:
    """Multigrid hierarchy of the general Sec. 4 system
    (alpha + sum_a beta_a L_a) x = alpha V + sum_a beta_a D_a^T G_a."""

    def __init__(self, shape, alpha, beta, dtype, opts=None, **kw):
        lib = load()
        nz, ny, nx = shape
        self.shape = tuple(shape)
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        o = opts or default_opts(**kw)
        _check(lib.gd_hierarchy_create(ctypes.byref(self._h), nx, ny, nz, float(alpha), float(beta[0]),
                                       float(beta[1]), float(beta[2]), gd_dtype(dtype), ctypes.byref(o),
                                       _stream()))

    def info(self, level=-1):
        n = ctypes.c_int()
        dims = (ctypes.c_int64 * 3)()
        coef = (ctypes.c_double * 4)()
        if level < 0:
            _check(_lib.gd_hierarchy_info(self._h, -1, ctypes.byref(n), None, None))
            return n.value
        _check(_lib.gd_hierarchy_info(self._h, level, ctypes.byref(n), dims, coef))
        return (dims[2], dims[1], dims[0]), tuple(coef)

    def rhs(self, V=None, Gx=None, Gy=None, Gz=None):
        for name, t in (("V", V), ("Gx", Gx), ("Gy", Gy), ("Gz", Gz)):
            if t is not None:
                _need(t, self.shape, self.dtype, name)
        b = _torch().empty(self.shape, dtype=self.dtype, device="cuda")
        _check(_lib.gd_rhs_general(self._h, _ptr(V), _ptr(Gx), _ptr(Gy), _ptr(Gz), _ptr(b), _stream()))
        return b

    def vcycle(self, x, b, ncycles=1):
        _need(x, self.shape, self.dtype, "x")
        _need(b, self.shape, self.dtype, "b")
        rr = ctypes.c_double()
        _check(_lib.gd_vcycle(self._h, _ptr(x), _ptr(b), int(ncycles), ctypes.byref(rr), _stream()))
        return rr.value

    def error_pairs(self, b, x_star, cycles):
        """(r_k, e_k) after `cycles` V-cycles from zero: b - A x_k and x_star - x_k."""
        _need(b, self.shape, self.dtype, "b")
        _need(x_star, self.shape, self.dtype, "x_star")
        r = _torch().empty_like(b)
        e = _torch().empty_like(b)
        _check(_lib.gd_mg_error_pairs(self._h, _ptr(b), _ptr(x_star), int(cycles), _ptr(r), _ptr(e), _stream()))
        return r, e

    def fcg(self, x, b, net=None, precond=0, rel_tol=1e-6, max_iter=200, check=True):
        """Flexible CG (x in/out); precond 0 V-cycle, 1 net, 2 V-cycle then net,
        3 net in place of the finest level's post-smoothing."""
        _need(x, self.shape, _torch().float32, "x")
        _need(b, self.shape, _torch().float32, "b")
        rep = Report()
        st = _lib.gd_fcg_solve(self._h, net._n if net is not None else None, _ptr(x), _ptr(b), int(precond),
                               float(rel_tol), int(max_iter), ctypes.byref(rep), _stream())
        if check:
            _check(st)
        d = rep.as_dict()
        d["iterations"] = d["cycles"]
        d["status"] = st
        return d

    def device_bytes(self):
        """(device bytes held, planes of the largest window; 0 unless streamed)."""
        b, w = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.gd_hierarchy_device_bytes(self._h, ctypes.byref(b), ctypes.byref(w)))
        return b.value, w.value

    def streamed_levels(self):
        n = ctypes.c_int()
        _check(_lib.gd_hierarchy_streamed_levels(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if self._h:
            _lib.gd_hierarchy_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_ptr(t):
    if t.is_cuda:
        raise ValueError("a streamed hierarchy takes host (CPU) tensors")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class StreamedHierarchy(Hierarchy):
    """A hierarchy whose finest level (and possibly the next large ones, see
    `levels`: 0 automatic, k > 0 at most k streamed levels) stays in host
    memory and is streamed through HBM in z-slabs of `slab` planes
    (Sec. 4.1); the other levels are resident.  vcycle takes CPU tensors
    (pinned ones let the copies overlap the kernels)."""

    def __init__(self, shape, alpha, beta, dtype, slab, levels=0, opts=None, **kw):
        lib = load()
        nz, ny, nx = shape
        self.shape = tuple(shape)
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        o = opts or default_opts(**kw)
        _check(lib.gd_hierarchy_create_streamed(ctypes.byref(self._h), nx, ny, nz, float(alpha), float(beta[0]),
                                                float(beta[1]), float(beta[2]), gd_dtype(dtype), ctypes.byref(o),
                                                int(slab), int(levels), _stream()))

    def vcycle(self, x, b, ncycles=1, relres=True):
        for t in (x, b):
            if tuple(t.shape) != self.shape or t.dtype != self.dtype:
                raise ValueError("x and b must have the hierarchy's shape and dtype")
        rr = ctypes.c_double()
        _check(_lib.gd_vcycle_streamed(self._h, _host_ptr(x), _host_ptr(b), int(ncycles),
                                       ctypes.byref(rr) if relres else None, _stream()))
        return rr.value if relres else None


def smooth_z_streamed(I0, beta=(1.0, 1.0, 4.0), out_dtype=None, slab=32, levels=0, device_budget=0, out=None,
                      opts=None, check=True, **kw):
    """Anisotropic diffusion (Eq. (1)) of a stack in HOST memory (CPU
    tensors, pinned ones copy fastest), streamed through HBM in z-slabs.
    Returns (I1 on the host, report)."""
    lib = load()
    torch = _torch()
    nz, ny, nx = I0.shape
    if out is None:
        out = torch.empty(I0.shape, dtype=out_dtype or I0.dtype, pin_memory=I0.is_pinned())
    if tuple(out.shape) != tuple(I0.shape):
        raise ValueError("out must have I0's shape")
    o = opts or default_opts(**kw)
    rep = Report()
    st = lib.gd_smooth_z_streamed(_host_ptr(I0), gd_dtype(I0.dtype), _host_ptr(out), gd_dtype(out.dtype), nx, ny, nz,
                                  float(beta[0]), float(beta[1]), float(beta[2]), ctypes.byref(o), int(slab),
                                  int(levels), int(device_budget), ctypes.byref(rep), _stream())
    if check:
        _check(st)
    return out, dict(rep.as_dict(), status=st)


def screened_poisson_streamed(I0, I1, alpha=0.01, beta_xy=(1.0, 1.0), out_dtype=None, slab=16, device_budget=0,
                              out=None, opts=None, check=True, **kw):
    """Eq. (2) for every slice of a [nz][ny][nx] stack in HOST memory, in
    batches of `slab` slices through HBM.  Returns (I2 on the host, report,
    per-slice reports)."""
    lib = load()
    torch = _torch()
    nz, ny, nx = I0.shape
    if tuple(I1.shape) != tuple(I0.shape):
        raise ValueError("I0 and I1 must share the shape")
    if out is None:
        out = torch.empty(I0.shape, dtype=out_dtype or I0.dtype, pin_memory=I0.is_pinned())
    o = opts or default_opts(**kw)
    rep = Report()
    per = (Report * nz)()
    st = lib.gd_screened_poisson_streamed(_host_ptr(I0), gd_dtype(I0.dtype), _host_ptr(I1), gd_dtype(I1.dtype),
                                          _host_ptr(out), gd_dtype(out.dtype), nx, ny, nz, float(alpha),
                                          float(beta_xy[0]), float(beta_xy[1]), ctypes.byref(o), int(slab),
                                          int(device_budget), ctypes.byref(rep), per, _stream())
    if check:
        _check(st)
    return out, dict(rep.as_dict(), status=st), [p.as_dict() for p in per]


class Net:
    """The learned preconditioner (BF16 U-Net run by the library's kernels)."""

    def __init__(self, seed=0, weights=None):
        """He-normal weights from `seed`, or a copy of `weights` (FP32 master
        weights in the layout of :meth:`get_params`)."""
        lib = load()
        self._n = ctypes.c_void_p()
        if weights is None:
            _check(lib.gd_net_create(ctypes.byref(self._n), None, 0, int(seed)), net=True)
        else:
            w = np.ascontiguousarray(weights, dtype=np.float32).ravel()
            _check(lib.gd_net_create(ctypes.byref(self._n), w.ctypes.data_as(ctypes.c_void_p), w.size, int(seed)),
                   net=True)

    @property
    def num_params(self):
        return int(_lib.gd_net_num_params(self._n))

    def get_params(self):
        out = np.empty(self.num_params, dtype=np.float32)
        _check(_lib.gd_net_get_params(self._n, out.ctypes.data_as(ctypes.c_void_p), out.size), net=True)
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.gd_net_set_params(self._n, p.ctypes.data_as(ctypes.c_void_p), p.size), net=True)

    def forward(self, r):
        """r: [batch][ny][nx] FP32 on the GPU -> z of the same shape."""
        _need(r, r.shape, _torch().float32, "r")
        if r.dim() != 3:
            raise ValueError("r must be [batch][ny][nx]")
        b, ny, nx = r.shape
        z = _torch().empty_like(r)
        _check(_lib.gd_net_forward(self._n, _ptr(r), _ptr(z), nx, ny, b, _stream()), net=True)
        return z

    def gradients(self, r, e):
        if r.dim() != 3:
            raise ValueError("r must be [batch][ny][nx]")
        _need(r, r.shape, _torch().float32, "r")
        _need(e, r.shape, _torch().float32, "e")
        b, ny, nx = r.shape
        g = np.empty(self.num_params, dtype=np.float32)
        loss = ctypes.c_double()
        _check(_lib.gd_net_gradients(self._n, _ptr(r), _ptr(e), nx, ny, b, g.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(loss), _stream()), net=True)
        return g, loss.value

    def train_step(self, r, e, lr=1e-3):
        if r.dim() != 3:
            raise ValueError("r must be [batch][ny][nx]")
        _need(r, r.shape, _torch().float32, "r")
        _need(e, r.shape, _torch().float32, "e")
        b, ny, nx = r.shape
        loss = ctypes.c_double()
        _check(_lib.gd_net_train_step(self._n, _ptr(r), _ptr(e), nx, ny, b, float(lr), ctypes.byref(loss),
                                      _stream()), net=True)
        return loss.value

    def set_timing(self, on=True):
        _check(_lib.gd_net_set_timing(self._n, int(bool(on))), net=True)

    def kernel_time(self, layer):
        """(total ms, launches, algorithmic FLOPs) of one layer's forward convolutions."""
        ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(_lib.gd_net_kernel_time(self._n, int(layer), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)),
               net=True)
        return ms.value, n.value, fl.value

    def close(self):
        if self._n:
            _lib.gd_net_destroy(self._n)
            self._n = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rb_sweep(x, b, alpha, w):
    """One red-black Gauss-Seidel sweep (returns the new x)."""
    lib = load()
    nz, ny, nx = x.shape
    out = _torch().empty_like(x)
    _check(lib.gd_rb_sweep(_ptr(x), _ptr(out), _ptr(b), gd_dtype(x.dtype), nx, ny, nz, float(alpha),
                           float(w[0]), float(w[1]), float(w[2]), _stream()))
    return out


def residual_restrict(x, b, alpha, w, c):
    """Residual restricted by summing children; returns (b_coarse, sum r^2)."""
    lib = load()
    nz, ny, nx = x.shape
    cs = (-(-nz // c[2]), -(-ny // c[1]), -(-nx // c[0]))
    bc = _torch().empty(cs, dtype=x.dtype, device=x.device)
    n2 = ctypes.c_double()
    _check(lib.gd_residual_restrict(_ptr(x), _ptr(b), _ptr(bc), gd_dtype(x.dtype), nx, ny, nz, int(c[0]),
                                    int(c[1]), int(c[2]), float(alpha), float(w[0]), float(w[1]), float(w[2]),
                                    ctypes.byref(n2), _stream()))
    return bc, n2.value


def prolong_add(e_coarse, x, c, mode=0):
    """x += P e_coarse in place (mode 0 trilinear, 1 constant); returns x."""
    lib = load()
    nz, ny, nx = x.shape
    _check(lib.gd_prolong_add(_ptr(e_coarse), _ptr(x), gd_dtype(x.dtype), nx, ny, nz, int(c[0]), int(c[1]),
                              int(c[2]), int(mode), _stream()))
    return x


SWEEP_STACK, SWEEP_STACK_PROLONG, SWEEP_SLICE, SWEEP_SLICE_PROLONG, SWEEP_STACK_ZERO, SWEEP_SLICE_ZERO = 0, 1, 2, 3, 4, 5


def kernel_time(variant=SWEEP_STACK):
    """(total ms, launches, algorithmic bytes per launch) of the finest-level
    relaxation launches of one variant recorded with opts.timing = 1."""
    lib = load()
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    by = ctypes.c_double()
    _check(lib.gd_get_kernel_time(int(variant), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
    return ms.value, n.value, by.value


def reset_kernel_time():
    load().gd_reset_kernel_time()


def sweep_config(shape, dtype):
    """Relaxation launch of the finest level of a (nz, ny, nx) grid: dict of
    tile, blocks target, tuned flag and measured ms per sweep."""
    nz, ny, nx = shape
    tx, ty, tuned = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    blocks, ms = ctypes.c_int64(), ctypes.c_double()
    _check(load().gd_sweep_config(nx, ny, nz, gd_dtype(dtype), ctypes.byref(tx), ctypes.byref(ty),
                                  ctypes.byref(blocks), ctypes.byref(tuned), ctypes.byref(ms)))
    return {"tile": (tx.value, ty.value), "blocks_target": blocks.value, "tuned": bool(tuned.value),
            "ms": ms.value}


def release_workspace():
    _check(load().gd_release_workspace())
