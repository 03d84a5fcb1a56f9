"""Thin ctypes binding of libhdsw (include/hdsw.h), same names as the C-ABI.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch is used for device memory and streams: arrays passed
to the device entry points are torch tensors on the GPU (complex128,
contiguous), and the context is bound to a torch stream.

If the shared library has not been built, importing this module raises;
there is no fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdsw.so")

HDSW_OK, HDSW_EINVAL, HDSW_ENOMEM, HDSW_EDEVICE, HDSW_ENOTFACTORED, \
    HDSW_ENOCONV, HDSW_EBUSY = range(7)
HDSW_FP64, HDSW_MIXED = 0, 1
KT_SOLVE, KT_GEMM, KT_FACTOR, KT_RESID, KT_SOLVE_SRC = range(5)

EXPORTED = [
    "hdsw_default_options", "hdsw_setup", "hdsw_factor", "hdsw_solve",
    "hdsw_apply_precond", "hdsw_apply_precond_noalloc", "hdsw_residual", "hdsw_query", "hdsw_timing_enable",
    "hdsw_timing_get", "hdsw_destroy", "hdsw_status_str", "hdsw_batch_reserve",
    "hdsw_batch_add", "hdsw_batch_step", "hdsw_batch_wait", "hdsw_batch_ready", "hdsw_batch_take",
    "hdsw_tuning_set", "hdsw_tuning_get",
]


class hdsw_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double)]


class hdsw_partition(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int * 3)]


DEV_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEV_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class hdsw_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("rounds", ctypes.c_int),
                ("pml_R", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("gmres_m", ctypes.c_int),
                ("dedup", ctypes.c_int), ("graphs", ctypes.c_int),
                ("hbm_budget", ctypes.c_size_t),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class hdsw_tuning(ctypes.Structure):
    _fields_ = [("solve_ng", ctypes.c_int), ("sweep_rw", ctypes.c_int),
                ("sweep_kb", ctypes.c_int), ("gemm_skinny", ctypes.c_int),
                ("sweep_nw", ctypes.c_int), ("sweep_sched", ctypes.c_int)]


class hdsw_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class HdswError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"libhdsw.so not built ({path}); run __graft_entry__.build() first")
    # The library has to bind to the HIP runtime that the caller's device
    # pointers and streams come from.  torch ships its own libamdhip64: when
    # torch is installed it is imported first, so the library resolves to
    # that runtime instead of loading a second one from the system (with two
    # runtimes in the process, torch's streams are invalid handles here).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    c_void_p, c_int = ctypes.c_void_p, ctypes.c_int
    lib.hdsw_default_options.argtypes = [ctypes.POINTER(hdsw_options)]
    lib.hdsw_default_options.restype = None
    lib.hdsw_setup.argtypes = [ctypes.POINTER(hdsw_grid), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(hdsw_partition), c_int,
                               ctypes.POINTER(hdsw_options), c_void_p,
                               ctypes.POINTER(c_void_p)]
    lib.hdsw_setup.restype = c_int
    lib.hdsw_factor.argtypes = [c_void_p]
    lib.hdsw_factor.restype = c_int
    lib.hdsw_solve.argtypes = [c_void_p, c_void_p, c_void_p, c_int,
                               ctypes.POINTER(hdsw_solve_info)]
    lib.hdsw_solve.restype = c_int
    lib.hdsw_apply_precond.argtypes = [c_void_p, c_void_p, c_void_p, c_int]
    lib.hdsw_apply_precond.restype = c_int
    lib.hdsw_apply_precond_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int]
    lib.hdsw_apply_precond_noalloc.restype = c_int
    lib.hdsw_residual.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    lib.hdsw_residual.restype = c_int
    lib.hdsw_query.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_size_t),
                               ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_size_t)]
    lib.hdsw_query.restype = c_int
    lib.hdsw_timing_enable.argtypes = [c_void_p, c_int]
    lib.hdsw_timing_enable.restype = c_int
    lib.hdsw_timing_get.argtypes = [c_void_p, c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.hdsw_timing_get.restype = c_int
    lib.hdsw_batch_reserve.argtypes = [c_void_p, c_int]
    lib.hdsw_batch_reserve.restype = c_int
    lib.hdsw_batch_add.argtypes = [c_void_p, c_void_p, c_int, ctypes.POINTER(c_int)]
    lib.hdsw_batch_add.restype = c_int
    lib.hdsw_batch_step.argtypes = [c_void_p]
    lib.hdsw_batch_step.restype = c_int
    lib.hdsw_batch_wait.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.hdsw_batch_wait.restype = c_int
    lib.hdsw_batch_ready.argtypes = [c_void_p]
    lib.hdsw_batch_ready.restype = c_int
    lib.hdsw_batch_take.argtypes = [c_void_p, c_int, c_void_p]
    lib.hdsw_batch_take.restype = c_int
    lib.hdsw_tuning_set.argtypes = [c_void_p, ctypes.POINTER(hdsw_tuning)]
    lib.hdsw_tuning_set.restype = c_int
    lib.hdsw_tuning_get.argtypes = [c_void_p, ctypes.POINTER(hdsw_tuning)]
    lib.hdsw_tuning_get.restype = c_int
    lib.hdsw_destroy.argtypes = [c_void_p]
    lib.hdsw_destroy.restype = None
    lib.hdsw_status_str.argtypes = [c_int]
    lib.hdsw_status_str.restype = ctypes.c_char_p
    return lib


_lib = load_library()


def hdsw_status_str(status):
    return _lib.hdsw_status_str(int(status)).decode()


def _check(status, what):
    if status != HDSW_OK:
        raise HdswError(status, f"{what}: {hdsw_status_str(status)}")


def hdsw_default_options(**kw):
    o = hdsw_options()
    _lib.hdsw_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# Per context: interior and global node counts, the reserved batch capacity
# and the allocator hooks that must outlive it (keyed by the handle's value).
_CTX = {}


def _dev_ptr(t, what, need=None):
    """Device address of a contiguous complex128 GPU tensor holding at least
    `need` elements."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128
            and t.is_contiguous()):
        raise TypeError(f"{what} must be a contiguous complex128 tensor on the GPU")
    if need is not None and t.numel() < need:
        raise ValueError(f"{what} holds {t.numel()} elements, the call needs {need}")
    return ctypes.c_void_p(t.data_ptr())


def _sizes(ctx):
    info = _CTX.get(ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx)
    if info is None:
        raise ValueError("unknown or destroyed context")
    return info


def torch_allocator_hooks(device=None):
    """Allocator hooks for hdsw_options that take every device allocation of
    a context from torch's caching allocator (uint8 tensors held until the
    library frees them).  Returns (dev_alloc, dev_free, live): pass the first
    two to hdsw_default_options(dev_alloc=..., dev_free=...); `live` maps
    each pointer the library holds to its tensor."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    live = {}

    def _alloc(nbytes, _ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        except RuntimeError:
            return None
        live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(ptr, _ctx):
        live.pop(int(ptr), None)

    return DEV_ALLOC_FN(_alloc), DEV_FREE_FN(_free), live


def hdsw_setup(kappa, h, nsub, pml_width, options=None, stream=None):
    """kappa: real array [n_z][n_y][n_x] (2D: [n_y][n_x]) on the host.
    Returns an opaque context handle (ctypes.c_void_p)."""
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    g = hdsw_grid()
    g.dim = kappa.ndim
    shp = list(reversed(kappa.shape)) + [1] * (3 - kappa.ndim)
    for a in range(3):
        g.n[a] = int(shp[a])
    g.h = float(h)
    p = hdsw_partition()
    ns = list(nsub) + [1] * (3 - len(nsub))
    for a in range(3):
        p.nsub[a] = int(ns[a])
    opt = options if options is not None else hdsw_default_options()
    if stream is None:
        s = None
    else:
        s = ctypes.c_void_p(int(stream))
    ctx = ctypes.c_void_p()
    st = _lib.hdsw_setup(ctypes.byref(g), kappa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         ctypes.byref(p), int(pml_width), ctypes.byref(opt), s,
                         ctypes.byref(ctx))
    _check(st, "hdsw_setup")
    nint = int(np.prod(kappa.shape))
    nglob = int(np.prod([int(x) + 2 * int(pml_width) for x in kappa.shape]))
    # the hooks' ctypes objects must live as long as the context
    _CTX[ctx.value] = dict(nint=nint, nglob=nglob, cap=0,
                           hooks=(opt.dev_alloc, opt.dev_free))
    return ctx


def hdsw_factor(ctx):
    _check(_lib.hdsw_factor(ctx), "hdsw_factor")


def hdsw_solve(ctx, f, x, nrhs, raise_on_noconv=True):
    """f, x: complex128 GPU tensors [nrhs][interior grid].  Returns a list of
    (iters, rel_residual) per RHS and the status."""
    info = (hdsw_solve_info * int(nrhs))()
    n = _sizes(ctx)["nint"] * int(nrhs)
    st = _lib.hdsw_solve(ctx, _dev_ptr(f, "f", n), _dev_ptr(x, "x", n), int(nrhs), info)
    if st != HDSW_ENOCONV or raise_on_noconv:
        _check(st, "hdsw_solve")
    return [(info[i].iters, info[i].rel_residual) for i in range(nrhs)], st


def hdsw_apply_precond(ctx, r, z, nrhs):
    n = _sizes(ctx)["nglob"] * int(nrhs)
    _check(_lib.hdsw_apply_precond(ctx, _dev_ptr(r, "r", n), _dev_ptr(z, "z", n), int(nrhs)),
           "hdsw_apply_precond")


def hdsw_apply_precond_noalloc(ctx, r, z, nrhs):
    """hdsw_apply_precond without any device allocation (workspaces from the
    library's fixed per-device array; overlapping calls on one device race)."""
    n = _sizes(ctx)["nglob"] * int(nrhs)
    _check(_lib.hdsw_apply_precond_noalloc(ctx, _dev_ptr(r, "r", n), _dev_ptr(z, "z", n),
                                           int(nrhs)), "hdsw_apply_precond_noalloc")


def hdsw_residual(ctx, b, x, r, nrhs):
    norms = (ctypes.c_double * int(nrhs))()
    n = _sizes(ctx)["nglob"] * int(nrhs)
    _check(_lib.hdsw_residual(ctx, _dev_ptr(b, "b", n), _dev_ptr(x, "x", n),
                              _dev_ptr(r, "r", n), int(nrhs), norms), "hdsw_residual")
    return np.array(norms[:])


def hdsw_query(ctx):
    fb, ws = ctypes.c_size_t(), ctypes.c_size_t()
    nops = ctypes.c_int()
    _check(_lib.hdsw_query(ctx, ctypes.byref(fb), ctypes.byref(nops), ctypes.byref(ws)),
           "hdsw_query")
    return fb.value, nops.value, ws.value


def hdsw_timing_enable(ctx, enable=True):
    """enable: True (every kernel class), False (none) or a bit mask of
    classes (bit k = class k of hdsw_timing_get)."""
    mask = (31 if enable else 0) if isinstance(enable, bool) else int(enable)
    _check(_lib.hdsw_timing_enable(ctx, mask), "hdsw_timing_enable")


def hdsw_timing_get(ctx, which):
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_longlong()
    _check(_lib.hdsw_timing_get(ctx, int(which), ctypes.byref(ms), ctypes.byref(n),
                                ctypes.byref(fl), ctypes.byref(by)), "hdsw_timing_get")
    return ms.value, n.value, fl.value, by.value


def hdsw_batch_reserve(ctx, capacity):
    _check(_lib.hdsw_batch_reserve(ctx, int(capacity)), "hdsw_batch_reserve")
    _sizes(ctx)["cap"] = int(capacity)


def hdsw_batch_add(ctx, f, nrhs):
    """f: complex128 GPU tensor [nrhs][interior grid].  Returns the slot ids."""
    slots = (ctypes.c_int * int(nrhs))()
    n = _sizes(ctx)["nint"] * int(nrhs)
    _check(_lib.hdsw_batch_add(ctx, _dev_ptr(f, "f", n), int(nrhs), slots), "hdsw_batch_add")
    return list(slots[:])


def hdsw_batch_step(ctx):
    _check(_lib.hdsw_batch_step(ctx), "hdsw_batch_step")


def hdsw_batch_wait(ctx, capacity):
    """Returns the relative residual of every slot (-1 for free slots)."""
    if int(capacity) < _sizes(ctx)["cap"]:
        raise ValueError(f"capacity {capacity} is below the reserved {_sizes(ctx)['cap']} slots")
    rel = (ctypes.c_double * int(capacity))()
    _check(_lib.hdsw_batch_wait(ctx, rel), "hdsw_batch_wait")
    return np.array(rel[:])


def hdsw_batch_ready(ctx):
    """True if the context's last step has finished."""
    st = _lib.hdsw_batch_ready(ctx)
    if st == HDSW_EBUSY:
        return False
    _check(st, "hdsw_batch_ready")
    return True


def hdsw_batch_take(ctx, slot, x=None):
    """Copies the slot's iterate to x (complex128 GPU tensor, interior grid)
    when given, and frees the slot."""
    xp = _dev_ptr(x, "x", _sizes(ctx)["nint"]) if x is not None else None
    _check(_lib.hdsw_batch_take(ctx, int(slot), xp), "hdsw_batch_take")


TUNING_FIELDS = ("solve_ng", "sweep_rw", "sweep_kb", "gemm_skinny", "sweep_nw",
                 "sweep_sched")


def hdsw_tuning_set(ctx, **fields):
    """Sets the kernels' launch parameters (0 = built-in rule); unknown
    fields raise TypeError, values outside the compiled lists HdswError."""
    t = hdsw_tuning()
    for k, v in fields.items():
        if k not in TUNING_FIELDS:
            raise TypeError(f"unknown tuning field {k}")
        setattr(t, k, int(v))
    _check(_lib.hdsw_tuning_set(ctx, ctypes.byref(t)), "hdsw_tuning_set")


def hdsw_tuning_get(ctx):
    t = hdsw_tuning()
    _check(_lib.hdsw_tuning_get(ctx, ctypes.byref(t)), "hdsw_tuning_get")
    return {k: getattr(t, k) for k in TUNING_FIELDS}


def hdsw_destroy(ctx):
    if ctx:
        _lib.hdsw_destroy(ctx)
        _CTX.pop(ctx.value, None)
