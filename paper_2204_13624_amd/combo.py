"""Thin Python binding of libcombo (include/combo.h): argument marshalling only.

Every function named combo_* mirrors the C entry point of the same name.  Host
arrays are numpy arrays (C-contiguous float64 / uint8 / int32); device arrays
are torch tensors on the context's GPU (PyTorch only provides the memory).
All computation happens in the HIP library; if the library is missing this
module raises instead of computing anything itself.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# COMBO_LIBRARY names another build of the library (e.g. a variant under test); default: the in-tree build
LIB_PATH = os.environ.get("COMBO_LIBRARY") or os.path.join(HERE, "libcombo.so")

COMBO_OK = 0
COMBO_E_INVAL = -1
COMBO_E_NOMEM = -2
COMBO_E_HIP = -3
COMBO_E_SIZE = -4
COMBO_E_NOCONV = -5
COMBO_E_INADMISSIBLE = -6
COMBO_E_NUMERIC = -7
COMBO_E_STATE = -8

COMBO_MEM_HOST = 0
COMBO_MEM_DEVICE = 1
COMBO_FP64 = 0
COMBO_MIXED = 1
COMBO_GREEN_GAMMA0 = 0
COMBO_GREEN_G = 1
COMBO_DISC_MS = 0
COMBO_DISC_WILLOT = 1
COMBO_DISC_STAGGERED = 2
COMBO_NORMALS_LAPLACE = 0
COMBO_NORMALS_BARYCENTRE = 1
COMBO_LAW_NEO_HOOKE = 0
COMBO_LAW_LINEAR = 1


class combo_material(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("lambda_", ctypes.c_double)]


class combo_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("tol_newton", ctypes.c_double),
        ("tol_cg", ctypes.c_double),
        ("max_newton", ctypes.c_int),
        ("max_cg", ctypes.c_int),
        ("max_laminate", ctypes.c_int),
        ("n_increments", ctypes.c_int),
        ("mu0", ctypes.c_double),
        ("kappa0", ctypes.c_double),
        ("warm_start_laminate", ctypes.c_int),
        ("want_tangent", ctypes.c_int),
        ("max_step_halvings", ctypes.c_int),
        ("max_cutbacks", ctypes.c_int),
        ("graph_chunk", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("line_search", ctypes.c_int),
        ("law", ctypes.c_int),
        ("batch_streams", ctypes.c_int),
    ]


class combo_stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("newton_iters", ctypes.c_int),
        ("cg_iters_total", ctypes.c_int),
        ("cg_iters_tangent", ctypes.c_int),
        ("increments_done", ctypes.c_int),
        ("step_halvings", ctypes.c_int),
        ("cutbacks", ctypes.c_int),
        ("laminate_iters_max", ctypes.c_int),
        ("laminate_iters_total", ctypes.c_longlong),
        ("laminate_backprojections", ctypes.c_longlong),
        ("laminate_failures", ctypes.c_longlong),
        ("eta_final", ctypes.c_double),
        ("time_ms_total", ctypes.c_double),
        ("time_ms_cg", ctypes.c_double),
        ("time_ms_material", ctypes.c_double),
        ("time_ms_residual", ctypes.c_double),
        ("time_ms_tangent", ctypes.c_double),
        ("cg_truncations", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "combo_abi_version": (_I, []),
    "combo_strerror": (ctypes.c_char_p, [_I]),
    "combo_default_options": (None, [ctypes.POINTER(combo_options)]),
    "combo_validate_microstructure": (_I, [_I, _I, _I, _P, _P, _P, ctypes.c_char_p, _I]),
    "combo_check_size": (_I, [_I]),
    "combo_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "combo_destroy": (_I, [_P]),
    "combo_last_error": (ctypes.c_char_p, [_P]),
    "combo_set_grid": (_I, [_P, _I, _I, _I, _D, _D, _D]),
    "combo_set_materials": (_I, [_P, ctypes.POINTER(combo_material)]),
    "combo_set_microstructure": (_I, [_P, _P, _P, _P, _I]),
    "combo_set_discretization": (_I, [_P, _I]),
    "combo_batch_set_discretization": (_I, [_P, _I]),
    "combo_get_grid": (_I, [_P] + [ctypes.POINTER(ctypes.c_int)] * 3 + [ctypes.POINTER(ctypes.c_double)] * 3),
    "combo_image_to_boxels": (_I, [_P, _P, _I, _I, _I, _I, _P, _P, _P, _I]),
    "combo_set_microstructure_from_image": (_I, [_P, _P, _I, _I, _I, _I, _I]),
    "combo_image_to_boxels_static": (_I, [_P, _P, _I, _I, _I, _I, _P, _P, _P]),
    "combo_set_options": (_I, [_P, ctypes.POINTER(combo_options)]),
    "combo_solve": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(combo_stats), _I]),
    "combo_eval_law": (_I, [_P, _P, _P, _P, _P, _P, _I]),
    "combo_apply_green": (_I, [_P, _I, _I, _P, _P, _I]),
    "combo_apply_operator": (_I, [_P, _I, _P, _P, _I]),
    "combo_profile_enable": (_I, [_P, _I]),
    "combo_profile_select": (_I, [_P, ctypes.c_uint]),
    "combo_profile_read": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "combo_profile_read_idle": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "combo_autotune": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "combo_set_schedule": (_I, [_P, _I, _I, _I]),
    "combo_get_schedule": (_I, [_P] + [ctypes.POINTER(_I)] * 6),
    "combo_batch_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "combo_batch_destroy": (_I, [_P]),
    "combo_batch_last_error": (ctypes.c_char_p, [_P]),
    "combo_batch_set_options": (_I, [_P, ctypes.POINTER(combo_options)]),
    "combo_batch_add": (_I, [_P, _I, _I, _I, _D, _D, _D, ctypes.POINTER(combo_material), _P, _P, _P, _I,
                             ctypes.POINTER(_I)]),
    "combo_batch_size": (_I, [_P]),
    "combo_batch_solve": (_I, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(combo_stats)]),
    "combo_batch_fields": (_I, [_P, _I, _P, _P, _I]),
}

KERNEL_NAMES = ["xpass_cg", "ypass_inv", "ypass_fwd", "zpass_inv", "zpass_fwd", "cg_update", "cg_finalize",
                "material", "residual", "newton_dir", "boxel_count", "boxel_normals"]

_lib = None


def load_library(path=None):
    """Load libcombo.so (built by paper_2204_13624_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError("libcombo.so not found at %s: build it with `python -m paper_2204_13624_amd.build`" % p)
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class ComboError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (strerror(status), status, msg))
        self.status = status


def strerror(status):
    return load_library().combo_strerror(status).decode()


def _check(ctx, status):
    if status != COMBO_OK:
        msg = load_library().combo_last_error(ctx).decode() if ctx else ""
        raise ComboError(status, msg)


# ---- pointer marshalling -----------------------------------------------------

def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, mem_kind) of a numpy array or torch tensor, or (None, None)."""
    if x is None:
        return None, None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        want = {np.float64: "torch.float64", np.uint8: "torch.uint8", np.int32: "torch.int32"}[dtype]
        if str(x.dtype) != want:
            raise TypeError("expected %s, got %s" % (want, x.dtype))
        if x.is_cuda:
            # the library works on its own stream: what torch has queued on its
            # stream for this tensor (the kernels that produced it) must be done
            import torch
            torch.cuda.current_stream(x.device).synchronize()
        return ctypes.c_void_p(x.data_ptr()), (COMBO_MEM_DEVICE if x.is_cuda else COMBO_MEM_HOST)
    if not isinstance(x, np.ndarray) or x.dtype != dtype or not x.flags.c_contiguous:
        raise TypeError("expected a C-contiguous numpy array of %s" % np.dtype(dtype))
    return ctypes.c_void_p(x.ctypes.data), COMBO_MEM_HOST


def _mem_kind(*kinds):
    ks = {k for k in kinds if k is not None}
    if len(ks) > 1:
        raise ValueError("mixing host and device buffers in one call")
    return ks.pop() if ks else COMBO_MEM_HOST


# ---- same-name wrappers ----------------------------------------------------------

def combo_abi_version():
    return load_library().combo_abi_version()


def combo_strerror(status):
    return strerror(status)


def combo_default_options():
    o = combo_options()
    load_library().combo_default_options(ctypes.byref(o))
    return o


def combo_check_size(n):
    return load_library().combo_check_size(int(n))


def combo_validate_microstructure(phase, c, N):
    """Host-only validation; returns (status, message)."""
    n3, n2, n1 = phase.shape
    ph = np.ascontiguousarray(phase, dtype=np.uint8)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    NN = np.ascontiguousarray(N, dtype=np.float64)
    buf = ctypes.create_string_buffer(256)
    st = load_library().combo_validate_microstructure(n1, n2, n3, ph.ctypes.data, cc.ctypes.data, NN.ctypes.data,
                                                      buf, 256)
    return st, buf.value.decode()


def combo_create(device=0, stream=None):
    ctx = ctypes.c_void_p()
    s = ctypes.c_void_p(stream) if stream else None
    st = load_library().combo_create(ctypes.byref(ctx), int(device), s)
    _check(None, st)
    return ctx


def combo_destroy(ctx):
    return load_library().combo_destroy(ctx)


def combo_last_error(ctx):
    return load_library().combo_last_error(ctx).decode()


def combo_set_grid(ctx, n1, n2, n3, l1=1.0, l2=1.0, l3=1.0):
    _check(ctx, load_library().combo_set_grid(ctx, int(n1), int(n2), int(n3), float(l1), float(l2), float(l3)))


def combo_set_materials(ctx, mats):
    arr = (combo_material * 2)()
    for i in range(2):
        arr[i].mu, arr[i].lambda_ = float(mats[i][0]), float(mats[i][1])
    _check(ctx, load_library().combo_set_materials(ctx, arr))


def combo_set_microstructure(ctx, phase, c, N):
    pp, k1 = _ptr(phase, np.uint8)
    cp, k2 = _ptr(c, np.float64)
    npt, k3 = _ptr(N, np.float64)
    _check(ctx, load_library().combo_set_microstructure(ctx, pp, cp, npt, _mem_kind(k1, k2, k3)))


def combo_image_to_boxels(ctx, chi, s, method=COMBO_NORMALS_LAPLACE, out=None):
    """Fine image chi [n3 s3, n2 s2, n1 s1] (uint8 0/1, numpy or torch) -> (phase, c, N) of the
    context's grid.  out = (phase, c, N) receives them (same memory kind as chi); else new
    numpy arrays (host image) or torch tensors on the image's device."""
    (n1, n2, n3), _ = combo_get_grid(ctx)
    if tuple(chi.shape) != (n3 * s[2], n2 * s[1], n1 * s[0]):
        raise ValueError("image shape %s does not match grid %s x boxel %s" % (tuple(chi.shape), (n1, n2, n3), tuple(s)))
    cp, kind = _ptr(chi, np.uint8)
    if out is None:
        if kind == COMBO_MEM_DEVICE:
            import torch
            dev = chi.device
            out = (torch.empty((n3, n2, n1), dtype=torch.uint8, device=dev),
                   torch.empty((n3, n2, n1), dtype=torch.float64, device=dev),
                   torch.empty((3, n3, n2, n1), dtype=torch.float64, device=dev))
        else:
            out = (np.zeros((n3, n2, n1), np.uint8), np.zeros((n3, n2, n1)), np.zeros((3, n3, n2, n1)))
    pp, k1 = _ptr(out[0], np.uint8)
    cc, k2 = _ptr(out[1], np.float64)
    nn, k3 = _ptr(out[2], np.float64)
    _check(ctx, load_library().combo_image_to_boxels(ctx, cp, int(s[0]), int(s[1]), int(s[2]), int(method),
                                                     pp, cc, nn, _mem_kind(kind, k1, k2, k3)))
    return out


def combo_image_to_boxels_static(ctx, chi, s, out, method=COMBO_NORMALS_LAPLACE):
    """combo_image_to_boxels into out = (phase, c, N), all device tensors, with the
    library's static device scratch (no allocation in the library)."""
    (n1, n2, n3), _ = combo_get_grid(ctx)
    if tuple(chi.shape) != (n3 * s[2], n2 * s[1], n1 * s[0]):
        raise ValueError("image shape %s does not match grid %s x boxel %s" % (tuple(chi.shape), (n1, n2, n3), tuple(s)))
    cp, kind = _ptr(chi, np.uint8)
    pp, k1 = _ptr(out[0], np.uint8)
    cc, k2 = _ptr(out[1], np.float64)
    nn, k3 = _ptr(out[2], np.float64)
    if _mem_kind(kind, k1, k2, k3) != COMBO_MEM_DEVICE:
        raise ValueError("combo_image_to_boxels_static takes device tensors only")
    _check(ctx, load_library().combo_image_to_boxels_static(ctx, cp, int(s[0]), int(s[1]), int(s[2]), int(method),
                                                            pp, cc, nn))
    return out


def combo_set_discretization(ctx, disc):
    _check(ctx, load_library().combo_set_discretization(ctx, int(disc)))


def combo_batch_set_discretization(b, disc):
    st = load_library().combo_batch_set_discretization(b, int(disc))
    if st != COMBO_OK:
        raise ComboError(st, load_library().combo_batch_last_error(b).decode())


def combo_get_grid(ctx):
    """((n1, n2, n3), (l1, l2, l3)) of the context."""
    n = [ctypes.c_int() for _ in range(3)]
    l = [ctypes.c_double() for _ in range(3)]
    _check(ctx, load_library().combo_get_grid(ctx, *[ctypes.byref(x) for x in n + l]))
    return tuple(x.value for x in n), tuple(x.value for x in l)


def combo_set_microstructure_from_image(ctx, chi, s, method=COMBO_NORMALS_LAPLACE):
    (n1, n2, n3), _ = combo_get_grid(ctx)
    if tuple(chi.shape) != (n3 * s[2], n2 * s[1], n1 * s[0]):
        raise ValueError("image shape %s does not match grid %s x boxel %s" % (tuple(chi.shape), (n1, n2, n3), tuple(s)))
    cp, kind = _ptr(chi, np.uint8)
    _check(ctx, load_library().combo_set_microstructure_from_image(ctx, cp, int(s[0]), int(s[1]), int(s[2]),
                                                                   int(method), kind))


def combo_set_options(ctx, opts):
    _check(ctx, load_library().combo_set_options(ctx, ctypes.byref(opts)))


def combo_solve(ctx, Fbar, F_init=None, F_out=None, P_out=None, want_tangent=False, want_phase=True):
    """Returns dict(Pbar 3x3, Abar 9x9 or None, Pbar_phase (2,3,3), stats dict); fields go to F_out/P_out."""
    fb = np.ascontiguousarray(np.asarray(Fbar, dtype=np.float64).reshape(9))
    Pbar = np.zeros(9)
    Abar = np.zeros(81) if want_tangent else None
    Pph = np.zeros(18) if want_phase else None
    st = combo_stats()
    fi, k1 = _ptr(F_init, np.float64)
    fo, k2 = _ptr(F_out, np.float64)
    po, k3 = _ptr(P_out, np.float64)
    status = load_library().combo_solve(
        ctx, fb.ctypes.data, fi, fo, po, Pbar.ctypes.data,
        Abar.ctypes.data if Abar is not None else None,
        Pph.ctypes.data if Pph is not None else None, ctypes.byref(st), _mem_kind(k1, k2, k3))
    out = dict(status=status, stats=st.as_dict(), Pbar=Pbar.reshape(3, 3),
               Abar=Abar.reshape(9, 9) if Abar is not None else None,
               Pbar_phase=Pph.reshape(2, 3, 3) if Pph is not None else None)
    if status != COMBO_OK:
        err = ComboError(status, combo_last_error(ctx))
        err.result = out
        raise err
    return out


def combo_eval_law(ctx, F, P=None, A=None, a=None, iters=None):
    fp, k0 = _ptr(F, np.float64)
    pp, k1 = _ptr(P, np.float64)
    ap, k2 = _ptr(A, np.float64)
    jp, k3 = _ptr(a, np.float64)
    ip, k4 = _ptr(iters, np.int32)
    return load_library().combo_eval_law(ctx, fp, pp, ap, jp, ip, _mem_kind(k0, k1, k2, k3, k4))


def combo_apply_green(ctx, which, precision, tau, out):
    tp, k1 = _ptr(tau, np.float64)
    op, k2 = _ptr(out, np.float64)
    _check(ctx, load_library().combo_apply_green(ctx, int(which), int(precision), tp, op, _mem_kind(k1, k2)))


def combo_apply_operator(ctx, precision, p, q):
    pp, k1 = _ptr(p, np.float64)
    qp, k2 = _ptr(q, np.float64)
    _check(ctx, load_library().combo_apply_operator(ctx, int(precision), pp, qp, _mem_kind(k1, k2)))


def combo_profile_enable(ctx, enable=True):
    _check(ctx, load_library().combo_profile_enable(ctx, 1 if enable else 0))


def combo_profile_select(ctx, kernels=None):
    """Time only these kernel classes while profiling (None: all)."""
    mask = 0xFFFFFFFF if kernels is None else sum(1 << int(k) for k in kernels)
    _check(ctx, load_library().combo_profile_select(ctx, mask))


def combo_profile_read(ctx, kernel):
    """(milliseconds, launches) accumulated for one kernel class."""
    ms = ctypes.c_double()
    nl = ctypes.c_longlong()
    _check(ctx, load_library().combo_profile_read(ctx, int(kernel), ctypes.byref(ms), ctypes.byref(nl)))
    return ms.value, nl.value


def combo_profile_read_idle(ctx, kernel):
    """(milliseconds, launches) of the launches that found the CG finished (left out above)."""
    ms = ctypes.c_double()
    nl = ctypes.c_longlong()
    _check(ctx, load_library().combo_profile_read_idle(ctx, int(kernel), ctypes.byref(ms), ctypes.byref(nl)))
    return ms.value, nl.value


def combo_profile_all(ctx):
    return {name: combo_profile_read(ctx, k) for k, name in enumerate(KERNEL_NAMES)}


def combo_profile_all_idle(ctx):
    return {name: combo_profile_read_idle(ctx, k) for k, name in enumerate(KERNEL_NAMES)}


def combo_autotune(ctx, precision):
    """Tune (or fetch the cached) schedule of the context's grid; returns (xv, yv, zv)."""
    v = [ctypes.c_int() for _ in range(3)]
    _check(ctx, load_library().combo_autotune(ctx, int(precision), *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def combo_set_schedule(ctx, xv, yv, zv):
    _check(ctx, load_library().combo_set_schedule(ctx, int(xv), int(yv), int(zv)))


def combo_get_schedule(ctx):
    """(xv, yv, zv), (number of x, y, z variants)."""
    v = [ctypes.c_int() for _ in range(6)]
    _check(ctx, load_library().combo_get_schedule(ctx, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v[:3]), tuple(x.value for x in v[3:])


# ---- batches ---------------------------------------------------------------------

def _bcheck(b, status):
    if status != COMBO_OK:
        raise ComboError(status, load_library().combo_batch_last_error(b).decode() if b else "")


def _mats_array(mats):
    arr = (combo_material * 2)()
    for i in range(2):
        arr[i].mu, arr[i].lambda_ = float(mats[i][0]), float(mats[i][1])
    return arr


def combo_batch_create(device=0, stream=None):
    b = ctypes.c_void_p()
    s = ctypes.c_void_p(stream) if stream else None
    _bcheck(None, load_library().combo_batch_create(ctypes.byref(b), int(device), s))
    return b


def combo_batch_destroy(b):
    return load_library().combo_batch_destroy(b)


def combo_batch_last_error(b):
    return load_library().combo_batch_last_error(b).decode()


def combo_batch_set_options(b, opts):
    _bcheck(b, load_library().combo_batch_set_options(b, ctypes.byref(opts)))


def combo_batch_add(b, n, l, mats, phase, c, N):
    """Append one RVE (n = (n1, n2, n3), l = (l1, l2, l3)); returns its index."""
    pp, k1 = _ptr(phase, np.uint8)
    cp, k2 = _ptr(c, np.float64)
    npt, k3 = _ptr(N, np.float64)
    idx = ctypes.c_int(-1)
    _bcheck(b, load_library().combo_batch_add(b, int(n[0]), int(n[1]), int(n[2]), float(l[0]), float(l[1]),
                                              float(l[2]), _mats_array(mats), pp, cp, npt, _mem_kind(k1, k2, k3),
                                              ctypes.byref(idx)))
    return idx.value


def combo_batch_size(b):
    return load_library().combo_batch_size(b)


def combo_batch_solve(b, Fbar, n_increments=None, want_tangent=False):
    """Fbar (m, 3, 3); returns dict(status, Pbar (m,3,3), Abar (m,9,9) or None, Pbar_phase (m,2,3,3), stats list)."""
    m = combo_batch_size(b)
    fb = np.ascontiguousarray(np.asarray(Fbar, dtype=np.float64).reshape(m, 9))
    ninc = None
    if n_increments is not None:
        ninc = np.ascontiguousarray(np.asarray(n_increments, dtype=np.int32).reshape(m))
    Pbar = np.zeros((m, 9))
    Abar = np.zeros((m, 81)) if want_tangent else None
    Pph = np.zeros((m, 18))
    stats = (combo_stats * m)()
    status = load_library().combo_batch_solve(
        b, fb.ctypes.data, ninc.ctypes.data if ninc is not None else None, Pbar.ctypes.data,
        Abar.ctypes.data if Abar is not None else None, Pph.ctypes.data, stats)
    out = dict(status=status, stats=[s.as_dict() for s in stats], Pbar=Pbar.reshape(m, 3, 3),
               Abar=Abar.reshape(m, 9, 9) if Abar is not None else None, Pbar_phase=Pph.reshape(m, 2, 3, 3))
    if status != COMBO_OK:
        err = ComboError(status, combo_batch_last_error(b))
        err.result = out
        raise err
    return out


def combo_batch_fields(b, i, F=None, P=None):
    fp, k1 = _ptr(F, np.float64)
    pp, k2 = _ptr(P, np.float64)
    _bcheck(b, load_library().combo_batch_fields(b, int(i), fp, pp, _mem_kind(k1, k2)))


# ---- convenience object ----------------------------------------------------------

class Solver:
    """One context: grid, materials, microstructure and options, then solve()."""

    def __init__(self, device=0, stream=None):
        self.ctx = combo_create(device, stream)
        self.n = None

    def close(self):
        if self.ctx:
            combo_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, ms, mats, **opts):
        """ms: object with n, l, phase, c, N (see synth.Microstructure)."""
        combo_set_grid(self.ctx, *ms.n, *ms.l)
        self.n = tuple(ms.n)
        combo_set_materials(self.ctx, mats)
        combo_set_microstructure(self.ctx, ms.phase, ms.c, ms.N)
        self.set_options(**opts)

    def set_options(self, **kw):
        o = combo_default_options()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        combo_set_options(self.ctx, o)
        self.opts = o

    def solve(self, Fbar, F_init=None, fields=False, want_tangent=False):
        n1, n2, n3 = self.n
        F_out = np.zeros((9, n3, n2, n1)) if fields else None
        P_out = np.zeros((9, n3, n2, n1)) if fields else None
        r = combo_solve(self.ctx, Fbar, F_init=F_init, F_out=F_out, P_out=P_out, want_tangent=want_tangent)
        if fields:
            r["F"] = F_out
            r["P"] = P_out
        return r
