"""ctypes binding of libgcb (include/gcb.h).  Argument marshalling only.

The functions carry the C names.  Arrays are torch tensors on the context's
device (or host numpy arrays where the C call accepts host memory); their
data pointers are handed to the library unchanged.  Every failing call raises
GcbError with the library's message.  If libgcb.so has not been built the
import fails loudly: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:
    # torch ships its own HIP runtime; loading it before libgcb.so makes the
    # library bind to that same runtime (two runtimes in one process do not
    # share devices or memory)
    import torch  # noqa: F401
except ImportError:
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GCB_LIBRARY", os.path.join(_HERE, "libgcb.so"))

GCB_OK, GCB_EINVAL, GCB_ENOFIELDS, GCB_ENOMEM, GCB_EHIP, GCB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GCB_F64, GCB_F32 = 0, 1
GCB_FORM_F64, GCB_FORM_MIXED = 0, 1
GCB_HOST, GCB_DEVICE = 0, 1
GCB_KERNEL_AUTO, GCB_KERNEL_GLOBAL, GCB_KERNEL_TILED = 0, 1, 2
GCB_FRAME_REDUCED, GCB_FRAME_EXACT = 0, 1
GCB_GYRATION_MU, GCB_GYRATION_UPERP, GCB_GYRATION_ZERO, GCB_GYRATION_PHASE = 0, 1, 2, 3
GCB_ARITH_EXACT, GCB_ARITH_FAST = 0, 1
GCB_ST_NONFINITE, GCB_ST_KAPPA, GCB_ST_QUAD, GCB_ST_BZERO, GCB_ST_FPRES, GCB_ST_HALO = 1, 2, 4, 8, 16, 32
GCB_ST_OUT = 64
GCB_ST_MIRROR = 128
GCB_TIMER_PUSH, GCB_TIMER_SORT, GCB_TIMER_BACKWARD, GCB_TIMER_OTHER = 0, 1, 2, 3
GCB_NTIMERS = 4

YEE_STAGGER = ((0.5, 0.0), (0.0, 0.5), (0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5))
YEE3_STAGGER = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5),
                (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


class GcbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gcb error {code}: {msg}")
        self.code = code


class gcb_grid_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double),
                ("dy", C.c_double), ("stagger", (C.c_double * 2) * 6),
                ("dtype", C.c_int32)]


class gcb_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("c", C.c_double), ("qm", C.c_double),
                ("f_rho", C.c_double), ("f_E", C.c_double), ("fp_tol", C.c_double),
                ("curvature", C.c_int32), ("n_iter", C.c_int32), ("form", C.c_int32),
                ("sort_every", C.c_int32), ("kernel", C.c_int32), ("tile", C.c_int32),
                ("replay", C.c_int32), ("frame", C.c_int32), ("gyration", C.c_int32),
                ("mirror", C.c_int32), ("mirror_tol", C.c_double), ("arith", C.c_int32),
                ("keep_order", C.c_int32)]


class gcb_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p),
                ("xp", C.c_void_p), ("yp", C.c_void_p), ("ux", C.c_void_p),
                ("uy", C.c_void_p), ("uz", C.c_void_p), ("qm", C.c_void_p),
                ("id", C.c_void_p), ("status", C.c_void_p)]


class gcb_stats(C.Structure):
    _fields_ = [("gca_steps", C.c_int64), ("boris_steps", C.c_int64),
                ("flagged", C.c_int64), ("halo_misses", C.c_int64),
                ("max_fp_residual", C.c_double), ("status_counts", C.c_int64 * 8)]


class gcb_gr_desc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nth", C.c_int32), ("r_min", C.c_double),
                ("r_max", C.c_double), ("spin", C.c_double), ("dtype", C.c_int32)]


class gcb_gr_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("r", C.c_void_p), ("th", C.c_void_p), ("ph", C.c_void_p),
                ("ur", C.c_void_p), ("uth", C.c_void_p), ("uph", C.c_void_p),
                ("qm", C.c_void_p), ("id", C.c_void_p), ("status", C.c_void_p)]


class gcb_grid3_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dtype", C.c_int32), ("d", C.c_double * 3),
                ("stagger", (C.c_double * 3) * 6)]


class gcb_particles3(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("xp", C.c_void_p), ("yp", C.c_void_p), ("zp", C.c_void_p),
                ("ux", C.c_void_p), ("uy", C.c_void_p), ("uz", C.c_void_p),
                ("qm", C.c_void_p), ("id", C.c_void_p), ("status", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "gcb_create": (C.c_int, [C.POINTER(P), C.c_int]),
        "gcb_destroy": (None, [P]),
        "gcb_last_error": (C.c_char_p, [P]),
        "gcb_load_fields": (C.c_int, [P, C.POINTER(gcb_grid_desc), C.POINTER(P * 3),
                                      C.POINTER(P * 3), C.c_int32, P]),
        "gcb_push": (C.c_int, [P, C.POINTER(gcb_particles), C.POINTER(gcb_params),
                               C.c_int32, P, C.POINTER(gcb_stats), P]),
        "gcb_push_noalloc": (C.c_int, [P, C.POINTER(gcb_particles), C.POINTER(gcb_params),
                                       C.c_int32, P, C.POINTER(gcb_stats), P]),
        "gcb_push_backward": (C.c_int, [P, C.POINTER(gcb_particles), C.POINTER(gcb_params),
                                        C.c_int32, C.POINTER(P * 7), C.POINTER(P * 7),
                                        C.POINTER(P * 3), C.POINTER(P * 3), P]),
        "gcb_kinetic_energy": (C.c_int, [P, C.POINTER(gcb_particles), C.POINTER(gcb_params),
                                         P, C.POINTER(P * 3), P]),
        "gcb_load_fields_gr": (C.c_int, [P, C.POINTER(gcb_gr_desc), C.POINTER(P * 3),
                                         C.POINTER(P * 3), C.c_int32, P]),
        "gcb_push_gr": (C.c_int, [P, C.POINTER(gcb_gr_particles), C.POINTER(gcb_params),
                                  C.c_int32, P, C.POINTER(gcb_stats), P]),
        "gcb_load_fields_3d": (C.c_int, [P, C.POINTER(gcb_grid3_desc), C.POINTER(P * 3),
                                         C.POINTER(P * 3), C.c_int32, P]),
        "gcb_push_3d": (C.c_int, [P, C.POINTER(gcb_particles3), C.POINTER(gcb_params),
                                  C.c_int32, P, C.POINTER(gcb_stats), P]),
        "gcb_push_backward_3d": (C.c_int, [P, C.POINTER(gcb_particles3), C.POINTER(gcb_params),
                                           C.c_int32, C.POINTER(P * 9), C.POINTER(P * 9),
                                           C.POINTER(P * 3), C.POINTER(P * 3), P]),
        "gcb_sincos": (C.c_int, [P, P, P, P, C.c_int64, P]),
        "gcb_set_timing": (C.c_int, [P, C.c_int32]),
        "gcb_get_timing": (C.c_int, [P, C.POINTER(C.c_double * GCB_NTIMERS),
                                     C.POINTER(C.c_int64 * GCB_NTIMERS)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("gcb_create", "gcb_destroy", "gcb_last_error", "gcb_load_fields", "gcb_push",
            "gcb_push_backward", "gcb_kinetic_energy", "gcb_set_timing", "gcb_get_timing",
            "gcb_load_fields_gr", "gcb_push_gr", "gcb_load_fields_3d", "gcb_push_3d",
            "gcb_push_backward_3d", "gcb_push_noalloc", "gcb_sincos")


def lib():
    return _lib


def _ptr(a):
    """Data pointer of a torch tensor / numpy array, or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stats_dict(st) -> dict:
    d = {k: getattr(st, k) for k, _ in gcb_stats._fields_}
    d["status_counts"] = list(d["status_counts"])
    return d


def _check(rc: int, ctx=None):
    if rc != GCB_OK:
        msg = _lib.gcb_last_error(ctx)
        raise GcbError(rc, msg.decode() if msg else "")


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def gcb_create(device: int = 0):
    # let torch set up its HIP context first: the caller's tensors live there
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    h = C.c_void_p()
    _check(_lib.gcb_create(C.byref(h), int(device)))
    return h


def gcb_destroy(ctx) -> None:
    _lib.gcb_destroy(ctx)


def gcb_last_error(ctx=None) -> str:
    m = _lib.gcb_last_error(ctx)
    return m.decode() if m else ""


def grid_desc(nx, ny, dx=1.0, dy=1.0, stagger=YEE_STAGGER, dtype=GCB_F64) -> gcb_grid_desc:
    d = gcb_grid_desc()
    d.nx, d.ny, d.dx, d.dy, d.dtype = int(nx), int(ny), float(dx), float(dy), int(dtype)
    for k in range(6):
        d.stagger[k][0] = float(stagger[k][0])
        d.stagger[k][1] = float(stagger[k][1])
    return d


def gcb_load_fields(ctx, desc: gcb_grid_desc, E, B, src=None, stream=None) -> None:
    """E, B: sequences of three (ny, nx) float64 arrays (numpy host or torch device)."""
    if src is None:
        src = GCB_HOST if isinstance(E[0], np.ndarray) else GCB_DEVICE
    for a in list(E) + list(B):
        if isinstance(a, np.ndarray):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        else:
            import torch
            assert a.dtype == torch.float64 and a.is_contiguous()
    Ea = (C.c_void_p * 3)(*[_ptr(a) for a in E])
    Ba = (C.c_void_p * 3)(*[_ptr(a) for a in B])
    sp = None if src == GCB_HOST and stream is None else _stream_ptr(stream)
    _check(_lib.gcb_load_fields(ctx, C.byref(desc), C.byref(Ea), C.byref(Ba), int(src), sp), ctx)


def params(dt=1.0, c=0.45, qm=-1.0, f_rho=0.4, f_E=1.0, fp_tol=1e-7, curvature=1,
           n_iter=4, form=GCB_FORM_F64, sort_every=0, kernel=GCB_KERNEL_AUTO,
           tile=0, replay=0, frame=GCB_FRAME_REDUCED,
           gyration=GCB_GYRATION_MU, mirror=0, mirror_tol=0.0,
           arith=GCB_ARITH_EXACT, keep_order=0) -> gcb_params:
    p = gcb_params()
    p.dt, p.c, p.qm, p.f_rho, p.f_E, p.fp_tol = dt, c, qm, f_rho, f_E, fp_tol
    p.curvature, p.n_iter, p.form = int(curvature), int(n_iter), int(form)
    p.sort_every, p.kernel, p.tile = int(sort_every), int(kernel), int(tile)
    p.replay, p.frame, p.gyration = int(replay), int(frame), int(gyration)
    p.mirror, p.mirror_tol = int(mirror), float(mirror_tol)
    p.arith, p.keep_order = int(arith), int(keep_order)
    return p


def particles(t: dict) -> gcb_particles:
    """Build the struct from a dict of tensors x, y, xp, yp, ux, uy, uz, status
    and optional qm, id."""
    p = gcb_particles()
    p.n = int(t["x"].shape[0])
    for k in ("x", "y", "xp", "yp", "ux", "uy", "uz", "status"):
        setattr(p, k, _ptr(t[k]))
    p.qm = _ptr(t.get("qm"))
    p.id = _ptr(t.get("id"))
    return p


def gcb_push(ctx, parts: gcb_particles, prm: gcb_params, n_steps: int, s_trace=None,
             want_stats: bool = False, stream=None):
    st = gcb_stats() if want_stats else None
    rc = _lib.gcb_push(ctx, C.byref(parts), C.byref(prm), int(n_steps), _ptr(s_trace),
                       C.byref(st) if st is not None else None, _stream_ptr(stream))
    _check(rc, ctx)
    if st is None:
        return None
    return _stats_dict(st)


def gcb_push_noalloc(ctx, parts: gcb_particles, prm: gcb_params, n_steps: int, s_trace=None,
                     want_stats: bool = False, stream=None):
    """gcb_push with the library's scratch taken from its fixed device array."""
    st = gcb_stats() if want_stats else None
    rc = _lib.gcb_push_noalloc(ctx, C.byref(parts), C.byref(prm), int(n_steps), _ptr(s_trace),
                               C.byref(st) if st is not None else None, _stream_ptr(stream))
    _check(rc, ctx)
    if st is None:
        return None
    return _stats_dict(st)


NOALLOC_SCRATCH_BYTES = 64 << 20


def gcb_push_backward(ctx, start: gcb_particles, prm: gcb_params, n_steps: int, lam_end,
                      lam_start, dE, dB, stream=None) -> None:
    le = (C.c_void_p * 7)(*[_ptr(a) for a in lam_end])
    ls = (C.c_void_p * 7)(*[_ptr(a) for a in lam_start])
    de = (C.c_void_p * 3)(*[_ptr(a) for a in dE])
    db = (C.c_void_p * 3)(*[_ptr(a) for a in dB])
    _check(_lib.gcb_push_backward(ctx, C.byref(start), C.byref(prm), int(n_steps),
                                  C.byref(le), C.byref(ls), C.byref(de), C.byref(db),
                                  _stream_ptr(stream)), ctx)


def gcb_sincos(ctx, x, s, c, stream=None):
    """s = sin x, c = cos x by the library's binary64 sin/cos (device tensors)."""
    _check(_lib.gcb_sincos(ctx, _ptr(x), _ptr(s), _ptr(c), int(x.numel()),
                           _stream_ptr(stream)), ctx)


def gcb_kinetic_energy(ctx, parts: gcb_particles, prm: gcb_params, out, lam_u=None,
                       stream=None) -> None:
    lu = (C.c_void_p * 3)(*[_ptr(a) for a in lam_u]) if lam_u is not None else None
    _check(_lib.gcb_kinetic_energy(ctx, C.byref(parts), C.byref(prm), _ptr(out),
                                   C.byref(lu) if lu is not None else None,
                                   _stream_ptr(stream)), ctx)


def gr_desc(nr, nth, r_min, r_max, spin, dtype=GCB_F64) -> gcb_gr_desc:
    d = gcb_gr_desc()
    d.nr, d.nth, d.r_min, d.r_max, d.spin, d.dtype = (int(nr), int(nth), float(r_min),
                                                      float(r_max), float(spin), int(dtype))
    return d


def gcb_load_fields_gr(ctx, desc: gcb_gr_desc, D, B, src=None, stream=None) -> None:
    # D, B are always binary64; desc.dtype selects the device copy
    """D, B: sequences of three (nth+1, nr+1) float64 arrays (numpy host or torch device)."""
    if src is None:
        src = GCB_HOST if isinstance(D[0], np.ndarray) else GCB_DEVICE
    for a in list(D) + list(B):
        if isinstance(a, np.ndarray):
            assert a.dtype == np.float64 and a.flags.c_contiguous
    Da = (C.c_void_p * 3)(*[_ptr(a) for a in D])
    Ba = (C.c_void_p * 3)(*[_ptr(a) for a in B])
    sp = None if src == GCB_HOST and stream is None else _stream_ptr(stream)
    _check(_lib.gcb_load_fields_gr(ctx, C.byref(desc), C.byref(Da), C.byref(Ba), int(src), sp),
           ctx)


def gr_particles(t: dict) -> gcb_gr_particles:
    """Build the struct from a dict of tensors r, th, ph, ur, uth, uph, status
    and optional qm, id."""
    p = gcb_gr_particles()
    p.n = int(t["r"].shape[0])
    for k in ("r", "th", "ph", "ur", "uth", "uph", "status"):
        setattr(p, k, _ptr(t[k]))
    p.qm = _ptr(t.get("qm"))
    p.id = _ptr(t.get("id"))
    return p


def gcb_push_gr(ctx, parts: gcb_gr_particles, prm: gcb_params, n_steps: int, s_trace=None,
                want_stats: bool = False, stream=None):
    st = gcb_stats() if want_stats else None
    rc = _lib.gcb_push_gr(ctx, C.byref(parts), C.byref(prm), int(n_steps), _ptr(s_trace),
                          C.byref(st) if st is not None else None, _stream_ptr(stream))
    _check(rc, ctx)
    if st is None:
        return None
    return _stats_dict(st)


def grid3_desc(nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, stagger=YEE3_STAGGER,
               dtype=GCB_F64) -> gcb_grid3_desc:
    d = gcb_grid3_desc()
    d.n[0], d.n[1], d.n[2] = int(nx), int(ny), int(nz)
    d.d[0], d.d[1], d.d[2] = float(dx), float(dy), float(dz)
    d.dtype = int(dtype)
    for k in range(6):
        for a in range(3):
            d.stagger[k][a] = float(stagger[k][a])
    return d


def gcb_load_fields_3d(ctx, desc: gcb_grid3_desc, E, B, src=None, stream=None) -> None:
    """E, B: sequences of three (nz, ny, nx) float64 arrays (numpy host or torch device)."""
    if src is None:
        src = GCB_HOST if isinstance(E[0], np.ndarray) else GCB_DEVICE
    for a in list(E) + list(B):
        if isinstance(a, np.ndarray):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        else:
            import torch
            assert a.dtype == torch.float64 and a.is_contiguous()
    Ea = (C.c_void_p * 3)(*[_ptr(a) for a in E])
    Ba = (C.c_void_p * 3)(*[_ptr(a) for a in B])
    sp = None if src == GCB_HOST and stream is None else _stream_ptr(stream)
    _check(_lib.gcb_load_fields_3d(ctx, C.byref(desc), C.byref(Ea), C.byref(Ba), int(src), sp),
           ctx)


def particles3(t: dict) -> gcb_particles3:
    """Build the struct from a dict of tensors x, y, z, xp, yp, zp, ux, uy, uz,
    status and optional qm, id."""
    p = gcb_particles3()
    p.n = int(t["x"].shape[0])
    for k in ("x", "y", "z", "xp", "yp", "zp", "ux", "uy", "uz", "status"):
        setattr(p, k, _ptr(t[k]))
    p.qm = _ptr(t.get("qm"))
    p.id = _ptr(t.get("id"))
    return p


def gcb_push_3d(ctx, parts: gcb_particles3, prm: gcb_params, n_steps: int, s_trace=None,
                want_stats: bool = False, stream=None):
    st = gcb_stats() if want_stats else None
    rc = _lib.gcb_push_3d(ctx, C.byref(parts), C.byref(prm), int(n_steps), _ptr(s_trace),
                          C.byref(st) if st is not None else None, _stream_ptr(stream))
    _check(rc, ctx)
    if st is None:
        return None
    return _stats_dict(st)


def gcb_push_backward_3d(ctx, start: gcb_particles3, prm: gcb_params, n_steps: int, lam_end,
                         lam_start, dE, dB, stream=None) -> None:
    """lam_end, lam_start: nine device arrays (x, y, z, xp, yp, zp, ux, uy, uz);
    dE, dB: three device float arrays of nz*ny*nx elements each (accumulated)."""
    le = (C.c_void_p * 9)(*[_ptr(a) for a in lam_end])
    ls = (C.c_void_p * 9)(*[_ptr(a) for a in lam_start])
    de = (C.c_void_p * 3)(*[_ptr(a) for a in dE])
    db = (C.c_void_p * 3)(*[_ptr(a) for a in dB])
    _check(_lib.gcb_push_backward_3d(ctx, C.byref(start), C.byref(prm), int(n_steps),
                                     C.byref(le), C.byref(ls), C.byref(de), C.byref(db),
                                     _stream_ptr(stream)), ctx)


def gcb_set_timing(ctx, enabled: bool) -> None:
    _check(_lib.gcb_set_timing(ctx, 1 if enabled else 0), ctx)


def gcb_get_timing(ctx):
    ms = (C.c_double * GCB_NTIMERS)()
    cnt = (C.c_int64 * GCB_NTIMERS)()
    _check(_lib.gcb_get_timing(ctx, C.byref(ms), C.byref(cnt)), ctx)
    return list(ms), list(cnt)
