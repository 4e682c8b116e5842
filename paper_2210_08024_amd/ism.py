"""Python binding of libism (include/ism.h): argument marshalling only.

Every computation runs in the HIP library; torch provides device memory and the
stream.  The binding raises if the built library is missing -- there is no CPU
fallback.  Function names follow the C entry points without the ``ism_`` prefix.
"""
import ctypes
import os
from dataclasses import dataclass, fields

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libism.so")
COEFF_PATH = os.path.join(ROOT, "data", "ism_coefficients.json")

F64, MIXED = 0, 1

ST_SUBSTEP_CAP, ST_NONFINITE, ST_T_FLOOR, ST_DENOM_GUARD, ST_FALLBACK, ST_TD_UNBRACKETED = 1, 2, 4, 8, 16, 32


class IsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ism error {code}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("dx_cm", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("Zg", "Zd", "chi0", "xi_cr0", "dvdr_kms_pc", "eps_sub", "fd_rel",
                                                "T_floor", "T_bb", "tau_opt_ratio")] + \
               [(k, ctypes.c_int32) for k in ("cr_mode", "kgr_const", "h2_rovib", "max_substeps", "order_cells",
                                               "pad_")]


@dataclass
class Params:
    """Mirror of ism_params (defaults of ism_params_default)."""
    Zg: float = 1.0
    Zd: float = 1.0
    chi0: float = 1.0
    xi_cr0: float = 2.0e-16
    dvdr_kms_pc: float = 1.0
    eps_sub: float = 0.1
    fd_rel: float = 1.0e-3
    T_floor: float = 1.0
    T_bb: float = 6.0
    tau_opt_ratio: float = 1.87
    cr_mode: int = 0
    kgr_const: int = 0
    h2_rovib: int = 1
    max_substeps: int = 100000
    order_cells: int = 1

    def _c(self):
        return _Params(**{f.name: getattr(self, f.name) for f in fields(self)}, pad_=0)


_lib = None
_inited = set()

_vp, _dp, _i64, _i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int32


def lib():
    """Load libism.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_08024_amd.build` "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.ism_init.argtypes = [ctypes.c_int, ctypes.c_char_p]
        L.ism_last_error.restype = ctypes.c_char_p
        L.ism_ndiag.restype = _i32
        L.ism_diag_name.argtypes = [_i32]
        L.ism_diag_name.restype = ctypes.c_char_p
        L.ism_params_default.argtypes = [ctypes.POINTER(_Params)]
        L.ism_columns6.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), ctypes.c_int] + [_vp] * 10
        L.ism_rates.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _i64] + [_vp] * 13
        L.ism_chem_cool_step.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _i64, _dp] + [_vp] * 17
        L.ism_chem_cool_step_noalloc.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _i64, _dp] + [_vp] * 17
        L.ism_surrogate_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_uint64]
        L.ism_surrogate_destroy.argtypes = [_vp]
        L.ism_surrogate_set_norm.argtypes = [_vp] * 5
        L.ism_surrogate_forward.argtypes = [_vp, _vp, _vp, _i64, _vp]
        L.ism_surrogate_backward.argtypes = [_vp, _vp, _vp, _vp, _i64, _vp]
        L.ism_surrogate_train_step.argtypes = [_vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp]
        L.ism_surrogate_get_params.argtypes = [_vp, _vp, _vp]
        L.ism_surrogate_set_params.argtypes = [_vp, _vp, _vp]
        L.ism_stream_release.argtypes = [_vp]
        L.ism_columns_beam.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), ctypes.c_int] + [_vp] * 10
        L.ism_columns_beam.restype = ctypes.c_int
        L.ism_local_shielding.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _i64] + [_vp] * 11
        L.ism_local_shielding.restype = ctypes.c_int
        L.ism_point_sources.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), ctypes.c_int, _i32,
                                        ctypes.c_void_p] + [_vp] * 8 + [_vp]
        L.ism_point_sources.restype = ctypes.c_int
        L.ism_ray_trace.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), ctypes.c_int, _i32,
                                    ctypes.c_void_p, ctypes.c_void_p] + [_vp] * 11 + [_vp]
        L.ism_ray_trace.restype = ctypes.c_int
        L.ism_radiation_force.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _i64] + [_vp] * 8 + \
            [_dp, _vp, _vp, _vp]
        L.ism_radiation_force.restype = ctypes.c_int
        L.ism_surrogate_pairs.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, _i64, _dp] + [_vp] * 14
        L.ism_chem_cool_step_surrogate.argtypes = [_vp, ctypes.POINTER(_Params), _i64, _dp] + [_vp] * 16 + \
            [_dp, _vp, _vp]
        for name in ("ism_init", "ism_shutdown", "ism_stream_release", "ism_columns6", "ism_rates",
                     "ism_chem_cool_step", "ism_chem_cool_step_noalloc") + SURROGATE_SYMBOLS:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


SURROGATE_SYMBOLS = ("ism_surrogate_create", "ism_surrogate_destroy", "ism_surrogate_set_norm",
                     "ism_surrogate_forward", "ism_surrogate_backward", "ism_surrogate_train_step",
                     "ism_surrogate_get_params", "ism_surrogate_set_params", "ism_surrogate_pairs",
                     "ism_chem_cool_step_surrogate")


def exported_symbols():
    return ["ism_params_default", "ism_init", "ism_shutdown", "ism_stream_release", "ism_last_error", "ism_ndiag",
            "ism_diag_name",
            "ism_columns6", "ism_rates", "ism_chem_cool_step", "ism_chem_cool_step_noalloc", "ism_point_sources",
            "ism_ray_trace", "ism_radiation_force", "ism_local_shielding", "ism_columns_beam"] + \
        list(SURROGATE_SYMBOLS)


def _check(rc):
    if rc != 0:
        raise IsmError(rc, lib().ism_last_error().decode())


def init(device=None, path=COEFF_PATH):
    """ism_init on `device` (default: torch's current device)."""
    dev = torch.cuda.current_device() if device is None else int(device)
    _check(lib().ism_init(dev, path.encode()))
    _inited.add(dev)


def stream_release(stream=None):
    """ism_stream_release: return the library scratch held for `stream` (default: torch's current)."""
    _check(lib().ism_stream_release(_stream(stream)))


def _ensure_init(t):
    dev = t.device.index if t.device.index is not None else torch.cuda.current_device()
    if dev not in _inited:
        init(dev)


def _ptr(t, dtype, n=None, name="array", allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr()


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _rdt(prec):
    return torch.float64 if prec == F64 else torch.float32


def columns_beam(n, xH2, xC, dx_cm, params, prec=F64, out=None, stream=None):
    """ism_columns_beam on an [nz, ny, nx] grid: a beam entering through x = 0 along +x."""
    _ensure_init(n)
    nz, ny, nx = n.shape
    N = n.numel()
    rd = _rdt(prec)
    if out is None:
        out = {k: torch.empty_like(n, dtype=rd) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
    g = _Grid(nx, ny, nz, 0, float(dx_cm))
    p = params._c()
    _check(lib().ism_columns_beam(ctypes.byref(g), ctypes.byref(p), prec, _ptr(n, torch.float64, N, "n"),
                                  _ptr(xH2, torch.float64, N, "xH2"),
                                  _ptr(xC, torch.float64, N, "xC", allow_none=True),
                                  *[_ptr(out[k], rd, N, k) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff")],
                                  _ptr(out.get("xi"), rd, N, "xi", allow_none=True), _stream(stream)))
    return out


def local_shielding(n, xH2, xC, L_cm, params, prec=F64, out=None, stream=None):
    """ism_local_shielding: radiation of cells shielded by their own column n L (Sec. 7.1.2)."""
    _ensure_init(n)
    N = n.numel()
    rd = _rdt(prec)
    if out is None:
        out = {k: torch.empty(N, dtype=rd, device=n.device) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C",
                                                                      "N_eff", "xi")}
    p = params._c()
    _check(lib().ism_local_shielding(
        ctypes.byref(p), prec, N, _ptr(n, torch.float64, N, "n"), _ptr(xH2, torch.float64, N, "xH2"),
        _ptr(xC, torch.float64, N, "xC", allow_none=True), _ptr(L_cm, torch.float64, N, "L_cm"),
        *[_ptr(out[k], rd, N, k) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff")],
        _ptr(out.get("xi"), rd, N, "xi", allow_none=True), _stream(stream)))
    return out


class _Source(ctypes.Structure):
    _fields_ = [("x_cm", ctypes.c_double), ("y_cm", ctypes.c_double), ("z_cm", ctypes.c_double),
                ("Q", ctypes.c_double), ("L_FUV", ctypes.c_double)]


def point_sources(n, xH2, xC, dx_cm, params, prec, sources, out, stream=None):
    """ism_point_sources: add the sources' radiation to out's chi_PE, chi_LW, chi_H2, chi_C and phi.

    n, xH2 (and xC or None): float64 device tensors shaped [nz, ny, nx]; sources: rows of
    (x_cm, y_cm, z_cm, Q, L_FUV); out: dict of device tensors of the path's dtype."""
    _ensure_init(n)
    nz, ny, nx = n.shape
    N = n.numel()
    rd = _rdt(prec)
    src = [tuple(float(v) for v in row) for row in sources]
    arr = (_Source * max(len(src), 1))(*[_Source(*r) for r in src])
    g = _Grid(nx, ny, nz, 0, float(dx_cm))
    p = params._c()
    _check(lib().ism_point_sources(
        ctypes.byref(g), ctypes.byref(p), prec, len(src), ctypes.cast(arr, ctypes.c_void_p),
        _ptr(n, torch.float64, N, "n"), _ptr(xH2, torch.float64, N, "xH2"),
        _ptr(xC, torch.float64, N, "xC", allow_none=True),
        *[_ptr(out[k], rd, N, k) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")], _stream(stream)))
    return out


class _ForceOptions(ctypes.Structure):
    _fields_ = [("T_destroy_K", ctypes.c_double), ("prad_ratio_max", ctypes.c_double)]


class _ArtOptions(ctypes.Structure):
    _fields_ = [("level0", ctypes.c_int32), ("max_level", ctypes.c_int32), ("rays_per_cell", ctypes.c_double),
                ("tau_max", ctypes.c_double)]


def ray_trace(n, xH2, xHp, xC, dx_cm, params, prec, sources, out, level0=4, max_level=13, rays_per_cell=4.0,
              tau_max=30.0, budget=False, stream=None):
    """ism_ray_trace: add the sources' radiation, by adaptive ray tracing, to out's chi_PE,
    chi_LW, chi_H2, chi_C and phi (and to out["flux"], [9, nz, ny, nx] of the path's dtype,
    when out holds one).

    n, xH2, xHp (and xC or None): float64 device tensors shaped [nz, ny, nx]; sources: rows of
    (x_cm, y_cm, z_cm, Q, L_FUV); out: dict of device tensors of the path's dtype.  With
    budget=True, out["budget"] receives the [nsrc, 6] escaped / dropped luminosities."""
    _ensure_init(n)
    nz, ny, nx = n.shape
    N = n.numel()
    rd = _rdt(prec)
    src = [tuple(float(v) for v in row) for row in sources]
    arr = (_Source * max(len(src), 1))(*[_Source(*r) for r in src])
    opt = _ArtOptions(int(level0), int(max_level), float(rays_per_cell), float(tau_max))
    g = _Grid(nx, ny, nz, 0, float(dx_cm))
    p = params._c()
    bud = None
    if budget:
        bud = torch.zeros((max(len(src), 1), 6), dtype=torch.float64, device=n.device)
        out["budget"] = bud
    _check(lib().ism_ray_trace(
        ctypes.byref(g), ctypes.byref(p), prec, len(src), ctypes.cast(arr, ctypes.c_void_p),
        ctypes.cast(ctypes.pointer(opt), ctypes.c_void_p),
        _ptr(n, torch.float64, N, "n"), _ptr(xH2, torch.float64, N, "xH2"), _ptr(xHp, torch.float64, N, "xHp"),
        _ptr(xC, torch.float64, N, "xC", allow_none=True),
        *[_ptr(out[k], rd, N, k) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")],
        _ptr(out.get("flux"), rd, 9 * N, "flux", allow_none=True),
        None if bud is None else ctypes.c_void_p(bud.data_ptr()), _stream(stream)))
    return out


def radiation_force(n, T, xH2, xHp, flux, params, prec, f_rad=None, dust_off=None, dt_s=0.0, mom=None, etot=None,
                    T_destroy=1.0e6, prad_ratio_max=50.0, stream=None):
    """ism_radiation_force: the force per volume of the traced radiation on the gas-dust mixture,
    with the grain-destruction switch, and optionally the momentum / energy source update.

    n, T, xH2, xHp: float64 device tensors of N cells; flux: [9, ...] of the path's dtype as
    ray_trace writes it.  Returns f_rad ([3, ...] of the path's dtype; allocated when None);
    dust_off (uint8, N) and mom ([3, ...] float64) / etot (float64) are updated in place."""
    _ensure_init(n)
    N = n.numel()
    rd = _rdt(prec)
    if f_rad is None:
        f_rad = torch.empty((3,) + tuple(n.shape), dtype=rd, device=n.device)
    opt = _ForceOptions(float(T_destroy), float(prad_ratio_max))
    p = params._c()
    _check(lib().ism_radiation_force(
        ctypes.byref(p), prec, N, _ptr(n, torch.float64, N, "n"), _ptr(T, torch.float64, N, "T"),
        _ptr(xH2, torch.float64, N, "xH2"), _ptr(xHp, torch.float64, N, "xHp"), _ptr(flux, rd, 9 * N, "flux"),
        ctypes.cast(ctypes.pointer(opt), ctypes.c_void_p), _ptr(f_rad, rd, 3 * N, "f_rad"),
        _ptr(dust_off, torch.uint8, N, "dust_off", allow_none=True), float(dt_s),
        _ptr(mom, torch.float64, 3 * N, "mom", allow_none=True), _ptr(etot, torch.float64, N, "etot", allow_none=True),
        _stream(stream)))
    return f_rad


def ndiag():
    return lib().ism_ndiag()


def diag_names():
    return [lib().ism_diag_name(k).decode() for k in range(ndiag())]


def columns6(n, xH2, xC, dx_cm, params, prec=F64, out=None, stream=None):
    """Six-ray columns on an [nz, ny, nx] grid.  Returns dict chi_PE, chi_LW, chi_H2, chi_C, N_eff, xi."""
    _ensure_init(n)
    nz, ny, nx = n.shape
    N = n.numel()
    rd = _rdt(prec)
    if out is None:
        out = {k: torch.empty_like(n, dtype=rd) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
    g = _Grid(nx, ny, nz, 0, float(dx_cm))
    p = params._c()
    _check(lib().ism_columns6(ctypes.byref(g), ctypes.byref(p), prec, _ptr(n, torch.float64, N, "n"),
                              _ptr(xH2, torch.float64, N, "xH2"),
                              _ptr(xC, torch.float64, N, "xC", allow_none=True),
                              *[_ptr(out[k], rd, N, k) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff")],
                              _ptr(out["xi"], rd, N, "xi", allow_none=True), _stream(stream)))
    return out


RAD_KEYS = ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi", "xi", "N_eff")


def rates(n, T, xH2, xHp, rad, params, prec=F64, out=None, stream=None):
    """Per-cell diagnostics [ndiag, ncell] (see diag_names())."""
    _ensure_init(n)
    N = n.numel()
    rd = _rdt(prec)
    if out is None:
        out = torch.empty((ndiag(), N), dtype=rd, device=n.device)
    p = params._c()
    _check(lib().ism_rates(ctypes.byref(p), prec, N, _ptr(n, torch.float64, N, "n"), _ptr(T, torch.float64, N, "T"),
                           _ptr(xH2, torch.float64, N, "xH2"), _ptr(xHp, torch.float64, N, "xHp"),
                           _ptr(rad["chi_PE"], rd, N, "chi_PE"), _ptr(rad["chi_LW"], rd, N, "chi_LW"),
                           _ptr(rad["chi_H2"], rd, N, "chi_H2"), _ptr(rad["chi_C"], rd, N, "chi_C"),
                           _ptr(rad.get("phi"), rd, N, "phi", allow_none=True), _ptr(rad["xi"], rd, N, "xi"),
                           _ptr(rad["N_eff"], rd, N, "N_eff"), _ptr(out, rd, None, "out"), _stream(stream)))
    return out


def chem_cool_step(n, T, xH2, xHp, rad, dt_s, params, prec=F64, want=("xCp", "xCO", "xe", "nsub", "status"),
                   out=None, stream=None):
    """In-place step of T, xH2, xHp (float64 device tensors).  Returns dict of the requested extra outputs.
    With params.order_cells == 2 the entry values of out["nsub"] are the ordering key; a binding-allocated
    nsub then starts at zero."""
    return _step("ism_chem_cool_step", n, T, xH2, xHp, rad, dt_s, params, prec, want, out, stream)


def chem_cool_step_noalloc(n, T, xH2, xHp, rad, dt_s, params, prec=F64, out=None, stream=None):
    """ism_chem_cool_step_noalloc: as chem_cool_step, the library allocating nothing (pass `out` to
    allocate nothing here either)."""
    return _step("ism_chem_cool_step_noalloc", n, T, xH2, xHp, rad, dt_s, params, prec,
                 ("xCp", "xCO", "xe", "nsub", "status"), out, stream)


def _step(symbol, n, T, xH2, xHp, rad, dt_s, params, prec, want, out, stream):
    _ensure_init(n)
    N = n.numel()
    rd = _rdt(prec)
    if out is None:
        out = {}
        for k in want:
            dt = torch.int32 if k == "nsub" else (torch.uint8 if k == "status" else rd)
            alloc = torch.zeros if (k == "nsub" and params.order_cells == 2) else torch.empty
            out[k] = alloc(N, dtype=dt, device=n.device)
    p = params._c()
    g = out.get
    _check(getattr(lib(), symbol)(
        ctypes.byref(p), prec, N, float(dt_s), _ptr(n, torch.float64, N, "n"), _ptr(T, torch.float64, N, "T"),
        _ptr(xH2, torch.float64, N, "xH2"), _ptr(xHp, torch.float64, N, "xHp"),
        _ptr(rad["chi_PE"], rd, N, "chi_PE"), _ptr(rad["chi_LW"], rd, N, "chi_LW"),
        _ptr(rad["chi_H2"], rd, N, "chi_H2"), _ptr(rad["chi_C"], rd, N, "chi_C"),
        _ptr(rad.get("phi"), rd, N, "phi", allow_none=True), _ptr(rad["xi"], rd, N, "xi"),
        _ptr(rad["N_eff"], rd, N, "N_eff"),
        _ptr(g("xCp"), rd, N, "xCp", True), _ptr(g("xCO"), rd, N, "xCO", True), _ptr(g("xe"), rd, N, "xe", True),
        _ptr(g("nsub"), torch.int32, N, "nsub", True), _ptr(g("status"), torch.uint8, N, "status", True),
        _stream(stream)))
    return out


# ---------------------------------------------------------------- learned surrogate
SURR_NIN, SURR_NOUT, SURR_NPARAM = 10, 3, 34819
SURR_STATE_FLOATS = 3 * SURR_NPARAM + 1 + 26


class Surrogate:
    """Handle of an ism_surrogate (10 -> 128 -> 128 -> 128 -> 3 SiLU MLP on the matrix cores)."""

    def __init__(self, seed=0, device=None):
        dev = torch.cuda.current_device() if device is None else int(device)
        if dev not in _inited:
            init(dev)
        self.device = dev
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(lib().ism_surrogate_create(ctypes.byref(h), ctypes.c_uint64(seed)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ism_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_norm(self, mu_x, sd_x, mu_y, sd_y):
        arrs = [(ctypes.c_float * k)(*[float(v) for v in a]) for a, k in
                ((mu_x, 10), (sd_x, 10), (mu_y, 3), (sd_y, 3))]
        _check(lib().ism_surrogate_set_norm(self._h, *[ctypes.cast(a, _vp) for a in arrs]))

    def forward(self, X, Y=None, stream=None):
        B = X.shape[0]
        if Y is None:
            Y = torch.empty((B, 3), dtype=torch.float32, device=X.device)
        _check(lib().ism_surrogate_forward(self._h, _ptr(X, torch.float32, B * 10, "X"),
                                           _ptr(Y, torch.float32, B * 3, "Y"), B, _stream(stream)))
        return Y

    def backward(self, X, dY, grad=None, stream=None):
        B = X.shape[0]
        if grad is None:
            grad = torch.empty(SURR_NPARAM, dtype=torch.float32, device=X.device)
        _check(lib().ism_surrogate_backward(self._h, _ptr(X, torch.float32, B * 10, "X"),
                                            _ptr(dY, torch.float32, B * 3, "dY"),
                                            _ptr(grad, torch.float32, SURR_NPARAM, "grad"), B, _stream(stream)))
        return grad

    def train_step(self, X, Y, lr, loss=None, stream=None):
        B = X.shape[0]
        _check(lib().ism_surrogate_train_step(self._h, _ptr(X, torch.float32, B * 10, "X"),
                                              _ptr(Y, torch.float32, B * 3, "Y"), B, ctypes.c_float(lr),
                                              _ptr(loss, torch.float32, 1, "loss", allow_none=True),
                                              _stream(stream)))
        return loss

    def get_params(self, stream=None):
        import numpy as np
        out = np.empty(SURR_STATE_FLOATS, dtype=np.float32)
        _check(lib().ism_surrogate_get_params(self._h, out.ctypes.data, _stream(stream)))
        return out

    def set_params(self, flat, stream=None):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.size != SURR_STATE_FLOATS:
            raise ValueError(f"state has {a.size} floats, expected {SURR_STATE_FLOATS}")
        _check(lib().ism_surrogate_set_params(self._h, a.ctypes.data, _stream(stream)))

    @staticmethod
    def state(theta, m=None, v=None, step=0, mu_x=None, sd_x=None, mu_y=None, sd_y=None):
        """Assemble a checkpoint vector (layout of ism_surrogate_get/set_params)."""
        import numpy as np
        z = np.zeros(SURR_NPARAM)
        parts = [theta, z if m is None else m, z if v is None else v, [step],
                 np.zeros(10) if mu_x is None else mu_x, np.ones(10) if sd_x is None else sd_x,
                 np.zeros(3) if mu_y is None else mu_y, np.ones(3) if sd_y is None else sd_y]
        return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts]).astype(np.float32)


def surrogate_pairs(n, T0, xH2_0, xHp_0, rad, dt_s, params, prec=MIXED, post=None, X=None, Y=None, stream=None):
    """Network inputs X [N][10] (and, given post = dict(T, xH2, xHp) after the step, targets Y [N][3])."""
    _ensure_init(n)
    N = n.numel()
    rd = _rdt(prec)
    if X is None:
        X = torch.empty((N, 10), dtype=torch.float32, device=n.device)
    if post is not None and Y is None:
        Y = torch.empty((N, 3), dtype=torch.float32, device=n.device)
    p = params._c()
    post = post or {}
    _check(lib().ism_surrogate_pairs(
        ctypes.byref(p), prec, N, float(dt_s), _ptr(n, torch.float64, N, "n"), _ptr(T0, torch.float64, N, "T0"),
        _ptr(xH2_0, torch.float64, N, "xH2_0"), _ptr(xHp_0, torch.float64, N, "xHp_0"),
        _ptr(rad["chi_PE"], rd, N, "chi_PE"), _ptr(rad.get("phi"), rd, N, "phi", allow_none=True),
        _ptr(rad["xi"], rd, N, "xi"), _ptr(rad["N_eff"], rd, N, "N_eff"),
        _ptr(post.get("T"), torch.float64, N, "T1", True), _ptr(post.get("xH2"), torch.float64, N, "xH2_1", True),
        _ptr(post.get("xHp"), torch.float64, N, "xHp_1", True), _ptr(X, torch.float32, N * 10, "X"),
        _ptr(Y, torch.float32, N * 3, "Y", True), _stream(stream)))
    return X, Y


def chem_cool_step_surrogate(surrogate, n, T, xH2, xHp, rad, dt_s, params, accept_tol=1e-6,
                             want=("xCp", "xCO", "xe", "nsub", "status"), out=None, n_fallback=None, stream=None):
    """ism_chem_cool_step_surrogate (MIXED): in-place T, xH2, xHp; surrogate None = identity seed."""
    _ensure_init(n)
    N = n.numel()
    rd = torch.float32
    if out is None:
        out = {}
        for k in want:
            dt = torch.int32 if k == "nsub" else (torch.uint8 if k == "status" else rd)
            out[k] = torch.empty(N, dtype=dt, device=n.device)
    p = params._c()
    g = out.get
    h = surrogate._h if surrogate is not None else None
    _check(lib().ism_chem_cool_step_surrogate(
        h, ctypes.byref(p), N, float(dt_s), _ptr(n, torch.float64, N, "n"), _ptr(T, torch.float64, N, "T"),
        _ptr(xH2, torch.float64, N, "xH2"), _ptr(xHp, torch.float64, N, "xHp"),
        _ptr(rad["chi_PE"], rd, N, "chi_PE"), _ptr(rad["chi_LW"], rd, N, "chi_LW"),
        _ptr(rad["chi_H2"], rd, N, "chi_H2"), _ptr(rad["chi_C"], rd, N, "chi_C"),
        _ptr(rad.get("phi"), rd, N, "phi", allow_none=True), _ptr(rad["xi"], rd, N, "xi"),
        _ptr(rad["N_eff"], rd, N, "N_eff"),
        _ptr(g("xCp"), rd, N, "xCp", True), _ptr(g("xCO"), rd, N, "xCO", True), _ptr(g("xe"), rd, N, "xe", True),
        _ptr(g("nsub"), torch.int32, N, "nsub", True), _ptr(g("status"), torch.uint8, N, "status", True),
        float(accept_tol), _ptr(n_fallback, torch.int64, 1, "n_fallback", True), _stream(stream)))
    return out
