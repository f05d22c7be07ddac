"""Thin ctypes binding of libmlcc.so (the C-ABI declared in include/mlcc.h).

Argument marshalling only: torch supplies device memory and the HIP stream,
every computation runs in the library's HIP kernels.  If the library is not
built this module raises on import; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlcc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_02121_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

MLCC_OK = 0
MLCC_ERR_INVALID = -1
MLCC_ERR_HIP = -2
MLCC_ERR_NOMEM = -3
MLCC_ERR_NOT_CONVERGED = -4
MLCC_ERR_STATE = -5
MLCC_ERR_MATCH = -7
MLCC_FP64 = 0
MLCC_MIXED = 1
MLCC_FP64_R32 = 2
MLCC_NOALLOC_MAX_PIXELS = 2048 * 2048
PRECISIONS = {"fp64": MLCC_FP64, "mixed": MLCC_MIXED, "fp64_r32": MLCC_FP64_R32}

EXPORTED = [
    "mlcc_create", "mlcc_destroy", "mlcc_set_stream", "mlcc_last_error", "mlcc_set_lenses",
    "mlcc_set_lenses_batched", "mlcc_cc_params_default", "mlcc_find_critical_curves",
    "mlcc_find_critical_curves_batched", "mlcc_map_caustics",
    "mlcc_caustic_crossings", "mlcc_caustic_distances",
    "mlcc_set_lenses_rect", "mlcc_rect_taylor_degree", "mlcc_num_roots",
    "mlcc_caustic_distances_directional", "mlcc_distance_histogram",
    "mlcc_caustic_crossings_noalloc",
]


class CCParams(ctypes.Structure):
    _fields_ = [("m_steps", ctypes.c_int64), ("n_subchains", ctypes.c_int32),
                ("max_iter_cold", ctypes.c_int32), ("max_iter_warm", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tol_step", ctypes.c_double),
                ("tol_inv_mu", ctypes.c_double), ("timing", ctypes.c_int32),
                ("predictor", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("watchdog_ms", ctypes.c_int32), ("star_sums", ctypes.c_int32),
                ("fmm_order", ctypes.c_int32), ("cold_restart_sweeps", ctypes.c_int32)]


class CCStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("root_updates", ctypes.c_int64),
                ("root_updates_f32", ctypes.c_int64), ("polish_updates", ctypes.c_int64),
                ("unconverged", ctypes.c_int64), ("rows_capped", ctypes.c_int64),
                ("rows_fallback", ctypes.c_int64),
                ("n_subchains", ctypes.c_int32), ("max_row_sweeps", ctypes.c_int32),
                ("cold_sweeps", ctypes.c_int32), ("polls", ctypes.c_int32),
                ("match_maxdist", ctypes.c_double), ("sweep_ms", ctypes.c_double),
                ("sweep_f32_ms", ctypes.c_double), ("polish_ms", ctypes.c_double),
                ("sweep_launches", ctypes.c_int64), ("sweep_f32_launches", ctypes.c_int64),
                ("polish_launches", ctypes.c_int64),
                ("algorithmic_flop", ctypes.c_double), ("algorithmic_flop_f32", ctypes.c_double),
                ("algorithmic_flop_polish", ctypes.c_double),
                ("persistent_ms", ctypes.c_double), ("persistent_launches", ctypes.c_int64),
                ("algorithmic_flop_sweep_roots", ctypes.c_double),
                ("fmm_near_terms", ctypes.c_int64), ("fmm_far_evals", ctypes.c_int64),
                ("cold_restarts", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class GridC(ctypes.Structure):
    _fields_ = [("center_re", ctypes.c_double), ("center_im", ctypes.c_double),
                ("half_width", ctypes.c_double), ("half_height", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_d = ctypes.c_double
_SIG = {
    "mlcc_create": ([ctypes.POINTER(_vp), ctypes.c_int, _vp], ctypes.c_int),
    "mlcc_destroy": ([_vp], None),
    "mlcc_set_stream": ([_vp, _vp], ctypes.c_int),
    "mlcc_last_error": ([], ctypes.c_char_p),
    "mlcc_set_lenses": ([_vp, _i64, _vp, _vp, _vp, _d, _d], ctypes.c_int),
    "mlcc_set_lenses_batched": ([_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "mlcc_cc_params_default": ([ctypes.POINTER(CCParams), _i64], None),
    "mlcc_find_critical_curves": ([_vp, ctypes.POINTER(CCParams), _vp, _vp, _vp, _vp, _vp,
                                   ctypes.POINTER(CCStats)], ctypes.c_int),
    "mlcc_find_critical_curves_batched": ([_vp, ctypes.POINTER(CCParams), _vp, _vp, _vp, _vp,
                                           _vp, _vp, ctypes.POINTER(CCStats)], ctypes.c_int),
    "mlcc_map_caustics": ([_vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
    "mlcc_caustic_crossings": ([_vp, _i64, _i64, _vp, _vp, _vp, ctypes.POINTER(GridC), _vp],
                               ctypes.c_int),
    "mlcc_caustic_crossings_noalloc": ([_vp, _i64, _i64, _vp, _vp, _vp, ctypes.POINTER(GridC),
                                        _vp], ctypes.c_int),
    "mlcc_caustic_distances": ([_vp, ctypes.POINTER(GridC), _vp, _vp, _vp], ctypes.c_int),
    "mlcc_set_lenses_rect": ([_vp, _i64, _vp, _vp, _vp, _d, _d, _d, _d, _d, ctypes.c_int32],
                             ctypes.c_int),
    "mlcc_rect_taylor_degree": ([_d, _d, _d, _d, _d, ctypes.POINTER(ctypes.c_int32)],
                                ctypes.c_int),
    "mlcc_num_roots": ([_vp, ctypes.POINTER(_i64)], ctypes.c_int),
    "mlcc_caustic_distances_directional": ([_vp, ctypes.POINTER(GridC), _vp, _d, _vp, _vp],
                                           ctypes.c_int),
    "mlcc_distance_histogram": ([_vp, _i64, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, _d, _vp], ctypes.c_int),
}
for _name, (_args, _res) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class MlccError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"mlcc error {code}: {message}")
        self.code = code


def _check(code: int):
    if code != MLCC_OK:
        raise MlccError(code, _lib.mlcc_last_error().decode())


def rect_taylor_degree(kappa_star: float, c1: float, c2: float, s: float, eps: float) -> int:
    """App. B truncation degree of a rectangular field's sheet for accuracy
    eps where |z| s < |c| (odd, and clear of the Arg(c) degeneracy)."""
    t = ctypes.c_int32(0)
    _check(_lib.mlcc_rect_taylor_degree(float(kappa_star), float(c1), float(c2), float(s),
                                        float(eps), ctypes.byref(t)))
    return int(t.value)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, device, what: str):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous {dtype} tensor on {device}")


@dataclass
class Grid:
    center_re: float
    center_im: float
    half_width: float
    half_height: float
    nx: int
    ny: int

    def c(self) -> GridC:
        return GridC(float(self.center_re), float(self.center_im), float(self.half_width),
                     float(self.half_height), int(self.nx), int(self.ny))


def as_grid(g) -> Grid:
    return Grid(g.center_re, g.center_im, g.half_width, g.half_height, g.nx, g.ny)


class Context:
    """One library context on one GPU.  Every call enqueues on torch's
    current stream of that device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = _vp()
        _check(_lib.mlcc_create(ctypes.byref(h), int(device),
                                _vp(torch.cuda.current_stream(self.device).cuda_stream)))
        self._h = h
        self.n = 0
        self.star_offsets = None   # set by set_lenses_batched

    def close(self):
        if getattr(self, "_h", None):
            _lib.mlcc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        _check(_lib.mlcc_set_stream(self._h, _vp(torch.cuda.current_stream(self.device).cuda_stream)))

    def set_lenses(self, x: torch.Tensor, y: torch.Tensor, m: torch.Tensor, kappa_s: float,
                   gamma: float):
        for t, w in ((x, "x"), (y, "y"), (m, "m")):
            _need(t, torch.float64, self.device, w)
        self._stream()
        _check(_lib.mlcc_set_lenses(self._h, x.numel(), _ptr(x), _ptr(y), _ptr(m),
                                    float(kappa_s), float(gamma)))
        self.n = x.numel()
        self.star_offsets = None

    def set_lenses_rect(self, x: torch.Tensor, y: torch.Tensor, m: torch.Tensor, kappa_s: float,
                        gamma: float, kappa_star: float, c1: float, c2: float, t: int):
        """A rectangular field (corner c1 + i c2, sheet of convergence
        -kappa_star Taylor-expanded to odd degree t): 2N + t - 1 roots per
        phase (num_roots())."""
        for a, w in ((x, "x"), (y, "y"), (m, "m")):
            _need(a, torch.float64, self.device, w)
        self._stream()
        _check(_lib.mlcc_set_lenses_rect(self._h, x.numel(), _ptr(x), _ptr(y), _ptr(m),
                                         float(kappa_s), float(gamma), float(kappa_star),
                                         float(c1), float(c2), int(t)))
        self.n = x.numel()
        self.star_offsets = None

    def num_roots(self) -> int:
        """Roots per phase of the current lenses."""
        n_r = _i64(0)
        _check(_lib.mlcc_num_roots(self._h, ctypes.byref(n_r)))
        return int(n_r.value)

    def set_lenses_batched(self, star_offsets, x: torch.Tensor, y: torch.Tensor, m: torch.Tensor,
                           kappa_s, gamma):
        """Several fields: field r holds stars star_offsets[r]:star_offsets[r+1]
        of x, y, m; kappa_s and gamma are per field."""
        for t, w in ((x, "x"), (y, "y"), (m, "m")):
            _need(t, torch.float64, self.device, w)
        off = (ctypes.c_int64 * len(star_offsets))(*[int(v) for v in star_offsets])
        nf = len(star_offsets) - 1
        if len(kappa_s) != nf or len(gamma) != nf:
            raise ValueError("kappa_s and gamma need one value per field")
        if int(star_offsets[-1]) != x.numel():
            raise ValueError("star_offsets[-1] must equal the number of stars")
        ks = (ctypes.c_double * nf)(*[float(v) for v in kappa_s])
        gs = (ctypes.c_double * nf)(*[float(v) for v in gamma])
        self._stream()
        _check(_lib.mlcc_set_lenses_batched(self._h, nf, off, _ptr(x), _ptr(y), _ptr(m), ks, gs))
        self.n = x.numel()
        self.star_offsets = [int(v) for v in star_offsets]

    def field_blocks(self, m_steps: int):
        """[(roots offset, chain_next offset, n_r)] of every field in the
        flat output arrays of a batched find_critical_curves call."""
        off = self.star_offsets or [0, self.n]
        return [((m_steps + 1) * 2 * a, 2 * a, 2 * (b - a)) for a, b in zip(off[:-1], off[1:])]

    @staticmethod
    def default_params(m_steps: int) -> CCParams:
        p = CCParams()
        _lib.mlcc_cc_params_default(ctypes.byref(p), int(m_steps))
        return p

    def find_critical_curves(self, m_steps: int, n_subchains: int = 0, tol_step: float = 1e-9,
                             tol_inv_mu: float = 1e-9, max_iter_cold: int = 500,
                             max_iter_warm: int = 100, timing: bool = False,
                             chain_next: bool = True, caustics: bool = False, out=None,
                             caustics_out=None, raise_on_error: bool = True,
                             precision: str = "fp64", predictor: int = 2,
                             schedule: str = "persistent", watchdog_ms: int = 0,
                             star_sums: str = "direct", fmm_order: int = 0,
                             cold_restart_sweeps: int = 0):
        """Returns (roots_re, roots_im, chain_next, stats, status), or with
        caustics=True (roots_re, roots_im, caus_re, caus_im, chain_next, stats,
        status).  One field: arrays are (m_steps + 1, n_r) float64 device
        tensors (n_r = 2N, or 2N + t - 1 for a rectangular field).  Several fields: flat tensors of (m_steps + 1) * 2 * (total
        stars) elements; field_blocks() gives each field's offsets."""
        p = self.default_params(m_steps)
        p.n_subchains = int(n_subchains)
        p.tol_step = float(tol_step)
        p.tol_inv_mu = float(tol_inv_mu)
        p.max_iter_cold = int(max_iter_cold)
        p.max_iter_warm = int(max_iter_warm)
        p.timing = int(bool(timing))
        p.precision = PRECISIONS[precision]
        p.predictor = int(predictor)
        p.schedule = {"rounds": 0, "persistent": 1}[schedule]
        p.watchdog_ms = int(watchdog_ms)
        p.star_sums = {"direct": 0, "fmm": 1}[star_sums]
        p.fmm_order = int(fmm_order)
        p.cold_restart_sweeps = int(cold_restart_sweeps)
        n_r = self.num_roots()
        shape = (m_steps + 1, n_r) if self.star_offsets is None else ((m_steps + 1) * n_r,)
        if out is None:
            rr = torch.empty(shape, dtype=torch.float64, device=self.device)
            ri = torch.empty_like(rr)
        else:
            rr, ri = out
        cr = ci = None
        if caustics:
            if caustics_out is None:
                cr, ci = torch.empty_like(rr), torch.empty_like(ri)
            else:
                cr, ci = caustics_out
        cn = torch.empty(n_r, dtype=torch.int32, device=self.device) if chain_next else None
        st = CCStats()
        self._stream()
        if self.star_offsets is None:
            code = _lib.mlcc_find_critical_curves(self._h, ctypes.byref(p), _ptr(rr), _ptr(ri),
                                                  _ptr(cr), _ptr(ci), _ptr(cn), ctypes.byref(st))
        else:
            offs = (ctypes.c_int64 * len(self.star_offsets))()
            code = _lib.mlcc_find_critical_curves_batched(self._h, ctypes.byref(p), offs, _ptr(rr),
                                                          _ptr(ri), _ptr(cr), _ptr(ci), _ptr(cn),
                                                          ctypes.byref(st))
            self.root_offsets = list(offs)
        if raise_on_error:
            _check(code)
        if caustics:
            return rr, ri, cr, ci, cn, st.as_dict(), code
        return rr, ri, cn, st.as_dict(), code

    def map_caustics(self, z_re: torch.Tensor, z_im: torch.Tensor, out=None):
        _need(z_re, torch.float64, self.device, "z_re")
        _need(z_im, torch.float64, self.device, "z_im")
        if out is None:
            wr, wi = torch.empty_like(z_re), torch.empty_like(z_im)
        else:
            wr, wi = out
        self._stream()
        _check(_lib.mlcc_map_caustics(self._h, z_re.numel(), _ptr(z_re), _ptr(z_im), _ptr(wr),
                                      _ptr(wi)))
        return wr, wi

    def caustic_crossings(self, w_re: torch.Tensor, w_im: torch.Tensor,
                          chain_next: Optional[torch.Tensor], grid, out=None,
                          noalloc: bool = False):
        """N_cc map; noalloc=True calls mlcc_caustic_crossings_noalloc (fixed
        device scratch, at most MLCC_NOALLOC_MAX_PIXELS pixels; `out` should
        then be given, or torch allocates it here)."""
        _need(w_re, torch.float64, self.device, "w_re")
        _need(w_im, torch.float64, self.device, "w_im")
        if w_re.dim() != 2 or w_re.shape != w_im.shape:
            raise ValueError("w_re, w_im must be (rows, n_r)")
        if chain_next is not None:
            _need(chain_next, torch.int32, self.device, "chain_next")
        g = as_grid(grid)
        ncc = out if out is not None else torch.empty((g.ny, g.nx), dtype=torch.int32,
                                                      device=self.device)
        self._stream()
        gc = g.c()
        fn = _lib.mlcc_caustic_crossings_noalloc if noalloc else _lib.mlcc_caustic_crossings
        _check(fn(self._h, w_re.shape[0], w_re.shape[1], _ptr(w_re), _ptr(w_im),
                  _ptr(chain_next), ctypes.byref(gc), _ptr(ncc)))
        return ncc

    def caustic_distances(self, grid, ncc: torch.Tensor, border_limited: bool = True, out=None):
        _need(ncc, torch.int32, self.device, "ncc")
        g = as_grid(grid)
        if out is None:
            dist = torch.empty((g.ny, g.nx), dtype=torch.float64, device=self.device)
            bl = torch.empty((g.ny, g.nx), dtype=torch.uint8, device=self.device) if border_limited else None
        else:
            dist, bl = out
        self._stream()
        gc = g.c()
        _check(_lib.mlcc_caustic_distances(self._h, ctypes.byref(gc), _ptr(ncc), _ptr(dist),
                                           _ptr(bl)))
        return dist, bl

    def caustic_distances_directional(self, grid, ncc: torch.Tensor, angle: float,
                                      border_limited: bool = True, out=None):
        """Moving source: distance along direction `angle` (radians from +y1)
        to the first caustic pixel entered; (dist, border_limited)."""
        _need(ncc, torch.int32, self.device, "ncc")
        g = as_grid(grid)
        if out is None:
            dist = torch.empty((g.ny, g.nx), dtype=torch.float64, device=self.device)
            bl = torch.empty((g.ny, g.nx), dtype=torch.uint8, device=self.device) if border_limited else None
        else:
            dist, bl = out
        self._stream()
        gc = g.c()
        _check(_lib.mlcc_caustic_distances_directional(self._h, ctypes.byref(gc), _ptr(ncc),
                                                       float(angle), _ptr(dist), _ptr(bl)))
        return dist, bl

    def distance_histogram(self, dist: torch.Tensor, border_limited: torch.Tensor, n_bins: int,
                           d_max: float, ncc: Optional[torch.Tensor] = None, ncc_lo: int = 0,
                           n_classes: int = 1, out=None):
        """int64 (n_classes, n_bins + 1) counts of non-border-limited pixels by
        distance bin (last column: d >= d_max), per N_cc class with ncc."""
        _need(dist, torch.float64, self.device, "dist")
        _need(border_limited, torch.uint8, self.device, "border_limited")
        if ncc is not None:
            _need(ncc, torch.int32, self.device, "ncc")
        counts = out if out is not None else torch.empty((n_classes, n_bins + 1),
                                                         dtype=torch.int64, device=self.device)
        self._stream()
        _check(_lib.mlcc_distance_histogram(self._h, dist.numel(), _ptr(dist), _ptr(border_limited),
                                            _ptr(ncc), int(ncc_lo), int(n_classes), int(n_bins),
                                            float(d_max), _ptr(counts)))
        return counts


def last_error() -> str:
    return _lib.mlcc_last_error().decode()


def library():
    return _lib
