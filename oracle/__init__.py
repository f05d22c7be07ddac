"""CPU oracle for the critical-curve / caustic / crossing-map / distance-map
path of Weisenbach (2025), "A GPU Code for Finding Microlensing Critical
Curves and Caustics".

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library and imports nothing from it; inputs arrive as plain
numpy arrays or duck-typed objects with the attributes
  field: x, y, m (float64 arrays), kappa_s, gamma (floats)
  grid:  center_re, center_im, half_width, half_height, nx, ny.

The arithmetic lives in mlcc_oracle.c (plain C, IEEE double); this module
only marshals arrays.  Each C function's header cites the passage of the
paper it follows.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

OK, ERR_INVALID, ERR_NOT_CONVERGED, ERR_NONFINITE, ERR_MATCH = 0, -1, -4, -6, -7

# Paper Sec. 3.2 (footnote on the cutoffs): |z^{a+1} - z^a| < 1e-9 theta_star
# or |mu| > 1e9.
TOL_STEP = 1e-9
TOL_INV_MU = 1e-9
QBITS = 24

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64
_d = ctypes.c_double


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        sig = {
            "orc_eval_F": [_i64, _D, _D, _D, _d, _d, _D, _d, _i64, _D, _D, _D, _D, _D, _D],
            "orc_lens_map": [_i64, _D, _D, _D, _d, _d, _D, _i64, _D, _D, _D, _D],
            "orc_inv_mu": [_i64, _D, _D, _D, _d, _d, _D, _i64, _D, _D, _D],
            "orc_seeds": [_i64, _D, _D, _D, _D, _D],
            "orc_aberth_row": [_i64, _D, _D, _D, _d, _d, _D, _d, _i64, _D, _D, _d, _d, _i64,
                               ctypes.c_int, _I64, _I64],
            "orc_subchain": [_i64, _D, _D, _D, _d, _d, _D, _i64, _i64, _i64, _i64, _d, _d, _i64,
                             _i64, ctypes.c_int, _D, _D, _I64],
            "orc_rect_dalpha": [_D, _i64, _D, _D, _D, _D],
            "orc_rect_alpha": [_D, ctypes.c_int, _i64, _D, _D, _D, _D],
            "orc_rect_taylor_degree": [_d, _d, _d, _d, _d],
            "orc_match": [_i64, _D, _D, _D, _D, _I32, _D],
            "orc_critical_curves": [_i64, _D, _D, _D, _d, _d, _D, _i64, _i64, _d, _d, _i64,
                                    _i64, ctypes.c_int, _D, _D, _I32, _I64, _D],
            "orc_num_roots": [_i64, _D],
            "orc_directional_distance": [_i64, _i64, _I32, _d, _d, _d, _D, _U8],
            "orc_distance_histogram": [_i64, _D, _U8, _I32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, _d, _I64],
            "orc_ncc_pixels": [_i64, _i64, _D, _D, _I32, _d, _d, _d, _d, _i64, _i64, _I32],
            "orc_ncc_rows": [_i64, _i64, _D, _D, _I32, _d, _d, _d, _d, _i64, _i64, _I32],
            "orc_ncc_at": [_i64, _i64, _D, _D, _I32, _d, _d, _d, _d, _i64, _i64, _i64, _I64,
                           _I64, _I64],
            "orc_caustic_mask": [_i64, _i64, _I32, _U8],
            "orc_edt_brute": [_i64, _i64, _I32, _d, _D, _U8, _I64],
            "orc_edt_twopass": [_i64, _i64, _I32, _d, _D, _U8, _I64],
            "orc_num_threads": [],
            "orc_set_num_threads": [ctypes.c_int],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int64 if name == "orc_num_roots" else ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _sheet(field):
    """(kappa_star, c1, c2, t) of a rectangular field as a float64 array, or
    None for a circular one."""
    sh = getattr(field, "sheet", None)
    return None if sh is None else np.ascontiguousarray(np.asarray(sh, dtype=np.float64))


def _star_args(field):
    x, y, m = _f64(field.x), _f64(field.y), _f64(field.m)
    sh = _sheet(field)
    return (x, y, m, sh), (x.shape[0], _p(x, _D), _p(y, _D), _p(m, _D),
                           float(field.kappa_s), float(field.gamma), _p(sh, _D))


def num_roots(field) -> int:
    """Roots per phase: 2N, plus t - 1 for a rectangular field (App. B)."""
    keep, sa = _star_args(field)
    return int(lib().orc_num_roots(sa[0], sa[6]))


def rect_taylor_degree(kappa_star, c1, c2, s, eps) -> int:
    """App. B truncation degree for accuracy eps where |z| s < |c|."""
    t = int(lib().orc_rect_taylor_degree(float(kappa_star), float(c1), float(c2), float(s),
                                         float(eps)))
    if t < 0:
        raise OracleError(t, "rect_taylor_degree")
    return t


def rect_dalpha_dzbar(sheet, z):
    """d alpha_s / d zbar of the rectangular sheet (App. B closed form)."""
    sh = np.ascontiguousarray(np.asarray(sheet, dtype=np.float64))
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).ravel())
    zr, zi = _f64(z.real), _f64(z.imag)
    dr, di = np.empty(z.shape[0]), np.empty(z.shape[0])
    lib().orc_rect_dalpha(_p(sh, _D), z.shape[0], _p(zr, _D), _p(zi, _D), _p(dr, _D), _p(di, _D))
    return dr + 1j * di


def rect_alpha(sheet, z, exact=False):
    """alpha_s of the rectangular sheet: App. B series truncated at t, or its
    closed form (exact=True)."""
    sh = np.ascontiguousarray(np.asarray(sheet, dtype=np.float64))
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).ravel())
    zr, zi = _f64(z.real), _f64(z.imag)
    ar, ai = np.empty(z.shape[0]), np.empty(z.shape[0])
    lib().orc_rect_alpha(_p(sh, _D), int(bool(exact)), z.shape[0], _p(zr, _D), _p(zi, _D),
                         _p(ar, _D), _p(ai, _D))
    return ar + 1j * ai


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> int:
    """Threads of the oracle's later parallel loops; returns the count in effect."""
    return int(lib().orc_set_num_threads(int(n)))


def phase(j, m_steps):
    """phi_j = 2 pi j / m_steps (Sec. 3.1 / Sec. 4.3), computed as the C side does."""
    return (2.0 * np.pi * np.asarray(j, dtype=np.float64)) / float(m_steps)


def eval_F(field, phi: float, z):
    z = np.ascontiguousarray(z, dtype=np.complex128).ravel()
    keep, sa = _star_args(field)
    zr, zi = _f64(z.real), _f64(z.imag)
    out = [np.empty(z.shape[0]) for _ in range(4)]
    lib().orc_eval_F(*sa, float(phi), z.shape[0], _p(zr, _D), _p(zi, _D),
                     *[_p(o, _D) for o in out])
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def lens_map(field, z):
    z = np.asarray(z, dtype=np.complex128)
    shape = z.shape
    z = z.ravel()
    keep, sa = _star_args(field)
    zr, zi = _f64(z.real), _f64(z.imag)
    wr, wi = np.empty(z.shape[0]), np.empty(z.shape[0])
    lib().orc_lens_map(*sa, z.shape[0], _p(zr, _D), _p(zi, _D), _p(wr, _D), _p(wi, _D))
    return (wr + 1j * wi).reshape(shape)


def inv_mu(field, z):
    z = np.asarray(z, dtype=np.complex128)
    shape = z.shape
    z = z.ravel()
    keep, sa = _star_args(field)
    zr, zi = _f64(z.real), _f64(z.imag)
    out = np.empty(z.shape[0])
    lib().orc_inv_mu(*sa, z.shape[0], _p(zr, _D), _p(zi, _D), _p(out, _D))
    return out.reshape(shape)


def seeds(field):
    keep, sa = _star_args(field)
    n = sa[0]
    n_r = num_roots(field)
    zr, zi = np.empty(n_r), np.empty(n_r)
    lib().orc_seeds(n, sa[1], sa[2], sa[6], _p(zr, _D), _p(zi, _D))
    return zr + 1j * zi


def aberth_row(field, phi: float, z0=None, tol_step=TOL_STEP, tol_mu=TOL_INV_MU,
               max_iter=10000, polish=True, allow_unconverged=False):
    """Roots of F(., phi) by Jacobi Aberth-Ehrlich sweeps from z0 (cold seeds
    when None).  Returns (roots, sweeps, updates, status)."""
    if z0 is None:
        z0 = seeds(field)
    z0 = np.asarray(z0, dtype=np.complex128)
    zr, zi = _f64(z0.real).copy(), _f64(z0.imag).copy()
    keep, sa = _star_args(field)
    sw, up = _i64(0), _i64(0)
    rc = lib().orc_aberth_row(*sa, float(phi), zr.shape[0], _p(zr, _D), _p(zi, _D),
                              float(tol_step), float(tol_mu), int(max_iter), int(polish),
                              ctypes.byref(sw), ctypes.byref(up))
    if rc not in (OK, ERR_NOT_CONVERGED) or (rc == ERR_NOT_CONVERGED and not allow_unconverged):
        raise OracleError(rc, "aberth_row")
    return zr + 1j * zi, sw.value, up.value, rc


def subchain(field, m_steps, lo, center, hi, tol_step=TOL_STEP, tol_mu=TOL_INV_MU,
             max_iter_cold=10000, max_iter_warm=10000, polish=True):
    """Rows lo..hi of the chain matrix grown from a cold start at `center`
    (Sec. 4.3).  Returns (roots (hi-lo+1, 2N) complex, stats dict)."""
    keep, sa = _star_args(field)
    n_r = num_roots(field)
    rows = hi - lo + 1
    rr, ri = np.empty(rows * n_r), np.empty(rows * n_r)
    st = np.zeros(5, dtype=np.int64)
    rc = lib().orc_subchain(*sa, int(m_steps), int(lo), int(center), int(hi), float(tol_step),
                            float(tol_mu), int(max_iter_cold), int(max_iter_warm), int(polish),
                            _p(rr, _D), _p(ri, _D), _p(st, _I64))
    if rc != OK:
        raise OracleError(rc, "subchain")
    return (rr + 1j * ri).reshape(rows, n_r), _stats(st)


def _stats(st):
    return {"sweeps": int(st[0]), "root_updates": int(st[1]), "capped_rows": int(st[2]),
            "max_warm_sweeps": int(st[3]), "cold_sweeps": int(st[4])}


def critical_curves(field, m_steps, n_sub=1, tol_step=TOL_STEP, tol_mu=TOL_INV_MU,
                    max_iter_cold=10000, max_iter_warm=10000, polish=True):
    """The (m_steps+1, 2N) chain matrix of Sec. 4.3 and chain_next.
    Returns (roots complex, chain_next int32, stats dict)."""
    keep, sa = _star_args(field)
    n_r = num_roots(field)
    rows = m_steps + 1
    rr, ri = np.empty(rows * n_r), np.empty(rows * n_r)
    cn = np.empty(n_r, dtype=np.int32)
    st = np.zeros(5, dtype=np.int64)
    md = _d(0.0)
    rc = lib().orc_critical_curves(*sa, int(m_steps), int(n_sub), float(tol_step),
                                   float(tol_mu), int(max_iter_cold), int(max_iter_warm),
                                   int(polish), _p(rr, _D), _p(ri, _D), _p(cn, _I32),
                                   _p(st, _I64), ctypes.byref(md))
    if rc != OK:
        raise OracleError(rc, "critical_curves")
    s = _stats(st)
    s["match_maxdist"] = md.value
    return (rr + 1j * ri).reshape(rows, n_r), cn, s


def match(a, b):
    """Nearest-neighbour bijection a -> b; returns (perm, maxdist)."""
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    ar, ai, br, bi = _f64(a.real), _f64(a.imag), _f64(b.real), _f64(b.imag)
    perm = np.empty(a.shape[0], dtype=np.int32)
    md = _d(0.0)
    rc = lib().orc_match(a.shape[0], _p(ar, _D), _p(ai, _D), _p(br, _D), _p(bi, _D),
                         _p(perm, _I32), ctypes.byref(md))
    if rc != OK:
        raise OracleError(rc, "match")
    return perm, md.value


def _grid_args(grid):
    return (float(grid.center_re), float(grid.center_im), float(grid.half_width),
            float(grid.half_height), int(grid.nx), int(grid.ny))


def _w_args(w, chain_next):
    """w: complex (rows, n_r), or a pair of real (rows, n_r) planes (re, im),
    which large maps pass to avoid a complex copy."""
    if isinstance(w, tuple):
        wr, wi = _f64(w[0]), _f64(w[1])
        if wr.ndim != 2 or wr.shape != wi.shape:
            raise ValueError("w planes must be two (rows, n_r) arrays")
    else:
        w = np.asarray(w, dtype=np.complex128)
        if w.ndim != 2:
            raise ValueError("w must be (rows, n_r)")
        wr, wi = _f64(w.real), _f64(w.imag)
    cn = None if chain_next is None else np.ascontiguousarray(chain_next, dtype=np.int32)
    return (wr, wi, cn), (wr.shape[0], wr.shape[1], _p(wr, _D), _p(wi, _D), _p(cn, _I32))


def ncc_pixels(w, chain_next, grid):
    """N_cc map by the definition (every pixel against every edge)."""
    keep, wa = _w_args(w, chain_next)
    out = np.empty((int(grid.ny), int(grid.nx)), dtype=np.int32)
    rc = lib().orc_ncc_pixels(*wa, *_grid_args(grid), _p(out, _I32))
    if rc != OK:
        raise OracleError(rc, "ncc_pixels")
    return out


def ncc_rows(w, chain_next, grid):
    """N_cc map built edge by edge with a per-row difference array."""
    keep, wa = _w_args(w, chain_next)
    out = np.empty((int(grid.ny), int(grid.nx)), dtype=np.int32)
    rc = lib().orc_ncc_rows(*wa, *_grid_args(grid), _p(out, _I32))
    if rc != OK:
        raise OracleError(rc, "ncc_rows")
    return out


def ncc_at(w, chain_next, grid, pix_r, pix_c):
    """N_cc at selected pixels (definition, edges streamed)."""
    keep, wa = _w_args(w, chain_next)
    pr = np.ascontiguousarray(pix_r, dtype=np.int64)
    pc = np.ascontiguousarray(pix_c, dtype=np.int64)
    out = np.empty(pr.shape[0], dtype=np.int64)
    rc = lib().orc_ncc_at(*wa, *_grid_args(grid), pr.shape[0], _p(pr, _I64), _p(pc, _I64),
                          _p(out, _I64))
    if rc != OK:
        raise OracleError(rc, "ncc_at")
    return out


def caustic_mask(ncc):
    ncc = np.ascontiguousarray(ncc, dtype=np.int32)
    ny, nx = ncc.shape
    out = np.empty((ny, nx), dtype=np.uint8)
    lib().orc_caustic_mask(nx, ny, _p(ncc, _I32), _p(out, _U8))
    return out


def _edt(fn, ncc, h):
    ncc = np.ascontiguousarray(ncc, dtype=np.int32)
    ny, nx = ncc.shape
    dist = np.empty((ny, nx))
    bl = np.empty((ny, nx), dtype=np.uint8)
    d2 = np.empty((ny, nx), dtype=np.int64)
    fn(nx, ny, _p(ncc, _I32), float(h), _p(dist, _D), _p(bl, _U8), _p(d2, _I64))
    return dist, bl, d2


def edt_brute(ncc, h):
    """(distance, border_limited, squared pixel distance) by brute force."""
    return _edt(lib().orc_edt_brute, ncc, h)


def edt_twopass(ncc, h):
    """(distance, border_limited, squared pixel distance), two-pass exact."""
    return _edt(lib().orc_edt_twopass, ncc, h)


def directional_distance(ncc, h, angle):
    """Moving source (Sec. 5.2): distance along the direction `angle` (from
    the +y1 axis) to the first caustic pixel entered, by brute force.
    Returns (dist, border_limited)."""
    ncc = np.ascontiguousarray(ncc, dtype=np.int32)
    ny, nx = ncc.shape
    dist = np.empty((ny, nx))
    bl = np.empty((ny, nx), dtype=np.uint8)
    rc = lib().orc_directional_distance(nx, ny, _p(ncc, _I32), float(h), float(np.cos(angle)),
                                        float(np.sin(angle)), _p(dist, _D), _p(bl, _U8))
    if rc != OK:
        raise OracleError(rc, "directional_distance")
    return dist, bl


def distance_histogram(dist, border_limited, n_bins, d_max, ncc=None, ncc_lo=0, n_classes=1):
    """Counts per distance bin of width d_max / n_bins (last column: d >=
    d_max), per N_cc class when ncc is given; border-limited pixels skipped."""
    dist = np.ascontiguousarray(dist, dtype=np.float64).ravel()
    bl = np.ascontiguousarray(border_limited, dtype=np.uint8).ravel()
    nc = None if ncc is None else np.ascontiguousarray(ncc, dtype=np.int32).ravel()
    counts = np.zeros((n_classes, n_bins + 1), dtype=np.int64)
    rc = lib().orc_distance_histogram(dist.shape[0], _p(dist, _D), _p(bl, _U8), _p(nc, _I32),
                                      int(ncc_lo), int(n_classes), int(n_bins),
                                      float(n_bins / d_max), _p(counts, _I64))
    if rc != OK:
        raise OracleError(rc, "distance_histogram")
    return counts
