"""Independent references used to pin the oracle (and, through it, the HIP
path).  Nothing here calls the oracle or the HIP library: each function is a
different route to a quantity the paper fixes.

* vector_lens_map: the paper's lens equation in vector form (Sec. 2.1,
  the micro-lens mapping with its diagonal macro matrix), with the
  compensating sheet alpha_s(x) = -kappa_star x of App. A.  The oracle uses
  the complex form of Sec. 3.1; agreement pins the conjugations and signs.
* wirtinger: finite-difference d/dz and d/dzbar of that vector map, for
  Witt's parametric condition dw/dz e^{i phi} - dw/dzbar = 0 (Sec. 3.1).
* companion_roots / mp_roots: the roots of the rationalised polynomial
  P(z) = F(z) prod (z - z_i)^2 (Sec. 3.1) expanded explicitly, solved by
  numpy's companion-matrix eigenvalues and by mpmath at 50 digits.
* chang_refsdal_*: closed forms for one star plus shear.
* cr_image_count: the number of images of the one-star-plus-shear lens at a
  source position, from the quartic its lens equation reduces to.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linear_sum_assignment


def vector_lens_map(field, x, y, kappa_star=0.37):
    """y = diag(1-k+g, 1-k-g) x - sum m_i (x - x_i)/|x - x_i|^2 - alpha_s(x),
    k = kappa_s + kappa_star, alpha_s(x) = -kappa_star x."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    k = field.kappa_s + kappa_star
    g = field.gamma
    y1 = (1 - k + g) * x
    y2 = (1 - k - g) * y
    for xi, yi, mi in zip(field.x, field.y, field.m):
        dx = x - xi
        dy = y - yi
        r2 = dx * dx + dy * dy
        y1 = y1 - mi * dx / r2
        y2 = y2 - mi * dy / r2
    y1 = y1 + kappa_star * x
    y2 = y2 + kappa_star * y
    return y1 + 1j * y2


def wirtinger(field, z, h=1e-6):
    """(dw/dz, dw/dzbar) by central differences of the vector lens map."""
    z = np.asarray(z, dtype=np.complex128)
    wx = (vector_lens_map(field, z.real + h, z.imag) - vector_lens_map(field, z.real - h, z.imag)) / (2 * h)
    wy = (vector_lens_map(field, z.real, z.imag + h) - vector_lens_map(field, z.real, z.imag - h)) / (2 * h)
    return 0.5 * (wx - 1j * wy), 0.5 * (wx + 1j * wy)


def jacobian_det(field, z, h=1e-6):
    """det(dy/dx) by central differences of the vector lens map."""
    z = np.asarray(z, dtype=np.complex128)
    wx = (vector_lens_map(field, z.real + h, z.imag) - vector_lens_map(field, z.real - h, z.imag)) / (2 * h)
    wy = (vector_lens_map(field, z.real, z.imag + h) - vector_lens_map(field, z.real, z.imag - h)) / (2 * h)
    return wx.real * wy.imag - wx.imag * wy.real


def poly_coeffs(field, phi):
    """Ascending coefficients of P(z) = c prod (z-z_i)^2 + sum_i m_i prod_{j!=i} (z-z_j)^2,
    c = gamma - (1 - kappa_s) e^{-i phi}."""
    P = np.polynomial.polynomial
    zs = np.asarray(field.x) + 1j * np.asarray(field.y)
    c = field.gamma - (1 - field.kappa_s) * np.exp(-1j * phi)
    sq = [P.polymul([-zi, 1.0], [-zi, 1.0]) for zi in zs]
    full = np.array([1.0 + 0j])
    for s in sq:
        full = P.polymul(full, s)
    tot = c * full
    for i, mi in enumerate(field.m):
        t = np.array([mi + 0j])
        for j, s in enumerate(sq):
            if j != i:
                t = P.polymul(t, s)
        tot = P.polyadd(tot, t)
    return tot


def companion_roots(field, phi):
    coeffs = poly_coeffs(field, phi)
    return np.roots(coeffs[::-1])


def mp_roots(field, phi, dps=50):
    import mpmath as mp
    with mp.workdps(dps):
        zs = [mp.mpc(a, b) for a, b in zip(field.x, field.y)]
        c = mp.mpf(field.gamma) - (1 - mp.mpf(field.kappa_s)) * mp.exp(-1j * mp.mpf(phi))
        # build P with mp arithmetic (descending coefficients)
        def pmul(a, b):
            out = [mp.mpc(0)] * (len(a) + len(b) - 1)
            for i, ai in enumerate(a):
                for j, bj in enumerate(b):
                    out[i + j] += ai * bj
            return out
        sq = [pmul([1, -zi], [1, -zi]) for zi in zs]
        full = [mp.mpc(1)]
        for s in sq:
            full = pmul(full, s)
        tot = [c * a for a in full]
        for i, mi in enumerate(field.m):
            t = [mp.mpc(mi)]
            for j, s in enumerate(sq):
                if j != i:
                    t = pmul(t, s)
            off = len(tot) - len(t)
            for q, v in enumerate(t):
                tot[off + q] += v
        r = mp.polyroots(tot, maxsteps=200, extraprec=400)
        return np.array([complex(v) for v in r])


def set_distance(a, b):
    """Max distance of the optimal bijection between two point sets."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    cost = np.abs(a[:, None] - b[None, :])
    ri, ci = linear_sum_assignment(cost)
    return float(cost[ri, ci].max())


def chang_refsdal_roots(z1, m, kappa_s, gamma, phi):
    """F = gamma + m/u^2 - (1-kappa_s) e^{-i phi} = 0, u = z - z1."""
    u = np.sqrt(m / ((1 - kappa_s) * np.exp(-1j * phi) - gamma))
    return np.array([z1 + u, z1 - u])


def chang_refsdal_caustic(z1, m, kappa_s, gamma, u):
    w1 = (1 - kappa_s) * z1 + gamma * np.conj(z1)
    return w1 + (1 - kappa_s) * u + gamma * np.conj(u) - m / np.conj(u)


def cr_image_count(w, m, kappa_s, gamma, tol=1e-7):
    """Images of w = a z + gamma conj(z) - m / conj(z) (star at the origin).

    With s = conj(z): z = Q / (a s), Q = w s - gamma s^2 + m, and the
    conjugate equation becomes a s Q (conj(w) - a s) - gamma Q^2 + m a^2 s^2 = 0,
    a quartic in s.  Its roots that satisfy the original equation are the
    images."""
    P = np.polynomial.polynomial
    a = 1.0 - kappa_s
    Q = np.array([m, w, -gamma], dtype=np.complex128)
    t1 = P.polymul(P.polymul([0, a], Q), [np.conj(w), -a])
    t2 = gamma * P.polymul(Q, Q)
    t3 = np.array([0, 0, m * a * a], dtype=np.complex128)
    poly = P.polyadd(P.polysub(t1, t2), t3)
    count = 0
    for s in np.roots(poly[::-1]):
        if abs(s) < 1e-12:
            continue
        z = np.polyval(Q[::-1], s) / (a * s)
        # the conjugate of z must be s, and the lens equation must hold
        res = abs(a * z + gamma * np.conj(z) - m / np.conj(z) - w)
        if abs(np.conj(z) - s) < tol * max(1, abs(s)) and res < tol * max(1, abs(w)):
            count += 1
    return count


def shoelace(poly):
    """Signed area of a closed polygon (positive = counter-clockwise)."""
    x, y = poly.real, poly.imag
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def loops_from_chains(rows_by_col, chain_next):
    """Assemble closed loops: follow column k over rows 0..m, then continue
    with column chain_next[k] until the starting column comes back."""
    n_r = rows_by_col.shape[1]
    seen = np.zeros(n_r, dtype=bool)
    loops = []
    for k0 in range(n_r):
        if seen[k0]:
            continue
        pts = []
        k = k0
        while not seen[k]:
            seen[k] = True
            pts.append(rows_by_col[:-1, k])
            k = int(chain_next[k])
        loops.append(np.concatenate(pts))
    return loops
