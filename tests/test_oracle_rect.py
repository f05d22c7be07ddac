"""Pins for the oracle's rectangular microlens field (Sec. 4.2, App. A, App. B),
CPU only.

The sheet enters the parametric equation through d alpha_s / d zbar, which
the oracle evaluates from the paper's closed form, and the lens map through
alpha_s, which it evaluates from the truncated series.  The pins reach the
same quantities by other routes: numerical integration of a uniform
rectangular sheet, finite-difference Wirtinger derivatives, the App. B error
bound, explicit polynomial roots, and the leading coefficients of the
rationalised polynomial (Vieta).
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from paper_2506_02121_amd import fields
from tests import parity

PHIS = [0.0, 0.9, 2.5, np.pi, 4.4]


def sheet_of(ks, c1, c2, t):
    return (float(ks), float(c1), float(c2), int(t))


def rectangle_deflection(ks, c1, c2, z):
    """Deflection of a uniform sheet of convergence -ks over [-c1, c1] x
    [-c2, c2]: -(ks/pi) int d^2z' / (conj(z) - conj(z')), with the x'
    integral done in closed form and the y' integral by quadrature."""
    x, y = z.real, z.imag

    def g(yp):
        return np.log(x + c1 + 1j * (yp - y)) - np.log(x - c1 + 1j * (yp - y))

    kw = dict(points=[y], limit=200, epsabs=1e-13, epsrel=1e-13)
    re = quad(lambda yp: g(yp).real, -c2, c2, **kw)[0]
    im = quad(lambda yp: g(yp).imag, -c2, c2, **kw)[0]
    return -(ks / np.pi) * (re + 1j * im)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("ks,c1,c2", [(0.4, 2.5, 3.8), (0.7, 5.0, 2.0)])
def test_closed_form_is_the_deflection_of_the_rectangle(ks, c1, c2):
    """Inside the field the App. B closed form (the series summed) is the
    deflection of the finite rectangular sheet."""
    sh = sheet_of(ks, c1, c2, 9)
    rng = np.random.default_rng(3)
    z = (2 * rng.random(6) - 1) * 0.9 * c1 + 1j * (2 * rng.random(6) - 1) * 0.9 * c2
    exact = oracle.rect_alpha(sh, z, exact=True)
    for k in range(z.shape[0]):
        ref = rectangle_deflection(ks, c1, c2, z[k])
        assert abs(exact[k] - ref) < 1e-10 * (1 + abs(ref))


@pytest.mark.parametrize("t,s", [(5, 2.0), (9, 1.5), (21, 1.25), (41, 1.1)])
def test_truncation_error_within_app_b_bound(t, s):
    ks, c1, c2 = 0.5, 3.0, 4.0
    sh = sheet_of(ks, c1, c2, t)
    ac = np.hypot(c1, c2)
    rng = np.random.default_rng(t)
    r = ac / s * np.sqrt(rng.random(200))
    z = r * np.exp(2j * np.pi * rng.random(200))
    err = np.abs(oracle.rect_alpha(sh, z) - oracle.rect_alpha(sh, z, exact=True))
    bound = ks / np.pi * 4 / (t + 1) * s ** -(t + 1) * ac * (s + 1) / (s - 1)
    assert err.max() <= bound
    # and the bound is not vacuous: the error is within a few orders of it
    assert err.max() > 1e-4 * bound


def test_series_derivatives_match_the_closed_form_derivative():
    """d alpha_s/dz = -kappa_star (the sheet extended to infinity) and
    d alpha_s/d zbar of the series equals App. B's closed form, by central
    differences of the series."""
    sh = sheet_of(0.45, 2.2, 3.1, 11)
    rng = np.random.default_rng(8)
    z = (2 * rng.random(8) - 1) * 1.5 + 1j * (2 * rng.random(8) - 1) * 1.5
    h = 1e-5
    ax = (oracle.rect_alpha(sh, z + h) - oracle.rect_alpha(sh, z - h)) / (2 * h)
    ay = (oracle.rect_alpha(sh, z + 1j * h) - oracle.rect_alpha(sh, z - 1j * h)) / (2 * h)
    d_dz = 0.5 * (ax - 1j * ay)
    d_dzbar = 0.5 * (ax + 1j * ay)
    assert np.abs(d_dz + 0.45).max() < 1e-8
    assert np.abs(d_dzbar - oracle.rect_dalpha_dzbar(sh, z)).max() < 1e-8


def test_taylor_degree_rule():
    for ks, c1, c2, s, eps in [(0.4, 2.0, 3.0, 1.3, 1e-6), (0.6, 10.0, 10.0, 1.5, 1e-9),
                               (0.2, 7.0, 1.0, 2.0, 1e-4)]:
        t = oracle.rect_taylor_degree(ks, c1, c2, s, eps)
        ac, th = np.hypot(c1, c2), np.arctan2(c2, c1)

        def bound(tt):
            return ks / np.pi * 4 / (tt + 1) * s ** -(tt + 1) * ac * (s + 1) / (s - 1)

        assert t % 2 == 1 and bound(t) <= eps
        r = np.fmod((t - 1) * th, np.pi)
        assert 0.1 * np.pi <= r <= 0.9 * np.pi
        # the smallest such t: every smaller odd degree breaks one condition
        for tt in range(1, t, 2):
            rr = np.fmod((tt - 1) * th, np.pi)
            assert bound(tt) > eps or not (0.1 * np.pi <= rr <= 0.9 * np.pi)


def sheet_poly(sh, degree):
    """Coefficients a_j (j = 0..degree) of conj(d alpha_s / d zbar) as a
    polynomial in z, recovered from samples on a circle by a discrete
    Fourier transform (exact for a polynomial of lower degree)."""
    K = 128
    rho = 0.5 * np.hypot(sh[1], sh[2])
    zk = rho * np.exp(2j * np.pi * np.arange(K) / K)
    vals = np.conj(oracle.rect_dalpha_dzbar(sh, zk))
    a = np.fft.fft(vals) / K / rho ** np.arange(K)
    assert np.abs(a[degree + 1:]).max() < 1e-12 * np.abs(a).max()
    return a[:degree + 1]


def rect_poly_roots(f, phi):
    """Roots of P = F prod (z - z_i)^2 for a rectangular field, expanded with
    numpy polynomial arithmetic."""
    sh = f.sheet
    a = sheet_poly(sh, sh[3])
    zs = f.x + 1j * f.y
    const = f.gamma - (1 - f.kappa_s) * np.exp(-1j * phi)
    # F numerator: (const - sum a_j z^j) prod (z - z_i)^2 + sum m_i prod_{j != i}(z - z_j)^2
    D = -a.copy()
    D[0] += const
    D = D[::-1]                      # numpy order: highest power first
    prod2 = np.array([1.0 + 0j])
    for z in zs:
        prod2 = np.polymul(prod2, np.polymul([1, -z], [1, -z]))
    P = np.polymul(D, prod2)
    for i, z in enumerate(zs):
        q = np.array([1.0 + 0j])
        for j, w in enumerate(zs):
            if j != i:
                q = np.polymul(q, np.polymul([1, -w], [1, -w]))
        P = np.polyadd(P, f.m[i] * q)
    P = np.trim_zeros(P, "f")
    # the leading coefficient can be a rounding residue when it should vanish
    while abs(P[0]) < 1e-12 * np.abs(P).max():
        P = P[1:]
    return np.roots(P)


@pytest.mark.parametrize("t", [3, 5, 7])
def test_rect_roots_are_the_polynomial_roots(t):
    """A 3-star rectangular field: the oracle finds 2N + t - 1 roots, the
    roots of the rationalised polynomial."""
    f = fields.rect_field(5, 3, kappa_star=0.4, gamma=0.25, aspect=1.3, t=t)
    assert oracle.num_roots(f) == 6 + t - 1
    for phi in PHIS:
        z, *_ = oracle.aberth_row(f, phi)
        ref = rect_poly_roots(f, phi)
        assert ref.shape[0] == z.shape[0]
        idx, d = parity.pair(ref, z)
        assert d.max() < 1e-8 * (1 + np.abs(ref).max())


@pytest.mark.parametrize("t", [3, 9, 21])
def test_rect_vieta_identities(t):
    """Sum r = 2 sum z_i; sum r^2 = 2 sum z_i^2 - 2 a_{t-3}/a_{t-1} (t >= 5),
    with a_j the sheet polynomial's coefficients and the constant term
    a_0 - (gamma - (1 - kappa_s) e^{-i phi}) for t = 3."""
    f = fields.rect_field(12, 40, kappa_star=0.5, gamma=0.3, aspect=1.7, t=t,
                          masses="salpeter")
    a = sheet_poly(f.sheet, t)
    zs = f.x + 1j * f.y
    for phi in [0.0, 2.0, np.pi]:
        z, *_ = oracle.aberth_row(f, phi)
        assert z.shape[0] == 2 * f.n + t - 1
        const = f.gamma - (1 - f.kappa_s) * np.exp(-1j * phi)
        lower = a[t - 3] - const if t == 3 else a[t - 3]
        s1 = 2 * zs.sum()
        s2 = 2 * (zs ** 2).sum() - 2 * lower / a[t - 1]
        assert abs(z.sum() - s1) < 1e-11 * np.abs(z).sum()
        assert abs((z ** 2).sum() - s2) < 1e-11 * (np.abs(z) ** 2).sum()


def test_rect_caustics_come_from_critical_points():
    """At every root the finite-difference Jacobian of the oracle's lens map
    is singular, and the App. C quantity 1/mu vanishes."""
    f = fields.rect_field(7, 12, kappa_star=0.5, kappa_s=0.05, gamma=0.35, aspect=1.2, t=9)
    h = 1e-6
    for phi in [0.4, 3.0]:
        z, *_ = oracle.aberth_row(f, phi)
        wx = (oracle.lens_map(f, z + h) - oracle.lens_map(f, z - h)) / (2 * h)
        wy = (oracle.lens_map(f, z + 1j * h) - oracle.lens_map(f, z - 1j * h)) / (2 * h)
        dwdz = 0.5 * (wx - 1j * wy)
        dwdzb = 0.5 * (wx + 1j * wy)
        det = np.abs(dwdz) ** 2 - np.abs(dwdzb) ** 2
        assert np.abs(det).max() < 1e-6
        assert np.abs(oracle.inv_mu(f, z)).max() < 1e-9
        # d w / d z = 1 - kappa_s (the sheet extended to infinity)
        assert np.abs(dwdz - (1 - f.kappa_s)).max() < 1e-7


def test_rect_chains_close_and_subchains_agree():
    f = fields.rect_field(9, 15, kappa_star=0.45, gamma=0.3, aspect=1.4, t=7)
    m_steps = 120
    R1, cn1, _ = oracle.critical_curves(f, m_steps, n_sub=1)
    R3, cn3, _ = oracle.critical_curves(f, m_steps, n_sub=3)
    assert R1.shape == (m_steps + 1, 2 * f.n + 6)
    assert sorted(cn1.tolist()) == list(range(R1.shape[1]))
    assert np.max(np.abs(R1[-1] - R1[0][cn1])) < 1e-8
    worst, _ = parity.compare_row_sets(R3, R1)
    assert worst < 1e-8
