"""Pins for the oracle's model and root finder (CPU only).

Each test reaches the quantity by a route that does not go through the
oracle's own formulas: the vector lens equation, finite-difference Wirtinger
derivatives, explicit polynomial roots, closed forms, exact identities.
"""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields
from tests import pins
from tests.conftest import make_lens

PHIS = [0.0, 0.7, np.pi / 2, 2.2, np.pi, 4.0, 5.9]


def small_field(n, seed, kappa_s=0.0, gamma=0.3, masses="equal"):
    return fields.random_field(seed, n, kappa_star=0.4, kappa_s=kappa_s, gamma=gamma,
                               masses=masses)


# --------------------------------------------------------------------------
# lens equation and the parametric condition (Sec. 2.1, Sec. 3.1, App. A)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kappa_s,gamma", [(0.0, 0.3), (0.2, 0.45), (-0.3, -0.2)])
def test_lens_map_equals_vector_form(kappa_s, gamma):
    f = small_field(25, 1, kappa_s, gamma, "salpeter")
    rng = np.random.default_rng(5)
    z = rng.normal(scale=3.0, size=200) + 1j * rng.normal(scale=3.0, size=200)
    w = oracle.lens_map(f, z)
    for ks in (0.1, 0.6):   # the compensating sheet cancels: no dependence on kappa_star
        v = pins.vector_lens_map(f, z.real, z.imag, kappa_star=ks)
        assert np.max(np.abs(w - v) / (1 + np.abs(v))) < 1e-12


@pytest.mark.parametrize("phi", PHIS)
def test_roots_satisfy_witt_parametric_condition(phi):
    """dw/dz e^{i phi} - dw/dzbar = 0 at every root, derivatives taken by
    finite differences of the vector-form lens equation."""
    f = small_field(12, 2, 0.1, 0.35)
    z, *_ = oracle.aberth_row(f, phi)
    dz, dzb = pins.wirtinger(f, z)
    res = np.abs(dz * np.exp(1j * phi) - dzb)
    assert res.max() < 1e-6
    # and the wrong phase sign would not vanish (guards the convention)
    if abs(np.sin(phi)) > 0.1:
        assert np.min(np.abs(dz * np.exp(-1j * phi) - dzb)) > 1e-3


def test_roots_are_critical_points_detJ_zero():
    f = small_field(15, 3, 0.0, 0.3)
    for phi in PHIS:
        z, *_ = oracle.aberth_row(f, phi)
        dz, dzb = pins.wirtinger(f, z)
        scale = np.abs(dz) ** 2 + np.abs(dzb) ** 2
        assert np.max(np.abs(pins.jacobian_det(f, z)) / scale) < 1e-6


def test_inv_mu_matches_jacobian_and_appC_identity():
    """1/mu from the oracle equals det J of the vector map, and obeys the
    App. C identity 1/mu = -|F|^2 - 2 Re(F (1-kappa_s) e^{i phi}) at any phi,
    hence |1/mu| <= |F| (|F| + 2|1-kappa_s|)."""
    f = small_field(20, 4, 0.15, 0.4, "salpeter")
    rng = np.random.default_rng(6)
    z = rng.normal(scale=2.5, size=300) + 1j * rng.normal(scale=2.5, size=300)
    im = oracle.inv_mu(f, z)
    dj = pins.jacobian_det(f, z)
    assert np.max(np.abs(im - dj) / (1 + np.abs(dj))) < 1e-6
    a = 1 - f.kappa_s
    for phi in PHIS:
        F, _ = oracle.eval_F(f, phi, z)
        ident = -np.abs(F) ** 2 - 2 * np.real(F * a * np.exp(1j * phi))
        assert np.max(np.abs(im - ident) / (1 + np.abs(im))) < 1e-9
        bound = np.abs(F) * (np.abs(F) + 2 * abs(a))
        assert np.all(np.abs(im) <= bound * (1 + 1e-12) + 1e-12)


def test_F_prime_is_derivative_of_F():
    f = small_field(10, 7, 0.0, 0.3, "salpeter")
    rng = np.random.default_rng(8)
    z = rng.normal(scale=2.0, size=50) + 1j * rng.normal(scale=2.0, size=50)
    h = 1e-6
    F0, Fp = oracle.eval_F(f, 1.3, z)
    Fa, _ = oracle.eval_F(f, 1.3, z + h)
    Fb, _ = oracle.eval_F(f, 1.3, z - h)
    Fc, _ = oracle.eval_F(f, 1.3, z + 1j * h)
    Fd, _ = oracle.eval_F(f, 1.3, z - 1j * h)
    # F is holomorphic in z: both directional derivatives agree with F'
    assert np.max(np.abs((Fa - Fb) / (2 * h) - Fp) / (1 + np.abs(Fp))) < 1e-5
    assert np.max(np.abs((Fc - Fd) / (2j * h) - Fp) / (1 + np.abs(Fp))) < 1e-5


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kappa_s", [0.0, 0.2, -0.4])
@pytest.mark.parametrize("mass", [1.0, 0.37])
def test_single_lens_ring_and_point_caustic(kappa_s, mass):
    z1 = 0.3 - 1.1j
    f = make_lens(z1, mass, kappa_s, 0.0)
    rho = np.sqrt(mass / (1 - kappa_s))
    for phi in PHIS:
        z, *_ = oracle.aberth_row(f, phi)
        exact = z1 + np.array([1, -1]) * rho * np.exp(0.5j * phi)
        assert pins.set_distance(z, exact) < 1e-12
        w = oracle.lens_map(f, z)
        assert np.max(np.abs(w - (1 - kappa_s) * z1)) < 1e-12


@pytest.mark.parametrize("kappa_s,gamma,mass", [(0.0, 0.3, 1.0), (0.2, 0.45, 0.5),
                                                (0.0, -0.6, 1.0), (0.3, 1.2, 0.8)])
def test_chang_refsdal_roots_caustic_and_cusps(kappa_s, gamma, mass):
    z1 = -0.4 + 0.25j
    f = make_lens(z1, mass, kappa_s, gamma)
    a = 1 - kappa_s
    for phi in PHIS:
        if phi == 0.0 and gamma > a:
            # one star, real seeds z1 +- 1 and a real F on the real u axis:
            # the iteration cannot leave that axis while the roots are
            # imaginary (a symmetric start of the paper's seed rule)
            continue
        z, *_ = oracle.aberth_row(f, phi)
        exact = pins.chang_refsdal_roots(z1, mass, kappa_s, gamma, phi)
        assert pins.set_distance(z, exact) < 1e-12
        w = oracle.lens_map(f, z)
        wexact = pins.chang_refsdal_caustic(z1, mass, kappa_s, gamma, exact - z1)
        assert pins.set_distance(w, wexact) < 1e-11
    w1 = a * z1 + gamma * np.conj(z1)
    if a - gamma > 0:   # cusps on the real axis at phi = 0
        z, *_ = oracle.aberth_row(f, 0.0)
        cusp = 2 * gamma * np.sqrt(mass / (a - gamma))
        assert pins.set_distance(oracle.lens_map(f, z) - w1, [cusp, -cusp]) < 1e-11
    if a + gamma > 0:   # and on the imaginary axis at phi = pi
        z, *_ = oracle.aberth_row(f, np.pi)
        cusp = 2j * gamma * np.sqrt(mass / (a + gamma))
        assert pins.set_distance(oracle.lens_map(f, z) - w1, [cusp, -cusp]) < 1e-11


def test_chang_refsdal_numbers():
    """kappa_s = 0, m = 1, gamma = 0.3: cusps at +-0.717137 and -+0.526235 i."""
    f = make_lens(0.0, 1.0, 0.0, 0.3)
    z, *_ = oracle.aberth_row(f, 0.0)
    assert pins.set_distance(oracle.lens_map(f, z), [0.7171371656, -0.7171371656]) < 1e-9
    z, *_ = oracle.aberth_row(f, np.pi)
    assert pins.set_distance(oracle.lens_map(f, z), [0.5262348115j, -0.5262348115j]) < 1e-9


# --------------------------------------------------------------------------
# explicit polynomial roots (Sec. 3.1 rationalisation)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 5, 8])
@pytest.mark.parametrize("kappa_s,gamma", [(0.0, 0.3), (0.2, 0.45)])
def test_roots_match_companion_matrix(n, kappa_s, gamma):
    f = small_field(n, 10 + n, kappa_s, gamma, "salpeter")
    for phi in [0.0, 1.1, np.pi, 4.4]:
        z, *_ = oracle.aberth_row(f, phi)
        assert z.shape[0] == 2 * n
        cr = pins.companion_roots(f, phi)
        assert cr.shape[0] == 2 * n
        # polish the eigenvalues (their error grows with the degree) with
        # plain Newton on the explicit polynomial before comparing
        P = np.polynomial.polynomial
        c = pins.poly_coeffs(f, phi)
        dc = P.polyder(c)
        for _ in range(3):
            cr = cr - P.polyval(cr, c) / P.polyval(cr, dc)
        assert pins.set_distance(z, cr) < 1e-9


@pytest.mark.parametrize("phi", [0.3, np.pi, 5.0])
def test_roots_match_multiprecision(phi):
    f = small_field(3, 21, 0.1, 0.25, "salpeter")
    z, *_ = oracle.aberth_row(f, phi)
    ref = pins.mp_roots(f, phi)
    assert ref.shape[0] == 6
    assert pins.set_distance(z, ref) < 1e-13


# --------------------------------------------------------------------------
# exact identities at any N (Vieta: top two coefficients of P)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(10, 0), (150, 1)])
def test_vieta_identities(n, seed):
    f = small_field(n, 30 + seed, 0.0, 0.3, "salpeter")
    zs = f.x + 1j * f.y
    M = f.m.sum()
    for phi in [0.0, 2.0, np.pi]:
        z, *_ = oracle.aberth_row(f, phi)
        c = f.gamma - (1 - f.kappa_s) * np.exp(-1j * phi)
        scale1 = np.abs(z).sum()
        scale2 = (np.abs(z) ** 2).sum()
        assert abs(z.sum() - 2 * zs.sum()) < 1e-12 * scale1 + 1e-9
        assert abs((z ** 2).sum() - (2 * (zs ** 2).sum() - 2 * M / c)) < 1e-12 * scale2 + 1e-9
        # all 2N roots distinct
        d = np.abs(z[:, None] - z[None, :]) + np.eye(z.shape[0]) * 1e9
        assert d.min() > 1e-6


# --------------------------------------------------------------------------
# metamorphic relations
# --------------------------------------------------------------------------

def _roots(f, phi):
    return oracle.aberth_row(f, phi)[0]


def test_translation_rotation_conjugation_scaling():
    f = small_field(9, 40, 0.1, 0.3, "salpeter")
    zs = f.x + 1j * f.y
    phi = 1.7
    z = _roots(f, phi)
    w = oracle.lens_map(f, z)
    t = 1.3 - 0.8j
    ft = make_lens(zs + t, f.m, f.kappa_s, f.gamma)
    zt = _roots(ft, phi)
    assert pins.set_distance(zt, z + t) < 1e-10
    a = 1 - f.kappa_s
    assert pins.set_distance(oracle.lens_map(ft, zt), w + a * t + f.gamma * np.conj(t)) < 1e-10
    fr = make_lens(-zs, f.m, f.kappa_s, f.gamma)
    zr = _roots(fr, phi)
    assert pins.set_distance(zr, -z) < 1e-10
    assert pins.set_distance(oracle.lens_map(fr, zr), -w) < 1e-10
    fc = make_lens(np.conj(zs), f.m, f.kappa_s, f.gamma)
    zc = _roots(fc, -phi)
    assert pins.set_distance(zc, np.conj(z)) < 1e-10
    assert pins.set_distance(oracle.lens_map(fc, zc), np.conj(w)) < 1e-10
    s = 2.5
    fs = make_lens(s * zs, s * s * f.m, f.kappa_s, f.gamma)
    zsc = _roots(fs, phi)
    assert pins.set_distance(zsc, s * z) < 1e-9
    assert pins.set_distance(oracle.lens_map(fs, zsc), s * w) < 1e-9


# --------------------------------------------------------------------------
# the iteration itself (Sec. 3.2)
# --------------------------------------------------------------------------

def test_cold_seeds_are_stars_plus_minus_one():
    f = small_field(7, 50)
    s = oracle.seeds(f)
    zs = f.x + 1j * f.y
    assert np.array_equal(s[0::2], zs + 1)
    assert np.array_equal(s[1::2], zs - 1)


def test_cutoffs_flag_roots_and_iteration_cap_reports():
    f = fields.tiny_field(0)
    z, sw, up, rc = oracle.aberth_row(f, np.pi, polish=False)
    assert rc == oracle.OK and 5 <= sw <= 60
    assert up <= sw * 20
    # one sweep cannot converge a cold start: the cap is reported, not hidden
    _, sw1, _, rc1 = oracle.aberth_row(f, np.pi, max_iter=1, allow_unconverged=True)
    assert rc1 == oracle.ERR_NOT_CONVERGED and sw1 == 1
    # with no |mu| test, the step test alone leaves steps below 1e-9 behind:
    # roots agree with a fully polished solve to far below the cutoff
    zp, *_ = oracle.aberth_row(f, np.pi, tol_mu=0.0, polish=False)
    assert pins.set_distance(zp, z) < 1e-9


def test_warm_start_needs_few_sweeps():
    """Sec. 3.2: seeding with the previous phase's roots cuts the sweeps."""
    f = small_field(60, 60, 0.0, 0.3)
    z0, cold, *_ = oracle.aberth_row(f, np.pi)
    _, warm, *_ = oracle.aberth_row(f, np.pi + 2 * np.pi / 2000, z0=z0)
    assert warm < cold and warm <= 4


def test_invalid_inputs_rejected():
    f = make_lens([0.0, 1.0], 1.0, 0.0, 1.0)   # |gamma| = |1 - kappa_s|
    with pytest.raises(oracle.OracleError):
        oracle.aberth_row(f, 0.5)
    g = make_lens([0.0, np.nan], 1.0, 0.0, 0.3)
    with pytest.raises(oracle.OracleError):
        oracle.aberth_row(g, 0.5)
