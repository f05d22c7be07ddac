"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle on
the same seeded inputs.  Marked `gpu`; each test prints its case first."""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields
from tests import parity, pins
from tests.conftest import Box, make_lens

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mlcc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_02121_amd import mlcc as m
    return m


@pytest.fixture(scope="module")
def ctx(mlcc):
    c = mlcc.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.array(a, copy=True), dtype=dtype).cuda()


def set_field(ctx, f):
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)


def host_c(re, im):
    return re.cpu().numpy() + 1j * im.cpu().numpy()


def gpu_roots(ctx, f, m_steps, **kw):
    set_field(ctx, f)
    rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(m_steps, caustics=True, **kw)
    torch.cuda.synchronize()
    gpu_roots.caustics = host_c(cr, ci)
    return host_c(rr, ri), cn.cpu().numpy(), st, (rr, ri, cn)


def check_roots_against_oracle(f, R_gpu, R_ref, label):
    Fp = np.stack([oracle.eval_F(f, oracle.phase(j, R_ref.shape[0] - 1), R_ref[j])[1]
                   for j in range(R_ref.shape[0])])
    bound = parity.root_bound(f, Fp)
    worst, ratio = parity.compare_row_sets(R_gpu, R_ref, bound)
    print(f"[{label}] max root distance {worst:.3e}, max distance/bound {ratio:.3f}", flush=True)
    assert ratio <= 1.0
    return worst


# --------------------------------------------------------------------------
# lens mapping
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,masses", [(1, "equal"), (37, "salpeter"), (46, "salpeter"), (300, "equal"),
                                     (1000, "equal")])
def test_map_caustics_matches_oracle(ctx, n, masses):
    say("map", n, masses)
    f = fields.random_field(7, n, kappa_star=0.4, kappa_s=0.2, gamma=0.45, masses=masses)
    set_field(ctx, f)
    rng = np.random.default_rng(n)
    z = rng.normal(scale=f.radius, size=1000 + n) + 1j * rng.normal(scale=f.radius, size=1000 + n)
    wr, wi = ctx.map_caustics(dev(z.real), dev(z.imag))
    w = host_c(wr, wi)
    ref = oracle.lens_map(f, z)
    err = float(np.max(np.abs(w - ref) / (1 + np.abs(ref))))
    print(f"[map n={n} {masses}] max relative error {err:.3e}", flush=True)
    assert err < 1e-12


def test_map_caustics_empty_and_errors(ctx, mlcc):
    say("map empty")
    f = fields.random_field(1, 5)
    set_field(ctx, f)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ctx.map_caustics(e, e)
    z = dev(np.zeros(4))
    with pytest.raises(mlcc.MlccError):
        ctx.map_caustics(z, z, out=(z, dev(np.zeros(4))))


# --------------------------------------------------------------------------
# roots: closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kappa_s,mass", [(0.0, 1.0), (0.2, 0.37)])
def test_single_lens_ring_gpu(ctx, kappa_s, mass):
    say("single lens", kappa_s, mass)
    z1 = 0.3 - 1.1j
    f = make_lens(z1, mass, kappa_s, 0.0)
    R, cn, st, (rr, ri, _) = gpu_roots(ctx, f, 64)
    rho = np.sqrt(mass / (1 - kappa_s))
    for j in range(65):
        phi = oracle.phase(j, 64)
        exact = z1 + np.array([1, -1]) * rho * np.exp(0.5j * phi)
        assert pins.set_distance(R[j], exact) < 1e-9
    wr, wi = ctx.map_caustics(rr.flatten(), ri.flatten())
    w = host_c(wr, wi)
    assert np.max(np.abs(w - (1 - kappa_s) * z1)) < 1e-9


def test_chang_refsdal_gpu(ctx):
    say("chang-refsdal")
    z1 = -0.4 + 0.25j
    f = make_lens(z1, 1.0, 0.0, 0.3)
    R, cn, st, (rr, ri, _) = gpu_roots(ctx, f, 400)
    for j in range(0, 401, 7):
        exact = pins.chang_refsdal_roots(z1, 1.0, 0.0, 0.3, oracle.phase(j, 400))
        assert pins.set_distance(R[j], exact) < 1e-9
    assert cn.tolist() == [1, 0]
    wr, wi = ctx.map_caustics(rr[0].contiguous(), ri[0].contiguous())
    cusp = 2 * 0.3 * np.sqrt(1.0 / 0.7)
    w1 = z1 + 0.3 * np.conj(z1)
    assert pins.set_distance(host_c(wr, wi) - w1, [cusp, -cusp]) < 1e-9


# --------------------------------------------------------------------------
# roots: oracle parity on seeded fields (several waves, ragged tail)
# --------------------------------------------------------------------------

CASES = [
    # name, n, masses, kappa_star, kappa_s, gamma, m_steps, n_sub
    ("tiny", 10, "equal", 0.3, 0.0, 0.3, 1000, 0),
    ("tiny_S1", 10, "equal", 0.3, 0.0, 0.3, 1000, 1),
    ("n37_salp", 37, "salpeter", 0.4, 0.2, 0.45, 200, 5),
    ("n100", 100, "equal", 0.5, 0.0, 0.3, 200, 4),
    ("n150_salp_S10", 150, "salpeter", 0.45, 0.1, 0.2, 200, 10),
]


@pytest.mark.parametrize("precision", ["fp64", "fp64_r32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_critical_curves_match_oracle(ctx, case, precision):
    """Both FP64 forms: the plain one (every term in double precision) and
    the one with FP32 root-root sums in warm rows."""
    name, n, masses, ks, kap_s, g, m_steps, S = case
    say("roots", case, precision)
    if name.startswith("tiny"):
        f = fields.tiny_field(0)
    else:
        f = fields.random_field(11, n, kappa_star=ks, kappa_s=kap_s, gamma=g, masses=masses)
    R, cn, st, (rr, ri, cnt) = gpu_roots(ctx, f, m_steps, n_subchains=S, precision=precision)
    print("[stats]", st, flush=True)
    # the plain form counts no FP32 work; the other runs its warm rows' root terms in FP32
    if precision == "fp64":
        assert st["algorithmic_flop_sweep_roots"] == 0.0 and st["root_updates_f32"] == 0
    else:
        assert st["algorithmic_flop_sweep_roots"] > 0.0
    R_ref, cn_ref, st_ref = oracle.critical_curves(f, m_steps, n_sub=1)
    check_roots_against_oracle(f, R, R_ref, name)
    # chain structure: row m = row 0 under chain_next, and the oracle grown
    # with the same subchains gives the same matrix column for column
    assert sorted(cn.tolist()) == list(range(2 * n))
    assert np.max(np.abs(R[-1] - R[0][cn])) < 1e-8
    R_s, cn_s, _ = oracle.critical_curves(f, m_steps, n_sub=st["n_subchains"])
    colwise = float(np.max(np.abs(R - R_s)))
    print(f"[{name}] column-wise distance to the oracle with S={st['n_subchains']}: {colwise:.3e}")
    assert colwise < 1e-8
    assert np.array_equal(cn, cn_s)
    # caustics: fused into the root finder, and by the standalone mapping
    W_fused = gpu_roots.caustics
    wr, wi = ctx.map_caustics(rr.flatten(), ri.flatten())
    W = host_c(wr, wi).reshape(R.shape)
    W_ref = oracle.lens_map(f, R_ref)
    worst = 0.0
    for j in range(R.shape[0]):
        idx, d = parity.pair(R_ref[j], R[j])
        Fp = oracle.eval_F(f, oracle.phase(j, m_steps), R_ref[j])[1]
        bw = 2 * abs(1 - f.kappa_s) * parity.root_bound(f, Fp) + 1e-11 * (1 + np.abs(W_ref[j]))
        assert np.all(np.abs(W[j][idx] - W_ref[j]) <= bw)
        assert np.all(np.abs(W_fused[j][idx] - W_ref[j]) <= bw)
        worst = max(worst, float(np.abs(W_fused[j][idx] - W_ref[j]).max()))
    print(f"[{name}] max caustic distance (fused) {worst:.3e}", flush=True)


MIXED_CASES = [
    ("tiny_mixed", 10, "equal", 0.3, 0.0, 0.3, 1000, 0),
    ("n100_mixed", 100, "equal", 0.5, 0.0, 0.3, 400, 4),
    ("n150_salp_mixed", 150, "salpeter", 0.45, 0.1, 0.2, 400, 10),
    ("n300_salp_mixed", 300, "salpeter", 0.4, 0.2, 0.45, 600, 6),
]


@pytest.mark.parametrize("case", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_precision_matches_oracle(ctx, case):
    """FP32 bulk sweeps + FP64 Newton polish: roots and caustics within the
    FP64 tolerance of the oracle."""
    name, n, masses, ks, kap_s, g, m_steps, S = case
    say("mixed", case)
    if name.startswith("tiny"):
        f = fields.tiny_field(0)
    else:
        f = fields.random_field(11, n, kappa_star=ks, kappa_s=kap_s, gamma=g, masses=masses)
    R, cn, st, (rr, ri, cnt) = gpu_roots(ctx, f, m_steps, n_subchains=S, precision="mixed")
    print("[stats]", {k: st[k] for k in ("root_updates", "root_updates_f32", "polish_updates",
                                         "rows_fallback", "sweeps")}, flush=True)
    assert st["root_updates_f32"] > 0 and st["polish_updates"] > 0
    R_ref, cn_ref, _ = oracle.critical_curves(f, m_steps, n_sub=1)
    worst = check_roots_against_oracle(f, R, R_ref, name)
    assert sorted(cn.tolist()) == list(range(2 * n))
    assert np.max(np.abs(R[-1] - R[0][cn])) < 1e-8
    W_fused = gpu_roots.caustics
    W_ref = oracle.lens_map(f, R_ref)
    wworst = 0.0
    for j in range(R.shape[0]):
        idx, d = parity.pair(R_ref[j], R[j])
        Fp = oracle.eval_F(f, oracle.phase(j, m_steps), R_ref[j])[1]
        bw = 2 * abs(1 - f.kappa_s) * parity.root_bound(f, Fp) + 1e-11 * (1 + np.abs(W_ref[j]))
        assert np.all(np.abs(W_fused[j][idx] - W_ref[j]) <= bw)
        wworst = max(wworst, float(np.abs(W_fused[j][idx] - W_ref[j]).max()))
    print(f"[{name}] mixed: max root error {worst:.3e}, max caustic error {wworst:.3e}", flush=True)



# Star and root counts whose partial tiles end in every mix of the shorter
# groups the term loops fall back to (8 terms share a reciprocal in full
# groups; a tile's remainder takes groups of 4, 2 and 1): stars 13 = 8+4+1,
# 15 = 8+4+2+1, 39 = 32+4+2+1, 46 = 40+4+2, 71 = 64+4+2+1; the other roots
# of a row past a block's own 64 end in remainders of 14 = 8+4+2 and 28 = 24+4.
TAIL_CASES = [(13, "equal"), (15, "salpeter"), (39, "equal"), (46, "salpeter"), (71, "equal")]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,masses", TAIL_CASES, ids=[f"n{c[0]}_{c[1]}" for c in TAIL_CASES])
def test_term_group_tails_match_oracle(ctx, n, masses, precision):
    say("group tails", n, masses, precision)
    f = fields.random_field(29, n, kappa_star=0.45, kappa_s=0.1, gamma=0.35, masses=masses)
    m_steps = 120
    R, cn, st, _ = gpu_roots(ctx, f, m_steps, n_subchains=2, precision=precision)
    R_ref, _, _ = oracle.critical_curves(f, m_steps, n_sub=1)
    check_roots_against_oracle(f, R, R_ref, f"tails n{n} {masses} {precision}")
    assert sorted(cn.tolist()) == list(range(2 * n))
    assert np.max(np.abs(R[-1] - R[0][cn])) < 1e-8

PREDICTOR_CASES = [
    # name, n, masses, kappa_star, kappa_s, gamma, m_steps, n_sub, precision, predictor
    ("n100_lin", 100, "equal", 0.5, 0.0, 0.3, 400, 4, "fp64", 1),
    ("n100_quad", 100, "equal", 0.5, 0.0, 0.3, 400, 4, "fp64", 2),
    ("n150_salp_quad", 150, "salpeter", 0.45, 0.1, 0.2, 400, 10, "fp64", 2),
    ("n300_salp_quad_mixed", 300, "salpeter", 0.4, 0.2, 0.45, 600, 6, "mixed", 2),
    ("tiny_quad", 10, "equal", 0.3, 0.0, 0.3, 1000, 0, "fp64", 2),
]


@pytest.mark.parametrize("case", PREDICTOR_CASES, ids=[c[0] for c in PREDICTOR_CASES])
def test_predictor_matches_oracle(ctx, case):
    """Warm rows started from an extrapolation along each chain: the same
    root sets within tolerance, the same chains as the oracle's warm start
    from the previous row, fewer updates than without it."""
    name, n, masses, ks, kap_s, g, m_steps, S, precision, pred = case
    say("predictor", case)
    if name.startswith("tiny"):
        f = fields.tiny_field(0)
    else:
        f = fields.random_field(11, n, kappa_star=ks, kappa_s=kap_s, gamma=g, masses=masses)
    R0, cn0, st0, _ = gpu_roots(ctx, f, m_steps, n_subchains=S, precision=precision,
                                predictor=0)
    R, cn, st, _ = gpu_roots(ctx, f, m_steps, n_subchains=S, precision=precision,
                             predictor=pred)
    W_fused = gpu_roots.caustics
    u0 = st0["root_updates"] + st0["root_updates_f32"] + st0["polish_updates"]
    u1 = st["root_updates"] + st["root_updates_f32"] + st["polish_updates"]
    print(f"[{name}] updates without / with predictor: {u0} / {u1}", flush=True)
    assert u1 < u0
    R_ref, _, _ = oracle.critical_curves(f, m_steps, n_sub=1)
    check_roots_against_oracle(f, R, R_ref, name)
    assert sorted(cn.tolist()) == list(range(2 * n))
    assert np.max(np.abs(R[-1] - R[0][cn])) < 1e-8
    R_s, cn_s, _ = oracle.critical_curves(f, m_steps, n_sub=st["n_subchains"])
    colwise = float(np.max(np.abs(R - R_s)))
    colwise0 = float(np.max(np.abs(R0 - R_s)))
    print(f"[{name}] column-wise distance to the oracle with S={st['n_subchains']}: "
          f"{colwise:.3e} (predictor {pred}), {colwise0:.3e} (previous-row start)")
    assert colwise < 1e-8 and colwise0 < 1e-8
    assert np.array_equal(cn, cn_s) and np.array_equal(cn0, cn_s)
    W_ref = oracle.lens_map(f, R_s)
    bound = np.stack([parity.root_bound(f, oracle.eval_F(f, oracle.phase(j, m_steps), R_s[j])[1])
                      for j in range(m_steps + 1)])
    assert np.all(np.abs(W_fused - W_ref) <= 2 * abs(1 - f.kappa_s) * bound
                  + 1e-11 * (1 + np.abs(W_ref)))


def test_determinism_bitwise(ctx):
    say("determinism")
    f = fields.random_field(5, 60, kappa_star=0.4, gamma=0.3, masses="salpeter")
    R1, cn1, _, _ = gpu_roots(ctx, f, 100, n_subchains=5)
    R2, cn2, _, _ = gpu_roots(ctx, f, 100, n_subchains=5)
    assert np.array_equal(R1.view(np.float64), R2.view(np.float64))
    assert np.array_equal(cn1, cn2)


def test_vieta_and_counts_any_size(ctx):
    say("vieta n=400")
    f = fields.random_field(21, 400, kappa_star=0.5, gamma=0.3)
    R, cn, st, _ = gpu_roots(ctx, f, 400)
    zs = f.x + 1j * f.y
    M = f.m.sum()
    for j in range(0, 401, 40):
        z = R[j]
        c = f.gamma - (1 - f.kappa_s) * np.exp(-1j * oracle.phase(j, 400))
        assert abs(z.sum() - 2 * zs.sum()) < 1e-9 * len(z)
        assert abs((z ** 2).sum() - (2 * (zs ** 2).sum() - 2 * M / c)) < 1e-9 * np.abs(z ** 2).sum()


def test_not_converged_is_reported(ctx, mlcc):
    say("iteration cap")
    f = fields.random_field(3, 20)
    set_field(ctx, f)
    rr, ri, cn, st, code = ctx.find_critical_curves(100, max_iter_cold=1, raise_on_error=False)
    assert code == mlcc.MLCC_ERR_NOT_CONVERGED
    assert st["rows_capped"] >= 1 and st["unconverged"] >= 1


def test_invalid_arguments(ctx, mlcc):
    say("invalid arguments")
    f = fields.random_field(3, 20)
    set_field(ctx, f)
    with pytest.raises(mlcc.MlccError):
        ctx.find_critical_curves(101)
    with pytest.raises(mlcc.MlccError):
        ctx.find_critical_curves(100, n_subchains=3)
    bad = make_lens([0.0, 1.0], 1.0, 0.0, 1.0)
    with pytest.raises(mlcc.MlccError):
        set_field(ctx, bad)
    dup = make_lens([0.5, 0.5], 1.0, 0.0, 0.3)
    with pytest.raises(mlcc.MlccError):
        set_field(ctx, dup)
    nan = make_lens([0.5, np.nan], 1.0, 0.0, 0.3)
    with pytest.raises(mlcc.MlccError):
        set_field(ctx, nan)
    # host memory where device memory is required
    x = torch.zeros(3, dtype=torch.float64)
    with pytest.raises(mlcc.MlccError):
        mlcc._check(mlcc.library().mlcc_set_lenses(ctx._h, 3, mlcc._ptr(x), mlcc._ptr(x),
                                                  mlcc._ptr(x), 0.0, 0.3))


# --------------------------------------------------------------------------
# crossing maps: bit-exact on identical vertices
# --------------------------------------------------------------------------

def _ncc_gpu(ctx, W, cn, grid):
    wr = dev(np.ascontiguousarray(W.real))
    wi = dev(np.ascontiguousarray(W.imag))
    c = None if cn is None else dev(cn, torch.int32)
    return ctx.caustic_crossings(wr, wi, c, grid).cpu().numpy()


def test_crossings_golden_diamond(ctx):
    say("ncc diamond")
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ncc_diamond.json")))
    W = (np.array(g["vertices_re"]) + 1j * np.array(g["vertices_im"]))[:, None]
    got = _ncc_gpu(ctx, W, np.array(g["chain_next"], dtype=np.int32), Box(**g["grid"]))
    assert np.array_equal(got, np.array(g["expected_rows_bottom_up"]))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_crossings_random_loops_bitexact(ctx, seed):
    say("ncc loops", seed)
    from tests.test_oracle_chains import random_loops
    W = random_loops(seed, 11, 700, scale=1.5, jitter=0.01)
    grid = Box(center_re=0.05, center_im=-0.1, half_width=3.0, half_height=2.4, nx=301, ny=257)
    ref = oracle.ncc_rows(W, None, grid)
    assert np.array_equal(_ncc_gpu(ctx, W, None, grid), ref)


def test_crossings_lattice_vertices_bitexact(ctx):
    say("ncc lattice")
    rng = np.random.default_rng(9)
    grid = Box(center_re=0.0, center_im=0.0, half_width=4.0, half_height=4.0, nx=16, ny=16)
    W = (rng.integers(-40, 41, size=(300, 7)) * 0.125) + 1j * (rng.integers(-40, 41, size=(300, 7)) * 0.125)
    cn = np.roll(np.arange(7), 3).astype(np.int32)
    assert np.array_equal(_ncc_gpu(ctx, W, cn, grid), oracle.ncc_pixels(W, cn, grid))


def test_crossings_of_oracle_caustics_bitexact(ctx):
    say("ncc tiny caustics")
    f = fields.tiny_field(0)
    R_ref, cn_ref, _ = oracle.critical_curves(f, 1000)
    W = oracle.lens_map(f, R_ref)
    grid = Box(center_re=0.0, center_im=0.0, half_width=8.0, half_height=8.0, nx=513, ny=509)
    ref = oracle.ncc_rows(W, cn_ref, grid)
    got = _ncc_gpu(ctx, W, cn_ref, grid)
    assert np.array_equal(got, ref)
    assert got.min() >= 0 and got.max() >= 1


def test_crossings_reject_bad_vertices(ctx, mlcc):
    say("ncc invalid")
    grid = Box(center_re=0.0, center_im=0.0, half_width=1.0, half_height=1.0, nx=4, ny=4)
    with pytest.raises(mlcc.MlccError):
        _ncc_gpu(ctx, np.array([[0.0], [1e30], [1j]]), None, grid)
    with pytest.raises(mlcc.MlccError):
        _ncc_gpu(ctx, np.array([[0.0], [np.nan]]), None, grid)
    with pytest.raises(mlcc.MlccError):
        _ncc_gpu(ctx, np.array([[0.0, 1.0], [1j, 2j]]), np.array([0, 5], dtype=np.int32), grid)


# --------------------------------------------------------------------------
# distance maps: exact squared distances
# --------------------------------------------------------------------------

def _dist_gpu(ctx, ncc, h, grid=None):
    ny, nx = ncc.shape
    if grid is None:
        grid = Box(center_re=0.0, center_im=0.0, half_width=0.5 * h * nx,
                   half_height=0.5 * h * ny, nx=nx, ny=ny)
    d, bl = ctx.caustic_distances(grid, dev(ncc, torch.int32))
    return d.cpu().numpy(), bl.cpu().numpy()


def test_distances_golden_plus(ctx):
    say("edt plus")
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "edt_plus.json")))
    ncc = np.array(g["ncc"], dtype=np.int32)
    d, bl = _dist_gpu(ctx, ncc, g["pixel_size"])
    d2 = np.array(g["expected_d2"])
    assert np.array_equal(np.rint((d / g["pixel_size"]) ** 2).astype(np.int64), d2)
    assert np.array_equal(bl, np.array(g["expected_border_limited"], dtype=np.uint8))


@pytest.mark.parametrize("seed,ny,nx", [(0, 97, 131), (1, 256, 256), (2, 64, 300)])
def test_distances_match_oracle(ctx, seed, ny, nx):
    say("edt", seed, ny, nx)
    from tests.test_oracle_chains import random_loops
    W = random_loops(seed, 15, 300, scale=1.4, jitter=0.02)
    grid = Box(center_re=0.0, center_im=0.0, half_width=3.0, half_height=3.0 * ny / nx, nx=nx, ny=ny)
    ncc = oracle.ncc_rows(W, None, grid)
    h = (2.0 * grid.half_width) / nx
    ref_d, ref_bl, ref_d2 = oracle.edt_twopass(ncc, h)
    d, bl = _dist_gpu(ctx, ncc, h, grid)
    assert np.array_equal(np.rint((d / h) ** 2).astype(np.int64), ref_d2)
    assert np.max(np.abs(d - ref_d) / np.maximum(ref_d, 1e-300)) <= 2.3e-16
    assert np.array_equal(bl, ref_bl)


@pytest.mark.parametrize("ny,nx,pixels", [(40, 1500, 1), (200, 1100, 3), (1300, 30, 2),
                                          (65, 64, 5)])
def test_distances_sparse_maps(ctx, ny, nx, pixels):
    """Few caustic pixels far apart: rows whose outward search runs past its
    window take the lower envelope instead; both must give the exact d^2.
    Odd band counts (rows not a multiple of 64) and single-column strips."""
    say("edt sparse", ny, nx, pixels)
    rng = np.random.default_rng(ny * 7 + nx)
    ncc = np.zeros((ny, nx), dtype=np.int32)
    for _ in range(pixels):
        r, c = int(rng.integers(0, ny)), int(rng.integers(0, nx))
        ncc[r:min(r + 3, ny), c:min(c + 2, nx)] = 1
    h = 0.01
    ref_d, ref_bl, ref_d2 = oracle.edt_twopass(ncc, h)
    d, bl = _dist_gpu(ctx, ncc, h)
    assert np.array_equal(np.rint((d / h) ** 2).astype(np.int64), ref_d2)
    assert np.array_equal(bl, ref_bl)


def test_distances_no_caustic(ctx):
    say("edt none")
    d, bl = _dist_gpu(ctx, np.full((7, 9), 3, dtype=np.int32), 0.1)
    assert np.all(np.isinf(d)) and np.all(bl == 1)


def test_distances_reject_oversized_maps(ctx, mlcc):
    """nx + ny above 30000 is refused before any kernel runs (the row pass
    keeps one envelope length per 64-column segment of a row in a fixed LDS
    array), so small buffers stand in for the map."""
    say("edt size limit")
    ncc = torch.zeros(16, dtype=torch.int32, device="cuda")
    dist = torch.zeros(16, dtype=torch.float64, device="cuda")
    big = mlcc.Grid(0.0, 0.0, 100.0, 75.0, 20000, 15000)
    with pytest.raises(mlcc.MlccError, match="30000"):
        ctx.caustic_distances(big, ncc, border_limited=False, out=(dist, None))
    torch.cuda.synchronize()
    assert float(dist.abs().sum()) == 0.0


# --------------------------------------------------------------------------
# end to end on the tiny field
# --------------------------------------------------------------------------

def test_end_to_end_tiny(ctx):
    say("end to end tiny")
    f = fields.tiny_field(0)
    R, cn, st, (rr, ri, cnt) = gpu_roots(ctx, f, 1000)
    wr, wi = ctx.map_caustics(rr.flatten(), ri.flatten())
    grid = Box(center_re=0.0, center_im=0.0, half_width=8.0, half_height=8.0, nx=256, ny=256)
    ncc = ctx.caustic_crossings(wr.view(rr.shape), wi.view(ri.shape), cnt, grid)
    dist, bl = ctx.caustic_distances(grid, ncc)
    ncc = ncc.cpu().numpy()
    R_ref, cn_ref, _ = oracle.critical_curves(f, 1000)
    W_ref = oracle.lens_map(f, R_ref)
    ncc_ref = oracle.ncc_rows(W_ref, cn_ref, grid)
    diff = np.argwhere(ncc != ncc_ref)
    # any disagreement must sit within a pixel of a caustic vertex
    h = 16.0 / 256
    pts = W_ref.ravel()
    for r, c in diff:
        p = (-8 + (c + 0.5) * h) + 1j * (-8 + (r + 0.5) * h)
        assert np.min(np.abs(pts - p)) < 2 * h
    print(f"[e2e] {len(diff)} differing pixels of {ncc.size}", flush=True)
    d_ref, bl_ref, _ = oracle.edt_twopass(ncc, h)
    assert np.array_equal(dist.cpu().numpy() > 0, d_ref > 0)
