"""Edge cases of the root finder on the GPU: the smallest phase grid, the
shortest subchains, a single star in every mode, iteration caps in the mixed
form, size limits, and one field through the batched entry point."""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields
from tests import parity
from tests.conftest import make_lens

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


def host_c(re, im):
    return re.cpu().numpy() + 1j * im.cpu().numpy()


def run(ctx, f, m_steps, **kw):
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(m_steps, caustics=True, **kw)
    torch.cuda.synchronize()
    return host_c(rr, ri), host_c(cr, ci), cn.cpu().numpy(), st, code


def against_oracle(f, R, W, cn, m_steps, S, colwise=True, relabelled=False):
    """relabelled: the seeds were taken in another star order (multipole
    sums take the stars in cell order), so the columns are matched at row 0
    first and must then agree in every row and in chain_next."""
    R_ref, cn_ref, _ = oracle.critical_curves(f, m_steps, n_sub=S)
    Fp = np.stack([oracle.eval_F(f, oracle.phase(j, m_steps), R_ref[j])[1]
                   for j in range(m_steps + 1)])
    bound = parity.root_bound(f, Fp)
    worst, ratio = parity.compare_row_sets(R, R_ref, bound)
    assert ratio <= 1.0
    n_r = R.shape[1]
    assert sorted(cn.tolist()) == list(range(n_r))
    assert np.max(np.abs(R[-1] - R[0][cn])) < 1e-8
    if colwise and relabelled:
        perm, _ = parity.pair(R_ref[0], R[0])
        assert float(np.max(np.abs(R[:, perm] - R_ref))) < 1e-8
        assert np.array_equal(cn[perm], perm[cn_ref])
    elif colwise:
        assert float(np.max(np.abs(R - R_ref))) < 1e-8
        assert np.array_equal(cn, cn_ref)
    W_ref = oracle.lens_map(f, R_ref)
    for j in range(m_steps + 1):
        idx, _ = parity.pair(R_ref[j], R[j])
        bw = 2 * abs(1 - f.kappa_s) * bound[j] + 1e-11 * (1 + np.abs(W_ref[j]))
        assert np.all(np.abs(W[j][idx] - W_ref[j]) <= bw)
    return worst


@pytest.mark.parametrize("precision,star_sums", [("fp64", "direct"), ("mixed", "direct"),
                                                 ("fp64", "fmm"), ("mixed", "fmm")])
def test_two_steps(ctx, precision, star_sums):
    """m = 2: one subchain, centre row 1, rows 0 and 2 at its ends."""
    say("m=2", precision, star_sums)
    f = fields.random_field(41, 12, kappa_star=0.4, gamma=0.35, masses="salpeter")
    R, W, cn, st, code = run(ctx, f, 2, precision=precision, star_sums=star_sums)
    assert R.shape == (3, 24) and st["n_subchains"] == 1
    against_oracle(f, R, W, cn, 2, 1, colwise=precision == "fp64", relabelled=star_sums == "fmm")


@pytest.mark.parametrize("precision,star_sums", [("fp64", "direct"), ("mixed", "direct"),
                                                 ("fp64", "fmm"), ("mixed", "fmm")])
def test_shortest_subchains(ctx, precision, star_sums):
    """S = m/2: every subchain is a centre row and its two neighbours, and
    every even row is a duplicated boundary."""
    say("S=m/2", precision, star_sums)
    f = fields.random_field(42, 20, kappa_star=0.5, gamma=0.25, masses="equal")
    m_steps = 40
    R, W, cn, st, code = run(ctx, f, m_steps, n_subchains=m_steps // 2, precision=precision,
                             star_sums=star_sums)
    assert st["n_subchains"] == m_steps // 2
    against_oracle(f, R, W, cn, m_steps, m_steps // 2, colwise=precision == "fp64",
                   relabelled=star_sums == "fmm")


@pytest.mark.parametrize("precision,predictor,star_sums", [
    ("fp64", 0, "direct"), ("fp64", 2, "direct"), ("mixed", 1, "direct"), ("mixed", 2, "direct"),
    ("fp64", 2, "fmm"), ("mixed", 2, "fmm")])
def test_single_star_every_mode(ctx, precision, predictor, star_sums):
    """N = 1: two roots on the ring |z - z1| = sqrt(m/(1 - kappa_s)), a
    point caustic at (1 - kappa_s) z1.  With multipole sums the one star is
    near for points in the grid and the expansion about it is exact outside."""
    say("single star", precision, predictor, star_sums)
    z1, mass, kap = -0.7 + 0.4j, 0.6, 0.15
    f = make_lens(z1, mass, kap, 0.0)
    m_steps = 96
    R, W, cn, st, code = run(ctx, f, m_steps, precision=precision, predictor=predictor,
                             star_sums=star_sums)
    rho = np.sqrt(mass / (1 - kap))
    assert np.max(np.abs(np.abs(R - z1) - rho)) < 1e-9
    assert np.max(np.abs(W - (1 - kap) * z1)) < 1e-8
    assert cn.tolist() == [1, 0]


def test_mixed_iteration_cap_is_reported(ctx, mlcc):
    """A cold start capped at one sweep in the mixed form ends in the FP64
    fallback, which reports the cap instead of running on."""
    say("mixed cap")
    f = fields.random_field(3, 20)
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    rr, ri, cn, st, code = ctx.find_critical_curves(100, max_iter_cold=1, precision="mixed",
                                                    raise_on_error=False)
    assert code == mlcc.MLCC_ERR_NOT_CONVERGED
    assert st["rows_capped"] >= 1


def test_size_limits_rejected(ctx, mlcc):
    """Limits are checked before any allocation."""
    say("size limits")
    f = fields.random_field(3, 5)
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    lib = mlcc.library()
    p = ctx.default_params((1 << 28) + 2)
    z = dev(np.zeros(4))
    code = lib.mlcc_find_critical_curves(ctx._h, p, mlcc._ptr(z), mlcc._ptr(z), None, None, None,
                                         None)
    assert code == mlcc.MLCC_ERR_INVALID
    p = ctx.default_params(100)
    p.predictor = 3
    code = lib.mlcc_find_critical_curves(ctx._h, p, mlcc._ptr(z), mlcc._ptr(z), None, None, None,
                                         None)
    assert code == mlcc.MLCC_ERR_INVALID
    with pytest.raises(mlcc.MlccError):
        ctx.set_lenses(dev(np.zeros(0)), dev(np.zeros(0)), dev(np.zeros(0)), 0.0, 0.3)


def test_one_field_batched_equals_single(ctx):
    """The batched entry point with one field gives the single-field result
    bit for bit (unequal masses: the same kernels run either way)."""
    say("one field batched")
    f = fields.random_field(44, 45, kappa_star=0.35, kappa_s=0.05, gamma=0.4, masses="salpeter")
    R1, W1, cn1, _, _ = run(ctx, f, 120, n_subchains=6)
    ctx.set_lenses_batched([0, 45], dev(f.x), dev(f.y), dev(f.m), [f.kappa_s], [f.gamma])
    rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(120, n_subchains=6, caustics=True)
    torch.cuda.synchronize()
    assert ctx.root_offsets == [0, rr.numel()]
    assert np.array_equal(host_c(rr, ri).reshape(R1.shape).view(np.float64), R1.view(np.float64))
    assert np.array_equal(host_c(cr, ci).reshape(W1.shape).view(np.float64), W1.view(np.float64))
    assert np.array_equal(cn.cpu().numpy(), cn1)


def test_mixed_restart_after_doubled_root(ctx):
    """A 3-star field whose cold start, finished by Newton steps, puts two
    columns on one root: the row identities catch it, and the row restarts
    from the seeds in FP64 instead of keeping the doubled root."""
    say("mixed doubled root")
    f = fields.random_field(2233, 3, kappa_star=0.3, kappa_s=0.1, gamma=0.35, masses="salpeter")
    m_steps, S = 64, 8
    R, W, cn, st, code = run(ctx, f, m_steps, n_subchains=S, precision="mixed")
    assert code == 0
    print("[stats]", {k: st[k] for k in ("rows_fallback", "polish_updates", "root_updates")})
    assert st["rows_fallback"] >= 1
    against_oracle(f, R, W, cn, m_steps, S, colwise=False)


def test_measured_valu_peak_is_plausible(mlcc):
    """The benchmark's FMA-chain probe (libvalu_probe.so) reports a rate between
    a third of and just above the published FP64 vector peak, 78.6 TFLOP/s,
    for FP64, and for unpacked FP32 (the published 157.3 TFLOP/s counts
    packed FP32 instructions, which issue two FMAs per lane)."""
    say("valu probe")
    from bench import valu_fma_tflops
    p64 = valu_fma_tflops("fp64")
    p32 = valu_fma_tflops("fp32")
    print("[probe] FP64", p64, "FP32", p32, flush=True)
    assert 0.33 * 78.6 < p64 < 1.1 * 78.6
    assert 0.33 * 78.6 < p32 < 1.1 * 157.3


def test_cold_start_from_second_seeds(ctx):
    """Every cold start made to begin again from the second set of start
    values (z_i +- i) after 4 sweeps, the path an FP64 cold start still
    unsettled after 100 sweeps takes: each restarts once, converges, and the
    chains it grows give the oracle's root sets and caustics in every row."""
    say("cold starts from the second seeds")
    f = fields.random_field(46, 25, kappa_star=0.45, kappa_s=0.1, gamma=0.3, masses="salpeter")
    m_steps, S = 120, 6
    R, W, cn, st, code = run(ctx, f, m_steps, n_subchains=S, cold_restart_sweeps=4)
    print("[stats]", {k: st[k] for k in ("cold_restarts", "cold_sweeps", "unconverged")})
    assert code == 0 and st["cold_restarts"] == S
    against_oracle(f, R, W, cn, m_steps, S, colwise=False)
