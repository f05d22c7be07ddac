"""GPU parity of the rectangular microlens field (Sec. 4.2, App. A, App. B)
against the CPU oracle on the same seeded inputs: root sets row by row,
column-wise chains with the same subchains, chain closure, fused and
standalone caustics, the crossing map of the GPU's own caustics, and the
argument checks of the entry points."""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields
from tests import parity
from tests.conftest import Box

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


def set_rect(ctx, f):
    ks, c1, c2, t = f.sheet
    ctx.set_lenses_rect(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma, ks, c1, c2, t)


CASES = [
    # name, seed, n, masses, kappa_star, kappa_s, gamma, aspect, t, m_steps, S
    ("n40_t9", 21, 40, "equal", 0.45, 0.0, 0.3, 1.5, 9, 200, 4),
    ("n60_t3", 22, 60, "salpeter", 0.4, 0.1, 0.25, 1.2, 3, 160, 2),
    ("n120_t21_auto", 23, 120, "salpeter", 0.5, 0.0, 0.35, 0.8, 21, 240, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rect_roots_and_caustics_match_oracle(ctx, case):
    name, seed, n, masses, ks, kap_s, g, aspect, t, m_steps, S = case
    say("rect", case)
    f = fields.rect_field(seed, n, kappa_star=ks, kappa_s=kap_s, gamma=g, aspect=aspect, t=t,
                          masses=masses)
    set_rect(ctx, f)
    n_r = 2 * n + t - 1
    assert ctx.num_roots() == n_r
    rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(m_steps, n_subchains=S,
                                                            caustics=True)
    torch.cuda.synchronize()
    assert code == 0 and rr.shape == (m_steps + 1, n_r)
    R, W, cnh = host_c(rr, ri), host_c(cr, ci), cn.cpu().numpy()
    print("[stats]", {k: st[k] for k in ("n_subchains", "sweeps", "root_updates",
                                         "cold_sweeps", "max_row_sweeps")}, flush=True)
    # root sets against the oracle grown as one chain, within the
    # conditioning-aware bound
    R_ref, cn_ref, _ = oracle.critical_curves(f, m_steps, n_sub=1)
    Fp = np.stack([oracle.eval_F(f, oracle.phase(j, m_steps), R_ref[j])[1]
                   for j in range(m_steps + 1)])
    bound = parity.root_bound(f, Fp)
    worst, ratio = parity.compare_row_sets(R, R_ref, bound)
    print(f"[{name}] roots {worst:.3e} (ratio {ratio:.3f})", flush=True)
    assert ratio <= 1.0
    # chains: closure, and column for column the oracle with the same S once
    # the columns are matched at row 0.  Which seed ends on which root in the
    # first subchain's cold start is not unique (any labelling is a valid
    # answer, and the iteration from the seeds is sensitive to rounding); the
    # relabelling at subchain boundaries carries that one permutation through
    # every later row, so the whole matrix and chain_next must agree up to it.
    assert sorted(cnh.tolist()) == list(range(n_r))
    assert np.max(np.abs(R[-1] - R[0][cnh])) < 1e-8
    R_s, cn_s, _ = oracle.critical_curves(f, m_steps, n_sub=st["n_subchains"])
    perm, _ = parity.pair(R_s[0], R[0])
    relabelled = int(np.count_nonzero(perm != np.arange(n_r)))
    colwise = float(np.max(np.abs(R[:, perm] - R_s)))
    print(f"[{name}] column-wise distance with S={st['n_subchains']}: {colwise:.3e} "
          f"({relabelled} columns labelled differently by the cold start)", flush=True)
    assert colwise < 1e-8
    assert np.array_equal(cnh[perm], perm[cn_s])
    # caustics: fused into the root finder, and the standalone map
    W_ref = oracle.lens_map(f, R_ref)
    wr, wi = ctx.map_caustics(rr.flatten(), ri.flatten())
    W2 = host_c(wr, wi).reshape(R.shape)
    wworst = 0.0
    for j in range(m_steps + 1):
        idx, _ = parity.pair(R_ref[j], R[j])
        bw = 2 * abs(1 - f.kappa_s) * bound[j] + 1e-11 * (1 + np.abs(W_ref[j]))
        assert np.all(np.abs(W[j][idx] - W_ref[j]) <= bw)
        assert np.all(np.abs(W2[j][idx] - W_ref[j]) <= bw)
        wworst = max(wworst, float(np.abs(W[j][idx] - W_ref[j]).max()))
    print(f"[{name}] caustics {wworst:.3e}", flush=True)
    # the crossing map of the GPU caustics equals the oracle's on the same vertices
    c1, c2 = f.sheet[1], f.sheet[2]
    grid = Box(center_re=0.0, center_im=0.0, half_width=0.8 * c1, half_height=0.8 * c2,
               nx=257, ny=251)
    ncc = ctx.caustic_crossings(cr, ci, cn, grid).cpu().numpy()
    ref = oracle.ncc_rows(W, cnh, grid)
    assert np.array_equal(ncc, ref)
    assert ncc.min() >= 0


def test_rect_map_caustics_matches_oracle(ctx):
    say("rect map")
    f = fields.rect_field(31, 50, kappa_star=0.4, kappa_s=0.2, gamma=0.45, aspect=2.0, t=17,
                          masses="salpeter")
    set_rect(ctx, f)
    rng = np.random.default_rng(4)
    z = (2 * rng.random(3000) - 1) * f.sheet[1] + 1j * (2 * rng.random(3000) - 1) * f.sheet[2]
    wr, wi = ctx.map_caustics(dev(z.real), dev(z.imag))
    w = host_c(wr, wi)
    ref = oracle.lens_map(f, z)
    assert np.max(np.abs(w - ref) / (1 + np.abs(ref))) < 1e-12


def test_rect_schedules_agree_bitwise(ctx):
    say("rect schedules")
    f = fields.rect_field(41, 70, kappa_star=0.5, gamma=0.3, aspect=1.3, t=13)
    set_rect(ctx, f)
    out = []
    for sched in ("rounds", "persistent"):
        rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(120, n_subchains=3, caustics=True,
                                                                schedule=sched)
        torch.cuda.synchronize()
        out.append([t.cpu().numpy() for t in (rr, ri, cr, ci, cn)])
    for a, b in zip(*out):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_rect_arguments(ctx, mlcc):
    say("rect arguments")
    f = fields.rect_field(1, 10, kappa_star=0.4, gamma=0.3, aspect=1.0, t=7)
    x, y, m = dev(f.x), dev(f.y), dev(f.m)
    c1 = f.sheet[1]
    # a square: Arg c = pi/4, (t - 1) pi/4 must stay clear of multiples of pi
    for bad_t in (2, 5, 9, 131):
        with pytest.raises(mlcc.MlccError):
            ctx.set_lenses_rect(x, y, m, 0.0, 0.3, 0.4, c1, c1, bad_t)
    with pytest.raises(mlcc.MlccError):
        ctx.set_lenses_rect(x, y, m, 0.0, 0.3, -0.4, c1, c1, 7)
    ctx.set_lenses_rect(x, y, m, 0.0, 0.3, 0.4, c1, c1, 7)
    assert ctx.num_roots() == 26
    with pytest.raises(mlcc.MlccError):
        ctx.find_critical_curves(20, precision="mixed")
    # the library's degree rule agrees with the oracle's reading of App. B
    for args in [(0.4, 2.0, 3.0, 1.3, 1e-6), (0.6, 10.0, 10.0, 1.5, 1e-9), (0.2, 7.0, 1.0, 2.0, 1e-4)]:
        assert mlcc.rect_taylor_degree(*args) == oracle.rect_taylor_degree(*args)
    # a plain field afterwards is a circular field again
    g = fields.random_field(2, 10)
    ctx.set_lenses(dev(g.x), dev(g.y), dev(g.m), g.kappa_s, g.gamma)
    assert ctx.num_roots() == 20


def test_rect_stalled_cold_start_recovers(ctx):
    """The rectangular workload's field with 250 subchains, where one cold
    start (row 13160) once left an iterate parked far from every root for
    the whole sweep cap.  Every cold start here is made to begin again from
    the second set of start values after 5 sweeps (cold starts need 11-30),
    the path a stalled cold start takes after 100: the z_i +- i seeds and the
    sheet's extra roots turned by half their spacing.  Rows of that subchain,
    and rows elsewhere, against cold-started oracle rows."""
    say("rect cold starts from the second seeds")
    wl = fields.workload("rect")
    f, m_steps = wl.field, wl.m_steps
    set_rect(ctx, f)
    rr, ri, cn, st, code = ctx.find_critical_curves(m_steps, n_subchains=250,
                                                    cold_restart_sweeps=5,
                                                    raise_on_error=False)
    torch.cuda.synchronize()
    print("[stats]", {k: st[k] for k in ("n_subchains", "sweeps", "cold_sweeps",
                                         "unconverged", "cold_restarts")}, flush=True)
    assert code == 0 and st["unconverged"] == 0 and st["cold_restarts"] == 250
    R = host_c(rr, ri)
    cnh = cn.cpu().numpy()
    assert np.max(np.abs(R[-1] - R[0][cnh])) < 1e-8
    worst = 0.0
    for j in (13121, 13140, 13160, 13180, 13199, 0, 10000):
        phi = oracle.phase(j, m_steps)
        z_ref, _, _, _ = oracle.aberth_row(f, phi)
        Fp = oracle.eval_F(f, phi, z_ref)[1]
        idx, d = parity.pair(z_ref, R[j])
        assert np.all(d <= parity.root_bound(f, Fp)), j
        worst = max(worst, float(d.max()))
    print(f"[rect stall] sampled rows within {worst:.3e} of the oracle", flush=True)
