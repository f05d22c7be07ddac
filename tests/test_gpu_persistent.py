"""The persistent scheduler (one launch, fronts advanced by the work group
that finishes their pass) against the round scheduler: every front runs the
same passes on the same data whatever the order, so results agree bit for
bit."""
import numpy as np
import pytest

from paper_2506_02121_amd import fields
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


def run_both(ctx, m_steps, **kw):
    out = {}
    for sched in ("rounds", "persistent"):
        rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(m_steps, caustics=True,
                                                                schedule=sched, **kw)
        torch.cuda.synchronize()
        out[sched] = ([t.cpu().numpy() for t in (rr, ri, cr, ci, cn)], st)
    return out


def assert_same(out):
    (a, sa), (b, sb) = out["rounds"], out["persistent"]
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    for k in ("root_updates", "root_updates_f32", "polish_updates", "rows_fallback",
              "n_subchains"):
        assert sa[k] == sb[k], k
    print("[stats] rounds", sa["sweeps"], "persistent passes on the longest front", sb["sweeps"],
          flush=True)


CASES = [
    # name, n, masses, kappa_star, kappa_s, gamma, m_steps, S, precision
    ("n100", 100, "equal", 0.5, 0.0, 0.3, 200, 4, "fp64"),
    ("n150_salp", 150, "salpeter", 0.45, 0.1, 0.2, 200, 10, "fp64"),
    ("n300_salp_mixed", 300, "salpeter", 0.4, 0.2, 0.45, 600, 6, "mixed"),
    ("n500_auto", 500, "equal", 0.5, 0.0, 0.3, 1000, 0, "fp64"),
    ("n500_auto_mixed", 500, "equal", 0.5, 0.0, 0.3, 1000, 0, "mixed"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_persistent_equals_rounds(ctx, case):
    name, n, masses, ks, kap_s, g, m_steps, S, precision = case
    say("persistent", case)
    f = fields.random_field(11, n, kappa_star=ks, kappa_s=kap_s, gamma=g, masses=masses)
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    assert_same(run_both(ctx, m_steps, n_subchains=S, precision=precision))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_persistent_batched_many_fronts(ctx, precision):
    say("persistent batched", precision)
    fs = [fields.random_field(3000 + i, 2 + i % 7, kappa_star=0.3, kappa_s=0.05 * (i % 3),
                              gamma=0.2 + 0.05 * (i % 5), masses="salpeter")
          for i in range(300)] + [make_lens(0.1 + 0.2j, 0.8, 0.0, 0.0)]
    off = np.concatenate([[0], np.cumsum([len(f.x) for f in fs])])
    ctx.set_lenses_batched(off, dev(np.concatenate([f.x for f in fs])),
                           dev(np.concatenate([f.y for f in fs])),
                           dev(np.concatenate([f.m for f in fs])),
                           [f.kappa_s for f in fs], [f.gamma for f in fs])
    assert_same(run_both(ctx, 64, n_subchains=8, precision=precision))


def test_persistent_cap_reported(ctx, mlcc):
    say("persistent cap")
    f = fields.random_field(3, 20)
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    for precision in ("fp64", "mixed"):
        rr, ri, cn, st, code = ctx.find_critical_curves(100, max_iter_cold=1, precision=precision,
                                                        schedule="persistent",
                                                        raise_on_error=False)
        assert code == mlcc.MLCC_ERR_NOT_CONVERGED
        assert st["rows_capped"] >= 1


def test_persistent_watchdog_ends_the_launch(ctx, mlcc):
    """A watchdog of 1 ms on a field whose every pass takes longer: the idle
    workers see no pass finish within the limit, the launch ends (every
    worker leaves through the abort flag it polls), the call reports
    MLCC_ERR_HIP, and the context works normally afterwards."""
    say("persistent watchdog")
    f = fields.random_field(12, 40000, kappa_star=0.5, masses="equal")
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    rr, ri, cn, st, code = ctx.find_critical_curves(2, n_subchains=1, schedule="persistent",
                                                    watchdog_ms=1, raise_on_error=False)
    torch.cuda.synchronize()
    assert code == mlcc.MLCC_ERR_HIP
    assert "no pass finished" in mlcc.library().mlcc_last_error().decode()
    g = fields.random_field(13, 30)
    ctx.set_lenses(dev(g.x), dev(g.y), dev(g.m), g.kappa_s, g.gamma)
    rr, ri, cn, st, code = ctx.find_critical_curves(100, schedule="persistent")
    assert code == 0
    with pytest.raises(mlcc.MlccError):
        ctx.find_critical_curves(100, watchdog_ms=-1)
