"""The allocation-free crossing map (mlcc_caustic_crossings_noalloc) against
mlcc_caustic_crossings, bit for bit, through the C-ABI: two calls in a row,
the second on a smaller input (fewer pixels, rows and roots), so that the
shared fixed scratch array still holds the first call's values when the
second begins.  Marked `gpu`; each test prints its case first."""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields

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


def caustics_of(ctx, f, m_steps):
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    rr, _, wr, wi, cn, _, _ = ctx.find_critical_curves(m_steps, caustics=True)
    torch.cuda.synchronize()
    return wr.view(rr.shape), wi.view(rr.shape), cn


def test_noalloc_equals_allocating_call_twice(mlcc, ctx):
    big = fields.random_field(11, 40, kappa_star=0.4, kappa_s=0.0, gamma=0.3, masses="salpeter")
    small = fields.random_field(12, 9, kappa_star=0.3, kappa_s=0.1, gamma=0.25, masses="equal")
    cases = [
        # the largest map the fixed scratch holds, then a smaller one
        ("max grid 2048^2", big, 600, mlcc.Grid(0.3, -0.2, 9.0, 9.0, 2048, 2048)),
        ("smaller input", small, 200, mlcc.Grid(0.0, 0.0, 5.0, 4.0, 301, 257)),
    ]
    for label, f, m_steps, grid in cases:
        say("noalloc", label, f.n, m_steps, grid.nx, grid.ny)
        wr, wi, cn = caustics_of(ctx, f, m_steps)
        ref = ctx.caustic_crossings(wr, wi, cn, grid)
        out = torch.full((grid.ny, grid.nx), -12345, dtype=torch.int32, device="cuda")
        got = ctx.caustic_crossings(wr, wi, cn, grid, out=out, noalloc=True)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), f"{label}: {int((a != b).sum())} pixels differ"
        assert b.max() > 0, "the map holds caustics"
        if grid.nx * grid.ny <= 301 * 257:   # and the oracle on the same vertices
            W = wr.cpu().numpy() + 1j * wi.cpu().numpy()
            assert np.array_equal(a, oracle.ncc_rows(W, cn.cpu().numpy(), grid))


def test_noalloc_rejects_maps_beyond_its_scratch(mlcc, ctx):
    say("noalloc over the limit")
    f = fields.random_field(12, 9, kappa_star=0.3, kappa_s=0.1, gamma=0.25, masses="equal")
    wr, wi, cn = caustics_of(ctx, f, 100)
    grid = mlcc.Grid(0.0, 0.0, 5.0, 5.0, 2049, 2048)
    with pytest.raises(mlcc.MlccError) as e:
        ctx.caustic_crossings(wr, wi, cn, grid, noalloc=True)
    assert e.value.code == mlcc.MLCC_ERR_INVALID
    assert "scratch" in str(e.value)
    # the entry point still works after the rejection
    grid = mlcc.Grid(0.0, 0.0, 5.0, 5.0, 64, 64)
    ref = ctx.caustic_crossings(wr, wi, cn, grid)
    got = ctx.caustic_crossings(wr, wi, cn, grid, noalloc=True)
    assert torch.equal(got, ref)
