"""GPU parity of the moving-source distances and distance histograms (Sec.
5.2, Figs. 5 bottom, 6, 7) with the CPU oracle: bit for bit on the same N_cc
maps (the crossing parameters are single correctly rounded divisions of exact
half-integer offsets on both sides), including axis and diagonal directions
whose rays run through pixel corners, and sampled pixels of a full-size
2048^2 map."""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields
from tests.conftest import Box
from tests.test_oracle_directional import blob_map

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


def grid_for(ny, nx, h):
    return Box(center_re=0.0, center_im=0.0, half_width=0.5 * nx * h, half_height=0.5 * ny * h,
               nx=nx, ny=ny)


ANGLES = [0.0, np.pi / 4, np.pi / 2, 0.3, 1.9, 0.75 * np.pi, np.pi, 1.25 * np.pi, 3.7, 1.5 * np.pi, 5.0,
          1.75 * np.pi]


@pytest.mark.parametrize("angle", ANGLES)
def test_directional_bitwise(ctx, angle):
    say("directional", angle)
    ncc = blob_map(11, 97, 83, n_blobs=9)
    h = 0.37
    d, bl = ctx.caustic_distances_directional(grid_for(97, 83, h), dev(ncc, torch.int32), angle)
    ref, rbl = oracle.directional_distance(ncc, h, angle)
    assert np.array_equal(bl.cpu().numpy(), rbl)
    assert np.array_equal(d.cpu().numpy().view(np.uint64), ref.view(np.uint64))


def test_directional_of_caustic_map(ctx):
    """On the crossing map of a field's own caustics."""
    say("directional of caustics")
    f = fields.tiny_field(0)
    ctx.set_lenses(dev(f.x), dev(f.y), dev(f.m), f.kappa_s, f.gamma)
    rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(1000, caustics=True)
    g = Box(center_re=0.0, center_im=0.0, half_width=6.0, half_height=6.0, nx=181, ny=181)
    ncc = ctx.caustic_crossings(cr, ci, cn, g)
    nh = ncc.cpu().numpy()
    for angle in (0.6, 2.5):
        d, bl = ctx.caustic_distances_directional(g, ncc, angle)
        ref, rbl = oracle.directional_distance(nh, 12.0 / 181, angle)
        assert np.array_equal(bl.cpu().numpy(), rbl)
        assert np.array_equal(d.cpu().numpy().view(np.uint64), ref.view(np.uint64))


def test_histograms_bitwise(ctx):
    say("histograms")
    ncc = blob_map(12, 120, 140, n_blobs=12)
    h = 0.5
    g = grid_for(120, 140, h)
    ncc_d = dev(ncc, torch.int32)
    for angle in (0.0, 1.2):
        d, bl = ctx.caustic_distances_directional(g, ncc_d, angle)
        dh, blh = oracle.directional_distance(ncc, h, angle)
        got = ctx.distance_histogram(d, bl, 40, 20.0).cpu().numpy()
        assert np.array_equal(got, oracle.distance_histogram(dh, blh, 40, 20.0))
        lo, ncls = int(ncc.min()), int(ncc.max() - ncc.min() + 1)
        got = ctx.distance_histogram(d, bl, 25, 10.0, ncc=ncc_d, ncc_lo=lo,
                                     n_classes=ncls).cpu().numpy()
        ref = oracle.distance_histogram(dh, blh, 25, 10.0, ncc=ncc, ncc_lo=lo, n_classes=ncls)
        assert np.array_equal(got, ref)


def slab_distance(mask, r, c, ca, sa):
    """The oracle's definition for one pixel, vectorised over the caustic
    pixels (the same half-integer divisions)."""
    qr, qc = np.nonzero(mask)
    with np.errstate(divide="ignore", invalid="ignore"):
        def near_far(lo, hi, comp):
            if comp == 0.0:
                inside = (lo < 0.0) & (hi > 0.0)
                return np.where(inside, -np.inf, np.inf), np.where(inside, np.inf, -np.inf)
            t1, t2 = lo / comp, hi / comp
            return np.minimum(t1, t2), np.maximum(t1, t2)
        nx_, fx = near_far((qc - c).astype(np.float64) - 0.5, (qc - c).astype(np.float64) + 0.5, ca)
        ny_, fy = near_far((qr - r).astype(np.float64) - 0.5, (qr - r).astype(np.float64) + 0.5, sa)
    tn, tf = np.maximum(nx_, ny_), np.minimum(fx, fy)
    ok = (tn < tf) & (tf > 0) & (tn >= 0)
    return tn[ok].min() if ok.any() else None


def test_directional_fullsize_samples(ctx):
    """A 2048^2 map: 64 sampled pixels against the definition, bit for bit."""
    say("directional 2048^2")
    ncc = blob_map(13, 2048, 2048, n_blobs=40)
    mask = oracle.caustic_mask(ncc)
    h = 40.0 / 2048
    angle = 2.1
    d, bl = ctx.caustic_distances_directional(grid_for(2048, 2048, h), dev(ncc, torch.int32), angle)
    d, bl = d.cpu().numpy(), bl.cpu().numpy()
    rng = np.random.default_rng(5)
    ca, sa = np.cos(angle), np.sin(angle)
    for _ in range(64):
        r, c = int(rng.integers(0, 2048)), int(rng.integers(0, 2048))
        if mask[r, c]:
            assert d[r, c] == 0.0 and bl[r, c] == 0
            continue
        t = slab_distance(mask, r, c, ca, sa)
        if t is None:
            assert bl[r, c] == 1
        else:
            assert bl[r, c] == 0 and d[r, c] == t * h


def test_directional_arguments(ctx, mlcc):
    say("directional arguments")
    ncc = dev(np.zeros((8, 8)), torch.int32)
    with pytest.raises(mlcc.MlccError):   # pixels not square
        ctx.caustic_distances_directional(Box(center_re=0, center_im=0, half_width=1.0,
                                              half_height=2.0, nx=8, ny=8), ncc, 0.1)
    with pytest.raises(mlcc.MlccError):
        ctx.caustic_distances_directional(grid_for(8, 8, 1.0), ncc, float("nan"))
    d, bl = ctx.caustic_distances_directional(grid_for(8, 8, 1.0), ncc, 0.1)
    with pytest.raises(mlcc.MlccError):
        ctx.distance_histogram(d, bl, 0, 1.0)
    with pytest.raises(mlcc.MlccError):
        ctx.distance_histogram(d, bl, 8192, 1.0)
    with pytest.raises(mlcc.MlccError):
        ctx.distance_histogram(d, bl, 8, -1.0)
    assert ctx.distance_histogram(d, bl, 8, 1.0).sum().item() == 0   # every pixel border-limited
