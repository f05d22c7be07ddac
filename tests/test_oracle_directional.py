"""Pins for the oracle's moving-source distances and distance histograms
(Sec. 5.2, Figs. 5 bottom, 6, 7), CPU only: row and column scans for the
axis directions, a fine ray march for oblique ones, the quarter-turn symmetry
of the pixel lattice, and counting identities of the histograms."""
import numpy as np
import pytest

import oracle


def blob_map(seed, ny, nx, n_blobs=6):
    """An N_cc-like integer map: overlapping discs with +1 inside each."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:ny, 0:nx]
    ncc = np.zeros((ny, nx), dtype=np.int32)
    for _ in range(n_blobs):
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        r = rng.uniform(2.0, 0.3 * min(nx, ny))
        ncc += ((yy - cy) ** 2 + (xx - cx) ** 2 < r * r).astype(np.int32)
    return ncc


def scan(mask, axis_step):
    """Distance in pixels along +x (axis_step = (0, 1)) etc. by a direct scan:
    k - 1/2 for the first caustic pixel k >= 1 cells away, 0 on a caustic
    pixel, the exit (cells to the edge + 1/2) with border flag otherwise."""
    ny, nx = mask.shape
    d = np.zeros((ny, nx))
    bl = np.zeros((ny, nx), dtype=np.uint8)
    dy, dx = axis_step
    for r in range(ny):
        for c in range(nx):
            if mask[r, c]:
                continue
            k = 1
            while True:
                rr, cc = r + k * dy, c + k * dx
                if not (0 <= rr < ny and 0 <= cc < nx):
                    d[r, c] = k - 0.5
                    bl[r, c] = 1
                    break
                if mask[rr, cc]:
                    d[r, c] = k - 0.5
                    break
                k += 1
    return d, bl


@pytest.mark.parametrize("angle,step", [(0.0, (0, 1)), (np.pi / 2, (1, 0)), (np.pi, (0, -1)),
                                        (1.5 * np.pi, (-1, 0))])
def test_axis_directions_are_scans(angle, step):
    ncc = blob_map(1, 37, 45)
    mask = oracle.caustic_mask(ncc)
    d, bl = oracle.directional_distance(ncc, 0.25, angle)
    ref, rbl = scan(mask, step)
    assert np.array_equal(bl, rbl)
    assert np.max(np.abs(d - 0.25 * ref)) < 1e-12
    assert np.all(d[mask == 1] == 0)


def march(mask, r, c, ca, sa, ds=1e-4):
    """First s at which the point (c, r) + s (ca, sa) lies inside a caustic
    pixel's square, or the exit from the map (with flag)."""
    ny, nx = mask.shape
    s = ds * np.arange(1, int((nx + ny) / ds) + 2)
    i = np.floor(c + s * ca + 0.5).astype(np.int64)
    j = np.floor(r + s * sa + 0.5).astype(np.int64)
    out = ~((i >= 0) & (i < nx) & (j >= 0) & (j < ny))
    first_out = int(np.argmax(out))
    hit = mask[np.clip(j, 0, ny - 1), np.clip(i, 0, nx - 1)].astype(bool) & ~out
    first_hit = int(np.argmax(hit)) if hit.any() else len(s)
    if first_hit < first_out:
        return s[first_hit], 0
    return s[first_out], 1


@pytest.mark.parametrize("angle", [0.3, 1.1, 2.2, 3.9, 5.5])
def test_oblique_directions_match_a_fine_march(angle):
    ncc = blob_map(2, 29, 33)
    mask = oracle.caustic_mask(ncc)
    d, bl = oracle.directional_distance(ncc, 1.0, angle)
    rng = np.random.default_rng(int(angle * 10))
    ca, sa = np.cos(angle), np.sin(angle)
    for _ in range(60):
        r, c = int(rng.integers(0, 29)), int(rng.integers(0, 33))
        if mask[r, c]:
            assert d[r, c] == 0
            continue
        s, b = march(mask, r, c, ca, sa)
        assert b == bl[r, c]
        assert abs(s - d[r, c]) < 2e-4


def test_quarter_turn_symmetry():
    """Turning the map by a quarter (np.rot90: (x, y) -> (y, nx - 1 - x)) and
    the direction with it gives the turned distances."""
    ncc = blob_map(3, 31, 31)
    for angle in [0.4, 2.0]:
        d, bl = oracle.directional_distance(ncc, 1.0, angle)
        d2, bl2 = oracle.directional_distance(np.rot90(ncc), 1.0, angle - np.pi / 2)
        assert np.array_equal(np.rot90(bl), bl2)
        assert np.max(np.abs(np.rot90(d) - d2)) < 1e-9


def test_no_caustic_gives_exit_distances():
    ncc = np.zeros((10, 14), dtype=np.int32)
    d, bl = oracle.directional_distance(ncc, 2.0, 0.0)
    assert np.all(bl == 1)
    assert np.allclose(d, 2.0 * (14 - 0.5 - np.arange(14))[None, :].repeat(10, 0))


def test_histograms_count_every_pixel_once():
    ncc = blob_map(4, 41, 39)
    d, bl = oracle.directional_distance(ncc, 0.5, 0.8)
    n_bins, d_max = 12, 6.0
    h = oracle.distance_histogram(d, bl, n_bins, d_max)
    assert h.sum() == np.count_nonzero(bl == 0)
    # away from bin edges the bins are numpy's
    edges = np.linspace(0.0, d_max, n_bins + 1)
    sel = (bl == 0) & (d < d_max)
    ref, _ = np.histogram(d[sel], bins=edges)
    assert np.array_equal(h[0, :n_bins], ref)
    assert h[0, n_bins] == np.count_nonzero((bl == 0) & (d >= d_max))
    # per class
    lo, ncls = int(ncc.min()), int(ncc.max() - ncc.min() + 1)
    hc = oracle.distance_histogram(d, bl, n_bins, d_max, ncc=ncc, ncc_lo=lo, n_classes=ncls)
    assert np.array_equal(hc.sum(axis=0), h[0])
    for k in range(ncls):
        assert hc[k].sum() == np.count_nonzero((bl == 0) & (ncc == lo + k))
