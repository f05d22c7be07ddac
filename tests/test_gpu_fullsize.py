"""Parity at the full workload sizes, in the launch configuration the
benchmark times (library-chosen subchains, fused caustics, per-launch event
timing), with direct and with fast-multipole star sums (Sec. 4.1).  The
oracle, which always sums every star directly, cannot redo whole runs of this size, so it checks
sampled rows (cold-started on their own), a window of subchain 0 grown
centre-out as the GPU grows it (the same columns once the two centre
rows are paired), and properties that
hold at any size: the row identities sum r = 2 sum z_i and
sum r^2 = 2 sum z_i^2 - 2M/c(phi), the closure row m = row 0 under
chain_next, the label of every column across every subchain boundary, and
the whole crossing and distance maps of the GPU's own caustic vertices,
pixel for pixel, against the oracle's edge-by-edge map and its exact
two-pass distance transform."""
import numpy as np
import pytest

import oracle
from paper_2506_02121_amd import fields
from tests import parity

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


def host_c(re, im):
    return re.cpu().numpy() + 1j * im.cpu().numpy()


def row_identities(f, rr, ri, m_steps, n_r):
    """Largest deviation of the two row identities over every row, relative
    to the scale of each sum (computed on the device in float64)."""
    dev = rr.device
    z = torch.complex(rr.view(m_steps + 1, n_r), ri.view(m_steps + 1, n_r))
    zs = f.x + 1j * f.y
    phi = 2 * np.pi * np.arange(m_steps + 1) / m_steps
    c = f.gamma - (1 - f.kappa_s) * np.exp(-1j * phi)
    want1 = 2 * zs.sum()
    want2 = torch.as_tensor(2 * (zs ** 2).sum() - 2 * f.m.sum() / c, device=dev)
    s1 = z.sum(dim=1)
    s2 = (z * z).sum(dim=1)
    scale2 = (z.abs() ** 2).sum(dim=1)
    e1 = float(((s1 - want1).abs() / n_r).max())
    e2 = float(((s2 - want2).abs() / scale2).max())
    return e1, e2


def check_sampled_rows(f, R_rows, W_rows, rows, m_steps, label):
    worst = wworst = 0.0
    for j, Rg, Wg in zip(rows, R_rows, W_rows):
        phi = oracle.phase(j, m_steps)
        z_ref, _, _, rc = oracle.aberth_row(f, phi)
        Fp = oracle.eval_F(f, phi, z_ref)[1]
        bound = parity.root_bound(f, Fp)
        idx, d = parity.pair(z_ref, Rg)
        assert np.all(d <= bound), (label, j, float((d / bound).max()))
        w_ref = oracle.lens_map(f, z_ref)
        bw = 2 * abs(1 - f.kappa_s) * bound + 1e-11 * (1 + np.abs(w_ref))
        assert np.all(np.abs(Wg[idx] - w_ref) <= bw), (label, j)
        worst = max(worst, float(d.max()))
        wworst = max(wworst, float(np.abs(Wg[idx] - w_ref).max()))
    print(f"[{label}] sampled rows {list(rows)}: max root distance {worst:.3e}, "
          f"max caustic distance {wworst:.3e}", flush=True)


def boundary_continuity(rr, ri, m_steps, S):
    """Across every subchain boundary row b (computed by two subchains and
    joined by relabelling) and at the closure, each root of row b+1 must have
    its own column's root of row b as nearest neighbour, and row b-1 likewise:
    a wrong relabelling breaks whole columns.  Returns the worst fraction of
    columns that keep their label."""
    L = m_steps // S
    worst = 1.0
    for b in range(L, m_steps, L):
        rb = host_c(rr[b], ri[b])
        for j in (b - 1, b + 1):
            idx, _ = parity.pair(host_c(rr[j], ri[j]), rb)
            worst = min(worst, float(np.mean(idx == np.arange(len(idx)))))
    return worst


def subchain0_window(st, m_steps, half):
    S = st["n_subchains"]
    L = m_steps // S
    c = L // 2
    return c - half, c, c + half


FULL = [
    # workload, precision (None: the workload's), sampled rows, half-width of the
    # subchain-0 window, whole crossing and distance maps, star sums
    ("n1k", None, 6, 40, True, "direct"),
    ("n10k", None, 2, 4, True, "direct"),
    ("n10k", "fp64_r32", 2, 4, False, "direct"),
    ("n10k_mixed", None, 2, 4, False, "direct"),
    ("n10k", None, 2, 4, False, "fmm"),
    ("n10k_mixed", None, 2, 4, False, "fmm"),
]


def case_id(c):
    return c[0] + ("_" + c[1] if c[1] else "") + ("_fmm" if c[5] == "fmm" else "")


def check_whole_maps(ctx, mlcc, wl, cr, ci, cnh, m_steps, n_r, name):
    """The crossing map of the GPU's caustics against the oracle's, every
    pixel, and the distance map of that N_cc map against the oracle's exact
    transform: squared pixel distances and border marks bit for bit."""
    grid = mlcc.as_grid(wl.grid)
    ncc_d = ctx.caustic_crossings(cr, ci, torch.as_tensor(cnh, device=cr.device), grid)
    dist_d, bl_d = ctx.caustic_distances(grid, ncc_d)
    torch.cuda.synchronize()
    ncc = ncc_d.cpu().numpy()
    wr = cr.view(m_steps + 1, n_r).cpu().numpy()
    wi = ci.view(m_steps + 1, n_r).cpu().numpy()
    ref = oracle.ncc_rows((wr, wi), cnh, grid)
    del wr, wi
    bad = int(np.count_nonzero(ncc != ref))
    print(f"[{name}] N_cc map {grid.nx}x{grid.ny}: {bad} pixels differ from the oracle "
          f"(max {int(ncc.max())}, {int(np.count_nonzero(ncc))} pixels inside caustics)",
          flush=True)
    assert bad == 0
    h = 2.0 * grid.half_width / grid.nx
    _, bl_ref, d2_ref = oracle.edt_twopass(ref, h)
    dist = dist_d.cpu().numpy()
    fin = np.isfinite(dist)
    assert np.array_equal(fin, d2_ref >= 0)
    d2 = np.full(dist.shape, -1, dtype=np.int64)
    d2[fin] = np.rint((dist[fin] / h) ** 2).astype(np.int64)
    assert np.array_equal(d2, d2_ref)
    assert np.array_equal(dist[fin], np.sqrt(d2_ref[fin].astype(np.float64)) * h)
    assert np.array_equal(bl_d.cpu().numpy(), bl_ref)
    print(f"[{name}] distance map: d^2 and border marks equal the oracle's on every pixel "
          f"(max distance {float(dist[fin].max()):.4f})", flush=True)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case", FULL, ids=[case_id(c) for c in FULL])
def test_full_size_single_field(mlcc, case):
    wl_name, prec, n_rows, half, maps, star_sums = case
    name = case_id(case)
    say("full size", name)
    wl = fields.workload(wl_name)
    f, m_steps = wl.field, wl.m_steps
    n_r = 2 * f.n
    ctx = mlcc.Context(0)
    try:
        dev = torch.device("cuda", 0)
        ctx.set_lenses(torch.as_tensor(f.x, device=dev), torch.as_tensor(f.y, device=dev),
                       torch.as_tensor(f.m, device=dev), f.kappa_s, f.gamma)
        rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(
            m_steps, timing=True, caustics=True, precision=prec or wl.precision,
            star_sums=star_sums)
        torch.cuda.synchronize()
        print("[stats]", {k: st[k] for k in ("n_subchains", "sweeps", "root_updates",
                                             "root_updates_f32", "rows_fallback",
                                             "match_maxdist")}, flush=True)
        # closure and the row identities, every row
        cnh = cn.cpu().numpy()
        assert sorted(cnh.tolist()) == list(range(n_r))
        last = host_c(rr[m_steps], ri[m_steps])
        first = host_c(rr[0], ri[0])
        assert np.max(np.abs(last - first[cnh])) < 1e-8
        e1, e2 = row_identities(f, rr, ri, m_steps, n_r)
        print(f"[{name}] row identities: {e1:.2e} (sum r, per root), {e2:.2e} (sum r^2, relative)",
              flush=True)
        assert e1 < 1e-9 and e2 < 1e-9
        keep = boundary_continuity(rr, ri, m_steps, st["n_subchains"])
        print(f"[{name}] columns keeping their label across subchain boundaries: {keep:.5f}",
              flush=True)
        assert keep == 1.0
        # sampled rows against cold-started oracle rows
        rng = np.random.default_rng(12345)
        rows = sorted(set([0, m_steps // 2, m_steps] +
                          rng.integers(1, m_steps, size=max(0, n_rows - 3)).tolist()))
        R_rows = [host_c(rr[j], ri[j]) for j in rows]
        W_rows = [host_c(cr[j], ci[j]) for j in rows]
        check_sampled_rows(f, R_rows, W_rows, rows, m_steps, name)
        # subchain 0 grown from its centre: which seed ends at which root of
        # the cold-started centre row is chaotic at this N (any rounding
        # difference reorders it), so the oracle's centre row is paired with
        # the GPU's; from there the warm-started rows must follow the same
        # columns
        lo, c, hi = subchain0_window(st, m_steps, half)
        if wl_name == "n1k":
            # grow the oracle's window on through the first boundary row, where
            # the GPU's columns continue only through the relabelling
            hi = m_steps // st["n_subchains"] + half
        R_win, _ = oracle.subchain(f, m_steps, lo, c, hi)
        G_win = host_c(rr[lo:hi + 1], ri[lo:hi + 1])
        idx, d = parity.pair(R_win[c - lo], G_win[c - lo])
        assert len(set(idx.tolist())) == n_r and d.max() < 1e-8
        colwise = float(np.max(np.abs(G_win[:, idx] - R_win)))
        print(f"[{name}] rows {lo}..{hi} of subchain 0, column-wise: {colwise:.3e}", flush=True)
        assert colwise < 1e-8
        if maps:
            check_whole_maps(ctx, mlcc, wl, cr, ci, cnh, m_steps, n_r, name)
    finally:
        ctx.close()
        torch.cuda.empty_cache()


@pytest.mark.timeout(900)
def test_full_size_batched(mlcc):
    """256 fields of uneven N in one call (mixed precision): every field's
    closure and row identities, the smallest fields against the whole oracle
    chain, and sampled rows of the largest field."""
    say("full size batched")
    wl = fields.workload("batched")
    fs, m_steps = wl.fields, wl.m_steps
    dev = torch.device("cuda", 0)
    off = np.concatenate([[0], np.cumsum([f.n for f in fs])]).astype(np.int64)
    ctx = mlcc.Context(0)
    try:
        ctx.set_lenses_batched(off, torch.as_tensor(np.concatenate([f.x for f in fs]), device=dev),
                               torch.as_tensor(np.concatenate([f.y for f in fs]), device=dev),
                               torch.as_tensor(np.concatenate([f.m for f in fs]), device=dev),
                               [f.kappa_s for f in fs], [f.gamma for f in fs])
        rr, ri, cr, ci, cn, st, code = ctx.find_critical_curves(
            m_steps, timing=True, caustics=True, precision=wl.precision)
        torch.cuda.synchronize()
        print("[stats]", {k: st[k] for k in ("n_subchains", "sweeps", "root_updates",
                                             "root_updates_f32", "rows_fallback")}, flush=True)
        blocks = ctx.field_blocks(m_steps)
        cnh = cn.cpu().numpy()
        worst1 = worst2 = 0.0
        for f, (o, co, n_r) in zip(fs, blocks):
            fr = rr[o:o + (m_steps + 1) * n_r]
            fi = ri[o:o + (m_steps + 1) * n_r]
            c_f = cnh[co:co + n_r]
            assert sorted(c_f.tolist()) == list(range(n_r))
            last = host_c(fr[m_steps * n_r:], fi[m_steps * n_r:])
            first = host_c(fr[:n_r], fi[:n_r])
            assert np.max(np.abs(last - first[c_f])) < 1e-8
            e1, e2 = row_identities(f, fr, fi, m_steps, n_r)
            worst1, worst2 = max(worst1, e1), max(worst2, e2)
        print(f"[batched] row identities over all fields: {worst1:.2e}, {worst2:.2e}", flush=True)
        assert worst1 < 1e-9 and worst2 < 1e-9
        order = np.argsort([f.n for f in fs])
        keep = 1.0
        for i in order[-4:]:
            o, co, n_r = blocks[i]
            fr = rr[o:o + (m_steps + 1) * n_r].view(m_steps + 1, n_r)
            fi = ri[o:o + (m_steps + 1) * n_r].view(m_steps + 1, n_r)
            keep = min(keep, boundary_continuity(fr, fi, m_steps, st["n_subchains"]))
        print(f"[batched] columns keeping their label across boundaries (4 largest fields): "
              f"{keep:.5f}", flush=True)
        assert keep == 1.0
        # the three smallest fields: the whole chain against the oracle
        for i in order[:3]:
            f = fs[i]
            o, co, n_r = blocks[i]
            R = host_c(rr[o:o + (m_steps + 1) * n_r], ri[o:o + (m_steps + 1) * n_r])
            R = R.reshape(m_steps + 1, n_r)
            R_ref, _, _ = oracle.critical_curves(f, m_steps, n_sub=1)
            Fp = np.stack([oracle.eval_F(f, oracle.phase(j, m_steps), R_ref[j])[1]
                           for j in range(m_steps + 1)])
            worst, ratio = parity.compare_row_sets(R, R_ref, parity.root_bound(f, Fp))
            print(f"[batched field {i}, N={f.n}] max root distance {worst:.3e} "
                  f"(ratio {ratio:.3f})", flush=True)
            assert ratio <= 1.0
        # the largest field: sampled rows
        i = order[-1]
        f = fs[i]
        o, co, n_r = blocks[i]
        rows = [0, 1234, m_steps // 2, m_steps]
        R_rows = [host_c(rr[o + j * n_r:o + (j + 1) * n_r], ri[o + j * n_r:o + (j + 1) * n_r])
                  for j in rows]
        W_rows = [host_c(cr[o + j * n_r:o + (j + 1) * n_r], ci[o + j * n_r:o + (j + 1) * n_r])
                  for j in rows]
        check_sampled_rows(f, R_rows, W_rows, rows, m_steps, f"batched field {i}, N={f.n}")
    finally:
        ctx.close()
        torch.cuda.empty_cache()
