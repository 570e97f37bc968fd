"""Parity of the HIP library (through the C ABI) with the CPU oracle.

uint8 data with unit weights must match bit for bit (int32 sums, exact detection
indices, S/N within 1e-12 relative since both sides evaluate (B - M)/S in fp64
from the same integers).  fp32 paths are held to the tolerances derived in the
design notes: all-positive sums within 1e-5 relative of fp64, mixed-sign sums
within 1e-5 of the sum of absolute terms.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check_detect(orc, y64, n, widths, mu, sg, snr, t, W, wmode="unit", w=None):
    M, S = orc.boxcar_norm(n, widths, mu, sg, wmode, w)
    so, to, wo = orc.boxcar_detect(y64, widths, M, S)
    snr, t, W = snr.cpu().numpy(), t.cpu().numpy(), W.cpu().numpy()
    assert np.allclose(snr, so, rtol=1e-12, atol=0)
    mism = np.nonzero((t != to) | (W != wo))[0]
    for d in mism:
        # Accept only a near-tie: the oracle's S/N at the GPU's (t, W) equals its best.
        j = list(widths).index(W[d])
        B = float(np.sum(y64[d, t[d]:t[d] + W[d]]))
        alt = (B - M[d, j]) / S[d, j]
        assert alt == pytest.approx(so[d], rel=1e-12), (d, t[d], W[d], to[d], wo[d])


def test_cfg1_full(dd, orc, otables):
    wl = workloads.cfg1()
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    x = _dev(wl.x)
    y = p.dedisperse(x)
    yo = orc.dedisperse_u8(wl.x, s, n)
    assert np.array_equal(y.cpu().numpy().astype(np.int64), yo)
    snr, t, W = p.search(x, wl.widths, wl.chan_mean, wl.chan_sigma)
    _check_detect(orc, yo.astype(np.float64), n, wl.widths, wl.chan_mean, wl.chan_sigma, snr, t, W)
    snr2, t2, W2 = p.detect(y, wl.widths, wl.chan_mean, wl.chan_sigma)
    assert np.array_equal(snr.cpu().numpy(), snr2.cpu().numpy())
    assert np.array_equal(t.cpu().numpy(), t2.cpu().numpy())
    d = int(np.argmax(snr.cpu().numpy()))
    assert abs(wl.dms[d] - 100.0) <= 10.0


@pytest.mark.parametrize("rule", ["allnonzero", "smear"])
def test_cfg2_reduced_all_outputs(dd, orc, otables, rule):
    # Several DM tiles and a ragged time tail: 96 trials over 4000 + 2246 samples.
    wl = workloads.cfg2(nsamp=6246, ndm=96, rule=rule)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=rule)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule)
    x = _dev(wl.x)
    y = p.dedisperse(x)
    yo = orc.dedisperse_u8(wl.x, s, n)
    assert np.array_equal(y.cpu().numpy().astype(np.int64), yo)
    snr, t, W = p.search(x, wl.widths, wl.chan_mean, wl.chan_sigma)
    _check_detect(orc, yo.astype(np.float64), n, wl.widths, wl.chan_mean, wl.chan_sigma, snr, t, W)


@pytest.fixture(scope="module")
def cfg2_full(dd, orc, otables, opar):
    # Full 336 x 65536 block and all 1024 trials: the oracle's sums of every trial (int64)
    # and its detection of every trial, run over trial ranges in host threads.
    wl = workloads.cfg2()
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    tout = wl.x.shape[1] - p.max_span + 1
    yo = opar.dedisperse_u8(wl.x, s, n, tout)
    y64 = yo.astype(np.float64)
    M, S = orc.boxcar_norm(n, wl.widths, wl.chan_mean, wl.chan_sigma)
    det = opar.detect(y64, wl.widths, M, S)
    return wl, p, n, yo, y64, M, S, det


def _check_detect_all(widths, y64, M, S, det, snr, t, W):
    so, to, wo = det
    snr, t, W = snr.cpu().numpy(), t.cpu().numpy(), W.cpu().numpy()
    assert np.allclose(snr, so, rtol=1e-12, atol=0)
    for d in np.nonzero((t != to) | (W != wo))[0]:
        j = list(widths).index(W[d])
        alt = (float(np.sum(y64[d, t[d]:t[d] + W[d]])) - M[d, j]) / S[d, j]
        assert alt == pytest.approx(so[d], rel=1e-12), (d, t[d], W[d], to[d], wo[d])


# The default shape, every matrix-core shape, and whatever the autotuner picks on this
# box (the launch configuration the benchmark times).
@pytest.mark.parametrize("tile", [-1, 8, 9, 10, 11, 12, "autotuned"])
def test_cfg2_full_size_all_trials(dd, orc, cfg2_full, tile):
    import torch
    wl, p, n, yo, y64, M, S, det = cfg2_full
    x = _dev(wl.x)
    mu = torch.as_tensor(wl.chan_mean, dtype=torch.float64).cuda()
    sg = torch.as_tensor(wl.chan_sigma, dtype=torch.float64).cuda()
    if tile == "autotuned":
        p.autotune(x, wl.widths, mu, sg)
    else:
        p.set_tile(tile)
    snr, t, W = p.search(x, wl.widths, mu, sg)
    if isinstance(tile, int) and tile >= 0:
        assert p.last_search_tile() == tile
    elif tile == "autotuned":
        assert 0 <= p.last_search_tile() <= 12
    _check_detect_all(wl.widths, y64, M, S, det, snr, t, W)
    if tile == -1:
        # the int32 dedispersion of every trial, bit for bit
        y = p.dedisperse(x)
        assert np.array_equal(y.cpu().numpy().astype(np.int64), yo)
        del y
    # The strongest injected pulses are found near their DM.
    sn = snr.cpu().numpy()
    for pl in wl.pulses[:4]:
        d = int(np.argmin(np.abs(wl.dms - pl.dm)))
        lo, hi = max(0, d - 3), min(len(wl.dms), d + 4)
        assert sn[lo:hi].max() > 6.0
    p.set_tile(-1)


def test_cfg3_channel_weights_fp32(dd, orc, otables):
    wl = workloads.cfg3(nsamp=20000, ndm=40)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule, wmode="channel",
                weights=wl.weights)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    y = p.dedisperse(_dev(wl.x)).cpu().numpy()
    yo = orc.dedisperse_f64(wl.x, s, n, "channel", wl.weights)
    rel = np.abs(y - yo) / np.abs(yo)
    assert rel.max() < 1e-5


def test_cfg3_full_size_sampled_points(dd, orc, otables):
    import torch
    wl = workloads.cfg3(nsamp=262144, ndm=4096)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule, wmode="channel",
                weights=wl.weights)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    x = _dev(wl.x)
    y = p.dedisperse(x)
    rng = np.random.default_rng(99)
    nout = y.shape[1]
    dd_ = rng.integers(0, 4096, 64)
    tt = rng.integers(0, nout, 64)
    tt[:2] = [0, nout - 1]
    got = y[torch.as_tensor(dd_).cuda(), torch.as_tensor(tt).cuda()].cpu().numpy()
    ref = orc.dedisperse_points(wl.x, s, n, np.zeros(64), dd_, tt, "channel", wl.weights)
    assert (np.abs(got - ref) / np.abs(ref)).max() < 1e-5


def _r14(got, ref):
    """Largest error of a gradient against its fp64 value, relative to
    max(|ref|, 1e-3 max|ref|): elementwise 1e-5 relative accuracy, with a floor for
    entries that cancel to near zero."""
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float((np.abs(np.asarray(got, dtype=np.float64) - ref) / scale).max())


def _tap_case(B=3, T=3000, D=24, C=40, K=8):
    rng = np.random.default_rng(1234)
    f = workloads.channel_centres(1.2, 0.336 * C / 336, C)
    dms = np.linspace(0, 300, D)
    x = rng.standard_normal((B, C, T)).astype(np.float32)
    w = (1.0 + 0.1 * rng.standard_normal((C, K))).astype(np.float32)
    return f, dms, x, w


def test_tap_weights_forward_and_backward(dd, orc, otables):
    f, dms, x, w = _tap_case()
    B, C, T = x.shape
    K = w.shape[1]
    p = dd.Plan(f, 0.001, 1e-3, dms, rule="fixed", ktaps=K, wmode="tap", weights=w)
    s, n = otables(p, f, 0.001, 1e-3, dms, "fixed", ktaps=K)
    xd = _dev(x)
    y = p.dedisperse(xd).cpu().numpy()
    yo = orc.dedisperse_f64(x, s, n, "tap", w)
    l1 = orc.dedisperse_f64(np.abs(x), s, n, "tap", np.abs(w))
    assert (np.abs(y - yo) / l1).max() < 1e-5
    rng = np.random.default_rng(5)
    g = rng.standard_normal(y.shape).astype(np.float32)
    gx, gw = p.backward(_dev(g), xd)
    gwo = orc.adjoint_w(x, s, n, g.astype(np.float64), "tap", K)
    gxo = orc.adjoint_x(T, s, n, g.astype(np.float64), "tap", w)
    gw = gw.cpu().numpy()
    assert _r14(gw, gwo) < 1e-5
    gxl1 = orc.adjoint_x(T, s, n, np.abs(g).astype(np.float64), "tap", np.abs(w))
    gx = gx.cpu().numpy()
    ok = gxl1 > 0
    assert _r14(gx, gxo) < 1e-5
    assert np.all(gx[~ok] == 0)
    # Sparse path: gradient of sum_e val_e y[b_e, d_e, t_e].
    bb = np.array([0, 1, 2, 2]); d_ = np.array([3, 0, 23, 10]); tt = np.array([5, 100, 0, y.shape[2] - 1])
    val = np.array([1.0, -2.0, 0.5, 3.0], np.float32)
    gs = p.backward_sparse(xd, bb, d_, tt, _dev(val)).cpu().numpy()
    gdense = np.zeros(y.shape)
    np.add.at(gdense, (bb, d_, tt), val.astype(np.float64))
    gso = orc.adjoint_w(x, s, n, gdense, "tap", K)
    assert np.allclose(gs, gso, rtol=1e-12, atol=1e-12)
    got = p.gather(xd, bb, d_, tt).cpu().numpy()
    ref = orc.dedisperse_points(x, s, n, bb, d_, tt, "tap", w)
    assert np.allclose(got, ref, rtol=2e-7, atol=1e-6)


@pytest.mark.parametrize("tile,xdtype,K", [(-1, "f32", 4), (-2, "f32", 4), (-1, "u8", 4),
                                           (-2, "u8", 4), (-1, "f32", 20), (-1, "u8", 37)])
def test_tap_backward_many_channel_groups(dd, orc, otables, tile, xdtype, K):
    """Dense tap-weight adjoint at 300 channels x 80 trials: the tiled transpose gather
    (several trial groups per channel tile, ragged channel and time tiles) and the
    general kernels (tile -2), both against the oracle; 20 and 37 taps take several
    tap slices in the weight gradient, the last one partly filled."""
    B, C, D, T = 2, 300, 80, 6000
    rng = np.random.default_rng(4321)
    f = workloads.channel_centres(1.2, 0.3, C)
    dms = np.linspace(0, 1000, D)
    if xdtype == "u8":
        x = rng.integers(0, 256, size=(B, C, T), dtype=np.uint8)
    else:
        x = rng.standard_normal((B, C, T)).astype(np.float32)
    w = (1.0 + 0.1 * rng.standard_normal((C, K))).astype(np.float32)
    p = dd.Plan(f, 0.001, 1e-3, dms, rule="fixed", ktaps=K, wmode="tap", weights=w)
    p.set_tile(tile)
    s, n = otables(p, f, 0.001, 1e-3, dms, "fixed", ktaps=K)
    assert int(s.max()) > 1000   # delays across a 32-channel tile reach ~150 samples
    nout = p.out_len(T)
    g = rng.standard_normal((B, D, nout)).astype(np.float32)
    gx, gw = p.backward(_dev(g), _dev(x))
    gwo = orc.adjoint_w(x, s, n, g.astype(np.float64), "tap", K)
    gxo = orc.adjoint_x(T, s, n, g.astype(np.float64), "tap", w)
    gw = gw.cpu().numpy()
    assert _r14(gw, gwo) < 1e-5
    gxl1 = orc.adjoint_x(T, s, n, np.abs(g).astype(np.float64), "tap", np.abs(w))
    gx = gx.cpu().numpy()
    ok = gxl1 > 0
    assert _r14(gx, gxo) < 1e-5
    assert np.all(gx[~ok] == 0)
    # the same call again gives the same bits (fixed reduction order)
    gx2, gw2 = p.backward(_dev(g), _dev(x))
    assert np.array_equal(gx2.cpu().numpy(), gx) and np.array_equal(gw2.cpu().numpy(), gw)


def test_u8_dedisperse_batched_unaligned_rows(dd, orc):
    """uint8 -> int32 dedispersion (the matrix-core kernel) of a batch of blocks whose
    rows start at odd byte offsets, with trials out of DM order, a channel that some
    trials skip (ntap 0), ragged trial and time counts; bit-exact against the oracle."""
    rng = np.random.default_rng(2024)
    C, D, B = 37, 50, 2
    f = workloads.channel_centres(1.35, 0.3, C)
    dms = ((np.arange(D) * 37) % D) * 3.0
    s = np.zeros((D, C), np.int32)
    n = np.zeros((D, C), np.int32)
    for d in range(D):
        s[d] = np.floor(4.15 * dms[d] * (1.0 / f ** 2 - 1.0 / f.max() ** 2)).astype(np.int32)
        n[d] = rng.integers(1, 8, size=C)
    n[::3, 5] = 0
    span = int(np.max(s + n))
    T = span + 700
    p = dd.Plan(f, 0.01, 1e-3, dms, rule="explicit", start=s, ntap=n)
    big = rng.integers(0, 256, size=(B, C, T + 3), dtype=np.uint8)
    xd = _dev(big)[:, :, 3:]        # rows start 3 bytes into each padded row
    assert xd.stride(1) == T + 3
    y = p.dedisperse(xd).cpu().numpy()
    x = np.ascontiguousarray(big[:, :, 3:])
    for b in range(B):
        assert np.array_equal(y[b].astype(np.int64), orc.dedisperse_u8(x[b], s, n)), b



@pytest.mark.parametrize("tile", [8, 9])
def test_fused_search_unaligned_rows(dd, orc, tile):
    """Fused search on the matrix cores (windows staged from the converted block) of a
    block whose rows start 3 bytes into rows of odd length, so the conversion takes its
    byte path; trials out of DM order, a channel some trials skip, ragged trial and time
    counts; detection against the oracle."""
    rng = np.random.default_rng(2025)
    C, D = 37, 50
    f = workloads.channel_centres(1.35, 0.3, C)
    dms = ((np.arange(D) * 37) % D) * 3.0
    s = np.zeros((D, C), np.int32)
    n = np.zeros((D, C), np.int32)
    for d in range(D):
        s[d] = np.floor(4.15 * dms[d] * (1.0 / f ** 2 - 1.0 / f.max() ** 2)).astype(np.int32)
        n[d] = rng.integers(1, 8, size=C)
    n[::3, 5] = 0
    span = int(np.max(s + n))
    T = span + 2300
    p = dd.Plan(f, 0.01, 1e-3, dms, rule="explicit", start=s, ntap=n)
    big = rng.integers(0, 256, size=(C, T + 5), dtype=np.uint8)
    xd = _dev(big)[:, 3:]           # rows start 3 bytes into rows of T + 5 bytes
    assert xd.stride(0) == T + 5
    x = np.ascontiguousarray(big[:, 3:])
    yo = orc.dedisperse_u8(x, s, n).astype(np.float64)
    widths = list(range(1, 33))
    mu, sg = np.full(C, 127.5), np.full(C, 73.9)
    p.set_tile(tile)
    snr, t, W = p.search(xd, widths, mu, sg)
    assert p.last_search_tile() == tile
    _check_detect(orc, yo, n, widths, mu, sg, snr, t, W)

def test_edge_cases(dd, orc):
    rng = np.random.default_rng(77)
    # Descending channel order, a channel with ntap = 0, nout = 1 and a single trial.
    C = 5
    f = workloads.channel_centres(1.2, 0.05, C)[::-1].copy()
    s = rng.integers(0, 7, size=(3, C)).astype(np.int32)
    n = rng.integers(0, 4, size=(3, C)).astype(np.int32)
    n[1, 2] = 0
    span = int(np.max(s + n))
    p = dd.Plan(f, 0.01, 1e-3, [0.0, 1.0, 2.0], rule="explicit", start=s, ntap=n)
    for T in (span, span + 1, span + 255, span + 257):
        x = rng.integers(0, 256, size=(C, T), dtype=np.uint8)
        y = p.dedisperse(_dev(x)).cpu().numpy()
        assert np.array_equal(y.astype(np.int64), orc.dedisperse_u8(x, s, n))
        widths = [1] if T - span + 1 < 3 else [1, 2, 3]
        snr, t, W = p.search(_dev(x), widths, np.full(C, 100.0), np.full(C, 10.0))
        yo = orc.dedisperse_u8(x, s, n).astype(np.float64)
        _check_detect(orc, yo, n, widths, np.full(C, 100.0), np.full(C, 10.0), snr, t, W)
    with pytest.raises(dd.DedispError):
        p.dedisperse(_dev(rng.integers(0, 256, size=(C, span - 1), dtype=np.uint8)))
    # A channel no trial uses (no window staged for it) in the fused search.
    n2 = n.copy()
    n2[:, 3] = 0
    p2 = dd.Plan(f, 0.01, 1e-3, [0.0, 1.0, 2.0], rule="explicit", start=s, ntap=n2)
    x = rng.integers(0, 256, size=(C, span + 300), dtype=np.uint8)
    snr, t, W = p2.search(_dev(x), [1, 2, 3], np.full(C, 100.0), np.full(C, 10.0))
    yo = orc.dedisperse_u8(x, s, n2).astype(np.float64)
    _check_detect(orc, yo, n2, [1, 2, 3], np.full(C, 100.0), np.full(C, 10.0), snr, t, W)
    # One channel, one trial: dedispersion and the fused search.
    p1 = dd.Plan([1.4], 0.01, 1e-3, [0.0])
    x = rng.integers(0, 256, size=(1, 33), dtype=np.uint8)
    assert np.array_equal(p1.dedisperse(_dev(x)).cpu().numpy()[0], x[0].astype(np.int32))
    _, n1 = p1.tables()
    snr, t, W = p1.search(_dev(x), [1, 2, 5], np.full(1, 120.0), np.full(1, 30.0))
    _check_detect(orc, x.astype(np.float64), np.asarray(n1), [1, 2, 5], np.full(1, 120.0),
                  np.full(1, 30.0), snr, t, W)


@pytest.mark.parametrize("tile", [-1, 0, 9, -2])
def test_search_zero_noise_deviation(dd, orc, otables, tile):
    # Zero channel means and deviations: a window of zeros has S/N 0 / 0 (NaN, which never
    # wins), any window with signal +inf (ties to the smaller width, then the earlier
    # start); trials whose series is all zeros have no candidate (-inf, -1, 0).
    wl = workloads.cfg2(nsamp=3000, ndm=40)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    p.set_tile(tile)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, "allnonzero")
    # signal only in the last samples of the most delayed channel: only the trials with
    # the largest delays there reach it
    x = np.zeros_like(wl.x)
    x[int(np.argmax(s[-1])), -4:] = 200
    C = x.shape[0]
    mu, sg = np.zeros(C), np.zeros(C)
    snr, t, W = p.search(_dev(x), wl.widths, mu, sg)
    yo = orc.dedisperse_u8(x, s, n).astype(np.float64)
    M, S = orc.boxcar_norm(n, wl.widths, mu, sg)
    so, to, wo = orc.boxcar_detect(yo, wl.widths, M, S)
    assert np.isposinf(so).any() and np.isneginf(so).any()
    assert np.array_equal(snr.cpu().numpy(), so)
    assert np.array_equal(t.cpu().numpy(), to) and np.array_equal(W.cpu().numpy(), wo)


def test_deterministic(dd):
    wl = workloads.cfg2(nsamp=5000, ndm=64)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    x = _dev(wl.x)
    a = p.search(x, wl.widths, wl.chan_mean, wl.chan_sigma)
    b = p.search(x, wl.widths, wl.chan_mean, wl.chan_sigma)
    for u, v in zip(a, b):
        assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())


@pytest.fixture(scope="module")
def cfg2_mid(orc):
    wl = workloads.cfg2(nsamp=9000, ndm=100)
    s = orc.delay_start(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    n = orc.taps_allnonzero(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    yo = orc.dedisperse_u8(wl.x, s, n).astype(np.float64)
    return wl, n, yo


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, -2])
def test_fused_search_every_tile_config(dd, orc, cfg2_mid, tile):
    # Ragged in both DM (100 trials) and time (6755 outputs) for every shape: 0-7 the
    # packed-add kernel, 8-12 the matrix-core kernel, -2 the unfused path.
    wl, n, yo = cfg2_mid
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    p.set_tile(tile)
    snr, t, W = p.search(_dev(wl.x), wl.widths, wl.chan_mean, wl.chan_sigma)
    assert p.last_search_tile() == (tile if tile >= 0 else -1)
    _check_detect(orc, yo, n, wl.widths, wl.chan_mean, wl.chan_sigma, snr, t, W)


@pytest.fixture(scope="module")
def cfg2_dense(orc):
    wl = workloads.cfg2(nsamp=9000, ndm=300)
    s = orc.delay_start(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    n = orc.taps_allnonzero(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    yo = orc.dedisperse_u8(wl.x, s, n).astype(np.float64)
    return wl, n, yo


@pytest.mark.parametrize("tile", [8, 9, 10, 11, 12])
def test_matrix_core_search_shapes(dd, orc, cfg2_dense, tile):
    # 300 trials: three DM tiles of 128 (or five of 64) trials with a ragged last tile,
    # ragged time.
    wl, n, yo = cfg2_dense
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    p.set_tile(tile)
    snr, t, W = p.search(_dev(wl.x), wl.widths, wl.chan_mean, wl.chan_sigma)
    assert p.last_search_tile() == tile
    _check_detect(orc, yo, n, wl.widths, wl.chan_mean, wl.chan_sigma, snr, t, W)


@pytest.mark.parametrize("tile", [8, 9, 10, 11, 12])
def test_matrix_core_short_series_odd_trials(dd, orc, otables, tile):
    # 37 trials (no DM tile full) and 100 outputs (one partial time tile): every
    # matrix-core shape, the fused search and the int32 dedispersion.
    wl = workloads.cfg2(nsamp=3000, ndm=37)
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, "allnonzero")
    T = p.max_span + 99
    x = np.ascontiguousarray(wl.x[:, :T])
    p.set_tile(tile)
    yo = orc.dedisperse_u8(x, s, n)
    y = p.dedisperse(_dev(x)).cpu().numpy()
    assert np.array_equal(y.astype(np.int64), yo)
    snr, t, W = p.search(_dev(x), wl.widths, wl.chan_mean, wl.chan_sigma)
    assert p.last_search_tile() == tile
    _check_detect(orc, yo.astype(np.float64), n, wl.widths, wl.chan_mean, wl.chan_sigma, snr, t, W)


def test_default_search_runs_on_the_matrix_cores(dd, orc, cfg2_mid):
    wl, n, yo = cfg2_mid
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    snr, t, W = p.search(_dev(wl.x), wl.widths, wl.chan_mean, wl.chan_sigma)
    assert p.last_search_tile() == 9     # two workgroups per CU, the untuned default
    _check_detect(orc, yo, n, wl.widths, wl.chan_mean, wl.chan_sigma, snr, t, W)


def test_fused_search_sparse_widths(dd, orc, cfg2_mid):
    wl, n, yo = cfg2_mid
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    widths = [3, 32, 7]
    snr, t, W = p.search(_dev(wl.x), widths, wl.chan_mean, wl.chan_sigma)
    assert p.last_search_tile() >= 0
    _check_detect(orc, yo, n, sorted(widths), wl.chan_mean, wl.chan_sigma, snr, t, W)


@pytest.mark.parametrize("ntap,fused", [(80, True), (90, False)])
def test_extreme_samples_near_int32_limits(dd, orc, opar, ntap, fused):
    # Saturated and alternating-extreme uint8 blocks on a plan whose sums come close to
    # the int32 limits the fused search accepts (255 * sum_c ntap * 49 < 2^30): 1024
    # channels of 80 samples (fused search, both int8 extremes through the x - 128
    # correction) and of 90 samples (beyond the fused search's limit: the unfused path),
    # against the oracle bit for bit.
    rng = np.random.default_rng(5150 + ntap)
    C, D = 1024, 64
    f = workloads.channel_centres(1.2, 0.3, C)
    s = np.sort(rng.integers(0, 40, size=(D, C)), axis=0).astype(np.int32)
    n = np.full((D, C), ntap, dtype=np.int32)
    p = dd.Plan(f, 0.3 / C, 1e-3, np.arange(D, dtype=np.float64), rule="explicit", start=s,
                ntap=n)
    span = int(np.max(s + n))
    T = span + 600
    widths = list(range(1, 33))
    mu, sg = np.full(C, 127.5), np.full(C, 40.0)
    blocks = [np.full((C, T), 255, np.uint8), np.zeros((C, T), np.uint8),
              np.where(rng.random((C, T)) < 0.5, 0, 255).astype(np.uint8)]
    for x in blocks:
        xd = _dev(x)
        yo = opar.dedisperse_u8(x, s, n, tout=T - span + 1)
        assert np.array_equal(p.dedisperse(xd).cpu().numpy().astype(np.int64), yo)
        snr, t, W = p.search(xd, widths, mu, sg)
        assert (p.last_search_tile() >= 0) == fused
        _check_detect(orc, yo.astype(np.float64), n, widths, mu, sg, snr, t, W)


@pytest.mark.parametrize("wmode,widths", [("unit", [1, 2, 7, 63]), ("unit", [1, 5, 64, 100, 250]),
                                          ("channel", list(range(1, 33))),
                                          ("tap", [1, 3, 8, 17])])
def test_detect_noise_tables_every_weight_mode(dd, orc, wmode, widths):
    # Detection of a given dedispersed series under every weight mode and width range
    # (the noise tables by tap-count buckets for unit and channel weights up to width 63,
    # the general ones for tap weights and wider boxcars): the GPU's series is handed to
    # the oracle's detector with the oracle's noise tables.
    rng = np.random.default_rng(909)
    C, D, T = 48, 24, 1500
    f = workloads.channel_centres(1.2, 0.048, C)
    dms = np.linspace(0.0, 300.0, D)
    w = None
    if wmode == "tap":
        K = 4
        w = (1.0 + 0.2 * rng.standard_normal((C, K))).astype(np.float32)
        p = dd.Plan(f, 0.001, 1e-3, dms, rule="fixed", ktaps=K, wmode="tap", weights=w)
    elif wmode == "channel":
        w = ((f / 1.2) ** -1.5).astype(np.float32)
        p = dd.Plan(f, 0.001, 1e-3, dms, rule="smear", wmode="channel", weights=w)
    else:
        p = dd.Plan(f, 0.001, 1e-3, dms, rule="allnonzero")
    s, n = p.tables()
    x = rng.integers(0, 256, size=(C, T), dtype=np.uint8)
    y = p.dedisperse(_dev(x))
    mu = 100.0 + 10.0 * rng.random(C)
    sg = 10.0 + 5.0 * rng.random(C)
    snr, t, W = p.detect(y, widths, mu, sg)
    y64 = y.cpu().numpy().astype(np.float64)
    M, S = orc.boxcar_norm(n, widths, mu, sg, wmode, w)
    so, to, wo = orc.boxcar_detect(y64, widths, M, S)
    snr, t, W = snr.cpu().numpy(), t.cpu().numpy(), W.cpu().numpy()
    assert np.allclose(snr, so, rtol=1e-9, atol=0)
    for d in np.nonzero((t != to) | (W != wo))[0]:
        j = list(widths).index(int(W[d]))
        B = float(np.sum(y64[d, t[d]:t[d] + W[d]]))
        assert (B - M[d, j]) / S[d, j] == pytest.approx(so[d], rel=1e-9)
