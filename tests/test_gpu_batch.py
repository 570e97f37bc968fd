"""Batched search over many beams (own DM grids from the trial-DM rule,
uneven lengths), eager and replayed from a HIP graph, checked against the oracle;
and the tile autotuner."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

EPS_08 = math.sqrt(0.8 ** -4 - 1.0)   # (eps^2 + 1)^(-1/4) = 0.8


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def dd():
    import paper_1301_3968_amd as dd
    return dd


@pytest.fixture(scope="module")
def beams(dd, orc, otables):
    rng = np.random.default_rng(4242)
    C = 96
    f = workloads.channel_centres(1.2, 0.336 * C / 336, C)
    out = []
    for b in range(5):
        T = int(rng.integers(3000, 9000))
        ntr = int(rng.integers(20, 70))
        dms = orc.trial_dms(0.0, 1e9, EPS_08 / 2, f, 0.001, 1e-3, cap=ntr)
        np.testing.assert_allclose(dd.trial_dms(0.0, 1e9, EPS_08 / 2, f, 0.001, 1e-3, cap=ntr),
                                   dms, rtol=1e-12)
        x = workloads.u8_noise(rng, C, T)
        p = dd.Plan(f, 0.001, 1e-3, dms, rule="allnonzero")
        s, n = otables(p, f, 0.001, 1e-3, dms, "allnonzero")
        yo = orc.dedisperse_u8(x, s, n).astype(np.float64)
        out.append((p, x, n, yo))
    return C, out


def _oracle_detect(orc, n, yo, widths, C):
    M, S = orc.boxcar_norm(n, widths, np.full(C, 128.0), np.full(C, 16.0))
    return orc.boxcar_detect(yo, widths, M, S), M, S


def _check(orc, beams_, widths, snr, t, W):
    C, bl = beams_
    off = 0
    for p, x, n, yo in bl:
        (so, to, wo), M, S = _oracle_detect(orc, n, yo, widths, C)
        D = len(so)
        s_, t_, w_ = snr[off:off + D], t[off:off + D], W[off:off + D]
        assert np.allclose(s_, so, rtol=1e-12, atol=0)
        for d in np.nonzero((t_ != to) | (w_ != wo))[0]:
            j = list(widths).index(w_[d])
            B = float(np.sum(yo[d, t_[d]:t_[d] + w_[d]]))
            assert (B - M[d, j]) / S[d, j] == pytest.approx(so[d], rel=1e-12)
        off += D


@pytest.mark.parametrize("kernel", ["matrix", "matrix-grid", "packed"])
def test_batch_eager_and_graph_replays(dd, orc, beams, kernel, monkeypatch):
    import torch
    C, bl = beams
    widths = list(range(1, 33))
    # the batch takes the matrix-core kernel unless the first plan forces a packed-add shape;
    # the matrix-core batch runs as a persistent launch unless one workgroup per tile is asked
    if kernel == "packed":
        bl[0][0].set_tile(4)
    if kernel == "matrix-grid":
        monkeypatch.setenv("DEDISP_BATCH_LAUNCH", "grid")
    try:
        B = dd.Batch([b[0] for b in bl], [b[1].shape[1] for b in bl], widths)
    finally:
        bl[0][0].set_tile(-1)
    assert B.total_trials == sum(b[0].ndm for b in bl)
    xs = [_dev(b[1]) for b in bl]
    mu = torch.full((C,), 128.0, dtype=torch.float64, device="cuda")
    sg = torch.full((C,), 16.0, dtype=torch.float64, device="cuda")
    eager = [v.cpu().numpy() for v in B.run(xs, mu, sg)]
    _check(orc, beams, widths, *eager)
    work = torch.empty(B.work_bytes, dtype=torch.uint8, device="cuda")
    outs = (torch.empty(B.total_trials, dtype=torch.float64, device="cuda"),
            torch.empty(B.total_trials, dtype=torch.int32, device="cuda"),
            torch.empty(B.total_trials, dtype=torch.int32, device="cuda"))
    for rep in range(3):
        for o in outs:
            o.fill_(-7)
        B.run(xs, mu, sg, work=work, outputs=outs, graph=True)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        for g, e in zip(got, eager):
            assert np.array_equal(g, e), rep
        # unrelated eager work between replays
        bl[0][0].search(xs[0], [1, 2, 4], mu, sg)
        torch.cuda.synchronize()


def test_batch_matches_single_plan_search(dd, beams):
    import torch
    C, bl = beams
    widths = [1, 3, 9, 27]
    B = dd.Batch([b[0] for b in bl], [b[1].shape[1] for b in bl], widths)
    xs = [_dev(b[1]) for b in bl]
    mu = torch.full((C,), 128.0, dtype=torch.float64, device="cuda")
    sg = torch.full((C,), 16.0, dtype=torch.float64, device="cuda")
    snr, t, W = [v.cpu().numpy() for v in B.run(xs, mu, sg)]
    off = 0
    for (p, x, n, yo), xd in zip(bl, xs):
        s1, t1, w1 = [v.cpu().numpy() for v in p.search(xd, widths, mu, sg)]
        D = p.ndm
        assert np.array_equal(s1, snr[off:off + D])
        assert np.array_equal(t1, t[off:off + D])
        assert np.array_equal(w1, W[off:off + D])
        off += D


def test_autotune_picks_a_working_shape(dd, orc, beams, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("DEDISP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    C, bl = beams
    p, x, n, yo = bl[0]
    xd = _dev(x)
    mu = torch.full((C,), 128.0, dtype=torch.float64, device="cuda")
    sg = torch.full((C,), 16.0, dtype=torch.float64, device="cuda")
    ref = [v.cpu().numpy() for v in p.search(xd, list(range(1, 33)), mu, sg)]
    ci = p.autotune(xd, list(range(1, 33)), mu, sg)
    assert 0 <= ci
    got = [v.cpu().numpy() for v in p.search(xd, list(range(1, 33)), mu, sg)]
    assert p.last_search_tile() == ci
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    # the second call is answered from the cache file
    assert (tmp_path / "tune.txt").read_text().count("\n") == 1
    assert p.autotune(xd, list(range(1, 33)), mu, sg) == ci
    assert (tmp_path / "tune.txt").read_text().count("\n") == 1
    p.set_tile(-1)


@pytest.mark.parametrize("kernel", ["matrix", "packed"])
def test_eager_call_between_graph_replays(dd, orc, beams, kernel):
    # A graph captured on inputs A, an eager call on other inputs B (own workspace and
    # outputs), then a replay of the graph after new data were written into A's
    # buffers: the replay must search A's new data, not B's, and the eager call B's.
    import torch
    C, bl = beams
    widths = list(range(1, 33))
    if kernel == "packed":
        bl[0][0].set_tile(4)
    try:
        B = dd.Batch([b[0] for b in bl], [b[1].shape[1] for b in bl], widths)
    finally:
        bl[0][0].set_tile(-1)
    rng = np.random.default_rng(777)
    data_b = [workloads.u8_noise(rng, C, b[1].shape[1]) for b in bl]
    data_a2 = [workloads.u8_noise(rng, C, b[1].shape[1]) for b in bl]
    xs_a = [_dev(b[1]) for b in bl]
    xs_b = [_dev(x) for x in data_b]
    mu = torch.full((C,), 128.0, dtype=torch.float64, device="cuda")
    sg = torch.full((C,), 16.0, dtype=torch.float64, device="cuda")
    work = torch.empty(B.work_bytes, dtype=torch.uint8, device="cuda")
    outs = (torch.empty(B.total_trials, dtype=torch.float64, device="cuda"),
            torch.empty(B.total_trials, dtype=torch.int32, device="cuda"),
            torch.empty(B.total_trials, dtype=torch.int32, device="cuda"))
    B.run(xs_a, mu, sg, work=work, outputs=outs, graph=True)
    torch.cuda.synchronize()
    _check(orc, beams, widths, *[o.cpu().numpy() for o in outs])
    eager_b = [v.cpu().numpy() for v in B.run(xs_b, mu, sg)]
    for xa, new in zip(xs_a, data_a2):
        xa.copy_(_dev(new))
    for o in outs:
        o.fill_(-7)
    B.run(xs_a, mu, sg, work=work, outputs=outs, graph=True)
    torch.cuda.synchronize()
    replay = [o.cpu().numpy() for o in outs]

    def with_data(data):
        out = []
        for (p, x, n, yo), xn in zip(bl, data):
            out.append((p, xn, n, orc.dedisperse_u8(xn, *_oracle_tables_of(orc, p, n)).astype(np.float64)))
        return C, out

    _check(orc, with_data(data_b), widths, *eager_b)
    _check(orc, with_data(data_a2), widths, *replay)


def _oracle_tables_of(orc, p, n):
    """The oracle's start table for plan p's trial DMs (the tap counts n are the
    oracle's already) and n."""
    s = orc.delay_start(p._freq, 0.001, 1e-3, p._dms).astype(np.int32)
    return s, n
