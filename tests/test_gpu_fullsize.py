"""Parity at the full sizes of the two training / serving patterns:

* the 36-beam batch (336 channels, 16384-131072 samples, 300-1200 trials per beam
  from the trial-DM rule of Section 5.3), eager and replayed from a HIP graph, with
  sampled trials of every beam (first, last, both sides of DM-tile boundaries and
  random ones) against the oracle's full-row detection;
* the 64-pulse, 336-channel, 32768-sample batch with 8 learnable taps per channel
  and 256 trials: the sparse weight adjoint of every weight against the oracle's
  per-pulse transpose, the matched-filter loss gradient against the oracle's fp64
  gradient and against 32 central differences of the oracle's loss (h = 1e-3), and
  the dense adjoint of a random output gradient at sampled channels (every tap).
"""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

EPS_08 = math.sqrt(0.8 ** -4 - 1.0)   # (eps^2 + 1)^(-1/4) = 0.8; grids spaced eps/2


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _r14(got, ref):
    """Largest gradient error relative to max(|ref|, 1e-3 max|ref|)."""
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float((np.abs(np.asarray(got, dtype=np.float64) - ref) / scale).max())


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


# ------------------------------------------------------------------ 36-beam batch

@pytest.fixture(scope="module")
def beams36(dd, orc, otables, opar):
    spec = workloads.cfg4_beams()
    C = 336
    f = workloads.channel_centres(1.2, 0.336, C)
    plans, data, picks, ref = [], [], [], []
    rng = np.random.default_rng(1301)
    for b in range(len(spec["nsamp"])):
        ntr = int(spec["ntrial"][b])
        dms = orc.trial_dms(0.0, 1e9, EPS_08 / 2, f, 0.001, 1e-3, cap=ntr)
        assert len(dms) == ntr
        np.testing.assert_allclose(dd.trial_dms(0.0, 1e9, EPS_08 / 2, f, 0.001, 1e-3, cap=ntr),
                                   dms, rtol=1e-12)
        x, _ = workloads.cfg4_beam_data(b, int(spec["nsamp"][b]), float(dms[0]), float(dms[-1]))
        p = dd.Plan(f, 0.001, 1e-3, dms, rule="allnonzero")
        s, n = otables(p, f, 0.001, 1e-3, dms, "allnonzero")
        # first and last trial, both sides of the 16- and 64-trial tile boundaries, random
        pk = {0, 15, 16, 63, 64, ntr - 1, ntr - 2} | set(int(v) for v in rng.integers(0, ntr, 3))
        pk = np.array(sorted(v for v in pk if 0 <= v < ntr))
        plans.append(p)
        data.append(x)
        picks.append(pk)
        ref.append((s[pk], n[pk], x.shape[1] - p.max_span + 1))
    widths = list(range(1, 33))
    mu, sg = np.full(C, 128.0), np.full(C, 16.0)

    def one(i):
        s, n, tout = ref[i]
        y = orc.dedisperse_u8(data[i], s, n, tout=tout).astype(np.float64)
        M, S = orc.boxcar_norm(n, widths, mu, sg)
        return y, M, S, orc.boxcar_detect(y, widths, M, S)

    oracle = opar.map(one, range(len(plans)))
    return C, plans, data, picks, oracle, widths


def _check_beams(plans, picks, oracle, widths, snr, t, W):
    off = 0
    for p, pk, (y, M, S, (so, to, wo)) in zip(plans, picks, oracle):
        s_, t_, w_ = snr[off + pk], t[off + pk], W[off + pk]
        assert np.allclose(s_, so, rtol=1e-12, atol=0)
        for i in np.nonzero((t_ != to) | (w_ != wo))[0]:
            j = widths.index(int(w_[i]))
            B = float(np.sum(y[i, t_[i]:t_[i] + w_[i]]))
            assert (B - M[i, j]) / S[i, j] == pytest.approx(so[i], rel=1e-12)
        off += p.ndm


def test_batch_36_beams_full_shape(dd, beams36):
    import torch
    C, plans, data, picks, oracle, widths = beams36
    B = dd.Batch(plans, [x.shape[1] for x in data], widths)
    assert B.total_trials == sum(p.ndm for p in plans)
    xs = [_dev(x) for x in data]
    mu = torch.full((C,), 128.0, dtype=torch.float64, device="cuda")
    sg = torch.full((C,), 16.0, dtype=torch.float64, device="cuda")
    eager = [v.cpu().numpy() for v in B.run(xs, mu, sg)]
    _check_beams(plans, picks, oracle, widths, *eager)
    work = torch.empty(B.work_bytes, dtype=torch.uint8, device="cuda")
    outs = tuple(torch.empty(B.total_trials, dtype=dt, device="cuda")
                 for dt in (torch.float64, torch.int32, torch.int32))
    for rep in range(2):
        for o in outs:
            o.fill_(-7)
        B.run(xs, mu, sg, work=work, outputs=outs, graph=True)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        for g, e in zip(got, eager):
            assert np.array_equal(g, e), rep


# --------------------------------------------------------- 64-pulse learnable profile

@pytest.fixture(scope="module")
def cfg5_full(dd, otables):
    import torch
    wl = workloads.cfg5()
    K = wl.extra["ktaps"]
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="fixed", ktaps=K, wmode="tap",
                weights=wl.weights)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, "fixed", ktaps=K)
    nout = p.out_len(wl.x.shape[2])
    b = np.arange(len(wl.pulses))
    d = np.array([q[1] for q in wl.pulses])
    t = np.array([min(q[2], nout - 1) for q in wl.pulses])
    x = torch.from_numpy(wl.x).cuda()
    return wl, p, s, n, nout, b, d, t, x


def _oracle_pulse_transpose(orc, opar, wl, s, n, nout, b, d, t):
    """d(sum_e y[b_e, d_e, t_e])/dw: per pulse, the oracle's weight adjoint of an output
    gradient that is 1 at that pulse's output only; summed over the pulses."""
    K = wl.weights.shape[1]

    def one(e):
        g = np.zeros((1, 1, nout))
        g[0, 0, t[e]] = 1.0
        return orc.adjoint_w(wl.x[b[e]:b[e] + 1], s[d[e]:d[e] + 1], n[d[e]:d[e] + 1], g, "tap", K)

    return np.sum(opar.map(one, range(len(b))), axis=0)


def _oracle_loss(orc, wl, s, n, b, d, t, w32):
    """L = -(1/B) sum_e y_e / ||w|| with y_e the outputs at the pulses (sigma = 1), fp64,
    for fp32 weights w32."""
    ye = orc.dedisperse_points(wl.x, s, n, b, d, t, "tap", w32)
    return -float(np.sum(ye)) / (len(b) * float(np.linalg.norm(w32.astype(np.float64))))


def test_cfg5_full_sparse_and_loss_gradients(dd, orc, opar, cfg5_full):
    import torch
    from paper_1301_3968_amd.autograd import matched_filter_loss
    wl, p, s, n, nout, b, d, t, x = cfg5_full
    B = len(b)
    G = p.backward_sparse(x, b, d, t, torch.ones(B, device="cuda")).cpu().numpy()
    Go = _oracle_pulse_transpose(orc, opar, wl, s, n, nout, b, d, t)
    assert G.shape == (336, 8)
    assert np.allclose(G, Go, rtol=1e-12, atol=1e-12 * np.abs(Go).max())
    # the loss gradient through autograd (library adjoint + the S/N normalisation)
    w = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
    L = matched_filter_loss(x, w, p, b, d, t, sparse=True)
    L.backward()
    g = w.grad.cpu().numpy().astype(np.float64)
    w64 = wl.weights.astype(np.float64)
    nw = float(np.linalg.norm(w64))
    ysum = float(np.sum(orc.dedisperse_points(wl.x, s, n, b, d, t, "tap", wl.weights)))
    ta, tb = Go / nw / B, ysum * w64 / nw ** 3 / B
    go = -(ta - tb)
    assert float(L) == pytest.approx(_oracle_loss(orc, wl, s, n, b, d, t, wl.weights), rel=1e-6)
    # the loss gradient is a difference of two terms delivered in fp32 (the adjoint's
    # fp64 G scaled, and the forward's outputs times w): its error is bounded relative
    # to the terms' magnitudes, not to their cancelling difference
    mag = np.abs(ta) + np.abs(tb)
    assert (np.abs(g - go) / np.maximum(mag, 1e-3 * mag.max())).max() < 1e-5
    # 32 central differences of the oracle's loss, h = 1e-3 (the perturbed weights are
    # fp32 values, so the step actually taken is divided out)
    rng = np.random.default_rng(32)
    h = np.float32(1e-3)
    for _ in range(32):
        c, k = int(rng.integers(0, 336)), int(rng.integers(0, 8))
        wp, wm = wl.weights.copy(), wl.weights.copy()
        wp[c, k] += h
        wm[c, k] -= h
        step = float(wp[c, k]) - float(wm[c, k])
        fd = (_oracle_loss(orc, wl, s, n, b, d, t, wp)
              - _oracle_loss(orc, wl, s, n, b, d, t, wm)) / step
        assert g[c, k] == pytest.approx(fd, rel=1e-5, abs=1e-5 * np.abs(go).max()), (c, k)


def test_cfg5_full_dense_adjoint_sampled_channels(dd, orc, opar, cfg5_full):
    import torch
    wl, p, s, n, nout, b, d, t, x = cfg5_full
    K = wl.weights.shape[1]
    rng = np.random.default_rng(55)
    g = rng.standard_normal((x.shape[0], len(wl.dms), nout)).astype(np.float32)
    _, gw = p.backward(_dev(g), x, need_x=False, need_w=True)
    gw = gw.cpu().numpy()
    g64 = g.astype(np.float64)
    del g
    chans = [0, 111, 222, 335]

    def one(c):
        return orc.adjoint_w(np.ascontiguousarray(wl.x[:, c:c + 1, :]), s[:, c:c + 1],
                             n[:, c:c + 1], g64, "tap", K)[0]

    ref = np.stack(opar.map(one, chans))
    assert _r14(gw[chans], ref) < 1e-5
