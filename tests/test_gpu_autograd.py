"""Gradients of the matched-filter S/N loss with respect to per-tap weights:
the library's sparse and dense adjoints against an fp64 oracle gradient and
oracle central differences (h = 1e-3)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(orc, otables):
    import torch
    import paper_1301_3968_amd as dd
    wl = workloads.cfg5(batch=4, nsamp=4096, ndm=32, nchan=48)
    K = wl.extra["ktaps"]
    p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="fixed", ktaps=K, wmode="tap",
                weights=wl.weights)
    s, n = otables(p, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, "fixed", ktaps=K)
    nout = p.out_len(wl.x.shape[2])
    b = np.arange(len(wl.pulses))
    d = np.array([pl[1] for pl in wl.pulses])
    t = np.array([min(pl[2], nout - 1) for pl in wl.pulses])
    x = torch.from_numpy(wl.x).cuda()
    return dd, wl, p, s, n, x, b, d, t


def _oracle_loss_grad(orc, wl, s, n, b, d, t, w64):
    """L = -(1/B) sum_e y_e / ||w|| and its gradient, in fp64 (sigma = 1)."""
    B = len(b)
    w32 = w64.astype(np.float32)
    ye = orc.dedisperse_points(wl.x, s, n, b, d, t, "tap", w32)
    nw = np.linalg.norm(w32.astype(np.float64))
    L = -np.sum(ye) / (B * nw)
    g = np.zeros((wl.x.shape[0], s.shape[0], wl.x.shape[2] - int(np.max(s + n)) + 1))
    np.add.at(g, (b, d, t), 1.0)
    dy = orc.adjoint_w(wl.x, s, n, g, "tap", w32.shape[1])      # d(sum_e y_e)/dw
    ta = dy / nw / B
    tb = np.sum(ye) * w32.astype(np.float64) / nw ** 3 / B
    return L, -(ta - tb), np.abs(ta) + np.abs(tb)


@pytest.mark.parametrize("sparse", [True, False])
def test_loss_gradient_matches_oracle(setup, orc, sparse):
    import torch
    from paper_1301_3968_amd.autograd import matched_filter_loss
    dd, wl, p, s, n, x, b, d, t = setup
    w = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
    L = matched_filter_loss(x, w, p, b, d, t, sparse=sparse)
    L.backward()
    Lo, go, mag = _oracle_loss_grad(orc, wl, s, n, b, d, t, wl.weights.astype(np.float64))
    assert float(L) == pytest.approx(Lo, rel=1e-5)
    g = w.grad.cpu().numpy().astype(np.float64)
    # the gradient is a difference of two terms delivered in fp32: its error is
    # bounded relative to the terms' magnitudes, not to their (cancelling) sum
    scale = np.maximum(mag, 1e-3 * mag.max())
    assert (np.abs(g - go) / scale).max() < 1e-5
    # the library's part, the weight adjoint, is fp64-exact against the oracle
    B = len(b)
    gw = p.backward_sparse(x, b, d, t, torch.ones(B, device="cuda")).cpu().numpy()
    gd = np.zeros((wl.x.shape[0], s.shape[0], wl.x.shape[2] - int(np.max(s + n)) + 1))
    np.add.at(gd, (b, d, t), 1.0)
    assert np.allclose(gw, orc.adjoint_w(wl.x, s, n, gd, "tap", wl.weights.shape[1]),
                       rtol=1e-12, atol=1e-12)


def test_gradient_central_differences(setup, orc):
    import torch
    from paper_1301_3968_amd.autograd import matched_filter_loss
    dd, wl, p, s, n, x, b, d, t = setup
    w = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
    matched_filter_loss(x, w, p, b, d, t).backward()
    g = w.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    h = 1e-3
    for _ in range(12):
        c, k = int(rng.integers(0, w.shape[0])), int(rng.integers(0, w.shape[1]))
        wp = wl.weights.astype(np.float64).copy()
        wm = wp.copy()
        wp[c, k] += h
        wm[c, k] -= h
        lp = _oracle_loss_grad(orc, wl, s, n, b, d, t, wp)[0]
        lm = _oracle_loss_grad(orc, wl, s, n, b, d, t, wm)[0]
        dh = float(np.float32(wp[c, k])) - float(np.float32(wm[c, k]))
        fd = (lp - lm) / dh
        assert g[c, k] == pytest.approx(fd, rel=1e-4, abs=1e-7 * np.abs(g).max())


def test_training_improves_snr(setup):
    import torch
    from paper_1301_3968_amd.autograd import matched_filter_loss
    dd, wl, p, s, n, x, b, d, t = setup
    w = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
    opt = torch.optim.Adam([w], lr=0.02)
    first = None
    for _ in range(30):
        opt.zero_grad()
        L = matched_filter_loss(x, w, p, b, d, t)
        L.backward()
        opt.step()
        first = float(L) if first is None else first
    assert float(matched_filter_loss(x, w, p, b, d, t)) < first


def test_training_approaches_the_dynamic_spectrum_matched_filter(setup, orc):
    # The loss is the negative mean S/N of <G, w> / ||w|| with G = d(sum_e y_e)/dw (the
    # sum is linear in w), so its optimum is w parallel to G (the dynamic-spectrum matched
    # filter of the batch's pulses, Section 4), with S/N ||G|| / B (Cauchy-Schwarz).
    import torch
    from paper_1301_3968_amd.autograd import matched_filter_loss
    dd, wl, p, s, n, x, b, d, t = setup
    B = len(b)
    g = np.zeros((wl.x.shape[0], s.shape[0], wl.x.shape[2] - int(np.max(s + n)) + 1))
    np.add.at(g, (b, d, t), 1.0)
    G = orc.adjoint_w(wl.x, s, n, g, "tap", wl.weights.shape[1])
    best = np.linalg.norm(G) / B
    w = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
    opt = torch.optim.Adam([w], lr=0.02)
    snr0 = -float(matched_filter_loss(x, w, p, b, d, t))
    for _ in range(300):
        opt.zero_grad()
        matched_filter_loss(x, w, p, b, d, t).backward()
        opt.step()
    snr = -float(matched_filter_loss(x, w, p, b, d, t))
    wl_ = w.detach().cpu().numpy().astype(np.float64)
    cos = float(np.sum(wl_ * G) / (np.linalg.norm(wl_) * np.linalg.norm(G)))
    assert snr0 < snr <= best * (1.0 + 1e-6)
    assert snr > 0.97 * best and cos > 0.97, (snr0, snr, best, cos)
