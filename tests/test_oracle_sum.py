"""Pins of the oracle's dedispersion sum, boxcar detector and adjoints.

Each test checks the oracle against something other than itself: numpy's
convolution and summation routines, exact invariants (linearity, the adjoint
identity), Monte Carlo noise statistics, or the physics of an injected pulse.
"""
import math

import numpy as np
import pytest

import workloads


def _tables(orc, f, bw, dt, dms, rule="smear"):
    s = orc.delay_start(f, bw, dt, dms)
    n = orc.taps_smear(f, bw, dt, dms) if rule == "smear" else orc.taps_allnonzero(f, bw, dt, dms)
    return s.astype(np.int32), n.astype(np.int32)


def test_dm0_single_tap_is_channel_sum(orc):
    # eq. p_dedisp at DM = 0 with one sample per channel: the plain sum over channels.
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, size=(7, 50), dtype=np.uint8)
    s = np.zeros((1, 7), np.int32)
    n = np.ones((1, 7), np.int32)
    y = orc.dedisperse_u8(x, s, n)
    assert np.array_equal(y[0], x.astype(np.int64).sum(axis=0))


def test_sum_matches_numpy_convolution(orc):
    # Each channel's run of n samples is a length-n box filter (np.convolve 'valid'),
    # shifted by the channel delay.
    rng = np.random.default_rng(2)
    C, T = 9, 700
    f = workloads.channel_centres(1.2, 0.3, C)
    bw = 0.3 / C
    dms = np.array([0.0, 37.0, 150.0, 401.5])
    s, n = _tables(orc, f, bw, 1e-3, dms)
    x = rng.integers(0, 256, size=(C, T), dtype=np.uint8)
    y = orc.dedisperse_u8(x, s, n)
    tout = y.shape[1]
    for d in range(len(dms)):
        ref = np.zeros(tout, np.int64)
        for c in range(C):
            box = np.convolve(x[c].astype(np.int64), np.ones(n[d, c], np.int64), "valid")
            ref += box[s[d, c]:s[d, c] + tout]
        assert np.array_equal(y[d], ref)
    yf = orc.dedisperse_f64(x, s, n)
    assert np.array_equal(yf, y.astype(np.float64))


def test_points_match_full(orc):
    rng = np.random.default_rng(3)
    C, T = 5, 200
    x = rng.standard_normal((2, C, T)).astype(np.float32)
    s = rng.integers(0, 20, size=(3, C)).astype(np.int32)
    n = rng.integers(0, 6, size=(3, C)).astype(np.int32)
    w = rng.standard_normal((C, 6)).astype(np.float32)
    n[:] = 6
    y = orc.dedisperse_f64(x, s, n, "tap", w)
    b = np.array([0, 1, 1, 0]); d = np.array([0, 2, 1, 2]); t = np.array([0, 5, y.shape[2] - 1, 17])
    p = orc.dedisperse_points(x, s, n, b, d, t, "tap", w)
    assert np.allclose(p, y[b, d, t], rtol=0, atol=1e-12)


def test_linearity_exact(orc):
    rng = np.random.default_rng(4)
    C, T = 6, 120
    s = rng.integers(0, 10, size=(4, C)).astype(np.int32)
    n = rng.integers(1, 5, size=(4, C)).astype(np.int32)
    x1 = rng.integers(-100, 100, size=(C, T)).astype(np.float64)
    x2 = rng.integers(-100, 100, size=(C, T)).astype(np.float64)
    a, b = 3.0, -7.0
    y = orc.dedisperse_f64(a * x1 + b * x2, s, n)
    assert np.array_equal(y, a * orc.dedisperse_f64(x1, s, n) + b * orc.dedisperse_f64(x2, s, n))


def test_injected_pulse_found_at_true_dm_and_time(orc):
    # A dispersed pulse (signal model of Section 2.1) must peak at its own DM
    # trial and arrival time.
    wl = workloads.cfg1()
    s, n = _tables(orc, wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, wl.rule)
    y = orc.dedisperse_u8(wl.x, s, n)
    M, S = orc.boxcar_norm(n, wl.widths, wl.chan_mean, wl.chan_sigma)
    snr, t, W = orc.boxcar_detect(y.astype(np.float64), wl.widths, M, S)
    d = int(np.argmax(snr))
    assert abs(wl.dms[d] - wl.pulses[0].dm) <= 10.0
    t_true = int(round(wl.pulses[0].t_arrival_s / wl.dt_s))
    assert abs(int(t[d]) + W[d] / 2 - t_true) <= W[d] / 2 + 2
    assert snr[d] > 20


def test_detect_matches_numpy_boxcar(orc):
    rng = np.random.default_rng(5)
    D, tout = 5, 400
    y = rng.integers(-1000, 1000, size=(D, tout)).astype(np.float64)
    y[2, 100:104] += 5000  # a clear pulse
    widths = np.array([1, 2, 3, 5, 8], np.int32)
    M = rng.uniform(-50, 50, size=(D, len(widths)))
    S = rng.uniform(10, 60, size=(D, len(widths)))
    snr, t, W = orc.boxcar_detect(y, widths, M, S)
    for d in range(D):
        best = (-math.inf, 0, 0)
        for j, w in enumerate(widths):
            B = np.convolve(y[d], np.ones(w), "valid")
            r = (B - M[d, j]) / S[d, j]
            k = int(np.argmax(r))  # first occurrence
            if r[k] > best[0]:
                best = (r[k], int(w), k)
        assert snr[d] == pytest.approx(best[0], rel=1e-14)
        assert (W[d], t[d]) == (best[1], best[2])


def test_norm_unit_width1_is_radiometer_sum(orc):
    # eq. P_N_dedisp: for one output sample, sigma_dedisp = sqrt(N_S) sigma_n.
    rng = np.random.default_rng(6)
    n = rng.integers(0, 9, size=(4, 11)).astype(np.int32)
    mu, sg = np.full(11, 128.0), np.full(11, 16.0)
    M, S = orc.boxcar_norm(n, [1], mu, sg)
    assert np.allclose(S[:, 0], np.sqrt(n.sum(axis=1)) * 16.0, rtol=1e-15)
    assert np.allclose(M[:, 0], 128.0 * n.sum(axis=1), rtol=1e-15)


@pytest.mark.parametrize("wmode", ["unit", "channel", "tap"])
def test_norm_matches_monte_carlo(orc, wmode):
    # On pure Gaussian noise the normalised boxcar S/N has mean 0 and std 1.
    rng = np.random.default_rng(7)
    C, T = 12, 40000
    mu = rng.uniform(50, 150, C)
    sg = rng.uniform(5, 20, C)
    K = 4
    s = rng.integers(0, 30, size=(3, C)).astype(np.int32)
    n = (np.full((3, C), K) if wmode == "tap" else rng.integers(1, 7, size=(3, C))).astype(np.int32)
    w = None
    if wmode == "channel":
        w = rng.uniform(0.2, 2.0, C).astype(np.float32)
    elif wmode == "tap":
        w = rng.uniform(-1.0, 2.0, (C, K)).astype(np.float32)
    x = mu[:, None] + sg[:, None] * rng.standard_normal((C, T))
    y = orc.dedisperse_f64(x, s, n, wmode, w)
    widths = [1, 3, 8]
    M, S = orc.boxcar_norm(n, widths, mu, sg, wmode, w)
    for d in range(3):
        for j, W in enumerate(widths):
            B = np.convolve(y[d], np.ones(W), "valid")
            z = (B - M[d, j]) / S[d, j]
            assert abs(np.mean(z)) < 0.05
            assert abs(np.std(z) - 1.0) < 0.03


def _explicit_matrix(C, T, s, n, w):
    """The linear map of eq. p_dedisp written out entry by entry: row (d, t) holds
    w[c, k] in column (c, t + s[d, c] + k) for every channel c and tap k < n[d, c]."""
    D = s.shape[0]
    tout = T - int(np.max(s + n)) + 1
    A = np.zeros((D * tout, C * T))
    for d in range(D):
        for t in range(tout):
            for c in range(C):
                for k in range(n[d, c]):
                    A[d * tout + t, c * T + t + s[d, c] + k] += w[c, k]
    return A, tout


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_matrix(orc, seed):
    # Tiny instances (C <= 4, T <= 32, D <= 4): y = A x, A^T g for both adjoints,
    # and unit weights as the all-ones special case, against the explicit matrix.
    rng = np.random.default_rng(100 + seed)
    C, T, D, K = int(rng.integers(1, 5)), int(rng.integers(16, 33)), int(rng.integers(1, 5)), 4
    s = rng.integers(0, 8, size=(D, C)).astype(np.int32)
    n = rng.integers(0, K + 1, size=(D, C)).astype(np.int32)
    n[0, 0] = max(n[0, 0], 1)
    w = rng.standard_normal((C, K)).astype(np.float32)
    w64 = w.astype(np.float64)
    A, tout = _explicit_matrix(C, T, s, n, w64)
    x = rng.standard_normal((C, T))
    y = orc.dedisperse_f64(x, s, n, "tap", w)
    assert y.shape == (D, tout)
    assert np.allclose(y.ravel(), A @ x.ravel(), rtol=0, atol=1e-12)
    g = rng.standard_normal((D, tout))
    assert np.allclose(orc.adjoint_x(T, s, n, g, "tap", w).ravel(), A.T @ g.ravel(),
                       rtol=0, atol=1e-12)
    # weight adjoint: column (c, k) of the Jacobian of y in w
    gw = orc.adjoint_w(x, s, n, g, "tap", K)
    for c in range(C):
        for k in range(K):
            e = np.zeros((C, K))
            e[c, k] = 1.0
            Ak, _ = _explicit_matrix(C, T, s, n, e)
            assert gw[c, k] == pytest.approx(float(g.ravel() @ (Ak @ x.ravel())), abs=1e-12)
    # unit weights on uint8: integer-exact
    A1, _ = _explicit_matrix(C, T, s, n, np.ones((C, K)))
    xu = rng.integers(0, 256, size=(C, T), dtype=np.uint8)
    yu = orc.dedisperse_u8(xu, s, n)
    assert np.array_equal(yu.ravel(), (A1 @ xu.ravel().astype(np.float64)).astype(np.int64))


def test_adjoint_dot_product_identity(orc):
    # <A x, g> = <x, A^T g> and <A_w x, g> linear in w: grad_w = A-adjoint in w.
    rng = np.random.default_rng(8)
    B, C, T, D, K = 2, 5, 90, 4, 3
    s = rng.integers(0, 12, size=(D, C)).astype(np.int32)
    n = np.full((D, C), K, np.int32)
    w = rng.standard_normal((C, K)).astype(np.float32)
    x = rng.integers(-5, 6, size=(B, C, T)).astype(np.float64)
    y = orc.dedisperse_f64(x, s, n, "tap", w)
    g = rng.integers(-5, 6, size=y.shape).astype(np.float64)
    gx = orc.adjoint_x(T, s, n, g, "tap", w)
    lhs = float(np.sum(y * g))
    rhs = float(np.sum(x * gx))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # Weight adjoint: y is linear in w, so <y(w), g> = sum_ck w_ck * gw_ck exactly.
    gw = orc.adjoint_w(x, s, n, g, "tap", K)
    assert lhs == pytest.approx(float(np.sum(w.astype(np.float64) * gw)), rel=1e-12)
    # Unit weights on uint8: integer identity.
    xu = rng.integers(0, 256, size=(C, T), dtype=np.uint8)
    nu = rng.integers(0, 5, size=(D, C)).astype(np.int32)
    yu = orc.dedisperse_u8(xu, s, nu)
    gu = rng.integers(-3, 4, size=yu.shape).astype(np.float64)
    gxu = orc.adjoint_x(T, s, nu, gu)
    assert int(np.sum(yu * gu.astype(np.int64))) == int(round(float(np.sum(xu * gxu))))


def test_weight_gradient_central_differences(orc):
    # Central finite differences (h = 1e-3) of L(w) = <g, y(w)> in fp64.
    rng = np.random.default_rng(9)
    B, C, T, D, K = 2, 4, 70, 3, 3
    s = rng.integers(0, 10, size=(D, C)).astype(np.int32)
    n = np.full((D, C), K, np.int32)
    x = rng.standard_normal((B, C, T))
    w = rng.standard_normal((C, K)).astype(np.float64)
    g = rng.standard_normal((B, D, T - int(np.max(s + n)) + 1))
    gw = orc.adjoint_w(x, s, n, g, "tap", K)
    h = 1e-3
    for c in range(C):
        for k in range(K):
            # weights go to the oracle as fp32; use exactly representable perturbations
            wp, wm = w.copy(), w.copy()
            wp[c, k] += h
            wm[c, k] -= h
            lp = np.sum(g * orc.dedisperse_f64(x, s, n, "tap", wp.astype(np.float32)))
            lm = np.sum(g * orc.dedisperse_f64(x, s, n, "tap", wm.astype(np.float32)))
            dwp = float(np.float32(wp[c, k])) - float(np.float32(wm[c, k]))
            fd = (lp - lm) / dwp
            assert fd == pytest.approx(gw[c, k], rel=1e-6, abs=1e-9)
