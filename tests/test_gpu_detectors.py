"""Section 4 detectors on the GPU path (tap-weighted, boxcar and greedy dedispersions of a
rendered 1 ms rectangular pulse at DM 30) against the oracle on the same cells: the
whole dedispersed series of each detector and the oracle's closed forms of its S/N, at
every channel width of the comparison, and the detectors' order at a finer sample time."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

GRID = [0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0]


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


def _oracle_detectors(orc, an, b, a=1.0):
    """The oracle's S/N of the four detectors and its dedispersed series for the test
    pulse at channel width b dnu_0 and sample time a tau."""
    tau, lead, dm = an.RES_TAU, 16, an.RES_DM
    lo, bw = an.RES_BAND
    C = max(1, int(round(bw / (b * an.res_delta_nu0()))))
    cw, dt = bw / C, a * tau
    f = workloads.channel_centres(lo, bw, C)
    s0 = orc.delay_start(f, cw, dt, [dm])[0]
    n0 = orc.taps_allnonzero(f, cw, dt, [dm], tau)[0]
    K = int(n0.max())
    T = int(np.max(s0 + n0)) + K + 2 * lead
    x = workloads.render_rect_pulse(f, cw, dt, T, dm, tau, lead * dt).astype(np.float64)
    P = x[np.arange(C)[:, None], lead + s0[:, None] + np.arange(K)[None, :]]
    scale = 1.0 / math.sqrt(C * tau)          # to units of P0 sqrt(beta tau) / k T_sys
    prof = P.sum(axis=0)
    on = np.nonzero(prof > 0.0)[0]
    snr = {"dsmf": orc.snr_dsmf(P.T, dt, 1.0) * scale,
           "mf": orc.snr_mf(P.T, dt, 1.0) * scale,
           "boxcar": orc.snr_bmf(P.T[on[0]:on[-1] + 1], dt, 1.0) * scale}
    s0 = s0.astype(np.int32)[None]
    full = np.full(s0.shape, K, np.int32)
    ser = {"dsmf": orc.dedisperse_f64(x, s0, full, "tap", P.astype(np.float32))[0],
           "mf": orc.dedisperse_f64(x, s0, full, "tap",
                                    np.broadcast_to(prof, (C, K)).astype(np.float32))[0],
           "boxcar": orc.dedisperse_f64(x, s0 + on[0], np.full(s0.shape, len(on), np.int32))[0]}
    s, n, _ = orc.greedy_tables(f, cw, dt, [dm], tau)
    ser["greedy"] = orc.dedisperse_f64(x, s.astype(np.int32), n.astype(np.int32))[0]
    snr["greedy"] = ser["greedy"].max() / math.sqrt(float(n.sum())) * math.sqrt(dt / (C * tau))
    return snr, ser


@pytest.mark.parametrize("b", GRID)
def test_detectors_match_oracle(dd, orc, an, b):
    ser = {}
    got, _, dt, cw = an.detector_snrs(dd, workloads, b, series=ser)
    ref, rser = _oracle_detectors(orc, an, b)
    for k, v in ref.items():
        assert got[k] == pytest.approx(v, rel=1e-5), k
        y = rser[k]
        np.testing.assert_allclose(ser[k], y, rtol=1e-5, atol=1e-6 * np.abs(y).max(), err_msg=k)
    # the dynamic-spectrum matched filter is the best linear detector (Cauchy-Schwarz)
    assert got["dsmf"] >= max(got.values()) * (1.0 - 1e-6)


def test_detector_order_at_finer_sample_time(dd, orc, an):
    # With dt = tau / 4 the time-series matched filter leads the greedy detector at fine
    # channel widths and trails it at coarse ones (the ordering Section 4 describes).
    fine, _, _, _ = an.detector_snrs(dd, workloads, 0.125, a=0.25)
    coarse, _, _, _ = an.detector_snrs(dd, workloads, 4.0, a=0.25)
    assert fine["mf"] > fine["greedy"]
    assert coarse["greedy"] > coarse["mf"]
    ref, _ = _oracle_detectors(orc, an, 0.125, a=0.25)
    for k, v in ref.items():
        assert fine[k] == pytest.approx(v, rel=1e-5), k
