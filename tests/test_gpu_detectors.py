"""Section 4 detectors on the GPU path (tap-weighted, boxcar and greedy dedispersions of a
rendered 1 ms rectangular pulse at DM 30) against the oracle's closed forms of the same
detectors on the same cells."""
import math

import numpy as np
import pytest

import bench
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


@pytest.mark.parametrize("b", [1.0, 4.0])
def test_detectors_match_oracle_closed_forms(dd, orc, b):
    got, _, dt, cw = bench.detector_snrs(dd, workloads, b)
    tau, lead = bench.RES_TAU, 16
    lo, bw = bench.RES_BAND
    C = int(round(bw / cw))
    f = workloads.channel_centres(lo, bw, C)
    s0 = orc.delay_start(f, cw, dt, [bench.RES_DM])[0]
    n0 = orc.taps_allnonzero(f, cw, dt, [bench.RES_DM], tau)[0]
    K = int(n0.max())
    T = int(np.max(s0 + n0)) + K + 2 * lead
    x = workloads.render_rect_pulse(f, cw, dt, T, bench.RES_DM, tau, lead * dt)
    P = x[np.arange(C)[:, None], lead + s0[:, None] + np.arange(K)[None, :]].astype(np.float64)
    scale = 1.0 / math.sqrt(C * tau)          # to units of P0 sqrt(beta tau) / k T_sys
    prof = P.sum(axis=0)
    on = np.nonzero(prof > 0.0)[0]
    ref = {"dsmf": orc.snr_dsmf(P.T, dt, 1.0) * scale,
           "mf": orc.snr_mf(P.T, dt, 1.0) * scale,
           "boxcar": orc.snr_bmf(P.T[on[0]:on[-1] + 1], dt, 1.0) * scale}
    s, n, _ = orc.greedy_tables(f, cw, dt, [bench.RES_DM], tau)
    y = orc.dedisperse_f64(x.astype(np.float64), s.astype(np.int32), n.astype(np.int32))[0]
    ref["greedy"] = y.max() / math.sqrt(float(n.sum())) * math.sqrt(dt / (C * tau))
    for k, v in ref.items():
        assert got[k] == pytest.approx(v, rel=1e-5), k
    # the dynamic-spectrum matched filter is the best linear detector (Cauchy-Schwarz)
    assert got["dsmf"] >= max(got.values()) * (1.0 - 1e-6)
