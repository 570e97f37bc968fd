"""Section 5.3 completeness curve on the GPU path (greedy sample sets, batched fp32
dedispersion, per-trial S/N) against the oracle on the same inputs: the 32-channel
21-23 GHz survey example with its 128 trial DMs."""
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


def test_completeness_curve_matches_oracle(dd, orc, otables):
    case = bench.COMPLETENESS_CASES[2]
    _, flo, band, C, dt, tau, lo, hi, eps = case
    f = workloads.channel_centres(flo, band, C)
    dms = orc.trial_dms(lo, hi, eps, f, band / C, dt)
    assert len(dms) == 128                               # the count the paper quotes
    pick = np.arange(0, 127, 9)
    true = np.concatenate([dms[pick], 0.5 * (dms[pick] + dms[pick + 1])])
    np.testing.assert_allclose(dd.trial_dms(lo, hi, eps, f, band / C, dt), dms, rtol=1e-12)
    plan, best, arg, snr, _ = bench.completeness_case(dd, workloads, case, true, chunk=8, dms=dms)
    s, n = otables(plan, f, band / C, dt, dms, "greedy", width_s=tau)
    T = plan.max_span + 128
    M, S = orc.boxcar_norm(n, [1], np.zeros(C), np.ones(C))
    norm = np.sqrt(dt / (C * tau))
    for i, dm in enumerate(true):
        x = workloads.render_rect_pulse(f, band / C, dt, T, float(dm), tau, 64 * dt)
        y = orc.dedisperse_f64(x.astype(np.float64), s, n)
        so, to, wo = orc.boxcar_detect(y, [1], M, S)
        # fp32 sums of positive terms: 1e-5 of the fp64 value
        np.testing.assert_allclose(snr[i], so * norm, rtol=1e-5, atol=0)
    # a pulse at a trial DM is found best at that trial
    assert np.array_equal(arg[:len(pick)], pick)
