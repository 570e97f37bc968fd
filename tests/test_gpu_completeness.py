"""Section 5.3 completeness curves on the GPU path (greedy sample sets, batched fp32
dedispersion, per-trial S/N) against the oracle on the same inputs, for the three survey
examples: the 32- and 256-channel 21-23 GHz grids of 128 trials (every trial's S/N for
sampled test pulses) and the 304-channel CRAFT grid of 442 trials (the trials about
each sampled test pulse's DM, where its largest S/N lies)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch  # noqa: F401
    import paper_1301_3968_amd as dd
    return dd


def _setup(dd, orc, an, k):
    case = an.COMPLETENESS_CASES[k]
    _, flo, band, C, dt, tau, lo, hi, eps = case
    f = workloads.channel_centres(flo, band, C)
    dms = orc.trial_dms(lo, hi, eps, f, band / C, dt)
    np.testing.assert_allclose(dd.trial_dms(lo, hi, eps, f, band / C, dt, cap=100000), dms,
                               rtol=1e-12)
    return case, f, dms


def _oracle_trial_snrs(orc, case, f, dms, idx, true):
    """Per test pulse, the oracle's width-1 S/N at trials idx (normalised like the GPU's)."""
    _, flo, band, C, dt, tau, lo, hi, eps = case
    s, n, _ = orc.greedy_tables(f, band / C, dt, dms[idx], tau)
    s, n = s.astype(np.int32), n.astype(np.int32)
    T = int(np.max(s + n)) + 128
    M, S = orc.boxcar_norm(n, [1], np.zeros(C), np.ones(C))
    norm = np.sqrt(dt / (C * tau))
    out = np.empty((len(true), len(idx)))
    for i, dm in enumerate(true):
        x = workloads.render_rect_pulse(f, band / C, dt, T, float(dm), tau, 64 * dt)
        y = orc.dedisperse_f64(x.astype(np.float64), s, n)
        out[i] = orc.boxcar_detect(y, [1], M, S)[0] * norm
    return out


@pytest.mark.parametrize("k", [1, 2])
def test_completeness_21_23ghz_every_trial(dd, orc, otables, an, k):
    case, f, dms = _setup(dd, orc, an, k)
    assert len(dms) == 128                               # the count the paper quotes
    pick = np.arange(0, 127, 9)
    true = np.concatenate([dms[pick], 0.5 * (dms[pick] + dms[pick + 1])])
    plan, best, arg, snr, _ = an.completeness_case(dd, workloads, case, true, chunk=8, dms=dms)
    _, flo, band, C, dt, tau, lo, hi, eps = case
    otables(plan, f, band / C, dt, dms, "greedy", width_s=tau)
    ref = _oracle_trial_snrs(orc, case, f, dms, np.arange(len(dms)), true)
    # fp32 sums of positive terms: 1e-5 of the fp64 value
    np.testing.assert_allclose(snr, ref, rtol=1e-5, atol=0)
    # a pulse at a trial DM is found best at that trial
    assert np.array_equal(arg[:len(pick)], pick)


def test_completeness_craft_grid(dd, orc, an):
    case, f, dms = _setup(dd, orc, an, 0)
    assert len(dms) == 442                               # the count the paper quotes
    pick = np.array([3, 77, 150, 260, 333, 420])
    true = np.concatenate([dms[pick], 0.5 * (dms[pick] + dms[pick + 1])])
    plan, best, arg, snr, _ = an.completeness_case(dd, workloads, case, true, chunk=6, dms=dms)
    near = np.unique(np.concatenate([pick - 1, pick, pick + 1, pick + 2]))
    ref = _oracle_trial_snrs(orc, case, f, dms, near, true)
    np.testing.assert_allclose(snr[:, near], ref, rtol=1e-5, atol=0)
    # the largest S/N of each test pulse lies at one of the trials beside its DM
    assert np.all(np.isin(arg, near))
    np.testing.assert_allclose(best, ref.max(axis=1), rtol=1e-5)
    assert np.array_equal(arg[:len(pick)], pick)
