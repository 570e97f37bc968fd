"""Pins of the oracle's sample-set tables and smearing constants against what the
delay law itself fixes: the band sweep the channel smears telescope to, the
hand-worked counts in tests/golden/smear_examples.csv, the first-order smear of
Section 3, and the defining property of DM_tau (Section 3) and Delta nu_0.

None of these compares against the library."""
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KAPPA_SI = 2.41e-16          # Section 2.1: t_d = DM / (kappa nu^2), nu in Hz, t in s


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip().split(",") for ln in fh if ln.strip() and not ln.startswith("#")]


def _delay_si(dm, nu_hz):
    """The Section 2.1 delay law in its own units (Hz, seconds)."""
    return dm / (KAPPA_SI * nu_hz * nu_hz)


# ------------------------------------------------------------------ smear taps (Section 3)

@pytest.mark.parametrize("flo,ftop,dm,dt,n", [tuple(float(v) for v in r)
                                               for r in _rows("smear_examples.csv")])
def test_smear_taps_hand_examples(orc, flo, ftop, dm, dt, n):
    centre, bw = 0.5 * (flo + ftop), ftop - flo
    got = orc.taps_smear(np.array([centre]), bw, dt, [dm])
    assert got.shape == (1, 1) and int(got[0, 0]) == int(n)


@pytest.mark.parametrize("flo,band,C,dt", [(1.2, 0.336, 336, 1e-3), (1.2, 0.3, 64, 1e-3),
                                           (0.7, 0.304, 304, 1e-3), (21.0, 2.0, 32, 1e-4)])
def test_smear_taps_telescope_to_band_sweep(orc, flo, band, C, dt):
    # Contiguous channels: the channel smears add up to the delay difference between the
    # band's two edges.  Each count is that smear rounded up, so the counts sum to the
    # sweep (in samples) plus less than one sample per channel.
    f = workloads.channel_centres(flo, band, C)
    dms = np.array([50.0, 333.3, 1000.0, 2000.0])
    n = orc.taps_smear(f, band / C, dt, dms)
    for i, dm in enumerate(dms):
        sweep = (_delay_si(dm, flo * 1e9) - _delay_si(dm, (flo + band) * 1e9)) / dt
        if sweep < C:      # the max(1, .) floor would dominate: not a telescoping case
            continue
        tot = int(n[i].sum())
        assert sweep - 1e-6 <= tot < sweep + C, (dm, tot, sweep)


@pytest.mark.parametrize("descending", [False, True])
def test_smear_run_reaches_next_channel_start(orc, descending):
    # t_A of a channel plus its smear is t_A of the channel below it (the lower edge of
    # one is the upper edge of the next), so the run [start, start + n) of every channel
    # ends at the next channel's start sample or one sample after it.
    f = workloads.channel_centres(1.2, 0.336, 336)
    if descending:
        f = f[::-1].copy()
    bw, dt = 0.001, 1e-3
    dms = np.linspace(1.0, 2000.0, 37)
    s = orc.delay_start(f, bw, dt, dms)
    n = orc.taps_smear(f, bw, dt, dms)
    order = np.argsort(-f)                # top of the band first
    s, n = s[:, order], n[:, order]
    gap = s[:, :-1] + n[:, :-1] - s[:, 1:]
    assert set(np.unique(gap)) <= {0, 1}, np.unique(gap)
    assert np.any(gap == 0) and np.any(gap == 1)


def test_smear_taps_first_order(orc):
    # Narrow channels: the smear is Section 3's first-order 2 DM dnu / (kappa nu_c^3),
    # to within one sample.
    C, flo, band, dt = 4096, 1.2, 0.3, 64e-6
    f = workloads.channel_centres(flo, band, C)
    dnu = band / C
    dms = np.array([10.0, 250.0, 1000.0])
    n = orc.taps_smear(f, dnu, dt, dms)
    for i, dm in enumerate(dms):
        first = 2.0 * dm * (dnu * 1e9) / (KAPPA_SI * (f * 1e9) ** 3) / dt
        assert np.all(np.abs(n[i] - np.maximum(1, np.ceil(first))) <= 1)


def test_smear_taps_dm_zero_and_monotone(orc):
    f = workloads.channel_centres(1.2, 0.3, 64)
    dms = np.arange(0.0, 400.0, 7.0)
    n = orc.taps_smear(f, 0.3 / 64, 1e-3, dms)
    assert np.all(n[0] == 1)                                  # no smear at DM 0
    assert np.all(np.diff(n, axis=0) >= 0)                    # grows with DM
    assert np.all(np.diff(n[-1][np.argsort(f)]) <= 0)         # larger at lower frequency


# ------------------------------------------------------- DM_tau, DM_diag and Delta nu_0

def test_dm_tau_at_dt_is_dm_diag(orc):
    # DM_diag is DM_tau with the sample time in place of tau'_av (Section 5.2).
    for flo, band, C, dt in [(1.2, 0.336, 336, 1e-3), (21.0, 2.0, 256, 1e-4)]:
        f = workloads.channel_centres(flo, band, C)
        assert orc.dm_tau(f, band / C, dt) == pytest.approx(orc.dm_diag(f, band / C, dt),
                                                            rel=1e-15)


@pytest.mark.parametrize("flo,band,C,tau", [(1.2, 0.336, 336, 1e-3), (0.7, 0.3, 300, 2e-3),
                                            (21.0, 2.0, 256, 1e-4)])
def test_dm_tau_defining_property(orc, flo, band, C, tau):
    # At DM_tau the mean intra-channel smear equals tau'_av.  Measured with the smear
    # tap counts on a sample grid 1e5 times finer than tau (each count is the channel's
    # two-edge smear rounded up to that grid).
    f = workloads.channel_centres(flo, band, C)
    dnu = band / C
    dmt = orc.dm_tau(f, dnu, tau)
    fine = tau * 1e-5
    n = orc.taps_smear(f, dnu, fine, [dmt])[0]
    mean_smear = float(np.mean(n)) * fine
    assert mean_smear == pytest.approx(tau, rel=2e-4)
    # and it scales as tau / dnu
    assert orc.dm_tau(f, dnu, 3 * tau) == pytest.approx(3 * dmt, rel=1e-14)
    assert orc.dm_tau(f, 2 * dnu, tau) == pytest.approx(0.5 * dmt, rel=1e-14)


def test_delta_nu0_defining_property(orc):
    # Delta nu_0: the channel width at which the mean smear at the given DM is tau'_av.
    flo, band, tau, dm = 0.7, 0.3, 1e-3, 30.0
    f = workloads.channel_centres(flo, band, 300)
    d0 = orc.delta_nu0(f, tau, dm)
    assert orc.dm_tau(f, d0, tau) == pytest.approx(dm, rel=1e-14)
    # on a grid of about that channel width, the mean two-edge smear is tau'_av scaled by
    # the grid's width over its own Delta nu_0
    C = int(round(band / d0))
    f2 = workloads.channel_centres(flo, band, C)
    d2 = orc.delta_nu0(f2, tau, dm)
    fine = tau * 1e-5
    n = orc.taps_smear(f2, band / C, fine, [dm])[0]
    assert float(np.mean(n)) * fine == pytest.approx(tau * (band / C) / d2, rel=2e-4)
