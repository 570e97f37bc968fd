"""Pins of the oracle's model-side functions against numbers the paper prints,
closed forms, brute force and invariants."""
import itertools
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.strip().split(",") for ln in fh if ln.strip() and not ln.startswith("#")]


TRIAL_EXAMPLES = [tuple(float(v) for v in r) for r in _rows("trial_dm_examples.csv")]
SCALARS = {r[0]: float(r[1]) for r in _rows("scalar_values.csv")}


# ---------------------------------------------------------------- trial DMs (Section 5.3)

@pytest.mark.parametrize("flo,bw,C,dt,eps,lo,hi,count,drop", TRIAL_EXAMPLES)
def test_trial_counts_printed_in_paper(orc, flo, bw, C, dt, eps, lo, hi, count, drop):
    C = int(C)
    f = workloads.channel_centres(flo, bw, C)
    dms = orc.trial_dms(lo, hi, eps, f, bw / C, dt)
    assert len(dms) == int(count)
    assert dms[0] == lo and dms[-1] <= hi
    assert np.all(np.diff(dms) > 0)


@pytest.mark.parametrize("eps,drop", [(r[4], r[8]) for r in TRIAL_EXAMPLES])
def test_dropouts_printed_in_paper(orc, eps, drop):
    # eq. dm error smearing limit at the printed eps, to the printed two digits
    assert round(orc.dropout(eps), 2) == drop


def test_exponential_grid_count():
    # the geometric comparison grid: ratio r from lo reaches hi after the printed count
    r, lo, hi = SCALARS["exp_grid_ratio"], SCALARS["exp_grid_lo"], SCALARS["exp_grid_hi"]
    n = int(math.floor(math.log(hi / lo) / math.log(r))) + 1
    assert n == int(SCALARS["exp_grid_trials"])


def test_trial_rule_limits(orc):
    # Far below DM_diag the spacing is uniform, 2 eps DM_diag / C; far above, geometric
    # with ratio 1 + 2 eps / C (the two limits stated after eq. trial DMs).
    f = workloads.channel_centres(1.2, 0.336, 336)
    diag = orc.dm_diag(f, 0.001, 1e-3)
    d = orc.trial_dms(0.0, 1e9, 1.0, f, 0.001, 1e-3, cap=20000)
    step0 = d[1] - d[0]
    assert step0 == pytest.approx(2.0 * diag / 336, rel=1e-12)
    big = d[d > 1000 * diag]
    assert big[1] / big[0] == pytest.approx(1 + 2.0 / 336, rel=1e-6)


def test_attenuation_at_half_spacing_equals_dropout(orc):
    # A DM error of half the trial spacing gives exactly the (eps^2+1)^-1/4 drop-out.
    f = workloads.channel_centres(0.7, 0.304, 304)
    diag = orc.dm_diag(f, 0.001, 1e-3)
    for dm in (10.0, 300.0, 2500.0):
        ddm = 1.492 / 304 * math.sqrt(dm * dm + diag * diag)
        assert orc.snr_attenuation(ddm, dm, diag, 0.0, 304) == pytest.approx(orc.dropout(1.492), rel=1e-12)


# ------------------------------------------------- rectangular pulse model (App. A)

def test_cell_power_without_dispersion(orc):
    # DM = 0: every frequency sees the same rectangle [0, tau); the cell power is the
    # overlap length times (P0/dt) int (nu/nu0)^-alpha dnu.
    tau, dt = 2.5e-3, 1e-3
    f_lo, f_hi, alpha = 0.8, 0.81, 1.5
    spec = (f_hi ** (1 - alpha) - f_lo ** (1 - alpha)) / (1 - alpha)
    for j, ov in [(0, 1e-3), (1, 1e-3), (2, 0.5e-3), (3, 0.0)]:
        got = orc.cell_power_rect(j * dt, dt, f_lo, f_hi, 0.0, tau, alpha_paper=alpha)
        assert got == pytest.approx(ov / dt * spec, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("alpha,scat", [(0.0, 0.0), (1.5, 0.0), (-1.0, 2e-4)])
def test_snr_closed_form_appendix(orc, alpha, scat):
    # A pulse matching the template, summed over every non-zero cell (eq. num_samples),
    # reaches eq. snr_approx exactly: all the pulse power lands in the selected cells.
    C, flo, dnu, dt, dm, tau = 6, 0.7, 0.004, 1e-3, 30.0, 1e-3
    f = workloads.channel_centres(flo, dnu * C, C)
    s = orc.delay_start(f, dnu, dt, [dm])[0]
    n = orc.taps_allnonzero(f, dnu, dt, [dm], tau, scat, -4.0)[0]
    ft, fl, fh = orc.channel_edges(f, dnu)
    tot = 0.0
    for c in range(C):
        for j in range(s[c], s[c] + n[c]):
            tot += orc.cell_power_rect(j * dt, dt, fl[c], ft[c], dm, tau, scat, -4.0, alpha,
                                       nu_top=fh)
    N = int(n.sum())
    beta = dnu * C
    br = orc.spectral_bracket(fl, dnu, alpha)
    assert orc.snr_dedisp(tot, N, dt, dnu) == pytest.approx(
        orc.snr_approx(1.0, beta, tau, 1.0, dnu, dt, N, br), rel=1e-9)


def _snr_allnonzero(orc, flo, beta, C, dt, dm, tau):
    """eq. snr with the eq. num_samples set for a pulse that lands wholly in it:
    sum Pbar = P0 tau beta / dt (alpha = 0), so SNR = P0 tau beta / sqrt(dt N_S dnu)."""
    f = workloads.channel_centres(flo, beta, C)
    dnu = beta / C
    N = int(orc.taps_allnonzero(f, dnu, dt, [dm], tau)[0].sum())
    return tau * beta / math.sqrt(dt * N * dnu), f


def test_table1_coarse_time_slope(orc):
    # Coarse dt, fine dnu: S/N proportional to dt^-1/2 (Table 1, right column).
    flo, beta, C, dm, tau = 0.7, 0.3, 3000, 30.0, 1e-3
    s1, _ = _snr_allnonzero(orc, flo, beta, C, 64 * tau, dm, tau)
    s2, _ = _snr_allnonzero(orc, flo, beta, C, 128 * tau, dm, tau)
    slope = math.log(s2 / s1) / math.log(2.0)
    assert slope == pytest.approx(-0.5, rel=0.02)


def test_table1_coarse_frequency_slope(orc):
    # Coarse dnu, fine dt: S/N proportional to dnu^-1/2 (Table 1, bottom row).
    flo, beta, dm, tau, dt = 0.7, 0.3, 3000.0, 1e-3, 1e-5
    f = workloads.channel_centres(flo, beta, 300)
    d0 = orc.delta_nu0(f, tau, dm)
    C1 = int(round(beta / (64 * d0)))
    C2 = int(round(beta / (128 * d0)))
    s1, _ = _snr_allnonzero(orc, flo, beta, C1, dt, dm, tau)
    s2, _ = _snr_allnonzero(orc, flo, beta, C2, dt, dm, tau)
    slope = math.log(s2 / s1) / math.log((beta / C2) / (beta / C1))
    assert slope == pytest.approx(-0.5, rel=0.02)


def test_nominal_resolution_rule(orc):
    # dt = tau'_av and mean smear = tau'_av (m = 1 in the m-rule): S/N ~ SNR'_0 / sqrt(3)
    # and, at m = 0.25, better than 80 % of SNR'_0 (Section 3).  SNR'_0 = sqrt(beta tau)
    # for P0 = kT = 1, alpha = 0, no scattering.
    flo, beta, dm, tau = 0.7, 0.3, 300.0, 1e-3
    f = workloads.channel_centres(flo, beta, 300)
    d0 = orc.delta_nu0(f, tau, dm)
    for m in (1.0, 0.5, 0.25):
        C = int(round(beta / (m * d0)))
        s, _ = _snr_allnonzero(orc, flo, beta, C, m * tau, dm, tau)
        ratio = s / math.sqrt(beta * tau)
        assert ratio == pytest.approx(1 / math.sqrt(1 + 2 * m), rel=0.01)
        if m == SCALARS["m_rule_m"]:
            assert round(ratio, 2) == SCALARS["m_rule_fraction_2dp"]


# ------------------------------------------------------------ selection rule (Section 2.2)

def _exhaustive(values):
    best = -math.inf
    for k in range(1, len(values) + 1):
        for sub in itertools.combinations(values, k):
            best = max(best, sum(sub) / math.sqrt(k))
    return best


def test_best_prefix_is_exhaustive_optimum(orc):
    rng = np.random.default_rng(11)
    for _ in range(30):
        v = rng.exponential(1.0, size=int(rng.integers(1, 11)))
        assert orc.best_prefix(v)[1] == pytest.approx(_exhaustive(list(v)), rel=1e-12)


def test_greedy_selection_matches_optimum_on_unimodal(orc):
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(60):
        v = rng.exponential(1.0, size=int(rng.integers(2, 11)))
        srt = np.sort(v)[::-1]
        f = np.cumsum(srt) / np.sqrt(np.arange(1, len(v) + 1))
        if not np.all(np.diff(np.sign(np.diff(f))) <= 0):
            continue   # objective not unimodal in k
        sel = orc.greedy_select(v, np.zeros(len(v), int), np.arange(len(v)))
        got = float(np.sum(v[sel])) / math.sqrt(len(sel))
        assert got == pytest.approx(_exhaustive(list(v)), rel=1e-12)
        checked += 1
    assert checked > 10


def test_greedy_stops_at_first_local_maximum(orc):
    # The procedure adds samples only while eq. sel_criterion holds, so it can stop
    # before the global optimum: {10, 1 x 99} stops after one sample.
    v = np.array([10.0] + [1.0] * 99)
    sel = orc.greedy_select(v, np.zeros(100, int), np.arange(100))
    assert len(sel) == 1
    assert orc.best_prefix(v)[0] == 100


def test_greedy_criterion_equivalent_to_snr_increase(orc):
    # eq. rel_snr > 1 exactly when eq. sel_criterion holds.
    rng = np.random.default_rng(13)
    for _ in range(200):
        tot = rng.uniform(0.1, 10)
        N = int(rng.integers(1, 50))
        p = rng.uniform(0, 3)
        crit = p > (math.sqrt((N + 1) / N) - 1) * tot
        rel = (1 + p / tot) * math.sqrt(N / (N + 1))
        if abs(rel - 1) > 1e-12:
            assert crit == (rel > 1)


# ---------------------------------------------------------------- detectors (Section 4)

def test_detectors_agree_for_perfectly_dedispersed_pulse(orc):
    P = np.full((5, 16), 0.7)
    dt, dnu = 1e-3, 1e-3
    tardis = orc.snr_dedisp(P.ravel(), P.size, dt, dnu)
    assert orc.snr_mf(P, dt, dnu) == pytest.approx(tardis, rel=1e-12)
    assert orc.snr_dsmf(P, dt, dnu) == pytest.approx(tardis, rel=1e-12)
    assert orc.snr_bmf(P, dt, dnu) == pytest.approx(tardis, rel=1e-12)


def test_dsmf_bounds_every_sample_set(orc):
    # Cauchy-Schwarz: no unweighted subset sum beats the dynamic-spectrum matched filter.
    rng = np.random.default_rng(14)
    P = rng.exponential(1.0, size=(6, 10))
    dsmf = orc.snr_dsmf(P, 1e-3, 1e-3)
    for _ in range(200):
        mask = rng.random(P.shape) < rng.uniform(0.1, 1.0)
        if not mask.any():
            continue
        assert orc.snr_dedisp(P[mask], int(mask.sum()), 1e-3, 1e-3) <= dsmf * (1 + 1e-12)
