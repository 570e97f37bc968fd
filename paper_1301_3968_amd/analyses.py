"""The paper's own analyses run through the library: the trial-DM completeness
curves (Section 5.3), the dedispersed profiles of test pulses with a DM error
(Sections 5.1-5.2), the peak S/N over time and frequency resolution and the detector
comparison (Section 4).

Each function renders noiseless rectangular test pulses with the `workloads` module
it is given (seeded inputs, no method arithmetic), dedisperses them with the library
(every sum on the GPU) and reads the S/N off the dedispersed series; only the
normalisation of the S/N and the choice of the best trial are done here on the host.
"""
from __future__ import annotations

import math
import time

import numpy as np


# Survey examples of Section 5.3: (name, band low edge GHz, bandwidth GHz, channels, dt s,
# test pulse width s, DM range, DM error factor).
COMPLETENESS_CASES = [
    ("700-1004 MHz, 304 x 1 MHz, 1 ms, 1 ms pulse", 0.700, 0.304, 304, 1e-3, 1e-3, 10.0, 3000.0, 1.492),
    ("21-23 GHz, 256 x 7.8125 MHz, 100 us, 100 us pulse", 21.0, 2.0, 256, 1e-4, 1e-4, 50.0, 10000.0, 0.580),
    ("21-23 GHz, 32 x 62.5 MHz, 100 us, 100 us pulse", 21.0, 2.0, 32, 1e-4, 1e-4, 50.0, 10000.0, 0.287),
]


def completeness_case(dd, workloads, case, true_dms, chunk=64, lead=64, dms=None):
    """Largest S/N over the trial DMs (eq. trial DMs) for a noiseless rectangular test pulse
    at each true DM, normalised to P0 sqrt(beta tau) / k T_sys (Section 5.3): greedy sample
    sets (Section 2.2) per trial, batched fp32 dedispersion, per-trial S/N at width 1 with
    unit noise per sample, largest over the trials on the host.  Returns (plan, S/N [n],
    best trial [n], per-trial S/N [n][D], seconds).  dms: the trial DMs (default: the
    library's eq. trial DMs for the case)."""
    import torch
    _, flo, band, C, dt, tau, lo, hi, eps = case
    f = workloads.channel_centres(flo, band, C)
    bw = band / C
    if dms is None:
        dms = dd.trial_dms(lo, hi, eps, f, bw, dt, cap=100000)
    plan = dd.Plan(f, bw, dt, dms, rule="greedy", width_s=tau)
    T = plan.max_span + 2 * lead
    D = len(dms)
    mean, sig = np.zeros(C), np.ones(C)
    work = torch.empty(plan.work_bytes(T, 1), dtype=torch.uint8, device="cuda")
    snr_all = np.empty((len(true_dms), D))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i0 in range(0, len(true_dms), chunk):
        dm_c = true_dms[i0:i0 + chunk]
        x = torch.zeros((len(dm_c), C, T), dtype=torch.float32, device="cuda")
        for b, dm in enumerate(dm_c):
            c, n, v = workloads.rect_pulse_cells(f, bw, dt, float(dm), tau, lead * dt)
            ok = (n >= 0) & (n < T)
            idx = torch.from_numpy(c[ok] * T + n[ok]).cuda()
            x[b].view(-1).index_put_((idx,), torch.from_numpy(v[ok].astype(np.float32)).cuda(),
                                     accumulate=True)
        y = plan.dedisperse(x)
        for b in range(len(dm_c)):
            snr, _, _ = plan.detect(y[b], [1], mean, sig, work=work)
            snr_all[i0 + b] = snr.cpu().numpy()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    norm = math.sqrt(dt / (C * tau))
    best = snr_all.max(axis=1) * norm
    return plan, best, snr_all.argmax(axis=1), snr_all * norm, secs


# Section 5.1 example: 700-1004 MHz, 1 MHz channels, 1 ms, 1 ms rectangular pulse, trial DM 30.
DM_ERROR_CASE = (0.700, 0.304, 304, 1e-3, 1e-3, 30.0)
KDM_S = 1.0 / (2.41e-16 * 1e18)     # dispersion constant, s GHz^2 / (pc cm^-3)


def dm_error_unit(case=DM_ERROR_CASE):
    """The DM-error unit of Section 5.2: (1/C) sqrt(DM^2 + DM_diag^2 + DM_tau^2), with DM_diag
    and DM_tau the DMs whose mean channel smearing equals dt and the pulse width."""
    flo, band, C, dt, tau, dm = case
    f = np.linspace(flo, flo + band, C, endpoint=False) + 0.5 * band / C
    bw = band / C
    inv3 = float(np.mean(f ** -3.0))
    dm_diag = dt / (2.0 * KDM_S * bw * inv3)
    dm_tau = tau / (2.0 * KDM_S * bw * inv3)
    return math.sqrt(dm * dm + dm_diag * dm_diag + dm_tau * dm_tau) / C


def dm_error_profiles(dd, workloads, xs, case=DM_ERROR_CASE, lead=64):
    """Dedispersed profiles (eq. rel_snr2) of rectangular test pulses at DM = trial + x units
    of DM error, through the greedy sample set of the trial DM: batched fp32 dedispersion
    of the rendered pulses.  Returns (plan, profiles [len(xs)][nout] relative to the
    matched pulse's peak, seconds)."""
    import torch
    flo, band, C, dt, tau, dm = case
    f = workloads.channel_centres(flo, band, C)
    bw = band / C
    plan = dd.Plan(f, bw, dt, [dm], rule="greedy", width_s=tau)
    T = plan.max_span + 2 * lead
    unit = dm_error_unit(case)
    dms = [dm] + [dm + float(x) * unit for x in xs]
    x = torch.zeros((len(dms), C, T), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, d in enumerate(dms):
        c, n, v = workloads.rect_pulse_cells(f, bw, dt, d, tau, lead * dt)
        ok = (n >= 0) & (n < T)
        idx = torch.from_numpy(c[ok] * T + n[ok]).cuda()
        x[b].view(-1).index_put_((idx,), torch.from_numpy(v[ok].astype(np.float32)).cuda(),
                                 accumulate=True)
    y = plan.dedisperse(x)[:, 0, :].cpu().numpy().astype(np.float64)
    secs = time.perf_counter() - t0
    return plan, y[1:] / y[0].max(), secs


# Section 4 example: 700 MHz - 1 GHz, 1 ms rectangular pulse, DM 30, no scattering.
RES_BAND = (0.700, 0.300)
RES_TAU, RES_DM = 1e-3, 30.0


def res_delta_nu0(band=RES_BAND, tau=RES_TAU, dm=RES_DM):
    """The channel width whose intra-channel smearing equals the pulse width, with the
    band-averaged nu^-3 (GHz)."""
    lo, bw = band
    inv3 = (lo ** -2 - (lo + bw) ** -2) / (2.0 * bw)       # mean of nu^-3 over the band
    return tau / (2.0 * KDM_S * dm * inv3)


def resolution_point(dd, workloads, a, b, rule, band=RES_BAND, tau=RES_TAU, dm=RES_DM, lead=16):
    """Peak dedispersed S/N (normalised to P0 sqrt(beta tau) / k T_sys) of the test pulse at
    time resolution a tau and channel width b dnu_0 (channel count rounded), sample sets by
    `rule`: fp32 dedispersion of one trial on the GPU.  Returns (S/N, plan, dt, channel
    width, rendered block)."""
    import torch
    lo, bw = band
    C = max(1, int(round(bw / (b * res_delta_nu0(band, tau, dm)))))
    cw = bw / C
    dt = a * tau
    f = workloads.channel_centres(lo, bw, C)
    plan = dd.Plan(f, cw, dt, [dm], rule=rule, width_s=tau)
    T = plan.max_span + 2 * lead
    x = workloads.render_rect_pulse(f, cw, dt, T, dm, tau, lead * dt)
    y = plan.dedisperse(torch.from_numpy(x).cuda())[0].cpu().numpy().astype(np.float64)
    _, n = plan.tables()
    snr = y.max() / math.sqrt(float(n.sum())) * math.sqrt(dt / (C * tau))
    return snr, plan, dt, cw, x


def detector_snrs(dd, workloads, b, band=RES_BAND, tau=RES_TAU, dm=RES_DM, lead=16, a=1.0,
                  series=None):
    """Section 4 detectors for the rendered test pulse at channel width b dnu_0 and dt = tau,
    each as a dedispersion of the block at the pulse's DM on the GPU (normalised to
    P0 sqrt(beta tau) / k T_sys, unit noise per sample): the dynamic-spectrum matched filter
    (tap weights = the pulse's own cells P), the time-series matched filter (every
    channel weighted by the channel sum of P at each tap), the time-series boxcar (unit
    weights over the pulse's dedispersed width in every channel) and the greedy detector
    (Section 2.2 sample set).  The sample time is a tau.  Returns ({name: S/N}, P [C][K],
    dt, channel width); when `series` is a dict it receives each detector's dedispersed
    series (before normalisation)."""
    import torch
    lo, bw = band
    C = max(1, int(round(bw / (b * res_delta_nu0(band, tau, dm)))))
    cw, dt = bw / C, a * tau
    f = workloads.channel_centres(lo, bw, C)
    p0 = dd.Plan(f, cw, dt, [dm], rule="allnonzero", width_s=tau)
    s0, n0 = p0.tables()
    K = int(n0.max())
    T = p0.max_span + K + 2 * lead
    x = workloads.render_rect_pulse(f, cw, dt, T, dm, tau, lead * dt)
    xd = torch.from_numpy(x).cuda()
    idx = lead + s0[0][:, None] + np.arange(K)[None, :]
    P = x[np.arange(C)[:, None], idx].astype(np.float64)        # [C][K] cells of the pulse
    norm = math.sqrt(dt / (C * tau))
    start = s0.copy()
    full = np.full((1, C), K, dtype=np.int32)

    def weighted(w):
        p = dd.Plan(f, cw, dt, [dm], rule="explicit", start=start, ntap=full, ktaps=K,
                    wmode="tap", weights=w.astype(np.float32))
        y = p.dedisperse(xd)[0].cpu().numpy().astype(np.float64)
        w32 = w.astype(np.float32).astype(np.float64)
        return y, y.max() / math.sqrt(float(np.sum(w32 ** 2))) * norm

    ys = {}
    out = {}
    ys["dsmf"], out["dsmf"] = weighted(P)
    prof = P.sum(axis=0)                                         # channel sum per tap
    ys["mf"], out["mf"] = weighted(np.broadcast_to(prof, (C, K)).copy())
    nt = int(np.count_nonzero(prof > 0.0))
    nts = np.full((1, C), nt, dtype=np.int32)
    first = int(np.argmax(prof > 0.0))
    pb = dd.Plan(f, cw, dt, [dm], rule="explicit", start=start + first, ntap=nts)
    yb = pb.dedisperse(xd)[0].cpu().numpy().astype(np.float64)
    out["boxcar"] = yb.max() / math.sqrt(float(C * nt)) * norm
    pg = dd.Plan(f, cw, dt, [dm], rule="greedy", width_s=tau)
    yg = pg.dedisperse(xd)[0].cpu().numpy().astype(np.float64)
    out["greedy"] = yg.max() / math.sqrt(float(pg.tables()[1].sum())) * norm
    if series is not None:
        series.update(ys, boxcar=yb, greedy=yg)
    return out, P, dt, cw
