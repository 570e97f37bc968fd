"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and renders synthetic dynamic spectra.
It holds none of the dedisperser's arithmetic (no delay tables, no tap
counts, no sums, no S/N): both the HIP library and the CPU oracle receive the
arrays it returns as plain inputs.

The injected pulses follow the signal model of Section 2.1 of the paper
(eqs. intrinsic_power, P_obs and Pavg): a pulse profile f(t) with a power-law
spectrum, delayed by the cold-plasma law t_d = DM / (kappa nu^2), broadened by
a unit-area scattering response h_d, and averaged over each dt x dnu cell.
Here f is a Gaussian, h_d a one-sided exponential with tau_s(nu) proportional
to nu^-4, and the cell average is taken by a mid-point rule over sub-channel
frequencies and the exact time integral of the exponentially modified
Gaussian.  Spectral indices are given in the S ~ nu^alpha convention.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import special

# Physical dispersion constant of the signal model: t_d = DM / (kappa nu^2)
# with kappa = 2.41e-16 pc cm^-3 s (Section 2.1).  In seconds for nu in GHz.
SIGNAL_KDM_S = 1.0 / (2.41e-16 * 1e18)


def channel_centres(f_lo_ghz: float, bw_ghz: float, nchan: int) -> np.ndarray:
    """Centres of `nchan` contiguous channels of width `bw_ghz/nchan` above f_lo."""
    d = bw_ghz / nchan
    return f_lo_ghz + (np.arange(nchan, dtype=np.float64) + 0.5) * d


@dataclasses.dataclass
class Pulse:
    dm: float              # pc cm^-3
    t_arrival_s: float     # arrival time at the top of the band
    fwhm_s: float
    amp: float             # peak of the un-smeared profile, in data units, at nu_ref
    alpha: float = 0.0     # S ~ (nu/nu_ref)^alpha
    tau_1ghz_s: float = 0.0
    nu_ref_ghz: float = 1.0
    beam: int = 0


def _exgauss_cdf(x: np.ndarray, sig: float, tau: np.ndarray) -> np.ndarray:
    """CDF of N(0, sig^2) + Exp(mean tau), evaluated elementwise (tau may be 0)."""
    z = x / sig
    out = special.ndtr(z)
    tau = np.broadcast_to(tau, x.shape)
    m = tau > 0
    if np.any(m):
        lam = 1.0 / tau[m]
        xm = x[m]
        expo = -lam * xm + 0.5 * (lam * sig) ** 2 + special.log_ndtr((xm - lam * sig * sig) / sig)
        out = out.copy()
        out[m] = out[m] - np.exp(expo)
    return out


def render_pulse(freqs_ghz: np.ndarray, chan_bw_ghz: float, dt_s: float, nsamp: int,
                 p: Pulse, nsub: int = 8) -> tuple[np.ndarray, np.ndarray]:
    """Cell-averaged pulse power per channel.

    Returns (t_first[C] int64, cells[C, L] float64): channel c holds
    cells[c, j] at sample t_first[c] + j.  Cells outside [0, nsamp) are
    dropped by the caller.
    """
    C = freqs_ghz.shape[0]
    nu_hi = float(np.max(freqs_ghz) + 0.5 * chan_bw_ghz)
    sub = (np.arange(nsub) + 0.5) / nsub - 0.5
    nu = freqs_ghz[:, None] + sub[None, :] * chan_bw_ghz          # [C, J]
    delay = p.t_arrival_s + SIGNAL_KDM_S * p.dm * (nu ** -2 - nu_hi ** -2)
    tau = p.tau_1ghz_s * nu ** -4.0
    sig = p.fwhm_s / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    area = sig * math.sqrt(2.0 * math.pi)                           # of the peak-1 Gaussian
    spec = (nu / p.nu_ref_ghz) ** p.alpha
    t_lo = np.floor((delay.min(axis=1) - 7.0 * sig) / dt_s).astype(np.int64) - 1
    t_hi = np.ceil((delay.max(axis=1) + 7.0 * sig + 12.0 * tau.max(axis=1)) / dt_s).astype(np.int64) + 1
    L = int(np.max(t_hi - t_lo)) + 1
    ts = (t_lo[:, None] + np.arange(L)[None, :]).astype(np.float64) * dt_s   # [C, L]
    a = ts[:, None, :] - delay[:, :, None]                                   # [C, J, L]
    g0 = _exgauss_cdf(a, sig, np.broadcast_to(tau[:, :, None], a.shape))
    g1 = _exgauss_cdf(a + dt_s, sig, np.broadcast_to(tau[:, :, None], a.shape))
    cell = (g1 - g0) / dt_s * area * spec[:, :, None]
    cells = p.amp * cell.mean(axis=1)
    return t_lo, cells


def rect_pulse_cells(freqs_ghz: np.ndarray, chan_bw_ghz: float, dt_s: float, dm: float,
                     width_s: float, t_arrival_s: float, nsub: int = 32):
    """Noiseless dispersed rectangular pulse (power 1 while it lasts) as cell means: the
    cells (channel, sample, value) it touches.  Each channel is cut into `nsub` sub-bands;
    in sub-band nu the pulse occupies [d(nu), d(nu) + width) with d(nu) = t_arrival +
    K DM (nu^-2 - nu_top^-2), nu_top the top of the band; a cell holds the mean over
    sub-bands of the fraction of [n dt, (n + 1) dt) it occupies.  Entries may repeat a
    cell (add them)."""
    C = freqs_ghz.shape[0]
    nu_top = float(np.max(freqs_ghz) + 0.5 * chan_bw_ghz)
    sub = (np.arange(nsub) + 0.5) / nsub - 0.5
    nu = freqs_ghz[:, None] + sub[None, :] * chan_bw_ghz                 # [C, J]
    d0 = t_arrival_s + SIGNAL_KDM_S * dm * (nu ** -2 - nu_top ** -2)     # pulse start
    d1 = d0 + width_s
    L = int(math.ceil(width_s / dt_s)) + 2
    n = np.floor(d0 / dt_s).astype(np.int64)[:, :, None] + np.arange(L)[None, None, :]
    lo = np.maximum(n * dt_s, d0[:, :, None])
    hi = np.minimum((n + 1) * dt_s, d1[:, :, None])
    frac = np.clip(hi - lo, 0.0, None) / dt_s / nsub                     # [C, J, L]
    cc = np.broadcast_to(np.arange(C)[:, None, None], n.shape)
    keep = frac > 0.0
    return cc[keep], n[keep], frac[keep]


def render_rect_pulse(freqs_ghz: np.ndarray, chan_bw_ghz: float, dt_s: float, nsamp: int,
                      dm: float, width_s: float, t_arrival_s: float, nsub: int = 32) -> np.ndarray:
    """rect_pulse_cells as a dense fp32 block [C, nsamp] (cells outside it dropped)."""
    c, n, v = rect_pulse_cells(freqs_ghz, chan_bw_ghz, dt_s, dm, width_s, t_arrival_s, nsub)
    x = np.zeros((freqs_ghz.shape[0], nsamp), dtype=np.float64)
    ok = (n >= 0) & (n < nsamp)
    np.add.at(x, (c[ok], n[ok]), v[ok])
    return x.astype(np.float32)


def add_pulse(x: np.ndarray, freqs_ghz: np.ndarray, chan_bw_ghz: float, dt_s: float, p: Pulse) -> None:
    """Add a rendered pulse in place into a float array x[C, T]."""
    C, T = x.shape
    t0, cells = render_pulse(freqs_ghz, chan_bw_ghz, dt_s, T, p)
    L = cells.shape[1]
    for c in range(C):
        a = int(t0[c])
        lo, hi = max(a, 0), min(a + L, T)
        if hi > lo:
            x[c, lo:hi] += cells[c, lo - a:hi - a]


def quantise_u8(xf: np.ndarray, mean: float = 128.0) -> np.ndarray:
    """clip(rint(mean + x), 0, 255) with round-half-even, as uint8."""
    return np.clip(np.rint(mean + xf), 0, 255).astype(np.uint8)


def u8_noise(rng: np.random.Generator, C: int, T: int, sigma: float = 16.0,
             block: int = 256) -> np.ndarray:
    """Quantised Gaussian noise N(128, sigma^2) as uint8, drawn in channel blocks."""
    out = np.empty((C, T), dtype=np.uint8)
    for c0 in range(0, C, block):
        c1 = min(C, c0 + block)
        z = rng.standard_normal((c1 - c0, T), dtype=np.float32)
        out[c0:c1] = np.clip(np.rint(128.0 + sigma * z), 0, 255).astype(np.uint8)
    return out


# ----------------------------------------------------------------------------------
# The five workloads.  Sizes, seeds and pulse recipes are fixed here; tests may
# shrink T or D explicitly through the keyword arguments.
# ----------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    freqs_ghz: np.ndarray
    chan_bw_ghz: float
    dt_s: float
    dms: np.ndarray
    widths: np.ndarray
    x: Optional[np.ndarray]
    pulses: list
    chan_mean: np.ndarray
    chan_sigma: np.ndarray
    rule: str
    weights: Optional[np.ndarray] = None
    extra: dict = dataclasses.field(default_factory=dict)


def cfg1(nsamp: int = 4096) -> Workload:
    """64 channels over 1.2-1.5 GHz, 1 ms, uint8 noise N(128,16^2), one 2 ms pulse at DM 100."""
    rng = np.random.default_rng(13011)
    C = 64
    f = channel_centres(1.2, 0.3, C)
    bw = 0.3 / C
    dt = 1e-3
    noise = 16.0 * rng.standard_normal((C, nsamp))
    p = Pulse(dm=100.0, t_arrival_s=2.0 * (nsamp / 4096.0), fwhm_s=2e-3, amp=128.0)
    add_pulse(noise, f, bw, dt, p)
    x = quantise_u8(noise)
    return Workload("cfg1_64ch_32dm", f, bw, dt, np.arange(32, dtype=np.float64) * 10.0,
                    np.array([1, 2, 4, 8], dtype=np.int32), x, [p],
                    np.full(C, 128.0), np.full(C, 16.0), "smear")


def cfg2(nsamp: int = 65536, ndm: int = 1024, rule: str = "allnonzero") -> Workload:
    """336 x 1 MHz channels at 1.2-1.536 GHz, 1 ms, 65536 uint8 samples, 16 pulses, 1024 DMs."""
    rng = np.random.default_rng(13012)
    C = 336
    f = channel_centres(1.2, 0.336, C)
    bw = 0.001
    dt = 1e-3
    noise = np.empty((C, nsamp), dtype=np.float64)
    for c0 in range(0, C, 64):
        c1 = min(C, c0 + 64)
        noise[c0:c1] = 16.0 * rng.standard_normal((c1 - c0, nsamp))
    dms = rng.uniform(50.0, 1900.0, size=16)
    pulses = []
    for i in range(16):
        t_arr = (512 + 4096 * i) * 1e-3
        if t_arr * 1e3 + 2500 > nsamp:
            continue
        p = Pulse(dm=float(dms[i]), t_arrival_s=t_arr, fwhm_s=(i + 1) * 1e-3, amp=16.0,
                  tau_1ghz_s=1e-3)
        add_pulse(noise, f, bw, dt, p)
        pulses.append(p)
    x = quantise_u8(noise)
    return Workload("cfg2_336ch_1024dm", f, bw, dt, np.linspace(0.0, 2000.0, ndm),
                    np.arange(1, 33, dtype=np.int32), x, pulses,
                    np.full(C, 128.0), np.full(C, 16.0), rule)


def cfg3(nsamp: int = 262144, ndm: int = 4096, nchan: int = 4096) -> Workload:
    """4096 channels over 1.2-1.5 GHz, 64 us, uint8 noise; fp32 weights (f/1.35 GHz)^-1.5."""
    rng = np.random.default_rng(13013)
    C = nchan
    f = channel_centres(1.2, 0.3, C)
    bw = 0.3 / C
    dt = 64e-6
    x = u8_noise(rng, C, nsamp)
    w = ((f / 1.35) ** -1.5).astype(np.float32)
    return Workload("cfg3_4096ch_4096dm_f32w", f, bw, dt, np.linspace(0.0, 1000.0, ndm),
                    np.arange(1, 33, dtype=np.int32), x, [], np.full(C, 128.0), np.full(C, 16.0),
                    "smear", weights=w)


def cfg4_beams(nbeam: int = 36, tmin: int = 16384, tmax: int = 131072,
               nmin: int = 300, nmax: int = 1200) -> dict:
    """Per-beam lengths and DM-grid sizes for the batched workload (seed 13014)."""
    rng = np.random.default_rng(13014)
    T = rng.integers(tmin, tmax + 1, size=nbeam)
    N = rng.integers(nmin, nmax + 1, size=nbeam)
    return {"nsamp": T.astype(np.int64), "ntrial": N.astype(np.int64)}


def cfg4_beam_data(b: int, nsamp: int, dm_lo: float, dm_hi: float, C: int = 336) -> tuple:
    """uint8 noise for beam b plus one 4 ms pulse at a DM inside [dm_lo, dm_hi] (seed 13014*1000+b)."""
    rng = np.random.default_rng(13014 * 1000 + b)
    f = channel_centres(1.2, 0.336, C)
    bw = 0.001
    dt = 1e-3
    noise = 16.0 * rng.standard_normal((C, nsamp))
    dm = float(rng.uniform(dm_lo, dm_hi))
    t_arr = float(rng.uniform(0.1, 0.5)) * nsamp * dt
    p = Pulse(dm=dm, t_arrival_s=t_arr, fwhm_s=4e-3, amp=16.0, tau_1ghz_s=1e-3, beam=b)
    add_pulse(noise, f, bw, dt, p)
    return quantise_u8(noise), p


def cfg5(batch: int = 64, nsamp: int = 32768, ndm: int = 256, ktaps: int = 8,
         nchan: int = 336) -> Workload:
    """Batch of fp32 N(0,1) filterbanks with one pulse each, for the learnable tap weights."""
    rng = np.random.default_rng(13015)
    C = nchan
    f = channel_centres(1.2, 0.336, C)
    bw = 0.001
    dt = 1e-3
    x = np.empty((batch, C, nsamp), dtype=np.float32)
    dms = np.linspace(0.0, 1000.0, ndm)
    pulses = []
    w0 = (1.0 + 0.1 * rng.standard_normal((C, ktaps))).astype(np.float32)
    # Output length bound used to place pulses: the largest sweep over the band at DM 1000.
    sweep = int(math.ceil(SIGNAL_KDM_S * 1000.0 * (1.2 ** -2 - 1.536 ** -2) / dt)) + ktaps
    tout_est = nsamp - sweep
    for b in range(batch):
        xb = rng.standard_normal((C, nsamp)).astype(np.float64)
        d_idx = int(rng.integers(0, ndm))
        lo, hi = 2048, max(2049, tout_est - 2048)
        if hi <= lo:
            lo, hi = 0, max(1, tout_est)
        t_b = int(rng.integers(lo, hi))
        p = Pulse(dm=float(dms[d_idx]), t_arrival_s=t_b * dt, fwhm_s=float(rng.uniform(1e-3, 8e-3)),
                  amp=0.5, alpha=float(rng.uniform(-2.0, 1.0)),
                  tau_1ghz_s=float(rng.uniform(0.0, 4e-3)), nu_ref_ghz=1.368, beam=b)
        add_pulse(xb, f, bw, dt, p)
        x[b] = xb.astype(np.float32)
        pulses.append((p, d_idx, t_b))
    return Workload("cfg5_b64_336ch_256dm_k8", f, bw, dt, dms, np.arange(1, 9, dtype=np.int32),
                    x, pulses, np.zeros(C), np.ones(C), "explicit", weights=w0,
                    extra={"ktaps": ktaps})
