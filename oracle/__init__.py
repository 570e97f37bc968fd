"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU implementation of what the dedispersion
library computes, written from the paper (Clarke, Macquart & Trott,
"Performance of a novel fast transients detection system").  Only `tests/`,
`__graft_entry__.smoke()` and the benchmark's CPU-baseline leg may import it;
the HIP library never does, and the two share no code.

Heavy loops (the dedispersion sum, the boxcar search and the adjoints) live in
`oracle.c` and run in int64 / double precision; table construction, the
trial-DM rule, the sample-selection rule and the closed forms are numpy /
Python in double precision.  Every function cites the passage it follows.

Parity status: every function here is pinned by a `-m "not gpu"` test
(tests/test_oracle_*.py) against a closed form, a library routine, a number
the paper prints, an invariant, or brute force.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

# Section 2.1: t_d = DM / (kappa nu^2), kappa = 2.41e-16 pc cm^-3 s.  With nu in
# GHz and t in seconds the delay constant is 1 / (kappa * 1e18).
KAPPA = 2.41e-16
KDM_PAPER = 1.0 / (KAPPA * 1e18)          # s GHz^2 cm^3 / pc  (= 4.149378e-3)
KDM_415 = 4.15e-3                          # the rounded constant, also supported


_SAN_LIB_PATH = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no FMA contraction); with sanitize,
    into liboracle_san.so with clang's AddressSanitizer and UndefinedBehaviorSanitizer
    (for runs that preload that runtime)."""
    if sanitize:
        clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
        subprocess.check_call([clang, "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-shared-libsan", "-fPIC", "-shared", "-o", _SAN_LIB_PATH, _SRC,
                               "-lm"])
        return _SAN_LIB_PATH
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", _LIB_PATH, _SRC, "-lm"])
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB")   # another build of oracle.c (the sanitized one)
        if not path:
            if not os.path.exists(_LIB_PATH):
                build(force=True)
            path = _LIB_PATH
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, ci = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
        L.oracle_dedisperse_u8.argtypes = [i32, i64, P, i64, i32, P, P, i64, P, i64]
        L.oracle_dedisperse_f64.argtypes = [i32, i32, i64, P, ci, i64, i64, i32, P, P, ci, i32, P,
                                            i64, P, i64, i64]
        L.oracle_boxcar_norm.argtypes = [i32, i32, P, ci, i32, P, P, P, i32, P, P, P]
        L.oracle_boxcar_detect.argtypes = [i32, i64, P, i64, i32, P, P, P, P, P, P]
        L.oracle_boxcar_detect.restype = None
        L.oracle_adjoint_w.argtypes = [i32, i32, i64, P, ci, i64, i64, i32, P, P, ci, i32, i64, P,
                                       i64, i64, P]
        L.oracle_adjoint_x.argtypes = [i32, i32, i64, i32, P, P, ci, i32, P, i64, P, i64, i64, P,
                                       i64, i64]
        L.oracle_dedisperse_points.argtypes = [i32, i64, P, ci, i64, i64, P, P, ci, i32, P, i32, P,
                                               P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


_DT = {np.dtype(np.uint8): 0, np.dtype(np.float32): 1, np.dtype(np.float64): 2,
       np.dtype(np.int32): 3}
_WMODE = {"unit": 0, "channel": 1, "tap": 2}


# ---------------------------------------------------------------------------------
# Channel geometry and the sample-set tables
# ---------------------------------------------------------------------------------

def channel_edges(freqs_ghz: np.ndarray, bw_ghz: float):
    """Top and bottom edges of each channel and the top of the band."""
    f = np.asarray(freqs_ghz, dtype=np.float64)
    ft = f + 0.5 * bw_ghz
    fl = f - 0.5 * bw_ghz
    fh = float(np.max(ft))
    return ft, fl, fh


def delay_start(freqs_ghz, bw_ghz, dt_s, dms, kdm=KDM_PAPER) -> np.ndarray:
    """start[d,c] = floor(t_A / dt), t_A = K DM (nu_top,c^-2 - nu_hi^-2).

    t_A is the earliest arrival of the pulse in channel c relative to the top of
    the band: the delay law of Section 2.1 at the channel's highest frequency
    (Section 3, definition of t_A)."""
    ft, fl, fh = channel_edges(freqs_ghz, bw_ghz)
    dm = np.asarray(dms, dtype=np.float64)[:, None]
    ta = kdm * dm * (1.0 / (ft * ft) - 1.0 / (fh * fh))[None, :] / dt_s
    return np.floor(ta).astype(np.int64)


def taps_smear(freqs_ghz, bw_ghz, dt_s, dms, kdm=KDM_PAPER) -> np.ndarray:
    """n[d,c] = max(1, ceil(intra-channel smear / dt)); the smear is the delay
    difference across the channel, K DM (nu_lo^-2 - nu_top^-2) (Section 3,
    Delta tau_c, taken between the two channel edges)."""
    ft, fl, fh = channel_edges(freqs_ghz, bw_ghz)
    dm = np.asarray(dms, dtype=np.float64)[:, None]
    sm = kdm * dm * (1.0 / (fl * fl) - 1.0 / (ft * ft))[None, :] / dt_s
    return np.maximum(1, np.ceil(sm)).astype(np.int64)


def pulse_width_at(f_ghz, width_s, scatter_1ghz_s, scatter_index):
    """Scatter-broadened width tau'(nu) = tau + tau_s,1GHz * nu^index (rectangle model, App. A)."""
    return width_s + scatter_1ghz_s * np.power(np.asarray(f_ghz, dtype=np.float64), scatter_index)


def taps_allnonzero(freqs_ghz, bw_ghz, dt_s, dms, width_s=0.0, scatter_1ghz_s=0.0,
                    scatter_index=-4.0, kdm=KDM_PAPER) -> np.ndarray:
    """eq. num_samples: every sample with non-zero pulse power.

    n[d,c] = max(1, ceil(t_B/dt) - floor(t_A/dt)) with t_A at the channel's top
    edge and t_B = K DM (nu_lo^-2 - nu_hi^-2) + tau'(nu_lo), the latest arrival
    of the pulse's trailing edge in the channel (the low edge, where both the
    delay and the scatter tail are largest).  The max(1, .) keeps one sample when
    t_A = t_B falls on a sample boundary (DM = 0 and tau' = 0)."""
    ft, fl, fh = channel_edges(freqs_ghz, bw_ghz)
    dm = np.asarray(dms, dtype=np.float64)[:, None]
    ta = kdm * dm * (1.0 / (ft * ft) - 1.0 / (fh * fh))[None, :] / dt_s
    taup = pulse_width_at(fl, width_s, scatter_1ghz_s, scatter_index)[None, :]
    tb = (kdm * dm * (1.0 / (fl * fl) - 1.0 / (fh * fh))[None, :] + taup) / dt_s
    return np.maximum(1, np.ceil(tb) - np.floor(ta)).astype(np.int64)


def out_len(nsamp: int, start: np.ndarray, ntap: np.ndarray) -> int:
    """Valid outputs of eq. p_dedisp for a finite block: T - max(start + ntap) + 1."""
    return int(nsamp - int(np.max(start + ntap)) + 1)


# ---------------------------------------------------------------------------------
# The dedispersion sum, the boxcar detector, the adjoints
# ---------------------------------------------------------------------------------

def dedisperse_u8(x: np.ndarray, start: np.ndarray, ntap: np.ndarray,
                  tout: Optional[int] = None) -> np.ndarray:
    """eq. p_dedisp with unit weights on uint8 data, int64 result [D, tout]."""
    x = np.ascontiguousarray(x, dtype=np.uint8)
    C, T = x.shape
    s = np.ascontiguousarray(start, dtype=np.int32)
    n = np.ascontiguousarray(ntap, dtype=np.int32)
    D = s.shape[0]
    if tout is None:
        tout = out_len(T, s, n)
    y = np.empty((D, tout), dtype=np.int64)
    rc = lib().oracle_dedisperse_u8(C, T, _p(x), T, D, _p(s), _p(n), tout, _p(y), tout)
    if rc != 0:
        raise ValueError("sample index outside the input block")
    return y


def dedisperse_f64(x: np.ndarray, start: np.ndarray, ntap: np.ndarray, wmode: str = "unit",
                   w: Optional[np.ndarray] = None, tout: Optional[int] = None) -> np.ndarray:
    """eq. p_dedisp with per-channel or per-tap weights in double precision.

    x is [C, T] or [B, C, T] (uint8, fp32 or fp64); returns [D, tout] or [B, D, tout]."""
    squeeze = x.ndim == 2
    xb = x[None] if squeeze else x
    xb = np.ascontiguousarray(xb)
    B, C, T = xb.shape
    s = np.ascontiguousarray(start, dtype=np.int32)
    n = np.ascontiguousarray(ntap, dtype=np.int32)
    D = s.shape[0]
    if tout is None:
        tout = out_len(T, s, n)
    K = 1
    if w is None:
        wa = np.zeros(1, dtype=np.float32)
    else:
        wa = np.ascontiguousarray(w, dtype=np.float32)
        if wmode == "tap":
            K = wa.shape[-1]
    y = np.empty((B, D, tout), dtype=np.float64)
    rc = lib().oracle_dedisperse_f64(B, C, T, _p(xb), _DT[xb.dtype], T, C * T, D, _p(s), _p(n),
                                     _WMODE[wmode], K, _p(wa), tout, _p(y), tout, D * tout)
    if rc != 0:
        raise ValueError("sample index outside the input block")
    return y[0] if squeeze else y


def dedisperse_points(x: np.ndarray, start, ntap, b, d, t, wmode: str = "unit",
                      w: Optional[np.ndarray] = None) -> np.ndarray:
    """eq. p_dedisp evaluated at selected outputs (b_e, d_e, t_e) only, in double."""
    xb = np.ascontiguousarray(x[None] if x.ndim == 2 else x)
    B, C, T = xb.shape
    s = np.ascontiguousarray(start, dtype=np.int32)
    n = np.ascontiguousarray(ntap, dtype=np.int32)
    pb = np.ascontiguousarray(b, dtype=np.int32)
    pd = np.ascontiguousarray(d, dtype=np.int32)
    pt = np.ascontiguousarray(t, dtype=np.int64)
    K = 1
    if w is None:
        wa = np.zeros(1, dtype=np.float32)
    else:
        wa = np.ascontiguousarray(w, dtype=np.float32)
        if wmode == "tap":
            K = wa.shape[-1]
    out = np.empty(pd.shape[0])
    rc = lib().oracle_dedisperse_points(C, T, _p(xb), _DT[xb.dtype], T, C * T, _p(s), _p(n),
                                        _WMODE[wmode], K, _p(wa), pd.shape[0], _p(pb), _p(pd),
                                        _p(pt), _p(out))
    if rc != 0:
        raise ValueError("sample index outside the input block")
    return out


def boxcar_norm(ntap: np.ndarray, widths: Sequence[int], mu: np.ndarray, sigma: np.ndarray,
                wmode: str = "unit", w: Optional[np.ndarray] = None):
    """Mean and standard deviation of every width-W boxcar of every trial's series
    under independent channel noise (eqs. P_N_dedisp and snr, extended to W
    consecutive outputs): M, S of shape [D, nW]."""
    n = np.ascontiguousarray(ntap, dtype=np.int32)
    D, C = n.shape
    wd = np.ascontiguousarray(widths, dtype=np.int32)
    K = 1
    if w is None:
        wa = np.zeros(1, dtype=np.float32)
    else:
        wa = np.ascontiguousarray(w, dtype=np.float32)
        if wmode == "tap":
            K = wa.shape[-1]
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    M = np.empty((D, wd.shape[0]))
    S = np.empty((D, wd.shape[0]))
    rc = lib().oracle_boxcar_norm(C, D, _p(n), _WMODE[wmode], K, _p(wa), _p(mu), _p(sg),
                                  wd.shape[0], _p(wd), _p(M), _p(S))
    if rc != 0:
        raise MemoryError
    return M, S


def boxcar_detect(y: np.ndarray, widths: Sequence[int], M: np.ndarray, S: np.ndarray):
    """Per trial, the best boxcar S/N = (B - M)/S over all widths and start times,
    with ties to the smaller width then the earlier start.  Returns (snr, t, W)."""
    yd = np.ascontiguousarray(y, dtype=np.float64)
    D, tout = yd.shape
    wd = np.ascontiguousarray(widths, dtype=np.int32)
    Mc = np.ascontiguousarray(M, dtype=np.float64)
    Sc = np.ascontiguousarray(S, dtype=np.float64)
    snr = np.empty(D)
    t = np.empty(D, dtype=np.int32)
    W = np.empty(D, dtype=np.int32)
    lib().oracle_boxcar_detect(D, tout, _p(yd), tout, wd.shape[0], _p(wd), _p(Mc), _p(Sc),
                               _p(snr), _p(t), _p(W))
    return snr, t, W


def adjoint_w(x: np.ndarray, start, ntap, g: np.ndarray, wmode: str = "tap", ktaps: int = 1):
    """Gradient of <g, y> with respect to the weights (transpose of eq. p_dedisp in w)."""
    xb = np.ascontiguousarray(x[None] if x.ndim == 2 else x)
    gb = np.ascontiguousarray(g[None] if g.ndim == 2 else g, dtype=np.float64)
    B, C, T = xb.shape
    s = np.ascontiguousarray(start, dtype=np.int32)
    n = np.ascontiguousarray(ntap, dtype=np.int32)
    D, tout = gb.shape[1], gb.shape[2]
    K = ktaps if wmode == "tap" else 1
    gw = np.empty((C, K))
    rc = lib().oracle_adjoint_w(B, C, T, _p(xb), _DT[xb.dtype], T, C * T, D, _p(s), _p(n),
                                _WMODE[wmode], K, tout, _p(gb), tout, D * tout, _p(gw))
    if rc != 0:
        raise ValueError("sample index outside the input block")
    return gw if wmode == "tap" else gw[:, 0]


def adjoint_x(nsamp: int, start, ntap, g: np.ndarray, wmode: str = "unit",
              w: Optional[np.ndarray] = None):
    """Gradient of <g, y> with respect to the input samples (transpose of eq. p_dedisp in x)."""
    squeeze = g.ndim == 2
    gb = np.ascontiguousarray(g[None] if squeeze else g, dtype=np.float64)
    B, D, tout = gb.shape
    s = np.ascontiguousarray(start, dtype=np.int32)
    n = np.ascontiguousarray(ntap, dtype=np.int32)
    C = s.shape[1]
    K = 1
    if w is None:
        wa = np.zeros(1, dtype=np.float32)
    else:
        wa = np.ascontiguousarray(w, dtype=np.float32)
        if wmode == "tap":
            K = wa.shape[-1]
    gx = np.empty((B, C, nsamp))
    rc = lib().oracle_adjoint_x(B, C, nsamp, D, _p(s), _p(n), _WMODE[wmode], K, _p(wa), tout,
                                _p(gb), tout, D * tout, _p(gx), nsamp, C * nsamp)
    if rc != 0:
        raise ValueError("sample index outside the input block")
    return gx[0] if squeeze else gx


# ---------------------------------------------------------------------------------
# Trial-DM selection (Section 5.3) and the smearing constants it uses
# ---------------------------------------------------------------------------------

def mean_inv_cube(freqs_ghz) -> float:
    """[ (1/C) sum_c nu_c^-3 ] with nu_c the channel centres (GHz)."""
    f = np.asarray(freqs_ghz, dtype=np.float64)
    return float(np.mean(f ** -3))


def dm_diag(freqs_ghz, bw_ghz, dt_s, kdm=KDM_PAPER) -> float:
    """DM at which the mean intra-channel smear equals dt (Section 5.2):
    DM_diag = dt kappa / (2 dnu) [mean nu^-3]^-1, kappa = 1/K in GHz units."""
    return dt_s / (kdm * 2.0 * bw_ghz) / mean_inv_cube(freqs_ghz)


def dm_tau(freqs_ghz, bw_ghz, tau_av_s, kdm=KDM_PAPER) -> float:
    """eq. DM_tau: DM at which the mean intra-channel smear equals tau'_av."""
    return tau_av_s / (kdm * 2.0 * bw_ghz) / mean_inv_cube(freqs_ghz)


def trial_dms(dm0: float, dm_max: float, eps: float, freqs_ghz, bw_ghz: float, dt_s: float,
              tau_av_s: float = 0.0, include_dm_tau: bool = False, cap: int = 1 << 30,
              kdm=KDM_PAPER) -> np.ndarray:
    """eq. trial DMs: DM_n = DM_0 + (2 eps / C) sum_{i<n} sqrt(DM_i^2 + DM_diag^2 + DM_tau^2).

    Trials are generated while DM_n <= dm_max (and at most `cap` of them).  The
    DM_tau term is optional: with it omitted the rule reproduces the trial counts
    the paper quotes for its survey examples."""
    C = len(freqs_ghz)
    a2 = dm_diag(freqs_ghz, bw_ghz, dt_s, kdm) ** 2
    if include_dm_tau:
        a2 += dm_tau(freqs_ghz, bw_ghz, tau_av_s, kdm) ** 2
    out = []
    acc = 0.0
    dm = dm0
    while dm <= dm_max and len(out) < cap:
        out.append(dm)
        acc += math.sqrt(dm * dm + a2)
        dm = dm0 + 2.0 * eps / C * acc
    return np.asarray(out)


def dropout(eps: float) -> float:
    """eq. dm error smearing limit: minimum relative S/N between trials, (eps^2+1)^(-1/4)."""
    return (eps * eps + 1.0) ** -0.25


def snr_attenuation(ddm, dm, dmdiag, dmtau, C):
    """eq. snrb/snri_approx: relative S/N for a DM error ddm."""
    return (C * C * ddm * ddm / (dm * dm + dmdiag * dmdiag + dmtau * dmtau) + 1.0) ** -0.25


# ---------------------------------------------------------------------------------
# Rectangular-pulse model (Appendix A) and the closed forms of Section 3
# ---------------------------------------------------------------------------------

def _overlap(a0, a1, b0, b1):
    return max(0.0, min(a1, b1) - max(a0, b0))


def cell_power_rect(t0: float, dt: float, f_lo: float, f_hi: float, dm: float, width_s: float,
                    scatter_1ghz_s: float = 0.0, scatter_index: float = -4.0,
                    alpha_paper: float = 0.0, nu0: float = 1.0, P0: float = 1.0,
                    nu_top: Optional[float] = None, kdm=KDM_PAPER) -> float:
    """eq. dispersed pulse (App. A): mean power in the cell [t0, t0+dt] x [f_lo, f_hi]
    of a rectangular scatter-broadened pulse of width tau'(nu) and height tau/tau',
    arriving at t = 0 at frequency `nu_top` (the top of the band).

    (P0/dt) int dnu' (nu'/nu0)^-alpha overlap([t0,t0+dt], [t_d, t_d + tau']) tau/tau'.
    The frequency integral is done by adaptive quadrature with the kink
    frequencies (where an edge of the delayed pulse crosses a cell edge) as
    breakpoints."""
    from scipy import integrate, optimize
    nt = f_hi if nu_top is None else nu_top

    def td(nu):
        return kdm * dm * (nu ** -2 - nt ** -2)

    def taup(nu):
        return width_s + scatter_1ghz_s * nu ** scatter_index

    def integrand(nu):
        d = td(nu)
        tp = taup(nu)
        return (nu / nu0) ** (-alpha_paper) * _overlap(t0, t0 + dt, d, d + tp) * (width_s / tp)

    pts = []
    for edge_fn in (lambda nu: td(nu), lambda nu: td(nu) + taup(nu)):
        for tc in (t0, t0 + dt):
            g0, g1 = edge_fn(f_lo) - tc, edge_fn(f_hi) - tc
            if g0 * g1 < 0:
                pts.append(optimize.brentq(lambda nu: edge_fn(nu) - tc, f_lo, f_hi, xtol=1e-15,
                                           rtol=1e-15))
    pts = sorted(set(pts))
    val, _ = integrate.quad(integrand, f_lo, f_hi, points=pts or None, limit=400,
                            epsabs=1e-16, epsrel=1e-13)
    return P0 * val / dt


def spectral_bracket(freqs_lo, bw_ghz, alpha_paper=0.0, nu0=1.0) -> float:
    """The bracketed term of eq. snr_approx: (1/beta) sum_c int_{nu_c}^{nu_c+dnu} (nu'/nu0)^-alpha."""
    f = np.asarray(freqs_lo, dtype=np.float64)
    beta = bw_ghz * len(f)
    if alpha_paper == 1.0:
        tot = np.sum(nu0 * np.log((f + bw_ghz) / f))
    else:
        e = 1.0 - alpha_paper
        tot = np.sum(nu0 ** alpha_paper * ((f + bw_ghz) ** e - f ** e) / e)
    return float(tot / beta)


def snr_approx(P0, beta, tau, kTsys, dnu, dt, N_S, bracket) -> float:
    """eq. snr_approx: peak S/N of a perfectly matched rectangular pulse."""
    return P0 * beta * tau / (kTsys * math.sqrt(dnu * dt * N_S)) * bracket


def delta_nu0(freqs_ghz, tau_av_s, dm, kdm=KDM_PAPER) -> float:
    """eq. delta_nu_0: spectral resolution where the mean intra-channel smear equals tau'_av."""
    return tau_av_s / (2.0 * dm * kdm) / mean_inv_cube(freqs_ghz)


def snr_dedisp(pbar_selected: np.ndarray, N_S: int, dt, dnu, kTsys=1.0) -> float:
    """eq. snr: sqrt(dt / (N_S dnu)) sum_{s in S} Pbar_s / (k T_sys)."""
    return math.sqrt(dt / (N_S * dnu)) * float(np.sum(pbar_selected)) / kTsys


def snr_mf(pbar_tc: np.ndarray, dt, dnu, kTsys=1.0) -> float:
    """Time-series matched filter (Section 4); pbar_tc[t, c]."""
    C = pbar_tc.shape[1]
    return math.sqrt(float(np.sum(np.sum(pbar_tc, axis=1) ** 2))) * math.sqrt(dt) / (
        kTsys * math.sqrt(dnu) * math.sqrt(C))


def snr_dsmf(pbar_tc: np.ndarray, dt, dnu, kTsys=1.0) -> float:
    """Dynamic-spectrum matched filter (Section 4)."""
    return math.sqrt(float(np.sum(pbar_tc ** 2))) * math.sqrt(dt) / (kTsys * math.sqrt(dnu))


def snr_bmf(pbar_tc: np.ndarray, dt, dnu, kTsys=1.0) -> float:
    """Time-series boxcar detector (Section 4)."""
    Nt, C = pbar_tc.shape
    return math.sqrt(dt / (C * Nt * dnu)) * float(np.sum(pbar_tc)) / kTsys


# ---------------------------------------------------------------------------------
# Sample selection (Section 2.2)
# ---------------------------------------------------------------------------------

def greedy_select(values: np.ndarray, chan: np.ndarray, tidx: np.ndarray) -> np.ndarray:
    """Section 2.2 procedure: start from the sample with the highest predicted power,
    then add samples in order of decreasing power while eq. sel_criterion holds,
    Pbar_next > (sqrt((N+1)/N) - 1) * sum_{s in S} Pbar_s.
    Order among equal powers: channel, then time, ascending.  Returns the indices
    (into `values`) of the selected samples."""
    order = sorted(range(len(values)), key=lambda i: (-values[i], chan[i], tidx[i]))
    if not order:
        return np.zeros(0, dtype=np.int64)
    sel = [order[0]]
    tot = float(values[order[0]])
    for i in order[1:]:
        N = len(sel)
        if float(values[i]) > (math.sqrt((N + 1) / N) - 1.0) * tot:
            sel.append(i)
            tot += float(values[i])
        else:
            break
    return np.asarray(sel, dtype=np.int64)


def best_prefix(values: np.ndarray) -> tuple[int, float]:
    """Exact optimum of sum(S)/sqrt(|S|) over all subsets: the best set of each size
    is the top-k, so scan the sorted prefixes.  Returns (k, objective)."""
    v = np.sort(np.asarray(values, dtype=np.float64))[::-1]
    best_k, best = 0, -math.inf
    acc = 0.0
    for k in range(1, len(v) + 1):
        acc += v[k - 1]
        f = acc / math.sqrt(k)
        if f > best:
            best, best_k = f, k
    return best_k, best


def greedy_tables(freqs_ghz, bw_ghz, dt_s, dms, width_s, scatter_1ghz_s=0.0, scatter_index=-4.0,
                  alpha_paper=0.0, nu0=1.0, kdm=KDM_PAPER):
    """Sample sets chosen by the Section 2.2 procedure for a rectangular pulse model
    arriving at t = 0 at the top of the band.  Candidates are every cell with
    non-zero predicted power (the eq. num_samples range); their powers come from
    eq. dispersed pulse.  Returns (start, ntap, objective[d]) where each channel's
    selection is stored as its contiguous run (ntap = 0 when none is selected)."""
    ft, fl, fh = channel_edges(freqs_ghz, bw_ghz)
    s0 = delay_start(freqs_ghz, bw_ghz, dt_s, dms, kdm)
    n0 = taps_allnonzero(freqs_ghz, bw_ghz, dt_s, dms, width_s, scatter_1ghz_s, scatter_index, kdm)
    D, C = s0.shape
    start = np.zeros((D, C), dtype=np.int64)
    ntap = np.zeros((D, C), dtype=np.int64)
    obj = np.zeros(D)
    for d in range(D):
        vals, ch, tj = [], [], []
        for c in range(C):
            for j in range(int(s0[d, c]), int(s0[d, c] + n0[d, c])):
                v = cell_power_rect(j * dt_s, dt_s, fl[c], ft[c], float(dms[d]), width_s,
                                    scatter_1ghz_s, scatter_index, alpha_paper, nu0, 1.0, fh, kdm)
                if v > 0.0:
                    vals.append(v)
                    ch.append(c)
                    tj.append(j)
        vals = np.asarray(vals)
        sel = greedy_select(vals, np.asarray(ch), np.asarray(tj))
        obj[d] = float(np.sum(vals[sel])) / math.sqrt(len(sel))
        for c in range(C):
            js = sorted(tj[i] for i in sel if ch[i] == c)
            if js:
                if js[-1] - js[0] + 1 != len(js):
                    raise ValueError("non-contiguous selection in a channel")
                start[d, c] = js[0]
                ntap[d, c] = len(js)
    return start, ntap, obj
