"""Host-side checks of libdedisp (no GPU needed): exported symbols, plan tables
against the oracle's independent tables, the trial-DM rule, and error paths."""
import ctypes
import re
import os

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dd():
    import paper_1301_3968_amd as dd
    return dd


def test_exports_every_declared_symbol(dd):
    from paper_1301_3968_amd import _lib
    with open(os.path.join(ROOT, "include", "dedisp.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"\b(dedisp_[a-z_]+)\s*\(", hdr))
    declared.discard("dedisp_plan_s")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(_lib.EXPORTS)


CASES = [
    ("cfg1", lambda: workloads.channel_centres(1.2, 0.3, 64), 0.3 / 64, 1e-3, np.arange(32) * 10.0),
    ("cfg2", lambda: workloads.channel_centres(1.2, 0.336, 336), 1e-3, 1e-3, np.linspace(0, 2000, 1024)),
    ("cfg3", lambda: workloads.channel_centres(1.2, 0.3, 4096), 0.3 / 4096, 64e-6, np.linspace(0, 1000, 4096)),
]


@pytest.mark.parametrize("name,fgen,bw,dt,dms", CASES)
@pytest.mark.parametrize("kdm", [0.0, 4.15e-3])
def test_tables_match_oracle(dd, orc, name, fgen, bw, dt, dms, kdm):
    f = fgen()
    K = kdm if kdm > 0 else orc.KDM_PAPER
    so = orc.delay_start(f, bw, dt, dms, K)
    for rule in ("smear", "allnonzero"):
        p = dd.Plan(f, bw, dt, dms, rule=rule, k_dm=kdm)
        s, n = p.tables()
        no = orc.taps_smear(f, bw, dt, dms, K) if rule == "smear" else orc.taps_allnonzero(f, bw, dt, dms, kdm=K)
        bad = np.argwhere((s != so) | (n != no))
        assert bad.size == 0, f"{name} {rule}: first mismatch at {bad[:3]}"
        assert p.max_span == int(np.max(so + no))


def test_allnonzero_with_width_and_scatter(dd, orc):
    f = workloads.channel_centres(1.2, 0.336, 336)
    dms = np.linspace(0, 2000, 257)
    p = dd.Plan(f, 1e-3, 1e-3, dms, rule="allnonzero", width_s=2.5e-3, scatter_s_1ghz=1e-3)
    s, n = p.tables()
    no = orc.taps_allnonzero(f, 1e-3, 1e-3, dms, 2.5e-3, 1e-3, -4.0)
    assert np.array_equal(n, no)
    assert np.array_equal(s, orc.delay_start(f, 1e-3, 1e-3, dms))


def test_descending_channels(dd, orc):
    f = workloads.channel_centres(1.2, 0.336, 336)[::-1].copy()
    dms = np.linspace(0, 2000, 64)
    p = dd.Plan(f, 1e-3, 1e-3, dms, rule="allnonzero")
    s, n = p.tables()
    assert np.array_equal(s, orc.delay_start(f, 1e-3, 1e-3, dms))
    assert np.array_equal(n, orc.taps_allnonzero(f, 1e-3, 1e-3, dms))


@pytest.mark.parametrize("flo,bw,C,dt,eps,lo,hi,count", [
    (0.7, 0.304, 304, 1e-3, 1.492, 10, 3000, 442),
    (21.0, 2.0, 256, 1e-4, 0.580, 50, 10000, 128),
    (21.0, 2.0, 32, 1e-4, 0.287, 50, 10000, 128),
])
def test_trial_dms_match_oracle(dd, orc, flo, bw, C, dt, eps, lo, hi, count):
    f = workloads.channel_centres(flo, bw, C)
    a = dd.trial_dms(lo, hi, eps, f, bw / C, dt)
    b = orc.trial_dms(lo, hi, eps, f, bw / C, dt)
    assert len(a) == len(b) == count
    assert np.allclose(a, b, rtol=1e-12, atol=0)
    a2 = dd.trial_dms(lo, hi, eps, f, bw / C, dt, tau_av_s=dt, include_dm_tau=True)
    b2 = orc.trial_dms(lo, hi, eps, f, bw / C, dt, tau_av_s=dt, include_dm_tau=True)
    assert len(a2) == len(b2) and np.allclose(a2, b2, rtol=1e-12)


def test_greedy_rule_matches_oracle_objective(dd, orc):
    # Section 2.2 selection on a small band: same set sizes and S/N objective.
    f = workloads.channel_centres(0.7, 0.032, 8)
    dms = np.array([0.0, 30.0, 120.0, 400.0])
    kw = dict(width_s=1e-3)
    p = dd.Plan(f, 0.004, 1e-3, dms, rule="greedy", **kw)
    s, n = p.tables()
    so, no, obj = orc.greedy_tables(f, 0.004, 1e-3, dms, 1e-3)
    assert np.array_equal(n.sum(axis=1), no.sum(axis=1))
    ft, fl, fh = orc.channel_edges(f, 0.004)
    for d in range(len(dms)):
        vals = [orc.cell_power_rect(j * 1e-3, 1e-3, fl[c], ft[c], dms[d], 1e-3, nu_top=fh)
                for c in range(len(f)) for j in range(s[d, c], s[d, c] + n[d, c])]
        got = sum(vals) / np.sqrt(len(vals))
        assert got == pytest.approx(obj[d], rel=1e-9)


def test_errors(dd):
    from paper_1301_3968_amd import _lib
    f = workloads.channel_centres(1.2, 0.336, 8)
    with pytest.raises(dd.DedispError) as e:
        dd.Plan(f, -1.0, 1e-3, [0.0])
    assert e.value.status == _lib.ERR_INVALID_ARG
    with pytest.raises(dd.DedispError) as e:
        dd.Plan(f, 1e-3, 1e-3, [float("nan")])
    assert e.value.status == _lib.ERR_INVALID_ARG
    with pytest.raises(dd.DedispError) as e:
        dd.Plan(f, 1e-3, 1e-3, [-5.0])
    assert e.value.status == _lib.ERR_INVALID_ARG
    p = dd.Plan(f, 1e-3, 1e-3, [0.0, 500.0])
    with pytest.raises(dd.DedispError) as e:
        p.out_len(p.max_span - 1)
    assert e.value.status == _lib.ERR_SHAPE
    assert p.out_len(p.max_span) == 1
    with pytest.raises(dd.DedispError) as e:
        dd.Plan(f, 1e-3, 1e-3, [0.0], rule="tap" if False else "fixed", ktaps=0)
    assert e.value.status == _lib.ERR_INVALID_ARG
    s = np.zeros((1, 8), np.int32)
    n = np.full((1, 8), 3, np.int32)
    with pytest.raises(dd.DedispError) as e:
        dd.Plan(f, 1e-3, 1e-3, [0.0], rule="explicit", start=s, ntap=n, wmode="tap", ktaps=4,
                weights=np.ones((8, 4), np.float32))
    assert e.value.status == _lib.ERR_UNSUPPORTED
    # The thread-local message describes the failure.
    assert b"ntap" in _lib.lib().dedisp_last_error()


def test_bench_refuses_more_than_one_gpu():
    # The benchmark measures one GPU; asked for more it says so and exits before any GPU work.
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _raw_call(dd, fn, *args):
    """Call a C-ABI entry point directly; returns (status, last error text)."""
    from paper_1301_3968_amd import _lib
    st = getattr(_lib.lib(), fn)(*args)
    return st, _lib.lib().dedisp_last_error().decode()


def test_overflow_predicted_before_device_work(dd):
    from paper_1301_3968_amd import _lib
    # 1000 channels of 9000-sample runs: 255 x 9e6 > 2^31 for one output
    C, D, n = 1000, 2, 9000
    f = workloads.channel_centres(1.2, 0.3, C)
    start = np.zeros((D, C), np.int32)
    ntap = np.full((D, C), n, np.int32)
    p = dd.Plan(f, 0.3 / C, 1e-3, [0.0, 1.0], rule="explicit", start=start, ntap=ntap)
    fake = ctypes.c_void_p(0x1000)     # never dereferenced: the check precedes device work
    T = n + 10
    st, msg = _raw_call(dd, "dedisp_dedisperse", p.handle, fake, _lib.U8, T, T, 0, 1, fake,
                        _lib.I32, 11, 0, None, None)
    assert st == _lib.ERR_OVERFLOW and "overflow" in msg
    # the same plan's fp32 output cannot overflow: the check lets it through (and the call
    # then needs a device, which this host may not have)
    # a plan whose single outputs fit but whose boxcar windows (64 outputs) would not
    ntap2 = np.full((D, C), 200, np.int32)    # 255 x 2e5 = 5.1e7 per output, x 64 > 2^31
    p2 = dd.Plan(f, 0.3 / C, 1e-3, [0.0, 1.0], rule="explicit", start=start, ntap=ntap2)
    w = np.arange(1, 33, dtype=np.int32)
    mu = np.full(C, 128.0)
    T2 = 5000
    wb = p2.work_bytes(T2, 32)
    st, msg = _raw_call(dd, "dedisp_search", p2.handle, fake, _lib.U8, T2, T2,
                        w.ctypes.data_as(ctypes.c_void_p), 32, fake, fake, fake, fake, fake,
                        fake, ctypes.c_size_t(wb), None)
    assert st == _lib.ERR_OVERFLOW and "window" in msg
    st, msg = _raw_call(dd, "dedisp_search_noalloc", p2.handle, fake, _lib.U8, T2, T2,
                        w.ctypes.data_as(ctypes.c_void_p), 32, fake, fake, fake, fake, fake, None)
    assert st == _lib.ERR_OVERFLOW
    # a delay beyond int32 samples is refused when the plan is made
    with pytest.raises(dd.DedispError) as e:
        dd.Plan(f, 0.3 / C, 1e-9, [1e6], rule="smear")
    assert e.value.status == _lib.ERR_OVERFLOW


def test_forced_allocation_failure(dd, monkeypatch):
    from paper_1301_3968_amd import _lib
    f = workloads.channel_centres(1.2, 0.3, 64)
    dms = np.arange(32) * 10.0
    # the first allocation (the plan), then the second (its tables), fail with OOM
    for k in ("1", "2"):
        monkeypatch.setenv("DEDISP_TEST_FAIL_ALLOC", k)
        with pytest.raises(dd.DedispError) as e:
            dd.Plan(f, 0.3 / 64, 1e-3, dms, rule="smear")
        assert e.value.status == _lib.ERR_OOM and "allocation" in str(e.value)
    # a count past the allocations a plan needs: the plan is made
    monkeypatch.setenv("DEDISP_TEST_FAIL_ALLOC", "3")
    p = dd.Plan(f, 0.3 / 64, 1e-3, dms, rule="smear")
    assert p.ndm == 32
    monkeypatch.delenv("DEDISP_TEST_FAIL_ALLOC")
    p2 = dd.Plan(f, 0.3 / 64, 1e-3, dms, rule="smear")
    assert np.array_equal(p.tables()[1], p2.tables()[1])


def test_plan_log_line():
    # DEDISP_LOG=1 prints one summary line per plan on stderr; without it nothing.
    import subprocess
    import sys
    code = ("import numpy as np, paper_1301_3968_amd as dd; "
            "f = 1.2 + 0.3 * (np.arange(64) + 0.5) / 64; "
            "dd.Plan(f, 0.3 / 64, 1e-3, np.arange(32) * 10.0, rule='smear')")
    env = dict(os.environ, DEDISP_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=ROOT, env=env)
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("dedisp: plan")]
    assert len(lines) == 1
    assert "32 trials x 64 channels" in lines[0] and "rule smear" in lines[0]
    env.pop("DEDISP_LOG")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=ROOT, env=env)
    assert r.returncode == 0 and "dedisp:" not in r.stderr


def test_merge_candidates_rejects_bad_arguments():
    # Argument checks of the stream merge run on the host, before anything is enqueued.
    import ctypes
    from paper_1301_3968_amd import _lib
    L = _lib.lib()
    p = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails its checks
    assert L.dedisp_merge_candidates(0, p, p, p, 0, p, p, p, None) == _lib.ERR_INVALID_ARG
    assert L.dedisp_merge_candidates(4, None, p, p, 0, p, p, p, None) == _lib.ERR_INVALID_ARG
    assert L.dedisp_merge_candidates(4, p, p, p, -1, p, p, p, None) == _lib.ERR_INVALID_ARG
    assert b"t_offset" in L.dedisp_last_error()


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "explicit", "short"])
def test_matrix_core_staging_tables_consistent(dd, which):
    """For every matrix-core shape the plan fits, the host tables of the two window
    stagings fill the same LDS pieces with the same window bytes and every K block reads
    inside its channel's staged region (the library's own host-side check)."""
    from paper_1301_3968_amd import _lib
    rng = np.random.default_rng(88)
    if which == "cfg1":
        wl = workloads.cfg1()
        p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule)
    elif which == "cfg2":
        wl = workloads.cfg2(nsamp=4096)
        p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    elif which == "short":   # 37 trials: no DM tile full
        wl = workloads.cfg2(nsamp=3000, ndm=37)
        p = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="allnonzero")
    else:                    # trials out of DM order, a channel no trial uses, runs of 1..7
        C, D = 37, 50
        f = workloads.channel_centres(1.35, 0.3, C)
        dms = ((np.arange(D) * 37) % D) * 3.0
        s = np.zeros((D, C), np.int32)
        n = rng.integers(1, 8, size=(D, C)).astype(np.int32)
        for d in range(D):
            s[d] = np.floor(4.15 * dms[d] * (1.0 / f ** 2 - 1.0 / f.max() ** 2)).astype(np.int32)
        n[:, 5] = 0
        p = dd.Plan(f, 0.01, 1e-3, dms, rule="explicit", start=s, ntap=n)
    fits = 0
    for shape in range(5):
        pieces = ctypes.c_int64(-1)
        st = _lib.lib().dedisp_check_search_tables(p.handle, shape, ctypes.byref(pieces))
        msg = _lib.lib().dedisp_last_error().decode()
        if st == _lib.ERR_UNSUPPORTED:
            assert "does not fit" in msg, msg
            continue
        assert st == 0, msg
        assert pieces.value > 0
        fits += 1
    assert fits >= 1
    assert _lib.lib().dedisp_check_search_tables(p.handle, 5, None) == _lib.ERR_INVALID_ARG
