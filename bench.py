"""Throughput of the fused dedispersion + boxcar search on one MI355X.

One step = one pass of the whole hot path over one block: the fused search
(dedispersion sum of every trial with its programmable profile, boxcar S/N
search over all widths, per-trial reduction) on the 336-channel, 65536-sample
uint8 block with 1024 trial DMs and widths 1..32, input already resident in HBM.
The metric is DM-trial x channel x output-sample sums per second.

Prints one JSON line (see the contract in the repository's design notes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9   # int32 vector lane-ops/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
PACKED_PEAK_OPS = 2 * VALU_PEAK_OPS    # two 16-bit adds per lane-op (packed uint16 adds)
HBM_PEAK_BYTES = 8e12                  # MI355X HBM3E peak, bytes/s
MFMA_I8_PEAK_OPS = 5.0e15              # dense int8 matrix-core ops/s (a multiply-add is 2 ops)
NUM_PACKED_SHAPES = 8                  # search shapes 0-7: packed-add kernel; 8 on: matrix cores
# sources of the search kernels (both kinds and their shared detection stage)
KERNEL_SRCS = [os.path.join(ROOT, "paper_1301_3968_amd", "csrc", f)
               for f in ("kernels_search.hip", "kernels_mfma.hip", "boxcar_row.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_search_336ch_65536s_1024dm.json")


def _src_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(tile: int):
    """HBM bytes per launch of the search kernel in tile shape `tile`, from the
    committed rocprofv3 counter runs (FETCH_SIZE + WRITE_SIZE, each scaled by what
    the counter reads for a plain copy of known size), if they were taken on the
    current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != _src_sha():
        return None
    return t.get("per_tile", {}).get(str(tile), {}).get("hbm_bytes_per_launch")


def _host_cpu():
    """(model name, logical CPUs) of the host this runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(wl, rule: str, ndm_single: int, ndm_threads: int):
    """The oracle as written (plain C loops, int64 sums, fp64 S/N), timed on the host on
    a bounded sample of the workload's trials: single-threaded, and on every host core
    (one thread per disjoint trial range, each running the unchanged oracle)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    # the oracle's own tables for the rule (not timed)
    start = oracle.delay_start(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    taps = {"smear": oracle.taps_smear, "allnonzero": oracle.taps_allnonzero}[rule]
    ntap = taps(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    T = wl.x.shape[1]
    C = wl.x.shape[0]
    tout = T - int(np.max(start + ntap)) + 1

    def run(pick):
        y = oracle.dedisperse_u8(wl.x, start[pick], ntap[pick], tout=tout)
        M, S = oracle.boxcar_norm(ntap[pick], wl.widths, wl.chan_mean, wl.chan_sigma)
        oracle.boxcar_detect(y.astype(np.float64), wl.widths, M, S)

    D = len(wl.dms)
    pick1 = np.linspace(0, D - 1, ndm_single).round().astype(int)
    t0 = time.perf_counter()
    run(pick1)
    dt1 = time.perf_counter() - t0
    model, ncpu = _host_cpu()
    nth = max(1, min(ncpu, ndm_threads))
    pickn = np.linspace(0, D - 1, ndm_threads).round().astype(int)
    parts = [p for p in np.array_split(pickn, nth) if len(p)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(len(parts)) as ex:
        list(ex.map(run, parts))
    dtn = time.perf_counter() - t0
    return {"value": ndm_threads * C * tout / dtn, "unit": "sums/s", "cores": len(parts),
            "kind": "oracle",
            "sample": f"{ndm_threads} of {D} trials (evenly spaced), full {C}x{T} block, "
                      f"dedisperse+norm+detect, {len(parts)} threads over disjoint trial "
                      f"ranges, {dtn:.1f} s",
            "host_cpu": model, "host_logical_cpus": ncpu,
            "single_thread": {"value": ndm_single * C * tout / dt1, "unit": "sums/s",
                              "cores": 1,
                              "sample": f"{ndm_single} of {D} trials (evenly spaced), "
                                        f"{dt1:.1f} s"}}


def _oracle_threads(jobs):
    """Run the oracle jobs (callables, each on its own part of a sample) on the host's
    cores; returns (seconds, threads)."""
    from concurrent.futures import ThreadPoolExecutor
    _, ncpu = _host_cpu()
    nth = max(1, min(ncpu, len(jobs)))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nth) as ex:
        list(ex.map(lambda f: f(), jobs))
    return time.perf_counter() - t0, nth


def _oracle_line(sums, seconds, nth, sample):
    model, ncpu = _host_cpu()
    return {"value": sums / seconds, "unit": "sums/s", "cores": nth, "kind": "oracle",
            "sample": f"{sample}, {nth} threads, {seconds:.1f} s", "host_cpu": model,
            "host_logical_cpus": ncpu}


def cpu_baseline_weighted(wl, ntrials: int = 16):
    """The oracle's fp64 channel-weighted sum on ntrials evenly spaced trials of the
    4096-channel block, one trial per thread."""
    import oracle
    start = oracle.delay_start(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    ntap = oracle.taps_smear(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    tout = wl.x.shape[1] - int(np.max(start + ntap)) + 1
    pick = np.linspace(0, len(wl.dms) - 1, ntrials).round().astype(int)
    jobs = [lambda d=d: oracle.dedisperse_f64(wl.x, start[d:d + 1], ntap[d:d + 1], "channel",
                                              wl.weights, tout=tout) for d in pick]
    sec, nth = _oracle_threads(jobs)
    return _oracle_line(ntrials * wl.x.shape[0] * tout, sec, nth,
                        f"{ntrials} of {len(wl.dms)} trials (evenly spaced), full "
                        f"{wl.x.shape[0]}x{wl.x.shape[1]} block, fp64 channel-weighted sum")


def cpu_baseline_batch(beams, widths, ntrials: int = 128):
    """The oracle's dedispersion + noise tables + detection on ntrials evenly spaced trials
    of each sampled beam (beams: list of (x, freqs, dms)), one (beam, trial range) per
    thread."""
    import oracle
    jobs, sums, desc = [], 0, []
    for x, f, dms in beams:
        start = oracle.delay_start(f, 0.001, 1e-3, dms).astype(np.int32)
        ntap = oracle.taps_allnonzero(f, 0.001, 1e-3, dms).astype(np.int32)
        tout = x.shape[1] - int(np.max(start + ntap)) + 1
        pick = np.linspace(0, len(dms) - 1, ntrials).round().astype(int)
        C = x.shape[0]
        mu, sg = np.full(C, 128.0), np.full(C, 16.0)
        for part in np.array_split(pick, 4):
            def job(x=x, s=start[part], n=ntap[part], tout=tout, mu=mu, sg=sg):
                y = oracle.dedisperse_u8(x, s, n, tout=tout)
                M, S = oracle.boxcar_norm(n, widths, mu, sg)
                oracle.boxcar_detect(y.astype(np.float64), widths, M, S)
            jobs.append(job)
        sums += ntrials * C * tout
        desc.append(f"{x.shape[1]}")
    sec, nth = _oracle_threads(jobs)
    return _oracle_line(sums, sec, nth,
                        f"{ntrials} evenly spaced trials of each of {len(beams)} beams "
                        f"(lengths {', '.join(desc)}), dedisperse+norm+detect")


def cpu_baseline_taps(wl, nbatch: int = 16, ntrials: int = 32):
    """The oracle's fp64 tap-weighted forward sum on nbatch pulses' blocks x ntrials
    evenly spaced trials of the 64-pulse batch, one (block, trial range) per thread."""
    import oracle
    start = oracle.delay_start(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms).astype(np.int32)
    K = wl.extra["ktaps"]
    ntap = np.full_like(start, K)
    tout = wl.x.shape[2] - int(np.max(start + ntap)) + 1
    pick = np.linspace(0, len(wl.dms) - 1, ntrials).round().astype(int)
    jobs = []
    for b in range(nbatch):
        for part in np.array_split(pick, 4):
            jobs.append(lambda b=b, part=part: oracle.dedisperse_f64(
                wl.x[b], start[part], ntap[part], "tap", wl.weights, tout=tout))
    sec, nth = _oracle_threads(jobs)
    return _oracle_line(nbatch * ntrials * wl.x.shape[1] * tout, sec, nth,
                        f"{nbatch} of {wl.x.shape[0]} pulse blocks x {ntrials} of "
                        f"{len(wl.dms)} trials, fp64 {K}-tap forward sum")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rule", default="allnonzero", choices=["allnonzero", "smear"])
    ap.add_argument("--cpu-sample-trials", type=int, default=64,
                    help="trials of the single-threaded oracle sample")
    ap.add_argument("--cpu-thread-trials", type=int, default=512,
                    help="trials of the all-cores oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the batch and autograd ratio measurements")
    ap.add_argument("--workload", default="search",
                    choices=["search", "batch", "weighted", "autograd", "completeness", "dm_error",
                             "resolution", "detectors", "lds"],
                    help="search: the headline fused search (default); batch: 36 beams in one "
                         "launch; weighted: 4096-channel fp32-weighted dedispersion; "
                         "autograd: forward / adjoint timing of the 8-tap learnable profile; "
                         "completeness: largest S/N over the trial DMs against a test pulse's DM; "
                         "dm_error: S/N attenuation with DM error about one trial DM; "
                         "resolution: peak S/N against the time and frequency resolution; "
                         "detectors: matched filters and boxcar against the greedy detector; "
                         "lds: LDS read rate of the lane address patterns of the matrix-core "
                         "operand reads (the probe_lds program, run as a child process)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (the reference kernel "
                         "for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU layout "
              "is described in the design notes and not run here.", file=sys.stderr)
        return 2

    if args.workload == "lds":
        # a child process of its own, started before this process touches the GPU
        probe = os.path.join(ROOT, "paper_1301_3968_amd", "probe_lds")
        if not os.path.exists(probe):
            print("probe_lds is not built (run the package's build first)", file=sys.stderr)
            return 1
        out = subprocess.run([probe], stdout=subprocess.PIPE, text=True)
        if out.returncode != 0:
            print(f"probe_lds failed with status {out.returncode}", file=sys.stderr)
            return out.returncode
        rates = [json.loads(ln) for ln in out.stdout.splitlines() if ln.startswith("{")]
        print(json.dumps({"metric": "LDS read bytes per clock per CU (16- and 8-byte lane reads)",
                          "unit": "B/clk/CU", "n_gpus": 1, "higher_is_better": True,
                          "data": "synthetic", "patterns": rates}))
        return 0

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))
        return 0

    import paper_1301_3968_amd as dd
    import workloads

    if args.workload != "search":
        return _other_workload(args, dd, workloads)
    print("generating the 336-channel workload", file=sys.stderr, flush=True)
    wl = workloads.cfg2(rule=args.rule)
    plan = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=args.rule)
    start, ntap = plan.tables()
    C, T = wl.x.shape
    D = len(wl.dms)
    nout = plan.out_len(T)
    nw = len(wl.widths)
    x = torch.from_numpy(wl.x).cuda()
    mu = torch.as_tensor(wl.chan_mean, dtype=torch.float64).cuda()
    sg = torch.as_tensor(wl.chan_sigma, dtype=torch.float64).cuda()
    work = torch.empty(plan.work_bytes(T, nw), dtype=torch.uint8, device="cuda")
    outs = (torch.empty(D, dtype=torch.float64, device="cuda"),
            torch.empty(D, dtype=torch.int32, device="cuda"),
            torch.empty(D, dtype=torch.int32, device="cuda"))

    def step():
        plan.search(x, wl.widths, mu, sg, work=work, outputs=outs)

    tile = plan.autotune(x, wl.widths, mu, sg, work=work)   # untimed: picks the tile shape
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K = args.steps
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for e in ev0 + ev1:
        e.record()
    torch.cuda.synchronize()
    plan.set_kernel_events(ev0, ev1)
    print(f"timing {K} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_kernel_events([], [])
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)]))
    ms_step = (t1 - t0) * 1e3 / K
    sums = float(D) * C * nout
    value = sums / ((t1 - t0) / K)

    # Algorithmic work of one launch of the dominant kernel, as the measurement rule
    # fixes it: one add per DM-trial x channel x output-sample sum (a trial's channel
    # term is one sample of a windowed sum), plus one subtract and one max per boxcar
    # window when the detection is fused into that kernel, i.e. (1 + 2 N_W / C) ops per
    # sum.  The fraction is taken against the peak of the unit the kernel runs on: the
    # dense int8 matrix-core rate for the matrix-core kernel, the int32 vector lane-op
    # rate for the packed-add kernel.
    fused = _fused(plan)
    ops = sums + (2.0 * D * nout * nw if fused else 0.0)
    kern_s = kern_ms * 1e-3
    mfma = fused and tile >= NUM_PACKED_SHAPES
    peak = MFMA_I8_PEAK_OPS if mfma else VALU_PEAK_OPS
    # algorithmic HBM bytes of a fused launch: the block read once, the per-(trial,
    # width) noise tables and the per-trial results
    alg_bytes = float(C) * T + D * nw * 16.0 + D * 16.0
    traffic = _traffic(tile) if fused else None
    roofline = {"bound": "mfma" if mfma else "alu",
                "achieved": ops / kern_s / 1e12, "peak": peak / 1e12,
                "unit": "TOP/s (int8 matrix cores)" if mfma else "Tops/s (int32 lane ops)",
                "frac": ops / kern_s / peak, "traffic": traffic,
                "kernel_ms": kern_ms, "ops_per_launch": ops, "sums_per_launch": sums,
                "algorithmic_bytes_per_launch": alg_bytes,
                "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None,
                # the same work against the vector units' peaks, for comparison
                "frac_of_int32_lane_op_peak": ops / kern_s / VALU_PEAK_OPS,
                "frac_of_packed_u16_peak": ops / kern_s / PACKED_PEAK_OPS}
    if mfma:
        # the plain definition of the sum on the matrix cores: one int8 multiply-add
        # (2 ops) per sample term, sum over (d, c) of ntap[d, c] terms per output
        roofline["useful_int8_ops_per_launch"] = 2.0 * nout * float(np.sum(ntap, dtype=np.int64))
    # the counted HBM bytes of one launch over its measured duration
    if traffic is not None:
        rate = traffic / kern_s
        roofline["traffic_rate"] = {"GB/s": rate / 1e9, "frac_of_hbm_peak": rate / HBM_PEAK_BYTES}
    line = {
        "metric": "DM-trial*channel*sample sums/s", "value": value, "unit": "sums/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded uint8 Gaussian noise + 16 injected dispersed pulses)",
        "config": {"workload": "336ch x 65536 samples uint8, 1024 trial DMs 0-2000, "
                               f"{args.rule} profile, boxcar widths 1-32",
                   "nchan": C, "nsamp": T, "ndm": D, "nout": nout, "widths": nw,
                   "rule": args.rule, "fused_search": bool(fused), "tile_config": tile},
        "roofline": roofline,
        # the "effective bandwidth" convention (one input byte per DM-channel-sample sum)
        # as a rate; a convention for comparing dedispersers, not a roofline fraction:
        # each input byte is reused by many trials in LDS and registers
        "effective_bandwidth": {"unit": "TB/s", "value": value / 1e12,
                                "convention": "one input byte per sum"},
    }
    if not args.no_extras:
        # the two serving / training patterns beside the headline: per-sum time of the
        # 36-beam batch against the headline's, and the adjoints against the forward
        mb = measure_batch(dd, workloads, 5, 2)
        mb["per_sum_time_over_headline"] = ((mb["ms_per_call"] / mb["total_sums"])
                                            / (ms_step / sums))
        line["batched"] = mb
        line["autograd"] = measure_autograd(dd, workloads, 3, 1)
    if not args.no_cpu_baseline:
        print("timing the oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, args.rule, args.cpu_sample_trials,
                                            args.cpu_thread_trials)
    print(json.dumps(line), flush=True)
    return 0


def _timed(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _other_workload(args, dd, workloads) -> int:
    """Secondary measurements (one JSON line each); not the headline metric."""
    import torch
    K, W = args.steps, args.warmup
    base = {"n_gpus": 1, "steps": K, "warmup": W, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "data": "synthetic"}
    if args.workload == "batch":
        m = measure_batch(dd, workloads, K, W, single=True,
                          keep_host=() if args.no_cpu_baseline else (0, 9, 18, 27))
        host = m.pop("host_beams", [])
        line = dict(base, metric="DM-trial*channel*sample sums/s (36-beam batch)",
                    value=m["sums_per_s"], unit="sums/s", ms_per_step=m["ms_per_call"],
                    dtype="int32", config=m)
        if host:
            print("timing the oracle on a sample", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline_batch(host, list(range(1, 33)))
    elif args.workload == "completeness":
        line = dict(base, **_completeness(dd, workloads, K, W))
    elif args.workload == "dm_error":
        line = dict(base, **_dm_error(dd, workloads))
    elif args.workload == "resolution":
        line = dict(base, **_resolution(dd, workloads))
    elif args.workload == "detectors":
        line = dict(base, **_detectors(dd, workloads))
    elif args.workload == "weighted":
        print("generating the 4096-channel block", file=sys.stderr, flush=True)
        wl = workloads.cfg3()
        p_ = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule=wl.rule, wmode="channel",
                     weights=wl.weights)
        x = torch.from_numpy(wl.x).cuda()
        nout = p_.out_len(x.shape[1])
        y = torch.empty((len(wl.dms), nout), dtype=torch.float32, device="cuda")
        t = _timed(lambda: p_.dedisperse(x, out=y[None]), K, W)
        sums = float(len(wl.dms)) * x.shape[0] * nout
        line = dict(base, metric="DM-trial*channel*sample sums/s (fp32 channel weights)",
                    value=sums / t, unit="sums/s", ms_per_step=t * 1e3, dtype="fp32",
                    config={"workload": "4096 ch x 262144 samples uint8, 4096 trial DMs, "
                                        "weights (f/1.35 GHz)^-1.5", "nout": nout})
        if not args.no_cpu_baseline:
            print("timing the oracle on a sample", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline_weighted(wl)
    else:
        m = measure_autograd(dd, workloads, K, W, train=True)
        line = dict(base, metric="DM-trial*channel*sample sums/s (8-tap fp32 forward)",
                    value=m["forward_sums_per_s"], unit="sums/s", ms_per_step=m["ms_forward"],
                    dtype="fp32", config=m)
        if not args.no_cpu_baseline:
            print("timing the oracle on a sample", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline_taps(workloads.cfg5())
    print(json.dumps(line), flush=True)
    return 0


def measure_batch(dd, workloads, K, W, single=False, keep_host=()):
    """The 36-beam batch (336 ch, lengths U{16384..131072}, trial-DM grids of 300-1200
    trials at 0.8 of optimal) searched in one call replayed from a HIP graph; eager
    calls and (single) the beams searched one plan at a time beside it.  The host data
    of the beams in keep_host are returned under "host_beams" (for the oracle's timing)."""
    import math

    import torch
    spec = workloads.cfg4_beams()
    C = 336
    f = workloads.channel_centres(1.2, 0.336, C)
    eps = math.sqrt(0.8 ** -4 - 1.0) / 2.0       # spacing one DM error apart, 0.8 of optimal
    plans, xs, host = [], [], []
    print("generating 36 beams", file=sys.stderr, flush=True)
    for b in range(len(spec["nsamp"])):
        dms = dd.trial_dms(0.0, 1e9, eps, f, 0.001, 1e-3, cap=int(spec["ntrial"][b]))
        x, _ = workloads.cfg4_beam_data(b, int(spec["nsamp"][b]), float(dms[0]), float(dms[-1]))
        plans.append(dd.Plan(f, 0.001, 1e-3, dms, rule="allnonzero"))
        xs.append(torch.from_numpy(x).cuda())
        if b in keep_host:
            host.append((x, f, np.asarray(dms)))
    widths = list(range(1, 33))
    B = dd.Batch(plans, [int(v) for v in spec["nsamp"]], widths)
    mu = torch.full((C,), 128.0, dtype=torch.float64, device="cuda")
    sg = torch.full((C,), 16.0, dtype=torch.float64, device="cuda")
    work = torch.empty(B.work_bytes, dtype=torch.uint8, device="cuda")
    outs = tuple(torch.empty(B.total_trials, dtype=dt, device="cuda")
                 for dt in (torch.float64, torch.int32, torch.int32))
    print("timing the batch", file=sys.stderr, flush=True)
    t_graph = _timed(lambda: B.run(xs, mu, sg, work=work, outputs=outs, graph=True), K, W)
    t_eager = _timed(lambda: B.run(xs, mu, sg, work=work, outputs=outs, graph=False), K, W)
    out = {"workload": "36 beams x 336 ch, lengths U{16384..131072}, trial-DM grids of "
                       "300-1200 trials (0.8 of optimal)",
           "total_trials": B.total_trials, "total_sums": B.total_sums,
           "ms_per_call": t_graph * 1e3, "sums_per_s": B.total_sums / t_graph,
           "ms_eager": t_eager * 1e3}
    if single:
        # per-sum cost of the same beams searched one plan at a time
        pw = [torch.empty(p_.work_bytes(x.shape[1], 32), dtype=torch.uint8, device="cuda")
              for p_, x in zip(plans, xs)]
        t_single = _timed(lambda: [p_.search(x, widths, mu, sg, work=w_) for p_, x, w_ in
                                   zip(plans, xs, pw)], K, W)
        out["ms_one_plan_at_a_time"] = t_single * 1e3
    if host:
        out["host_beams"] = host
    return out


def measure_autograd(dd, workloads, K, W, train=False):
    """The 64-pulse, 336-channel, 32768-sample fp32 batch with 8 learnable taps per
    channel and 256 trials: forward, dense adjoint (weight gradient of a dense output
    gradient), sparse adjoint (the matched-filter loss reads 64 outputs), one loss step;
    with train, 300 Adam steps from the initial weights against the loss optimum."""
    import torch
    from paper_1301_3968_amd.autograd import matched_filter_loss
    print("generating the 64-pulse batch", file=sys.stderr, flush=True)
    wl = workloads.cfg5()
    Kt = wl.extra["ktaps"]
    p_ = dd.Plan(wl.freqs_ghz, wl.chan_bw_ghz, wl.dt_s, wl.dms, rule="fixed", ktaps=Kt,
                 wmode="tap", weights=wl.weights)
    x = torch.from_numpy(wl.x).cuda()
    nout = p_.out_len(x.shape[2])
    bi = np.arange(len(wl.pulses))
    di = np.array([q[1] for q in wl.pulses])
    ti = np.array([min(q[2], nout - 1) for q in wl.pulses])
    w = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
    y = torch.empty((x.shape[0], len(wl.dms), nout), dtype=torch.float32, device="cuda")
    print("timing forward and adjoints", file=sys.stderr, flush=True)
    t_fwd = _timed(lambda: p_.dedisperse(x, weights=w.detach(), out=y), K, W)
    g = torch.zeros_like(y)
    g[torch.as_tensor(bi).cuda(), torch.as_tensor(di).cuda(), torch.as_tensor(ti).cuda()] = 1.0
    t_adj_dense = _timed(lambda: p_.backward(g, x, need_x=False, need_w=True,
                                             weights=w.detach()), K, W)
    del g
    val = torch.ones(len(bi), device="cuda")
    t_adj_sparse = _timed(lambda: p_.backward_sparse(x, bi, di, ti, val), K, W)

    def step():
        w.grad = None
        matched_filter_loss(x, w, p_, bi, di, ti, sparse=True).backward()
    t_train = _timed(step, K, W)
    sums = float(x.shape[0]) * len(wl.dms) * x.shape[1] * nout
    out = {"workload": "64 x 336 ch x 32768 fp32, 256 trial DMs, 8 taps",
           "ms_forward": t_fwd * 1e3, "forward_sums_per_s": sums / t_fwd,
           "ms_adjoint_dense": t_adj_dense * 1e3, "ms_adjoint_sparse": t_adj_sparse * 1e3,
           "ms_sparse_loss_step": t_train * 1e3,
           "ratio_fwd_plus_dense_adjoint": (t_fwd + t_adj_dense) / t_fwd,
           "ratio_dense_adjoint": t_adj_dense / t_fwd,
           "ratio_fwd_plus_sparse_adjoint": (t_fwd + t_adj_sparse) / t_fwd}
    if train:
        # training from the initial weights against the optimum of the loss: w parallel to
        # G = d(sum of the pulses' outputs)/dw, the batch's dynamic-spectrum matched filter
        G = p_.backward_sparse(x, bi, di, ti, val).cpu().numpy()
        wt = torch.from_numpy(wl.weights.copy()).cuda().requires_grad_(True)
        opt = torch.optim.Adam([wt], lr=0.02)
        out["snr_initial_weights"] = -float(matched_filter_loss(x, wt, p_, bi, di, ti).detach())
        for _ in range(300):
            opt.zero_grad()
            matched_filter_loss(x, wt, p_, bi, di, ti).backward()
            opt.step()
        out["snr_after_300_adam_steps"] = -float(matched_filter_loss(x, wt, p_, bi, di,
                                                                     ti).detach())
        out["snr_matched_filter_optimum"] = float(np.linalg.norm(G)) / len(bi)
    return out


def _completeness(dd, workloads, K, W):
    """Section 5.3 completeness curves: the S/N at every trial DM (peaks) and half-way
    between adjacent trials (troughs) for the three survey examples."""
    from paper_1301_3968_amd.analyses import COMPLETENESS_CASES, completeness_case
    out = {"metric": "completeness points/s (largest S/N over trial DMs per test pulse)",
           "unit": "points/s", "dtype": "fp32", "config": {"workload": "completeness", "cases": []}}
    total_pts, total_s = 0, 0.0
    for case in COMPLETENESS_CASES:
        f = workloads.channel_centres(case[1], case[2], case[3])
        dms = dd.trial_dms(case[6], case[7], case[8], f, case[2] / case[3], case[4], cap=100000)
        true = np.concatenate([dms, 0.5 * (dms[:-1] + dms[1:])])
        completeness_case(dd, workloads, case, true[:8])          # warm-up
        plan, best, arg, _, secs = completeness_case(dd, workloads, case, true)
        D = len(dms)
        pk, tr = best[:D], best[D:]
        ratio = tr / (0.5 * (pk[:-1] + pk[1:]))
        q = max(1, D // 10)
        out["config"]["cases"].append({
            "name": case[0], "trials": D, "points": len(true), "seconds": secs,
            "peak_snr_first_tenth": float(np.mean(pk[:q])),
            "peak_snr_last_tenth": float(np.mean(pk[-q:])),
            "trough_over_peak_mean": float(np.mean(ratio)),
            "trough_over_peak_min": float(np.min(ratio)),
            "trough_over_peak_max": float(np.max(ratio)),
            "dropout_closed_form": (case[8] ** 2 + 1.0) ** -0.25,
            "pulse_found_at_own_trial": float(np.mean(arg[:D] == np.arange(D)))})
        total_pts += len(true)
        total_s += secs
    out["value"] = total_pts / total_s
    out["ms_per_step"] = total_s * 1e3
    return out


def _dm_error(dd, workloads):
    """Section 5.2: peak relative S/N against the normalised DM error, beside the closed
    form of eq. snrb/snri_approx, (x^2 + 1)^(-1/4)."""
    from paper_1301_3968_amd.analyses import dm_error_profiles, dm_error_unit
    xs = np.linspace(-8.0, 8.0, 161)
    dm_error_profiles(dd, workloads, xs[:4])                  # warm-up
    _, prof, secs = dm_error_profiles(dd, workloads, xs)
    peak = prof.max(axis=1)
    closed = (xs * xs + 1.0) ** -0.25
    pick = [0, 40, 60, 70, 75, 80, 85, 90, 100, 120, 160]
    return {"metric": "DM-error profiles/s (dedispersed test pulses about one trial DM)",
            "value": len(xs) / secs, "unit": "profiles/s", "ms_per_step": secs * 1e3,
            "dtype": "fp32",
            "config": {"workload": "700-1004 MHz x 304 ch, 1 ms, 1 ms pulse, trial DM 30, "
                                   "DM error -8..8 units",
                       "dm_error_unit": dm_error_unit(),
                       "x": [float(xs[i]) for i in pick],
                       "peak_relative_snr": [float(peak[i]) for i in pick],
                       "closed_form": [float(closed[i]) for i in pick],
                       "max_abs_difference": float(np.max(np.abs(peak - closed)))}}


def _resolution(dd, workloads):
    """Section 4: peak S/N over a grid of dt / tau and dnu / dnu_0 with greedy sample sets
    (Section 2.2) and with every non-zero sample (eq. num_samples)."""
    from paper_1301_3968_amd.analyses import res_delta_nu0, resolution_point
    grid = [0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0]
    t0 = time.perf_counter()
    g = np.array([[resolution_point(dd, workloads, a, b, "greedy")[0] for b in grid] for a in grid])
    z = np.array([[resolution_point(dd, workloads, a, b, "allnonzero")[0] for b in grid]
                  for a in grid])
    secs = time.perf_counter() - t0
    diag = np.array([g[i, i] for i in range(len(grid))])
    return {"metric": "resolution grid points/s (peak S/N, greedy and all-nonzero sample sets)",
            "value": 2 * len(grid) ** 2 / secs, "unit": "points/s", "ms_per_step": secs * 1e3,
            "dtype": "fp32",
            "config": {"workload": "700 MHz-1 GHz, 1 ms rectangular pulse, DM 30, dt/tau and "
                                   "dnu/dnu0 in 1/8..8",
                       "dnu0_mhz": res_delta_nu0() * 1e3, "grid": grid,
                       "snr_greedy": g.tolist(), "snr_allnonzero": z.tolist(),
                       "greedy_over_allnonzero_max": float(np.max(g / z)),
                       "greedy_over_allnonzero_min": float(np.min(g / z)),
                       "diagonal_greedy": diag.tolist(),
                       "diagonal_closed_form": [float((1.0 + 2.0 * m) ** -0.5) for m in grid]}}


def _detectors(dd, workloads):
    """Section 4: the four detectors against the channel width, at dt = tau and at
    dt = tau / 4 (with the finer sample time the time-series matched filter leads the
    greedy detector at fine channel widths, as the paper describes)."""
    from paper_1301_3968_amd.analyses import detector_snrs
    grid = [0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0]
    names = ["dsmf", "mf", "boxcar", "greedy"]
    t0 = time.perf_counter()
    res = {a: [detector_snrs(dd, workloads, b, a=a)[0] for b in grid] for a in (1.0, 0.25)}
    secs = time.perf_counter() - t0
    cfg = {"workload": "700 MHz-1 GHz, 1 ms rectangular pulse, DM 30, dt = tau and tau/4, "
                       "dnu/dnu0 in 1/8..8", "dnu_over_dnu0": grid}
    for a, rs in res.items():
        key = "dt_tau" if a == 1.0 else "dt_quarter_tau"
        cfg[key] = {**{k: [float(r[k]) for r in rs] for k in names},
                    "dsmf_best_everywhere": bool(all(r["dsmf"] >= max(r[k] for k in names) - 1e-9
                                                     for r in rs)),
                    "mf_over_greedy": [float(r["mf"] / r["greedy"]) for r in rs]}
    return {"metric": "detector comparisons/s (four detectors per channel width)",
            "value": 2 * len(grid) / secs, "unit": "points/s", "ms_per_step": secs * 1e3,
            "dtype": "fp32", "config": cfg}


def _fused(plan) -> bool:
    return bool(getattr(plan, "fused_search", lambda: False)())


if __name__ == "__main__":
    sys.exit(main())
