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
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9   # int32 vector lane-ops/s: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
KERNEL_SRC = os.path.join(ROOT, "paper_1301_3968_amd", "csrc", "kernels_search.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_search_cfg2.json")


def _src_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(launches_per_step: int):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on the current kernel source; otherwise None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != _src_sha():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(wl, start, ntap, ndm_sample: int):
    import numpy as np

    import oracle
    pick = np.linspace(0, len(wl.dms) - 1, ndm_sample).round().astype(int)
    T = wl.x.shape[1]
    tout = T - int(np.max(start + ntap)) + 1
    t0 = time.perf_counter()
    y = oracle.dedisperse_u8(wl.x, start[pick], ntap[pick], tout=tout)
    M, S = oracle.boxcar_norm(ntap[pick], wl.widths, wl.chan_mean, wl.chan_sigma)
    oracle.boxcar_detect(y.astype(np.float64), wl.widths, M, S)
    dt = time.perf_counter() - t0
    sums = ndm_sample * wl.x.shape[0] * tout
    return {"value": sums / dt, "unit": "sums/s", "cores": 1, "kind": "oracle",
            "sample": f"{ndm_sample} of {len(wl.dms)} trials (evenly spaced), full "
                      f"{wl.x.shape[0]}x{T} block, dedisperse+norm+detect, single thread, "
                      f"{dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rule", default="allnonzero", choices=["allnonzero", "smear"])
    ap.add_argument("--cpu-sample-trials", type=int, default=48)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (the reference kernel "
                         "for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU layout "
              "is described in the design notes and not run here.", file=sys.stderr)
        return 2

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

    # Algorithmic integer ops of one launch of the dominant kernel: one add per
    # DM-channel-sample sum, plus one subtract and one max per boxcar window
    # evaluation when the detection is fused into that kernel.
    fused = os.environ.get("DEDISP_BENCH_UNFUSED") is None and _fused(plan)
    ops = sums + (2.0 * D * nout * nw if fused else 0.0)
    achieved = ops / (kern_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS, "traffic": _traffic(1),
                "kernel_ms": kern_ms, "ops_per_launch": ops}
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
    }
    if not args.no_cpu_baseline:
        print("timing the oracle on a sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, start, ntap, args.cpu_sample_trials)
    print(json.dumps(line), flush=True)
    return 0


def _fused(plan) -> bool:
    return bool(getattr(plan, "fused_search", lambda: False)())


if __name__ == "__main__":
    sys.exit(main())
