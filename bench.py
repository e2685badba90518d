"""Throughput of the GRFFE DG-FD step on one MI355X.

Workload (default): flat-space current sheet, periodic cube [-1,1]^3 with 8^3
elements of DG degree 5 (6^3 GLL nodes; 11^3 FD subcells when flagged),
eta = 1e6, CFL 0.25, seeded 1e-3 noise on B_y and E_z, adaptive DG-FD
control (about a quarter of the elements stay on FD).  One step = one
IMEX-SSP3(4,3,3) step of the whole domain (three explicit substeps, pointwise
implicit solves, filter, indicator, DG<->FD switching).

Metric: grid-point updates per second per RK substep (a DG node on DG
elements, an FD cell on FD elements, counted for each of the three substeps).

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (timed live with HIP events on its launch stream) and the CPU oracle
timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6

# Algorithmic bytes per DG node per substep moved by the register scheme:
# substep 1 reads U^n, writes U_3 and the accumulator (216 B); substep 2 reads
# U^n, U_3, A and writes U_4, A (360 B); substep 3 reads U^n, U_4, A and writes
# U^{n+1} (288 B).  Mean 288 B; the flat metric adds nothing.
DG_BYTES_PER_NODE = {1: 216.0, 2: 360.0, 3: 288.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sheet")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design note, "
                                   "rerun with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I

    torch.cuda.set_device(0)
    w = I.workload(args.workload)
    N = w["degree"]
    n3, m3 = (N + 1) ** 3, (2 * N + 1) ** 3
    p = grffe.default_params(eta=w["eta"], cfl=w["cfl"])
    exc = I.excision_mask(w) if w.get("curved") else None
    bg = None
    if w.get("curved"):
        raise SystemExit("the benchmark workload is flat; curved workloads are parity cases")
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p, bg=bg, excised=exc)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    u_fd = I.initial_data(w, xf, yf, zf)
    dom.init_from_fd(torch.from_numpy(u_fd.reshape(9, dom.E, -1)).cuda())
    dt = dom.dt()
    dom.step(args.warmup, dt)
    torch.cuda.synchronize()
    n_dg0, n_fd0 = dom.counts()
    print(f"# warm: {n_dg0} DG + {n_fd0} FD elements, dt {dt:.6e}", file=sys.stderr, flush=True)

    # timed region: the whole step; the dominant kernel is timed with HIP events
    dom.timing_enable(grffe.KERNEL_FAMILIES["dg_substep"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(args.steps, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = dom.timing_read()
    dom.timing_enable(0)
    n_dg1, n_fd1 = dom.counts()
    secs = t1 - t0
    pts = 0.5 * ((n_dg0 + n_dg1) * n3 + (n_fd0 + n_fd1) * m3)
    updates = pts * 3 * args.steps
    value = updates / secs
    # roofline: fused DG substep kernel, HBM bound; algorithmic bytes per launch
    n_dg = 0.5 * (n_dg0 + n_dg1)
    bytes_per_launch = n_dg * n3 * (sum(DG_BYTES_PER_NODE.values()) / 3.0)
    avg_s = (k_ms / 1e3) / max(k_launches, 1)
    achieved = bytes_per_launch / avg_s / 1e9
    print(f"# {args.steps} steps in {secs:.4f} s; dg_substep {k_launches} launches, mean {avg_s * 1e6:.2f} us",
          file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_sample_steps)

    out = {
        "metric": "grid-point updates/s per RK substep, FP64 vs mixed, at stated L2 error",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "flat current sheet, periodic [-1,1]^3, 8^3 elements DG-P5 / FD 11^3, "
                               "eta 1e6, CFL 0.25, adaptive DG-FD, seed 1002",
                   "elements": int(dom.E), "fd_elements": [int(n_fd0), int(n_fd1)],
                   "points_per_substep": pts, "dt": dt},
        "roofline": {"kernel": "k_dg_substep (fused DG substep)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "mean_launch_us": avg_s * 1e6, "launches": int(k_launches)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_baseline(w, steps):
    """The oracle (numpy FP64, one thread) on the same workload for `steps` steps."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import step as OS
    from oracle.domain import Domain as ODomain
    from paper_2404_01531_amd import inputs as I

    N = w["degree"]
    with threadpool_limits(limits=1):
        odom = ODomain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=dict(eta=w["eta"], cfl=w["cfl"]))
        xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
        st = OS.initial_state(odom, I.initial_data(w, xf, yf, zf))
        dt = odom.dt()
        t0 = time.perf_counter()
        pts = 0.0
        for _ in range(steps):
            nfd = int((st.rep == 1).sum())
            pts += 3 * ((odom.E - nfd) * (N + 1) ** 3 + nfd * (2 * N + 1) ** 3)
            st = OS.step(odom, st, dt)
        secs = time.perf_counter() - t0
    return {"value": pts / secs, "unit": "grid-point updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} step(s) of the same 8^3-element sheet workload from its initial state, "
                      f"numpy FP64 on one host core, {secs:.1f} s"}


if __name__ == "__main__":
    main()
