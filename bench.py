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
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic FP64 flops per subcell face per direction of the FD flux kernel:
# WENO5-Z of ten components (U and J~^d) on both sides, 20 x 78 = 1560; the two
# face fluxes F(U_L), F(U_R), 2 x 75 = 150; Rusanov 36; one cell-centred flux
# and the fourth-order corrector 75 + 36 = 111; flux difference 18.
FD_FLOP_PER_FACE = 1560 + 150 + 36 + 111 + 18

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
    ap.add_argument("--cpu-sample-steps", type=int, default=5)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def copy_probe():
    """A plain copy kernel of known size: 512 MiB read, 512 MiB written."""
    import torch
    n = 512 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8}))


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
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

    # timed region: the whole step; the dominant kernel (FD face fluxes) is timed
    # with HIP events recorded on its launch stream around every launch
    dom.timing_enable(grffe.KERNEL_FAMILIES["fd_flux"])
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
    m = 2 * N + 1
    n_fd = 0.5 * (n_fd0 + n_fd1)
    flop_per_launch = n_fd * 3 * (m + 1) * m * m * FD_FLOP_PER_FACE
    avg_s = (k_ms / 1e3) / max(k_launches, 1)
    achieved = flop_per_launch / avg_s / 1e12
    print(f"# {args.steps} steps in {secs:.4f} s; fd_flux {k_launches} launches, mean {avg_s * 1e6:.2f} us",
          file=sys.stderr, flush=True)
    # secondary: the fused DG substep kernel (HBM bound) timed over a short extra run
    dom.timing_enable(grffe.KERNEL_FAMILIES["dg_substep"])
    dom.step(max(1, args.steps // 10), dt)
    dg_ms, dg_launches = dom.timing_read()
    dom.timing_enable(0)
    n_dg = 0.5 * (n_dg0 + n_dg1)
    dg_bytes = n_dg * n3 * (sum(DG_BYTES_PER_NODE.values()) / 3.0)
    dg_avg = (dg_ms / 1e3) / max(dg_launches, 1)

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
        "roofline": {"kernel": "k_fd_flux (FD subcell WENO5-Z face fluxes)", "bound": "alu",
                     "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": None,
                     "mean_launch_us": avg_s * 1e6, "launches": int(k_launches),
                     "flop_per_launch": flop_per_launch},
        "roofline_dg": {"kernel": "k_dg_substep (fused DG substep)", "bound": "hbm",
                        "achieved": dg_bytes / dg_avg / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": dg_bytes / dg_avg / 1e9 / HBM_PEAK_GBS, "mean_launch_us": dg_avg * 1e6,
                        "bytes_per_launch": dg_bytes},
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
