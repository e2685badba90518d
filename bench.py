"""Throughput of the GRFFE DG-FD step on one MI355X.

Workload (the JSON line): the Kerr-Schild black hole, M = 1, a = 0.9, uniform seed
field B0 = 1 with the ideal E, [-40,40]^3 cut into 16^3 elements of DG degree 5
(6^3 GLL nodes; 11^3 FD subcells when flagged), the 8 elements meeting r < 1.8
excised, no-incoming-Poynting outer faces, eta = 1e5, CFL 0.25, adaptive DG-FD
control from an all-DG start.  One step = one IMEX-SSP3(4,3,3) step of the whole
domain (three explicit substeps, pointwise implicit solves, filter, indicator,
DG<->FD switching), FP64; the same in the mixed mode beside it.

Metric: grid-point updates per second per RK substep (a DG node on DG elements, an
FD cell on FD elements, counted for each of the three substeps).

Prints one JSON line with the throughput, the roofline of the dominant kernel (the
fused curved DG substep, timed live with HIP events on its launch stream), the
whole step's algorithmic HBM rate, the error against the oracle on sampled elements,
and the oracle timed on a bounded sample on the host.
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
# The curved background adds its 26 FP64 fields per node, read once per substep.
DG_BG_BYTES_PER_NODE = 26 * 8.0

# Kernel timing: HIP events on the launches of one step in every TIMING_PERIOD of
# the timed region.
TIMING_PERIOD = 10

# HBM bytes per FD element per launch of k_fd_flux (FP64, flat): rocprofv3 FETCH_SIZE
# and WRITE_SIZE runs on the current-sheet 8^3 workload (KiB per dispatch, 12
# dispatches with 128 FD elements: fetch 14825.0, write 36232.7), each scaled by what
# the same counter reads for a plain 512 MiB device copy (fetch x 2.0, write x 1.0).
# Valid for the kernel source whose hash is FD_FLUX_TRAFFIC_SRC; reported as null for
# any other source.
FD_FLUX_TRAFFIC_PER_FD_ELEMENT = (2.0 * 14825.0 + 1.0 * 36232.7) * 1024.0 / 128.0
FD_FLUX_TRAFFIC_SRC = "b4e40c45594c6e0f"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--only", choices=("sheet", "batch", "adjoint_adaptive", "shell_wald", "vacuum_wald", "shell_scale",
                                        "shell_hybrid"),
                    default=None,
                    help="run one secondary workload alone and print its record (profiling runs)")
    ap.add_argument("--shell-degrees", default="5,7,9",
                    help="degrees of the exact-Wald shell rows (--only shell_wald)")
    ap.add_argument("--spins", default="0,0.5,0.7,0.8", help="spins of the vacuum Wald runs (--only vacuum_wald)")
    ap.add_argument("--coords", choices=("cartesian", "spherical"), default="spherical",
                    help="Kerr-Schild coordinates of the vacuum Wald runs (--only vacuum_wald)")
    ap.add_argument("--contraction", choices=("valu", "mfma"), default="valu",
                    help="DG derivative contraction engine of the black-hole domains (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=12)
    ap.add_argument("--extras", choices=("core", "all", "none"), default="core",
                    help="also measure the batch, sheet, full-length black-hole and adjoint workloads (core), "
                         "and the paper's accuracy experiments (all); nested in the JSON line")
    ap.add_argument("--extra-steps", type=int, default=30)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--rotator", action="store_true",
                    help="only run the rotating-star spin-down sweep (inclinations 0, 30, 45, 60, 90 degrees, "
                         "two periods each, about 7 minutes) and fit L = L0 (k1 + k2 sin^2 theta)")
    ap.add_argument("--rotator-frame", choices=("inertial", "rotating"), default="inertial",
                    help="grid at rest or rotating with the star (the rotating frame's shift; its CFL step is "
                         "smaller by the shift's speed at the box corners)")
    ap.add_argument("--rotator-angles", default="0,30,45,60,90", help="inclinations in degrees")
    ap.add_argument("--rotator-periods", type=float, default=2.0)
    return ap.parse_args()


def rotator_sweep(frame="inertial", degrees=(0.0, 30.0, 45.0, 60.0, 90.0), periods=2.0):
    """Spin-down luminosity against inclination (Sec. IV C, oblique rotator): one JSON
    line per angle, then the least-squares fit of L / L(0) = k1 + k2 sin^2 theta
    (when the first angle is 0 and there are three or more)."""
    import math

    import numpy as np
    L = []
    angles = [math.radians(a) for a in degrees]
    for th in angles:
        r = run_rotator(th, periods=periods, frame=frame)
        print(json.dumps(r), flush=True)
        L.append(r["luminosity"])
    if len(angles) >= 3 and angles[0] == 0.0:
        s2 = np.sin(np.asarray(angles)) ** 2
        k2, k1 = np.polyfit(s2, np.asarray(L) / L[0], 1)
        print(json.dumps({"fit": "L/L(0) = k1 + k2 sin^2 theta", "frame": frame, "k1": float(k1), "k2": float(k2)}),
              flush=True)


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


def run_workload(w, precision, steps, warmup, families):
    """Start-up, warm-up and `steps` timed steps of workload w at one precision.
    Returns the timing record and the final state (device tensors)."""
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I

    N = w["degree"]
    n3, m3 = (N + 1) ** 3, (2 * N + 1) ** 3
    p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], precision=precision)
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    u_fd = I.initial_data(w, xf, yf, zf)
    dom.init_from_fd(torch.from_numpy(u_fd.reshape(9, dom.E, -1)).cuda())
    dt = dom.dt()
    dom.step(warmup, dt)
    torch.cuda.synchronize()
    n_dg0, n_fd0 = dom.counts()
    # timed region: the whole step; the listed kernel families are timed with HIP
    # events attached to their own dispatches on the launch stream, in one step of
    # every TIMING_PERIOD (the events cost a few microseconds per timed launch)
    dom.timing_enable(*families, period=TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(steps, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {f: dom.timing_read(f) for f in families}
    dom.timing_enable()
    n_dg1, n_fd1 = dom.counts()
    secs = t1 - t0
    pts = 0.5 * ((n_dg0 + n_dg1) * n3 + (n_fd0 + n_fd1) * m3)
    rec = dict(secs=secs, value=pts * 3 * steps / secs, pts=pts, dt=dt, E=dom.E, n_dg=(n_dg0, n_dg1),
               n_fd=(n_fd0, n_fd1), kern=kern)
    return rec, dom.get_state()


def state_diff(a, b):
    """Max and RMS difference per variable group (E~, B~, psi~, phi~, q~) of two
    states, each relative to the group's scale in `b` (floored at 1e-3 of the whole
    state's), over the elements held in the same representation by both."""
    import numpy as np
    dga, fda, repa = (x.cpu().numpy() for x in a)
    dgb, fdb, repb = (x.cpu().numpy() for x in b)
    same = repa == repb
    groups = ((0, 3), (3, 6), (6, 7), (7, 8), (8, 9))
    mx = np.zeros(5)
    sq = np.zeros(5)
    ref_sq = np.zeros(5)
    cnt = np.zeros(5)
    ref_max = np.zeros(5)
    for r, A, B in ((0, dga, dgb), (1, fda, fdb)):
        el = np.nonzero(same & (repb == r))[0]
        if el.size == 0:
            continue
        A, B = A[:, el], B[:, el]
        for g, (lo, hi) in enumerate(groups):
            d = A[lo:hi] - B[lo:hi]
            mx[g] = max(mx[g], np.abs(d).max())
            sq[g] += (d ** 2).sum()
            ref_sq[g] += (B[lo:hi] ** 2).sum()
            cnt[g] += d.size
            ref_max[g] = max(ref_max[g], np.abs(B[lo:hi]).max())
    rms_ref = np.sqrt(ref_sq / np.maximum(cnt, 1))
    rms_all = np.sqrt(ref_sq.sum() / max(cnt.sum(), 1))
    max_all = ref_max.max()
    rel_max = mx / np.maximum(ref_max, 1e-3 * max_all)
    rel_l2 = np.sqrt(sq / np.maximum(cnt, 1)) / np.maximum(rms_ref, 1e-3 * rms_all)
    names = ["E", "B", "psi", "phi", "q"]
    return {"max": dict(zip(names, rel_max.tolist())), "l2": dict(zip(names, rel_l2.tolist())),
            "elements_compared": int(same.sum()), "elements_rep_differs": int((~same).sum())}


def _dg_nodes(w):
    """DG node coordinates of workload w from the library's own GLL nodes."""
    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    return I.points(w["n_elem"], w["lower"], w["upper"], grffe.operator(w["degree"], 0))


def _time_steps(step, steps, warmup):
    import torch
    step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


CONTRACTION = 0  # DG derivative contraction engine of the black-hole domains (--contraction)


def kerr_schild_domain(precision, n_elem=16):
    """The Kerr-Schild black-hole domain (M = 1, a = 0.9, B0 = 1, Wald-like data with
    the ideal E), [-40,40]^3 with n_elem^3 DG-P5 elements, elements meeting r < 1.8
    excised, every element on DG.  Returns (domain, workload, excision mask, DG node
    coordinates)."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    w = I.workload("kerr_schild", n_elem=(n_elem,) * 3)
    N = w["degree"]
    x, y, z = _dg_nodes(w)
    with np.errstate(all="ignore"):
        bg = I.background(w, x, y, z)
        u = I.initial_data(w, x, y, z)
    exc = I.excision_mask(w)
    E, n3 = int(np.prod(w["n_elem"])), (N + 1) ** 3
    bg = bg.reshape(26, E, n3)
    u = u.reshape(9, E, n3)
    bg[:, exc.astype(bool)] = 0.0
    bg[0, exc.astype(bool)] = 1.0
    bg[4, exc.astype(bool)] = bg[7, exc.astype(bool)] = bg[9, exc.astype(bool)] = 1.0
    u[:, exc.astype(bool)] = 0.0
    p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], precision=precision)
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p,
                       bg=torch.from_numpy(np.ascontiguousarray(bg)).cuda(), excised=exc)
    m3 = (2 * N + 1) ** 3
    dom.set_contraction(CONTRACTION)
    dom.set_state(torch.from_numpy(np.ascontiguousarray(u)).cuda(),
                  torch.zeros((9, E, m3), dtype=torch.float64, device="cuda"),
                  torch.zeros(E, dtype=torch.int32, device="cuda"))
    return dom, w, exc, (x, y, z)


def run_kerr_schild(steps, warmup, precision, n_elem=16, families=None):
    """Kerr-Schild black hole (M = 1, a = 0.9, B0 = 1, Wald-like data with the ideal
    E), [-40,40]^3 with n_elem^3 DG-P5 elements, elements meeting r < 1.8 excised,
    every element starting on DG: `warmup` untimed steps, then `steps` timed steps.
    The listed kernel families are timed with HIP events attached to their own
    dispatches on the launch stream, on the launches of one step in every
    TIMING_PERIOD (family 1, the fused DG substep, is the dominant kernel)."""
    import torch

    from paper_2404_01531_amd import grffe
    dom, w, exc, _ = kerr_schild_domain(precision, n_elem)
    N = w["degree"]
    n3, m3 = (N + 1) ** 3, (2 * N + 1) ** 3
    dt = dom.dt()
    fams = tuple(families) if families else (grffe.KERNEL_FAMILIES["dg_substep"],)
    dom.step(warmup, dt)
    torch.cuda.synchronize()
    n_dg0, n_fd0 = dom.counts()
    dom.timing_enable(*fams, period=min(TIMING_PERIOD, max(1, steps // 2)))
    secs = _time_steps(lambda k: dom.step(k, dt), steps, 0)
    kern = {f: dom.timing_read(f) for f in fams}
    dom.timing_enable()
    n_dg1, n_fd1 = dom.counts()
    n_bad = dom.check_finite()
    state = dom.get_state()
    dom.close()
    pts = 0.5 * ((n_dg0 + n_dg1) * n3 + (n_fd0 + n_fd1) * m3)
    n_dg = 0.5 * (n_dg0 + n_dg1)
    fam = grffe.KERNEL_FAMILIES["dg_substep"]
    k_ms, k_n = kern[fam]
    byt = n_dg * n3 * (sum(DG_BYTES_PER_NODE.values()) / 3.0 + DG_BG_BYTES_PER_NODE)
    avg = (k_ms / 1e3) / max(k_n, 1)
    # the whole step's algorithmic bytes: every DG node and FD cell moves the register
    # scheme's mean 288 B and reads its 208 B of background in each of three substeps
    step_bytes = 3 * pts * (sum(DG_BYTES_PER_NODE.values()) / 3.0 + DG_BG_BYTES_PER_NODE)
    ms = secs * 1e3 / steps
    names = {v: k for k, v in grffe.KERNEL_FAMILIES.items()}
    rec = {"workload": f"Kerr-Schild black hole M=1 a=0.9, uniform seed field B0=1 with the ideal E, [-40,40]^3, "
                       f"{n_elem}^3 elements DG-P5 (FD 11^3 when flagged), {int(exc.sum())} elements excised "
                       f"(r < 1.8), eta 1e5, CFL 0.25, adaptive DG-FD, start on DG",
           "dtype": "f64" if precision == 0 else "mixed",
           "value": pts * 3 * steps / secs, "unit": "grid-point updates/s", "steps": steps,
           "ms_per_step": ms, "dt": dt, "elements": int(dom.E), "live_elements": int(dom.E - exc.sum()),
           "elements_dg_fd": [[int(n_dg0), int(n_fd0)], [int(n_dg1), int(n_fd1)]],
           "points_per_substep": pts, "non_finite_elements": n_bad,
           "roofline": {"kernel": "k_dg_substep (fused DG substep, curved)", "bound": "hbm",
                        "achieved": byt / avg / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": byt / avg / 1e9 / HBM_PEAK_GBS, "traffic": None, "mean_launch_us": avg * 1e6,
                        "launches": int(k_n), "bytes_per_launch": byt},
           "step_hbm": {"algorithmic_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / (ms / 1e3) / 1e9,
                        "frac": step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
           "kernels_mean_us": {names[f]: {"mean_us": kern[f][0] * 1e3 / max(kern[f][1], 1),
                                          "launches": int(kern[f][1])} for f in fams}}
    return rec, state


def run_kerr_schild_full(precision=0, n_elem=16, steps=1000, segment=100):
    """The Kerr-Schild configuration over its full length (1000 steps, t = 61.5M) from
    the initial data: the rate of every 100-step segment and of the whole run, with the
    FD element count at each segment's end (the elements by the box's outer faces
    switch to FD as the transient meets the no-incoming-Poynting faces)."""
    import torch
    dom, w, exc, _ = kerr_schild_domain(precision, n_elem)
    N = w["degree"]
    n3, m3 = (N + 1) ** 3, (2 * N + 1) ** 3
    dt = dom.dt()
    rows, tot_pts, tot_secs = [], 0.0, 0.0
    a0, f0 = dom.counts()
    for s in range(0, steps, segment):
        secs = _time_steps(lambda k: dom.step(k, dt), segment, 0)
        a1, f1 = dom.counts()
        pts = 0.5 * ((a0 + a1) * n3 + (f0 + f1) * m3) * 3 * segment
        rows.append({"steps": [s + 1, s + segment], "fd_elements_end": int(f1), "ms_per_step": secs * 1e3 / segment,
                     "value": pts / secs})
        tot_pts += pts
        tot_secs += secs
        a0, f0 = a1, f1
    n_bad = dom.check_finite()
    dom.close()
    torch.cuda.empty_cache()
    return {"workload": f"the Kerr-Schild {n_elem}^3 configuration over its full {steps} steps (t = {steps * dt:.1f}M)",
            "dtype": "f64" if precision == 0 else "mixed", "value": tot_pts / tot_secs,
            "unit": "grid-point updates/s", "ms_per_step": tot_secs * 1e3 / steps, "segments": rows,
            "non_finite_elements": n_bad}


GOLDEN_KS = os.path.join(ROOT, "tests", "golden", "kerr_schild_16_p5_10steps.npz")


def kerr_schild_parity(precision, floor):
    """Error of the Kerr-Schild 16^3 run against the oracle: the library's first 10 steps
    from the initial data against the stored oracle run of the same configuration
    (tests/golden/kerr_schild_16_p5_10steps.npz, written by make_kerr_schild_16.py
    beside it from the oracle and the seeded inputs), on its sampled elements.  Per
    variable group (E~, B~, psi~, phi~, q~): the largest and the RMS difference, each
    relative to the group's own scale floored at `floor` times the whole state's."""
    import numpy as np
    ref = np.load(GOLDEN_KS)
    dom, w, exc, _ = kerr_schild_domain(precision, 16)
    N = w["degree"]
    dt = dom.dt()
    mism = 0
    for k in range(int(ref["steps"])):
        dom.step(1, dt)
        _, _, rep = dom.get_state()
        mism = max(mism, int((rep.cpu().numpy() != ref["rep"][k]).sum()))
    dg, fd, rep = (x.cpu().numpy() for x in dom.get_state())
    dom.close()
    E = dg.shape[1]
    got = np.concatenate([dg[:, ref["dg_elements"]].reshape(9, -1), fd[:, ref["fd_elements"]].reshape(9, -1)], axis=1)
    want = np.concatenate([ref["dg_values"].reshape(9, -1), ref["fd_values"].reshape(9, -1)], axis=1)
    groups = ((0, 3), (3, 6), (6, 7), (7, 8), (8, 9))
    names = ["E", "B", "psi", "phi", "q"]
    amax, rms_all = np.abs(want).max(), np.sqrt(np.mean(want ** 2))
    mx, l2 = {}, {}
    for nm, (a, b) in zip(names, groups):
        d = got[a:b] - want[a:b]
        mx[nm] = float(np.abs(d).max() / max(np.abs(want[a:b]).max(), floor * amax))
        l2[nm] = float(np.sqrt(np.mean(d ** 2)) / max(np.sqrt(np.mean(want[a:b] ** 2)), floor * rms_all))
    return {"reference": "stored oracle run (tests/golden/kerr_schild_16_p5_10steps.npz)",
            "steps": int(ref["steps"]), "dt": float(ref["dt"]),
            "sampled_elements": {"dg": int(ref["dg_elements"].size), "fd": int(ref["fd_elements"].size)},
            "representation_mismatches": mism, "group_scale_floor": floor, "max": mx, "l2": l2}


def run_rotator(theta, periods=2.0, n_elem=24, half_width=12.0, r_measure=6.0, samples=8, frame="inertial"):
    """Rotating magnetised star (Sec. IV C): the regularised dipole of inclination
    theta inside a perfect conductor of radius R = 1 rotating at Omega = 0.2 about z,
    flat space, [-half_width, half_width]^3 with n_elem^3 P5 elements (one element per
    R at the defaults), no-incoming-Poynting faces, eta = 1e5, CFL 0.25, adaptive
    DG/FD.  After `periods` rotation periods the Poynting luminosity through the
    sphere r = r_measure (Eq. of the spin-down luminosity; FD elements taken through
    R to their DG polynomial) is averaged over the last tenth of a period.
    frame = "rotating": the grid rotates with the star (flat space with the rotating
    frame's shift, the conductor at rest on the grid); its normal observers are the
    inertial ones, so E, B and the luminosity are measured the same way."""
    import math

    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    from paper_2404_01531_amd.poynting import SphereFlux
    w = I.workload("rotator", n_elem=(n_elem,) * 3, lower=(-half_width,) * 3, upper=(half_width,) * 3, theta=theta,
                   frame=frame)
    N = w["degree"]
    p = grffe.default_params(eta=w["eta"], cfl=w["cfl"])
    bg = None
    if frame == "rotating":
        bg = I.background(w, *_dg_nodes(w)).reshape(26, int(np.prod(w["n_elem"])), -1)
        bg = torch.from_numpy(np.ascontiguousarray(bg)).cuda()
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p, bg=bg)
    del bg
    dom.set_conductor(w["centre"], w["radius"], 0.0 if frame == "rotating" else w["omega"])
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    E = int(np.prod(w["n_elem"]))
    dom.init_from_fd(torch.from_numpy(np.ascontiguousarray(I.initial_data(w, xf, yf, zf).reshape(9, E, -1))).cuda())
    del xf, yf, zf
    dt = dom.dt()
    period = 2.0 * math.pi / w["omega"]
    total = int(math.ceil(periods * period / dt))
    tail = int(math.ceil(0.1 * period / dt))
    flux = SphereFlux(w, R=r_measure)

    def luminosity():
        dg, fd, rep = dom.get_state()
        el = torch.nonzero(rep == 1).flatten().to(torch.int32)
        if el.numel():
            dg[:, el.long()] = dom.reconstruct_fd_to_dg(fd[:, el.long()].contiguous(), el)
        return float(flux(dg))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < total - tail:
        k = min(1000, total - tail - done)
        dom.step(k, dt)
        done += k
        torch.cuda.synchronize()
        print(f"# rotator theta {theta:.3f} ({frame} frame): step {done} of {total}", file=sys.stderr, flush=True)
    Ls = []
    chunk = max(1, tail // samples)
    done = total - tail
    while done < total:
        k = min(chunk, total - done)
        dom.step(k, dt)
        done += k
        Ls.append(luminosity())
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    n_dg, n_fd = dom.counts()
    # where the FD elements are: the band around the equatorial plane beyond the
    # light cylinder (the current sheet) against the polar caps inside it
    _, _, rep = dom.get_state()
    on_fd = rep.cpu().numpy() == 1
    h = (w["upper"][0] - w["lower"][0]) / w["n_elem"][0]
    idx = np.arange(E)
    ne = w["n_elem"][0]
    cx, cy, cz = (w["lower"][0] + h * (0.5 + v) for v in (idx % ne, (idx // ne) % ne, idx // (ne * ne)))
    rho = np.hypot(cx, cy)
    lc = 1.0 / w["omega"]
    sheet = (np.abs(cz) < 1.5 * h) & (rho > 1.2 * lc) & (rho < 2.0 * lc)
    polar = (np.abs(cz) > 1.2 * lc) & (np.abs(cz) < 2.0 * lc) & (rho < 0.6 * lc)
    L0 = 4.0 * math.pi * w["mu"] ** 2 * w["omega"] ** 4
    return {"theta": theta, "frame": frame, "steps": total, "dt": dt, "t": total * dt, "seconds": secs,
            "luminosity": float(np.mean(Ls)), "luminosity_spread": float(np.ptp(Ls)),
            "luminosity_over_4pi_mu2_omega4": float(np.mean(Ls)) / L0, "elements_dg_fd": [int(n_dg), int(n_fd)],
            "fd_fraction_equatorial_band": float(on_fd[sheet].mean()), "fd_fraction_polar": float(on_fd[polar].mean()),
            "non_finite_elements": dom.check_finite()}


def run_batch(steps, warmup, precision, use_graph=True):
    """64 independent flat periodic domains (n^3 elements, n ~ U{4..12}, degree
    N ~ U{3..7}, wave or sheet), each advanced by its own CFL step, one call per step
    (every pool on the VALU contraction)."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    ws = I.batch_workloads()
    b = grffe.Batch([dict(n_elem=w["n_elem"], lower=w["lower"], upper=w["upper"], degree=w["degree"],
                          bc=w["bc"]) for w in ws], params=dict(eta=1e6, cfl=0.25, precision=precision))
    nodes = 0
    for k, w in enumerate(ws):
        N = w["degree"]
        E, n3, m3 = int(np.prod(w["n_elem"])), (N + 1) ** 3, (2 * N + 1) ** 3
        x, y, z = _dg_nodes(w)
        u = I.initial_data(w, x, y, z).reshape(9, E, n3)
        b.set_state(k, torch.from_numpy(np.ascontiguousarray(u)).cuda(),
                    torch.zeros((9, E, m3), dtype=torch.float64, device="cuda"),
                    torch.zeros(E, dtype=torch.int32, device="cuda"))
        nodes += E * n3
    torch.cuda.synchronize()
    b.step(warmup, use_graph=use_graph)
    torch.cuda.synchronize()

    def points():
        tot = fd = 0
        for k, w in enumerate(ws):
            N = w["degree"]
            a, f = b.counts(k)
            tot += a * (N + 1) ** 3 + f * (2 * N + 1) ** 3
            fd += f
        return tot, fd

    p0, f0 = points()
    secs = _time_steps(lambda k: b.step(k, use_graph=use_graph), steps, 0)
    p1, f1 = points()
    pts = 0.5 * (p0 + p1)
    return {"workload": "64 flat periodic domains on [-1,1]^3, n^3 elements n~U{4..12}, DG degree ~U{3..7}, "
                        "wave or sheet, eta 1e6, CFL 0.25, adaptive DG-FD, one HIP-graph launch per step",
            "dtype": "f64" if precision == 0 else "mixed", "domains": len(ws), "dg_nodes": nodes,
            "degrees": sorted({w["degree"] for w in ws}), "value": pts * 3 * steps / secs,
            "unit": "grid-point updates/s", "steps": steps, "ms_per_step": secs * 1e3 / steps,
            "fd_elements": [int(f0), int(f1)],
            "hbm_GBps_dg_state": (nodes * sum(DG_BYTES_PER_NODE.values())) * steps / secs / 1e9,
            "contraction_per_degree": "valu"}


def run_adjoint(steps=200, every=20, check_steps=10):
    """The adjoint workload: Kerr-Schild black hole (a = 0.9), [-40,40]^3 with 8^3
    DG-P5 elements (all DG, 8 excised), initial field with four seeded parameters
    (B0, tilt, dipole amplitude, dipole offset from the spin axis); objective the
    outgoing Poynting flux through r = 20 integrated over the steps; its gradient
    with respect to the parameters through the checkpointed step adjoint, timed
    against the forward run.  The gradient is checked by central differences of the
    objective over `check_steps` steps: over the full horizon the objective crosses
    many flips of the boundary state's inward/outward switch (it is piecewise
    smooth in the parameters), and differences at any step size straddle some."""
    import torch

    from paper_2404_01531_amd import inputs as I
    from paper_2404_01531_amd.poynting import AdjointWorkload, time_integral, time_integral_gradient
    w = I.workload("kerr_schild", n_elem=(8, 8, 8))
    aw = AdjointWorkload(w)
    params = I.adjoint_parameters()
    u0 = aw.initial(params)
    du = aw.initial_derivatives(params)
    time_integral(aw.dom, u0, 2, aw.dt, aw.L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi = time_integral(aw.dom, u0, steps, aw.dt, aw.L)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # one step adjoint against one forward step
    lam = torch.ones_like(u0)
    aw.dom.step_adjoint(u0, lam, aw.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        lam = aw.dom.step_adjoint(u0, lam, aw.dt)
    torch.cuda.synchronize()
    t_adj1 = (time.perf_counter() - t0) / 20
    t0 = time.perf_counter()
    phi_g, lam0 = time_integral_gradient(aw.dom, u0, steps, aw.dt, every, aw.L)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    grad = {k: float((lam0 * du[k]).sum()) for k in aw.PARAMS}
    _, lam_c = time_integral_gradient(aw.dom, u0, check_steps, aw.dt, every, aw.L)
    check = {}
    for k in aw.PARAMS:
        g = float((lam_c * du[k]).sum())
        row = {"adjoint": g}
        errs = []
        for rel in (1e-4, 1e-5, 1e-6):
            h = rel * max(1.0, abs(params[k]))
            fd = (aw.phi(dict(params, **{k: params[k] + h}), check_steps)
                  - aw.phi(dict(params, **{k: params[k] - h}), check_steps)) / (2 * h)
            row[f"fd_rel_step_{rel:g}"] = fd
            errs.append(abs(g - fd) / max(abs(fd), 1e-300))
        row["best_rel_err"] = min(errs)
        check[k] = row
    aw.close()
    return {"workload": f"Kerr-Schild a=0.9, [-40,40]^3, 8^3 elements DG-P5 (all DG), {int(aw.exc.sum())} excised; "
                        f"Phi = sum_n dt * (outgoing Poynting flux through r=20, 32x64 points) over {steps} steps; "
                        f"gradient w.r.t. (B0, tilt, dipole amplitude, dipole offset), checkpoints every {every}",
            "dtype": "f64", "parameters": params, "phi": phi, "phi_from_gradient_pass": phi_g,
            "forward_ms_per_step": t_fwd * 1e3 / steps,
            "step_adjoint_ms": t_adj1 * 1e3,
            "step_adjoint_over_forward": t_adj1 / (t_fwd / steps),
            "gradient_ms_total": t_grad * 1e3,
            "gradient_over_forward": t_grad / t_fwd,
            "gradient": grad,
            "gradient_check_steps": check_steps,
            "gradient_check": check,
            "gradient_check_note": "central differences of the objective at three relative steps; the objective is "
                                   "piecewise smooth (the boundary state's inward/outward switch flips at isolated "
                                   "parameter values), so a step whose window holds a flip disagrees with every "
                                   "other step and with the adjoint"}


def run_adjoint_adaptive(steps=200, every=20, check_steps=10):
    """The adjoint workload with the hybrid control on (the paper's eta = 1e5, adaptive
    indicator; elements go to FD near the hole and where the dipole is sharp): Phi over
    `steps` steps and its gradient with the forward pass's decisions frozen
    (rollbacks and switches back of every step, grffe_step_adjoint_frozen).  The
    gradient check over `check_steps` steps lists central differences at three small
    relative steps with a flag for perturbed runs whose decisions differ."""
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    from paper_2404_01531_amd.poynting import AdjointWorkload, time_integral, time_integral_gradient
    w = I.workload("kerr_schild", n_elem=(8, 8, 8))
    aw = AdjointWorkload(w, hybrid=grffe.HYBRID_ADAPTIVE)
    params = I.adjoint_parameters()
    u0 = aw.initial(params)
    du = aw.initial_derivatives(params)
    time_integral(aw.dom, u0, 2, aw.dt, aw.L)
    # the forward pass alone (steps only) and with the objective evaluated every step
    aw.dom.set_state(u0, torch.zeros(aw.dom.fd_shape(), dtype=torch.float64, device="cuda"),
                     torch.zeros(aw.E, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    aw.dom.step(steps, aw.dt)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    log = []
    t0 = time.perf_counter()
    phi = time_integral(aw.dom, u0, steps, aw.dt, aw.L, log)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    n_fd = [int(r.sum()) for r in log]
    # one frozen step adjoint (re-runs its step) from a state with FD elements
    st = aw.dom.get_state()
    mu = (torch.ones_like(st[0]), torch.ones_like(st[1]))
    aw.dom.step_adjoint_frozen(*st, *mu, aw.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        aw.dom.step_adjoint_frozen(*st, *mu, aw.dt)
    torch.cuda.synchronize()
    t_adj1 = (time.perf_counter() - t0) / 10
    aw.dom.set_state(*st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    aw.dom.step(10, aw.dt)
    torch.cuda.synchronize()
    t_step_late = (time.perf_counter() - t0) / 10
    t0 = time.perf_counter()
    phi_g, lam0 = time_integral_gradient(aw.dom, u0, steps, aw.dt, every, aw.L)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    grad = {k: float((lam0 * du[k]).sum()) for k in aw.PARAMS}
    log_c = []
    _, lam_c = time_integral_gradient(aw.dom, u0, check_steps, aw.dt, every, aw.L, log_c)
    check = {}
    for k in aw.PARAMS:
        g = float((lam_c * du[k]).sum())
        row = {"adjoint": g}
        for rel in (1e-6, 1e-7, 1e-8):
            h = rel * max(1.0, abs(params[k]))
            lp, lm = [], []
            fd = (aw.phi(dict(params, **{k: params[k] + h}), check_steps, lp)
                  - aw.phi(dict(params, **{k: params[k] - h}), check_steps, lm)) / (2 * h)
            same = all(torch.equal(a, b) and torch.equal(a, c) for a, b, c in zip(log_c, lp, lm))
            row[f"fd_rel_step_{rel:g}"] = {"value": fd, "rel_err": abs(g - fd) / max(abs(fd), 1e-300),
                                           "same_decisions": bool(same)}
        check[k] = row
    aw.close()
    return {"workload": f"Kerr-Schild a=0.9, [-40,40]^3, 8^3 elements DG-P5 / FD 11^3, {int(aw.exc.sum())} excised, "
                        f"eta 1e5, adaptive DG-FD (start on DG); Phi = sum_n dt * (outgoing Poynting flux through "
                        f"r=20, 32x64 points, FD elements through R) over {steps} steps; gradient w.r.t. (B0, tilt, "
                        f"dipole amplitude, dipole offset) with the forward pass's decisions frozen, checkpoints "
                        f"every {every}",
            "dtype": "f64", "parameters": params, "phi": phi, "phi_from_gradient_pass": phi_g,
            "fd_elements_every_20_steps": n_fd[::20], "fd_elements_end": n_fd[-1] if n_fd else 0,
            "forward_steps_only_ms_per_step": t_steps * 1e3 / steps,
            "forward_with_objective_ms_per_step": t_fwd * 1e3 / steps,
            "step_ms_at_end_state": t_step_late * 1e3,
            "step_adjoint_frozen_ms_at_end_state": t_adj1 * 1e3,
            "step_adjoint_over_step_at_end_state": t_adj1 / t_step_late,
            "gradient_ms_total": t_grad * 1e3,
            "gradient_over_forward_with_objective": t_grad / t_fwd,
            "gradient": grad,
            "gradient_check_steps": check_steps,
            "gradient_check": check,
            "gradient_check_note": "the frozen-decision gradient of a piecewise-smooth objective; with elements on FD "
                                   "at eta = 1e5 the objective is rough at small scales (stiff relaxation over "
                                   "WENO5-Z weights), so the differences approach the adjoint only as the step "
                                   "shrinks"}


def roofline_fd(rec, N, counted=True):
    """FP64-ALU roofline of the FD face-flux kernel from the run record's timed launches;
    the counter traffic is attached only to the counted source and workload."""
    from paper_2404_01531_amd import grffe
    m = 2 * N + 1
    k_ms, k_n = rec["kern"][grffe.KERNEL_FAMILIES["fd_flux"]]
    n_fd = 0.5 * sum(rec["n_fd"])
    flop = n_fd * 3 * (m + 1) * m * m * FD_FLOP_PER_FACE
    avg = (k_ms / 1e3) / max(k_n, 1)
    ach = flop / avg / 1e12
    return {"kernel": "k_fd_flux (FD subcell WENO5-Z face fluxes)", "bound": "alu", "achieved": ach,
            "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_VALU_PEAK_TFLOPS,
            "traffic": (FD_FLUX_TRAFFIC_PER_FD_ELEMENT * n_fd
                        if counted and kernel_source_hash() == FD_FLUX_TRAFFIC_SRC else None),
            "mean_launch_us": avg * 1e6, "launches": int(k_n), "flop_per_launch": flop}


def roofline_dg(rec, N):
    """HBM roofline of the fused flat DG substep kernel from the run record's timed launches."""
    from paper_2404_01531_amd import grffe
    k_ms, k_n = rec["kern"][grffe.KERNEL_FAMILIES["dg_substep"]]
    n_dg = 0.5 * sum(rec["n_dg"])
    byt = n_dg * (N + 1) ** 3 * (sum(DG_BYTES_PER_NODE.values()) / 3.0)
    avg = (k_ms / 1e3) / max(k_n, 1)
    return {"kernel": "k_dg_substep (fused DG substep)", "bound": "hbm", "achieved": byt / avg / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": byt / avg / 1e9 / HBM_PEAK_GBS,
            "mean_launch_us": avg * 1e6, "launches": int(k_n), "bytes_per_launch": byt}


def run_sheet_sweep(steps, warmup, sizes=(16, 32)):
    """The benchmark's current sheet on the same domain with n^3 elements (h = 2/n):
    the element-count diagnostic, FP64, adaptive DG-FD, the sheet workload's seed."""
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    fam = (grffe.KERNEL_FAMILIES["fd_flux"], grffe.KERNEL_FAMILIES["dg_substep"])
    rows = []
    for n in sizes:
        w = I.workload("sheet", n_elem=(n, n, n))
        rec, st = run_workload(w, 0, steps, warmup, fam)
        del st
        torch.cuda.empty_cache()
        rf, rd = roofline_fd(rec, w["degree"], counted=False), roofline_dg(rec, w["degree"])
        rows.append({"n_elem": n, "elements": int(rec["E"]), "fd_elements": [int(x) for x in rec["n_fd"]],
                     "value": rec["value"], "ms_per_step": rec["secs"] * 1e3 / steps, "dt": rec["dt"],
                     "fd_flux_tflops": rf["achieved"], "fd_flux_mean_us": rf["mean_launch_us"],
                     "dg_substep_gbs": rd["achieved"], "dg_substep_frac": rd["frac"],
                     "dg_substep_mean_us": rd["mean_launch_us"]})
    return {"workload": "current sheet, periodic [-1,1]^3, n^3 elements DG-P5 / FD 11^3, eta 1e6, CFL 0.25, "
                        "adaptive DG-FD, seed 1002, fp64 (element-count diagnostic)",
            "unit": "grid-point updates/s", "steps": steps, "rows": rows}


def run_forced_fractions(steps, warmup, fractions=(0.0, 0.1, 0.2, 0.5, 1.0), w=None):
    """The controlled experiment of the paper's performance section: the partition is
    forced (no indicator, no rollback) with the elements of lowest y on FD, a fraction
    x of them, and the step's wall-clock time is compared with the all-FD run; the ideal
    speedup 1 / (x + (1 - x)/f) uses the measured all-DG / all-FD ratio f.  Workload w
    (default: the benchmark sheet, 8^3 P5 elements)."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    w = w or I.workload("sheet")
    N = w["degree"]
    E = int(np.prod(w["n_elem"]))
    n3, m3 = (N + 1) ** 3, (2 * N + 1) ** 3
    x, y, z = _dg_nodes(w)
    u_dg = torch.from_numpy(np.ascontiguousarray(I.initial_data(w, x, y, z).reshape(9, E, n3))).cuda()
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    u_fd = torch.from_numpy(np.ascontiguousarray(I.initial_data(w, xf, yf, zf).reshape(9, E, m3))).cuda()
    nx, ny, nz = w["n_elem"]
    iy = (np.arange(E) // nx) % ny
    order = np.lexsort((np.arange(E), iy))  # y-major: the lowest-y elements first
    p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], hybrid=grffe.HYBRID_FORCED)
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p)
    if I.BC_DIRICHLET in tuple(w["bc"]):
        dom.set_boundary_state(I.boundary_states(w))
    dt = dom.dt()
    rows = []
    for frac in fractions:
        rep = np.zeros(E, np.int32)
        rep[order[:int(round(frac * E))]] = 1
        dom.set_state(u_dg, u_fd, torch.from_numpy(rep).cuda())
        secs = _time_steps(lambda k: dom.step(k, dt), steps, warmup)
        n_fd = int(rep.sum())
        pts = (E - n_fd) * n3 + n_fd * m3
        rows.append({"fd_fraction": n_fd / E, "fd_elements": n_fd, "ms_per_step": secs * 1e3 / steps,
                     "G_updates_per_s": pts * 3 * steps / secs / 1e9})
    t_fd = rows[-1]["ms_per_step"]
    f = t_fd / rows[0]["ms_per_step"]
    for r in rows:
        r["speedup_vs_all_fd"] = t_fd / r["ms_per_step"]
        r["ideal_speedup"] = 1.0 / (r["fd_fraction"] + (1.0 - r["fd_fraction"]) / f)
    dom.close()
    return {"dg_over_fd_speedup_f": f, "rows": rows,
            "paper_context": "one CPU core: f = 9.6 (108K vs 69K zone-cycles/s per core), 3.3x (ideal 5.2x) at 10% "
                             "FD, 2.6x (ideal 3.5x) at 20% FD"}


def run_forced_fractions_sheet(steps, warmup):
    r = run_forced_fractions(steps, warmup)
    return {"workload": "current sheet 8^3 DG-P5 elements, partition forced with the lowest-y elements on FD "
                        "(the paper's controlled DG/FD experiment on the benchmark sheet, fp64)", **r}


def run_forced_fractions_alfven(steps, warmup):
    """The paper's own set-up of the controlled experiment: the stationary Alfven wave on
    (8, 32, 8) elements (cubic, h = 0.375: [-1.5, 1.5] x [-6, 6] x [-1.5, 1.5]; the paper
    gives the element counts, not the extents), Dirichlet faces at the ends of x."""
    from paper_2404_01531_amd import inputs as I
    w = I.workload("alfven_1d", n_elem=(8, 32, 8), lower=(-1.5, -6.0, -1.5), upper=(1.5, 6.0, 1.5))
    r = run_forced_fractions(steps, warmup, w=w)
    return {"workload": "stationary Alfven wave, (8, 32, 8) DG-P5 elements on [-1.5,1.5]x[-6,6]x[-1.5,1.5], "
                        "Dirichlet x faces, partition forced with the lowest-y elements on FD (fp64)", **r}


def run_accuracy_smooth_wave(crossings=20):
    """The paper's accuracy comparison of the DG and FD grids: the smooth fast wave
    (E_z = -B_y = sin(pi x), lambda = 2) on [0, 2]^3 with 4^3 P5 elements, periodic,
    evolved for `crossings` crossing times with every element on DG (filtered and
    unfiltered) or every element on FD (with and without the fourth-order
    corrector).  Reported: the RMS over the grid points of |B - B_exact| after each
    crossing, B_exact(x, t) = B(x - t, 0).  The time step is the CFL step rounded
    down to a whole number of steps per crossing."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    w = I.workload("smooth_fast_wave")
    N = w["degree"]
    E = int(np.prod(w["n_elem"]))
    n3, m3 = (N + 1) ** 3, (2 * N + 1) ** 3
    x, y, z = _dg_nodes(w)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    lam = w["wavelength"]
    variants = (("dg_filtered", dict(hybrid=grffe.HYBRID_DG_ONLY)),
                ("dg_unfiltered", dict(hybrid=grffe.HYBRID_DG_ONLY, filter_on=0)),
                ("fd4", dict(hybrid=grffe.HYBRID_FORCED, fd_order=4)),
                ("fd2", dict(hybrid=grffe.HYBRID_FORCED, fd_order=2)))
    out = {}
    for name, over in variants:
        p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], **over)
        dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p)
        on_fd = over["hybrid"] == grffe.HYBRID_FORCED
        u_dg = torch.from_numpy(np.ascontiguousarray(I.initial_data(w, x, y, z).reshape(9, E, n3))).cuda()
        u_fd = torch.from_numpy(np.ascontiguousarray(I.initial_data(w, xf, yf, zf).reshape(9, E, m3))).cuda()
        dom.set_state(u_dg, u_fd, torch.full((E,), 1 if on_fd else 0, dtype=torch.int32, device="cuda"))
        per = int(np.ceil(lam / dom.dt()))
        dt = lam / per
        xs = (xf if on_fd else x).reshape(E, -1)
        errs = []
        t0 = time.perf_counter()
        for k in range(1, crossings + 1):
            dom.step(per, dt)
            g, f, _ = dom.get_state()
            u = (f if on_fd else g).cpu().numpy().reshape(9, E, -1)
            ex = I.smooth_fast_wave(xs - k * lam, lam)  # periodic: x - k lambda is x
            errs.append(float(np.sqrt(np.mean((u[3:6] - ex[3:6]) ** 2))))
        torch.cuda.synchronize()
        out[name] = {"rms_B_error_per_crossing": errs, "steps_per_crossing": per, "dt": dt,
                     "secs": time.perf_counter() - t0}
        dom.close()
    return {"workload": "smooth fast wave E_z = -B_y = sin(pi x) on [0,2]^3 periodic, 4^3 DG-P5 / FD 11^3 elements, "
                        "eta 1e6, CFL 0.3 (the paper's accuracy comparison of the DG and FD grids)", **out}


def run_exact_wald(levels=(2, 4, 8, 16), degrees=(5, 7, 9), t_end=5.0):
    """Convergence on the exact a = 0 Wald field (Sec. IV B, the paper's exact-Wald
    table, here on a Cartesian box): Kerr-Schild background, M = 1, the box
    [4, 28] x [-12, 12]^2 beside the hole with n^3 elements, every face a Dirichlet
    face holding the exact field point by point, all elements on DG, evolved to
    t = 5M; the RMS over the nodes of |B~ - B~_exact| and the measured order."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    lo, hi = (4.0, -12.0, -12.0), (28.0, 12.0, 12.0)
    rows = []
    for N in degrees:
        prev = None
        for n in levels:
            w = dict(n_elem=(n, n, n), lower=lo, upper=hi, degree=N)
            ref = grffe.operator(N, 0)
            x, y, z = I.points(w["n_elem"], lo, hi, ref)
            E, n3, m3 = n ** 3, (N + 1) ** 3, (2 * N + 1) ** 3
            bg = I.kerr_schild_background(x, y, z, 1.0, 0.0).reshape(26, E, n3)
            u = I.wald_a0(x, y, z).reshape(9, E, n3)
            p = grffe.default_params(eta=1e6, cfl=0.25, hybrid=grffe.HYBRID_DG_ONLY)
            dom = grffe.Domain(w["n_elem"], lo, hi, N, (I.BC_DIRICHLET,) * 6, params=p,
                               bg=torch.from_numpy(np.ascontiguousarray(bg)).cuda())
            fdg, ffd = I.boundary_field(w, I.wald_a0, ref)
            dom.set_boundary_field(torch.from_numpy(fdg).cuda(), torch.from_numpy(ffd).cuda())
            dom.set_state(torch.from_numpy(np.ascontiguousarray(u)).cuda(),
                          torch.zeros((9, E, m3), dtype=torch.float64, device="cuda"),
                          torch.zeros(E, dtype=torch.int32, device="cuda"))
            steps = int(np.ceil(t_end / dom.dt()))
            dt = t_end / steps
            dom.step(steps, dt)
            g = dom.get_state()[0].cpu().numpy().reshape(9, E, n3)
            dom.close()
            err = float(np.sqrt(np.mean((g[3:6] - u[3:6]) ** 2)))
            rows.append({"degree": N, "n_elem": n, "dt": dt, "rms_B_error": err,
                         "order": None if prev is None else float(np.log2(prev / err))})
            prev = err
    return {"workload": "exact a=0 Wald field, Kerr-Schild M=1, box [4,28]x[-12,12]^2 beside the hole, n^3 elements, "
                        "per-point Dirichlet faces, all DG, t = 5M (the paper's exact-Wald convergence test on a "
                        "Cartesian box)", "rows": rows}


# The exact-Wald table of Sec. IV B 1 as printed: (degree, n_radial, n_angular) ->
# (dt/M, L2 error of B~ at t = 5M, order).  The P5 high-resolution error is at odds
# with its own order (4.72 implies 1.04e-6 from the row above).
EXACT_WALD_TABLE = {(5, 1, 1): (2.90e-2, 8.71e-4, None), (5, 2, 2): (1.15e-2, 2.74e-5, 4.99),
                    (5, 4, 4): (5.76e-3, 4.11e-8, 4.72), (7, 1, 1): (1.62e-2, 1.23e-5, None),
                    (7, 2, 2): (6.29e-3, 1.51e-7, 6.35), (7, 4, 4): (3.14e-3, 1.29e-9, 6.87),
                    (9, 1, 1): (1.03e-2, 2.75e-7, None), (9, 2, 2): (3.95e-3, 2.03e-9, 7.08),
                    (9, 4, 4): (1.97e-3, 8.04e-12, 7.98)}


def _shell_faces(u, n):
    """(9, E, n^3) -> (9, E, 6, n^2): the values at the nodes of each element face,
    node t1 + n t2 along the face's two tangential axes in increasing order."""
    import numpy as np
    v = u.reshape(u.shape[0], u.shape[1], n, n, n)  # axes (k, j, i)
    faces = [v[..., 0], v[..., -1], v[..., 0, :], v[..., -1, :], v[:, :, 0], v[:, :, -1]]
    return np.stack([f.reshape(u.shape[0], u.shape[1], n * n) for f in faces], axis=2)


def run_shell_wald(cases=tuple(EXACT_WALD_TABLE), t_end=5.0):
    """The exact-Wald convergence test on the paper's grid (Sec. IV B 1): the shell
    1.99M..20M of six cubed-sphere wedges (equiangular and logarithmic maps),
    Kerr-Schild a = 0, eta = 0, CFL 0.3, outflow inner sphere, the exact solution as
    the outer Dirichlet state, data evaluated on the FD grid and reconstructed to DG,
    t = 5M (the last step shortened to land on it).  Per row: time step, error of B~,
    order, the printed values, and the time per step of the curved-element DG step."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    rows, prev = [], {}
    for N, nr, na in cases:
        n = N + 1
        x = grffe.shell_points(N, nr, na, 1.99, 20.0)
        xf = grffe.shell_points(N, nr, na, 1.99, 20.0, fd=True)
        E = x.shape[1]
        bg = I.kerr_schild_background(x[0], x[1], x[2], 1.0, 0.0)
        uex = I.wald_a0(x[0], x[1], x[2], 1.0, 1.0)
        p = grffe.default_params(eta=0.0, cfl=0.3, hybrid=grffe.HYBRID_DG_ONLY)
        dom = grffe.Domain.shell(N, nr, na, 1.99, 20.0, grffe.BC_OUTFLOW, grffe.BC_DIRICHLET, params=p,
                                 bg=torch.from_numpy(np.ascontiguousarray(bg)).cuda())
        dom.set_boundary_field(torch.from_numpy(np.ascontiguousarray(_shell_faces(uex, n))).cuda(), None)
        dom.init_from_fd(torch.from_numpy(np.ascontiguousarray(I.wald_a0(xf[0], xf[1], xf[2], 1.0, 1.0))).cuda())
        dt = dom.dt()
        n_full = int(np.floor(t_end / dt + 1e-9))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dom.step(n_full)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(n_full, 1)
        rest = t_end - n_full * dt
        if rest > 1e-12:
            dom.step(1, rest)
        u = dom.get_dg().cpu().numpy()
        dom.close()
        err = float(np.sqrt(((u[3:6] - uex[3:6]) ** 2).sum(axis=0).mean()))
        dt_p, err_p, order_p = EXACT_WALD_TABLE[(N, nr, na)]
        order = float(np.log2(prev[N] / err)) if N in prev else None
        prev[N] = err
        rows.append({"degree": N, "elements": f"{nr}x{6 * na * na}", "dt": dt, "dt_paper": dt_p,
                     "B_error": err, "B_error_paper": err_p, "order": order, "order_paper": order_p,
                     "steps": n_full + (1 if rest > 1e-12 else 0), "ms_per_step": ms,
                     "node_updates_per_s": E * n ** 3 / (ms * 1e-3)})
    return {"workload": "exact a=0 Wald field on the spherical shell 1.99M..20M of six cubed-sphere wedges, "
                        "Kerr-Schild M=1, eta=0, CFL 0.3, outflow inner / Dirichlet outer sphere, all DG, t = 5M",
            "rows": rows}


def _shell_sample(u, pts, N, nr, na, r_in, r_out, nodes):
    """Values (C, P) of the nodal DG data u (C, E, n^3) of a shell at the points pts
    (3, P): the wedge and element from the inverse map, then the element's Lagrange
    interpolant at the reference coordinates."""
    import numpy as np
    n = N + 1
    x = np.asarray(pts, np.float64)
    k = np.argmax(np.abs(x), axis=0)
    P = x.shape[1]
    idx = np.arange(P)
    xk = x[k, idx]
    s = np.sign(xk)
    X = x[(k + 1) % 3, idx] / xk
    Y = s * x[(k + 2) % 3, idx] / xk
    r = np.sqrt((x * x).sum(axis=0))
    ref = [4.0 / np.pi * np.arctan(X), 4.0 / np.pi * np.arctan(Y),
           2.0 * np.log(r / r_in) / np.log(r_out / r_in) - 1.0]
    cnt = (na, na, nr)
    cell, xi = [], []
    for d in range(3):
        t = 0.5 * (ref[d] + 1.0) * cnt[d]
        c = np.clip(np.floor(t), 0, cnt[d] - 1).astype(np.int64)
        cell.append(c)
        xi.append(2.0 * (t - c) - 1.0)
    w = 2 * k + (s < 0)
    e = ((w * nr + cell[2]) * na + cell[1]) * na + cell[0]
    L = []
    for d in range(3):
        l = np.ones((n, P))
        for j in range(n):
            for m in range(n):
                if m != j:
                    l[j] *= (xi[d] - nodes[m]) / (nodes[j] - nodes[m])
        L.append(l)
    basis = np.einsum("kp,jp,ip->pkji", L[2], L[1], L[0]).reshape(P, n ** 3)  # node i + n (j + n k)
    return np.stack([(u[c][e] * basis).sum(axis=1) for c in range(u.shape[0])])


def hemisphere_flux(u, N, nr, na, r_in, r_out, nodes, R, n_mu=48, n_phi=96):
    """Flux of B~ through the upper hemisphere of the coordinate sphere of radius R:
    Gauss-Legendre in cos(theta) on [0, 1], uniform in phi."""
    import numpy as np
    g, gw = np.polynomial.legendre.leggauss(n_mu)
    mu, wmu = 0.5 * (g + 1.0), 0.5 * gw
    ph = 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    st = np.sqrt(1.0 - MU ** 2)
    nrm = np.stack([st * np.cos(PH), st * np.sin(PH), MU]).reshape(3, -1)
    B = _shell_sample(u[3:6], R * nrm, N, nr, na, r_in, r_out, nodes)
    Bn = (B * nrm).sum(axis=0).reshape(n_mu, n_phi)
    return float((wmu[:, None] * Bn).sum() * (2.0 * np.pi / n_phi) * R * R)


def run_vacuum_wald(spins=(0.0, 0.5, 0.7, 0.8), degree=5, n_radial=16, n_angular=4, r_in=None, r_out=125.0,
                    t_end=125.0, cfl=0.25, checks=(80.0, 100.0, 125.0), coords="cartesian"):
    """The vacuum Wald problem (Sec. IV B 2) on the shell: Kerr background of spin a
    (M = 1), Wald's magnetic field with E = 0 at t = 0, eta = 0, outflow inner sphere
    inside the horizon, no-incoming-Poynting outer sphere, all DG.  coords
    "spherical": the Cartesian projection of spherical Kerr-Schild coordinates
    (Appendix B), inner sphere at M as in the paper, the horizon the sphere r_+;
    "cartesian": Kerr-Schild Cartesian coordinates, inner sphere at 1.2M (inside the
    horizon, outside the ring singularity for a <= 0.9), the horizon the ellipsoid
    sharing its equator with the sphere of radius sqrt(r_+^2 + a^2), through whose
    upper hemisphere the flux is measured (B~ is divergence-free between the two).
    The flux of B~ through the upper half of the horizon is compared with King's
    closed form (Eq. vacuum wald magnetic flux) at the check times."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    N = degree
    sph = coords == "spherical"
    if r_in is None:
        r_in = 1.0 if sph else 1.2
    bgf = I.spherical_kerr_schild_background if sph else I.kerr_schild_background
    datf = I.wald_vacuum_spherical if sph else I.wald_vacuum
    nodes = np.asarray(grffe.operator(N, 0))
    rows = []
    for a in spins:
        x = grffe.shell_points(N, n_radial, n_angular, r_in, r_out)
        xf = grffe.shell_points(N, n_radial, n_angular, r_in, r_out, fd=True)
        bg = bgf(x[0], x[1], x[2], 1.0, a)
        p = grffe.default_params(eta=0.0, cfl=cfl, hybrid=grffe.HYBRID_DG_ONLY)
        dom = grffe.Domain.shell(N, n_radial, n_angular, r_in, r_out, grffe.BC_OUTFLOW,
                                 grffe.BC_NO_INCOMING_POYNTING, params=p,
                                 bg=torch.from_numpy(np.ascontiguousarray(bg)).cuda())
        dom.init_from_fd(torch.from_numpy(np.ascontiguousarray(datf(xf[0], xf[1], xf[2], 1.0, a))).cuda())
        dt = dom.dt()
        rp = 1.0 + np.sqrt(1.0 - a * a)
        R = rp if sph else np.sqrt(rp * rp + a * a)
        king = I.king_flux(a)
        t, flux, t0 = 0.0, {}, time.perf_counter()
        steps = 0
        for tc in checks:
            n = int(round((tc - t) / dt))
            chunk = 2000
            while n > 0:
                k = min(chunk, n)
                dom.step(k)
                n -= k
                steps += k
                t += k * dt
                torch.cuda.synchronize()
                print(f"#   vacuum Wald a = {a}: t = {t:.1f}M", file=sys.stderr, flush=True)
            u = dom.get_dg().cpu().numpy()
            if not np.all(np.isfinite(u)):
                flux[tc] = None
                break
            flux[tc] = hemisphere_flux(u, N, n_radial, n_angular, r_in, r_out, nodes, R)
        wall = time.perf_counter() - t0
        dom.close()
        rows.append({"spin": a, "dt": dt, "steps": steps, "wall_s": wall, "r_plus": rp,
                     "flux": {str(k): v for k, v in flux.items()}, "king": king,
                     "rel_error_last": None if flux.get(checks[-1]) is None else flux[checks[-1]] / king - 1.0})
    return {"workload": f"vacuum Wald problem on the shell r = {r_in}M..{r_out}M, {n_radial}x{6 * n_angular ** 2} "
                        f"P{degree} elements, Kerr M=1 ({coords} Kerr-Schild coordinates), eta=0, CFL {cfl}, "
                        "outflow inner / no-incoming-Poynting outer sphere, all DG", "rows": rows}


def run_shell_scale(steps=20, warmup=5, degree=5, n_radial=32, n_angular=8, spin=0.7):
    """The curved-element DG step at a full-chip size: the magnetospheric-Wald grid of
    Sec. IV B 3 (32 x 384 elements; here P5 from 1.2M to 125M in Cartesian
    Kerr-Schild coordinates, a = 0.7, the vacuum Wald data, eta = 1e5, all DG), timed
    over `steps` steps; the DG substep's mean launch from HIP events and its
    algorithmic HBM fraction (the box kernel's bytes per node plus 72 B of inverse
    Jacobian)."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    N, n = degree, degree + 1
    r_in, r_out = 1.2, 125.0
    x = grffe.shell_points(N, n_radial, n_angular, r_in, r_out)
    E = x.shape[1]
    bg = I.kerr_schild_background(x[0], x[1], x[2], 1.0, spin)
    p = grffe.default_params(eta=1e5, cfl=0.25, hybrid=grffe.HYBRID_DG_ONLY)
    dom = grffe.Domain.shell(N, n_radial, n_angular, r_in, r_out, grffe.BC_OUTFLOW, grffe.BC_NO_INCOMING_POYNTING,
                             params=p, bg=torch.from_numpy(np.ascontiguousarray(bg)).cuda())
    del bg
    # the data set at the nodes (the FD start-up grid of 16 M cells is not needed for timing)
    dom.set_state(torch.from_numpy(np.ascontiguousarray(I.wald_vacuum(x[0], x[1], x[2], 1.0, spin))).cuda(),
                  torch.zeros((9, E, (2 * N + 1) ** 3), dtype=torch.float64, device="cuda"),
                  torch.zeros(E, dtype=torch.int32, device="cuda"))
    dom.step(warmup)
    fam = grffe.KERNEL_FAMILIES["dg_substep"]
    dom.timing_enable(fam, period=TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tot, launches = dom.timing_read(fam)
    dom.timing_enable()
    ok = bool(torch.isfinite(dom.get_dg()).all().item())
    dom.close()
    nodes = E * n ** 3
    mean_us = tot * 1e3 / max(launches, 1)
    per_node = sum(DG_BYTES_PER_NODE.values()) / 3.0 + DG_BG_BYTES_PER_NODE + 72.0
    achieved = nodes * per_node / (mean_us * 1e-6) / 1e9
    return {"workload": f"shell {r_in}M..{r_out}M, {n_radial}x{6 * n_angular ** 2} P{N} elements, Kerr-Schild a={spin} "
                        "(Cartesian KS), vacuum Wald data, eta 1e5, all DG", "elements": E, "dg_nodes": nodes,
            "ms_per_step": ms, "node_updates_per_s": 3 * nodes / (ms * 1e-3), "finite": ok,
            "dg_mapped_mean_us": mean_us, "launches": launches, "algorithmic_bytes_per_node": per_node,
            "achieved_GBps": achieved, "frac_hbm": achieved / 8000.0}


def run_shell_hybrid_scale(steps=20, warmup=3, degree=5, n_radial=32, n_angular=8, spin=0.7):
    """The hybrid step on curved elements at the same full-chip size: the grid of
    run_shell_scale with FD subcells (second order) on a band of elements about the
    equator near the hole -- where the magnetospheric-Wald run of Sec. IV B 3 keeps
    its troubled elements, the equatorial current sheet -- held there (forced
    partition).  Timed over `steps` steps; the curved FD flux kernel's mean launch and
    its FP64 rate (WENO5-Z of twelve components at 78 flop each side of every face,
    1872 flop per face: a lower bound of its arithmetic) against the vector peak."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    N, n, m = degree, degree + 1, 2 * degree + 1
    r_in, r_out = 1.2, 125.0
    x = grffe.shell_points(N, n_radial, n_angular, r_in, r_out)
    E = x.shape[1]
    bg = I.kerr_schild_background(x[0], x[1], x[2], 1.0, spin)
    p = grffe.default_params(eta=1e5, cfl=0.25, hybrid=grffe.HYBRID_FORCED, fd_order=2)
    dom = grffe.Domain.shell(N, n_radial, n_angular, r_in, r_out, grffe.BC_OUTFLOW, grffe.BC_NO_INCOMING_POYNTING,
                             params=p, bg=torch.from_numpy(np.ascontiguousarray(bg)).cuda())
    del bg
    c = x.mean(axis=2)
    rc = np.sqrt((c * c).sum(axis=0))
    band = (rc < 4.0) & (np.abs(c[2]) < 0.2 * rc)
    fd_e = np.nonzero(band)[0]
    u = torch.from_numpy(np.ascontiguousarray(I.wald_vacuum(x[0], x[1], x[2], 1.0, spin))).cuda()
    el = torch.from_numpy(fd_e.astype(np.int32)).cuda()
    fd = torch.zeros((9, E, m ** 3), dtype=torch.float64, device="cuda")
    fd[:, el.long()] = dom.project_dg_to_fd(u, el)
    rep = torch.zeros(E, dtype=torch.int32, device="cuda")
    rep[el.long()] = 1
    u[:, el.long()] = 0.0
    dom.set_state(u, fd, rep)
    del u, fd
    dom.step(warmup)
    fams = {k: grffe.KERNEL_FAMILIES[k] for k in ("dg_substep", "fd_flux", "fd_update", "fd_stage", "fd_trace",
                                                   "dg_slab")}
    dom.timing_enable(*fams.values(), period=TIMING_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    times = {}
    for k, f in fams.items():
        tot, launches = dom.timing_read(f)
        times[k] = {"mean_us": tot * 1e3 / max(launches, 1), "launches": launches}
    dom.timing_enable()
    dg, fdd, r = dom.get_state()
    ok = bool(torch.isfinite(dg).all().item() and torch.isfinite(fdd).all().item())
    n_fd = int(r.sum().item())
    dom.close()
    faces = n_fd * 3 * (m + 1) * m * m
    flux_us = times["fd_flux"]["mean_us"]
    tflops = faces * 1872.0 / (flux_us * 1e-6) / 1e12
    updates = 3 * ((E - n_fd) * n ** 3 + n_fd * m ** 3)
    return {"workload": f"shell {r_in}M..{r_out}M, {n_radial}x{6 * n_angular ** 2} P{N} elements, Kerr-Schild "
                        f"a={spin} (Cartesian KS), vacuum Wald data, eta 1e5, {n_fd} elements on FD (second "
                        "order) in an equatorial band r < 4M, forced partition", "elements": E, "fd_elements": n_fd,
            "ms_per_step": ms, "point_updates_per_s": updates / (ms * 1e-3), "finite": ok, "kernels": times,
            "fd_flux_weno_tflops": tflops, "fd_flux_frac_fp64_valu_weno_only": tflops / 78.6}


def run_adjoint_frozen(steps=40, every=20):
    """The benchmark's current sheet, 8^3 P5 elements, with the start-up DG/FD
    partition held fixed (forced mode): forward steps, one-step adjoints through DG
    and FD elements and their coupling, and the checkpointed gradient of a linear
    functional of the end state, timed against the forward run."""
    import numpy as np
    import torch

    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    from paper_2404_01531_amd.autograd import GRFFEStepFrozen
    w = I.workload("sheet")
    N = w["degree"]
    p0 = grffe.default_params(eta=w["eta"], cfl=w["cfl"])
    d0 = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p0)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    d0.init_from_fd(torch.from_numpy(I.initial_data(w, xf, yf, zf).reshape(9, d0.E, -1)).cuda())
    dg, fd, rep = d0.get_state()
    dg, fd, rep = dg.clone(), fd.clone(), rep.clone()
    d0.close()
    p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], hybrid=grffe.HYBRID_FORCED)
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p)
    dt = dom.dt()
    gen = np.random.default_rng(1006)
    wd = torch.from_numpy(gen.standard_normal(tuple(dg.shape))).cuda()
    wf = torch.from_numpy(gen.standard_normal(tuple(fd.shape))).cuda()
    GRFFEStepFrozen.apply(dg, fd, rep, dom, 2, dt, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        GRFFEStepFrozen.apply(dg, fd, rep, dom, steps, dt, every)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    ld, lf = dom.step_adjoint_frozen(dg, fd, rep, wd, wf, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        ld, lf = dom.step_adjoint_frozen(dg, fd, rep, ld, lf, dt)
    torch.cuda.synchronize()
    t_adj1 = (time.perf_counter() - t0) / 10
    a = dg.clone().requires_grad_(True)
    b = fd.clone().requires_grad_(True)
    t0 = time.perf_counter()
    gN, fN, _ = GRFFEStepFrozen.apply(a, b, rep, dom, steps, dt, every)
    ((wd * gN).sum() + (wf * fN).sum()).backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    n_fd = int((rep == 1).sum())
    out = {"workload": f"current sheet, 8^3 elements DG-P5, start-up partition frozen ({n_fd} FD elements), "
                       f"J = <w, U_N> after {steps} steps, checkpoints every {every}",
           "dtype": "f64", "forward_ms_per_step": t_fwd * 1e3 / steps,
           "step_adjoint_ms": t_adj1 * 1e3,
           "step_adjoint_over_forward": t_adj1 / (t_fwd / steps),
           "gradient_ms_total": t_grad * 1e3,
           "gradient_over_forward": t_grad / t_fwd,
           "grad_norm": float(torch.sqrt((a.grad ** 2).sum() + (b.grad ** 2).sum()))}
    dom.close()
    return out


def sheet_line(steps, warmup):
    """The flat current sheet (8^3 DG-P5 elements, about a quarter on FD): FP64 and mixed
    rates with the FD face-flux kernel's FP64-ALU roofline and the flat DG substep's
    HBM roofline."""
    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd import inputs as I
    w = I.workload("sheet")
    N = w["degree"]
    fam_fd, fam_dg = grffe.KERNEL_FAMILIES["fd_flux"], grffe.KERNEL_FAMILIES["dg_substep"]
    out, states = {}, {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        rec, st = run_workload(w, prec, steps, warmup, (fam_fd, fam_dg))
        states[name] = st
        out[name] = {"value": rec["value"], "ms_per_step": rec["secs"] * 1e3 / steps,
                     "fd_elements": [int(x) for x in rec["n_fd"]], "points_per_substep": rec["pts"],
                     "roofline_fd_flux": roofline_fd(rec, N, counted=prec == 0), "roofline_dg": roofline_dg(rec, N)}
    out["mixed"]["error_vs_fp64_run"] = state_diff(states["mixed"], states["fp64"])
    out["workload"] = ("flat current sheet, periodic [-1,1]^3, 8^3 elements DG-P5 / FD 11^3, eta 1e6, CFL 0.25, "
                       "adaptive DG-FD, seed 1002")
    out["steps"] = steps
    return out


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.rotator:
        rotator_sweep(args.rotator_frame, tuple(float(a) for a in args.rotator_angles.split(",")),
                      args.rotator_periods)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design note, "
                                   "rerun with --gpus 1"}))
        sys.exit(2)
    import torch

    from paper_2404_01531_amd import grffe

    torch.cuda.set_device(0)
    global CONTRACTION
    CONTRACTION = grffe.CONTRACTION_MFMA if args.contraction == "mfma" else grffe.CONTRACTION_VALU
    if args.only == "sheet":
        print(json.dumps(sheet_line(args.steps, args.warmup)))
        return
    if args.only == "batch":
        print(json.dumps(run_batch(args.steps, args.warmup, 0)))
        return
    if args.only == "adjoint_adaptive":
        print(json.dumps(run_adjoint_adaptive()))
        return
    if args.only == "shell_scale":
        print(json.dumps(run_shell_scale(args.steps, args.warmup)))
        return
    if args.only == "shell_hybrid":
        print(json.dumps(run_shell_hybrid_scale(args.steps, args.warmup)))
        return
    if args.only == "vacuum_wald":
        print(json.dumps(run_vacuum_wald(tuple(float(v) for v in args.spins.split(",")), coords=args.coords)))
        return
    if args.only == "shell_wald":
        degs = {int(v) for v in args.shell_degrees.split(",")}
        print(json.dumps(run_shell_wald(tuple(c for c in EXACT_WALD_TABLE if c[0] in degs))))
        return
    fams = tuple(sorted(grffe.KERNEL_FAMILIES.values()))
    res, states = {}, {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        rec, st = run_kerr_schild(args.steps, args.warmup, prec, families=fams)
        res[name], states[name] = rec, st
        print(f"# kerr-schild 16^3 {name}: {args.steps} steps, {rec['ms_per_step']:.4f} ms/step, "
              f"{rec['elements_dg_fd']} DG/FD elements; dg_substep mean {rec['roofline']['mean_launch_us']:.1f} us "
              f"over {rec['roofline']['launches']} launches", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    f64, mix = res["fp64"], res["mixed"]
    f64["roofline"]["traffic"] = dg_substep_traffic(f64)
    err64 = kerr_schild_parity(0, 1.0)
    errmx = kerr_schild_parity(1, 1e-3)
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_sample_steps)
    out = {
        "metric": "grid-point updates/s per RK substep, FP64 vs mixed, at stated L2 error",
        "value": f64["value"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f64["workload"], "elements": f64["elements"], "live_elements": f64["live_elements"],
                   "elements_dg_fd": f64["elements_dg_fd"], "points_per_substep": f64["points_per_substep"],
                   "dt": f64["dt"]},
        "roofline": f64["roofline"],
        "step_hbm": f64["step_hbm"],
        "kernels_mean_us": f64["kernels_mean_us"],
        "error_vs_oracle": err64,
        "mixed": {"value": mix["value"], "ms_per_step": mix["ms_per_step"],
                  "dtype": "f64 state, f32 fluxes and DG contractions", "elements_dg_fd": mix["elements_dg_fd"],
                  "roofline": mix["roofline"], "step_hbm": mix["step_hbm"], "error_vs_oracle": errmx,
                  "error_vs_fp64_run": state_diff(states["mixed"], states["fp64"])},
        "cpu_baseline": cpu,
    }
    del states
    torch.cuda.empty_cache()
    if args.extras != "none":
        ex = {}
        jobs = [("batch_64_fp64", lambda: run_batch(max(args.extra_steps // 3, 3), 1, 0)),
                ("batch_64_mixed", lambda: run_batch(max(args.extra_steps // 3, 3), 1, 1)),
                ("sheet_8^3", lambda: sheet_line(args.extra_steps, 2)),
                ("kerr_schild_16^3_full_run", lambda: run_kerr_schild_full()),
                ("sheet_element_sweep_16^3_32^3", lambda: run_sheet_sweep(args.extra_steps, 2)),
                ("forced_fd_fraction_sheet_8^3", lambda: run_forced_fractions_sheet(args.extra_steps, 2)),
                ("adjoint_poynting_kerr_schild_8^3", lambda: run_adjoint()),
                ("adjoint_poynting_kerr_schild_8^3_adaptive", lambda: run_adjoint_adaptive()),
                ("adjoint_sheet_8^3_frozen_partition", lambda: run_adjoint_frozen()),
                ("exact_wald_shell_table", lambda: run_shell_wald()),
                ("shell_32x384_p5", lambda: run_shell_scale(args.extra_steps, 3)),
                ("shell_32x384_p5_hybrid", lambda: run_shell_hybrid_scale(args.extra_steps, 3))]
        if args.extras == "all":
            jobs += [("vacuum_wald_king_flux", lambda: run_vacuum_wald()),
                     ("accuracy_smooth_fast_wave_4^3", lambda: run_accuracy_smooth_wave(20)),
                     ("exact_wald_convergence", lambda: run_exact_wald()),
                     ("forced_fd_fraction_alfven_8x32x8", lambda: run_forced_fractions_alfven(args.extra_steps, 2))]
        for name, fn in jobs:
            print(f"# extra workload {name}", file=sys.stderr, flush=True)
            ex[name] = fn()
            print(f"#   {json.dumps(ex[name])[:300]}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        out["extras"] = ex
    print(json.dumps(out))


# HBM bytes per DG node per launch of the curved k_dg_substep (FP64) on the Kerr-Schild
# 16^3 workload: rocprofv3 FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch, 14
# dispatches per substep with 4064-4088 DG elements; fetch 166814 / 216046 / 215350,
# write 123750 / 123760 / 61891 for substeps 1 / 2 / 3), each scaled by what the same
# counter reads for a plain 512 MiB device copy (fetch x 2.0, write x 1.0), averaged
# over the substeps and divided by 4072 x 216 nodes: 584.4 B against the 496 B of
# algorithmic traffic.  Most of the excess (~88 B per node) is the neighbours' face
# states the surface term reads (6 x 36 x 9 FP64 values per element, 72 B per node),
# which the algorithmic figure leaves out.  Valid for the kernel source whose hash is
# DG_TRAFFIC_SRC; reported as null for any other source.
DG_TRAFFIC_PER_NODE = 584.4
DG_TRAFFIC_SRC = "b14332371343b5da"


def dg_substep_traffic(rec):
    """Counted HBM bytes per launch of the curved DG substep for this run's DG node
    count, or None when the counters were taken on other kernel sources."""
    if DG_TRAFFIC_PER_NODE is None or kernel_source_hash("kernels_dg.hip") != DG_TRAFFIC_SRC:
        return None
    n_dg = 0.5 * sum(x[0] for x in rec["elements_dg_fd"])
    return DG_TRAFFIC_PER_NODE * n_dg * 216


# The library headers each counted kernel source includes (directly or through
# another header).
KERNEL_HEADERS = {"kernels_dg.hip": ("common.h", "physics.h", "grffe_internal.h"),
                  "kernels_fd.hip": ("fd_common.h", "common.h", "physics.h", "grffe_internal.h")}


def kernel_source_hash(main="kernels_fd.hip"):
    """SHA-256 (first 16 hex digits) of a kernel source and the headers it includes."""
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(ROOT, "paper_2404_01531_amd", "csrc")
    for f in (main,) + KERNEL_HEADERS[main]:
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(steps):
    """The oracle (numpy FP64) on a bounded sample of the benchmark's Kerr-Schild
    workload: the octant [-40, 0]^3 of the same grid (8^3 of its 16^3 elements, h = 5,
    the same background, data and parameters; the element at the hole excised, the cut
    faces outer faces), `steps` steps from the initial data, on every host core the
    process may use (numpy's BLAS threads; the elementwise work is single-threaded)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import operators as ops
    from oracle import step as OS
    from oracle.domain import Domain as ODomain
    from paper_2404_01531_amd import inputs as I

    w = I.workload("kerr_schild", n_elem=(8, 8, 8), lower=(-40.0,) * 3, upper=(0.0,) * 3)
    N = w["degree"]
    x, y, z = I.points(w["n_elem"], w["lower"], w["upper"], ops.gll(N)[0])
    with np.errstate(all="ignore"):
        bg = I.background(w, x, y, z)
        u = I.initial_data(w, x, y, z)
    exc = I.excision_mask(w).astype(bool)
    bg[:, exc] = 0.0
    bg[0, exc] = 1.0
    bg[4, exc] = bg[7, exc] = bg[9, exc] = 1.0
    u[:, exc] = 0.0
    odom = ODomain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], excised=exc, bg=bg,
                   params=dict(eta=w["eta"], cfl=w["cfl"]))
    st = OS.State(u, np.zeros((9, odom.E, odom.m, odom.m, odom.m)), np.zeros(odom.E, np.int64))
    dt = odom.dt()
    t0 = time.perf_counter()
    pts = 0.0
    for _ in range(steps):
        nfd = int((st.rep[odom.active] == 1).sum())
        pts += 3 * ((int(odom.active.sum()) - nfd) * (N + 1) ** 3 + nfd * (2 * N + 1) ** 3)
        st = OS.step(odom, st, dt)
    secs = time.perf_counter() - t0
    threads = max([int(t.get("num_threads", 1)) for t in threadpool_info()] or [1])
    return {"value": pts / secs, "unit": "grid-point updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
            "sample": f"{steps} step(s) of the octant [-40,0]^3 of the Kerr-Schild 16^3 grid (8^3 of its elements, "
                      f"same element size, background, data and parameters) from the initial data, numpy FP64 with "
                      f"{threads} BLAS thread(s), {secs:.1f} s"}


if __name__ == "__main__":
    main()
