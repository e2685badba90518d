"""Writes kerr_schild_16_p5_10steps.npz: the oracle's run of the Kerr-Schild black-hole
configuration (16^3 DG-P5 elements on [-40, 40]^3, a = 0.9, B0 = 1, eta = 1e5,
CFL 0.25, the adaptive hybrid control, every element starting on DG) over 10 steps.

Stored: the time step, the representation after every step (10, E), the smallest
relative distance |ratio / threshold - 1| of any indicator ratio to its threshold
in each substep and end-of-step check (10, 4: how far every decision is from a
tie), and the final values of a fixed sample of elements (DG elements next to the hole, on the
outer faces and edges, random interior ones; FD elements as found).  Calls only the
oracle and the seeded inputs; about five minutes on one host core.

    python tests/golden/make_kerr_schild_16.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import step as OS  # noqa: E402
from oracle.domain import DG, FD, Domain  # noqa: E402

from helpers import kerr_schild_config  # noqa: E402

OUT = os.path.join(HERE, "kerr_schild_16_p5_10steps.npz")
STEPS = 10


def sample_dg(odom, exc, rng):
    """Element ids: every live element with an excised neighbour, the outer corners,
    some face and edge elements, and random interior ones (32 in all)."""
    E = odom.E
    nx, ny, nz = odom.n_elem
    hole = [e for e in range(E) if not exc[e] and any(exc[o] for o in _box_nbrs(odom, e))]
    corners = [odom.index(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)]
    faces = [odom.index(0, 7, 8), odom.index(15, 8, 7), odom.index(8, 0, 3), odom.index(3, 15, 12),
             odom.index(5, 9, 0), odom.index(11, 2, 15), odom.index(0, 0, 9), odom.index(15, 15, 4)]
    picked = list(dict.fromkeys(hole[::3] + corners + faces))
    rest = [e for e in range(E) if not exc[e] and e not in picked]
    picked += list(rng.choice(rest, 32 - len(picked), replace=False)) if len(picked) < 32 else []
    return np.array(sorted(picked[:32]), np.int64)


def _box_nbrs(odom, e):
    x, y, z = odom.coords(e)
    out = []
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        c = (x + dx, y + dy, z + dz)
        if all(0 <= c[i] < odom.n_elem[i] for i in range(3)):
            out.append(odom.index(*c))
    return out


def main():
    w, bg, u, exc = kerr_schild_config(16)
    odom = Domain(w["n_elem"], w["lower"], w["upper"], w["degree"], w["bc"], excised=exc, bg=bg,
                  params=dict(eta=w["eta"], cfl=w["cfl"]))
    st = OS.State(u, np.zeros((9, odom.E, odom.m, odom.m, odom.m)), np.zeros(odom.E, np.int64))
    dt = odom.dt()
    reps, ratios = [], []
    t0 = time.time()
    for k in range(STEPS):
        log = []
        st = OS.step(odom, st, dt, log=log)
        reps.append(st.rep.astype(np.int8))
        margin = np.full(4, np.inf)
        for entry in log:
            if entry[0] == "substep":
                _, kk, el, ratio, thr = entry
                slot = kk - 1
            else:
                _, el, ratio, thr = entry
                slot = 3
            if len(ratio):
                margin[slot] = np.abs(ratio / thr - 1.0).min()
        ratios.append(margin)
        print(f"step {k + 1}: {int((st.rep == FD).sum())} FD elements, {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(1003)
    dg_el = sample_dg(odom, exc, rng)
    dg_el = dg_el[st.rep[dg_el] == DG]
    fd_all = np.nonzero(st.rep == FD)[0]
    fd_el = fd_all[np.linspace(0, fd_all.size - 1, min(6, fd_all.size)).astype(np.int64)] if fd_all.size else fd_all
    np.savez_compressed(OUT, dt=dt, steps=STEPS, rep=np.array(reps), margins=np.array(ratios), dg_elements=dg_el,
                        dg_values=st.dg[:, dg_el], fd_elements=fd_el, fd_values=st.fd[:, fd_el])
    print(f"wrote {OUT}: {dg_el.size} DG and {fd_el.size} FD elements sampled")


if __name__ == "__main__":
    main()
