"""grffe_check_finite_noalloc (no device allocation: a fixed library array holds the
per-element flags and their count) against grffe_check_finite, through the C ABI,
on two calls in a row, the second on a smaller domain."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2404_01531_amd import inputs as I

from helpers import make_pair, to_dev

pytestmark = pytest.mark.gpu


def _count(fn, ldom, stream):
    n = ctypes.c_int32(-1)
    rc = fn(ldom._h, ctypes.byref(n), stream)
    return rc, n.value


def test_check_finite_noalloc_matches_allocating_entry_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_01531_amd import grffe
    L = grffe.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # first a 4x3x2 sheet with non-finite values planted in four elements (two of
    # them past the second domain's last element), then a 2x2x1 sheet with one
    for n_elem, plant in (((4, 3, 2), (1, 5, 17, 23)), ((2, 2, 1), (2,))):
        w = I.workload("sheet", n_elem=n_elem, degree=3)
        _, ldom, _ = make_pair(w, dict(eta=w["eta"], cfl=w["cfl"]))
        xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], w["degree"])
        ldom.init_from_fd(to_dev(I.initial_data(w, xf, yf, zf)))
        for label in ("healthy", "planted"):
            if label == "planted":
                dg, fd, rep = ldom.get_state()
                r = rep.cpu().numpy()
                for e in plant:
                    if r[e] == 0:
                        dg[4, e, 3] = float("nan")
                    else:
                        fd[1, e, 7] = float("inf")
                ldom.set_state(dg, fd, rep)
            print(f"check_finite_noalloc: sheet {n_elem} {label}", flush=True)
            sys.stdout.flush()
            rc_a, n_a = _count(L.grffe_check_finite, ldom, stream)
            rc_b, n_b = _count(L.grffe_check_finite_noalloc, ldom, stream)
            expect = 0 if label == "healthy" else len(plant)
            assert (rc_a, n_a) == (rc_b, n_b) == ((0, 0) if expect == 0 else (-4, expect)), \
                (n_elem, label, rc_a, n_a, rc_b, n_b)
            rc_c, n_c = _count(L.grffe_check_finite_noalloc, ldom, stream)
            assert (rc_c, n_c) == (rc_b, n_b)
