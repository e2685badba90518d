"""Troubled-cell indicator (Sec. III C 3, Eq. (persson tci)) and DG<->FD transfer.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py).

The indicator is applied to u = |B~| = sqrt(gamma_ij B~^i B~^j) at the DG
nodes.  u_hat is u with its lowest modes removed; an element is troubled
when sqrt(sum u_hat^2 / sum u^2) > (N + 1 - M)^(-alpha), sums over the nodes.

Two readings of removing the lowest M modes are provided:
* mode 2 (default): u_hat = u - (L (x) L (x) L) u with L = V diag(p < M) V^-1,
  i.e. every mode with at least one index >= M is kept;
* mode 1: u_hat = (H (x) H (x) H) u with H = V diag(p >= M) V^-1, i.e. only
  modes whose three indices are all >= M (the printed triple sum).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from . import physics as ph


def tci_ratio(U_dg, geo, N, M, mode=2):
    """Indicator ratio per element of U_dg (9, E, n, n, n) with geometry at the nodes."""
    Bt = U_dg[3:6]
    u = np.sqrt(ph.dot(Bt, Bt, geo))
    u = np.broadcast_to(u, U_dg.shape[1:])
    if mode == 2:
        uh = u - ops.apply_3d(ops.mode_mask_matrix(N, M, True), u)
    else:
        uh = ops.apply_3d(ops.mode_mask_matrix(N, M, False), u)
    num = (uh ** 2).sum(axis=(-1, -2, -3))
    den = (u ** 2).sum(axis=(-1, -2, -3))
    return np.where(den > 0.0, np.sqrt(num / np.where(den > 0.0, den, 1.0)), 0.0)


def tci_threshold(N, M, alpha):
    return float(N + 1 - M) ** (-alpha)


def troubled(U_dg, geo, N, M, alpha, mode=2):
    return tci_ratio(U_dg, geo, N, M, mode) > tci_threshold(N, M, alpha)


def project_dg_to_fd(U_dg, N):
    """Sec. III C 2: DG polynomial evaluated at the subcell centres, P (x) P (x) P."""
    return ops.apply_3d(ops.projection_matrix(N), U_dg)


def reconstruct_fd_to_dg(U_fd, N):
    """Sec. III C 1: reconstruction from subcell centres to GLL nodes, R (x) R (x) R."""
    return ops.apply_3d(ops.reconstruction_matrix(N), U_fd)
