"""One-dimensional operators of the DG and FD grids (FP64, plain formulas).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct CPU
reference the HIP path is checked against; it is imported only by the tests,
the smoke check and the benchmark's CPU-baseline leg, and shares no code with
the HIP library.

Everything here follows Sec. III A (nodal DG on Legendre-Gauss-Lobatto
points, modal Legendre representation, exponential filter) and Sec. III C
(2N+1 subcells, DG<->FD transfer).  All matrices act along one reference
axis; the 3D operators are tensor products.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre(p, x):
    """Legendre polynomial L_p(x) by Bonnet's three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    if p == 0:
        return np.ones_like(x)
    l0, l1 = np.ones_like(x), x.copy()
    for n in range(1, p):
        l0, l1 = l1, ((2 * n + 1) * x * l1 - n * l0) / (n + 1)
    return l1


@lru_cache(maxsize=None)
def gll(N):
    """Legendre-Gauss-Lobatto nodes and weights for degree N (Sec. III A).

    Nodes: -1, the N-1 roots of L_N', +1.  Weights: 2 / (N (N+1) L_N(x)^2).
    The interior roots come from numpy's Legendre root finder and are then
    polished with Newton steps on L_N'.
    """
    c = np.zeros(N + 1)
    c[N] = 1.0
    dc = npleg.legder(c)
    ddc = npleg.legder(dc)
    r = np.sort(np.real(npleg.legroots(dc))) if N > 1 else np.zeros(0)
    for _ in range(5):
        r = r - npleg.legval(r, dc) / npleg.legval(r, ddc)
    x = np.concatenate([[-1.0], r, [1.0]])
    # enforce the exact symmetry of the node set
    x = 0.5 * (x - x[::-1])
    w = 2.0 / (N * (N + 1) * legendre(N, x) ** 2)
    return x, w


def lagrange_matrix(nodes, points):
    """M[k, j] = l_j(points[k]) for the Lagrange basis of ``nodes`` (plain product formula)."""
    nodes = np.asarray(nodes, np.float64)
    points = np.asarray(points, np.float64)
    n = nodes.size
    M = np.ones((points.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                M[:, j] *= (points - nodes[m]) / (nodes[j] - nodes[m])
    return M


def lagrange_derivative_matrix(nodes):
    """D[i, j] = l_j'(x_i), from differentiating the Lagrange product term by term."""
    x = np.asarray(nodes, np.float64)
    n = x.size
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            s = 0.0
            for k in range(n):
                if k == j:
                    continue
                prod = 1.0 / (x[j] - x[k])
                for m in range(n):
                    if m != j and m != k:
                        prod *= (x[i] - x[m]) / (x[j] - x[m])
                s += prod
            D[i, j] = s
    return D


@lru_cache(maxsize=None)
def diff_matrix(N):
    return lagrange_derivative_matrix(gll(N)[0])


@lru_cache(maxsize=None)
def vandermonde(N):
    """V[n, p] = L_p(xi_n): nodal values of the modal basis of Eq. (modal expansion)."""
    x, _ = gll(N)
    return np.stack([legendre(p, x) for p in range(N + 1)], axis=1)


@lru_cache(maxsize=None)
def filter_matrix(N, a=36.0, b=50.0):
    """V diag(sigma) V^-1 with sigma_n = exp(-a (n/N)^(2b)) (Eq. exponential filter)."""
    V = vandermonde(N)
    n = np.arange(N + 1)
    sigma = np.exp(-a * (n / N) ** (2 * b))
    return V @ np.diag(sigma) @ np.linalg.inv(V)


@lru_cache(maxsize=None)
def mode_mask_matrix(N, M, keep_low):
    """V diag(1[p < M]) V^-1 (keep_low) or V diag(1[p >= M]) V^-1 (not keep_low)."""
    V = vandermonde(N)
    p = np.arange(N + 1)
    s = (p < M) if keep_low else (p >= M)
    return V @ np.diag(s.astype(np.float64)) @ np.linalg.inv(V)


def fd_centres(N):
    """Reference cell centres of the 2N+1 uniform subcells, spacing 2/(2N+1) (Sec. III C 1)."""
    m = 2 * N + 1
    return -1.0 + (2.0 * np.arange(m) + 1.0) / m


def fd_faces(N):
    """Reference positions of the 2N+2 subcell faces."""
    m = 2 * N + 1
    return -1.0 + 2.0 * np.arange(m + 1) / m


@lru_cache(maxsize=None)
def projection_matrix(N):
    """DG -> FD: P[k, j] = l_j(xhat_k), the DG polynomial evaluated at cell centres."""
    return lagrange_matrix(gll(N)[0], fd_centres(N))


@lru_cache(maxsize=None)
def face_eval_matrix(N):
    """DG polynomial evaluated at the 2N+2 subcell faces."""
    return lagrange_matrix(gll(N)[0], fd_faces(N))


@lru_cache(maxsize=None)
def reconstruction_matrix(N):
    """FD -> DG: R[j, k], the least-squares inverse of the projection (Sec. III C 1).

    The cell-centre values of one axis are fitted in the least-squares sense
    by a polynomial of degree N (the DG space), using all 2N+1 cells, and the
    fit is evaluated at the GLL nodes: R = V(nodes) pinv(V(centres)) with V
    the Legendre Vandermonde matrix of degree N, i.e. R = (P^T P)^-1 P^T.  R is
    exact on polynomials of degree <= N, so R P = I.  (The exact-Wald table's
    P7 and P9 errors come out only with the fit of degree N; a fit of degree 5
    leaves them 1.7 and 66 times larger.)
    """
    x, _ = gll(N)
    xc = fd_centres(N)
    Vc = np.stack([legendre(p, xc) for p in range(N + 1)], axis=1)
    Vn = np.stack([legendre(p, x) for p in range(N + 1)], axis=1)
    return Vn @ np.linalg.solve(Vc.T @ Vc, Vc.T)


def apply_1d(A, u, axis):
    """Apply the matrix A along ``axis`` of u (out[..., i, ...] = sum_j A[i, j] u[..., j, ...])."""
    u = np.moveaxis(u, axis, -1)
    out = u @ A.T
    return np.moveaxis(out, -1, axis)


def apply_3d(A, u):
    """Tensor-product operator A (x) A (x) A on the last three axes."""
    for ax in (-1, -2, -3):
        u = apply_1d(A, u, ax)
    return u


def tci_M(N):
    """Number of low modes removed by the indicator: M=3 for N>=5, else floor((N+1)/2) >= 2."""
    return max(2, min(3, (N + 1) // 2))


def ssp_rk3_c():
    """Time-stepper constant c of Eq. (spectre DG CFL condition) for SSP-RK3.

    Half the extent of the stability region of 1 + z + z^2/2 + z^3/6 on the
    negative real axis (the same convention gives 1.39 for classic RK4).
    """
    # root of R(x) = -1 on the negative axis: 1 + x + x^2/2 + x^3/6 + 1 = 0
    r = np.roots([1.0 / 6.0, 0.5, 1.0, 2.0])
    r = r[np.abs(np.imag(r)) < 1e-12].real
    return float(-r.min()) / 2.0
