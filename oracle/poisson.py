"""CPU FP64 oracle of the electrostatic potential solve (Sec. 3.3, Eqs.
FD:PoissonDiscrete, Phi:correction, phi:BC:discrete and the discrete multipole
moments; CG with a block-Jacobi preconditioner and l_max = 6 from Sec. 4).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: the tests, the smoke
check and the CPU-baseline leg of the benchmark are its only callers.

Grid functions are flat arrays of n1*n2*n3 values, index k + n3*(j + n2*i);
node (i, j, k) (0-based) sits at ((i+1) h, (j+1) h, (k+1) h).  Positions in the
multipole expansion are measured from the centre of the domain,
((n_d + 1) h / 2 per axis): the paper does not name the expansion centre.

Functions and the passages they follow:

* ``real_harmonics``      orthonormal real spherical harmonics Y_lm, l <= l_max,
                          from SciPy's complex ones (a library routine).
* ``multipole_moments``   Q_lm = h^3 sum |x|^l Y_lm(x) f(x) (the moments that
                          follow Eq. phi:BC:discrete).
* ``boundary_potential``  Eq. phi:BC:discrete at given points.
* ``charge_correction``   Eq. Phi:correction, with the off-grid values from a
                          callable (the multipole expansion, or any function).
* ``poisson_apply``       -(1/4 pi) lap_h phi with zero Dirichlet padding, the
                          operator of Eq. FD:PoissonDiscrete.
* ``block_jacobi``        the block-Jacobi preconditioner on B^3 blocks of nodes.
* ``poisson_solve``       Eq. FD:PoissonDiscrete solved by preconditioned CG.
"""
from __future__ import annotations

import math
from typing import Callable, Sequence

import numpy as np

from . import fd_weights, laplacian

FOUR_PI = 4.0 * math.pi


def node_positions(n: Sequence[int], h: float):
    """Coordinates of the nodes along each axis, relative to the domain centre."""
    return [(np.arange(1, n[d] + 1) - 0.5 * (n[d] + 1)) * h for d in range(3)]


def real_harmonics(lmax: int, x, y, z) -> np.ndarray:
    """Y_lm(x/|x|) for l = 0..lmax, m = -l..l, stacked as index l*l + l + m:
    sqrt(2) (-1)^m Re Y_l^m for m > 0, sqrt(2) (-1)^m Im Y_l^|m| for m < 0,
    Y_l^0 for m = 0, from scipy.special.sph_harm_y (orthonormal on the sphere).
    At the origin the direction is taken as +z."""
    from scipy.special import sph_harm_y

    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    r = np.sqrt(x * x + y * y + z * z)
    polar = np.arccos(np.clip(np.where(r > 0, z / np.where(r > 0, r, 1.0), 1.0), -1.0, 1.0))
    azim = np.arctan2(y, x)
    out = np.empty(((lmax + 1) ** 2,) + r.shape)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), polar, azim)
            if m > 0:
                v = math.sqrt(2.0) * (-1) ** m * c.real
            elif m < 0:
                v = math.sqrt(2.0) * (-1) ** m * c.imag
            else:
                v = c.real
            out[l * l + l + m] = v
    return out


def _grid_xyz(n, h):
    xs = node_positions(n, h)
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


def multipole_moments(n: Sequence[int], h: float, f: np.ndarray, lmax: int) -> np.ndarray:
    """Q_lm = h^3 sum_x |x|^l Y_lm(x) f(x) over the grid."""
    X, Y, Z = _grid_xyz(n, h)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    Ylm = real_harmonics(lmax, X, Y, Z)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    Q = np.zeros((lmax + 1) ** 2)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            i = l * l + l + m
            Q[i] = h ** 3 * np.sum(r ** l * Ylm[i] * f)
    return Q


def boundary_potential(Q: np.ndarray, lmax: int, x, y, z) -> np.ndarray:
    """phi(x) = sum_lm 4 pi / ((2l+1) |x|^(l+1)) Y_lm(x) Q_lm (Eq.
    phi:BC:discrete), for points away from the origin."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    r = np.sqrt(x * x + y * y + z * z)
    Ylm = real_harmonics(lmax, x, y, z)
    phi = np.zeros(r.shape)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            i = l * l + l + m
            phi += FOUR_PI / ((2 * l + 1) * r ** (l + 1)) * Ylm[i] * Q[i]
    return phi


def charge_correction(n: Sequence[int], h: float, no: int, phi_off: Callable) -> np.ndarray:
    """d of Eq. Phi:correction on the grid: -(1/4 pi) sum_p w_p times the sum of
    phi over the six neighbours at distance p that lie off the grid (indicator
    1 there, 0 on the grid; the p = 0 term is the node itself, always on the
    grid).  phi_off(x, y, z) gives phi at off-grid positions (relative to the
    domain centre); only nodes one axis step off a face are ever needed."""
    w = fd_weights(no, h)
    xs = node_positions(n, h)
    d = np.zeros(tuple(n))
    for ax in range(3):
        for side in (-1, 1):
            for p in range(1, no + 1):
                # grid nodes whose neighbour at distance p along ax, on this side, is off the grid
                if side > 0:
                    idx = np.arange(max(0, n[ax] - p), n[ax])
                else:
                    idx = np.arange(0, min(p, n[ax]))
                if idx.size == 0:
                    continue
                off = (idx + side * p + 1 - 0.5 * (n[ax] + 1)) * h  # coordinate of the off-grid neighbour
                coords = list(xs)
                coords[ax] = off
                X, Y, Z = np.meshgrid(*coords, indexing="ij")
                sl = [slice(None)] * 3
                sl[ax] = idx
                d[tuple(sl)] += w[p] * phi_off(X, Y, Z)
    return (-d / FOUR_PI).reshape(-1)


def poisson_apply(n: Sequence[int], h: float, no: int, phi: np.ndarray) -> np.ndarray:
    """-(1/4 pi) lap_h phi with phi = 0 off the grid."""
    return -laplacian(n, h, no, phi) / FOUR_PI


def block_jacobi(n: Sequence[int], h: float, no: int, B=4) -> Callable:
    """The block-Jacobi preconditioner: the nodes are cut into blocks of
    B[0] x B[1] x B[2] nodes (B an int: a cube), ragged at the high end of
    each axis, and each block of the residual is multiplied by the inverse of
    the operator restricted to that block (a dense matrix, the same for every
    block of one shape)."""
    B = (B, B, B) if np.isscalar(B) else tuple(int(b) for b in B)
    w = fd_weights(no, h)
    inv = {}

    def block_matrix(shape):
        m = int(np.prod(shape))
        A = np.zeros((m, m))
        pts = [(a, b, c) for a in range(shape[0]) for b in range(shape[1]) for c in range(shape[2])]
        where = {p: t for t, p in enumerate(pts)}
        for t, p in enumerate(pts):
            A[t, t] += 6.0 * w[0]
            for ax in range(3):
                for q in range(1, no + 1):
                    for s in (-1, 1):
                        nb = list(p)
                        nb[ax] += s * q
                        u = where.get(tuple(nb))
                        if u is not None:
                            A[t, u] += w[q]
        return np.linalg.inv(-A / FOUR_PI)

    starts = [list(range(0, n[d], B[d])) for d in range(3)]

    def apply(r: np.ndarray) -> np.ndarray:
        R = np.asarray(r, dtype=np.float64).reshape(tuple(n))
        Z = np.zeros_like(R)
        for i0 in starts[0]:
            for j0 in starts[1]:
                for k0 in starts[2]:
                    sl = (slice(i0, min(i0 + B[0], n[0])), slice(j0, min(j0 + B[1], n[1])),
                          slice(k0, min(k0 + B[2], n[2])))
                    shape = tuple(s.stop - s.start for s in sl)
                    if shape not in inv:
                        inv[shape] = block_matrix(shape)
                    Z[sl] = (inv[shape] @ R[sl].reshape(-1)).reshape(shape)
        return Z.reshape(-1)

    return apply


def poisson_solve(n: Sequence[int], h: float, no: int, charge: np.ndarray, lmax: int = 6, tol: float = 1e-10,
                  maxit: int = 2000, block: int = 4, phi_off: Callable = None):
    """phi on the grid from -(1/4 pi) lap_h phi = charge - d (Eq.
    FD:PoissonDiscrete), zero Dirichlet, with d from the multipole expansion of
    the charge to l_max (or from phi_off when given), by CG with the
    block-Jacobi preconditioner, from phi = 0, until ||r||_2 <= tol ||rhs||_2.
    Returns (phi, iterations, final relative residual, rhs)."""
    charge = np.asarray(charge, dtype=np.float64).reshape(-1)
    if phi_off is None:
        Q = multipole_moments(n, h, charge, lmax)
        phi_off = lambda X, Y, Z: boundary_potential(Q, lmax, X, Y, Z)  # noqa: E731
    rhs = charge - charge_correction(n, h, no, phi_off)
    M = block_jacobi(n, h, no, block)
    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = M(r)
    p = z.copy()
    rz = float(np.dot(r, z))
    bnorm = float(np.linalg.norm(rhs))
    it = 0
    while np.linalg.norm(r) > tol * bnorm and it < maxit:
        q = poisson_apply(n, h, no, p)
        alpha = rz / float(np.dot(p, q))
        x += alpha * p
        r -= alpha * q
        z = M(r)
        rz_new = float(np.dot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, float(np.linalg.norm(r) / bnorm), rhs
