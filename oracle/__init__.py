"""CPU FP64 oracle for the Chebyshev-filter hot path (arXiv:1603.04334).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  Nothing here is imported by, or
imports, the HIP library or its Python binding; the two sides share only the
seeded input generator.

Orbital blocks are NumPy arrays of shape (ns, nd): row c is orbital c, i.e. the
column-major N_d x N_s matrix of the paper (Sec. 3.1, last paragraph) with
leading dimension nd.

Functions and the passages they follow:

* ``fd_weights``        Sec. 3.1 Eq. weightsLap (C).
* ``laplacian``         Sec. 3.1 Eq. FD:Laplacian with zero Dirichlet padding (C).
* ``h_apply``           Sec. 2 Eq. EL operator, discretised per Sec. 3.1 incl.
                        Eq. non-localPS:FD (C).
* ``cheb_filter``       Sec. 3.4 Eq. ChebFilter / Alg. 2 (C), scaled form.
* ``lanczos``           Sec. 4 (extremal eigenvalues by a few Lanczos steps).
* ``select_bounds``     Alg. 2 inputs lambda_1, lambda_c, lambda_Nd from Ritz values.
* ``rayleigh_ritz``     Sec. 3.4 Eq. SubspaceGeneralizedEigenproblem and the
                        H_s, M_s definitions that follow it.
* ``rotate``            Sec. 3.4 Eq. OrbitalTransformation.
* ``fermi_level``       Sec. 3.4 Eq. FermiEnergyConstraintFormulation (the
                        occupation constraint 2 sum_n g_n = N_e) and the
                        occupations g_n; Sec. 4 (k_B T = 1e-3 Ha).
* ``density``           Sec. 3.4, the electron density rho = (2/h^3) sum_n g_n psi_n^2.
* ``chefsi_passes``     Sec. 3.4 last paragraph and Sec. 4: repeated CheFSI
                        passes (filter, Rayleigh-Ritz, Fermi level, rotation)
                        with the cutoff set to the previous Fermi level + 0.1 Ha.
* ``gradient_weights``  Sec. 3.1, the weights of Eq. gradient:approximate.
* ``gradient``          Sec. 3.1 Eq. gradient:approximate with zero Dirichlet padding.
* ``nonlocal_force``    Sec. 3.6 Eqs. NonlocForce:Discrete and NonLocForce:U:W
                        (Alg. 4): Y_Jnlm, W_Jnlm and the nonlocal atomic force.
* ``dense_hamiltonian`` brute-force N_d x N_d matrix for tiny grids.
* ``cheb_closed_form``  C_m(x) from its trigonometric/hyperbolic definition.

The electrostatic potential solve (Sec. 3.3) lives in ``oracle.poisson``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sparc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle (gcc, OpenMP) in place."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Atom(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int * 3), ("ext", ctypes.c_int * 3), ("nproj", ctypes.c_int),
                ("chi", ctypes.POINTER(ctypes.c_double)), ("gamma", ctypes.POINTER(ctypes.c_double))]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        lib.oracle_fd_weights.argtypes = [ci, ctypes.c_double, dp]
        lib.oracle_laplacian.argtypes = [ci, ci, ci, ctypes.c_double, ci, ci, dp, dp]
        lib.oracle_h_apply.argtypes = [ci, ci, ci, ctypes.c_double, ci, ci, dp, ci, ctypes.POINTER(_Atom),
                                       dp, i64, dp, i64, ci]
        lib.oracle_cheb_filter.argtypes = [ci, ci, ci, ctypes.c_double, ci, ci, dp, ci, ctypes.POINTER(_Atom),
                                           dp, i64, dp, i64, ci, ci, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ci]
        lib.oracle_num_threads.restype = ci
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


# ----------------------------------------------------------------------------- operator pieces

def fd_weights(no: int, h: float) -> np.ndarray:
    """w_0..w_{n_o} of Sec. 3.1 Eq. weightsLap (FP64)."""
    w = np.zeros(16)
    _load().oracle_fd_weights(int(no), float(h), _dp(w))
    return w[: no + 1].copy()


def laplacian(n: Sequence[int], h: float, no: int, f: np.ndarray, bc: int = 0) -> np.ndarray:
    """lap_h f of Sec. 3.1 Eq. FD:Laplacian on one grid function (FP64)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    out = np.empty_like(f)
    _load().oracle_laplacian(int(n[0]), int(n[1]), int(n[2]), float(h), int(no), int(bc), _dp(f), _dp(out))
    return out


class _AtomTable:
    """Keeps the ctypes atom array and the buffers it points to alive."""

    def __init__(self, atoms):
        self.bufs = []
        self.arr = (_Atom * max(1, len(atoms)))()
        for i, a in enumerate(atoms):
            chi = np.ascontiguousarray(a.chi, dtype=np.float64).reshape(-1)
            gam = np.ascontiguousarray(a.gamma, dtype=np.float64)
            self.bufs += [chi, gam]
            self.arr[i].lo[:] = list(a.lo)
            self.arr[i].ext[:] = list(a.ext)
            self.arr[i].nproj = int(a.chi.shape[0])
            self.arr[i].chi = _dp(chi)
            self.arr[i].gamma = _dp(gam)
        self.n = len(atoms)


def _block(X: np.ndarray, nd: int) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X.reshape(1, -1)
    if X.shape[1] != nd:
        raise ValueError("orbital block must have shape (ns, nd)")
    return X


def h_apply(cluster, X: np.ndarray, bc: int = 0) -> np.ndarray:
    """H X for an orbital block (ns, nd): -1/2 lap_h + diag(V_eff) + V_nl."""
    nd = cluster.nd
    X = _block(X, nd)
    Y = np.empty_like(X)
    at = _AtomTable(cluster.atoms)
    n = cluster.n
    _load().oracle_h_apply(n[0], n[1], n[2], cluster.h, cluster.radius, bc, _dp(np.ascontiguousarray(cluster.veff)),
                           at.n, at.arr, _dp(X), nd, _dp(Y), nd, X.shape[0])
    return Y


def cheb_filter(cluster, X: np.ndarray, m: int, a0: float, a: float, b: float,
                scaled: bool = True, bc: int = 0) -> np.ndarray:
    """Chebyshev filter of Sec. 3.4 on an orbital block (ns, nd).

    scaled=True returns C_m((H-c)/e) X / C_m((a0-c)/e) (the normalised form of
    Alg. 2); scaled=False returns C_m((H-c)/e) X (Eq. ChebFilter as written).
    """
    if m < 1:
        raise ValueError("degree m must be >= 1")
    if not (a0 < a < b):
        raise ValueError("need a0 < a < b")
    nd = cluster.nd
    X = _block(X, nd)
    Y = np.empty_like(X)
    at = _AtomTable(cluster.atoms)
    n = cluster.n
    _load().oracle_cheb_filter(n[0], n[1], n[2], cluster.h, cluster.radius, bc,
                               _dp(np.ascontiguousarray(cluster.veff)), at.n, at.arr,
                               _dp(X), nd, _dp(Y), nd, X.shape[0], int(m), float(a0), float(a), float(b),
                               1 if scaled else 0)
    return Y


# ----------------------------------------------------------------------------- spectral bounds

def lanczos(cluster, k: int, v0: np.ndarray, bc: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """k steps of Lanczos on H with full re-orthogonalisation (FP64).

    Sec. 4 determines the extremal eigenvalues of H "using a few iterations of
    the Lanczos method"; step count, start vector and re-orthogonalisation are
    not stated, so: start from v0/|v0|, and after the three-term update remove
    the components along all previous basis vectors twice (classical
    Gram-Schmidt, repeated).  Returns (alpha[k], beta[k-1], theta[k]) where
    theta are the eigenvalues of the tridiagonal T_k, ascending.
    """
    import scipy.linalg

    nd = cluster.nd
    if not 1 <= k <= nd:
        raise ValueError("need 1 <= k <= N_d")
    V = np.zeros((k, nd))
    alpha = np.zeros(k)
    beta = np.zeros(max(k - 1, 0))
    V[0] = v0 / np.linalg.norm(v0)
    for j in range(k):
        w = h_apply(cluster, V[j], bc)[0]
        alpha[j] = V[j] @ w
        w = w - alpha[j] * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        for _ in range(2):
            w = w - V[: j + 1].T @ (V[: j + 1] @ w)
        if j + 1 < k:
            beta[j] = np.linalg.norm(w)
            if beta[j] == 0.0:
                raise ArithmeticError("Lanczos breakdown: invariant subspace reached")
            V[j + 1] = w / beta[j]
    theta = scipy.linalg.eigh_tridiagonal(alpha, beta, eigvals_only=True) if k > 1 else alpha.copy()
    return alpha, beta, np.sort(theta)


def upper_bound(cluster) -> float:
    """A guaranteed upper bound on lambda_max(H).

    -1/2 lap_h with zero padding is a Kronecker sum of three finite sections of
    a symmetric Toeplitz operator, so each 1D part is bounded by the maximum of
    its symbol s(t) = -1/2 (2 w_0 + 2 sum_p w_p cos(p t)).  The symbol maximum is
    taken on a fine grid of t and widened by the Lipschitz bound of s times the
    grid step.  V_eff contributes max V_eff, and each atom's V_nl,J is bounded
    by h^3 max(gamma_J, 0) * trace(chi_J^T chi_J).
    """
    w = fd_weights(cluster.radius, cluster.h)
    t = np.linspace(0.0, math.pi, 20001)
    p = np.arange(1, len(w))
    s = -0.5 * (2 * w[0] + 2 * (w[1:, None] * np.cos(p[:, None] * t[None, :])).sum(axis=0))
    lip = 0.5 * 2 * float(np.sum(np.abs(w[1:]) * p))
    smax = float(s.max()) + lip * (t[1] - t[0])
    bound = 3 * smax + float(np.max(cluster.veff))
    h3 = cluster.h ** 3
    for a in cluster.atoms:
        g = float(np.max(a.gamma))
        if g > 0:
            bound += h3 * g * float(np.sum(a.chi * a.chi))
    return bound


def select_bounds(theta: np.ndarray, nwant: int = 8, shift: float = 0.1, bfactor: float = 1.01,
                  ubound: Optional[float] = None) -> Tuple[float, float, float]:
    """Filter bounds (a0, a, b) from ascending Lanczos Ritz values.

    a0 = theta_1 (stands in for lambda_1 of Alg. 2), a = theta_nwant + shift
    (the cutoff lambda_c), b = bfactor * theta_max (lambda_Nd), clamped to the
    guaranteed upper bound when that is smaller.
    """
    theta = np.sort(np.asarray(theta, dtype=np.float64))
    a0 = float(theta[0])
    a = float(theta[min(nwant, len(theta)) - 1] + shift)
    b = float(bfactor * theta[-1])
    if ubound is not None and ubound < b:
        b = float(ubound)
    if not (a0 < a < b):
        raise ValueError("degenerate bounds a0=%g a=%g b=%g" % (a0, a, b))
    return a0, a, b


# ----------------------------------------------------------------------------- Rayleigh-Ritz

def rayleigh_ritz(cluster, Y: np.ndarray, bc: int = 0):
    """Projection onto the filtered block and the generalized eigenproblem.

    H_s = Y^T H Y, M_s = Y^T Y (the h^3 quadrature factor cancels), then
    H_s y = theta M_s y solved as a symmetric-definite problem (LAPACK via
    SciPy).  Returns (theta ascending, eigenvectors as columns, H_s, M_s).
    """
    import scipy.linalg

    Y = _block(Y, cluster.nd)
    HY = h_apply(cluster, Y, bc)
    Hs = Y @ HY.T
    Ms = Y @ Y.T
    Hs = 0.5 * (Hs + Hs.T)
    theta, vec = scipy.linalg.eigh(Hs, Ms)
    return theta, vec, Hs, Ms


def rotate(Y: np.ndarray, vec: np.ndarray) -> np.ndarray:
    """Psi = Psi_f Q with Psi_f column-major (rows of Y are columns of Psi_f)."""
    return (np.asarray(Y, dtype=np.float64).T @ vec).T.copy()


# ----------------------------------------------------------------------------- occupations and density

KT_DEFAULT = 1e-3  # smearing k_B T of the paper's runs (Sec. 4), Hartree


def occupations(theta, lambda_f: float, kT: float = KT_DEFAULT) -> np.ndarray:
    """g_n = 1 / (1 + exp((theta_n - lambda_f) / kT)) (Sec. 3.4), evaluated as
    exp(-x)/(1 + exp(-x)) for x > 0 so that no exponential overflows."""
    x = (np.asarray(theta, dtype=np.float64) - float(lambda_f)) / float(kT)
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def fermi_level(theta, ne: float, kT: float = KT_DEFAULT) -> float:
    """The Fermi energy lambda_f: the root of 2 sum_n g_n(lambda_f) = N_e
    (Sec. 3.4 Eq. FermiEnergyConstraintFormulation).  The left side increases
    strictly with lambda_f from 0 to 2 N_s, so for 0 < N_e < 2 N_s the root is
    unique; it is bracketed 50 k_B T beyond the extreme eigenvalues and found
    by bisection until the bracket stops shrinking (the paper uses Brent's
    method, Sec. 4, which converges to the same root).

    The constraint is evaluated as 2 ((#{theta_n <= l} - N_e / 2)
    + sum_{theta_n > l} g_n - sum_{theta_n <= l} (1 - g_n)), with 1 - g_n = g_n(2 l - theta_n)
    by the symmetry of the Fermi-Dirac function: the same value as
    2 sum_n g_n - N_e, but without the cancellation of 1 - g_n, so that the
    root stays determined across gaps up to about 1400 k_B T (beyond that the
    tails underflow and every point of the gap satisfies the constraint)."""
    th = np.asarray(theta, dtype=np.float64)
    ns = th.size
    if not 0.0 < ne < 2.0 * ns:
        raise ValueError("need 0 < N_e < 2 N_s")

    def f(lf):
        below = th <= lf
        tails = occupations(th[~below], lf, kT).sum() - occupations(2.0 * lf - th[below], lf, kT).sum()
        # the integer part first, so that tails below its rounding unit survive
        return 2.0 * ((below.sum() - 0.5 * ne) + tails)
    lo, hi = th.min() - 50.0 * kT, th.max() + 50.0 * kT
    while f(lo) > 0:
        lo -= 50.0 * kT
    while f(hi) < 0:
        hi += 50.0 * kT
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def density(Psi: np.ndarray, g, h: float) -> np.ndarray:
    """rho(x) = (2/h^3) sum_n g_n psi_n(x)^2 (Sec. 3.4) for an orbital block
    (ns, nd) whose rows are the orbitals."""
    Psi = np.asarray(Psi, dtype=np.float64)
    if Psi.ndim == 1:
        Psi = Psi.reshape(1, -1)
    g = np.asarray(g, dtype=np.float64)
    rho = np.zeros(Psi.shape[1])
    for n in range(Psi.shape[0]):
        rho += g[n] * Psi[n] * Psi[n]
    return 2.0 / h ** 3 * rho


# ----------------------------------------------------------------------------- gradient and nonlocal force

def gradient_weights(no: int, h: float) -> np.ndarray:
    """w~_1..w~_{n_o} of Eq. gradient:approximate (Sec. 3.1):
    w~_p = (-1)^(p+1) / (h p) * (n_o!)^2 / ((n_o - p)! (n_o + p)!).  Returned
    with index 0 unused (zero), so that w[p] is w~_p."""
    w = np.zeros(no + 1)
    f = math.factorial
    for p in range(1, no + 1):
        w[p] = (-1.0) ** (p + 1) / (h * p) * (f(no) ** 2 / (f(no - p) * f(no + p)))
    return w


def gradient(n: Sequence[int], h: float, no: int, f: np.ndarray) -> np.ndarray:
    """nabla_h f of Eq. gradient:approximate on one grid function: (3, N_d),
    component d the central difference along axis d (e_1 along the slowest
    index i), with f = 0 at every index outside the grid (Sec. 3.1)."""
    w = gradient_weights(no, h)
    F = np.zeros((n[0] + 2 * no, n[1] + 2 * no, n[2] + 2 * no))
    F[no:no + n[0], no:no + n[1], no:no + n[2]] = np.asarray(f, dtype=np.float64).reshape(n)
    out = np.zeros((3,) + tuple(n))
    for d in range(3):
        for p in range(1, no + 1):
            plus = [slice(no, no + n[a]) for a in range(3)]
            minus = [slice(no, no + n[a]) for a in range(3)]
            plus[d] = slice(no + p, no + p + n[d])
            minus[d] = slice(no - p, no - p + n[d])
            out[d] += w[p] * (F[tuple(plus)] - F[tuple(minus)])
    return out.reshape(3, -1)


def nonlocal_force(cluster, Psi: np.ndarray, g) -> np.ndarray:
    """Nonlocal atomic forces f_J (natoms, 3) of Sec. 3.6 Eq.
    NonlocForce:Discrete, following Alg. 4: for each atom J, the gradient
    nabla_h psi_n at the points of J's cube (Eq. gradient:approximate, psi = 0
    off the grid), Y_Jnlm = h^3 sum psi_n chi_Jlm and W_Jnlm = h^3 sum
    (nabla_h psi_n) chi_Jlm over the cube (Eq. NonLocForce:U:W), then
    f_J = -4 sum_n g_n sum_lm gamma_Jl Y_Jnlm W_Jnlm.  Psi: (ns, nd) block;
    g: the ns occupations."""
    Psi = _block(Psi, cluster.nd)
    g = np.asarray(g, dtype=np.float64)
    n, h, no = cluster.n, cluster.h, cluster.radius
    w = gradient_weights(no, h)
    h3 = h ** 3
    ns = Psi.shape[0]
    f = np.zeros((len(cluster.atoms), 3))
    for k in range(ns):
        P = np.zeros((n[0] + 2 * no, n[1] + 2 * no, n[2] + 2 * no))
        P[no:no + n[0], no:no + n[1], no:no + n[2]] = Psi[k].reshape(n)
        for J, a in enumerate(cluster.atoms):
            lo, ext = a.lo, a.ext
            cube = tuple(slice(no + lo[d], no + lo[d] + ext[d]) for d in range(3))
            psi = P[cube]
            grad = np.zeros((3,) + tuple(ext))
            for d in range(3):
                for p in range(1, no + 1):
                    plus, minus = list(cube), list(cube)
                    plus[d] = slice(no + lo[d] + p, no + lo[d] + ext[d] + p)
                    minus[d] = slice(no + lo[d] - p, no + lo[d] + ext[d] - p)
                    grad[d] += w[p] * (P[tuple(plus)] - P[tuple(minus)])
            for q in range(a.nproj):
                Y = h3 * np.sum(psi * a.chi[q])
                for d in range(3):
                    W = h3 * np.sum(grad[d] * a.chi[q])
                    f[J, d] += -4.0 * g[k] * a.gamma[q] * Y * W
    return f


# ----------------------------------------------------------------------------- CheFSI passes

CUTOFF_SHIFT = 0.1  # lambda_c = previous Fermi energy + 0.1 Ha (Sec. 4)


def chefsi_passes(cluster, X: np.ndarray, m, passes: int, ne: float, a0: float, a: float, b: float,
                  kT: float = KT_DEFAULT, shift: float = CUTOFF_SHIFT, bc: int = 0):
    """``passes`` CheFSI steps on the orbital block X (Sec. 3.4): filter with
    bounds (a0, cutoff, b), Rayleigh-Ritz, Fermi level of the Ritz values,
    rotation.  The first pass uses the cutoff ``a``; each later pass the
    previous pass's Fermi level plus ``shift`` (Sec. 4).  b (lambda_Nd of
    Alg. 2) stays fixed: without a density update H does not change between
    the passes of the first SCF iteration (Sec. 3.4, last paragraph).  a0
    (lambda_1 of Alg. 2) stays fixed too, unless a cutoff falls at or below
    it: the Lanczos estimate of lambda_1 was then too high, and a0 becomes
    the lowest Ritz value of the previous pass (also an upper bound of
    lambda_1, below that pass's Fermi level).  a0 only scales the filter's
    output, so the filtered subspace and the Ritz values do not depend on it.
    m: one degree for every pass, or a sequence of per-pass degrees.  Returns
    (rotated block, list of per-pass dicts with a0, the cutoff, degree, Ritz
    values and Fermi level)."""
    degrees = [int(m)] * passes if np.isscalar(m) else [int(d) for d in m]
    if len(degrees) != passes:
        raise ValueError("one degree per pass")
    X = _block(X, cluster.nd)
    cutoff = float(a)
    a0 = float(a0)
    record = []
    for p in range(passes):
        Y = cheb_filter(cluster, X, degrees[p], a0, cutoff, b, bc=bc)
        theta, vec, _, _ = rayleigh_ritz(cluster, Y, bc)
        lf = fermi_level(theta, ne, kT)
        X = rotate(Y, vec)
        record.append(dict(a0=a0, cutoff=cutoff, degree=degrees[p], theta=theta, lambda_f=lf))
        cutoff = lf + shift
        if cutoff <= a0:
            a0 = float(theta[0])
    return X, record


# ----------------------------------------------------------------------------- closed forms, brute force

def cheb_closed_form(m: int, x) -> np.ndarray:
    """C_m(x) = cos(m acos x) on [-1,1], sign(x)^m cosh(m acosh|x|) outside."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


def filter_gain(lam, m: int, a0: float, a: float, b: float) -> np.ndarray:
    """Scalar gain of the scaled filter at eigenvalue lam: C_m(l(lam))/C_m(l(a0))."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    return cheb_closed_form(m, (np.asarray(lam) - c) / e) / cheb_closed_form(m, np.array([(a0 - c) / e]))[0]


def fornberg_second_derivative(no: int):
    """Exact rational central weights c_{-no..no} of d^2/dx^2 on the unit-spaced
    stencil, from the moment conditions sum_j c_j j^q = q! [q == 2], q = 0..2no.

    An independent route to the Laplacian weights (Gauss-Jordan over
    fractions.Fraction); returns c_0..c_no (symmetric stencil)."""
    return _fornberg_central(no, 2)


def fornberg_first_derivative(no: int):
    """Exact rational central weights of d/dx on the unit-spaced stencil (the
    same moment conditions with q! [q == 1]); returns c_0..c_no (c_0 = 0,
    c_{-p} = -c_p).  An independent route to the gradient weights."""
    return _fornberg_central(no, 1)


def _fornberg_central(no: int, order: int):
    from fractions import Fraction

    pts = list(range(-no, no + 1))
    N = len(pts)
    rhs = Fraction(math.factorial(order))
    A = [[Fraction(j) ** q for j in pts] + [rhs if q == order else Fraction(0)] for q in range(N)]
    for col in range(N):
        piv = next(r for r in range(col, N) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(N):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [vr - f * vc for vr, vc in zip(A[r], A[col])]
    c = [A[i][N] for i in range(N)]
    return [c[no + p] for p in range(no + 1)]


def dense_hamiltonian(cluster, bc: int = 0) -> np.ndarray:
    """Brute-force dense H (N_d x N_d) for tiny grids.

    Built from 1D pieces rather than the stencil loop: the second-difference
    matrix D_d (size n_d) has c_0/h^2 on the diagonal and c_p/h^2 on the p-th
    off-diagonals (exact Fornberg weights), truncated at the walls for bc = 0
    or folded with odd reflection for bc = 1; the 3D Laplacian is the Kronecker
    sum D_x (+) D_y (+) D_z with x slowest.  Then H = -1/2 L + diag(V) +
    h^3 sum_J sum_p gamma_p chi_p chi_p^T with chi_p embedded in the grid.
    """
    n = cluster.n
    nd = cluster.nd
    if nd > 4096:
        raise ValueError("dense_hamiltonian is for tiny grids only")
    c = [float(v) for v in fornberg_second_derivative(cluster.radius)]
    h2 = cluster.h ** 2

    def d1(nn):
        D = np.zeros((nn, nn))
        for i in range(nn):
            for off in range(-cluster.radius, cluster.radius + 1):
                j = i + off
                coef = c[abs(off)] / h2
                if 0 <= j < nn:
                    D[i, j] += coef
                elif bc == 1:
                    per = 2 * (nn + 1)
                    r = (j + 1) % per
                    if r == 0 or r == nn + 1:
                        continue
                    if r <= nn:
                        D[i, r - 1] += coef
                    else:
                        D[i, per - r - 1] -= coef
        return D

    I = [np.eye(v) for v in n]
    L = (np.kron(d1(n[0]), np.kron(I[1], I[2])) + np.kron(I[0], np.kron(d1(n[1]), I[2]))
         + np.kron(I[0], np.kron(I[1], d1(n[2]))))
    H = -0.5 * L + np.diag(cluster.veff)
    h3 = cluster.h ** 3
    for a in cluster.atoms:
        for p in range(a.chi.shape[0]):
            full = np.zeros(n)
            full[a.lo[0]:a.lo[0] + a.ext[0], a.lo[1]:a.lo[1] + a.ext[1], a.lo[2]:a.lo[2] + a.ext[2]] = a.chi[p]
            v = full.reshape(-1)
            H += h3 * a.gamma[p] * np.outer(v, v)
    return H


def toeplitz_1d(no: int, h: float, nn: int) -> np.ndarray:
    """-1/2 times the zero-padded 1D second-difference matrix (exact weights)."""
    c = [float(v) for v in fornberg_second_derivative(no)]
    D = np.zeros((nn, nn))
    for i in range(nn):
        for off in range(-no, no + 1):
            j = i + off
            if 0 <= j < nn:
                D[i, j] = c[abs(off)] / h ** 2
    return -0.5 * D
