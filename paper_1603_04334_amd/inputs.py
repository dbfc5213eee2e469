"""Seeded synthetic cluster generator.

This module builds the *inputs* of the Chebyshev-filter hot path: a uniform
grid, a local effective potential sampled at the grid nodes, Kleinman-Bylander
projector values on each atom's cube, projector energies, and blocks of random
orbitals.  It holds none of the method's arithmetic (no finite-difference
weights, no Hamiltonian application, no filter): both the HIP library and the
CPU oracle consume the arrays it returns, and neither imports the other.

Conventions (the paper is silent on these; the readings are fixed here):

* Grid (Sec. 3.1): nodes ``i = 1..n`` per axis sit at ``x_i = i*h``; the two
  zero-Dirichlet walls are at ``0`` and ``(n+1)*h``.  Arrays use 0-based index
  ``i0 = i-1`` and the linear index ``k + n3*(j + n2*i)`` (z fastest).
* Local potential: ``V_eff(x) = sum_J -Z_J exp(-|x-R_J|^2 / (2 sigma_J^2))``
  evaluated at every node in FP64 (no cutoff).
* Projectors (Sec. 2, Eq. V_nl; Sec. 3.1 Eq. non-localPS:FD): for each atom
  ``chi_Jlm(x) = exp(-r^2/(2*0.7^2)) * Y_lm(x-R_J)`` for ``r <= 2.5`` bohr and
  0 beyond, with orthonormal real spherical harmonics ordered ``l = 0,1,2``
  then ``m = -l..l``, and ``Y_lm := 0`` at ``r = 0`` for ``l >= 1``.  The
  projector is stored over the cube of nodes with ``|x_d - R_d| <= 2.5`` on
  every axis (the paper uses cubes rather than spheres around atoms, Sec. 3.2).
  ``gamma_Jl`` is drawn per (atom, l) and shared by the ``2l+1`` values of m.
* Randomness: NumPy PCG64 streams derived from ``SeedSequence(seed)`` with a
  distinct spawn key per quantity; orbital column ``n`` has a stream of its
  own, so any subset of columns can be regenerated without the rest.
"""
from __future__ import annotations

import dataclasses
import math
from functools import lru_cache
from typing import List, Optional, Sequence, Tuple

import numpy as np

# spawn keys of the independent random streams
_KEY_POS, _KEY_Z, _KEY_SIGMA, _KEY_GAMMA, _KEY_X, _KEY_LANCZOS, _KEY_MISC = range(7)

PROJ_WIDTH = 0.7     # Gaussian width of the radial projector factor (bohr)
PROJ_CUTOFF = 2.5    # projector cutoff radius (bohr)
WALL_MARGIN = 4.0    # minimum atom distance from the domain walls (bohr)


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=seed, spawn_key=tuple(key))))


@dataclasses.dataclass
class Atom:
    pos: np.ndarray          # (3,) bohr
    Z: int
    sigma: float
    lo: Tuple[int, int, int]     # first 0-based node index of the projector cube, per axis
    ext: Tuple[int, int, int]    # cube extent per axis
    chi: np.ndarray          # (nproj, ext0, ext1, ext2) float64, z fastest
    gamma: np.ndarray        # (nproj,) float64

    @property
    def nproj(self) -> int:
        return int(self.chi.shape[0])


@dataclasses.dataclass
class Cluster:
    n: Tuple[int, int, int]
    h: float
    radius: int
    veff: np.ndarray         # (N_d,) float64, linear index k + n3*(j + n2*i)
    atoms: List[Atom]
    seed: int

    @property
    def nd(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nproj_total(self) -> int:
        return sum(a.nproj for a in self.atoms)


# ----------------------------------------------------------------------------- spherical harmonics

def real_ylm(lmax: int, dx: np.ndarray, dy: np.ndarray, dz: np.ndarray) -> List[np.ndarray]:
    """Orthonormal real spherical harmonics Y_lm(r_hat), l = 0..lmax, m = -l..l.

    Returned in the order (0,0), (1,-1), (1,0), (1,1), (2,-2), ..., (2,2).
    For l >= 1 the value at r = 0 is defined as 0.
    """
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    safe = np.where(r > 0, r, 1.0)
    x, y, z = dx / safe, dy / safe, dz / safe
    nz = (r > 0).astype(np.float64)
    out = [np.full_like(r, 0.5 / math.sqrt(math.pi))]
    if lmax >= 1:
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        out += [c1 * y * nz, c1 * z * nz, c1 * x * nz]
    if lmax >= 2:
        c2 = 0.5 * math.sqrt(15.0 / math.pi)
        c20 = 0.25 * math.sqrt(5.0 / math.pi)
        c22 = 0.25 * math.sqrt(15.0 / math.pi)
        out += [c2 * x * y * nz, c2 * y * z * nz, c20 * (3 * z * z - 1.0) * nz,
                c2 * x * z * nz, c22 * (x * x - y * y) * nz]
    if lmax >= 3:
        raise ValueError("lmax <= 2 supported")
    return out


# ----------------------------------------------------------------------------- cluster construction

def node_coords(n: int, h: float) -> np.ndarray:
    """Coordinates of the n nodes of one axis: x_i = i*h, i = 1..n."""
    return (np.arange(n, dtype=np.float64) + 1.0) * h


def _place_atoms(rng: np.random.Generator, natoms: int, n: Sequence[int], h: float,
                 margin: float, min_dist: float) -> np.ndarray:
    lo = np.full(3, margin)
    hi = (np.asarray(n, dtype=np.float64) + 1.0) * h - margin
    if np.any(hi < lo):
        raise ValueError("domain too small for the wall margin")
    pos = np.zeros((natoms, 3))
    placed = 0
    tries = 0
    while placed < natoms:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place atoms with the requested spacing")
        p = lo + (hi - lo) * rng.random(3)
        if placed and min_dist > 0:
            d = np.sqrt(((pos[:placed] - p) ** 2).sum(axis=1))
            if np.any(d < min_dist):
                continue
        pos[placed] = p
        placed += 1
    return pos


def _projector_cube(n: Sequence[int], h: float, R: np.ndarray, lmax: int):
    lo, ext, coords = [], [], []
    for d in range(3):
        xs = node_coords(n[d], h)
        idx = np.nonzero(np.abs(xs - R[d]) <= PROJ_CUTOFF)[0]
        if idx.size == 0:
            raise ValueError("projector cube is empty")
        lo.append(int(idx[0]))
        ext.append(int(idx.size))
        coords.append(xs[idx] - R[d])
    dx, dy, dz = np.meshgrid(coords[0], coords[1], coords[2], indexing="ij")
    r2 = dx * dx + dy * dy + dz * dz
    radial = np.exp(-r2 / (2.0 * PROJ_WIDTH ** 2)) * (r2 <= PROJ_CUTOFF ** 2)
    chi = np.stack([radial * y for y in real_ylm(lmax, dx, dy, dz)])
    return tuple(lo), tuple(ext), np.ascontiguousarray(chi)


def make_cluster(n: Sequence[int] | int, h: float, natoms: int, zmax: int, lmax: int, seed: int,
                 radius: int = 6, min_dist: float = 2.0, margin: float = WALL_MARGIN,
                 gamma_range: float = 2.0) -> Cluster:
    """Build one synthetic cluster (positions, Z, sigma, gamma, V_eff, projectors)."""
    if isinstance(n, int):
        n = (n, n, n)
    n = tuple(int(v) for v in n)
    pos = _place_atoms(_rng(seed, _KEY_POS), natoms, n, h, margin, min_dist)
    Z = _rng(seed, _KEY_Z).integers(1, zmax + 1, size=natoms)
    sig = _rng(seed, _KEY_SIGMA).uniform(0.8, 1.2, size=natoms)
    gam_l = _rng(seed, _KEY_GAMMA).uniform(-gamma_range, gamma_range, size=(natoms, lmax + 1))

    xs, ys, zs = (node_coords(n[d], h) for d in range(3))
    veff = np.zeros(n, dtype=np.float64)
    for J in range(natoms):
        gx = np.exp(-((xs - pos[J, 0]) ** 2) / (2 * sig[J] ** 2))
        gy = np.exp(-((ys - pos[J, 1]) ** 2) / (2 * sig[J] ** 2))
        gz = np.exp(-((zs - pos[J, 2]) ** 2) / (2 * sig[J] ** 2))
        veff -= Z[J] * gx[:, None, None] * gy[None, :, None] * gz[None, None, :]

    atoms = []
    for J in range(natoms):
        lo, ext, chi = _projector_cube(n, h, pos[J], lmax)
        gamma = np.concatenate([np.full(2 * l + 1, gam_l[J, l]) for l in range(lmax + 1)])
        atoms.append(Atom(pos=pos[J].copy(), Z=int(Z[J]), sigma=float(sig[J]), lo=lo, ext=ext,
                          chi=chi, gamma=gamma.astype(np.float64)))
    return Cluster(n=n, h=float(h), radius=int(radius), veff=veff.reshape(-1), atoms=atoms, seed=seed)


def free_cluster(n: Sequence[int] | int, h: float, v0: float = 0.0, radius: int = 6) -> Cluster:
    """A cluster with constant potential v0 and no atoms (closed-form test cases)."""
    if isinstance(n, int):
        n = (n, n, n)
    n = tuple(int(v) for v in n)
    nd = n[0] * n[1] * n[2]
    return Cluster(n=n, h=float(h), radius=int(radius), veff=np.full(nd, float(v0)), atoms=[], seed=0)


def orbitals(nd: int, ns: int, seed: int, cols: Optional[Sequence[int]] = None,
             dtype=np.float64) -> np.ndarray:
    """N(0,1) orbital block, column-major: returns an array of shape (ncols, nd).

    Column c is drawn from its own stream, so ``orbitals(..., cols=[c])`` equals
    row c of the full block.
    """
    cols = range(ns) if cols is None else cols
    out = np.empty((len(cols), nd), dtype=dtype)
    for i, c in enumerate(cols):
        if not 0 <= c < ns:
            raise IndexError(c)
        out[i] = _rng(seed, _KEY_X, int(c)).standard_normal(nd)
    return out


def device_orbitals(nd: int, ns: int, seed: int, dtype=None, device: str = "cuda"):
    """N(0,1) orbital block of shape (ns, nd) drawn on the device by torch's
    seeded generator (Philox), for blocks too large to draw on the host
    (600 columns of a 160^3 grid are 2.5e9 values).  The same seed gives the
    same block; the FP32 block is drawn in FP32 and the FP64 block is its
    exact widening, so both dtypes start from the same values.  Columns are
    copied to the host where a CPU check needs them."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    X = torch.randn(ns, nd, generator=gen, device=device, dtype=torch.float32)
    if dtype is not None and dtype != torch.float32:
        X = X.to(dtype)
    return X


def lanczos_start(nd: int, seed: int) -> np.ndarray:
    """N(0,1) start vector of the spectral-bound Lanczos pass (not normalised)."""
    return _rng(seed, _KEY_LANCZOS).standard_normal(nd)


def round_to_f32(a: np.ndarray) -> np.ndarray:
    """Round-to-nearest FP32 copy, promoted back to FP64 (what an FP32 run sees)."""
    return a.astype(np.float32).astype(np.float64)


def round_cluster_f32(c: Cluster) -> Cluster:
    """The cluster as an FP32 run stores it: V_eff and chi rounded once to FP32.

    gamma is not rounded: the library folds h^3*gamma into the FP64 gathered
    coefficients before rounding them.
    """
    atoms = [dataclasses.replace(a, chi=round_to_f32(a.chi)) for a in c.atoms]
    return dataclasses.replace(c, veff=round_to_f32(c.veff), atoms=atoms)


# ----------------------------------------------------------------------------- workload recipes

@dataclasses.dataclass(frozen=True)
class FilterCase:
    name: str
    n: int
    h: float
    natoms: int
    zmax: int
    lmax: int
    ns: int
    m: int
    seed: int
    min_dist: float = 2.0


# Single-cluster workloads (grid edge, spacing, atoms, projectors per atom,
# orbitals, filter degree) with the paper's production stencil order n_o = 6.
SMALL = FilterCase("cluster24_h0.5_2atoms_8orb_m20", 24, 0.5, 2, 4, 1, 8, 20, seed=1, min_dist=0.0)
MEDIUM = FilterCase("cluster96_h0.4_16atoms_64orb_m24", 96, 0.4, 16, 8, 1, 64, 24, seed=2)
LARGE = FilterCase("cluster160_h0.35_128atoms_600orb_m30", 160, 0.35, 128, 8, 2, 600, 30, seed=3)
CASES = {c.name: c for c in (SMALL, MEDIUM, LARGE)}


@lru_cache(maxsize=8)
def case_cluster(name: str) -> Cluster:
    c = CASES[name]
    return make_cluster(c.n, c.h, c.natoms, c.zmax, c.lmax, c.seed, min_dist=c.min_dist)


def batch_recipe(seed: int = 4, nclusters: int = 64) -> List[dict]:
    """Uneven-cluster batch: grid edge in {32,40,...,96}, h = 0.45, atoms 2..24
    scaled with volume, orbitals U{16..128}, degree U{16..28}."""
    rng = _rng(seed, _KEY_MISC)
    edges = np.arange(32, 97, 8)
    out = []
    for i in range(nclusters):
        n = int(rng.choice(edges))
        natoms = int(round(2 + 22 * (n ** 3 - 32 ** 3) / (96 ** 3 - 32 ** 3)))
        out.append(dict(n=n, h=0.45, natoms=natoms, zmax=8, lmax=1,
                        ns=int(rng.integers(16, 129)), m=int(rng.integers(16, 29)), seed=1000 * seed + i))
    return out


def serving_recipe(seed: int = 5, nclusters: int = 64, rate: float = 200.0,
                   steps_per_cluster: int = 5, edge_range=(24, 128), ns_range=(8, 256),
                   fp32_share: float = 0.8) -> List[dict]:
    """Serving stream of cluster sessions.  Each session is one cluster with
    ``steps_per_cluster`` filtered-subspace passes, run one after another;
    sessions arrive as a Poisson process whose request rate (passes per
    second) is ``rate``, i.e. sessions at rate / steps_per_cluster.  Clusters:
    grid edge log-uniform in [24,128] (rounded to a multiple of 8), h = 0.45,
    atoms clamp(round(64 (n/128)^3), 1, 64), degree U{20..30}, FP32 with
    probability 0.8.  The orbital count follows the paper's rule (Sec. 4)
    N_s = N_e/2 + 30 with N_e = sum of the cluster's Z (the same Z that
    ``make_cluster`` draws), clamped to ``ns_range``.  Returns sessions in
    arrival order: dicts with the cluster, ``t_arrive`` and ``steps``."""
    rng = _rng(seed, _KEY_MISC, 1)
    clusters = []
    for i in range(nclusters):
        e = math.exp(rng.uniform(math.log(edge_range[0]), math.log(edge_range[1])))
        n = int(max(edge_range[0], min(edge_range[1], 8 * round(e / 8))))
        natoms = int(min(64, max(1, round(64 * (n / 128.0) ** 3))))
        cseed = 100000 + 1000 * seed + i
        ne = int(_rng(cseed, _KEY_Z).integers(1, 8 + 1, size=natoms).sum())
        ns = int(min(ns_range[1], max(ns_range[0], (ne + 1) // 2 + 30)))
        clusters.append(dict(n=n, h=0.45, natoms=natoms, zmax=8, lmax=1, ns=ns, ne=ne,
                             m=int(rng.integers(20, 31)),
                             fp32=bool(rng.random() < fp32_share), seed=cseed))
    # arrival gaps come from their own stream, so the clusters do not depend on the rate
    arr = _rng(seed, _KEY_MISC, 2)
    t = 0.0
    sessions = []
    for c in clusters:
        t += arr.exponential(steps_per_cluster / rate)
        sessions.append(dict(cluster=c, t_arrive=t, steps=steps_per_cluster))
    return sessions
