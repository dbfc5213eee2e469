"""Dump and replay of one filter job (inputs and outputs in a NumPy .npz file).

A job is the operator's cluster (grid, spacing, stencil radius, V_eff and the
atoms' projector cubes), the orbital block X, the filter's degree and bounds
(Sec. 3.4 Eq. ChebFilter / Alg. 2) and the block Y the library returned.  The
file holds plain arrays only (``numpy.load`` with ``allow_pickle=False``
reads it), so a job captured on one machine can be re-run elsewhere and
compared bit for bit: the library's results do not depend on scheduling.
"""
from __future__ import annotations

import numpy as np

from . import inputs


def save_filter_job(path, cluster: inputs.Cluster, X, m: int, a0: float, a: float, b: float, Y) -> None:
    """Write the job to ``path`` (.npz).  X and Y are (ns, N_d) host arrays or
    device tensors of the same dtype (float64 or float32)."""
    X = _host(X)
    Y = _host(Y)
    if X.shape != Y.shape or X.dtype != Y.dtype or X.shape[1] != cluster.nd:
        raise ValueError("X and Y must be (ns, N_d) blocks of one dtype")
    at = cluster.atoms
    np.savez(
        path,
        n=np.asarray(cluster.n, dtype=np.int64), h=np.float64(cluster.h), radius=np.int64(cluster.radius),
        seed=np.int64(cluster.seed), veff=np.asarray(cluster.veff, dtype=np.float64),
        atom_pos=np.asarray([x.pos for x in at], dtype=np.float64).reshape(len(at), 3),
        atom_Z=np.asarray([x.Z for x in at], dtype=np.int64),
        atom_sigma=np.asarray([x.sigma for x in at], dtype=np.float64),
        atom_lo=np.asarray([x.lo for x in at], dtype=np.int64).reshape(len(at), 3),
        atom_ext=np.asarray([x.ext for x in at], dtype=np.int64).reshape(len(at), 3),
        atom_nproj=np.asarray([x.nproj for x in at], dtype=np.int64),
        chi=np.concatenate([x.chi.ravel() for x in at]) if at else np.zeros(0),
        gamma=np.concatenate([x.gamma.ravel() for x in at]) if at else np.zeros(0),
        X=X, Y=Y, m=np.int64(m), bounds=np.asarray([a0, a, b], dtype=np.float64))


def load_filter_job(path):
    """(cluster, X, m, (a0, a, b), Y) from a file written by save_filter_job."""
    with np.load(path, allow_pickle=False) as z:
        atoms = []
        off = goff = 0
        for i in range(len(z["atom_Z"])):
            ext = tuple(int(v) for v in z["atom_ext"][i])
            npj = int(z["atom_nproj"][i])
            cnt = npj * ext[0] * ext[1] * ext[2]
            atoms.append(inputs.Atom(pos=z["atom_pos"][i].copy(), Z=int(z["atom_Z"][i]),
                                     sigma=float(z["atom_sigma"][i]),
                                     lo=tuple(int(v) for v in z["atom_lo"][i]), ext=ext,
                                     chi=z["chi"][off:off + cnt].reshape((npj,) + ext).copy(),
                                     gamma=z["gamma"][goff:goff + npj].copy()))
            off += cnt
            goff += npj
        cl = inputs.Cluster(n=tuple(int(v) for v in z["n"]), h=float(z["h"]), radius=int(z["radius"]),
                            veff=z["veff"].copy(), atoms=atoms, seed=int(z["seed"]))
        a0, a, b = (float(v) for v in z["bounds"])
        return cl, z["X"].copy(), int(z["m"]), (a0, a, b), z["Y"].copy()


def replay_filter_job(path):
    """Run the saved job again through the library on the current device:
    (Y now, Y saved, True when they are equal bit for bit)."""
    import torch

    from . import binding

    cl, X, m, (a0, a, b), Y = load_filter_job(path)
    op = binding.Operator(cl)
    Xd = torch.from_numpy(X).cuda()
    Yn = op.cheb_filter(Xd, m, a0, a, b).cpu().numpy()
    return Yn, Y, bool(np.array_equal(Yn, Y))


def _host(t):
    if hasattr(t, "detach"):
        t = t.detach().cpu().numpy()
    return np.ascontiguousarray(t)
