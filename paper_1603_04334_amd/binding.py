"""ctypes binding of libsparcfilter.so.

Argument marshalling only: every computation happens in the HIP library.
The raw entry points keep the C names (``sparc_h_apply`` ...); ``Operator``
wraps an op handle and turns torch device tensors into pointers, leading
dimensions and the current HIP stream.  Orbital blocks are torch tensors of
shape (ns, ld>=N_d) on the GPU: row c is orbital c, i.e. the column-major
N_d x ns block of the C ABI with leading dimension ``X.stride(0)``.

If the library has not been built this module raises on use; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsparcfilter.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sparc_filter.h")

SPARC_OK, SPARC_PENDING = 0, 1
SPARC_E_ARG, SPARC_E_SHAPE, SPARC_E_BOUNDS, SPARC_E_NOMEM, SPARC_E_HIP = -1, -2, -3, -4, -5
SPARC_E_BUSY, SPARC_E_TICKET, SPARC_E_JOB, SPARC_E_WORKSPACE, SPARC_E_BREAKDOWN, SPARC_E_ALIAS = -6, -7, -8, -9, -10, -11
SPARC_F64, SPARC_F32 = 0, 1
_STATUS_NAMES = {0: "SPARC_OK", 1: "SPARC_PENDING", -1: "SPARC_E_ARG", -2: "SPARC_E_SHAPE", -3: "SPARC_E_BOUNDS",
                 -4: "SPARC_E_NOMEM", -5: "SPARC_E_HIP", -6: "SPARC_E_BUSY", -7: "SPARC_E_TICKET", -8: "SPARC_E_JOB",
                 -9: "SPARC_E_WORKSPACE", -10: "SPARC_E_BREAKDOWN", -11: "SPARC_E_ALIAS"}


def status_name(status: int) -> str:
    return _STATUS_NAMES.get(int(status), f"status {status}")


class SparcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class sparc_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double), ("radius", ctypes.c_int32)]


class sparc_atom(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("ext", ctypes.c_int32 * 3), ("nproj", ctypes.c_int32),
                ("chi", ctypes.POINTER(ctypes.c_double)), ("gamma", ctypes.POINTER(ctypes.c_double))]


class sparc_batch_job(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
                ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64), ("ns", ctypes.c_int32), ("m", ctypes.c_int32),
                ("a0", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double)]


class sparc_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("workers", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("first_passes", ctypes.c_int32), ("kT", ctypes.c_double)]


class sparc_cluster_desc(ctypes.Structure):
    _fields_ = [("grid", sparc_grid), ("veff", ctypes.POINTER(ctypes.c_double)), ("natoms", ctypes.c_int32),
                ("atoms", ctypes.POINTER(sparc_atom)), ("dtype", ctypes.c_int32), ("ns", ctypes.c_int32),
                ("m", ctypes.c_int32), ("X0", ctypes.c_void_p), ("ldx0", ctypes.c_int64), ("v0", ctypes.c_void_p),
                ("ne", ctypes.c_double)]


class sparc_filter_job(ctypes.Structure):
    _fields_ = [("cluster", ctypes.c_uint64), ("desc", ctypes.POINTER(sparc_cluster_desc)), ("release", ctypes.c_int32),
                ("ritz", ctypes.POINTER(ctypes.c_double))]


class sparc_job_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("step", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double), ("lambda_min", ctypes.c_double),
                ("updates", ctypes.c_int64), ("lambda_f", ctypes.c_double), ("passes", ctypes.c_int32),
                ("halvings", ctypes.c_int32), ("error", ctypes.c_char * 128)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_dbl = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "sparc_op_create": (_i32, [ctypes.POINTER(sparc_grid), _dp, _i32, ctypes.POINTER(sparc_atom), ctypes.POINTER(_vp)]),
    "sparc_op_destroy": (_i32, [_vp]),
    "sparc_op_nd": (_i64, [_vp]),
    "sparc_op_nproj": (_i32, [_vp]),
    "sparc_workspace_bytes": (_sz, [_vp, _i32, _i32, _i32]),
    "sparc_h_apply": (_i32, [_vp, _i32, _vp, _i64, _vp, _i64, _i32, _vp, _sz, _vp]),
    "sparc_cheb_filter": (_i32, [_vp, _i32, _vp, _i64, _vp, _i64, _i32, _i32, _dbl, _dbl, _dbl, _vp, _sz, _vp]),
    "sparc_lanczos_workspace_bytes": (_sz, [_vp, _i32]),
    "sparc_lanczos": (_i32, [_vp, _i32, _vp, _dp, _dp, _dp, _vp, _sz, _vp]),
    "sparc_upper_bound": (_i32, [_vp, _dp]),
    "sparc_select_bounds": (_i32, [_dp, _i32, _i32, _dbl, _dbl, _dbl, _dp, _dp, _dp]),
    "sparc_rr_workspace_bytes": (_sz, [_vp, _i32, _i32]),
    "sparc_rayleigh_ritz": (_i32, [_vp, _i32, _vp, _i64, _i32, _dp, _vp, _vp, _sz, _vp]),
    "sparc_rotate": (_i32, [_i32, _vp, _i64, _i64, _i32, _vp, _vp, _i64, _vp, _sz, _vp]),
    "sparc_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "sparc_cleared_hip_errors": (_i64, []),
    "sparc_stream_copy": (_i32, [_vp, _vp, _sz, _vp]),
    "sparc_fermi_level": (_i32, [_dp, _i32, _dbl, _dbl, _dp, _dp]),
    "sparc_density": (_i32, [_i32, _vp, _i64, _i64, _i32, _vp, _dbl, _vp, _vp]),
    "sparc_poisson_create": (_i32, [ctypes.POINTER(sparc_grid), _i32, _vp, ctypes.POINTER(_vp)]),
    "sparc_poisson_destroy": (_i32, [_vp]),
    "sparc_poisson_workspace_bytes": (_sz, [_vp]),
    "sparc_poisson_solve": (_i32, [_vp, _vp, _vp, _i32, _dbl, _i32, ctypes.POINTER(_i32), _dp, _dp, _vp, _sz, _vp]),
    "sparc_force_workspace_bytes": (_sz, [_vp, _i32]),
    "sparc_nonlocal_force": (_i32, [_vp, _i32, _vp, _i64, _i32, _vp, _vp, _vp, _sz, _vp]),
    "sparc_chefsi_workspace_bytes": (_sz, [_vp, _i32, _i32]),
    "sparc_chefsi": (_i32, [_vp, _i32, _vp, _i64, _i32, _i32, _i32, _dbl, _dbl, _dbl, _dbl, _dbl, _dp, _dp,
                            ctypes.POINTER(_i32), _vp, _vp, _sz, _vp]),
    "sparc_h_apply_noalloc": (_i32, [_vp, _i32, _vp, _i64, _vp, _i64, _i32, _vp]),
    "sparc_noalloc_scratch_bytes": (_sz, []),
    "sparc_last_error": (ctypes.c_char_p, []),
    "sparc_profile_enable": (_i32, [_i32]),
    "sparc_profile_read": (_i32, [_i32, ctypes.POINTER(_i64), _dp]),
    "sparc_profile_reset": (_i32, []),
    "sparc_op_set_launch": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32]),
    "sparc_autotune": (_i32, [_vp, _i32, _i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                              ctypes.POINTER(_i32), ctypes.POINTER(_i32), _dp]),
    "sparc_rotate_workspace_bytes": (ctypes.c_size_t, [_i32, _i32]),
    "sparc_server_create": (_i32, [ctypes.POINTER(sparc_server_cfg), ctypes.POINTER(_vp)]),
    "sparc_filter_submit": (_i32, [_vp, ctypes.POINTER(sparc_filter_job), ctypes.POINTER(ctypes.c_uint64)]),
    "sparc_filter_poll": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(sparc_job_result)]),
    "sparc_server_stats": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                  ctypes.POINTER(ctypes.c_uint64)]),
    "sparc_server_destroy": (_i32, [_vp]),
    "sparc_server_clusters": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "sparc_clock": (ctypes.c_double, []),
    "sparc_cluster_footprint": (ctypes.c_uint64, [ctypes.POINTER(sparc_cluster_desc), _i32]),
    "sparc_batch_create": (_i32, [ctypes.POINTER(sparc_batch_job), _i32, _i32, ctypes.POINTER(_vp)]),
    "sparc_batch_run": (_i32, [_vp, _vp]),
    "sparc_batch_check": (_i32, [_vp, _vp, ctypes.POINTER(_i32)]),
    "sparc_batch_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "sparc_batch_destroy": (_i32, [_vp]),
    "sparc_step_config": (_i32, [_vp, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
}


def lib():
    """Load libsparcfilter.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the HIP library is required; there is no fallback)")
        # Load torch's HIP runtime first when torch is present: the library then
        # binds to the same runtime instance as the tensors it is handed.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> Sequence[str]:
    """Names of the functions declared in include/sparc_filter.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sparc_[a-z0-9_]+)\s*\(", text)))


def check(status: int, what: str = "") -> int:
    if status < 0:
        msg = lib().sparc_last_error().decode(errors="replace")
        raise SparcError(status, f"{what}: {msg}" if what else msg)
    return status


# ----------------------------------------------------------------------------- raw entry points

def _fn(name):
    def call(*args):
        return getattr(lib(), name)(*args)
    call.__name__ = name
    return call


for _name in _SIGS:
    globals()[_name] = _fn(_name)


# ----------------------------------------------------------------------------- convenience wrapper

def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return SPARC_F64
    if t.dtype == torch.float32:
        return SPARC_F32
    raise TypeError("orbital blocks must be float64 or float32")


def _block(t, nd: int, name: str):
    if t.dim() != 2 or t.shape[1] != nd or t.stride(1) != 1:
        raise ValueError(f"{name} must have shape (ns, nd={nd}) with unit stride along nd")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return t.shape[0], t.stride(0)


class Operator:
    """An op handle built from an ``inputs.Cluster``."""

    def __init__(self, cluster):
        self.cluster = cluster
        g, atoms, veff, keep = _cluster_arrays(cluster)
        h = _vp()
        check(lib().sparc_op_create(ctypes.byref(g), veff.ctypes.data_as(_dp), len(cluster.atoms), atoms,
                                    ctypes.byref(h)), "sparc_op_create")
        self.handle = h
        self.nd = int(lib().sparc_op_nd(h))

    def close(self):
        if getattr(self, "handle", None):
            lib().sparc_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- workspaces
    def workspace(self, dtype_code: int, ns: int, which: int, device=None):
        import torch
        nb = int(lib().sparc_workspace_bytes(self.handle, dtype_code, ns, which))
        return torch.empty(max(nb, 1), dtype=torch.uint8, device=device or "cuda")

    # -- entry points
    def h_apply(self, X, Y=None, ws=None, stream=None):
        import torch
        ns, ldx = _block(X, self.nd, "X")
        if Y is None:
            Y = torch.empty_like(X)
        _, ldy = _block(Y, self.nd, "Y")
        dt = _dtype_code(X)
        if ws is None:
            ws = self.workspace(dt, ns, 0, X.device)
        check(lib().sparc_h_apply(self.handle, dt, _ptr(X), ldx, _ptr(Y), ldy, ns, _ptr(ws), ws.numel(),
                                  _stream(stream)), "sparc_h_apply")
        return Y

    def cheb_filter(self, X, m: int, a0: float, a: float, b: float, Y=None, ws=None, stream=None):
        import torch
        ns, ldx = _block(X, self.nd, "X")
        if Y is None:
            Y = torch.empty_like(X)
        _, ldy = _block(Y, self.nd, "Y")
        dt = _dtype_code(X)
        if ws is None:
            ws = self.workspace(dt, ns, 1, X.device)
        check(lib().sparc_cheb_filter(self.handle, dt, _ptr(X), ldx, _ptr(Y), ldy, ns, int(m), float(a0),
                                      float(a), float(b), _ptr(ws), ws.numel(), _stream(stream)),
              "sparc_cheb_filter")
        return Y

    def lanczos(self, k: int, v0, stream=None, ws=None):
        import torch
        if v0.dtype != torch.float64 or v0.numel() != self.nd or not v0.is_cuda:
            raise ValueError("v0 must be a device float64 vector of N_d values")
        nb = int(lib().sparc_lanczos_workspace_bytes(self.handle, k))
        if ws is None:
            ws = torch.empty(nb, dtype=torch.uint8, device=v0.device)
        nb = ws.numel()
        alpha = np.zeros(k)
        beta = np.zeros(max(k - 1, 1))
        theta = np.zeros(k)
        check(lib().sparc_lanczos(self.handle, int(k), _ptr(v0), alpha.ctypes.data_as(_dp), beta.ctypes.data_as(_dp),
                                  theta.ctypes.data_as(_dp), _ptr(ws), nb, _stream(stream)), "sparc_lanczos")
        return alpha, beta[: k - 1], theta

    def upper_bound(self) -> float:
        ub = ctypes.c_double()
        check(lib().sparc_upper_bound(self.handle, ctypes.byref(ub)), "sparc_upper_bound")
        return ub.value

    def rayleigh_ritz(self, Yf, want_vectors: bool = True, stream=None):
        import torch
        ns, ldy = _block(Yf, self.nd, "Y")
        dt = _dtype_code(Yf)
        nb = int(lib().sparc_rr_workspace_bytes(self.handle, dt, ns))
        ws = torch.empty(nb, dtype=torch.uint8, device=Yf.device)
        theta = np.zeros(ns)
        evec = torch.empty((ns, ns), dtype=torch.float64, device=Yf.device) if want_vectors else None
        check(lib().sparc_rayleigh_ritz(self.handle, dt, _ptr(Yf), ldy, ns, theta.ctypes.data_as(_dp),
                                        _ptr(evec) if evec is not None else None, _ptr(ws), nb, _stream(stream)),
              "sparc_rayleigh_ritz")
        # evec is column-major ns x ns: as a torch (ns, ns) row-major tensor it is Q^T
        return theta, evec

    def nonlocal_force(self, Psi, occ, force=None, ws=None, stream=None):
        """Nonlocal atomic forces (natoms, 3) FP64 of the (ns, nd) block Psi with
        device FP64 occupations occ (ns,)."""
        import torch
        ns, ld = _block(Psi, self.nd, "Psi")
        natoms = len(self.cluster.atoms)
        if occ.dtype != torch.float64 or occ.numel() != ns or not occ.is_cuda or not occ.is_contiguous():
            raise ValueError("occ must be a contiguous device float64 tensor of ns entries")
        if force is None:
            force = torch.zeros(max(natoms, 1), 3, dtype=torch.float64, device=Psi.device)
        if ws is None:
            ws = torch.empty(max(1, int(lib().sparc_force_workspace_bytes(self.handle, ns))), dtype=torch.uint8,
                             device=Psi.device)
        check(lib().sparc_nonlocal_force(self.handle, _dtype_code(Psi), _ptr(Psi), ld, ns, _ptr(occ), _ptr(force),
                                         _ptr(ws), ws.numel(), _stream(stream)), "sparc_nonlocal_force")
        return force[:natoms]

    def chefsi(self, X, m: int, passes: int, ne: float, a0: float, a: float, b: float, kT: float = 1e-3,
               rho=None, ws=None, stream=None):
        """``passes`` CheFSI passes on X in place; returns (theta (passes, ns),
        lambda_f (passes,), degrees (passes,))."""
        import torch
        ns, ld = _block(X, self.nd, "X")
        dt = _dtype_code(X)
        if ws is None:
            ws = torch.empty(max(1, int(lib().sparc_chefsi_workspace_bytes(self.handle, dt, ns))), dtype=torch.uint8,
                             device=X.device)
        if rho is not None and (rho.dtype != torch.float64 or rho.numel() != self.nd or not rho.is_contiguous()):
            raise ValueError("rho must be a contiguous float64 tensor of N_d entries")
        theta = np.zeros((passes, ns))
        lf = np.zeros(passes)
        deg = np.zeros(passes, dtype=np.int32)
        check(lib().sparc_chefsi(self.handle, dt, _ptr(X), ld, ns, int(m), int(passes), float(ne), float(kT), float(a0),
                                 float(a), float(b), theta.ctypes.data_as(_dp), lf.ctypes.data_as(_dp),
                                 deg.ctypes.data_as(ctypes.POINTER(_i32)), _ptr(rho) if rho is not None else None,
                                 _ptr(ws), ws.numel(), _stream(stream)), "sparc_chefsi")
        return theta, lf, deg

    def set_launch(self, dtype_code: int, tile_z: int = 0, tile_y: int = 0, chunk_x: int = 0, col_group: int = 0,
                   col_block: int = 0):
        check(lib().sparc_op_set_launch(self.handle, dtype_code, tile_z, tile_y, chunk_x, col_group, col_block),
              "sparc_op_set_launch")

    def autotune(self, dtype_code: int, ns: int, stream=None):
        """(tile_z, tile_y, chunk_x, col_group, col_block, microseconds per step)"""
        tz, ty, cx, cg, cb = _i32(), _i32(), _i32(), _i32(), _i32()
        us = ctypes.c_double()
        check(lib().sparc_autotune(self.handle, dtype_code, ns, _stream(stream), ctypes.byref(tz), ctypes.byref(ty),
                                   ctypes.byref(cx), ctypes.byref(cg), ctypes.byref(cb), ctypes.byref(us)),
              "sparc_autotune")
        return tz.value, ty.value, cx.value, cg.value, cb.value, us.value

    def step_config(self, dtype_code: int, ns: int):
        """(tile_z, tile_y, chunk_x, col_group, col_block)"""
        tz, ty, cx, cg, cb = _i32(), _i32(), _i32(), _i32(), _i32()
        check(lib().sparc_step_config(self.handle, dtype_code, ns, ctypes.byref(tz), ctypes.byref(ty),
                                      ctypes.byref(cx), ctypes.byref(cg), ctypes.byref(cb)), "sparc_step_config")
        return tz.value, ty.value, cx.value, cg.value, cb.value


def stream_copy(dst, src, stream=None):
    """dst[:] = src with the library's reference copy kernel (device tensors
    of equal byte size, a multiple of 16)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("dst and src must have the same byte size")
    check(lib().sparc_stream_copy(_ptr(dst), _ptr(src), nb, _stream(stream)), "sparc_stream_copy")
    return dst


def select_bounds(theta, nwant: int = 8, shift: float = 0.1, bfactor: float = 1.01, ubound: float = 0.0):
    th = np.ascontiguousarray(np.sort(np.asarray(theta, dtype=np.float64)))
    a0, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(lib().sparc_select_bounds(th.ctypes.data_as(_dp), len(th), int(nwant), float(shift), float(bfactor),
                                    float(ubound), ctypes.byref(a0), ctypes.byref(a), ctypes.byref(b)),
          "sparc_select_bounds")
    return a0.value, a.value, b.value


def fermi_level(theta, ne: float, kT: float = 1e-3):
    """(lambda_f, occupations) for host eigenvalues theta and N_e electrons."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    occ = np.empty_like(th)
    lf = ctypes.c_double()
    check(lib().sparc_fermi_level(th.ctypes.data_as(_dp), len(th), float(ne), float(kT), ctypes.byref(lf),
                                  occ.ctypes.data_as(_dp)), "sparc_fermi_level")
    return lf.value, occ


def density(Psi, occ, h: float, rho=None, stream=None):
    """rho = (2/h^3) sum_n occ[n] Psi[n]^2 for an (ns, nd) device block;
    occ: device FP64 (ns,), rho: device FP64 (nd,) (allocated if None)."""
    import torch
    ns, nd = Psi.shape[0], Psi.shape[1]
    ld = _block(Psi, nd, "Psi")[1]
    if occ.dtype != torch.float64 or occ.numel() != ns or not occ.is_cuda or not occ.is_contiguous():
        raise ValueError("occ must be a contiguous device float64 tensor of ns entries")
    if rho is None:
        rho = torch.empty(nd, dtype=torch.float64, device=Psi.device)
    if rho.dtype != torch.float64 or rho.numel() != nd or not rho.is_contiguous():
        raise ValueError("rho must be a contiguous float64 tensor of nd entries")
    check(lib().sparc_density(_dtype_code(Psi), _ptr(Psi), ld, nd, ns, _ptr(occ), float(h), _ptr(rho),
                              _stream(stream)), "sparc_density")
    return rho


def rotate(Y, Qt, out=None, ws=None, stream=None):
    """Psi = Psi_f Q; Y and out are (ns, nd) blocks, Qt the (ns, ns) tensor
    returned by ``Operator.rayleigh_ritz`` (column-major Q)."""
    import torch
    ns, ldy = Y.shape[0], Y.stride(0)
    nd = Y.shape[1]
    if out is None:
        out = torch.empty_like(Y)
    dt = _dtype_code(Y)
    if ws is None:
        ws = torch.empty(max(1, int(lib().sparc_rotate_workspace_bytes(dt, ns))), dtype=torch.uint8, device=Y.device)
    check(lib().sparc_rotate(dt, _ptr(Y), ldy, nd, ns, _ptr(Qt), _ptr(out), out.stride(0), _ptr(ws), ws.numel(),
                             _stream(stream)), "sparc_rotate")
    return out


class Poisson:
    """Electrostatic potential solver for one grid (n, h, stencil radius)."""

    def __init__(self, n, h: float, radius: int = 6, lmax: int = 6, block=(4, 4, 4)):
        g = sparc_grid()
        g.n[0], g.n[1], g.n[2] = (int(v) for v in n)
        g.h = float(h)
        g.radius = int(radius)
        self.nd = int(n[0]) * int(n[1]) * int(n[2])
        self.lmax = int(lmax)
        blk = (_i32 * 3)(*[int(b) for b in block])
        hd = _vp()
        check(lib().sparc_poisson_create(ctypes.byref(g), int(lmax), ctypes.cast(blk, _vp), ctypes.byref(hd)),
              "sparc_poisson_create")
        self.handle = hd

    def solve(self, charge, phi=None, use_guess: bool = False, tol: float = 1e-10, max_iter: int = 5000, ws=None,
              stream=None):
        """Returns (phi, iterations, relative residual, moments Q_lm)."""
        import torch
        if charge.dtype != torch.float64 or charge.numel() != self.nd or not charge.is_cuda:
            raise ValueError("charge must be a device float64 tensor of N_d values")
        if phi is None:
            phi = torch.zeros(self.nd, dtype=torch.float64, device=charge.device)
        if ws is None:
            ws = torch.empty(int(lib().sparc_poisson_workspace_bytes(self.handle)), dtype=torch.uint8,
                             device=charge.device)
        it = _i32()
        res = ctypes.c_double()
        mom = np.zeros((self.lmax + 1) ** 2)
        check(lib().sparc_poisson_solve(self.handle, _ptr(charge), _ptr(phi), 1 if use_guess else 0, float(tol),
                                        int(max_iter), ctypes.byref(it), ctypes.byref(res), mom.ctypes.data_as(_dp),
                                        _ptr(ws), ws.numel(), _stream(stream)), "sparc_poisson_solve")
        return phi, it.value, res.value, mom

    def close(self):
        if getattr(self, "handle", None):
            lib().sparc_poisson_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of Chebyshev filters (one per job) run as one unit.

    jobs: sequence of (Operator, X, Y, m, a0, a, b) with X, Y device blocks of
    the same dtype.  mode: 0 persistent + HIP graph, 1 persistent, 2 one grouped
    launch per level, 3 the plain filters one after another, 4 mode 2 in a HIP
    graph, 5 the plain filters on the batch's four streams."""

    def __init__(self, jobs, mode: int = 0):
        arr = (sparc_batch_job * len(jobs))()
        self._refs = []
        for i, (op, X, Y, m, a0, a, b) in enumerate(jobs):
            ns, ldx = _block(X, op.nd, "X")
            _, ldy = _block(Y, op.nd, "Y")
            arr[i].op = op.handle
            arr[i].dtype = _dtype_code(X)
            arr[i].X = _ptr(X)
            arr[i].ldx = ldx
            arr[i].Y = _ptr(Y)
            arr[i].ldy = ldy
            arr[i].ns = ns
            arr[i].m = int(m)
            arr[i].a0, arr[i].a, arr[i].b = float(a0), float(a), float(b)
            self._refs += [op, X, Y]
        h = _vp()
        check(lib().sparc_batch_create(arr, len(jobs), int(mode), ctypes.byref(h)), "sparc_batch_create")
        self.handle = h

    def run(self, stream=None):
        check(lib().sparc_batch_run(self.handle, _stream(stream)), "sparc_batch_run")

    def check(self, stream=None) -> int:
        ab = _i32()
        lib().sparc_batch_check(self.handle, _stream(stream), ctypes.byref(ab))
        return ab.value

    def info(self):
        items, levels, grid = _i64(), _i32(), _i32()
        check(lib().sparc_batch_info(self.handle, ctypes.byref(items), ctypes.byref(levels), ctypes.byref(grid)))
        return items.value, levels.value, grid.value

    def close(self):
        if getattr(self, "handle", None):
            lib().sparc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cluster_arrays(cluster):
    """ctypes grid, atom array and the host buffers they point to."""
    g = sparc_grid()
    g.n[:] = list(cluster.n)
    g.h = cluster.h
    g.radius = cluster.radius
    keep = []
    atoms = (sparc_atom * max(1, len(cluster.atoms)))()
    for i, a in enumerate(cluster.atoms):
        chi = np.ascontiguousarray(a.chi, dtype=np.float64).reshape(-1)
        gam = np.ascontiguousarray(a.gamma, dtype=np.float64)
        keep += [chi, gam]
        atoms[i].lo[:] = list(a.lo)
        atoms[i].ext[:] = list(a.ext)
        atoms[i].nproj = a.chi.shape[0]
        atoms[i].chi = chi.ctypes.data_as(_dp)
        atoms[i].gamma = gam.ctypes.data_as(_dp)
    veff = np.ascontiguousarray(cluster.veff, dtype=np.float64)
    keep.append(veff)
    return g, atoms, veff, keep


def default_electrons(ns: int) -> float:
    """Electron count for ns orbitals by the paper's sizing rule ns = N_e/2 + 30
    (Sec. 4); for blocks of 60 orbitals or fewer, half of them occupied."""
    return float(2 * (ns - 30)) if ns > 60 else float(ns)


def cluster_desc(cluster, X0, v0, m: int, ne: float = None):
    """sparc_cluster_desc for an inputs.Cluster with device tensors X0 (ns, ld)
    and v0 (N_d, float64); ne defaults to ``default_electrons(ns)``."""
    g, atoms, veff, keep = _cluster_arrays(cluster)
    ns, ld = _block(X0, cluster.nd, "X0")
    d = sparc_cluster_desc()
    d.grid = g
    d.veff = veff.ctypes.data_as(_dp)
    d.natoms = len(cluster.atoms)
    d.atoms = atoms
    d.dtype = _dtype_code(X0)
    d.ns = ns
    d.m = int(m)
    d.X0 = _ptr(X0)
    d.ldx0 = ld
    d.v0 = _ptr(v0)
    d.ne = float(default_electrons(ns) if ne is None else ne)
    return d, keep + [atoms, X0, v0]


def cluster_footprint(cluster, X0, v0, m: int, lanczos_steps: int = 0) -> int:
    d, keep = cluster_desc(cluster, X0, v0, m, ne=1.0)
    return int(lib().sparc_cluster_footprint(ctypes.byref(d), int(lanczos_steps)))


def clock() -> float:
    return float(lib().sparc_clock())


class Server:
    """Request server: one SCF iteration's CheFSI passes per request on resident clusters."""

    def __init__(self, workers: int = 4, budget: int = 0, lanczos_steps: int = 0, first_passes: int = 0,
                 kT: float = 0.0):
        cfg = sparc_server_cfg(int(budget), int(workers), int(lanczos_steps), int(first_passes), float(kT))
        h = _vp()
        check(lib().sparc_server_create(ctypes.byref(cfg), ctypes.byref(h)), "sparc_server_create")
        self.handle = h
        self._keep = {}

    def submit(self, cluster_id: int, desc=None, release: bool = False, ritz=None) -> int:
        """desc: (sparc_cluster_desc, keep) from cluster_desc() for the cluster's first request."""
        job = sparc_filter_job()
        job.cluster = int(cluster_id)
        if desc is not None:
            job.desc = ctypes.pointer(desc[0])
            self._keep[int(cluster_id)] = desc[1]  # X0 and v0 must outlive admission
        job.release = 1 if release else 0
        if ritz is not None:
            job.ritz = ritz.ctypes.data_as(_dp)
        t = ctypes.c_uint64()
        check(lib().sparc_filter_submit(self.handle, ctypes.byref(job), ctypes.byref(t)), "sparc_filter_submit")
        return t.value

    def poll(self, ticket: int):
        r = sparc_job_result()
        st = lib().sparc_filter_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(r))
        if st == SPARC_PENDING:
            return None
        check(st, "sparc_filter_poll")
        return {"status": r.status, "step": r.step, "t_submit": r.t_submit, "t_start": r.t_start, "t_end": r.t_end,
                "lambda_min": r.lambda_min, "updates": r.updates, "lambda_f": r.lambda_f, "passes": r.passes,
                "halvings": r.halvings, "error": r.error.decode(errors="replace")}

    def stats(self):
        d, p, r, u = _i64(), _i64(), _i64(), ctypes.c_uint64()
        check(lib().sparc_server_stats(self.handle, ctypes.byref(d), ctypes.byref(p), ctypes.byref(r), ctypes.byref(u)))
        return {"done": d.value, "pending": p.value, "running": r.value, "hbm_used": u.value}

    def clusters(self):
        """(host cluster records held, retired cluster ids)."""
        n, r = _i64(), _i64()
        check(lib().sparc_server_clusters(self.handle, ctypes.byref(n), ctypes.byref(r)))
        return n.value, r.value

    def close(self):
        if getattr(self, "handle", None):
            lib().sparc_server_destroy(self.handle)
            self.handle = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class profile:
    """Per-kernel HIP-event timing inside the library (0 = fused recurrence step,
    1 = gather, 2 = scatter, 3 = fused step without Y_{k-1})."""

    @staticmethod
    def enable(on: bool = True):
        check(lib().sparc_profile_enable(1 if on else 0))

    @staticmethod
    def reset():
        check(lib().sparc_profile_reset())

    @staticmethod
    def read(kernel: int):
        n = _i64()
        ms = ctypes.c_double()
        check(lib().sparc_profile_read(int(kernel), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value
