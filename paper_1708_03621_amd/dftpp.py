"""Thin ctypes binding of libdftpp.so (C ABI in include/dftpp.h).

Every function here has the name of the C entry point it calls and only
marshals arguments: device arrays are passed as torch tensors (their
data_ptr), host arrays as NumPy arrays, handles as opaque pointers.  All
computation happens in the library's HIP kernels; there is no fallback.  A
non-zero status raises DppError with the library's error text.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdftpp.so")

DPP_F64 = 0
DPP_F32 = 1
DPP_STATUS_NOTPD = 1
DPP_STATUS_NONFINITE = 2
DPP_STATUS_NOBANDS = 4

STATUS_NAMES = {0: "DPP_OK", -1: "DPP_EINVAL", -2: "DPP_ENOMEM", -3: "DPP_EDEVICE", -4: "DPP_ENOTPD",
                -5: "DPP_ENOCONV", -6: "DPP_EUNSUPPORTED"}


class DppError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

_vp = C.c_void_p
_i = C.c_int
_i64 = C.c_int64
_d = C.c_double
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_szp = C.POINTER(C.c_size_t)

class dpp_system_desc(C.Structure):
    _fields_ = [("R", _dp), ("S", _ip), ("ecut", _d), ("nk", _i), ("kpts", _dp), ("wk", _dp), ("nb", _i),
                ("n_electrons", _d), ("nat", _i), ("tau", _dp), ("Z", _dp), ("rc", _dp), ("has_proj", _ip),
                ("rp", _d), ("D", _d), ("prec", _i)]


class dpp_energy(C.Structure):
    _fields_ = [("E_el", _d), ("E_kin", _d), ("E_nl", _d), ("E_loc", _d), ("E_H", _d), ("E_xc", _d)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class dpp_scf_desc(C.Structure):
    _fields_ = [("nat", _i), ("tau", _dp), ("Z", _dp), ("sigma", _d), ("d_n_start", _vp), ("n_inner", _i),
                ("n_inner_first", _i)]


DPP_FIELD_VLOC, DPP_FIELD_VEFF, DPP_FIELD_N, DPP_FIELD_NIN, DPP_FIELD_NOUT = range(5)

# name -> argtypes (all return int status except where noted)
SIGNATURES = {
    "dpp_ctx_create": [_i, _vp, C.POINTER(_vp)],
    "dpp_ctx_destroy": [_vp],
    "dpp_ctx_status": [_vp, _i, _ip],
    "dpp_grid_create": [_vp, _dp, _ip, C.POINTER(_vp)],
    "dpp_grid_destroy": [_vp],
    "dpp_grid_info": [_vp, _dp, _i64p],
    "dpp_basis_create": [_vp, _dp, _d, C.POINTER(_vp)],
    "dpp_basis_destroy": [_vp],
    "dpp_basis_info": [_vp, _i64p, _i32p],
    "dpp_basis_export": [_vp, _vp, _vp],
    "dpp_workspace_size": [_vp, _i, _i, _szp],
    "dpp_grid_workspace_size": [_vp, _szp],
    "dpp_I": [_vp, _i, _vp, _i64, _vp, _i, _vp],
    "dpp_Idag": [_vp, _i, _vp, _vp, _i64, _i, _i, _vp],
    "dpp_J": [_vp, _i, _vp, _vp, _vp],
    "dpp_Jdag": [_vp, _i, _vp, _vp, _vp],
    "dpp_O": [_vp, _i, _vp, _i64, _vp, _i64],
    "dpp_L": [_vp, _i, _vp, _i64, _vp, _i64],
    "dpp_K": [_vp, _i, _vp, _i64, _vp, _i64],
    "dpp_ham_create": [_vp, _i, _dp, _ip, _d, _d, C.POINTER(_vp)],
    "dpp_ham_destroy": [_vp],
    "dpp_ham_set_potential": [_vp, _vp],
    "dpp_apply_H": [_vp, _i, _vp, _i64, _vp, _i64, _i, _vp],
    "dpp_overlap": [_vp, _i, _vp, _i64, _i, _vp, _i64, _d, _vp, _i, _vp],
    "dpp_rotate": [_vp, _i, _vp, _i64, _i, _vp, _d, _vp, _i64, _i],
    "dpp_cholesky_inverse": [_vp, _i, _i, _vp, _vp],
    "dpp_cholesky_orthonormalize": [_vp, _i, _vp, _i64, _vp, _vp],
    "dpp_ortho_workspace_size": [_vp, _i, _szp],
    "dpp_subspace_eigh": [_vp, _i, _i, _vp, _vp, _vp, _vp],
    "dpp_eigh_workspace_size": [_i, _i, _szp],
    "dpp_subspace_eigh_noalloc": [_vp, _i, _i, _vp, _vp, _vp],
    "dpp_density_accumulate": [_vp, _i, _vp, _i64, _vp, _d, _vp, _i, _vp],
    "dpp_hartree": [_vp, _vp, _vp, _vp, _vp],
    "dpp_pcm_workspace_size": [_vp, C.POINTER(C.c_size_t)],
    "dpp_gga_workspace_size": [_vp, C.POINTER(C.c_size_t)],
    "dpp_gga_pbe": [_vp, _vp, _vp, _vp, _vp],
    "dpp_system_set_xc": [_vp, _i],
    "dpp_system_set_smearing": [_vp, C.c_double],
    "dpp_system_smearing_state": [_vp, _i, _dp, _dp],
    "dpp_pcm_solve": [_vp, _vp, _vp, C.c_double, _i, _vp, _dp, C.POINTER(C.c_int), _dp, _vp],
    "dpp_lda_pz81": [_vp, _vp, _vp, _vp, _vp],
    "dpp_local_potential": [_vp, _i, _dp, _dp, _dp, _vp, _vp],
    "dpp_start_density": [_vp, _i, _dp, _dp, _d, _vp, _vp],
    "dpp_grid_dot": [_vp, _vp, _vp, _d, _vp, _vp],
    "dpp_system_create": [_vp, C.POINTER(dpp_system_desc), C.POINTER(_vp)],
    "dpp_batch_create": [_vp, _i, C.POINTER(dpp_system_desc), C.POINTER(_vp)],
    "dpp_system_dims": [_vp, _ip, _ip, _i64p, _i64p, _i64p],
    "dpp_system_cells": [_vp, _ip, _i64p, _i64p],
    "dpp_set_graph_mode": [_vp, _i],
    "dpp_scf_cell_residuals": [_vp, _dp],
    "dpp_system_destroy": [_vp],
    "dpp_system_layout": [_vp, _i64p, _i64p],
    "dpp_system_field": [_vp, _i, C.POINTER(_vp)],
    "dpp_system_copy_field": [_vp, _i, _vp],
    "dpp_cg_V_init": [_vp, _vp, _i, _d, C.POINTER(dpp_energy)],
    "dpp_cg_V_step": [_vp, _vp, C.POINTER(dpp_energy), _ip],
    "dpp_cg_B_init": [_vp, _vp, _vp, _dp],
    "dpp_cg_B_step": [_vp, _vp, _dp],
    "dpp_band_eigenvalues": [_vp, _vp, _dp],
    "dpp_scf_init": [_vp, C.POINTER(dpp_scf_desc)],
    "dpp_scf_iteration": [_vp, _vp, C.POINTER(dpp_energy), _dp],
    "dpp_system_fillings": [_vp, _dp],
    "dpp_system_forces": [_vp, _vp, _vp, _vp, _vp, _dp],
    "dpp_system_set_positions": [_vp, _dp],
    "dpp_system_counters": [_vp, _i64p],
    "dpp_set_precision_policy": [_vp, _i, _d],
    "dpp_scf_status": [_vp, _dp, _ip, _ip],
    "dpp_system_apply_H": [_vp, _vp, _vp],
    "dpp_system_tune": [_vp, _vp, _vp, _i],
    "dpp_system_tune_report": [_vp, C.c_char_p, C.c_size_t],
    "dpp_system_set_launch_choice": [_vp, _i, _i],
    "dpp_net_create": [_vp, _ip, _i, C.POINTER(_vp)],
    "dpp_net_destroy": [_vp],
    "dpp_net_num_params": [_vp, _ip],
    "dpp_net_set_params": [_vp, C.POINTER(C.c_float)],
    "dpp_net_get_params": [_vp, C.POINTER(C.c_float), C.POINTER(C.c_float)],
    "dpp_net_forward": [_vp, _i, _vp, _d, _vp],
    "dpp_net_backward": [_vp, _i, _vp, _vp, _d, _dp],
    "dpp_net_adam_step": [_vp, _d],
    "dpp_net_train_epoch": [_vp, _i, _vp, _vp, _d, _i, _d, _ip, _dp],
    "dpp_net_predict_density": [_vp, _vp, _d, _d, _vp],
    "dpp_timer_enable": [_vp, _i],
    "dpp_timer_reset": [_vp],
    "dpp_timer_read": [_vp, _i, _dp, _i64p, _dp, _dp],
}

TIMER_KINDS = {"planes_in": 0, "xz_h": 1, "planes_out": 2, "xz_density": 3, "overlap": 4, "rotate": 5,
               "cholesky": 6, "eigh": 7, "fullbox": 8, "fields": 9, "blockops": 10, "xz_io": 11, "net": 12,
               "linesearch": 13, "masked": 14}


def load(path: str = LIB_PATH):
    """Load the library (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libdftpp.so not built at {path}; run paper_1708_03621_amd.build")
    lib = C.CDLL(path)
    lib.dpp_last_error.restype = C.c_char_p
    lib.dpp_last_error.argtypes = []
    lib.dpp_version.restype = C.c_int
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    _lib = lib
    return lib


def _call(name, *args):
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        raise DppError(st, lib.dpp_last_error().decode())
    return st


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _hd(a):
    """Host double array pointer (keeps a contiguous copy alive via the return)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


# ---------------------------------------------------------------- setup ----

def dpp_ctx_create(device: int = 0, stream=None):
    out = _vp()
    s = None if stream is None else C.c_void_p(int(stream))
    _call("dpp_ctx_create", device, s, C.byref(out))
    return out


def dpp_ctx_destroy(ctx):
    _call("dpp_ctx_destroy", ctx)


def dpp_ctx_status(ctx, clear: bool = True) -> int:
    v = C.c_int(0)
    _call("dpp_ctx_status", ctx, 1 if clear else 0, C.byref(v))
    return v.value


def dpp_grid_create(ctx, R, S):
    R = np.ascontiguousarray(np.asarray(R, float).reshape(3, 3))
    Sa = (C.c_int * 3)(*[int(s) for s in S])
    out = _vp()
    _call("dpp_grid_create", ctx, R.ctypes.data_as(_dp), C.cast(Sa, _ip), C.byref(out))
    return out


def dpp_grid_destroy(grid):
    _call("dpp_grid_destroy", grid)


def dpp_grid_info(grid):
    om = C.c_double()
    N = C.c_int64()
    _call("dpp_grid_info", grid, C.byref(om), C.byref(N))
    return om.value, N.value


def dpp_basis_create(grid, k_red, ecut: float):
    k, kp = _hd(np.asarray(k_red, float).reshape(3))
    out = _vp()
    _call("dpp_basis_create", grid, kp, float(ecut), C.byref(out))
    return out


def dpp_basis_destroy(basis):
    _call("dpp_basis_destroy", basis)


def dpp_basis_info(basis):
    npw = C.c_int64()
    ext = (C.c_int32 * 6)()
    _call("dpp_basis_info", basis, C.byref(npw), C.cast(ext, _i32p))
    return npw.value, list(ext)


def dpp_basis_export(basis, d_index=None, d_kG2=None):
    _call("dpp_basis_export", basis, _ptr(d_index), _ptr(d_kG2))


def dpp_workspace_size(basis, nb: int, prec: int = DPP_F64) -> int:
    v = C.c_size_t()
    _call("dpp_workspace_size", basis, nb, prec, C.byref(v))
    return v.value


def dpp_grid_workspace_size(grid) -> int:
    v = C.c_size_t()
    _call("dpp_grid_workspace_size", grid, C.byref(v))
    return v.value


def dpp_ortho_workspace_size(basis, nb: int) -> int:
    v = C.c_size_t()
    _call("dpp_ortho_workspace_size", basis, nb, C.byref(v))
    return v.value


def dpp_eigh_workspace_size(nb: int, batch: int) -> int:
    v = C.c_size_t()
    _call("dpp_eigh_workspace_size", nb, batch, C.byref(v))
    return v.value


# ------------------------------------------------------------ operators ----

def dpp_I(basis, nb, C_, ldC, grid_out, prec, ws):
    _call("dpp_I", basis, nb, _ptr(C_), ldC, _ptr(grid_out), prec, _ptr(ws))


def dpp_Idag(basis, nb, grid, C_out, ldC, accumulate, prec, ws):
    _call("dpp_Idag", basis, nb, _ptr(grid), _ptr(C_out), ldC, int(accumulate), prec, _ptr(ws))


def dpp_J(grid, nf, x, y, ws):
    _call("dpp_J", grid, nf, _ptr(x), _ptr(y), _ptr(ws))


def dpp_Jdag(grid, nf, x, y, ws):
    _call("dpp_Jdag", grid, nf, _ptr(x), _ptr(y), _ptr(ws))


def dpp_O(basis, nb, x, ldin, out, ldout):
    _call("dpp_O", basis, nb, _ptr(x), ldin, _ptr(out), ldout)


def dpp_L(basis, nb, x, ldin, out, ldout):
    _call("dpp_L", basis, nb, _ptr(x), ldin, _ptr(out), ldout)


def dpp_K(basis, nb, x, ldin, out, ldout):
    _call("dpp_K", basis, nb, _ptr(x), ldin, _ptr(out), ldout)


def dpp_ham_create(basis, tau, has_proj, rp: float, D: float):
    tau = np.ascontiguousarray(np.asarray(tau, float).reshape(-1, 3))
    hp = np.ascontiguousarray(np.asarray(has_proj, dtype=np.int32).reshape(-1))
    out = _vp()
    _call("dpp_ham_create", basis, len(hp), tau.ctypes.data_as(_dp), hp.ctypes.data_as(_ip), float(rp),
          float(D), C.byref(out))
    return out


def dpp_ham_destroy(ham):
    _call("dpp_ham_destroy", ham)


def dpp_ham_set_potential(ham, d_Veff):
    _call("dpp_ham_set_potential", ham, _ptr(d_Veff))


def dpp_apply_H(ham, nb, C_, ldC, HC, ldHC, prec, ws):
    _call("dpp_apply_H", ham, nb, _ptr(C_), ldC, _ptr(HC), ldHC, prec, _ptr(ws))


# --------------------------------------------------------- contractions ----

def dpp_overlap(basis, nbA, A, ldA, nbB, B, ldB, scale, U, ws, prec=DPP_F64):
    _call("dpp_overlap", basis, nbA, _ptr(A), ldA, nbB, _ptr(B), ldB, float(scale), _ptr(U), prec, _ptr(ws))


def dpp_rotate(basis, nbX, X, ldX, nbO, M, beta, out, ldout, prec=DPP_F64):
    _call("dpp_rotate", basis, nbX, _ptr(X), ldX, nbO, _ptr(M), float(beta), _ptr(out), ldout, prec)


def dpp_cholesky_inverse(ctx, nb, batch, U, Rinv):
    _call("dpp_cholesky_inverse", ctx, nb, batch, _ptr(U), _ptr(Rinv))


def dpp_cholesky_orthonormalize(basis, nb, Y, ldY, Rinv, ws):
    _call("dpp_cholesky_orthonormalize", basis, nb, _ptr(Y), ldY, _ptr(Rinv), _ptr(ws))


def dpp_subspace_eigh(ctx, nb, batch, H, eig, vecs, ws):
    _call("dpp_subspace_eigh", ctx, nb, batch, _ptr(H), _ptr(eig), _ptr(vecs), _ptr(ws))


def dpp_subspace_eigh_noalloc(ctx, nb, batch, H, eig, vecs):
    _call("dpp_subspace_eigh_noalloc", ctx, nb, batch, _ptr(H), _ptr(eig), _ptr(vecs))


# ------------------------------------------------- densities, potentials ----

def dpp_density_accumulate(basis, nb, psi, ldpsi, d_f, wk, d_n, prec, ws):
    _call("dpp_density_accumulate", basis, nb, _ptr(psi), ldpsi, _ptr(d_f), float(wk), _ptr(d_n), prec, _ptr(ws))


def dpp_hartree(grid, d_n, d_VH, d_EH, ws):
    _call("dpp_hartree", grid, _ptr(d_n), _ptr(d_VH), _ptr(d_EH), _ptr(ws))


def dpp_pcm_workspace_size(grid):
    v = C.c_size_t()
    _call("dpp_pcm_workspace_size", grid, C.byref(v))
    return v.value


def dpp_pcm_solve(grid, d_eps, d_rho, tol, max_iter, d_phi, ws):
    """Returns (A_diel, iterations, relative residual); phi(r) into d_phi (or None)."""
    A, it, rel = C.c_double(), C.c_int(), C.c_double()
    _call("dpp_pcm_solve", grid, _ptr(d_eps), _ptr(d_rho), float(tol), int(max_iter), _ptr(d_phi), C.byref(A),
          C.byref(it), C.byref(rel), _ptr(ws))
    return A.value, it.value, rel.value


def dpp_gga_workspace_size(grid):
    v = C.c_size_t()
    _call("dpp_gga_workspace_size", grid, C.byref(v))
    return v.value


def dpp_gga_pbe(grid, d_n, d_vxc, d_Exc, ws):
    _call("dpp_gga_pbe", grid, _ptr(d_n), _ptr(d_vxc), _ptr(d_Exc), _ptr(ws))


DPP_XC_LDA_PZ81, DPP_XC_PBE = 0, 1


def dpp_system_set_xc(sys_, functional):
    _call("dpp_system_set_xc", sys_, int(functional))


def dpp_system_set_smearing(sys_, sigma):
    _call("dpp_system_set_smearing", sys_, float(sigma))


def dpp_system_smearing_state(sys_, ncells=1):
    """Returns (mu, sigma S) arrays of the last smeared SCF iteration."""
    mu = np.zeros(ncells)
    ts = np.zeros(ncells)
    _call("dpp_system_smearing_state", sys_, int(ncells), mu.ctypes.data_as(_dp), ts.ctypes.data_as(_dp))
    return mu, ts


def dpp_lda_pz81(grid, d_n, d_vxc, d_Exc, ws):
    _call("dpp_lda_pz81", grid, _ptr(d_n), _ptr(d_vxc), _ptr(d_Exc), _ptr(ws))


def dpp_local_potential(grid, tau, Z, rc, d_Vloc, ws):
    tau = np.ascontiguousarray(np.asarray(tau, float).reshape(-1, 3))
    Z = np.ascontiguousarray(np.asarray(Z, float).reshape(-1))
    rc = np.ascontiguousarray(np.asarray(rc, float).reshape(-1))
    _call("dpp_local_potential", grid, len(Z), tau.ctypes.data_as(_dp), Z.ctypes.data_as(_dp),
          rc.ctypes.data_as(_dp), _ptr(d_Vloc), _ptr(ws))


def dpp_start_density(grid, tau, Z, sigma, d_n, ws):
    tau = np.ascontiguousarray(np.asarray(tau, float).reshape(-1, 3))
    Z = np.ascontiguousarray(np.asarray(Z, float).reshape(-1))
    _call("dpp_start_density", grid, len(Z), tau.ctypes.data_as(_dp), Z.ctypes.data_as(_dp), float(sigma),
          _ptr(d_n), _ptr(ws))


def dpp_grid_dot(grid, d_a, d_b, scale, d_out, ws):
    _call("dpp_grid_dot", grid, _ptr(d_a), _ptr(d_b), float(scale), _ptr(d_out), _ptr(ws))


# --------------------------------------------------------------- drivers ----

def _system_desc(keep, R, S, ecut, kpts, wk, nb, n_electrons, tau, Z, rc, has_proj, rp, D, prec):
    def arr(a, dt):
        keep.append(np.ascontiguousarray(np.asarray(a, dtype=dt).reshape(-1)))
        return keep[-1]

    Ra = arr(np.asarray(R, float).reshape(3, 3), np.float64)
    Sa = arr(S, np.int32)
    ka = arr(kpts, np.float64)
    wa = arr(wk, np.float64)
    ta = arr(tau, np.float64)
    Za = arr(Z, np.float64)
    ra = arr(rc, np.float64)
    ha = arr(has_proj, np.int32)
    return dpp_system_desc(Ra.ctypes.data_as(_dp), Sa.ctypes.data_as(_ip), float(ecut), len(wa), ka.ctypes.data_as(_dp),
                           wa.ctypes.data_as(_dp), int(nb), float(n_electrons), len(Za), ta.ctypes.data_as(_dp),
                           Za.ctypes.data_as(_dp), ra.ctypes.data_as(_dp), ha.ctypes.data_as(_ip), float(rp), float(D),
                           int(prec))


def dpp_system_create(ctx, R, S, ecut, kpts, wk, nb, n_electrons, tau, Z, rc, has_proj, rp, D, prec=DPP_F64):
    """Host arrays are kept alive for the duration of the call."""
    keep = []
    d = _system_desc(keep, R, S, ecut, kpts, wk, nb, n_electrons, tau, Z, rc, has_proj, rp, D, prec)
    out = _vp()
    _call("dpp_system_create", ctx, C.byref(d), C.byref(out))
    return out


def dpp_batch_create(ctx, cells, prec=DPP_F64):
    """cells: list of dicts with the dpp_system_create arguments R, S, ecut,
    kpts, wk, nb, n_electrons, tau, Z, rc, has_proj, rp, D."""
    keep = []
    arr = (dpp_system_desc * len(cells))()
    for i, c in enumerate(cells):
        arr[i] = _system_desc(keep, c["R"], c["S"], c["ecut"], c["kpts"], c["wk"], c["nb"], c["n_electrons"],
                              c["tau"], c["Z"], c["rc"], c["has_proj"], c["rp"], c["D"], prec)
    out = _vp()
    _call("dpp_batch_create", ctx, len(cells), arr, C.byref(out))
    return out


def dpp_system_dims(sys_):
    nc, ni = C.c_int(), C.c_int()
    tot, ns, ng = C.c_int64(), C.c_int64(), C.c_int64()
    _call("dpp_system_dims", sys_, C.byref(nc), C.byref(ni), C.byref(tot), C.byref(ns), C.byref(ng))
    return nc.value, ni.value, tot.value, ns.value, ng.value


def dpp_system_cells(sys_):
    nc = dpp_system_dims(sys_)[0]
    item0 = np.zeros(nc + 1, np.int32)
    foff = np.zeros(nc + 1, np.int64)
    state0 = np.zeros(nc + 1, np.int64)
    _call("dpp_system_cells", sys_, item0.ctypes.data_as(_ip), foff.ctypes.data_as(_i64p),
          state0.ctypes.data_as(_i64p))
    return item0, foff, state0


def dpp_set_graph_mode(sys_, on=True):
    _call("dpp_set_graph_mode", sys_, 1 if on else 0)


def dpp_system_tune(sys_, Y, HY, reps=5):
    _call("dpp_system_tune", sys_, _ptr(Y), _ptr(HY), int(reps))


DPP_CHOICE_OVERLAP, DPP_CHOICE_ROTATE_PT, DPP_CHOICE_XPASS = 0, 1, 2


def dpp_system_set_launch_choice(sys_, which, value):
    _call("dpp_system_set_launch_choice", sys_, int(which), int(value))


def dpp_system_tune_report(sys_) -> str:
    buf = C.create_string_buffer(4096)
    _call("dpp_system_tune_report", sys_, buf, C.c_size_t(4096))
    return buf.value.decode()


def dpp_scf_cell_residuals(sys_):
    r = np.zeros(dpp_system_dims(sys_)[0])
    _call("dpp_scf_cell_residuals", sys_, r.ctypes.data_as(_dp))
    return r


def dpp_system_destroy(sys_):
    _call("dpp_system_destroy", sys_)


def dpp_system_layout(sys_, nk=None):
    """Offsets (nitems + 1) and npw (nitems) of the packed layout."""
    if nk is None:
        nk = dpp_system_dims(sys_)[1]
    off = (C.c_int64 * (nk + 1))()
    npw = (C.c_int64 * nk)()
    _call("dpp_system_layout", sys_, C.cast(off, _i64p), C.cast(npw, _i64p))
    return list(off), list(npw)


def dpp_system_field(sys_, which):
    p = _vp()
    _call("dpp_system_field", sys_, int(which), C.byref(p))
    return p.value


def dpp_system_copy_field(sys_, which, d_out):
    _call("dpp_system_copy_field", sys_, int(which), _ptr(d_out))


def dpp_cg_V_init(sys_, Y, nocc, f):
    E = dpp_energy()
    _call("dpp_cg_V_init", sys_, _ptr(Y), int(nocc), float(f), C.byref(E))
    return E.as_dict()


def dpp_cg_V_step(sys_, Y):
    E = dpp_energy()
    st = C.c_int(0)
    _call("dpp_cg_V_step", sys_, _ptr(Y), C.byref(E), C.byref(st))
    return E.as_dict(), bool(st.value)


def dpp_cg_B_init(sys_, Y, d_Veff, nk):
    Eb = np.zeros(nk)
    vp = d_Veff if isinstance(d_Veff, int) else d_Veff.data_ptr()
    _call("dpp_cg_B_init", sys_, _ptr(Y), C.c_void_p(vp), Eb.ctypes.data_as(_dp))
    return Eb


def dpp_cg_B_step(sys_, Y, nk):
    Eb = np.zeros(nk)
    _call("dpp_cg_B_step", sys_, _ptr(Y), Eb.ctypes.data_as(_dp))
    return Eb


def dpp_band_eigenvalues(sys_, Y, nk, nb):
    e = np.zeros((nk, nb))
    _call("dpp_band_eigenvalues", sys_, _ptr(Y), e.ctypes.data_as(_dp))
    return e


def dpp_scf_init(sys_, tau=None, Z=None, sigma=1.0, d_n_start=None, n_inner=3, n_inner_first=0, cells=None):
    """One cell (tau, Z or d_n_start) or, with `cells`, a list of dicts with
    keys tau, Z, sigma, d_n_start (any may be absent) for every cell."""
    keep = []

    def desc(tau_, Z_, sigma_, start_):
        sp = None if start_ is None else C.c_void_p(start_.data_ptr())
        if tau_ is not None:
            ta = np.ascontiguousarray(np.asarray(tau_, float).reshape(-1))
            Za = np.ascontiguousarray(np.asarray(Z_, float).reshape(-1))
            keep.extend([ta, Za])
            return dpp_scf_desc(len(Za), ta.ctypes.data_as(_dp), Za.ctypes.data_as(_dp), float(sigma_), sp,
                                int(n_inner), int(n_inner_first))
        return dpp_scf_desc(0, None, None, float(sigma_), sp, int(n_inner), int(n_inner_first))

    if cells is None:
        cells = [dict(tau=tau, Z=Z, sigma=sigma, d_n_start=d_n_start)]
    arr = (dpp_scf_desc * len(cells))()
    for i, c in enumerate(cells):
        arr[i] = desc(c.get("tau"), c.get("Z"), c.get("sigma", sigma), c.get("d_n_start"))
    _call("dpp_scf_init", sys_, arr)


def dpp_scf_iteration(sys_, Y, nk=None, nb=None):
    """One cell with nk, nb given: (energy dict, eig (nk, nb)).  Otherwise:
    (list of energy dicts per cell, eig over all states)."""
    ncells, _, _, nstates, _ = dpp_system_dims(sys_)
    E = (dpp_energy * ncells)()
    e = np.zeros(nstates)
    _call("dpp_scf_iteration", sys_, _ptr(Y), E, e.ctypes.data_as(_dp))
    if ncells == 1 and nk is not None and nb is not None:
        return E[0].as_dict(), e.reshape(nk, nb)
    return [x.as_dict() for x in E], e


def dpp_system_fillings(sys_, nk, nb):
    f = np.zeros((nk, nb))
    _call("dpp_system_fillings", sys_, f.ctypes.data_as(_dp))
    return f


def dpp_system_forces(sys_, Y, F_loc, F_nl, F_ion, ncells):
    """Forces into caller-owned device tensors (3 per atom, or None); returns
    the ionic energy of every cell."""
    e = np.zeros(ncells)
    _call("dpp_system_forces", sys_, _ptr(Y), _ptr(F_loc), _ptr(F_nl), _ptr(F_ion), e.ctypes.data_as(_dp))
    return e


def dpp_system_set_positions(sys_, tau):
    t = np.ascontiguousarray(tau, dtype=np.float64).reshape(-1)
    _call("dpp_system_set_positions", sys_, t.ctypes.data_as(_dp))


def dpp_set_precision_policy(sys_, bulk, refine_residual):
    _call("dpp_set_precision_policy", sys_, int(bulk), float(refine_residual))


def dpp_scf_status(sys_):
    r = C.c_double()
    p = C.c_int()
    n = C.c_int()
    _call("dpp_scf_status", sys_, C.byref(r), C.byref(p), C.byref(n))
    return r.value, p.value, n.value


def dpp_system_counters(sys_):
    v = C.c_int64()
    _call("dpp_system_counters", sys_, C.byref(v))
    return v.value


def dpp_system_apply_H(sys_, Y, HY):
    _call("dpp_system_apply_H", sys_, _ptr(Y), _ptr(HY))


def dpp_timer_enable(ctx, on=True):
    _call("dpp_timer_enable", ctx, 1 if on else 0)


def dpp_timer_reset(ctx):
    _call("dpp_timer_reset", ctx)


def dpp_timer_read(ctx, kind):
    """Summed (ms, launches, algorithmic bytes, flops) of one kernel class."""
    ms = C.c_double()
    n = C.c_int64()
    by = C.c_double()
    fl = C.c_double()
    k = TIMER_KINDS[kind] if isinstance(kind, str) else int(kind)
    _call("dpp_timer_read", ctx, k, C.byref(ms), C.byref(n), C.byref(by), C.byref(fl))
    return ms.value, n.value, by.value, fl.value


# ------------------------------------------------- learned start density ----

def dpp_net_create(ctx, S, max_batch):
    Sa = (C.c_int * 3)(*[int(x) for x in S])
    out = _vp()
    _call("dpp_net_create", ctx, C.cast(Sa, _ip), int(max_batch), C.byref(out))
    return out


def dpp_net_destroy(net):
    _call("dpp_net_destroy", net)


def dpp_net_num_params(net):
    v = C.c_int()
    _call("dpp_net_num_params", net, C.byref(v))
    return v.value


def dpp_net_set_params(net, params):
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    _call("dpp_net_set_params", net, a.ctypes.data_as(C.POINTER(C.c_float)))


def dpp_net_get_params(net):
    n = dpp_net_num_params(net)
    p = np.zeros(n, np.float32)
    g = np.zeros(n, np.float32)
    _call("dpp_net_get_params", net, p.ctypes.data_as(C.POINTER(C.c_float)), g.ctypes.data_as(C.POINTER(C.c_float)))
    return p, g


def dpp_net_forward(net, batch, d_n0, nbar, d_y=None):
    _call("dpp_net_forward", net, int(batch), _ptr(d_n0), float(nbar), _ptr(d_y))


def dpp_net_backward(net, batch, d_n0, d_nconv, nbar):
    l = C.c_double()
    _call("dpp_net_backward", net, int(batch), _ptr(d_n0), _ptr(d_nconv), float(nbar), C.byref(l))
    return l.value


def dpp_net_adam_step(net, lr):
    _call("dpp_net_adam_step", net, float(lr))


def dpp_net_train_epoch(net, nsamples, d_n0, d_nconv, nbar, batch, lr, order):
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    l = C.c_double()
    _call("dpp_net_train_epoch", net, int(nsamples), _ptr(d_n0), _ptr(d_nconv), float(nbar), int(batch), float(lr),
          o.ctypes.data_as(_ip), C.byref(l))
    return l.value


def dpp_net_predict_density(net, d_n0, n_electrons, omega, d_n_out):
    _call("dpp_net_predict_density", net, _ptr(d_n0), float(n_electrons), float(omega), _ptr(d_n_out))


def exported_symbols():
    """Names the binding expects the library to export."""
    return ["dpp_last_error", "dpp_version"] + list(SIGNATURES)
