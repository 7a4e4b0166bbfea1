"""Density, Hartree solve, total energy and its gradient (FP64 oracle).

Electronic state of one cell: per k-point a block Y_k (npw_k, nb) of
unorthonormalized coefficients; psi_k = Y_k R_k^{-1} from the Cholesky factor
of U_k = Y_k^dag O Y_k (Sec. 2.1, integrals as dot products with O).

  density   n_j = sum_k w_k sum_i f_ki |(I psi_ki)_j|^2,  (Omega/N) sum_j n_j = N_e
  Hartree   n~ = J n;  V_H(G) = 4 pi n~(G) / |G|^2 for G != 0, 0 at G = 0
            (coulomb operator of Sec. 2.1, diagonal in plane waves);
            V_H(r) = Re[I V_H];  E_H = (Omega/2) sum_{G!=0} 4 pi |n~|^2 / |G|^2
  energies  E_kin = sum_k w_k sum_i f_ki (Omega/2) sum_G |k+G|^2 |psi_Gi|^2
            E_nl  = sum_k w_k sum_i f_ki D sum_a |(P_k^dag psi_ki)_a|^2
            E_loc = (Omega/N) sum_j V_loc,j n_j;  E_xc = (Omega/N) sum_j n_j eps_xc
            (LDA PZ81, oracle/xc.py; with System.xc = "pbe" E_xc and v_xc
            come from oracle/gga.py)
            E_el  = E_kin + E_nl + E_loc + E_H + E_xc   (ion-ion excluded)
  gradient  with equal fillings f on the minimized block (energy invariant
            under Y -> Y M), dE/dY_k^dag = w_k f (H_k Y - O Y U^{-1} Y^dag H_k Y) U^{-1},
            H_k the Kohn-Sham operator with V_eff = V_loc + V_H + v_xc.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import operators as ops
from .basis import Basis, box_G2, cell_volume, gsphere
from .transforms import I, J, I_full
from .xc import lda_pz81


@dataclasses.dataclass
class System:
    """One cell with its k-point bases and pseudopotential data."""
    R: np.ndarray
    S: tuple
    bases: List[Basis]
    wk: np.ndarray
    Vloc: np.ndarray            # real grid
    P: List[np.ndarray]         # per k (npw, nproj)
    D: float
    n_electrons: int
    nat: int
    xc: str = "lda"             # "lda" (PZ81, oracle/xc.py) or "pbe" (oracle/gga.py)

    @property
    def omega(self) -> float:
        return cell_volume(self.R)

    @property
    def N(self) -> int:
        return int(np.prod(self.S))


def build_system(cell, with_local=True, with_projectors=True, xc="lda") -> System:
    """Set up bases, V_loc and projectors for a workloads.Cell (xc: "lda" or "pbe")."""
    from workloads import PROJ_D, PROJ_RP
    bases = [gsphere(cell.R, cell.S, k, cell.ecut) for k in cell.kpts]
    if with_local:
        Vloc = ops.local_potential(cell.R, cell.S, cell.tau, cell.Z, cell.rc)
    else:
        Vloc = np.zeros(cell.S)
    hp = cell.has_proj if with_projectors else np.zeros(cell.nat, bool)
    P = [ops.projectors(b, cell.tau, hp, PROJ_RP) for b in bases]
    return System(np.asarray(cell.R, float), tuple(cell.S), bases, np.asarray(cell.wk, float),
                  Vloc, P, PROJ_D, cell.n_electrons, cell.nat, xc)


def density(psis, fills, sys: System) -> np.ndarray:
    n = np.zeros(sys.S)
    for k, b in enumerate(sys.bases):
        X = I(psis[k], b)
        for i in range(psis[k].shape[1]):
            if fills[k][i] != 0.0:
                n += sys.wk[k] * fills[k][i] * np.abs(X[i]) ** 2
    return n


def hartree(n: np.ndarray, R) -> tuple:
    """Return (V_H(r), E_H) for a real density n on the box."""
    S = n.shape
    omega = cell_volume(R)
    nt = J(n)
    G2 = box_G2(R, S)
    kern = np.where(G2 > 0, 4.0 * np.pi / np.where(G2 > 0, G2, 1.0), 0.0)
    VHt = kern * nt
    EH = 0.5 * omega * float(np.sum(kern * np.abs(nt) ** 2))
    return np.real(I_full(VHt)), EH


def potentials(n: np.ndarray, sys: System):
    """V_eff and the density-dependent energy terms for density n."""
    VH, EH = hartree(n, sys.R)
    dV = sys.omega / sys.N
    if sys.xc == "pbe":
        from .gga import pbe_on_grid
        vxc, Exc = pbe_on_grid(n, sys.R)
    else:
        eps, vxc = lda_pz81(n)
        Exc = float(dV * np.sum(n * eps))
    Eloc = float(dV * np.sum(sys.Vloc * n))
    return sys.Vloc + VH + vxc, dict(E_H=EH, E_xc=Exc, E_loc=Eloc)


def band_energies(psis, fills, sys: System):
    """E_kin and E_nl from orthonormal psi."""
    Ekin = 0.0
    Enl = 0.0
    for k, b in enumerate(sys.bases):
        f = np.asarray(fills[k], float)
        colk = 0.5 * b.omega * np.sum(b.kG2[:, None] * np.abs(psis[k]) ** 2, axis=0)
        Ekin += sys.wk[k] * float(np.sum(f * colk))
        if sys.P[k].shape[1] > 0:
            Pi = sys.P[k].conj().T @ psis[k]
            Enl += sys.wk[k] * sys.D * float(np.sum(f * np.sum(np.abs(Pi) ** 2, axis=0)))
    return Ekin, Enl


def orthonormalize_all(Ys, sys: System):
    out = []
    for k, b in enumerate(sys.bases):
        psi, Rm, Rinv = ops.cholesky_orthonormalize(Ys[k], b)
        out.append((psi, Rinv))
    return out


def total_energy(Ys, fills, sys: System, return_parts=False):
    """E_el for unorthonormalized blocks Y (orthonormalized internally)."""
    psis = [p for p, _ in orthonormalize_all(Ys, sys)]
    n = density(psis, fills, sys)
    Veff, parts = potentials(n, sys)
    Ekin, Enl = band_energies(psis, fills, sys)
    E = Ekin + Enl + parts["E_loc"] + parts["E_H"] + parts["E_xc"]
    if return_parts:
        parts.update(E_kin=Ekin, E_nl=Enl, E_el=E)
        return E, parts, n, Veff
    return E


def energy_and_gradient(Ys, f: float, sys: System):
    """E_el and dE/dY^dag per k for blocks with equal filling f (protocol V)."""
    fills = [np.full(Y.shape[1], f) for Y in Ys]
    E, parts, n, Veff = total_energy(Ys, fills, sys, return_parts=True)
    grads = []
    for k, b in enumerate(sys.bases):
        Y = Ys[k]
        U = ops.overlap(Y, Y, b)
        Uinv = np.linalg.inv(U)
        HY = ops.apply_H(Y, b, Veff, sys.P[k], sys.D)
        g = sys.wk[k] * f * (HY - ops.O(Y, b) @ (Uinv @ (Y.conj().T @ HY))) @ Uinv
        grads.append(g)
    return E, grads


def band_energy_and_gradient(Y, b: Basis, Veff, P, D):
    """Protocol B objective at fixed H: Tr(U^{-1} Y^dag H Y) and its gradient."""
    U = ops.overlap(Y, Y, b)
    Uinv = np.linalg.inv(U)
    HY = ops.apply_H(Y, b, Veff, P, D)
    Hs = Y.conj().T @ HY
    E = float(np.real(np.trace(Uinv @ Hs)))
    g = (HY - ops.O(Y, b) @ (Uinv @ Hs)) @ Uinv
    return E, g


def start_density(cell, sigma: float) -> np.ndarray:
    """Superposition of atomic Gaussians:
    n0(G) = (1/Omega) sum_a Z_a exp(-G^2 sigma^2 / 4) exp(-i G.tau_a);  n0(r) = Re[I n0]."""
    from .basis import box_G
    R = np.asarray(cell.R, float)
    omega = cell_volume(R)
    G = box_G(R, cell.S)
    G2 = np.sum(G * G, axis=-1)
    nt = np.zeros(G2.shape, complex)
    for a in range(cell.nat):
        nt += cell.Z[a] * np.exp(-G2 * sigma * sigma / 4.0) * np.exp(-1j * (G @ cell.tau[a]))
    return np.real(I_full(nt / omega))


def residual_norm(psi, eps, b: Basis, Veff, P, D) -> float:
    """max_i ||(H - eps_i O) psi_i||_2 / sqrt(Omega)."""
    Hpsi = ops.apply_H(psi, b, Veff, P, D)
    r = Hpsi - ops.O(psi, b) * eps[None, :]
    return float(np.max(np.linalg.norm(r, axis=0)) / np.sqrt(b.omega))
