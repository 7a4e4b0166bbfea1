"""Diagonal operators, pseudopotential model, Hamiltonian and overlap.

Sec. 2.1: O (overlap, diagonal in plane waves; integrals are dot products
with O) and the pointwise product of a real-space field with I(...).
The remaining DFT++ diagonals follow the plane-wave convention with
O = Omega (no 1/sqrt(Omega) in the coefficients):
  O   = Omega
  L   = -Omega |k+G|^2          (Laplacian; kinetic operator is -L/2)
  K   = 1 / (1 + |k+G|^2 / 2)   (preconditioner)

Pseudopotential model of the synthetic workloads:
  local  v_a(G) = -4 pi Z_a exp(-G^2 r_c^2 / 4) / (Omega G^2),  v_a(0) = 0
         (the Fourier transform of -Z erf(r/r_c)/r; G = 0 term dropped)
  V_loc(G) = sum_a v_a(|G|) exp(-i G.tau_a),  V_loc(r) = Re[I V_loc]
  nonlocal P_k[G,a] = beta(|k+G|) exp(-i G.tau_a), beta(q) = exp(-q^2 r_p^2/2)
         (continuum transform of a unit-integral Gaussian of width r_p; the
         per-atom phase exp(-i k.tau) cancels in P D P^dag and is dropped)
Kohn-Sham operator on a block C (npw, nb):
  H C = -L/2 C + (Omega/N) I^dag(V_eff * I C) + P D P^dag C.
"""
from __future__ import annotations

import numpy as np

from .basis import Basis, box_G, cell_volume, reciprocal_basis
from .transforms import I, Idag, I_full


def O(C: np.ndarray, b: Basis) -> np.ndarray:
    return b.omega * C


def L(C: np.ndarray, b: Basis) -> np.ndarray:
    d = -b.omega * b.kG2
    return d[:, None] * C if C.ndim == 2 else d * C


def K(C: np.ndarray, b: Basis) -> np.ndarray:
    d = 1.0 / (1.0 + 0.5 * b.kG2)
    return d[:, None] * C if C.ndim == 2 else d * C


def local_potential_G(R, S, tau, Z, rc) -> np.ndarray:
    """Reciprocal-space local pseudopotential on the full box."""
    omega = cell_volume(R)
    G = box_G(R, S)
    G2 = np.sum(G * G, axis=-1)
    safe = np.where(G2 > 0, G2, 1.0)
    Vt = np.zeros(G2.shape, complex)
    for a in range(len(Z)):
        v = -4.0 * np.pi * Z[a] * np.exp(-G2 * rc[a] ** 2 / 4.0) / (omega * safe)
        v = np.where(G2 > 0, v, 0.0)
        Vt += v * np.exp(-1j * (G @ tau[a]))
    return Vt


def local_potential(R, S, tau, Z, rc) -> np.ndarray:
    """V_loc(r) on the grid: Re[I V_loc(G)]."""
    return np.real(I_full(local_potential_G(R, S, tau, Z, rc)))


def projectors(b: Basis, tau, has_proj, rp) -> np.ndarray:
    """P_k (npw, nproj) for the atoms that carry the Gaussian s-projector."""
    beta = np.exp(-b.kG2 * rp * rp / 2.0)
    G = b.n @ reciprocal_basis(b.R).T       # G alone, without k
    cols = [beta * np.exp(-1j * (G @ tau[a])) for a in range(len(tau)) if has_proj[a]]
    if not cols:
        return np.zeros((b.npw, 0), complex)
    return np.stack(cols, axis=1)


def apply_H(C: np.ndarray, b: Basis, Veff: np.ndarray, P: np.ndarray | None, D: float) -> np.ndarray:
    """Kohn-Sham Hamiltonian on a block C (npw, nb)."""
    out = -0.5 * L(C, b)
    out = out + (b.omega / b.N) * Idag(Veff[None] * I(C, b), b)
    if P is not None and P.shape[1] > 0:
        out = out + P @ (D * (P.conj().T @ C))
    return out


def overlap(A: np.ndarray, B: np.ndarray, b: Basis) -> np.ndarray:
    """A^dag O B."""
    return A.conj().T @ O(B, b)


PIVOT_RTOL = 1e-14


def cholesky_orthonormalize(Y: np.ndarray, b: Basis):
    """U = Y^dag O Y = R^dag R (R upper, positive diagonal); psi = Y R^{-1}.

    Returns (psi, R, Rinv).  Raises numpy.linalg.LinAlgError if U is not
    positive definite.
    """
    U = overlap(Y, Y, b)
    Lc = np.linalg.cholesky(U)      # U = Lc Lc^dag
    Rm = Lc.conj().T
    # numerically rank-deficient blocks: a pivot R_jj^2 at or below
    # PIVOT_RTOL * max_i U_ii is treated as not positive definite
    if np.min(np.real(np.diag(Rm))) ** 2 <= PIVOT_RTOL * np.max(np.real(np.diag(U))):
        raise np.linalg.LinAlgError("overlap not positive definite")
    Rinv = np.linalg.inv(Rm)
    return Y @ Rinv, Rm, Rinv


def dense_hamiltonian(b: Basis, Veff: np.ndarray, P: np.ndarray | None, D: float) -> np.ndarray:
    """Explicit npw x npw matrix of H: kinetic + Omega * V~[(n - n') mod S] + P D P^dag.

    V~ = J V_eff.  With the index taken modulo the box this is exactly the
    FFT operator used by apply_H (no dealiasing).
    """
    Vt = np.fft.fftn(Veff) / Veff.size
    S = np.array(b.S)
    dn = b.n[:, None, :] - b.n[None, :, :]
    dm = np.mod(dn, S)
    Vmat = Vt[dm[..., 0], dm[..., 1], dm[..., 2]]
    H = b.omega * Vmat + np.diag(0.5 * b.omega * b.kG2)
    if P is not None and P.shape[1] > 0:
        H = H + D * (P @ P.conj().T)
    return H
