"""Forces on the ions (FP64 oracle; test infrastructure only: tests/, the
smoke check and the CPU baseline use it, the library never does).

The paper lists ionic and lattice optimization among the solver's features
(Table 1) and drives it from its input language (Sec. 3, the ionic
minimization of the example).  The force on ion a is -dE/dtau_a, with E the
electronic energy E_el of this model plus the electrostatic energy of the
point ions in a uniform compensating background.  The plane-wave basis does
not depend on the positions, so at a self-consistent state the force is the
sum of the explicit position derivatives below (Hellmann-Feynman); at any
state each of them is the exact derivative of its energy term at fixed
density or fixed wavefunctions.

  local     E_loc = (Omega/N) sum_j n_j V_loc(r_j) = Omega Re sum_G conj(n~(G)) V(G)
            with n~ = J n and V(G) = sum_a v_a(|G|) exp(-i G.tau_a) (box G, the
            operators module's model), so
            F_a = -Omega sum_G G v_a(G) Im[conj(n~(G)) exp(-i G.tau_a)]
  nonlocal  E_nl = sum_k w_k sum_i f_ki D sum_a |Pi_ai|^2, Pi = P_k^dag psi_k;
            dP_k[G,a]/dtau_a = -i G P_k[G,a] (G without k), so
            F_a = -sum_k w_k sum_i f_ki D 2 Re[conj(Pi_ai) (dP_a^dag psi_k)_i]
  ions      Ewald summation with splitting parameter eta (any eta > 0 gives
            the same energy):
            E_ion = 1/2 sum_{a,b} sum'_L Z_a Z_b erfc(eta r)/r
                    + (2 pi/Omega) sum_{G!=0} exp(-G^2/(4 eta^2))/G^2 |S(G)|^2
                    - (eta/sqrt(pi)) sum_a Z_a^2 - pi (sum_a Z_a)^2/(2 Omega eta^2)
            r = |tau_a - tau_b + L| (L = 0 omitted for a = b), S(G) = sum_a Z_a exp(i G.tau_a)
            F_a = sum_b sum'_L Z_a Z_b [erfc(eta r)/r^2 + (2 eta/sqrt(pi)) exp(-eta^2 r^2)/r] (d/r)
                  + (4 pi/Omega) Z_a sum_{G!=0} exp(-G^2/(4 eta^2))/G^2 G Im[exp(i G.tau_a) conj(S(G))]
            with d = tau_a - tau_b + L.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .basis import box_G, cell_volume, reciprocal_basis
from .transforms import J

EWALD_TOL = 36.0  # exp(-36) ~ 2e-16: both Ewald sums are cut where their terms fall below it


def local_forces(R, S, tau, Z, rc, n) -> np.ndarray:
    """(nat, 3) -dE_loc/dtau at the fixed real density n on the box."""
    omega = cell_volume(R)
    G = box_G(R, S)
    G2 = np.sum(G * G, axis=-1)
    nt = J(n)
    F = np.zeros((len(Z), 3))
    for a in range(len(Z)):
        v = np.where(G2 > 0, -4.0 * np.pi * Z[a] * np.exp(-G2 * rc[a] ** 2 / 4.0) / (omega * np.where(G2 > 0, G2, 1.0)),
                     0.0)
        c = np.conj(nt) * np.exp(-1j * (G @ tau[a]))
        F[a] = -omega * np.sum(G * (v * c.imag)[..., None], axis=(0, 1, 2))
    return F


def nonlocal_forces(bases, wk, psis, fills, tau, has_proj, rp, D) -> np.ndarray:
    """(nat, 3) -dE_nl/dtau at fixed orthonormal psi (per k: (npw, nb)) and fillings."""
    F = np.zeros((len(tau), 3))
    atoms = [a for a in range(len(tau)) if has_proj[a]]
    for k, b in enumerate(bases):
        G = b.n @ reciprocal_basis(b.R).T
        beta = np.exp(-b.kG2 * rp * rp / 2.0)
        f = np.asarray(fills[k], float)
        for a in atoms:
            p = beta * np.exp(-1j * (G @ tau[a]))
            Pi = p.conj() @ psis[k]
            for d in range(3):
                dPi = (-1j * G[:, d] * p).conj() @ psis[k]
                F[a, d] -= wk[k] * D * np.sum(f * 2.0 * np.real(np.conj(Pi) * dPi))
    return F


def ewald_eta(R, nat) -> float:
    """A splitting parameter that balances the two sums."""
    omega = cell_volume(R)
    return math.sqrt(math.pi) * (nat / omega ** 2) ** (1.0 / 6.0)


def _image_range(R, rcut):
    """Per lattice direction i, how many images along a_i reach within rcut of
    the cell: lattice planes along a_i are 2 pi / |b_i| apart."""
    B = reciprocal_basis(R)  # columns b_i with b_i . a_j = 2 pi delta_ij
    return [int(math.ceil(rcut * np.linalg.norm(B[:, i]) / (2.0 * math.pi))) + 1 for i in range(3)]


def ewald(R, tau, Z, eta=None):
    """(E_ion, F (nat, 3)) of point charges Z at tau in a compensating background."""
    R = np.asarray(R, float)
    tau = np.asarray(tau, float)
    Z = np.asarray(Z, float)
    nat = len(Z)
    omega = cell_volume(R)
    if eta is None:
        eta = ewald_eta(R, nat)
    rcut = math.sqrt(EWALD_TOL) / eta
    gcut = 2.0 * eta * math.sqrt(EWALD_TOL)
    E = 0.0
    F = np.zeros((nat, 3))
    # real space
    nr = _image_range(R, rcut)
    for n in itertools.product(*[range(-m, m + 1) for m in nr]):
        L = R @ np.array(n, float)
        for a in range(nat):
            for b in range(nat):
                if a == b and n == (0, 0, 0):
                    continue
                d = tau[a] - tau[b] + L
                r = float(np.linalg.norm(d))
                if r > rcut:
                    continue
                E += 0.5 * Z[a] * Z[b] * math.erfc(eta * r) / r
                g = math.erfc(eta * r) / r ** 2 + 2.0 * eta / math.sqrt(math.pi) * math.exp(-(eta * r) ** 2) / r
                F[a] += Z[a] * Z[b] * g * d / r
    # reciprocal space
    B = reciprocal_basis(R)
    # G = sum_i m_i b_i has m_i = G . a_i / (2 pi), so |m_i| <= gcut |a_i| / (2 pi)
    ng = [int(math.ceil(gcut * np.linalg.norm(R[:, i]) / (2.0 * math.pi))) + 1 for i in range(3)]
    for m in itertools.product(*[range(-k, k + 1) for k in ng]):
        if m == (0, 0, 0):
            continue
        G = B @ np.array(m, float)
        G2 = float(G @ G)
        if G2 > gcut * gcut:
            continue
        w = math.exp(-G2 / (4.0 * eta * eta)) / G2
        ph = np.exp(1j * (tau @ G))
        Sg = np.sum(Z * ph)
        E += 2.0 * math.pi / omega * w * abs(Sg) ** 2
        F += (4.0 * math.pi / omega) * w * (Z * np.imag(ph * np.conj(Sg)))[:, None] * G[None, :]
    # self and background terms (position independent)
    E -= eta / math.sqrt(math.pi) * float(np.sum(Z * Z))
    E -= math.pi * float(np.sum(Z)) ** 2 / (2.0 * omega * eta * eta)
    return E, F
