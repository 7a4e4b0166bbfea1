"""Pins for the local pseudopotential, projectors, Hartree solve and start
density against closed forms, quadrature and an independent Ewald sum."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from oracle import basis, energy, operators as ops
from tests._golden import constants


def ewald_madelung_sc(eta=0.6, nr=6, ng=8):
    """alpha for a point charge in a unit simple-cubic cell with background."""
    L = 1.0
    s_real = 0.0
    for i in range(-nr, nr + 1):
        for j in range(-nr, nr + 1):
            for k in range(-nr, nr + 1):
                if i == j == k == 0:
                    continue
                t = math.sqrt(i * i + j * j + k * k)
                s_real += math.erfc(eta * t * 6) / t
    e = eta * 6
    s_rec = 0.0
    for i in range(-ng, ng + 1):
        for j in range(-ng, ng + 1):
            for k in range(-ng, ng + 1):
                if i == j == k == 0:
                    continue
                g2 = (2 * math.pi) ** 2 * (i * i + j * j + k * k)
                s_rec += math.exp(-g2 / (4 * e * e)) / g2
    E = 0.5 * (s_real + 4 * math.pi * s_rec - 2 * e / math.sqrt(math.pi) - math.pi / (e * e))
    return -2.0 * E * L


def test_madelung_constant_from_ewald():
    alpha = ewald_madelung_sc()
    assert abs(alpha - constants()["madelung_sc"]) < 1e-10


def test_erf_potential_is_radial_fourier_transform():
    L = 9.0
    R = np.eye(3) * L
    S = (12, 12, 12)
    rc = 0.5
    Vt = ops.local_potential_G(R, S, np.zeros((1, 3)), np.array([1.0]), np.array([rc]))
    G = basis.box_G(R, S)
    omega = L ** 3
    for idx in [(1, 0, 0), (2, 1, 0), (3, 2, 1), (5, 5, 4)]:
        g = float(np.linalg.norm(G[idx]))
        # FT of -erf(r/rc)/r = -4 pi / G^2 + FT of erfc(r/rc)/r (short ranged)
        short, _ = integrate.quad(lambda r: special.erfc(r / rc) * math.sin(g * r), 0, 30 * rc, limit=400)
        ft = -4 * math.pi / g ** 2 + 4 * math.pi / g * short
        assert abs(omega * Vt[idx] - ft) < 1e-9 * abs(ft)
    assert Vt[0, 0, 0] == 0.0


def _gaussian_on_grid(R, S, centres, width, charges, images=2):
    L = R[0, 0]
    j = np.stack(np.meshgrid(*[np.arange(s) / s for s in S], indexing="ij"), -1)
    r = j @ R.T
    out = np.zeros(S)
    for c, q in zip(centres, charges):
        for t in np.ndindex(2 * images + 1, 2 * images + 1, 2 * images + 1):
            shift = (np.array(t) - images) * L
            d2 = np.sum((r - c - shift) ** 2, axis=-1)
            out += q * (math.pi * width ** 2) ** -1.5 * np.exp(-d2 / width ** 2)
    return out


def test_hartree_gaussian_closed_form():
    L, Q, sigma = 10.0, 2.0, 1.0
    R = np.eye(3) * L
    S = (48, 48, 48)
    n = _gaussian_on_grid(R, S, [np.array([3.1, 4.2, 5.3])], sigma, [Q])
    VH, EH = energy.hartree(n, R)
    alpha = constants()["madelung_sc"]
    exact = Q * Q / (sigma * math.sqrt(2 * math.pi)) - 0.5 * Q * Q * alpha / L + math.pi * Q * Q * sigma ** 2 / L ** 3
    assert abs(EH - exact) < 1e-8
    # E_H = (1/2) integral n V_H
    assert abs(0.5 * L ** 3 / n.size * np.sum(n * VH) - EH) < 1e-10


def test_local_potential_is_potential_of_ionic_gaussians():
    L = 8.0
    R = np.eye(3) * L
    S = (48, 48, 48)
    tau = np.array([[1.0, 2.0, 3.0], [5.5, 4.0, 6.5]])
    Z = np.array([1.0, 4.0])
    rc = np.array([0.8, 0.9])
    V = ops.local_potential(R, S, tau, Z, rc)
    rho = np.zeros(S)
    for a in range(2):
        rho += _gaussian_on_grid(R, S, [tau[a]], rc[a], [-Z[a]])
    VH, _ = energy.hartree(rho, R)
    assert np.max(np.abs(V - VH)) < 1e-8 * np.max(np.abs(V))


def test_projector_is_overlap_with_gaussian():
    # <p_a | exp(i (k+G).r)> over all space by quadrature on a fine grid
    R = np.eye(3) * 7.0
    b = basis.gsphere(R, (20, 20, 20), np.array([0.5, 0.0, 0.5]), 3.0)
    tau = np.array([[1.3, -0.4, 2.2]])
    rp = 1.0
    P = ops.projectors(b, tau, [True], rp)
    x = np.linspace(-7, 7, 141)
    h = x[1] - x[0]
    X, Y, Zc = np.meshgrid(x, x, x, indexing="ij")
    p = (2 * math.pi * rp * rp) ** -1.5 * np.exp(-(X ** 2 + Y ** 2 + Zc ** 2) / (2 * rp * rp))
    for g in [0, 7, b.npw // 2, b.npw - 1]:
        q = b.kG[g]
        integrand = p * np.exp(1j * (q[0] * (X + tau[0, 0]) + q[1] * (Y + tau[0, 1]) + q[2] * (Zc + tau[0, 2])))
        val = integrand.sum() * h ** 3
        kcart = q - b.n[g] @ basis.reciprocal_basis(R).T
        # oracle drops exp(i k.tau): <p|psi> = conj(P) * exp(i k.tau)
        ref = np.conj(P[g, 0]) * np.exp(1j * kcart @ tau[0])
        assert abs(val - ref) < 1e-8


def test_start_density_normalized_and_gaussian():
    cell = W.tiny_cell(nat=2, L=8.0, S=(40, 40, 40), Z=(1, 4))
    n0 = energy.start_density(cell, 1.0)
    omega = 8.0 ** 3
    assert abs(omega / n0.size * n0.sum() - 5.0) < 1e-10
    ref = _gaussian_on_grid(cell.R, cell.S, cell.tau, 1.0, cell.Z)
    assert np.max(np.abs(n0 - ref)) < 1e-9
