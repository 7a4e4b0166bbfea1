"""Pins of the LinearPCM oracle (oracle/pcm.py), on the CPU.

  * uniform eps = c: the solve gives phi~ = 4 pi rho~ / (c |G'|^2) on every
    solved mode, and on a grid without Nyquist modes A_diel = (1/c - 1) E_H(rho)
    with E_H from the oracle's Hartree solve (oracle/energy.py), a separate code path;
    c = 1 gives A_diel = 0;
  * a direct dense solve: on a 5 x 6 x 7 box the operator, assembled column
    by column on real-space delta fields, is solved by least squares and
    matches the CG solution;
  * a layered dielectric eps(z) with rho(z): the 1D continuum solution by
    quadrature, eps phi' = -4 pi Q + C with C fixed by periodicity, gives phi
    and A_diel, which the spectral solve reproduces at a fine grid;
  * the operator is symmetric and positive on real fields, and A_diel < 0 for
    a non-uniform eps >= 1 (screening lowers the electrostatic energy).
"""
import numpy as np
import pytest

import workloads as W
from oracle import energy as oe, pcm


def _random_real_field(rng, S):
    return rng.standard_normal(S)


@pytest.mark.parametrize("S,c", [((12, 13, 14), 4.0), ((9, 11, 13), 78.4)])
def test_uniform_eps_closed_form(S, c):
    R = np.array([[9.0, 0.4, 0.0], [0.0, 8.5, 0.3], [0.2, 0.0, 9.4]])
    rng = np.random.default_rng(3)
    rho = _random_real_field(rng, S)
    eps = np.full(S, c)
    phit, it, rel = pcm.solve(R, S, eps, rho, tol=1e-13)
    assert rel <= 1e-13
    Gp = pcm.spectral_G(R, S)
    G2p = np.sum(Gp * Gp, axis=-1)
    mask = G2p > 0
    expect = np.zeros_like(phit)
    expect[mask] = 4 * np.pi * pcm.J(rho)[mask] / (c * G2p[mask])
    assert np.max(np.abs(phit - expect)) < 1e-12 * np.max(np.abs(expect))
    if all(s % 2 for s in S):  # no Nyquist modes: G' = G
        A = pcm.a_diel(R, S, phit, rho)
        EH = oe.hartree(rho, R)[1]
        assert abs(A - (1.0 / c - 1.0) * EH) < 1e-11 * abs(EH)
        phi1, _, _ = pcm.solve(R, S, np.ones(S), rho, tol=1e-13)
        assert abs(pcm.a_diel(R, S, phi1, rho)) < 1e-12 * abs(EH)


def test_dense_direct_solve():
    S = (5, 6, 7)
    R = np.array([[6.0, 0.3, 0.0], [0.1, 6.5, 0.0], [0.0, 0.2, 7.0]])
    rng = np.random.default_rng(5)
    eps = 1.0 + 20.0 * rng.uniform(0, 1, S)
    rho = _random_real_field(rng, S)
    Gp = pcm.spectral_G(R, S)
    mask = pcm.solved_modes(R, S)
    N = int(np.prod(S))
    # the operator on real fields, in real space: columns from delta fields
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        h = np.where(mask, pcm.hessian(np.where(mask, pcm.J(e.reshape(S)), 0.0), eps, Gp), 0.0)
        A[:, j] = np.real(pcm.I(h)).reshape(-1)
    b = np.real(pcm.I(np.where(mask, pcm.J(rho), 0.0))).reshape(-1)
    x = np.linalg.lstsq(A, b, rcond=1e-12)[0]
    # project out the null space (modes outside the solve) before comparing
    xd = np.real(pcm.I(np.where(mask, pcm.J(x.reshape(S)), 0.0)))
    phit, it, rel = pcm.solve(R, S, eps, rho, tol=1e-13, max_iter=2000)
    assert rel <= 1e-13
    phi = np.real(pcm.I(phit))
    assert np.max(np.abs(phi - xd)) < 1e-9 * np.max(np.abs(xd))


def _layered(M, L=10.0):
    z = np.arange(M) * L / M
    k = 2 * np.pi / L
    rho = np.cos(k * z) + 0.6 * np.sin(2 * k * z + 0.3) - 0.25 * np.cos(3 * k * z)
    eps = 1.0 + 30.0 * np.exp(-2.0 * (1 + np.cos(k * z - 0.7)))
    return z, rho, eps


def _continuum_1d(L, area, fine=4000):
    """phi and A_diel of the layered case by quadrature (trapezoid on a fine periodic grid)."""
    z, rho, eps = _layered(fine, L)
    dz = L / fine
    # Q(z) = int_0^z rho (rho has zero mean); exact for the trigonometric rho
    k = 2 * np.pi / L
    Q = (np.sin(k * z) / k - 0.6 * (np.cos(2 * k * z + 0.3) - np.cos(0.3)) / (2 * k)
         - 0.25 * np.sin(3 * k * z) / (3 * k))
    C = 4 * np.pi * np.sum(Q / eps) / np.sum(1.0 / eps)
    dphi = (-4 * np.pi * Q + C) / eps
    C0 = 4 * np.pi * np.mean(Q)
    dphi0 = -4 * np.pi * Q + C0
    # A_diel = (1/2) int (phi - phi0) rho = -(1/2) int (phi - phi0)' Q (by parts, periodic)
    return -0.5 * area * np.sum((dphi - dphi0) * Q) * dz


@pytest.mark.parametrize("M", [45, 61])
def test_layered_dielectric_matches_continuum(M):
    L, Lxy = 10.0, 3.0
    R = np.diag([Lxy, Lxy, L])
    S = (3, 3, M)
    _, rho1, eps1 = _layered(M, L)
    rho = np.broadcast_to(rho1, S).copy()
    eps = np.broadcast_to(eps1, S).copy()
    A, phi, it, rel = pcm.get_adiel(R, S, eps, rho, tol=1e-13, max_iter=3000)
    assert rel <= 1e-13
    Aref = _continuum_1d(L, Lxy * Lxy)
    # spectral accuracy of eps * dphi/dz on M points
    assert abs(A - Aref) < 1e-7 * abs(Aref), (A, Aref)
    assert Aref < 0


def test_operator_symmetric_positive_and_sign_of_adiel():
    c = W.pcm_case("small")
    R, S, eps, rho = c["R"], c["S"], c["eps"], c["rho"]
    Gp = pcm.spectral_G(R, S)
    mask = pcm.solved_modes(R, S)
    rng = np.random.default_rng(9)
    a = np.where(mask, pcm.J(rng.standard_normal(S)), 0.0)
    b = np.where(mask, pcm.J(rng.standard_normal(S)), 0.0)
    Ha = np.where(mask, pcm.hessian(a, eps, Gp), 0.0)
    Hb = np.where(mask, pcm.hessian(b, eps, Gp), 0.0)
    assert abs(pcm.dot(a, Hb) - pcm.dot(Ha, b)) < 1e-12 * abs(pcm.dot(a, Hb))
    assert pcm.dot(a, Ha) > 0 and pcm.dot(b, Hb) > 0
    A, phi, it, rel = pcm.get_adiel(R, S, eps, rho, tol=1e-11)
    assert rel <= 1e-11 and A < 0
