"""Pins for protocol V (variational minimization), its gradient, protocol S
(SCF with Pulay mixing) and the fillings: finite differences, monotone
descent, the jellium closed form and SCF fixed point = variational minimum."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, energy, minimize, operators as ops, scf, xc


def _system(nat=2, Z=(1, 1), fold=(1, 1, 1), L=6.0, ecut=3.0, S=(12, 12, 12), seed=7):
    cell = W.tiny_cell(nat=nat, L=L, ecut=ecut, S=S, nb=2, Z=Z, fold=fold, seed=seed)
    return cell, energy.build_system(cell)


def _random_Y(sys, nb, seed):
    shapes = [(nb, b.npw) for b in sys.bases]
    return [y.T.copy() for y in W.initial_wavefunctions(seed, shapes)]


def test_gradient_matches_finite_differences():
    cell, sys = _system(Z=(4, 1), fold=(2, 1, 1))
    Y = _random_Y(sys, 2, 5)
    f = 1.25
    E, g = energy.energy_and_gradient(Y, f, sys)
    rng = np.random.default_rng(6)
    Dl = [rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape) for y in Y]
    h = 1e-5
    fills = [np.full(2, f)] * len(Y)
    Ep = energy.total_energy(minimize.axpy(Y, h, Dl), fills, sys)
    Em = energy.total_energy(minimize.axpy(Y, -h, Dl), fills, sys)
    fd = (Ep - Em) / (2 * h)
    an = minimize.dot(g, Dl)
    assert abs(fd - an) < 1e-6 * abs(an)


def test_gradient_vanishes_on_rotations():
    # E is invariant under Y -> Y M, so the gradient is O-orthogonal to span(Y)
    cell, sys = _system(Z=(4, 4))
    Y = _random_Y(sys, 2, 9)
    E, g = energy.energy_and_gradient(Y, 2.0, sys)
    for y, gk, b in zip(Y, g, sys.bases):
        assert np.max(np.abs(y.conj().T @ gk)) < 1e-12 * np.max(np.abs(gk)) * b.npw


def test_protocol_V_descends_monotonically():
    cell, sys = _system(Z=(4, 1), fold=(1, 1, 2))
    Y = _random_Y(sys, 2, 12)
    cg = minimize.protocol_V(Y, sys, 2.0, 25)
    h = np.array(cg.history)
    assert len(h) >= 20
    assert np.all(np.diff(h) <= 1e-12 * np.abs(h[:-1]))
    # the gradient has fallen by orders of magnitude
    Y0 = [ops.cholesky_orthonormalize(y, b)[0] for y, b in zip(Y, sys.bases)]
    g0 = energy.energy_and_gradient(Y0, 2.0, sys)[1]
    assert minimize.dot(cg.g, cg.g) < 1e-6 * minimize.dot(g0, g0)


def test_jellium_closed_form():
    # no atoms: uniform density, E = E_kin + Omega n eps_xc(n), eps_i = |G_i|^2/2 + v_xc(n)
    L = 6.0
    cell = W.tiny_cell(nat=2, L=L, ecut=3.0, S=(12, 12, 12), nb=8, Z=(0, 0))
    sys = energy.build_system(cell, with_local=False, with_projectors=False)
    sys.n_electrons = 14
    Y = _random_Y(sys, 8, 3)
    nbar = 14.0 / L ** 3
    res = scf.scf(sys, Y, np.full(cell.S, nbar), n_iter=10, n_inner=15)
    eps_xc, v_xc = xc.lda_pz81(np.array([nbar]))
    g1 = 2 * math.pi / L
    Ekin = 2 * 6 * 0.5 * g1 ** 2
    Eref = Ekin + L ** 3 * nbar * eps_xc[0]
    assert abs(res["energies"][-1] - Eref) < 1e-9
    assert np.max(np.abs(res["n_out"] - nbar)) < 1e-6 * nbar
    eig = res["eigs"][0]
    ref = np.array([0.0] + [0.5 * g1 ** 2] * 6 + [g1 ** 2]) + v_xc[0]
    assert np.max(np.abs(eig[:7] - ref[:7])) < 1e-7
    assert abs(eig[7] - ref[7]) < 1e-7


def test_scf_fixed_point_equals_variational_minimum():
    cell, sys = _system(Z=(4, 4), L=6.5, ecut=3.0, S=(15, 15, 15), seed=21)
    nb = 4
    Y = _random_Y(sys, nb, 22)
    cgv = minimize.protocol_V(Y, sys, 2.0, 120)
    Ev = cgv.E
    n0 = energy.start_density(cell, W.START_SIGMA)
    res = scf.scf(sys, Y, n0, n_iter=40, n_inner=3, etol_per_atom=1e-12)
    Es = res["energies"][-1]
    assert abs(Ev - Es) / sys.nat < 1e-8
    # variational principle: every SCF output energy lies above the minimum
    assert min(res["energies"]) >= Ev - 1e-9


def test_aufbau_fillings():
    eigs = [np.array([0.0, 1.0, 2.0]), np.array([0.5, 1.0 + 1e-8, 3.0])]
    f = scf.aufbau_fillings(eigs, np.array([0.5, 0.5]), 3.0)
    # states 0.0 and 0.5 hold 1 electron each (2 w_k); the degenerate pair at 1.0 shares 1
    assert np.allclose(f[0], [2.0, 1.0, 0.0]) and np.allclose(f[1], [2.0, 1.0, 0.0])
    f = scf.aufbau_fillings([np.array([-1.0, 0.2, 0.4])], np.array([1.0]), 3.0)
    assert np.allclose(f[0], [2.0, 1.0, 0.0])
    with pytest.raises(ValueError):
        scf.aufbau_fillings([np.array([0.0])], np.array([1.0]), 4.0)
