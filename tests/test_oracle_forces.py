"""Pins of the oracle's forces on the ions (oracle/forces.py).

  * Ewald: the simple-cubic Madelung constant (tests/golden/constants.txt),
    independence of the splitting parameter (energy and forces), central
    differences of the energy, zero net force, zero forces on the ideal
    diamond lattice (inversion symmetry);
  * local and nonlocal forces: central differences of E_loc at a fixed density
    and of E_nl at fixed wavefunctions, the energies computed by the
    operators module (independent of the force formulas);
  * Hellmann-Feynman: at a converged SCF state, the central difference of the
    converged energy E_el + E_ion equals the sum of the three forces;
  * ionic minimization (oracle/relax.py): it lowers the energy and ends below
    its force tolerance.
"""
import numpy as np
import pytest

import workloads as W
from oracle import energy as oe, forces as of, operators as ops, scf as oscf
from tests._golden import constants

H = 1e-4
SKEW = np.array([[7.0, 0.5, 0.0], [0.0, 6.6, 0.7], [0.4, 0.0, 7.3]])


def _skew_cell():
    return W.tiny_cell(nat=3, L=7.0, ecut=3.5, S=(16, 15, 18), nb=6, Z=(4, 1, 4), fold=(2, 1, 1), R=SKEW, seed=31)


def _fd(fn, tau, a, d, h=H):
    tp, tm = tau.copy(), tau.copy()
    tp[a, d] += h
    tm[a, d] -= h
    return -(fn(tp) - fn(tm)) / (2 * h)


@pytest.mark.parametrize("L", [1.0, 3.7])
def test_ewald_simple_cubic_madelung(L):
    E, F = of.ewald(np.eye(3) * L, np.zeros((1, 3)), np.array([1.0]))
    assert abs(E * L + constants()["madelung_sc"] / 2) < 1e-10
    assert np.max(np.abs(F)) < 1e-12


def test_ewald_splitting_independent():
    rng = np.random.default_rng(1)
    tau = rng.uniform(0, 6, (4, 3))
    Z = np.array([1.0, 4.0, 1.0, 4.0])
    E1, F1 = of.ewald(SKEW, tau, Z, eta=0.4)
    E2, F2 = of.ewald(SKEW, tau, Z, eta=0.9)
    assert abs(E1 - E2) < 1e-10
    assert np.max(np.abs(F1 - F2)) < 1e-10
    assert np.max(np.abs(F1.sum(axis=0))) < 1e-12


def test_ewald_forces_are_energy_derivatives():
    rng = np.random.default_rng(2)
    tau = rng.uniform(0, 6, (4, 3))
    Z = np.array([1.0, 4.0, 1.0, 4.0])
    _, F = of.ewald(SKEW, tau, Z)
    for a, d in [(0, 0), (1, 2), (3, 1), (2, 0)]:
        fd = _fd(lambda t: of.ewald(SKEW, t, Z)[0], tau, a, d)
        assert abs(fd - F[a, d]) < 1e-7 * max(1.0, abs(F[a, d]))


def test_ewald_ideal_diamond_has_no_force():
    cell = W.config2()
    # the undisplaced diamond positions of the cell
    _, F = of.ewald(cell.R, cell.tau, cell.Z)
    assert np.max(np.abs(F)) < 1e-10


def test_local_forces_are_energy_derivatives():
    cell = _skew_cell()
    s = oe.build_system(cell)
    n = W.random_density(5, cell.S)
    F = of.local_forces(cell.R, cell.S, cell.tau, cell.Z, cell.rc, n)
    dV = s.omega / s.N

    def Eloc(tau):
        return dV * np.sum(n * ops.local_potential(cell.R, cell.S, tau, cell.Z, cell.rc))

    for a, d in [(0, 0), (1, 1), (2, 2), (0, 2)]:
        assert abs(_fd(Eloc, cell.tau, a, d) - F[a, d]) < 1e-8


def test_nonlocal_forces_are_energy_derivatives():
    cell = _skew_cell()
    s = oe.build_system(cell)
    rng = np.random.default_rng(3)
    psis, fills = [], []
    for b in s.bases:
        Y = rng.standard_normal((b.npw, cell.nb)) + 1j * rng.standard_normal((b.npw, cell.nb))
        psis.append(ops.cholesky_orthonormalize(Y, b)[0])
        fills.append(rng.uniform(0, 2, cell.nb))
    F = of.nonlocal_forces(s.bases, s.wk, psis, fills, cell.tau, cell.has_proj, W.PROJ_RP, W.PROJ_D)

    def Enl(tau):
        E = 0.0
        for k, b in enumerate(s.bases):
            Pi = ops.projectors(b, tau, cell.has_proj, W.PROJ_RP).conj().T @ psis[k]
            E += s.wk[k] * W.PROJ_D * np.sum(fills[k] * np.sum(np.abs(Pi) ** 2, axis=0))
        return E

    assert np.all(F[~cell.has_proj] == 0.0)
    for a, d in [(0, 0), (2, 1), (0, 2), (2, 2)]:
        assert abs(_fd(Enl, cell.tau, a, d) - F[a, d]) < 1e-9


# two Z = 4 atoms (local and nonlocal parts) 3 bohr apart: protocol S
# converges in ~40 iterations, and every band is filled
HF_TAU = np.array([[2.2, 2.6, 3.0], [4.6, 4.1, 3.4]])


def _hf_cell(tau):
    c = W.tiny_cell(nat=2, L=7.0, ecut=4.0, S=(16, 16, 16), nb=4, Z=(4, 4), seed=11)
    c.tau = tau.copy()
    return c


def _converged(cell):
    s = oe.build_system(cell)
    blocks = W.initial_wavefunctions(cell.y0_seed, [(cell.nb, b.npw) for b in s.bases])
    res = oscf.scf(s, [b.T.copy() for b in blocks], oe.start_density(cell, W.START_SIGMA), 150, n_inner=4,
                   etol_per_atom=1e-13)
    assert abs(res["energies"][-1] - res["energies"][-2]) < 1e-12
    return s, res


def oracle_forces(s, cell, res):
    """Local + nonlocal + Ewald at the SCF state res (psi, fillings, n_out)."""
    fills = oscf.aufbau_fillings(res["eigs"], s.wk, s.n_electrons)
    Fl = of.local_forces(cell.R, cell.S, cell.tau, cell.Z, cell.rc, res["n_out"])
    Fn = of.nonlocal_forces(s.bases, s.wk, res["Y"], fills, cell.tau, cell.has_proj, W.PROJ_RP, W.PROJ_D)
    Fi = of.ewald(cell.R, cell.tau, cell.Z)[1]
    return Fl, Fn, Fi


def test_hellmann_feynman_at_convergence():
    cell = _hf_cell(HF_TAU)
    s, res = _converged(cell)
    Fl, Fn, Fi = oracle_forces(s, cell, res)
    F = Fl + Fn + Fi
    assert np.max(np.abs(Fn)) > 1e-3  # every part matters at this geometry
    h = 2e-3

    def E(tau):
        c = _hf_cell(tau)
        _, r = _converged(c)
        return r["energies"][-1] + of.ewald(c.R, c.tau, c.Z)[0]

    for a, d in [(0, 0), (1, 2)]:
        # O(h^2) truncation of the central difference is ~1e-6 here
        assert abs(_fd(E, HF_TAU, a, d, h) - F[a, d]) < 2e-6


# a stretched bond (4.0 bohr) that contracts to the minimum near 3.64 bohr;
# along this path the highest filled and lowest empty levels stay apart, so
# every aufbau SCF converges (between 3.2 and 3.5 bohr they cross, and SCF
# without smearing does not converge)
RELAX_TAU = np.array([[1.748, 4.171, 3.9308], [5.042, 2.519, 2.5392]])


def test_relaxation_reaches_force_tolerance():
    """The oracle's ionic minimization lowers the energy and ends below the
    force tolerance (the trajectory the GPU relaxation is compared with)."""
    from oracle import relax as orx
    cell = _hf_cell(RELAX_TAU)
    r = orx.relax(orx.energy_forces(cell), RELAX_TAU, ftol=1e-3, max_steps=30)
    E = [h[0] for h in r["history"]]
    assert E[-1] < E[0] - 0.02
    # at the end every force component is below the tolerance, the energy is
    # the lowest of the trajectory, and the bond is at the minimum
    assert np.max(np.abs(r["F"])) < 1e-3
    assert E[-1] <= min(E) + 1e-9
    assert abs(np.linalg.norm(r["tau"][0] - r["tau"][1]) - 3.643) < 0.01
