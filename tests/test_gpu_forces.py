"""GPU parity of the forces on the ions (dpp_system_forces) with the oracle.

After SCF iterations on the GPU, the oracle (oracle/forces.py) evaluates the
local, nonlocal and Ewald forces from the GPU's own state: its orthonormal
wavefunctions, fillings and output density, so both sides see the same
inputs and the bar is FP64 rounding (1e-9 hartree/bohr on forces of order
0.01-1, 1e-9 hartree on the ionic energy).  Cases: two projector atoms in a
cubic box; three atoms with two k-points in a skewed cell; config 3 (64
atoms, 90^3, 128 bands) itself.  Then, end to end on the GPU alone: at a
converged SCF state the summed force equals the central difference of the
converged energy E_el + E_ion (Hellmann-Feynman), to the difference's O(h^2)
truncation.  Moving the ions in place (dpp_system_set_positions) gives the
forces of a system created at the new positions, and the ionic minimization
driven through the library (paper_1708_03621_amd/relax.py) follows the
oracle's (oracle/relax.py) step by step.
"""
import numpy as np
import pytest

import workloads as W
from oracle import energy as oe, forces as of
from tests._gpu import Device, log
from tests._systems import make_gpu_system, packed_Y, unpack

pytestmark = pytest.mark.gpu
TOL_F = 1e-9
TOL_E = 1e-9
HF_TAU = np.array([[2.2, 2.6, 3.0], [4.6, 4.1, 3.4]])
SKEW = np.array([[7.0, 0.5, 0.0], [0.0, 6.6, 0.7], [0.4, 0.0, 7.3]])


@pytest.fixture(scope="module")
def dev():
    return Device()


def _hf_cell(tau=HF_TAU):
    c = W.tiny_cell(nat=2, L=7.0, ecut=4.0, S=(16, 16, 16), nb=4, Z=(4, 4), seed=11)
    c.tau = np.array(tau, float)
    return c


def _skew_cell():
    return W.tiny_cell(nat=3, L=7.0, ecut=3.5, S=(16, 15, 18), nb=6, Z=(4, 1, 4), fold=(2, 1, 1), R=SKEW, seed=31)


def _run(dev, cell, nit):
    sysg, off, npw = make_gpu_system(dev, cell)
    Y, _ = packed_Y(dev, cell, npw)
    dev.D.dpp_scf_init(sysg, cell.tau, cell.Z, W.START_SIGMA)
    E = None
    for _ in range(nit):
        E, _ = dev.D.dpp_scf_iteration(sysg, Y, len(cell.kpts), cell.nb)
    return sysg, Y, off, npw, E["E_el"]


def _gpu_forces(dev, sysg, Y, nat):
    F = [dev.zeros((nat, 3), dev.torch.float64) for _ in range(3)]
    Eion = dev.D.dpp_system_forces(sysg, Y, F[0], F[1], F[2], 1)
    return [dev.host(f) for f in F], Eion[0]


@pytest.mark.parametrize("name,nit", [("hf", 3), ("skew", 3), ("config3", 2)])
def test_forces_match_oracle_at_gpu_state(dev, name, nit):
    cell = {"hf": _hf_cell, "skew": _skew_cell, "config3": W.config3}[name]()
    log(f"forces {name} after {nit} SCF iterations")
    sysg, Y, off, npw, _ = _run(dev, cell, nit)
    (Fl, Fn, Fi), Eion = _gpu_forces(dev, sysg, Y, cell.nat)
    # the GPU state, handed to the oracle
    psis = [b.T.copy() for b in unpack(dev, Y, cell, off, npw)]
    fills = dev.D.dpp_system_fillings(sysg, len(cell.kpts), cell.nb)
    nout = dev.field(sysg, dev.D.DPP_FIELD_NOUT, cell.S)
    dev.D.dpp_system_destroy(sysg)
    s = oe.build_system(cell)
    ol = of.local_forces(cell.R, cell.S, cell.tau, cell.Z, cell.rc, nout)
    on = of.nonlocal_forces(s.bases, s.wk, psis, fills, cell.tau, cell.has_proj, W.PROJ_RP, W.PROJ_D)
    oE, oi = of.ewald(cell.R, cell.tau, cell.Z)
    for label, g, o in [("local", Fl, ol), ("nonlocal", Fn, on), ("ions", Fi, oi)]:
        d = np.max(np.abs(g - o))
        log(f"{label}: max |F| {np.max(np.abs(o)):.3e}, max |dF| {d:.2e}")
        assert d < TOL_F
    log(f"E_ion gpu {Eion:.12f} oracle {oE:.12f}")
    assert abs(Eion - oE) < TOL_E


def test_forces_are_converged_energy_derivatives(dev):
    """Hellmann-Feynman on the GPU alone: converged SCF (FP64) at the
    geometry and at +-h along two coordinates."""
    nit = 120

    def converged_E(tau):
        c = _hf_cell(tau)
        sysg, Y, _, _, Eel = _run(dev, c, nit)
        _, Eion = _gpu_forces(dev, sysg, Y, c.nat)
        res, _, _ = dev.D.dpp_scf_status(sysg)
        dev.D.dpp_system_destroy(sysg)
        return Eel + Eion, res

    cell = _hf_cell()
    sysg, Y, _, _, _ = _run(dev, cell, nit)
    (Fl, Fn, Fi), _ = _gpu_forces(dev, sysg, Y, cell.nat)
    res, _, _ = dev.D.dpp_scf_status(sysg)
    dev.D.dpp_system_destroy(sysg)
    F = Fl + Fn + Fi
    log(f"converged band residual {res:.1e}; F[0] {F[0]}")
    h = 2e-3
    for a, d in [(0, 0), (1, 2)]:
        tp, tm = HF_TAU.copy(), HF_TAU.copy()
        tp[a, d] += h
        tm[a, d] -= h
        Ep, rp = converged_E(tp)
        Em, rm = converged_E(tm)
        fd = -(Ep - Em) / (2 * h)
        log(f"atom {a} dir {d}: fd {fd:.9f} force {F[a, d]:.9f} (residuals {rp:.1e} {rm:.1e})")
        assert abs(fd - F[a, d]) < 2e-6


def test_set_positions_equals_fresh_system(dev):
    moved = HF_TAU + np.array([[0.13, -0.07, 0.05], [-0.02, 0.11, -0.09]])
    cell = _hf_cell()
    sysg, off, npw = make_gpu_system(dev, cell)
    Y, _ = packed_Y(dev, cell, npw)
    dev.D.dpp_scf_init(sysg, cell.tau, cell.Z, W.START_SIGMA)
    dev.D.dpp_scf_iteration(sysg, Y, 1, cell.nb)
    _gpu_forces(dev, sysg, Y, cell.nat)  # force tables built at the old positions
    dev.D.dpp_system_set_positions(sysg, moved)
    Y2, _ = packed_Y(dev, cell, npw)  # same seeded start as the fresh system
    dev.D.dpp_scf_init(sysg, moved, cell.Z, W.START_SIGMA)
    for _ in range(3):
        E1, _ = dev.D.dpp_scf_iteration(sysg, Y2, 1, cell.nb)
    F1, Ei1 = _gpu_forces(dev, sysg, Y2, cell.nat)
    dev.D.dpp_system_destroy(sysg)
    fresh = _hf_cell(moved)
    sys2, Y3, _, _, E2 = _run(dev, fresh, 3)
    F2, Ei2 = _gpu_forces(dev, sys2, Y3, fresh.nat)
    dev.D.dpp_system_destroy(sys2)
    log(f"moved in place {E1['E_el']:.12f} fresh {E2:.12f}")
    assert abs(E1["E_el"] - E2) < 1e-11
    assert abs(Ei1 - Ei2) < 1e-11
    for a, b in zip(F1, F2):
        assert np.max(np.abs(a - b)) < 1e-11


# a stretched bond contracting to its minimum (3.64 bohr) through geometries
# where every aufbau SCF converges (see tests/test_oracle_forces.py)
RELAX_TAU = np.array([[1.748, 4.171, 3.9308], [5.042, 2.519, 2.5392]])


def test_relaxation_matches_oracle(dev):
    from oracle import relax as orx
    from paper_1708_03621_amd import relax as grx
    cell = _hf_cell(RELAX_TAU)
    g = grx.GpuCell(dev.D, dev.torch, dev.ctx, cell)
    rg = grx.relax(g.energy_forces, RELAX_TAU, ftol=1e-3, max_steps=30)
    log(f"gpu: {len(rg['history'])} steps, SCF iterations {g.scf_iterations}")
    g.close()
    ro = orx.relax(orx.energy_forces(cell), RELAX_TAU, ftol=1e-3, max_steps=30)
    for k, (a, b) in enumerate(zip(rg["history"], ro["history"])):
        log(f"step {k}: E gpu {a[0]:.10f} oracle {b[0]:.10f}  max|F| {a[1]:.2e} {b[1]:.2e}")
    # Each SCF stops when one energy change falls below 1e-12 Ha/atom, which
    # leaves a density error of order sqrt(1e-11) ~ 3e-6; the forces carry it
    # at first order, so the next positions differ by ~1e-5 bohr and the step
    # energies by ~5e-7 Ha (forces ~0.05 Ha/bohr): bar 1e-6 Ha/atom.  At the
    # end both are at the minimum, within the force tolerance: positions to
    # 2e-3 bohr.
    assert len(rg["history"]) == len(ro["history"])
    Eg = np.array([h[0] for h in rg["history"]])
    Eo = np.array([h[0] for h in ro["history"]])
    assert np.max(np.abs(Eg - Eo)) / cell.nat < 1e-6
    log(f"final positions differ by {np.max(np.abs(rg['tau'] - ro['tau'])):.2e} bohr")
    assert np.max(np.abs(rg["tau"] - ro["tau"])) < 2e-3
    assert rg["history"][-1][1] < 1e-3
