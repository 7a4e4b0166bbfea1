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
truncation.
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
