"""GPU parity of the Fermi-Dirac smeared SCF (dpp_system_set_smearing) with
the oracle's (oracle/scf.py, smearing=sigma).

Five SCF iterations on a sheared two-k cell with 9 electrons (an odd count,
so the highest level is partly filled) at sigma = 0.02 Ha: free energies
E - sigma S per iteration to 1e-8 Ha/atom and eigenvalues to 1e-7 Ha (the
bars of the aufbau SCF parity test), fillings to 1e-8, mu and sigma S to
1e-9.  A width of 1e-6 Ha on a cell with a gap reproduces the aufbau SCF to
the same bars.
"""
import numpy as np
import pytest

import workloads as W
from oracle import energy as oe, scf as oscf
from tests._gpu import Device, log
from tests._systems import make_gpu_system, packed_Y

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return Device()


def _cell():
    return W.tiny_cell(nat=3, L=7.0, ecut=3.5, S=(16, 15, 18), nb=6, Z=(4, 1, 4), fold=(2, 1, 2),
                       R=np.array([[7.0, 0.5, 0.0], [0.0, 6.6, 0.7], [0.4, 0.0, 7.3]]), seed=31)


def _run(dev, cell, sigma, nit):
    sysg, off, npw = make_gpu_system(dev, cell)
    if sigma is not None:
        dev.D.dpp_system_set_smearing(sysg, sigma)
    Y, blocks = packed_Y(dev, cell, npw)
    dev.D.dpp_scf_init(sysg, cell.tau, cell.Z, W.START_SIGMA)
    Eg = []
    for _ in range(nit):
        E, e = dev.D.dpp_scf_iteration(sysg, Y, len(cell.kpts), cell.nb)
        Eg.append(E["E_el"])
    fills = dev.D.dpp_system_fillings(sysg, len(cell.kpts), cell.nb)
    mu = ts = None
    if sigma:
        mu, ts = dev.D.dpp_system_smearing_state(sysg, 1)
    dev.D.dpp_system_destroy(sysg)
    return Eg, e, fills, mu, ts, blocks


def test_smeared_scf_matches_oracle(dev):
    cell = _cell()
    sig, nit = 0.02, 5
    log(f"smeared SCF sigma={sig}, N_e={cell.n_electrons}")
    Eg, e, fills, mu, ts, blocks = _run(dev, cell, sig, nit)
    s = oe.build_system(cell)
    res = oscf.scf(s, [b.T.copy() for b in blocks], oe.start_density(cell, W.START_SIGMA), nit, smearing=sig)
    log(f"gpu F {Eg}\noracle F {res['energies']}\nmu {mu[0]:.12f} / {res['mu']:.12f}, TS {ts[0]:.3e} / {res['TS']:.3e}")
    assert np.max(np.abs(np.array(Eg) - np.array(res["energies"]))) / cell.nat < 1e-8
    assert np.max(np.abs(e - np.array(res["eigs"]))) < 1e-7
    assert max(np.max(np.abs(np.asarray(fills[k]) - res["fills"][k])) for k in range(len(cell.kpts))) < 1e-8
    assert abs(mu[0] - res["mu"]) < 1e-9 and abs(ts[0] - res["TS"]) < 1e-9
    assert res["TS"] > 1e-4  # the smearing acts: fractional fillings carry entropy


def test_tiny_width_reproduces_aufbau(dev):
    cell = W.config2()
    nit = 3
    Ea, ea, _, _, _, _ = _run(dev, cell, None, nit)
    Es, es, _, mu, ts, _ = _run(dev, cell, 1e-6, nit)
    log(f"aufbau {Ea} smeared {Es} TS {ts[0]:.2e}")
    assert np.max(np.abs(np.array(Ea) - np.array(Es))) / cell.nat < 1e-8
    assert np.max(np.abs(ea - es)) < 1e-7


def test_forces_are_free_energy_derivatives_at_level_crossing(dev):
    """The two-atom cell at 3.35 bohr, inside the window where the highest
    filled and lowest empty levels cross and the aufbau SCF does not settle.
    With two empty bands (6 bands, 8 electrons) and sigma = 0.01 Ha the SCF
    converges (within 35 iterations here; the two crossing levels, 4 mHa
    apart, share two electrons), and the force on the ions equals the central
    difference of the converged free energy E - sigma S + E_ion
    (Hellmann-Feynman for the smeared functional: the fillings are
    stationary), to the difference's O(h^2) truncation."""
    sig, h, nit = 0.01, 2e-3, 80
    u = np.array([2.4, 1.5, 0.4]) / np.linalg.norm([2.4, 1.5, 0.4])
    mid = np.array([3.4, 3.35, 3.2])
    tau0 = np.stack([mid - 1.675 * u, mid + 1.675 * u])

    def cell_at(tau):
        c = W.tiny_cell(nat=2, L=7.0, ecut=4.0, S=(16, 16, 16), nb=6, Z=(4, 4), seed=11)
        c.tau = np.array(tau, float)
        return c

    def converged(tau, with_forces=False):
        c = cell_at(tau)
        sysg, off, npw = make_gpu_system(dev, c)
        dev.D.dpp_system_set_smearing(sysg, sig)
        Y, _ = packed_Y(dev, c, npw)
        dev.D.dpp_scf_init(sysg, c.tau, c.Z, W.START_SIGMA)
        Es = []
        for _ in range(nit):
            E, _ = dev.D.dpp_scf_iteration(sysg, Y, 1, c.nb)
            Es.append(E["E_el"])
        F = [dev.zeros((2, 3), dev.torch.float64) for _ in range(3)]
        Eion = dev.D.dpp_system_forces(sysg, Y, F[0], F[1], F[2], 1)[0]
        Ftot = sum(dev.host(f) for f in F)
        fills = dev.D.dpp_system_fillings(sysg, 1, c.nb)
        dev.D.dpp_system_destroy(sysg)
        assert abs(Es[-1] - Es[-2]) < 1e-11, Es[-5:]
        return Es[-1] + Eion, Ftot, fills

    E0, F0, fills = converged(tau0)
    log(f"fillings at 3.35 bohr: {fills}; F[0] {F0[0]}")
    assert np.any((fills > 1e-3) & (fills < 2 - 1e-3))  # the levels near the Fermi level share electrons
    for a, d in [(0, 0), (1, 2)]:
        tp, tm = tau0.copy(), tau0.copy()
        tp[a, d] += h
        tm[a, d] -= h
        fd = -(converged(tp)[0] - converged(tm)[0]) / (2 * h)
        log(f"atom {a} dir {d}: fd {fd:.9f} force {F0[a, d]:.9f}")
        assert abs(fd - F0[a, d]) < 2e-6
