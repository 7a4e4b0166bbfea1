"""Pins of the Fermi-Dirac fillings (oracle/scf.py fermi_fillings), on the CPU.

  * electron count: sum_k w_k sum_i f_ki = N_e to rounding;
  * two levels holding two electrons: mu is their mean by symmetry, and the
    fillings and entropy have closed forms;
  * small width with a gap: the fillings equal the aufbau fillings;
  * Mermin's variational property: at fixed levels the fillings minimize
    sum w f eps - sigma S(f) over fillings with the same electron count (the
    first-order change vanishes, the second-order change is positive).
"""
import numpy as np

from oracle import scf as oscf


def _entropy(fills, wk):
    S = 0.0
    for k, f in enumerate(fills):
        g = np.clip(np.asarray(f) / 2.0, 1e-300, 1 - 1e-16)
        S -= 2.0 * wk[k] * float(np.sum(g * np.log(g) + (1 - g) * np.log(1 - g)))
    return S


def test_electron_count():
    rng = np.random.default_rng(3)
    eigs = [np.sort(rng.uniform(-0.5, 0.5, 9)) for _ in range(4)]
    wk = np.array([0.1, 0.2, 0.3, 0.4])
    for ne in (3.0, 7.3, 11.0):
        f, mu, S = oscf.fermi_fillings(eigs, wk, ne, 0.02)
        assert abs(sum(float(np.sum(wk[k] * f[k])) for k in range(4)) - ne) < 1e-12


def test_two_levels_closed_form():
    e1, e2, sig = -0.3, 0.1, 0.05
    f, mu, S = oscf.fermi_fillings([np.array([e1, e2])], np.array([1.0]), 2.0, sig)
    assert abs(mu - 0.5 * (e1 + e2)) < 1e-14
    g1 = 1.0 / (1.0 + np.exp((e1 - e2) / (2 * sig)))
    assert abs(f[0][0] - 2 * g1) < 1e-14 and abs(f[0][1] - 2 * (1 - g1)) < 1e-14
    Sref = -2 * 2 * (g1 * np.log(g1) + (1 - g1) * np.log(1 - g1))
    assert abs(S - Sref) < 1e-13


def test_small_width_equals_aufbau():
    eigs = [np.array([-0.4, -0.2, 0.1, 0.3]), np.array([-0.35, -0.15, 0.12, 0.4])]
    wk = np.array([0.5, 0.5])
    f, mu, S = oscf.fermi_fillings(eigs, wk, 4.0, 1e-4)
    fa = oscf.aufbau_fillings(eigs, wk, 4.0)
    assert max(np.max(np.abs(a - b)) for a, b in zip(f, fa)) < 1e-12
    assert -0.15 < mu < 0.1 and S < 1e-100 + 1e-12


def test_fillings_minimize_free_energy_at_fixed_levels():
    rng = np.random.default_rng(8)
    eigs = [np.sort(rng.uniform(-0.3, 0.3, 7)) for _ in range(3)]
    wk = np.array([0.25, 0.25, 0.5])
    sig, ne = 0.03, 6.5
    f, mu, S = oscf.fermi_fillings(eigs, wk, ne, sig)
    assert abs(S - _entropy(f, wk)) < 1e-12

    def F(fl):
        return sum(float(np.sum(wk[k] * fl[k] * eigs[k])) for k in range(3)) - sig * _entropy(fl, wk)

    # a direction that keeps every occupation inside (0, 1) for small steps
    # (scaled by g (1 - g)) and keeps the electron count
    g = [fk / 2.0 for fk in f]
    r = [rng.standard_normal(7) for _ in range(3)]
    wgt = [wk[k] * g[k] * (1 - g[k]) for k in range(3)]
    c = sum(float(np.sum(wgt[k] * r[k])) for k in range(3)) / sum(float(np.sum(wgt[k])) for k in range(3))
    d = [2.0 * g[k] * (1 - g[k]) * (r[k] - c) for k in range(3)]
    h = 1e-4
    Fp = F([f[k] + h * d[k] for k in range(3)])
    Fm = F([f[k] - h * d[k] for k in range(3)])
    F0 = F(f)
    assert abs(Fp - Fm) / (2 * h) < 1e-8  # stationary
    assert Fp > F0 and Fm > F0             # a minimum
