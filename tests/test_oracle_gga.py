"""Pins of the PBE oracle (oracle/gga.py), on the CPU.

  * PW92 against the oracle's PZ81 correlation (oracle/xc.py, pinned on its
    own): two fits of the same uniform-gas correlation energies, within
    1 mHa per electron for r_s in [0.5, 20]; its high-density limit (the
    RPA coefficient (1 - ln 2)/pi^2 of ln r_s and the constant -0.046644) and
    low-density limit (-0.4335 / r_s).  The intermediate-density parameters
    b2 and b3 are pinned only by the 1 mHa window (a 7% change of b3 stays
    inside it);
  * exchange enhancement F_x: the gradient expansion 1 + mu s^2 at small s
    and the bound 1 + kappa at large s;
  * correlation H: H / t^2 -> beta as t -> 0 (the gradient expansion) and
    H -> -eps_c as t -> infinity (correlation vanishes for a rapidly varying
    density);
  * the hydrogen atom (n = e^{-2r}/pi, fully polarized, E_x[n, 0] =
    E_x^unpol[2n] / 2): LDA exchange in closed form, -(81/256) 6^{1/3}
    pi^{-2/3}, and the PBE exchange energy of the PBE paper's table, -0.306 Ha;
  * complex-step derivatives against central differences, the uniform-
    density potential against the closed LDA exchange potential plus
    eps_c - (r_s/3) d eps_c / d r_s, and the grid potential against central
    differences of E_xc (which checks the divergence term).
"""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import gga, xc


def test_pw92_close_to_pz81():
    rs = np.linspace(0.5, 20.0, 400)
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    eps, _ = xc.lda_pz81(n)
    ec_pz = eps + 0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0)
    assert np.max(np.abs(gga.pw92_ec(rs) - ec_pz)) < 1e-3


def test_pw92_asymptotes():
    # high density: eps_c = a ln r_s + c1 + ..., with a the exact RPA
    # coefficient (1 - ln 2) / pi^2 and c1 = 2 a ln(2 a b1) = -0.046644
    rs = 1e-9
    slope = (gga.pw92_ec(rs * 1.01) - gga.pw92_ec(rs / 1.01)) / (2 * np.log(1.01))
    assert abs(slope - (1 - np.log(2)) / np.pi ** 2) < 1e-4 * slope
    assert abs(gga.pw92_ec(rs) - slope * np.log(rs) - (-0.046644)) < 2e-5
    # low density: eps_c -> -d0 / r_s with d0 = alpha1 / b4 = 0.4335 (the
    # next term is O(r_s^{-3/2}))
    rs = 1e9
    assert abs(gga.pw92_ec(rs) * rs + 0.4335) < 1e-4


def test_fx_limits():
    s2 = 1e-6  # (F_x - 1) / s^2 = mu / (1 + mu s^2 / kappa)
    assert abs((gga.fx_pbe(s2) - 1.0) / s2 - gga.MU) < 1e-6 * gga.MU
    assert abs(gga.fx_pbe(1e14) - (1.0 + gga.KAPPA)) < 1e-12
    s2 = np.linspace(0, 50, 1000)
    assert np.all(np.diff(gga.fx_pbe(s2)) > 0)


@pytest.mark.parametrize("rs", [0.3, 1.0, 4.0, 12.0])
def test_h_limits(rs):
    ec = gga.pw92_ec(rs)
    t2 = 1e-9
    assert abs(gga.h_pbe(ec, t2) / t2 - gga.BETA) < 1e-6 * gga.BETA
    assert abs(gga.h_pbe(ec, 1e14) + ec) < 1e-9 * abs(ec)
    assert gga.h_pbe(ec, 0.0) == 0.0


def _h_atom_exchange(lda):
    def f(r):
        n = 2.0 * np.exp(-2.0 * r) / np.pi
        sig = 0.0 if lda else (4.0 * np.exp(-2.0 * r) / np.pi) ** 2
        return 4.0 * np.pi * r * r * float(np.real(gga.ex_pbe(n, sig)))
    return 0.5 * quad(f, 0.0, 60.0, limit=400, epsabs=1e-14, epsrel=1e-13)[0]


def test_hydrogen_atom_exchange():
    closed = -(81.0 / 256.0) * 6.0 ** (1.0 / 3.0) * np.pi ** (-2.0 / 3.0)
    assert abs(_h_atom_exchange(True) - closed) < 1e-12
    # PBE exchange energy of the hydrogen atom, -0.306 Ha (to the table's 3 decimals)
    assert abs(_h_atom_exchange(False) - (-0.306)) < 5e-4


def test_complex_step_derivatives():
    rng = np.random.default_rng(4)
    n = 10.0 ** rng.uniform(-5, 1, 50)
    sig = (n ** (4.0 / 3.0)) ** 2 * 10.0 ** rng.uniform(-3, 2, 50)
    e, en, es = gga.e_and_derivatives(n, sig)
    def d5(f, x, h):  # five-point central difference, O(h^4)
        return (f(x - 2 * h) - 8 * f(x - h) + 8 * f(x + h) - f(x + 2 * h)) / (12 * h)

    for i in range(50):
        fd = d5(lambda x: gga.e_and_derivatives(x, sig[i])[0], n[i], 1e-4 * n[i])
        assert abs(fd - en[i]) < 1e-8 * abs(en[i])
        # e varies weakly with sigma (de/dsigma sigma << e): the difference is
        # rounding-limited at ~3e-5 relative; any dropped term is O(1)
        fd = d5(lambda x: gga.e_and_derivatives(n[i], x)[0], sig[i], 5e-2 * sig[i])
        assert abs(fd - es[i]) < 1e-4 * abs(es[i])


def test_uniform_density_potential():
    rs = np.array([0.4, 1.0, 3.0, 9.0])
    n = 3.0 / (4.0 * np.pi * rs ** 3)
    e, en, _ = gga.e_and_derivatives(n, np.zeros_like(n))
    vx = (4.0 / 3.0) * (-0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0))
    h = 1e-6 * rs
    dec = (gga.pw92_ec(rs + h) - gga.pw92_ec(rs - h)) / (2 * h)
    vc = gga.pw92_ec(rs) - rs / 3.0 * dec
    assert np.max(np.abs(en - (vx + vc)) / np.abs(vx + vc)) < 1e-8


def test_grid_potential_is_functional_derivative():
    R = np.array([[7.0, 0.3, 0.0], [0.0, 6.6, 0.4], [0.2, 0.0, 7.2]])
    S = (16, 15, 18)
    fr = np.stack(np.meshgrid(*[np.arange(s) / s for s in S], indexing="ij"), axis=-1)
    r = fr @ R.T
    c1, c2 = R @ np.array([0.4, 0.5, 0.45]), R @ np.array([0.7, 0.3, 0.6])

    def blob(c, w):
        d = fr - np.linalg.solve(R, c)
        d -= np.round(d)
        x = d @ R.T
        return np.exp(-np.sum(x * x, axis=-1) / (2 * w * w))

    n = 0.3 * blob(c1, 1.1) + 0.2 * blob(c2, 0.9) + 1e-3
    dn = np.cos(2 * np.pi * fr[..., 0]) * np.sin(2 * np.pi * fr[..., 1] + 0.4) * 1e-3 + 2e-4 * blob(c2, 1.3)
    v, E = gga.pbe_on_grid(n, R)
    h = 1e-2
    E = [gga.pbe_on_grid(n + k * h * dn, R)[1] for k in (-2, -1, 1, 2)]
    dV = abs(np.linalg.det(R)) / n.size
    lhs = (E[0] - 8 * E[1] + 8 * E[2] - E[3]) / (12 * h)  # O(h^4)
    rhs = dV * np.sum(v * dn)
    assert abs(lhs - rhs) < 1e-7 * abs(rhs), (lhs, rhs)
    del r
