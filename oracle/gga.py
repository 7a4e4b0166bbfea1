"""GGA exchange-correlation: PBE, spin-unpolarized, FP64 (test infrastructure only).

Table 1 and Sec. 2.2 list semilocal (GGA) functionals; PBE is the common
one.  Per grid point, with sigma = |grad n|^2, k_F = (3 pi^2 n)^{1/3},
r_s = (3 / (4 pi n))^{1/3}, k_s = sqrt(4 k_F / pi):
  exchange     e_x = n eps_x^LDA F_x(s),  eps_x^LDA = -(3/4)(3/pi)^{1/3} n^{1/3},
               s^2 = sigma / (4 k_F^2 n^2),
               F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa)
  correlation  e_c = n (eps_c^PW92(r_s) + H),  t^2 = sigma / (4 k_s^2 n^2),
               H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
               A = (beta/gamma) / (exp(-eps_c^PW92 / gamma) - 1)
  PW92         eps_c = -2 a (1 + alpha1 r_s)
                       ln(1 + 1 / (2 a (b1 r_s^{1/2} + b2 r_s + b3 r_s^{3/2} + b4 r_s^2)))
  kappa = 0.804, beta = 0.06672455060314922, mu = beta pi^2 / 3,
  gamma = (1 - ln 2) / pi^2; a = 0.031091, alpha1 = 0.21370, b1 = 7.5957,
  b2 = 3.5876, b3 = 1.6382, b4 = 0.49294.
Densities below 1e-16 (negative ones included) give e = 0 and no derivatives.

Energy and potential on the grid (the functional derivative of
E_xc = (Omega/N) sum_r e(n, sigma)):
  v_xc = de/dn - 2 div(de/dsigma grad n),
with grad and div spectral on the full box: J, times i G', I (real part), G'
as in the LinearPCM oracle (the Nyquist index of an even axis counts as 0).
The pointwise derivatives de/dn and de/dsigma are taken by complex-step
differentiation (f'(x) = Im f(x + i h) / h), exact to rounding.

Pinned by tests/test_oracle_gga.py: PW92 against the oracle's PZ81 (two
fits of the same correlation energies, within 1 mHa) and its high- and
low-density limits (b2 and b3 only through the 1 mHa window), the limits of F_x
and H (gradient expansions and the bounds 1 + kappa, H -> -eps_c), the
hydrogen-atom PBE and LDA exchange energies, complex-step against central
differences, and the potential against central differences of E_xc.
"""
from __future__ import annotations

import numpy as np

from .basis import cell_volume

KAPPA = 0.804
BETA = 0.06672455060314922
MU = BETA * np.pi ** 2 / 3.0
GAMMA = (1.0 - np.log(2.0)) / np.pi ** 2
PW_A, PW_ALPHA1 = 0.031091, 0.21370
PW_B = (7.5957, 3.5876, 1.6382, 0.49294)
N_FLOOR = 1e-16


def pw92_ec(rs):
    """PW92 correlation energy per electron (unpolarized); complex-safe."""
    srs = np.sqrt(rs)
    den = 2.0 * PW_A * (PW_B[0] * srs + PW_B[1] * rs + PW_B[2] * rs * srs + PW_B[3] * rs * rs)
    return -2.0 * PW_A * (1.0 + PW_ALPHA1 * rs) * np.log1p(1.0 / den)


def fx_pbe(s2):
    return 1.0 + KAPPA - KAPPA / (1.0 + MU * s2 / KAPPA)


def h_pbe(ec, t2):
    A = (BETA / GAMMA) / (np.exp(-ec / GAMMA) - 1.0)
    At2 = A * t2
    return GAMMA * np.log1p((BETA / GAMMA) * t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2))


def ex_pbe(n, sigma):
    """Exchange part n eps_x^LDA F_x(s) alone; complex-safe."""
    kF = (3.0 * np.pi ** 2 * n) ** (1.0 / 3.0)
    ex_lda = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0)
    return n * ex_lda * fx_pbe(sigma / (4.0 * kF * kF * n * n))


def e_pbe(n, sigma):
    """Energy density e(n, sigma) (hartree / bohr^3) for n >= N_FLOOR; complex-safe."""
    kF = (3.0 * np.pi ** 2 * n) ** (1.0 / 3.0)
    rs = (3.0 / (4.0 * np.pi * n)) ** (1.0 / 3.0)
    ks = np.sqrt(4.0 * kF / np.pi)
    ex_lda = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0)
    s2 = sigma / (4.0 * kF * kF * n * n)
    t2 = sigma / (4.0 * ks * ks * n * n)
    ec = pw92_ec(rs)
    return n * ex_lda * fx_pbe(s2) + n * (ec + h_pbe(ec, t2))


def e_and_derivatives(n, sigma):
    """(e, de/dn, de/dsigma) per point by complex steps; zero below the density floor."""
    n = np.asarray(n, float)
    sigma = np.asarray(sigma, float)
    ok = n >= N_FLOOR
    nn = np.where(ok, n, 1.0)
    ss = np.where(ok, sigma, 0.0)
    hn = 1e-20 * nn
    hs = 1e-20 * np.maximum(ss, 1e-30)
    e = np.real(e_pbe(nn + 0j, ss + 0j))
    en = np.imag(e_pbe(nn + 1j * hn, ss + 0j)) / hn
    es = np.imag(e_pbe(nn + 0j, ss + 1j * hs)) / hs
    return np.where(ok, e, 0.0), np.where(ok, en, 0.0), np.where(ok, es, 0.0)


def _Gp(R, S):
    from .pcm import spectral_G
    return spectral_G(R, S)


def gradient_real(n, R):
    """grad n on the grid: Re I(i G'_d J n), shape (3,) + S."""
    S = n.shape
    Gp = _Gp(R, S)
    nt = np.fft.fftn(n) / n.size
    return np.stack([np.real(n.size * np.fft.ifftn(1j * Gp[..., d] * nt)) for d in range(3)])


def divergence_real(h, R):
    """div h on the grid for h of shape (3,) + S (real fields)."""
    S = h.shape[1:]
    Gp = _Gp(R, S)
    N = int(np.prod(S))
    acc = np.zeros(S, complex)
    for d in range(3):
        acc += 1j * Gp[..., d] * (np.fft.fftn(h[d]) / N)
    return np.real(N * np.fft.ifftn(acc))


def pbe_on_grid(n, R):
    """(v_xc, E_xc) of a real density on the box with lattice R."""
    g = gradient_real(n, R)
    sigma = np.sum(g * g, axis=0)
    e, en, es = e_and_derivatives(n, sigma)
    v = en - 2.0 * divergence_real(es[None] * g, R)
    return v, float(cell_volume(R) / n.size * np.sum(e))
