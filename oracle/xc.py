"""LDA exchange-correlation: Slater exchange + Perdew-Zunger 1981 correlation.

Sec. 2.2 lists LDA among the semilocal functionals; the workloads use the
spin-unpolarized form.  Per grid point, with r_s = (3 / (4 pi n))^{1/3}:
  exchange     eps_x = -(3/4) (3/pi)^{1/3} n^{1/3},   v_x = (4/3) eps_x
  correlation  r_s >= 1 (Pade in sqrt(r_s)):
                 eps_c = g / (1 + b1 sqrt(r_s) + b2 r_s)
                 v_c   = eps_c (1 + 7/6 b1 sqrt(r_s) + 4/3 b2 r_s) / (1 + b1 sqrt(r_s) + b2 r_s)
               r_s < 1 (high-density expansion):
                 eps_c = A ln r_s + B + C r_s ln r_s + D r_s
                 v_c   = A ln r_s + (B - A/3) + 2/3 C r_s ln r_s + (2D - C)/3 r_s
  g = -0.1423, b1 = 1.0529, b2 = 0.3334, A = 0.0311, B = -0.048,
  C = 0.0020, D = -0.0116.  Densities below 1e-16 (including negative
  values) give eps = v = 0.
v = d(n eps)/dn is the potential; E_xc = (Omega/N) sum_j n_j eps_xc(n_j).
"""
from __future__ import annotations

import numpy as np

PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
N_FLOOR = 1e-16


def lda_pz81(n: np.ndarray):
    """Return (eps_xc, v_xc) arrays of the same shape as n."""
    n = np.asarray(n, float)
    ok = n >= N_FLOOR
    nn = np.where(ok, n, 1.0)
    rs = (3.0 / (4.0 * np.pi * nn)) ** (1.0 / 3.0)
    ex = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * nn ** (1.0 / 3.0)
    vx = (4.0 / 3.0) * ex
    srs = np.sqrt(rs)
    den = 1.0 + PZ_BETA1 * srs + PZ_BETA2 * rs
    ec_lo = PZ_GAMMA / den
    vc_lo = ec_lo * (1.0 + (7.0 / 6.0) * PZ_BETA1 * srs + (4.0 / 3.0) * PZ_BETA2 * rs) / den
    lrs = np.log(rs)
    ec_hi = PZ_A * lrs + PZ_B + PZ_C * rs * lrs + PZ_D * rs
    vc_hi = PZ_A * lrs + (PZ_B - PZ_A / 3.0) + (2.0 / 3.0) * PZ_C * rs * lrs + ((2.0 * PZ_D - PZ_C) / 3.0) * rs
    hi = rs < 1.0
    ec = np.where(hi, ec_hi, ec_lo)
    vc = np.where(hi, vc_hi, vc_lo)
    eps = np.where(ok, ex + ec, 0.0)
    v = np.where(ok, vx + vc, 0.0)
    return eps, v


def exc_energy(n: np.ndarray, omega: float) -> float:
    eps, _ = lda_pz81(n)
    return float(omega / n.size * np.sum(n * eps))
