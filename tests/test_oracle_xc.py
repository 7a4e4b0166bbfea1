"""Pins for LDA (Slater + PZ81): literature HEG values, exact limits,
v = d(n eps)/dn by finite differences, branch continuity."""
import math

import numpy as np
import pytest

from oracle import xc
from tests._golden import constants


def n_of_rs(rs):
    return 3.0 / (4.0 * math.pi * rs ** 3)


def test_exchange_is_slater():
    # at very high density exchange dominates: eps * rs -> -0.458165... (textbook)
    c = constants()["slater_coeff"]
    for rs in (1e-7, 1e-6):
        eps, v = xc.lda_pz81(np.array([n_of_rs(rs)]))
        assert abs(eps[0] * rs + c) < 1e-5 * c
        assert abs(v[0] * rs + 4.0 / 3.0 * c) < 1e-5 * c


@pytest.mark.parametrize("rs,key", [(1.0, "heg_ec_rs1"), (2.0, "heg_ec_rs2"), (5.0, "heg_ec_rs5"), (10.0, "heg_ec_rs10")])
def test_correlation_matches_qmc_fit(rs, key):
    c = constants()
    eps, _ = xc.lda_pz81(np.array([n_of_rs(rs)]))
    ec = eps[0] + c["slater_coeff"] / rs
    assert abs(ec - c[key]) < 1e-3


def test_high_density_coefficient_is_rpa():
    c = constants()
    # eps_c(rs) - eps_c(rs/e) -> A as rs -> 0 (log slope)
    rs = 1e-4
    e1, _ = xc.lda_pz81(np.array([n_of_rs(rs)]))
    e2, _ = xc.lda_pz81(np.array([n_of_rs(rs / math.e)]))
    ec1 = e1[0] + c["slater_coeff"] / rs
    ec2 = e2[0] + c["slater_coeff"] / (rs / math.e)
    assert abs((ec1 - ec2) - c["rpa_A"]) < 2e-4


@pytest.mark.parametrize("rs", [0.2, 0.7, 0.99, 1.01, 1.5, 3.0, 8.0, 30.0])
def test_potential_is_derivative(rs):
    n = n_of_rs(rs)
    h = n * 1e-5
    ep, _ = xc.lda_pz81(np.array([n + h]))
    em, _ = xc.lda_pz81(np.array([n - h]))
    _, v = xc.lda_pz81(np.array([n]))
    fd = ((n + h) * ep[0] - (n - h) * em[0]) / (2 * h)
    assert abs(fd - v[0]) < 1e-8 * abs(v[0])


def test_branch_continuity_and_floor():
    n1 = n_of_rs(1.0)
    a, va = xc.lda_pz81(np.array([n1 * (1 + 1e-12)]))
    b, vb = xc.lda_pz81(np.array([n1 * (1 - 1e-12)]))
    assert 1e-6 < abs(a[0] - b[0]) < 1e-4    # PZ81's small jump at rs = 1
    assert abs(va[0] - vb[0]) < 1e-4
    eps, v = xc.lda_pz81(np.array([0.0, -1e-3, 5e-17]))
    assert np.all(eps == 0) and np.all(v == 0)
