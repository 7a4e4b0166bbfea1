"""GPU parity of the LinearPCM solve (dpp_pcm_solve) with the oracle
(oracle/pcm.py) on the same seeded eps(r) and rho(r).

Both run the same preconditioned CG to a relative residual of 1e-12 (1e-10
at 90^3).  A residual of t leaves a solution error of at most kappa t, with
kappa the preconditioned condition number, bounded by max eps / min eps = 78.4
for the vacuum-inverse preconditioner; so phi agrees to about 1e-10 relative
and A_diel, linear in phi at fixed rho, to the same order: bars 1e-9 (1e-7 at
90^3).  Iteration counts may differ by one where the residual crosses the
threshold within rounding.  Edge cases: eps = 1 (the preconditioner is the
exact inverse: one iteration, A_diel = 0), and max_iter = 0 (phi = 0,
A_diel = -E_H over the solved modes).
"""
import numpy as np
import pytest

import workloads as W
from oracle import energy as oe, pcm
from tests._gpu import Device, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return Device()


def _gpu_solve(dev, R, S, eps, rho, tol, max_iter):
    D = dev.D
    g = dev.grid(R, S)
    ws = dev.ws(D.dpp_pcm_workspace_size(g))
    phi = dev.empty(S, dev.torch.float64)
    A, it, rel = D.dpp_pcm_solve(g, dev.tensor(eps), dev.tensor(rho), tol, max_iter, phi, ws)
    out = dev.host(phi)
    D.dpp_grid_destroy(g)
    return A, out, it, rel


@pytest.mark.parametrize("kind,tol,bar", [("small", 1e-12, 1e-9), ("skew", 1e-12, 1e-9), ("config3", 1e-10, 1e-7)])
def test_pcm_matches_oracle(dev, kind, tol, bar):
    c = W.pcm_case(kind)
    R, S, eps, rho = c["R"], c["S"], c["eps"], c["rho"]
    log(f"pcm {kind} S={S} tol={tol}")
    A, phi, it, rel = _gpu_solve(dev, R, S, eps, rho, tol, 1000)
    Ao, phio, ito, relo = pcm.get_adiel(R, S, eps, rho, tol=tol, max_iter=1000)
    log(f"gpu A={A:.15e} it={it} rel={rel:.2e}; oracle A={Ao:.15e} it={ito} rel={relo:.2e}")
    assert rel <= tol and abs(it - ito) <= 1
    assert abs(A - Ao) < bar * abs(Ao)
    assert np.max(np.abs(phi - phio)) < bar * np.max(np.abs(phio))


def test_pcm_edge_cases(dev):
    R = np.array([[9.0, 0.4, 0.0], [0.0, 8.5, 0.3], [0.2, 0.0, 9.4]])
    S = (9, 15, 25)  # odd: no Nyquist modes, so the solved modes are all G != 0
    rho = np.random.default_rng(3).standard_normal(S)
    EH = oe.hartree(rho, R)[1]
    A, phi, it, rel = _gpu_solve(dev, R, S, np.ones(S), rho, 1e-12, 100)
    log(f"eps = 1: A={A:.3e} it={it} rel={rel:.2e} (E_H {EH:.3e})")
    assert it == 1 and rel <= 1e-12 and abs(A) < 1e-12 * abs(EH)
    A0, phi0, it0, _ = _gpu_solve(dev, R, S, np.full(S, 5.0), rho, 1e-12, 0)
    assert it0 == 0 and np.all(phi0 == 0.0)
    assert abs(A0 + EH) < 1e-12 * abs(EH)
