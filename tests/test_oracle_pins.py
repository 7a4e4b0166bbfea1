"""Pins for the oracle parts that the step-by-step parity tests rest on:
the band residual that drives the FP64 refinement switch, the Pulay (DIIS)
step of the SCF mixing (Sec. 2.1 names Pulay mixing), the published PZ81
correlation constants (LDA, Sec. 2.2) and Adam beyond its first step.

Each check is against something other than the oracle's own formula: an
exact eigenpair of the explicit plane-wave Hamiltonian matrix, an
independently posed constrained least-squares problem, the constants as
published with the continuity they were built for, and the closed form of
Adam under a constant gradient."""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import convnet as cn, energy, operators as ops, scf, xc
from tests._golden import constants


# ------------------------------------------------------------- residual ---
def _tiny_dense(seed=5):
    R = np.array([[6.8, 0.4, 0.0], [0.0, 6.5, 0.3], [0.2, 0.0, 7.1]])
    cell = W.tiny_cell(nat=2, L=7.0, ecut=2.0, S=(14, 14, 14), nb=4, Z=(4, 1), fold=(2, 1, 1), R=R, seed=seed)
    s = energy.build_system(cell)
    Veff = s.Vloc + W.random_potential(17, cell.S, 0.2)
    return cell, s, Veff


def test_residual_norm_vanishes_at_exact_eigenpairs():
    cell, s, Veff = _tiny_dense()
    for k, b in enumerate(s.bases):
        H = ops.dense_hamiltonian(b, Veff, s.P[k], s.D)
        # H c = O c eps with O = Omega: generalized problem, c^dag O c = 1
        eps, C = scipy.linalg.eigh(H, b.omega * np.eye(b.npw))
        psi, e = C[:, :4], eps[:4]
        r = energy.residual_norm(psi, e, b, Veff, s.P[k], s.D)
        assert r < 1e-10 * max(1.0, np.max(np.abs(e)))


def test_residual_norm_closed_form_of_a_perturbed_eigenpair():
    """psi_i + delta_i v with v a known sphere vector: the residual of column i
    is delta_i ||(H - eps_i Omega) v|| / sqrt(Omega) with H the dense matrix,
    and the reported value is the largest over the columns."""
    cell, s, Veff = _tiny_dense(seed=9)
    b = s.bases[1]
    H = ops.dense_hamiltonian(b, Veff, s.P[1], s.D)
    eps, C = scipy.linalg.eigh(H, b.omega * np.eye(b.npw))
    rng = np.random.default_rng(3)
    v = rng.standard_normal(b.npw) + 1j * rng.standard_normal(b.npw)
    deltas = np.array([1e-3, 4e-3, 2e-3])
    psi = C[:, :3] + v[:, None] * deltas[None, :]
    expect = [deltas[i] * np.linalg.norm((H - eps[i] * b.omega * np.eye(b.npw)) @ v) / math.sqrt(b.omega)
              for i in range(3)]
    got = energy.residual_norm(psi, eps[:3], b, Veff, s.P[1], s.D)
    assert abs(got - max(expect)) < 1e-9 * max(expect)
    # the largest is not the first column: a "first column" or "sum" reading fails
    assert int(np.argmax(expect)) == 1 and abs(sum(expect) - max(expect)) > 0.1 * max(expect)


# ---------------------------------------------------------------- Pulay ---
def _pulay_expected(hist, alpha):
    """Mixed density from the last history entries, posed independently:
    minimize ||sum_i c_i R_i|| subject to sum_i c_i = 1 by eliminating c_m
    (c_m = 1 - sum_{i<m} c_i) and solving the unconstrained least-squares
    problem with numpy.linalg.lstsq."""
    m = len(hist)
    Rm = hist[-1][1].reshape(-1)
    if m == 1:
        c = np.array([1.0])
    else:
        A = np.stack([hist[i][1].reshape(-1) - Rm for i in range(m - 1)], axis=1)
        x = np.linalg.lstsq(A, -Rm, rcond=None)[0]
        c = np.append(x, 1.0 - x.sum())
    return sum(c[i] * (hist[i][0] + alpha * hist[i][1]) for i in range(m)), c


@pytest.mark.parametrize("steps", [1, 2, 3, 5, 8, 11])
def test_pulay_step_is_constrained_least_squares(steps):
    S = (6, 5, 4)
    omega = 123.0
    rng = np.random.default_rng(100 + steps)
    mixer = scf.Pulay(omega, int(np.prod(S)))
    hist = []
    n_in = rng.random(S)
    for t in range(steps):
        # residuals of decreasing size with random directions
        n_out = n_in + (0.5 ** t) * rng.standard_normal(S)
        out = mixer.mix(n_in, n_out)
        hist.append((n_in.copy(), n_out - n_in))
        hist = hist[-8:]
        if t == 0:
            # the first iteration is linear mixing
            assert np.max(np.abs(out - (n_in + 0.5 * (n_out - n_in)))) < 1e-15
        ref, c = _pulay_expected(hist, 0.5)
        assert abs(c.sum() - 1.0) < 1e-12
        assert np.max(np.abs(out - ref)) < 1e-10 * np.max(np.abs(ref))
        n_in = out


def test_pulay_coefficients_minimize_the_residual_norm():
    """Any other affine combination of the residuals is longer."""
    S = (5, 5, 5)
    rng = np.random.default_rng(7)
    mixer = scf.Pulay(50.0, 125)
    hist = []
    n_in = rng.random(S)
    for t in range(5):
        n_out = n_in + rng.standard_normal(S)
        out = mixer.mix(n_in, n_out)
        hist.append((n_in.copy(), n_out - n_in))
        n_in = out
    _, c = _pulay_expected(hist, 0.5)
    Rs = np.stack([h[1].reshape(-1) for h in hist], axis=1)
    best = np.linalg.norm(Rs @ c)
    for _ in range(50):
        d = rng.standard_normal(len(c))
        d -= d.mean()                       # keeps sum c = 1
        assert np.linalg.norm(Rs @ (c + 1e-3 * d)) >= best


# ----------------------------------------------------------------- PZ81 ---
def test_pz81_constants_are_the_published_ones():
    g = constants()
    pub = [("pz81_gamma", xc.PZ_GAMMA), ("pz81_beta1", xc.PZ_BETA1), ("pz81_beta2", xc.PZ_BETA2),
           ("pz81_A", xc.PZ_A), ("pz81_B", xc.PZ_B), ("pz81_C", xc.PZ_C), ("pz81_D", xc.PZ_D)]
    for key, val in pub:
        assert val == g[key], key


def test_pz81_high_density_constants_follow_from_continuity():
    """Perdew and Zunger fixed B and D by continuity of eps_c and of
    d eps_c / d r_s at r_s = 1 given the low-density Pade fit and A, C.
    Solving those two conditions with the published gamma, beta1, beta2, A
    and C gives B and D to the published precision."""
    g = constants()
    gam, b1, b2 = g["pz81_gamma"], g["pz81_beta1"], g["pz81_beta2"]
    A, C = g["pz81_A"], g["pz81_C"]
    den = 1.0 + b1 + b2
    e1 = gam / den
    de1 = -gam * (0.5 * b1 + b2) / den ** 2          # d/drs of gamma/(1 + b1 sqrt(rs) + b2 rs) at rs = 1
    # high-density branch at rs = 1: value B + D, slope A + C + D
    D = de1 - A - C
    B = e1 - D
    assert abs(D - g["pz81_D"]) < 5e-5
    assert abs(B - g["pz81_B"]) < 5e-4
    # the oracle's two branches meet with jumps of that rounding size only
    n1 = 3.0 / (4.0 * math.pi)
    lo, _ = xc.lda_pz81(np.array([n1 * (1 - 1e-12)]))
    hi, _ = xc.lda_pz81(np.array([n1 * (1 + 1e-12)]))
    assert abs(lo[0] - hi[0]) < 5e-5
    # slopes of eps_c on both sides (central differences inside each branch)
    h = 1e-4
    rs = np.array([1 - 2 * h, 1 - h, 1 + h, 1 + 2 * h])
    e = xc.lda_pz81(3.0 / (4.0 * math.pi * rs ** 3))[0] + g["slater_coeff"] / rs
    slope_hi = (e[1] - e[0]) / h      # rs < 1: high-density branch
    slope_lo = (e[3] - e[2]) / h      # rs > 1: Pade branch
    assert abs(slope_hi - (A + C + g["pz81_D"])) < 1e-3
    assert abs(slope_lo - de1) < 1e-3


# ----------------------------------------------------------------- Adam ---
def _params(seed=3):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((2, 1, 3, 3, 3)), rng.standard_normal(2)),
            (rng.standard_normal((1, 2, 3, 3, 3)), rng.standard_normal(1))]


@pytest.mark.parametrize("steps", [1, 2, 5, 12])
def test_adam_constant_gradient_moves_lr_per_step(steps):
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2, so every step moves each parameter by -lr g / (|g| + eps)."""
    params = _params()
    rng = np.random.default_rng(11)
    grads = [(rng.choice([-3.0, -0.5, 0.7, 2.0], W.shape), rng.choice([-1.5, 0.25], b.shape)) for W, b in params]
    lr, eps = 1e-2, 1e-8
    opt = cn.Adam(params, lr=lr, eps=eps)
    p = params
    for _ in range(steps):
        p = opt.step(p, grads)
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, p, grads):
        for x0, x1, g in ((W0, W1, gW), (b0, b1, gb)):
            expect = -lr * steps * g / (np.abs(g) + eps)
            assert np.max(np.abs((x1 - x0) - expect)) < 1e-12


def test_adam_is_invariant_to_gradient_scale():
    """Adam's step depends on g only through m / sqrt(v): scaling every
    gradient by a constant leaves the trajectory unchanged (up to eps)."""
    params = _params(5)
    rng = np.random.default_rng(13)
    seq = [[(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params] for _ in range(6)]
    runs = []
    for scale in (1.0, 1000.0):
        opt = cn.Adam(params, lr=1e-2, eps=1e-12)
        p = params
        for g in seq:
            p = opt.step(p, [(scale * gW, scale * gb) for gW, gb in g])
        runs.append(p)
    for (Wa, ba), (Wb, bb) in zip(*runs):
        assert np.max(np.abs(Wa - Wb)) < 1e-9 and np.max(np.abs(ba - bb)) < 1e-9
    # and the trajectory does depend on the gradients' history (bias
    # correction and momentum at work): reversing the sequence changes it
    opt = cn.Adam(params, lr=1e-2, eps=1e-12)
    p = params
    for g in seq[::-1]:
        p = opt.step(p, g)
    assert max(np.max(np.abs(a[0] - b[0])) for a, b in zip(p, runs[0])) > 1e-4
