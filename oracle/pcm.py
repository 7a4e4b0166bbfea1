"""LinearPCM: the dielectric Poisson solve and the solvation energy, FP64
(test infrastructure only).

Sec. 2.1, Eq. (1): -4 pi rho = div(eps grad phi); Eq. (2):
A_diel = (1/2) int (phi - K rho) rho, K the unscreened Coulomb operator.
Listing 1 poses Eq. (1) as a linear problem on reciprocal-space fields,
hessian(phi~) = rho~ with hessian(x) = (-1/(4 pi)) div(J(eps * I(grad x))),
solved by conjugate gradients, and evaluates Eq. (2) as
(1/2) dot(phi~ - coulomb(rho~), O rho~).

Conventions (the library's own, listed as readings):
  * J x = fftn(x) / N and I y = N ifftn(y) on the full box (J I = 1), so a
    real field's coefficients are Hermitian; O = Omega, so that
    dot(a, O b) = Omega sum_G conj(a) b = int a*(r) b(r) dr;
  * grad x -> i G' x, div v -> sum_d i G'_d v_d with G' = B m', where m' is the
    signed frequency m of each axis except that the Nyquist index of an even
    axis counts as 0 (the spectral derivative of a real field stays real);
  * modes with G' = 0 (G = 0 and the pure-Nyquist modes) carry no part of
    the solve: phi~ is zero there and rho~ there is dropped (a neutralizing
    background for any net charge);
  * coulomb(rho~) = 4 pi rho~ / |G|^2 for G != 0 and 0 at G = 0; on the
    modes outside the solve it is zeroed too, so phi - K rho only compares
    what the solve determines;
  * CG is preconditioned by the inverse of the vacuum operator,
    M = 4 pi / |G'|^2 on the solved modes; inner products are real parts of
    sum_G conj(a) b; start phi~ = 0; stop when ||r|| <= tol ||rho~||.

Pinned by tests/test_oracle_pcm.py: uniform eps (closed form), a dense
direct solve on a small box, a layered dielectric against the continuum
solution by quadrature, symmetry and positivity of the operator, and the
sign and vacuum limit of A_diel.
"""
from __future__ import annotations

import numpy as np

from .basis import box_frequencies, cell_volume, reciprocal_basis


def spectral_G(R, S) -> np.ndarray:
    """G' = B m' for every box point (Nyquist index of even axes -> 0), shape S + (3,)."""
    m = box_frequencies(S).astype(float)
    for d, s in enumerate(S):
        if s % 2 == 0:
            m[..., d] = np.where(m[..., d] == -s // 2, 0.0, m[..., d])
    return m @ reciprocal_basis(R).T


def solved_modes(R, S) -> np.ndarray:
    """Boolean mask of the modes that take part in the solve (G' != 0)."""
    Gp = spectral_G(R, S)
    return np.sum(Gp * Gp, axis=-1) > 0.0


def J(x):
    return np.fft.fftn(x) / x.size


def I(y):
    return y.size * np.fft.ifftn(y)


def gradient(x, Gp):
    """i G' x for each Cartesian direction: shape (3,) + S."""
    return np.stack([1j * Gp[..., d] * x for d in range(3)])


def divergence(v, Gp):
    return sum(1j * Gp[..., d] * v[d] for d in range(3))


def hessian(x, eps, Gp):
    """(-1/(4 pi)) div(J(eps * I(grad x))); I of a Hermitian field is real."""
    g = gradient(x, Gp)
    w = np.stack([J(eps * np.real(I(g[d]))) for d in range(3)])
    return (-1.0 / (4.0 * np.pi)) * divergence(w, Gp)


def dot(a, b) -> float:
    return float(np.real(np.vdot(a, b)))


def coulomb(rt, R, S):
    """4 pi rho~ / |G|^2 (G != 0), zero at G = 0."""
    G = box_frequencies(S) @ reciprocal_basis(R).T
    G2 = np.sum(G * G, axis=-1)
    out = np.zeros_like(rt)
    nz = G2 > 0
    out[nz] = 4.0 * np.pi * rt[nz] / G2[nz]
    return out


def solve(R, S, eps, rho, tol=1e-10, max_iter=1000):
    """Preconditioned CG for hessian(phi~) = rho~ on the solved modes.
    Returns (phi~, iterations, relative residual)."""
    Gp = spectral_G(R, S)
    G2p = np.sum(Gp * Gp, axis=-1)
    mask = G2p > 0.0
    M = np.zeros(G2p.shape)
    M[mask] = 4.0 * np.pi / G2p[mask]
    b = np.where(mask, J(rho), 0.0)
    x = np.zeros_like(b)
    r = b.copy()
    z = M * r
    p = z.copy()
    rz = dot(r, z)
    bn = np.sqrt(dot(b, b))
    it, rel = 0, (np.sqrt(dot(r, r)) / bn if bn > 0 else 0.0)
    while it < max_iter and rel > tol:
        q = np.where(mask, hessian(p, eps, Gp), 0.0)
        alpha = rz / dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        rel = np.sqrt(dot(r, r)) / bn
        if rel <= tol:
            break
        z = M * r
        rz_new = dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, rel


def a_diel(R, S, phit, rho):
    """(1/2) dot(phi~ - coulomb(rho~), O rho~) over the solved modes (Eq. (2))."""
    omega = cell_volume(R)
    mask = solved_modes(R, S)
    rt = np.where(mask, J(rho), 0.0)
    return 0.5 * omega * dot(phit - np.where(mask, coulomb(rt, R, S), 0.0), rt)


def get_adiel(R, S, eps, rho, tol=1e-10, max_iter=1000):
    """Listing 1's getAdiel: solve, then Eq. (2).  Returns (A_diel, phi(r), iterations, residual)."""
    phit, it, rel = solve(R, S, eps, rho, tol, max_iter)
    return a_diel(R, S, phit, rho), np.real(I(phit)), it, rel
