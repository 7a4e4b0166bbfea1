"""Preconditioned nonlinear CG for band minimization (FP64 oracle).

Sec. 2.1 names Minimize (variational minimization by linear/nonlinear CG)
and Sec. 2.2 the variational minimization of the total energy.  The paper
gives no step rules, so this fixes one protocol that both implementations
follow step for step:

* inner product  <A, B> = sum_k 2 Re Tr(A_k^dag B_k); preconditioner K per k.
* direction      D = -K g + beta D_prev,
                 beta = max(0, <g - g_prev, K g> / <g_prev, K g_prev>)
                 (Polak-Ribiere), beta = 0 on the first step and after a
                 failed line minimization; if d0 = <g, D> >= 0, D = -K g.
* line search    trial step a_t (first 0.3/s, then the last accepted step);
                 fit E(a) = E0 + d0 a + c a^2 from E(a_t); a* = -d0/(2c) if
                 c > 0 else 2 a_t, clamped to 10 a_t; accept a* if
                 E(a*) <= E0, else a_t if E(a_t) <= E0, else halve a_t and
                 retry (at most 6 tries).  After a failure, one more line
                 minimization along -K g; if that fails as well the state is
                 stationary.
* the starting block is orthonormalized once (Y <- Y R^{-1}), so the first
  trial step 0.3/s is on the scale of the wavefunctions; after that Y is not
  re-orthonormalized between steps: the objective orthonormalizes.
"""
from __future__ import annotations

from typing import Callable, List

import numpy as np

MAX_TRIES = 6


def dot(A: List[np.ndarray], B: List[np.ndarray]) -> float:
    return float(sum(2.0 * np.real(np.vdot(a, b)) for a, b in zip(A, B)))


def axpy(Y, a, D):
    return [y + a * d for y, d in zip(Y, D)]


class CG:
    """State machine for one minimization (one objective over a list of blocks)."""

    def __init__(self, Y, objective: Callable, energy_only: Callable, precond: Callable, alpha0: float):
        self.Y = [y.copy() for y in Y]
        self.objective = objective
        self.energy_only = energy_only
        self.precond = precond
        self.alpha_t = alpha0
        self.E = None
        self.g = None
        self.g_prev = self.Kg_prev = self.D_prev = None
        self.reset = True
        self.stationary = False
        self.history = []

    def _linemin(self, D, d0):
        E0 = self.E
        a_t = self.alpha_t
        for _ in range(MAX_TRIES):
            E_t = self.energy_only(axpy(self.Y, a_t, D))
            c = (E_t - E0 - d0 * a_t) / (a_t * a_t)
            a_s = -d0 / (2.0 * c) if c > 0 else 2.0 * a_t
            a_s = min(a_s, 10.0 * a_t)
            Ys = axpy(self.Y, a_s, D)
            E_s, g_s = self.objective(Ys)
            if E_s <= E0:
                return True, a_s, Ys, E_s, g_s
            if E_t <= E0:
                Yt = axpy(self.Y, a_t, D)
                E_t2, g_t = self.objective(Yt)
                return True, a_t, Yt, E_t2, g_t
            a_t *= 0.5
        return False, None, None, None, None

    def step(self) -> bool:
        """One CG step; returns False once stationary."""
        if self.stationary:
            return False
        if self.E is None:
            self.E, self.g = self.objective(self.Y)
            self.history.append(self.E)
        g = self.g
        Kg = self.precond(g)
        if self.reset or self.g_prev is None:
            beta = 0.0
        else:
            beta = max(0.0, (dot(g, Kg) - dot(self.g_prev, Kg)) / dot(self.g_prev, self.Kg_prev))
        D = [-kg for kg in Kg] if beta == 0.0 else [-kg + beta * dp for kg, dp in zip(Kg, self.D_prev)]
        d0 = dot(g, D)
        steepest = beta == 0.0
        if d0 >= 0.0:
            D = [-kg for kg in Kg]
            d0 = dot(g, D)
            steepest = True
        ok, a, Yn, En, gn = self._linemin(D, d0)
        if not ok and not steepest:
            D = [-kg for kg in Kg]
            d0 = dot(g, D)
            ok, a, Yn, En, gn = self._linemin(D, d0)
        if not ok:
            self.stationary = True
            self.reset = True
            return False
        self.g_prev, self.Kg_prev, self.D_prev = g, Kg, D
        self.Y, self.E, self.g = Yn, En, gn
        self.alpha_t = a
        self.reset = False
        self.history.append(En)
        return True


def protocol_V(Ys, sys, f: float, nsteps: int):
    """Direct minimization of E_el over the occupied blocks with filling f."""
    from .energy import energy_and_gradient, total_energy
    from .operators import K

    def objective(Y):
        return energy_and_gradient(Y, f, sys)

    def energy_only(Y):
        return total_energy(Y, [np.full(y.shape[1], f) for y in Y], sys)

    def precond(g):
        return [K(gk, b) for gk, b in zip(g, sys.bases)]

    from .operators import cholesky_orthonormalize
    Ys = [cholesky_orthonormalize(y, b)[0] for y, b in zip(Ys, sys.bases)]
    s = sys.omega * f * float(np.max(sys.wk))
    cg = CG(Ys, objective, energy_only, precond, 0.3 / s)
    for _ in range(nsteps):
        if not cg.step():
            break
    return cg


def protocol_B(Y, b, Veff, P, D, nsteps: int):
    """Band-energy minimization at fixed H for one k-point."""
    from .energy import band_energy_and_gradient
    from .operators import K

    def objective(Yl):
        E, g = band_energy_and_gradient(Yl[0], b, Veff, P, D)
        return E, [g]

    def energy_only(Yl):
        return objective(Yl)[0]

    def precond(g):
        return [K(g[0], b)]

    from .operators import cholesky_orthonormalize
    Y = cholesky_orthonormalize(Y, b)[0]
    cg = CG([Y], objective, energy_only, precond, 0.3 / b.omega)
    for _ in range(nsteps):
        if not cg.step():
            break
    return cg
