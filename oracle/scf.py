"""Self-consistent field iteration with Pulay mixing (FP64 oracle).

Sec. 2.1 names Pulay mixing for self-consistency; Sec. 2.2 contrasts SCF
with variational minimization.  One iteration, for input density n_in:
  1. V_eff = V_loc + V_H[n_in] + v_xc[n_in]
  2. per k: a fixed number of band-energy CG steps at that V_eff (CG state
     restarted every iteration, wavefunctions warm-started)
  3. subspace diagonalization: psi = Y R^{-1}, H~ = psi^dag H psi,
     H~ V = V diag(eps), Y <- psi V
  4. aufbau fillings over all (k, band) states, each holding 2 w_k
     electrons; a degenerate set (|d eps| < 1e-6 Ha) straddling the Fermi
     level shares the remaining electrons equally.  With a smearing width
     sigma instead Fermi-Dirac fillings 2 / (1 + exp((eps - mu) / sigma)),
     mu by bisection on the electron count, and the reported energy is the
     free energy E - sigma S (Table 1: smearing for metals)
  5. n_out from psi and the fillings; E_el evaluated with n_out
  6. Pulay (DIIS) mixing of n_in: history 8, alpha 0.5, first iteration
     linear n_in + alpha (n_out - n_in); later the residual combination
     sum_i c_i R_i of least norm with sum_i c_i = 1 gives
     n_in = sum_i c_i (n_in,i + alpha R_i).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from .energy import band_energies, density, potentials
from .minimize import protocol_B

DEGEN_TOL = 1e-6


def aufbau_fillings(eigs, wk, n_electrons: float, tol: float = DEGEN_TOL):
    """Fillings per k (list of arrays) from eigenvalues per k."""
    states = [(float(e), k, i) for k, ek in enumerate(eigs) for i, e in enumerate(ek)]
    states.sort(key=lambda s: (s[0], s[1], s[2]))
    fills = [np.zeros(len(ek)) for ek in eigs]
    remaining = float(n_electrons)
    j = 0
    while j < len(states) and remaining > 1e-12:
        e0 = states[j][0]
        grp = [states[j]]
        j += 1
        while j < len(states) and states[j][0] - e0 < tol:
            grp.append(states[j])
            j += 1
        cap = sum(2.0 * wk[k] for _, k, _ in grp)
        if cap <= remaining + 1e-12:
            for _, k, i in grp:
                fills[k][i] = 2.0
            remaining -= cap
        else:
            frac = remaining / cap
            for _, k, i in grp:
                fills[k][i] = 2.0 * frac
            remaining = 0.0
    if remaining > 1e-9:
        raise ValueError("not enough bands for the electron count")
    return fills


SMEAR_BRACKET = 40.0   # bisection bracket: [min eps - 40 sigma, max eps + 40 sigma]
SMEAR_ITERS = 200      # bisection halvings (the bracket stops shrinking in FP64 well before)


def fermi_fillings(eigs, wk, n_electrons: float, sigma: float):
    """Fermi-Dirac fillings of width sigma (hartree), spin-unpolarized:
    f = 2 / (1 + exp((eps - mu) / sigma)) with mu by bisection so that
    sum_k w_k sum_i f_ki = N_e.  Returns (fills per k, mu, S) with the entropy
    S = -2 sum_k w_k sum_i [g ln g + (1 - g) ln(1 - g)], g = f / 2; the SCF
    reports the free energy E - sigma S."""
    e = [np.asarray(ek, float) for ek in eigs]
    lo = min(float(ek.min()) for ek in e) - SMEAR_BRACKET * sigma
    hi = max(float(ek.max()) for ek in e) + SMEAR_BRACKET * sigma
    cap = sum(2.0 * wk[k] * len(ek) for k, ek in enumerate(e))
    if cap < n_electrons - 1e-9:
        raise ValueError("not enough bands for the electron count")

    def count(mu):  # exp overflows to inf far above mu: those states hold 0
        with np.errstate(over="ignore"):
            return sum(float(np.sum(2.0 * wk[k] / (1.0 + np.exp((ek - mu) / sigma)))) for k, ek in enumerate(e))

    for _ in range(SMEAR_ITERS):
        mid = 0.5 * (lo + hi)
        if count(mid) < n_electrons:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    fills, S = [], 0.0
    for k, ek in enumerate(e):
        x = (ek - mu) / sigma
        with np.errstate(over="ignore"):
            g = 1.0 / (1.0 + np.exp(x))       # occupation per spin
            gc = 1.0 / (1.0 + np.exp(-x))     # 1 - g without cancellation
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(g > 0, g * np.log(g), 0.0) + np.where(gc > 0, gc * np.log(gc), 0.0)
        S -= 2.0 * wk[k] * float(np.sum(t))
        fills.append(2.0 * g)
    return fills, mu, S


class Pulay:
    def __init__(self, omega: float, N: int, alpha: float = 0.5, history: int = 8):
        self.alpha = alpha
        self.maxh = history
        self.dV = omega / N
        self.hist = []

    def mix(self, n_in, n_out):
        R = n_out - n_in
        self.hist.append((n_in.copy(), R))
        if len(self.hist) > self.maxh:
            self.hist.pop(0)
        m = len(self.hist)
        if m == 1:
            return n_in + self.alpha * R
        A = np.zeros((m + 1, m + 1))
        for i in range(m):
            for j in range(m):
                A[i, j] = self.dV * float(np.sum(self.hist[i][1] * self.hist[j][1]))
        A[m, :m] = 1.0
        A[:m, m] = 1.0
        rhs = np.zeros(m + 1)
        rhs[m] = 1.0
        c = np.linalg.solve(A, rhs)[:m]
        out = np.zeros_like(n_in)
        for i in range(m):
            out += c[i] * (self.hist[i][0] + self.alpha * self.hist[i][1])
        return out


def subspace_rotate(Y, b, Veff, P, D):
    psi, _, _ = ops.cholesky_orthonormalize(Y, b)
    Hpsi = ops.apply_H(psi, b, Veff, P, D)
    Hs = psi.conj().T @ Hpsi
    Hs = 0.5 * (Hs + Hs.conj().T)
    eps, V = np.linalg.eigh(Hs)
    return psi @ V, eps


def scf(sys, Ys, n_in, n_iter: int, n_inner: int = 3, callback=None, etol_per_atom=None, n_inner_first=None,
        smearing=None):
    """Run protocol S; returns dict with energies per iteration, final Y, eigs, n.

    n_inner_first (default n_inner): band-CG steps of the first iteration, so
    that the bands can be converged in the start potential before mixing.
    smearing (hartree, default none): Fermi-Dirac fillings of that width
    instead of aufbau; the energies are then the free energies E - sigma S,
    and the result carries mu, the entropy term sigma S and the fillings."""
    Ys = [y.copy() for y in Ys]
    pulay = Pulay(sys.omega, sys.N)
    energies = []
    eigs = None
    n_out = None
    Veff_last = None
    for it in range(n_iter):
        Veff, _ = potentials(n_in, sys)
        new_Y, eigs = [], []
        for k, b in enumerate(sys.bases):
            steps = n_inner_first if (it == 0 and n_inner_first is not None) else n_inner
            cg = protocol_B(Ys[k], b, Veff, sys.P[k], sys.D, steps)
            Yk, ek = subspace_rotate(cg.Y[0], b, Veff, sys.P[k], sys.D)
            new_Y.append(Yk)
            eigs.append(ek)
        Ys = new_Y
        TS, mu = 0.0, None
        if smearing:
            fills, mu, S = fermi_fillings(eigs, sys.wk, sys.n_electrons, smearing)
            TS = smearing * S
        else:
            fills = aufbau_fillings(eigs, sys.wk, sys.n_electrons)
        n_out = density(Ys, fills, sys)
        _, parts = potentials(n_out, sys)
        Ekin, Enl = band_energies(Ys, fills, sys)
        E = Ekin + Enl + parts["E_loc"] + parts["E_H"] + parts["E_xc"] - TS
        energies.append(E)
        if callback is not None:
            callback(it, E, eigs, n_out)
        Veff_last = Veff
        n_in = pulay.mix(n_in, n_out)
        if etol_per_atom is not None and it > 0 and abs(energies[-1] - energies[-2]) < etol_per_atom * sys.nat:
            break
    return dict(energies=energies, Y=Ys, eigs=eigs, n_out=n_out, n_in=n_in, Veff=Veff_last, fills=fills, mu=mu,
                TS=TS)
