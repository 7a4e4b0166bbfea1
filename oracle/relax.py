"""Ionic minimization with the oracle's SCF and forces (FP64; test
infrastructure only).

Table 1 lists ion optimization and Sec. 3's example relaxes the positions;
the paper does not fix the minimizer, so this one is the library's reading
written out plainly: E = E_el + E_ion of an SCF converged until one energy
change per atom falls below etol; F = local + nonlocal + ionic forces (Hellmann-
Feynman); Polak-Ribiere conjugate gradients on the positions (beta clipped at
0, restarted along F when F . d <= 0); per line one trial step of `trial`
bohr for the farthest-moving atom, then the secant zero of
g(a) = -F(tau + a d) . d, clipped to [0.1, 4] trial steps (4 trial steps if
g did not rise).  Each SCF starts from the superposition density at the new
positions and the previous orthonormal wavefunctions.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import energy as oe
from . import forces as of
from . import scf as oscf


def energy_forces(cell, etol=1e-12, max_scf=300, sigma=None):
    """A function tau -> (E, F) for the cell's species, box and cutoff."""
    import workloads as W
    sig = W.START_SIGMA if sigma is None else sigma
    state = {}

    def ef(tau):
        c = dataclasses.replace(cell, tau=np.array(tau, float))
        s = oe.build_system(c)
        Ys = state.get("Y")
        if Ys is None:
            blocks = W.initial_wavefunctions(c.y0_seed, [(c.nb, b.npw) for b in s.bases])
            Ys = [b.T.copy() for b in blocks]
        res = oscf.scf(s, Ys, oe.start_density(c, sig), max_scf, etol_per_atom=etol)
        state["Y"] = res["Y"]
        fills = oscf.aufbau_fillings(res["eigs"], s.wk, s.n_electrons)
        F = of.local_forces(c.R, c.S, c.tau, c.Z, c.rc, res["n_out"])
        F = F + of.nonlocal_forces(s.bases, s.wk, res["Y"], fills, c.tau, c.has_proj, W.PROJ_RP, W.PROJ_D)
        E_ion, F_ion = of.ewald(c.R, c.tau, c.Z)
        return res["energies"][-1] + E_ion, F + F_ion

    return ef


def relax(ef, tau0, ftol=1e-3, max_steps=40, trial=0.1):
    tau = np.array(tau0, float)
    E, F = ef(tau)
    history = [(E, float(np.abs(F).max()))]
    d, F_old = F.copy(), None
    for _ in range(max_steps):
        if np.abs(F).max() < ftol:
            break
        if F_old is not None:
            beta = max(0.0, float((F * (F - F_old)).sum() / (F_old * F_old).sum()))
            d = F + beta * d
            if (F * d).sum() <= 0.0:
                d = F.copy()
        g0 = -float((F * d).sum())
        a_t = trial / float(np.sqrt((d * d).sum(axis=1)).max())
        _, F_t = ef(tau + a_t * d)
        g_t = -float((F_t * d).sum())
        a = a_t * g0 / (g0 - g_t) if g_t > g0 else 4.0 * a_t
        a = float(np.clip(a, 0.1 * a_t, 4.0 * a_t))
        tau = tau + a * d
        F_old = F
        E, F = ef(tau)
        history.append((E, float(np.abs(F).max())))
    return dict(tau=tau, E=E, F=F, history=history)
