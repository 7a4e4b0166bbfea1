"""Ionic minimization (Table 1: ion optimization; Sec. 3: the example relaxes
the ionic positions before its solvated calculation), driven through the C ABI.

Energy E = E_el + E_ion of a converged SCF at the positions, force from
dpp_system_forces (local + nonlocal + ionic; Hellmann-Feynman at convergence).
Minimizer: nonlinear conjugate gradients on the positions (Polak-Ribiere,
restarted along the force when the direction stops descending); each line
minimization takes one trial step that moves the farthest-moving atom by
`trial` bohr and then the secant step to the zero of the directional
derivative g(a) = -F(tau + a d) . d, kept within [0.1, 4] trial steps.  Every
SCF starts from the superposition density at the new positions and warm
wavefunctions.

Every numerical step runs in libdftpp; this module sequences the calls.
"""
from __future__ import annotations

import numpy as np


class GpuCell:
    """One cell as a library system; energy_forces(tau) -> (E, F (nat, 3))."""

    def __init__(self, D, torch, ctx, cell, etol=1e-12, max_scf=300, start_sigma=None):
        import workloads as W
        self.D, self.torch, self.cell = D, torch, cell
        self.etol, self.max_scf = etol, max_scf
        self.sigma = W.START_SIGMA if start_sigma is None else start_sigma
        self.sys = D.dpp_system_create(ctx, cell.R, cell.S, cell.ecut, cell.kpts, cell.wk, cell.nb, cell.n_electrons,
                                       cell.tau, cell.Z.astype(float), cell.rc, cell.has_proj.astype(int), W.PROJ_RP,
                                       W.PROJ_D, D.DPP_F64)
        _, npw = D.dpp_system_layout(self.sys, len(cell.kpts))
        blocks = W.initial_wavefunctions(cell.y0_seed, [(cell.nb, n) for n in npw])
        self.Y = torch.from_numpy(np.concatenate([b.reshape(-1) for b in blocks])).to("cuda:0")
        self.tau = np.array(cell.tau, float)
        self.scf_iterations = []

    def energy_forces(self, tau):
        D, c = self.D, self.cell
        tau = np.asarray(tau, float)
        if not np.array_equal(tau, self.tau):
            D.dpp_system_set_positions(self.sys, tau)
            self.tau = tau.copy()
        D.dpp_scf_init(self.sys, tau, c.Z.astype(float), self.sigma)
        E_prev = None
        for it in range(self.max_scf):
            E, _ = D.dpp_scf_iteration(self.sys, self.Y, len(c.kpts), c.nb)
            E_el = E["E_el"]
            if E_prev is not None and abs(E_el - E_prev) < self.etol * c.nat:
                break
            E_prev = E_el
        self.scf_iterations.append(it + 1)
        F = [self.torch.zeros((c.nat, 3), dtype=self.torch.float64, device="cuda:0") for _ in range(3)]
        E_ion = D.dpp_system_forces(self.sys, self.Y, F[0], F[1], F[2], 1)[0]
        self.torch.cuda.synchronize()
        return E_el + E_ion, sum(f.cpu().numpy() for f in F)

    def close(self):
        self.D.dpp_system_destroy(self.sys)


def relax(energy_forces, tau0, ftol=1e-3, max_steps=40, trial=0.1):
    """Conjugate-gradient minimization of the energy over the positions."""
    tau = np.array(tau0, float)
    E, F = energy_forces(tau)
    hist = [(E, float(np.max(np.abs(F))))]
    d = F.copy()
    F_prev = None
    for _ in range(max_steps):
        if np.max(np.abs(F)) < ftol:
            break
        if F_prev is not None:
            beta = max(0.0, float(np.sum(F * (F - F_prev)) / np.sum(F_prev * F_prev)))
            d = F + beta * d
            if np.sum(F * d) <= 0.0:
                d = F.copy()
        g0 = -float(np.sum(F * d))
        at = trial / float(np.max(np.linalg.norm(d, axis=1)))
        _, Ft = energy_forces(tau + at * d)
        gt = -float(np.sum(Ft * d))
        a = at * g0 / (g0 - gt) if gt > g0 else 4.0 * at
        a = min(max(a, 0.1 * at), 4.0 * at)
        tau = tau + a * d
        F_prev = F
        E, F = energy_forces(tau)
        hist.append((E, float(np.max(np.abs(F)))))
    return dict(tau=tau, E=E, F=F, history=hist)
