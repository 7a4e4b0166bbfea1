"""Learned initial density for SCF (form 4), driven through the C ABI.

Pipeline:
  1. training data: the superposition start density n0 and the converged
     density n_conv of every training geometry, from the library's own SCF
     (cells run together as batches: one launch per pass for the whole batch);
  2. training: the library's network kernels (forward, backward, Adam) on
     the resident (n0, n_conv) pairs;
  3. evaluation: on held-out geometries, SCF from the superposition density
     and from the learned density; per cell the number of iterations after
     which the energy stays within 1e-6 Ha/atom of the plain start's final
     energy, and the difference of the two final energies.

Every numerical step runs in libdftpp; this module sequences the calls.
Usage: python -m paper_1708_03621_amd.learned --train 512 --eval 64
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


class Runner:
    """SCF of a list of cells as one batch system (graph replay after the
    first iteration)."""

    def __init__(self, D, torch, ctx, n_inner=3, n_inner_first=3, graph=True):
        self.D, self.torch, self.ctx = D, torch, ctx
        self.dev = torch.device("cuda:0")
        self.n_inner, self.n_inner_first, self.graph = n_inner, n_inner_first, graph

    def system(self, cells):
        import workloads as W
        D = self.D
        descs = [dict(R=c.R, S=c.S, ecut=c.ecut, kpts=c.kpts, wk=c.wk, nb=c.nb, n_electrons=c.n_electrons, tau=c.tau,
                      Z=c.Z.astype(float), rc=c.rc, has_proj=c.has_proj.astype(int), rp=W.PROJ_RP, D=W.PROJ_D)
                 for c in cells]
        s = D.dpp_batch_create(self.ctx, descs, D.DPP_F64)
        D.dpp_set_graph_mode(s, self.graph)
        off, npw = D.dpp_system_layout(s)
        item0, foff, _ = D.dpp_system_cells(s)
        blocks = []
        for ci, c in enumerate(cells):
            blocks += W.initial_wavefunctions(c.y0_seed, [(c.nb, npw[k]) for k in range(item0[ci], item0[ci + 1])])
        Y = self.torch.from_numpy(np.concatenate([b.reshape(-1) for b in blocks])).to(self.dev)
        return s, Y, foff

    def start_densities(self, cells):
        """Superposition start densities of the cells, (ncells, S0, S1, S2)."""
        import workloads as W
        D = self.D
        s, _, foff = self.system(cells)
        D.dpp_scf_init(s, cells=[dict(tau=c.tau, Z=c.Z, sigma=W.START_SIGMA) for c in cells])
        n0 = self.torch.empty(int(foff[-1]), dtype=self.torch.float64, device=self.dev)
        D.dpp_system_copy_field(s, D.DPP_FIELD_NIN, n0)
        self.torch.cuda.synchronize()
        D.dpp_system_destroy(s)
        return n0.view((len(cells),) + tuple(cells[0].S))

    def scf(self, cells, n_start, max_iter=200, tol_atom=1e-10):
        """SCF of all cells from device start densities (ncells, S...);
        returns energies (iterations, ncells), the last n_out per cell and
        per cell whether it converged.  Stops once every cell changed by less
        than tol_atom per atom in two consecutive iterations."""
        D = self.D
        s, Y, _ = self.system(cells)
        D.dpp_scf_init(s, cells=[dict(d_n_start=n_start[i]) for i in range(len(cells))],
                       n_inner=self.n_inner, n_inner_first=self.n_inner_first)
        nat = np.array([c.nat for c in cells])
        E = []
        conv = np.zeros(len(cells), bool)
        for it in range(max_iter):
            e, _ = D.dpp_scf_iteration(s, Y)
            E.append([x["E_el"] for x in e])
            if it >= 2:
                a = np.abs(np.array(E[-1]) - np.array(E[-2])) / nat
                b = np.abs(np.array(E[-2]) - np.array(E[-3])) / nat
                conv = (a < tol_atom) & (b < tol_atom)
                if np.all(conv):
                    break
        nout = self.torch.empty(n_start.shape, dtype=self.torch.float64, device=self.dev)
        D.dpp_system_copy_field(s, D.DPP_FIELD_NOUT, nout)
        self.torch.cuda.synchronize()
        D.dpp_system_destroy(s)
        return np.array(E), nout, conv


def iterations_to(E, E_ref, nat, tol=1e-6):
    """First iteration (1-based) after which |E_i - E_ref| / nat < tol holds for good."""
    for i in range(len(E)):
        if all(abs(e - E_ref) / nat < tol for e in E[i:]):
            return i + 1
    return None


def run(n_train=512, n_eval=64, epochs=40, batch=8, lr=1e-3, n_inner_first=3, seed=502, max_iter=200,
        scf_batch=64, n_inner=3, log=_log):
    import torch

    import workloads as W
    from paper_1708_03621_amd import dftpp as D

    ctx = D.dpp_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    R = Runner(D, torch, ctx, n_inner=n_inner, n_inner_first=n_inner_first)
    train = W.config5("train", n_train)
    evals = W.config5("eval", n_eval)
    S = train[0].S
    omega = float(abs(np.linalg.det(train[0].R)))
    ne = float(train[0].n_electrons)
    nbar = ne / omega
    t0 = time.time()
    n0s, ncs, scf_iters = [], [], []
    for i in range(0, len(train), scf_batch):
        cells = train[i:i + scf_batch]
        n0 = R.start_densities(cells)
        E, nc, _ = R.scf(cells, n0, max_iter=max_iter)
        n0s.append(n0)
        ncs.append(nc)
        scf_iters.append(len(E))
        log(f"training data {i + len(cells)}/{len(train)} ({len(E)} SCF iterations)")
    n0_all = torch.cat(n0s).contiguous()
    nc_all = torch.cat(ncs).contiguous()
    t_data = time.time() - t0
    net = D.dpp_net_create(ctx, S, batch)
    D.dpp_net_set_params(net, W.net_flatten(W.net_init_params(501)))
    rng = np.random.default_rng(seed)
    losses = []
    t1 = time.time()
    for ep in range(epochs):
        order = rng.permutation(len(train)).astype(np.int32)
        losses.append(D.dpp_net_train_epoch(net, len(train), n0_all, nc_all, nbar, batch, lr, order))
        if (ep + 1) % 10 == 0:
            log(f"epoch {ep + 1}: loss {losses[-1]:.3e}")
    torch.cuda.synchronize()
    t_train = time.time() - t1
    # held-out evaluation: the same cells from both starts
    rows = []
    t2 = time.time()
    for i in range(0, len(evals), scf_batch):
        cells = evals[i:i + scf_batch]
        n0 = R.start_densities(cells)
        nl = torch.empty_like(n0)
        for j in range(len(cells)):
            D.dpp_net_predict_density(net, n0[j], ne, omega, nl[j])
        Ep, nconv, cp = R.scf(cells, n0, max_iter=max_iter)
        El, _, cl = R.scf(cells, nl, max_iter=max_iter)
        for j, c in enumerate(cells):
            E_ref = Ep[-1, j]
            l1 = float(torch.sum(torch.abs(nconv[j])))
            rows.append(dict(plain=iterations_to(Ep[:, j], E_ref, c.nat),
                             learned=iterations_to(El[:, j], E_ref, c.nat),
                             converged_plain=bool(cp[j]), converged_learned=bool(cl[j]),
                             dE_per_atom=abs(El[-1, j] - Ep[-1, j]) / c.nat, E=E_ref,
                             start_err_plain=float(torch.sum(torch.abs(n0[j] - nconv[j]))) / l1,
                             start_err_learned=float(torch.sum(torch.abs(nl[j] - nconv[j]))) / l1))
    t_eval = time.time() - t2
    D.dpp_net_destroy(net)
    ip = [r["plain"] for r in rows if r["plain"]]
    il = [r["learned"] for r in rows if r["learned"]]
    both = [r for r in rows if r["converged_plain"] and r["converged_learned"]]
    return dict(n_train=len(train), n_eval=len(evals), nb=train[0].nb, epochs=epochs, batch=batch, lr=lr,
                n_inner=n_inner, n_inner_first=n_inner_first, max_iter=max_iter,
                cells_converged_both=len(both),
                iters_plain_mean_converged=float(np.mean([r["plain"] for r in both])) if both else None,
                iters_learned_mean_converged=float(np.mean([r["learned"] for r in both])) if both else None,
                iters_saved_per_cell=[r["plain"] - r["learned"] for r in both],
                loss_first=losses[0], loss_last=losses[-1], train_data_s=t_data, train_s=t_train, eval_s=t_eval,
                scf_iters_train_batches=scf_iters,
                iters_plain_mean=float(np.mean(ip)) if ip else None,
                iters_learned_mean=float(np.mean(il)) if il else None,
                start_err_plain_mean=float(np.mean([r["start_err_plain"] for r in rows])),
                start_err_learned_mean=float(np.mean([r["start_err_learned"] for r in rows])),
                max_dE_per_atom=max(r["dE_per_atom"] for r in rows), rows=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--first", type=int, default=3, help="band-CG steps of the first SCF iteration")
    ap.add_argument("--inner", type=int, default=3, help="band-CG steps of every later SCF iteration")
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--scf-batch", type=int, default=64, help="cells per batched SCF system")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    res = run(args.train, args.eval, args.epochs, n_inner_first=args.first, max_iter=args.max_iter,
              scf_batch=args.scf_batch, n_inner=args.inner)
    js = json.dumps(res)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(js + "\n")
    print(js, flush=True)


if __name__ == "__main__":
    main()
