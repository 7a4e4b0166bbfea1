"""Learned initial density for SCF (form 4), driven through the C ABI.

Pipeline:
  1. training data: for each training geometry, the superposition start
     density n0 and the converged density n_conv from the library's own SCF;
  2. training: the library's network kernels (forward, backward, Adam) on
     the resident (n0, n_conv) pairs;
  3. evaluation: on held-out geometries, SCF iterations until the energy
     stays within 1e-6 Ha/atom of the converged energy, starting from the
     superposition density and from the learned density; the converged
     energies of both starts must agree.

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
    def __init__(self, D, torch, ctx, n_inner=3, n_inner_first=3):
        self.D, self.torch, self.ctx = D, torch, ctx
        self.dev = torch.device("cuda:0")
        self.n_inner, self.n_inner_first = n_inner, n_inner_first

    def system(self, cell):
        import workloads as W
        D = self.D
        s = D.dpp_system_create(self.ctx, cell.R, cell.S, cell.ecut, cell.kpts, cell.wk, cell.nb, cell.n_electrons,
                                cell.tau, cell.Z.astype(float), cell.rc, cell.has_proj.astype(int), W.PROJ_RP,
                                W.PROJ_D, D.DPP_F64)
        off, npw = D.dpp_system_layout(s, len(cell.kpts))
        blocks = W.initial_wavefunctions(cell.y0_seed, [(cell.nb, n) for n in npw])
        Y = self.torch.from_numpy(np.concatenate([b.reshape(-1) for b in blocks])).to(self.dev)
        return s, Y

    def start_density(self, cell):
        import workloads as W
        D = self.D
        g = D.dpp_grid_create(self.ctx, cell.R, cell.S)
        ws = self.torch.empty(D.dpp_grid_workspace_size(g), dtype=self.torch.uint8, device=self.dev)
        n0 = self.torch.empty(tuple(cell.S), dtype=self.torch.float64, device=self.dev)
        D.dpp_start_density(g, cell.tau, cell.Z.astype(float), W.START_SIGMA, n0, ws)
        self.torch.cuda.synchronize()
        D.dpp_grid_destroy(g)
        return n0

    def scf(self, cell, n_start, max_iter=80, tol_atom=1e-10):
        """SCF from a device start density; returns energies and the last n_out."""
        D = self.D
        s, Y = self.system(cell)
        D.dpp_scf_init(s, d_n_start=n_start, n_inner=self.n_inner, n_inner_first=self.n_inner_first)
        nk = len(cell.kpts)
        E = []
        for it in range(max_iter):
            e, _ = D.dpp_scf_iteration(s, Y, nk, cell.nb)
            E.append(e["E_el"])
            if it >= 2 and abs(E[-1] - E[-2]) / cell.nat < tol_atom and abs(E[-2] - E[-3]) / cell.nat < tol_atom:
                break
        nout = self.torch.empty(tuple(cell.S), dtype=self.torch.float64, device=self.dev)
        D.dpp_system_copy_field(s, D.DPP_FIELD_NOUT, nout)
        self.torch.cuda.synchronize()
        D.dpp_system_destroy(s)
        return E, nout


def iterations_to(E, E_ref, nat, tol=1e-6):
    """First iteration (1-based) after which |E_i - E_ref| / nat < tol holds for good."""
    for i in range(len(E)):
        if all(abs(e - E_ref) / nat < tol for e in E[i:]):
            return i + 1
    return None


def run(n_train=512, n_eval=64, epochs=40, batch=8, lr=1e-3, n_inner_first=3, seed=502, log=_log):
    import torch

    import workloads as W
    from paper_1708_03621_amd import dftpp as D

    ctx = D.dpp_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    R = Runner(D, torch, ctx, n_inner=3, n_inner_first=n_inner_first)
    train = W.config5("train", n_train)
    evals = W.config5("eval", n_eval)
    S = train[0].S
    omega = float(abs(np.linalg.det(train[0].R)))
    ne = float(train[0].n_electrons)
    nbar = ne / omega
    t0 = time.time()
    n0s, ncs, scf_iters = [], [], []
    for i, cell in enumerate(train):
        n0 = R.start_density(cell)
        E, nc = R.scf(cell, n0)
        n0s.append(n0)
        ncs.append(nc)
        scf_iters.append(len(E))
        if (i + 1) % 32 == 0:
            log(f"training data {i + 1}/{len(train)}")
    n0_all = torch.stack(n0s).contiguous()
    nc_all = torch.stack(ncs).contiguous()
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
    # held-out evaluation
    rows = []
    for cell in evals:
        n0 = R.start_density(cell)
        Ep, nconv = R.scf(cell, n0)
        nl = torch.empty_like(n0)
        D.dpp_net_predict_density(net, n0, ne, omega, nl)
        El, _ = R.scf(cell, nl)
        E_ref = Ep[-1]
        l1 = float(torch.sum(torch.abs(nconv)))
        rows.append(dict(plain=iterations_to(Ep, E_ref, cell.nat), learned=iterations_to(El, E_ref, cell.nat),
                         dE_per_atom=abs(El[-1] - Ep[-1]) / cell.nat, E=Ep[-1],
                         start_err_plain=float(torch.sum(torch.abs(n0 - nconv))) / l1,
                         start_err_learned=float(torch.sum(torch.abs(nl - nconv))) / l1))
    D.dpp_net_destroy(net)
    ip = [r["plain"] for r in rows if r["plain"]]
    il = [r["learned"] for r in rows if r["learned"]]
    return dict(n_train=len(train), n_eval=len(evals), epochs=epochs, batch=batch, lr=lr,
                n_inner=3, n_inner_first=n_inner_first,
                loss_first=losses[0], loss_last=losses[-1], train_data_s=t_data, train_s=t_train,
                scf_iters_train_mean=float(np.mean(scf_iters)),
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
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    res = run(args.train, args.eval, args.epochs, n_inner_first=args.first)
    js = json.dumps(res)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(js + "\n")
    print(js, flush=True)


if __name__ == "__main__":
    main()
