"""Build a library system (C ABI) and the matching oracle system from one
workloads.Cell, plus seeded initial wavefunctions in both layouts."""
import numpy as np

import workloads as W


def make_gpu_system(dev, cell, prec=0, with_local=True, with_projectors=True):
    D = dev.D
    Z = cell.Z.astype(float) if with_local else np.zeros(cell.nat)
    hp = cell.has_proj.astype(int) if with_projectors else np.zeros(cell.nat, int)
    sys_ = D.dpp_system_create(dev.ctx, cell.R, cell.S, cell.ecut, cell.kpts, cell.wk, cell.nb,
                               cell.n_electrons, cell.tau, Z, cell.rc, hp, W.PROJ_RP, W.PROJ_D, prec)
    off, npw = D.dpp_system_layout(sys_, len(cell.kpts))
    return sys_, off, npw


def packed_Y(dev, cell, npw):
    """Seeded Y0 (workloads generator) packed as the library layout."""
    blocks = W.initial_wavefunctions(cell.y0_seed, [(cell.nb, n) for n in npw])
    flat = np.concatenate([b.reshape(-1) for b in blocks])
    return dev.tensor(flat), blocks


def unpack(dev, Y, cell, off, npw):
    h = dev.host(Y)
    return [h[off[k]:off[k + 1]].reshape(cell.nb, npw[k]) for k in range(len(npw))]
