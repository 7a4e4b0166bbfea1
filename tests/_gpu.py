"""Shared helpers for the GPU parity tests (HIP library through the C ABI)."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class Device:
    """One library context on torch's current HIP stream."""

    def __init__(self):
        import torch
        from paper_1708_03621_amd import dftpp as D
        self.torch = torch
        self.D = D
        self.dev = torch.device("cuda:0")
        self.stream = torch.cuda.current_stream()
        self.ctx = D.dpp_ctx_create(0, self.stream.cuda_stream)

    def sync(self):
        self.torch.cuda.synchronize()

    def tensor(self, a, dtype=None):
        t = self.torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            t = t.to(dtype)
        return t.to(self.dev)

    def empty(self, shape, dtype):
        return self.torch.empty(shape, dtype=dtype, device=self.dev)

    def zeros(self, shape, dtype):
        return self.torch.zeros(shape, dtype=dtype, device=self.dev)

    def ws(self, nbytes):
        return self.torch.empty(max(int(nbytes), 256), dtype=self.torch.uint8, device=self.dev)

    def host(self, t):
        self.sync()
        return t.cpu().numpy()

    def field(self, sys_, which, S):
        """Copy of a system's internal real-space field to host."""
        t = self.torch.empty(tuple(S), dtype=self.torch.float64, device=self.dev)
        self.D.dpp_system_copy_field(sys_, which, t)
        return self.host(t)

    def grid(self, R, S):
        return self.D.dpp_grid_create(self.ctx, R, S)

    def basis(self, grid, k, ecut):
        return self.D.dpp_basis_create(grid, k, ecut)


def block_to_gpu(dev, C_math):
    """Oracle (npw, nb) block -> device band-major (nb, npw) complex128."""
    return dev.tensor(np.ascontiguousarray(C_math.T), dev.torch.complex128)


def block_from_gpu(dev, t):
    return dev.host(t).T.copy()


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)
