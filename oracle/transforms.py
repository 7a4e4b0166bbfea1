"""The Fourier operators I, I^dag, J, J^dag (Sec. 2.1: I and J transform
between reciprocal and real space, using FFTs).

Conventions (DFT++, unnormalized I):
  (I C)_j     = sum_G C_G exp(+i G.r_j)          sphere -> box
  (I^dag X)_G = sum_j X_j exp(-i G.r_j)          box -> sphere
  J x         = FFT(x) / N                       box -> box, J = I^{-1}
  J^dag y     = IFFT(y)                           (NumPy normalization)
so I^dag I = N on the sphere and J I = 1 on full-box fields.  r_j are the
grid points R (j0/S0, j1/S1, j2/S2); G.r_j = 2 pi n.(j/S).
The library FFT (numpy.fft) serves as the DFT step; tests pin it against
explicit sums.
"""
from __future__ import annotations

import numpy as np

from .basis import Basis


def scatter(C: np.ndarray, b: Basis) -> np.ndarray:
    """Place sphere coefficients (npw,) into a zero box of shape S."""
    box = np.zeros(int(np.prod(b.S)), complex)
    box[b.index] = C
    return box.reshape(b.S)


def I(C: np.ndarray, b: Basis) -> np.ndarray:
    """Sphere -> grid. C is (npw,) or (npw, nb); returns S or (nb,)+S."""
    if C.ndim == 1:
        return b.N * np.fft.ifftn(scatter(C, b))
    return np.stack([I(C[:, i], b) for i in range(C.shape[1])])


def Idag(X: np.ndarray, b: Basis) -> np.ndarray:
    """Grid -> sphere (adjoint of I). X is S or (nb,)+S; returns (npw,) or (npw, nb)."""
    if X.ndim == 3:
        return np.fft.fftn(X).reshape(-1)[b.index]
    return np.stack([Idag(X[i], b) for i in range(X.shape[0])], axis=1)


def J(x: np.ndarray) -> np.ndarray:
    return np.fft.fftn(x) / x.size


def Jdag(y: np.ndarray) -> np.ndarray:
    return np.fft.ifftn(y)


def I_full(y: np.ndarray) -> np.ndarray:
    """Full-box reciprocal -> real (inverse of J)."""
    return y.size * np.fft.ifftn(y)


def Idag_full(x: np.ndarray) -> np.ndarray:
    return np.fft.fftn(x)
