"""Plane-wave basis: G-sphere per k-point and the box frequency map.

Sec. 2.1 (GridInfo: the plane-wave grid and its Fourier transforms).  For a
Bloch vector k (reduced coordinates) the basis holds every reciprocal
lattice vector G = B n, n integer, with kinetic energy |k+G|^2/2 <= Ecut,
evaluated in FP64.  Canonical order is lexicographic on (n0, n1, n2), each
ascending.  Each sphere point maps to the linear box index
(i0*S1 + i1)*S2 + i2 with i_d = n_d mod S_d.

Full-box fields use the frequency map m -> n = m if m < S/2 else m - S
(for even S the Nyquist index S/2 maps to -S/2).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def reciprocal_basis(R: np.ndarray) -> np.ndarray:
    """B = 2 pi R^{-T}: columns b_i with b_i . a_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(R, float)).T


def cell_volume(R: np.ndarray) -> float:
    return float(abs(np.linalg.det(np.asarray(R, float))))


@dataclasses.dataclass
class Basis:
    R: np.ndarray
    S: tuple
    k: np.ndarray          # reduced k-point
    ecut: float
    n: np.ndarray          # (npw, 3) integer Miller indices, canonical order
    index: np.ndarray      # (npw,) linear box index
    kG: np.ndarray         # (npw, 3) Cartesian k+G
    kG2: np.ndarray        # (npw,) |k+G|^2

    @property
    def npw(self) -> int:
        return len(self.index)

    @property
    def omega(self) -> float:
        return cell_volume(self.R)

    @property
    def N(self) -> int:
        return int(np.prod(self.S))


def gsphere(R, S, k_red, ecut) -> Basis:
    """Enumerate the G-sphere of k in canonical order (Sec. 2.1, GridInfo)."""
    R = np.asarray(R, float)
    S = tuple(int(s) for s in S)
    B = reciprocal_basis(R)
    k = np.asarray(k_red, float)
    gmax = np.sqrt(2.0 * ecut)
    # n_d + k_d = a_d . (k+G) / 2pi, so |n_d + k_d| <= gmax |a_d| / 2pi
    ranges = []
    for d in range(3):
        ext = gmax * np.linalg.norm(R[:, d]) / (2.0 * np.pi)
        lo = int(np.floor(-ext - k[d])) - 1
        hi = int(np.ceil(ext - k[d])) + 1
        ranges.append(np.arange(lo, hi + 1))
    n0, n1, n2 = np.meshgrid(*ranges, indexing="ij")
    n = np.stack([n0.ravel(), n1.ravel(), n2.ravel()], axis=1)  # lexicographic
    kG = (n + k) @ B.T
    kG2 = np.sum(kG * kG, axis=1)
    keep = 0.5 * kG2 <= ecut
    n, kG, kG2 = n[keep], kG[keep], kG2[keep]
    for d in range(3):
        if n.size and (n[:, d].max() - n[:, d].min() + 1) > S[d]:
            raise ValueError("G-sphere does not fit in the FFT box along axis %d" % d)
    i = np.mod(n, np.array(S))
    index = (i[:, 0] * S[1] + i[:, 1]) * S[2] + i[:, 2]
    return Basis(R, S, k, float(ecut), n.astype(np.int64), index.astype(np.int64), kG, kG2)


def box_frequencies(S) -> np.ndarray:
    """Integer frequency n for every box point, shape S + (3,)."""
    axes = []
    for s in S:
        m = np.arange(s)
        axes.append(np.where(m < s / 2.0, m, m - s))
    f0, f1, f2 = np.meshgrid(*axes, indexing="ij")
    return np.stack([f0, f1, f2], axis=-1)


def box_G(R, S) -> np.ndarray:
    """Cartesian G for every box point under the frequency map, shape S + (3,)."""
    return box_frequencies(S) @ reciprocal_basis(R).T


def box_G2(R, S) -> np.ndarray:
    G = box_G(R, S)
    return np.sum(G * G, axis=-1)
