"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds geometry, k-point lists, band counts and seeded random
numbers only.  It performs none of the method's arithmetic (no basis
construction, no transform, no potential): both sides receive the same
arrays from here and compute everything else themselves.

All random draws use ``numpy.random.default_rng(seed)``.  Random numbers
that the method consumes (initial wavefunction coefficients) are produced
here for a caller-supplied basis size, so each side builds its own basis and
asks for coefficients of the size it found.

Workloads (plane-wave DFT, atomic units: bohr, hartree):

* ``config1``: cubic cell L = 10, two Z=1 atoms at seeded uniform positions
  at least 1.5 bohr apart (minimum image), Ecut 8, grid 24^3, 4 bands,
  Gamma point only, local pseudopotential only.
* ``config2``: diamond-structure cubic cell a = 10.26, 8 atoms Z=4 with a
  Gaussian s-projector each, Ecut 12, grid 40^3, 16 bands, Gamma-centred
  2x2x2 k folding (8 k-points).
* ``config3``: 2x2x2 supercell of config2 (64 atoms) displaced by seeded
  N(0, 0.1^2) per Cartesian component, Gamma only, Ecut 15, grid 90^3,
  128 bands.
* ``config4``: 48 independent cubic cells with random edge, atom count,
  species, band count and k folding (batched throughput).
* ``config5``: config2 cell displaced by N(0, 0.3^2), 512 training and 64
  held-out geometries, 16 bands (learned initial density).
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Sequence, Tuple

import numpy as np

# Pseudopotential model parameters per valence charge Z (local erf radius
# r_c, and whether the species carries the Gaussian s-projector).
SPECIES = {
    1: dict(rc=0.5, projector=False),
    4: dict(rc=0.7, projector=True),
}
PROJ_RP = 1.0      # Gaussian projector width (bohr)
PROJ_D = 2.0       # projector coupling (hartree)
START_SIGMA = 1.0  # width of the superposition-of-Gaussians start density


@dataclasses.dataclass
class Cell:
    """One periodic system: everything a solver needs, no derived arithmetic."""
    name: str
    R: np.ndarray             # (3,3) lattice vectors as COLUMNS (bohr)
    tau: np.ndarray           # (nat,3) Cartesian positions (bohr)
    Z: np.ndarray             # (nat,) valence charges
    ecut: float               # hartree
    S: Tuple[int, int, int]   # FFT box
    nb: int                   # bands per k-point
    kpts: np.ndarray          # (nk,3) reduced k-points
    wk: np.ndarray            # (nk,) k weights, sum 1
    y0_seed: int              # seed for the initial wavefunctions

    @property
    def nat(self) -> int:
        return len(self.Z)

    @property
    def n_electrons(self) -> int:
        return int(np.sum(self.Z))

    @property
    def rc(self) -> np.ndarray:
        return np.array([SPECIES[int(z)]["rc"] for z in self.Z], float)

    @property
    def has_proj(self) -> np.ndarray:
        return np.array([SPECIES[int(z)]["projector"] for z in self.Z], bool)


def initial_wavefunctions(seed: int, shapes: Sequence[Tuple[int, int]]) -> List[np.ndarray]:
    """Complex128 coefficients, Re and Im i.i.d. N(0,1), one array per k-point.

    ``shapes`` lists (nb, npw) per k-point in k order; the returned arrays are
    band-major (nb, npw) in canonical sphere order.  One generator stream
    covers all k-points: for each k, the real block then the imaginary block.
    """
    rng = np.random.default_rng(seed)
    out = []
    for nb, npw in shapes:
        re = rng.standard_normal((nb, npw))
        im = rng.standard_normal((nb, npw))
        out.append(re + 1j * im)
    return out


def _min_image_ok(frac: np.ndarray, R: np.ndarray, dmin: float) -> bool:
    n = len(frac)
    for a in range(n):
        for b in range(a + 1, n):
            d = frac[a] - frac[b]
            d -= np.round(d)
            # search neighbouring images as well (exact for any cell shape
            # whose reduced minimum image lies within one shell)
            best = np.inf
            for s in itertools.product((-1, 0, 1), repeat=3):
                best = min(best, float(np.linalg.norm(R @ (d + np.array(s)))))
            if best < dmin:
                return False
    return True


def _uniform_positions(rng, R, nat, dmin=1.5, max_tries=100000):
    for _ in range(max_tries):
        frac = rng.random((nat, 3))
        if _min_image_ok(frac, R, dmin):
            return (R @ frac.T).T
    raise RuntimeError("could not place atoms")


def gamma_centred_kpoints(fold: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Gamma-centred folding: k = (i0/f0, i1/f1, i2/f2), lexicographic, equal weights."""
    ks = [np.array([i / fold[0], j / fold[1], l / fold[2]])
          for i in range(fold[0]) for j in range(fold[1]) for l in range(fold[2])]
    k = np.array(ks, float)
    return k, np.full(len(k), 1.0 / len(k))


DIAMOND_FRAC = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


def config1() -> Cell:
    L = 10.0
    R = np.eye(3) * L
    rng = np.random.default_rng(101)
    tau = _uniform_positions(rng, R, 2)
    k, w = gamma_centred_kpoints((1, 1, 1))
    return Cell("config1", R, tau, np.array([1, 1]), 8.0, (24, 24, 24), 4, k, w, 102)


def diamond_cell(displace_sigma: float = 0.0, seed: int | None = None, name="config2",
                 reject_below: float | None = None, nb: int = 16) -> Cell:
    a = 10.26
    R = np.eye(3) * a
    base = (R @ DIAMOND_FRAC.T).T
    if displace_sigma > 0:
        rng = np.random.default_rng(seed)
        while True:
            tau = base + rng.normal(0.0, displace_sigma, base.shape)
            if reject_below is None or _min_image_ok((np.linalg.inv(R) @ tau.T).T, R, reject_below):
                break
    else:
        tau = base.copy()
    k, w = gamma_centred_kpoints((2, 2, 2))
    return Cell(name, R, tau, np.full(8, 4), 12.0, (40, 40, 40), nb, k, w, 201)


def config2() -> Cell:
    return diamond_cell()


def config3() -> Cell:
    a = 10.26
    L = 2 * a
    R = np.eye(3) * L
    frac = []
    for i, j, l in itertools.product(range(2), repeat=3):
        for f in DIAMOND_FRAC:
            frac.append((f + np.array([i, j, l])) / 2.0)
    frac = np.array(frac)
    rng = np.random.default_rng(301)
    tau = (R @ frac.T).T + rng.normal(0.0, 0.1, (64, 3))
    k, w = gamma_centred_kpoints((1, 1, 1))
    return Cell("config3", R, tau, np.full(64, 4), 15.0, (90, 90, 90), 128, k, w, 302)


def smooth235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def config4() -> List[Cell]:
    """48 cells for the batched-throughput workload (seed 401, Y0 seeds 402+c)."""
    rng = np.random.default_rng(401)
    ecut = 10.0
    folds = [(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2)]
    cells = []
    for c in range(48):
        L = float(rng.uniform(8.0, 14.0))
        R = np.eye(3) * L
        nat = int(rng.integers(2, 17))
        Z = rng.choice([1, 4], size=nat)
        tau = _uniform_positions(rng, R, nat)
        # box: smallest 2/3/5-smooth size holding products of sphere functions
        nmax = int(math.floor(math.sqrt(2 * ecut) * L / (2 * math.pi)))
        s = max(24, 4 * nmax + 1)
        while not smooth235(s):
            s += 1
        s = min(s, 48)
        ne = int(np.sum(Z))
        nb = max(int(rng.integers(4, 33)), (ne + 1) // 2)
        fold = folds[int(rng.integers(0, 4))]
        k, w = gamma_centred_kpoints(fold)
        cells.append(Cell(f"config4_cell{c}", R, tau, Z.astype(int), ecut, (s, s, s), nb, k, w, 402 + c))
    return cells


CONFIG5_NB = 16


def config5(split: str = "train", count: int | None = None) -> List[Cell]:
    """Displaced diamond cells: seeds 5000-5511 (train) or 6000-6063 (held out).

    16 bands per k-point (N_e / 2): with empty bands some displaced cells put
    two levels within the degeneracy width of the Fermi level and their SCF
    never settles under sharp fillings; with exactly the occupied count every
    cell converges."""
    if split == "train":
        seeds = range(5000, 5512)
    elif split == "eval":
        seeds = range(6000, 6064)
    else:
        raise ValueError(split)
    seeds = list(seeds)[: count if count is not None else None]
    return [diamond_cell(0.3, s, name=f"config5_{split}_{s}", reject_below=1.5, nb=CONFIG5_NB) for s in seeds]


def tiny_cell(nat=2, L=6.0, ecut=3.0, S=(12, 12, 12), nb=3, Z=(1, 1), seed=7,
              fold=(1, 1, 1), R=None) -> Cell:
    """Small cell for fast CPU self-checks and parity cases (non-cubic R allowed)."""
    R = np.eye(3) * L if R is None else np.asarray(R, float)
    rng = np.random.default_rng(seed)
    tau = _uniform_positions(rng, R, nat, dmin=1.0)
    k, w = gamma_centred_kpoints(fold)
    return Cell(f"tiny{seed}", R, tau, np.array(Z[:nat]), ecut, tuple(S), nb, k, w, seed + 1)


def random_potential(seed: int, S: Sequence[int], scale: float = 0.5) -> np.ndarray:
    """Seeded smooth-ish real field on the box (for operator parity cases)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(tuple(S))


def random_density(seed: int, S: Sequence[int], mean: float = 0.05) -> np.ndarray:
    """Seeded positive field on the box (for LDA/Hartree parity cases)."""
    rng = np.random.default_rng(seed)
    return mean * rng.gamma(2.0, 0.5, tuple(S))


NET_CHANNELS = (1, 16, 16, 16, 1)


def net_init_params(seed: int = 501):
    """Seeded initial weights of the learned-density network as a list of
    (W, b) per layer, W of shape (co, ci, 3, 3, 3): N(0, 2 / (ci * 27)) draws
    (the output layer scaled by 0.1 so the first correction is small), zero
    biases.  Random numbers only; both the oracle and the library start here."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(4):
        ci, co = NET_CHANNELS[l], NET_CHANNELS[l + 1]
        std = math.sqrt(2.0 / (ci * 27)) * (0.1 if l == 3 else 1.0)
        params.append((rng.normal(0.0, std, (co, ci, 3, 3, 3)), np.zeros(co)))
    return params


def net_flatten(params) -> np.ndarray:
    """Flat float32 vector in the library's order: W1, b1, W2, b2, W3, b3, W4, b4."""
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params]).astype(np.float32)


# ------------------------------------------------------------- LinearPCM inputs
# The solvation model takes eps(r) and rho(r) as given (the paper leaves the
# cavity's construction out); these inputs follow the common density-based
# cavity: eps = 1 + (eps_b - 1) s(n), s(n) = erfc(ln(n / n_c) / (sigma sqrt 2)) / 2,
# water-like eps_b = 78.4, n_c = 7e-4 bohr^-3, sigma = 0.6.  rho = ions
# (Gaussians of width 0.6 bohr, charge Z) minus electrons (Gaussians of width
# 1 bohr, Z electrons per atom): neutral up to sampling.
PCM_EPS_B, PCM_NC, PCM_SIGMA = 78.4, 7e-4, 0.6
PCM_ION_WIDTH, PCM_EL_WIDTH = 0.6, 1.0


def gaussians_on_box(R, S, tau, q, width):
    """sum_a q_a exp(-|r - tau_a|^2 / (2 w^2)) / (2 pi w^2)^(3/2), minimum image."""
    R = np.asarray(R, float)
    grids = np.meshgrid(*[np.arange(s) / s for s in S], indexing="ij")
    frac = np.stack(grids, axis=-1)
    out = np.zeros(tuple(S))
    Rinv = np.linalg.inv(R)
    norm = (2.0 * np.pi * width * width) ** -1.5
    for a in range(len(tau)):
        d = frac - Rinv @ np.asarray(tau[a], float)
        d -= np.round(d)
        r = d @ R.T
        out += q[a] * norm * np.exp(-np.sum(r * r, axis=-1) / (2.0 * width * width))
    return out


def pcm_case(kind: str = "small"):
    """Seeded LinearPCM input: dict(R, S, tau, Z, n, eps, rho).
    small: cubic 10 bohr, (20, 24, 25), two atoms; skew: a sheared cell,
    (24, 25, 27), three atoms; config3: config 3's cell and 90^3 grid with the
    8-atom diamond cube of its first octant centred in the box (a cluster in
    the dielectric)."""
    from scipy.special import erfc
    if kind == "small":
        R = np.eye(3) * 10.0
        S = (20, 24, 25)
        tau = np.array([[4.4, 5.1, 5.0], [5.9, 4.8, 5.3]])
        Z = np.array([4.0, 1.0])
    elif kind == "skew":
        R = np.array([[11.0, 0.8, 0.0], [0.0, 10.4, 0.9], [0.6, 0.0, 11.3]])
        S = (24, 25, 27)
        rng = np.random.default_rng(41)
        tau = R @ np.array([0.5, 0.5, 0.5]) + rng.normal(0.0, 0.9, (3, 3))
        Z = np.array([4.0, 1.0, 1.0])
    elif kind == "config3":
        c3 = config3()
        R, S = c3.R, c3.S
        a = R[0, 0] / 2.0
        tau = DIAMOND_FRAC * a + (np.diag(R) - a) / 2.0
        Z = np.full(len(tau), 4.0)
    else:
        raise ValueError(kind)
    n = gaussians_on_box(R, S, tau, Z, PCM_EL_WIDTH)
    s = 0.5 * erfc(np.log(np.maximum(n, 1e-300) / PCM_NC) / (PCM_SIGMA * np.sqrt(2.0)))
    eps = 1.0 + (PCM_EPS_B - 1.0) * s
    rho = gaussians_on_box(R, S, tau, Z, PCM_ION_WIDTH) - n
    return dict(R=np.asarray(R, float), S=tuple(S), tau=tau, Z=Z, n=n, eps=eps, rho=rho)
