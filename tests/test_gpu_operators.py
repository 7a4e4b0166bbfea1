"""GPU parity of the DFT++ operators against the FP64 oracle, through the C ABI.

Cases span several tiles and ragged tails (odd box sizes, non-cubic cells,
k != 0, band counts that are not multiples of 16) plus the workload shapes.
Tolerances: FP64 paths 1e-11 relative to the largest output magnitude (the
kernels and NumPy differ only in summation order, ~1e-15 per term over
<= 1e5 terms); FP32 FFT paths 2e-5 relative.
"""
import numpy as np
import pytest

import workloads as W
from oracle import basis as ob, energy as oe, operators as oo, transforms as ot, xc as oxc
from tests._gpu import Device, block_from_gpu, block_to_gpu, log, rel_err

pytestmark = pytest.mark.gpu

NONCUBIC = np.array([[7.0, 0.5, 0.0], [0.0, 6.6, 0.7], [0.4, 0.0, 7.3]])


@pytest.fixture(scope="module")
def dev():
    return Device()


def _cases():
    c1, c2, c3 = W.config1(), W.config2(), W.config3()
    return [
        ("noncubic_k", NONCUBIC, (15, 16, 18), np.array([0.25, -0.5, 0.1]), 4.0),
        ("cfg1", c1.R, c1.S, c1.kpts[0], c1.ecut),
        ("cfg2_k0", c2.R, c2.S, c2.kpts[0], c2.ecut),
        ("cfg2_k7", c2.R, c2.S, c2.kpts[7], c2.ecut),
        ("cfg3", c3.R, c3.S, c3.kpts[0], c3.ecut),
    ]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_gsphere(dev, case):
    name, R, S, k, ecut = case
    log(f"gsphere {name}")
    ref = ob.gsphere(R, S, k, ecut)
    g = dev.grid(R, S)
    b = dev.basis(g, k, ecut)
    npw, ext = dev.D.dpp_basis_info(b)
    assert npw == ref.npw
    assert ext == [ref.n[:, 0].min(), ref.n[:, 0].max(), ref.n[:, 1].min(), ref.n[:, 1].max(),
                   ref.n[:, 2].min(), ref.n[:, 2].max()]
    idx = dev.zeros(npw, dev.torch.int32)
    kg2 = dev.zeros(npw, dev.torch.float64)
    dev.D.dpp_basis_export(b, idx, kg2)
    assert np.array_equal(dev.host(idx), ref.index)
    assert rel_err(dev.host(kg2), ref.kG2) < 1e-14


def test_basis_rejects_box_too_small(dev):
    g = dev.grid(np.eye(3) * 10.0, (8, 8, 8))
    with pytest.raises(dev.D.DppError):
        dev.basis(g, np.zeros(3), 8.0)


@pytest.mark.parametrize("case", _cases()[:4], ids=lambda c: c[0])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_I_and_Idag(dev, case, prec):
    name, R, S, k, ecut = case
    log(f"I/Idag {name} prec={prec}")
    torch = dev.torch
    ref = ob.gsphere(R, S, k, ecut)
    g = dev.grid(R, S)
    b = dev.basis(g, k, ecut)
    nb = 5
    rng = np.random.default_rng(11)
    C = rng.standard_normal((ref.npw, nb)) + 1j * rng.standard_normal((ref.npw, nb))
    cdt = torch.complex128 if prec == 0 else torch.complex64
    Cg = block_to_gpu(dev, C).to(cdt)
    out = dev.empty((nb,) + tuple(S), cdt)
    ws = dev.ws(dev.D.dpp_workspace_size(b, nb, prec))
    dev.D.dpp_I(b, nb, Cg, ref.npw, out, prec, ws)
    tol = 1e-12 if prec == 0 else 2e-6
    assert rel_err(dev.host(out), ot.I(C, ref)) < tol
    X = rng.standard_normal((nb,) + tuple(S)) + 1j * rng.standard_normal((nb,) + tuple(S))
    Xg = dev.tensor(X, cdt)
    Co = dev.zeros((nb, ref.npw), cdt)
    dev.D.dpp_Idag(b, nb, Xg, Co, ref.npw, 0, prec, ws)
    assert rel_err(block_from_gpu(dev, Co), ot.Idag(X, ref)) < tol
    # accumulate mode adds on top
    dev.D.dpp_Idag(b, nb, Xg, Co, ref.npw, 1, prec, ws)
    assert rel_err(block_from_gpu(dev, Co), 2 * ot.Idag(X, ref)) < tol


def test_J_Jdag(dev):
    log("J/Jdag")
    R, S = NONCUBIC, (15, 16, 18)
    g = dev.grid(R, S)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2,) + S) + 1j * rng.standard_normal((2,) + S)
    xg = dev.tensor(x, dev.torch.complex128)
    y = dev.empty((2,) + S, dev.torch.complex128)
    ws = dev.ws(dev.D.dpp_grid_workspace_size(g))
    dev.D.dpp_J(g, 2, xg, y, ws)
    assert rel_err(dev.host(y), np.stack([ot.J(x[0]), ot.J(x[1])])) < 1e-13
    dev.D.dpp_Jdag(g, 2, xg, y, ws)
    assert rel_err(dev.host(y), np.stack([ot.Jdag(x[0]), ot.Jdag(x[1])])) < 1e-13


def _ham_case(name):
    if name == "tiny_proj_k":
        cell = W.tiny_cell(nat=3, L=7.0, ecut=4.0, S=(16, 15, 18), Z=(4, 1, 4), fold=(2, 2, 1),
                           R=NONCUBIC)
        return cell, 3, 7
    if name == "cfg1":
        return W.config1(), 0, 4
    if name == "cfg2":
        return W.config2(), 7, 16
    if name == "cfg3":
        return W.config3(), 0, 8
    raise KeyError(name)


@pytest.mark.parametrize("name", ["tiny_proj_k", "cfg1", "cfg2", "cfg3"])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_apply_H(dev, name, prec):
    log(f"apply_H {name} prec={prec}")
    cell, kidx, nb = _ham_case(name)
    sys_ = oe.build_system(cell)
    ref = sys_.bases[kidx]
    Veff = sys_.Vloc + W.random_potential(5, cell.S, 0.2)
    rng = np.random.default_rng(17)
    C = rng.standard_normal((ref.npw, nb)) + 1j * rng.standard_normal((ref.npw, nb))
    HC_ref = oo.apply_H(C, ref, Veff, sys_.P[kidx], sys_.D)
    g = dev.grid(cell.R, cell.S)
    b = dev.basis(g, cell.kpts[kidx], cell.ecut)
    ham = dev.D.dpp_ham_create(b, cell.tau, cell.has_proj.astype(int), W.PROJ_RP, W.PROJ_D)
    Vg = dev.tensor(Veff, dev.torch.float64)
    dev.D.dpp_ham_set_potential(ham, Vg)
    Cg = block_to_gpu(dev, C)
    HCg = dev.empty((nb, ref.npw), dev.torch.complex128)
    ws = dev.ws(dev.D.dpp_workspace_size(b, nb, prec))
    dev.D.dpp_apply_H(ham, nb, Cg, ref.npw, HCg, ref.npw, prec, ws)
    tol = 1e-11 if prec == 0 else 2e-5
    assert rel_err(block_from_gpu(dev, HCg), HC_ref) < tol


def test_diagonal_operators(dev):
    log("O/L/K")
    ref = ob.gsphere(NONCUBIC, (15, 16, 18), np.array([0.25, -0.5, 0.1]), 4.0)
    g = dev.grid(NONCUBIC, (15, 16, 18))
    b = dev.basis(g, ref.k, 4.0)
    rng = np.random.default_rng(2)
    C = rng.standard_normal((ref.npw, 3)) + 1j * rng.standard_normal((ref.npw, 3))
    Cg = block_to_gpu(dev, C)
    out = dev.empty((3, ref.npw), dev.torch.complex128)
    for fn, ofn in [(dev.D.dpp_O, oo.O), (dev.D.dpp_L, oo.L), (dev.D.dpp_K, oo.K)]:
        fn(b, 3, Cg, ref.npw, out, ref.npw)
        assert rel_err(block_from_gpu(dev, out), ofn(C, ref)) < 1e-15


@pytest.mark.parametrize("nbA,nbB,npw", [(1, 1, 7), (5, 3, 700), (16, 16, 2134), (33, 20, 1045),
                                        (128, 128, 23847), (8, 128, 23847)])
def test_overlap(dev, nbA, nbB, npw):
    log(f"overlap {nbA}x{nbB} npw={npw}")
    L = (npw / 1.51) ** (1 / 3) * 1.0
    # a basis with at least npw points; use its first npw coefficients via ld
    g = dev.grid(np.eye(3) * 20.52, (90, 90, 90))
    b = dev.basis(g, np.zeros(3), 15.0)
    nfull, _ = dev.D.dpp_basis_info(b)
    rng = np.random.default_rng(nbA * 100 + nbB)
    A = rng.standard_normal((nbA, nfull)) + 1j * rng.standard_normal((nbA, nfull))
    B = rng.standard_normal((nbB, nfull)) + 1j * rng.standard_normal((nbB, nfull))
    U = dev.empty((nbA, nbB), dev.torch.complex128)
    ws = dev.ws(2 ** 26)
    dev.D.dpp_overlap(b, nbA, dev.tensor(A), nfull, nbB, dev.tensor(B), nfull, 2.5, U, ws)
    ref = 2.5 * A.conj() @ B.T
    assert rel_err(dev.host(U), ref) < 1e-12


@pytest.mark.parametrize("nbX,nbO", [(1, 1), (5, 3), (16, 16), (64, 128), (128, 128), (128, 130)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_rotate(dev, nbX, nbO, beta):
    log(f"rotate {nbX}->{nbO} beta={beta}")
    g = dev.grid(np.eye(3) * 10.26, (40, 40, 40))
    b = dev.basis(g, np.array([0.5, 0.5, 0.5]), 12.0)
    npw, _ = dev.D.dpp_basis_info(b)
    rng = np.random.default_rng(nbX + 7 * nbO)
    X = rng.standard_normal((nbX, npw)) + 1j * rng.standard_normal((nbX, npw))
    M = rng.standard_normal((nbX, nbO)) + 1j * rng.standard_normal((nbX, nbO))
    O0 = rng.standard_normal((nbO, npw)) + 1j * rng.standard_normal((nbO, npw))
    out = dev.tensor(O0)
    dev.D.dpp_rotate(b, nbX, dev.tensor(X), npw, nbO, dev.tensor(M), beta, out, npw)
    ref = (X.T @ M).T + beta * O0
    assert rel_err(dev.host(out), ref) < 1e-12


# Mixed-precision contractions (DPP_F32).  A^dag B on split-BF16 MFMA: every
# real input x is rounded to FP32 and split into hi + lo (BF16 each), with
# hi + lo = x (1 + d), |d| <= 2^-16 + 2^-24, d uniform in sign at about half
# that size; all four split products are exact in FP32, so one real product
# carries d_a + d_b, about 2^-17 rms.  The per-element statistical scale is
# therefore sigma_ij = 2^-17 sqrt(sum_g |a_g|^2 |b_g|^2); a correct kernel stays
# well inside 8 sigma over a whole matrix, while plain BF16 (no lo parts) is
# ~2^8 times larger and dropping the lo lo' product biases the Gram diagonal by
# ~2^-18/3 of sum |a|^2 (> 8 sigma at these sizes).
def _split_sigma(A, B):
    return 2.0 ** -17 * np.sqrt((np.abs(A) ** 2) @ (np.abs(B) ** 2).T)


@pytest.mark.parametrize("which,nbA,nbB", [("cfg1", 5, 3), ("cfg2", 16, 16), ("cfg2", 33, 20),
                                           ("cfg3", 128, 128), ("cfg3", 64, 128), ("cfg3", 1, 1)])
@pytest.mark.parametrize("gram", [False, True])
def test_overlap_split_bf16(dev, which, nbA, nbB, gram):
    log(f"overlap f32 {which} {nbA}x{nbB} gram={gram}")
    cell = {"cfg1": W.config1, "cfg2": W.config2, "cfg3": W.config3}[which]()
    g = dev.grid(cell.R, cell.S)
    b = dev.basis(g, cell.kpts[-1], cell.ecut)
    npw, _ = dev.D.dpp_basis_info(b)
    rng = np.random.default_rng(nbA * 131 + nbB + (7 if gram else 0))
    ld = npw + 3  # ragged leading dimension
    A = rng.standard_normal((nbA, ld)) + 1j * rng.standard_normal((nbA, ld))
    B = A[:nbB] if gram else rng.standard_normal((nbB, ld)) + 1j * rng.standard_normal((nbB, ld))
    if gram:
        nbB = min(nbA, nbB)
    U = dev.empty((nbA, nbB), dev.torch.complex128)
    ws = dev.ws(2 ** 26)
    dev.D.dpp_overlap(b, nbA, dev.tensor(A), ld, nbB, dev.tensor(B[:nbB]), ld, 2.5, U, ws, dev.D.DPP_F32)
    a, bb = A[:, :npw], B[:nbB, :npw]
    ref = 2.5 * a.conj() @ bb.T
    err = np.abs(dev.host(U) - ref) / (2.5 * _split_sigma(a, bb))
    log(f"max |err|/sigma = {err.max():.2f}")
    assert err.max() < 8.0


def _f32_bound(X, M, K):
    """Worst-case error of X M with X and M rounded to FP32 and an FP32 sum of
    K complex terms (2K real products per component): (2K + 4) 2^-24 times
    sum_k (|Re M|+|Im M|)(|Re X|+|Im X|)."""
    m1 = np.abs(M.real) + np.abs(M.imag)
    x1 = np.abs(X.real) + np.abs(X.imag)
    return (2 * K + 4) * 2.0 ** -24 * (x1.T @ m1).T


@pytest.mark.parametrize("nbX,nbO", [(1, 1), (5, 3), (16, 16), (64, 128), (128, 128), (128, 130)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_rotate_f32(dev, nbX, nbO, beta):
    log(f"rotate f32 {nbX}->{nbO} beta={beta}")
    g = dev.grid(np.eye(3) * 10.26, (40, 40, 40))
    b = dev.basis(g, np.array([0.5, 0.5, 0.5]), 12.0)
    npw, _ = dev.D.dpp_basis_info(b)
    rng = np.random.default_rng(3 * nbX + 11 * nbO)
    X = rng.standard_normal((nbX, npw)) + 1j * rng.standard_normal((nbX, npw))
    M = rng.standard_normal((nbX, nbO)) + 1j * rng.standard_normal((nbX, nbO))
    O0 = rng.standard_normal((nbO, npw)) + 1j * rng.standard_normal((nbO, npw))
    out = dev.tensor(O0)
    dev.D.dpp_rotate(b, nbX, dev.tensor(X), npw, nbO, dev.tensor(M), beta, out, npw, dev.D.DPP_F32)
    ref = (X.T @ M).T + beta * O0
    bound = _f32_bound(X, M, nbX) + 1e-15 * np.abs(ref)
    err = np.abs(dev.host(out) - ref)
    log(f"max err/bound = {(err / bound).max():.3e}")
    assert np.all(err <= bound)
    # and well above BF16-level accuracy: the typical error is at FP32 rounding
    assert np.sqrt(np.mean(err ** 2)) < 1e-5 * np.sqrt(np.mean(np.abs(ref) ** 2))


@pytest.mark.parametrize("nb", [1, 4, 16, 33, 64, 65, 100, 128])
def test_cholesky_orthonormalize(dev, nb):
    log(f"cholesky nb={nb}")
    cell = W.config2() if nb <= 16 else W.config3()
    ref = ob.gsphere(cell.R, cell.S, cell.kpts[-1], cell.ecut)
    g = dev.grid(cell.R, cell.S)
    b = dev.basis(g, cell.kpts[-1], cell.ecut)
    rng = np.random.default_rng(nb)
    Y = rng.standard_normal((ref.npw, nb)) + 1j * rng.standard_normal((ref.npw, nb))
    psi_ref, R_ref, Rinv_ref = oo.cholesky_orthonormalize(Y, ref)
    Yg = block_to_gpu(dev, Y)
    Rinv = dev.empty((nb, nb), dev.torch.complex128)
    ws = dev.ws(dev.D.dpp_ortho_workspace_size(b, nb))
    dev.D.dpp_cholesky_orthonormalize(b, nb, Yg, ref.npw, Rinv, ws)
    assert dev.D.dpp_ctx_status(dev.ctx) == 0
    psi = block_from_gpu(dev, Yg)
    assert rel_err(dev.host(Rinv), Rinv_ref) < 1e-11
    assert rel_err(psi, psi_ref) < 1e-11
    assert np.max(np.abs(psi.conj().T @ (ref.omega * psi) - np.eye(nb))) < 1e-11


@pytest.mark.parametrize("nb", [4, 40, 128])
def test_cholesky_flags_rank_deficient(dev, nb):
    log(f"cholesky rank-deficient nb={nb}")
    cell = W.config2()
    ref = ob.gsphere(cell.R, cell.S, cell.kpts[0], cell.ecut)
    g = dev.grid(cell.R, cell.S)
    b = dev.basis(g, cell.kpts[0], cell.ecut)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((ref.npw, nb)) + 1j * rng.standard_normal((ref.npw, nb))
    Y[:, nb - 2] = Y[:, 1]
    Yg = block_to_gpu(dev, Y)
    ws = dev.ws(dev.D.dpp_ortho_workspace_size(b, nb))
    dev.D.dpp_ctx_status(dev.ctx, True)
    dev.D.dpp_cholesky_orthonormalize(b, nb, Yg, ref.npw, None, ws)
    assert dev.D.dpp_ctx_status(dev.ctx, True) & dev.D.DPP_STATUS_NOTPD
    assert dev.D.dpp_ctx_status(dev.ctx, True) == 0


@pytest.mark.parametrize("nb", [1, 2, 5, 16, 33, 64, 65, 100, 128])
def test_subspace_eigh(dev, nb):
    log(f"eigh nb={nb}")
    rng = np.random.default_rng(nb)
    batch = 7 if nb >= 33 else 3
    H = rng.standard_normal((batch, nb, nb)) + 1j * rng.standard_normal((batch, nb, nb))
    H = H + np.conj(np.transpose(H, (0, 2, 1)))
    if nb >= 5:
        H[1] = np.diag(np.arange(nb, dtype=float)) + 0j     # already diagonal
        H[2, :2, :2] = np.array([[1.0, 0.0], [0.0, 1.0]])   # a degenerate block
    if nb >= 33:
        Q, _ = np.linalg.qr(rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb)))
        # shells of equal eigenvalues (free-electron-like multiplicities)
        ev = np.sort(np.repeat(0.1875 * np.arange(nb), 12)[:nb])
        H[3] = (Q * ev) @ Q.conj().T
        # a cluster spaced at 1e-9 inside an otherwise spread spectrum
        ev = np.sort(rng.standard_normal(nb))
        ev[5:13] = ev[5] + 1e-9 * np.arange(8)
        H[4] = 1e3 * ((Q * ev) @ Q.conj().T)
        H[5] = np.eye(nb) + 0j                               # every eigenvalue equal
        # one cluster of nb eigenvalues 1e-7 apart (larger than a block cluster)
        H[6] = (Q * (1.0 + 1e-7 * np.arange(nb))) @ Q.conj().T
    eig = dev.empty((batch, nb), dev.torch.float64)
    vec = dev.empty((batch, nb, nb), dev.torch.complex128)
    ws = dev.ws(dev.D.dpp_eigh_workspace_size(nb, batch))
    dev.D.dpp_subspace_eigh(dev.ctx, nb, batch, dev.tensor(H), eig, vec, ws)
    e = dev.host(eig)
    V = dev.host(vec)
    for i in range(batch):
        ref = np.linalg.eigvalsh(H[i])
        scale = max(1.0, np.max(np.abs(ref)))
        assert np.max(np.abs(e[i] - ref)) < 1e-12 * scale * nb
        assert np.max(np.abs(H[i] @ V[i] - V[i] * e[i][None, :])) < 1e-11 * scale * nb
        assert np.max(np.abs(V[i].conj().T @ V[i] - np.eye(nb))) < 1e-12 * nb


@pytest.mark.parametrize("name", ["tiny_proj_k", "cfg2", "cfg3"])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_density(dev, name, prec):
    log(f"density {name} prec={prec}")
    cell, kidx, nb = _ham_case(name)
    ref = ob.gsphere(cell.R, cell.S, cell.kpts[kidx], cell.ecut)
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((ref.npw, nb)) + 1j * rng.standard_normal((ref.npw, nb))
    f = rng.uniform(0, 2, nb)
    f[1] = 0.0
    wk = 0.125
    nref = np.zeros(cell.S)
    X = ot.I(psi, ref)
    for i in range(nb):
        nref += wk * f[i] * np.abs(X[i]) ** 2
    g = dev.grid(cell.R, cell.S)
    b = dev.basis(g, cell.kpts[kidx], cell.ecut)
    n0 = rng.uniform(0, 1, cell.S)
    ng = dev.tensor(n0)
    ws = dev.ws(dev.D.dpp_workspace_size(b, nb, prec))
    dev.D.dpp_density_accumulate(b, nb, block_to_gpu(dev, psi), ref.npw, dev.tensor(f), wk, ng, prec, ws)
    tol = 1e-12 if prec == 0 else 2e-5
    assert rel_err(dev.host(ng) - n0, nref) < tol


@pytest.mark.parametrize("cfg", ["noncubic", "cfg2", "cfg3"])
def test_fields(dev, cfg):
    log(f"fields {cfg}")
    if cfg == "noncubic":
        cell = W.tiny_cell(nat=3, L=7.0, ecut=4.0, S=(16, 15, 18), Z=(4, 1, 4), R=NONCUBIC)
    elif cfg == "cfg2":
        cell = W.config2()
    else:
        cell = W.config3()
    g = dev.grid(cell.R, cell.S)
    ws = dev.ws(dev.D.dpp_grid_workspace_size(g))
    omega = ob.cell_volume(cell.R)
    # local potential and start density
    V = dev.empty(cell.S, dev.torch.float64)
    dev.D.dpp_local_potential(g, cell.tau, cell.Z, cell.rc, V, ws)
    Vref = oo.local_potential(cell.R, cell.S, cell.tau, cell.Z, cell.rc)
    assert rel_err(dev.host(V), Vref) < 1e-12
    n = dev.empty(cell.S, dev.torch.float64)
    dev.D.dpp_start_density(g, cell.tau, cell.Z, W.START_SIGMA, n, ws)
    nref = oe.start_density(cell, W.START_SIGMA)
    assert rel_err(dev.host(n), nref) < 1e-12
    # Hartree on that density
    VH = dev.empty(cell.S, dev.torch.float64)
    EH = dev.zeros(1, dev.torch.float64)
    dev.D.dpp_hartree(g, dev.tensor(nref), VH, EH, ws)
    VHref, EHref = oe.hartree(nref, cell.R)
    assert rel_err(dev.host(VH), VHref) < 1e-12
    assert abs(dev.host(EH)[0] - EHref) < 1e-12 * abs(EHref)
    # LDA (include negative and tiny densities)
    nx = nref.copy()
    nx.reshape(-1)[:7] = [-1e-3, 0.0, 1e-17, 1e-16, 5e-16, 0.2387, 10.0]
    vxc = dev.empty(cell.S, dev.torch.float64)
    Exc = dev.zeros(1, dev.torch.float64)
    dev.D.dpp_lda_pz81(g, dev.tensor(nx), vxc, Exc, ws)
    eps_ref, v_ref = oxc.lda_pz81(nx)
    assert rel_err(dev.host(vxc), v_ref) < 1e-13
    Eref = omega / nx.size * np.sum(nx * eps_ref)
    assert abs(dev.host(Exc)[0] - Eref) < 1e-12 * abs(Eref)
    # grid dot
    out = dev.zeros(1, dev.torch.float64)
    dev.D.dpp_grid_dot(g, dev.tensor(nref), dev.tensor(Vref), 0.5, out, ws)
    assert abs(dev.host(out)[0] - 0.5 * np.sum(nref * Vref)) < 1e-12 * np.sum(np.abs(nref * Vref))
