"""The allocation-free eigensolver entry point (static device workspace)
against the workspace one, through the C ABI: two calls in a row, the second
smaller than the first, each equal to dpp_subspace_eigh on the same input."""
import numpy as np
import pytest

from tests._gpu import Device, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return Device()


def _hermitian(rng, batch, nb):
    H = rng.standard_normal((batch, nb, nb)) + 1j * rng.standard_normal((batch, nb, nb))
    return H + np.conj(np.transpose(H, (0, 2, 1)))


def _both(dev, H):
    batch, nb, _ = H.shape
    Hg = dev.tensor(H)
    eig_a = dev.empty((batch, nb), dev.torch.float64)
    vec_a = dev.empty((batch, nb, nb), dev.torch.complex128)
    ws = dev.ws(dev.D.dpp_eigh_workspace_size(nb, batch))
    dev.D.dpp_subspace_eigh(dev.ctx, nb, batch, Hg, eig_a, vec_a, ws)
    eig_b = dev.zeros((batch, nb), dev.torch.float64)
    vec_b = dev.zeros((batch, nb, nb), dev.torch.complex128)
    dev.D.dpp_subspace_eigh_noalloc(dev.ctx, nb, batch, Hg, eig_b, vec_b)
    return dev.host(eig_a), dev.host(vec_a), dev.host(eig_b), dev.host(vec_b)


def test_noalloc_eigh_equals_workspace_eigh(dev):
    rng = np.random.default_rng(11)
    for batch, nb in [(3, 128), (2, 65), (1, 24)]:  # each call smaller than the one before
        log(f"noalloc eigh batch={batch} nb={nb}")
        H = _hermitian(rng, batch, nb)
        ea, va, eb, vb = _both(dev, H)
        assert np.array_equal(ea, eb)
        assert np.max(np.abs(va - vb)) <= 1e-13
        for i in range(batch):
            ref = np.linalg.eigvalsh(H[i])
            assert np.max(np.abs(eb[i] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))) * nb


def test_noalloc_eigh_rejects_oversize(dev):
    nb, batch = 128, 8  # needs more workspace than the static array holds
    H = dev.zeros((batch, nb, nb), dev.torch.complex128)
    eig = dev.empty((batch, nb), dev.torch.float64)
    vec = dev.empty((batch, nb, nb), dev.torch.complex128)
    with pytest.raises(Exception, match="static array"):
        dev.D.dpp_subspace_eigh_noalloc(dev.ctx, nb, batch, H, eig, vec)
