"""GPU parity of the learned-density network (forward, loss, backward, Adam,
prediction) against the FP64 oracle run with the same BF16-rounded weights.
The GPU accumulates in FP32: tolerances 1e-4 relative on activations and
1e-3 relative per gradient tensor (cosine > 0.9999)."""
import numpy as np
import pytest

from oracle import convnet as cn
from tests._gpu import Device, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return Device()


def bf16_round(a):
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def flatten(params):
    import workloads as W
    return W.net_flatten(params)


def unflatten(vec, like):
    out, o = [], 0
    for W, b in like:
        w = vec[o:o + W.size].reshape(W.shape)
        o += W.size
        bb = vec[o:o + b.size]
        o += b.size
        out.append((w, bb))
    return out


@pytest.mark.parametrize("S,batch", [((12, 10, 8), 2), ((40, 40, 40), 1)])
def test_forward_backward_adam(dev, S, batch):
    log(f"convnet S={S} batch={batch}")
    params = cn.init_params(501)
    # make the last layer non-trivial so every gradient is exercised
    params[3] = (params[3][0] * 10.0, params[3][1] + 0.01)
    flat = flatten(params)
    p32 = unflatten(flat.astype(np.float64), params)
    pq = [(bf16_round(W), b.astype(np.float32).astype(np.float64)) for W, b in p32]
    rng = np.random.default_rng(7)
    n0 = rng.gamma(3.0, 0.01, (batch,) + S)
    nc = n0 * (1.0 + 0.2 * rng.standard_normal((batch,) + S))
    nbar = 0.03
    net = dev.D.dpp_net_create(dev.ctx, S, batch)
    dev.D.dpp_net_set_params(net, flat)
    n0g, ncg = dev.tensor(n0), dev.tensor(nc)
    y = dev.empty((batch,) + S, dev.torch.float32)
    dev.D.dpp_net_forward(net, batch, n0g, nbar, y)
    loss = dev.D.dpp_net_backward(net, batch, n0g, ncg, nbar)
    yg = dev.host(y)
    _, grads = dev.D.dpp_net_get_params(net)
    Lref, gsum = 0.0, None
    for b in range(batch):
        yo, _ = cn.forward(pq, (n0[b] / nbar)[None])
        assert np.max(np.abs(yg[b] - yo[0])) < 1e-4 * np.max(np.abs(yo[0]))
        L, gr = cn.loss_and_grads(pq, (n0[b] / nbar)[None], (nc[b] - n0[b]) / nbar)
        Lref += L / batch
        fl = flatten([(gW / batch, gb / batch) for gW, gb in gr]).astype(np.float64)
        gsum = fl if gsum is None else gsum + fl
    assert abs(loss - Lref) < 1e-4 * Lref
    o = 0
    for l, (W, bb) in enumerate(params):
        for j, size in enumerate((W.size, bb.size)):
            a, r = grads[o:o + size].astype(np.float64), gsum[o:o + size]
            o += size
            if l == 3 and j == 1:
                # the loss sees y - mean(y): the output bias has an exactly zero
                # gradient, so only its size relative to the weights' is checked
                scale = np.linalg.norm(gsum[o - size - W.size:o - size])
                assert np.linalg.norm(a) < 1e-5 * scale and np.linalg.norm(r) < 1e-9 * scale, (a, r, scale)
                continue
            rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            cos = a @ r / max(np.linalg.norm(a) * np.linalg.norm(r), 1e-30)
            assert rel < 1e-3 and cos > 0.9999, (l, size, rel, cos)
    # Adam step from the GPU gradients vs the oracle Adam (FP64)
    dev.D.dpp_net_adam_step(net, 1e-3)
    p_after, _ = dev.D.dpp_net_get_params(net)
    opt = cn.Adam(p32, lr=1e-3)
    ref = flatten(opt.step(p32, unflatten(grads.astype(np.float64), params)))
    assert np.max(np.abs(p_after - ref)) < 1e-6
    dev.D.dpp_net_destroy(net)


def test_predict_density(dev):
    log("convnet predict")
    S = (16, 15, 18)
    params = cn.init_params(501)
    params[3] = (params[3][0] * 10.0, params[3][1])
    flat = flatten(params)
    pq = [(bf16_round(W), b.astype(np.float32).astype(np.float64)) for W, b in
          unflatten(flat.astype(np.float64), params)]
    rng = np.random.default_rng(9)
    n0 = rng.gamma(3.0, 0.01, S)
    net = dev.D.dpp_net_create(dev.ctx, S, 1)
    dev.D.dpp_net_set_params(net, flat)
    out = dev.empty(S, dev.torch.float64)
    dev.D.dpp_net_predict_density(net, dev.tensor(n0), 32.0, 1080.0, out)
    ng = dev.host(out)
    ref = cn.predict_density(pq, n0, 32.0, 1080.0)
    assert np.all(ng >= 0)
    assert abs(1080.0 / ng.size * ng.sum() - 32.0) < 1e-10
    assert np.max(np.abs(ng - ref)) < 1e-5 * np.max(ref)
    dev.D.dpp_net_destroy(net)


def test_learned_start_small(dev):
    """Small end-to-end run of the learned start: training data from the
    library's SCF, training on the GPU, held-out evaluation with the bands
    converged in every SCF iteration (8 band-CG steps, 30 in the first).  The
    trained network must reduce the start-density error, both starts must
    converge (two energy changes below 1e-10 Ha/atom), and their converged
    energies must agree within 1e-6 Ha/atom.

    The saving in SCF iterations is not asserted here: single displaced cells
    range from 76 iterations slower to 65 faster, so four held-out cells
    cannot resolve the mean gain (this run: 20.75 plain, 23.0 learned).  The
    gain is measured over 64 held-out cells by learned.py (mean 27.1 -> 23.1,
    median 22.5 -> 16.0, 45 of 64 faster, one-sided sign test p = 2.5e-4)."""
    log("learned start: 24 train, 4 eval")
    from paper_1708_03621_amd import learned
    res = learned.run(n_train=24, n_eval=4, epochs=30, batch=8, lr=2e-3, n_inner=8, n_inner_first=30, max_iter=400,
                      log=log)
    log(f"loss {res['loss_first']:.3e} -> {res['loss_last']:.3e}; start error plain "
        f"{res['start_err_plain_mean']:.3e} learned {res['start_err_learned_mean']:.3e}; iters "
        f"{res['iters_plain_mean']} -> {res['iters_learned_mean']}")
    assert res["loss_last"] < 0.5 * res["loss_first"]
    assert res["start_err_learned_mean"] < res["start_err_plain_mean"]
    assert res["cells_converged_both"] == res["n_eval"]
    assert res["max_dE_per_atom"] < 1e-6
