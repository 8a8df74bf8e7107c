"""GPU parity of the learned block preconditioner's kernels against the FP64
reference network (oracle/convnet.py): forward pass, loss and gradients (the
gradient check), one Adam step, and a training run on solver-generated pairs.

The GPU network computes in FP32; tolerances are FP32-level (relative 1e-5 on
outputs and loss, 1e-4 on gradient norms).
"""
import numpy as np
import pytest

import synth
from oracle import convnet

pytestmark = pytest.mark.gpu

SIZES = [(24, 32), (32, 32), (32, 24)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_06902_amd import dd

    c = dd.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _layers(w):
    out, k = [], 0
    for a, b in SIZES:
        out.append(np.asarray(w[k:k + 81 * a * b], dtype=np.float64).reshape(81, a, b))
        k += 81 * a * b
    return out


def _acts():
    from paper_2211_06902_amd import dd

    return [(dd.NN_LINEAR, "linear"), (dd.NN_RELU, "relu")]


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("extent", [(4, 4, 4, 4), (3, 2, 4, 5)])
def test_forward_matches_oracle(ctx, extent, k):
    code, act = _acts()[k]
    w = synth.convnet_weights(21, scale=1.0, identity=(code == 0))
    net = ctx.nn_create(extent, w, act=code)
    S = int(np.prod(extent))
    rng = np.random.default_rng(22)
    X = rng.standard_normal((3, S, 24))
    Y = net.apply(_dev(X.astype(np.float32))).cpu().numpy()
    Ws = _layers(w)
    for i in range(3):
        ref = convnet.forward(X[i].reshape(tuple(extent) + (24,)), Ws, act)[0].reshape(S, 24)
        assert np.linalg.norm(Y[i] - ref) <= 1e-5 * np.linalg.norm(ref)
    net.close()


def _toy_pairs(ctx, n_rhs, seed):
    """8^4 lattice in 16 blocks of 4^4; random sources and targets in the solver layout."""
    L = (8, 8, 8, 8)
    blk = ctx.make_blocks(L, -1, [[4, 4]] * 4)
    src = synth.gaussian_complex((n_rhs, 8**4, 4, 3), seed)
    sol = synth.gaussian_complex((n_rhs, 8**4, 4, 3), seed + 1)
    return blk, src, sol


def _oracle_batch(src, sol, pairs, nb):
    S = 4**4
    X, T = [], []
    for p in pairs:
        r, b = divmod(int(p), nb)
        X.append(convnet.spinor_to_channels(src[r, b * S:(b + 1) * S], (4, 4, 4, 4)))
        T.append(convnet.spinor_to_channels(sol[r, b * S:(b + 1) * S], (4, 4, 4, 4)))
    return np.asarray(X), np.asarray(T)


@pytest.mark.parametrize("k", [0, 1])
def test_loss_and_gradients_match_oracle(ctx, k):
    """The gradient check: the GPU backward pass against the FP64 analytic gradients."""
    code, act = _acts()[k]
    blk, src, sol = _toy_pairs(ctx, 2, 31)
    w = synth.convnet_weights(32, scale=1.0, identity=(code == 0))
    net = ctx.nn_create((4, 4, 4, 4), w, act=code)
    pairs = [0, 5, 17, 30]
    loss, g = net.loss_grad(blk, _dev(src), _dev(sol), 2, pairs, mask_even=1)
    X, T = _oracle_batch(src, sol, pairs, blk.n_blocks)
    mask = (np.indices((4, 4, 4, 4)).sum(axis=0) % 2 == 0).astype(float)
    lref, gref = convnet.loss_and_grad(X, T, _layers(w), mask, act)
    assert abs(loss - lref) <= 1e-5 * lref
    for gl, gr in zip(_layers(g), gref):
        assert np.linalg.norm(gl - gr) <= 1e-4 * np.linalg.norm(gr)
    net.close()
    blk.close()


def test_adam_step_matches_oracle(ctx):
    from paper_2211_06902_amd import dd

    blk, src, sol = _toy_pairs(ctx, 1, 41)
    w = synth.convnet_weights(42)
    net = ctx.nn_create((4, 4, 4, 4), w)
    lr = 1e-3
    p = dd.nn_train_params(epochs=1, batch=16, lr=lr)
    net.train(blk, _dev(src), _dev(sol), 1, params=p)
    w1 = net.weights()
    X, T = _oracle_batch(src, sol, range(16), blk.n_blocks)
    mask = (np.indices((4, 4, 4, 4)).sum(axis=0) % 2 == 0).astype(float)
    _, gref = convnet.loss_and_grad(X, T, _layers(w), mask)
    g = np.concatenate([x.reshape(-1) for x in gref])
    wref, _, _ = convnet.adam_step(w.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    # the first Adam step moves each weight by lr * sign(g): compare where the gradient sign is certain
    sure = np.abs(g) > 1e-3 * np.abs(g).max()
    assert sure.mean() > 0.5
    assert np.max(np.abs(w1[sure] - wref[sure])) <= 1e-6 + 1e-5 * lr
    assert np.max(np.abs(w1 - w)) <= lr * 1.0001
    net.close()
    blk.close()


def test_training_on_solver_pairs_lowers_validation_loss(ctx):
    """Train on (source, D^{-1} source) pairs of 4^4 blocks (sources on even sites) made by the
    block solver; the held-out loss must fall well below that of the untrained network."""
    import torch

    from paper_2211_06902_amd import dd

    L = (8, 8, 8, 8)
    kappa = 0.12
    blk = ctx.make_blocks(L, -1, [[4, 4]] * 4)
    U = synth.gauge_field(L, 0.3, 51)
    g = ctx.load_gauge(blk, _dev(U), "f32")
    even = (np.indices((4, 4, 4, 4)).sum(axis=0).reshape(-1) % 2 == 0)

    def pairs(n, seed):
        b = synth.gaussian_complex((n, 8**4, 4, 3), seed)
        b.reshape(n, 16, 256, 4, 3)[:, :, ~even] = 0.0
        bd = _dev(b)
        x, info, st = ctx.block_solve(blk, g, kappa, bd, params=dd.solve_params(inner_prec="f32"))
        assert st == dd.DD_OK
        return bd, x

    src, sol = pairs(24, 52)
    vsrc, vsol = pairs(8, 53)
    net = ctx.nn_create((4, 4, 4, 4), synth.convnet_weights(54))
    p = dd.nn_train_params(epochs=1, batch=16, lr=2e-3)
    tl0, vl0 = net.train(blk, src, sol, 24, vsrc, vsol, 8, params=dd.nn_train_params(epochs=1, batch=16, lr=1e-9))
    p = dd.nn_train_params(epochs=25, batch=16, lr=2e-3)
    tl, vl = net.train(blk, src, sol, 24, vsrc, vsol, 8, params=p)
    print("val loss untrained %.4f -> %s" % (vl0[0], np.array2string(vl[::6], precision=4)))
    assert vl[-1] < 0.5 * vl0[0]
    assert tl[-1] < tl[0]
    net.close()
    g.close()
    blk.close()
    torch.cuda.synchronize()
