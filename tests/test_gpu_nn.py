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


def _bf16_forward(X, Ws, act):
    """The network with BF16 weights, input and hidden activations (FP64 sums)."""
    from oracle import precision

    r = precision.round_bf16
    h = r(X)
    for l, W in enumerate(Ws):
        z = convnet.conv(h, r(W))
        if l < 2:
            h = r(np.maximum(z, 0.0) if act == "relu" else z)
    return z


@pytest.mark.parametrize("k", [0, 1])
def test_bf16_matrix_core_forward_matches_rounded_oracle(ctx, k):
    code, act = _acts()[k]
    extent = (4, 4, 4, 4)
    w = synth.convnet_weights(23, scale=1.0, identity=(code == 0))
    net = ctx.nn_create(extent, w, act=code)
    S = 256
    rng = np.random.default_rng(24)
    X = rng.standard_normal((5, S, 24)).astype(np.float32)
    Y = net.apply(_dev(X), prec="bf16").cpu().numpy()
    Ws = _layers(w)
    for i in range(5):
        xi = X[i].astype(np.float64).reshape(extent + (24,))
        ref = _bf16_forward(xi, Ws, act).reshape(S, 24)
        exact = convnet.forward(xi, Ws, act)[0].reshape(S, 24)
        assert np.linalg.norm(Y[i] - ref) <= 2e-3 * np.linalg.norm(ref)
        assert np.linalg.norm(Y[i] - exact) <= 3e-2 * np.linalg.norm(exact)
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


@pytest.fixture(scope="module")
def toy(ctx):
    """8^4 lattice in 16 blocks of 4^4 (kappa 0.12, links exp(0.3 i H)), (source, solution)
    pairs made by the block solver with sources on even sites, and a network trained on them."""
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
    _, vl0 = net.train(blk, src, sol, 24, vsrc, vsol, 8, params=dd.nn_train_params(epochs=1, batch=16, lr=1e-9))
    tl, vl = net.train(blk, src, sol, 24, vsrc, vsol, 8, params=dd.nn_train_params(epochs=25, batch=16, lr=2e-3))
    yield dict(L=L, U=U, kappa=kappa, blk=blk, g=g, net=net, vl0=vl0, tl=tl, vl=vl)
    net.close()
    g.close()
    blk.close()


def test_training_on_solver_pairs_lowers_validation_loss(toy):
    """Held-out loss of the trained network well below that of the untrained one."""
    print("val loss untrained %.4f -> %s" % (toy["vl0"][0], np.array2string(toy["vl"][::6], precision=4)))
    assert toy["vl"][-1] < 0.5 * toy["vl0"][0]
    assert toy["tl"][-1] < toy["tl"][0]


@pytest.mark.parametrize("cycles", [0, 1])
def test_fgmres_with_trained_network(ctx, toy, cycles):
    """Flexible GMRES with the network's first directions: same FP64 1e-10 solutions, fewer Krylov steps."""
    from oracle import geometry, wilson
    from tests import _cfg

    from paper_2211_06902_amd import dd

    b = synth.spinor_field(toy["L"], 4, 61)[:, _cfg.block_sites(toy["L"], geometry.tile_boxes(toy["L"], [[4, 4]] * 4))]
    bd = _dev(b)
    base = dict(method=dd.GMRES, restart=8, inner_prec="f32")
    x0, i0, s0 = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd, params=dd.solve_params(**base))
    x1, i1, s1 = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd,
                                 params=dd.solve_params(precond=toy["net"], precond_cycles=cycles, **base))
    print("GMRES(8) steps per pair: plain %.1f, with network (every %d cycles) %.1f" %
          (i0["iters"].mean(), cycles, i1["iters"].mean()))
    assert s0 == dd.DD_OK and s1 == dd.DD_OK
    assert np.all(i1["true_relres"] <= 1e-10)
    assert _cfg.rel_err(x1.cpu().numpy(), x0.cpu().numpy()) <= 1e-8
    boxes = geometry.tile_boxes(toy["L"], [[4, 4]] * 4)
    xh = x1.cpu().numpy()
    for k in (0, 9):
        sl = slice(256 * k, 256 * (k + 1))
        r = b[2, sl] - wilson.dirac_box(toy["L"], -1, toy["kappa"], toy["U"], boxes[k][:4], boxes[k][4:8], xh[2, sl])
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[2, sl])
    assert i1["iters"].mean() < i0["iters"].mean()


def test_bicgstab_right_preconditioned_by_trained_network(ctx, toy):
    """BiCGStab on Dhat N u = f with the linear network N: same 1e-10 solutions, fewer iterations,
    and graph replay identical to eager launches."""
    from oracle import geometry
    from tests import _cfg

    from paper_2211_06902_amd import dd

    b = synth.spinor_field(toy["L"], 4, 62)[:, _cfg.block_sites(toy["L"], geometry.tile_boxes(toy["L"], [[4, 4]] * 4))]
    bd = _dev(b)
    x0, i0, s0 = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd, params=dd.solve_params(inner_prec="f32"))
    x1, i1, s1 = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd,
                                 params=dd.solve_params(inner_prec="f32", precond=toy["net"], use_graph=1))
    x2, i2, s2 = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd,
                                 params=dd.solve_params(inner_prec="f32", precond=toy["net"], use_graph=0))
    print("BiCGStab iterations per pair: plain %.1f, right-preconditioned by the network %.1f" %
          (i0["iters"].mean(), i1["iters"].mean()))
    assert s0 == dd.DD_OK and s1 == dd.DD_OK and s2 == dd.DD_OK
    assert np.all(i1["true_relres"] <= 1e-10)
    assert _cfg.rel_err(x1.cpu().numpy(), x0.cpu().numpy()) <= 1e-8
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert i1["iters"].mean() < i0["iters"].mean()


def test_bicgstab_rejects_a_relu_network(ctx, toy):
    from paper_2211_06902_amd import dd

    net = ctx.nn_create((4, 4, 4, 4), synth.convnet_weights(74), act=dd.NN_RELU)
    with pytest.raises(dd.DDError):
        ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], _dev(synth.gaussian_complex((1, 8**4, 4, 3), 75)),
                        params=dd.solve_params(precond=net))
    net.close()


def test_fgmres_with_an_untrained_network_still_converges(ctx, toy):
    from paper_2211_06902_amd import dd

    net = ctx.nn_create((4, 4, 4, 4), synth.convnet_weights(71, scale=1.0, identity=False))
    b = _dev(synth.gaussian_complex((2, 8**4, 4, 3), 72))
    x, info, st = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], b,
                                  params=dd.solve_params(method=dd.GMRES, restart=8, precond=net, precond_cycles=1))
    assert st == dd.DD_OK and np.all(info["true_relres"] <= 1e-10)
    net.close()


def test_network_on_blocks_of_another_extent_is_rejected(ctx, toy):
    from paper_2211_06902_amd import dd

    blk = ctx.make_blocks(toy["L"], -1, [[8]] * 4)
    g = ctx.load_gauge(blk, _dev(toy["U"]), "f32")
    with pytest.raises(dd.DDError):
        ctx.block_solve(blk, g, toy["kappa"], _dev(synth.gaussian_complex((1, 8**4, 4, 3), 73)),
                        params=dd.solve_params(method=dd.GMRES, precond=toy["net"]))
    g.close()
    blk.close()


def test_network_parity_modes_change_nothing(ctx, toy):
    """Inside the solver the BF16 network gets an even half field (odd sites zero) and only its even
    output sites are used: the LDS kernel then skips the taps that reach the zero odd sites (layer 1)
    and the odd output rows (layer 3).  The solve is the same as with the global-gather kernel, which
    multiplies everything."""
    from oracle import geometry
    from tests import _cfg

    from paper_2211_06902_amd import dd

    b = synth.spinor_field(toy["L"], 4, 63)[:, _cfg.block_sites(toy["L"], geometry.tile_boxes(toy["L"], [[4, 4]] * 4))]
    bd = _dev(b)
    prm = dd.solve_params(inner_prec="f32", precond=toy["net"])
    out = []
    try:
        for k in (0, 1):
            ctx.tune_set(dd.TUNE_NN_KERNEL, k)
            x, info, st = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd, params=prm)
            assert st == dd.DD_OK
            out.append((x.cpu().numpy(), info["iters"].copy()))
    finally:
        ctx.tune_set(dd.TUNE_NN_KERNEL, 1)
    assert np.array_equal(out[0][1], out[1][1])
    assert _cfg.rel_err(out[1][0], out[0][0]) <= 1e-12


def test_network_preconditioned_bicgstab_with_dhat_walk(ctx, toy):
    """BiCGStab with the network as right preconditioner applies Dhat to M p and M s; with one walk
    segment per block it takes the one-kernel x0-walk of Dhat (intermediate in LDS, the dot with rh or
    with s fused).  Same solve as with two hop launches: every pair to tolerance, same solution, the same
    iteration counts up to rounding at the stopping test."""
    from oracle import geometry
    from tests import _cfg

    from paper_2211_06902_amd import dd

    b = synth.spinor_field(toy["L"], 4, 64)[:, _cfg.block_sites(toy["L"], geometry.tile_boxes(toy["L"], [[4, 4]] * 4))]
    bd = _dev(b)
    prm = dd.solve_params(inner_prec="f32", precond=toy["net"])
    out = []
    try:
        ctx.tune_set(dd.TUNE_HOP_WALK, 1)
        for k in (0, -1):
            ctx.tune_set(dd.TUNE_DHAT_WALK, k)
            x, info, st = ctx.block_solve(toy["blk"], toy["g"], toy["kappa"], bd, params=prm)
            assert st == dd.DD_OK
            assert np.all(info["true_relres"] <= 1e-10)
            out.append((x.cpu().numpy(), info["iters"].astype(np.int64)))
    finally:
        ctx.tune_set(dd.TUNE_HOP_WALK, 0)
        ctx.tune_set(dd.TUNE_DHAT_WALK, 0)
    assert np.max(np.abs(out[0][1] - out[1][1])) <= 2
    assert _cfg.rel_err(out[0][0], out[1][0]) <= 1e-9


def test_network_preconditioned_bicgstab_with_clover(ctx, toy):
    """BiCGStab right-preconditioned by the network on the clover operator (the network trained on
    Wilson pairs is a perturbation away from the clover inverse, which right preconditioning allows):
    every pair to tolerance with the one-kernel Dhat and with two hop launches, the same solution, and
    the true residual of two blocks on the oracle's clover operator; flexible GMRES with the network
    gives the same solution."""
    from oracle import clover, geometry
    from tests import _cfg

    from paper_2211_06902_amd import dd

    L, kappa, csw = toy["L"], toy["kappa"], 1.4
    g = ctx.load_gauge(toy["blk"], _dev(toy["U"]), "f32").set_clover(_dev(toy["U"]), kappa, csw)
    boxes = geometry.tile_boxes(L, [[4, 4]] * 4)
    b = synth.spinor_field(L, 3, 65)[:, _cfg.block_sites(L, boxes)]
    bd = _dev(b)
    prm = dd.solve_params(inner_prec="f32", precond=toy["net"])
    out = []
    try:
        ctx.tune_set(dd.TUNE_HOP_WALK, 1)
        for k in (0, -1):
            ctx.tune_set(dd.TUNE_DHAT_WALK, k)
            x, info, st = ctx.block_solve(toy["blk"], g, kappa, bd, params=prm)
            assert st == dd.DD_OK and np.all(info["true_relres"] <= 1e-10), k
            out.append(x.cpu().numpy())
    finally:
        ctx.tune_set(dd.TUNE_HOP_WALK, 0)
        ctx.tune_set(dd.TUNE_DHAT_WALK, 0)
    assert _cfg.rel_err(out[0], out[1]) <= 1e-9
    A = clover.clover_matrix(L, toy["U"], kappa, csw)
    off = _cfg.site_offsets(boxes)
    for k in (0, len(boxes) - 1):
        sl = slice(off[k], off[k + 1])
        for r in range(3):
            Dx = clover.dirac_clover_box(L, -1, kappa, csw, toy["U"], boxes[k][:4], boxes[k][4:8], out[0][r, sl], A=A)
            assert np.linalg.norm(b[r, sl] - Dx) <= 1e-10 * np.linalg.norm(b[r, sl]), (k, r)
    # flexible GMRES with the network's first directions on the same operator
    xg, infog, st = ctx.block_solve(toy["blk"], g, kappa, bd,
                                    params=dd.solve_params(method=dd.GMRES, inner_prec="f32", precond=toy["net"]))
    assert st == dd.DD_OK and np.all(infog["true_relres"] <= 1e-10)
    assert _cfg.rel_err(xg.cpu().numpy(), out[0]) <= 1e-9
    g.close()
