"""Surrogate MLP kernels (BF16 MFMA, FP32 accumulation) against the FP64 reference."""
import numpy as np
import pytest

from oracle import mlp_ref
from tests.philox_ref import philox4x32_10

pytestmark = pytest.mark.gpu

N_IN = 8


@pytest.fixture(scope="module")
def ctx():
    import paper_1806_00205_amd as rt
    c = rt.Context(0)
    yield c
    c.close()


def _data(seed, B):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, N_IN)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 7]).astype(np.float32)
    return X, t


def test_params_roundtrip(ctx):
    s = ctx.srg_create(N_IN, 256, 4, seed=3)
    p = ctx.srg_params(s)
    assert p.size == mlp_ref.n_params(N_IN)
    q = np.random.default_rng(0).normal(size=p.size).astype(np.float32) * 0.01
    ctx.srg_set_params(s, q)
    assert np.array_equal(ctx.srg_params(s), q)


@pytest.mark.parametrize("B", [64, 1000, 4096 + 7])
def test_forward_matches_reference(ctx, B):
    s = ctx.srg_create(N_IN, 256, 4, seed=1)
    p = ctx.srg_params(s)
    X, _ = _data(2, B)
    y = ctx.srg_predict(s, X).cpu().numpy().astype(np.float64)
    pv = mlp_ref.gpu_visible_params(p, N_IN)
    yr, _ = mlp_ref.forward(pv, mlp_ref.round_bf16(X), N_IN)
    # BF16 activations between layers: relative error of a few 2^-8 steps
    err = np.abs(y - yr)
    assert np.max(err) <= 0.03 * np.max(np.abs(yr)) + 1e-3, np.max(err)
    assert np.sqrt(np.mean(err ** 2)) <= 0.01 * np.sqrt(np.mean(yr ** 2)) + 1e-4


def test_predict_across_chunks_and_tiny(ctx):
    s = ctx.srg_create(N_IN, 256, 4, seed=4)
    X, _ = _data(5, (1 << 18) + 77)
    y_all = ctx.srg_predict(s, X).cpu().numpy()
    y_head = ctx.srg_predict(s, X[:1]).cpu().numpy()
    y_tail = ctx.srg_predict(s, X[-100:]).cpu().numpy()
    assert y_head[0] == y_all[0]
    assert np.array_equal(y_tail, y_all[-100:])


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_reference(ctx, seed):
    s = ctx.srg_create(N_IN, 256, 4, seed=10 + seed)
    p = ctx.srg_params(s)
    X, t = _data(20 + seed, 512)
    loss, g = ctx.srg_gradient(s, X, t)
    pv = mlp_ref.gpu_visible_params(p, N_IN)
    lr, gr = mlp_ref.loss_and_grad(pv, mlp_ref.round_bf16(X), t, N_IN)
    assert loss == pytest.approx(lr, rel=1e-2)
    g = g.astype(np.float64)
    cos = g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr))
    rel = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    # observed 5e-4 to 1e-3: the bfloat16 storage between layers (next test)
    assert cos > 0.9999 and rel < 5e-3, (cos, rel)
    # every parameter block, separately
    n_in, W = N_IN, 256
    bounds = [0, W * n_in, W * n_in + W]
    o = bounds[-1]
    for _ in range(3):
        o += W * W
        bounds.append(o)
        o += W
        bounds.append(o)
    bounds += [o + W, o + W + 1]
    for a, b in zip(bounds[:-1], bounds[1:]):
        ga, gb = g[a:b], gr[a:b]
        if np.linalg.norm(gb) > 0:
            assert np.linalg.norm(ga - gb) <= 1e-2 * np.linalg.norm(gb) + 1e-7, (a, b)


def _bf16_rounded_grad(p, X, t, n_in, width=256, depth=4):
    """Gradient with the GPU's storage rounding: inputs, weights, hidden
    activations and the hidden layers' backward signals held as bfloat16,
    everything else (pre-activations, sums, output layer) in FP64."""
    r = lambda a: mlp_ref.round_bf16(np.asarray(a, dtype=np.float32)).astype(np.float64)
    Ws, bs, w_out, b_out = mlp_ref.unpack(mlp_ref.gpu_visible_params(p, n_in), n_in, width, depth)
    h = r(X)
    hs, zs = [h], []
    for W, b in zip(Ws, bs):
        z = h @ W.T + b
        h = r(mlp_ref.gelu(z))
        zs.append(z)
        hs.append(h)
    t = np.asarray(t, dtype=np.float64)
    B = h.shape[0]
    dy = 2.0 * (h @ w_out + b_out - t) / B
    parts_out = [hs[-1].T @ dy, np.array([dy.sum()])]
    G = r(np.outer(dy, w_out) * mlp_ref.gelu_d(zs[-1]))
    gW, gb = [None] * depth, [None] * depth
    for l in range(depth - 1, -1, -1):
        gW[l] = G.T @ hs[l]
        gb[l] = G.sum(axis=0)
        if l > 0:
            G = r((G @ Ws[l]) * mlp_ref.gelu_d(zs[l - 1]))
    parts = []
    for l in range(depth):
        parts += [gW[l].ravel(), gb[l]]
    return np.concatenate(parts + parts_out)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_deviation_is_the_bf16_storage(ctx, seed):
    """What separates the GPU gradient from the FP64 one (about 1e-3) is the
    bfloat16 storage of activations and backward signals between layers:
    with that rounding reproduced on the host the agreement is about ten
    times closer (what remains is FP32 summation order and values that round
    to the other side of a bfloat16 step)."""
    s = ctx.srg_create(N_IN, 256, 4, seed=10 + seed)
    p = ctx.srg_params(s)
    X, t = _data(20 + seed, 512)
    _, g = ctx.srg_gradient(s, X, t)
    g = g.astype(np.float64)
    ge = _bf16_rounded_grad(p, mlp_ref.round_bf16(X), t, N_IN)
    _, gr = mlp_ref.loss_and_grad(mlp_ref.gpu_visible_params(p, N_IN), mlp_ref.round_bf16(X), t, N_IN)
    rel_e = np.linalg.norm(g - ge) / np.linalg.norm(ge)
    rel_r = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    rel_er = np.linalg.norm(ge - gr) / np.linalg.norm(gr)
    print(f"GPU vs bf16-rounded {rel_e:.2e}, GPU vs FP64 {rel_r:.2e}, bf16-rounded vs FP64 {rel_er:.2e}")
    assert rel_e < 5e-4, rel_e
    assert rel_e < 0.25 * rel_r, (rel_e, rel_r)


@pytest.mark.parametrize("batch", [32, 4128, 16384 + 4128])
def test_gradient_of_one_tile_and_of_many_tiles_per_workgroup(ctx, batch):
    """One 32-row tile (one workgroup); 129 tiles in 129 workgroups; and a
    batch of two passes (16384 rows as two tiles in each of 256 workgroups,
    whose bias and loss sums each workgroup adds up in its slice, then 4128
    rows whose weight gradients are added to the first pass's): the gradient
    still carries only the BF16 storage error against the host evaluation with
    the same rounding."""
    s = ctx.srg_create(N_IN, 256, 4, seed=44)
    p = ctx.srg_params(s)
    X, t = _data(60, batch)
    loss, g = ctx.srg_gradient(s, X, t)
    ge = _bf16_rounded_grad(p, mlp_ref.round_bf16(X), t, N_IN)
    rel_e = np.linalg.norm(g.astype(np.float64) - ge) / np.linalg.norm(ge)
    assert rel_e < 5e-4, rel_e
    lr, _ = mlp_ref.loss_and_grad(mlp_ref.gpu_visible_params(p, N_IN), mlp_ref.round_bf16(X), t, N_IN)
    assert loss == pytest.approx(lr, rel=1e-2)


def test_adamw_step_matches_numpy(ctx):
    """Three AdamW steps (decoupled weight decay, bias-corrected moments)
    element by element against numpy fed with the same gradients."""
    s = ctx.srg_create(N_IN, 256, 4, seed=5)
    X, t = _data(40, 256)
    p = ctx.srg_params(s).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lr, wd, b1, b2, eps = 1e-3, 1e-2, 0.9, 0.999, 1e-8
    for step in range(1, 4):
        _, g = ctx.srg_gradient(s, X, t)  # the gradient the step will use (deterministic)
        ctx.srg_train_step(s, X, t, lr=lr, weight_decay=wd)
        g = g.astype(np.float64)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p - lr * ((m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps) + wd * p)
        got = ctx.srg_params(s).astype(np.float64)
        err = np.abs(got - p)
        assert np.max(err - 1e-6 * np.abs(p)) <= 2e-8, (step, float(np.max(err)))


def test_training_loop_graph_replays_equal_eager(ctx):
    """The device training loop replayed as a HIP graph gives bit for bit the
    parameters of the same launches issued one by one: three rounds, each a
    replayed call after an eager one on a twin network, with other GPU work
    and synchronisation in between."""
    import torch
    X, t = _data(50, 4096)
    Xd, td = torch.tensor(X, device="cuda:0"), torch.tensor(t, device="cuda:0")
    a = ctx.srg_create(N_IN, 256, 4, seed=9)
    b = ctx.srg_create(N_IN, 256, 4, seed=9)
    lr = np.full(40, 1e-3, dtype=np.float32)
    for rnd in range(3):
        la = ctx.srg_train(a, Xd, td, 256, lr, weight_decay=1e-4, seed=77, use_graph=False)
        lb = ctx.srg_train(b, Xd, td, 256, lr, weight_decay=1e-4, seed=77, use_graph=True)
        assert np.array_equal(la, lb), rnd
        assert np.array_equal(ctx.srg_params(a), ctx.srg_params(b)), rnd
        ctx.srg_predict(a, Xd[:1000])  # other work between replays
        torch.cuda.synchronize()


def test_training_loop_of_two_passes_per_step(ctx):
    """A batch of 16384 + 2048 rows takes two passes of the weight-gradient
    kernel per step, the step's bookkeeping (loss, AdamW constants, step
    counter) on the last one only: the loop's losses are those of the
    same-seed loop replayed as a graph, and its first loss is the batch loss
    of the rows the first step draws, evaluated on the host."""
    import torch
    X, t = _data(51, 50000)
    Xd, td = torch.tensor(X, device="cuda:0"), torch.tensor(t, device="cuda:0")
    batch = 16384 + 2048
    a = ctx.srg_create(N_IN, 256, 4, seed=12)
    b = ctx.srg_create(N_IN, 256, 4, seed=12)
    p0 = ctx.srg_params(a)
    lr = np.full(5, 1e-3, dtype=np.float32)
    la = ctx.srg_train(a, Xd, td, batch, lr, seed=5, use_graph=False)
    lb = ctx.srg_train(b, Xd, td, batch, lr, seed=5, use_graph=True)
    assert np.array_equal(la, lb)
    assert np.array_equal(ctx.srg_params(a), ctx.srg_params(b))
    # rows of step 0: batch row r is source row floor(u n / 2^32), u the first
    # word of Philox4x32-10 keyed by the seed at counter (r, 0, 0, 0)
    ctr = np.zeros((batch, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(batch, dtype=np.uint32)
    u = philox4x32_10(ctr, np.array([5, 0], dtype=np.uint32))[:, 0].astype(np.uint64)
    rows = ((u * np.uint64(len(X))) >> np.uint64(32)).astype(np.int64)
    lr0, _ = mlp_ref.loss_and_grad(mlp_ref.gpu_visible_params(p0, N_IN), mlp_ref.round_bf16(X[rows]), t[rows], N_IN)
    assert float(la[0]) == pytest.approx(lr0, rel=1e-2)
    assert np.all(np.isfinite(la)) and la[-1] < la[0]


def test_training_loop_converges(ctx):
    import torch
    s = ctx.srg_create(N_IN, 256, 4, seed=8)
    X, t = _data(31, 8192)
    Xd, td = torch.tensor(X, device="cuda:0"), torch.tensor(t, device="cuda:0")
    losses = ctx.srg_train(s, Xd, td, 1024, np.full(400, 1e-3, dtype=np.float32), seed=3)
    assert np.all(np.isfinite(losses)) and losses.shape == (400,)
    y = ctx.srg_predict(s, Xd).cpu().numpy()
    mse = float(np.mean((y - t) ** 2))
    assert mse < float(losses[0]) / 20, (float(losses[0]), mse)


def test_training_converges(ctx):
    import torch
    s = ctx.srg_create(N_IN, 256, 4, seed=7)
    X, t = _data(30, 8192)
    Xd = torch.tensor(X, device="cuda:0")
    td = torch.tensor(t, device="cuda:0")
    first = None
    for it in range(400):
        idx = torch.randint(0, 8192, (1024,), device="cuda:0",
                            generator=torch.Generator(device="cuda:0").manual_seed(it))
        loss = ctx.srg_train_step(s, Xd[idx].contiguous(), td[idx].contiguous(), lr=1e-3)
        first = loss if first is None else first
    y = ctx.srg_predict(s, Xd).cpu().numpy()
    mse = float(np.mean((y - t) ** 2))
    assert mse < first / 20, (first, mse)


def test_rejects_bad_shapes(ctx):
    import paper_1806_00205_amd as rt
    s = ctx.srg_create(N_IN, 256, 4, seed=0)
    X, t = _data(0, 100)
    with pytest.raises(rt.RtmcError):
        ctx.srg_gradient(s, X, t)  # batch not a multiple of 32
    with pytest.raises(rt.RtmcError):
        ctx.srg_create(N_IN, 128, 4, seed=0)


@pytest.mark.parametrize("n_in,B", [(8, 128 * 3 + 1), (5, 64), (32, 1000), (1, 130), (31, 257)])
def test_fused_prediction_matches_reference_any_width(ctx, n_in, B):
    """The fused inference kernel (all layers in one workgroup, activations in
    LDS) against the FP64 reference, for input counts that fill a different
    part of the padded first layer and a ragged final tile."""
    s = ctx.srg_create(n_in, 256, 4, seed=20 + n_in)
    p = ctx.srg_params(s)
    rng = np.random.default_rng(n_in)
    X = rng.normal(size=(B, n_in)).astype(np.float32)
    y = ctx.srg_predict(s, X).cpu().numpy().astype(np.float64)
    yr, _ = mlp_ref.forward(mlp_ref.gpu_visible_params(p, n_in), mlp_ref.round_bf16(X), n_in)
    err = np.abs(y - yr)
    assert np.max(err) <= 0.03 * np.max(np.abs(yr)) + 1e-3, np.max(err)


def test_fused_prediction_agrees_with_training_forward(ctx):
    """Two GPU forward paths -- the fused inference kernel and the layer-by-layer
    GEMMs of training -- differ only in FP32 summation order: the training loss
    against the fused predictions as targets is ~0."""
    s = ctx.srg_create(N_IN, 256, 4, seed=31)
    X, _ = _data(32, 2048)
    y = ctx.srg_predict(s, X).cpu().numpy()
    loss, _ = ctx.srg_gradient(s, X, y)
    assert loss <= 1e-8 * float(np.mean(y.astype(np.float64) ** 2)) + 1e-12, (loss, float(np.mean(y ** 2)))


@pytest.mark.slow
def test_surrogate_gains_over_rtmc_on_held_out_foams(ctx):
    """End to end at small scale: RTMC traces yields on 96 training foams, the
    network is trained on them with the GPU kernels, and on 16 held-out foams
    it is (a) closer to RTMC than a foam-blind predictor (the mean training
    yield at the nearest (E, theta) points), so it has learned the foam's
    effect, and (b) far faster than RTMC itself at the same error."""
    from paper_1806_00205_amd.surrogate import run_experiment
    out, _ = run_experiment(ctx, n_train=96, points_per_foam=32, n_test=16, train_primaries=20000,
                            eval_primaries=100000, steps=2000, seed=5, log=lambda *a: None, sizes=(24, 32, 40),
                            workers=0, batch_foams=32)
    print(f"held-out MAE {out['mae']:.4f}, foam-blind MAE {out['foam_blind_mae']:.4f}, gain {out['gain']:.3g}")
    # observed: MAE 0.046 against 0.100 foam-blind, gain about 200 (the full-size
    # experiment, 1024 training foams of 64^3-192^3: MAE 0.010, gain about 3000)
    assert out["mae"] < 0.08, out["mae"]
    assert out["mae"] < 0.7 * out["foam_blind_mae"], (out["mae"], out["foam_blind_mae"])
    assert out["gain"] > 50, out["gain"]
