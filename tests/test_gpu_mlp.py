"""GPU MLP kernels against the float64 oracle with the same bfloat16 rounding
points.  Tolerances: float32 accumulation of K <= 256 bf16 products differs
from float64 by ~1e-6 relative, and a bf16 rounding tie can flip one input
by 2^-8; outputs are compared at 1e-3 and gradients at 1e-2 of their scale."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _setup(sfg, shape_t, batch, seed):
    import torch
    rng = np.random.default_rng(seed)
    shape = sfg.mlp_shape(*shape_t)
    P = sfg.mlp_param_count(shape)
    _, total = omlp.layers(*shape_t)
    assert P == total
    params = rng.normal(0, 1.0 / np.sqrt(shape_t[1]), size=P).astype(np.float32)
    x = rng.normal(size=(batch, shape_t[0])).astype(np.float32)
    t = rng.normal(size=(batch, shape_t[2])).astype(np.float32)
    g = dict(params=torch.tensor(params).cuda(), x=torch.tensor(x).cuda(), t=torch.tensor(t).cuda(),
             ws=sfg.workspace(sfg.mlp_workspace_bytes(shape, batch)))
    return shape, params, x, t, g


def _close(a, b, rel):
    scale = np.max(np.abs(b)) + 1e-30
    np.testing.assert_allclose(a, b, rtol=rel, atol=rel * scale)


@pytest.mark.parametrize("shape_t,batch", [((10, 256, 34, 3), 1000), ((10, 256, 34, 3), 1),
                                           ((5, 70, 7, 2), 63), ((3, 40, 130, 1), 257)])
def test_mlp_forward_backward(sfg, shape_t, batch):
    import torch
    shape, params, x, t, g = _setup(sfg, shape_t, batch, 7 + batch)
    y = sfg.mlp_forward(shape, g["params"], g["x"], g["ws"])
    torch.cuda.synchronize()
    yo, cache = omlp.forward(shape_t, params.astype(np.float64), x.astype(np.float64))
    _close(y.cpu().numpy(), yo, 1e-3)
    # loss gradient on the GPU against the oracle's, then backward from the same dy
    lws = sfg.workspace(4 * batch)
    dy, loss = sfg.mlp_mse_grad(y, g["t"], lws)
    dyo, losso = omlp.mse_grad(y.cpu().numpy().astype(np.float64), t.astype(np.float64))
    _close(dy.cpu().numpy(), dyo, 1e-5)
    assert abs(float(loss.item()) - losso) <= 1e-5 * abs(losso)
    grad, dx = sfg.mlp_backward(shape, g["params"], dy, g["ws"], want_dx=True)
    torch.cuda.synchronize()
    go, dxo = omlp.backward(shape_t, params.astype(np.float64), cache, dy.cpu().numpy().astype(np.float64))
    _close(grad.cpu().numpy(), go, 1e-2)
    _close(dx.cpu().numpy(), dxo, 1e-2)


def test_mse_mask_and_weights(sfg):
    import torch
    rng = np.random.default_rng(5)
    y = rng.normal(size=(50, 9)).astype(np.float32)
    t = rng.normal(size=(50, 9)).astype(np.float32)
    mask = (rng.uniform(size=y.shape) > 0.3).astype(np.float32)
    w = rng.uniform(0.1, 3, size=9).astype(np.float32)
    dy, loss = sfg.mlp_mse_grad(torch.tensor(y).cuda(), torch.tensor(t).cuda(), sfg.workspace(200),
                                mask=torch.tensor(mask).cuda(), col_weight=torch.tensor(w).cuda())
    dyo, losso = omlp.mse_grad(y.astype(np.float64), t.astype(np.float64), mask, w)
    _close(dy.cpu().numpy(), dyo, 1e-6)
    assert abs(float(loss.item()) - losso) <= 1e-5 * losso


def test_adam_matches_oracle(sfg):
    import torch
    rng = np.random.default_rng(6)
    p = rng.normal(size=1000).astype(np.float32)
    po, mo, vo = p.astype(np.float64), np.zeros(1000), np.zeros(1000)
    pg, m, v = torch.tensor(p).cuda(), torch.zeros(1000).cuda(), torch.zeros(1000).cuda()
    for step in range(1, 6):
        gr = rng.normal(size=1000).astype(np.float32)
        sfg.adam_step(pg, torch.tensor(gr).cuda(), m, v, step, lr=1e-2)
        po, mo, vo = omlp.adam(po, gr.astype(np.float64), mo, vo, step, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pg.cpu().numpy(), po, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(sfg):
    """A few hundred Adam steps on a smooth synthetic regression."""
    import torch
    shape_t = (4, 64, 3, 2)
    shape = sfg.mlp_shape(*shape_t)
    rng = np.random.default_rng(8)
    B = 512
    x = rng.uniform(-1, 1, size=(B, 4)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]), x[:, 1] * x[:, 2], np.cos(x[:, 3])], 1).astype(np.float32)
    P = sfg.mlp_param_count(shape)
    params = torch.tensor(rng.normal(0, 0.3, size=P).astype(np.float32)).cuda()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    xg, tg = torch.tensor(x).cuda(), torch.tensor(t).cuda()
    ws, lws = sfg.workspace(sfg.mlp_workspace_bytes(shape, B)), sfg.workspace(4 * B)
    losses = []
    for step in range(1, 401):
        y = sfg.mlp_forward(shape, params, xg, ws)
        dy, loss = sfg.mlp_mse_grad(y, tg, lws)
        grad, _ = sfg.mlp_backward(shape, params, dy, ws)
        sfg.adam_step(params, grad, m, v, step, lr=3e-3)
        if step in (1, 400):
            losses.append(float(loss.item()))
    assert losses[1] < 0.1 * losses[0], losses


def _fused_step(sfg, shape, batch, params, x, t, rows=None, mask=None, cw=None, lr=1e-2):
    import torch
    p = params.clone()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    grad = torch.empty_like(p)
    lr_dev = torch.tensor([lr], dtype=torch.float32, device="cuda")
    step_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = sfg.workspace(sfg.mlp_train_workspace_bytes(shape, batch))
    loss = sfg.mlp_train_step(shape, batch, p, x, t, m, v, lr_dev, step_dev, ws, rows=rows, mask=mask,
                              col_weight=cw, grad=grad)
    torch.cuda.synchronize()
    assert int(step_dev.item()) == 1
    return p, grad, float(loss.item())


@pytest.mark.parametrize("shape_t,batch", [((10, 256, 34, 3), 1000), ((10, 256, 34, 3), 4096), ((10, 256, 34, 3), 1),
                                           ((5, 70, 7, 2), 63), ((3, 40, 130, 1), 257)])
def test_fused_step_matches_oracle(sfg, shape_t, batch):
    """mlp_train_step: the gradient it applies equals the oracle's (forward,
    loss gradient and backward in float64 with the same bf16 rounding points)
    at the tolerances above, its loss the oracle's, and the parameters after
    the step the oracle's Adam applied to that gradient."""
    shape, params, x, t, g = _setup(sfg, shape_t, batch, 70 + batch)
    p, grad, loss = _fused_step(sfg, shape, batch, g["params"], g["x"], g["t"])
    yo, cache = omlp.forward(shape_t, params.astype(np.float64), x.astype(np.float64))
    dyo, losso = omlp.mse_grad(yo, t.astype(np.float64))
    go, _ = omlp.backward(shape_t, params.astype(np.float64), cache, dyo)
    _close(grad.cpu().numpy(), go, 1e-2)
    assert abs(loss - losso) <= 1e-3 * abs(losso), (loss, losso)
    gpu_grad = grad.cpu().numpy().astype(np.float64)
    po, _, _ = omlp.adam(params.astype(np.float64), gpu_grad, np.zeros_like(gpu_grad), np.zeros_like(gpu_grad), 1,
                         lr=1e-2)
    np.testing.assert_allclose(p.cpu().numpy(), po, rtol=1e-5, atol=1e-6)


def test_fused_step_rows_mask_weights_equal_unfused(sfg):
    """A shuffled batch (rows), a mask and column weights: the fused step's
    gradient and loss equal the unfused kernels' on the gathered batch
    (float32 summation order only)."""
    import torch
    shape_t, batch, N = (10, 256, 34, 3), 777, 2000
    shape, params, _, _, g = _setup(sfg, shape_t, 1, 9)
    rng = np.random.default_rng(10)
    X = torch.tensor(rng.normal(size=(N, 10)).astype(np.float32)).cuda()
    T = torch.tensor(rng.normal(size=(N, 34)).astype(np.float32)).cuda()
    M = torch.tensor((rng.uniform(size=(N, 34)) > 0.2).astype(np.float32)).cuda()
    cw = torch.tensor(rng.uniform(0.2, 2.0, size=34).astype(np.float32)).cuda()
    rows = torch.tensor(rng.permutation(N)[:batch]).cuda()
    _, grad, loss = _fused_step(sfg, shape, batch, g["params"], X, T, rows=rows, mask=M, cw=cw)
    ws = sfg.workspace(sfg.mlp_workspace_bytes(shape, batch))
    y = sfg.mlp_forward(shape, g["params"], X[rows].contiguous(), ws)
    dy, loss_u = sfg.mlp_mse_grad(y, T[rows].contiguous(), sfg.workspace(4 * batch), mask=M[rows].contiguous(),
                                  col_weight=cw)
    grad_u, _ = sfg.mlp_backward(shape, g["params"], dy, ws)
    torch.cuda.synchronize()
    _close(grad.cpu().numpy(), grad_u.cpu().numpy(), 1e-3)
    assert abs(loss - float(loss_u.item())) <= 1e-5 * abs(loss)


def test_fused_step_graph_replays_equal_eager(sfg):
    """The fused step captured into a HIP graph: every replay, with eager
    library work and synchronisations between replays, equals the eager
    step on the same state."""
    import torch
    shape_t, batch = (10, 256, 34, 3), 512
    shape, params, x, t, g = _setup(sfg, shape_t, batch, 12)
    ws = sfg.workspace(sfg.mlp_train_workspace_bytes(shape, batch))
    lr_dev = torch.tensor([3e-3], dtype=torch.float32, device="cuda")

    def state():
        return (g["params"].clone(), torch.zeros_like(g["params"]), torch.zeros_like(g["params"]),
                torch.zeros(1, dtype=torch.int32, device="cuda"))

    pe, me, ve, se = state()
    eager = []
    for _ in range(3):
        sfg.mlp_train_step(shape, batch, pe, g["x"], g["t"], me, ve, lr_dev, se, ws)
        eager.append(pe.clone())
    pg, mg, vg, sg_ = state()
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    sfg.mlp_train_step(shape, batch, pg, g["x"], g["t"], mg, vg, lr_dev, sg_, ws, loss=loss)  # eager first step
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sfg.mlp_train_step(shape, batch, pg, g["x"], g["t"], mg, vg, lr_dev, sg_, ws, loss=loss)
    torch.cuda.synchronize()
    # capture does not run the step: state is still after one step
    assert torch.equal(pg, eager[0])
    for rep in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(pg, eager[rep + 1]), rep
        sfg.mlp_forward(shape, pg, g["x"], sfg.workspace(sfg.mlp_workspace_bytes(shape, batch)))  # eager work between
        torch.cuda.synchronize()
    assert int(sg_.item()) == 3


def _rne_bf16(v):
    """float32 -> bfloat16 -> float64 by the definition of rounding to nearest
    even on the bit pattern (finite inputs)."""
    u = v.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _rounding_cases(rng, n):
    """n float32 values in [2^-8, 2^9) of either sign: random patterns, exact
    ties with even and odd upper halves, and the neighbours of ties."""
    hi = (rng.integers(0x3B80, 0x4400, size=n) | (rng.integers(0, 2, size=n) << 15)).astype(np.uint32)
    lo = rng.choice(np.array([0x8000, 0x7FFF, 0x8001, 0x0000, 0xFFFF, 0x0001], dtype=np.uint32), size=n)
    lo = np.where(rng.uniform(size=n) < 0.3, rng.integers(0, 1 << 16, size=n).astype(np.uint32), lo)
    return ((hi << 16) | lo).astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("fused", [False, True])
def test_input_rounding_is_nearest_even(sfg, fused):
    """At batch one the first layer's weight gradient is dZb_0[j] * bf16(x_i),
    a product of two bf16 values and so exact in float32: its ratio to the
    entry of x_0 = 1 is bf16(x_i) itself.  Every such ratio equals rounding to
    nearest even by its definition, ties (both parities) and their
    neighbours included, in the unfused kernels and in the fused step."""
    import torch
    rng = np.random.default_rng(77 + fused)
    D = 256 if fused else 4096
    shape_t = (D, 16, 8, 1)
    shape = sfg.mlp_shape(*shape_t)
    P = sfg.mlp_param_count(shape)
    checked = 0
    for call in range(8 if fused else 2):
        params = rng.normal(0, 1.0 / D, size=P).astype(np.float32)
        x = np.concatenate([[np.float32(1.0)], _rounding_cases(rng, D - 1)]).astype(np.float32)[None, :]
        t = rng.normal(size=(1, 8)).astype(np.float32)
        pt, xt, tt = torch.tensor(params).cuda(), torch.tensor(x).cuda(), torch.tensor(t).cuda()
        if fused:
            _, grad, _ = _fused_step(sfg, shape, 1, pt, xt, tt)
            grad = grad.cpu().numpy()
        else:
            ws = sfg.workspace(sfg.mlp_workspace_bytes(shape, 1))
            y = sfg.mlp_forward(shape, pt, xt, ws)
            dy, _ = sfg.mlp_mse_grad(y, tt, sfg.workspace(4))
            grad, _ = sfg.mlp_backward(shape, pt, dy, ws)
            torch.cuda.synchronize()
            grad = grad.cpu().numpy()
        W0 = grad[:16 * D].reshape(16, D).astype(np.float64)
        j = int(np.argmax(np.abs(W0[:, 0])))
        assert W0[j, 0] != 0.0
        np.testing.assert_array_equal(W0[j] / W0[j, 0], _rne_bf16(x[0]), err_msg=f"call {call}")
        checked += D
    assert checked >= 2000
