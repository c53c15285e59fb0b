"""The learned warm start's HIP kernels (BF16 MFMA products, SiLU, MSE, Adam,
features, state mapping) against the FP64 oracle in oracle/mlp.py, through
the C ABI."""
import sys

import numpy as np
import pytest

from oracle import mlp as OM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BF16_TOL = 2e-2  # BF16 operands: 8-bit significands, FP32 accumulation


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def api():
    from paper_2404_14195_amd import api as A
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return A


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def init_theta(seed):
    """torch.nn.Linear's default ranges, U(-1/sqrt(in), 1/sqrt(in))."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(OM.SIZES[:-1], OM.SIZES[1:]):
        a = 1.0 / np.sqrt(i)
        parts += [rng.uniform(-a, a, o * i), rng.uniform(-a, a, o)]
    return np.concatenate(parts).astype(np.float32)


def blocks(vec):
    out, at = [], 0
    for i, o in zip(OM.SIZES[:-1], OM.SIZES[1:]):
        out.append(vec[at:at + o * i])
        at += o * i
        out.append(vec[at:at + o])
        at += o
    return out


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b)


class Net:
    def __init__(self, api, theta, batch):
        self.api = api
        self.master = dev(theta, torch.float32)
        self.packed = torch.empty(api.mlp_packed_count(), dtype=torch.bfloat16, device="cuda")
        api.mlp_pack(self.master, self.packed)
        self.ws = api.mlp_workspace(batch, True)


@pytest.mark.parametrize("M,N,K", [(200, 37, 96), (64, 128, 32), (130, 5, 64), (1, 16, 32)])
def test_gemm_bf16_exact_on_small_integers(api, M, N, K):
    """Small integers are exact in BF16 and their products and sums exact in
    FP32, so the MFMA product must equal the integer product bit for bit; a
    wrong lane layout or a transposed operand cannot pass."""
    rng = np.random.default_rng(M * 1000 + N)
    A = rng.integers(-8, 9, (M, K))
    Bt = rng.integers(-8, 9, (N, K))
    C = api.gemm_bf16(dev(A, torch.bfloat16), dev(Bt, torch.bfloat16))
    np.testing.assert_array_equal(C.cpu().numpy(), (A @ Bt.T).astype(np.float32))


def test_gemm_bf16_argument_errors(api):
    from paper_2404_14195_amd._lib import MPFError
    A = torch.zeros((4, 40), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(MPFError):
        api.gemm_bf16(A, A)  # K = 40 is not a multiple of 32


def test_forward_parity(api):
    theta = init_theta(1)
    B = 1000  # 15 full 64-row tiles and a ragged one
    x = np.random.default_rng(2).normal(size=(B, 5)).astype(np.float32)
    net = Net(api, theta, B)
    y = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    api.mlp_forward(net.master, net.packed, dev(x, torch.float32), y, net.ws)
    y_o, _ = OM.forward(theta.astype(np.float64), x.astype(np.float64))
    yg = y.cpu().numpy()
    print(f"[mlp fwd] rel err {rel(yg, y_o):.3e}", flush=True)
    assert rel(yg, y_o) <= BF16_TOL
    assert np.abs(yg - y_o).max() <= 5 * BF16_TOL * np.abs(y_o).max()
    # inference and training mode give the same outputs
    y2 = torch.empty_like(y)
    api.mlp_forward(net.master, net.packed, dev(x, torch.float32), y2, net.ws, train=True)
    assert torch.equal(y, y2)


def test_forward_rows_gather(api):
    theta = init_theta(3)
    x = np.random.default_rng(4).normal(size=(300, 5)).astype(np.float32)
    rows = np.random.default_rng(5).permutation(300)[:129]
    net = Net(api, theta, 300)
    ya = torch.empty((129, 4), dtype=torch.float32, device="cuda")
    yb = torch.empty((129, 4), dtype=torch.float32, device="cuda")
    api.mlp_forward(net.master, net.packed, dev(x, torch.float32), ya, net.ws, rows=dev(rows, torch.int64))
    api.mlp_forward(net.master, net.packed, dev(x[rows], torch.float32), yb, net.ws)
    assert torch.equal(ya, yb)


@pytest.mark.parametrize("B", [700, 70000])
def test_backward_parity_and_determinism(api, B):
    """Gradients of every parameter block within the BF16 tolerance of the
    FP64 oracle's, bitwise identical on a second call."""
    theta = init_theta(6)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(B, 5)).astype(np.float32)
    dy = rng.normal(size=(B, 4)).astype(np.float32)
    net = Net(api, theta, B)
    y = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    grad = torch.empty(theta.size, dtype=torch.float32, device="cuda")
    api.mlp_forward(net.master, net.packed, dev(x, torch.float32), y, net.ws, train=True)
    api.mlp_backward(net.packed, dev(dy, torch.float32), grad, net.ws)
    g1 = grad.cpu().numpy()
    api.mlp_backward(net.packed, dev(dy, torch.float32), grad, net.ws)
    assert np.array_equal(g1, grad.cpu().numpy())
    _, cache = OM.forward(theta.astype(np.float64), x.astype(np.float64))
    g_o = OM.backward(theta.astype(np.float64), cache, dy.astype(np.float64))
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    errs = {nm: rel(a, b) for nm, a, b in zip(names, blocks(g1), blocks(g_o))}
    print(f"[mlp bwd B={B}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) <= BF16_TOL


def test_mse_parity(api):
    rng = np.random.default_rng(8)
    B = 333
    y = rng.normal(size=(B, 4)).astype(np.float32)
    t = rng.normal(size=(500, 4)).astype(np.float32)
    rows = rng.integers(0, 500, B)
    dy = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    api.mlp_mse(dev(y, torch.float32), dev(t, torch.float32), dy, loss, api.reduce_workspace(4 * B, "cuda"),
                rows=dev(rows, torch.int64))
    l_o, dy_o = OM.mse(y.astype(np.float64), t[rows].astype(np.float64))
    assert loss.item() == pytest.approx(l_o, rel=1e-6)
    np.testing.assert_allclose(dy.cpu().numpy(), dy_o, rtol=1e-6, atol=1e-12)


def test_adam_parity(api):
    rng = np.random.default_rng(9)
    n = 34308
    p = rng.normal(size=n).astype(np.float32)
    pg, mg, vg = dev(p, torch.float32), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    po, mo, vo = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        api.adam_step(pg, dev(g, torch.float32), mg, vg, t, 1e-3)
        po, mo, vo = OM.adam_step(po, g.astype(np.float64), mo, vo, t, 1e-3)
    np.testing.assert_allclose(pg.cpu().numpy(), po, rtol=0, atol=1e-6)
    np.testing.assert_allclose(mg.cpu().numpy(), mo, rtol=1e-5, atol=1e-7)


def test_features_parity(api, small_cloud):
    c = small_cloud
    x = api.mlp_features(dev(c.pos.T, torch.float64), c.r, 0.77)
    x_o = OM.features(c.pos, c.r, 0.77)
    np.testing.assert_allclose(x.cpu().numpy(), x_o, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_to_state_parity(api, dtype):
    rng = np.random.default_rng(10)
    n, n_int = 1234, 1000
    y = rng.normal(size=(n, 4)).astype(np.float32)
    v = torch.empty((3, n), dtype=dtype, device="cuda")
    p = torch.empty(n, dtype=dtype, device="cuda")
    vmax = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    api.mlp_to_state(dev(y, torch.float32), n_int, 0.05, 2.0, v, p, vmax)
    v_o, p_o = OM.to_state(y.astype(np.float64), n_int, 0.05, 2.0)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    np.testing.assert_allclose(v.cpu().numpy(), v_o, rtol=tol, atol=tol * 0.1)
    np.testing.assert_allclose(p.cpu().numpy(), p_o, rtol=tol, atol=tol * 2)
    assert vmax.item() == pytest.approx(np.sqrt((v_o ** 2).sum(0)).max(), rel=tol)


def test_training_tracks_the_oracle(api):
    """The same 150 Adam steps on a smooth regression, GPU (BF16 products)
    and oracle (FP64): both reduce the loss tenfold and the two loss curves
    stay within a factor 1.5 of each other."""
    rng = np.random.default_rng(11)
    N, B = 4096, 512
    x = rng.uniform(-0.5, 0.5, (N, 5)).astype(np.float32)
    t = np.column_stack([np.sin(3 * x[:, 0]), x[:, 1] * x[:, 2], np.exp(-4 * (x ** 2).sum(1)), x[:, 3] - x[:, 4]])
    t = t.astype(np.float32)
    theta = init_theta(12)
    net = Net(api, theta, B)
    xg, tg = dev(x, torch.float32), dev(t, torch.float32)
    y = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(theta.size, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    rws = api.reduce_workspace(4 * B, "cuda")
    th, mo, vo = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    lg, lo = [], []
    lr = 2e-3
    for step in range(1, 151):
        rows = rng.integers(0, N, B)
        rg = dev(rows, torch.int64)
        api.mlp_forward(net.master, net.packed, xg, y, net.ws, rows=rg, train=True)
        api.mlp_mse(y, tg, dy, loss, rws, rows=rg)
        api.mlp_backward(net.packed, dy, grad, net.ws)
        api.adam_step(net.master, grad, m, v, step, lr)
        api.mlp_pack(net.master, net.packed)
        lg.append(loss.item())
        yo, cache = OM.forward(th, x[rows].astype(np.float64))
        l, d = OM.mse(yo, t[rows].astype(np.float64))
        lo.append(l)
        th, mo, vo = OM.adam_step(th, OM.backward(th, cache, d), mo, vo, step, lr)
    a, b = np.mean(lg[-10:]), np.mean(lo[-10:])
    print(f"[mlp train] loss {lg[0]:.3e} -> gpu {a:.3e}, oracle {b:.3e}", flush=True)
    assert a < 0.1 * lg[0] and b < 0.1 * lo[0]
    assert 1 / 1.5 <= a / b <= 1.5


def test_mlp_argument_errors(api):
    from paper_2404_14195_amd._lib import MPFError
    net = Net(api, init_theta(0), 200)
    x = torch.zeros((200, 5), dtype=torch.float32, device="cuda")
    y = torch.empty((200, 4), dtype=torch.float32, device="cuda")
    small = api.mlp_workspace(8, False)  # sized for one 64-row tile, the batch needs four
    with pytest.raises(MPFError):
        api.mlp_forward(net.master, net.packed, x, y, small)
    with pytest.raises(MPFError):
        api.adam_step(net.master, net.master, net.master, net.master, 0, 1e-3)  # step must be >= 1


def test_fused_training_loop_matches_separate_calls(api):
    """mpf_mlp_train runs exactly the kernels of the separate calls in the same
    order, so three steps through it and through the separate calls give
    identical parameters, moments and loss."""
    rng = np.random.default_rng(13)
    N, B = 3000, 256
    x = dev(rng.normal(size=(N, 5)).astype(np.float32), torch.float32)
    t = dev(rng.normal(size=(N, 4)).astype(np.float32), torch.float32)
    rows = dev(rng.permutation(N)[:3 * B], torch.int64)
    theta = init_theta(14)
    a, b = Net(api, theta, B), Net(api, theta, B)
    ma, va, ga = (torch.zeros(theta.size, device="cuda") for _ in range(3))
    mb, vb, gb = (torch.zeros(theta.size, device="cuda") for _ in range(3))
    y = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rws = api.reduce_workspace(4 * B, "cuda")
    total = 0.0
    lr, ratio = 1e-3, 1.0  # a constant rate: both sides then pass the same float
    for i in range(3):
        r = rows[i * B:(i + 1) * B]
        api.mlp_forward(a.master, a.packed, x, y, a.ws, rows=r, train=True)
        api.mlp_mse(y, t, dy, loss, rws, rows=r)
        total += loss.item()
        api.mlp_backward(a.packed, dy, ga, a.ws)
        api.adam_step(a.master, ga, ma, va, i + 1, lr * ratio ** i)
        api.mlp_pack(a.master, a.packed)
    loss_sum = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.mlp_train(b.master, b.packed, mb, vb, gb, x, t, rows, B, 0, lr, ratio, loss_sum, api.mlp_train_workspace(B))
    assert torch.equal(a.master, b.master) and torch.equal(ma, mb) and torch.equal(va, vb)
    assert torch.equal(a.packed, b.packed)
    assert loss_sum.item() == pytest.approx(total, rel=1e-15)


@pytest.mark.parametrize("n,count", [(1, 1), (1000, 1000), (4097, 4097), (12_800_000, 12_800_000), (300, 129)])
def test_shuffle_rows_is_a_seeded_permutation(api, n, count):
    a = api.shuffle_rows(n, count, 7).cpu().numpy()
    b = api.shuffle_rows(n, count, 7).cpu().numpy()
    c = api.shuffle_rows(n, count, 8).cpu().numpy()
    assert np.array_equal(a, b)
    assert len(np.unique(a)) == count and a.min() >= 0 and a.max() < n
    if count == n:
        assert np.array_equal(np.sort(a), np.arange(n))
    if n > 1:
        assert not np.array_equal(a, c)


@pytest.mark.parametrize("B", [37, 700, 70001])
def test_fused_gradient_parity_and_determinism(api, B):
    """The fused training step's gradient and loss of one batch (gathered
    through rows, a ragged last tile) against the FP64 oracle within the BF16
    tolerance, against the layered kernels to rounding, and bitwise identical
    on a second call."""
    theta = init_theta(16)
    rng = np.random.default_rng(17)
    N = B + 50
    x = rng.normal(size=(N, 5)).astype(np.float32)
    t = rng.normal(size=(N, 4)).astype(np.float32)
    rows = rng.permutation(N)[:B]
    net = Net(api, theta, B)
    xg, tg, rg = dev(x, torch.float32), dev(t, torch.float32), dev(rows, torch.int64)
    grad = torch.empty(theta.size, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = api.mlp_fused_workspace(B)
    api.mlp_grad_fused(net.master, net.packed, xg, tg, grad, ws, rows=rg, loss=loss)
    g1, l1 = grad.cpu().numpy(), loss.item()
    api.mlp_grad_fused(net.master, net.packed, xg, tg, grad, ws, rows=rg, loss=loss)
    assert np.array_equal(g1, grad.cpu().numpy()) and l1 == loss.item()
    yo, cache = OM.forward(theta.astype(np.float64), x[rows].astype(np.float64))
    l_o, d_o = OM.mse(yo, t[rows].astype(np.float64))
    g_o = OM.backward(theta.astype(np.float64), cache, d_o)
    names = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    errs = {nm: rel(a, b) for nm, a, b in zip(names, blocks(g1), blocks(g_o))}
    # the layered kernels on the same batch
    y = torch.empty((B, 4), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    loss2 = torch.empty(1, dtype=torch.float64, device="cuda")
    gl = torch.empty_like(grad)
    api.mlp_forward(net.master, net.packed, xg, y, net.ws, rows=rg, train=True)
    api.mlp_mse(y, tg, dy, loss2, api.reduce_workspace(4 * B, "cuda"), rows=rg)
    api.mlp_backward(net.packed, dy, gl, net.ws)
    e_lay = {nm: rel(a, b) for nm, a, b in zip(names, blocks(g1), blocks(gl.cpu().numpy()))}
    print(f"[mlp fused B={B}] loss {l1:.6e} (oracle {l_o:.6e}, layered {loss2.item():.6e}); vs oracle "
          + " ".join(f"{k}={v:.2e}" for k, v in errs.items()) + "; vs layered "
          + " ".join(f"{k}={v:.2e}" for k, v in e_lay.items()), flush=True)
    assert l1 == pytest.approx(l_o, rel=BF16_TOL)
    assert max(errs.values()) <= BF16_TOL
    assert max(e_lay.values()) <= 1e-2


def test_fused_training_tracks_the_layered_training(api):
    """100 fused Adam steps (one host call) and 100 layered ones from the same
    parameters on the same minibatches: both reduce the loss and end within a
    factor 1.2 of each other."""
    rng = np.random.default_rng(21)
    N, B, steps = 8192, 1024, 100
    x = rng.uniform(-0.5, 0.5, (N, 5)).astype(np.float32)
    t = np.column_stack([np.sin(3 * x[:, 0]), x[:, 1] * x[:, 2], np.exp(-4 * (x ** 2).sum(1)), x[:, 3] - x[:, 4]])
    t = t.astype(np.float32)
    theta = init_theta(22)
    xg, tg = dev(x, torch.float32), dev(t, torch.float32)
    rows = dev(rng.integers(0, N, steps * B), torch.int64)
    out = {}
    for name, fused in (("fused", True), ("layered", False)):
        net = Net(api, theta, B)
        m = torch.zeros(theta.size, dtype=torch.float32, device="cuda")
        v = torch.zeros_like(m)
        grad = torch.empty_like(m)
        ls = torch.zeros(1, dtype=torch.float64, device="cuda")
        if fused:
            api.mlp_train_fused(net.master, net.packed, m, v, grad, xg, tg, rows[:B * 10], B, 0, 2e-3, 1.0, ls,
                                api.mlp_fused_workspace(B))
            first = ls.item() / 10
            api.mlp_train_fused(net.master, net.packed, m, v, grad, xg, tg, rows[B * 10:], B, 10, 2e-3, 1.0, ls,
                                api.mlp_fused_workspace(B))
        else:
            ws = api.mlp_train_workspace(B)
            api.mlp_train(net.master, net.packed, m, v, grad, xg, tg, rows[:B * 10], B, 0, 2e-3, 1.0, ls, ws)
            first = ls.item() / 10
            api.mlp_train(net.master, net.packed, m, v, grad, xg, tg, rows[B * 10:], B, 10, 2e-3, 1.0, ls, ws)
        out[name] = (first, ls.item() / (steps - 10))
    print(f"[mlp fused training] {out}", flush=True)
    for first, last in out.values():
        assert last < 0.2 * first
    assert 1 / 1.2 <= out["fused"][1] / out["layered"][1] <= 1.2


def test_fused_update_equals_grad_adam_and_pack(api):
    """The fused training loop's reduction kernel also takes the Adam step and
    rewrites the BF16 copies.  Three steps of mpf_mlp_train_fused against the
    same steps as mpf_mlp_grad_fused + mpf_adam_step + mpf_mlp_pack: the
    gradient sums are the same kernel's, so the parameters and moments agree
    to the rounding of the Adam expression (1e-6), and the packed copy equals
    mpf_mlp_pack of the fused run's own parameters bit for bit (the same
    round-to-nearest-even of the same values, padding untouched)."""
    rng = np.random.default_rng(23)
    N, B = 5000, 700  # a ragged last tile
    x = dev(rng.normal(size=(N, 5)).astype(np.float32), torch.float32)
    t = dev(rng.normal(size=(N, 4)).astype(np.float32), torch.float32)
    rows = dev(rng.permutation(N)[:3 * B], torch.int64)
    theta = init_theta(24)
    a, b = Net(api, theta, B), Net(api, theta, B)
    ma, va, ga = (torch.zeros(theta.size, device="cuda") for _ in range(3))
    mb, vb, gb = (torch.zeros(theta.size, device="cuda") for _ in range(3))
    ws = api.mlp_fused_workspace(B)
    lr = 1e-3
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for i in range(3):
        api.mlp_grad_fused(a.master, a.packed, x, t, ga, ws, rows=rows[i * B:(i + 1) * B], loss=loss)
        api.adam_step(a.master, ga, ma, va, i + 1, lr)
        api.mlp_pack(a.master, a.packed)
    loss_sum = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.mlp_train_fused(b.master, b.packed, mb, vb, gb, x, t, rows, B, 0, lr, 1.0, loss_sum, ws)
    assert torch.allclose(a.master, b.master, rtol=1e-6, atol=1e-9)
    assert torch.allclose(ma, mb, rtol=1e-6, atol=1e-12) and torch.allclose(va, vb, rtol=1e-6, atol=1e-15)
    ref = torch.empty_like(b.packed)
    api.mlp_pack(b.master, ref)
    assert torch.equal(ref.view(torch.int16), b.packed.view(torch.int16))
