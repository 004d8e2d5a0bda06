"""GPU surrogate-network kernels against the FP64 reference (oracle/mlp.py).

BF16 operands carry 8 significant bits (relative rounding 2^-9), so a dot
product of K terms is accurate to about 2^-9 relative to the sum of the
absolute terms; the tests bound errors by 3e-2 relative to the typical
output magnitude (forward) and to the gradient's norm (backward).  The FP64
reference itself is pinned by central differences on the CPU.
"""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2107_07104_amd import fib as F

from gpu_helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [[5, 64, 64, 64, 4], [57, 128, 128, 57], [3, 40, 7]]
CASES = [(s, "silu") for s in SHAPES] + [([57, 128, 128, 57], "relu"), ([3, 40, 7], "relu")]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def _net(sizes, seed, act="silu"):
    params = M.init_params(sizes, seed)
    rng = np.random.default_rng(seed)
    params = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    net = F.Mlp(sizes, act=act)
    net.set_params(M.flatten(params).astype(np.float32))
    return net, params


@pytest.mark.parametrize("sizes,act", CASES)
def test_forward_matches_reference(sizes, act):
    say(f"[mlp forward] {sizes} {act}")
    net, params = _net(sizes, 5, act)
    rng = np.random.default_rng(6)
    B = 1000  # several chunks and a ragged last chunk
    X = rng.standard_normal((B, sizes[0]))
    O = net.forward(torch.as_tensor(X, dtype=torch.float32, device="cuda")).cpu().numpy()
    ref, _ = M.forward(params, X, act)
    err = np.max(np.abs(O - ref)) / np.max(np.abs(ref))
    say("   rel err", err)
    assert err < 3e-2
    np.testing.assert_array_equal(net.get_params(), M.flatten(params).astype(np.float32))
    net.close()


@pytest.mark.parametrize("sizes,act", CASES)
def test_gradient_matches_reference(sizes, act):
    say(f"[mlp gradient] {sizes} {act}")
    net, params = _net(sizes, 7, act)
    rng = np.random.default_rng(8)
    B = 777
    X = rng.standard_normal((B, sizes[0]))
    T = rng.standard_normal((B, sizes[-1]))
    g, loss = net.gradient(torch.as_tensor(X, dtype=torch.float32, device="cuda"),
                           torch.as_tensor(T, dtype=torch.float32, device="cuda"))
    g = g.cpu().numpy()
    ref = M.flatten(M.backward(params, X, T, act))
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ref_loss = M.loss(params, X, T, act)
    say("   rel err", err, "loss", float(loss.item()), ref_loss)
    assert err < 3e-2
    assert abs(float(loss.item()) - ref_loss) < 3e-2 * ref_loss
    # deterministic: the same call gives the same bits
    g2, _ = net.gradient(torch.as_tensor(X, dtype=torch.float32, device="cuda"),
                         torch.as_tensor(T, dtype=torch.float32, device="cuda"))
    np.testing.assert_array_equal(g, g2.cpu().numpy())
    net.close()


def test_adam_step_and_training_reduce_the_loss():
    sizes = [5, 64, 64, 64, 4]
    say("[mlp adam]")
    net, params = _net(sizes, 9)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((4096, 5))
    # a smooth target the network can fit
    T = np.stack([np.sin(X[:, 0]) + 0.5 * X[:, 1], X[:, 2] * X[:, 3], np.tanh(X[:, 4]),
                  0.3 * X[:, 0] - X[:, 2]], axis=1)
    Xt = torch.as_tensor(X, dtype=torch.float32, device="cuda")
    Tt = torch.as_tensor(T, dtype=torch.float32, device="cuda")
    # one step against the reference update computed from the GPU gradient
    g, _ = net.gradient(Xt, Tt)
    g = g.cpu().numpy().astype(np.float64)
    p0 = net.get_params().astype(np.float64)
    net.adam_step(Xt, Tt, 1e-3)
    p1 = net.get_params().astype(np.float64)
    m = 0.1 * g
    v = 0.001 * g * g
    expect = p0 - 1e-3 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    np.testing.assert_allclose(p1, expect, rtol=1e-5, atol=1e-7)
    losses = []
    loss = torch.empty(1, device="cuda")
    for it in range(300):
        net.adam_step(Xt, Tt, 3e-3, loss)
        if it % 50 == 0:
            losses.append(float(loss.item()))
    say("   losses", losses)
    assert losses[-1] < 0.2 * losses[0]
    net.close()
