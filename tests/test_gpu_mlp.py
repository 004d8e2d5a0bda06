"""GPU surrogate-network kernels against the FP64 reference (oracle/mlp.py).

BF16 operands carry 8 significant bits (relative rounding 2^-9), so a dot
product of K terms is accurate to about 2^-9 relative to the sum of the
absolute terms; the tests bound errors by 3e-2 relative to the typical
output magnitude (forward) and, element by element, to the largest
gradient entry of the same weight matrix or bias vector (backward; for
ReLU against the reference with bfloat16 operands, whose 0/1 derivative
decisions are those of the device).  Adam
runs on the FP32 masters: over ten steps fed with the GPU's own gradients
it matches the FP64 update of oracle/mlp.py to FP32 rounding.  The FP64
reference itself is pinned on the CPU (central differences, closed forms).
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
    ref_layers = M.backward(params, X, T, act)
    ref = M.flatten(ref_layers)
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    ref_loss = M.loss(params, X, T, act)
    say("   rel err", err, "loss", float(loss.item()), ref_loss)
    assert err < 3e-2
    # element by element, per layer: every weight and bias gradient against
    # the largest entry of its own array.  ReLU's derivative is a 0/1
    # decision on the sign of each pre-activation, so that reference takes
    # it from bfloat16-rounded operands as the matrix cores do (a
    # pre-activation within BF16 rounding of zero would otherwise switch a
    # sample's whole contribution through that unit)
    if act == "relu":
        ref_layers = M.backward(params, X, T, act, bf16=True)
    gl = M.unflatten(g.astype(np.float64), sizes)
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(gl, ref_layers)):
        for name, a, r in (("W", gW, rW), ("b", gb, rb)):
            scale = np.max(np.abs(r))
            worst = np.max(np.abs(a - r)) / scale
            say(f"   layer {li + 1} {name}{list(r.shape)}: max |g - g_ref| / max |g_ref| = "
                f"{worst:.2e}")
            assert worst < 3e-2, (li, name)
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


@pytest.mark.parametrize("sizes,act", [([5, 64, 64, 64, 4], "silu"), ([57, 128, 128, 57], "relu")])
def test_adam_matches_the_reference_over_ten_steps(sizes, act):
    """Ten GPU Adam steps, each on the gradient the GPU computes at the
    current parameters (deterministic: the same bits the step uses), against
    the FP64 Adam of oracle/mlp.py fed with those gradients."""
    say(f"[mlp adam x10] {sizes} {act}")
    net, params = _net(sizes, 12, act)
    rng = np.random.default_rng(13)
    B = 1500
    Xt = torch.as_tensor(rng.standard_normal((B, sizes[0])), dtype=torch.float32, device="cuda")
    Tt = torch.as_tensor(rng.standard_normal((B, sizes[-1])), dtype=torch.float32, device="cuda")
    state = {}
    lr = 3e-3
    for t in range(1, 11):
        # the reference steps from the GPU's FP32 parameters of this step, so
        # parameter rounding does not accumulate; its moments are its own
        p_prev = M.unflatten(net.get_params().astype(np.float64), sizes)
        g, _ = net.gradient(Xt, Tt)
        g = M.unflatten(g.cpu().numpy().astype(np.float64), sizes)
        net.adam_step(Xt, Tt, lr)
        flat_ref = M.flatten(M.adam_step(p_prev, g, state, lr=lr))
        p_gpu = net.get_params().astype(np.float64)
        # FP32 parameters, moments and update: two ulp of each parameter plus
        # a small fraction of the step size
        tol = 3e-7 * np.abs(flat_ref) + 1e-5 * lr
        bad = np.abs(p_gpu - flat_ref) > tol
        say(f"   step {t}: max |p - p_ref| {np.max(np.abs(p_gpu - flat_ref)):.2e}, "
            f"beyond tolerance {int(bad.sum())}")
        assert not bad.any()
        assert state["t"] == t
    net.close()
