"""Pins of the FP64 surrogate-network reference (oracle/mlp.py).

* SiLU and its derivative at closed-form points (SiLU(0) = 0, SiLU'(0) = 1/2,
  SiLU(z) -> z and SiLU'(z) -> 1 for large z, SiLU(z) -> 0 for z -> -inf);
* a one-layer (linear) network's gradient equals the normal-equation form
  (O - T)^T X / (B n) written as a matrix product;
* a hand-computed two-layer example;
* backpropagation of the full network against central finite differences;
* the first Adam step moves every parameter by lr * sign(g) (bias-corrected
  moments give m/sqrt(v) = g/|g| at t = 1);
* Adam beyond the first step: with a constant gradient the bias-corrected
  moments are exactly g and g^2 at every step, so every step moves by
  lr * sign(g) (a wrong step count or bias correction breaks this from t = 2
  on); hand-computed three-step examples with alternating signs and with a
  changing magnitude (these separate beta1 from beta2);
* bfloat16 operand rounding: exact ties-to-even cases, agreement with
  torch's float32 -> bfloat16 conversion, and a network whose weights and
  inputs are bfloat16 values computes its first layer exactly as without
  rounding;
* ReLU: closed forms, a ReLU network whose pre-activations are all positive
  is the product of its affine maps, one whose hidden pre-activations are
  all negative outputs its last bias, and its backpropagation matches
  central differences away from the kinks.
"""
import numpy as np
import pytest

from oracle import mlp as M


def test_silu_closed_forms():
    assert M.silu(0.0) == 0.0
    assert M.silu_grad(0.0) == pytest.approx(0.5)
    assert M.silu(40.0) == pytest.approx(40.0, rel=1e-15)
    assert M.silu_grad(40.0) == pytest.approx(1.0, rel=1e-15)
    assert abs(M.silu(-40.0)) < 1e-15
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(M.silu_grad(z), (M.silu(z + h) - M.silu(z - h)) / (2 * h),
                               rtol=1e-8, atol=1e-10)


def test_linear_network_gradient_is_the_normal_equation_form():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((7, 3))
    T = rng.standard_normal((7, 2))
    params = [(rng.standard_normal((2, 3)), rng.standard_normal(2))]
    (gW, gb), = M.backward(params, X, T)
    O = X @ params[0][0].T + params[0][1]
    np.testing.assert_allclose(gW, (O - T).T @ X / (7 * 2), rtol=1e-13)
    np.testing.assert_allclose(gb, (O - T).sum(axis=0) / (7 * 2), rtol=1e-13)


def test_hand_computed_two_layer_example():
    # x = 1, hidden z = 2x + 0 = 2, a = SiLU(2) = 2/(1+e^-2), out = 3a + 1
    params = [(np.array([[2.0]]), np.array([0.0])), (np.array([[3.0]]), np.array([1.0]))]
    O, _ = M.forward(params, np.array([[1.0]]))
    a = 2.0 / (1.0 + np.exp(-2.0))
    assert O[0, 0] == pytest.approx(3.0 * a + 1.0, rel=1e-15)
    # target 0: loss = 0.5 (3a+1)^2; dL/db2 = 3a+1; dL/dW2 = (3a+1) a;
    # dL/dW1 = (3a+1) * 3 * SiLU'(2) * x
    g = M.backward(params, np.array([[1.0]]), np.array([[0.0]]))
    e = 3.0 * a + 1.0
    s = 1.0 / (1.0 + np.exp(-2.0))
    assert g[1][1][0] == pytest.approx(e)
    assert g[1][0][0, 0] == pytest.approx(e * a)
    assert g[0][0][0, 0] == pytest.approx(e * 3.0 * s * (1.0 + 2.0 * (1.0 - s)))


@pytest.mark.parametrize("sizes", [[5, 8, 8, 4], [6, 12, 5]])
def test_backprop_matches_central_differences(sizes):
    rng = np.random.default_rng(1)
    params = M.init_params(sizes, seed=3)
    X = rng.standard_normal((9, sizes[0]))
    T = rng.standard_normal((9, sizes[-1]))
    g = M.flatten([(gW, gb) for gW, gb in M.backward(params, X, T)])
    theta = M.flatten(params)
    h = 1e-6
    num = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num[i] = (M.loss(M.unflatten(tp, sizes), X, T) - M.loss(M.unflatten(tm, sizes), X, T)) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-10)


def test_first_adam_step_moves_by_lr_times_sign():
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([0.0]))]
    new = M.adam_step(params, grads, {}, lr=0.01)
    np.testing.assert_allclose(new[0][0], [[1.0 - 0.01, -2.0 + 0.01]], rtol=1e-6)
    assert new[0][1][0] == 0.5


def test_adam_with_a_constant_gradient_moves_by_lr_every_step():
    W0, b0 = np.array([[1.0, -2.0, 0.25]]), np.array([0.5])
    gW, gb = np.array([[0.3, -4.0, 1e-3]]), np.array([2.0])
    state, p = {}, [(W0, b0)]
    for t in range(1, 8):
        p = M.adam_step(p, [(gW, gb)], state, lr=0.01)
        np.testing.assert_allclose(p[0][0], W0 - t * 0.01 * gW / (np.abs(gW) + 1e-8),
                                   rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(p[0][1], b0 - t * 0.01 * 2.0 / (2.0 + 1e-8), rtol=1e-12)
    assert state["t"] == 7


def test_adam_hand_computed_three_steps():
    """Kingma & Ba's update by hand (eps = 0).  Gradients +g, -g, +g (|g| fixed, so the
    bias-corrected second moment is g^2 at every step):
      t=1: m = 0.1 g,               m/(1-0.9)   = g,          step -lr
      t=2: m = 0.09 g - 0.1 g,      m/(1-0.81)  = -g/19,      step +lr/19
      t=3: m = -0.009 g + 0.1 g,    m/(1-0.729) = 91 g/271,   step -91 lr/271
    Gradients 1 then 3 on one parameter:
      t=2: m = 0.09 + 0.3 = 0.39,   v = 0.000999 + 0.009 = 0.009999,
           m_hat = 39/19,           v_hat = 0.009999/0.001999 = 9999/1999."""
    lr, g = 0.01, 0.7
    state, p = {}, [(np.array([[0.0]]), np.array([0.0]))]
    want = [-lr, -lr + lr / 19.0, -lr + lr / 19.0 - 91.0 * lr / 271.0]
    for t, sgn in enumerate((1.0, -1.0, 1.0)):
        p = M.adam_step(p, [(np.array([[sgn * g]]), np.array([-sgn * g]))], state, lr=lr, eps=0.0)
        assert p[0][0][0, 0] == pytest.approx(want[t], rel=1e-9)
        assert p[0][1][0] == pytest.approx(-want[t], rel=1e-9)
    state, p = {}, [(np.array([[0.0]]), np.array([0.0]))]
    p = M.adam_step(p, [(np.array([[1.0]]), np.array([1.0]))], state, lr=lr, eps=0.0)
    p = M.adam_step(p, [(np.array([[3.0]]), np.array([3.0]))], state, lr=lr, eps=0.0)
    step2 = (39.0 / 19.0) / np.sqrt(9999.0 / 1999.0)
    assert p[0][0][0, 0] == pytest.approx(-lr - lr * step2, rel=1e-9)


def test_param_count_of_the_surrogate_shapes():
    assert M.n_params([5, 64, 64, 64, 4]) == 8964
    assert M.n_params([57, 128, 128, 57]) == 31289


def test_relu_closed_forms():
    assert M.relu(-1.5) == 0.0 and M.relu(2.5) == 2.5 and M.relu(0.0) == 0.0
    assert M.relu_grad(-1.5) == 0.0 and M.relu_grad(2.5) == 1.0 and M.relu_grad(0.0) == 0.0


def test_relu_network_in_its_linear_region_is_the_product_of_affine_maps():
    rng = np.random.default_rng(4)
    sizes = [3, 6, 5, 2]
    # positive weights and inputs keep every pre-activation positive
    params = [(rng.uniform(0.1, 1.0, (sizes[i + 1], sizes[i])), rng.uniform(0.1, 1.0, sizes[i + 1]))
              for i in range(3)]
    X = rng.uniform(0.1, 1.0, (4, 3))
    O, (zs, _) = M.forward(params, X, "relu")
    assert all((z > 0).all() for z in zs[:-1])
    (W1, b1), (W2, b2), (W3, b3) = params
    A = W3 @ W2 @ W1
    c = W3 @ (W2 @ b1 + b2) + b3
    np.testing.assert_allclose(O, X @ A.T + c, rtol=1e-13)
    # negative first-layer biases switch every hidden unit off: output = b3
    params_off = [(W1, -10.0 * np.ones(6)), (W2, b2), (W3, b3)]
    O_off, _ = M.forward(params_off, X, "relu")
    z2 = np.maximum(b2, 0.0)
    np.testing.assert_allclose(O_off, np.tile(W3 @ z2 + b3, (4, 1)), rtol=1e-13)


def test_relu_backprop_matches_central_differences():
    sizes = [5, 8, 8, 4]
    rng = np.random.default_rng(12)
    params = M.init_params(sizes, seed=13)
    params = [(W, 0.2 * rng.standard_normal(b.shape)) for W, b in params]
    X = rng.standard_normal((9, sizes[0]))
    T = rng.standard_normal((9, sizes[-1]))
    _, (zs, _) = M.forward(params, X, "relu")
    h = 1e-7
    # no hidden pre-activation within reach of a kink for steps of size h
    assert min(np.min(np.abs(z)) for z in zs[:-1]) > 1e-4
    g = M.flatten(M.backward(params, X, T, "relu"))
    theta = M.flatten(params)
    num = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num[i] = (M.loss(M.unflatten(tp, sizes), X, T, "relu") -
                  M.loss(M.unflatten(tm, sizes), X, T, "relu")) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-9)


def test_bf16_rounding():
    one = 1.0
    # spacing of bfloat16 at 1 is 2^-7: halfway cases go to the even neighbour
    assert M.round_bf16(one + 2.0 ** -8) == 1.0
    assert M.round_bf16(one + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7
    assert M.round_bf16(one + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert M.round_bf16(-(one + 3 * 2.0 ** -8)) == -(1.0 + 2 * 2.0 ** -7)
    assert M.round_bf16(0.0) == 0.0
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(3).standard_normal(10000) * 10.0 ** np.random.default_rng(4).integers(-6, 6, 10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.round_bf16(x), ref)


def test_bf16_operands_change_nothing_for_bf16_values():
    rng = np.random.default_rng(5)
    sizes = [6, 8, 3]
    params = [(M.round_bf16(W), b) for W, b in M.init_params(sizes, seed=6)]
    X = M.round_bf16(rng.standard_normal((4, 6)))
    _, (z_plain, _) = M.forward(params, X, "relu")
    _, (z_bf, _) = M.forward(params, X, "relu", bf16=True)
    np.testing.assert_array_equal(z_plain[0], z_bf[0])
