"""Pins of the oracle's 1D diffusion step (lumped linear FE + Crank-Nicolson)
and of its Thomas solver.

* Thomas against LAPACK's pivoted LU (numpy.linalg.solve) on random
  diagonally dominant systems and on the actual Crank-Nicolson matrices.
* Closed-form eigenmodes (Crank-Nicolson and implicit Euler): with the
  lumped mass matrix and no-flux ends,
  v_k(i) = cos(k pi i / (N-1)) is an exact eigenvector of M_L^{-1} K with
  eigenvalue -(4/h^2) sin^2(k pi / (2 (N-1))), so one Crank-Nicolson step
  multiplies it by (1 + dt c lam / 2) / (1 - dt c lam / 2), c = sigma/(Am Cm).
* Discrete charge conservation: sum_i w_i V_i with the lumped weights
  w = h (1/2, 1, ..., 1, 1/2) is invariant (1^T K = 0).
* Discrete maximum principle when r = c dt / h^2 <= 1.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _dd_system(rng, n):
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    d = np.abs(a) + np.abs(c) + rng.uniform(0.1, 2.0, n)
    d *= rng.choice([-1.0, 1.0], n)
    b = rng.standard_normal(n)
    return a, d, c, b


def _dense(a, d, c):
    n = d.size
    A = np.diag(d)
    for i in range(1, n):
        A[i, i - 1] = a[i]
    for i in range(n - 1):
        A[i, i + 1] = c[i]
    return A


@pytest.mark.parametrize("n", list(range(1, 17)) + [63, 200])
def test_thomas_matches_pivoted_lu(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        a, d, c, b = _dd_system(rng, n)
        x = O.thomas(a, d, c, b)
        ref = np.linalg.solve(_dense(a, d, c), b)
        assert np.max(np.abs(x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def _cn_matrix(n, r):
    """Crank-Nicolson left-hand matrix written from the lumped FE stencils."""
    a = np.full(n, -0.5 * r)
    c = np.full(n, -0.5 * r)
    d = np.full(n, 1.0 + r)
    if n >= 2:
        c[0] = -r
        a[n - 1] = -r
    if n == 1:
        d[0] = 1.0
    return a, d, c


@pytest.mark.parametrize("n,r", [(2, 0.0766), (3, 0.0766), (16, 0.383), (1000, 0.0766)])
def test_thomas_on_cn_matrices(n, r):
    rng = np.random.default_rng(7)
    a, d, c = _cn_matrix(n, r)
    b = rng.uniform(-80, 30, n)
    x = O.thomas(a, d, c, b)
    ref = np.linalg.solve(_dense(a, d, c), b)
    assert np.max(np.abs(x - ref)) < 1e-12


def _cfg(dt):
    return O.Config(dt_0D=dt, dt_1D=dt, dt_split=dt)


@pytest.mark.parametrize("N", [2, 3, 17, 200])
@pytest.mark.parametrize("dt", [1e-3, 5e-3, 0.05])
def test_cn_cosine_eigenmodes(N, dt):
    cfg = _cfg(dt)
    c = cfg.sigma / (cfg.Am * cfg.Cm)
    i = np.arange(N)
    for k in range(N):
        v = np.cos(k * np.pi * i / (N - 1))
        lam = -(4.0 / cfg.h ** 2) * np.sin(k * np.pi / (2 * (N - 1))) ** 2
        g = (1 + 0.5 * dt * c * lam) / (1 - 0.5 * dt * c * lam)
        out = O.diffusion(cfg, [N], v, dt)
        assert np.max(np.abs(out - g * v)) < 1e-12


@pytest.mark.parametrize("N", [2, 17, 200])
@pytest.mark.parametrize("dt", [1e-3, 0.05])
def test_implicit_euler_cosine_eigenmodes(N, dt):
    """theta = 1 (eq. implicit_euler with the lumped mass): the same cosine
    eigenvectors are damped by exactly 1 / (1 - dt c lambda_k)."""
    cfg = O.Config(dt_0D=dt, dt_1D=dt, dt_split=dt, theta=1.0)
    c = cfg.sigma / (cfg.Am * cfg.Cm)
    i = np.arange(N)
    for k in range(N):
        v = np.cos(k * np.pi * i / (N - 1))
        lam = -(4.0 / cfg.h ** 2) * np.sin(k * np.pi / (2 * (N - 1))) ** 2
        out = O.diffusion(cfg, [N], v, dt)
        assert np.max(np.abs(out - v / (1 - dt * c * lam))) < 1e-12


def test_theta_outside_the_stable_range_is_rejected():
    with pytest.raises(RuntimeError):
        O.diffusion(O.Config(theta=0.4), [10], np.zeros(10), 1e-3)


def test_cn_conserves_lumped_charge_and_max_principle():
    rng = np.random.default_rng(3)
    lengths = np.array([1, 2, 5, 100, 1481], dtype=np.int32)
    V = rng.uniform(-85.0, 35.0, lengths.sum())
    cfg = _cfg(1e-3)
    r = cfg.sigma / (cfg.Am * cfg.Cm) * cfg.dt_1D / cfg.h ** 2
    assert r <= 1.0
    out = V.copy()
    off = np.concatenate([[0], np.cumsum(lengths)])
    for _ in range(20):
        prev = out
        out = O.diffusion(cfg, lengths, prev, cfg.dt_1D)
        for f, n in enumerate(lengths):
            s = slice(off[f], off[f + 1])
            w = np.ones(n)
            if n > 1:
                w[0] = w[-1] = 0.5
            q0, q1 = np.dot(w, prev[s]), np.dot(w, out[s])
            assert abs(q1 - q0) <= 1e-13 * np.sum(np.abs(w * prev[s]))
            assert out[s].min() >= prev[s].min() - 1e-12
            assert out[s].max() <= prev[s].max() + 1e-12


def test_diffusion_substeps():
    # span = 2 dt_1D is two Crank-Nicolson steps of width dt_1D
    rng = np.random.default_rng(4)
    V = rng.uniform(-80, 20, 50)
    cfg = O.Config(dt_1D=1e-3)
    a = O.diffusion(cfg, [50], V, 2e-3)
    b = O.diffusion(cfg, [50], O.diffusion(cfg, [50], V, 1e-3), 1e-3)
    np.testing.assert_array_equal(a, b)


def test_fibers_are_independent():
    rng = np.random.default_rng(5)
    lengths = [7, 1, 30]
    V = rng.uniform(-80, 20, sum(lengths))
    cfg = _cfg(5e-3)
    whole = O.diffusion(cfg, lengths, V, 5e-3)
    parts = np.concatenate([O.diffusion(cfg, [7], V[:7], 5e-3), V[7:8],
                            O.diffusion(cfg, [30], V[8:], 5e-3)])
    np.testing.assert_array_equal(whole, parts)


def test_only_sigma_over_am_cm_enters_the_diffusion():
    # eq. monodomain: the fiber operator is sigma / (Am Cm) times the second
    # derivative, so doubling Cm or Am and halving sigma give the same step
    from dataclasses import replace
    rng = np.random.default_rng(8)
    V = rng.uniform(-80, 20, 40)
    base = _cfg(5e-3)
    ref = O.diffusion(replace(base, sigma=base.sigma / 2), [40], V, 5e-3)
    assert np.max(np.abs(ref - O.diffusion(base, [40], V, 5e-3))) > 1e-3  # sigma matters
    for cfg in (replace(base, Cm=2 * base.Cm), replace(base, Am=2 * base.Am)):
        np.testing.assert_allclose(O.diffusion(cfg, [40], V, 5e-3), ref, rtol=0, atol=1e-11)
