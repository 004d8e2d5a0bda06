"""EMG step (static bidomain solve on the 3D mesh) on the GPU against the FP64
oracle of oracle/emg.py.

* the right-hand side -K_{sigma_i} P V_m from the device state equals the
  oracle's from the same V_m within the rounding bound of an FP32 stencil
  sum, 2^-24 x 64 x max_i sum_j |K_ij| |V_j| (the terms cancel strongly where
  the mesh is fine along the fibers);
* phi_e after conjugate gradients to a relative residual of 1e-7 equals the
  oracle's direct solve from the same V_m to 1e-4 of its largest value (the
  residual bound times the condition number of the preconditioned system,
  a few hundred on these meshes, plus FP32 rounding);
* the same on a bundle of the 57-state model during an action potential;
* V_m linear along the fibers gives phi_e = -sigma_i / (sigma_i + sigma_el)
  V_m up to a constant;
* CG driven far past the FP32 accuracy of phi_e (relative residual 1e-9)
  converges and stays at the oracle's solution: the stencil in difference
  form keeps the constant vector an exact null vector of the FP32 operator
  and the residual is kept at zero mean in every iteration (without either,
  a 3 x 7 x 121 mesh diverges below a relative residual of about 1e-7);
* a resting V_m gives phi_e = 0 without an iteration; a repeated solve from
  the same V_m starts at the previous phi_e and needs at most a few
  iterations (the true residual of the FP32 iterate sits near the tolerance);
* at the benchmark's size (37 x 37 fibers of 1481 nodes, every 10th node:
  37 x 37 x 149 = 2.0e5 mesh nodes) phi_e during a propagating wave equals
  the oracle's FP64 conjugate-gradient solution (the direct solve does not
  fit this mesh) to 1e-5 of its largest value after a deep solve, and to
  1e-3 after the benchmark's tolerance 1e-6;
* malformed bundles are refused.
"""
import numpy as np
import pytest

from oracle import emg as E
from paper_2107_07104_amd import fib as F
from paper_2107_07104_amd import inputs as I

from gpu_helpers import gpu_solver, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIG = dict(sigma_i=8.93, sigma_el=6.7, sigma_et=3.35)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.lib()


def _bundle(nx, ny, n, t_end=3.0):
    return I.batched_hh(n_fibers=nx * ny, n_min=n, n_max=n, t_end=t_end, onset_max=1.0)


def _oracle(s, nx, ny, n, m, hxy, h):
    V = s.get_state()[0]
    V3 = E.prolongate(V, nx, ny, n, m)
    g = E.Grid(nx, ny, (n - 1) // m + 1, hxy, hxy, m * h)
    return E.solve(g, V3, SIG["sigma_i"], SIG["sigma_el"], SIG["sigma_et"]), g, V3


@pytest.mark.parametrize("nx,ny,n,m", [(5, 4, 301, 10), (8, 8, 1001, 25), (3, 7, 121, 1)])
def test_phi_matches_oracle_during_a_propagating_wave(nx, ny, n, m):
    w = _bundle(nx, ny, n)
    s = gpu_solver(w)
    s.run(0, 2500)
    s.sync()
    hxy = 0.05
    emg = F.Emg(s, nx, ny, m, hxy, hxy, **SIG)
    it, rel = emg.solve(tol=1e-7, max_iter=5000)
    (phi_o, b_o), g, V3 = _oracle(s, nx, ny, n, m, hxy, w.h)
    b = emg.rhs()
    phi = emg.phi()
    Ki = E.stiffness_3d(g, (0.0, 0.0, SIG["sigma_i"]))
    bound = 64 * 2.0 ** -24 * np.max(abs(Ki) @ np.abs(V3 - V3.min()))
    eb = np.max(np.abs(b - b_o)) / bound
    ep = np.max(np.abs(phi - phi_o)) / np.max(np.abs(phi_o))
    say(f"[emg] {nx}x{ny}x{g.nz}: {it} iterations, residual {rel:.2e}; rhs err {eb:.2e} "
        f"of the bound {bound:.2e}, "
        f"phi err {ep:.2e}, max |phi| {np.max(np.abs(phi_o)):.3f} mV, V range "
        f"{V3.min():.1f}..{V3.max():.1f}")
    assert rel <= 1e-7 and it > 0
    assert eb < 1.0
    assert ep < 1e-4
    assert abs(phi.mean()) < 1e-6 * np.max(np.abs(phi_o))
    emg.close()
    s.close()


@pytest.mark.parametrize("nx,ny,n,m", [(3, 7, 121, 1), (5, 4, 301, 10)])
def test_deep_solve_converges_and_stays_at_the_solution(nx, ny, n, m):
    w = _bundle(nx, ny, n)
    s = gpu_solver(w)
    s.run(0, 2500)
    s.sync()
    emg = F.Emg(s, nx, ny, m, 0.05, 0.05, **SIG)
    it, rel = emg.solve(tol=1e-9, max_iter=3000)
    (phi_o, _), _, _ = _oracle(s, nx, ny, n, m, 0.05, w.h)
    ep = np.max(np.abs(emg.phi() - phi_o)) / np.max(np.abs(phi_o))
    say(f"[emg deep] {nx}x{ny}x{n}/{m}: {it} iterations, residual {rel:.2e}, phi err {ep:.2e}")
    assert rel <= 1e-9 and it < 3000
    assert ep < 1e-4
    emg.close()
    s.close()


def test_bench_size_bundle_matches_oracle():
    nx = ny = 37
    n, m, hxy = 1481, 10, 0.05
    say(f"[emg bench size] {nx}x{ny}x{n}, every {m}th node")
    w = _bundle(nx, ny, n)
    s = gpu_solver(w)
    s.run(0, 2500)
    s.sync()
    V = s.get_state()[0]
    V3 = E.prolongate(V, nx, ny, n, m)
    g = E.Grid(nx, ny, (n - 1) // m + 1, hxy, hxy, m * w.h)
    phi_o, _ = E.solve(g, V3, SIG["sigma_i"], SIG["sigma_el"], SIG["sigma_et"], method="cg")
    emg = F.Emg(s, nx, ny, m, hxy, hxy, **SIG)
    # the benchmark's tolerance, then deeper from there
    it1, rel1 = emg.solve(tol=1e-6, max_iter=5000)
    e1 = np.max(np.abs(emg.phi() - phi_o)) / np.max(np.abs(phi_o))
    it2, rel2 = emg.solve(tol=1e-9, max_iter=5000)
    e2 = np.max(np.abs(emg.phi() - phi_o)) / np.max(np.abs(phi_o))
    say(f"   tol 1e-6: {it1} iterations, residual {rel1:.2e}, phi err {e1:.2e}; "
        f"tol 1e-9: {it2} more, residual {rel2:.2e}, phi err {e2:.2e}; "
        f"max |phi| {np.max(np.abs(phi_o)):.3f} mV")
    assert rel1 <= 1e-6 and rel2 <= 1e-9
    # FP32 iterates reach a few 1e-6 of max |phi| (measured 1.1e-6); at the
    # benchmark's tolerance the residual bound leaves 3.8e-5 (measured)
    assert e2 < 1e-5
    assert e1 < 1e-3
    emg.close()
    s.close()


def test_st57_bundle_matches_oracle():
    # V_m is state row 0 of the 57-state model too
    nx, ny, n, m = 4, 3, 241, 8
    w = I.st57_bundle(n_fibers=nx * ny, n_nodes=n, t_end=1.0, onset_max=0.1)
    s = gpu_solver(w)
    s.run(0, 1200)
    s.sync()
    emg = F.Emg(s, nx, ny, m, 0.05, 0.05, **SIG)
    it, rel = emg.solve(tol=1e-7, max_iter=5000)
    (phi_o, _), _, V3 = _oracle(s, nx, ny, n, m, 0.05, w.h)
    ep = np.max(np.abs(emg.phi() - phi_o)) / np.max(np.abs(phi_o))
    say(f"[emg st57] {it} iterations, residual {rel:.2e}, phi err {ep:.2e}, "
        f"V range {V3.min():.1f}..{V3.max():.1f}")
    assert V3.max() - V3.min() > 50.0     # an action potential is in the mesh
    assert rel <= 1e-7 and ep < 1e-4
    emg.close()
    s.close()


def test_fiber_aligned_linear_vm_gives_the_bidomain_ratio():
    nx, ny, n, m = 4, 5, 201, 10
    w = _bundle(nx, ny, n)
    s = gpu_solver(w)
    y = s.get_state()
    z = np.tile(np.arange(n) * w.h, nx * ny)
    y[0] = -75.0 + 400.0 * z          # mV, linear along every fiber
    s.set_state(y)
    emg = F.Emg(s, nx, ny, m, 0.05, 0.05, **SIG)
    it, rel = emg.solve(tol=1e-7, max_iter=5000)
    V3 = E.prolongate(s.get_state()[0], nx, ny, n, m)
    want = -SIG["sigma_i"] / (SIG["sigma_i"] + SIG["sigma_el"]) * V3
    want -= want.mean()
    err = np.max(np.abs(emg.phi() - want)) / np.max(np.abs(want))
    say(f"[emg linear] {it} iterations, relative error {err:.2e}")
    assert err < 1e-4
    emg.close()
    s.close()


def test_rest_gives_zero_and_a_repeated_solve_starts_converged():
    nx, ny, n, m = 4, 4, 101, 5
    w = _bundle(nx, ny, n)
    s = gpu_solver(w)
    s.init_state()                    # every node at the resting state
    emg = F.Emg(s, nx, ny, m, 0.05, 0.05, **SIG)
    it, rel = emg.solve(tol=1e-7, max_iter=100)
    assert it == 0 and rel == 0.0
    assert np.all(emg.phi() == 0.0)
    s.init_state(vm_noise=w.vm_noise.astype(np.float32))
    s.run(0, 1500)
    it1, _ = emg.solve(tol=1e-6, max_iter=5000)
    it2, rel2 = emg.solve(tol=1e-6, max_iter=5000)
    say(f"[emg warm start] first {it1}, repeated {it2} iterations")
    assert it1 > 0 and it2 <= 3 and rel2 <= 1e-6
    emg.close()
    s.close()


def test_malformed_bundles_are_refused():
    w = _bundle(3, 3, 101)
    s = gpu_solver(w)
    for args in ((3, 4, 10), (3, 3, 7), (1, 9, 10), (3, 3, 0)):
        with pytest.raises(F.FibError) as e:
            F.Emg(s, *args, 0.05, 0.05, **SIG)
        assert e.value.code == F.FIB_EINVAL
    s.close()
    w2 = I.batched_hh(n_fibers=4, n_min=100, n_max=120, t_end=0.1)
    s2 = gpu_solver(w2)
    with pytest.raises(F.FibError):
        F.Emg(s2, 2, 2, 1, 0.05, 0.05, **SIG)
    s2.close()
