"""Pins of the EMG oracle (static bidomain step on a structured cuboid).

* the Kronecker assembly of one trilinear element equals Gauss quadrature of
  grad N_a . D grad N_b with the trilinear shape functions written out;
* constants span the null space, the matrices are symmetric positive
  semi-definite;
* a linear potential leaves every interior row zero and its boundary rows
  add up to the flux D grad u . n through each face;
* a manufactured cosine solution with homogeneous Neumann data converges at
  second order in the nodal values;
* P is the injection of every m-th fiber node;
* for V_m linear along the fibers, phi_e = -sigma_i / (sigma_i + sigma_el) V_m
  (up to a constant): the k / (k + 1) ratio of the thesis's derivation of
  the monodomain equation from the bidomain equations.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import emg as E


def _coords(g):
    x = np.arange(g.nx) * g.hx
    y = np.arange(g.ny) * g.hy
    z = np.arange(g.nz) * g.hz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


def test_element_matrix_matches_gauss_quadrature():
    hx, hy, hz = 0.3, 0.5, 0.7
    D = (1.3, 0.4, 2.1)
    g = E.Grid(2, 2, 2, hx, hy, hz)
    K = E.stiffness_3d(g, D).toarray()
    # trilinear shape functions on [0,hx]x[0,hy]x[0,hz], node (i,j,k) -> (k*2+j)*2+i
    gp = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
    Kq = np.zeros((8, 8))
    for a, b_, c in itertools.product(gp, gp, gp):  # reference coordinates in [0,1]
        grads = []
        for k, j, i in itertools.product((0, 1), (0, 1), (0, 1)):
            fx = a if i else 1 - a
            fy = b_ if j else 1 - b_
            fz = c if k else 1 - c
            dx = (1 if i else -1) / hx * fy * fz
            dy = (1 if j else -1) / hy * fx * fz
            dz = (1 if k else -1) / hz * fx * fy
            grads.append(np.array([dx, dy, dz]))
        w = hx * hy * hz / 8.0
        for p_, q_ in itertools.product(range(8), range(8)):
            Kq[p_, q_] += w * np.dot(grads[p_] * D, grads[q_])
    np.testing.assert_allclose(K, Kq, rtol=1e-12, atol=1e-12)


def test_null_space_symmetry_and_semi_definiteness():
    g = E.Grid(4, 3, 5, 0.1, 0.2, 0.3)
    for D in ((1.0, 1.0, 1.0), (0.0, 0.0, 2.0), (0.3, 0.7, 1.9)):
        K = E.stiffness_3d(g, D)
        assert np.max(np.abs(K @ np.ones(g.n))) < 1e-12
        Kd = K.toarray()
        np.testing.assert_allclose(Kd, Kd.T, atol=1e-14)
        assert np.linalg.eigvalsh(Kd).min() > -1e-10


def test_linear_potential_interior_rows_and_face_fluxes():
    g = E.Grid(5, 4, 6, 0.2, 0.25, 0.5)
    D = (0.7, 1.1, 2.3)
    X, Y, Z = _coords(g)
    Lx, Ly, Lz = (g.nx - 1) * g.hx, (g.ny - 1) * g.hy, (g.nz - 1) * g.hz
    K = E.stiffness_3d(g, D)
    for grad, u in (((1, 0, 0), X), ((0, 1, 0), Y), ((0, 0, 1), Z)):
        r = K @ u
        inner = ((X > 0) & (X < Lx - 1e-12) & (Y > 0) & (Y < Ly - 1e-12) & (Z > 0)
                 & (Z < Lz - 1e-12))
        assert np.max(np.abs(r[inner])) < 1e-12
        # the rows of the face where the coordinate is maximal integrate
        # the outward flux D grad u . n over that face
        ax = int(np.argmax(grad))
        coord, L = (X, Y, Z)[ax], (Lx, Ly, Lz)[ax]
        area = (Ly * Lz, Lx * Lz, Lx * Ly)[ax]
        top = np.abs(coord - L) < 1e-12
        assert r[top].sum() == pytest.approx(D[ax] * area, rel=1e-12)
        assert r.sum() == pytest.approx(0.0, abs=1e-12)


def test_manufactured_cosine_converges_at_second_order():
    D = (0.6, 0.9, 1.7)
    L = (1.0, 0.8, 1.3)
    errs = []
    for n in (6, 11, 21):
        g = E.Grid(n, n, n, L[0] / (n - 1), L[1] / (n - 1), L[2] / (n - 1))
        X, Y, Z = _coords(g)
        phi = np.cos(np.pi * X / L[0]) * np.cos(np.pi * Y / L[1]) * np.cos(np.pi * Z / L[2])
        lam = sum(d * (np.pi / l) ** 2 for d, l in zip(D, L))
        K = E.stiffness_3d(g, D)
        # the consistent 3D mass is the Kronecker product of the 1D masses
        Mx, My, Mz = E.mass_1d(g.nx, g.hx), E.mass_1d(g.ny, g.hy), E.mass_1d(g.nz, g.hz)
        M3 = sp.kron(Mz, sp.kron(My, Mx))
        x = E.solve_neumann(K, M3 @ (lam * phi))
        errs.append(np.max(np.abs(x - (phi - phi.mean()))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.6 < r2 < 4.4


def test_prolongation_is_the_injection_of_every_mth_node():
    nx, ny, n, m = 3, 2, 13, 4
    rng = np.random.default_rng(5)
    V = rng.standard_normal(nx * ny * n)
    V3 = E.prolongate(V, nx, ny, n, m)
    nz = (n - 1) // m + 1
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                assert V3[(k * ny + j) * nx + i] == V[(j * nx + i) * n + k * m]


def test_fiber_aligned_linear_potential_gives_the_bidomain_ratio():
    g = E.Grid(4, 5, 9, 0.05, 0.05, 0.1)
    X, Y, Z = _coords(g)
    s_i, s_el, s_et = 8.93, 6.7, 3.35
    phi, b = E.solve(g, 2.5 * Z, s_i, s_el, s_et)
    want = -s_i / (s_i + s_el) * 2.5 * Z
    np.testing.assert_allclose(phi, want - want.mean(), atol=1e-11)
    # a constant V_m drives no current
    phi0, b0 = E.solve(g, np.full(g.n, -75.0), s_i, s_el, s_et)
    assert np.max(np.abs(b0)) < 1e-11 and np.max(np.abs(phi0)) < 1e-11


@pytest.mark.parametrize("nx,ny,nz,hz", [(5, 4, 31, 0.1), (3, 7, 121, 0.01), (6, 6, 9, 0.25)])
def test_cg_route_equals_the_direct_solve(nx, ny, nz, hz):
    """The FP64 conjugate-gradient route (for meshes too large for the
    bordered LU) returns the direct solve's zero-mean solution, and its
    residual, computed here from the matrices, is at the requested level."""
    g = E.Grid(nx, ny, nz, 0.05, 0.07, hz)
    rng = np.random.default_rng(nx * ny * nz)
    z = np.arange(nz) * hz
    V3 = np.tile(-75.0 + 100.0 * np.exp(-((z - z.mean()) / (3 * hz)) ** 2), nx * ny)
    V3 = V3.reshape(nx * ny, nz).T.ravel() + rng.uniform(-1.0, 1.0, g.n)
    pd, b = E.solve(g, V3, 8.93, 6.7, 3.35)
    pc, b2 = E.solve(g, V3, 8.93, 6.7, 3.35, method="cg")
    np.testing.assert_array_equal(b, b2)
    assert np.max(np.abs(pc - pd)) <= 1e-9 * np.max(np.abs(pd))
    Kt = E.stiffness_3d(g, (3.35, 3.35, 6.7 + 8.93))
    bz = b - b.mean()
    assert np.linalg.norm(Kt @ pc - bz) <= 1e-12 * np.linalg.norm(bz)
    assert abs(pc.mean()) < 1e-12 * np.max(np.abs(pc))
