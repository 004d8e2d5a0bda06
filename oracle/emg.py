"""FP64 oracle of the static bidomain (EMG) step on a structured cuboid.

TEST INFRASTRUCTURE ONLY: the reference that the GPU EMG solve is checked
against.  Only tests/, the smoke check and bench.py's parity legs use it; it
shares nothing with the GPU library.

What it computes (thesis eq. discretized_fibers_2 and eq. discretized_fibers_3,
the static first bidomain equation eq. bidomain1 with the homogeneous Neumann
conditions of eq. monodomain_bc):

    V_3D = P V_fibers,
    K_{sigma_i + sigma_e} phi_e = -K_{sigma_i} V_3D,

on a 3D mesh of trilinear hexahedra whose nodes are the fiber nodes of a
bundle of nfx x nfy parallel fibers (along z) sampled at every m-th node
(section on mesh generation: the 3D mesh is sampled from the fiber points,
so P is the injection of those nodes).  The conduction tensors are
sigma_i = sigma_i a (x) a with the fiber direction a = e_z, and sigma_e =
diag(sigma_et, sigma_et, sigma_el).  phi_e is determined up to a constant;
the oracle returns the zero-mean solution.

Stiffness matrices of Q1 elements on a tensor grid with a diagonal tensor
are sums of Kronecker products of the 1D linear-element matrices,
    K_D = d_x K_x (x) M_y (x) M_z + d_y M_x (x) K_y (x) M_z + d_z M_x (x) M_y (x) K_z,
with the 1D stiffness (1/h) tridiag(-1, 2, -1) (corner entries 1) and the
consistent 1D mass (h/6) tridiag(1, 4, 1) (corner entries 2) -- the tables
stencils_laplace and stencils_mass_laplace in 1D.  Node (i, j, k) has
index (k ny + j) nx + i.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class Grid:
    nx: int          # fibers along x
    ny: int          # fibers along y
    nz: int          # 3D nodes along each fiber
    hx: float        # fiber spacing in x (cm)
    hy: float        # fiber spacing in y (cm)
    hz: float        # 3D mesh width along the fibers (cm): m * h

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def stiffness_1d(n: int, h: float) -> sp.csr_matrix:
    """1D linear-element stiffness on n nodes (n >= 2)."""
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    off = np.full(n - 1, -1.0)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr") / h


def mass_1d(n: int, h: float) -> sp.csr_matrix:
    """1D linear-element consistent mass on n nodes (n >= 2)."""
    main = np.full(n, 4.0)
    main[0] = main[-1] = 2.0
    off = np.ones(n - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr") * (h / 6.0)


def stiffness_3d(g: Grid, d) -> sp.csr_matrix:
    """K_D for the diagonal tensor D = diag(d[0], d[1], d[2]) (x fastest)."""
    Kx, Mx = stiffness_1d(g.nx, g.hx), mass_1d(g.nx, g.hx)
    Ky, My = stiffness_1d(g.ny, g.hy), mass_1d(g.ny, g.hy)
    Kz, Mz = stiffness_1d(g.nz, g.hz), mass_1d(g.nz, g.hz)
    # index (k ny + j) nx + i: z is the slowest, so Kronecker order z, y, x
    K = (d[0] * sp.kron(Mz, sp.kron(My, Kx)) + d[1] * sp.kron(Mz, sp.kron(Ky, Mx))
         + d[2] * sp.kron(Kz, sp.kron(My, Mx)))
    return K.tocsr()


def prolongate(V_fibers: np.ndarray, nx: int, ny: int, n_nodes: int, m: int) -> np.ndarray:
    """V_3D = P V: fiber f = j nx + i holds nodes 0..n_nodes-1; the 3D node
    (i, j, k) takes fiber node k m (eq. discretized_fibers_2)."""
    nz = (n_nodes - 1) // m + 1
    V = np.asarray(V_fibers, dtype=np.float64).reshape(ny * nx, n_nodes)
    V3 = V[:, ::m][:, :nz]                  # [fiber, k]
    return np.ascontiguousarray(V3.T).reshape(-1)  # k slowest, then fiber = j nx + i


def solve_neumann(K: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """Zero-mean solution of the singular Neumann system K x = b, with the
    zero-mean condition as one extra row and column (a bordered system)."""
    n = K.shape[0]
    one = np.ones((n, 1))
    Kb = sp.bmat([[K, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]], format="csc")
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]


def solve_neumann_cg(K: sp.csr_matrix, b: np.ndarray, rtol: float = 1e-13) -> np.ndarray:
    """Zero-mean solution of the same singular system for meshes too large for
    the direct solve: the right-hand side's mean (zero in exact arithmetic:
    every column of K sums to zero) is removed, FP64 conjugate gradients with
    the diagonal as preconditioner (SciPy's `cg`) run to a relative residual of
    `rtol`, and the iterate's mean is removed.  CG on a consistent
    semi-definite system stays in the range of K."""
    bz = b - b.mean()
    d = K.diagonal()
    M = sp.diags(1.0 / d)
    x, info = spla.cg(K, bz, rtol=rtol, atol=0.0, maxiter=20 * K.shape[0], M=M)
    if info != 0:
        raise RuntimeError(f"CG did not converge (info {info})")
    return x - x.mean()


def solve(g: Grid, V3: np.ndarray, sigma_i: float, sigma_el: float, sigma_et: float,
          method: str = "direct"):
    """Zero-mean phi_e of K_{sigma_i + sigma_e} phi_e = -K_{sigma_i} V3, and the
    right-hand side; method "direct" (bordered sparse LU) or "cg" (FP64
    conjugate gradients to a relative residual of 1e-13)."""
    Ki = stiffness_3d(g, (0.0, 0.0, sigma_i))
    Kt = stiffness_3d(g, (sigma_et, sigma_et, sigma_el + sigma_i))
    b = -(Ki @ V3)
    if method == "cg":
        return solve_neumann_cg(Kt, b), b
    return solve_neumann(Kt, b), b
