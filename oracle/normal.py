"""Oracle: damped normal equations, Schur complement, reduced RHS, back-substitution.

Test infrastructure only. Section 2.1 of the paper: LM solves
(J^T J + D) delta = -J^T f  (the printed right-hand side drops the transpose;
read as -J^T f). With J = [F E]:
    A = F^T F + D_c   (9x9 blocks per camera),
    C = E^T E + D_p   (3x3 blocks per point),
    W = F^T E         (9x3 blocks per observation),
    S = A - W C^-1 W^T  (the Schur complement, 9x9 blocks).
The reduced right-hand side and back-substitution follow from block
elimination (the paper does not write them):
    b = -g_c + W C^-1 g_p,   S delta_c = b,   delta_p = -C^-1 (g_p + W^T delta_c),
with g = J^T f. Damping D = lam * diag(J^T J) (Marquardt scaling; no clamping).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def assemble_J(F, E, obs_cam, obs_pt, n_cam, n_pt):
    """Sparse J [2 n_obs, 9 n_cam + 3 n_pt] from the per-observation blocks."""
    n = obs_cam.shape[0]
    rows_F = np.repeat(2 * np.arange(n)[:, None] + np.arange(2)[None, :], 9, axis=1).reshape(n, 2, 9)
    cols_F = np.broadcast_to((9 * obs_cam)[:, None, None] + np.arange(9)[None, None, :], (n, 2, 9))
    rows_E = np.repeat(2 * np.arange(n)[:, None] + np.arange(2)[None, :], 3, axis=1).reshape(n, 2, 3)
    cols_E = np.broadcast_to(9 * n_cam + (3 * obs_pt)[:, None, None] + np.arange(3)[None, None, :],
                             (n, 2, 3))
    rows = np.concatenate([rows_F.ravel(), rows_E.ravel()])
    cols = np.concatenate([cols_F.ravel(), cols_E.ravel()])
    vals = np.concatenate([F.ravel(), E.ravel()])
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * n, 9 * n_cam + 3 * n_pt))


def block_sum(idx, blocks, n):
    """sum of blocks[o] into out[idx[o]] (plain scatter-add)."""
    out = np.zeros((n,) + blocks.shape[1:])
    np.add.at(out, idx, blocks)
    return out


class Normal:
    """Damped normal-equation blocks of one LM step (all FP64)."""

    def __init__(self, F, E, f, obs_cam, obs_pt, n_cam, n_pt, lam=1e-4, D=None):
        self.F, self.E, self.f = F, E, f
        self.obs_cam, self.obs_pt = obs_cam, obs_pt
        self.n_cam, self.n_pt = n_cam, n_pt
        A0 = block_sum(obs_cam, np.einsum("nki,nkj->nij", F, F), n_cam)
        C0 = block_sum(obs_pt, np.einsum("nki,nkj->nij", E, E), n_pt)
        self.g_c = block_sum(obs_cam, np.einsum("nki,nk->ni", F, f), n_cam)
        self.g_p = block_sum(obs_pt, np.einsum("nki,nk->ni", E, f), n_pt)
        if D is None:
            Dc = lam * np.einsum("nii->ni", A0)
            Dp = lam * np.einsum("nii->ni", C0)
        else:
            Dc = D[: 9 * n_cam].reshape(n_cam, 9)
            Dp = D[9 * n_cam:].reshape(n_pt, 3)
        self.Dc, self.Dp = Dc, Dp
        self.A0, self.C0 = A0, C0
        self.A = A0 + np.einsum("ni,ij->nij", Dc, np.eye(9))
        self.C = C0 + np.einsum("ni,ij->nij", Dp, np.eye(3))
        self.Cinv = np.linalg.inv(self.C)
        self.Y = np.einsum("nki,nkj->nij", F, E)          # W blocks F_o^T E_o, [n,9,3]

    # ---- explicit operators
    def H_sparse(self):
        """J^T J + D as a sparse matrix (the plain definition)."""
        J = assemble_J(self.F, self.E, self.obs_cam, self.obs_pt, self.n_cam, self.n_pt)
        d = np.concatenate([self.Dc.ravel(), self.Dp.ravel()])
        return (J.T @ J + sp.diags(d)).tocsc()

    def W_sparse(self):
        n = self.obs_cam.shape[0]
        rows = (9 * self.obs_cam)[:, None, None] + np.arange(9)[None, :, None]
        cols = (3 * self.obs_pt)[:, None, None] + np.arange(3)[None, None, :]
        return sp.csr_matrix((self.Y.ravel(), (np.broadcast_to(rows, (n, 9, 3)).ravel(),
                                               np.broadcast_to(cols, (n, 9, 3)).ravel())),
                             shape=(9 * self.n_cam, 3 * self.n_pt))

    def Cinv_sparse(self):
        return sp.block_diag(list(self.Cinv), format="csr") if self.n_pt < 50 else \
            _blockdiag(self.Cinv)

    def A_sparse(self):
        return _blockdiag(self.A)

    def S_sparse(self):
        """Explicit Schur complement S = A - W C^-1 W^T (sparse, 9x9 blocks)."""
        W = self.W_sparse()
        return (self.A_sparse() - W @ self.Cinv_sparse() @ W.T).tocsr()

    def S_dense(self):
        return self.S_sparse().toarray()

    # ---- implicit operator (Section 3.6)
    def S_apply(self, x):
        """S x = A x - F^T (E (C^-1 (E^T (F x)))) without forming S."""
        x = np.asarray(x).reshape(self.n_cam, 9)
        s = np.einsum("nkj,nj->nk", self.F, x[self.obs_cam])                 # F x
        z = block_sum(self.obs_pt, np.einsum("nki,nk->ni", self.E, s), self.n_pt)  # E^T
        u = np.einsum("pij,pj->pi", self.Cinv, z)                             # C^-1
        w = np.einsum("nkj,nj->nk", self.E, u[self.obs_pt])                   # E
        y = block_sum(self.obs_cam, np.einsum("nki,nk->ni", self.F, w), self.n_cam)  # F^T
        return (np.einsum("cij,cj->ci", self.A, x) - y).ravel()

    # ---- right-hand sides and recovery (block elimination)
    def reduce_rhs(self, r_c, r_p):
        """Camera right-hand side of the Schur system for H [x_c; x_p] = [r_c; r_p]:
        b = r_c - W C^-1 r_p."""
        v = np.einsum("pij,pj->pi", self.Cinv, r_p.reshape(self.n_pt, 3))
        return (r_c.reshape(self.n_cam, 9)
                - block_sum(self.obs_cam, np.einsum("nij,nj->ni", self.Y, v[self.obs_pt]),
                            self.n_cam)).ravel()

    def recover_points(self, x_c, r_p):
        """x_p = C^-1 (r_p - W^T x_c)."""
        x_c = x_c.reshape(self.n_cam, 9)
        wt = block_sum(self.obs_pt, np.einsum("nij,ni->nj", self.Y, x_c[self.obs_cam]), self.n_pt)
        return np.einsum("pij,pj->pi", self.Cinv, r_p.reshape(self.n_pt, 3) - wt)

    def rhs(self):
        """b for the LM step: r = -g."""
        return self.reduce_rhs(-self.g_c.ravel(), -self.g_p.ravel())

    def block_jacobi_blocks(self):
        """Diagonal 9x9 blocks of S: S_cc = A_c - sum_{o in c} Y_o C_p^-1 Y_o^T."""
        YCY = np.einsum("nij,njk,nlk->nil", self.Y, self.Cinv[self.obs_pt], self.Y)
        return self.A - block_sum(self.obs_cam, YCY, self.n_cam)


def _blockdiag(blocks):
    n, b, _ = blocks.shape
    rows = (b * np.arange(n))[:, None, None] + np.arange(b)[None, :, None]
    cols = (b * np.arange(n))[:, None, None] + np.arange(b)[None, None, :]
    return sp.csr_matrix((blocks.ravel(), (np.broadcast_to(rows, blocks.shape).ravel(),
                                           np.broadcast_to(cols, blocks.shape).ravel())),
                         shape=(n * b, n * b))


def solve_full(nrm: Normal):
    """The plain definition: solve (J^T J + D) delta = -J^T f directly (sparse LU).
    Returns (delta_c [n_cam, 9], delta_p [n_pt, 3])."""
    g = np.concatenate([nrm.g_c.ravel(), nrm.g_p.ravel()])
    d = ScaledLU(nrm.H_sparse()).solve(-g)
    nc = 9 * nrm.n_cam
    return d[:nc].reshape(nrm.n_cam, 9), d[nc:].reshape(nrm.n_pt, 3)


class ScaledLU:
    """Sparse LU of H after symmetric Jacobi scaling s H s, s = diag(H)^-1/2.
    The scaling leaves the solution unchanged and keeps the factorization
    accurate when parameters live on very different scales."""

    def __init__(self, H):
        self.s = 1.0 / np.sqrt(H.diagonal())
        Dm = sp.diags(self.s)
        self.lu = spla.splu((Dm @ H @ Dm).tocsc())

    def solve(self, rhs):
        return self.s * self.lu.solve(self.s * rhs)


def cholesky_solve(S, b):
    """Dense Cholesky S = L L^T, then two triangular solves (small S only)."""
    L = np.linalg.cholesky(S)
    from scipy.linalg import solve_triangular
    y = solve_triangular(L, b, lower=True)
    return solve_triangular(L.T, y, lower=False)
