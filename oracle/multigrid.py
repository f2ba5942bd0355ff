"""Oracle: unsmoothed-aggregation multigrid preconditioner and PCG.

Test infrastructure only. Follows the paper:
  * Algorithm 1 (Section 2.3): V-cycle -- smooth, residual, restrict with R = P^T,
    recurse from x_c = 0, prolong, smooth; direct solve on the coarsest level;
    coarse operators by the Galerkin product A_{l+1} = R A_l P.
  * Section 3.3: tentative prolongation -- per aggregate, the near-nullspace rows
    of its members are factored K_agg = Q R; Q becomes the aggregate's block of P,
    R its rows of the coarse near-nullspace (16 columns, so 16x16 coarse blocks).
  * Section 3.4: Chebyshev smoother on the point-block-Jacobi matrix D, bounds
    [0.3, 1.1] * lambda_max(D^-1 A), lambda_max from generalized Lanczos on
    A x = lambda D x limited to 5 operator applications; two pre- and two
    post-smoothing iterations.

Readings where the paper is silent:
  * QR: Householder, thin Q, sign fixed so that diag(R) >= 0. When K_agg is rank
    deficient all 16 orthonormal columns are kept (P stays orthonormal and
    16 wide); those extra columns are not unique.
  * Chebyshev: Saad's Chebyshev acceleration (Iterative Methods for Sparse
    Linear Systems, 2nd ed., Algorithm 12.1) applied to D^-1 A; "two
    iterations" = two steps of that recurrence. The pre-smoother's residual is
    reused as the V-cycle residual.
  * Lanczos start vector: v_i = (splitmix64(seed ^ i) >> 11) 2^-53 - 1/2 over the
    level's dof index i, seed = 0x9E3779B97F4A7C15 ^ level; splitmix64 as
    published by Steele, Lea and Flood (2014) and Vigna: z = x + 0x9E3779B97F4A7C15,
    z = (z ^ z>>30) * 0xBF58476D1CE4E5B9, z = (z ^ z>>27) * 0x94D049BB133111EB,
    out = z ^ z>>31.
  * Coarsest direct solve (Algorithm 1's direct solve): Cholesky of the
    equilibrated matrix s S s with s = diag(S)^-1/2, which has the same inverse
    as S up to the scaling and keeps the factor accurate when the camera
    parameters live on very different scales. No shift is added: the coarsest
    operator P^T S P is symmetric positive definite whenever S is (P has
    orthonormal columns on disjoint rows).
  * Coarsening stops when a level has <= 128 nodes, or the next level would keep
    more than 0.9 of the nodes, or at 12 levels.
  * PCG: Saad Algorithm 9.1 from x0 = 0; stop when ||r||_2 <= rtol ||b||_2 on the
    recursively updated residual.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.linalg import solve_triangular

from . import aggregation as agglib

GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


@dataclasses.dataclass
class MGOptions:
    agg_cap: int = 20
    cheb_degree: int = 2
    lanczos_steps: int = 5
    cheb_lo: float = 0.3
    cheb_hi: float = 1.1
    coarse_max_nodes: int = 128
    max_levels: int = 12
    min_ratio: float = 0.9
    smooth_prolongator: bool = False   # Section 3.5's comparison: P = (I - w D^-1 S) P_tent
    smooth_omega: float = 4.0 / 3.0    # w = smooth_omega / lambda_max(D^-1 S)


def splitmix64(x):
    """Elementwise splitmix64 on python ints (exact 64-bit arithmetic)."""
    z = (int(x) + GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def lanczos_start(n, level):
    seed = GOLDEN ^ level
    return np.array([(splitmix64(seed ^ i) >> 11) * 2.0 ** -53 - 0.5 for i in range(n)])


# ------------------------------------------------------------ prolongation

def tentative_prolongator(Krows, agg, n_agg):
    """Krows: [n, bs, 16] near-nullspace rows per node. Returns
    (P blocks [n, bs, 16], coarse K rows [n_agg, 16, 16], P as sparse)."""
    n, bs, m = Krows.shape
    Pb = np.zeros((n, bs, m))
    Kc = np.zeros((n_agg, m, m))
    for a in range(n_agg):
        mem = np.nonzero(agg == a)[0]          # ascending member order
        Ka = Krows[mem].reshape(-1, m)
        Q, R = householder_qr(Ka)
        Pb[mem] = Q.reshape(len(mem), bs, m)
        Kc[a] = R
    rows = (bs * np.arange(n))[:, None, None] + np.arange(bs)[None, :, None]
    cols = (m * agg)[:, None, None] + np.arange(m)[None, None, :]
    P = sp.csr_matrix((Pb.ravel(), (np.broadcast_to(rows, Pb.shape).ravel(),
                                    np.broadcast_to(cols, Pb.shape).ravel())),
                      shape=(n * bs, n_agg * m))
    return Pb, Kc, P


def householder_qr(K):
    """Thin Householder QR with diag(R) >= 0 (K has at least as many rows as
    columns). Uses LAPACK's Householder factorization, then fixes signs."""
    if K.shape[0] < K.shape[1]:
        raise ValueError("aggregate has fewer rows than near-nullspace columns")
    Q, R = np.linalg.qr(K, mode="reduced")
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


# ------------------------------------------------------------ smoother pieces

def block_diagonal(S, bs):
    """Diagonal bs x bs blocks of a (sparse or dense) matrix: [n, bs, bs]."""
    n = S.shape[0] // bs
    Sd = S.toarray() if sp.issparse(S) and S.shape[0] <= 4096 else S
    out = np.zeros((n, bs, bs))
    if sp.issparse(Sd):
        Sd = Sd.tocsr()
        for i in range(n):
            out[i] = Sd[i * bs:(i + 1) * bs, i * bs:(i + 1) * bs].toarray()
    else:
        for i in range(n):
            out[i] = Sd[i * bs:(i + 1) * bs, i * bs:(i + 1) * bs]
    return out


def apply_blocks(Binv, r):
    n, bs, _ = Binv.shape
    return np.einsum("nij,nj->ni", Binv, r.reshape(n, bs)).ravel()


def lanczos_lmax(apply_A, Dinv, v0, steps):
    """Largest eigenvalue estimate of A x = lambda D x by `steps` steps of the
    generalized Lanczos process in the D inner product. Only D^-1 is needed:
    u_j = D v_j is carried along."""
    u = v0.copy()                       # u_1 = D v_1 up to scale: take v1 = D^-1 u1
    v = apply_blocks(Dinv, u)
    nrm = np.sqrt(v @ u)
    v, u = v / nrm, u / nrm
    v_prev = np.zeros_like(v)
    u_prev = np.zeros_like(u)
    alphas, betas = [], []
    beta = 0.0
    for j in range(steps):
        Av = apply_A(v)
        alpha = Av @ v
        alphas.append(alpha)
        # w = D^-1 A v - alpha v - beta v_prev ; D w = A v - alpha u - beta u_prev
        Dw = Av - alpha * u - beta * u_prev
        w = apply_blocks(Dinv, Av) - alpha * v - beta * v_prev
        b2 = w @ Dw
        if j == steps - 1:
            break
        if b2 <= 1e-300 or np.sqrt(b2) <= 1e-14 * abs(alpha):
            break
        beta = np.sqrt(b2)
        betas.append(beta)
        v_prev, u_prev = v, u
        v, u = w / beta, Dw / beta
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    return float(np.linalg.eigvalsh(T)[-1])


def chebyshev(apply_A, Dinv, b, x, lmax, steps, lo=0.3, hi=1.1, r=None, need_residual=True):
    """`steps` steps of Chebyshev acceleration on D^-1 A over [lo, hi] * lmax,
    starting from x (r = b - A x may be passed in). Returns (x, r); when
    need_residual is False the last update of r is skipped and r is None."""
    alpha, beta = lo * lmax, hi * lmax
    theta = 0.5 * (beta + alpha)
    delta = 0.5 * (beta - alpha)
    sigma1 = theta / delta
    rho = 1.0 / sigma1
    if r is None:
        r = b - apply_A(x)
    d = apply_blocks(Dinv, r) / theta
    for k in range(steps):
        x = x + d
        if k == steps - 1 and not need_residual:
            return x, None
        r = r - apply_A(d)
        if k == steps - 1:
            break
        rho_next = 1.0 / (2.0 * sigma1 - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * apply_blocks(Dinv, r)
        rho = rho_next
    return x, r


def chebyshev_pre(apply_A, Dinv, b, lmax, steps, lo, hi):
    """Pre-smoothing from x = 0; also returns the residual b - A x."""
    return chebyshev(apply_A, Dinv, b, np.zeros_like(b), lmax, steps, lo, hi, r=b.copy())


def chebyshev_post(apply_A, Dinv, b, x, lmax, steps, lo, hi):
    x, _ = chebyshev(apply_A, Dinv, b, x, lmax, steps, lo, hi, need_residual=False)
    return x


# ------------------------------------------------------------ hierarchy

@dataclasses.dataclass
class Level:
    S: object               # sparse matrix of this level
    bs: int                 # block size (9 at level 0, 16 above)
    W: object = None        # covisibility counts of this level's nodes
    agg: np.ndarray = None  # aggregate of every node (None on the coarsest level)
    n_agg: int = 0
    P: object = None        # tentative prolongator to the next level
    Pb: np.ndarray = None
    Kc: np.ndarray = None
    Dinv: np.ndarray = None
    lmax: float = 0.0
    chol: np.ndarray = None  # coarsest level: Cholesky factor of the equilibrated matrix
    cscale: np.ndarray = None  # coarsest level: equilibration diag(S)^-1/2


def smoothed_prolongator(S, bs, P, lmax, omega_scale=4.0 / 3.0):
    """Smoothed aggregation (Section 3.5 weighs it against the unsmoothed P the
    paper uses): one damped block-Jacobi sweep applied to the tentative
    prolongator, P_s = (I - w D^-1 S) P with D the bs x bs block diagonal of S
    and w = omega_scale / lambda_max(D^-1 S) (the usual 4/3 of Vanek et al.)."""
    Dinv = np.linalg.inv(block_diagonal(S, bs))
    Dinv_s = sp.block_diag(list(Dinv), format="csr")
    return (P - (omega_scale / lmax) * (Dinv_s @ (S @ P))).tocsr()


def build_hierarchy(S0, K0, W0, opts: MGOptions = MGOptions(), apply_S0=None):
    """Set up the whole hierarchy from the explicit level-0 Schur complement S0,
    the camera near-nullspace rows K0 [n_cam, 9, 16] and the covisibility W0."""
    levels = []
    S, K, W, bs = S0, K0, W0, 9
    while True:
        lev = Level(S=S, bs=bs, W=W)
        levels.append(lev)
        n = W.shape[0]
        l = len(levels) - 1
        if n <= opts.coarse_max_nodes or len(levels) == opts.max_levels:
            break
        agg, n_agg = agglib.aggregate(W, opts.agg_cap)
        if n_agg > opts.min_ratio * n:
            break
        Pb, Kc, P = tentative_prolongator(K, agg, n_agg)
        if opts.smooth_prolongator:
            Dinv_l = np.linalg.inv(block_diagonal(S, bs))
            lm = lanczos_lmax(lambda x, S=S: S @ x, Dinv_l, lanczos_start(S.shape[0], l), opts.lanczos_steps)
            P = smoothed_prolongator(S, bs, sp.csr_matrix(P), lm, opts.smooth_omega)
        lev.agg, lev.n_agg, lev.Pb, lev.Kc, lev.P = agg, n_agg, Pb, Kc, P
        S = (P.T @ S @ P).tocsr()
        W = agglib.coarse_covisibility(W, agg, n_agg)
        K, bs = Kc, 16
    for l, lev in enumerate(levels):
        if l == len(levels) - 1:
            Sd = lev.S.toarray() if sp.issparse(lev.S) else lev.S
            # direct solve on the equilibrated matrix s S s, s = diag(S)^-1/2
            # (same inverse; keeps the factorization accurate when the camera
            # parameters live on very different scales)
            lev.cscale = 1.0 / np.sqrt(np.diag(Sd))
            Ss = Sd * lev.cscale[:, None] * lev.cscale[None, :]
            lev.chol = np.linalg.cholesky(Ss)
        else:
            Dblk = block_diagonal(lev.S, lev.bs)
            lev.Dinv = np.linalg.inv(Dblk)
            A = (lambda x, S=lev.S: S @ x)
            v0 = lanczos_start(lev.S.shape[0], l)
            lev.lmax = lanczos_lmax(A, lev.Dinv, v0, opts.lanczos_steps)
    return levels


def vcycle(levels, b, opts: MGOptions = MGOptions(), l=0):
    """Algorithm 1 with x = 0 on entry."""
    lev = levels[l]
    if l == len(levels) - 1:
        y = solve_triangular(lev.chol, lev.cscale * b, lower=True)
        return lev.cscale * solve_triangular(lev.chol.T, y, lower=False)
    A = (lambda v, S=lev.S: S @ v)
    x, r = chebyshev_pre(A, lev.Dinv, b, lev.lmax, opts.cheb_degree, opts.cheb_lo, opts.cheb_hi)
    rc = lev.P.T @ r
    xc = vcycle(levels, rc, opts, l + 1)
    x = x + lev.P @ xc
    x = chebyshev_post(A, lev.Dinv, b, x, lev.lmax, opts.cheb_degree, opts.cheb_lo, opts.cheb_hi)
    return x


# ------------------------------------------------------------ PCG

@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    rel_res: float          # recursive residual norm / ||b||
    converged: bool
    history: list


def pcg(apply_A, apply_M, b, rtol, max_iter=10000, forcing=None):
    """Saad Algorithm 9.1, x0 = 0, stop on ||r|| <= rtol ||b||.

    forcing = tau additionally stops on the Nash-Sofer rule of Section 2.1
    (a constant forcing sequence, Section 5): with the quadratic model
    Q_i = 1/2 x_i^T A x_i - x_i^T b of iterate i (Q_0 = 0), stop once
    i (Q_i - Q_{i-1}) / Q_i <= tau. Q_i is evaluated from its definition."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return PCGResult(x, 0, 0.0, True, [])
    z = apply_M(r)
    p = z.copy()
    rz = r @ z
    hist = []
    q_prev = 0.0
    for it in range(1, max_iter + 1):
        Ap = apply_A(p)
        pAp = p @ Ap
        if pAp <= 0 or rz <= 0:
            raise np.linalg.LinAlgError("PCG breakdown: operator or preconditioner not SPD")
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rn = np.linalg.norm(r)
        hist.append(rn / bn)
        if rn <= rtol * bn:
            return PCGResult(x, it, rn / bn, True, hist)
        if forcing is not None:
            q = 0.5 * (x @ apply_A(x)) - x @ b
            if it * (q - q_prev) / q <= forcing:
                return PCGResult(x, it, rn / bn, True, hist)
            q_prev = q
        z = apply_M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return PCGResult(x, max_iter, hist[-1], False, hist)
