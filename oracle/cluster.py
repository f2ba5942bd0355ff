"""Oracle: the visibility-based block-Jacobi preconditioner the paper compares
against (Section 2.2, the block-Jacobi preconditioner of Kushal and Agarwal
formed from camera visibility; results in Section 5).

Test infrastructure only. The preconditioner is the inverse of the
block-diagonal part of S over clusters of cameras: M^-1 r restricted to a
cluster c is (S_cc)^-1 r_c with S_cc the principal submatrix of S on the
cluster's 9m unknowns. Reading (the paper does not say how the clusters are
formed): the clusters are the level-0 aggregates of Algorithm 2, which group
cameras by the same visibility strength, at most 20 per aggregate except the
leftovers; a camera outside every aggregate (a single-level hierarchy) is a
cluster of its own, which is point block Jacobi.
"""
from __future__ import annotations

import numpy as np

from . import aggregation as agglib


def clusters(W0, opts):
    """Cluster id of every camera: the level-0 aggregates when the multigrid
    hierarchy has a second level (the same stop rule as the hierarchy: more
    than coarse_max_nodes cameras, more than one level allowed, and
    aggregation keeping at most min_ratio of the nodes); otherwise one camera
    per cluster."""
    n = W0.shape[0]
    single = (np.arange(n), n)
    if n <= opts.coarse_max_nodes or opts.max_levels == 1:
        return single
    agg, n_agg = agglib.aggregate(W0, opts.agg_cap)
    if n_agg > opts.min_ratio * n:
        return single
    return agg, n_agg


def cluster_inverses(S, agg, n_agg):
    """For S (9n x 9n, dense or scipy sparse) and the aggregate id of every
    camera: (members of each cluster in ascending order, dense inverse of its
    principal submatrix)."""
    S = S.toarray() if hasattr(S, "toarray") else np.asarray(S)
    out = []
    for a in range(n_agg):
        mem = np.flatnonzero(agg == a)
        idx = (9 * mem[:, None] + np.arange(9)[None, :]).ravel()
        out.append((mem, np.linalg.inv(S[np.ix_(idx, idx)])))
    return out


def apply(blocks, r):
    """z = M^-1 r for the cluster inverses of cluster_inverses."""
    z = np.zeros_like(r)
    for mem, inv in blocks:
        idx = (9 * mem[:, None] + np.arange(9)[None, :]).ravel()
        z[idx] = inv @ r[idx]
    return z
