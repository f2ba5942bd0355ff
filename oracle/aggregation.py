"""Oracle: visibility strength of connection and greedy aggregation (Section 3.2).

Test infrastructure only.

Strength of connection (Section 3.2): with v_k the 0/1 vector of points seen by
camera k, G_ij = v_i^T v_j / (|v_i| |v_j|) for i != j and 0 on the diagonal.
Writing W = V V^T (integer covisibility counts; W_ii = |v_i|^2),
G_ij = W_ij / sqrt(W_ii W_jj). Both sides of the method evaluate this in
IEEE FP64 exactly as written: float(W_ij) / sqrt(float(W_ii) * float(W_jj)).

Aggregation (Algorithm 2): visit nodes in index order; an unaggregated node i
scans its neighbours j by decreasing G_ij and either forms a new aggregate
{i, j} with the first unaggregated one, or joins the first neighbour's
aggregate holding fewer than 20 nodes.

Readings where the paper is silent:
  * equal strengths: the lower neighbour index comes first;
  * "20 dofs" is read as 20 nodes (cameras at level 0, aggregates above);
  * a node still unaggregated after the sweep joins the aggregate of its first
    neighbour in the same order, even past the cap; a node with no neighbour
    becomes a singleton aggregate;
  * aggregate ids are numbered in creation order; members ascend;
  * coarse strength: an aggregate's visibility vector is the sum of its
    members', so W_{l+1} = Ahat^T W_l Ahat with Ahat the 0/1 aggregate matrix,
    and G_{l+1} is computed from W_{l+1} by the same formula.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

AGG_CAP = 20


def covisibility(obs_cam, obs_pt, n_cam, n_pt):
    """W = V V^T as a sparse int64 matrix (V: n_cam x n_pt, 0/1)."""
    V = sp.csr_matrix((np.ones(obs_cam.shape[0], dtype=np.int64), (obs_cam, obs_pt)),
                      shape=(n_cam, n_pt))
    if V.max() > 1:
        raise ValueError("duplicate (camera, point) observation")
    return (V @ V.T).tocsr()


def strength(W_ij, W_ii, W_jj):
    return float(W_ij) / np.sqrt(float(W_ii) * float(W_jj))


def neighbour_order(W):
    """For every node, its neighbours sorted by decreasing G (ties: lower index)."""
    W = W.tocsr()
    W.sort_indices()
    diag = W.diagonal()
    orders = []
    for i in range(W.shape[0]):
        cols = W.indices[W.indptr[i]:W.indptr[i + 1]]
        vals = W.data[W.indptr[i]:W.indptr[i + 1]]
        nb = [(-strength(v, diag[i], diag[j]), int(j)) for j, v in zip(cols, vals) if j != i]
        nb.sort()
        orders.append([j for _, j in nb])
    return orders


def aggregate(W, cap=AGG_CAP):
    """Algorithm 2 plus the leftover rule. Returns (agg_id [n] int64, n_agg)."""
    n = W.shape[0]
    orders = neighbour_order(W)
    agg = -np.ones(n, dtype=np.int64)
    size = []
    for i in range(n):
        if agg[i] != -1:
            continue
        for j in orders[i]:
            if agg[j] == -1:
                agg[i] = agg[j] = len(size)
                size.append(2)
                break
            if size[agg[j]] < cap:
                agg[i] = agg[j]
                size[agg[j]] += 1
                break
    for i in range(n):
        if agg[i] != -1:
            continue
        if orders[i]:
            a = agg[orders[i][0]]
            agg[i] = a
            size[a] += 1
        else:
            agg[i] = len(size)
            size.append(1)
    return agg, len(size)


def coarse_covisibility(W, agg, n_agg):
    """W_{l+1} = Ahat^T W Ahat."""
    n = W.shape[0]
    Ahat = sp.csr_matrix((np.ones(n, dtype=np.int64), (np.arange(n), agg)), shape=(n, n_agg))
    return (Ahat.T @ W @ Ahat).tocsr()
