"""Oracle: visibility strength of connection and greedy aggregation (Section 3.2).

Test infrastructure only.

Strength of connection (Section 3.2): with v_k the 0/1 vector of points seen by
camera k, G_ij = v_i^T v_j / (|v_i| |v_j|) for i != j and 0 on the diagonal.
Writing W = V V^T (integer covisibility counts; W_ii = |v_i|^2),
G_ij = W_ij / sqrt(W_ii W_jj). The aggregation only ever compares two strengths
of the same row, G_ij against G_ik, and since every quantity is a positive
integer that comparison is decided exactly, without rounding:
    G_ij > G_ik  <=>  W_ij^2 W_kk > W_ik^2 W_jj
(Python integers, so no product overflows).

Aggregation (Algorithm 2): nodes are visited in index order. A node that is
not yet in an aggregate is grouped with the strongest neighbour it may join:
a neighbour that is itself ungrouped starts a new aggregate of the two, a
grouped one lends its aggregate if that still holds fewer than 20 nodes.

Readings where the paper is silent:
  * equal strengths (equal as exact rationals): the lower neighbour index comes
    first;
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

import functools

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
    """G_ij as a float (for reports; the ordering never uses it)."""
    return float(W_ij) / np.sqrt(float(W_ii) * float(W_jj))


def compare_strength(w_ij, w_jj, w_ik, w_kk):
    """Sign of G_ij - G_ik for two neighbours j, k of the same row i, exactly:
    +1, 0 or -1 as W_ij^2 W_kk is greater than, equal to or less than
    W_ik^2 W_jj (W_ii cancels)."""
    lhs = int(w_ij) * int(w_ij) * int(w_kk)
    rhs = int(w_ik) * int(w_ik) * int(w_jj)
    return (lhs > rhs) - (lhs < rhs)


def neighbour_order(W):
    """For every node, its neighbours sorted by decreasing G (ties: lower index)."""
    W = W.tocsr()
    W.sort_indices()
    diag = [int(d) for d in W.diagonal()]
    orders = []
    for i in range(W.shape[0]):
        cols = W.indices[W.indptr[i]:W.indptr[i + 1]]
        vals = W.data[W.indptr[i]:W.indptr[i + 1]]
        nb = [(int(j), int(v)) for j, v in zip(cols, vals) if j != i]

        def before(a, b):          # a = (j, W_ij), b = (k, W_ik): -1 if a comes first
            c = compare_strength(a[1], diag[a[0]], b[1], diag[b[0]])
            if c != 0:
                return -c
            return (a[0] > b[0]) - (a[0] < b[0])

        nb.sort(key=functools.cmp_to_key(before))
        orders.append([j for j, _ in nb])
    return orders


def aggregate(W, cap=AGG_CAP):
    """Algorithm 2 plus the leftover rule. Returns (agg_id [n] int64, n_agg)."""
    n = W.shape[0]
    orders = neighbour_order(W)
    agg = -np.ones(n, dtype=np.int64)
    members = []                   # members[a]: nodes of aggregate a, in joining order

    def partner(i):
        """Strongest neighbour that i may be grouped with (None if every neighbour
        sits in a full aggregate): ungrouped, or in an aggregate below the cap."""
        return next((j for j in orders[i] if agg[j] < 0 or len(members[agg[j]]) < cap), None)

    for i in range(n):
        if agg[i] >= 0:
            continue
        j = partner(i)
        if j is None:
            continue                # a leftover, placed after the sweep
        if agg[j] < 0:
            agg[i] = agg[j] = len(members)
            members.append([i, j])
        else:
            agg[i] = agg[j]
            members[agg[j]].append(i)
    for i in np.nonzero(agg < 0)[0]:
        if orders[i]:               # every neighbour of a leftover is grouped by now
            agg[i] = agg[orders[i][0]]
            members[agg[i]].append(int(i))
        else:
            agg[i] = len(members)
            members.append([int(i)])
    return agg, len(members)


def coarse_covisibility(W, agg, n_agg):
    """W_{l+1} = Ahat^T W Ahat."""
    n = W.shape[0]
    Ahat = sp.csr_matrix((np.ones(n, dtype=np.int64), (np.arange(n), agg)), shape=(n, n_agg))
    return (Ahat.T @ W @ Ahat).tocsr()
