"""Oracle: the Huber loss of the paper's robust error metrics (Section 5.4)
and the reweighted least-squares problem an LM step solves with it.

Test infrastructure only. The paper applies a loss to x = |f_o|^2, the squared
norm of an observation's reprojection error: loss(x) = x for x <= 1 and
2 sqrt(x) - 1 above. Reading (the paper gives only the unit scale): with scale
a the loss is rho(s) = s for s <= a^2 and 2 a sqrt(s) - a^2 above, which is the
paper's loss at a = 1 and stays continuously differentiable at s = a^2.

The objective becomes 1/2 sum_o rho(|f_o|^2). An LM step linearises it by
iteratively reweighted least squares: each observation's residual and
Jacobian rows are multiplied by sqrt(rho'(s_o)), so that J~^T f~ is the exact
gradient of the objective and J~^T J~ its Gauss-Newton matrix with the
curvature of rho left out. (Triggs et al., "Bundle adjustment -- a modern
synthesis", 2000, Section 4.3, add a rank-one curvature term where rho'' > 0;
Huber's rho'' is 0 inside and negative outside, where that term is dropped.)
"""
from __future__ import annotations

import numpy as np


def huber(s, a=1.0):
    """rho(s) elementwise."""
    s = np.asarray(s, dtype=np.float64)
    out = s.copy()
    big = s > a * a
    out[big] = 2.0 * a * np.sqrt(s[big]) - a * a
    return out


def huber_derivative(s, a=1.0):
    """rho'(s): 1 inside, a / sqrt(s) outside."""
    s = np.asarray(s, dtype=np.float64)
    out = np.ones_like(s)
    big = s > a * a
    out[big] = a / np.sqrt(s[big])
    return out


def weights(f, loss, a=1.0):
    """sqrt(rho'(|f_o|^2)) per observation for f [n_obs, 2]; None = squared loss."""
    if loss is None or loss == "squared":
        return np.ones(f.shape[0])
    if loss != "huber":
        raise ValueError(loss)
    return np.sqrt(huber_derivative(np.sum(f * f, axis=1), a))


def objective(f, loss, a=1.0):
    """1/2 sum_o rho(|f_o|^2)."""
    s = np.sum(f * f, axis=1)
    if loss is None or loss == "squared":
        return 0.5 * float(np.sum(s))
    return 0.5 * float(np.sum(huber(s, a)))
