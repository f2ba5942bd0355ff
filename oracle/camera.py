"""Oracle: reprojection residual and its Jacobian blocks (plain numpy, FP64).

Test infrastructure only. Section 2.1 of the paper: the objective is the squared
sum of reprojection errors f_i(x) over all camera-point observations, and the
step equation needs J = df/dx = [F E] with F = df/dx_c (2x9 per observation)
and E = df/dx_p (2x3 per observation).

The paper names a "9-parameter camera" with a simple projective model but never
writes it out (Sections 2.1 and 6). Reading: the camera of the Bundle Adjustment
in the Large datasets cited in Section 4,
    x_cam = R(w) X + t,   p = -(x_cam.x, x_cam.y)/x_cam.z,
    r = 1 + k1 |p|^2 + k2 |p|^4,   pi = f r p,   f_o = pi_o - u_o,
with R(w) = I + a [w]x + b [w]x^2, a = sin(th)/th, b = (1 - cos th)/th^2.

The rotation derivative here is taken by the product rule on that (a, b) form,
which is a different derivation from the right-Jacobian form a kernel would
use; the two meet only through the finite-difference and parity checks.
"""
from __future__ import annotations

import math

import numpy as np

# Series switch: below this angle a, b and their derivatives come from their
# Taylor series, whose terms are generated from the factorial definitions.
_SERIES_THETA = 0.25
_NTERMS = 8


def _series(theta2, first, step):
    """sum_{n>=0} (-1)^n c_n theta^(2n) where c_n is given by `step(n)`."""
    out = np.zeros_like(theta2)
    pw = np.ones_like(theta2)
    for n in range(first, first + _NTERMS):
        out += ((-1) ** n) * step(n) * pw
        pw = pw * theta2
    return out


def rotation_coeffs(theta):
    """a = sin t/t, b = (1-cos t)/t^2, da = a'(t)/t, db = b'(t)/t (elementwise)."""
    theta = np.asarray(theta, dtype=np.float64)
    t2 = theta * theta
    small = theta < _SERIES_THETA
    ts = np.where(small, 1.0, theta)  # avoids 0/0 in the closed forms
    s, c = np.sin(ts), np.cos(ts)
    a_cf = s / ts
    b_cf = (1.0 - c) / (ts * ts)
    da_cf = (ts * c - s) / ts ** 3
    db_cf = (ts * s - 2.0 * (1.0 - c)) / ts ** 4
    f = math.factorial
    # a = sum (-1)^n t^2n/(2n+1)!,  b = sum (-1)^n t^2n/(2n+2)!
    a_s = _series(t2, 0, lambda n: 1.0 / f(2 * n + 1))
    b_s = _series(t2, 0, lambda n: 1.0 / f(2 * n + 2))
    # a'/t = sum_{n>=1} (-1)^n 2n t^(2n-2)/(2n+1)!  (shift index: m = n-1)
    da_s = -_series(t2, 0, lambda m: 2.0 * (m + 1) / f(2 * m + 3))
    db_s = -_series(t2, 0, lambda m: 2.0 * (m + 1) / f(2 * m + 4))
    pick = lambda x, y: np.where(small, x, y)
    return pick(a_s, a_cf), pick(b_s, b_cf), pick(da_s, da_cf), pick(db_s, db_cf)


def skew(w):
    """[w]x for a batch of 3-vectors: [..., 3] -> [..., 3, 3]."""
    w = np.asarray(w)
    z = np.zeros(w.shape[:-1])
    return np.stack([np.stack([z, -w[..., 2], w[..., 1]], -1),
                     np.stack([w[..., 2], z, -w[..., 0]], -1),
                     np.stack([-w[..., 1], w[..., 0], z], -1)], -2)


def rotation_matrix(omega):
    """R(w) = I + a[w]x + b[w]x^2 for a batch of angle-axis vectors."""
    omega = np.asarray(omega, dtype=np.float64)
    th = np.linalg.norm(omega, axis=-1)
    a, b, _, _ = rotation_coeffs(th)
    K = skew(omega)
    return np.eye(3) + a[..., None, None] * K + b[..., None, None] * (K @ K)


def project(cams, pts, obs_cam, obs_pt):
    """Projected pixel pi_o for every observation, and x_cam."""
    cam = cams[obs_cam]
    X = pts[obs_pt]
    R = rotation_matrix(cam[:, 0:3])
    xc = np.einsum("nij,nj->ni", R, X) + cam[:, 3:6]
    p = -xc[:, 0:2] / xc[:, 2:3]
    n2 = np.sum(p * p, axis=1)
    r = 1.0 + cam[:, 7] * n2 + cam[:, 8] * n2 * n2
    return cam[:, 6, None] * r[:, None] * p, xc


def residuals(cams, pts, obs_cam, obs_pt, uv):
    """f_o = pi_o - u_o, shape [n_obs, 2]."""
    pi, _ = project(cams, pts, obs_cam, obs_pt)
    return pi - uv


def objective(cams, pts, obs_cam, obs_pt, uv):
    """Half the squared sum of reprojection errors (Section 2.1; the 1/2 does
    not change the step)."""
    f = residuals(cams, pts, obs_cam, obs_pt, uv)
    return 0.5 * float(np.sum(f * f))


def jacobian_blocks(cams, pts, obs_cam, obs_pt):
    """F [n_obs, 2, 9] = d pi / d camera, E [n_obs, 2, 3] = d pi / d point.

    Chain rule through x_cam:
      d pi/d x_cam = f (r I + (2 k1 + 4 k2 |p|^2) p p^T) . dp/dx_cam,
      dp/dx_cam = [[-1/z, 0, x/z^2], [0, -1/z, y/z^2]],
      d x_cam/d t = I,  d x_cam/d X = R,
      d x_cam/d w_k = da_k [w]x X + a [e_k]x X + db_k [w]x^2 X
                      + b ([e_k]x [w]x + [w]x [e_k]x) X,
      with da_k = (a'(th)/th) w_k and db_k = (b'(th)/th) w_k;
      d pi/d f = r p,  d pi/d k1 = f |p|^2 p,  d pi/d k2 = f |p|^4 p.
    """
    cam = cams[obs_cam]
    X = pts[obs_pt]
    w = cam[:, 0:3]
    th = np.linalg.norm(w, axis=1)
    a, b, da, db = rotation_coeffs(th)
    K = skew(w)
    K2 = K @ K
    R = np.eye(3) + a[:, None, None] * K + b[:, None, None] * K2
    xc = np.einsum("nij,nj->ni", R, X) + cam[:, 3:6]
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    p = -xc[:, 0:2] / xc[:, 2:3]
    n2 = np.sum(p * p, axis=1)
    f, k1, k2 = cam[:, 6], cam[:, 7], cam[:, 8]
    r = 1.0 + k1 * n2 + k2 * n2 * n2
    n = xc.shape[0]
    dpdx = np.zeros((n, 2, 3))
    dpdx[:, 0, 0] = -1.0 / z
    dpdx[:, 0, 2] = x / (z * z)
    dpdx[:, 1, 1] = -1.0 / z
    dpdx[:, 1, 2] = y / (z * z)
    dpid_p = f[:, None, None] * (r[:, None, None] * np.eye(2)
                                 + (2.0 * k1 + 4.0 * k2 * n2)[:, None, None]
                                 * np.einsum("ni,nj->nij", p, p))
    M = dpid_p @ dpdx                               # d pi / d x_cam  [n,2,3]
    KX = np.einsum("nij,nj->ni", K, X)
    K2X = np.einsum("nij,nj->ni", K2, X)
    dRX = np.zeros((n, 3, 3))                       # column k = d(RX)/dw_k
    for k in range(3):
        ek = np.zeros(3)
        ek[k] = 1.0
        Ek = skew(ek)
        term = (da * w[:, k])[:, None] * KX + a[:, None] * (X @ Ek.T) \
            + (db * w[:, k])[:, None] * K2X \
            + b[:, None] * (np.einsum("ij,njk,nk->ni", Ek, K, X)
                            + np.einsum("nij,jk,nk->ni", K, Ek, X))
        dRX[:, :, k] = term
    F = np.zeros((n, 2, 9))
    F[:, :, 0:3] = M @ dRX
    F[:, :, 3:6] = M
    F[:, :, 6] = r[:, None] * p
    F[:, :, 7] = (f * n2)[:, None] * p
    F[:, :, 8] = (f * n2 * n2)[:, None] * p
    E = M @ R
    return F, E


def jacobian_fd(cams, pts, obs_cam, obs_pt, rel_step=1e-6):
    """Central-difference F and E (used only to check jacobian_blocks)."""
    n = obs_cam.shape[0]
    F = np.zeros((n, 2, 9))
    E = np.zeros((n, 2, 3))
    for k in range(9):
        h = rel_step * np.maximum(1.0, np.abs(cams[:, k]))
        cp, cm = cams.copy(), cams.copy()
        cp[:, k] += h
        cm[:, k] -= h
        d = (project(cp, pts, obs_cam, obs_pt)[0] - project(cm, pts, obs_cam, obs_pt)[0])
        F[:, :, k] = d / (2.0 * h[obs_cam][:, None])
    for k in range(3):
        h = rel_step * np.maximum(1.0, np.abs(pts[:, k]))
        pp, pm = pts.copy(), pts.copy()
        pp[:, k] += h
        pm[:, k] -= h
        d = (project(cams, pp, obs_cam, obs_pt)[0] - project(cams, pm, obs_cam, obs_pt)[0])
        E[:, :, k] = d / (2.0 * h[obs_pt][:, None])
    return F, E
