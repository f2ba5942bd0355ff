"""Oracle: near-nullspace of the camera system (Section 3.1 of the paper).

Test infrastructure only. For monocular cameras and no fixed camera, J^T J has a
7-dimensional nullspace: 3 rotations, 3 translations and 1 scaling of the whole
world. The paper augments it with 9 columns that are constant in each of the 9
camera parameters, 16 columns in all.

Gauge modes, written as the first-order change of the parameters under the
world similarity X' = (1 + s)(I + [e]x) X + tau, which leaves every x_cam
(up to the common scale, to which the projection is blind) unchanged:
    tau_k : d omega = 0,                    d t = -R e_k,   d X = e_k
    e_k   : d omega = -J_r(omega)^-1 e_k,   d t = 0,        d X = e_k x X
    s     : d omega = 0,                    d t = t,        d X = X
where J_r is the right Jacobian of SO(3): R(omega + d) = R(omega) exp([J_r d]x).
This oracle obtains J_r^-1 by inverting J_r numerically (J_r = I - b [w]x +
c [w]x^2, b = (1 - cos th)/th^2, c = (th - sin th)/th^3).

Column order (a reading; the paper gives none): the 9 constant columns, then
tau_1..3, e_1..3, s. Intrinsic rows (f, k1, k2) of the gauge columns are 0.
"""
from __future__ import annotations

import math

import numpy as np

from .camera import rotation_matrix, skew


def _jr_coeffs(theta):
    """b = (1-cos)/t^2, c = (t - sin)/t^3, series below 0.25."""
    theta = np.asarray(theta, dtype=np.float64)
    small = theta < 0.25
    ts = np.where(small, 1.0, theta)
    b_cf = (1.0 - np.cos(ts)) / ts ** 2
    c_cf = (ts - np.sin(ts)) / ts ** 3
    t2 = theta * theta
    b_s = np.zeros_like(theta)
    c_s = np.zeros_like(theta)
    pw = np.ones_like(theta)
    for n in range(8):
        b_s += (-1) ** n * pw / math.factorial(2 * n + 2)
        c_s += (-1) ** n * pw / math.factorial(2 * n + 3)
        pw = pw * t2
    return np.where(small, b_s, b_cf), np.where(small, c_s, c_cf)


def right_jacobian(omega):
    omega = np.asarray(omega, dtype=np.float64)
    b, c = _jr_coeffs(np.linalg.norm(omega, axis=-1))
    K = skew(omega)
    return np.eye(3) - b[..., None, None] * K + c[..., None, None] * (K @ K)


def camera_nullspace(cams):
    """K rows per camera: [n_cam, 9, 16]."""
    n = cams.shape[0]
    K = np.zeros((n, 9, 16))
    K[:, :, 0:9] = np.eye(9)
    R = rotation_matrix(cams[:, 0:3])
    Jr_inv = np.linalg.inv(right_jacobian(cams[:, 0:3]))
    for k in range(3):
        K[:, 3:6, 9 + k] = -R[:, :, k]
        K[:, 0:3, 12 + k] = -Jr_inv[:, :, k]
    K[:, 3:6, 15] = cams[:, 3:6]
    return K


def point_gauge(pts):
    """Point rows of the 7 gauge modes: [n_pt, 3, 7] (tau, e, s order)."""
    n = pts.shape[0]
    N = np.zeros((n, 3, 7))
    N[:, :, 0:3] = np.eye(3)
    for k in range(3):
        ek = np.zeros(3)
        ek[k] = 1.0
        N[:, :, 3 + k] = np.cross(ek[None, :], pts)
    N[:, :, 6] = pts
    return N


def full_gauge(cams, pts):
    """The 7 gauge vectors of J^T J over all parameters: [9 n_cam + 3 n_pt, 7]."""
    Kc = camera_nullspace(cams)[:, :, 9:16].reshape(-1, 7)
    Np = point_gauge(pts).reshape(-1, 7)
    return np.vstack([Kc, Np])
