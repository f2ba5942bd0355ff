"""Seeded synthetic bundle-adjustment scenes.

This module only synthesises inputs. It holds none of the solver's arithmetic:
no Jacobians, no normal equations, no preconditioner. To write pixel
observations it does need a forward camera model (Section 4 of the paper
builds its datasets the same way: ground truth first, then visibility and
projection, then noise). That forward model is written here on rotation
matrices built from look-at frames, never from the angle-axis vector the
solver consumes; the angle-axis parameters are obtained with the matrix
logarithm. The oracle's zero-residual check therefore compares two
independently written camera models.

Camera parameters per camera, in order:
    [w0 w1 w2 | t0 t1 t2 | f | k1 k2]
with x_cam = R(w) X + t, the camera looking down its -z axis,
p = -(x_cam.x, x_cam.y) / x_cam.z, and pixel = f (1 + k1 |p|^2 + k2 |p|^4) p
(the 9-parameter camera of the Bundle Adjustment in the Large datasets the
paper cites in Section 4).

Scenes (seeds are fixed per scene so every run sees the same input):
    ring       cameras on a circle looking inward, points in the unit ball
    city       random walk on a street grid, facade points
    path       one long smooth path without loop closures
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

UP = np.array([0.0, 0.0, 1.0])


@dataclasses.dataclass
class Scene:
    name: str
    cams_true: np.ndarray  # [n_cam, 9] float64
    pts_true: np.ndarray   # [n_pt, 3]
    cams: np.ndarray       # [n_cam, 9] perturbed initial parameters
    pts: np.ndarray        # [n_pt, 3] perturbed initial points
    obs_cam: np.ndarray    # [n_obs] int32
    obs_pt: np.ndarray     # [n_obs] int32
    uv: np.ndarray         # [n_obs, 2] noisy observations of the truth
    uv_clean: np.ndarray   # [n_obs, 2] noise-free projections of the truth

    @property
    def n_cam(self):
        return self.cams.shape[0]

    @property
    def n_pt(self):
        return self.pts.shape[0]

    @property
    def n_obs(self):
        return self.obs_cam.shape[0]

    def summary(self) -> dict:
        k = np.bincount(self.obs_pt, minlength=self.n_pt)
        return {"name": self.name, "n_cam": int(self.n_cam), "n_pt": int(self.n_pt),
                "n_obs": int(self.n_obs), "obs_per_pt_mean": float(k.mean()),
                "obs_per_pt_max": int(k.max())}


# ---------------------------------------------------------------- geometry

def look_rotations(dirs: np.ndarray) -> np.ndarray:
    """World->camera rotation matrices whose camera -z axis points along dirs."""
    d = dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
    z_ax = -d
    x_ax = np.cross(d, UP)
    bad = np.linalg.norm(x_ax, axis=1) < 1e-9
    x_ax[bad] = np.array([1.0, 0.0, 0.0])
    x_ax /= np.linalg.norm(x_ax, axis=1, keepdims=True)
    y_ax = np.cross(z_ax, x_ax)
    return np.stack([x_ax, y_ax, z_ax], axis=1)  # rows are the camera axes


def _forward_project(Rm, t, f, k1, k2, X):
    """Forward model on rotation matrices (used only to synthesise pixels)."""
    xc = np.einsum("nij,nj->ni", Rm, X) + t
    p = -xc[:, :2] / xc[:, 2:3]
    n2 = np.sum(p * p, axis=1)
    s = f * (1.0 + k1 * n2 + k2 * n2 * n2)
    return s[:, None] * p, xc[:, 2]


def sine_field(P, amplitude, wavelength):
    """Long-range displacement of world positions P [n, 3]: x moves with
    sin(2 pi y / wavelength), y with sin(2 pi x / wavelength), both by
    `amplitude` metres. Smooth, so nearby cameras and points move together."""
    w = 2.0 * np.pi / wavelength
    return amplitude * np.column_stack([np.sin(w * P[:, 1]), np.sin(w * P[:, 0]), np.zeros(P.shape[0])])


def _finish(name, rng, centers, dirs, X, obs_cam, obs_pt, sigma_px=1.0, sigma_par=1e-2, long_range=None):
    """Truth parameters, noise-free and noisy pixels, perturbed initial values.
    long_range = (amplitude, wavelength) adds sine_field to the initial camera
    centres and points on top of the local noise (the long-range error of the
    paper's scaling experiment); it draws no random numbers."""
    n_cam = centers.shape[0]
    Rm = look_rotations(dirs)
    omega = Rotation.from_matrix(Rm).as_rotvec()
    t = -np.einsum("nij,nj->ni", Rm, centers)
    f = np.full(n_cam, 500.0)
    k1 = rng.normal(0.0, 1e-3, n_cam)
    k2 = rng.normal(0.0, 1e-3, n_cam)
    cams_true = np.column_stack([omega, t, f, k1, k2])
    order = np.lexsort((obs_cam, obs_pt))
    obs_cam = obs_cam[order].astype(np.int32)
    obs_pt = obs_pt[order].astype(np.int32)
    uv_clean, z = _forward_project(Rm[obs_cam], t[obs_cam], f[obs_cam], k1[obs_cam],
                                   k2[obs_cam], X[obs_pt])
    if np.any(z >= 0):
        raise RuntimeError("synthetic scene has a point behind an observing camera")
    uv = uv_clean + rng.normal(0.0, sigma_px, uv_clean.shape)
    # Initial values: every parameter perturbed by N(0, sigma_par). The pose is
    # perturbed about the camera's own centre (a rotation of that size in the
    # camera frame, the centre moved by that many metres); adding noise to w
    # with t held fixed would swing each camera about the world origin by
    # sigma_par times its distance from it.
    dR = Rotation.from_rotvec(rng.normal(0.0, sigma_par, (n_cam, 3))).as_matrix()
    Rp = np.einsum("nij,njk->nik", dR, Rm)
    cp = centers + rng.normal(0.0, sigma_par, centers.shape)
    if long_range is not None:
        cp = cp + sine_field(centers, *long_range)
    cams = np.column_stack([Rotation.from_matrix(Rp).as_rotvec(), -np.einsum("nij,nj->ni", Rp, cp),
                            f + rng.normal(0.0, sigma_par, n_cam), k1 + rng.normal(0.0, sigma_par, n_cam),
                            k2 + rng.normal(0.0, sigma_par, n_cam)])
    pts = X + rng.normal(0.0, sigma_par, X.shape)
    if long_range is not None:
        pts = pts + sine_field(X, *long_range)
    return Scene(name, cams_true, X.copy(), cams, pts, obs_cam, obs_pt, uv, uv_clean)


# ---------------------------------------------------------------- ring scene

def ring_scene(n_cam=64, n_pt=4000, cap=8, seed=0, radius=5.0, half_angle_deg=15.0,
               name="ring"):
    """Cameras on a circle of the given radius in the z=0 plane, looking at the
    origin; points uniform in the unit ball; each point is seen by the cameras
    whose view cone contains it, keeping the `cap` nearest (ties -> lower index)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = 2.0 * np.pi * np.arange(n_cam) / n_cam
    centers = np.column_stack([radius * np.cos(ang), radius * np.sin(ang), np.zeros(n_cam)])
    dirs = -centers / radius
    # uniform in the unit ball
    v = rng.normal(size=(n_pt, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    X = v * rng.uniform(0.0, 1.0, (n_pt, 1)) ** (1.0 / 3.0)
    rel = X[:, None, :] - centers[None, :, :]                  # [n_pt, n_cam, 3]
    dist = np.linalg.norm(rel, axis=2)
    cosang = np.einsum("pcj,cj->pc", rel, dirs) / dist
    vis = cosang > math.cos(math.radians(half_angle_deg))
    key = np.where(vis, dist, np.inf)
    order = np.lexsort((np.broadcast_to(np.arange(n_cam), key.shape), key), axis=1)
    obs_cam, obs_pt = [], []
    for p in range(n_pt):
        sel = [c for c in order[p] if vis[p, c]][:cap]
        obs_cam.extend(sel)
        obs_pt.extend([p] * len(sel))
    return _finish(name, rng, centers, dirs, X, np.array(obs_cam), np.array(obs_pt))


# ---------------------------------------------------------------- street grids

_DIRS = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])


def grid_walk(rng, n_cam, n_blocks, block_len, spacing=1.0, revisit_every=None):
    """Random walk along the streets of an n_blocks x n_blocks grid.

    Cameras are dropped every `spacing` metres, facing the direction of travel.
    With `revisit_every`, once that many cameras have passed since the walk
    last re-entered a street segment it had already driven, each turn is
    chosen to head for an earlier part of the walk until it re-enters one.
    """
    steps = int(round(block_len / spacing))
    node = rng.integers(0, n_blocks + 1, size=2)
    d = int(rng.integers(0, 4))
    centers, dirs = [], []
    visited = set()
    since = 0
    while len(centers) < n_cam:
        opts = []
        for nd in range(4):
            if nd == (d + 2) % 4 and len(centers) > 0:
                continue
            nxt = node + _DIRS[nd].astype(int)
            if np.all(nxt >= 0) and np.all(nxt <= n_blocks):
                opts.append(nd)
        if revisit_every is not None and since >= revisit_every and len(centers) > 0:
            seg_opts = [nd for nd in opts if _seg(node, nd) in visited]
            if seg_opts:
                d = seg_opts[int(rng.integers(0, len(seg_opts)))]
            else:
                # head toward a camera placed well before the current stretch
                old = np.asarray(centers[int(rng.integers(0, max(1, len(centers) - revisit_every)))])
                tgt = old / block_len
                best = min(opts, key=lambda nd: np.abs(node + _DIRS[nd] - tgt).sum()
                           + 1e-3 * rng.random())
                d = best
        else:
            d = opts[int(rng.integers(0, len(opts)))]
        seg = _seg(node, d)
        if seg in visited:
            since = 0
        visited.add(seg)
        start = node * block_len
        for s in range(steps):
            centers.append(start + s * spacing * _DIRS[d])
            dirs.append(_DIRS[d])
            since += 1
        node = node + _DIRS[d].astype(int)
    c2 = np.asarray(centers[:n_cam])
    d2 = np.asarray(dirs[:n_cam])
    cam_h = 2.0
    return (np.column_stack([c2, np.full(n_cam, cam_h)]),
            np.column_stack([d2, np.zeros(n_cam)]))


def _seg(node, d):
    a = tuple(int(v) for v in node)
    b = tuple(int(v) for v in node + _DIRS[d].astype(int))
    return (a, b) if a < b else (b, a)


def _choose_observers(rng, centers, dirs, X, k_want, max_dist, half_angle_deg, knn=48,
                      min_dist=2.0):
    """For each point the k nearest cameras that see it (frustum, at least
    min_dist and at most max_dist away: a point almost on a camera's centre
    would project anywhere once the parameters are perturbed)."""
    tree = cKDTree(centers)
    dist, idx = tree.query(X, k=knn, distance_upper_bound=max_dist, workers=-1)
    n_cam = centers.shape[0]
    valid = idx < n_cam
    idx_c = np.where(valid, idx, 0)
    rel = X[:, None, :] - centers[idx_c]
    cosang = np.einsum("pkj,pkj->pk", rel, dirs[idx_c]) / np.maximum(dist, 1e-12)
    valid &= cosang > math.cos(math.radians(half_angle_deg))
    valid &= dist >= min_dist
    rank = np.cumsum(valid, axis=1)
    take = valid & (rank <= k_want[:, None])
    n_vis = take.sum(axis=1)
    return idx_c, take, n_vis


def city_scene(n_cam, n_pt, n_blocks, block_len, k_sampler, seed, name,
               revisit_every=None, max_dist=15.0, half_angle_deg=60.0, chunk=1_000_000, long_range=None):
    """Street-view scene: a walk on a street grid and facade points at +-2 m
    lateral, 0-8 m high, each observed by its k nearest viewing cameras."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centers, dirs = grid_walk(rng, n_cam, n_blocks, block_len, revisit_every=revisit_every)
    X_all, oc_all, op_all = [], [], []
    have = 0
    while have < n_pt:
        m = min(chunk, int((n_pt - have) * 1.15) + 64)
        a = rng.integers(0, n_cam, m)
        ahead = rng.uniform(3.0, 12.0, m)
        side = np.where(rng.random(m) < 0.5, -2.0, 2.0)
        h = rng.uniform(0.0, 8.0, m)
        lat = np.cross(dirs[a], UP)
        X = centers[a] + ahead[:, None] * dirs[a] + side[:, None] * lat
        X[:, 2] = h
        k_want = k_sampler(rng, m)
        idx, take, n_vis = _choose_observers(rng, centers, dirs, X, k_want, max_dist,
                                             half_angle_deg)
        ok = np.nonzero(n_vis >= 2)[0][: n_pt - have]
        pid = have + np.arange(ok.size)
        t_ok = take[ok]
        oc_all.append(idx[ok][t_ok])
        op_all.append(np.repeat(pid, t_ok.sum(axis=1)))
        X_all.append(X[ok])
        have += ok.size
    X = np.concatenate(X_all)
    return _finish(name, rng, centers, dirs, X, np.concatenate(oc_all), np.concatenate(op_all),
                   long_range=long_range)


def scaling_scene(k):
    """City of k x k blocks of 10 m with 5 cameras and 1,500 points per block and
    a sine-wave long-range error (0.5 m over one city width): the growing-
    diameter problems of the paper's scaling experiment (Section 5.2)."""
    return city_scene(5 * k * k, 1500 * k * k, k, 10.0, _k_geometric, seed=100 + k, name=f"sine{k}",
                      long_range=(0.5, 10.0 * k))


def path_scene(n_cam, n_pt, seed, name, spacing=0.5, chunk=2_000_000):
    """One long smooth path without loop closures; each point is seen by k
    consecutive cameras (k = 3 + Binomial(5, 0.65)) and sits 5-30 m ahead of
    the last of them, 2-10 m to the side, -1..5 m above the camera."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.arange(n_cam) * spacing
    ph = rng.uniform(0.0, 2.0 * np.pi, 3)
    heading = (0.6 * np.sin(2 * np.pi * s / 1300.0 + ph[0])
               + 0.3 * np.sin(2 * np.pi * s / 410.0 + ph[1])
               + 0.15 * np.sin(2 * np.pi * s / 97.0 + ph[2]))
    d2 = np.column_stack([np.cos(heading), np.sin(heading)])
    c2 = np.concatenate([[0.0, 0.0]] + [[0.0, 0.0]] * 0).reshape(1, 2) + \
        np.vstack([np.zeros(2), np.cumsum(spacing * d2[:-1], axis=0)])
    centers = np.column_stack([c2, np.full(n_cam, 1.5)])
    dirs = np.column_stack([d2, np.zeros(n_cam)])
    X_all, oc_all, op_all = [], [], []
    have = 0
    while have < n_pt:
        m = min(chunk, int((n_pt - have) * 1.05) + 64)
        k = 3 + rng.binomial(5, 0.65, m)
        first = rng.integers(0, n_cam - k + 1)
        last = first + k - 1
        ahead = rng.uniform(5.0, 30.0, m)
        lat = rng.uniform(2.0, 10.0, m) * np.where(rng.random(m) < 0.5, -1.0, 1.0)
        h = rng.uniform(-1.0, 5.0, m)
        side = np.cross(dirs[last], UP)
        X = centers[last] + ahead[:, None] * dirs[last] + lat[:, None] * side
        X[:, 2] = centers[last, 2] + h
        # every observer must have the point in front of it
        kmax = 8
        off = np.arange(kmax)
        cams_k = first[:, None] + np.minimum(off[None, :], (k - 1)[:, None])
        front = np.einsum("pkj,pkj->pk", X[:, None, :] - centers[cams_k], dirs[cams_k]) > 1.0
        ok = np.nonzero(front.all(axis=1))[0][: n_pt - have]
        pid = have + np.arange(ok.size)
        kk = k[ok]
        oc_all.append((np.repeat(first[ok], kk) + _ragged_arange(kk)))
        op_all.append(np.repeat(pid, kk))
        X_all.append(X[ok])
        have += ok.size
    X = np.concatenate(X_all)
    return _finish(name, rng, centers, dirs, X, np.concatenate(oc_all), np.concatenate(op_all))


def _ragged_arange(counts):
    counts = np.asarray(counts, dtype=np.int64)
    starts = np.repeat(np.cumsum(counts) - counts, counts)
    return np.arange(counts.sum()) - starts


def _k_geometric(rng, m, p=0.11, kmin=2, kmax=12):
    """k = kmin + Geometric failures, conditioned on k <= kmax (by resampling)."""
    k = np.full(m, kmax + 1)
    bad = np.ones(m, dtype=bool)
    while bad.any():
        k[bad] = kmin + rng.geometric(p, bad.sum()) - 1
        bad = k > kmax
    return k


def _k_powerlaw(rng, m, alpha=0.75, kmin=2, kmax=15):
    ks = np.arange(kmin, kmax + 1)
    w = ks.astype(float) ** (-alpha)
    return rng.choice(ks, size=m, p=w / w.sum())


# ---------------------------------------------------------------- named scenes

def make_scene(name: str) -> Scene:
    """The named synthetic workloads.

    ring64    64 cameras / 4,000 points / cap 8 (seed 0)            -- small FP64 step
    city2k    2,000 cameras / 600k points, 20x20 grid of 10 m blocks (seed 1)
    path10k   10,000 cameras / 4M points, 5 km path, 0.5 m spacing (seed 2)
    ring20    20 cameras / 800 points / cap 8 (seed 3)             -- finite differences
    city30k   30,000 cameras / 12M points, 40x40 grid of 100 m blocks,
              loop closures every 500 cameras (seed 4)
    Smaller shapes of the same generators for tests:
    city200   200 cameras / 20k points, 6x6 grid of 10 m blocks (seed 11)
    path500   500 cameras / 40k points (seed 12)
    city1k    1,000 cameras / 150k points, 12x12 grid (seed 13)
    sine<k>   k x k city blocks with a sine-wave long-range error (scaling_scene)
    """
    if name == "ring64":
        return ring_scene(64, 4000, 8, seed=0, name=name)
    if name == "ring20":
        return ring_scene(20, 800, 8, seed=3, name=name)
    if name == "city2k":
        return city_scene(2000, 600_000, 20, 10.0, _k_geometric, seed=1, name=name)
    if name == "path10k":
        return path_scene(10_000, 4_000_000, seed=2, name=name)
    if name == "city30k":
        return city_scene(30_000, 12_000_000, 40, 100.0, _k_powerlaw, seed=4, name=name,
                          revisit_every=500)
    if name == "city200":
        return city_scene(200, 20_000, 6, 10.0, _k_geometric, seed=11, name=name)
    if name == "city1k":
        return city_scene(1000, 150_000, 12, 10.0, _k_geometric, seed=13, name=name)
    if name == "path500":
        return path_scene(500, 40_000, seed=12, name=name)
    if name.startswith("sine") and name[4:].isdigit():
        return scaling_scene(int(name[4:]))
    raise KeyError(name)


def tiny_scene(n_cam, n_pt, seed, k_min=2, k_max=None, shuffle=True) -> Scene:
    """Small random scenes (for randomized checks): cameras on a noisy ring,
    points near the centre, each point seen by k random cameras that view it;
    observations optionally shuffled out of point order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = 2 * np.pi * np.arange(n_cam) / n_cam + rng.normal(0, 0.05, n_cam)
    r = 6.0 + rng.normal(0, 0.3, n_cam)
    centers = np.column_stack([r * np.cos(ang), r * np.sin(ang), rng.normal(0, 0.3, n_cam)])
    dirs = -centers + rng.normal(0, 0.1, centers.shape)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    X = rng.normal(0, 0.7, (n_pt, 3))
    k_max = k_max or n_cam
    oc, op = [], []
    for p in range(n_pt):
        k = int(rng.integers(k_min, min(k_max, n_cam) + 1))
        sel = np.sort(rng.choice(n_cam, size=k, replace=False))
        oc.extend(sel)
        op.extend([p] * k)
    sc = _finish(f"tiny{n_cam}x{n_pt}s{seed}", rng, centers, dirs, X, np.array(oc), np.array(op))
    if shuffle:
        perm = rng.permutation(sc.n_obs)
        sc.obs_cam, sc.obs_pt = sc.obs_cam[perm], sc.obs_pt[perm]
        sc.uv, sc.uv_clean = sc.uv[perm], sc.uv_clean[perm]
    return sc


# ---------------------------------------------------------------- cache

_FIELDS = ("cams_true", "pts_true", "cams", "pts", "obs_cam", "obs_pt", "uv", "uv_clean")


def cached_scene(name: str, cache_dir: str | None) -> Scene:
    """make_scene(name), kept as <cache_dir>/<name>.npz (plain arrays, no pickled
    objects) so that repeated runs on one machine skip the generation. With
    cache_dir None the scene is generated every time."""
    import os
    if not cache_dir:
        return make_scene(name)
    path = os.path.join(cache_dir, f"{name}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return Scene(name, *(z[f] for f in _FIELDS))
    sc = make_scene(name)
    os.makedirs(cache_dir, exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **{f: getattr(sc, f) for f in _FIELDS})
    os.replace(tmp, path)
    return sc
