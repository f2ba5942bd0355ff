"""The long-range error of the scaling scenes: an exact, smooth displacement
added to the initial values on top of the local noise, truth untouched."""
import numpy as np

from oracle.camera import project, rotation_matrix
from scenes import city_scene, make_scene, sine_field
from scenes.generate import _k_geometric


def test_sine_field_is_added_exactly_and_leaves_the_truth():
    args = (5 * 16, 1500 * 16, 4, 10.0, _k_geometric, 104, "t")
    plain = city_scene(*args)
    wavy = city_scene(*args, long_range=(0.5, 40.0))
    for a, b in ((plain.cams_true, wavy.cams_true), (plain.pts_true, wavy.pts_true), (plain.uv, wavy.uv)):
        assert np.array_equal(a, b)
    assert np.allclose(wavy.pts - plain.pts, sine_field(plain.pts_true, 0.5, 40.0), atol=1e-12)
    # camera centres -R^T t moved by the field at the true centre (plus the same local noise)
    def centres(c):
        R = rotation_matrix(c[:, :3])
        return -np.einsum("nji,nj->ni", R, c[:, 3:6])
    d = centres(wavy.cams) - centres(plain.cams)
    assert np.allclose(d, sine_field(centres(plain.cams_true), 0.5, 40.0), atol=1e-6)


def test_sine_field_is_smooth_and_long_range():
    P = np.random.default_rng(0).uniform(0, 100, (2000, 3))
    u = sine_field(P, 0.5, 100.0)
    assert np.abs(u).max() <= 0.5 and np.abs(u).max() > 0.45
    # displacement differences between points 1 m apart stay below 2 pi a / lambda
    Q = P + np.array([1.0, 0.0, 0.0])
    assert np.abs(sine_field(Q, 0.5, 100.0) - u).max() <= 2 * np.pi * 0.5 / 100.0 + 1e-12


def test_scaling_scene_is_valid():
    sc = make_scene("sine4")
    assert sc.n_cam == 80 and sc.n_pt == 24000
    _, xc = project(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt)
    assert np.all(xc[:, 2] < 0)            # every point in front of its observers at the start
    assert np.all(np.bincount(sc.obs_pt, minlength=sc.n_pt) >= 2)
