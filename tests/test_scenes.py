"""The seeded input generators are deterministic and have the stated shapes."""
import numpy as np

from paper_2603_18707_amd import scenes


def _eq(a, b):
    return all(np.array_equal(getattr(a, k), getattr(b, k)) for k in ("means3d", "scales", "quats", "opacities", "sh"))


def test_tiny_deterministic():
    a, ca = scenes.workload_tiny()
    b, cb = scenes.workload_tiny()
    assert _eq(a, b) and np.array_equal(ca.viewmat, cb.viewmat)
    assert a.n == 1000 and a.sh.shape == (1000, 1, 3) and a.means3d.dtype == np.float32
    assert ca.width == ca.height == 128 and abs(ca.fx - 64 / np.tan(np.radians(30))) < 1e-4
    assert np.allclose(np.linalg.norm(a.quats, axis=1), 1, atol=1e-6)
    assert np.all((a.opacities > 0) & (a.opacities < 1))


def test_cluster_scene_shapes_and_seed():
    a = scenes.cluster_scene(5000, seed=2)
    b = scenes.cluster_scene(5000, seed=2)
    c = scenes.cluster_scene(5000, seed=3)
    assert _eq(a, b) and not _eq(a, c)
    assert a.sh.shape == (5000, 16, 3) and a.sh_degree == 3
    assert np.all(np.abs(a.means3d) <= 10.0)


def test_camera_conventions():
    cam = scenes.orbit_camera(1920, 1080, 0.0)
    # the camera at (0, 0, -30) sees the origin at depth 30 on the optical axis
    p = cam.viewmat @ np.array([0, 0, 0, 1.0])
    assert np.allclose(p[:3], [0, 0, 30], atol=1e-5)
    R = cam.viewmat[:3, :3].astype(np.float64)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-6) and np.linalg.det(R) > 0
    assert cam.cx == 960.0 and cam.cy == 540.0


def test_sample_pixels():
    p = scenes.sample_pixels(100, 50, 300, seed=4)
    assert p.shape == (300, 2) and len({tuple(x) for x in p}) == 300
    assert p[:, 0].max() < 100 and p[:, 1].max() < 50
    assert np.array_equal(p, scenes.sample_pixels(100, 50, 300, seed=4))
