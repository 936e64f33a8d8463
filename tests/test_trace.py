"""CPU tests of the serving workload's request generator: arrivals,
view-cone geometry, level of detail by distance, determinism."""
import numpy as np

import synth


def test_poisson_arrivals_and_determinism():
    ids, lods, t = synth.camera_trace(512, 512, 256, rate=2e5, duration_s=0.5, seed=3, t0_s=1.0)
    n = len(ids)
    # Poisson count: mean 1e5, sd ~316
    assert abs(n - 1e5) < 5 * 316
    assert (np.diff(t.astype(np.int64)) >= 0).all() and t[-1] < 0.5e9
    gaps = np.diff(t.astype(np.float64)) * 1e-9
    assert abs(gaps.mean() - 1 / 2e5) < 0.03 / 2e5
    # exponential gaps: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.03
    ids2, lods2, t2 = synth.camera_trace(512, 512, 256, rate=2e5, duration_s=0.5, seed=3, t0_s=1.0)
    assert (ids == ids2).all() and (lods == lods2).all() and (t == t2).all()


def test_requests_lie_in_the_volume_and_the_view_cone():
    nx, ny, nz = 2048, 1024, 512
    ids, lods, t = synth.camera_trace(nx, ny, nz, rate=1e5, duration_s=0.2, seed=4, t0_s=3.0)
    nbx, nby, nbz = nx // 32, ny // 32, nz // 32
    assert ids.max() < nbx * nby * nbz
    # brick centres against the camera at each request time
    bx, by, bz = ids % nbx, (ids // nbx) % nby, ids // (nbx * nby)
    c = np.stack([bx, by, bz], 1) * 32.0 + 16.0
    ctrl = synth.camera_path(nx, ny, nz, seed=7)
    assert (ctrl >= 0.15 * np.array([nx, ny, nz]) - 1e-9).all()
    pos, tan = synth.camera_pose(ctrl, ((t * 1e-9 + 3.0) / 20.0) % 1.0)
    v = c - pos
    d = np.linalg.norm(v, axis=1)
    fwd = tan / np.linalg.norm(tan, axis=1, keepdims=True)
    far = d > 64  # the brick centre is within half a brick diagonal of the sampled point
    cosang = (v[far] * fwd[far]).sum(1) / d[far]
    # half angle 30 deg, widened by the brick size at distance > 64
    assert (cosang > np.cos(np.radians(30 + np.degrees(np.arcsin(28 / 64))))).all()
    assert d.max() < 3000 + 28


def test_lod_follows_distance():
    # a long thin volume lets the camera see far: all three LODs occur, and
    # the level grows with the distance of the brick from the camera
    nx, ny, nz = 8192, 256, 256
    ids, lods, t = synth.camera_trace(nx, ny, nz, rate=1e5, duration_s=0.3, seed=5, d_max=6000.0, d0=1000.0)
    assert set(np.unique(lods)) <= {0, 1, 2}
    nbx, nby = nx // 32, ny // 32
    c = np.stack([ids % nbx, (ids // nbx) % nby, ids // (nbx * nby)], 1) * 32.0 + 16.0
    pos, _ = synth.camera_pose(synth.camera_path(nx, ny, nz, seed=7), ((t * 1e-9) / 20.0) % 1.0)
    d = np.linalg.norm(c - pos, axis=1)
    slack = 28.0
    assert (d[lods == 0] < 1000 + slack).all()
    assert (d[lods == 1] > 1000 - slack).all() and (d[lods == 1] < 2000 + slack).all()
    assert (d[lods == 2] > 2000 - slack).all()


def test_camera_path_passes_through_its_control_points():
    # uniform Catmull-Rom: at u = i / 8 the curve is at control point i and
    # its tangent (per unit of segment parameter) is half the difference of
    # the neighbouring control points
    ctrl = synth.camera_path(100, 200, 300, seed=9)
    assert ((ctrl >= [15, 30, 45]) & (ctrl <= [85, 170, 255])).all()
    pos, tan = synth.camera_pose(ctrl, np.arange(8) / 8.0)
    np.testing.assert_allclose(pos, ctrl, atol=1e-9)
    # tangent at a control point: half the difference of its neighbours
    np.testing.assert_allclose(tan, 0.5 * (np.roll(ctrl, -1, 0) - np.roll(ctrl, 1, 0)), atol=1e-9)
