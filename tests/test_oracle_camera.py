"""Pin of the oracle's pinhole camera (ray generation, Section 3.6 / Algorithm 2) against the
geometry of a pinhole with a vertical field of view: the pixel at normalised device coordinates
(u, v) = (2 px / W - 1, 1 - 2 py / H) looks along a ray that makes the angle
atan(sqrt((u tan(fov/2) aspect)^2 + (v tan(fov/2))^2)) with the viewing axis, leans toward the
camera's right for u > 0 and toward its up vector for v > 0, and starts at the eye.  A camera
that used tan(fov) for tan(fov/2), swapped the aspect ratio or flipped an image axis fails."""
import math
import types

import numpy as np
import pytest


def _cam(eye, target, up, fov, w, h):
    return types.SimpleNamespace(eye=list(eye), target=list(target), up=list(up), fov_y_deg=fov,
                                 width=w, height=h)


def _frame(cam):
    f = np.subtract(cam.target, cam.eye).astype(float)
    f /= np.linalg.norm(f)
    r = np.cross(f, cam.up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return f, r, u


CAMERAS = [
    _cam((2.2, 0.5, 0.5), (0.5, 0.5, 0.5), (0, 0, 1), 40.0, 160, 90),
    _cam((-0.4, 1.9, 1.3), (0.45, 0.55, 0.5), (0, 0, 1), 40.0, 128, 128),
    _cam((0.5, -1.5, 0.9), (0.5, 0.5, 0.4), (0, 0, 1), 65.0, 90, 200),
]


@pytest.mark.parametrize("ci", range(len(CAMERAS)))
def test_pixel_angles_follow_the_pinhole_model(orc, ci):
    cam = CAMERAS[ci]
    f, r, u = _frame(cam)
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    aspect = cam.width / cam.height
    W, H = cam.width, cam.height
    # corners, edge midpoints, the centre and a few interior pixel centres
    pts = [(0, 0), (W, 0), (0, H), (W, H), (W / 2, 0), (W / 2, H), (0, H / 2), (W, H / 2),
           (W / 2, H / 2), (0.5, 0.5), (W - 0.5, 3.5), (W / 3 + 0.5, 2 * H / 3 + 0.5)]
    for px, py in pts:
        o, d = orc.camera_ray(cam, px, py)
        np.testing.assert_allclose(o, cam.eye, rtol=0, atol=1e-15)
        assert abs(np.linalg.norm(d) - 1.0) < 1e-14
        nu, nv = 2.0 * px / W - 1.0, 1.0 - 2.0 * py / H
        expect = math.atan(math.hypot(nu * th * aspect, nv * th))
        got = math.atan2(float(np.linalg.norm(np.cross(d, f))), float(np.dot(d, f)))
        assert got == pytest.approx(expect, abs=1e-12), (px, py)
        # orientation: right for u > 0, up for v > 0, in the proportion of the two offsets
        dr, du, df = float(np.dot(d, r)), float(np.dot(d, u)), float(np.dot(d, f))
        assert dr / df == pytest.approx(nu * th * aspect, abs=1e-12)
        assert du / df == pytest.approx(nv * th, abs=1e-12)


def test_vertical_and_horizontal_half_angles(orc):
    cam = CAMERAS[0]
    f, _, _ = _frame(cam)
    half = math.radians(cam.fov_y_deg) / 2.0
    _, top = orc.camera_ray(cam, cam.width / 2, 0)
    assert math.acos(float(np.dot(top, f))) == pytest.approx(half, abs=1e-12)
    _, side = orc.camera_ray(cam, 0, cam.height / 2)
    hh = math.atan(math.tan(half) * cam.width / cam.height)
    assert math.acos(float(np.dot(side, f))) == pytest.approx(hh, abs=1e-12)
    # the top row looks up (+z here), the left column to the camera's left
    assert top[2] > f[2]
    _, r, _ = _frame(cam)
    assert float(np.dot(side, r)) < 0.0
