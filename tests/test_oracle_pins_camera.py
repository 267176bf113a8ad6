"""Pins of the FP64 oracle's differentiable camera (section 3.4: rays from a
pinhole through the pixel centres, the closest intersection in front of the
projection plane, bilinear texture sampling so that the image has non-zero
derivatives with respect to the state).

Each expected value comes from geometry or a construction, never from the
renderer itself:

* a texture that is a linear function of the texel coordinates is
  reproduced exactly by bilinear sampling, so a pixel's colour reads back
  the texel coordinates of its hit point: the ground point below a camera
  looking straight down, and the point of a sphere nearest a camera on its
  axis (l = -e_x of the body frame), also with the body turned
* the nearer of two spheres on one ray is seen; a sphere between the camera
  and the projection plane is not; a ray that hits nothing is 0
* the colour of the sphere's nearest point changes with the body's rotation
  as the linear texture says, and not with its position along the ray
* the reverse-mode gradient of sum(w * image) with respect to the bodies'
  positions and rotations equals central differences (pixels away from the
  silhouettes, where the hit object does not change)
"""
import numpy as np
import pytest

from oracle import Camera, Oracle
from paper_1611_01652_amd import workloads as W

NX, NY = 33, 17
ALPHA, BETA, GAMMA = 0.01, 0.02, 0.1


def _linear_texture(nx=NX, ny=NY):
    a, b = np.meshgrid(np.arange(nx), np.arange(ny))
    return ALPHA * a + BETA * b + GAMMA


def _cam(pos, axes, focal=1.0, pitch=0.01, width=9, height=5):
    c = Camera()
    c.pos[:] = list(pos)
    c.axes[:] = list(np.asarray(axes, np.float64).reshape(9))
    c.focal, c.pitch, c.width, c.height = focal, pitch, width, height
    return c


def _scene(centres, radii, rotations=None, ground=False):
    w = W.free_spheres(np.asarray(centres, np.float64), radii, [1.0] * len(radii), ground=ground)
    if rotations is not None:
        for k, R in enumerate(rotations):
            w.x0[k, 3:12] = np.asarray(R, np.float64).reshape(9)
    return w


LOOK_X = [[0, -1, 0], [0, 0, 1], [1, 0, 0]]   # right, up, optical axis: looking along +x


def test_ground_point_below_a_camera_looking_down():
    # camera at height 2 looking down (-z), right = +x, up = +y: pixel (i, j)
    # sees the ground at 2 (u, v) / f with (u, v) its offset on the plane
    cam = _cam((0.3, 0.4, 2.0), [[1, 0, 0], [0, 1, 0], [0, 0, -1]], focal=1.0, pitch=0.05, width=7, height=5)
    w = _scene([[50.0, 50.0, 5.0]], [0.1], ground=True)   # a sphere far out of view
    img = Oracle(w).render(cam, _linear_texture(), _linear_texture(), cell=0.1)
    for j in range(5):
        for i in range(7):
            u, v = (i + 0.5 - 3.5) * 0.05, (2.5 - j - 0.5) * 0.05
            hx, hy = 0.3 + 2.0 * u, 0.4 + 2.0 * v
            assert img[0, j, i] == pytest.approx(ALPHA * hx / 0.1 + BETA * hy / 0.1 + GAMMA, abs=1e-12)


@pytest.mark.parametrize("turn", [0.0, 0.4, -1.1])
def test_nearest_point_of_a_sphere_on_the_axis(turn):
    # the centre pixel (odd image) looks along +x at a sphere centred on the
    # axis: it hits the point nearest the camera, h - c = -r e_x (world); in
    # the body frame l = R^T (-e_x), read through the linear texture
    R = W._rot((0, 0, 1), turn)
    w = _scene([[3.0, 0.0, 0.0]], [1.0], rotations=[R])
    cam = _cam((0, 0, 0), LOOK_X, width=9, height=5)
    img = Oracle(w).render(cam, _linear_texture(), _linear_texture(), cell=1.0)
    l = R.T @ np.array([-1.0, 0.0, 0.0])
    u, v = (l[0] + 1) * (NX - 1) / 2, (l[1] + 1) * (NY - 1) / 2
    assert img[0, 2, 4] == pytest.approx(ALPHA * u + BETA * v + GAMMA, abs=1e-12)


def test_occlusion_and_the_projection_plane():
    # two spheres on the optical axis, turned differently: the nearer one is
    # seen.  With the projection plane pushed beyond the nearer sphere, the
    # farther one is seen.  Off both spheres the rays hit nothing.
    Ra, Rb = W._rot((0, 0, 1), 0.5), W._rot((0, 0, 1), -0.7)
    w = _scene([[3.0, 0.0, 0.0], [6.0, 0.0, 0.0]], [0.5, 0.5], rotations=[Ra, Rb])
    tex = _linear_texture()

    def expect(R):
        l = R.T @ np.array([-1.0, 0.0, 0.0])
        return ALPHA * (l[0] + 1) * (NX - 1) / 2 + BETA * (l[1] + 1) * (NY - 1) / 2 + GAMMA

    img = Oracle(w).render(_cam((0, 0, 0), LOOK_X, focal=1.0, pitch=0.2), tex, tex, cell=1.0)
    assert img[0, 2, 4] == pytest.approx(expect(Ra), abs=1e-12)
    assert img[0, 0, 0] == 0.0   # (the corner ray passes 0.57 m beside the first sphere's centre)
    img = Oracle(w).render(_cam((0, 0, 0), LOOK_X, focal=4.0, pitch=0.2), tex, tex, cell=1.0)
    assert img[0, 2, 4] == pytest.approx(expect(Rb), abs=1e-12)


def test_nearest_point_colour_follows_rotation_not_axial_position():
    R = W._rot((0, 0, 1), 0.3)
    tex = _linear_texture()
    cols = []
    for x in (2.0, 3.0, 5.0):
        w = _scene([[x, 0.0, 0.0]], [1.0], rotations=[R])
        cols.append(Oracle(w).render(_cam((0, 0, 0), LOOK_X), tex, tex, cell=1.0)[0, 2, 4])
    assert cols[0] == pytest.approx(cols[1], abs=1e-12) and cols[1] == pytest.approx(cols[2], abs=1e-12)
    # its derivatives.  In R (row-major in x[3:12]): l_x = sum_k R_k0 q_k / r
    # and l_y = sum_k R_k1 q_k / r with q = -r e_x, so only R_00 and R_01
    # count, by -alpha (NX - 1) / 2 and -beta (NY - 1) / 2.  In the position:
    # along the ray, nothing; sideways by d, the hit moves to q = (-sqrt(r^2 -
    # d^2), -d, 0), so dl/dp_y = R^T (0, -1, 0) and dl/dp_z = R^T (0, 0, -1)
    w = _scene([[3.0, 0.0, 0.0]], [1.0], rotations=[R])
    wts = np.zeros((1, 5, 9))
    wts[0, 2, 4] = 1.0
    g = Oracle(w).render_grad(_cam((0, 0, 0), LOOK_X), tex, tex, 1.0, wts)
    ku, kv = ALPHA * (NX - 1) / 2, BETA * (NY - 1) / 2
    want = np.zeros(18)
    want[1] = -ku * R[1, 0] - kv * R[1, 1]
    want[2] = -ku * R[2, 0] - kv * R[2, 1]
    want[3], want[4] = -ku, -kv
    np.testing.assert_allclose(g[0], want, atol=1e-12)


def _fd(o, cam, ts, tg, cell, wts, x, b, k, h=1e-6):
    xp, xm = x.copy(), x.copy()
    xp[b, k] += h
    xm[b, k] -= h
    return ((o.render(cam, ts, tg, cell, x=xp) * wts).sum() - (o.render(cam, ts, tg, cell, x=xm) * wts).sum()) / (2 * h)


def test_gradient_equals_central_differences():
    # two turned spheres over a textured ground, a camera looking at them from
    # an oblique angle; smooth synthetic textures; weights on the pixels whose
    # hit object is the same after moving any body by 1e-4
    Ra, Rb = W._rot((1, 2, 0.5), 0.8), W._rot((0.3, -1, 1), -0.6)
    w = _scene([[0.2, 0.1, 0.35], [-0.35, 0.3, 0.3]], [0.3, 0.25], rotations=[Ra, Rb], ground=True)
    c = W.pinhole_camera((0.4, -2.5, 1.2), (0.0, 0.1, 0.3), focal=1.0, pitch=1.0 / 40, width=36, height=24)
    cam = _cam(c["pos"], c["axes"], c["focal"], c["pitch"], c["width"], c["height"])
    ts, tg = W.synthetic_texture(24, 12, 1), W.synthetic_texture(16, 16, 2)
    o = Oracle(w)
    x = np.asarray(w.x0, np.float64)
    base = o.render(cam, ts, tg, 0.2)
    # hit classes: perturbing any coordinate by 1e-4 must not change a weighted pixel's object
    stable = np.ones(base.shape, bool)
    for b in range(2):
        for k in (0, 1, 2):
            for s in (-1e-4, 1e-4):
                xp = x.copy()
                xp[b, k] += s
                stable &= np.abs(o.render(cam, ts, tg, 0.2, x=xp) - base) < 1e-2
    rng = np.random.default_rng(5)
    wts = rng.normal(size=base.shape) * stable
    assert stable.sum() > 0.8 * stable.size and (base > 0).sum() > 0.9 * base.size
    g = o.render_grad(cam, ts, tg, 0.2, wts, x=x)
    for b in range(2):
        for k in list(range(12)):
            fd = _fd(o, cam, ts, tg, 0.2, wts, x, b, k)
            assert g[b, k] == pytest.approx(fd, rel=2e-5, abs=2e-6), (b, k, g[b, k], fd)
    assert np.abs(g[:, 12:]).max() == 0.0
