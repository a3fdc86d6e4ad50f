"""Checks that tie the analytic-image oracle (oracle/shapes.py) to facts
outside itself: direct quadrature of the defining integral over the body,
the exact voxel image of a box that the voxel grid resolves, convergence of
voxelised balls, and the volume fraction.  Each function returns a
non-negative error; ALL maps a name to (function, bound).  The mutation tests
plant mistakes in the oracle and require one of these to fail."""
import numpy as np

from oracle import gsm as O
from oracle import shapes as S


def _ball_integral_quadrature(G, centre, axes, n=48):
    """(integral over the ellipsoid {sum ((r-r0)_a / axes_a)^2 <= 1} of
    exp(-i G . r) dr) by Gauss-Legendre in radius and cos(theta) and the
    trapezoid rule in phi (exact for the periodic phi integrand), written
    as an integral over the unit ball after r = r0 + diag(axes) s."""
    xr, wr = np.polynomial.legendre.leggauss(n)
    rr = 0.5 * (xr + 1.0)            # radius nodes on [0, 1]
    wr = 0.5 * wr
    xt, wt = np.polynomial.legendre.leggauss(n)   # cos(theta) on [-1, 1]
    phi = 2 * np.pi * np.arange(2 * n) / (2 * n)
    wp = 2 * np.pi / (2 * n)
    st = np.sqrt(1 - xt ** 2)
    sx = rr[:, None, None] * st[None, :, None] * np.cos(phi)[None, None, :]
    sy = rr[:, None, None] * st[None, :, None] * np.sin(phi)[None, None, :]
    sz = rr[:, None, None] * xt[None, :, None] * np.ones_like(phi)[None, None, :]
    w = (wr * rr ** 2)[:, None, None] * wt[None, :, None] * wp
    a = np.asarray(axes, float)
    arg = G[0] * a[0] * sx + G[1] * a[1] * sy + G[2] * a[2] * sz
    val = np.sum(w * np.exp(-1j * arg))
    return np.prod(a) * val * np.exp(-1j * np.dot(G, centre))


def _sample_ns(n_max, count, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(-m, m + 1)) for m in n_max) for _ in range(count)]


def err_sphere_quadrature():
    period = (1.0, 0.9, 1.2)
    sph = {"kind": "sphere", "centre": (0.45, 0.5, 0.62), "size": 0.31, "eps": 4.0}
    nmax = (5, 4, 6)
    c = S.shape_factor(sph, period, nmax)
    err = 0.0
    for n in _sample_ns(nmax, 16, 1) + [(0, 0, 0), (5, -4, 6)]:
        G = 2 * np.pi * np.array(n, float) / np.array(period)
        ref = _ball_integral_quadrature(G, np.array(sph["centre"]), (0.31,) * 3) / np.prod(period)
        got = c[n[2] + nmax[2], n[1] + nmax[1], n[0] + nmax[0]]
        err = max(err, abs(got - ref))
    return err


def err_ellipsoid_quadrature():
    period = (1.0, 0.8, 1.2)
    ell = {"kind": "ellipsoid", "centre": (0.5, 0.4, 0.6), "size": (0.35, 0.25, 0.15), "eps": 6.0}
    nmax = (6, 5, 4)
    c = S.shape_factor(ell, period, nmax)
    err = 0.0
    for n in _sample_ns(nmax, 16, 2) + [(0, 0, 0), (-6, 5, 4)]:
        G = 2 * np.pi * np.array(n, float) / np.array(period)
        ref = _ball_integral_quadrature(G, np.array(ell["centre"]), ell["size"]) / np.prod(period)
        got = c[n[2] + nmax[2], n[1] + nmax[1], n[0] + nmax[0]]
        err = max(err, abs(got - ref))
    return err


def _box_voxels(v, lo, hi, eps_in, eps_out):
    """Voxel body of an axis-aligned box whose faces lie on voxel faces
    (lo, hi in voxel units per axis, x first)."""
    e = np.full((v[2], v[1], v[0]), float(eps_out))
    e[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = eps_in
    return e


def err_box_matches_voxel_image():
    """A box whose faces are voxel faces is the voxel body itself: its
    analytic image equals the exact voxel image (box_image of gsm.py)."""
    period = (1.0, 1.3, 0.7)
    v = (8, 10, 4)
    lo, hi = (2, 1, 1), (5, 7, 3)
    vox = _box_voxels(v, lo, hi, 9.0, 2.25)
    centre = [0.5 * (lo[a] + hi[a]) / v[a] * period[a] for a in range(3)]
    half = [0.5 * (hi[a] - lo[a]) / v[a] * period[a] for a in range(3)]
    box = {"kind": "box", "centre": centre, "size": half, "eps": 9.0}
    nmax = (9, 7, 11)
    err = 0.0
    for inverse in (False, True):
        ref = O.box_image(1.0 / vox if inverse else vox, nmax)
        got = S.shape_image(period, 2.25, [box], nmax, inverse=inverse)
        err = max(err, np.abs(got - ref).max())
    return err


def err_two_boxes_sum():
    """Two disjoint boxes: the image of the union equals the voxel image."""
    period = (1.0, 1.0, 1.0)
    v = (8, 8, 8)
    vox = _box_voxels(v, (0, 0, 0), (2, 4, 8), 3.0, 1.5)
    vox[1:3, 5:8, 4:8] = 6.0
    shapes = [{"kind": "box", "centre": (0.125, 0.25, 0.5), "size": (0.125, 0.25, 0.5), "eps": 3.0},
              {"kind": "box", "centre": (0.75, 0.8125, 0.25), "size": (0.25, 0.1875, 0.125), "eps": 6.0}]
    nmax = (6, 6, 6)
    return float(np.abs(S.shape_image(period, 1.5, shapes, nmax) - O.box_image(vox, nmax)).max())


def err_sphere_voxel_convergence():
    """Centre-sampled voxel balls converge to the analytic ball image: the
    error at 96^3 voxels is below that at 24^3 by more than 2x and below
    1e-3 (the voxel surface error falls like 1/V)."""
    period = (1.0, 1.0, 1.0)
    nmax = (3, 3, 3)
    sph = {"kind": "sphere", "centre": (0.5, 0.5, 0.5), "size": 0.3, "eps": 4.0}
    ref = S.shape_image(period, 1.0, [sph], nmax)
    errs = []
    for v in (24, 96):
        u = (np.arange(v) + 0.5) / v - 0.5
        r2 = u[:, None, None] ** 2 + u[None, :, None] ** 2 + u[None, None, :] ** 2
        vox = np.where(r2 <= 0.09, 4.0, 1.0)
        errs.append(np.abs(O.box_image(vox, nmax) - ref).max())
    if not errs[1] < errs[0] / 2:
        return np.inf
    return errs[1]


def err_zero_order_is_mean():
    """c_0 = eps_h + sum (eps_i - eps_h) f_i with f_i the volume fractions
    of a ball (4 pi r^3 / 3) and a box (product of sides)."""
    period = (1.0, 1.1, 0.9)
    shapes = [{"kind": "sphere", "centre": (0.3, 0.3, 0.3), "size": 0.2, "eps": 5.0},
              {"kind": "box", "centre": (0.75, 0.8, 0.6), "size": (0.1, 0.2, 0.15), "eps": 2.0}]
    c = S.shape_image(period, 1.2, shapes, (1, 1, 1))
    cell = 1.0 * 1.1 * 0.9
    ref = 1.2 + (5.0 - 1.2) * (4 * np.pi * 0.2 ** 3 / 3) / cell + (2.0 - 1.2) * (0.2 * 0.4 * 0.3) / cell
    return abs(c[1, 1, 1] - ref)


ALL = {
    "sphere_quadrature": (err_sphere_quadrature, 1e-13),
    "ellipsoid_quadrature": (err_ellipsoid_quadrature, 1e-13),
    "box_equals_voxel_image": (err_box_matches_voxel_image, 1e-14),
    "two_boxes_union": (err_two_boxes_sum, 1e-14),
    "sphere_voxel_convergence": (err_sphere_voxel_convergence, 1e-3),
    "zero_order_mean": (err_zero_order_is_mean, 1e-15),
}
