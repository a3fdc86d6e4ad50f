"""FP64 CPU oracle of analytic Fourier images of permittivity bodies.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product library.

The paper prefers exact Fourier images of simple shapes (spheres and
polyhedra, combined to build a structure) to samples of the permittivity on
a mesh ("Calculation details"; also the remark below Eq.(4) that no transform
to coordinate space is made).  For a host of permittivity eps_h holding
inclusions i of permittivity eps_i that overlap neither each other nor their
own periodic images,

    eps(r) = eps_h + sum_i (eps_i - eps_h) chi_i(r),
    c_n    = (1/|cell|) integral_cell eps(r) exp(-i G_n . r) dr
           = eps_h delta_n0 + sum_i (eps_i - eps_h) S_i(G_n),
    S_i(G) = (1/|cell|) integral_{body i} exp(-i G . r) dr,

with G_n = 2 pi (n_x/Lambda_x, n_y/Lambda_y, n_z/Lambda_z).  The shape
factors S are the textbook integrals:

* ball of radius R centred at r0: (4 pi R^3 / 3|cell|) * 3 j1(u)/u *
  exp(-i G . r0), u = |G| R (j1 the spherical Bessel function of order 1);
* axis-aligned ellipsoid with semi-axes (a, b, c): the ball's formula with
  volume 4 pi a b c / 3 and u = |(a G_x, b G_y, c G_z)| (the affine image of
  the unit ball);
* axis-aligned box with half-sides (a, b, c): (8 a b c / |cell|) *
  sinc(a G_x) sinc(b G_y) sinc(c G_z) * exp(-i G . r0), sinc(x) = sin(x)/x.

The same formulas with 1/eps in place of eps give the coefficients of the
inverse permittivity that the H-field formulation, Eq.(5), uses.

Shapes are dicts {"kind": "sphere" | "ellipsoid" | "box", "centre": (x, y, z),
"size": radius | semi-axes | half-sides, "eps": value}.  Coefficient arrays
have shape (2Nz+1, 2Ny+1, 2Nx+1), index n + N_a, like box_image in gsm.py.
"""
import numpy as np
import scipy.special


def reciprocal_vectors(period, n_max):
    """G_n on the grid |n_a| <= N_a: arrays gx, gy, gz broadcastable to
    (2Nz+1, 2Ny+1, 2Nx+1)."""
    lx, ly, lz = (float(p) for p in period)
    nx = np.arange(-n_max[0], n_max[0] + 1, dtype=np.float64)
    ny = np.arange(-n_max[1], n_max[1] + 1, dtype=np.float64)
    nz = np.arange(-n_max[2], n_max[2] + 1, dtype=np.float64)
    gx = (2 * np.pi * nx / lx)[None, None, :]
    gy = (2 * np.pi * ny / ly)[None, :, None]
    gz = (2 * np.pi * nz / lz)[:, None, None]
    return gx, gy, gz


def _ball_factor(u):
    """3 j1(u) / u, equal to 1 at u = 0 (scipy's spherical Bessel function)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.ones_like(u)
    nz = u > 0
    out[nz] = 3.0 * scipy.special.spherical_jn(1, u[nz]) / u[nz]
    return out


def _sinc(x):
    """sin(x)/x with the value 1 at 0 (numpy's sinc is sin(pi x)/(pi x))."""
    return np.sinc(np.asarray(x, dtype=np.float64) / np.pi)


def shape_factor(shape, period, n_max):
    """S(G_n) of one shape (see the module docstring)."""
    gx, gy, gz = reciprocal_vectors(period, n_max)
    cell = float(np.prod(np.asarray(period, dtype=np.float64)))
    r0 = np.asarray(shape["centre"], dtype=np.float64)
    phase = np.exp(-1j * (gx * r0[0] + gy * r0[1] + gz * r0[2]))
    kind = shape["kind"]
    if kind == "sphere":
        a = b = c = float(shape["size"] if np.ndim(shape["size"]) == 0 else shape["size"][0])
    else:
        a, b, c = (float(s) for s in shape["size"])
    if kind in ("sphere", "ellipsoid"):
        vol = 4.0 * np.pi * a * b * c / 3.0
        u = np.sqrt((a * gx) ** 2 + (b * gy) ** 2 + (c * gz) ** 2)
        return vol / cell * _ball_factor(u) * phase
    if kind == "box":
        vol = 8.0 * a * b * c
        return vol / cell * _sinc(a * gx) * _sinc(b * gy) * _sinc(c * gz) * phase
    raise ValueError(f"unknown shape kind {kind!r}")


def shape_image(period, eps_host, shapes, n_max, inverse=False):
    """c_n of a host with non-overlapping inclusions, |n_a| <= N_a.

    inverse=True gives the coefficients of 1/eps instead (Eq.(5)'s
    inverse-permittivity matrix, found "just in the same way", as the paper's
    "Calculation details" puts it)."""
    f = (lambda e: 1.0 / float(e)) if inverse else (lambda e: float(e))
    shape_ = (2 * n_max[2] + 1, 2 * n_max[1] + 1, 2 * n_max[0] + 1)
    c = np.zeros(shape_, dtype=np.complex128)
    c[n_max[2], n_max[1], n_max[0]] = f(eps_host)
    for s in shapes:
        c += (f(s["eps"]) - f(eps_host)) * shape_factor(s, period, n_max)
    return c


def volume_fraction(period, shapes):
    """Sum of the inclusions' volumes over the cell volume."""
    cell = float(np.prod(np.asarray(period, dtype=np.float64)))
    tot = 0.0
    for s in shapes:
        if s["kind"] == "sphere":
            r = float(s["size"] if np.ndim(s["size"]) == 0 else s["size"][0])
            tot += 4.0 * np.pi * r ** 3 / 3.0
        elif s["kind"] == "ellipsoid":
            tot += 4.0 * np.pi * float(np.prod(s["size"])) / 3.0
        else:
            tot += 8.0 * float(np.prod(s["size"]))
    return tot / cell
