"""Seeded synthetic inputs: voxel bodies, sweep points and drives.

This module holds input generation only (voxelisation of simple shapes,
seeded random draws); it contains none of the method's arithmetic and is the
one piece shared by the product path's tests/benchmark and the CPU oracle.

Units: lengths in units of the x period (Lambda_x = 1 unless stated);
voxel arrays have shape (Vz, Vy, Vx), x fastest; voxel (i, j, l) occupies
[i, i+1) x [j, j+1) x [l, l+1) in units of Lambda_a / V_a.  Inclusions are
centred at the middle of the cell.  Shapes are voxelised by sampling the
voxel centre, except axis-aligned slab boundaries, which are averaged by
partial volume (exact for a piecewise-constant stack).
"""
import numpy as np


def _centres(v, length):
    return (np.arange(v) + 0.5) * (length / v)


def ellipsoid(vox, period, semi_axes, eps_in, eps_out=1.0):
    """Ellipsoid centred in the cell, voxel-centre sampled.

    vox = (Vx, Vy, Vz); period = (Lx, Ly, Lz); semi_axes = (ax, ay, az).
    """
    vx, vy, vz = vox
    x = _centres(vx, period[0]) - 0.5 * period[0]
    y = _centres(vy, period[1]) - 0.5 * period[1]
    z = _centres(vz, period[2]) - 0.5 * period[2]
    r2 = ((z[:, None, None] / semi_axes[2]) ** 2 + (y[None, :, None] / semi_axes[1]) ** 2
          + (x[None, None, :] / semi_axes[0]) ** 2)
    eps = np.full((vz, vy, vx), float(eps_out))
    eps[r2 <= 1.0] = float(eps_in)
    return eps


def sphere(v, radius, eps_in, eps_out=1.0, period=1.0):
    """Sphere of the given radius centred in a cubic cell of V^3 voxels."""
    return ellipsoid((v, v, v), (period,) * 3, (radius,) * 3, eps_in, eps_out)


def layered_stack(vz, fill, eps1, eps2, vxy=1):
    """Two-layer stack along z: eps1 for z < fill * Lz, eps2 above.

    The voxel cut by the interface gets the partial-volume average, so the
    voxel body is the exact piecewise-constant stack when fill * Vz is an
    integer and its closest voxel model otherwise.  Shape (vz, vxy, vxy).
    """
    z0 = np.arange(vz) / vz
    z1 = (np.arange(vz) + 1) / vz
    frac1 = np.clip((fill - z0) / (z1 - z0), 0.0, 1.0)
    col = frac1 * eps1 + (1.0 - frac1) * eps2
    return np.broadcast_to(col[:, None, None], (vz, vxy, vxy)).copy()


def woodpile(v=128, eps_rod=10.0, eps_bg=1.0):
    """Four-layer woodpile, rods of width and height Lambda/4.

    Layer l occupies z in [l/4, (l+1)/4); layer 0 rods run along x at
    y in [1/8, 3/8), layer 1 along y at x in [1/8, 3/8), layer 2 along x at
    y in [5/8, 7/8), layer 3 along y at x in [5/8, 7/8).  With v a multiple
    of 8 every edge falls on a voxel face, so the voxel body is exact.
    """
    assert v % 8 == 0
    e = np.full((v, v, v), float(eps_bg))
    q = v // 4
    lo, hi = v // 8, 3 * v // 8
    lo2, hi2 = 5 * v // 8, 7 * v // 8
    e[0 * q:1 * q, lo:hi, :] = eps_rod
    e[1 * q:2 * q, :, lo:hi] = eps_rod
    e[2 * q:3 * q, lo2:hi2, :] = eps_rod
    e[3 * q:4 * q, :, lo2:hi2] = eps_rod
    return e


def _periodic_gaussian_smooth(field, sigma):
    v = field.shape[0]
    d = np.minimum(np.abs(np.arange(v)), v - np.abs(np.arange(v)))
    g1 = np.exp(-0.5 * (d / sigma) ** 2)
    g1 /= g1.sum()
    ker = g1[:, None, None] * g1[None, :, None] * g1[None, None, :]
    return np.real(np.fft.ifftn(np.fft.fftn(field) * np.fft.fftn(ker)))


def smooth_random_field(v=32, seed=4, sigma=3.0, lo=1.0, hi=10.0, stretch=True):
    """Gaussian-smoothed seeded uniform random field on a periodic V^3 grid.

    stretch=True: s = smooth(U[0,1]); eps = clip(mid + half * (s - mean) /
    max|s - mean|, lo, hi), which spans [lo, hi].  stretch=False: the literal
    clip(smooth(U[lo, hi]), lo, hi), which smoothing leaves nearly uniform.
    """
    rng = np.random.default_rng(seed)
    if stretch:
        s = _periodic_gaussian_smooth(rng.uniform(0.0, 1.0, (v, v, v)), sigma)
        d = s - s.mean()
        mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        return np.clip(mid + half * d / np.max(np.abs(d)), lo, hi)
    s = _periodic_gaussian_smooth(rng.uniform(lo, hi, (v, v, v)), sigma)
    return np.clip(s, lo, hi)


def transverse_drive(khat):
    """Unit polarisation normalise(z x khat); x when khat is along z."""
    khat = np.asarray(khat, dtype=np.float64)
    a = np.cross([0.0, 0.0, 1.0], khat)
    n = np.linalg.norm(a)
    if n < 1e-12:
        return np.array([1.0, 0.0, 0.0])
    return a / n


def random_directions(n, seed):
    """n unit vectors uniform on the sphere (normalised Gaussian draws)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def orthorhombic_sweep(n=256, seed=3, r_lo=0.2, r_hi=0.45, m_lo=6, m_hi=16):
    """Sweep points of the uneven batched workload.

    Draw order from one PCG64 stream: Lambda_x / lambda ~ U[r_lo, r_hi],
    Gaussian direction draws, order counts M ~ U{m_lo..m_hi}.
    Returns (wavelength[n], khat[n, 3], M[n]).
    """
    rng = np.random.default_rng(seed)
    r = rng.uniform(r_lo, r_hi, n)
    g = rng.standard_normal((n, 3))
    m = rng.integers(m_lo, m_hi + 1, n)
    return 1.0 / r, g / np.linalg.norm(g, axis=1, keepdims=True), m


# ------------------------------------------------------------- workloads ----

def sphere_lattice_small():
    """Cubic lattice Lambda = 0.3 lambda, sphere r = 0.3 Lambda, eps 4 in vacuum,
    16^3 voxels, M = 3, normal incidence along z, x polarisation."""
    return dict(eps=sphere(16, 0.3, 4.0), period=(1.0, 1.0, 1.0), wavelength=1.0 / 0.3,
                k_hat=(0.0, 0.0, 1.0), M=(3, 3, 3), drives=[(1.0, 0.0, 0.0)])


def sphere_lattice_m15():
    """The same sphere lattice on 64^3 voxels at M = 15 (31^3 harmonics)."""
    return dict(eps=sphere(64, 0.3, 4.0), period=(1.0, 1.0, 1.0), wavelength=1.0 / 0.3,
                k_hat=(0.0, 0.0, 1.0), M=(15, 15, 15),
                drives=[(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)])


def sphere_lattice_table1(M):
    """Table 1's workload: a cubic lattice of spheres of refractive index 3
    (eps 9) in air.  The paper states neither the radius nor the period;
    taken here as r = 0.3 Lambda and Lambda = 0.3 lambda, on 64^3 voxels;
    normal incidence along z, x polarisation, M orders per axis (2M + 1
    harmonics: 15, 31, 63 stand for the table's 16, 32, 64)."""
    return dict(eps=sphere(64, 0.3, 9.0), period=(1.0, 1.0, 1.0), wavelength=1.0 / 0.3,
                k_hat=(0.0, 0.0, 1.0), M=(M, M, M), drives=[(1.0, 0.0, 0.0)])


def layered_stack_m15():
    """Stack f = 0.4, eps1 = 2.25, eps2 = 9 along z on 64 voxels, M = 15."""
    return dict(eps=layered_stack(64, 0.4, 2.25, 9.0), period=(1.0, 1.0, 1.0),
                wavelength=1.0 / 0.3, k_hat=(0.0, 0.0, 1.0), M=(15, 15, 15),
                drives=[(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)])
