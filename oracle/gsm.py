"""FP64 CPU oracle of the GSM linear system, Eq.(4) of arXiv 1501.01752.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product library.

Conventions (stated here so that a reader can check them against the paper):

* Voxel permittivities ``eps`` have shape (Vz, Vy, Vx) (x fastest); voxel
  (ix, iy, iz) occupies the box [ix, ix+1) x [iy, iy+1) x [iz, iz+1) in units of
  Lambda_a / V_a.  Per-axis parameters are given in (x, y, z) order.
* Harmonics m = (mx, my, mz) with |m_a| <= M_a (the truncation to N_a
  harmonics per axis of the section on truncation, with N_a = 2 M_a + 1).
  Field arrays have shape (3, 2Mz+1, 2My+1, 2Mx+1): component, then m with
  offsets M_a.  Flattened unknown vectors use the same order.
* All wave-vectors are normalised by k0 = 2 pi / lambda:
  q_m = k_inc / k0 + (mx lambda/Lx, my lambda/Ly, mz lambda/Lz)
  (Bloch wave-vectors k_am = k_a^inc + m_a K_a, K_a = 2 pi / Lambda_a,
  defined right after Eq.(4)).
* Fourier coefficients of permittivity have shape (2Nz+1, 2Ny+1, 2Nx+1),
  index n + N_a; c_n = (1/|cell|) * integral over the cell of
  eps(r) exp(-i G_n . r).
"""
import os

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse.linalg

# FFTs of the FFT route run on the host threads this process may use (the
# same DFT as numpy's; only the rounding order can differ): OMP_NUM_THREADS
# when set, else the CPU affinity
def _fft_workers():
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    if hasattr(os, "sched_getaffinity"):
        return max(1, len(os.sched_getaffinity(0)))
    return os.cpu_count() or 1


FFT_WORKERS = _fft_workers()


# ---------------------------------------------------------------- geometry --

def _axis_box_factor(n_max, v):
    """F[n, j] = (1/Lambda) * integral over voxel j of exp(-2 pi i n x / Lambda).

    In the unit coordinate u = x / Lambda the voxel j is [j/v, (j+1)/v), so the
    integral of exp(-2 pi i n u) du is 1/v for n = 0 and
    (exp(-2 pi i n (j+1)/v) - exp(-2 pi i n j/v)) / (-2 pi i n) otherwise.
    """
    n = np.arange(-n_max, n_max + 1, dtype=np.float64)[:, None]
    j = np.arange(v, dtype=np.float64)[None, :]
    out = np.empty((n.shape[0], v), dtype=np.complex128)
    nz = n[:, 0] != 0
    nn = n[nz]
    out[nz] = (np.exp(-2j * np.pi * nn * (j + 1) / v)
               - np.exp(-2j * np.pi * nn * j / v)) / (-2j * np.pi * nn)
    out[~nz] = 1.0 / v
    return out


def box_image(eps, n_max):
    """Exact Fourier coefficients of a piecewise-constant voxel body.

    The paper prefers exact Fourier images of the permittivity to samples on a
    mesh (the "Calculation details" section and the remark below Eq.(4) on the
    Toeplitz matrix).  For a voxel body the exact image is the sum over voxels
    of eps_v times the integral of exp(-i G_n . r) over the voxel box, divided
    by the cell volume; the box integral factorises over axes.

    eps   : (Vz, Vy, Vx) real array.
    n_max : (Nx, Ny, Nz), largest |n_a| kept.
    Returns c with shape (2Nz+1, 2Ny+1, 2Nx+1), c[nz+Nz, ny+Ny, nx+Nx].
    """
    eps = np.asarray(eps, dtype=np.float64)
    vz, vy, vx = eps.shape
    fx = _axis_box_factor(n_max[0], vx)
    fy = _axis_box_factor(n_max[1], vy)
    fz = _axis_box_factor(n_max[2], vz)
    return np.einsum('zyx,az,by,cx->abc', eps, fz, fy, fx, optimize=True)


# ------------------------------------------------------------- harmonics ----

def harmonic_q(k_inc, wavelength, period, M):
    """Normalised Bloch wave-vectors q_m = k_m / k0, shape (N1z, N1y, N1x, 3).

    k_am = k_a^inc + m_a K_a with K_a = 2 pi / Lambda_a (text after Eq.(4)).
    """
    k0 = 2.0 * np.pi / wavelength
    q0 = np.asarray(k_inc, dtype=np.float64) / k0
    b = wavelength / np.asarray(period, dtype=np.float64)
    mx = np.arange(-M[0], M[0] + 1)
    my = np.arange(-M[1], M[1] + 1)
    mz = np.arange(-M[2], M[2] + 1)
    q = np.empty((mz.size, my.size, mx.size, 3))
    q[..., 0] = q0[0] + mx[None, None, :] * b[0]
    q[..., 1] = q0[1] + my[None, :, None] * b[1]
    q[..., 2] = q0[2] + mz[:, None, None] * b[2]
    return q


def green_tensor(q, eps_b):
    """Per-harmonic Green factor of Eq.(4), normalised by k0^2.

    (k_b^2 delta_ab - k_am k_bm) / (k_m^2 - k_b^2) with k_b^2 = k0^2 eps_b
    becomes (eps_b I - q q^T) / (|q|^2 - eps_b).
    """
    q = np.asarray(q, dtype=np.float64)
    q2 = np.sum(q * q, axis=-1)
    eye = np.eye(3)
    num = eps_b * eye - q[..., :, None] * q[..., None, :]
    return num / (q2 - eps_b)[..., None, None]


def singular_margin(q, eps_b):
    """min over m of | |q_m|^2 - eps_b |: Eq.(4) requires k_m^2 != k_b^2."""
    q2 = np.sum(np.asarray(q) ** 2, axis=-1)
    return float(np.min(np.abs(q2 - eps_b)))


# ------------------------------------------------------- dense route (O1) ---

def _flat_orders(M):
    mx = np.arange(-M[0], M[0] + 1)
    my = np.arange(-M[1], M[1] + 1)
    mz = np.arange(-M[2], M[2] + 1)
    gz, gy, gx = np.meshgrid(mz, my, mx, indexing='ij')
    return gx.ravel(), gy.ravel(), gz.ravel()


def toeplitz(c, M):
    """T[m, m'] = c_{m - m'} over the truncated harmonic set (flattened)."""
    nz0 = (c.shape[0] - 1) // 2
    ny0 = (c.shape[1] - 1) // 2
    nx0 = (c.shape[2] - 1) // 2
    assert nx0 >= 2 * M[0] and ny0 >= 2 * M[1] and nz0 >= 2 * M[2]
    mx, my, mz = _flat_orders(M)
    dx = mx[:, None] - mx[None, :]
    dy = my[:, None] - my[None, :]
    dz = mz[:, None] - mz[None, :]
    return c[dz + nz0, dy + ny0, dx + nx0]


def zero_index(M):
    """Flat index of the harmonic m = 0."""
    return (M[2] * (2 * M[1] + 1) + M[1]) * (2 * M[0] + 1) + M[0]


def assemble_dense(c, M, q, eps_b):
    """Dense matrix A of Eq.(4) written as A E = E_inc.

    E_am - sum_b G_ab(q_m) sum_m' (Delta eps / eps_b)_{m-m'} E_bm' = E^inc_am,
    with (Delta eps / eps_b)_n = c_n / eps_b - delta_n0 for a homogeneous basis
    medium eps_b.  Unknowns ordered (component, m).
    """
    T = toeplitz(c, M)
    n = T.shape[0]
    Vm = T / eps_b - np.eye(n)
    G = green_tensor(q, eps_b).reshape(n, 3, 3)
    A = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            A[a * n:(a + 1) * n, b * n:(b + 1) * n] = -G[:, a, b][:, None] * Vm
    A += np.eye(3 * n)
    return A


def incident_rhs(M, a):
    """E^inc_am = delta_m0 a_a (plane-wave incident field, text after Eq.(4))."""
    n = (2 * M[0] + 1) * (2 * M[1] + 1) * (2 * M[2] + 1)
    b = np.zeros(3 * n, dtype=np.complex128)
    i0 = zero_index(M)
    for comp in range(3):
        b[comp * n + i0] = a[comp]
    return b


def solve_dense(c, M, q, eps_b, drives):
    """Route O1: LU solve of the dense truncated system, one column per drive.

    Returns E with shape (n_drive, 3, N1z, N1y, N1x).
    """
    A = assemble_dense(c, M, q, eps_b)
    B = np.stack([incident_rhs(M, a) for a in drives], axis=1)
    X = scipy.linalg.solve(A, B)
    shape = (3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    return np.stack([X[:, p].reshape(shape) for p in range(X.shape[1])])


# --------------------------------------------------------- FFT route (O2) ---

def contrast_convolution_fft(c, M, eps_b, x, P):
    """w_m = sum_m' (Delta eps / eps_b)_{m-m'} x_m' computed with FFTs.

    The Toeplitz product by FFT, the step the paper singles out as the most
    costly (section on the truncation):
    coefficients and field are placed on a P^3 grid at n mod P, taken to real
    space, multiplied point by point and taken back.  With P >= 4 M_a + 1 on
    every axis the cropped result equals the truncated Toeplitz product.
    x : (3, N1z, N1y, N1x).   P : (Px, Py, Pz).
    """
    Px, Py, Pz = P
    assert Px >= 4 * M[0] + 1 and Py >= 4 * M[1] + 1 and Pz >= 4 * M[2] + 1
    nz0 = (c.shape[0] - 1) // 2
    ny0 = (c.shape[1] - 1) // 2
    nx0 = (c.shape[2] - 1) // 2
    grid = np.zeros((Pz, Py, Px), dtype=np.complex128)
    for nz in range(-2 * M[2], 2 * M[2] + 1):
        for ny in range(-2 * M[1], 2 * M[1] + 1):
            nx = np.arange(-2 * M[0], 2 * M[0] + 1)
            grid[nz % Pz, ny % Py, nx % Px] = c[nz + nz0, ny + ny0, nx + nx0] / eps_b
    grid[0, 0, 0] -= 1.0
    g = scipy.fft.ifftn(grid, workers=FFT_WORKERS) * (Px * Py * Pz)
    mz = np.arange(-M[2], M[2] + 1) % Pz
    my = np.arange(-M[1], M[1] + 1) % Py
    mx = np.arange(-M[0], M[0] + 1) % Px
    X = np.zeros((3, Pz, Py, Px), dtype=np.complex128)
    X[:, mz[:, None, None], my[None, :, None], mx[None, None, :]] = x
    xr = scipy.fft.ifftn(X, axes=(1, 2, 3), workers=FFT_WORKERS) * (Px * Py * Pz)
    W = scipy.fft.fftn(xr * g[None], axes=(1, 2, 3), workers=FFT_WORKERS) / (Px * Py * Pz)
    return W[:, mz[:, None, None], my[None, :, None], mx[None, None, :]]


def apply_operator_fft(c, M, q, eps_b, x, P):
    """y = x - G(q_m) . w_m with w the FFT contrast convolution (Eq.(4))."""
    w = contrast_convolution_fft(c, M, eps_b, x, P)
    G = green_tensor(q, eps_b)                      # (N1z, N1y, N1x, 3, 3)
    gw = np.einsum('zyxab,bzyx->azyx', G, w)
    return x - gw


def solve_fft_gmres(c, M, q, eps_b, a, P, rtol=1e-12, restart=30, maxiter=2000,
                    x0=None):
    """Route O2: the same operator applied by FFT, solved by restarted GMRES.

    GMRES is the Krylov method the paper uses (section "Calculation details").
    Returns (E with shape (3, N1z, N1y, N1x), number of GMRES iterations).
    """
    shape = (3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    n = int(np.prod(shape))

    def mv(v):
        return apply_operator_fft(c, M, q, eps_b, v.reshape(shape), P).ravel()

    op = scipy.sparse.linalg.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    b = incident_rhs(M, a)
    count = [0]

    def cb(_):
        count[0] += 1

    x, info = scipy.sparse.linalg.gmres(
        op, b, x0=None if x0 is None else np.asarray(x0).ravel(), rtol=rtol,
        atol=0.0, restart=restart, maxiter=maxiter, callback=cb,
        callback_type='pr_norm')
    if info != 0:
        raise RuntimeError(f'oracle GMRES did not converge (info={info})')
    return x.reshape(shape), count[0]


def apply_operator_at(c, M, q, eps_b, x, orders):
    """(A x)_m of Eq.(4) at the listed output orders m = (mx, my, mz) only,
    each written out from the definition:
    (A x)_m = x_m - G(q_m) sum_m' (c_{m-m'}/eps_b - delta_mm') x_m'.
    One output costs a pass over all N inputs (for checks at sizes where the
    whole product would not fit the host's time).  x: (3, N1z, N1y, N1x).
    Returns (len(orders), 3)."""
    x = np.asarray(x, dtype=np.complex128)
    nz0 = (c.shape[0] - 1) // 2
    ny0 = (c.shape[1] - 1) // 2
    nx0 = (c.shape[2] - 1) // 2
    mzs = np.arange(-M[2], M[2] + 1)[:, None, None]
    mys = np.arange(-M[1], M[1] + 1)[None, :, None]
    mxs = np.arange(-M[0], M[0] + 1)[None, None, :]
    out = np.zeros((len(orders), 3), dtype=np.complex128)
    for k, (mx, my, mz) in enumerate(orders):
        cm = c[mz - mzs + nz0, my - mys + ny0, mx - mxs + nx0] / eps_b     # c_{m-m'}/eps_b over m'
        w = np.array([np.sum(cm * x[comp]) for comp in range(3)])
        w -= x[:, mz + M[2], my + M[1], mx + M[0]]                          # - delta_mm' x_m'
        G = green_tensor(q[mz + M[2], my + M[1], mx + M[0]], eps_b)
        out[k] = x[:, mz + M[2], my + M[1], mx + M[0]] - G @ w
    return out


def relative_residual(c, M, q, eps_b, a, E, P):
    """||b - A E||_2 / ||b||_2 over all 3N unknowns of Eq.(4)."""
    b = incident_rhs(M, a)
    r = b - apply_operator_fft(c, M, q, eps_b, E, P).ravel()
    return float(np.linalg.norm(r) / np.linalg.norm(b))


# ------------------------------------------------------- effective tensor ---

def displacement_zero_order(c, M, E):
    """(T(eps) E)_0 = sum_m' c_{-m'} E_m': zeroth Fourier order of eps E."""
    T0 = toeplitz(c, M)[zero_index(M)]
    return np.array([np.dot(T0, E[comp].ravel()) for comp in range(3)])


def eps_eff_from_fields(c, M, fields):
    """Field-averaged tensor eps_eff = D0 E0^-1 from three independent drives.

    fields : (3, 3, N1z, N1y, N1x), one solved field per drive.
    D0 and E0 hold the zeroth Fourier orders of eps E and of E as columns.
    """
    i0 = zero_index(M)
    E0 = np.stack([f.reshape(3, -1)[:, i0] for f in fields], axis=1)
    D0 = np.stack([displacement_zero_order(c, M, f) for f in fields], axis=1)
    return D0 @ np.linalg.inv(E0)


def operator_L(c, M, q):
    """L = K(q_m) - T(eps) with K(q) = |q|^2 I - q q^T (units of k0^2).

    Multiplying Eq.(4) by the inverse Green factor gives L E = delta_m0 s:
    the Fourier form of curl curl E - k0^2 eps E = source.
    """
    T = toeplitz(c, M)
    n = T.shape[0]
    qf = q.reshape(n, 3)
    K = np.sum(qf * qf, axis=1)[:, None, None] * np.eye(3) - qf[:, :, None] * qf[:, None, :]
    L = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    for a in range(3):
        L[a * n:(a + 1) * n, a * n:(a + 1) * n] -= T
        for b in range(3):
            L[a * n + np.arange(n), b * n + np.arange(n)] += K[:, a, b]
    return L


def eps_eff_schur(c, M, q):
    """eps_eff = c_0 I + T_0r (K_r - T_rr)^-1 T_r0 (elimination of m != 0).

    Eliminating every harmonic but the zeroth from L E = delta_m0 s leaves
    (K_0 - eps_eff) E_0 = s with this eps_eff; it depends neither on eps_b nor
    on the drive.
    """
    L = operator_L(c, M, q)
    n = L.shape[0] // 3
    i0 = zero_index(M)
    zero = np.array([a * n + i0 for a in range(3)])
    rest = np.setdiff1d(np.arange(3 * n), zero)
    L_0r = L[np.ix_(zero, rest)]
    L_r0 = L[np.ix_(rest, zero)]
    L_rr = L[np.ix_(rest, rest)]
    c0 = c[(c.shape[0] - 1) // 2, (c.shape[1] - 1) // 2, (c.shape[2] - 1) // 2]
    return c0 * np.eye(3) + L_0r @ np.linalg.solve(L_rr, L_r0)


# ------------------------------------------------------- 1D stack (z only) --

def solve_stack_1d(c1d, Mz, q0, bz, eps_b, a):
    """Eq.(4) restricted to the harmonics (0, 0, mz) of a z-layered body.

    When c_n vanishes unless nx = ny = 0 the Toeplitz matrix couples only
    harmonics with equal (mx, my); the Green factor is diagonal in m; the
    incident field lives at m = 0.  So the solution lives on (0, 0, mz).
    c1d : coefficients c_(0,0,n) for n in [-2Mz, 2Mz].   bz = lambda / Lz.
    Returns e with shape (3, 2Mz+1).
    """
    mz = np.arange(-Mz, Mz + 1)
    n = mz.size
    T = c1d[(mz[:, None] - mz[None, :]) + 2 * Mz]
    q = np.zeros((n, 3))
    q[:, :] = q0
    q[:, 2] += mz * bz
    G = green_tensor(q, eps_b)
    Vm = T / eps_b - np.eye(n)
    A = np.eye(3 * n, dtype=np.complex128)
    for i in range(3):
        for j in range(3):
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] -= G[:, i, j][:, None] * Vm
    b = np.zeros(3 * n, dtype=np.complex128)
    b[np.arange(3) * n + Mz] = a
    return np.linalg.solve(A, b).reshape(3, n)
