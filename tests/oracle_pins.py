"""Checks that tie the CPU oracle to facts outside itself.

Each function returns a non-negative error; the tests compare it with a
bound, and the mutation tests plant plausible mistakes in the oracle and
require that at least one of these checks fails.  Nothing here re-types the
oracle's formulas: the references are closed forms, an exact ODE solution,
quadrature, the shift theorem, symmetry and the paper's printed scalars.
"""
import numpy as np

from oracle import gsm as O
from exact_stack_1d import ExactStack
from paper_1501_01752_amd import inputs


def _gauss_box_image(eps, n_max, order=30):
    """c_n by Gauss-Legendre quadrature over each voxel, loops in Python."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    vz, vy, vx = eps.shape
    out = np.zeros((2 * n_max[2] + 1, 2 * n_max[1] + 1, 2 * n_max[0] + 1), complex)
    ns = [np.arange(-n, n + 1) for n in n_max]
    for iz in range(vz):
        for iy in range(vy):
            for ix in range(vx):
                # nodes in unit coordinates inside the voxel
                ux = (ix + 0.5 + 0.5 * xg) / vx
                uy = (iy + 0.5 + 0.5 * xg) / vy
                uz = (iz + 0.5 + 0.5 * xg) / vz
                fx = (np.exp(-2j * np.pi * ns[0][:, None] * ux[None]) * wg).sum(1) * 0.5 / vx
                fy = (np.exp(-2j * np.pi * ns[1][:, None] * uy[None]) * wg).sum(1) * 0.5 / vy
                fz = (np.exp(-2j * np.pi * ns[2][:, None] * uz[None]) * wg).sum(1) * 0.5 / vz
                out += eps[iz, iy, ix] * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    return out


def err_box_image_quadrature(seed=0):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, 5.0, (2, 3, 3))
    nmax = (4, 3, 5)
    ref = _gauss_box_image(eps, nmax)
    return float(np.abs(O.box_image(eps, nmax) - ref).max())


def err_box_image_slab():
    """Voxel-aligned slab vs the exact step-function Fourier series."""
    vz, fill, e1, e2 = 16, 0.375, 2.0, 7.0
    eps = inputs.layered_stack(vz, fill, e1, e2)
    c = O.box_image(eps, (0, 0, 20))[:, 0, 0]
    n = np.arange(-20, 21)
    ref = np.empty(n.size, complex)
    nz = n != 0
    ref[nz] = (e1 - e2) * (1 - np.exp(-2j * np.pi * n[nz] * fill)) / (2j * np.pi * n[nz])
    ref[~nz] = fill * e1 + (1 - fill) * e2
    return float(np.abs(c - ref).max())


def err_box_image_shift():
    """Shift theorem: rolling the body by one voxel along x multiplies c_n by
    exp(-2 pi i n_x / V_x)."""
    eps = inputs.sphere(8, 0.3, 4.0)
    eps = eps * (1.0 + 0.1 * np.arange(8)[None, None, :])  # break symmetry
    c = O.box_image(eps, (3, 3, 3))
    c2 = O.box_image(np.roll(eps, 1, axis=2), (3, 3, 3))
    nx = np.arange(-3, 4)
    return float(np.abs(c2 - c * np.exp(-2j * np.pi * nx / 8)[None, None, :]).max())


def err_green_eigen():
    """G q = -q (longitudinal) and G t = eps_b t / (|q|^2 - eps_b) for t _|_ q."""
    rng = np.random.default_rng(1)
    q = rng.normal(size=(20, 3))
    eb = 2.7
    G = O.green_tensor(q, eb)
    e1 = np.abs(np.einsum('nab,nb->na', G, q) + q).max()
    t = np.cross(q, rng.normal(size=(20, 3)))
    lam_t = eb / (np.sum(q * q, 1) - eb)
    e2 = np.abs(np.einsum('nab,nb->na', G, t) - lam_t[:, None] * t).max()
    return float(max(e1, e2))


def _setup(eps, M, k_hat=(0.0, 0.0, 1.0), wavelength=1.0 / 0.3, period=(1.0, 1.0, 1.0),
           n_inc=1.0):
    k0 = 2 * np.pi / wavelength
    kinc = n_inc * k0 * np.asarray(k_hat, float)
    c = O.box_image(eps, tuple(2 * m for m in M))
    q = O.harmonic_q(kinc, wavelength, period, M)
    return c, q


def err_trivial_contrast():
    """Uniform eps equal to eps_b: E = E_inc exactly."""
    M = (2, 2, 2)
    eps = np.full((4, 4, 4), 2.0)
    c, q = _setup(eps, M)
    E = O.solve_dense(c, M, q, 2.0, [np.array([0.3, -0.5, 0.8])])[0]
    ref = O.incident_rhs(M, np.array([0.3, -0.5, 0.8])).reshape(E.shape)
    return float(np.abs(E - ref).max())


def err_homogeneous_closed_form(route='dense'):
    """Homogeneous eps_h != eps_b: only m = 0 is excited and
    E_0 = transverse(a) (|q|^2 - eps_b)/(|q|^2 - eps_h) + longitudinal(a) eps_b/eps_h."""
    M = (2, 2, 2)
    eh, eb = 3.1, 1.7
    eps = np.full((4, 4, 4), eh)
    khat = np.array([0.3, -0.2, 0.9])
    khat /= np.linalg.norm(khat)
    c, q = _setup(eps, M, k_hat=khat, n_inc=0.8)
    a = np.array([0.2 + 0.1j, 1.0, -0.4])
    if route == 'dense':
        E = O.solve_dense(c, M, q, eb, [a])[0]
    else:
        E, _ = O.solve_fft_gmres(c, M, q, eb, a, (9, 9, 9), rtol=1e-14)
    q0 = q[M[2], M[1], M[0]]
    u = q0 / np.linalg.norm(q0)
    al = u * np.dot(u, a)
    at = a - al
    qq = np.dot(q0, q0)
    e0 = at * (qq - eb) / (qq - eh) + al * eb / eh
    ref = np.zeros_like(E)
    ref[:, M[2], M[1], M[0]] = e0
    return float(np.abs(E - ref).max())


def err_stack_exact(Mz=40, route='1d'):
    """Layered stack, k || z, transverse drive: Fourier coefficients of the
    truncated solve against the exact continuum ODE solution."""
    lam = 1.0 / 0.3
    lz = 2 * np.pi / lam
    fill, e1, e2, eb, qn = 0.375, 2.25, 9.0, 3.0, 1.0
    vox = inputs.layered_stack(64, fill, e1, e2)
    c = O.box_image(vox, (0, 0, 2 * Mz))
    ex = ExactStack([(fill * lz, e1), ((1 - fill) * lz, e2)], qn, (qn * qn - eb))
    m = np.arange(-Mz, Mz + 1)
    ref = ex.fourier(m)
    if route == '1d':
        e = O.solve_stack_1d(c[:, 0, 0], Mz, np.array([0, 0, qn]), lam, eb,
                             np.array([1.0, 0, 0]))[0]
    else:
        M = (1, 1, Mz)
        c3 = O.box_image(vox, (2, 2, 2 * Mz))
        q = O.harmonic_q(np.array([0, 0, qn * 2 * np.pi / lam]), lam, (1, 1, 1), M)
        E = O.solve_dense(c3, M, q, eb, [np.array([1.0, 0, 0])])[0]
        e = E[0, :, M[1], M[0]]
        if np.abs(E[:, :, [0, 2], :]).max() + np.abs(E[:, :, :, [0, 2]]).max() > 1e-13:
            return 1.0
    return float(np.abs(e - ref).max() / np.abs(ref).max())


def err_stack_eps_xx_exact(Mz=40):
    """eps_xx of the stack (k || z) against <eps E>/<E> of the exact ODE field."""
    lam = 1.0 / 0.3
    lz = 2 * np.pi / lam
    fill, e1, e2, qn = 0.375, 2.25, 9.0, 1.0
    vox = inputs.layered_stack(64, fill, e1, e2)
    M = (1, 1, Mz)
    c = O.box_image(vox, (2, 2, 2 * Mz))
    q = O.harmonic_q(np.array([0, 0, qn * 2 * np.pi / lam]), lam, (1, 1, 1), M)
    ee = O.eps_eff_from_fields(c, M, O.solve_dense(c, M, q, 3.0, np.eye(3)))
    ex = ExactStack([(fill * lz, e1), ((1 - fill) * lz, e2)], qn, 1.0)
    z = np.array([0.0])
    ref = ex.fourier(z, weight_eps=True)[0] / ex.fourier(z)[0]
    return float(abs(ee[0, 0] - ref) / abs(ref))


def eps_eff_case(eps, M, k_hat=(0, 0, 1.0), eps_b=None, drives=None, wavelength=1.0 / 0.3,
                 period=(1.0, 1.0, 1.0), n_inc=1.0):
    c, q = _setup(eps, M, k_hat=k_hat, wavelength=wavelength, period=period, n_inc=n_inc)
    eb = float(np.mean(eps)) if eps_b is None else eps_b
    drives = np.eye(3) if drives is None else drives
    E = O.solve_dense(c, M, q, eb, drives)
    return O.eps_eff_from_fields(c, M, E), c, q, E


def asym_body():
    eps = inputs.ellipsoid((6, 5, 7), (1.0, 0.9, 1.1), (0.3, 0.25, 0.35), 5.0)
    eps[1, 2, 3] = 8.0
    eps[4, 0, 1] = 2.5
    return eps


def err_schur_vs_fields():
    eps = asym_body()
    M = (2, 2, 2)
    ee, c, q, _ = eps_eff_case(eps, M, k_hat=(0.3, 0.4, 0.866), period=(1.0, 0.9, 1.1))
    return float(np.abs(ee - O.eps_eff_schur(c, M, q)).max())


def err_eps_b_and_drive_invariance():
    eps = asym_body()
    M = (2, 2, 2)
    kw = dict(k_hat=(0.3, 0.4, 0.866), period=(1.0, 0.9, 1.1))
    e1 = eps_eff_case(eps, M, eps_b=2.0, **kw)[0]
    rng = np.random.default_rng(5)
    D = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    e2 = eps_eff_case(eps, M, eps_b=4.5, drives=D, **kw)[0]
    return float(np.abs(e1 - e2).max())


def err_hermitian_reciprocal():
    eps = asym_body()
    M = (2, 2, 2)
    k = np.array([0.3, 0.4, 0.866])
    e1 = eps_eff_case(eps, M, k_hat=k, period=(1.0, 0.9, 1.1))[0]
    e2 = eps_eff_case(eps, M, k_hat=-k, period=(1.0, 0.9, 1.1))[0]
    return float(max(np.abs(e1 - e1.conj().T).max(), np.abs(e2 - e1.T).max()))


def err_translation_covariance():
    """Rolling the body by t: eps_eff unchanged, E_m -> exp(-i G_m t) E_m."""
    eps = asym_body()
    M = (2, 2, 2)
    kw = dict(k_hat=(0.3, 0.4, 0.866), period=(1.0, 0.9, 1.1), eps_b=3.0)
    e1, _, _, E1 = eps_eff_case(eps, M, **kw)
    e2, _, _, E2 = eps_eff_case(np.roll(eps, 2, axis=2), M, **kw)   # shift x by 2/6
    mx = np.arange(-M[0], M[0] + 1)
    ph = np.exp(-2j * np.pi * mx * 2 / 6)
    return float(max(np.abs(e1 - e2).max(),
                     np.abs(E2 - E1 * ph[None, None, None, None, :]).max()))


def err_cubic_isotropy():
    """Sphere centred in a cubic cell (O_h): eps_eff = e I at k = 0;
    at k || z, eps_xx = eps_yy and the off-diagonal entries vanish."""
    eps = inputs.sphere(8, 0.3, 4.0)
    M = (2, 2, 2)
    e0 = eps_eff_case(eps, M, n_inc=0.0)[0]
    ez = eps_eff_case(eps, M)[0]
    off = ez - np.diag(np.diag(ez))
    return float(max(np.abs(e0 - e0[0, 0] * np.eye(3)).max(), abs(ez[0, 0] - ez[1, 1]),
                     np.abs(off).max()))


def err_stack_long_wavelength():
    """eps_xx of a stack tends to <eps> as Lambda/lambda -> 0 with an
    O((Lambda/lambda)^2) correction: returns the spread of err/r^2."""
    vox = inputs.layered_stack(16, 0.375, 2.25, 9.0)
    M = (1, 1, 6)
    mean = vox.mean()
    ratios = []
    for r in (0.02, 0.01, 0.005):
        ee = eps_eff_case(vox, M, wavelength=1.0 / r, eps_b=2.0)[0]
        ratios.append(abs(ee[0, 0] - mean) / r ** 2)
    return float(abs(ratios[0] / ratios[2] - 1.0))


def err_fft_vs_dense():
    eps = asym_body()
    M = (2, 2, 2)
    c, q = _setup(eps, M, k_hat=(0.3, 0.4, 0.866), period=(1.0, 0.9, 1.1))
    a = np.array([1.0, 0.5j, -0.25])
    E1 = O.solve_dense(c, M, q, 3.0, [a])[0]
    E2, _ = O.solve_fft_gmres(c, M, q, 3.0, a, (9, 10, 12), rtol=1e-14)
    return float(np.abs(E1 - E2).max() / np.abs(E1).max())


ALL = {
    'box_image_quadrature': (err_box_image_quadrature, 1e-13),
    'box_image_slab': (err_box_image_slab, 1e-14),
    'box_image_shift': (err_box_image_shift, 1e-14),
    'green_eigen': (err_green_eigen, 1e-12),
    'trivial_contrast': (err_trivial_contrast, 1e-15),
    'homogeneous_dense': (lambda: err_homogeneous_closed_form('dense'), 1e-13),
    'homogeneous_fft': (lambda: err_homogeneous_closed_form('fft'), 1e-12),
    'stack_exact_1d': (lambda: err_stack_exact(40, '1d'), 1e-5),
    'stack_exact_3d': (lambda: err_stack_exact(12, '3d'), 1e-3),
    'stack_eps_xx_exact': (err_stack_eps_xx_exact, 2e-5),
    'schur_vs_fields': (err_schur_vs_fields, 1e-10),
    'eps_b_drive_invariance': (err_eps_b_and_drive_invariance, 1e-10),
    'hermitian_reciprocal': (err_hermitian_reciprocal, 1e-10),
    'translation_covariance': (err_translation_covariance, 1e-12),
    'cubic_isotropy': (err_cubic_isotropy, 1e-12),
    'stack_long_wavelength': (err_stack_long_wavelength, 0.02),
    'fft_vs_dense': (err_fft_vs_dense, 1e-11),
}
