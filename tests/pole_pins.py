"""Checks that tie the pole-search oracle (oracle/poles.py) to facts outside
itself: meromorphic test functions with known poles and amplitudes, the
singularity of the Eq.(4) operator at a found pole (a singular value of the
dense matrix from oracle/gsm.py's independent assembly), the residue as the
limit (kappa - eta) xi(kappa) of dense solves, and the paper's printed
effective index of Fig. 2 as a loose physical check.  ALL maps a name to
(function, bound); the mutation tests require one of them to fail for each
planted mistake."""
import numpy as np

from oracle import gsm as O
from oracle import poles as OP


def _near_errors(eta_true, zeta_true, eta, zeta):
    e = z = 0.0
    for t, zt in zip(eta_true, zeta_true):
        j = int(np.argmin(np.abs(eta - t)))
        e = max(e, abs(eta[j] - t))
        z = max(z, abs(zeta[j] - zt) / abs(zt))
    return e, z


def err_polynomial_regular_part():
    """Three poles and a polynomial regular part of degree N_d - N_p - 1:
    P xi is a polynomial of degree N_d - 1, so every divided difference of
    order N_d vanishes and the poles and amplitudes are exact."""
    eta_t = np.array([2.52 - 0.02j, 2.71 + 0.01j, 2.96 + 0.05j])
    zeta_t = np.array([0.3 + 0.1j, -0.2j, 0.7])
    Np, Nd = 3, 10
    k = OP.kappa_mesh(2.41, 2.93, Np, Nd)
    reg = lambda x: 0.3 - 0.2 * x + 0.05 * x ** 2 + 0.01j * x ** 3 - 0.002 * x ** 4 + 1e-3 * x ** 6
    xi = np.array([np.sum(zeta_t / (kk - eta_t)) + reg(kk) for kk in k])
    eta, zeta = OP.pole_search(k, xi, Np, Nd)
    e, z = _near_errors(eta_t, zeta_t, eta, zeta)
    return max(e, 1e-3 * z)


def err_meromorphic_regular_part():
    """Two poles near the mesh, three far ones and an exponential: with
    N_p = 5, N_d = 10 the near poles come out to rounding."""
    eta_t = np.array([2.6513 + 0.0j, 2.7504 + 0.001j])
    zeta_t = np.array([0.4, 0.1 - 0.05j])
    far = np.array([6.0 + 1j, -3.0, 8.0 - 2j])
    Np, Nd = 5, 10
    k = OP.kappa_mesh(2.41, 2.93, Np, Nd)
    xi = np.array([np.sum(zeta_t / (kk - eta_t)) + np.sum(1.0 / (kk - far)) + np.exp(0.3 * kk) for kk in k])
    eta, zeta = OP.pole_search(k, xi, Np, Nd)
    e, z = _near_errors(eta_t, zeta_t, eta, zeta)
    return max(e, 1e-3 * z)


def fig2_case(M, eps_host=2.25):
    """Fig. 2's lattice: cubic air cavities of side Lambda/2 centred in a host,
    Lambda = 0.3 lambda (exact on 4^3 voxels); xi = E_x,0 for k || z, x drive."""
    vox = np.full((4, 4, 4), float(eps_host))
    vox[1:3, 1:3, 1:3] = 1.0
    lam = 1 / 0.3
    return vox, (1.0, 1.0, 1.0), lam


def dense_xi(vox, period, lam, M, kappas, eps_b, k_hat=(0, 0, 1), drive=(1.0, 0, 0), comp=0):
    c = O.box_image(vox, tuple(2 * m for m in M))
    kh = np.asarray(k_hat, float) / np.linalg.norm(k_hat)
    out = []
    for kk in kappas:
        q = O.harmonic_q(kk * kh, lam, period, M)
        E = O.solve_dense(c, M, q, eps_b, [np.asarray(drive, complex)])[0]
        out.append(E.reshape(3, -1)[comp, O.zero_index(M)])
    return np.array(out), c


def fig2_poles(M, eps_host=2.25, n_lo=1.30, n_hi=1.60, eps_b=3.5):
    vox, period, lam = fig2_case(M, eps_host)
    k0 = 2 * np.pi / lam
    kap = OP.kappa_mesh(n_lo * k0, n_hi * k0, 5, 10)
    xi, c = dense_xi(vox, period, lam, M, kap, eps_b)
    eta, zeta = OP.pole_search(kap, xi, 5, 10)
    j = OP.dominant_pole(eta, zeta, kap[0], kap[-1])
    return eta, zeta, j, c, k0, lam, period


def err_operator_singular_at_pole():
    """The dominant pole makes the truncated operator L = K - T(eps) of
    Eq.(4) singular: its smallest singular value over its largest."""
    M = (2, 2, 2)
    eta, zeta, j, c, k0, lam, period = fig2_poles(M)
    if j < 0:
        return np.inf
    q = O.harmonic_q(np.array([0.0, 0.0, eta[j].real]), lam, period, M)
    s = np.linalg.svd(O.operator_L(c, M, q), compute_uv=False)
    return s[-1] / s[0]


def err_residue_limit():
    """zeta = lim (kappa - eta) xi(kappa): dense solves at eta (1 +- 1e-6),
    averaged to cancel the first-order term."""
    M = (2, 2, 2)
    eta, zeta, j, c, k0, lam, period = fig2_poles(M)
    if j < 0:
        return np.inf
    vox, period, lam = fig2_case(M)
    e = eta[j].real
    d = 1e-6 * e
    xi, _ = dense_xi(vox, period, lam, M, [e + d, e - d], 3.5)
    lim = 0.5 * (d * xi[0] + (-d) * xi[1])
    return abs(lim - zeta[j]) / abs(zeta[j])


def err_fig2_effective_index():
    """Loose physical check: the paper's Fig. 2 gives n_eff = 1.441688 for
    n = 1.5 (its converged value, truncation unstated); at 7^3 harmonics the
    pole lies within 2.5e-3 of it."""
    eta, zeta, j, c, k0, lam, period = fig2_poles((3, 3, 3))
    return abs(eta[j].real / k0 - 1.441688) if j >= 0 else np.inf


ALL = {
    "polynomial_regular_part": (err_polynomial_regular_part, 1e-9),
    "meromorphic_regular_part": (err_meromorphic_regular_part, 1e-10),
    "operator_singular_at_pole": (err_operator_singular_at_pole, 1e-12),
    "residue_limit": (err_residue_limit, 1e-8),
    "fig2_effective_index": (err_fig2_effective_index, 2.5e-3),
}
