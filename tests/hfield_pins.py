"""Checks that tie the H-field oracle (oracle/hfield.py, Eq.(5)) to facts
outside itself: a uniform medium equal to the basis gives the incident field,
the closed form of a homogeneous medium, the transversality q_m . H_m = 0
that Eq.(5) forces for a transverse drive, and Maxwell's curl relation
between the modes of the two formulations: at a mode found from the pinned
E-field system, H* = q x E* (the curl of the mode's E field) solves the
H-field system, to a residual that falls with the order count for a smooth
permittivity.  ALL maps a name to (function, bound)."""
import numpy as np

from oracle import gsm as O
from oracle import hfield as OH
from oracle import poles as OP


def _asym_body():
    rng = np.random.default_rng(21)
    eps = rng.uniform(1.0, 6.0, (3, 4, 5))
    return eps, (1.0, 0.9, 1.2)


def err_uniform_is_incident():
    """eps = eps_b everywhere: delta - eps_b eta = 0, so H = H^inc exactly."""
    M = (2, 1, 2)
    eta = OH.inverse_box_image(np.full((3, 3, 3), 2.5), tuple(2 * m for m in M))
    q = O.harmonic_q(np.array([0.3, 0.1, 1.2]), 1.0, (1.0, 1.0, 1.0), M)
    a = np.array([0.2, 1.0 - 0.5j, 0.1])
    H = OH.solve_dense_h(eta, M, q, 2.5, [a])[0]
    ref = O.incident_rhs(M, a)
    return float(np.abs(H.ravel() - ref).max())


def err_homogeneous_closed_form():
    """eps = eps_h != eps_b: only m = 0 is excited; the part of a across q_0
    is scaled by (|q|^2 - eps_b) eps_h / (eps_b (|q|^2 - eps_h)), the part
    along q_0 is unchanged (it is not a field of any mode)."""
    M = (1, 2, 1)
    eh, eb = 4.0, 2.0
    eta = OH.inverse_box_image(np.full((2, 2, 2), eh), tuple(2 * m for m in M))
    q0 = np.array([0.4, -0.3, 1.1])
    q = O.harmonic_q(2 * np.pi * q0, 1.0, (1.0, 0.8, 1.3), M)     # k_inc = k0 q0 at lambda = 1
    a = np.array([1.0, 0.5j, -0.2])
    H = OH.solve_dense_h(eta, M, q, eb, [a])[0].reshape(3, -1)
    i0 = O.zero_index(M)
    qq = q0 @ q0
    al = (a @ q0) / qq * q0
    ref = al + (a - al) * (qq - eb) * eh / (eb * (qq - eh))
    rest = np.delete(H, i0, axis=1)
    return max(float(np.abs(H[:, i0] - ref).max()), float(np.abs(rest).max()))


def err_transverse():
    """a . q_0 = 0 gives q_m . H_m = 0 at every harmonic (Eq.(5) adds only
    q_m x w_m to the incident field)."""
    eps, period = _asym_body()
    M = (2, 2, 1)
    eta = OH.inverse_box_image(eps, tuple(2 * m for m in M))
    q0 = np.array([0.3, 0.2, 0.9])
    q = O.harmonic_q(2 * np.pi * q0, 1.0, period, M)
    a = np.cross(q0, [0.0, 1.0, 0.3]) * (1 + 0.5j)
    H = OH.solve_dense_h(eta, M, q, 3.0, [a])[0]
    div = np.einsum('czyx,zyxc->zyx', H, q)
    return float(np.abs(div).max() / np.abs(H).max())


def smooth_body(nmax, grid=48):
    """A smooth, non-symmetric permittivity (three cosines with phases) and
    the coefficients of eps and 1/eps, from an FFT of their samples on a
    fine grid (spectrally accurate for |n| <= nmax)."""
    u = np.arange(grid) / grid
    z, y, x = np.meshgrid(u, u, u, indexing='ij')
    eps = (3.0 + 0.8 * np.cos(2 * np.pi * x + 0.4) + 0.6 * np.sin(2 * np.pi * (y + z) + 0.2)
           + 0.3 * np.cos(2 * np.pi * (x - 2 * y) + 1.1))

    def coef(f):
        F = np.fft.fftn(f) / f.size
        nz = np.arange(-nmax[2], nmax[2] + 1) % grid
        ny = np.arange(-nmax[1], nmax[1] + 1) % grid
        nx = np.arange(-nmax[0], nmax[0] + 1) % grid
        return F[np.ix_(nz, ny, nx)]
    return coef(eps), coef(1.0 / eps)


SMOOTH = {"lam": 1 / 0.35, "khat": (0.2, 0.1, 1.0), "eps_b": 5.0, "window": (1.55, 1.85)}


def mode_residual(m):
    """Residual |A_H (q x E*)| / |q x E*| of the curl of the E-form mode E*
    (the pole of E_x,0 inside the window, the null vector of L by one inverse
    iteration) under the H-form operator, and the E-form mode's n_eff."""
    M = (m, m, m)
    c, eta = smooth_body(tuple(2 * k for k in M))
    lam = SMOOTH["lam"]
    k0 = 2 * np.pi / lam
    kh = np.asarray(SMOOTH["khat"], float)
    kh /= np.linalg.norm(kh)
    period = (1.0, 1.0, 1.0)
    kap = OP.kappa_mesh(SMOOTH["window"][0] * k0, SMOOTH["window"][1] * k0, 5, 10)
    xi = []
    for kk in kap:
        q = O.harmonic_q(kk * kh, lam, period, M)
        E = O.solve_dense(c, M, q, SMOOTH["eps_b"], [np.array([1.0, 0, 0])])[0]
        xi.append(E.reshape(3, -1)[0, O.zero_index(M)])
    eta_p, zeta_p = OP.pole_search(kap, np.array(xi), 5, 10)
    j = OP.dominant_pole(eta_p, zeta_p, kap[0], kap[-1])
    ks = eta_p[j].real
    q = O.harmonic_q(ks * kh, lam, period, M)
    L = O.operator_L(c, M, q)
    x = np.linalg.solve(L, np.random.default_rng(0).standard_normal(L.shape[0]))
    H = np.cross(q.reshape(-1, 3), x.reshape(3, -1).T).T.ravel()
    AH = OH.assemble_dense_h(eta, M, q, SMOOTH["eps_b"])
    return np.linalg.norm(AH @ H) / np.linalg.norm(H), ks / k0


def err_curl_of_e_mode():
    """Residual at 7^3 harmonics below 2e-4, and 4x below that at 5^3."""
    r2, _ = mode_residual(2)
    r3, _ = mode_residual(3)
    if not r3 < r2 / 4:
        return np.inf
    return r3


ALL = {
    "uniform_is_incident": (err_uniform_is_incident, 1e-15),
    "homogeneous_closed_form": (err_homogeneous_closed_form, 1e-14),
    "transverse_field": (err_transverse, 1e-13),
    "curl_of_e_mode": (err_curl_of_e_mode, 2e-4),
}
