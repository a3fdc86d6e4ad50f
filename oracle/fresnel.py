"""FP64 CPU oracle of the Fresnel normal surface, the last step of the
pole-search retrieval of arXiv 1501.01752 ("Modes in 3D crystals": each
propagation direction of the effective medium carries two refractive
indices, the solutions of the Fresnel normal equation; the uniaxial and
biaxial examples read the principal indices off propagation along the
lattice axes).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product library.

A plane wave E exp(i k0 n k.r) (k a unit vector) in a homogeneous medium of
real symmetric permittivity tensor eps obeys k x (k x E) n^2 + eps E = 0,
i.e. (eps - n^2 (I - k k^T)) E = 0.  Its indices are the roots t = n^2 of
det(eps - t (I - k k^T)) = 0.  The projector I - k k^T has rank 2, so the
determinant is a quadratic in t: two indices per direction.
"""
import numpy as np
import scipy.optimize


def projector(k_hat):
    """I - k k^T for the unit vector along k_hat."""
    k = np.asarray(k_hat, dtype=np.float64)
    k = k / np.linalg.norm(k)
    return np.eye(3) - np.outer(k, k)


def normal_polynomial(eps, k_hat):
    """Coefficients (c2, c1, c0) of det(eps - t P) = c2 t^2 + c1 t + c0: the
    determinant sampled at t = 0, 1, 2 (it is exactly quadratic), then the
    interpolating parabola."""
    eps = np.asarray(eps, dtype=np.float64)
    P = projector(k_hat)
    d = [np.linalg.det(eps - t * P) for t in (0.0, 1.0, 2.0)]
    c0 = d[0]
    c2 = (d[2] - 2.0 * d[1] + d[0]) / 2.0
    c1 = d[1] - d[0] - c2
    return c2, c1, c0


def indices(eps, k_hat):
    """The two refractive indices (ascending) of direction k_hat."""
    c2, c1, c0 = normal_polynomial(eps, k_hat)
    t = np.sort(np.roots([c2, c1, c0]).real)
    return np.sqrt(t)


def _eps_of(p, diagonal):
    if diagonal:
        return np.diag(p)
    e = np.empty((3, 3))
    e[0, 0], e[1, 1], e[2, 2] = p[0], p[1], p[2]
    e[0, 1] = e[1, 0] = p[3]
    e[0, 2] = e[2, 0] = p[4]
    e[1, 2] = e[2, 1] = p[5]
    return e


def _form_row(k, diagonal):
    """Coefficients of the 3 (diagonal) or 6 tensor parameters in k^T e k."""
    if diagonal:
        return k * k
    return np.array([k[0] ** 2, k[1] ** 2, k[2] ** 2, 2 * k[0] * k[1], 2 * k[0] * k[2], 2 * k[1] * k[2]])


def initial_tensor(k_hats, n_pairs, diagonal=False):
    """The product of a direction's two roots is det(eps) / (k^T eps k), so
    E = eps / det(eps) has k^T E k = 1 / (n1^2 n2^2): a linear least-squares
    problem for E, then eps = E / sqrt(det E)."""
    k_hats = np.asarray(k_hats, dtype=np.float64).reshape(-1, 3)
    k_hats = k_hats / np.linalg.norm(k_hats, axis=1, keepdims=True)
    t = np.asarray(n_pairs, dtype=np.float64).reshape(-1, 2) ** 2
    A = np.array([_form_row(k, diagonal) for k in k_hats])
    E = _eps_of(np.linalg.lstsq(A, 1.0 / (t[:, 0] * t[:, 1]), rcond=None)[0], diagonal)
    return E / np.sqrt(np.linalg.det(E))


def fit(k_hats, n_pairs, diagonal=False):
    """Real symmetric tensor (diagonal: principal axes along x, y, z) whose
    normal surface passes closest to the observed directions and their two
    indices each: least squares on det(eps - n^2 P) / n^6 by SciPy's
    trust-region solver, from the linear estimate of initial_tensor."""
    k_hats = np.asarray(k_hats, dtype=np.float64).reshape(-1, 3)
    n_pairs = np.asarray(n_pairs, dtype=np.float64).reshape(-1, 2)
    Ps = [projector(k) for k in k_hats for _ in range(2)]
    t = n_pairs.ravel() ** 2

    def resid(p):
        e = _eps_of(p, diagonal)
        return np.array([np.linalg.det(e - ti * Pi) / ti ** 3 for ti, Pi in zip(t, Ps)])

    e0 = initial_tensor(k_hats, n_pairs, diagonal)
    p0 = np.diag(e0).copy() if diagonal else np.array([e0[0, 0], e0[1, 1], e0[2, 2], e0[0, 1], e0[0, 2],
                                                       e0[1, 2]])
    sol = scipy.optimize.least_squares(resid, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
    return _eps_of(sol.x, diagonal), float(np.sqrt(np.mean(sol.fun ** 2)))
