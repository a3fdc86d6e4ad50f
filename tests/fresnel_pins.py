"""Pins of the Fresnel normal-surface oracle: closed forms of crystal optics
that do not go through its determinant.  Each pin returns an error to hold
below its tolerance.

- isotropic medium: both indices sqrt(eps) in every direction;
- diagonal tensor, propagation along an axis: the indices are the square
  roots of the two other principal values (the field lies along them);
- uniaxial medium (optic axis z, principal indices n_o, n_e): an ordinary
  index n_o and an extraordinary one with 1/n^2 = cos^2(th)/n_o^2 +
  sin^2(th)/n_e^2 at the angle th from the optic axis;
- biaxial medium (e1 < e2 < e3) in the x-z plane: one wave with E along y
  (n^2 = e2) and one with D in the plane, 1/n^2 = D.eps^-1.D; both meet
  at the wave-normal optic axis, cos^2(th) = (1/e2 - 1/e3) / (1/e1 - 1/e3);
- rotation: indices of R eps R^T along R k equal those of eps along k;
- the fit: exact data of a known tensor give that tensor back (full
  symmetric from both indices of 12 directions; diagonal from the axes),
  and data perturbed by 1e-6 move it by about as much.
"""
import numpy as np

from oracle import fresnel as F


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


def _dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def isotropic():
    err = 0.0
    for k in _dirs(8, 1):
        n = F.indices(2.7 * np.eye(3), k)
        err = max(err, np.abs(n - np.sqrt(2.7)).max())
    return err


def diagonal_axes():
    e = np.array([1.7, 2.6, 3.9])
    err = 0.0
    for ax in range(3):
        k = np.eye(3)[ax]
        want = np.sort(np.sqrt(np.delete(e, ax)))
        err = max(err, np.abs(F.indices(np.diag(e), k) - want).max())
    return err


def uniaxial_extraordinary():
    no, ne = 1.45, 1.62
    eps = np.diag([no ** 2, no ** 2, ne ** 2])
    err = 0.0
    for th in np.linspace(0.05, 1.5, 9):
        k = np.array([np.sin(th) * np.cos(0.3), np.sin(th) * np.sin(0.3), np.cos(th)])
        n_ext = 1.0 / np.sqrt(np.cos(th) ** 2 / no ** 2 + np.sin(th) ** 2 / ne ** 2)
        want = np.sort([no, n_ext])
        err = max(err, np.abs(F.indices(eps, k) - want).max())
    return err


def biaxial_plane_and_optic_axis():
    e1, e2, e3 = 2.0, 2.5, 3.4
    eps = np.diag([e1, e2, e3])
    err = 0.0
    for th in np.linspace(0.1, 1.4, 7):
        k = np.array([np.sin(th), 0.0, np.cos(th)])
        d = np.array([np.cos(th), 0.0, -np.sin(th)])
        n_d = 1.0 / np.sqrt(d @ np.linalg.inv(eps) @ d)
        err = max(err, np.abs(F.indices(eps, k) - np.sort([np.sqrt(e2), n_d])).max())
    th = np.arccos(np.sqrt((1 / e2 - 1 / e3) / (1 / e1 - 1 / e3)))
    n = F.indices(eps, [np.sin(th), 0.0, np.cos(th)])
    return max(err, np.abs(n - np.sqrt(e2)).max())


def rotation_covariance():
    eps = np.array([[2.1, 0.2, -0.1], [0.2, 2.9, 0.3], [-0.1, 0.3, 3.3]])
    R = _rot(5)
    err = 0.0
    for k in _dirs(6, 6):
        err = max(err, np.abs(F.indices(R @ eps @ R.T, R @ k) - F.indices(eps, k)).max())
    return err


def fit_full_tensor():
    eps = np.array([[2.3, 0.15, -0.2], [0.15, 2.8, 0.1], [-0.2, 0.1, 3.1]])
    ks = _dirs(12, 9)
    got, rms = F.fit(ks, [F.indices(eps, k) for k in ks])
    return max(np.abs(got - eps).max(), rms)


def fit_noisy_data():
    """Indices perturbed by 1e-6 relative: the fit moves by about as much."""
    eps = np.array([[2.3, 0.15, -0.2], [0.15, 2.8, 0.1], [-0.2, 0.1, 3.1]])
    ks = _dirs(16, 10)
    rng = np.random.default_rng(11)
    ns = [F.indices(eps, k) * (1 + 1e-6 * rng.normal(size=2)) for k in ks]
    got, _ = F.fit(ks, ns)
    return np.abs(got - eps).max()


def fit_diagonal_from_axes():
    e = np.array([2.2, 2.5, 2.9])
    ks = np.eye(3)
    got, rms = F.fit(ks, [F.indices(np.diag(e), k) for k in ks], diagonal=True)
    return max(np.abs(got - np.diag(e)).max(), rms)


ALL = {
    "isotropic": (isotropic, 1e-13),
    "diagonal_axes": (diagonal_axes, 1e-13),
    "uniaxial_extraordinary": (uniaxial_extraordinary, 1e-12),
    "biaxial_plane_and_optic_axis": (biaxial_plane_and_optic_axis, 1e-7),
    "rotation_covariance": (rotation_covariance, 1e-12),
    "fit_full_tensor": (fit_full_tensor, 1e-9),
    "fit_noisy_data": (fit_noisy_data, 2e-5),
    "fit_diagonal_from_axes": (fit_diagonal_from_axes, 1e-10),
}
