"""Dense FP64 derivative of the effective tensor with respect to voxel
permittivities (forward / tangent mode) and central finite differences.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

For drive p the field solves A E_p = b_p with A = I - G (T(eps)/eps_b - I)
(Eq.(4)); eps_eff = D0 E0^-1 with E0 = [E_p,0] and D0 = [(T E_p)_0].  A voxel
perturbation d eps_v changes the coefficients by dc_n = phi_{n,v}, the exact
Fourier image of that voxel's box, hence dA = -G dT / eps_b (eps_b held
fixed), dE_p = -A^-1 dA E_p, dE0 = [dE_p,0], dD0 = [(dT E_p)_0 + (T dE_p)_0]
and d eps_eff = (dD0 - eps_eff dE0) E0^-1.  For a real loss L(eps_eff) with
Gbar = dL/d conj(eps_eff), dL = 2 Re sum_ij conj(Gbar_ij) d eps_eff_ij.
"""
import numpy as np
import scipy.linalg

from oracle import gsm as O


def _fields_and_tensor(c, M, q, eps_b):
    A = O.assemble_dense(c, M, q, eps_b)
    lu = scipy.linalg.lu_factor(A)
    B = np.stack([O.incident_rhs(M, e) for e in np.eye(3)], axis=1)
    X = scipy.linalg.lu_solve(lu, B)
    n = X.shape[0] // 3
    i0 = O.zero_index(M)
    T = O.toeplitz(c, M)
    E0 = np.stack([X[np.arange(3) * n + i0, p] for p in range(3)], axis=1)
    D0 = np.stack([np.array([T[i0] @ X[a * n:(a + 1) * n, p] for a in range(3)]) for p in range(3)], axis=1)
    return lu, X, T, E0, D0, D0 @ np.linalg.inv(E0)


def loss_and_tangent(eps, M, k_inc, wavelength, period, eps_b, target, voxels):
    """L = ||eps_eff - target||_F^2 and dL/d eps_v for each flat voxel index v."""
    eps = np.asarray(eps, dtype=np.float64)
    c = O.box_image(eps, tuple(2 * m for m in M))
    q = O.harmonic_q(k_inc, wavelength, period, M)
    lu, X, T, E0, D0, ee = _fields_and_tensor(c, M, q, eps_b)
    gbar = ee - target
    L = float(np.sum(np.abs(ee - target) ** 2))
    n = X.shape[0] // 3
    i0 = O.zero_index(M)
    G = O.green_tensor(q, eps_b).reshape(n, 3, 3)
    E0inv = np.linalg.inv(E0)
    out = []
    for v in voxels:
        unit = np.zeros(eps.size)
        unit[v] = 1.0
        dc = O.box_image(unit.reshape(eps.shape), tuple(2 * m for m in M))
        dT = O.toeplitz(dc, M)
        # dA X = -G (dT X) / eps_b, component-wise over the 3 field components
        dTX = np.stack([dT @ X[a * n:(a + 1) * n] for a in range(3)])      # (3, n, 3)
        dAX = -np.einsum('mab,bmp->amp', G, dTX) / eps_b                   # (3, n, 3)
        dX = -scipy.linalg.lu_solve(lu, dAX.reshape(3 * n, 3))
        dE0 = np.stack([dX[np.arange(3) * n + i0, p] for p in range(3)], axis=1)
        dD0 = np.stack([np.array([dT[i0] @ X[a * n:(a + 1) * n, p] + T[i0] @ dX[a * n:(a + 1) * n, p]
                                  for a in range(3)]) for p in range(3)], axis=1)
        dee = (dD0 - ee @ dE0) @ E0inv
        out.append(2.0 * np.real(np.sum(np.conj(gbar) * dee)))
    return L, ee, np.array(out)


def loss_fd(eps, M, k_inc, wavelength, period, eps_b, target, voxels, h=1e-6):
    """Central finite differences of L at the given voxels (dense solves)."""
    eps = np.asarray(eps, dtype=np.float64)
    q = O.harmonic_q(k_inc, wavelength, period, M)

    def L_of(e):
        c = O.box_image(e, tuple(2 * m for m in M))
        ee = _fields_and_tensor(c, M, q, eps_b)[-1]
        return float(np.sum(np.abs(ee - target) ** 2))
    out = []
    for v in voxels:
        ep = eps.copy().ravel()
        em = eps.copy().ravel()
        ep[v] += h
        em[v] -= h
        out.append((L_of(ep.reshape(eps.shape)) - L_of(em.reshape(eps.shape))) / (2 * h))
    return np.array(out)
