"""FP64 CPU oracle of the magnetic-field system, Eq.(5) of arXiv 1501.01752.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product library.

Eq.(5) written with normalised wave-vectors q_m = k_m / k0 (the factor k0^2
cancels between k_bm k_sm' and k_b^2 - k_m^2):

    H_m = H^inc_m + q_m x w_m / (eps_b - |q_m|^2),
    w_m = sum_m' [delta_mm' - eps_b eta_{m-m'}] (q_m' x H_m'),

where eta_n are the Fourier coefficients of 1/eps (the paper's
(eps_b/eps)_n = eps_b eta_n, found "just in the same way" as those of eps,
"Calculation details") and x is the vector product (the Levi-Civita sums of
Eq.(5)).  The incident field is H^inc_m = delta_m0 a.  Conventions of
arrays follow oracle/gsm.py: fields (3, N1z, N1y, N1x), coefficients
(2Nz+1, 2Ny+1, 2Nx+1) indexed n + N.
"""
import numpy as np
import scipy.linalg
import scipy.sparse.linalg

from . import gsm as O


def inverse_box_image(eps, n_max):
    """eta_n of a voxel body: the exact image of the piecewise-constant 1/eps."""
    return O.box_image(1.0 / np.asarray(eps, dtype=np.float64), n_max)


def cross_matrix(q):
    """[q]_x per harmonic, shape (..., 3, 3): [q]_x v = q x v."""
    q = np.asarray(q, dtype=np.float64)
    Z = np.zeros(q.shape[:-1])
    return np.stack([np.stack([Z, -q[..., 2], q[..., 1]], -1),
                     np.stack([q[..., 2], Z, -q[..., 0]], -1),
                     np.stack([-q[..., 1], q[..., 0], Z], -1)], -2)


def assemble_dense_h(eta, M, q, eps_b):
    """Dense matrix A_H = I - B_H of Eq.(5) over the unknowns
    [component][mz][my][mx] (route O1 for the H field)."""
    T = O.toeplitz(eta, M)              # eta_{m-m'}
    n = T.shape[0]
    conv = np.eye(n) - eps_b * T        # delta_mm' - eps_b eta_{m-m'}
    qf = np.asarray(q, dtype=np.float64).reshape(n, 3)
    X = cross_matrix(qf)                # (n, 3, 3)
    den = 1.0 / (eps_b - np.sum(qf * qf, axis=1))
    B = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    # B[(a,m),(u,m')] = sum_g X_m[a,g] den_m conv[m,m'] X_m'[g,u]
    for a in range(3):
        for u in range(3):
            blk = np.zeros((n, n), dtype=np.complex128)
            for g in range(3):
                blk += (X[:, a, g] * den)[:, None] * conv * X[None, :, g, u]
            B[a * n:(a + 1) * n, u * n:(u + 1) * n] = blk
    return np.eye(3 * n) - B


def solve_dense_h(eta, M, q, eps_b, drives):
    """LU solve of Eq.(5) with H^inc_m = delta_m0 a, one column per drive;
    returns (n_drive, 3, N1z, N1y, N1x)."""
    A = assemble_dense_h(eta, M, q, eps_b)
    B = np.stack([O.incident_rhs(M, a) for a in drives], axis=1)
    X = scipy.linalg.solve(A, B)
    shape = (3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    return np.stack([X[:, p].reshape(shape) for p in range(X.shape[1])])


def apply_operator_fft_h(eta, M, q, eps_b, x, P):
    """A_H x with the Toeplitz product by FFT on a P grid (route O2): the
    convolution with delta - eps_b eta of each component of q x x."""
    x = np.asarray(x, dtype=np.complex128).reshape((3,) + tuple(2 * m + 1 for m in M[::-1]))
    qv = np.asarray(q, dtype=np.float64)
    u = np.cross(qv, np.moveaxis(x, 0, -1))            # q_m x x_m, (N1z, N1y, N1x, 3)
    u = np.moveaxis(u, -1, 0)
    # (delta - eps_b eta) * u = u - eps_b (eta * u); eps_b eta * u = convolution
    # with c' = eps_b eta, done by the E-form routine with eps_b' = 1:
    # contrast_convolution_fft(c, M, 1, v, P) = T(c) v - v
    tv = O.contrast_convolution_fft(eps_b * eta, M, 1.0, u, P) + u
    w = u - tv
    den = 1.0 / (eps_b - np.sum(qv * qv, axis=-1))
    bw = np.moveaxis(np.cross(qv, np.moveaxis(w, 0, -1)) * den[..., None], -1, 0)
    return (x - bw).ravel()


def solve_fft_gmres_h(eta, M, q, eps_b, a, P, rtol=1e-12, restart=30, maxiter=2000):
    """Eq.(5) by SciPy GMRES(restart) on the FFT operator (route O2 for H)."""
    n = 3 * (2 * M[0] + 1) * (2 * M[1] + 1) * (2 * M[2] + 1)
    op = scipy.sparse.linalg.LinearOperator((n, n), dtype=np.complex128,
                                            matvec=lambda v: apply_operator_fft_h(eta, M, q, eps_b, v, P))
    b = O.incident_rhs(M, np.asarray(a, dtype=np.complex128))
    x, info = scipy.sparse.linalg.gmres(op, b, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter)
    return x.reshape((3,) + tuple(2 * m + 1 for m in M[::-1])), info
