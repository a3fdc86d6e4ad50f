"""Exact continuum solution of a plane-wave-driven layered medium (test pin).

Independent of any Fourier truncation: for a stack eps(z) made of layers
(thickness_j, eps_j) and a drive along z, the transverse field solves the
ordinary differential equation obtained from curl curl E - k0^2 eps E = source
(the form the GSM system takes after multiplication by the inverse Green
factor):

    -E''(z) - eps(z) E(z) = s exp(i q z),     E(z + L) = exp(i q L) E(z),

in units where k0 = 1.  In each layer E = A exp(i kz) + B exp(-i kz) +
s exp(i q z) / (q^2 - eps_j) with kz = sqrt(eps_j); E and E' are continuous at
every interface and Bloch-periodic across the cell.  Fourier coefficients
E_m = (1/L) int_0^L E(z) exp(-i (q + m K) z) dz, K = 2 pi / L, follow in
closed form from integrals of exponentials.
"""
import numpy as np


def _int_exp(beta, za, zb):
    beta = np.asarray(beta, dtype=np.complex128)
    out = np.empty(np.broadcast(beta, za).shape, dtype=np.complex128)
    small = np.abs(beta) < 1e-14
    out[small] = zb - za
    b = beta[~small]
    out[~small] = (np.exp(1j * b * zb) - np.exp(1j * b * za)) / (1j * b)
    return out


class ExactStack:
    def __init__(self, layers, q, s):
        """layers: list of (thickness, eps) in units of 1/k0; q: Bloch wave
        number along z (units of k0); s: source amplitude."""
        self.layers = [(float(t), float(e)) for t, e in layers]
        self.q = float(q)
        self.s = complex(s)
        self.L = sum(t for t, _ in self.layers)
        z = [0.0]
        for t, _ in self.layers:
            z.append(z[-1] + t)
        self.z = z
        nl = len(self.layers)
        kz = [np.sqrt(e) for _, e in self.layers]
        part = [self.s / (self.q ** 2 - e) for _, e in self.layers]
        self.kz, self.part = kz, part
        # unknowns (A_j, B_j); equations: continuity of E, E' at interior
        # interfaces and Bloch periodicity between the last and first layer.
        mat = np.zeros((2 * nl, 2 * nl), dtype=np.complex128)
        rhs = np.zeros(2 * nl, dtype=np.complex128)
        row = 0
        for j in range(nl):
            jn = (j + 1) % nl
            zj = self.z[j + 1]
            zn = self.z[j + 1] if jn != 0 else 0.0
            ph = 1.0 if jn != 0 else np.exp(1j * self.q * self.L)
            # E_j(zj) = ph * E_jn(zn)
            mat[row, 2 * j] = np.exp(1j * kz[j] * zj)
            mat[row, 2 * j + 1] = np.exp(-1j * kz[j] * zj)
            mat[row, 2 * jn] -= ph * np.exp(1j * kz[jn] * zn)
            mat[row, 2 * jn + 1] -= ph * np.exp(-1j * kz[jn] * zn)
            rhs[row] = ph * part[jn] * np.exp(1j * self.q * zn) - part[j] * np.exp(1j * self.q * zj)
            row += 1
            mat[row, 2 * j] = 1j * kz[j] * np.exp(1j * kz[j] * zj)
            mat[row, 2 * j + 1] = -1j * kz[j] * np.exp(-1j * kz[j] * zj)
            mat[row, 2 * jn] -= ph * 1j * kz[jn] * np.exp(1j * kz[jn] * zn)
            mat[row, 2 * jn + 1] -= ph * (-1j) * kz[jn] * np.exp(-1j * kz[jn] * zn)
            rhs[row] = (ph * part[jn] * 1j * self.q * np.exp(1j * self.q * zn)
                        - part[j] * 1j * self.q * np.exp(1j * self.q * zj))
            row += 1
        self.coef = np.linalg.solve(mat, rhs)

    def fourier(self, m, weight_eps=False):
        """(1/L) int E(z) exp(-i(q + mK)z) dz (times eps(z) if weight_eps)."""
        m = np.asarray(m, dtype=np.float64)
        K = 2 * np.pi / self.L
        out = np.zeros(m.shape, dtype=np.complex128)
        for j, (_, e) in enumerate(self.layers):
            za, zb = self.z[j], self.z[j + 1]
            A, B = self.coef[2 * j], self.coef[2 * j + 1]
            base = -(self.q + m * K)
            term = (A * _int_exp(base + self.kz[j], za, zb)
                    + B * _int_exp(base - self.kz[j], za, zb)
                    + self.part[j] * _int_exp(base + self.q, za, zb))
            out += (e if weight_eps else 1.0) * term
        return out / self.L
