"""Shared helpers of the GPU parity tests: build the same seeded case for the
HIP library and for the CPU oracle."""
import sys

import numpy as np

from oracle import gsm as O
from paper_1501_01752_amd import inputs


def say(msg):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    sys.stdout.write(f"[gpu-case] {msg}\n")
    sys.stdout.flush()


def torch_dev():
    import torch
    return torch.device("cuda:0")


def k_vector(wavelength, k_hat, n_inc=1.0):
    k0 = 2 * np.pi / wavelength
    k = np.asarray(k_hat, dtype=np.float64)
    k = k / np.linalg.norm(k) if np.linalg.norm(k) > 0 else k
    return n_inc * k0 * k


def oracle_case(eps, period, wavelength, k_inc, M):
    c = O.box_image(eps, tuple(2 * m for m in M))
    q = O.harmonic_q(k_inc, wavelength, period, M)
    return c, q


def asym_body():
    eps = inputs.ellipsoid((6, 5, 7), (1.0, 0.9, 1.1), (0.3, 0.25, 0.35), 5.0)
    eps[1, 2, 3] = 8.0
    eps[4, 0, 1] = 2.5
    return eps


def seeded_field(shape, seed, dtype=np.complex128):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(dtype)


def to_torch(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch_dev())


def rel_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def oracle_P(M):
    """An FFT size per axis the oracle may use: any P >= 4M + 1 gives the same
    operator; 2-3-5 smooth sizes keep numpy fast."""
    out = []
    for m in M:
        p = 4 * m + 1
        while True:
            r = p
            for f in (2, 3, 5):
                while r % f == 0:
                    r //= f
            if r == 1:
                break
            p += 1
        out.append(p)
    return tuple(out)


def fp32_operator_tol(P):
    """Bound on max|y - y_ref| / max|y_ref| for one complex64 application of
    the operator on a grid of P points: each output passes six transforms of
    log2 P butterfly levels (x, y, z, forward and inverse), and the rounding
    of a level is at most the unit roundoff u32 = 2^-24 = 6.0e-8 relative to
    the largest value; the contrast multiply and the Green epilogue add a
    few u32 more.  6 log2(P) u32 + 4 u32: 2.4e-6 at P = 64, 2.8e-6 at 128."""
    import math
    return (6 * math.log2(P) + 4) * 6.0e-8
