"""The H-field oracle (Eq.(5)) against a uniform and a homogeneous medium,
transversality and the curl of the E-field system's modes (no GPU), its FFT
route against its dense matrix, and planted mistakes these pins must catch."""
import numpy as np
import pytest

import hfield_pins as P
from oracle import gsm as O
from oracle import hfield as OH


@pytest.mark.parametrize("name", sorted(P.ALL))
def test_hfield_pin(name):
    fn, tol = P.ALL[name]
    err = fn()
    assert err <= tol, f"{name}: {err:.3e} > {tol:.0e}"


def test_fft_route_equals_dense_matrix():
    eps, period = P._asym_body()
    M = (2, 3, 1)
    eta = OH.inverse_box_image(eps, tuple(2 * m for m in M))
    q = O.harmonic_q(np.array([0.5, -0.2, 2.0]), 1.3, period, M)
    x = np.random.default_rng(4).standard_normal(3 * 5 * 7 * 3) * (1 + 0.3j)
    A = OH.assemble_dense_h(eta, M, q, 2.7)
    y = OH.apply_operator_fft_h(eta, M, q, 2.7, x, (13, 13, 13))
    assert np.abs(y - A @ x).max() <= 1e-13 * np.abs(A @ x).max()


def _any_pin_fails():
    failed = []
    for name, (fn, tol) in P.ALL.items():
        try:
            err = fn()
        except Exception:
            err = np.inf
        if not (err <= tol):
            failed.append(name)
    return failed


def _m_transposed(mp):
    orig = O.toeplitz
    mp.setattr(OH, "O", type("Oproxy", (), {k: staticmethod(getattr(O, k)) if callable(getattr(O, k)) else getattr(O, k)
                                            for k in dir(O) if not k.startswith("__")}))
    OH.O.toeplitz = staticmethod(lambda c, M: orig(c, M).T)


def _m_denominator_sign(mp):
    orig = OH.assemble_dense_h

    def a(eta, M, q, eps_b):
        return 2 * np.eye(orig(eta, M, q, eps_b).shape[0]) - orig(eta, M, q, eps_b)
    mp.setattr(OH, "assemble_dense_h", a)
    orig_s = OH.solve_dense_h

    def s(eta, M, q, eps_b, drives):
        import scipy.linalg
        A = a(eta, M, q, eps_b)
        B = np.stack([O.incident_rhs(M, d) for d in drives], axis=1)
        X = scipy.linalg.solve(A, B)
        shape = (3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
        return np.stack([X[:, k].reshape(shape) for k in range(X.shape[1])])
    mp.setattr(OH, "solve_dense_h", s)


def _m_eps_not_inverse(mp):
    """The image of eps in place of that of 1/eps."""
    mp.setattr(OH, "inverse_box_image", lambda eps, n: O.box_image(eps, n))
    orig = P.smooth_body
    mp.setattr(P, "smooth_body", lambda nmax, grid=48: (orig(nmax, grid)[0], orig(nmax, grid)[0]))


def _m_missing_eps_b(mp):
    orig = OH.assemble_dense_h
    mp.setattr(OH, "assemble_dense_h", lambda eta, M, q, eps_b: orig(eta / eps_b, M, q, eps_b))
    orig_s = OH.solve_dense_h
    mp.setattr(OH, "solve_dense_h", lambda eta, M, q, eps_b, d: orig_s(eta / eps_b, M, q, eps_b, d))


def _m_cross_transposed(mp):
    orig = OH.cross_matrix
    mp.setattr(OH, "cross_matrix", lambda q: np.swapaxes(orig(q), -1, -2) * np.array([1, 1, -1])[:, None])


MUTATIONS = {
    "transposed_toeplitz": _m_transposed,
    "denominator_sign": _m_denominator_sign,
    "eps_for_inverse": _m_eps_not_inverse,
    "missing_eps_b": _m_missing_eps_b,
    "cross_product_rows": _m_cross_transposed,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_hfield_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    assert _any_pin_fails(), f"planted mistake {name} passed every pin"
