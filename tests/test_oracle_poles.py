"""The pole-search oracle against test functions with known poles, the
singular operator at a found pole, the residue as a limit and the paper's
Fig. 2 index (no GPU), and planted mistakes these pins must catch."""
import numpy as np
import pytest

import pole_pins as P
from oracle import poles as OP


@pytest.mark.parametrize("name", sorted(P.ALL))
def test_pole_pin(name):
    fn, tol = P.ALL[name]
    err = fn()
    assert err <= tol, f"{name}: {err:.3e} > {tol:.0e}"


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


def _m_xi_in_denominator(mp):
    """Eq.(9) as printed: xi_i in the denominator."""
    orig = OP.polynomial_coefficients
    mp.setattr(OP, "polynomial_coefficients",
               lambda kappa, xi, n_poles, n_div: orig(kappa, 1.0 / np.asarray(xi), n_poles, n_div))


def _m_rhs_sign(mp):
    orig = OP.polynomial_coefficients

    def pc(kappa, xi, n_poles, n_div):
        # solve with the right-hand side's sign flipped: p -> the coefficients
        # of a different monic polynomial
        return -orig(kappa, xi, n_poles, n_div) - 2 * np.eye(1, n_poles, 0)[0]
    mp.setattr(OP, "polynomial_coefficients", pc)


def _m_companion_reversed(mp):
    orig = OP.companion_roots
    mp.setattr(OP, "companion_roots", lambda p: orig(np.asarray(p)[::-1]))


def _m_residue_no_poly(mp):
    def res(kappa, xi, eta):
        kappa = np.asarray(kappa, complex)
        out = []
        for k in range(len(eta)):
            lag = np.array([np.prod([(eta[k] - kappa[j]) / (kappa[i] - kappa[j])
                                     for j in range(len(kappa)) if j != i]) for i in range(len(kappa))])
            den = np.prod([eta[k] - eta[i] for i in range(len(eta)) if i != k])
            out.append(np.sum(np.asarray(xi) * lag) / den)      # P(kappa_i) dropped
        return np.array(out)
    mp.setattr(OP, "residues", res)


def _m_weights_unsigned(mp):
    orig = OP.divided_difference_weights
    mp.setattr(OP, "divided_difference_weights", lambda kappa: np.abs(orig(kappa)))


def _m_one_window(mp):
    """Every row from the first window (a singular or meaningless system)."""
    def pc(kappa, xi, n_poles, n_div):
        kappa = np.asarray(kappa, complex)
        xi = np.asarray(xi, complex)
        A = np.zeros((n_poles, n_poles), complex)
        rhs = np.zeros(n_poles, complex)
        for s in range(n_poles):
            kk = kappa[:n_div + 1]
            wx = OP.divided_difference_weights(kk) * xi[:n_div + 1] * (1 + 1e-3 * s)
            for k in range(n_poles):
                A[s, k] = np.sum(kk ** k * wx)
            rhs[s] = -np.sum(kk ** n_poles * wx)
        return np.linalg.lstsq(A, rhs, rcond=None)[0]
    mp.setattr(OP, "polynomial_coefficients", pc)


MUTATIONS = {
    "xi_in_denominator": _m_xi_in_denominator,
    "rhs_sign": _m_rhs_sign,
    "companion_reversed": _m_companion_reversed,
    "residue_without_P": _m_residue_no_poly,
    "weights_unsigned": _m_weights_unsigned,
    "single_window": _m_one_window,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pole_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    assert _any_pin_fails(), f"planted mistake {name} passed every pin"
