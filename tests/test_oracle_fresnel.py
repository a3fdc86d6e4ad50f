"""The Fresnel normal-surface oracle against closed forms of crystal optics
(no GPU), and planted mistakes those pins must catch."""
import numpy as np
import pytest

import fresnel_pins as P
from oracle import fresnel as F


@pytest.mark.parametrize("name", sorted(P.ALL))
def test_fresnel_pin(name):
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


def _m_projector_plus(mp):
    """I + k k^T instead of I - k k^T."""
    def proj(k_hat):
        k = np.asarray(k_hat, dtype=np.float64)
        k = k / np.linalg.norm(k)
        return np.eye(3) + np.outer(k, k)
    mp.setattr(F, "projector", proj)


def _m_unnormalised_direction(mp):
    mp.setattr(F, "projector", lambda k_hat: np.eye(3) - np.outer(k_hat, k_hat) * 0.81)


def _m_indices_are_squares(mp):
    """n^2 reported as n."""
    def ind(eps, k_hat):
        c2, c1, c0 = F.normal_polynomial(eps, k_hat)
        return np.sort(np.roots([c2, c1, c0]).real)
    mp.setattr(F, "indices", ind)


def _m_inverse_tensor(mp):
    """The impermeability eps^-1 put where eps belongs."""
    orig = F.normal_polynomial
    mp.setattr(F, "normal_polynomial", lambda eps, k_hat: orig(np.linalg.inv(eps), k_hat))


def _m_transposed_offdiagonal(mp):
    """Off-diagonal fit parameters written into the wrong slots."""
    def eps_of(p, diagonal):
        if diagonal:
            return np.diag(p)
        e = np.diag(p[:3]).astype(float)
        e[0, 1] = e[1, 0] = p[5]
        e[0, 2] = e[2, 0] = p[3]
        e[1, 2] = e[2, 1] = p[4]
        return e
    orig_fit = F.fit

    def fit(k_hats, n_pairs, diagonal=False):
        got, rms = orig_fit(k_hats, n_pairs, diagonal)
        if diagonal:
            return got, rms
        p = np.array([got[0, 0], got[1, 1], got[2, 2], got[0, 1], got[0, 2], got[1, 2]])
        return eps_of(p, False), rms
    mp.setattr(F, "fit", fit)


MUTATIONS = {
    "projector_plus": _m_projector_plus,
    "unnormalised_direction": _m_unnormalised_direction,
    "indices_are_squares": _m_indices_are_squares,
    "inverse_tensor": _m_inverse_tensor,
    "transposed_offdiagonal": _m_transposed_offdiagonal,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_fresnel_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    assert _any_pin_fails(), f"planted mistake {name} passed every pin"
