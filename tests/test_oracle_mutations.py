"""Plant plausible mistakes in the CPU oracle (on the CPU, via monkeypatch)
and require that at least one pin catches each of them."""
import numpy as np
import pytest

import oracle_pins as P
from oracle import gsm as O


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


def _m_transposed_toeplitz(mp):
    orig = O.toeplitz
    mp.setattr(O, "toeplitz", lambda c, M: orig(c, M).T)


def _m_green_sign(mp):
    orig = O.green_tensor
    mp.setattr(O, "green_tensor", lambda q, eb: -orig(q, eb))


def _m_green_no_qq(mp):
    def g(q, eb):
        q2 = np.sum(np.asarray(q) ** 2, axis=-1)
        return eb * np.eye(3) / (q2 - eb)[..., None, None]
    mp.setattr(O, "green_tensor", g)


def _m_q_minus(mp):
    orig = O.harmonic_q

    def hq(k_inc, wl, period, M):
        q = orig(k_inc, wl, period, M)
        q0 = np.asarray(k_inc, float) / (2 * np.pi / wl)
        return 2 * q0 - q            # q0 - m K instead of q0 + m K
    mp.setattr(O, "harmonic_q", hq)


def _m_box_conj(mp):
    orig = O._axis_box_factor
    mp.setattr(O, "_axis_box_factor", lambda n, v: np.conj(orig(n, v)))


def _m_d0_wrong_index(mp):
    def d0(c, M, E):
        T0 = O.toeplitz(c, M)[:, O.zero_index(M)]   # c_{m'} instead of c_{-m'}
        return np.array([np.dot(T0, E[k].ravel()) for k in range(3)])
    mp.setattr(O, "displacement_zero_order", d0)


def _m_dropped_delta(mp):
    orig = O.assemble_dense

    def ad(c, M, q, eb):
        n = O.toeplitz(c, M).shape[0]
        G = O.green_tensor(q, eb).reshape(n, 3, 3)
        A = orig(c, M, q, eb)
        for a in range(3):
            for b in range(3):
                A[a * n:(a + 1) * n, b * n:(b + 1) * n] -= np.diag(G[:, a, b])
        return A
    mp.setattr(O, "assemble_dense", ad)


def _m_fft_unscaled(mp):
    orig = O.contrast_convolution_fft
    mp.setattr(O, "contrast_convolution_fft",
               lambda c, M, eb, x, Pp: orig(c, M, eb, x, Pp) * 1.0001)


MUTATIONS = {
    "transposed_toeplitz": _m_transposed_toeplitz,
    "green_sign": _m_green_sign,
    "green_missing_qq": _m_green_no_qq,
    "harmonic_minus": _m_q_minus,
    "box_image_conjugate": _m_box_conj,
    "d0_wrong_index": _m_d0_wrong_index,
    "dropped_delta": _m_dropped_delta,
    "fft_route_scale": _m_fft_unscaled,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    failed = _any_pin_fails()
    assert failed, f"planted mistake {name} passed every pin"
