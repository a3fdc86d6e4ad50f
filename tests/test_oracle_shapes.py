"""The analytic-image oracle against quadrature, exact voxel images and
convergence (no GPU), and planted mistakes that these pins must catch."""
import numpy as np
import pytest

import shape_pins as P
from oracle import shapes as S


@pytest.mark.parametrize("name", sorted(P.ALL))
def test_shape_pin(name):
    fn, tol = P.ALL[name]
    err = fn()
    assert err <= tol, f"{name}: {err:.3e} > {tol:.0e}"


def test_hermitian_symmetry():
    """A real permittivity has c_{-n} = conj(c_n)."""
    shapes = [{"kind": "ellipsoid", "centre": (0.3, 0.6, 0.2), "size": (0.2, 0.15, 0.1), "eps": 7.0},
              {"kind": "box", "centre": (0.7, 0.2, 0.7), "size": (0.1, 0.1, 0.2), "eps": 3.0}]
    c = S.shape_image((1.0, 0.9, 1.1), 1.5, shapes, (4, 5, 3))
    assert np.abs(c - np.conj(c[::-1, ::-1, ::-1])).max() < 1e-15


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


def _m_phase_sign(mp):
    orig = S.shape_factor

    def f(shape, period, n_max):
        s = dict(shape)
        s["centre"] = tuple(-np.asarray(shape["centre"], float))
        return orig(s, period, n_max)
    mp.setattr(S, "shape_factor", f)


def _m_diameter(mp):
    orig = S.shape_factor

    def f(shape, period, n_max):
        s = dict(shape)
        if s["kind"] != "box":
            s["size"] = 2 * np.asarray(s["size"], float)
        return orig(s, period, n_max)
    mp.setattr(S, "shape_factor", f)


def _m_ball_j1_no_3(mp):
    mp.setattr(S, "_ball_factor", lambda u: np.where(np.asarray(u) > 0, 1.0, 1.0) *
               np.where(np.asarray(u) > 0, np.sinc(np.asarray(u) / np.pi), 1.0))


def _m_sinc_unscaled(mp):
    mp.setattr(S, "_sinc", lambda x: np.sinc(np.asarray(x, float)))


def _m_box_full_sides(mp):
    orig = S.shape_factor

    def f(shape, period, n_max):
        s = dict(shape)
        if s["kind"] == "box":
            s["size"] = tuple(0.5 * np.asarray(s["size"], float))
        return orig(s, period, n_max)
    mp.setattr(S, "shape_factor", f)


def _m_no_two_pi(mp):
    orig = S.reciprocal_vectors
    mp.setattr(S, "reciprocal_vectors",
               lambda period, n_max: tuple(g / (2 * np.pi) for g in orig(period, n_max)))


def _m_inverse_ignored(mp):
    orig = S.shape_image
    mp.setattr(S, "shape_image", lambda period, eh, shapes, n_max, inverse=False:
               orig(period, eh, shapes, n_max, inverse=False))


def _m_axes_swapped(mp):
    orig = S.reciprocal_vectors

    def rv(period, n_max):
        gx, gy, gz = orig(period, n_max)
        return gx, gy, gz * 0 + np.moveaxis(gz, 0, 0)[::-1]   # harmonic order of z reversed
    mp.setattr(S, "reciprocal_vectors", rv)


MUTATIONS = {
    "phase_sign": _m_phase_sign,
    "diameter_for_radius": _m_diameter,
    "ball_factor": _m_ball_j1_no_3,
    "sinc_scaled_by_pi": _m_sinc_unscaled,
    "box_full_sides": _m_box_full_sides,
    "no_two_pi": _m_no_two_pi,
    "inverse_ignored": _m_inverse_ignored,
    "z_orders_reversed": _m_axes_swapped,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_shape_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    assert _any_pin_fails(), f"planted mistake {name} passed every pin"
