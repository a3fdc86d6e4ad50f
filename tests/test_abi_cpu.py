"""The C-ABI library loads and exports every symbol include/gsm.h declares;
host-side validation and error codes (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1501_01752_amd import gsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gsm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gsm.lib()
    names = _declared()
    assert "gsm_solve" in names and "gsm_plan" in names and "gsm_eff_tensor" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.gsm_version() == 100


def test_binding_covers_declared_symbols():
    assert set(_declared()) <= set(gsm._SIGS)


def test_solver_opts_layout_matches_the_library():
    """The library's defaults fill exactly the binding's struct: a buffer of
    sentinel bytes larger than the struct keeps its tail, and every field
    reads back the documented default where the binding expects it."""
    L = gsm.lib()
    size = C.sizeof(gsm.SolverOpts)
    buf = (C.c_ubyte * (size + 64))(*([0xA5] * (size + 64)))
    L.gsm_solver_opts_default(C.cast(buf, C.POINTER(gsm.SolverOpts)))
    assert bytes(buf[size:]) == b"\xa5" * 64
    o = gsm.SolverOpts.from_buffer_copy(bytes(buf[:size]))
    assert (o.tol, o.inner_tol, o.restart, o.max_iter, o.max_refine) == (1e-9, 1e-5, 30, 5000, 200)
    assert (o.precision, o.method, o.flags) == (gsm.GSM_MIXED, gsm.GSM_GMRES, 0)
    assert not o.x0 and o.group_max == 32 and o.formulation == gsm.GSM_FORM_E


def test_strerror_and_defaults():
    L = gsm.lib()
    assert L.gsm_strerror(gsm.GSM_E_SINGULAR)
    o = gsm.default_opts()
    assert o.tol == 1e-9 and o.inner_tol == 1e-5 and o.restart == 30
    assert o.precision == gsm.GSM_MIXED


@pytest.mark.parametrize("M,P", [((0, 0, 0), 4), ((1, 1, 1), 8), ((3, 3, 3), 16), ((3, 1, 0), 16),
                                 ((7, 2, 2), 32), ((8, 2, 2), 36), ((1, 9, 0), 40), ((10, 10, 10), 48),
                                 ((0, 0, 11), 48), ((12, 12, 12), 64), ((15, 15, 15), 64), ((16, 6, 6), 72),
                                 ((17, 17, 17), 72), ((18, 0, 0), 128),
                                 ((31, 31, 31), 128), ((32, 0, 0), 256), ((63, 63, 63), 256),
                                 ((2, 64, 1), 512), ((127, 127, 127), 512)])
def test_fft_size(M, P):
    assert gsm.fft_size(M) == P
    assert P >= 4 * max(M) + 1


def test_fft_size_unsupported():
    assert gsm.fft_size((128, 0, 0)) == gsm.GSM_E_UNSUPPORTED


def _geom(eps, period=(1.0, 1.0, 1.0)):
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    g = gsm.Geometry()
    for a in range(3):
        g.period[a] = period[a]
    g.nvox[0], g.nvox[1], g.nvox[2] = eps.shape[2], eps.shape[1], eps.shape[0]
    g.eps = eps.ctypes.data_as(C.POINTER(C.c_double))
    return g, eps


def _popts(m=(3, 3, 3)):
    o = gsm.PlanOpts()
    for a in range(3):
        o.m_max[a] = m[a]
    return o


def _validate(geo=None, po=None, insts=()):
    arr = gsm.instances_array(list(insts)) if insts else None
    return gsm.lib().gsm_plan_validate(C.byref(geo) if geo else None, C.byref(po) if po else None,
                                       len(insts), arr)


def test_validate_ok():
    g, keep = _geom(np.full((4, 4, 4), 2.0))
    inst = gsm.make_instance(1 / 0.3, (0, 0, 2 * np.pi * 0.3), (3, 3, 3))
    assert _validate(g, _popts(), [inst]) == gsm.GSM_OK


def test_validate_nan_voxel():
    e = np.full((4, 4, 4), 2.0)
    e[1, 2, 3] = np.nan
    g, keep = _geom(e)
    assert _validate(g) == gsm.GSM_E_NONFINITE
    assert b"eps" in gsm.lib().gsm_last_error()


def test_validate_bad_sizes():
    g, keep = _geom(np.full((4, 4, 4), 2.0), period=(1.0, -1.0, 1.0))
    assert _validate(g) == gsm.GSM_E_ARG
    assert _validate(None, _popts((128, 0, 0))) == gsm.GSM_E_UNSUPPORTED
    g, keep = _geom(np.full((4, 4, 4), -2.0))
    assert _validate(g) == gsm.GSM_E_ARG


def test_validate_instance_errors():
    g, keep = _geom(np.full((4, 4, 4), 2.0))
    bad = gsm.make_instance(-1.0, (0, 0, 1), (3, 3, 3))
    assert _validate(g, _popts(), [bad]) == gsm.GSM_E_ARG
    big = gsm.make_instance(1.0, (0, 0, 1), (5, 3, 3))
    assert _validate(g, _popts(), [big]) == gsm.GSM_E_ARG
    nod = gsm.make_instance(1.0, (0, 0, 1), (3, 3, 3), drives=[])
    assert _validate(g, _popts(), [nod]) == gsm.GSM_E_ARG


def test_validate_singular_explicit_eps_b():
    # |q_0|^2 = 1 for |k_inc| = k0: eps_b = 1 puts the m = 0 harmonic on the light cone
    g, keep = _geom(np.full((4, 4, 4), 2.0))
    lam = 1 / 0.3
    inst = gsm.make_instance(lam, (0, 0, 2 * np.pi / lam), (3, 3, 3), eps_b=1.0)
    assert _validate(g, _popts(), [inst]) == gsm.GSM_E_SINGULAR
    inst.eps_b = 1.2
    assert _validate(g, _popts(), [inst]) == gsm.GSM_OK


def test_validate_auto_eps_b_dodges_light_cone():
    # uniform vacuum: <eps> = 1 = |q_0|^2, the policy must pick another eps_b
    g, keep = _geom(np.full((4, 4, 4), 1.0))
    lam = 1 / 0.3
    inst = gsm.make_instance(lam, (0, 0, 2 * np.pi / lam), (3, 3, 3))
    assert _validate(g, _popts(), [inst]) == gsm.GSM_OK


def test_profile_sampling_arguments():
    L = gsm.lib()
    assert L.gsm_profile_begin_sampled(b"pass_b", 0) == gsm.GSM_E_ARG
    assert L.gsm_profile_begin_sampled(None, -3) == gsm.GSM_E_ARG
    assert L.gsm_profile_begin_sampled(b"no_such_class", 2) == gsm.GSM_E_ARG
    assert L.gsm_plan_graph_stats(None, None, None) == gsm.GSM_E_ARG


def _brute_margin(lam, k_inc, M, period, eb):
    """min over the truncated harmonic set of | |q_m|^2 - eb |, every harmonic."""
    k0 = 2 * np.pi / lam
    ax = [np.asarray(k_inc[a]) / k0 + np.arange(-M[a], M[a] + 1) * lam / period[a] for a in range(3)]
    q2 = ax[0][None, None, :] ** 2 + ax[1][None, :, None] ** 2 + ax[2][:, None, None] ** 2
    return float(np.abs(q2 - eb).min())


def test_light_cone_check_matches_every_harmonic():
    """The light-cone refusal for an explicit eps_b (|q_m|^2 within 1e-3 eps_b
    of eps_b for some harmonic) against a scan of every harmonic: random
    lattices, directions, order counts and eps_b, plus eps_b placed on a
    shell and just inside and outside the 1e-3 band around it."""
    rng = np.random.default_rng(17)
    checked = 0
    for t in range(300):
        period = tuple(0.3 + 1.5 * rng.random(3))
        M = tuple(int(v) for v in rng.integers(0, 7, 3))
        lam = 0.5 + 4 * rng.random()
        d = rng.normal(size=3)
        if t % 4 == 0:
            d[:2] = 0.0  # normal incidence
        k_inc = (1.0 if t % 3 else 2.5 * rng.random()) * 2 * np.pi / lam * d / np.linalg.norm(d)
        g, keep = _geom(np.full((2, 2, 2), 2.0), period)
        po = _popts(tuple(max(m, 1) for m in M))
        k0 = 2 * np.pi / lam
        m = [int(rng.integers(-M[a], M[a] + 1)) for a in range(3)]
        shell = sum((k_inc[a] / k0 + m[a] * lam / period[a]) ** 2 for a in range(3))
        for eb in (0.3 + 8 * rng.random(), shell, shell * (1 + 0.5e-3), shell * (1 - 2e-3), shell * (1 + 2e-3)):
            if eb <= 0:
                continue
            inst = gsm.make_instance(lam, k_inc, M, eps_b=eb)
            want = gsm.GSM_E_SINGULAR if _brute_margin(lam, k_inc, M, period, eb) < 1e-3 * eb else gsm.GSM_OK
            assert _validate(g, po, [inst]) == want, (t, eb)
            checked += want == gsm.GSM_E_SINGULAR
    assert checked > 300  # the shell cases really hit the band


def _shape_body(shapes, period=(1.0, 1.0, 1.0), eps_host=1.0):
    arr = (gsm.Shape * max(len(shapes), 1))()
    for i, (kind, centre, size, eps) in enumerate(shapes):
        arr[i].kind = kind
        for a in range(3):
            arr[i].centre[a] = centre[a]
            arr[i].size[a] = size[a]
        arr[i].eps = eps
    b = gsm.ShapeBody()
    for a in range(3):
        b.period[a] = period[a]
    b.eps_host, b.n_shapes, b.shapes = eps_host, len(shapes), arr
    return b, arr


def test_shape_plan_argument_errors_without_device():
    """gsm_plan_shapes checks its body before it touches a device."""
    L = gsm.lib()
    h = C.c_void_p()
    ok = (gsm.GSM_SHAPE_SPHERE, (0.5, 0.5, 0.5), (0.3, 0, 0), 4.0)
    for bad, code in [((7, (0.5, 0.5, 0.5), (0.3, 0, 0), 4.0), gsm.GSM_E_ARG),          # kind
                      ((gsm.GSM_SHAPE_SPHERE, (0.5, 0.5, 0.5), (0.6, 0, 0), 4.0), gsm.GSM_E_ARG),  # 1.2 > period
                      ((gsm.GSM_SHAPE_BOX, (0.5, 0.5, 0.5), (0.2, 0.0, 0.2), 4.0), gsm.GSM_E_ARG),  # zero side
                      ((gsm.GSM_SHAPE_ELLIPSOID, (0.5, np.nan, 0.5), (0.2, 0.1, 0.2), 4.0), gsm.GSM_E_NONFINITE),
                      ((gsm.GSM_SHAPE_SPHERE, (0.5, 0.5, 0.5), (0.3, 0, 0), -1.0), gsm.GSM_E_ARG)]:
        b, keep = _shape_body([ok, bad])
        assert L.gsm_plan_shapes(C.byref(b), C.byref(_popts()), C.byref(h)) == code
    b, keep = _shape_body([ok], eps_host=0.0)
    assert L.gsm_plan_shapes(C.byref(b), C.byref(_popts()), C.byref(h)) == gsm.GSM_E_ARG


def test_coefficient_plan_argument_errors_without_device():
    """gsm_plan_from_coeffs refuses too few orders and the image of a
    permittivity that is not real, before it touches a device."""
    from oracle import gsm as O
    L = gsm.lib()
    h = C.c_void_p()
    vox = np.random.default_rng(3).uniform(1, 4, (3, 4, 5))

    def body(c, emin=1.0, emax=4.0):
        c = np.ascontiguousarray(c, dtype=np.complex128)
        b = gsm.CoeffBody()
        b.period[0] = b.period[1] = b.period[2] = 1.0
        b.n_max[0], b.n_max[1], b.n_max[2] = (c.shape[2] - 1) // 2, (c.shape[1] - 1) // 2, (c.shape[0] - 1) // 2
        b.coef = c.ctypes.data_as(C.POINTER(C.c_double))
        b.eps_min, b.eps_max = emin, emax
        return b, c

    b, keep = body(O.box_image(vox, (5, 5, 5)))                       # 5 < 2 m_max = 6
    assert L.gsm_plan_from_coeffs(C.byref(b), C.byref(_popts()), C.byref(h)) == gsm.GSM_E_ARG
    c = O.box_image(vox, (6, 6, 6))
    c[7, 6, 6] += 0.1j                                                 # no longer Hermitian
    b, keep = body(c)
    assert L.gsm_plan_from_coeffs(C.byref(b), C.byref(_popts()), C.byref(h)) == gsm.GSM_E_ARG
    b, keep = body(O.box_image(vox, (6, 6, 6)), emin=3.0, emax=2.0)
    assert L.gsm_plan_from_coeffs(C.byref(b), C.byref(_popts()), C.byref(h)) == gsm.GSM_E_ARG
