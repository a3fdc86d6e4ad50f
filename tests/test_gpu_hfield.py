"""The H-field system of Eq.(5) (HIP path through the C ABI) against the
CPU oracle: the images of 1/eps, the operator (FP64 and FP32) at several FFT
grids and order counts, solves against dense LU and the FFT-GMRES route, the
pole search on the H system against the oracle's, and the agreement of the E
and H systems' effective index at 31^3 harmonics."""
import numpy as np
import pytest

from gpu_common import asym_body, k_vector, oracle_P, rel_err, say, seeded_field, to_torch
from oracle import gsm as O
from oracle import hfield as OH
from oracle import poles as OP
from oracle import shapes as OS
from paper_1501_01752_amd import inputs

import pole_pins as PP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def G():
    from paper_1501_01752_amd import gsm
    return gsm


def test_inverse_coefficients_voxels_and_shapes():
    gsm = G()
    eps = asym_body()
    mmax = (2, 3, 1)
    say("inverse coefficients")
    plan = gsm.Plan(eps, (1.0, 0.9, 1.1), mmax)
    ref = OH.inverse_box_image(eps, tuple(2 * m for m in mmax))
    assert np.abs(plan.inverse_coefficients() - ref).max() <= 1e-13 * np.abs(ref).max()
    plan.close()
    shapes = [{"kind": "sphere", "centre": (0.5, 0.5, 0.5), "size": 0.3, "eps": 6.0},
              {"kind": "box", "centre": (0.1, 0.15, 0.2), "size": (0.05, 0.1, 0.08), "eps": 2.0}]
    plan = gsm.Plan.from_shapes((1.0, 1.0, 1.0), 1.5, shapes, (4, 4, 4))
    ref = OS.shape_image((1.0, 1.0, 1.0), 1.5, shapes, (8, 8, 8), inverse=True)
    assert np.abs(plan.inverse_coefficients() - ref).max() <= 1e-13 * np.abs(ref).max()
    plan.close()


APPLY_CASES = {
    "asym_m231": (asym_body, (1.0, 0.9, 1.1), (2, 3, 1), 1.7, (0.3, -0.2, 1.0)),
    "sphere_m7": (lambda: inputs.sphere(16, 0.3, 4.0), (1.0, 1.0, 1.0), (7, 7, 7), 1 / 0.3, (0.0, 0.0, 1.0)),
    "random_m12": (lambda: inputs.smooth_random_field(16, seed=4), (1.0, 1.0, 1.0), (12, 5, 9), 1 / 0.3,
                   (0.2, 0.4, 1.0)),
    "ellipsoid_m16": (lambda: inputs.ellipsoid((32, 32, 32), (1.0, 0.8, 1.2), (0.35, 0.25, 0.15), 6.0),
                      (1.0, 0.8, 1.2), (16, 4, 3), 2.5, (0.5, 0.1, 0.8)),
}


@pytest.mark.parametrize("name", sorted(APPLY_CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_h_matches_oracle(name, precision):
    gsm = G()
    mk, period, M, lam, kh = APPLY_CASES[name]
    eps = mk()
    k = k_vector(lam, kh)
    plan = gsm.Plan(eps, period, M)
    inst = gsm.make_instance(lam, k, M, [(1.0, 0, 0), (0, 1.0, 0)])
    eb = plan.basis_eps(inst)
    inst.eps_b = eb
    shape = (3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    x = seeded_field((2,) + shape, 31)
    say(f"apply H {name} {precision} M={M} P={gsm.fft_size(M)}")
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    xt = to_torch(x.ravel() if precision == "fp64" else x.ravel().astype(np.complex64))
    y = plan.apply([inst], xt, precision=prec, mode=gsm.GSM_APPLY_FORWARD_H).cpu().numpy()
    y = y.astype(np.complex128).reshape((2,) + shape)
    eta = OH.inverse_box_image(eps, tuple(2 * m for m in M))
    q = O.harmonic_q(k, lam, period, M)
    for d in range(2):
        xd = x[d] if precision == "fp64" else x[d].astype(np.complex64).astype(np.complex128)
        ref = OH.apply_operator_fft_h(eta, M, q, eb, xd, oracle_P(M)).reshape(shape)
        tol = 1e-13 if precision == "fp64" else 1e-6
        assert rel_err(y[d], ref) <= tol, rel_err(y[d], ref)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_h_vs_dense(precision):
    gsm = G()
    w = inputs.sphere_lattice_small()
    M = w["M"]
    lam = w["wavelength"]
    k = k_vector(lam, (0.3, 0.1, 1.0))
    plan = gsm.Plan(w["eps"], w["period"], M)
    a1 = np.cross(k / np.linalg.norm(k), [1.0, 0.0, 0.0])
    inst = gsm.make_instance(lam, k, M, [tuple(a1), (0.2, 1.0, 0.1j)])
    inst.eps_b = plan.basis_eps(inst)
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    say(f"solve H vs dense {precision}")
    H, info, st = plan.solve([inst], gsm.default_opts(tol=1e-12, precision=prec, formulation=gsm.GSM_FORM_H))
    assert st == gsm.GSM_OK
    eta = OH.inverse_box_image(w["eps"], tuple(2 * m for m in M))
    q = O.harmonic_q(k, lam, w["period"], M)
    ref = OH.solve_dense_h(eta, M, q, inst.eps_b, [a1, np.array([0.2, 1.0, 0.1j])]).ravel()
    assert rel_err(H.cpu().numpy(), ref) <= 1e-10
    plan.close()


def test_solve_h_m8_vs_fft_gmres_oracle():
    """17^3 harmonics (P = 64 on the device, 36 in the oracle), oblique
    incidence on the 64^3-voxel sphere lattice, mixed precision."""
    gsm = G()
    w = inputs.sphere_lattice_m15()
    M = (8, 8, 8)
    lam = w["wavelength"]
    k = k_vector(lam, (0.2, -0.3, 1.0))
    plan = gsm.Plan(w["eps"], w["period"], M)
    a = np.cross(k / np.linalg.norm(k), [0.0, 1.0, 0.0])
    inst = gsm.make_instance(lam, k, M, [tuple(a)])
    inst.eps_b = plan.basis_eps(inst)
    say("solve H M=8 vs FFT-GMRES oracle")
    H, info, st = plan.solve([inst], gsm.default_opts(tol=1e-11, formulation=gsm.GSM_FORM_H))
    assert st == gsm.GSM_OK and info[0]["rel_residual"] <= 1e-11
    eta = OH.inverse_box_image(w["eps"], tuple(2 * m for m in M))
    q = O.harmonic_q(k, lam, w["period"], M)
    ref, code = OH.solve_fft_gmres_h(eta, M, q, inst.eps_b, a, oracle_P(M), rtol=1e-12)
    assert code == 0
    assert rel_err(H.cpu().numpy(), ref.ravel()) <= 1e-9
    plan.close()


def test_pole_search_h_matches_oracle_at_m3():
    """The pole search on Eq.(5), xi = the y component of the zeroth H
    order under a y drive (k || z), against the oracle's dense H solves and
    fit."""
    gsm = G()
    M = (3, 3, 3)
    vox, period, lam = PP.fig2_case(M)
    k0 = 2 * np.pi / lam
    plan = gsm.Plan(vox, period, M)
    q = gsm.make_pole_query(lam, (0, 0, 1), M, 1.30 * k0, 1.60 * k0, drive=(0, 1, 0), component=1, eps_b=3.5)
    say("pole search H fig2 M=3")
    res, st = plan.pole_search([q], gsm.default_opts(tol=1e-12, precision=gsm.GSM_FP64,
                                                     formulation=gsm.GSM_FORM_H))
    r = res[0]
    assert st == gsm.GSM_OK and r["best"] >= 0
    kap = OP.kappa_mesh(1.30 * k0, 1.60 * k0, 5, 10)
    eta = OH.inverse_box_image(vox, tuple(2 * m for m in M))
    xi = []
    for kk in kap:
        qh = O.harmonic_q(np.array([0.0, 0.0, kk]), lam, period, M)
        Hs = OH.solve_dense_h(eta, M, qh, 3.5, [np.array([0.0, 1.0, 0.0])])[0]
        xi.append(Hs.reshape(3, -1)[1, O.zero_index(M)])
    e_ref, z_ref = OP.pole_search(kap, np.array(xi), 5, 10)
    j = OP.dominant_pole(e_ref, z_ref, kap[0], kap[-1])
    assert abs(r["eta"][r["best"]] - e_ref[j]) <= 1e-9 * abs(e_ref[j])
    plan.close()


def test_e_and_h_effective_index_agree_m15():
    """Fig. 2's lattice (n = 1.5 host) at 31^3 harmonics: the E and H
    systems' poles agree to the truncation error (the paper's Fig. 2 shows
    both converging to one index)."""
    gsm = G()
    M = (15, 15, 15)
    vox, period, lam = PP.fig2_case(M)
    k0 = 2 * np.pi / lam
    plan = gsm.Plan(vox, period, M)
    qe = gsm.make_pole_query(lam, (0, 0, 1), M, 1.36 * k0, 1.52 * k0)
    qh = gsm.make_pole_query(lam, (0, 0, 1), M, 1.36 * k0, 1.52 * k0, drive=(0, 1, 0), component=1)
    say("E and H poles M=15")
    re_, st1 = plan.pole_search([qe], gsm.default_opts(tol=1e-10))
    rh_, st2 = plan.pole_search([qh], gsm.default_opts(tol=1e-10, formulation=gsm.GSM_FORM_H))
    ne, nh = re_[0]["n_eff"], rh_[0]["n_eff"]
    assert re_[0]["best"] >= 0 and rh_[0]["best"] >= 0
    assert abs(ne - nh) <= 5e-3, (ne, nh)
    assert abs(ne - 1.441688) <= 3e-3 and abs(nh - 1.441688) <= 5e-3, (ne, nh)
    plan.close()


def test_h_refusals():
    gsm = G()
    w = inputs.sphere_lattice_small()
    M = w["M"]
    plan = gsm.Plan(w["eps"], w["period"], M)
    inst = gsm.make_instance(w["wavelength"], k_vector(w["wavelength"], (0, 0, 1)), M)
    say("H refusals")
    with pytest.raises(gsm.GsmError) as e:
        plan.eff_tensor([inst], gsm.default_opts(formulation=gsm.GSM_FORM_H))
    assert e.value.status == gsm.GSM_E_ARG
    c = O.box_image(w["eps"], tuple(2 * m for m in M))
    pc = gsm.Plan.from_coeffs(w["period"], c, 1.0, 4.0, M)   # no coefficients of 1/eps
    with pytest.raises(gsm.GsmError) as e:
        pc.solve([inst], gsm.default_opts(formulation=gsm.GSM_FORM_H))
    assert e.value.status == gsm.GSM_E_ARG
    pc.close()
    plan.close()
