"""Plans of analytic shape bodies and of given coefficients (HIP path
through the C ABI) against the CPU oracle: the device's analytic images
against oracle/shapes.py, solves and effective tensors on such plans
against dense LU and the Schur form built from the oracle's images, a
coefficient plan against the voxel plan of the same body, and the refusal
of voxel gradients on plans without voxels."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import k_vector, say
from oracle import gsm as O
from oracle import shapes as OS
from paper_1501_01752_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def G():
    from paper_1501_01752_amd import gsm
    return gsm


MIXED_BODY = {
    "period": (1.0, 0.9, 1.2),
    "eps_host": 1.5,
    "shapes": [
        {"kind": "sphere", "centre": (0.3, 0.35, 0.4), "size": 0.2, "eps": 6.0},
        {"kind": "ellipsoid", "centre": (0.72, 0.6, 0.85), "size": (0.15, 0.12, 0.2), "eps": 3.0},
        {"kind": "box", "centre": (0.75, 0.2, 0.3), "size": (0.12, 0.08, 0.1), "eps": 9.0},
    ],
}

FIG3_BODY = {  # air spheres of radius 0.125 lambda in n = 1.5 at Lambda = 0.3 lambda
    "period": (1.0, 1.0, 1.0),
    "eps_host": 2.25,
    "shapes": [{"kind": "sphere", "centre": (0.5, 0.5, 0.5), "size": 0.125 / 0.3, "eps": 1.0}],
}


@pytest.mark.parametrize("name,mmax", [("mixed", (4, 3, 5)), ("mixed", (15, 15, 15)), ("fig3", (6, 6, 6))])
def test_shape_coefficients(name, mmax):
    body = MIXED_BODY if name == "mixed" else FIG3_BODY
    say(f"shape plan coefficients {name} m_max={mmax}")
    plan = G().Plan.from_shapes(body["period"], body["eps_host"], body["shapes"], mmax)
    got = plan.coefficients()
    ref = OS.shape_image(body["period"], body["eps_host"], body["shapes"], tuple(2 * m for m in mmax))
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shape_plan_solve_vs_dense(precision):
    gsm = G()
    body = MIXED_BODY
    M = (3, 3, 3)
    lam = 1 / 0.35
    k = k_vector(lam, (0.2, -0.3, 1.0))
    say(f"shape plan solve {precision}")
    plan = gsm.Plan.from_shapes(body["period"], body["eps_host"], body["shapes"], M)
    inst = gsm.make_instance(lam, k, M, [(1.0, 0.0, 0.0), (0.0, 0.6, 0.8j)])
    inst.eps_b = plan.basis_eps(inst)
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    E, info, st = plan.solve([inst], gsm.default_opts(tol=1e-12, precision=prec))
    assert st == gsm.GSM_OK
    c = OS.shape_image(body["period"], body["eps_host"], body["shapes"], (6, 6, 6))
    q = O.harmonic_q(k, lam, body["period"], M)
    ref = O.solve_dense(c, M, q, inst.eps_b, [np.array([1.0, 0, 0]), np.array([0, 0.6, 0.8j])]).ravel()
    got = E.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    plan.close()


def test_shape_plan_eff_tensor_vs_schur():
    """Fig. 3's lattice (air spheres, r = 0.125 lambda, n = 1.5 host,
    Lambda = 0.3 lambda) at k = n k0 z: the effective tensor from the
    device's analytic image against the Schur form of the oracle's."""
    gsm = G()
    body = FIG3_BODY
    M = (4, 4, 4)
    lam = 1 / 0.3
    k = k_vector(lam, (0, 0, 1), n_inc=1.4)
    say("shape plan eff tensor")
    plan = gsm.Plan.from_shapes(body["period"], body["eps_host"], body["shapes"], M)
    inst = gsm.make_instance(lam, k, M)
    ee, _, info, st = plan.eff_tensor([inst], gsm.default_opts(tol=1e-12, precision=gsm.GSM_FP64))
    assert st == gsm.GSM_OK
    c = OS.shape_image(body["period"], body["eps_host"], body["shapes"], (8, 8, 8))
    ref = O.eps_eff_schur(c, M, O.harmonic_q(k, lam, body["period"], M))
    assert np.abs(ee[0] - ref).max() <= 1e-10 * np.abs(ref).max()
    # cubic symmetry with k || z: eps_xx = eps_yy, no off-diagonal terms
    assert abs(ee[0][0, 0] - ee[0][1, 1]) <= 1e-10 * abs(ee[0][0, 0])
    assert np.abs(ee[0] - np.diag(np.diag(ee[0]))).max() <= 1e-10 * abs(ee[0][0, 0])
    plan.close()


def test_coefficient_plan_equals_voxel_plan():
    """The oracle's voxel image handed over as coefficients gives the voxel
    plan's solution (the two images agree to rounding)."""
    gsm = G()
    w = inputs.sphere_lattice_small()
    M = w["M"]
    k = k_vector(w["wavelength"], (0.3, 0.0, 1.0))
    c = O.box_image(w["eps"], tuple(2 * m + 1 for m in M))   # one more order than needed
    say("coefficient plan vs voxel plan")
    pc = gsm.Plan.from_coeffs(w["period"], c, float(w["eps"].min()), float(w["eps"].max()), M)
    pv = gsm.Plan(w["eps"], w["period"], M)
    got_c = pc.coefficients()
    inner = c[1:-1, 1:-1, 1:-1]
    assert np.array_equal(got_c, inner)
    inst = gsm.make_instance(w["wavelength"], k, M)
    # the two plans' mean permittivities (c_0 against the voxel sum) agree
    # to rounding; the same basis permittivity is given to both
    assert abs(pc.basis_eps(inst) - pv.basis_eps(inst)) <= 1e-14 * pv.basis_eps(inst)
    inst.eps_b = pv.basis_eps(inst)
    opts = gsm.default_opts(tol=1e-12, precision=gsm.GSM_FP64)
    Ec, _, st1 = pc.solve([inst], opts)
    Ev, _, st2 = pv.solve([inst], opts)
    assert st1 == st2 == gsm.GSM_OK
    a, b = Ec.cpu().numpy(), Ev.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()
    pc.close()
    pv.close()


def test_voxel_gradient_refused_without_voxels():
    import torch
    gsm = G()
    body = FIG3_BODY
    M = (2, 2, 2)
    plan = gsm.Plan.from_shapes(body["period"], body["eps_host"], body["shapes"], M)
    inst = gsm.make_instance(1 / 0.3, k_vector(1 / 0.3, (0, 0, 1)), M)
    say("vjp refused on a shape plan")
    ee, E, info, st = plan.eff_tensor([inst], gsm.default_opts(tol=1e-10), save_fields=True)
    arr = gsm.instances_array([inst])
    opts = gsm.default_opts(tol=1e-10)
    ws = plan.workspace([inst], opts)
    grad = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    gb = np.eye(3, dtype=np.complex128)
    info = (gsm.SolveInfo * 3)()
    st = gsm.lib().gsm_eff_tensor_vjp(plan.handle, 1, arr, C.byref(opts), C.c_void_p(E.data_ptr()),
                                      ee.ctypes.data_as(C.c_void_p), gb.ctypes.data_as(C.c_void_p),
                                      C.c_void_p(grad.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                      info, None)
    assert st == gsm.GSM_E_ARG
    assert float(grad.abs().max()) == 0.0
    plan.close()
