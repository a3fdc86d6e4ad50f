"""BiCGStab route of the HIP solver against the CPU oracle: the same field
as the dense LU solution at small order counts (FP64 and mixed precision,
forward and adjoint), the full-size layered stack against the exact 1D
reduction, and the argument check on the Krylov storage it needs."""
import numpy as np
import pytest

from gpu_common import asym_body, k_vector, oracle_case, rel_err, say, seeded_field, to_torch
from oracle import gsm as O
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


def _opts(gsm, **kw):
    kw.setdefault("method", gsm.GSM_BICGSTAB)
    kw.setdefault("restart", 5)
    return gsm.default_opts(**kw)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bicgstab_sphere_m3_vs_dense_lu(precision):
    gsm = G()
    w = inputs.sphere_lattice_small()
    k = k_vector(w["wavelength"], w["k_hat"])
    drives = [(1, 0, 0), (0, 0.3, 1j)]
    inst = gsm.make_instance(w["wavelength"], k, w["M"], drives)
    plan = gsm.Plan(w["eps"], w["period"], w["M"])
    inst.eps_b = plan.basis_eps(inst)
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    say(f"bicgstab sphere M=3 {precision}")
    E, info, st = plan.solve([inst], _opts(gsm, tol=1e-12, precision=prec))
    assert st == gsm.GSM_OK and all(i["rel_residual"] <= 1e-12 for i in info)
    c, q = oracle_case(w["eps"], w["period"], w["wavelength"], k, w["M"])
    ref = O.solve_dense(c, w["M"], q, inst.eps_b, [np.array(a, complex) for a in drives])
    assert rel_err(E.cpu().numpy(), ref.ravel()) <= 1e-10
    # two operator applications per iteration
    assert all(i["iterations"] % 2 == 0 and i["iterations"] > 0 for i in info)


def test_bicgstab_oblique_aniso_batch_vs_dense_lu():
    """Uneven batch (two order-count groups), oblique incidence, mixed precision."""
    gsm = G()
    eps = asym_body()
    period = (1.0, 0.9, 1.1)
    plan = gsm.Plan(eps, period, (3, 3, 3))
    cases = [(1 / 0.35, (0.3, 0.4, 0.866), (2, 3, 1), (0.2, 1.0, -0.4j)),
             (1 / 0.3, (1, 0, 0), (3, 3, 3), (0, 1, 0)),
             (1 / 0.35, (0.6, 0, 0.8), (2, 3, 1), (0, 1, 0.5))]
    insts = []
    for lam, kh, M, a in cases:
        inst = gsm.make_instance(lam, k_vector(lam, kh), M, [a])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
    say("bicgstab uneven batch of 3")
    E, info, st = plan.solve(insts, _opts(gsm, tol=1e-11))
    assert st == gsm.GSM_OK
    E = E.cpu().numpy()
    off = 0
    for inst, (lam, kh, M, a) in zip(insts, cases):
        c, q = oracle_case(eps, period, lam, k_vector(lam, kh), M)
        ref = O.solve_dense(c, M, q, inst.eps_b, [np.array(a, complex)]).ravel()
        assert rel_err(E[off:off + ref.size], ref) <= 1e-9
        off += ref.size


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bicgstab_adjoint_vs_dense(precision):
    gsm = G()
    eps = asym_body()
    period, lam, M = (1.0, 0.9, 1.1), 1 / 0.35, (2, 1, 3)
    k = k_vector(lam, (0.3, 0.4, 0.866))
    inst = gsm.make_instance(lam, k, M, [(1, 0, 0), (0, 1, 0)])
    plan = gsm.Plan(eps, period, M)
    inst.eps_b = plan.basis_eps(inst)
    shape = (2, 3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    rhs = seeded_field(shape, seed=23)
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    say(f"bicgstab adjoint solve {precision}")
    lam_gpu, info, st = plan.solve_adjoint([inst], to_torch(rhs.ravel()), _opts(gsm, tol=1e-12, precision=prec))
    assert st == gsm.GSM_OK
    c, q = oracle_case(eps, period, lam, k, M)
    A = O.assemble_dense(c, M, q, inst.eps_b)
    ref = np.linalg.solve(A.conj().T, rhs.reshape(2, -1).T).T
    assert rel_err(lam_gpu.cpu().numpy(), ref.ravel()) <= 1e-10


def test_bicgstab_trivial_contrast():
    """Uniform eps = eps_b: A = I, one iteration reaches the exact field."""
    gsm = G()
    lam = 1 / 0.3
    a = np.array([0.3, -0.5, 0.8])
    inst = gsm.make_instance(lam, k_vector(lam, (0, 0, 1)), (3, 3, 3), [tuple(a)])
    inst.eps_b = 2.0
    plan = gsm.Plan(np.full((8, 8, 8), 2.0), (1, 1, 1), (3, 3, 3))
    say("bicgstab uniform eps = eps_b")
    E, info, st = plan.solve([inst], _opts(gsm, tol=1e-13))
    assert st == gsm.GSM_OK and info[0]["iterations"] <= 4
    ref = O.incident_rhs((3, 3, 3), a)
    assert np.abs(E.cpu().numpy() - ref).max() <= 1e-13


def test_bicgstab_stack_m15_vs_1d_reduction():
    """Full-size layered stack (31^3 harmonics, 64^3 grid), mixed precision."""
    gsm = G()
    w = inputs.layered_stack_m15()
    k = k_vector(w["wavelength"], w["k_hat"])
    inst = gsm.make_instance(w["wavelength"], k, w["M"], w["drives"])
    plan = gsm.Plan(w["eps"], w["period"], w["M"])
    inst.eps_b = plan.basis_eps(inst)
    say("bicgstab cfg2 stack M=15 mixed")
    E, info, st = plan.solve([inst], _opts(gsm, tol=1e-11))
    assert st == gsm.GSM_OK
    E = E.cpu().numpy()
    M = w["M"]
    c1 = O.box_image(w["eps"], (0, 0, 30))[:, 0, 0]
    n = E.size // 2
    for d, a in enumerate(w["drives"]):
        Ed = E[d * n:(d + 1) * n].reshape(3, 31, 31, 31)
        ref = O.solve_stack_1d(c1, 15, k / (2 * np.pi / w["wavelength"]), w["wavelength"], inst.eps_b,
                               np.array(a, complex))
        assert rel_err(Ed[:, :, M[1], M[0]], ref) <= 1e-9


def test_bicgstab_needs_six_vectors():
    gsm = G()
    w = inputs.sphere_lattice_small()
    inst = gsm.make_instance(w["wavelength"], k_vector(w["wavelength"], w["k_hat"]), w["M"], [(1, 0, 0)])
    plan = gsm.Plan(w["eps"], w["period"], w["M"])
    inst.eps_b = plan.basis_eps(inst)
    say("bicgstab restart=4 rejected")
    with pytest.raises(gsm.GsmError) as e:
        plan.solve([inst], _opts(gsm, restart=4))
    assert e.value.status == gsm.GSM_E_ARG
