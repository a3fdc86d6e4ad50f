"""Adjoint solve and the gradient of the effective tensor (HIP path) against
the CPU oracle: dense A^-H at small order counts, the oracle's forward-mode
(tangent) derivative on sampled voxels, torch.autograd.gradcheck on a tiny
body, and central finite differences of the GPU forward at the 32^3 / M = 12
inverse-design size."""
import numpy as np
import pytest

from gpu_common import asym_body, k_vector, oracle_case, rel_err, say, seeded_field, to_torch
from oracle import grad as OG
from oracle import gsm as O
from paper_1501_01752_amd import inputs

pytestmark = pytest.mark.gpu

TARGET = np.diag([4.0, 5.0, 6.0]).astype(complex)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def G():
    from paper_1501_01752_amd import gsm
    return gsm


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_adjoint_vs_dense(precision):
    gsm = G()
    eps = asym_body()
    period, lam, M = (1.0, 0.9, 1.1), 1 / 0.35, (2, 1, 3)
    k = k_vector(lam, (0.3, 0.4, 0.866))
    inst = gsm.make_instance(lam, k, M, [(1, 0, 0), (0, 1, 0)])
    plan = gsm.Plan(eps, period, M)
    inst.eps_b = plan.basis_eps(inst)
    shape = (2, 3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    rhs = seeded_field(shape, seed=21)
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    say(f"adjoint solve {precision}")
    lam_gpu, info, st = plan.solve_adjoint([inst], to_torch(rhs.ravel()), gsm.default_opts(tol=1e-12, precision=prec))
    assert st == gsm.GSM_OK
    c, q = oracle_case(eps, period, lam, k, M)
    A = O.assemble_dense(c, M, q, inst.eps_b)
    ref = np.linalg.solve(A.conj().T, rhs.reshape(2, -1).T).T
    assert rel_err(lam_gpu.cpu().numpy(), ref.ravel()) <= 1e-10


def _grad_case(v, M, lam=1 / 0.3):
    eps = inputs.smooth_random_field(v, seed=4)
    k = k_vector(lam, (0, 0, 1))
    return eps, k, lam


@pytest.mark.parametrize("v,M", [(8, (2, 2, 2)), (6, (2, 1, 3))])
def test_gradient_vs_tangent_oracle(v, M):
    gsm = G()
    eps, k, lam = _grad_case(v, M)
    plan = gsm.Plan(eps, (1, 1, 1), M)
    inst = gsm.make_instance(lam, k, M)
    inst.eps_b = plan.basis_eps(inst)
    opts = gsm.default_opts(tol=1e-12)
    say(f"eff tensor + vjp V={v} M={M}")
    ee, E, info, st = plan.eff_tensor([inst], opts, save_fields=True)
    gbar = (ee - TARGET[None])
    grad, info2, st2 = plan.eff_tensor_vjp([inst], E, ee, gbar, opts)
    grad = grad.cpu().numpy().ravel()
    rng = np.random.default_rng(5)
    vox = rng.choice(eps.size, 24, replace=False)
    L, ee_ref, g_ref = OG.loss_and_tangent(eps, M, k, lam, (1, 1, 1), inst.eps_b, TARGET, vox)
    assert np.abs(ee[0] - ee_ref).max() <= 1e-9 * np.abs(ee_ref).max()
    assert np.abs(grad[vox] - g_ref).max() <= 1e-8 * np.abs(g_ref).max()


def test_autograd_function_gradcheck():
    import torch
    gsm = G()
    M = (1, 1, 1)
    lam = 1 / 0.3
    eps = torch.tensor(inputs.smooth_random_field(4, seed=9, lo=2.0, hi=5.0), dtype=torch.float64,
                       device="cuda:0", requires_grad=True)
    inst = gsm.make_instance(lam, k_vector(lam, (0.2, 0.1, 0.97)), M)
    inst.eps_b = 3.3
    opts = gsm.default_opts(tol=1e-14, precision=gsm.GSM_FP64)
    fn = gsm.eff_tensor_fn()
    target = torch.tensor(TARGET, device="cuda:0")

    def loss(e):
        ee = fn.apply(e, (1.0, 1.0, 1.0), M, [inst], opts)
        return (ee - target).abs().pow(2).sum()
    say("gradcheck EffTensorFn")
    assert torch.autograd.gradcheck(loss, (eps,), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_inverse_design_gradient_vs_finite_differences():
    """32^3 voxel field in [1, 10], M = 12, three drives: the adjoint gradient
    of ||eps_eff - diag(4, 5, 6)||_F^2 (complex64 + FP64 refinement to 1e-9)
    against central differences (h = 1e-6) on the 64 seeded voxels
    rng(44).choice(32768, 64).  The difference solves run in FP64 to 1e-14
    (warm-started from the base field), so their noise, about
    1e-14 * |L| / h, stays far below the per-voxel gradients.  Per voxel:
    |g_adj - g_fd| <= 1e-4 |g_fd| + 1e-6 max|g_fd|; the absolute floor is that
    FD noise with room, and a relative error of 1e-4 is the finite-difference
    truncation and the adjoint's mixed-precision solve error together."""
    gsm = G()
    M = (12, 12, 12)
    lam = 1 / 0.3
    eps = inputs.smooth_random_field(32, seed=4)
    k = k_vector(lam, (0, 0, 1))
    plan = gsm.Plan(eps, (1, 1, 1), M)
    inst = gsm.make_instance(lam, k, M)
    inst.eps_b = plan.basis_eps(inst)
    opts = gsm.default_opts(tol=1e-9)
    say("inverse design forward + vjp 32^3 M=12")
    ee, E, info, st = plan.eff_tensor([inst], opts, save_fields=True)
    grad, _, _ = plan.eff_tensor_vjp([inst], E, ee, ee - TARGET[None], opts)
    grad = grad.cpu().numpy().ravel()
    vox = np.random.default_rng(44).choice(eps.size, 64, replace=False)
    fd_opts = gsm.default_opts(tol=1e-14, precision=gsm.GSM_FP64)
    fd_opts.x0 = E.data_ptr()  # the base fields (three drives, the solve's layout)
    h = 1e-6
    fd = []
    for j, v in enumerate(vox):
        vals = []
        for sgn in (+1, -1):
            e2 = eps.copy().ravel()
            e2[v] += sgn * h
            p2 = gsm.Plan(e2.reshape(eps.shape), (1, 1, 1), M)
            ee2, _, _, st2 = p2.eff_tensor([inst], fd_opts)
            assert st2 == gsm.GSM_OK
            vals.append(float(np.sum(np.abs(ee2[0] - TARGET) ** 2)))
            p2.close()
        fd.append((vals[0] - vals[1]) / (2 * h))
        if j % 16 == 15:
            say(f"finite differences: {j + 1} of 64 voxels")
    fd = np.array(fd)
    err = np.abs(grad[vox] - fd)
    say(f"max |g_adj - g_fd| / |g_fd| = {np.max(err / np.abs(fd)):.3e}, max|g_fd| = {np.abs(fd).max():.3e}, "
        f"max abs err = {err.max():.3e}")
    assert np.all(err <= 1e-4 * np.abs(fd) + 1e-6 * np.abs(fd).max()), (grad[vox], fd)


def test_repeated_calls_allocate_nothing():
    """Once a plan has its contrast grids and the scheduler its pinned words
    (the first calls), repeated gsm_solve, gsm_eff_tensor (fields kept by the
    caller or left in the workspace) and gsm_eff_tensor_vjp calls make no
    device or pinned-host allocation: every buffer they need is carved from
    the caller's workspace.  The library counts its own allocations.  The
    repeated gradients are bit-identical."""
    gsm = G()
    eps, k, lam = _grad_case(8, (2, 2, 2))
    M = (2, 2, 2)
    plan = gsm.Plan(eps, (1, 1, 1), M)
    inst = gsm.make_instance(lam, k, M)
    inst.eps_b = plan.basis_eps(inst)
    opts = gsm.default_opts(tol=1e-11)
    say("first eff tensor + vjp (plan state is built here)")
    ee, E, _, _ = plan.eff_tensor([inst], opts, save_fields=True)
    g0, _, _ = plan.eff_tensor_vjp([inst], E, ee, ee - TARGET[None], opts)
    plan.solve([inst], opts)
    g0 = g0.cpu().numpy()
    n0 = gsm.allocation_stats()
    for r in range(3):
        say(f"repeated calls {r}")
        ee2, _, _, st = plan.eff_tensor([inst], opts)
        assert st == gsm.GSM_OK and np.array_equal(ee2, ee)
        g, _, _ = plan.eff_tensor_vjp([inst], E, ee, ee - TARGET[None], opts)
        assert np.array_equal(g.cpu().numpy(), g0)
        plan.solve([inst], opts)
    assert gsm.allocation_stats() == n0
