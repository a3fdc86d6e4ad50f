"""Launch graphs of the GMRES cycle (HIP path).

A solve whose Arnoldi steps run as captured launch graphs must equal, bit
for bit, the same solve issued as separate launches (the graphs hold the
same kernels with the same arguments), on the first call (capture) and on
every later call that replays the cached graphs, with other GPU work and
synchronisations in between; and it must match the CPU oracle.  Separate
launches are used without GSM_SOLVE_GRAPH, for BiCGStab and while launches
are being timed.
"""
import numpy as np
import pytest

from gpu_common import asym_body, k_vector, oracle_case, rel_err, say
from oracle import gsm as O
from paper_1501_01752_amd import inputs

pytestmark = pytest.mark.gpu

PERIOD = (1.0, 0.9, 1.1)
CASES = [(1 / 0.35, (0.3, 0.4, 0.866), (2, 3, 1), (0.2, 1.0, -0.4j)),
         (1 / 0.3, (1, 0, 0), (3, 3, 3), (0, 1, 0)),
         (1 / 0.35, (0.6, 0, 0.8), (2, 3, 1), (0, 1, 0.5))]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def G():
    from paper_1501_01752_amd import gsm
    return gsm


def _batch(gsm, plan):
    insts = []
    for lam, kh, M, a in CASES:
        inst = gsm.make_instance(lam, k_vector(lam, kh), M, [a])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
    return insts


def _other_gpu_work(gsm, plan):
    """Eager work between replays: torch kernels, a solve issued as separate
    launches on another batch, host synchronisations."""
    import torch
    a = torch.randn(1 << 20, device="cuda:0")
    (a * 2 + 1).sum().item()
    inst = gsm.make_instance(1 / 0.3, k_vector(1 / 0.3, (0, 0, 1)), (2, 2, 2), [(1, 0, 0)])
    inst.eps_b = plan.basis_eps(inst)
    _, _, st = plan.solve([inst], gsm.default_opts(tol=1e-10))
    assert st == gsm.GSM_OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("restart", [30, 7, 1])
def test_graph_solve_equals_separate_launches(precision, restart):
    import torch
    gsm = G()
    eps = asym_body()
    plan = gsm.Plan(eps, PERIOD, (3, 3, 3))
    insts = _batch(gsm, plan)
    prec = gsm.GSM_MIXED if precision == "mixed" else gsm.GSM_FP64
    kw = dict(tol=1e-12, precision=prec, restart=restart)
    say(f"separate launches, {precision}, restart {restart}")
    E_ref, info_ref, st = plan.solve(insts, gsm.default_opts(**kw))
    assert st == gsm.GSM_OK
    assert plan.graph_stats() == (0, 0)
    say(f"launch graphs, first call, {precision}, restart {restart}")
    E1, info1, st = plan.solve(insts, gsm.default_opts(flags=gsm.GSM_SOLVE_GRAPH, **kw))
    assert st == gsm.GSM_OK
    cap1, run1 = plan.graph_stats()
    assert cap1 > 0 and run1 >= cap1
    assert torch.equal(E1, E_ref)
    assert [i["iterations"] for i in info1] == [i["iterations"] for i in info_ref]
    for rep in range(3):
        _other_gpu_work(gsm, plan)
        say(f"launch graphs, replay {rep}")
        E2, info2, st = plan.solve(insts, gsm.default_opts(flags=gsm.GSM_SOLVE_GRAPH, **kw))
        assert st == gsm.GSM_OK
        cap2, run2 = plan.graph_stats()
        assert cap2 == cap1, "identical call captured again instead of replaying"
        assert run2 > run1
        run1 = run2
        assert torch.equal(E2, E_ref), rep
    E = E_ref.cpu().numpy()
    off = 0
    for inst, (lam, kh, M, a) in zip(insts, CASES):
        c, q = oracle_case(eps, PERIOD, lam, k_vector(lam, kh), M)
        ref = O.solve_dense(c, M, q, inst.eps_b, [np.array(a, complex)]).ravel()
        assert rel_err(E[off:off + ref.size], ref) <= 1e-10
        off += ref.size


def test_graph_stack_m15_vs_1d_reduction():
    """Full-size layered stack (31^3 harmonics, 64^3 grid, GMRES(30), mixed
    precision) through launch graphs: the exact 1D reduction, and the same
    bits as separate launches."""
    import torch
    gsm = G()
    w = inputs.layered_stack_m15()
    k = k_vector(w["wavelength"], w["k_hat"])
    inst = gsm.make_instance(w["wavelength"], k, w["M"], w["drives"])
    plan = gsm.Plan(w["eps"], w["period"], w["M"])
    inst.eps_b = plan.basis_eps(inst)
    say("launch graphs, stack M=15")
    E, info, st = plan.solve([inst], gsm.default_opts(tol=1e-11, flags=gsm.GSM_SOLVE_GRAPH))
    assert st == gsm.GSM_OK and plan.graph_stats()[0] > 0
    say("separate launches, stack M=15")
    E_sep, _, st = plan.solve([inst], gsm.default_opts(tol=1e-11))
    assert st == gsm.GSM_OK and torch.equal(E, E_sep)
    E = E.cpu().numpy()
    c1 = O.box_image(w["eps"], (0, 0, 30))[:, 0, 0]
    n = E.size // 2
    for d, a in enumerate(w["drives"]):
        Ed = E[d * n:(d + 1) * n].reshape(3, 31, 31, 31)
        ref = O.solve_stack_1d(c1, 15, k / (2 * np.pi / w["wavelength"]), w["wavelength"], inst.eps_b,
                               np.array(a, complex))
        assert rel_err(Ed[:, :, 15, 15], ref) <= 1e-9


def test_no_graph_for_bicgstab_timed_launches_or_by_default():
    gsm = G()
    eps = asym_body()
    plan = gsm.Plan(eps, PERIOD, (3, 3, 3))
    insts = _batch(gsm, plan)
    say("bicgstab: separate launches")
    _, _, st = plan.solve(insts, gsm.default_opts(tol=1e-11, method=gsm.GSM_BICGSTAB, restart=6,
                                                  flags=gsm.GSM_SOLVE_GRAPH))
    assert st == gsm.GSM_OK and plan.graph_stats() == (0, 0)
    say("gmres while profiling: separate launches")
    gsm.profile_begin()
    try:
        _, _, st = plan.solve(insts, gsm.default_opts(tol=1e-11, flags=gsm.GSM_SOLVE_GRAPH))
    finally:
        stats = gsm.profile_end()
    assert st == gsm.GSM_OK and plan.graph_stats() == (0, 0)
    assert any(name.startswith("cgs_update") for name in stats)
    say("gmres without the flag: separate launches")
    _, _, st = plan.solve(insts, gsm.default_opts(tol=1e-11))
    assert st == gsm.GSM_OK and plan.graph_stats() == (0, 0)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_graph_adjoint_solve_equals_separate_launches(precision):
    """The adjoint Arnoldi steps (Green tensor before the convolution) in
    launch graphs: the same bits as separate launches, on the capture and on
    a replay, and the dense adjoint solution of the oracle."""
    import torch
    from gpu_common import seeded_field, to_torch
    gsm = G()
    eps = asym_body()
    period, lam, M = (1.0, 0.9, 1.1), 1 / 0.35, (2, 1, 3)
    k = k_vector(lam, (0.3, 0.4, 0.866))
    inst = gsm.make_instance(lam, k, M, [(1, 0, 0), (0, 1, 0)])
    plan = gsm.Plan(eps, period, M)
    inst.eps_b = plan.basis_eps(inst)
    rhs = seeded_field((2, 3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1), seed=29)
    prec = gsm.GSM_FP64 if precision == "fp64" else gsm.GSM_MIXED
    kw = dict(tol=1e-12, precision=prec)
    say(f"adjoint, separate launches, {precision}")
    ref_gpu, _, st = plan.solve_adjoint([inst], to_torch(rhs.ravel()), gsm.default_opts(**kw))
    assert st == gsm.GSM_OK
    for call in ("capture", "replay"):
        say(f"adjoint, launch graphs ({call}), {precision}")
        got, _, st = plan.solve_adjoint([inst], to_torch(rhs.ravel()),
                                        gsm.default_opts(flags=gsm.GSM_SOLVE_GRAPH, **kw))
        assert st == gsm.GSM_OK and torch.equal(got, ref_gpu), call
    cap, run = plan.graph_stats()
    assert cap > 0 and run > cap
    c, q = oracle_case(eps, period, lam, k, M)
    A = O.assemble_dense(c, M, q, inst.eps_b)
    ref = np.linalg.solve(A.conj().T, rhs.reshape(2, -1).T).T
    assert rel_err(ref_gpu.cpu().numpy(), ref.ravel()) <= 1e-10
