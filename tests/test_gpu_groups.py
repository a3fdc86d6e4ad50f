"""Splitting a call's systems into launch groups (solver option group_max).

Every system's arithmetic is its own (per-system blocks, partial sums and
refinement decisions), so the solution of each system must not depend on
which systems share its group: the same bits with no limit, one system per
group, an uneven split and the default; and the oracle's dense solution.
"""
import numpy as np
import pytest
import torch

from gpu_common import asym_body, k_vector, oracle_case, rel_err, say
from oracle import gsm as O

pytestmark = pytest.mark.gpu

PERIOD = (1.0, 0.9, 1.1)
M = (2, 3, 1)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _batch(gsm, plan):
    """Seven instances of one (M, P) with two drives each (14 systems) and one
    of another order count."""
    insts = []
    rng = np.random.default_rng(17)
    for i in range(7):
        lam = 1 / rng.uniform(0.25, 0.4)
        kh = rng.normal(size=3)
        inst = gsm.make_instance(lam, k_vector(lam, kh), M, [(1, 0, 0), (0, 1, 0.5)])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
    inst = gsm.make_instance(1 / 0.3, k_vector(1 / 0.3, (0, 0, 1)), (1, 1, 1), [(1, 0, 0)])
    inst.eps_b = plan.basis_eps(inst)
    insts.append(inst)
    return insts


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_group_split_gives_identical_solutions(precision):
    from paper_1501_01752_amd import gsm
    plan = gsm.Plan(asym_body(), PERIOD, M)
    insts = _batch(gsm, plan)
    prec = gsm.GSM_MIXED if precision == "mixed" else gsm.GSM_FP64
    results = {}
    for gmax in (0, 1, 5, 32):
        say(f"group_max={gmax} {precision}")
        E, info, st = plan.solve(insts, gsm.default_opts(tol=1e-11, precision=prec, group_max=gmax))
        assert st == gsm.GSM_OK
        results[gmax] = (E, [i["iterations"] for i in info])
    E0, it0 = results[0]
    for gmax, (E, it) in results.items():
        assert torch.equal(E, E0), gmax
        assert it == it0, gmax
    # first instance, first drive, against the dense oracle
    inst = insts[0]
    c, q = oracle_case(asym_body(), PERIOD, inst.wavelength, np.array(inst.k_inc), M)
    ref = O.solve_dense(c, M, q, inst.eps_b, [np.array((1, 0, 0), complex)]).ravel()
    assert rel_err(E0[:ref.size].cpu().numpy(), ref) <= 1e-9
    plan.close()


def test_negative_group_max_rejected():
    from paper_1501_01752_amd import gsm
    plan = gsm.Plan(asym_body(), PERIOD, M)
    insts = _batch(gsm, plan)
    with pytest.raises(gsm.GsmError) as e:
        plan.solve(insts, gsm.default_opts(group_max=-1))
    assert e.value.status == gsm.GSM_E_ARG
    plan.close()
