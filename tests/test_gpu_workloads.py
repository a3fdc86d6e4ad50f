"""The two large batched workloads at full size, checked against the CPU
oracle through what it can afford one by one: the oracle's own FFT operator
evaluates the relative residual of sampled GPU fields (an independent check
of every harmonic at once), small members are solved by the oracle outright,
and members of the batch equal the same instance solved alone.

  * uneven sweep: 256 (omega, k) points on an orthorhombic ellipsoid lattice
    (1 : 0.8 : 1.2, semi-axes 0.35 / 0.25 / 0.15, eps 6, 64^3 voxels), order
    counts 6..16 drawn per instance, one call (11 order-count groups);
  * woodpile: four-layer rods of eps 10 (128^3 voxels, exact), Lambda =
    0.4 lambda, M = 31 (63^3 harmonics, 128^3 grid), 16 seeded directions in
    one batched call.
"""
import numpy as np
import pytest

from gpu_common import k_vector, oracle_P, oracle_case, rel_err, say
from oracle import gsm as O
from paper_1501_01752_amd import inputs

pytestmark = pytest.mark.gpu

PERIOD3 = (1.0, 0.8, 1.2)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def G():
    from paper_1501_01752_amd import gsm
    return gsm


@pytest.fixture(scope="module")
def sweep():
    gsm = G()
    lam, khat, Ms = inputs.orthorhombic_sweep()
    eps = inputs.ellipsoid((64, 64, 64), PERIOD3, (0.35, 0.25, 0.15), 6.0)
    plan = gsm.Plan(eps, PERIOD3, (16, 16, 16))
    insts, drives = [], []
    for i in range(lam.size):
        a = inputs.transverse_drive(khat[i])
        M = (int(Ms[i]),) * 3
        inst = gsm.make_instance(lam[i], k_vector(lam[i], khat[i]), M, [tuple(a)])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
        drives.append(a)
    say("uneven sweep: 256 instances, M 6..16, one call")
    E, info, st = plan.solve(insts, gsm.default_opts(tol=1e-11))
    sizes = gsm.system_sizes(insts)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return dict(plan=plan, eps=eps, lam=lam, khat=khat, Ms=Ms, insts=insts, drives=drives,
                E=E.cpu().numpy(), info=info, st=st, offs=offs)


def test_sweep_all_converged(sweep):
    gsm = G()
    assert sweep["st"] == gsm.GSM_OK
    assert len(sweep["info"]) == 256
    assert all(i["status"] == gsm.GSM_OK and i["rel_residual"] <= 1e-11 for i in sweep["info"])
    # the order counts really are uneven and cover the whole range
    assert set(int(m) for m in sweep["Ms"]) == set(range(6, 17))


def _member(sweep, i):
    M = (int(sweep["Ms"][i]),) * 3
    k = k_vector(sweep["lam"][i], sweep["khat"][i])
    c, q = oracle_case(sweep["eps"], PERIOD3, sweep["lam"][i], k, M)
    shape = (3, 2 * M[2] + 1, 2 * M[1] + 1, 2 * M[0] + 1)
    E = sweep["E"][sweep["offs"][i]:sweep["offs"][i + 1]].reshape(shape)
    return M, c, q, E


def test_sweep_residual_by_oracle_operator(sweep):
    """Largest, smallest and seeded members: the oracle's FFT operator gives
    residual <= 1e-10 for the GPU field."""
    Ms = sweep["Ms"]
    picks = [int(np.argmax(Ms)), int(np.argmin(Ms))]
    picks += list(np.random.default_rng(31).choice(256, 4, replace=False))
    for i in picks:
        M, c, q, E = _member(sweep, i)
        say(f"oracle residual of sweep member {i} M={M[0]}")
        r = O.relative_residual(c, M, q, sweep["insts"][i].eps_b, sweep["drives"][i].astype(complex), E,
                                oracle_P(M))
        assert r <= 1e-10, (i, r)


def test_sweep_small_members_vs_oracle_solve(sweep):
    Ms = sweep["Ms"]
    small = [i for i in range(256) if Ms[i] == 6][:2]
    for i in small:
        M, c, q, E = _member(sweep, i)
        say(f"oracle solve of sweep member {i} M=6")
        ref, _ = O.solve_fft_gmres(c, M, q, sweep["insts"][i].eps_b, sweep["drives"][i].astype(complex),
                                   oracle_P(M), rtol=1e-12)
        assert rel_err(E, ref) <= 1e-9


def test_sweep_member_equals_single(sweep):
    gsm = G()
    for i in (0, 137):
        say(f"single solve of sweep member {i}")
        Es, _, st = sweep["plan"].solve([sweep["insts"][i]], gsm.default_opts(tol=1e-11))
        assert st == gsm.GSM_OK
        E = sweep["E"][sweep["offs"][i]:sweep["offs"][i + 1]]
        assert rel_err(E, Es.cpu().numpy()) <= 1e-9


def test_woodpile_m31_batch():
    gsm = G()
    eps = inputs.woodpile(128, 10.0)
    lam, M = 2.5, (31, 31, 31)
    plan = gsm.Plan(eps, (1, 1, 1), M)
    dirs = inputs.random_directions(16, seed=5)
    insts, drives = [], []
    for kh in dirs:
        a = inputs.transverse_drive(kh)
        inst = gsm.make_instance(lam, k_vector(lam, kh), M, [tuple(a)])
        inst.eps_b = plan.basis_eps(inst)
        insts.append(inst)
        drives.append(a)
    say("woodpile M=31 P=128, 16 directions, mixed, tol 1e-9")
    E, info, st = plan.solve(insts, gsm.default_opts(tol=1e-9))
    assert st == gsm.GSM_OK
    assert all(i["rel_residual"] <= 1e-9 and i["fft_size"] == 128 for i in info)
    E = E.cpu().numpy()
    n = 3 * 63 ** 3
    for s in (0, 9):
        say(f"oracle residual of woodpile direction {s}")
        c, q = oracle_case(eps, (1, 1, 1), lam, k_vector(lam, dirs[s]), M)
        r = O.relative_residual(c, M, q, insts[s].eps_b, drives[s].astype(complex),
                                E[s * n:(s + 1) * n].reshape(3, 63, 63, 63), (128, 128, 128))
        assert r <= 1e-9 * (1 + 1e-6), (s, r)
        assert abs(r - info[s]["rel_residual"]) <= 1e-12, (s, r, info[s]["rel_residual"])
