"""Different plans solved at the same time from different host threads (the
library keeps per-thread state for the profiler and the error message, and a
plan's resources to itself): each thread's result equals, bit for bit, the
same solve made alone, with and without launch timing."""
import threading

import pytest

from gpu_common import k_vector, say
from paper_1501_01752_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _bodies(gsm):
    out = []
    for w in (inputs.sphere_lattice_small(), inputs.layered_stack_m15()):
        k = k_vector(w["wavelength"], w["k_hat"])
        plan = gsm.Plan(w["eps"], w["period"], w["M"])
        dirs = inputs.random_directions(6, seed=11)
        insts = []
        for kh in [w["k_hat"]] + list(dirs):
            inst = gsm.make_instance(w["wavelength"], k_vector(w["wavelength"], kh), w["M"],
                                     [tuple(inputs.transverse_drive(kh))])
            inst.eps_b = plan.basis_eps(inst)
            insts.append(inst)
        out.append((plan, insts))
    return out


@pytest.mark.parametrize("profiled", [False, True])
def test_two_plans_from_two_threads(profiled):
    import torch
    from paper_1501_01752_amd import gsm
    bodies = _bodies(gsm)
    opts = gsm.default_opts(tol=1e-10)
    say("two plans, one after the other")
    alone = [plan.solve(insts, opts)[0] for plan, insts in bodies]
    streams = [torch.cuda.Stream() for _ in bodies]
    results = [None] * len(bodies)
    errors = []

    def run(i):
        try:
            plan, insts = bodies[i]
            with torch.cuda.stream(streams[i]):
                E, info, st = plan.solve(insts, opts, stream=streams[i].cuda_stream)
            streams[i].synchronize()
            results[i] = (E, st)
        except Exception as e:  # reported by the main thread
            errors.append(e)

    say(f"two plans from two threads (profiled={profiled})")
    if profiled:
        gsm.profile_begin(only="pass_b", every=2)
    try:
        threads = [threading.Thread(target=run, args=(i,)) for i in range(len(bodies))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
    finally:
        stats = gsm.profile_end() if profiled else None
    assert not errors, errors
    for i, (E, st) in enumerate(results):
        assert st == gsm.GSM_OK
        assert torch.equal(E, alone[i]), i
    if profiled:
        assert stats["pass_b_c64"]["launches"] > 0 and stats["pass_b_c64"]["flops"] > 0


def test_plan_before_any_torch_call():
    """A fresh process that makes a plan and solves before it has touched
    torch.cuda: the binding loads PyTorch's HIP runtime before the library,
    so both use one runtime (otherwise torch would find no device)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import numpy as np\n"
        "from paper_1501_01752_amd import gsm, inputs\n"
        "w = inputs.sphere_lattice_small()\n"
        "plan = gsm.Plan(w['eps'], w['period'], w['M'])\n"
        "lam = w['wavelength']\n"
        "inst = gsm.make_instance(lam, (0, 0, 2 * np.pi / lam), w['M'], [(1, 0, 0)])\n"
        "E, info, st = plan.solve([inst])\n"
        "print('ok', st, info[0]['rel_residual'])\n" % root)
    say("fresh process: plan and solve before torch.cuda")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().startswith("ok 0"), r.stdout
