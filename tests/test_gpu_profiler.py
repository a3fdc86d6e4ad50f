"""Launch profiler (HIP path): per-class launch counts, algorithmic bytes and
flops, a single profiled class, and sampled timing (one launch in k)."""
import pytest

from gpu_common import k_vector, say
from paper_1501_01752_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _case():
    from paper_1501_01752_amd import gsm
    w = inputs.sphere_lattice_small()
    k = k_vector(w["wavelength"], w["k_hat"])
    plan = gsm.Plan(w["eps"], w["period"], w["M"])
    inst = gsm.make_instance(w["wavelength"], k, w["M"], [(1, 0, 0), (0, 1, 0)])
    inst.eps_b = plan.basis_eps(inst)
    return gsm, plan, inst


def test_every_class_counted():
    gsm, plan, inst = _case()
    say("profile every class, sphere M=3")
    gsm.profile_begin()
    try:
        _, info, st = plan.solve([inst], gsm.default_opts(tol=1e-11))
    finally:
        stats = gsm.profile_end()
    assert st == gsm.GSM_OK
    for c in ("pass_a_c64", "pass_b_c64", "pass_c_c64", "cgs_update_c64", "cgs_finish_c64", "pass_a_c128"):
        assert c in stats and stats[c]["launches"] > 0 and stats[c]["ms"] > 0, c
    # the three passes run together: one launch each per operator application
    assert stats["pass_a_c64"]["launches"] == stats["pass_b_c64"]["launches"] == stats["pass_c_c64"]["launches"]
    for c in ("pass_a_c64", "pass_b_c64", "pass_c_c64"):
        assert stats[c]["bytes"] > 0 and stats[c]["flops"] > 0, c
    # every Krylov iteration of the two systems is one complex64 operator application
    assert stats["pass_b_c64"]["launches"] >= max(i["iterations"] for i in info)


def test_one_class_and_sampling():
    gsm, plan, inst = _case()
    say("profile pass_b only")
    gsm.profile_begin(only="pass_b")
    try:
        plan.solve([inst], gsm.default_opts(tol=1e-11))
    finally:
        full = gsm.profile_end()
    assert set(full) <= {"pass_b_c64", "pass_b_c128"} and "pass_b_c64" in full
    say("profile pass_b, one launch in 3")
    gsm.profile_begin(only="pass_b", every=3)
    try:
        plan.solve([inst], gsm.default_opts(tol=1e-11))
    finally:
        samp = gsm.profile_end()
    assert set(samp) <= {"pass_b_c64", "pass_b_c128"}
    # one counter per class (both precisions); launch counts of two identical
    # solves can differ by the few gated steps the host issues past the end
    # of a cycle
    n_full = sum(v["launches"] for v in full.values())
    n_samp = sum(v["launches"] for v in samp.values())
    assert abs(n_samp - n_full / 3) <= 4, (n_full, n_samp)
    assert samp["pass_b_c64"]["flops"] > 0
