"""Codelet families and the autotuner (HIP path) against the CPU oracle.

Every combination of codelet families (fewest-operation or plain radix-4,
chosen per FFT stage) must apply the same operator: each is forced through a
tuning-cache entry and checked against the oracle's FFT operator.  An
autotuned plan must solve to the oracle's field, write one cache entry per
(M, P, precision), and a second plan reading that cache must reuse it.
"""
import itertools

import numpy as np
import pytest

from gpu_common import fp32_operator_tol, k_vector, oracle_case, rel_err, say, seeded_field, to_torch
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


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _sphere_case(M):
    eps = inputs.sphere(32, 0.3, 4.0)
    lam = 1 / 0.3
    k = k_vector(lam, (0.2, 0.3, 0.93))
    return eps, (1.0, 1.0, 1.0), lam, k


@pytest.mark.parametrize("precision", ["c64", "c128"])
@pytest.mark.parametrize("M", [7, 15])
def test_every_family_combination_applies_the_operator(tmp_path, precision, M):
    gsm = G()
    Ms = (M, M, M)
    P = gsm.fft_size(Ms)
    eps, period, lam, k = _sphere_case(Ms)
    c, q = oracle_case(eps, period, lam, k, Ms)
    shape = (3, 2 * M + 1, 2 * M + 1, 2 * M + 1)
    dt = np.complex64 if precision == "c64" else np.complex128
    prec = gsm.GSM_MIXED if precision == "c64" else gsm.GSM_FP64
    tol = fp32_operator_tol(P) if precision == "c64" else 1e-13
    x = seeded_field(shape, seed=5, dtype=dt)
    ref = None
    for fam in itertools.product((0, 1), repeat=4):
        cache = tmp_path / f"tune_{''.join(map(str, fam))}.txt"
        cache.write_text(f"{_arch()} P={P} M={M},{M},{M} {precision} S=1 "
                         f"fam={fam[0]},{fam[1]},{fam[2]},{fam[3]}\n")
        plan = gsm.Plan(eps, period, Ms, tune_cache=str(cache))
        inst = gsm.make_instance(lam, k, Ms, [(1, 0.5j, 0)])
        inst.eps_b = plan.basis_eps(inst)
        assert plan.tuning(Ms, prec) == (list(fam), True)
        if ref is None:
            ref = O.apply_operator_fft(c, Ms, q, inst.eps_b, x.astype(np.complex128), (P, P, P))
        say(f"apply {precision} M={M} families {fam}")
        y = plan.apply([inst], to_torch(x.ravel()), precision=prec).cpu().numpy().reshape(shape)
        assert rel_err(y, ref) <= tol, fam
        plan.close()


def test_autotuned_solve_and_cache(tmp_path):
    gsm = G()
    w = inputs.sphere_lattice_small()
    k = k_vector(w["wavelength"], w["k_hat"])
    cache = tmp_path / "tune.txt"
    plan = gsm.Plan(w["eps"], w["period"], w["M"], autotune=True, tune_cache=str(cache))
    assert plan.tuning(w["M"])[1] is False
    inst = gsm.make_instance(w["wavelength"], k, w["M"], [(1, 0, 0), (0, 0.3, 1j)])
    inst.eps_b = plan.basis_eps(inst)
    say("autotuned solve sphere M=3")
    E, info, st = plan.solve([inst], gsm.default_opts(tol=1e-12))
    assert st == gsm.GSM_OK
    c, q = oracle_case(w["eps"], w["period"], w["wavelength"], k, w["M"])
    ref = O.solve_dense(c, w["M"], q, inst.eps_b, [np.array([1, 0, 0]), np.array([0, 0.3, 1j])])
    assert rel_err(E.cpu().numpy(), ref.ravel()) <= 1e-10
    fam, tuned = plan.tuning(w["M"])
    assert tuned
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and " P=16 M=3,3,3 c64 " in lines[0]
    assert lines[0].split()[0] == _arch()
    # a second plan reads the entry and does not tune again
    plan2 = gsm.Plan(w["eps"], w["period"], w["M"], autotune=True, tune_cache=str(cache))
    assert plan2.tuning(w["M"]) == (fam, True)
    say("solve with cached tuning")
    E2, _, st2 = plan2.solve([inst], gsm.default_opts(tol=1e-12))
    assert st2 == gsm.GSM_OK and rel_err(E2.cpu().numpy(), ref.ravel()) <= 1e-10
    assert len(cache.read_text().splitlines()) == 1


def test_untuned_plan_uses_defaults():
    gsm = G()
    eps = inputs.sphere(16, 0.3, 4.0)
    plan = gsm.Plan(eps, (1, 1, 1), (15, 15, 15))
    assert plan.tuning((15, 15, 15), gsm.GSM_MIXED) == ([0, 0, 0, 0], False)
    assert plan.tuning((15, 15, 15), gsm.GSM_FP64) == ([0, 0, 0, 1], False)
