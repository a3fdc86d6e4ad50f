"""The HIP FFT codelet generator against numpy.fft (no GPU): evaluates the
generated data-flow graph numerically for every codelet the kernels use."""
import importlib.util
import os

import numpy as np
import pytest

_here = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location(
    "gen_fft", os.path.join(_here, "..", "paper_1501_01752_amd", "csrc", "gen_fft.py"))
gen = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(gen)


def _evaluate(n, in_slots, out_slots, sign, xin, family=0):
    b, outs = gen.build_codelet(n, in_slots, out_slots, sign, family)
    vals = {}
    for i, op in enumerate(b.g.nodes):
        if op[0] == 'in':
            vals[i] = xin[op[1]].real if op[2] == 0 else xin[op[1]].imag
        elif op[0] == 'add':
            vals[i] = vals[op[1]] + vals[op[2]]
        elif op[0] == 'sub':
            vals[i] = vals[op[1]] - vals[op[2]]
        elif op[0] == 'mul':
            vals[i] = vals[op[1]] * float(op[2])

    def r(x):
        if x is None:
            return 0.0
        return -vals[x[0]] if x[1] else vals[x[0]]
    return np.array([r(o.re) + 1j * r(o.im) for o in outs])


@pytest.mark.parametrize("family", gen.FAMILIES)
@pytest.mark.parametrize("spec", gen.codelet_specs(), ids=lambda s: s[0])
def test_codelet_matches_numpy(spec, family):
    name, n, ins, outs, sign = spec
    rng = np.random.default_rng(n)
    xin = rng.normal(size=len(ins)) + 1j * rng.normal(size=len(ins))
    full = np.zeros(n, complex)
    full[ins] = xin
    ref = np.fft.ifft(full) * n if sign > 0 else np.fft.fft(full)
    got = _evaluate(n, ins, outs, sign, xin, family)
    assert np.abs(got - ref[outs]).max() < 1e-13 * np.sqrt(n) * np.abs(xin).max() * 4


@pytest.mark.parametrize("n", [6, 12, 20, 24, 40, 45, 48, 60, 72, 96])
def test_mixed_radix_sizes(n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    got = _evaluate(n, list(range(n)), list(range(n)), -1, x)
    assert np.abs(got - np.fft.fft(x)).max() < 1e-12 * n


def test_twiddle_table_exact_points():
    for n in (8, 16, 32):
        assert gen._cs(n // 4, n) == (0.0, 1.0)
        assert gen._cs(n // 2, n) == (-1.0, 0.0)


def test_family_zero_has_fewest_operations():
    """The fewest-operation family never needs more operations than the plain
    radix-4 one, and at the plane pass's main size it needs clearly fewer."""
    for name, n, ins, outs, sign in gen.codelet_specs():
        b0, o0 = gen.build_codelet(n, ins, outs, sign, 0)
        b1, o1 = gen.build_codelet(n, ins, outs, sign, 1)
        assert gen._ops(b0, o0) <= gen._ops(b1, o1), name
    i, o = gen.expand_slots(64, 15)
    b0, o0 = gen.build_codelet(64, i, o, +1, 0)
    b1, o1 = gen.build_codelet(64, i, o, +1, 1)
    assert gen._ops(b0, o0) < 0.85 * gen._ops(b1, o1)
