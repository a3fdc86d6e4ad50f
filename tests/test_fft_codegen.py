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


def _evaluate(n, in_slots, out_slots, sign, xin):
    b, outs = gen.build_codelet(n, in_slots, out_slots, sign)
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


@pytest.mark.parametrize("spec", gen.codelet_specs(), ids=lambda s: s[0])
def test_codelet_matches_numpy(spec):
    name, n, ins, outs, sign = spec
    rng = np.random.default_rng(n)
    xin = rng.normal(size=len(ins)) + 1j * rng.normal(size=len(ins))
    full = np.zeros(n, complex)
    full[ins] = xin
    ref = np.fft.ifft(full) * n if sign > 0 else np.fft.fft(full)
    got = _evaluate(n, ins, outs, sign, xin)
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
