"""Host model of the four-step lane transform of the FFT passes (no GPU):
the ownership rule that gives each lane of a line one order per slot, and
the exchange it implies, checked against a direct DFT for every (P, lanes)
split the kernels use.  The model restates the kernels' index arithmetic
(slot s, block m = bitrev(t) mod R taken from the lowest block, radix-2
butterflies between lanes H apart, slot twiddle e^{2 pi i s t / P}); the
device kernels themselves are checked by the GPU operator parity tests."""
import numpy as np
import pytest

# (P, values per lane) of the splits that take the four-step form
SPLITS = [(128, 32), (128, 16), (256, 32), (256, 16), (512, 32), (512, 16)]


def _bitrev(t, nb):
    return int(format(t, f"0{nb}b")[::-1], 2) if nb else 0


def _shape(P, L):
    R = P // L
    N = P // R
    K = (P - 1) // 4
    mlo = -((K + N - 1) // N)
    nb = R.bit_length() - 1
    blocks = [mlo + (_bitrev(t, nb) - mlo) % R for t in range(R)]
    return R, N, K, nb, blocks


@pytest.mark.parametrize("P,L", SPLITS)
def test_every_order_has_one_owner(P, L):
    R, N, K, _, blocks = _shape(P, L)
    owners = {}
    for t in range(R):
        for s in range(N):
            k = s + N * blocks[t]
            if -K <= k <= K:
                assert k not in owners, (k, owners[k], t)
                owners[k] = t
    assert sorted(owners) == list(range(-K, K + 1))


def _butterfly_twiddle(t, h, sign):
    return np.exp(sign * 2j * np.pi * (t & (h - 1)) / (2 * h)) if t & h else 1.0


@pytest.mark.parametrize("P,L", SPLITS)
@pytest.mark.parametrize("kmax_frac", [1.0, 0.4, 0.0])
def test_exchange_equals_direct_transform(P, L, kmax_frac):
    R, N, K, nb, blocks = _shape(P, L)
    kmax = int(K * kmax_frac)
    rng = np.random.default_rng(P + L)
    ks = np.arange(-K, K + 1)
    X = np.where(np.abs(ks) <= kmax, rng.normal(size=ks.size) + 1j * rng.normal(size=ks.size), 0)
    pos = np.arange(P)
    want = np.exp(2j * np.pi * np.outer(pos, ks) / P) @ X
    # expand: lane t loads the order of its block in each slot, then a
    # decimation-in-time exchange across the lanes, the slot twiddle and the
    # lane's N-point inverse DFT give positions R j + t
    got = np.empty(P, complex)
    A = np.zeros((R, N), complex)
    for s in range(N):
        v = np.array([X[s + N * blocks[t] + K] if abs(s + N * blocks[t]) <= kmax else 0 for t in range(R)])
        for st in range(nb):
            h = 1 << st
            w = v * np.array([_butterfly_twiddle(t, h, +1) for t in range(R)])
            sg = np.array([-1 if t & h else 1 for t in range(R)])
            v = w[np.arange(R) ^ h] + sg * w
        A[:, s] = v * np.exp(2j * np.pi * s * np.arange(R) / P)
    j = np.arange(N)
    for t in range(R):
        got[R * j + t] = np.exp(2j * np.pi * np.outer(j, np.arange(N)) / N) @ A[t]
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
    # crop: the lane's N-point forward DFT, the conjugate slot twiddle, then a
    # decimation-in-frequency exchange leaves lane t with its block's order
    x = rng.normal(size=P) + 1j * rng.normal(size=P)
    zwant = np.exp(-2j * np.pi * np.outer(ks, pos) / P) @ x
    z = np.array([np.fft.fft(x[t::R]) for t in range(R)])
    zgot = {}
    for s in range(N):
        v = z[:, s] * np.exp(-2j * np.pi * s * np.arange(R) / P)
        for st in reversed(range(nb)):
            h = 1 << st
            sg = np.array([-1 if t & h else 1 for t in range(R)])
            v = (v[np.arange(R) ^ h] + sg * v) * np.array([_butterfly_twiddle(t, h, -1) for t in range(R)])
        for t in range(R):
            k = s + N * blocks[t]
            if abs(k) <= kmax:
                zgot[k] = v[t]
    assert sorted(zgot) == list(range(-kmax, kmax + 1))
    err = max(abs(zgot[k] - zwant[k + K]) for k in zgot)
    assert err <= 1e-12 * np.abs(zwant).max()
