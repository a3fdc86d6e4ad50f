#!/usr/bin/env python3
"""Generate straight-line, pruned FFT codelets for the GSM pass kernels.

Each codelet computes a length-N DFT restricted to a set of non-zero input
residues and a set of wanted output residues,

    out[j] = sum_{k in inputs} in[k] * exp(sign * 2 pi i * k * j / N),

built as a data-flow graph of real additions and constant multiplications
from several factorisations (decimation in time or in frequency, radix 4 or
split radix, mixed radix 2, 3, 5 otherwise; each also by network
transposition of the transposed problem), keeping the one with the fewest
operations.  Zero inputs are propagated, multiplications by 0, +-1 and +-i
disappear, and only the operations that feed a wanted output are emitted.  The result is a
``__device__ __forceinline__`` template over the real type (float or double)
that works on register arrays, so every twiddle is a literal constant.

Usage: gen_fft.py OUT_HEADER
"""
import math
import struct
import os
import sys
from fractions import Fraction

# --------------------------------------------------------------- DAG --------


class Graph:
    def __init__(self):
        self.nodes = []          # (op, args...)
        self.memo = {}

    def node(self, *key):
        if key in self.memo:
            return self.memo[key]
        self.nodes.append(key)
        idx = len(self.nodes) - 1
        self.memo[key] = idx
        return idx


ZERO = None   # a real value that is exactly zero


def neg(x):
    if x is ZERO:
        return ZERO
    return (x[0], not x[1])


class Builder:
    """Real-valued expressions as (node, negated) references."""

    def __init__(self):
        self.g = Graph()

    def inp(self, slot, part):
        return (self.g.node('in', slot, part), False)

    def add(self, x, y):
        if x is ZERO:
            return y
        if y is ZERO:
            return x
        if x[1] and y[1]:
            return neg(self.add(neg(x), neg(y)))
        if x[1]:
            return self._sub(y, neg(x))
        if y[1]:
            return self._sub(x, neg(y))
        a, b = sorted((x[0], y[0]))
        return (self.g.node('add', a, b), False)

    def _sub(self, x, y):          # x, y positive references
        if x[0] == y[0]:
            return ZERO
        return (self.g.node('sub', x[0], y[0]), False)

    def sub(self, x, y):
        return self.add(x, neg(y))

    def mul(self, x, c):
        if x is ZERO or c == 0.0:
            return ZERO
        if c == 1.0:
            return x
        if c == -1.0:
            return neg(x)
        if c < 0:
            return neg(self.mul(x, -c))
        return (self.g.node('mul', x[0], repr(float(c))), x[1])


def _cs(num, den):
    """exp(2 pi i num/den) with exact values at multiples of pi/4."""
    f = Fraction(num, den) % 1
    exact = {Fraction(0): (1.0, 0.0), Fraction(1, 4): (0.0, 1.0), Fraction(1, 2): (-1.0, 0.0),
             Fraction(3, 4): (0.0, -1.0)}
    if f in exact:
        return exact[f]
    r = math.sqrt(0.5)
    eighth = {Fraction(1, 8): (r, r), Fraction(3, 8): (-r, r), Fraction(5, 8): (-r, -r),
              Fraction(7, 8): (r, -r)}
    if f in eighth:
        return eighth[f]
    ang = 2.0 * math.pi * float(f)
    return (math.cos(ang), math.sin(ang))


class C:
    """Complex value as a pair of real references."""

    def __init__(self, re, im):
        self.re, self.im = re, im

    def is_zero(self):
        return self.re is ZERO and self.im is ZERO


def cadd(b, x, y):
    return C(b.add(x.re, y.re), b.add(x.im, y.im))


def csub(b, x, y):
    return C(b.sub(x.re, y.re), b.sub(x.im, y.im))


def ctw(b, x, num, den):
    """x * exp(2 pi i num / den)."""
    if x.is_zero():
        return x
    c, s = _cs(num, den)
    if s == 0.0:
        return C(b.mul(x.re, c), b.mul(x.im, c))
    if c == 0.0:     # +-i
        return C(b.mul(x.im, -s), b.mul(x.re, s))
    if abs(abs(c) - abs(s)) < 1e-300:
        # (c + i s) with |c| = |s| = r: two adds and two multiplications
        r = abs(c)
        re = b.sub(b.mul(x.re, c / r), b.mul(x.im, s / r))
        im = b.add(b.mul(x.re, s / r), b.mul(x.im, c / r))
        return C(b.mul(re, r), b.mul(im, r))
    re = b.sub(b.mul(x.re, c), b.mul(x.im, s))
    im = b.add(b.mul(x.re, s), b.mul(x.im, c))
    return C(re, im)


def _radix(n):
    for r in (4, 2, 3, 5):
        if n % r == 0:
            return r
    raise ValueError(f'size {n} is not 2,3,5-smooth')


def _zeros(n):
    return [C(ZERO, ZERO) for _ in range(n)]


def _mul_i(b, x, s):
    """x * (s i) for s = +1 or -1 (free: a swap and a sign)."""
    if s > 0:
        return C(neg(x.im), x.re)
    return C(x.im, neg(x.re))


def _butterfly(b, t, n, sign):
    """Length-r DFT of the already twiddled t (r = len(t)) with the usual
    shared partial sums for r = 2 and 4, plain sums otherwise."""
    r = len(t)
    if NAIVE_BUTTERFLIES:
        r = -r
    if r == 2:
        return [cadd(b, t[0], t[1]), csub(b, t[0], t[1])]
    if r == 4:
        a0 = cadd(b, t[0], t[2])
        a1 = csub(b, t[0], t[2])
        a2 = cadd(b, t[1], t[3])
        a3 = _mul_i(b, csub(b, t[1], t[3]), sign)
        return [cadd(b, a0, a2), cadd(b, a1, a3), csub(b, a0, a2), csub(b, a1, a3)]
    r = abs(r)
    out = []
    for q in range(r):
        acc = C(ZERO, ZERO)
        for j in range(r):
            acc = cadd(b, acc, ctw(b, t[j], sign * j * q, r))
        out.append(acc)
    return out


def dft_dit(b, xs, n, sign, split):
    """Decimation in time (split radix 2/4 for powers of two when `split`,
    else radix 4, 2, 3, 5); xs: n complex values (possibly zero)."""
    if n == 1:
        return list(xs)
    if all(x.is_zero() for x in xs):
        return _zeros(n)
    if split and n % 4 == 0 and (n & (n - 1)) == 0:
        e = dft_dit(b, xs[0::2], n // 2, sign, split)
        o1 = dft_dit(b, xs[1::4], n // 4, sign, split)
        o3 = dft_dit(b, xs[3::4], n // 4, sign, split)
        out = [None] * n
        q = n // 4
        for k in range(q):
            u = ctw(b, o1[k], sign * k, n)
            v = ctw(b, o3[k], sign * 3 * k, n)
            sm = cadd(b, u, v)
            df = _mul_i(b, csub(b, u, v), sign)
            out[k] = cadd(b, e[k], sm)
            out[k + 2 * q] = csub(b, e[k], sm)
            out[k + q] = cadd(b, e[k + q], df)
            out[k + 3 * q] = csub(b, e[k + q], df)
        return out
    r = 2 if (split and n == 2) else _radix(n)
    m = n // r
    subs = [dft_dit(b, xs[j::r], m, sign, split) for j in range(r)]
    out = [None] * n
    for k in range(m):
        t = [ctw(b, subs[j][k], sign * j * k, n) for j in range(r)]
        for qq, v in enumerate(_butterfly(b, t, n, sign)):
            out[k + qq * m] = v
    return out


def dft_dif(b, xs, n, sign, split):
    """Decimation in frequency, the transpose of dft_dit's factorisation."""
    if n == 1:
        return list(xs)
    if all(x.is_zero() for x in xs):
        return _zeros(n)
    if split and n % 4 == 0 and (n & (n - 1)) == 0:
        q = n // 4
        ev = [cadd(b, xs[i], xs[i + 2 * q]) for i in range(2 * q)]
        u1, u3 = [], []
        for i in range(q):
            a = csub(b, xs[i], xs[i + 2 * q])
            c = _mul_i(b, csub(b, xs[i + q], xs[i + 3 * q]), sign)
            u1.append(ctw(b, cadd(b, a, c), sign * i, n))
            u3.append(ctw(b, csub(b, a, c), sign * 3 * i, n))
        e = dft_dif(b, ev, 2 * q, sign, split)
        o1 = dft_dif(b, u1, q, sign, split)
        o3 = dft_dif(b, u3, q, sign, split)
        out = [None] * n
        for k in range(2 * q):
            out[2 * k] = e[k]
        for k in range(q):
            out[4 * k + 1] = o1[k]
            out[4 * k + 3] = o3[k]
        return out
    r = 2 if (split and n == 2) else _radix(n)
    m = n // r
    # butterflies across the r blocks of length m, twiddle, then r sub-DFTs
    cols = []
    for i in range(m):
        t = [xs[i + j * m] for j in range(r)]
        cols.append(_butterfly(b, t, n, sign))
    out = [None] * n
    for qq in range(r):
        sub = [ctw(b, cols[i][qq], sign * qq * i, n) for i in range(m)]
        y = dft_dif(b, sub, m, sign, split)
        for k in range(m):
            out[k * r + qq] = y[k]
    return out


def dft(b, xs, n, sign):
    """Radix-4 decimation in time (the reference factorisation)."""
    return dft_dit(b, xs, n, sign, False)


# ------------------------------------------------------------- emitter ------

ALGORITHMS = (('dit', False), ('dit', True), ('dif', False), ('dif', True))
# Two families of every codelet: 0 = the fewest operations over the
# factorisations below; 1 = radix-4 decimation in time with plain butterfly
# sums (more additions, shorter live ranges, so fewer registers where a whole
# long transform sits in one lane).  The kernels take the family as a
# template parameter and the library's autotuner picks per pass by timing.
FAMILIES = (0, 1)
NAIVE_BUTTERFLIES = False


def _build(n, in_slots, out_slots, sign, algo):
    b = Builder()
    xs = [C(ZERO, ZERO) for _ in range(n)]
    for i, s in enumerate(in_slots):
        xs[s] = C(b.inp(i, 0), b.inp(i, 1))
    kind, split = algo
    ys = (dft_dit if kind == 'dit' else dft_dif)(b, xs, n, sign, split)
    outs = [ys[s] for s in out_slots]
    return b, outs


def _live(b, outs):
    """Nodes the outputs depend on."""
    nodes = b.g.nodes
    used = set()
    stack = []
    for o in outs:
        for r in (o.re, o.im):
            if r is not ZERO:
                stack.append(r[0])
    while stack:
        i = stack.pop()
        if i in used:
            continue
        used.add(i)
        op = nodes[i]
        if op[0] in ('add', 'sub'):
            stack += [op[1], op[2]]
        elif op[0] == 'mul':
            stack.append(op[1])
    return used


def _ops(b, outs):
    return sum(1 for i in _live(b, outs) if b.g.nodes[i][0] != 'in')


def _transpose(b, outs, n_in):
    """Network transposition.  The codelet is a real linear map from its
    2 n_in input parts to the parts of `outs`; the transposed graph computes
    the transposed map (for a DFT of sign s restricted to input set I and
    output set O, that is the DFT of sign -s from O to I, the DFT matrix being
    symmetric).  Every fan-out of the original becomes an addition."""
    nodes = b.g.nodes
    live = _live(b, outs)
    t = Builder()
    adj = {}

    def contribute(i, ref):
        if ref is ZERO:
            return
        adj[i] = ref if i not in adj else t.add(adj[i], ref)

    for j, o in enumerate(outs):
        for part, r in ((0, o.re), (1, o.im)):
            if r is ZERO:
                continue
            x = t.inp(j, part)
            contribute(r[0], neg(x) if r[1] else x)
    res = [[ZERO, ZERO] for _ in range(n_in)]
    for i in sorted(live, reverse=True):
        if i not in adj:
            continue
        a = adj[i]
        op = nodes[i]
        if op[0] == 'add':
            contribute(op[1], a)
            contribute(op[2], a)
        elif op[0] == 'sub':
            contribute(op[1], a)
            contribute(op[2], neg(a))
        elif op[0] == 'mul':
            contribute(op[1], t.mul(a, float(op[2])))
        else:  # input
            res[op[1]][op[2]] = a
    return t, [C(r[0], r[1]) for r in res]


def build_codelet(n, in_slots, out_slots, sign, family=0):
    """The cheapest (fewest real operations after pruning) of: the
    decimation-in-time and -in-frequency factorisations, radix 4 or split
    radix, built directly for this pattern of non-zero inputs and wanted
    outputs, and the transposes of the same factorisations built for the
    transposed pattern (output set to input set, opposite sign).  Family 1
    is the plain radix-4 form only."""
    global NAIVE_BUTTERFLIES
    best = None
    saved = NAIVE_BUTTERFLIES
    algos = ALGORITHMS
    if family == 1:
        NAIVE_BUTTERFLIES = True
        algos = (('dit', False),)
    for algo in algos:
        cands = [_build(n, in_slots, out_slots, sign, algo)]
        if family == 0:
            tb, touts = _build(n, out_slots, in_slots, -sign, algo)
            cands.append(_transpose(tb, touts, len(out_slots)))
        for b, outs in cands:
            cost = _ops(b, outs)
            if best is None or cost < best[0]:
                best = (cost, b, outs)
    NAIVE_BUTTERFLIES = saved
    return best[1], best[2]


def emit(name, n, in_slots, out_slots, sign, family=0):
    b, outs = build_codelet(n, in_slots, out_slots, sign, family)
    nodes = b.g.nodes
    used = _live(b, outs)
    lines = []
    nin, nout = len(in_slots), len(out_slots)
    lines.append(f'// {name}: N={n}, {nin} non-zero inputs, {nout} outputs, sign {sign:+d}')
    lines.append('template <typename T>')
    lines.append(f'__device__ __forceinline__ void {name}(const T (&ir)[{nin}], const T (&ii)[{nin}],'
                 f' T (&orr)[{nout}], T (&oi)[{nout}]) {{')
    nflop = 0
    for i in sorted(used):
        op = nodes[i]
        if op[0] == 'in':
            src = 'ir' if op[2] == 0 else 'ii'
            lines.append(f'  const T v{i} = {src}[{op[1]}];')
        elif op[0] == 'add':
            lines.append(f'  const T v{i} = v{op[1]} + v{op[2]};')
            nflop += 1
        elif op[0] == 'sub':
            lines.append(f'  const T v{i} = v{op[1]} - v{op[2]};')
            nflop += 1
        elif op[0] == 'mul':
            lines.append(f'  const T v{i} = v{op[1]} * T({op[2]});')
            nflop += 1

    def ref(r):
        if r is ZERO:
            return 'T(0)'
        return ('-' if r[1] else '') + f'v{r[0]}'
    for j, o in enumerate(outs):
        lines.append(f'  orr[{j}] = {ref(o.re)};')
        lines.append(f'  oi[{j}] = {ref(o.im)};')
    lines.append('}')
    lines.insert(1, f'// real operations: {nflop}')
    return '\n'.join(lines) + '\n', nflop


def expand_slots(n, k):
    return [x % n for x in range(-k, k + 1)], list(range(n))


def crop_slots(n, k):
    return list(range(n)), [x % n for x in range(-k, k + 1)]


# FFT grid sizes of the pass kernels: the powers of two, and between 32 and
# 128 the 2-3-smooth sizes whose pruned transforms (and lane splits) cost
# less than the next power of two for the order counts they serve: 36
# (M = 8), 40 (M = 9), 48 (M = 10, 11), 72 (M = 16, 17).  Sizes with a
# factor 5 or an odd lane length cost more operations than 64 (50, 54, 60).
GRID_SIZES = (4, 8, 16, 32, 36, 40, 48, 64, 72, 128)
MIXED_SIZES = tuple(p for p in GRID_SIZES if p & (p - 1))


def lane_length(p, lane_max):
    """Values per lane when a length-p transform is split over the fewest
    lanes R (a power of two dividing p) that leave at most lane_max each."""
    r = 1
    while p // r > lane_max:
        r *= 2
    assert p % r == 0, (p, lane_max)
    return p // r


def codelet_specs():
    """(name, N, in_slots, out_slots, sign) for every codelet the kernels use.

    expand (e): inputs at residues of -K..K, all N outputs, sign +1 (field to
    real space); crop (c): all N inputs, outputs at -K..K, sign -1; full (f).
    """
    specs = []
    pairs = set()
    fulls = set()
    # A length-P transform (orders |k| <= K = (P-1)//4) is split over R lanes
    # of length N = P / R: at most 32 values per lane in complex64, 16 in
    # complex128 (the kernels' rule).  When 2K+1 > N the orders fold and the
    # lane runs a full length-N transform.
    for p in GRID_SIZES:
        k = (p - 1) // 4
        for lane_max in (64, 32, 16):
            n = lane_length(p, lane_max)
            if 2 * k + 1 <= n:
                pairs.add((n, k))
            else:
                fulls.add(n)
    for n, k in sorted(pairs):
        i, o = expand_slots(n, k)
        specs.append((f'fft_e{n}_{k}', n, i, o, +1))
        i, o = crop_slots(n, k)
        specs.append((f'fft_c{n}_{k}', n, i, o, -1))
    for n in sorted(fulls):
        specs.append((f'fft_fp{n}', n, list(range(n)), list(range(n)), +1))
        specs.append((f'fft_fm{n}', n, list(range(n)), list(range(n)), -1))
    return specs


def twiddle_table(n):
    vals = [_cs(j, n) for j in range(n)]
    body = ',\n'.join(f'  {{{c!r}, {s!r}}}' for c, s in vals)
    return f'__device__ constexpr double kTw{n}[{n}][2] = {{\n{body}\n}};\n'


def _f32(x):
    # the binary32 value nearest x (ties to even), written so that it parses back exactly
    return repr(struct.unpack('f', struct.pack('f', x))[0]) + 'f'


def twiddle_table_f32(n):
    vals = [_cs(j, n) for j in range(n)]
    body = ',\n'.join(f'  {{{_f32(c)}, {_f32(s)}}}' for c, s in vals)
    return f'__device__ constexpr float kTw{n}f[{n}][2] = {{\n{body}\n}};\n'


def dispatch(name, n, nin, nout, kind, param, family):
    return (f'template <> struct Codelet{kind}<{n}, {param}, {family}> {{\n'
            f'  template <typename T> __device__ static __forceinline__ void run('
            f'const T (&ir)[{nin}], const T (&ii)[{nin}], T (&orr)[{nout}], T (&oi)[{nout}]) {{\n'
            f'    {name}<T>(ir, ii, orr, oi);\n  }}\n}};\n')


def main(path):
    out = ['// Generated by gen_fft.py: straight-line pruned DFT codelets. Do not edit.',
           '#pragma once', '#include <hip/hip_runtime.h>', '',
           '// CodeletE<N, K>: inputs at residues of -K..K (in that order), all N outputs,',
           '//   out[j] = sum_k in[k] exp(+2 pi i k j / N).',
           '// CodeletC<N, K>: all N inputs, outputs at residues of -K..K,',
           '//   out[k] = sum_j in[j] exp(-2 pi i k j / N).',
           '// CodeletF<N, S>: full transform with sign S (+1 or -1).',
           '// The last parameter is the family: 0 fewest operations, 1 plain radix 4.',
           'template <int N, int K, int F> struct CodeletE;',
           'template <int N, int K, int F> struct CodeletC;',
           'template <int N, int S, int F> struct CodeletF;', '']
    total = 0
    for family in FAMILIES:
        for name, n, i, o, s in codelet_specs():
            fname = f'{name}_f{family}'
            src, nf = emit(fname, n, i, o, s, family)
            out.append(src)
            total += nf
            if name.startswith('fft_e'):
                out.append(dispatch(fname, n, len(i), len(o), 'E', (len(i) - 1) // 2, family))
            elif name.startswith('fft_c'):
                out.append(dispatch(fname, n, len(i), len(o), 'C', (len(o) - 1) // 2, family))
            else:
                out.append(dispatch(fname, n, len(i), len(o), 'F', s, family))
    # roots of unity: order 512 for the powers of two, order 720 (a multiple of
    # every mixed size) for the others
    for n in (8, 16, 32, 64, 128, 512, 720):
        out.append(twiddle_table(n))
    # complex64 copy of the order-512 roots, for twiddles indexed at run time
    out.append(twiddle_table_f32(512))
    with open(path, 'w') as f:
        f.write('\n'.join(out))
    with open(os.path.join(os.path.dirname(path), 'fft_opcount.h'), 'w') as f:
        f.write(opcount_table())


def opcount_table():
    """Real operations (add, sub, mul each one) of the unsplit pruned length-P
    transforms for orders |k| <= K in their fewest-operation factorisation:
    the algorithmic work of one expand and one crop, for every supported P
    and every K <= (P - 1) / 4."""
    lines = ['// Generated by gen_fft.py: real operations of pruned length-P DFTs. Do not edit.',
             '#pragma once', '',
             f'// kPrunedOps[pruned_ops_row(P)][K] = {{expand (2K+1 -> P), crop (P -> 2K+1)}},',
             f'// P in {GRID_SIZES}',
             f'static const int kPrunedGrid[{len(GRID_SIZES)}] = {{{", ".join(str(p) for p in GRID_SIZES)}}};',
             'inline int pruned_ops_row(int P) {',
             f'  for (int i = 0; i < {len(GRID_SIZES)}; ++i)',
             '    if (kPrunedGrid[i] == P) return i;',
             '  return -1;',
             '}',
             f'static const int kPrunedOps[{len(GRID_SIZES)}][32][2] = {{']
    rows = []
    for p in GRID_SIZES:
        vals = []
        for k in range(32):
            if k <= (p - 1) // 4:
                i, o = expand_slots(p, k)
                b, outs = build_codelet(p, i, o, +1, 0)
                fe = _ops(b, outs)
                i, o = crop_slots(p, k)
                b, outs = build_codelet(p, i, o, -1, 0)
                fc = _ops(b, outs)
            else:
                fe = fc = 0
            vals.append(f'{{{fe}, {fc}}}')
        rows.append('  {' + ', '.join(vals) + '}')
    lines.append(',\n'.join(rows))
    lines.append('};')
    return '\n'.join(lines) + '\n'


if __name__ == '__main__':
    main(sys.argv[1])
