"""Host checks of the bit-level identities the multi-generation kernels use
(one bit per cell in LDS, bit-sliced neighbour counts).

The expressions below are the kernels' own (csrc/smap_ca2k.hpp,
csrc/smap_ca3k.hpp), evaluated on Python integers; each is checked
exhaustively against its plain definition: the byte/bit packing multiplies,
the full adder of a row and its shifted copies, the sums of bit-sliced
numbers, and the B3/S23 and B6/S567 rules on the count with the centre
(Section 5.1: a cell is born on 3 or 6 live neighbours and survives on 2-3
or 5-7).
"""
import itertools

M32 = 0xFFFFFFFF


def pack4(d):
    return ((d * 0x01020408) & M32) >> 24 & 0xF


def unpack4(v):
    return ((v & 0xF) * 0x00204081) & M32 & 0x01010101


def test_pack_and_unpack_every_pattern():
    for bits in range(16):
        d = sum(((bits >> k) & 1) << (8 * k) for k in range(4))   # four 0/1 bytes
        assert pack4(d) == bits
        assert unpack4(bits) == d


def _slices(values, nbits):
    """Bit-slice a list of small integers: plane b holds bit b of each."""
    return [sum(((v >> b) & 1) << i for i, v in enumerate(values)) for b in range(nbits)]


def _unslice(planes, count):
    return [sum(((p >> i) & 1) << b for b, p in enumerate(planes)) for i in range(count)]


def _row_sum(L, a, R):
    # the kernels' horizontal full adder: s0 = L ^ a ^ R, s1 = majority
    la = L ^ a
    return la ^ R, (L & a) | (R & la)


def _add3_2(a, b, c):
    # three 2-bit numbers -> 4 bits (the kernels' add3_2)
    t0, k0 = a[0] ^ b[0], a[0] & b[0]
    x1 = a[1] ^ b[1]
    t1, k1 = x1 ^ k0, (a[1] & b[1]) | (k0 & x1)
    q0, m0 = t0 ^ c[0], t0 & c[0]
    y1 = t1 ^ c[1]
    q1, m1 = y1 ^ m0, (t1 & c[1]) | (m0 & y1)
    return [q0, q1, k1 ^ m1, k1 & m1]


def _add_ripple(x, y, width):
    out, cr = [], 0
    for b in range(width):
        xb = x[b] if b < len(x) else 0
        yb = y[b] if b < len(y) else 0
        t = xb ^ yb
        out.append(t ^ cr)
        cr = (xb & yb) | (cr & t)
    return out, cr


def test_row_full_adder_counts_three_cells():
    for L, a, R in itertools.product((0, 1), repeat=3):
        s0, s1 = _row_sum(L, a, R)
        assert s0 + 2 * s1 == L + a + R


def test_add3_2_all_operands():
    vals = list(itertools.product(range(4), repeat=3))       # every triple of 2-bit numbers
    a, b, c = (_slices([v[k] for v in vals], 2) for k in range(3))
    got = _unslice(_add3_2(a, b, c), len(vals))
    assert got == [sum(v) for v in vals]


def test_two_ripple_adds_of_in_plane_sums():
    # T = Sp + Sc + Sn with each in-plane sum at most 9: 5 bits, at most 27
    vals = list(itertools.product(range(10), repeat=3))
    sp, sc, sn = (_slices([v[k] for v in vals], 4) for k in range(3))
    u, cr = _add_ripple(sp, sc, 4)
    u.append(cr)
    t, cr2 = _add_ripple(u, sn, 4)
    t.append(u[4] ^ cr2)
    assert not any(u[4] & cr2 for _ in [0])                # no carry out of bit 4
    assert _unslice(t, len(vals)) == [sum(v) for v in vals]


def test_b3s23_on_bits_matches_the_rule():
    # T = 3x3 count including the centre (0..9); next = born on 3, survives on 2-3
    cases = [(t, alive) for t in range(10) for alive in (0, 1) if not (alive and t == 0)]
    q = _slices([t for t, _ in cases], 4)
    ca = sum(alive << i for i, (_, alive) in enumerate(cases))
    res = ~q[3] & ((q[0] & q[1] & ~q[2]) | (ca & ~q[0] & ~q[1] & q[2]))
    for i, (t, alive) in enumerate(cases):
        neighbours = t - alive
        want = (neighbours in (2, 3)) if alive else (neighbours == 3)
        assert ((res >> i) & 1) == int(want), (t, alive)


def test_b6s567_on_bits_matches_the_rule():
    # T = 3x3x3 count including the centre (0..27); born on 6, survives on 5-7
    cases = [(t, alive) for t in range(28) for alive in (0, 1) if not (alive and t == 0)]
    tt = _slices([t for t, _ in cases], 5)
    cc = sum(alive << i for i, (_, alive) in enumerate(cases))
    e67 = ~tt[4] & ~tt[3] & tt[2] & tt[1]
    e8 = ~tt[4] & tt[3] & ~tt[2] & ~tt[1] & ~tt[0]
    res = (e67 & (~tt[0] | cc)) | (cc & e8)
    for i, (t, alive) in enumerate(cases):
        neighbours = t - alive
        want = (5 <= neighbours <= 7) if alive else (neighbours == 6)
        assert ((res >> i) & 1) == int(want), (t, alive)


def test_keep_bits_clears_left_of_box_and_past_the_hypotenuse():
    def keep_bits(x, y, n):
        if y < 0 or x <= -32:
            return 0
        hi = n - y - x + 1
        m = M32 if hi >= 32 else (0 if hi <= 0 else (1 << hi) - 1)
        if x < 0:
            m &= (M32 << (-x)) & M32
        return m
    for n in (0, 5, 40, 100):
        for y in range(-3, n + 3):
            for x in range(-48, n + 8, 4):
                m = keep_bits(x, y, n)
                for b in range(32):
                    cell = x + b
                    want = y >= 0 and 0 <= cell and cell + y <= n
                    assert ((m >> b) & 1) == int(want), (n, x, y, b)
