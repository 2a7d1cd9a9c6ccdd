"""Pins of the oracle's message log (every bit a party sends during a
comparison) against what the gates of App. C/D must send.

For an ABY3 AND gate the three parties' messages z_0, z_1, z_2 XOR to the
product of the opened inputs (App. C: z_p = x_p y_p + x_{p-1} y_p +
x_p y_{p-1} + alpha_p with alpha_0 + alpha_1 + alpha_2 = 0).  In BitExtract
(App. D) the inputs of every gate follow from the plain integers of the
three input components: the FA-layer gate of bit i multiplies
(x0_i ^ x2_i) by (x1_i ^ x2_i), and the ripple gate of bit i multiplies
(A_i ^ c_i) by (B_i ^ c_i) for A = the FA carries shifted up one bit,
B = x0 ^ x1 ^ x2 and c_i the carry into bit i of A + B.  Those products are
computed here with Python integers, independently of the oracle's
bit-sliced gates.  In the 3OT the receiver's output c1 is w_c ^ k_{choice},
so c1 ^ w_c equals one of the two values party 0 sent.  The per-party split
of the log gives the bits each party sends.
"""
import numpy as np
import pytest

import oracle as orc


def _bits(log, m, row, col):
    return int((int(log[m, row, col // 64]) >> (col % 64)) & 1)


def _gate_products(x, m):
    """Opened AND products of BitExtract over bits 0..m of x[0]+x[1]+x[2]:
    (FA products of bits 0..m-1, ripple products of bits 1..m-1)."""
    bit = lambda v, i: (v >> i) & 1  # noqa: E731
    fa = [(bit(x[0], i) ^ bit(x[2], i)) & (bit(x[1], i) ^ bit(x[2], i)) for i in range(m)]
    maj = [bit(x[0], i) & bit(x[1], i) | bit(x[0], i) & bit(x[2], i) | bit(x[1], i) & bit(x[2], i)
           for i in range(m + 1)]
    A = [0] + maj[:m]
    B = [bit(x[0], i) ^ bit(x[1], i) ^ bit(x[2], i) for i in range(m + 1)]
    rip, c = [None], 0                      # carry into bit 1 is A_0 B_0 = 0
    for i in range(1, m):
        z = (A[i] ^ c) & (B[i] ^ c)
        rip.append(z)
        c = z ^ c
    return fa, rip


def _check_bit_extract(log, g0, m, comps, row, col):
    fa, rip = _gate_products(comps, m)
    for i in range(m):
        g = g0 + (0 if i == 0 else 2 * i - 1)
        assert _bits(log, 3 * g, row, col) ^ _bits(log, 3 * g + 1, row, col) ^ _bits(log, 3 * g + 2, row, col) == fa[i]
        if i >= 1:
            g = g0 + 2 * i
            got = _bits(log, 3 * g, row, col) ^ _bits(log, 3 * g + 1, row, col) ^ _bits(log, 3 * g + 2, row, col)
            assert got == rip[i], (i, row, col)


def _check_ot(log, base, k, row, col):
    val = lambda off: sum(_bits(log, base + off + j, row, col) << j for j in range(k))  # noqa: E731
    k0, k1, wc, c1 = val(0), val(k), val(2 * k), val(3 * k)
    assert (c1 ^ wc) in (k0, k1)


def _random_components(rng, rows, n, mask=0xFFFF):
    return rng.integers(0, mask + 1, (3, rows, n), dtype=np.uint64).astype(np.uint16 if mask == 0xFFFF else np.uint32)


def test_mpclift_message_log(keys):
    _, party = keys
    rng = np.random.default_rng(5)
    rows, n = 2, 130                          # three words, the last ragged
    rot = [0, 3]
    d = _random_components(rng, rows, n)
    x = _random_components(rng, rows, n)
    match, ml, y, counts, log = orc.compare(party, d, x, 1, rot, 11, 64, want_aux=True, want_msg=True)
    assert log.shape == (406, rows, 3) and orc.msg_count(0) == 406
    # bits sent per comparison: 94 AND messages each, plus the 3OT roles
    assert list(counts) == [94 * rows * n, 156 * rows * n, 125 * rows * n, 125 * rows * n]
    for row in range(rows):
        for col in list(range(0, n, 7)) + [n - 1]:
            xs = [int(x[p, row, col]) for p in range(3)]
            _check_bit_extract(log, 0, 17, xs, row, col)                      # Lift: 33 gates
            ys = [int(y[p, row, col]) for p in range(3)]
            _check_bit_extract(log, 33, 31, ys, row, col)                     # MSB: 61 gates
            _check_ot(log, 282, 15, row, col)
            _check_ot(log, 342, 16, row, col)
    # columns past n send nothing
    assert not any(int(log[m, r, 2]) >> (n % 64) for m in range(406) for r in range(rows))
    # the log is a pure addition: the match components are unchanged
    assert np.array_equal(match, orc.compare(party, d, x, 1, rot, 11, 64))


@pytest.mark.parametrize("variant", [orc.CMPV_PLAIN, orc.CMPV_LIFT18, orc.CMPV_CONST32])
def test_variant_message_logs(keys, variant):
    _, party = keys
    rng = np.random.default_rng(6 + variant)
    rows, n = 2, 100
    rot = [-2, 5]
    if variant == orc.CMPV_CONST32:
        d = _random_components(rng, rows, n, 0xFFFFFFFF)
        x = _random_components(rng, rows, n, 0xFFFFFFFF)
        ml_pub = None
    else:
        d = _random_components(rng, rows, n)
        x = None if variant == orc.CMPV_PLAIN else _random_components(rng, rows, n)
        ml_pub = rng.integers(0, 12801, (rows, n)) if variant == orc.CMPV_PLAIN else None
    match, y, counts, log = orc.compare_variant(party, variant, d, x, ml_pub, 1, rot, 3, 0, want_aux=True,
                                                want_msg=True)
    nmsg = {orc.CMPV_PLAIN: 87, orc.CMPV_LIFT18: 210, orc.CMPV_CONST32: 183}[variant]
    assert log.shape[0] == nmsg == orc.msg_count(variant)
    assert counts[1] + counts[2] + counts[3] == nmsg * rows * n
    for row in range(rows):
        for col in list(range(0, n, 9)) + [n - 1]:
            ys = [int(y[p, row, col]) for p in range(3)]
            if variant == orc.CMPV_PLAIN:
                _check_bit_extract(log, 0, 15, ys, row, col)
            elif variant == orc.CMPV_CONST32:
                _check_bit_extract(log, 0, 31, ys, row, col)
            else:
                xs = [int(x[p, row, col]) for p in range(3)]
                _check_bit_extract(log, 0, 17, xs, row, col)
                _check_bit_extract(log, 33, 17, ys, row, col)
                _check_ot(log, 198, 1, row, col)
                _check_ot(log, 202, 2, row, col)
