"""Random words of the 16-bit stochastic rounding (host-side check, no GPU).

The step kernels give opposite pair k of a cell the word A ^ rotr(B, r_k),
with A the per-(cell, step) hash and B = xorshift32(A) (Marsaglia's 13/17/5
triple), and the rest value the word after the last pair; an FP16 conversion
reads the top 13 bits of its word, the pair's second value the top 13 bits
of the word shifted left by 13.  Every word is linear over GF(2) in the 32
bits of A, so two windows are independent and jointly uniform for a uniform
A exactly when their 26 x 32 matrix has full rank.  This test reads the
rotation table from the kernel source and checks that for both velocity
sets (9 pairs + rest, 13 pairs + rest).
"""
import itertools
import os
import re

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2402_10809_amd", "csrc", "step.hpp")


def rotations():
    txt = open(SRC).read()
    m = re.search(r"SR_ROT\[(\d+)\]\s*=\s*\{([^}]*)\}", txt)
    assert m, "rotation table not found"
    vals = [int(v) for v in m.group(2).split(",")]
    assert len(vals) == int(m.group(1))
    return vals


# A bit vector is a Python int over the 32 bits of A; a word is a list of 32
# such forms, word[i] being bit i of the word.
IDENT = [1 << i for i in range(32)]


def shl(w, s):
    return [w[i - s] if i >= s else 0 for i in range(32)]


def shr(w, s):
    return [w[i + s] if i + s < 32 else 0 for i in range(32)]


def xor(a, b):
    return [x ^ y for x, y in zip(a, b)]


def xorshift32(w):
    w = xor(w, shl(w, 13))
    w = xor(w, shr(w, 17))
    return xor(w, shl(w, 5))


def rotr(w, r):
    return [w[(i + r) % 32] for i in range(32)]


def rank(rows):
    rows, rk = list(rows), 0
    for bit in range(32):
        piv = next((i for i in range(rk, len(rows)) if rows[i] >> bit & 1), None)
        if piv is None:
            continue
        rows[rk], rows[piv] = rows[piv], rows[rk]
        for i in range(len(rows)):
            if i != rk and rows[i] >> bit & 1:
                rows[i] ^= rows[rk]
        rk += 1
    return rk


def fp16_windows(rots, npairs):
    B = xorshift32(IDENT)
    win = []
    for k in range(npairs + 1):
        w = xor(IDENT, rotr(B, rots[k]))
        win.append(w[19:32])              # top 13 bits
        if k < npairs:
            win.append(w[6:19])           # top 13 bits of the word << 13
    return win


def test_rotation_table_is_distinct_and_in_range():
    r = rotations()
    assert len(r) >= 14 and len(set(r)) == len(r) and all(0 <= v < 32 for v in r)


def test_every_two_fp16_windows_are_independent():
    r = rotations()
    for npairs in (9, 13):  # D3Q19, D3Q27
        win = fp16_windows(r, npairs)
        assert len(win) == 2 * npairs + 1
        assert all(rank(w) == 13 for w in win)
        bad = [(i, j) for (i, a), (j, b) in itertools.combinations(enumerate(win), 2) if rank(a + b) < 26]
        assert not bad, f"{npairs} pairs: dependent windows {bad[:5]}"


def test_the_check_catches_a_bad_table():
    # all pairs sharing one rotation: their first windows coincide
    win = fp16_windows([3] * 14, 9)
    assert any(rank(a + b) < 26 for a, b in itertools.combinations(win, 2))
