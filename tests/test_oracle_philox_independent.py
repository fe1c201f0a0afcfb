"""Bit-level pin of the oracle's random numbers by a second, independent generator.

The paper fixes only that the normals xi_n are i.i.d. N(0, 1) (Sec. 3.1); both
implementations draw them from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11) followed by Box-Muller. This file holds a
vectorised numpy implementation written from the SC'11 description, in a different
form from the oracle's C loop:

* the counter is two (left, right) pairs of 32-bit words, (x0, x1) and (x2, x3); a
  round multiplies each left word by its own multiplier (0xD2511F53 for x0,
  0xCD9E8D57 for x2) into a 64-bit product, and the new words are the high half of
  the *other* pair's product xor the right word xor the round key, followed by the
  low half of that other product;
* round r's key is the base key plus r times the Weyl constants (0x9E3779B9,
  0xBB67AE85) modulo 2^32, computed directly instead of bumped in place;
* ten rounds.

Its words must equal the oracle's bit for bit, and the oracle's normals must be the
Box-Muller pair of those words (u from the high 52 bits of (r1:r0), v from (r3:r2),
z0 = rho cos 2 pi v, z1 = rho sin 2 pi v) at the counter (block, sample_lo, sample_hi,
level | stream << 8) under the key (seed_lo, seed_hi).

Two known-answer vectors of Philox4x32-10 (the all-zero and the all-ones counter and
key), as published with the Random123 library and quoted in this project's code review,
pin both implementations to the published generator.
"""
import numpy as np
import pytest

import workloads as W

MASK32 = np.uint64(0xFFFFFFFF)
MUL = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
WEYL = (0x9E3779B9, 0xBB67AE85)
ROUNDS = 10


def philox_np(ctr, key):
    """Philox4x32-10 on arrays: ctr (n, 4), key (n, 2), 32-bit values in any integer
    dtype; returns (n, 4) uint64 holding 32-bit words."""
    x = np.asarray(ctr, dtype=np.uint64) & MASK32
    k = np.asarray(key, dtype=np.uint64) & MASK32
    left = [x[:, 0].copy(), x[:, 2].copy()]
    right = [x[:, 1].copy(), x[:, 3].copy()]
    for r in range(ROUNDS):
        rk = [(k[:, j] + np.uint64((r * WEYL[j]) & 0xFFFFFFFF)) & MASK32 for j in range(2)]
        prod = [left[j] * MUL[j] for j in range(2)]          # < 2^64: exact in uint64
        hi = [p >> np.uint64(32) for p in prod]
        lo = [p & MASK32 for p in prod]
        # pair 0 takes pair 1's product and vice versa
        new_left = [hi[1] ^ right[0] ^ rk[0], hi[0] ^ right[1] ^ rk[1]]
        new_right = [lo[1], lo[0]]
        left, right = new_left, new_right
    return np.stack([left[0], right[0], left[1], right[1]], axis=1)


def box_muller_np(words):
    """Uniforms (2m + 1) 2^-53 with m the top 52 bits of (r1:r0) and of (r3:r2), then
    rho = sqrt(-2 ln u), (rho cos 2 pi v, rho sin 2 pi v)."""
    w = np.asarray(words, dtype=np.uint64)
    def unif(hi, lo):
        m = ((hi << np.uint64(32)) | lo) >> np.uint64(12)
        return ((m << np.uint64(1)) | np.uint64(1)).astype(np.float64) * 2.0**-53
    u = unif(w[:, 1], w[:, 0])
    v = unif(w[:, 3], w[:, 2])
    rho = np.sqrt(-2.0 * np.log(u))
    theta = 2.0 * np.pi * v
    return rho * np.cos(theta), rho * np.sin(theta)


# (counter, key, output): Philox4x32-10 known-answer vectors
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_known_answers(orc, ctr, key, out):
    assert [int(v) for v in philox_np([ctr], [key])[0]] == list(out)
    assert orc.philox(list(ctr), list(key)) == list(out)


def test_oracle_words_equal_independent_generator(orc):
    rng = np.random.default_rng(20161222)
    n = 10000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    # edge words: zero, all ones, the counters the paths use (small block, reserved blocks)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0xFFFFFFFE, 7, 1, 3 | (5 << 8)]]
    key[:4] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [42, 0], [0xFFFFFFFF, 0x7FFFFFFF]]
    ref = philox_np(ctr, key)
    got = np.array([orc.philox([int(c) for c in ctr[i]], [int(k) for k in key[i]])
                    for i in range(n)], dtype=np.uint64)
    mism = np.nonzero(np.any(got != ref, axis=1))[0]
    assert mism.size == 0, f"{mism.size} of {n} blocks differ, first at {mism[:5]}"


def test_oracle_normals_are_box_muller_of_the_counter_words(orc):
    """The counter layout, the key, the word order of the two uniforms and the
    cos/sin assignment: every oracle normal equals the independent generator's."""
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(3000):
        level = int(rng.integers(0, 31))
        sample = int(rng.integers(0, 2**40))
        block = int(rng.integers(0, 2**32))
        seed = int(rng.integers(0, 2**63))
        stream = int(rng.integers(0, 2**24))
        cases.append((level, sample, block, seed, stream))
    cases += [(0, 0, 0, 42, 0), (12, 9999, 0xFFFFFFFF, 42, 0), (5, 2**33 + 3, 0xFFFFFFFE, 2**63, 2**24 - 1)]
    ctr = [[b, s & 0xFFFFFFFF, s >> 32, (lv & 0xFF) | (st << 8)] for lv, s, b, _, st in cases]
    key = [[sd & 0xFFFFFFFF, sd >> 32] for _, _, _, sd, _ in cases]
    z0, z1 = box_muller_np(philox_np(ctr, key))
    got = np.array([orc.normals(W.problem(seed=sd, stream_id=st), lv, s, b)
                    for lv, s, b, sd, st in cases])
    # libm and numpy may round log, cos and sin differently in the last place
    tol = 1e-14 * np.maximum(1.0, np.abs(np.stack([z0, z1], axis=1)))
    assert np.all(np.abs(got[:, 0] - z0) <= tol[:, 0])
    assert np.all(np.abs(got[:, 1] - z1) <= tol[:, 1])


def test_independent_generator_is_not_trivially_the_oracle():
    """Self-check of the pin: the numpy generator is sensitive to each of the mistakes
    the oracle could plausibly make (it would not pin them otherwise)."""
    ctr = np.array([[0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]], dtype=np.uint64)
    key = np.array([[0xA4093822, 0x299F31D0]], dtype=np.uint64)
    base = philox_np(ctr, key)
    global MUL, ROUNDS
    saved = (MUL, ROUNDS)
    try:
        MUL = (saved[0][1], saved[0][0])
        assert not np.array_equal(philox_np(ctr, key), base)
        MUL, ROUNDS = saved[0], 9
        assert not np.array_equal(philox_np(ctr, key), base)
    finally:
        MUL, ROUNDS = saved
    assert np.array_equal(philox_np(ctr, key), base)
