"""Pins of the oracle's sample codec (64 bits per sample: 3 x 18-bit
quantised position + 10-bit log radius; 32 bits per colour: RGBA8; the wire
format of Sec. 4.1 and Sec. 5): hand-computed words, the error bounds of a
round trip, idempotence on decoded values, clamping and monotonicity."""
import math

import numpy as np
import pytest

import oracle

LO, SIZE, RU = -0.25, 1.5, 0.0015
CELL = SIZE / 2 ** 18


def test_hand_computed_words():
    assert oracle.encode_position([LO, LO, LO], RU, LO, SIZE, RU) == 512 << 54
    q = (12345, 200000, 7)
    c = [LO + (qi + 0.5) * CELL for qi in q]
    r = RU * 2 ** (70 / 64)  # code 582
    assert oracle.encode_position(c, r, LO, SIZE, RU) == q[0] | q[1] << 18 | q[2] << 36 | 582 << 54
    assert oracle.encode_colour([1.0, 0.0, 0.5, 1.0]) == 0xFF8000FF
    assert oracle.encode_colour([0.2, 0.4, 0.6, 0.8]) == 51 | 102 << 8 | 153 << 16 | 204 << 24


def test_round_trip_error_bounds():
    rng = np.random.default_rng(4)
    n = 20000
    cr = np.empty((n, 4), dtype=np.float32)
    cr[:, :3] = rng.uniform(LO, LO + SIZE, (n, 3))
    cr[:, 3] = RU * 2 ** rng.uniform(-6, 6, n)
    col = rng.uniform(0, 1, (n, 4))
    pos, words = oracle.encode(cr, col, LO, SIZE, RU)
    dcr, dcol = oracle.decode(pos, words, LO, SIZE, RU)
    c64 = cr[:, :3].astype(np.float64)
    assert np.abs(dcr[:, :3] - c64).max() <= CELL / 2 + 2e-7   # half a cell, plus float rounding of the output
    rel = np.abs(dcr[:, 3] - cr[:, 3].astype(np.float64)) / cr[:, 3]
    assert rel.max() <= 2 ** (1 / 128) - 1 + 1e-6              # half a radius step
    assert np.abs(dcol - col).max() <= 1 / 510 + 1e-7


def test_decoded_values_encode_to_the_same_words():
    rng = np.random.default_rng(9)
    n = 5000
    pos = (rng.integers(0, 2 ** 18, (n, 3)).astype(np.uint64) << np.array([0, 18, 36], dtype=np.uint64)).sum(axis=1)
    pos |= rng.integers(0, 1024, n).astype(np.uint64) << np.uint64(54)
    words = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    cr, col = oracle.decode(pos, words, LO, SIZE, RU)
    p2, w2 = oracle.encode(cr, col.astype(np.float64), LO, SIZE, RU)
    assert np.array_equal(p2, pos) and np.array_equal(w2, words)


def test_clamping_and_monotone_codes():
    hi = 2 ** 18 - 1
    assert oracle.encode_position([LO - 1, LO + SIZE + 1, math.nan], RU, LO, SIZE, RU) == 0 | hi << 18 | 0 << 36 | 512 << 54
    assert oracle.encode_position([LO, LO, LO], RU * 2 ** -20, LO, SIZE, RU) >> 54 == 0
    assert oracle.encode_position([LO, LO, LO], RU * 2 ** 20, LO, SIZE, RU) >> 54 == 1023
    assert oracle.encode_colour([-0.5, 2.0, math.nan, 0.5]) == 0 | 255 << 8 | 0 << 16 | 128 << 24
    xs = np.sort(np.random.default_rng(1).uniform(LO, LO + SIZE, 3000))
    codes = [oracle.encode_position([x, LO, LO], RU, LO, SIZE, RU) & (2 ** 18 - 1) for x in xs]
    assert all(a <= b for a, b in zip(codes, codes[1:]))
