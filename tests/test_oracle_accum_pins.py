"""Pins of the oracle's temporal accumulation (Sec. 7: samples kept across
frames; the merge policy is this library's reading) against cases whose
answer is fixed by construction, not by the oracle's formula:
* hand-placed centres at known cells, on cell boundaries and outside the box,
  with ages at the limit;
* random centres placed strictly inside randomly chosen cells (or pushed
  outside the box from a border cell), the survivors found by set membership
  of the chosen cells;
* merging the same frame twice equals one merge with a history one frame
  older;
* the merged layout: frame first, survivors in order, ages, capacity cut."""
import numpy as np
import pytest

import oracle

LO = np.array([-1.0, 0.5, 2.0])
SIZE = 1.0
GRID = 4  # cell side 0.25: every boundary below is exact in float


def _at(cell, frac=(0.5, 0.5, 0.5)):
    """A centre at LO + side (cell + frac), radius 0.01."""
    side = SIZE / GRID
    p = LO + side * (np.asarray(cell, dtype=np.float64) + np.asarray(frac, dtype=np.float64))
    return [float(np.float32(p[0])), float(np.float32(p[1])), float(np.float32(p[2])), 0.01]


def _arr(rows):
    return np.asarray(rows, dtype=np.float32).reshape(-1, 4)


def test_hand_placed_cells():
    frame = _arr([_at((0, 0, 0)), _at((1, 2, 3), (0.2, 0.4, 0.6)), _at((3, 3, 3), (0.9, 0.9, 0.9))])
    side = SIZE / GRID
    hist = [
        _at((0, 0, 0), (0.8, 0.2, 0.96)),          # 0: frame cell (0,0,0) -> dropped
        _at((3, 2, 1)),                            # 1: the transposed cell of (1,2,3) -> kept
        _at((1, 2, 3), (0.04, 0.96, 0.04)),        # 2: frame cell (1,2,3) -> dropped
        _at((1, 2, 3), (0.0, 0.0, 0.0)),           # 3: on the cell's lower corner -> (1,2,3), dropped
        _at((0, 2, 3), (0.999, 0.0, 0.0)),         # 4: just below that corner in x -> (0,2,3), kept
        [float(LO[0] - 0.5), *_at((0, 2, 3))[1:]],  # 5: outside in x, border cell (0,2,3) -> kept
        [float(LO[0] - 0.3), float(LO[1] - 2.0), *_at((0, 0, 0))[2:]],  # 6: outside, clamps to (0,0,0) -> dropped
        [float(LO[0] + 1.7), float(LO[1] + 1.3), float(LO[2] + SIZE), 0.01],  # 7: clamps to (3,3,3) -> dropped
        _at((2, 0, 0)),                            # 8: free cell, age 2 -> 3 <= max_age: kept
        _at((2, 1, 0)),                            # 9: free cell, age 3 -> 4 > max_age: dropped
    ]
    age = np.array([0, 0, 0, 0, 0, 0, 0, 0, 2, 3], dtype=np.uint8)
    assert side == 0.25
    got = oracle.accumulate_survivors(frame, _arr(hist), age, LO, SIZE, GRID, max_age=3)
    assert got.tolist() == [1, 4, 5, 8]


def test_age_limits():
    hist = _arr([_at((0, 0, 0)), _at((1, 0, 0)), _at((2, 0, 0))])
    empty = _arr([])
    ages = np.array([0, 1, 2], dtype=np.uint8)
    assert oracle.accumulate_survivors(empty, hist, ages, LO, SIZE, GRID, 0).tolist() == []
    assert oracle.accumulate_survivors(empty, hist, ages, LO, SIZE, GRID, 1).tolist() == [0]
    assert oracle.accumulate_survivors(empty, hist, ages, LO, SIZE, GRID, 2).tolist() == [0, 1]
    assert oracle.accumulate_survivors(empty, hist, ages, LO, SIZE, GRID, 255).tolist() == [0, 1, 2]
    big = np.array([254, 255, 0], dtype=np.uint8)  # age 255 + 1 exceeds every limit
    assert oracle.accumulate_survivors(empty, hist, big, LO, SIZE, GRID, 255).tolist() == [0, 2]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_cells_by_construction(seed):
    rng = np.random.default_rng(seed)
    grid, lo, size = 16, np.array([0.25, -0.75, 1.5]), 2.0
    side = size / grid

    def place(cells, outside):
        frac = rng.uniform(0.05, 0.95, cells.shape)
        p = lo + side * (cells + frac)
        # push some border-cell centres out of the box along that axis: their cell stays the border cell
        for a in range(3):
            low = outside & (cells[:, a] == 0)
            high = outside & (cells[:, a] == grid - 1)
            p[low, a] = lo[a] - rng.uniform(0.0, 1.0, low.sum()) - 1e-3
            p[high, a] = lo[a] + size + rng.uniform(0.0, 1.0, high.sum()) + 1e-3
        out = np.zeros((len(cells), 4), dtype=np.float32)
        out[:, :3] = p
        out[:, 3] = 0.01
        # the float rounding of a centre must not cross a boundary: fractions stay 0.05 away
        return out

    # cells drawn from a small range so that frame and history share many
    fc = rng.integers(0, grid, (300, 3))
    fc[:40] = rng.choice([0, grid - 1], (40, 3))
    hc = np.concatenate([fc[rng.integers(0, 300, 250)], rng.integers(0, grid, (250, 3))])
    hc[:60] = rng.choice([0, grid - 1], (60, 3))
    frame = place(fc.astype(np.float64), rng.uniform(size=300) < 0.5)
    hist = place(hc.astype(np.float64), rng.uniform(size=500) < 0.5)
    age = rng.integers(0, 6, 500).astype(np.uint8)
    max_age = 4
    occupied = {tuple(c) for c in fc.tolist()}
    want = [i for i in range(500) if age[i] + 1 <= max_age and tuple(hc[i].tolist()) not in occupied]
    got = oracle.accumulate_survivors(frame, hist, age, lo, size, grid, max_age)
    assert len(want) > 50 and len(want) < 450
    assert got.tolist() == want


def test_merging_a_frame_twice():
    rng = np.random.default_rng(7)
    lo, size, grid = 0.0, 1.0, 32

    def rand(n):
        a = np.zeros((n, 4), dtype=np.float32)
        a[:, :3] = rng.uniform(-0.1, 1.1, (n, 3))
        a[:, 3] = 0.01
        return a

    f = {"cr": rand(400), "rgba": rng.uniform(size=(400, 4)).astype(np.float32)}
    h = {"cr": rand(900), "rgba": rng.uniform(size=(900, 4)).astype(np.float32),
         "age": rng.integers(0, 4, 900).astype(np.uint8)}
    once = oracle.accumulate(f, h, lo, size, grid, max_age=4)
    twice = oracle.accumulate(f, once, lo, size, grid, max_age=4)
    older = dict(h, age=(h["age"] + 1).astype(np.uint8))
    direct = oracle.accumulate(f, older, lo, size, grid, max_age=4)
    for k in ("cr", "rgba", "age"):
        assert np.array_equal(twice[k], direct[k])
    # the first copy of the frame (age 1 after the second merge) is gone entirely
    assert not np.any(twice["age"] == 1) and np.sum(once["age"] == 0) == 400
    assert len(twice["cr"]) < len(once["cr"])


def test_merged_layout_and_capacity():
    frame = {"cr": _arr([_at((0, 0, 0)), _at((1, 1, 1))]), "rgba": np.eye(2, 4, dtype=np.float32),
             "src": np.array([5, 9], dtype=np.uint32)}
    hist = {"cr": _arr([_at((3, 3, 3)), _at((0, 0, 0)), _at((2, 2, 2))]),
            "rgba": np.arange(12, dtype=np.float32).reshape(3, 4), "src": np.array([1, 2, 3], dtype=np.uint32),
            "age": np.array([0, 0, 1], dtype=np.uint8)}
    m = oracle.accumulate(frame, hist, LO, SIZE, GRID, max_age=2)
    assert m["kept"].tolist() == [0, 2]
    assert np.array_equal(m["cr"], np.concatenate([frame["cr"], hist["cr"][[0, 2]]]))
    assert np.array_equal(m["rgba"][2:], hist["rgba"][[0, 2]])
    assert m["src"].tolist() == [5, 9, 1, 3]
    assert m["age"].tolist() == [0, 0, 1, 2]
    cut = oracle.accumulate(frame, hist, LO, SIZE, GRID, max_age=2, capacity=3)
    assert cut["src"].tolist() == [5, 9, 1] and cut["age"].tolist() == [0, 0, 1]
