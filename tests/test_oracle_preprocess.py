"""Pins of the preprocessing oracle (half-sampling, fiber mask, per-pixel
rows) against a hand-worked example, brute force and closed forms. CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import preprocess as pp

GOLD = os.path.join(os.path.dirname(__file__), "golden", "preprocess_example.json")


def test_hand_example():
    d = json.load(open(GOLD))
    stack = np.array(d["stack"], dtype=np.uint16)
    assert np.array_equal(pp.half_sample(stack), np.array(d["half"]))
    E = pp.energy(stack)
    assert np.array_equal(E, np.array(d["energy"], dtype=np.float64))
    for frac in ("0.999", "0.7", "0.4"):
        assert pp.fiber_mask(E, float(frac)).tolist() == d["mask_" + frac]
    assert np.array_equal(pp.gather_rows(stack, np.array(d["mask_0.7"])), np.array(d["rows_0.7"]))


def test_half_sample_keeps_odd_one_based_indices():
    n, H, W = 3, 6, 8
    i, y, x = np.meshgrid(np.arange(n), np.arange(H), np.arange(W), indexing="ij")
    stack = i * 10000 + (y + 1) * 100 + (x + 1)  # value encodes 1-based row and column
    h = pp.half_sample(stack)
    assert h.shape == (n, H // 2, W // 2)
    assert np.all((h // 100) % 100 % 2 == 1) and np.all(h % 100 % 2 == 1)


def test_energy_and_rows_by_loops():
    g = np.random.default_rng(0)
    stack = g.integers(0, 4096, size=(7, 6, 4)).astype(np.uint16)
    E = np.zeros(6, dtype=np.float64)
    for i in range(7):
        for r in range(3):
            for c in range(2):
                E[r * 2 + c] += float(stack[i, 2 * r, 2 * c])
    assert np.array_equal(pp.energy(stack), E)
    pix = np.array([1, 4, 5])
    rows = pp.gather_rows(stack, pix)
    for k, p in enumerate(pix):
        for i in range(7):
            assert rows[k, i] == stack[i, 2 * (p // 2), 2 * (p % 2)]


@pytest.mark.parametrize("seed", range(6))
def test_mask_is_minimal_brightest_set_by_brute_force(seed):
    g = np.random.default_rng(seed)
    E = g.integers(0, 6, size=9).astype(np.float64)  # ties are frequent
    for frac in (0.3, 0.5, 0.9, 0.999, 1.0):
        m = pp.fiber_mask(E, frac)
        total = E.sum()
        best = None
        for r in range(0, 10):
            ok = [c for c in itertools.combinations(range(9), r) if E[list(c)].sum() >= frac * total]
            if ok:
                best = r
                break
        assert len(m) == best
        # among the minimal sets, the brightest-first one with ties broken by index
        key = sorted(range(9), key=lambda i: (-E[i], i))[:best]
        assert m.tolist() == sorted(key)


def test_mask_special_cases():
    assert pp.fiber_mask(np.zeros(16), 0.999).size == 0
    E = np.array([0.0, 3.0, 0.0, 1.0, 2.0, 0.0])
    assert pp.fiber_mask(E, 1.0).tolist() == [1, 3, 4]  # every lit pixel, none of the dark ones
    assert pp.fiber_mask(E, 1e-9).tolist() == [1]        # the brightest pixel alone


def test_disk_holding_the_energy_is_the_mask():
    # a fiber core (disk) of uniform brightness and a dim background holding
    # less than 0.1 % of the total: the mask is exactly the disk
    n = 32
    y, x = np.mgrid[0:n, 0:n]
    disk = (y - 15.5) ** 2 + (x - 15.5) ** 2 <= 11.0 ** 2
    E = np.where(disk, 1000.0, 0.0) + np.where(disk, 0.0, 1e-3)
    assert np.array_equal(pp.fiber_mask(E.reshape(-1), 0.999), np.flatnonzero(disk.reshape(-1)))
