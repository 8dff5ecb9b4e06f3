"""The 4-sub-sweep ordering of the oracle (the alternative the paper suggests in Sec. II.A.2).

Pins: the classes are conflict-free for the 19-point stencil (checked over all offsets); so a
snapshot sub-sweep equals cell-by-cell Gauss-Seidel in any order (brute force at 6^3), which the
red-black colouring does not satisfy (its diagonal neighbours share a colour); and both orderings
reach the same solution (the fixed point does not depend on the ordering).
Measured, parity unpinned: on lognormal fields both orderings take the same number of V-cycles.
"""
import itertools

import numpy as np
import pytest

import inputs
from oracle import multigrid as mg
from oracle import operator as op

OFFSETS = [o for o in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(map(abs, o)) <= 2]


def test_classes_are_conflict_free_and_balanced():
    assert len(OFFSETS) == 18
    n = 8
    cls = mg.four_colour_classes(n)
    for o in OFFSETS:
        assert not np.any(np.roll(cls, o, axis=(0, 1, 2)) == cls), o
    assert np.bincount(cls.ravel()).tolist() == [n ** 3 // 4] * 4
    # the red-black colouring is not: the edge (diagonal) neighbours share the colour
    red = mg.red_mask(n)
    assert np.all(np.roll(red, (1, 1, 0), axis=(0, 1, 2)) == red)


def _sequential(theta, delta, mask, m, order):
    th = theta.copy()
    for c in order:
        if not mask[c]:
            continue
        L = op.laplacian(th, 1.0) - (op.source(th, delta, 1.0) - m)
        th[c] = th[c] + L[c] / 6.0
    return th


def test_snapshot_sub_sweep_is_exact_gauss_seidel():
    n = 6
    rng = np.random.default_rng(40)
    theta = 0.05 * rng.standard_normal((n, n, n))
    delta = rng.uniform(-0.5, 0.5, (n, n, n))
    m = float(op.source(theta, delta, 1.0).mean())
    cells = list(itertools.product(range(n), repeat=3))
    cls = mg.four_colour_classes(n)
    for c in range(4):
        mask = cls == c
        snap = mg.class_sweep(theta, delta, None, 1.0, mask, m)
        for seed in (0, 1):
            order = [cells[t] for t in np.random.default_rng(seed).permutation(len(cells))]
            np.testing.assert_allclose(_sequential(theta, delta, mask, m, order), snap, rtol=0, atol=1e-15)
    # red-black: the sequential order changes the result
    red = mg.red_mask(n)
    snap = mg.class_sweep(theta, delta, None, 1.0, red, m)
    seq = _sequential(theta, delta, red, m, cells)
    assert np.abs(seq - snap).max() > 1e-6


def test_orderings_reach_the_same_solution():
    delta = inputs.lognormal(16, 0.6, 3.0, 41)
    a, ia = mg.solve(delta, tol=1e-11)
    b, ib = mg.solve(delta, tol=1e-11, ordering="4c")
    assert ia["converged"] and ib["converged"]
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-9 * np.abs(a).max())


def test_cycle_counts_are_alike():
    """Measured, parity unpinned (no independent value for a cycle count)."""
    delta = inputs.lognormal(32, 1.0, 2.0, 1002)
    _, ia = mg.solve(delta, tol=1e-8)
    _, ib = mg.solve(delta, tol=1e-8, ordering="4c")
    print(f"32^3 lognormal sigma_g = 1: V-cycles to 1e-8, red-black {ia['cycles']}, 4 classes {ib['cycles']}")
    assert abs(ia["cycles"] - ib["cycles"]) <= 1


def test_unknown_ordering_is_rejected():
    with pytest.raises(ValueError):
        mg.sweep(np.zeros((4, 4, 4)), np.zeros((4, 4, 4)), None, 1.0, ordering="8c")
