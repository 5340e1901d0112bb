"""Host logic: the X^T z accumulation of the z pass is exact in any order.

Each wave's float32 tile sum is rounded to a multiple of 2^-24 by adding and
subtracting C = 1.5 * 2^28 in float64 before it enters a float64
accumulator.  Multiples of 2^-24 below 2^29 in magnitude are exactly
representable in float64 (53-bit significand), so every partial sum is exact
and the total does not depend on which block summed which tiles or in what
order -- the property that keeps dynamically dealt tiles reproducible.
"""
import numpy as np

C = 1.5 * 2.0**28


def on_grid(v):
    v = np.asarray(v, np.float64)
    return (v + C) - C


def test_rounding_is_to_the_grid():
    rng = np.random.default_rng(3)
    v = (rng.standard_normal(100_000) * 10.0 ** rng.uniform(-6, 6, 100_000)).astype(np.float32)
    v = v[np.abs(v) < 2.0**26]
    q = on_grid(v)
    assert np.all(q * 2.0**24 == np.round(q * 2.0**24))       # multiples of 2^-24
    assert np.all(np.abs(q - v.astype(np.float64)) <= 2.0**-25)  # round to nearest


def test_sums_do_not_depend_on_order():
    rng = np.random.default_rng(4)
    # tile sums of the size the z pass produces (8 rows of |x z| ~ 1), 2^17 of them
    v = (rng.standard_normal(1 << 17) * 8.0).astype(np.float32)
    q = on_grid(v)
    ref = None
    for seed in range(5):
        perm = np.random.default_rng(seed).permutation(q.size)
        # block partials of uneven sizes, then a sum of the partials
        cuts = np.sort(np.random.default_rng(100 + seed).choice(q.size, 479, replace=False))
        parts = [np.sum(c, dtype=np.float64) for c in np.split(q[perm], cuts)]
        s = 0.0
        for x in parts:
            s += x
        ref = s if ref is None else ref
        assert s == ref
    assert ref == np.sum(q.astype(object))  # equals the exact rational sum


def test_unrounded_sums_do_depend_on_order():
    # the same experiment without the rounding: float64 sums of float32 values
    # of mixed magnitude differ between orders, so the rounding is what matters
    rng = np.random.default_rng(5)
    v = (rng.standard_normal(1 << 17) * 10.0 ** rng.uniform(-3, 3, 1 << 17)).astype(np.float64)
    sums = set()
    for seed in range(5):
        perm = np.random.default_rng(seed).permutation(v.size)
        s = 0.0
        for x in np.array_split(v[perm], 480):
            s += np.sum(x)
        sums.add(s)
    assert len(sums) > 1
