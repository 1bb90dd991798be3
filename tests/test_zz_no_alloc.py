"""The no-allocation RCS entry point (cavity_rcs_many_noalloc) against cavity_rcs_many:
two calls in a row on the same device-wide scratch, the second with fewer pairs on a
smaller plan, each equal to the allocating entry point within rounding (the same
aperture-transform partial sums, added on the device in the same order); pairs beyond the
scratch are rejected on the host."""
import numpy as np
import pytest

import paper_2008_01966_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _pairs(nsol, per, rng):
    idx = np.repeat(np.arange(nsol), per)
    th = rng.uniform(0.0, 0.5 * np.pi, idx.size)
    ph = rng.uniform(0.0, 2 * np.pi, idx.size)
    return idx, th, ph


def test_noalloc_rcs_matches_allocating_entry_point():
    rng = np.random.default_rng(7)
    big = W.small_cases()[2]
    print(f"\n[case] {big.name}: 6 solutions x 7 directions", flush=True)
    plan = P.Plan.from_cavity(big.cavity)
    incs = [(0.2 + 0.2 * i, 0.5 * i, i % 2) for i in range(6)]
    plan.solve_batch([t for t, _, _ in incs], [f for _, f, _ in incs], [p for _, _, p in incs],
                     field=False)
    idx, th, ph = _pairs(6, 7, rng)
    ref = plan.rcs_many(idx, th, ph)
    got = plan.rcs_many_noalloc(idx, th, ph)
    assert got.shape == ref.shape == (42, 2)
    assert np.all(ref > 0)
    d1 = float(np.abs(got - ref).max() / ref.max())
    print(f"[compare] first call, 42 pairs: max rel diff {d1:.1e}", flush=True)
    assert d1 <= 1e-13
    # a pair count beyond the 4 MiB scratch is refused before any device work
    n_big = 20000
    with pytest.raises(P.CavityError) as e:
        plan.rcs_many_noalloc(np.zeros(n_big, int), np.full(n_big, 0.3), np.zeros(n_big))
    assert e.value.status == 1
    plan.close()

    small = W.vacuum_1x1x05()
    print(f"[case] {small.name}: 1 solution x 3 directions", flush=True)
    plan2 = P.Plan.from_cavity(small.cavity)
    plan2.solve(0.4, 0.9, W.TM, field=False)
    idx, th, ph = _pairs(1, 3, rng)
    ref2 = plan2.rcs_many(idx, th, ph)
    got2 = plan2.rcs_many_noalloc(idx, th, ph)
    d2 = float(np.abs(got2 - ref2).max() / ref2.max())
    print(f"[compare] second call, 3 pairs: max rel diff {d2:.1e}", flush=True)
    assert got2.shape == (3, 2) and d2 <= 1e-13
    with pytest.raises(P.CavityError):
        plan2.rcs_many_noalloc([1], [0.1], [0.0])      # no such solution
    assert plan2.rcs_many_noalloc([], [], []).shape == (0, 2)
    plan2.close()
