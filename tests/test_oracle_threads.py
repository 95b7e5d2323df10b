"""The oracle shares its rows among OpenMP threads; every node's arithmetic is
the same whatever the thread count, so states, moments and monitors are
bitwise equal for one thread and for all of them."""
import os

import numpy as np
import pytest

from paper_1610_01388_amd import inputs


@pytest.mark.parametrize("op", ["PR", "IR", "PRI"])
@pytest.mark.parametrize("lat", [0, 2])
def test_threads_bitwise_equal(orc, lat, op):
    dims = (37, 11, 1) if lat == 0 else (19, 13, 9)
    N = int(np.prod(dims))
    mask = (inputs.uniform_array(5, N) < 0.2).astype(np.uint8)
    oop = {"PR": orc.PR, "IR": orc.IR, "PRI": orc.PRI}[op]
    g = (2e-5, -1e-5, 5e-6 if lat else 0.0)
    rh = orc.rheology(oop, 0.1, 5e-5, 1e4, 1e-8, 0.25, g)
    results = []
    keep = orc.set_threads(0)
    try:
        for threads in (1, max(2, os.cpu_count() or 2)):
            assert orc.set_threads(threads) == threads
            d = orc.Domain(lat, dims, (1, 0, 1), rh, mask)
            d.step(12)
            results.append((d.get_state(), d.moments(), d.monitors()))
            d.close()
    finally:
        orc.set_threads(keep)
    (P1, t1), m1, mon1 = results[0]
    (P2, t2), m2, mon2 = results[1]
    assert np.array_equal(P1, P2) and np.array_equal(t1, t2)
    for a, b in zip(m1, m2):
        assert np.array_equal(a, b)
    assert np.array_equal(mon1["flux"], mon2["flux"]) and mon1["mass"] == mon2["mass"]
