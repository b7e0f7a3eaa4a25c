"""The batched workload's orbits (tests/golden/batched_orbits.txt, written by
make_batched_orbits.py with the oracle): the stored targets are the recipe's
seeded draws, and each stored apocentre speed gives, integrated in the
composite host at the workload's dt, an orbit whose eccentricity
e = (r_apo - r_peri) / (r_apo + r_peri) (Sec. 2.3) is the target."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

from paper_2602_13385_amd import inputs as I  # noqa: E402


def test_stored_orbits_have_the_target_eccentricities(O):
    import make_batched_orbits as M
    rows = np.loadtxt(os.path.join(HERE, "golden", "batched_orbits.txt"))
    w = I.config4()
    assert np.array_equal(rows[:, 0], np.arange(10))
    assert np.allclose(rows[:, 1], w.extra["e_target"], rtol=0, atol=1e-15)
    assert np.allclose(rows[:, 2], w.extra["r_apo"], rtol=0, atol=1e-12)
    H = M.host()
    for i, (e1, e2) in enumerate(w.extra["plane"]):
        c = w.centres[i]
        assert np.allclose(c[:3], rows[i, 2] * e1) and np.allclose(c[3:], rows[i, 3] * e2)
        e = M.eccentricity(H, rows[i, 2], e1, e2, rows[i, 3], w.dt)
        assert e == pytest.approx(rows[i, 1], abs=1e-4), (i, e, rows[i, 1])
        # the speed is below the circular speed: the start is the apocentre
        assert rows[i, 3] < M.circular_speed(H, rows[i, 2], e1)
