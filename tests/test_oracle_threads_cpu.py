"""The oracle's OpenMP build (used only to time the oracle on all host
cores) gives the single-thread build's state exactly: each parallel row loop
writes only its own nodes and keeps the per-node order of operations."""
import numpy as np

import oracle as O
from paper_2302_04120_amd import workloads as WL


def test_openmp_build_state_equals_single_thread_state():
    prm, ini, _ = WL.bubble(n=48, radii=(12,), batch=1, seed=3)
    states = []
    for threads in (0, 3):
        ph = O.Phase(48, 48, prm, threads=threads)
        ph.init(ini["phi"][0], ini["p"][0], ini["ux"][0], ini["uy"][0])
        ph.step(15)
        states.append(ph.get_state())
    assert O.Phase(8, 8, prm, threads=3).threads == 3
    for a, b in zip(*states):
        np.testing.assert_array_equal(a, b)
