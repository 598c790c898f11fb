"""The oracle's threaded timing entry point (centres shared among OpenMP
threads, per-thread force arrays) gives the single-threaded oracle's
energy, forces and virial up to the order of the final sums."""
import numpy as np

from oracle import oracle, params
from paper_1607_02904_amd import inputs


import pytest


@pytest.mark.parametrize("threads", [0, 1])
def test_threaded_oracle_equals_serial(threads):
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=900, nmax=1000, seed=5)[0]
    tab = params.sic()
    nl = oracle.neighbours(x, box, 3.0)
    e1, f1, w1, _ = oracle.compute(x, t, box, tab, nlist=nl)
    e2, f2, w2, nthr = oracle.compute_threads(x, t, box, tab, nl, threads=threads)
    assert nthr >= 1 and (threads == 0 or nthr == threads)
    assert abs(e2 - e1) <= 1e-13 * abs(e1)
    assert np.linalg.norm(f2 - f1) <= 1e-13 * np.linalg.norm(f1)
    assert np.linalg.norm(w2 - w1) <= 1e-13 * np.linalg.norm(w1)
