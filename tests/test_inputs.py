"""Seeded input generators and the benchmark's work counter (CPU only)."""
import numpy as np
import pytest

from oracle import params
from paper_1607_02904_amd import inputs


def test_diamond_counts_and_box():
    x, box = inputs.diamond(3, 5.431)
    assert x.shape == (216, 3)
    assert np.allclose(box, 3 * 5.431)
    # nearest-neighbour distance a*sqrt(3)/4
    d = np.linalg.norm(x[4] - x[0])
    assert abs(d - 5.431 * np.sqrt(3) / 4) < 1e-12


def test_generators_are_seeded():
    a = inputs.si_bulk(ncell=3)
    b = inputs.si_bulk(ncell=3)
    assert np.array_equal(a[0], b[0])
    c = inputs.si_bulk(ncell=3, seed=99)
    assert not np.array_equal(a[0], c[0])


def test_antisites_keep_composition():
    x, t, box = inputs.sic_bulk(ncell=6)
    assert t.sum() * 2 == len(t)
    ideal = inputs.zincblende_types(len(t))
    assert abs(np.mean(t != ideal) - 0.10) < 0.01


def test_fitting_frames_strain_range():
    frames = inputs.si_frames(nframes=8)
    sides = np.array([f[2][0] for f in frames]) / (4 * 5.431)
    assert np.all(np.abs(sides - 1.0) <= 0.03 + 1e-12)
    assert len(set(np.round(sides, 9))) == 8


def test_liquid_batch_recipe():
    confs = inputs.sic_liquid_batch(nconf=200)
    n = np.array([len(c[1]) for c in confs])
    assert n.min() >= 64 and n.max() <= 4096
    # log-uniform sizes: median near sqrt(64*4096) = 512
    assert 250 < np.median(n) < 1000
    for x, t, box in confs:
        assert np.min(box) >= 6.0  # twice the 3.0 A list cutoff
        # volume-preserving stretch by factors drawn in [0.8, 1.25]
        assert box.max() / box.min() <= 1.25 / 0.8 + 1e-12
        assert np.all((x >= 0) & (x < box))
        rho = len(t) / np.prod(box)
        assert 0.94 * 8 / 4.36 ** 3 < rho < 1.06 * 8 / 4.36 ** 3


def test_bench_work_counter_matches_oracle_lists(orc):
    import bench
    x, t, box = inputs.si_bulk(ncell=6, seed=5)
    tab = params.single(params.SI_B)
    L, P, T = bench.count_work(x, t, box, tab, 3.7, 3.2)
    cnt, lst = orc.neighbours(x, box, 3.7)
    assert L == cnt.sum()
    cin, _ = orc.neighbours(x, box, 3.2)
    assert P == cin.sum()
    assert T == int(np.sum(cin * (cin - 1)))
