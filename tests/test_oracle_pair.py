"""Pins of the pair-potential oracle (truncated Lennard-Jones, the paper's
Algorithm 1 form) against facts that do not restate its formula: the
dimer's minimum and zero crossing, lattice energies fixed by coordination
numbers, finite differences of the energy (forces and virial), and the
conservation of momentum."""
import numpy as np

from oracle import pair

EPS, SIG = 0.0104, 3.40  # argon-like, eV and Angstrom


def test_dimer_minimum_and_zero_crossing():
    rmin = 2.0 ** (1.0 / 6.0) * SIG
    box = np.array([30.0, 30.0, 30.0])
    x = np.array([[1.0, 1.0, 1.0], [1.0 + rmin, 1.0, 1.0]])
    e, f, w = pair.lj_compute(x, box, EPS, SIG, 10.0)
    assert abs(e + EPS) <= 1e-15
    assert np.abs(f).max() <= 1e-15
    x[1, 0] = 1.0 + SIG
    e, f, w = pair.lj_compute(x, box, EPS, SIG, 10.0)
    assert abs(e) <= 1e-15  # rounding of the positions
    assert f[1, 0] > 0.0 and abs(f[0, 0] + f[1, 0]) <= 1e-15  # repulsive at r = sigma


def _simple_cubic(nc, a):
    g = np.arange(nc) * a
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return x, np.full(3, nc * a)


def test_simple_cubic_lattice_shells():
    """6 first neighbours at a, 12 second at sqrt(2) a: E/N = 3 V(a) when
    a < r_c < sqrt(2) a, plus 6 V(sqrt(2) a) when sqrt(2) a < r_c < sqrt(3) a;
    forces vanish by symmetry."""
    a = 3.9
    x, box = _simple_cubic(6, a)
    v = lambda r: 4 * EPS * ((SIG / r) ** 12 - (SIG / r) ** 6)
    e1, f1, _ = pair.lj_compute(x, box, EPS, SIG, 1.2 * a)
    e2, f2, _ = pair.lj_compute(x, box, EPS, SIG, 1.6 * a)
    n = len(x)
    assert abs(e1 / n - 3 * v(a)) <= 1e-14
    assert abs(e2 / n - (3 * v(a) + 6 * v(np.sqrt(2) * a))) <= 1e-14
    assert np.abs(f1).max() <= 1e-14 and np.abs(f2).max() <= 1e-14


def _cluster(seed, n=40):
    rng = np.random.default_rng(seed)
    box = np.array([14.0, 15.0, 16.0])
    # jittered grid: no pair closer than ~2.6 A and none near the cutoff shell
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(3), indexing="ij"),
                 axis=-1).reshape(-1, 3)[:n] * np.array([3.5, 3.75, 5.3])
    return g + rng.normal(0.0, 0.2, g.shape), box


def test_forces_are_minus_the_energy_gradient():
    x, box = _cluster(1)
    rc = 6.0
    e, f, _ = pair.lj_compute(x, box, EPS, SIG, rc)
    h = 1e-5
    for a in (0, 7, 19):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, k] += h
            xm[a, k] -= h
            fd = -(pair.lj_compute(xp, box, EPS, SIG, rc)[0] - pair.lj_compute(xm, box, EPS, SIG, rc)[0]) / (2 * h)
            assert abs(fd - f[a, k]) <= 1e-7 * max(1.0, abs(f[a, k])), (a, k, fd, f[a, k])
    assert np.abs(f.sum(axis=0)).max() <= 1e-14


def test_virial_is_minus_the_strain_derivative():
    x, box = _cluster(2)
    rc = 6.0
    _, _, w = pair.lj_compute(x, box, EPS, SIG, rc)
    h = 1e-6
    for k in range(3):
        s = np.ones(3)
        s[k] = 1 + h
        ep = pair.lj_compute(x * s, box * s, EPS, SIG, rc)[0]
        s[k] = 1 - h
        em = pair.lj_compute(x * s, box * s, EPS, SIG, rc)[0]
        assert abs(-(ep - em) / (2 * h) - w[k]) <= 1e-7 * max(1.0, abs(w[k])), (k, w[k])


def test_pair_enumeration_equals_the_loop_over_all_pairs():
    """lj_compute_pairs (pairs within r_c found by a k-d tree, for large
    systems) gives the energy, forces and virial of lj_compute (every pair
    visited), on a perturbed lattice and on a dense random gas."""
    rng = np.random.default_rng(12)
    a = 3.8
    g = np.arange(8) * a
    x1 = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + rng.normal(0, 0.3, (512, 3))
    box1 = np.full(3, 8 * a)
    box2 = np.array([22.0, 25.0, 21.0])
    x2 = rng.uniform(0, 1, (400, 3)) * box2
    for x, box, rc in ((x1, box1, 8.5), (x2, box2, 9.0)):
        e, f, w = pair.lj_compute(x, box, EPS, SIG, rc)
        e2, f2, w2 = pair.lj_compute_pairs(x, box, EPS, SIG, rc)
        assert abs(e2 - e) <= 1e-12 * abs(e)
        assert np.linalg.norm(f2 - f) <= 1e-12 * np.linalg.norm(f)
        assert np.linalg.norm(w2 - w) <= 1e-12 * np.linalg.norm(w)

