"""FP64 CPU oracle of a pair potential over a periodic cell (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg
use it).

The paper's Algorithm 1 (Section II) is the plain pair-potential loop
E = 1/2 sum_i sum_{j in N_i} V(r_ij) that the Tersoff algorithms extend; the
pair potential here is Lennard-Jones, truncated (not shifted) at r_c:

    V(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6)   for r < r_c, 0 beyond.

Everything is written out over all pairs (i < j) with the minimum image, no
neighbour list: energy, forces F_a = -dE/dx_a and the virial
W = sum over pairs of d_ij (x) f_j (d_ij = x_j - x_i, f_j the pair's force on
j), the same convention as the Tersoff oracle's virial.
"""
import numpy as np


def lj_pair(r, eps, sigma):
    """V(r) and -dV/dr / r (the factor that turns d_ij into the force on j)."""
    s6 = (sigma / r) ** 6
    v = 4.0 * eps * (s6 * s6 - s6)
    g = 24.0 * eps * (2.0 * s6 * s6 - s6) / (r * r)
    return v, g


def lj_compute(x, box, eps, sigma, rc):
    """Energy, forces [n][3] and virial [xx, yy, zz, xy, xz, yz] of the
    truncated Lennard-Jones potential, O(N^2) over pairs with the minimum
    image (every box side must be at least 2 r_c)."""
    x = np.asarray(x, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(x)
    e = 0.0
    f = np.zeros((n, 3))
    w = np.zeros(6)
    for i in range(n - 1):
        d = x[i + 1:] - x[i]
        d -= box * np.round(d / box)
        r = np.sqrt(np.sum(d * d, axis=1))
        m = r < rc
        if not np.any(m):
            continue
        js = np.nonzero(m)[0] + i + 1
        dm = d[m]
        v, g = lj_pair(r[m], eps, sigma)
        e += float(np.sum(v))
        fj = g[:, None] * dm  # force on j from the pair (i, j)
        np.add.at(f, js, fj)
        f[i] -= np.sum(fj, axis=0)
        w += np.array([np.sum(dm[:, 0] * fj[:, 0]), np.sum(dm[:, 1] * fj[:, 1]),
                       np.sum(dm[:, 2] * fj[:, 2]), np.sum(dm[:, 0] * fj[:, 1]),
                       np.sum(dm[:, 0] * fj[:, 2]), np.sum(dm[:, 1] * fj[:, 2])])
    return e, f, w


def lj_compute_pairs(x, box, eps, sigma, rc):
    """The same energy, forces and virial as lj_compute, with the pairs
    within r_c enumerated by a k-d tree over the periodic box (a library
    primitive standing in for the loop over all pairs, for systems too large
    for it); the sums are the definition's, pair by pair."""
    from scipy.spatial import cKDTree
    x = np.asarray(x, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(x)
    xw = x - np.floor(x / box) * box
    pairs = cKDTree(xw, boxsize=box).query_pairs(rc, output_type="ndarray")
    f = np.zeros((n, 3))
    if len(pairs) == 0:
        return 0.0, f, np.zeros(6)
    i, j = pairs[:, 0], pairs[:, 1]
    d = x[j] - x[i]
    d -= box * np.round(d / box)
    r = np.sqrt(np.sum(d * d, axis=1))
    m = r < rc
    i, j, d, r = i[m], j[m], d[m], r[m]
    v, g = lj_pair(r, eps, sigma)
    fj = g[:, None] * d
    np.add.at(f, j, fj)
    np.add.at(f, i, -fj)
    w = np.array([np.sum(d[:, 0] * fj[:, 0]), np.sum(d[:, 1] * fj[:, 1]), np.sum(d[:, 2] * fj[:, 2]),
                  np.sum(d[:, 0] * fj[:, 1]), np.sum(d[:, 0] * fj[:, 2]), np.sum(d[:, 1] * fj[:, 2])])
    return float(np.sum(v)), f, w
