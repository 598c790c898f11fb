"""Seeded synthetic atomic configurations.

The paper measures on LAMMPS's Si benchmark: diamond-cubic silicon on a
perfect lattice, every atom with four nearest neighbours (Section VI).  That
input file is not shipped; these generators build configurations of the same
structure and size, plus the two-species and disordered variants used for
testing and measurement.  Everything is seeded (NumPy PCG64).

This module holds geometry only (lattices, displacements, species labels,
box shapes).  It contains no part of the potential, so both the GPU path and
the FP64 reference may consume its output.
"""
import math

import numpy as np

DIAMOND_BASIS = np.array([
    [0.00, 0.00, 0.00], [0.00, 0.50, 0.50], [0.50, 0.00, 0.50], [0.50, 0.50, 0.00],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])
SEED_BASE = 1607


def seed_for(config, frame=0):
    """Seed convention: 1607 + 10 * config index + frame."""
    return SEED_BASE + 10 * config + frame


def diamond(nx, a, ny=None, nz=None):
    """Diamond-cubic lattice of nx*ny*nz conventional cells (8 atoms each).
    Returns positions [N,3] (float64) and the orthorhombic box [3].
    Sub-lattice A (fcc sites) comes first within each cell."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
    x = (cells[:, None, :] + DIAMOND_BASIS[None, :, :]).reshape(-1, 3) * a
    box = np.array([nx * a, ny * a, nz * a], dtype=np.float64)
    return x, box


def zincblende_types(n_atoms):
    """Species for a diamond() lattice read as zincblende: fcc sites species 0
    (Si), the (1/4,1/4,1/4)-shifted sites species 1 (C)."""
    per = np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.int32)
    return np.tile(per, n_atoms // 8)


def perturb(x, sigma, rng):
    """Independent Gaussian displacement of every Cartesian component."""
    return x + rng.normal(0.0, sigma, size=x.shape)


def antisite_swap(types, frac, rng):
    """Exchange species on floor(frac/2 * N) randomly chosen sites of each
    species, so that `frac` of all sites end up on the wrong sub-lattice while
    the composition stays unchanged."""
    types = types.copy()
    n = types.size
    k = int(math.floor(0.5 * frac * n))
    a = rng.choice(np.flatnonzero(types == 0), size=k, replace=False)
    b = rng.choice(np.flatnonzero(types == 1), size=k, replace=False)
    types[a] = 1
    types[b] = 0
    return types


def wrap(x, box):
    """Fold positions into [0, L) per axis."""
    return x - np.floor(x / box) * box


# --------------------------------------------------------------------------
# Workloads (sizes and structure of the measured configurations)
# --------------------------------------------------------------------------

def si_small(sigma=0.05, ncell=4, a=5.431, seed=None):
    """512-atom Si diamond (4^3 cells, a = 5.431 A), Gaussian sigma 0.05 A."""
    rng = np.random.default_rng(seed_for(0) if seed is None else seed)
    x, box = diamond(ncell, a)
    x = perturb(x, sigma, rng)
    return wrap(x, box), np.zeros(len(x), dtype=np.int32), box


def si_bulk(ncell=40, sigma=0.1, a=5.431, seed=None):
    """Si diamond ncell^3 cells (20 -> 64,000 atoms, 40 -> 512,000 atoms),
    Gaussian sigma 0.1 A, zero initial velocities."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    x, box = diamond(ncell, a)
    x = perturb(x, sigma, rng)
    return wrap(x, box), np.zeros(len(x), dtype=np.int32), box


def sic_bulk(ncell=50, a=4.36, antisite=0.10, sigma=0.1, seed=None):
    """SiC zincblende ncell^3 cells (50 -> 1,000,000 atoms), 10 % antisites,
    Gaussian sigma 0.1 A.  Species 0 = Si, 1 = C."""
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    x, box = diamond(ncell, a)
    t = zincblende_types(len(x))
    t = antisite_swap(t, antisite, rng)
    x = perturb(x, sigma, rng)
    return wrap(x, box), t, box


def si_frames(nframes=64, ncell=4, a=5.431, sigma=0.15, strain=0.03):
    """Fitting frames: 512-atom Si cells, each with its own isotropic strain
    s ~ U(-0.03, 0.03) and Gaussian sigma 0.15 A.  Frame f uses seed 1607+30+f."""
    frames = []
    for f in range(nframes):
        rng = np.random.default_rng(seed_for(3, f))
        s = rng.uniform(-strain, strain)
        x, box = diamond(ncell, a * (1.0 + s))
        x = perturb(x, sigma, rng)
        frames.append((wrap(x, box), np.zeros(len(x), dtype=np.int32), box))
    return frames


def sic_liquid_batch(nconf=1024, nmin=64, nmax=4096, a=4.36, sigma=0.3, rho_jitter=0.05,
                     aspect=(0.8, 1.25), min_side=6.0, seed=None):
    """Many uneven disordered SiC configurations.

    Atom count N_c = round(exp(U(ln nmin, ln nmax))); start from the smallest
    cubic zincblende supercell with 8 n^3 >= N_c (50/50 species), delete random
    sites down to N_c, scale the box to the zincblende number density times
    U(1 - rho_jitter, 1 + rho_jitter), stretch the axes by volume-preserving
    log-uniform factors in `aspect`, then displace every component by a
    Gaussian of width sigma.  A box with a side below `min_side` is redrawn."""
    rng = np.random.default_rng(seed_for(4) if seed is None else seed)
    rho0 = 8.0 / a ** 3
    out = []
    while len(out) < nconf:
        nc = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        nc = max(nmin, min(nmax, nc))
        m = 1
        while 8 * m ** 3 < nc:
            m += 1
        xs, _ = diamond(m, 1.0)
        ts = zincblende_types(len(xs))
        keep = np.sort(rng.choice(len(xs), size=nc, replace=False))
        xs, ts = xs[keep] / m, ts[keep]  # fractional coordinates in [0,1)
        rho = rho0 * rng.uniform(1.0 - rho_jitter, 1.0 + rho_jitter)
        side = (nc / rho) ** (1.0 / 3.0)
        f = np.exp(rng.uniform(math.log(aspect[0]), math.log(aspect[1]), size=3))
        f /= np.prod(f) ** (1.0 / 3.0)
        box = side * f
        if np.min(box) < min_side:
            continue
        x = perturb(xs * box, sigma, rng)
        out.append((wrap(x, box), ts.astype(np.int32), box))
    return out
