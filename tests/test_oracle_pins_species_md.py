"""More pins of the FP64 oracle (CPU): the per-triplet parameter lookup of two
species, a brute force that shares no code with the oracle, and the time
integration of the molecular-dynamics reference.

The expected values here come from an evaluator written in this file directly
from Tersoff's two-element formulation (Phys. Rev. B 39, 5566 (1989)): per
species parameters, mixed pair parameters (geometric A, B and cutoff radii,
arithmetic lambda, mu, chi on B), the angular function and beta, n of the
centre atom, and Tersoff's own cutoff written with R, S and a cosine.  It reads
no parameter table, so a mistake in how the oracle's table is filled or
looked up (which entry gives the cutoff of r_ik, whose angular parameters a
triplet uses) changes the oracle's result and not this one.
"""
import math

import numpy as np
import pytest

from oracle import params
from paper_1607_02904_amd import inputs

# ---------------------------------------------------------------------------
# Tersoff (1989) evaluator, independent of the oracle code and its tables
# ---------------------------------------------------------------------------

ELEMENTS = {0: params.SI_C, 1: params.CARBON}  # species 0 = Si, 1 = C
CHI = {frozenset([0]): 1.0, frozenset([1]): 1.0, frozenset([0, 1]): 0.9776}


def _pair(si, sj, elements):
    """Mixed pair parameters of species si, sj (Tersoff 1989, Eqs. 1-2)."""
    a, b = elements[si], elements[sj]
    chi = CHI[frozenset([si, sj])] if elements is ELEMENTS else 1.0
    return dict(A=math.sqrt(a["A"] * b["A"]), B=chi * math.sqrt(a["B"] * b["B"]),
                lam=0.5 * (a["lam1"] + b["lam1"]), mu=0.5 * (a["lam2"] + b["lam2"]),
                R=math.sqrt(a["Rt"] * b["Rt"]), S=math.sqrt(a["St"] * b["St"]))


def _fc_rs(r, R, S):
    """Tersoff's cutoff: 1 below R, 1/2 + 1/2 cos(pi (r - R)/(S - R)) up to S."""
    if r < R:
        return 1.0
    if r > S:
        return 0.0
    return 0.5 + 0.5 * math.cos(math.pi * (r - R) / (S - R))


def energy_1989(centres, cpos, cspec, cand_pos, cand_spec, cand_id, elements=ELEMENTS,
                with_scale=False):
    """E = 1/2 sum over centre atoms i and candidate atoms j != i of
    fc(r_ij) [A_ij exp(-lam_ij r_ij) - b_ij B_ij exp(-mu_ij r_ij)], with
    b_ij = (1 + beta_i^n_i zeta_ij^n_i)^(-1/(2 n_i)),
    zeta_ij = sum_{k != i, j} fc(r_ik) g_i(theta_ijk) exp(lam3_i^m (r_ij - r_ik)^m),
    g_i = 1 + c_i^2/d_i^2 - c_i^2 / (d_i^2 + (h_i - cos theta)^2).
    cand_*: every atom (periodic images included) that may neighbour a
    centre; cand_id[q] is the identity of candidate q (centre index in the
    home image, or -1) so that a centre skips itself.  with_scale: also
    return sum |1/2 V_ij|, the scale of the rounding of the sum (disordered
    cells nearly cancel)."""
    e = 0.0
    scale = 0.0
    for ci in range(len(cpos)):
        si = int(cspec[ci])
        el = elements[si]
        d = cand_pos - cpos[ci]
        r = np.sqrt((d * d).sum(1))
        near = [q for q in range(len(r)) if cand_id[q] != centres[ci] and r[q] < 3.5]
        for j in near:
            sj = int(cand_spec[j])
            pj = _pair(si, sj, elements)
            rij = float(r[j])
            fij = _fc_rs(rij, pj["R"], pj["S"])
            if fij == 0.0:
                continue
            zeta = 0.0
            for k in near:
                if k == j:
                    continue
                pk = _pair(si, int(cand_spec[k]), elements)
                rik = float(r[k])
                cos = float(np.dot(d[j], d[k])) / (rij * rik)
                g = 1.0 + el["c"] ** 2 / el["d"] ** 2 - el["c"] ** 2 / (el["d"] ** 2 + (el["h"] - cos) ** 2)
                u = el["lam3"] * (rij - rik)
                zeta += _fc_rs(rik, pk["R"], pk["S"]) * el["gamma"] * g * math.exp(u ** int(el["m"]))
            b = (1.0 + (el["beta"] * zeta) ** el["n"]) ** (-0.5 / el["n"])
            v = 0.5 * fij * (pj["A"] * math.exp(-pj["lam"] * rij) - b * pj["B"] * math.exp(-pj["mu"] * rij))
            e += v
            scale += abs(v)
    return (e, scale) if with_scale else e


def cluster_energy(pos, spec, elements=ELEMENTS):
    n = len(pos)
    return energy_1989(np.arange(n), pos, spec, pos, spec, np.arange(n), elements)


def periodic_energy(x, spec, box, nimg, elements=ELEMENTS, with_scale=False):
    """The same sum over a periodic cell: candidates are all atoms in all
    images with shifts in [-nimg, nimg]^3 (no list, no minimum image)."""
    n = len(x)
    sh = np.array([[a, b, c] for a in range(-nimg, nimg + 1) for b in range(-nimg, nimg + 1)
                   for c in range(-nimg, nimg + 1)], dtype=np.float64)
    cand = (x[None, :, :] + (sh * box)[:, None, :]).reshape(-1, 3)
    cspec = np.tile(spec, len(sh))
    home = np.flatnonzero((sh == 0).all(1))[0]
    cid = np.full(len(cand), -1)
    cid[home * n:(home + 1) * n] = np.arange(n)
    return energy_1989(np.arange(n), x, spec, cand, cspec, cid, elements, with_scale)


def _at(r, theta_deg, phi_deg=0.0):
    t, p = math.radians(theta_deg), math.radians(phi_deg)
    return np.array([r * math.cos(t), r * math.sin(t) * math.cos(p), r * math.sin(t) * math.sin(p)])


# ---------------------------------------------------------------------------
# mixed-species clusters: the per-triplet lookup
# ---------------------------------------------------------------------------

def _clusters():
    """(name, positions, species).  Distances are chosen so that a wrong
    lookup changes the energy:
    * si_centre: Si i with a Si neighbour j at 2.35 A (inside the Si-Si R) and
      a C neighbour k at 2.40 A, inside the Si-C switching band (2.205-2.510)
      but below the Si-Si R (2.7): the r_ik cutoff must be the (i,k) one;
    * c_centre: C i with a C neighbour at 1.5 A and a Si neighbour at 2.40 A,
      beyond the C-C cutoff (2.1): the r_ik cutoff from (i,j) would drop k;
      the angular terms of both pairs must be C's;
    * mixed_4 and mixed_5: several species around one centre, pairs in the
      switching bands of Si-Si (2.7-3.0), Si-C and C-C (1.8-2.1)."""
    o = np.zeros(3)
    cl = []
    cl.append(("si_centre", np.array([o, _at(2.35, 0), _at(2.40, 109.47)]), [0, 0, 1]))
    cl.append(("c_centre", np.array([o, _at(1.5, 0), _at(2.40, 100.0)]), [1, 1, 0]))
    cl.append(("mixed_4", np.array([o, _at(2.80, 0), _at(2.30, 105.0), _at(1.95, 115.0, 120.0)]),
               [0, 0, 1, 1]))
    cl.append(("mixed_5", np.array([o, _at(2.05, 0), _at(2.45, 95.0), _at(2.85, 118.0, 125.0),
                                    _at(1.6, 112.0, 240.0)]), [1, 0, 0, 0, 1]))
    return cl


@pytest.mark.parametrize("perm", [0, 1, 2])
@pytest.mark.parametrize("name,pos,spec", _clusters(), ids=lambda v: v if isinstance(v, str) else "")
def test_mixed_species_cluster_energy(orc, name, pos, spec, perm):
    """Oracle (table P[ti][tj][tk] from params.sic) = Tersoff 1989 evaluated
    directly, for clusters in vacuum, with the atoms in three orders (j and k
    exchanged, centre moved)."""
    spec = np.array(spec, dtype=np.int32)
    order = [np.arange(len(spec)), np.r_[0, np.arange(len(spec))[1:][::-1]],
             np.roll(np.arange(len(spec)), 1)][perm]
    pos = pos[order] + 12.0
    spec = spec[order]
    want = cluster_energy(pos, spec)
    e, f, _, ea = orc.compute(pos, spec, np.array([40.0, 40.0, 40.0]), params.sic())
    assert abs(e - want) <= 1e-13 * abs(want), (e, want)
    assert abs(ea.sum() - e) <= 1e-13 * abs(e)


def test_mixed_species_cluster_forces_fd(orc):
    """Oracle forces on the five-atom mixed cluster = minus the central
    difference of the Tersoff 1989 energy (h = 1e-5 A, 4-point stencil)."""
    name, pos, spec = _clusters()[3]
    pos = pos + 12.0
    spec = np.array(spec, dtype=np.int32)
    _, f, _, _ = orc.compute(pos, spec, np.array([40.0] * 3), params.sic())
    h = 1e-5
    fd = np.zeros_like(pos)
    for a in range(len(pos)):
        for c in range(3):
            def e_at(s):
                p = pos.copy()
                p[a, c] += s
                return cluster_energy(p, spec)
            fd[a, c] = -(8 * (e_at(h) - e_at(-h)) - (e_at(2 * h) - e_at(-2 * h))) / (12 * h)
    assert np.linalg.norm(f - fd) <= 1e-8 * np.linalg.norm(fd)


def test_cutoff_forms_agree():
    """The table's (R, D) sine switch equals Tersoff's (R, S) cosine switch
    with R_table = (R + S)/2, D = (S - R)/2 (the oracle uses the former)."""
    for el in (params.SI_C, params.CARBON, params.SI_B):
        Rt, St = el["Rt"], el["St"]
        R, D = 0.5 * (Rt + St), 0.5 * (St - Rt)
        for r in np.linspace(Rt - 0.1, St + 0.1, 41):
            sine = 1.0 if r < R - D else (0.0 if r > R + D else 0.5 - 0.5 * math.sin(math.pi * (r - R) / (2 * D)))
            assert abs(sine - _fc_rs(r, Rt, St)) <= 1e-15


# ---------------------------------------------------------------------------
# brute force with periodic images, sharing no code with the oracle
# ---------------------------------------------------------------------------

def test_independent_bruteforce_si_b(orc):
    """64-atom Si(B) cell (2x2x2 diamond, sigma 0.15): the oracle over its
    cell list = the Tersoff sum over explicit images (this file's evaluator,
    m = 3 and lambda3 != 0 exercised)."""
    x, t, box = inputs.si_small(sigma=0.15, ncell=2, seed=11)
    el = {0: params.SI_B}
    want = periodic_energy(x, t, box, 1, el)
    e = orc.compute(x, t, box, params.single(params.SI_B))[0]
    assert abs(e - want) <= 1e-13 * abs(want)


def test_independent_bruteforce_sic_liquid(orc):
    """Disordered SiC (64-300 atoms, sigma 0.3, many pairs in the switching
    bands): the oracle = the explicit-image Tersoff 1989 sum, to 1e-13 of
    the sum of the terms' magnitudes (these cells' repulsive and attractive
    parts cancel to a small total, which the summation order then rounds)."""
    for seed in (21, 22):
        x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=64, nmax=300, seed=seed)[0]
        want, scale = periodic_energy(x, t, box, 1, with_scale=True)
        e = orc.compute(x, t, box, params.sic())[0]
        assert abs(e - want) <= 1e-13 * scale, (seed, e, want, scale)


def test_independent_bruteforce_single_cell_images(orc):
    """One 8-atom diamond cell (box below twice the cutoff, so only explicit
    images work): the oracle's image brute force = this file's."""
    x, box = inputs.diamond(1, 5.431)
    x = inputs.perturb(x, 0.1, np.random.default_rng(5))
    t = np.zeros(8, dtype=np.int32)
    want = periodic_energy(x, t, box, 1, {0: params.SI_B})
    e = orc.compute_images(x, t, box, params.single(params.SI_B), 1)[0]
    assert abs(e - want) <= 1e-13 * abs(want)


# ---------------------------------------------------------------------------
# time integration (metal units)
# ---------------------------------------------------------------------------

def test_force_to_acceleration_constant_from_codata():
    """eV / (Angstrom amu) in Angstrom / ps^2 from the SI values (CODATA 2018:
    e = 1.602176634e-19 C exactly, u = 1.66053906660e-27 kg)."""
    from oracle import oracle
    ev, amu = 1.602176634e-19, 1.66053906660e-27
    acc_si = ev / 1e-10 / amu           # m / s^2
    want = acc_si * 1e10 / 1e24          # Angstrom / ps^2
    assert abs(oracle.FTM2V - want) <= 1e-12 * want


def _md_system():
    x, t, box = inputs.si_small(sigma=0.1, ncell=2, seed=17)
    rng = np.random.default_rng(18)
    v = rng.normal(0.0, 5.0, size=x.shape)   # Angstrom / ps (a few hundred K)
    v -= v.mean(0)
    return x, t, box, v


def _total_energy(orc, x, t, box, tab, v, mass):
    e = orc.compute(x, t, box, tab)[0]
    return e + 0.5 * mass * float((v * v).sum()) / orc.FTM2V


def test_velocity_verlet_is_time_reversible(orc):
    """40 steps forward, velocities negated, 40 steps back: the positions
    return to the start (velocity Verlet is symmetric in time)."""
    x0, t, box, v0 = _md_system()
    tab = params.single(params.SI_B)
    m = [28.0855]
    x1, v1, _, _ = orc.velocity_verlet(x0, v0, t, box, tab, m, 0.001, 40)
    x2, v2, _, _ = orc.velocity_verlet(x1, -v1, t, box, tab, m, 0.001, 40)
    d = x2 - x0
    d -= box * np.round(d / box)
    assert np.abs(d).max() <= 1e-10
    assert np.abs(v2 + v0).max() <= 1e-8


def test_velocity_verlet_energy_error_scales_with_dt_squared(orc):
    """Largest deviation of the total energy (potential + kinetic with the
    CODATA constant) over 20 fs with dt = 2 fs and dt = 1 fs: ratio ~ 4."""
    x0, t, box, v0 = _md_system()
    tab = params.single(params.SI_B)
    mass = 28.0855
    dev = []
    for dt, nsteps in ((0.002, 10), (0.001, 20)):
        x, v = x0.copy(), v0.copy()
        e0 = _total_energy(orc, x, t, box, tab, v, mass)
        worst = 0.0
        step = 2 if dt == 0.001 else 1  # compare at the same times
        for k in range(nsteps // step):
            x, v, _, _ = orc.velocity_verlet(x, v, t, box, tab, [mass], dt, step)
            worst = max(worst, abs(_total_energy(orc, x, t, box, tab, v, mass) - e0))
        dev.append(worst)
    ratio = dev[0] / dev[1]
    assert 3.0 < ratio < 5.0, (dev, ratio)
