"""GPU parity of the forward path (energy, forces, virial, per-atom energy)
against the FP64 oracle, through the C ABI.

Bars: FP64 path <= 1e-12 relative (energy, norm-wise forces, Frobenius
virial); mixed path <= 1e-5 norm-wise on forces and <= 1e-7 relative on the
energy, |dE| <= 1e-7 |E|, with a per-atom floor: where |E|/N is below
E_FLOOR = 1 eV/atom the bar is 1e-7 eV per atom.  The floor only matters for
disordered cells whose repulsive and attractive parts cancel to a few per
cent (|E| -> 0 while each pair term keeps its size): the rounding error of
the FP32 arithmetic has no systematic sign, so the error of the sum scales
with the sum of the term magnitudes (about 40 eV/atom in liquid SiC), not
with |E|, and a relative error of a vanishing energy is not defined.
Crystals (|E|/N > 4 eV/atom) and liquid cells with |E|/N >= 1 eV/atom are
held to the plain relative bar.  Every mixed case prints its |dE|/|E| and
|dE|/N.
Single-precision mode (positions rounded to FP32, FP32 accumulators): the
rounding of a coordinate of up to ~30 A costs ~2e-6 A, i.e. ~1e-6 of a bond
length; the pair exponentials magnify a relative error in r by lambda r ~ 8
and the forces, differences of such terms, by a further order, so the bars
are 2e-5 on the energy (relative to E_rep - E_att) and 2e-4 norm-wise on
forces, virial and per-atom energies.
"""
import numpy as np
import pytest
import torch

from oracle import params
from paper_1607_02904_amd import inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIX_F_TOL = 1e-5
MIX_E_TOL = 1e-7
E_FLOOR = 1.0  # eV/atom, see the module docstring
SP_F_TOL = 2e-4
SP_E_TOL = 2e-5


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def gpu_eval(model, x, t, box, precision, skin=0.0, per_atom=True):
    xd, td = _dev(x), _dev(t, torch.int32)
    model.build_nlist(xd, td, box, skin)
    o = model.compute(xd, td, box, precision, per_atom=per_atom)
    torch.cuda.synchronize()
    model.sync()
    return (float(o["energy"].item()), o["forces"].cpu().numpy(), o["virial"].cpu().numpy(),
            o["e_atom"].cpu().numpy() if per_atom else None)


@pytest.fixture(scope="module")
def si_model():
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    tab = table_element("Si(B)")
    tab[0, 0, 0, params.IDX["R"]] = 2.85
    tab[0, 0, 0, params.IDX["D"]] = 0.15
    m = Tersoff(tab, masses=[28.0855])
    yield m
    m.close()


@pytest.fixture(scope="module")
def sic_model():
    from paper_1607_02904_amd.tersoff import Tersoff, table_sic
    m = Tersoff(table_sic(), masses=[28.0855, 12.011])
    yield m
    m.close()


def _si_table_oracle():
    return params.single(params.SI_B, R=2.85, D=0.15)


def energy_scale(orc, x, t, box, table):
    """S = E_rep - E_att: the repulsive (f_R) and attractive (b f_A) parts of
    the energy, each from the oracle with the other part switched off.  The
    single mode's energy bar is taken relative to it (its error comes from
    rounding the positions to FP32 and scales with the size of the terms)."""
    rep = table.copy()
    rep[..., params.IDX["B"]] = 0.0
    att = table.copy()
    att[..., params.IDX["A"]] = 0.0
    return orc.compute(x, t, box, rep)[0] - orc.compute(x, t, box, att)[0]


def mixed_energy_ok(e, er, n, tag=""):
    """The mixed-path energy bar: |dE| <= 1e-7 max(|E|, E_FLOOR N); prints
    the achieved relative and per-atom errors."""
    d = abs(e - er)
    print("mixed energy %s: |dE|/|E| = %.2e, |dE|/N = %.2e eV (E/N = %+.3f eV)"
          % (tag, d / abs(er) if er else float("inf"), d / max(n, 1), er / max(n, 1)))
    return d <= MIX_E_TOL * max(abs(er), E_FLOOR * n)


def _check(gpu, ref, precision, sp_scale=None):
    """sp_scale: energy scale of the single mode's bar (default |E|)."""
    e, f, w, ea = gpu
    er, fr, wr, ear = ref
    n = len(f)
    if np.abs(fr).max() < 1e-8:
        # perfect lattice: forces vanish, so the bar is absolute
        assert np.abs(f).max() <= (1e-10 if precision == 0 else 1e-5 if precision == 1 else 1e-4)
        fr = f = np.zeros(1)
    if precision == 0:
        assert abs(e - er) <= FP64_TOL * abs(er), (e, er)
        assert _rel(f, fr) <= FP64_TOL, _rel(f, fr)
        assert _rel(w, wr) <= FP64_TOL, _rel(w, wr)
        if ea is not None:
            assert _rel(ea, ear) <= FP64_TOL
    else:
        if precision == 1:
            ftol = MIX_F_TOL
            assert mixed_energy_ok(e, er, n), (e, er)
        else:
            ftol = SP_F_TOL
            assert abs(e - er) <= SP_E_TOL * (abs(er) if sp_scale is None else sp_scale), (e, er)
        assert _rel(f, fr) <= ftol, _rel(f, fr)
        assert _rel(w, wr) <= ftol, _rel(w, wr)
        if ea is not None:
            assert _rel(ea, ear) <= ftol, _rel(ea, ear)


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp64", "mixed", "single"])
def test_si_512(orc, si_model, precision):
    """512-atom Si diamond, sigma 0.05, Si(B) with R = 2.85, D = 0.15."""
    x, t, box = inputs.si_small()
    ref = orc.compute(x, t, box, _si_table_oracle())
    _check(gpu_eval(si_model, x, t, box, precision), ref, precision)


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp64", "mixed", "single"])
@pytest.mark.parametrize("seed", [0, 1])
def test_sic_liquid(orc, sic_model, precision, seed):
    """Disordered SiC with many pairs in the cutoff transition region,
    several hundred atoms (several workgroups, ragged last one)."""
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=700, nmax=1500, seed=100 + seed)[0]
    ref = orc.compute(x, t, box, params.sic())
    sp = energy_scale(orc, x, t, box, params.sic()) if precision == 2 else None
    _check(gpu_eval(sic_model, x, t, box, precision), ref, precision, sp_scale=sp)


SCHEDULES = [(1, 8, 0), (1, 13, 0), (1, 32, 1), (1, 64, 2), (1, 40, 0), (1, 1, 0),
             (2, 1, 0), (2, 7, 0), (2, 16, 0), (2, 32, 0), (3, 0, 0)]


@pytest.mark.parametrize("kernel,atoms,kmax", SCHEDULES)
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_schedules_and_kmax_fallback(orc, sic_model, kernel, atoms, kmax, precision):
    """Both force kernels, every atoms-per-workgroup/wavefront choice and the
    k_max fallback (recompute dzeta/dx_k beyond k_max) reach the same result."""
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=600, nmax=700, seed=7)[0]
    ref = orc.compute(x, t, box, params.sic())
    sic_model.set_schedule(kernel, atoms, kmax)
    try:
        _check(gpu_eval(sic_model, x, t, box, precision), ref, precision)
    finally:
        sic_model.set_schedule(0, 0, 0)


@pytest.mark.parametrize("kernel", [1, 2, 3])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_si_512_both_kernels(orc, si_model, kernel, precision):
    x, t, box = inputs.si_small()
    ref = orc.compute(x, t, box, _si_table_oracle())
    si_model.set_schedule(kernel, 0, 0)
    try:
        _check(gpu_eval(si_model, x, t, box, precision), ref, precision)
    finally:
        si_model.set_schedule(0, 0, 0)


def test_perfect_lattice_zero_force(si_model):
    x, box = inputs.diamond(4, 5.431)
    t = np.zeros(len(x), dtype=np.int32)
    e, f, w, ea = gpu_eval(si_model, x, t, box, 0)
    assert np.max(np.abs(f)) < 1e-10
    assert abs(e / len(x) - (-4.630412064213)) < 1e-11


def test_zincblende_closed_form(sic_model, orc):
    x, box = inputs.diamond(4, 4.36)
    t = inputs.zincblende_types(len(x))
    ref = orc.compute(x, t, box, params.sic())
    _check(gpu_eval(sic_model, x, t, box, 0), ref, 0)


def test_skin_and_atom_order_do_not_matter(sic_model):
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=800, nmax=900, seed=11)[0]
    e0, f0, w0, _ = gpu_eval(sic_model, x, t, box, 0, skin=0.0)
    e1, f1, w1, _ = gpu_eval(sic_model, x, t, box, 0, skin=0.5)
    assert abs(e1 - e0) <= 1e-13 * abs(e0)
    assert _rel(f1, f0) <= 1e-13
    p = np.random.default_rng(0).permutation(len(x))
    e2, f2, w2, _ = gpu_eval(sic_model, x[p], t[p], box, 0)
    assert abs(e2 - e0) <= 1e-13 * abs(e0)
    assert _rel(f2, f0[p]) <= 1e-13


def test_small_and_degenerate(sic_model, orc):
    # dimer in vacuum (zeta = 0), an isolated atom, a carbon trimer
    box = np.array([20.0, 20.0, 20.0])
    x = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 3.2], [10.0, 10.0, 10.0], [15.0, 15.0, 15.0],
                  [16.4, 15.0, 15.0], [15.7, 16.2, 15.0]])
    t = np.array([0, 0, 1, 1, 1, 1], dtype=np.int32)
    ref = orc.compute(x, t, box, params.sic())
    _check(gpu_eval(sic_model, x, t, box, 0), ref, 0)


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp64", "mixed", "single"])
def test_empty_system(sic_model, precision):
    xd = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    td = torch.zeros(0, dtype=torch.int32, device="cuda")
    box = np.array([20.0, 20.0, 20.0])
    sic_model.build_nlist(xd, td, box, 0.0)
    o = sic_model.compute(xd, td, box, precision)
    torch.cuda.synchronize()
    assert float(o["energy"].item()) == 0.0
    assert float(o["virial"].abs().sum().item()) == 0.0
    if precision < 2:
        p = sic_model.pair_compute(xd, box, 0.05, 2.1, 2.5, precision)
        torch.cuda.synchronize()
        assert float(p["energy"].item()) == 0.0
        assert float(p["virial"].abs().sum().item()) == 0.0


def test_accumulate_flag(si_model):
    from paper_1607_02904_amd.tersoff import ACCUMULATE, ENERGY, FORCES
    x, t, box = inputs.si_small(sigma=0.05, seed=3)
    xd, td = _dev(x), _dev(t, torch.int32)
    si_model.build_nlist(xd, td, box, 0.0)
    o = si_model.compute(xd, td, box, 0, virial=False)
    e = torch.zeros(1, dtype=torch.float64, device="cuda") + 1.0
    f = torch.ones((len(x), 3), dtype=torch.float64, device="cuda")
    si_model._chk(si_model._L.ters_compute(si_model._h, len(x), xd.data_ptr(), td.data_ptr(),
                                           np.ascontiguousarray(box).ctypes.data, 0,
                                           ENERGY | FORCES | ACCUMULATE, e.data_ptr(), f.data_ptr(),
                                           None, None))
    torch.cuda.synchronize()
    assert abs(float(e.item()) - 1.0 - float(o["energy"].item())) < 1e-9
    assert torch.allclose(f - 1.0, o["forces"], rtol=0, atol=1e-12)


def test_errors_are_reported(si_model):
    from paper_1607_02904_amd.tersoff import TersoffError
    x, t, box = inputs.si_small()
    xd, td = _dev(x), _dev(t, torch.int32)
    with pytest.raises(TersoffError) as ei:
        si_model.build_nlist(xd, td, np.array([5.0, 30.0, 30.0]), 0.0)
    assert ei.value.name == "TERS_ERR_BOX_TOO_SMALL"
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(TersoffError) as ei:
        si_model.build_nlist(_dev(bad), td, box, 0.0)
    assert ei.value.name == "TERS_ERR_NOT_FINITE"
    tab = si_model.table.copy()
    tab[0, 0, 0, params.IDX["n"]] = -1.0
    with pytest.raises(TersoffError) as ei:
        si_model.set_params(tab)
    assert ei.value.name == "TERS_ERR_PARAMS"
    with pytest.raises(TersoffError) as ei:
        si_model.compute(xd[:10], td[:10], box, 0)
    assert ei.value.name == "TERS_ERR_NO_LIST"
    # a species outside [0, ntypes): the list build refuses it (the force
    # kernels never see it); a valid build afterwards works again
    for bad_t in (1, -1):
        tb = td.clone()
        tb[7] = bad_t
        with pytest.raises(TersoffError) as ei:
            si_model.build_nlist(xd, tb, box, 0.0)
        assert ei.value.name == "TERS_ERR_INVALID_ARG"
    si_model.build_nlist(xd, td, box, 0.0)
    si_model.compute(xd, td, box, 0)
    si_model.sync()
    # the binding checks dtypes and layout before anything reaches the library
    with pytest.raises(TypeError):
        si_model.build_nlist(xd, td.long(), box, 0.0)
    with pytest.raises(TypeError):
        si_model.build_nlist(xd.float(), td, box, 0.0)
    with pytest.raises(ValueError):
        si_model.build_nlist(xd.t().contiguous().t(), td, box, 0.0)
    with pytest.raises(TypeError):
        si_model.build_nlist(xd.cpu(), td, box, 0.0)


# ---------------------------------------------------------------------------
# full sizes: total energy exact, forces on sampled atoms
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def si512k(orc):
    """Si diamond 40^3 cells = 512,000 atoms, sigma 0.1 (the molecular-dynamics
    workload) with the published Si(B) table (R = 3.0, D = 0.2), as the
    benchmark runs it; oracle energy and virial, and forces and per-atom
    energies of 48 sampled atoms from the oracle's local evaluation."""
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    x, t, box = inputs.si_bulk(40)
    tab = params.single(params.SI_B)
    nl = orc.neighbours(x, box, 3.2 + 0.5)
    sample = np.random.default_rng(5).choice(len(x), size=48, replace=False)
    fs, es = orc.forces_on(x, t, box, tab, sample, nlist=nl)
    eref, _, wref, _ = orc.compute(x, t, box, tab, nlist=nl)
    m = Tersoff(table_element("Si(B)"), masses=[28.0855])
    yield x, t, box, sample, fs, es, eref, wref, m
    m.close()


# (kernel, atoms): the workgroup schedule, and the wavefront schedule with 32
# atoms per wavefront that the autotuner picks for this workload
@pytest.mark.parametrize("kernel,atoms", [(1, 0), (2, 32)], ids=["workgroup", "wave32"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_si_512k_full_size(si512k, precision, kernel, atoms):
    """512,000-atom Si in the benchmark's launch configuration (skin 0.5)."""
    x, t, box, sample, fs, es, eref, wref, m = si512k
    m.set_schedule(kernel, atoms, 0)
    try:
        e, f, w, ea = gpu_eval(m, x, t, box, precision, skin=0.5)
    finally:
        m.set_schedule(0, 0, 0)
    tol_f = FP64_TOL if precision == 0 else MIX_F_TOL
    if precision == 0:
        assert abs(e - eref) <= FP64_TOL * abs(eref)
    else:
        assert mixed_energy_ok(e, eref, len(x), "Si 512k")
    assert _rel(f[sample], fs) <= tol_f
    assert _rel(ea[sample], es) <= tol_f
    assert _rel(w, wref) <= tol_f
    # translation invariance at full size
    assert np.linalg.norm(f.sum(0)) <= 1e-9 * len(x) ** 0.5


def test_si_512k_full_size_single(si512k):
    """The single mode (all FP32, the paper's all-single mode) on the
    512,000-atom Si workload in the launch configuration the benchmark times
    for it (wavefront schedule, 32 atoms per wavefront, skin 0.5): energy,
    virial, and forces and per-atom energies of the sampled atoms against
    the oracle, at the single mode's bars."""
    x, t, box, sample, fs, es, eref, wref, m = si512k
    m.set_schedule(2, 32, 0)
    try:
        e, f, w, ea = gpu_eval(m, x, t, box, 2, skin=0.5)
    finally:
        m.set_schedule(0, 0, 0)
    print("single 512k: |dE|/|E| = %.2e, forces %.2e, per-atom %.2e, virial %.2e"
          % (abs(e - eref) / abs(eref), _rel(f[sample], fs), _rel(ea[sample], es), _rel(w, wref)))
    assert abs(e - eref) <= SP_E_TOL * abs(eref)
    assert _rel(f[sample], fs) <= SP_F_TOL
    assert _rel(ea[sample], es) <= SP_F_TOL
    assert _rel(w, wref) <= SP_F_TOL


def test_si_512k_md_full_size(orc, si512k):
    """20 velocity-Verlet steps (1 fs) of the 512,000-atom Si workload in the
    benchmark's launch configuration (wavefront schedule, 32 atoms per
    wavefront, skin 0.5, eight steps per graph launch, rebuilds on the
    device), in FP64 and in mixed precision from the same start: the forces
    on the sampled atoms and the energy of each end state agree with the
    oracle's evaluation of that state, the two precisions follow the same
    trajectory, the list was rebuilt on the device, and the total energy is
    conserved to within the integrator's fluctuation (1e-3 eV per atom; a
    wrong kick or drift factor moves it by far more)."""
    from oracle import oracle as O
    x, t, box, sample, fs, es, eref, wref, m = si512k
    tab = params.single(params.SI_B)
    mass = 28.0855
    n = len(x)
    td = _dev(t, torch.int32)
    ends = {}
    m.set_schedule(2, 32, 0)
    try:
        for prec in (0, 1):
            xd = _dev(x).clone()
            v = torch.zeros_like(xd)
            f = torch.empty_like(xd)
            m.build_nlist(xd, td, box, 0.5)
            m.compute(xd, td, box, prec, energy=False, virial=False, out={"forces": f})
            r0 = m.rebuilds()
            tr = m.md_run(xd, v, f, td, box, 0.001, 20, 0.5, prec)
            torch.cuda.synchronize()
            m.sync()
            ends[prec] = (xd.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy(),
                          float(tr[19].item()), m.rebuilds() - r0)
    finally:
        m.set_schedule(0, 0, 0)
    for prec in (0, 1):
        xe, ve, fe, epot, reb = ends[prec]
        assert reb >= 1, reb
        nl = orc.neighbours(xe, box, 3.2 + 0.5)
        fs_e, _ = orc.forces_on(xe, t, box, tab, sample, nlist=nl)
        e_ref, _, _, _ = orc.compute(xe, t, box, tab, nlist=nl)
        if prec == 0:
            assert _rel(fe[sample], fs_e) <= FP64_TOL
            assert abs(epot - e_ref) <= FP64_TOL * abs(e_ref), (epot, e_ref)
        else:
            assert _rel(fe[sample], fs_e) <= MIX_F_TOL
            assert mixed_energy_ok(epot, e_ref, n, "Si 512k MD")
        ekin = 0.5 * mass * float((ve * ve).sum()) / O.FTM2V
        print("precision %d: rebuilds %d, sampled force error %.2e, energy error %.2e, "
              "total energy change %.2e eV/atom" % (prec, reb, _rel(fe[sample], fs_e),
                                                    abs(epot - e_ref) / abs(e_ref),
                                                    (epot + ekin - eref) / n))
        assert abs(epot + ekin - eref) / n <= 1e-3, (epot + ekin - eref) / n
    dx = np.max(np.abs(ends[1][0] - ends[0][0]))
    print("mixed vs FP64 position difference after 20 steps: %.2e A" % dx)
    assert dx <= 1e-6


@pytest.fixture(scope="module")
def sic1m(orc):
    """SiC zincblende 50^3 cells = 1,000,000 atoms, 10 % antisites, sigma 0.1,
    skin 0.5, with oracle references (32 sampled atoms for the forces)."""
    x, t, box = inputs.sic_bulk(50)
    tab = params.sic()
    nl = orc.neighbours(x, box, 3.0 + 0.5)
    sample = np.random.default_rng(9).choice(len(x), size=32, replace=False)
    fs, es = orc.forces_on(x, t, box, tab, sample, nlist=nl)
    eref, _, wref, _ = orc.compute(x, t, box, tab, nlist=nl)
    return x, t, box, sample, fs, es, eref, wref


# the wavefront schedule with 24 atoms per wavefront is the autotuner's pick
@pytest.mark.parametrize("kernel,atoms", [(1, 0), (2, 24)], ids=["workgroup", "wave24"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_sic_1m_full_size(sic1m, sic_model, precision, kernel, atoms):
    """1,000,000-atom SiC in the benchmark's launch configuration."""
    x, t, box, sample, fs, es, eref, wref = sic1m
    sic_model.set_schedule(kernel, atoms, 0)
    try:
        e, f, w, ea = gpu_eval(sic_model, x, t, box, precision, skin=0.5)
    finally:
        sic_model.set_schedule(0, 0, 0)
    tol_f = FP64_TOL if precision == 0 else MIX_F_TOL
    if precision == 0:
        assert abs(e - eref) <= FP64_TOL * abs(eref)
    else:
        assert mixed_energy_ok(e, eref, len(x), "SiC 1M")
    assert _rel(f[sample], fs) <= tol_f
    assert _rel(ea[sample], es) <= tol_f
    assert _rel(w, wref) <= tol_f
    assert np.linalg.norm(f.sum(0)) <= 1e-9 * len(x) ** 0.5


@pytest.mark.parametrize("kernel", [1, 2])
def test_force_modes_agree_and_gather_is_reproducible(orc, sic_model, kernel):
    """Owner-gather (no atomics) and atomic scatter give the same forces; the
    gather mode is bitwise reproducible run to run."""
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=900, nmax=1200, seed=12)[0]
    ref = orc.compute(x, t, box, params.sic())
    sic_model.set_schedule(kernel, 0, 0)
    try:
        sic_model.set_force_mode(gather=False)
        scat = gpu_eval(sic_model, x, t, box, 0)
        sic_model.set_force_mode(gather=True)
        g1 = gpu_eval(sic_model, x, t, box, 0)
        g2 = gpu_eval(sic_model, x, t, box, 0)
    finally:
        sic_model.set_force_mode(gather=True)
        sic_model.set_schedule(0, 0, 0)
    _check(scat, ref, 0)
    _check(g1, ref, 0)
    assert np.array_equal(g1[1], g2[1])
    assert _rel(scat[1], g1[1]) <= 1e-14


def test_single_precision_is_its_own_mode(orc, sic_model):
    """The single mode rounds positions and accumulates in FP32: its result
    differs from the mixed path's (which is far closer to the oracle), while
    both meet their bars; on a perfect lattice the forces vanish up to the
    rounding of the positions to FP32 (~1e-6 A on a 22 A box: 1e-4 eV/A)."""
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=700, nmax=1500, seed=100)[0]
    ref = orc.compute(x, t, box, params.sic())
    mixed = gpu_eval(sic_model, x, t, box, 1)
    single = gpu_eval(sic_model, x, t, box, 2)
    assert not np.array_equal(mixed[1], single[1])
    assert _rel(mixed[1], ref[1]) < _rel(single[1], ref[1])
    xl, tl, bl = inputs.si_small(sigma=0.0)
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    m = Tersoff(table_element("Si(B)"))
    try:
        e, f, w, ea = gpu_eval(m, xl, tl, bl, 2)
        assert np.abs(f).max() <= 1e-4
    finally:
        m.close()


def test_single_precision_forward_only(si_model):
    """No adjoint and no parameter gradient in the single mode: the library
    refuses them with TERS_ERR_UNSUPPORTED (7)."""
    from paper_1607_02904_amd.tersoff import TersoffError
    x, t, box = inputs.si_small()
    xd, td = _dev(x), _dev(t, torch.int32)
    si_model.build_nlist(xd, td, box, 0.0)
    with pytest.raises(TersoffError) as ei:
        si_model.compute(xd, td, box, 2, param_grad=True)
    assert ei.value.code == 7
    with pytest.raises(TersoffError) as ei:
        si_model.backward(xd, td, box, 1.0, torch.zeros_like(xd), precision=2)
    assert ei.value.code == 7


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_filter_off_gives_the_same_result(orc, sic_model, precision):
    """Without the filter (every skin-list entry takes a lane, the cutoff is
    applied inside the K loops) the wavefront schedule still meets the
    oracle's bars: the filter changes the speed, not the result."""
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=700, nmax=1500, seed=101)[0]
    ref = orc.compute(x, t, box, params.sic())
    sic_model.set_schedule(2, 16, 0)
    sic_model.set_filter(False)
    try:
        xd, td = _dev(x), _dev(t, torch.int32)
        sic_model.build_nlist(xd, td, box, 0.5)  # skin entries present
        o = sic_model.compute(xd, td, box, precision, per_atom=True)
        torch.cuda.synchronize()
        sic_model.sync()
        got = (float(o["energy"].item()), o["forces"].cpu().numpy(), o["virial"].cpu().numpy(),
               o["e_atom"].cpu().numpy())
    finally:
        sic_model.set_filter(True)
        sic_model.set_schedule(0, 0, 0)
    _check(got, ref, precision)


@pytest.mark.parametrize("skin", [0.0, 0.5])
def test_list_is_the_exact_list_up_to_the_rounding_margin(sic_model, skin):
    """The device list tests distances in FP32 on positions wrapped into the
    box, with the radius widened by a bound of that rounding: it holds every
    pair within r_list (counted here in FP64 with a k-d tree, both
    directions) and nothing beyond r_list + 1e-3 A."""
    from scipy.spatial import cKDTree
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=1500, nmax=3000, seed=102)[0]
    xd, td = _dev(x), _dev(t, torch.int32)
    sic_model.build_nlist(xd, td, box, skin)
    st = sic_model.nlist_stats()
    n, entries, longest, cap = st["n"], st["entries"], st["longest"], st["capacity"]
    tab = params.sic()
    rlist = float(np.max(tab[..., params.IDX["R"]] + tab[..., params.IDX["D"]])) + skin
    xw = x - np.floor(x / box) * box
    tree = cKDTree(xw, boxsize=box)
    exact = 2 * len(tree.query_pairs(rlist))
    wide = 2 * len(tree.query_pairs(rlist + 1e-3))
    assert n == len(x) and longest <= cap
    assert exact <= entries <= wide, (exact, entries, wide)


# diamond Si boxes (conventional cells per axis) for the list build's cell
# grid: with a 3.5 A list radius a side of two cells (10.86 A) holds exactly
# three grid cells, the smallest grid the build treats with cell-fixed images
CELL_GRIDS = {"three_cells_per_axis": (2, 2, 2), "elongated": (2, 5, 3), "slab": (5, 4, 2)}


@pytest.mark.parametrize("shape", list(CELL_GRIDS))
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_list_build_cell_grids(orc, si_model, shape, precision):
    """The list build takes each candidate's periodic image from the cell grid
    (a near run of cells and, across the periodic seam, a far run per row):
    boxes with exactly three grid cells along an axis, elongated boxes and
    every seam, with a skin, against the oracle."""
    nx, ny, nz = CELL_GRIDS[shape]
    rng = np.random.default_rng(inputs.seed_for(9, 100 * nx + 10 * ny + nz))
    x, box = inputs.diamond(nx, 5.431, ny, nz)
    x = inputs.wrap(inputs.perturb(x, 0.1, rng), box)
    t = np.zeros(len(x), dtype=np.int32)
    ref = orc.compute(x, t, box, _si_table_oracle())
    _check(gpu_eval(si_model, x, t, box, precision, skin=0.5), ref, precision)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_disordered_si_close_contacts(orc, precision):
    """Disordered single-species Si cells (the batched recipe with Si's
    lattice constant: sites thinned, sigma 0.3 A), four with contacts of
    0.28-0.52 A, where (beta zeta)^n of Si(B) leaves the FP64 range and b is
    about (beta zeta)^(-1/2): energy, forces, virial and per-atom energies
    against the oracle."""
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    confs = inputs.sic_liquid_batch(nconf=256, a=5.431, seed=77)
    model = Tersoff(table_element("Si(B)"), masses=[28.0855])
    try:
        for c in (174, 100, 222, 50):
            x, _, box = confs[c]
            t = np.zeros(len(x), dtype=np.int32)
            ref = orc.compute(x, t, box, params.single(params.SI_B))
            _check(gpu_eval(model, x, t, box, precision), ref, precision)
    finally:
        model.close()


@pytest.mark.parametrize("skin", [2.0, 3.0])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_list_build_crowded_cells(orc, skin, precision):
    """Large cells (a wide skin) on 8,000 Si atoms, each case on a model of
    its own (list capacity from 16): with skin 2.0 A about eight atoms per
    cell, so cells on both sides of the binning pass's eight-atom bucket, and
    capacity 32; with skin 3.0 A about eleven per cell, most of them past the
    bucket, and capacity 64.  Either way one tile of the cell pass holds all
    the atoms, more than it stages at a time.  The list holds every pair
    within r_list and nothing beyond r_list + 1e-3 A (k-d tree count in
    FP64), and the evaluation matches the oracle."""
    from scipy.spatial import cKDTree
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    tab = table_element("Si(B)")
    tab[0, 0, 0, params.IDX["R"]] = 2.85
    tab[0, 0, 0, params.IDX["D"]] = 0.15
    model = Tersoff(tab, masses=[28.0855])
    try:
        rng = np.random.default_rng(inputs.seed_for(13, int(skin * 10)))
        x, box = inputs.diamond(10, 5.431)
        x = inputs.wrap(inputs.perturb(x, 0.1, rng), box)
        t = np.zeros(len(x), dtype=np.int32)
        xd, td = _dev(x), _dev(t, torch.int32)
        model.build_nlist(xd, td, box, skin)
        st = model.nlist_stats()
        rlist = 3.0 + skin
        tree = cKDTree(x, boxsize=box)
        exact = 2 * len(tree.query_pairs(rlist))
        wide = 2 * len(tree.query_pairs(rlist + 1e-3))
        assert st["n"] == len(x) and st["longest"] <= st["capacity"]
        assert exact <= st["entries"] <= wide, (exact, st["entries"], wide)
        assert st["capacity"] == (32 if skin == 2.0 else 64), st
        ref = orc.compute(x, t, box, _si_table_oracle())
        _check(gpu_eval(model, x, t, box, precision, skin=skin), ref, precision)
    finally:
        model.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_list_capacity_growth_to_64(orc, si_model, precision):
    """A 2.6 A skin gives every Si atom 33 or 34 list neighbours (the shells at
    2.35, 3.84, 4.50 and 5.43 A lie within r_list = 5.6 A): the capacity
    grows to 64 and the build stores the entries as it finds them instead of
    collecting them in LDS; the forces only see the in-cutoff pairs."""
    x, t, box = inputs.si_small()
    ref = orc.compute(x, t, box, _si_table_oracle())
    got = gpu_eval(si_model, x, t, box, precision, skin=2.6)
    st = si_model.nlist_stats()
    assert st["capacity"] == 64 and 32 < st["longest"] <= 64, st
    _check(got, ref, precision)


@pytest.mark.parametrize("seed,nmin", [(12, 80), (15, 80)])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_list_build_single_cell_axes(orc, sic_model, seed, nmin, precision):
    """Boxes with sides between two and three list radii hold a single grid
    cell along those axes; there the build takes the minimum image of every
    candidate.  Disordered SiC cells with one or two such axes and one axis of
    three cells, with a skin, against the oracle."""
    x, t, box = inputs.sic_liquid_batch(nconf=1, nmin=nmin, nmax=nmin + 8, seed=seed)[0]
    cells = [int(np.floor(b / 3.5)) for b in box]
    assert min(cells) < 3 <= max(cells), (box, cells)
    ref = orc.compute(x, t, box, params.sic())
    _check(gpu_eval(sic_model, x, t, box, precision, skin=0.5), ref, precision)


def test_thread_schedule_is_forward_only(si_model):
    """The thread-per-atom schedule has no adjoint: ters_backward refuses it
    with TERS_ERR_UNSUPPORTED (7)."""
    from paper_1607_02904_amd.tersoff import TersoffError
    x, t, box = inputs.si_small()
    xd, td = _dev(x), _dev(t, torch.int32)
    si_model.build_nlist(xd, td, box, 0.0)
    si_model.set_schedule(3, 0, 0)
    try:
        with pytest.raises(TersoffError) as ei:
            si_model.backward(xd, td, box, 1.0, torch.zeros_like(xd), precision=0)
        assert ei.value.code == 7
    finally:
        si_model.set_schedule(0, 0, 0)
