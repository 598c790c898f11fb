"""GPU molecular dynamics (velocity Verlet with device-side list rebuilds,
graph-captured step) and batched evaluation (many configurations, one graph
launch) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import params
from paper_1607_02904_amd import inputs

pytestmark = pytest.mark.gpu
MASS_SI = 28.0855


@pytest.fixture(scope="module")
def si_model():
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    m = Tersoff(table_element("Si(B)"), masses=[MASS_SI])
    yield m
    m.close()


def _md_gpu(model, x, t, box, nsteps, skin, precision=0, use_graph=True, dt=0.001):
    xd = torch.as_tensor(x, device="cuda").clone()
    td = torch.as_tensor(t, device="cuda")
    v = torch.zeros_like(xd)
    f = torch.empty_like(xd)
    model.build_nlist(xd, td, box, skin)
    model.compute(xd, td, box, precision, energy=False, virial=False, out={"forces": f})
    tr = model.md_run(xd, v, f, td, box, dt, nsteps, skin, precision, use_graph=use_graph)
    torch.cuda.synchronize()
    model.sync()
    return xd.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy(), tr.cpu().numpy()[:nsteps]


@pytest.mark.parametrize("use_graph,kernel", [(True, 1), (False, 1), (True, 2), (True, 3)])
def test_md_matches_oracle_verlet(orc, si_model, use_graph, kernel):
    """30 steps of 1 fs on a 1000-atom Si cell (sigma 0.1, v0 = 0), list with
    skin 0.5 rebuilt on the device when due, against the oracle's velocity
    Verlet that rebuilds its list at every step."""
    x, t, box = inputs.si_bulk(ncell=5, seed=21)
    si_model.set_schedule(kernel, 0, 0)
    try:
        xg, vg, fg, trg = _md_gpu(si_model, x, t, box, 30, 0.5, use_graph=use_graph)
    finally:
        si_model.set_schedule(0, 0, 0)
    xo, vo, fo, tro = orc.velocity_verlet(x, np.zeros_like(x), t, box, params.single(params.SI_B),
                                          [MASS_SI], 0.001, 30)
    assert np.max(np.abs(xg - xo)) < 1e-10
    assert np.max(np.abs(vg - vo)) < 1e-8
    assert np.max(np.abs(trg - tro)) <= 1e-11 * abs(tro[0])


def test_md_graph_equals_eager_and_rebuilds_happen(si_model):
    x, t, box = inputs.si_bulk(ncell=5, seed=22)
    a = _md_gpu(si_model, x, t, box, 40, 0.1, use_graph=True)
    r0 = si_model.rebuilds()
    b = _md_gpu(si_model, x, t, box, 40, 0.1, use_graph=False)
    r1 = si_model.rebuilds()
    assert r1 - r0 > 0  # a small skin forces device-side rebuilds
    assert np.array_equal(a[0], b[0]) or np.max(np.abs(a[0] - b[0])) < 1e-12
    c = _md_gpu(si_model, x, t, box, 40, 0.5, use_graph=True)
    # the skin never changes the trajectory beyond rounding
    assert np.max(np.abs(a[0] - c[0])) < 1e-10


def _total_energy_deviation(model, x, t, box, dt, total_time, chunk):
    """Largest |E_kin + E_pot - E_0| per atom along a trajectory, sampled
    every `chunk` steps (list rebuilt on the device as needed)."""
    n = len(t)
    xd = torch.as_tensor(x, device="cuda").clone()
    td = torch.as_tensor(t, device="cuda")
    v = torch.zeros_like(xd)
    f = torch.empty_like(xd)
    model.build_nlist(xd, td, box, 0.5)
    o = model.compute(xd, td, box, 0, virial=False, out={"forces": f})
    e0 = float(o["energy"].item())
    dev = 0.0
    for _ in range(int(round(total_time / dt / chunk))):
        tr = model.md_run(xd, v, f, td, box, dt, chunk, 0.5, 0)
        torch.cuda.synchronize()
        ke = 0.5 * MASS_SI * float((v ** 2).sum().item()) / O.FTM2V
        dev = max(dev, abs(float(tr[chunk - 1].item()) + ke - e0) / n)
    model.sync()
    return dev


def test_md_energy_conservation(si_model):
    """Velocity Verlet conserves the total energy up to an O(dt^2)
    oscillation: halving dt divides the largest deviation by about four, and
    the deviation stays small."""
    x, t, box = inputs.si_bulk(ncell=6, seed=23)
    d1 = _total_energy_deviation(si_model, x, t, box, 0.001, 0.2, 10)
    d2 = _total_energy_deviation(si_model, x, t, box, 0.0005, 0.2, 20)
    assert d1 < 1e-3
    assert 3.0 < d1 / d2 < 5.5, (d1, d2)


def test_md_mixed_runs_and_tracks_fp64(si_model):
    x, t, box = inputs.si_bulk(ncell=5, seed=24)
    a = _md_gpu(si_model, x, t, box, 20, 0.5, precision=0)
    b = _md_gpu(si_model, x, t, box, 20, 0.5, precision=1)
    assert np.max(np.abs(a[0] - b[0])) < 1e-5
    assert np.max(np.abs(a[3] - b[3]) / np.abs(a[3])) < 1e-6


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def batch_setup():
    from paper_1607_02904_amd.tersoff import Tersoff, table_sic
    confs = inputs.sic_liquid_batch(nconf=24, nmin=64, nmax=700, seed=55)
    model = Tersoff(table_sic(), masses=[28.0855, 12.011])
    yield confs, model
    model.close()


def _cat(confs):
    nat = np.array([len(c[1]) for c in confs], dtype=np.int32)
    boxes = np.array([c[2] for c in confs])
    x = np.concatenate([c[0] for c in confs])
    t = np.concatenate([c[1] for c in confs])
    return nat, boxes, x, t


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_forward_matches_oracle(orc, batch_setup, precision):
    from paper_1607_02904_amd.tersoff import BatchPlan
    confs, model = batch_setup
    nat, boxes, x, t = _cat(confs)
    plan = BatchPlan(model, nat, boxes, precision=precision)
    N = int(nat.sum())
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    e = torch.empty(len(confs), dtype=torch.float64, device="cuda")
    f = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    w = torch.empty((len(confs), 6), dtype=torch.float64, device="cuda")
    plan.run(xd, td, e, f, w)
    torch.cuda.synchronize()
    model.sync()
    e, f, w = e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy()
    off = plan.offsets
    _check_batch(orc, confs, off, e, f, w, precision)
    plan.close()


def _check_batch(orc, confs, off, e, f, w, precision):
    """Every configuration against the oracle: FP64 1e-12; mixed forces and
    virial 1e-5 and the mixed energy bar of the forward tests."""
    from test_gpu_forward import mixed_energy_ok
    tol_f = 1e-12 if precision == 0 else 1e-5
    for c, (xc, tc, bc) in enumerate(confs):
        er, fr, wr, ear = orc.compute(xc, tc, bc, params.sic())
        if precision == 0:
            assert abs(e[c] - er) <= 1e-12 * abs(er), (c, e[c], er)
        else:
            assert mixed_energy_ok(e[c], er, len(tc), "config %d (%d atoms)" % (c, len(tc))), c
        fc = f[off[c]:off[c + 1]]
        assert np.linalg.norm(fc - fr) <= tol_f * np.linalg.norm(fr), c
        assert np.linalg.norm(w[c] - wr) <= tol_f * np.linalg.norm(wr), c


def _run_plan(model, confs, precision, adjoint=False, seed=3):
    from paper_1607_02904_amd.tersoff import BatchPlan
    nat, boxes, x, t = _cat(confs)
    plan = BatchPlan(model, nat, boxes, precision=precision)
    N = int(nat.sum())
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    e = torch.empty(len(confs), dtype=torch.float64, device="cuda")
    f = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    w = torch.empty((len(confs), 6), dtype=torch.float64, device="cuda")
    args = [xd, td, e, f, w]
    if adjoint:
        g = torch.Generator("cuda").manual_seed(seed)
        eb = torch.rand(len(confs), dtype=torch.float64, device="cuda", generator=g) * 1e-3
        fb = torch.randn((N, 3), dtype=torch.float64, device="cuda", generator=g) * 0.1
        xg = torch.empty_like(f)
        pg = torch.empty((2, 2, 2, 14), dtype=torch.float64, device="cuda")
        args += [eb, fb, xg, pg]
    plan.run(*args)
    torch.cuda.synchronize()
    model.sync()
    return plan, args


def test_batch_extreme_sizes(orc, batch_setup):
    """Configurations of 4,096 atoms (the largest of the batched workload) and
    of 64 atoms in the smallest boxes (about 6-9 A a side, one cell per axis)
    in one batch, FP64 and mixed, in the launch configuration the plan's
    autotuner picks."""
    _, model = batch_setup
    confs = (inputs.sic_liquid_batch(nconf=2, nmin=4096, nmax=4096, seed=60)
             + inputs.sic_liquid_batch(nconf=6, nmin=64, nmax=64, seed=61)
             + inputs.sic_liquid_batch(nconf=4, nmin=64, nmax=4096, seed=62))
    assert min(np.min(c[2]) for c in confs) < 8.0
    for precision in (0, 1):
        plan, (xd, td, e, f, w) = _run_plan(model, confs, precision)
        sch = plan.schedule()
        print("batch extreme sizes, precision %d: schedule %s" % (precision, sch))
        assert sch["kernel"] == 2 and sch["workgroups"] > 0  # the persistent launch
        _check_batch(orc, confs, plan.offsets, e.cpu().numpy(), f.cpu().numpy(),
                     w.cpu().numpy(), precision)
        plan.close()


@pytest.mark.parametrize("nconf", [1, 3])
def test_batch_few_chunks(orc, batch_setup, nconf):
    """Batches of one and of three 64-atom configurations: far fewer chunks
    than the device holds wavefronts, so the persistent launches take a grid
    sized to the chunks (one workgroup per chunk of the forward pass, at least
    eight: one per XCD queue), and wavefronts find queues used up while others
    still work.  Forward against the oracle, FP64 and mixed; the adjoint
    against the single-system entry points."""
    _, model = batch_setup
    confs = inputs.sic_liquid_batch(nconf=nconf, nmin=64, nmax=64, seed=70 + nconf)
    for precision in (0, 1):
        plan, out = _run_plan(model, confs, precision, adjoint=True, seed=9)
        xd, td, e, f, w, eb, fb, xg, pg = out
        sch = plan.schedule()
        chunks = nconf * -(-64 // sch["atoms"])
        assert 8 <= sch["workgroups"] <= max(8, chunks), (sch, chunks)
        _check_batch(orc, confs, plan.offsets, e.cpu().numpy(), f.cpu().numpy(),
                     w.cpu().numpy(), precision)
        off = plan.offsets
        pg_sum = np.zeros((2, 2, 2, 14))
        xg_all = xg.cpu().numpy()
        # FP64 element by element; mixed as the norm of the difference (the
        # same schedule, FP32 sums in another order)
        model.set_schedule(sch["kernel"], sch["atoms"], 0)
        try:
            for c, (xc, tc, bc) in enumerate(confs):
                xcd = torch.as_tensor(xc, device="cuda")
                tcd = torch.as_tensor(tc, device="cuda")
                model.build_nlist(xcd, tcd, bc, 0.0)
                xgc, pgc = model.backward(xcd, tcd, bc, float(eb[c].item()),
                                          fb[off[c]:off[c + 1]].contiguous(), precision)
                torch.cuda.synchronize()
                pg_sum += pgc.cpu().numpy()
                a, b = xg_all[off[c]:off[c + 1]], xgc.cpu().numpy()
                if precision == 0:
                    assert np.allclose(a, b, rtol=1e-11, atol=1e-12)
                else:
                    assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b)
        finally:
            model.set_schedule(0, 0, 0)
        a = pg.cpu().numpy()
        if precision == 0:
            assert np.allclose(a, pg_sum, rtol=1e-11, atol=1e-12)
        else:
            assert np.linalg.norm(a - pg_sum) <= 1e-6 * np.linalg.norm(pg_sum)
        plan.close()


def test_batch_mixed_adjoint_matches_single_calls(batch_setup):
    """The batched mixed forward + adjoint (the benchmark's batched figure, in
    the plan's autotuned schedule) equals per-configuration calls of the
    single-system entry points in the same schedule."""
    confs, model = batch_setup
    plan, args = _run_plan(model, confs, 1, adjoint=True)
    xd, td, e, f, w, eb, fb, xg, pg = args
    sch = plan.schedule()
    print("batched mixed adjoint schedule:", sch)
    off = plan.offsets
    pg_sum = np.zeros((2, 2, 2, 14))
    xg_all = xg.cpu().numpy()
    model.set_schedule(sch["kernel"], sch["atoms"], 0)
    try:
        worst = 0.0
        for c, (xc, tc, bc) in enumerate(confs):
            xcd = torch.as_tensor(xc, device="cuda")
            tcd = torch.as_tensor(tc, device="cuda")
            model.build_nlist(xcd, tcd, bc, 0.0)
            xgc, pgc = model.backward(xcd, tcd, bc, float(eb[c].item()),
                                      fb[off[c]:off[c + 1]].contiguous(), 1)
            torch.cuda.synchronize()
            pg_sum += pgc.cpu().numpy()
            a, b = xg_all[off[c]:off[c + 1]], xgc.cpu().numpy()
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            worst = max(worst, rel)
            assert rel <= 1e-6, (c, rel)
    finally:
        model.set_schedule(0, 0, 0)
    relp = np.linalg.norm(pg.cpu().numpy() - pg_sum) / np.linalg.norm(pg_sum)
    print("batched vs single mixed adjoint: x %.2e, params %.2e" % (worst, relp))
    assert relp <= 1e-6
    plan.close()


def test_batch_full_size(orc, batch_setup):
    """The benchmark's batched workload at full size (1,024 SiC configurations
    of 64-4,096 atoms, 1,026,326 atoms), mixed forward + adjoint in the plan's
    autotuned schedule: 16 sampled configurations (the smallest and the
    largest among them) against the oracle (energy, forces, virial) and
    their position gradients against per-configuration calls of the
    single-system entry points in the same schedule; the parameter gradient
    (a sum over every configuration) against the sum of all 1,024
    per-configuration calls."""
    _, model = batch_setup
    confs = inputs.sic_liquid_batch(nconf=1024)
    sizes = np.array([len(c[1]) for c in confs])
    assert sizes.sum() == 1026326
    rng = np.random.default_rng(17)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))}
                  | set(int(v) for v in rng.choice(len(confs), size=14, replace=False)))
    plan, args = _run_plan(model, confs, 1, adjoint=True)
    xd, td, e, f, w, eb, fb, xg, pg = args
    sch = plan.schedule()
    print("full-size batch schedule:", sch)
    off = plan.offsets
    e_all, f_all, w_all, xg_all = (a.cpu().numpy() for a in (e, f, w, xg))
    sub = [confs[c] for c in pick]
    sub_off = [0]
    for c in pick:
        sub_off.append(sub_off[-1] + len(confs[c][1]))
    f_sub = np.concatenate([f_all[off[c]:off[c + 1]] for c in pick])
    _check_batch(orc, sub, sub_off, e_all[pick], f_sub, w_all[pick], 1)
    pg_sum = np.zeros((2, 2, 2, 14))
    model.set_schedule(sch["kernel"], sch["atoms"], 0)
    try:
        worst = 0.0
        for c, (xc, tc, bc) in enumerate(confs):
            xcd = torch.as_tensor(xc, device="cuda")
            tcd = torch.as_tensor(tc, device="cuda")
            model.build_nlist(xcd, tcd, bc, 0.0)
            xgc, pgc = model.backward(xcd, tcd, bc, float(eb[c].item()),
                                      fb[off[c]:off[c + 1]].contiguous(), 1)
            pg_sum += pgc.cpu().numpy()
            if c in pick:
                a, b = xg_all[off[c]:off[c + 1]], xgc.cpu().numpy()
                rel = np.linalg.norm(a - b) / np.linalg.norm(b)
                worst = max(worst, rel)
                assert rel <= 1e-6, (c, rel)
    finally:
        model.set_schedule(0, 0, 0)
    relp = np.linalg.norm(pg.cpu().numpy() - pg_sum) / np.linalg.norm(pg_sum)
    print("full-size batch vs single mixed adjoint: x %.2e, params %.2e" % (worst, relp))
    assert relp <= 1e-6
    plan.close()


def test_batch_graph_replays_and_adjoint(batch_setup):
    """Three graph replays with eager work in between give identical results;
    the batched adjoint equals per-configuration adjoints summed."""
    from paper_1607_02904_amd.tersoff import BatchPlan
    confs, model = batch_setup
    nat, boxes, x, t = _cat(confs)
    plan = BatchPlan(model, nat, boxes, precision=0)
    N = int(nat.sum())
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    g = torch.Generator("cuda").manual_seed(3)
    eb = torch.rand(len(confs), dtype=torch.float64, device="cuda", generator=g) * 1e-3
    fb = torch.randn((N, 3), dtype=torch.float64, device="cuda", generator=g) * 0.1
    outs = []
    for rep in range(3):
        e = torch.empty(len(confs), dtype=torch.float64, device="cuda")
        f = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        w = torch.empty((len(confs), 6), dtype=torch.float64, device="cuda")
        xg = torch.empty_like(f)
        pg = torch.empty((2, 2, 2, 14), dtype=torch.float64, device="cuda")
        plan.run(xd, td, e, f, w, eb, fb, xg, pg)
        torch.cuda.synchronize()
        _ = (xd * 2.0).sum().item()  # unrelated eager work between replays
        outs.append([a.cpu().numpy().copy() for a in (e, f, w, xg, pg)])
    for k in range(5):
        assert np.allclose(outs[0][k], outs[1][k], rtol=1e-13, atol=1e-13)
        assert np.allclose(outs[0][k], outs[2][k], rtol=1e-13, atol=1e-13)
    # per-configuration reference through the single-system entry points
    pg_sum = np.zeros((2, 2, 2, 14))
    off = plan.offsets
    xg_all = outs[0][3]
    for c, (xc, tc, bc) in enumerate(confs):
        xcd = torch.as_tensor(xc, device="cuda")
        tcd = torch.as_tensor(tc, device="cuda")
        model.build_nlist(xcd, tcd, bc, 0.0)
        xgc, pgc = model.backward(xcd, tcd, bc, float(eb[c].item()), fb[off[c]:off[c + 1]].contiguous(), 0)
        torch.cuda.synchronize()
        pg_sum += pgc.cpu().numpy()
        assert np.allclose(xg_all[off[c]:off[c + 1]], xgc.cpu().numpy(), rtol=1e-11, atol=1e-12)
    assert np.allclose(outs[0][4], pg_sum, rtol=1e-11, atol=1e-12)
    plan.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_batch_alternating_runs_replay_their_own_graphs(batch_setup, precision):
    """Forward-only runs and runs with the adjoint alternate on one plan (the
    fitting loop): each replays the graph of its own argument set, also after
    runs with four other argument sets have replaced both graphs in the
    plan's cache, and gives the results of its first run; a run that asks
    for the gradients alone gives those of a run with the forward pass."""
    from paper_1607_02904_amd.tersoff import BatchPlan
    confs, model = batch_setup
    nat, boxes, x, t = _cat(confs)
    plan = BatchPlan(model, nat, boxes, precision=precision)
    N, C = int(nat.sum()), len(confs)
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    g = torch.Generator("cuda").manual_seed(5)
    eb = torch.rand(C, dtype=torch.float64, device="cuda", generator=g) * 1e-3
    fb = torch.randn((N, 3), dtype=torch.float64, device="cuda", generator=g) * 0.1

    def bufs():
        return (torch.empty(C, dtype=torch.float64, device="cuda"),
                torch.empty((N, 3), dtype=torch.float64, device="cuda"),
                torch.empty((C, 6), dtype=torch.float64, device="cuda"),
                torch.empty((N, 3), dtype=torch.float64, device="cuda"),
                torch.empty((2, 2, 2, 14), dtype=torch.float64, device="cuda"))

    e, f, w, xg, pg = bufs()

    def run(adjoint):
        for a in (e, f, w, xg, pg):
            a.fill_(float("nan"))
        if adjoint:
            plan.run(xd, td, e, f, w, eb, fb, xg, pg)
        else:
            plan.run(xd, td, e, f, w)
        torch.cuda.synchronize()
        return [a.cpu().numpy().copy() for a in ((e, f, w, xg, pg) if adjoint else (e, f, w))]

    first_f, first_a = run(False), run(True)
    for k in range(3):
        assert np.allclose(first_a[k], first_f[k], rtol=1e-13, atol=1e-13)
    # gradients alone (no forward outputs: the graph leaves the forward pass out)
    xg.fill_(float("nan"))
    pg.fill_(float("nan"))
    plan.run(xd, td, None, None, None, eb, fb, xg, pg)
    torch.cuda.synchronize()
    assert np.allclose(xg.cpu().numpy(), first_a[3], rtol=1e-13, atol=1e-13)
    assert np.allclose(pg.cpu().numpy(), first_a[4], rtol=1e-13, atol=1e-13)
    for rep in range(2):
        for _ in range(2):
            got_f, got_a = run(False), run(True)
            for k in range(3):
                assert np.allclose(got_f[k], first_f[k], rtol=1e-13, atol=1e-13)
            for k in range(5):
                assert np.isfinite(got_a[k]).all()
                assert np.allclose(got_a[k], first_a[k], rtol=1e-13, atol=1e-13)
        if rep == 0:
            held = [bufs() for _ in range(4)]  # four other argument sets (all live)
            for e2, f2, w2, xg2, pg2 in held:
                plan.run(xd, td, e2, f2, w2, eb, fb, xg2, pg2)
                torch.cuda.synchronize()
                assert np.allclose(xg2.cpu().numpy(), first_a[3], rtol=1e-13, atol=1e-13)
            del held
    plan.close()


def test_md_run_timed_matches_md_run(si_model):
    """The timed MD entry point runs the same steps (launched one by one, with
    events around the force kernel) and reports a positive kernel time."""
    x, t, box = inputs.si_bulk(ncell=5, seed=25)
    a = _md_gpu(si_model, x, t, box, 12, 0.3, use_graph=True)
    xd = torch.as_tensor(x, device="cuda").clone()
    td = torch.as_tensor(t, device="cuda")
    v = torch.zeros_like(xd)
    f = torch.empty_like(xd)
    si_model.build_nlist(xd, td, box, 0.3)
    si_model.compute(xd, td, box, 0, energy=False, virial=False, out={"forces": f})
    tr, us = si_model.md_run_timed(xd, v, f, td, box, 0.001, 12, 0.3, 0)
    torch.cuda.synchronize()
    si_model.sync()
    assert us > 0.0
    assert np.array_equal(xd.cpu().numpy(), a[0])
    assert np.array_equal(tr.cpu().numpy()[:12], a[3])


def _energy_series(model, x, t, box, precision, steps, chunk):
    n = len(t)
    xd = torch.as_tensor(x, device="cuda").clone()
    td = torch.as_tensor(t, device="cuda")
    v = torch.zeros_like(xd)
    f = torch.empty_like(xd)
    model.build_nlist(xd, td, box, 0.5)
    o = model.compute(xd, td, box, precision, virial=False, out={"forces": f})
    out = [float(o["energy"].item())]
    trace = torch.empty(chunk, dtype=torch.float64, device="cuda")
    for _ in range(steps // chunk):
        model.md_run(xd, v, f, td, box, 0.001, chunk, 0.5, precision, trace=trace)
        ke = 0.5 * MASS_SI * float((v * v).sum().item()) / O.FTM2V
        out.append(float(trace[chunk - 1].item()) + ke)
    model.sync()
    return np.array(out)


@pytest.mark.parametrize("precision", [1, 2], ids=["mixed", "single"])
def test_long_run_total_energy_tracks_fp64(si_model, precision):
    """5,000 NVE steps of 4,096 Si atoms: the mixed (or all-FP32) path's total
    energy stays within 2e-5 relative of the FP64 path's at every sample (the
    bound the paper reports for its reduced-precision modes over long runs);
    both stay within the O(dt^2) oscillation of velocity Verlet at 1 fs (1e-3
    eV per atom from the start) and do not drift after the first sample (1e-4
    eV per atom)."""
    x, t, box = inputs.si_bulk(ncell=8, seed=26)
    e64 = _energy_series(si_model, x, t, box, 0, 5000, 500)
    emx = _energy_series(si_model, x, t, box, precision, 5000, 500)
    n = len(t)
    assert np.max(np.abs(emx - e64) / np.abs(e64)) < 2e-5
    for e in (e64, emx):
        assert np.max(np.abs(e - e[0])) / n < 1e-3
        assert (e[1:].max() - e[1:].min()) / n < 1e-4


def test_batch_builds_lists_only_when_atoms_moved(orc, batch_setup):
    """A plan builds its lists again only when an atom is not where the last
    build found it.  The same positions again: the same results (lists
    reused).  Positions permuted within every configuration (types kept): the
    oracle's results for the new positions, which a reused list would miss
    entirely.  A species out of range with unchanged positions, and a list
    that overflowed, are still reported by every run."""
    from paper_1607_02904_amd.tersoff import TersoffError
    confs, model = batch_setup
    confs = confs[:6]
    plan, (xd, td, e, f, w) = _run_plan(model, confs, 0)
    first = [a.cpu().numpy().copy() for a in (e, f, w)]
    plan.run(xd, td, e, f, w)
    model.sync()
    for a, b in zip(first, (e, f, w)):
        assert np.allclose(a, b.cpu().numpy(), rtol=1e-13, atol=1e-13)
    nat, boxes, x, t = _cat(confs)
    off = plan.offsets
    xp = x.copy()
    for c in range(len(confs)):  # reverse the atoms' positions in each configuration
        xp[off[c]:off[c + 1]] = x[off[c]:off[c + 1]][::-1]
    xd.copy_(torch.as_tensor(xp, device="cuda"))
    plan.run(xd, td, e, f, w)
    model.sync()
    moved = [(xp[off[c]:off[c + 1]], confs[c][1], confs[c][2]) for c in range(len(confs))]
    _check_batch(orc, moved, off, e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy(), 0)
    # a species outside the table, positions unchanged
    tbad = td.clone()
    tbad[3] = 7
    plan.run(xd, tbad, e, f, w)
    with pytest.raises(TersoffError) as ei:
        model.sync()
    assert ei.value.name == "TERS_ERR_INVALID_ARG"
    plan.run(xd, td, e, f, w)
    model.sync()
    # an overflowing list is reported by the run that builds it and, with the
    # positions unchanged, by the next run too
    xs = xp.copy()
    for c in range(len(confs)):
        xs[off[c]:off[c + 1]] = 0.7 * inputs.wrap(xp[off[c]:off[c + 1]], boxes[c])
    xd.copy_(torch.as_tensor(xs, device="cuda"))
    for _ in range(2):
        plan.run(xd, td, e, f, w)
        with pytest.raises(TersoffError) as ei:
            model.sync()
        assert ei.value.name == "TERS_ERR_NLIST_OVERFLOW"
    xd.copy_(torch.as_tensor(x, device="cuda"))
    plan.run(xd, td, e, f, w)
    model.sync()
    _check_batch(orc, confs, off, e.cpu().numpy(), f.cpu().numpy(), w.cpu().numpy(), 0)
    plan.close()


def test_batch_run_reports_list_overflow(batch_setup):
    """A plan sizes its list on its first run; a later run whose atoms are
    packed more densely overflows the rows.  The graph latches the error in
    the plan's error word and ters_sync reports it (TERS_ERR_NLIST_OVERFLOW);
    the word is cleared once read, and a run at the original density is
    clean again."""
    from paper_1607_02904_amd.tersoff import TersoffError
    confs, model = batch_setup
    confs = confs[:6]
    plan, (xd, td, e, f, w) = _run_plan(model, confs, 0)
    model.sync()
    nat, boxes, x, t = _cat(confs)
    off = plan.offsets
    xs = x.copy()
    for c in range(len(confs)):  # pack every configuration into 70 % of its box
        xs[off[c]:off[c + 1]] = 0.7 * inputs.wrap(x[off[c]:off[c + 1]], boxes[c])
    xd.copy_(torch.as_tensor(xs, device="cuda"))
    plan.run(xd, td, e, f, w)
    with pytest.raises(TersoffError) as ei:
        model.sync()
    assert ei.value.name == "TERS_ERR_NLIST_OVERFLOW"
    xd.copy_(torch.as_tensor(x, device="cuda"))
    plan.run(xd, td, e, f, w)
    model.sync()
    plan.close()
