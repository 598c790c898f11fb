"""Benchmark: Tersoff atom-steps/s on one MI355X (FP64 vs mixed vs batched).

Headline workload: Si diamond 40^3 cells = 512,000 atoms, Gaussian sigma 0.1 A,
Si(B) parameters, neighbour skin 0.5 A, velocity-Verlet molecular dynamics with
dt = 1 fs.  One step = one velocity-Verlet step: half kick + drift (with the
rebuild test), neighbour rebuild when due, one full energy/force evaluation,
half kick.  `value` is the mixed-precision path (FP32 arithmetic, FP64
accumulators); the FP64 path is measured in the same run.  Also reported:
two-species SiC 1,000,000 atoms (one mixed evaluation), a batch of 1,024
uneven SiC configurations evaluated forward + adjoint in one graph launch, and
the total energy along a 100,000-step NVE run (32,768 atoms) in FP64 and mixed.

Prints one JSON line.  Options: --gpus N (only 1 is supported), --steps K,
--warmup W, --no-cpu (skip the CPU baseline), --quick (smaller extras).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK = 78.6e12      # MI355X vector FP64, FLOP/s
FP32_PEAK = 157.3e12     # MI355X vector FP32 (packed), FLOP/s

# Algorithmic work of one evaluation, from the counts of list entries L,
# in-cutoff (ordered) pairs P and triplets T of the configuration.
#
# Reported model (the work-per-unit figures of the design, counting an FMA as
# one op): per list entry 16 ops (distance and compare), per in-cutoff
# neighbour 6 ops + sqrt + reciprocal, per pair 45 ops + 5 transcendentals +
# 1 division, per triplet 70 ops + reciprocal + exponential (no exponential
# when lambda3 = 0).  Ops become flops at 1.9 flops per op (the FMA share of
# the definition: ~1.1 k ops are ~1.9 k flops per Si atom), and every
# transcendental, reciprocal or division counts as one flop.
OPS_PER_ENTRY = 16
OPS_PER_NEIGH = 6
OPS_PER_PAIR = 45
OPS_PER_TRIPLET = 70
FLOPS_PER_OP = 1.9 / 1.1
# A lower count, made by hand from the kernels' own formulas (FMA = 2 flops,
# transcendental = 1): per entry 9, per neighbour 8, per pair 46, per triplet
# 74.  Reported beside the model for reference.
BUILDER_FLOPS = (9, 8, 46, 74)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--ncell", type=int, default=40)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--md-only", action="store_true", help="only the headline MD workload")
    ap.add_argument("--workload", choices=["batch", "fitting"],
                    help="run one of the other workloads alone and print its figures as one "
                         "JSON object (no headline line; for kernel traces of that workload)")
    return ap.parse_args()


def count_work(x, t, box, table, rlist, rcut_pair):
    """List entries L, in-cutoff pairs P and triplets T of a configuration,
    counted on the host with a cell list (numpy)."""
    from scipy.spatial import cKDTree
    xw = x - np.floor(x / box) * box
    tree = cKDTree(xw, boxsize=box)
    pairs = tree.query_pairs(rlist, output_type="ndarray")
    L = 2 * len(pairs)
    d = xw[pairs[:, 1]] - xw[pairs[:, 0]]
    d -= box * np.round(d / box)
    r = np.linalg.norm(d, axis=1)
    inc = r < rcut_pair
    P = 2 * int(inc.sum())
    deg = np.bincount(pairs[inc].ravel(), minlength=len(x))
    T = int(np.sum(deg * (deg - 1)))
    return L, P, T


def flops_of(L, P, T, lam3=True):
    """Algorithmic flops of one evaluation (the reported model above)."""
    ops = OPS_PER_ENTRY * L + (OPS_PER_NEIGH + OPS_PER_PAIR) * P + OPS_PER_TRIPLET * T
    trans = 2 * P + 6 * P + (2 if lam3 else 1) * T
    return FLOPS_PER_OP * ops + trans


def builder_flops_of(L, P, T):
    e, nb, p, t = BUILDER_FLOPS
    return e * L + nb * P + p * P + t * T


VALU_MIX_SUMMARY = os.path.join(ROOT, "profiles", "force_wave_si512k_%s_valu_mix.txt")


def counter_flops_of(sched, tname, n):
    """FP32 and FP64 flops per launch of the force kernel from the committed
    instruction-count summary (64 lanes per wave instruction, FMA = 2, a
    transcendental = 1), or None when there is none for this kernel and
    launch shape or its sources have changed since it was taken."""
    from paper_1607_02904_amd import profsum
    path = VALU_MIX_SUMMARY % tname
    if sched["kernel"] != 2 or not os.path.exists(path):
        return None
    s = profsum.read_summary(path)
    grid = 64 * ((n + sched["atoms"] - 1) // sched["atoms"])
    if s.get("kernel_sources_sha256") != profsum.kernel_hash() or int(s.get("grid", -1)) != grid:
        return None
    out = {}
    for prec in ("F32", "F64"):
        add = float(s["SQ_INSTS_VALU_ADD_%s" % prec])
        mul = float(s["SQ_INSTS_VALU_MUL_%s" % prec])
        fma = float(s["SQ_INSTS_VALU_FMA_%s" % prec])
        trans = float(s["SQ_INSTS_VALU_TRANS_%s" % prec])
        out[prec] = 64.0 * (add + mul + 2.0 * fma + trans)
    out["valu_insts"] = float(s["SQ_INSTS_VALU"])
    return out


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "force_wave_si512k_%s_traffic.txt")


def traffic_of(sched, tname, n):
    """HBM bytes per launch of the force kernel from the committed counter
    summary, or None when there is none for this kernel and launch shape or
    the kernel's sources have changed since it was taken."""
    from paper_1607_02904_amd import profsum
    path = TRAFFIC_SUMMARY % tname
    if sched["kernel"] != 2 or not os.path.exists(path):
        return None
    s = profsum.read_summary(path)
    grid = 64 * ((n + sched["atoms"] - 1) // sched["atoms"])
    if s.get("kernel_sources_sha256") != profsum.kernel_hash() or int(s.get("grid", -1)) != grid:
        return None
    return float(s["traffic_bytes_per_launch"])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported "
              "(multi-GPU spatial decomposition is design only)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1607_02904_amd import inputs
    from paper_1607_02904_amd.tersoff import (FP64, MIXED, SINGLE, BatchPlan, Tersoff,
                                              table_element, table_sic)

    dev = "cuda"
    if args.workload:
        out = {}
        if args.workload == "batch":
            run_batch(args, out, dev)
        else:
            print("bench: fitting frames", file=sys.stderr, flush=True)
            out["fitting_64x512"] = run_fitting(dev)
        print(json.dumps(out), flush=True)
        return
    if args.copy_probe:
        # plain copy of known size: 256 MiB read + 256 MiB written per launch
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    print("bench: building inputs", file=sys.stderr, flush=True)
    x, t, box = inputs.si_bulk(args.ncell)
    n = len(x)
    tab = table_element("Si(B)")
    skin = 0.5
    dt = 0.001
    model = Tersoff(tab, masses=[28.0855])
    td = torch.as_tensor(t, device=dev)
    x0 = torch.as_tensor(x, device=dev)

    # schedule per precision chosen by the library's autotuner on this input
    model.build_nlist(x0, td, box, skin)
    tuned = {}
    for prec in (FP64, MIXED, SINGLE):
        us = model.autotune(x0, td, box, prec)
        tuned[prec] = us

    mass = 28.0855
    # (g/mol) (A/ps)^2 in eV: 1e4 amu m^2 s^-2 / e
    mvv2e = 1.66053906660e-27 * 1e4 / 1.602176634e-19
    etot = []

    def kinetic(v):
        return 0.5 * mass * mvv2e * float((v * v).sum().item())

    def run_md(precision, skin=skin, kernel_times=True):
        xd = x0.clone()
        v = torch.zeros_like(xd)
        f = torch.empty_like(xd)
        model.build_nlist(xd, td, box, skin)
        model.compute(xd, td, box, precision, energy=False, virial=False, out={"forces": f})
        trace = torch.empty(max(args.warmup, args.steps, 1), dtype=torch.float64, device=dev)
        model.md_run(xd, v, f, td, box, dt, args.warmup, skin, precision, trace=trace)
        torch.cuda.synchronize()
        # total energy (potential after the last step + kinetic, whose
        # velocities are those of the same instant) before and after the timed
        # steps, read outside the timed region
        e0 = None
        if args.warmup > 0:
            e0 = float(trace[args.warmup - 1].item()) + kinetic(v)
        r0 = model.rebuilds()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        model.md_run(xd, v, f, td, box, dt, args.steps, skin, precision, trace=trace)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        model.sync()
        reb = model.rebuilds() - r0
        tr = trace[:args.steps].cpu().numpy()
        etot.append(None if e0 is None else
                    (float(tr[-1]) + kinetic(v) - e0) / n)
        if not kernel_times:
            return el, reb, tr, None
        # force-kernel duration: HIP events on the library's stream around every
        # force launch of K further steps of the same trajectory (launched one
        # by one; the timed region above replays the captured step)
        _, fus = model.md_run_timed(xd, v, f, td, box, dt, args.steps, skin, precision, trace=trace)
        torch.cuda.synchronize()
        return el, reb, tr, fus

    print("bench: MD fp64", file=sys.stderr, flush=True)
    el64, reb64, tr64, f64us = run_md(FP64)
    etot64 = etot[-1]
    print("bench: MD mixed", file=sys.stderr, flush=True)
    elmx, rebmx, trmx, fmxus = run_md(MIXED)
    etotmx = etot[-1]
    elsp = None
    if not args.md_only:
        print("bench: MD single", file=sys.stderr, flush=True)
        elsp, rebsp, trsp, fspus = run_md(SINGLE)

    # back-to-back launches of the force kernel alone on the start configuration
    model.build_nlist(x0, td, box, skin)
    sched = model.schedules()
    k64 = model.profile_forward(x0, td, box, FP64, reps=20)
    kmx = model.profile_forward(x0, td, box, MIXED, reps=20)
    L, P, T = count_work(x, t, box, tab, 3.2 + skin, 3.2)
    fl = flops_of(L, P, T)
    flb = builder_flops_of(L, P, T)

    def roof(us, us_b2b, peak, sch, tname):
        ach = fl / (us * 1e-6)
        r = {"bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
             "frac": ach / peak, "traffic": traffic_of(sch, tname, n),
             "kernel": ("k_force_wave<%s, true, false, false, false>" % tname if sch["kernel"] == 2
                        else "k_force<%s, true, false, ...>" % tname),
             "kernel_us": us, "kernel_us_timing": "HIP events around each force launch of %d MD "
                                                  "steps" % args.steps,
             "kernel_us_back_to_back": us_b2b,
             "flops_per_launch": fl,
             "flops_model": "16/6/45/70 ops per entry/neighbour/pair/triplet x 1.9/1.1 flops per "
                            "op + 8 transcendentals per pair + 2 per triplet",
             "builder_count": {"flops_per_launch": flb, "achieved": flb / (us * 1e-6) / 1e12,
                               "frac": flb / (us * 1e-6) / peak},
             "units": {"entries": L, "pairs": P, "triplets": T}}
        cf = counter_flops_of(sch, tname, n)
        if cf is not None:
            prec = "F32" if tname == "float" else "F64"
            ca = cf[prec] / (us * 1e-6)
            r["counter"] = {"flops_per_launch": cf[prec], "achieved": ca / 1e12, "frac": ca / peak,
                            "other_precision_flops_per_launch": cf["F64" if prec == "F32" else "F32"],
                            "valu_insts_per_launch": cf["valu_insts"],
                            "source": os.path.relpath(VALU_MIX_SUMMARY % tname, ROOT)}
        else:
            r["counter"] = None
        return r

    # ablation of the paper's design choices on this hardware: time to forces
    # (force kernel, plus the gather pass in owner-gather mode; back-to-back
    # launches on the start configuration) for the workgroup schedule (Alg. 3
    # with k_max), the wavefront schedule with 32 atoms per wavefront (the
    # fused I x J mapping, scheme (b)) and with one (lanes over the j of one
    # atom, scheme (a)), and thread per atom (scheme (c)); owner gather vs
    # FP64 atomic scatter; the wavefront schedule without the filter; and
    # whole MD steps with skin 0 (rebuild every step) vs the headline skin
    ablation = None
    if not args.md_only:
        print("bench: ablation", file=sys.stderr, flush=True)
        fk = {}
        for prec, tag in ((MIXED, "mixed"), (FP64, "fp64")):
            for kern, atoms, name in ((1, 64, "workgroup_64"), (2, 32, "wavefront_32"),
                                      (2, 1, "wavefront_1_scheme_a")):
                for gather in (True, False):
                    model.set_schedule(kern, atoms, 0)
                    model.set_force_mode(gather)
                    fk["%s_%s_%s" % (tag, name, "gather" if gather else "atomic")] = \
                        model.profile_forward(x0, td, box, prec, reps=10, with_gather=True)
        model.set_schedule(3, 0, 0)  # thread per atom (the paper's scheme (c)), atomics
        for prec, tag in ((MIXED, "mixed"), (FP64, "fp64")):
            fk["%s_thread_per_atom_atomic" % tag] = \
                model.profile_forward(x0, td, box, prec, reps=10, with_gather=True)
        model.set_force_mode(True)
        model.set_schedule(2, 32, 0)
        model.set_filter(False)  # every skin-list entry takes a lane
        for prec, tag in ((MIXED, "mixed"), (FP64, "fp64")):
            fk["%s_wavefront_32_gather_filter_off" % tag] = \
                model.profile_forward(x0, td, box, prec, reps=10, with_gather=True)
        model.set_filter(True)
        # the paper's Algorithm 2 (every dzeta/dx_k recomputed in the second K
        # loop) against Algorithm 3 with k_max derivatives stored per pair
        # (workgroup schedule, 64 atoms per workgroup)
        for prec, tag in ((MIXED, "mixed"), (FP64, "fp64")):
            for km, name in ((-1, "alg2"), (1, "alg3_kmax1"), (2, "alg3_kmax2"), (4, "alg3_kmax4"),
                             (0, "alg3_kmax_all")):
                model.set_schedule(1, 64, km)
                fk["%s_workgroup_64_%s" % (tag, name)] = \
                    model.profile_forward(x0, td, box, prec, reps=10, with_gather=True)
        model.set_schedule(sched["mixed"]["kernel"], sched["mixed"]["atoms"], 0)
        el0, reb0, _, _ = run_md(MIXED, skin=0.0, kernel_times=False)
        ablation = {"time_to_forces_us": fk,
                    "md_mixed_atom_steps_per_s": {"skin_0": n * args.steps / el0,
                                                  "skin_%g" % skin: n * args.steps / elmx},
                    "md_mixed_rebuilds": {"skin_0": reb0, "skin_%g" % skin: rebmx},
                    "schedule_in_md_runs": sched["mixed"]}

    value = n * args.steps / elmx
    out = {
        "metric": "Tersoff atom-steps/s: FP64 vs mixed vs batched on 1 MI355X; % vector peak",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elmx / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Si diamond, sigma 0.1 A)",
        "config": {"workload": "Si diamond 40^3 cells = %d atoms, Si(B), skin 0.5 A, "
                               "velocity Verlet dt 1 fs, mixed precision" % n,
                   "atoms": n, "skin": skin, "dt_fs": 1.0, "precision": "mixed"},
        "roofline": roof(fmxus, kmx, FP32_PEAK, sched["mixed"], "float"),
        "fp64": {"value": n * args.steps / el64, "unit": "atom-steps/s",
                 "ms_per_step": 1000.0 * el64 / args.steps, "rebuilds": reb64,
                 "schedule": sched["fp64"], "roofline": roof(f64us, k64, FP64_PEAK, sched["fp64"],
                                                              "double")},
        "single": None if elsp is None else {
            "value": n * args.steps / elsp, "unit": "atom-steps/s",
            "ms_per_step": 1000.0 * elsp / args.steps, "rebuilds": rebsp, "kernel_us": fspus,
            "note": "all-FP32 mode (FP32 positions and accumulators), the paper's Opt-S"},
        "ablation": ablation,
        "mixed": {"rebuilds": rebmx, "schedule": sched["mixed"],
                  "potential_energy_change_per_atom": float((trmx[-1] - trmx[0]) / n),
                  "total_energy_drift_per_atom": etotmx,
                  "fp64_total_energy_drift_per_atom": etot64,
                  "fp64_vs_mixed_energy_rel": float(abs(trmx[-1] - tr64[-1]) / abs(tr64[-1]))},
    }

    # ---- the same molecular dynamics at 64,000 atoms (20^3 cells) --------------
    if not args.md_only:
        print("bench: MD 64k", file=sys.stderr, flush=True)
        out["md_64k"] = run_md_size(args, 20, dev)

    # ---- one FP64 evaluation of 512 atoms: latency -----------------------------
    if not args.md_only:
        print("bench: latency 512", file=sys.stderr, flush=True)
        out["latency_512"] = run_latency(dev)

    # ---- fitting: loss and its gradient over 64 frames of 512 atoms -------------
    if not args.md_only:
        print("bench: fitting frames", file=sys.stderr, flush=True)
        out["fitting_64x512"] = run_fitting(dev)

    # ---- a pair potential on the same list (Algorithm 1): Lennard-Jones --------
    if not args.md_only:
        print("bench: pair potential", file=sys.stderr, flush=True)
        model.build_nlist(x0, td, box, skin)
        entries = model.nlist_stats()["entries"]
        # bytes an evaluation must move at least: the list entries, counts and
        # cell order, every position once and the forces written
        lj_bytes = 4.0 * entries + 8.0 * n + 24.0 * n + 24.0 * n
        pl = {}
        for prec, tag in ((MIXED, "mixed"), (FP64, "fp64")):
            model.pair_compute(x0, box, 0.05, 2.1, 3.0, prec)
            torch.cuda.synchronize()
            reps = 20
            t0 = time.perf_counter()
            for _ in range(reps):
                model.pair_compute(x0, box, 0.05, 2.1, 3.0, prec)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / reps
            # device time of an evaluation (kernel and energy reduction, stream order)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                model.pair_compute(x0, box, 0.05, 2.1, 3.0, prec)
            e1.record()
            torch.cuda.synchronize()
            dus = e0.elapsed_time(e1) / reps * 1e3
            pl[tag] = {"value": n / el, "unit": "atom-steps/s", "ms_per_eval": el * 1e3,
                       "device_us_per_eval": dus,
                       "roofline": {"bound": "hbm", "achieved": lj_bytes / (dus * 1e-6) / 1e9,
                                    "peak": 8000.0, "unit": "GB/s",
                                    "frac": lj_bytes / (dus * 1e-6) / 8e12, "traffic": None,
                                    "algorithmic_bytes": lj_bytes}}
        out["pair_lj"] = dict(pl, note="truncated Lennard-Jones (eps 0.05 eV, sigma 2.1 A, "
                                       "r_c 3.0 A) over the Tersoff list of the headline "
                                       "configuration; one evaluation, outputs allocated per call; "
                                       "algorithmic bytes = 4 per list entry + 56 per atom")

    # ---- two-species SiC, 1,000,000 atoms, one mixed evaluation ----------------
    if not args.quick and not args.md_only:
        print("bench: SiC 1M", file=sys.stderr, flush=True)
        xs, ts, bs = inputs.sic_bulk(50)
        ms = Tersoff(table_sic(), masses=[28.0855, 12.011])
        xsd = torch.as_tensor(xs, device=dev)
        tsd = torch.as_tensor(ts, device=dev)
        ms.build_nlist(xsd, tsd, bs, 0.5)
        ms.autotune(xsd, tsd, bs, MIXED)
        o = ms.compute(xsd, tsd, bs, MIXED)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            ms.compute(xsd, tsd, bs, MIXED, out=o)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        kus = ms.profile_forward(xsd, tsd, bs, MIXED, reps=10)
        out["sic_1m_mixed"] = {"value": len(xs) / el, "unit": "atom-steps/s", "ms_per_eval": el * 1e3,
                               "kernel_us": kus, "schedule": ms.schedules()["mixed"]}
        ms.autotune(xsd, tsd, bs, FP64)
        o = ms.compute(xsd, tsd, bs, FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ms.compute(xsd, tsd, bs, FP64, out=o)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        kus = ms.profile_forward(xsd, tsd, bs, FP64, reps=10)
        out["sic_1m_fp64"] = {"value": len(xs) / el, "unit": "atom-steps/s", "ms_per_eval": el * 1e3,
                              "kernel_us": kus, "schedule": ms.schedules()["fp64"]}
        ms.close()
        del xsd, tsd

    # ---- batched: 1,024 uneven SiC configurations, forward + adjoint ----------
    if not args.md_only:
        run_batch(args, out, dev)

    # ---- long NVE run: mixed vs FP64 energy (the paper's accuracy check) ------
    if not args.md_only:
        run_accuracy(args, out, dev)

    # ---- CPU baseline: the FP64 oracle on the host ----------------------------
    if not args.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        from oracle import oracle as orc
        from oracle import params as oparams
        otab = oparams.single(oparams.SI_B)
        nl = orc.neighbours(x, box, 3.2 + skin)
        # the oracle's source compiled with gcc -O3 -march=native, one thread
        orc.compute_threads(x, t, box, otab, nl, threads=1)  # build and warm up
        reps = 0
        t0 = time.perf_counter()
        while True:
            orc.compute_threads(x, t, box, otab, nl, threads=1)
            reps += 1
            if time.perf_counter() - t0 > 10.0 or reps >= 50:
                break
        elc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * reps / elc, "unit": "atom-steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "%d full FP64 force evaluations (Algorithm 2) of the same "
                                         "%d-atom configuration over a prebuilt skin list, one "
                                         "thread, gcc -O3 -march=native; list build and "
                                         "integration not timed" % (reps, n)}
        # the same oracle with the centres shared among the host's threads
        # (OpenMP, per-thread force arrays, gcc -O3 -march=native)
        orc.compute_threads(x, t, box, otab, nl)  # build and warm up
        reps = 0
        t0 = time.perf_counter()
        while True:
            _, _, _, nthr = orc.compute_threads(x, t, box, otab, nl)
            reps += 1
            if time.perf_counter() - t0 > 10.0 or reps >= 200:
                break
        elc = time.perf_counter() - t0
        out["cpu_baseline_all_cores"] = {
            "value": n * reps / elc, "unit": "atom-steps/s", "cores": nthr, "kind": "oracle",
            "sample": "%d full FP64 force evaluations of the same %d-atom configuration over a "
                      "prebuilt skin list, %d OpenMP threads, gcc -O3 -march=native; list build "
                      "and integration not timed" % (reps, n, nthr)}
    model.close()
    print(json.dumps(out), flush=True)


def run_md_size(args, ncell, dev):
    """Velocity-Verlet MD of Si diamond ncell^3 cells (sigma 0.1 A, skin 0.5 A,
    dt 1 fs), FP64 and mixed, with the autotuned schedules: atom-steps/s of
    the whole step over args.steps graph-replayed steps."""
    import torch

    from paper_1607_02904_amd import inputs
    from paper_1607_02904_amd.tersoff import FP64, MIXED, Tersoff, table_element
    x, t, box = inputs.si_bulk(ncell)
    n = len(x)
    m = Tersoff(table_element("Si(B)"), masses=[28.0855])
    td = torch.as_tensor(t, device=dev)
    x0 = torch.as_tensor(x, device=dev)
    m.build_nlist(x0, td, box, 0.5)
    res = {"atoms": n, "unit": "atom-steps/s", "steps": args.steps}
    for prec, tag in ((FP64, "fp64"), (MIXED, "mixed")):
        m.autotune(x0, td, box, prec)
        xd = x0.clone()
        v = torch.zeros_like(xd)
        f = torch.empty_like(xd)
        m.build_nlist(xd, td, box, 0.5)
        m.compute(xd, td, box, prec, energy=False, virial=False, out={"forces": f})
        m.md_run(xd, v, f, td, box, 0.001, args.warmup, 0.5, prec)
        torch.cuda.synchronize()
        r0 = m.rebuilds()
        t0 = time.perf_counter()
        m.md_run(xd, v, f, td, box, 0.001, args.steps, 0.5, prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[tag] = {"value": n * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                    "rebuilds": m.rebuilds() - r0, "schedule": m.schedules()[tag]}
    m.close()
    return res


def run_latency(dev, reps=50):
    """Si diamond 4^3 cells = 512 atoms (sigma 0.05 A, Si(B) with R = 2.85,
    D = 0.15, skin 0): wall time of one FP64 evaluation (energy, forces,
    virial) on a prebuilt list, and of list build plus evaluation, each the
    median over `reps` synchronised calls."""
    import torch

    from paper_1607_02904_amd import inputs
    from paper_1607_02904_amd.tersoff import FP64, Tersoff, table_element
    x, t, box = inputs.si_small()
    tab = table_element("Si(B)")
    tab[0, 0, 0, 10] = 2.85
    tab[0, 0, 0, 11] = 0.15
    m = Tersoff(tab)
    xd = torch.as_tensor(x, device=dev)
    td = torch.as_tensor(t, device=dev)
    m.build_nlist(xd, td, box, 0.0)
    o = m.compute(xd, td, box, FP64)
    torch.cuda.synchronize()
    ev, full = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        m.compute(xd, td, box, FP64, out=o)
        torch.cuda.synchronize()
        ev.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        m.build_nlist(xd, td, box, 0.0)
        m.compute(xd, td, box, FP64, out=o)
        torch.cuda.synchronize()
        full.append(time.perf_counter() - t0)
    m.close()
    return {"atoms": len(x), "eval_us_median": 1e6 * float(np.median(ev)),
            "build_and_eval_us_median": 1e6 * float(np.median(full)),
            "note": "wall time per synchronised call (launch latency included); the list build "
                    "synchronises to read its longest row"}


def run_fitting(dev, nframes=64, reps=5):
    """The fitting workload: 64 Si frames of 512 atoms (sigma 0.15 A, +-3 %
    strain), references E_ref, F_ref from the FP64 GPU path at a table whose
    continuous fields are scaled by (1 + 0.01 N(0,1)) (h shifted), loss
    sum_f (E_f - E_ref,f)^2 / N^2 + 0.1 sum |F - F_ref|^2.  One evaluation of
    loss and gradient = a batched forward (energies and forces of all frames)
    and a batched adjoint with the cotangents of that loss (one plan, graph
    launches; the adjoint run asks for no forward outputs, so its graph
    holds the list build and the adjoint alone).  Reported per precision: atom-steps/s of the whole
    loss-and-gradient evaluation, and the largest relative error of the 14
    parameter gradients against central differences (h = 1e-6 relative) of
    the same loss evaluated by the FP64 GPU path."""
    import torch

    from paper_1607_02904_amd import inputs
    from paper_1607_02904_amd.tersoff import FP64, MIXED, BatchPlan, Tersoff, table_element
    frames = inputs.si_frames(nframes)
    nat = np.array([len(f[1]) for f in frames], dtype=np.int32)
    boxes = np.array([f[2] for f in frames])
    N = int(nat.sum())
    xc = torch.as_tensor(np.concatenate([f[0] for f in frames]), device=dev)
    tc = torch.as_tensor(np.concatenate([f[1] for f in frames]), device=dev)
    tab = table_element("Si(B)")
    rng = np.random.default_rng(1607 + 33)
    ref_tab = tab.copy()
    for fld in range(14):
        if fld == 0:
            continue
        if ref_tab[0, 0, 0, fld] == 0.0:
            ref_tab[0, 0, 0, fld] = 0.01 * rng.normal() if fld == 5 else 0.0
        else:
            ref_tab[0, 0, 0, fld] *= 1.0 + 0.01 * rng.normal()
    natd = torch.as_tensor(nat, device=dev, dtype=torch.float64)
    e = torch.empty(nframes, dtype=torch.float64, device=dev)
    f = torch.empty((N, 3), dtype=torch.float64, device=dev)
    w = torch.empty((nframes, 6), dtype=torch.float64, device=dev)
    eb = torch.empty(nframes, dtype=torch.float64, device=dev)
    fb = torch.empty((N, 3), dtype=torch.float64, device=dev)
    xg = torch.empty_like(f)
    pg = torch.empty((1, 1, 1, 14), dtype=torch.float64, device=dev)

    def model_at(table):
        return Tersoff(table, masses=[28.0855])

    mref = model_at(ref_tab)
    pref = BatchPlan(mref, nat, boxes, precision=FP64)
    pref.run(xc, tc, e, f, w)
    torch.cuda.synchronize()
    e_ref, f_ref = e.clone(), f.clone()
    pref.close()
    mref.close()

    def loss_of(table, precision=FP64):
        m = model_at(table)
        p = BatchPlan(m, nat, boxes, precision=precision)
        p.run(xc, tc, e, f, w)
        torch.cuda.synchronize()
        L = float((((e - e_ref) / natd) ** 2).sum().item() + 0.1 * ((f - f_ref) ** 2).sum().item())
        p.close()
        m.close()
        return L

    res = {"frames": nframes, "atoms": N, "unit": "atom-steps/s (loss + gradient)"}
    for prec, tag in ((FP64, "fp64"), (MIXED, "mixed")):
        m = model_at(tab)
        p = BatchPlan(m, nat, boxes, precision=prec)

        def loss_and_grad():
            p.run(xc, tc, e, f, w)
            torch.subtract(e, e_ref, out=eb)
            eb.mul_(2.0).div_(natd * natd)
            torch.subtract(f, f_ref, out=fb)
            fb.mul_(0.2)
            p.run(xc, tc, None, None, None, eb, fb, xg, pg)  # gradients alone

        loss_and_grad()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            loss_and_grad()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        g = pg.cpu().numpy().reshape(14).copy()
        p.close()
        m.close()
        res[tag] = {"value": N / el, "ms_per_loss_and_gradient": 1e3 * el, "gradient": g.tolist()}
    # central differences of the FP64 loss for the 13 continuous fields (the
    # library takes m in {1, 3} only; dE/dm is checked against the oracle's
    # continuation by the tests)
    fd = np.zeros(14)
    for fld in range(1, 14):
        th = tab[0, 0, 0, fld]
        # R and D (fields 10, 11) move the cutoff, where dF/dR jumps: a step
        # that straddles a pair distance at R + D sees that jump, so their
        # step is 1e-8 (relative)
        rel = 1e-8 if fld in (10, 11) else 1e-6
        h = rel * abs(th) if th != 0.0 else rel
        tp, tm = tab.copy(), tab.copy()
        tp[0, 0, 0, fld] += h
        tm[0, 0, 0, fld] -= h
        fd[fld] = (loss_of(tp) - loss_of(tm)) / (2.0 * h)
    scale = np.abs(fd).max()
    for tag in ("fp64", "mixed"):
        g = np.array(res[tag].pop("gradient"))[1:]
        fd_ = fd[1:]
        err = np.abs(g - fd_) / np.maximum(np.abs(fd_), 1e-3 * scale)
        res[tag]["fd_rel_err_per_field"] = [float("%.3g" % v) for v in err]
        res[tag]["fd_max_rel_err"] = float(err.max())
        res[tag]["fd_norm_rel_err"] = float(np.linalg.norm(g - fd_) / np.linalg.norm(fd_))
    res["fd"] = "central differences (h = 1e-6 relative, absolute where the field is 0; 1e-8 " \
                "for the cutoff fields R and D) of the loss evaluated by the FP64 GPU path; m " \
                "excluded (the forward takes m in {1, 3} only)"
    return res


FTM2V = 9648.533215665328  # eV/(Angstrom amu) -> Angstrom/ps^2 (metal units, CODATA 2018)


def run_accuracy(args, out, dev):
    """Total energy along a long NVE trajectory of Si diamond 16^3 cells
    (32,768 atoms, sigma 0.1 A, v0 = 0, dt 1 fs, skin 0.5 A) in FP64, in the
    mixed precision and in the single-precision mode: the largest relative
    difference of each total energy from the FP64 one, and each path's largest
    total-energy deviation per atom from its start.  The paper checks its
    precision modes the same way (a long run of about 32,000 Si atoms, FP64
    as reference)."""
    import torch

    from paper_1607_02904_amd import inputs
    from paper_1607_02904_amd.tersoff import FP64, MIXED, SINGLE, Tersoff, table_element
    print("bench: accuracy run", file=sys.stderr, flush=True)
    steps = 10000 if args.quick else 100000
    chunk = 2000
    x, t, box = inputs.si_bulk(16, seed=inputs.seed_for(6))
    n = len(x)
    mass = 28.0855
    m = Tersoff(table_element("Si(B)"), masses=[mass])
    td = torch.as_tensor(t, device=dev)
    series = {}
    t0 = time.perf_counter()
    for prec in (FP64, MIXED, SINGLE):
        xd = torch.as_tensor(x, device=dev).clone()
        v = torch.zeros_like(xd)
        f = torch.empty_like(xd)
        m.build_nlist(xd, td, box, 0.5)
        e0 = m.compute(xd, td, box, prec, virial=False, out={"forces": f})["energy"]
        etot = [float(e0.item())]
        trace = torch.empty(chunk, dtype=torch.float64, device=dev)
        for _ in range(steps // chunk):
            m.md_run(xd, v, f, td, box, 0.001, chunk, 0.5, prec, trace=trace)
            ke = 0.5 * mass * float((v * v).sum().item()) / FTM2V
            etot.append(float(trace[chunk - 1].item()) + ke)
        series[prec] = np.array(etot)
    el = time.perf_counter() - t0
    m.close()
    e64, emx, esp = series[FP64], series[MIXED], series[SINGLE]
    out["accuracy"] = {
        "atoms": n, "steps": steps, "dt_fs": 1.0, "sample_every": chunk,
        "max_rel_dev_mixed_vs_fp64": float(np.max(np.abs(emx - e64) / np.abs(e64))),
        "max_rel_dev_single_vs_fp64": float(np.max(np.abs(esp - e64) / np.abs(e64))),
        "max_drift_per_atom_fp64_eV": float(np.max(np.abs(e64 - e64[0])) / n),
        "max_drift_per_atom_mixed_eV": float(np.max(np.abs(emx - emx[0])) / n),
        "max_drift_per_atom_single_eV": float(np.max(np.abs(esp - esp[0])) / n),
        "seconds": el,
    }


def run_batch(args, out, dev):
    import torch

    from paper_1607_02904_amd import inputs
    from paper_1607_02904_amd.tersoff import MIXED, BatchPlan, Tersoff, table_sic
    print("bench: batch", file=sys.stderr, flush=True)
    nconf = 256 if args.quick else 1024
    confs = inputs.sic_liquid_batch(nconf=nconf)
    nat = np.array([len(c[1]) for c in confs], dtype=np.int32)
    boxes = np.array([c[2] for c in confs])
    xc = torch.as_tensor(np.concatenate([c[0] for c in confs]), device=dev)
    tc = torch.as_tensor(np.concatenate([c[1] for c in confs]), device=dev)
    mb = Tersoff(table_sic(), masses=[28.0855, 12.011])
    plan = BatchPlan(mb, nat, boxes, precision=MIXED)
    N = int(nat.sum())
    e = torch.empty(nconf, dtype=torch.float64, device=dev)
    f = torch.empty((N, 3), dtype=torch.float64, device=dev)
    w = torch.empty((nconf, 6), dtype=torch.float64, device=dev)
    eb = torch.full((nconf,), 1e-3, dtype=torch.float64, device=dev)
    fb = torch.randn((N, 3), dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(0)) * 0.1
    xg = torch.empty_like(f)
    pg = torch.empty((2, 2, 2, 14), dtype=torch.float64, device=dev)
    # a plan builds its lists again only when an atom moved since the last
    # build: the timed launches alternate between the positions and a copy
    # displaced by 1e-9 A, so that every launch builds every list
    xc2 = xc + 1e-9
    for xx in (xc, xc2):
        plan.run(xx, tc, e, f, w, eb, fb, xg, pg)
    torch.cuda.synchronize()
    reps = 10
    # the same positions every launch: the lists are reused
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run(xc2, tc, e, f, w, eb, fb, xg, pg)
    torch.cuda.synchronize()
    els = (time.perf_counter() - t0) / reps
    # the reported figure (timed last, so that a kernel trace ends with it)
    t0 = time.perf_counter()
    for r in range(reps):
        plan.run(xc2 if r % 2 else xc, tc, e, f, w, eb, fb, xg, pg)
    torch.cuda.synchronize()
    elb = (time.perf_counter() - t0) / reps
    mb.sync()
    out["batched"] = {"value": N / elb, "unit": "atom-steps/s (forward + adjoint)", "configs": nconf,
                      "atoms": N, "ms_per_launch": elb * 1e3,
                      "ms_per_launch_positions_unchanged": els * 1e3,
                      "note": "every timed launch builds the lists (positions alternate by 1e-9 A); "
                              "ms_per_launch_positions_unchanged: the lists reused",
                      "schedule": plan.schedule()}
    plan.close()
    mb.close()


if __name__ == "__main__":
    main()
