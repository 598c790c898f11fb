"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It wraps ``tersoff_oracle.c`` (plain C, FP64, the paper's
Algorithm 2) with ctypes and adds the plain NumPy pieces that sit around the
potential: the fitting loss and velocity-Verlet time integration.

The shared library is compiled by the build step (``__graft_entry__.build``);
if it is missing it is compiled here with gcc.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tersoff_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

# "metal" units: force/mass in eV/(Angstrom amu) -> Angstrom/ps^2, from the
# SI values of the elementary charge (exact) and the atomic mass constant
# (CODATA 2018): (1.602176634e-19 J / 1e-10 m) / 1.66053906660e-27 kg in m/s^2,
# times 1e10 Angstrom/m and 1e-24 s^2/ps^2
FTM2V = 1.602176634e-19 / 1.66053906660e-27 * 1e-4
MASS = {"Si": 28.0855, "C": 12.011}


def build(force=True):
    """Compile the oracle with gcc (-O2, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_LIB_THREADS = os.path.join(_HERE, "_build", "liboracle_threads.so")
_lib_threads = None


def build_threads():
    """The same source compiled for timing on all host cores: -O3
    -march=native -fopenmp (built on the machine that runs it, since
    -march=native targets that machine's CPU)."""
    os.makedirs(os.path.dirname(_LIB_THREADS), exist_ok=True)
    tmp = _LIB_THREADS + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared",
                           "-std=c99", "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_THREADS)
    return _LIB_THREADS


def compute_threads(x, types, box, table, nlist, threads=0):
    """Energy, forces and virial over a prebuilt list with the centres shared
    among the OpenMP threads (OMP_NUM_THREADS, or at most `threads` when it is
    positive); returns (E, F, W, threads used)."""
    global _lib_threads
    if _lib_threads is None:
        L = ctypes.CDLL(build_threads())
        P, I = ctypes.c_void_p, ctypes.c_int
        L.orc_tersoff_threads.argtypes = [I, P, P, P, I, P, P, P, I, I, P, P, P]
        L.orc_tersoff_threads.restype = I
        _lib_threads = L
    x = _f64(x, (-1, 3))
    box = _f64(box, (3,))
    table = _f64(table)
    types = np.ascontiguousarray(types, dtype=np.int32)
    count, lst = nlist
    n = x.shape[0]
    e = np.zeros(1)
    f = np.zeros((n, 3))
    w = np.zeros(6)
    nthr = _lib_threads.orc_tersoff_threads(n, _p(x), _p(types), _p(box), table.shape[0], _p(table),
                                            _p(count), _p(lst), lst.shape[1], int(threads), _p(e),
                                            _p(f), _p(w))
    if nthr <= 0:
        raise RuntimeError("oracle threaded compute failed (%d)" % nthr)
    return float(e[0]), f, w, nthr


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.orc_neigh_brute.argtypes = [I, P, P, D, I, P, P, P]
        L.orc_neigh_cells.argtypes = [I, P, P, D, I, P, P, P]
        L.orc_tersoff.argtypes = [I, P, P, P, I, P, P, P, I, I, P, P, P, P, P]
        L.orc_tersoff_images.argtypes = [I, P, P, P, I, P, I, P, P, P, P]
        for f in (L.orc_neigh_brute, L.orc_neigh_cells, L.orc_tersoff, L.orc_tersoff_images):
            f.restype = I
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def neighbours(x, box, rlist, method="cells", cap=None):
    """Full neighbour list {j != i: r_ij <= rlist} (minimum image).
    Returns (count[n], list[n, cap]) with rows sorted by j."""
    x = _f64(x, (-1, 3))
    box = _f64(box, (3,))
    n = x.shape[0]
    fn = lib().orc_neigh_cells if method == "cells" else lib().orc_neigh_brute
    cap = cap or 32
    while True:
        count = np.zeros(n, dtype=np.int32)
        lst = np.full((n, cap), -1, dtype=np.int32)
        need = np.zeros(1, dtype=np.int32)
        rc = fn(n, _p(x), _p(box), float(rlist), cap, _p(count), _p(lst), _p(need))
        if rc == 3:
            cap = int(need[0])
            continue
        if rc == 2:
            raise ValueError("box side below twice the list cutoff")
        if rc != 0:
            raise RuntimeError("oracle neighbour build failed (%d)" % rc)
        return count, lst


def compute(x, types, box, table, rlist=None, nlist=None, centres=None):
    """Energy, forces [n,3], virial [6] (xx yy zz xy xz yz) and per-atom
    energy [n] by Algorithm 2 over a full neighbour list.

    rlist defaults to the largest cutoff in the table.  With ``centres`` only
    the terms rooted at those atoms are summed (see orc_tersoff)."""
    x = _f64(x, (-1, 3))
    box = _f64(box, (3,))
    table = _f64(table)
    nt = table.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    n = x.shape[0]
    if nlist is None:
        if rlist is None:
            rlist = float(np.max(table[..., 10] + table[..., 11]))
        nlist = neighbours(x, box, rlist)
    count, lst = nlist
    cen = None if centres is None else np.ascontiguousarray(centres, dtype=np.int32)
    e = np.zeros(1)
    f = np.zeros((n, 3))
    w = np.zeros(6)
    ea = np.zeros(n)
    rc = lib().orc_tersoff(n, _p(x), _p(types), _p(box), nt, _p(table), _p(count), _p(lst),
                           lst.shape[1], 0 if cen is None else cen.size, _p(cen),
                           _p(e), _p(f), _p(w), _p(ea))
    if rc != 0:
        raise RuntimeError("oracle compute failed (%d)" % rc)
    return float(e[0]), f, w, ea


def compute_images(x, types, box, table, nimg):
    """Brute force with explicit periodic images (no lists, no minimum image)."""
    x = _f64(x, (-1, 3))
    box = _f64(box, (3,))
    table = _f64(table)
    types = np.ascontiguousarray(types, dtype=np.int32)
    n = x.shape[0]
    e = np.zeros(1)
    f = np.zeros((n, 3))
    w = np.zeros(6)
    ea = np.zeros(n)
    rc = lib().orc_tersoff_images(n, _p(x), _p(types), _p(box), table.shape[0], _p(table), int(nimg),
                                  _p(e), _p(f), _p(w), _p(ea))
    if rc != 0:
        raise RuntimeError("oracle brute force failed (%d)" % rc)
    return float(e[0]), f, w, ea


def forces_on(x, types, box, table, atoms, nlist=None, rlist=None):
    """Exact forces on the listed atoms and exact per-atom energies of them,
    computed from the terms rooted at each atom and at its in-list neighbours
    only, so that single outputs of very large systems can be checked."""
    x = _f64(x, (-1, 3))
    if rlist is None:
        rlist = float(np.max(table[..., 10] + table[..., 11]))
    if nlist is None:
        nlist = neighbours(x, box, rlist)
    count, lst = nlist
    atoms = np.asarray(atoms, dtype=np.int64)
    cen = set(int(a) for a in atoms)
    for a in atoms:
        cen.update(int(j) for j in lst[a, :count[a]])
    cen = np.array(sorted(cen), dtype=np.int32)
    _, f, _, ea = compute(x, types, box, table, nlist=nlist, centres=cen)
    return f[atoms], ea[atoms]


def loss(frames, table, refs, wf=0.1):
    """Fitting loss sum_frames (E - E_ref)^2 / N^2 + wf * sum_a |F_a - F_ref,a|^2.
    frames: list of (x, types, box); refs: list of (E_ref, F_ref)."""
    total = 0.0
    for (x, t, box), (er, fr) in zip(frames, refs):
        e, f, _, _ = compute(x, t, box, table)
        n = len(t)
        total += (e - er) ** 2 / n ** 2 + wf * float(np.sum((f - fr) ** 2))
    return total


def velocity_verlet(x, v, types, box, table, masses, dt, nsteps):
    """Plain velocity Verlet (metal units; dt in ps), with the neighbour list
    rebuilt at every force evaluation.  Returns x, v, f, energy trace."""
    x = _f64(x, (-1, 3)).copy()
    v = _f64(v, (-1, 3)).copy()
    m = np.asarray(masses, dtype=np.float64)[np.asarray(types)][:, None]
    e, f, _, _ = compute(x, types, box, table)
    trace = []
    for _ in range(nsteps):
        v += 0.5 * dt * FTM2V * f / m
        x += dt * v
        e, f, _, _ = compute(x, types, box, table)
        v += 0.5 * dt * FTM2V * f / m
        trace.append(e)
    return x, v, f, np.array(trace)
