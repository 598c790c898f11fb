"""Python binding of libtersoff (ctypes over torch device tensors).

Argument marshalling only: every step of the computation runs in the HIP
library.  Torch supplies device memory and the current stream.  If the shared
library is missing, loading fails with an error; there is no fallback.

Units: Angstrom, eV, amu, ps.  Positions float64 [n, 3] on the GPU, species
int32 [n] on the GPU, box: three side lengths (host sequence).
"""
import ctypes
import os
import sys

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtersoff.so")

FP64 = 0
MIXED = 1
SINGLE = 2  # everything in FP32 (forward only)
ENERGY, FORCES, VIRIAL, PER_ATOM_E, ACCUMULATE, PARAM_GRAD = 1, 2, 4, 8, 16, 32
NFIELD = 14
FIELDS = ("m", "gamma", "lam3", "c", "d", "h", "n", "beta", "lam2", "B", "R", "D", "lam1", "A")

STATUS = {0: "TERS_OK", 1: "TERS_ERR_INVALID_ARG", 2: "TERS_ERR_BOX_TOO_SMALL",
          3: "TERS_ERR_NLIST_OVERFLOW", 4: "TERS_ERR_PARAMS", 5: "TERS_ERR_NOT_FINITE",
          6: "TERS_ERR_HIP", 7: "TERS_ERR_UNSUPPORTED", 8: "TERS_ERR_NO_LIST"}

EXPORTS = ("ters_create", "ters_destroy", "ters_set_stream", "ters_sync", "ters_last_error",
           "ters_set_params", "ters_build_nlist", "ters_needs_rebuild", "ters_nlist_stats",
           "ters_compute", "ters_compute_ex", "ters_backward", "ters_md_run", "ters_md_run_timed",
           "ters_md_rebuilds",
           "ters_batch_plan", "ters_batch_run", "ters_plan_destroy", "ters_plan_schedule",
           "ters_set_schedule", "ters_get_schedule", "ters_set_force_mode", "ters_set_filter", "ters_autotune",
           "ters_profile_forward", "ters_pair_compute", "ters_compute_static",
           "ters_table_sic",
           "ters_table_element", "ters_version")

_lib = None
_finalizing = sys.is_finalizing  # kept: module globals are cleared at shutdown


class TersoffError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code
        self.name = STATUS.get(code, str(code))


def load_library(path=LIB_PATH):
    """Load libtersoff.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libtersoff.so not built (run python -m paper_1607_02904_amd.build)")
    L = ctypes.CDLL(path)
    P, I32, U32, D, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double, ctypes.c_int64
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "ters_create": [PP, ctypes.c_int, P],
        "ters_destroy": [P],
        "ters_set_stream": [P, P],
        "ters_sync": [P],
        "ters_set_params": [P, I32, P, P],
        "ters_build_nlist": [P, I32, P, P, P, D],
        "ters_needs_rebuild": [P, P, P],
        "ters_nlist_stats": [P, P],
        "ters_compute": [P, I32, P, P, P, ctypes.c_int, U32, P, P, P, P],
        "ters_compute_ex": [P, I32, P, P, P, ctypes.c_int, U32, P, P, P, P, P],
        "ters_compute_static": [P, I32, P, P, P, ctypes.c_int, U32, P, P, P, P],
        "ters_backward": [P, I32, P, P, P, ctypes.c_int, D, P, P, P],
        "ters_md_run": [P, I32, P, P, P, P, P, D, I32, D, ctypes.c_int, P, ctypes.c_int],
        "ters_md_run_timed": [P, I32, P, P, P, P, P, D, I32, D, ctypes.c_int, P, P],
        "ters_md_rebuilds": [P, P],
        "ters_batch_plan": [P, I32, P, P, ctypes.c_int, U32, PP],
        "ters_batch_run": [P, P, P, P, P, P, P, P, P, P],
        "ters_plan_destroy": [P],
        "ters_plan_schedule": [P, P],
        "ters_set_schedule": [P, I32, I32, I32],
        "ters_set_force_mode": [P, I32],
        "ters_set_filter": [P, I32],
        "ters_pair_compute": [P, I32, P, P, D, D, D, ctypes.c_int, U32, P, P, P],
        "ters_get_schedule": [P, I32, P],
        "ters_autotune": [P, I32, P, P, P, ctypes.c_int, P],
        "ters_profile_forward": [P, I32, P, P, P, ctypes.c_int, I32, I32, P],
        "ters_table_sic": [P],
        "ters_table_element": [I32, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ters_last_error.argtypes = [P]
    L.ters_last_error.restype = ctypes.c_char_p
    L.ters_version.argtypes = []
    L.ters_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(t, dtype=torch.float64, name="tensor", rows=None, cols=None):
    """Device address of a tensor handed to the library, after checking what
    the C interface assumes of it: on a GPU, contiguous, of the given dtype
    (float64 for positions, forces and cotangents, int32 for species) and,
    when given, of the given leading size and row width."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, not %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if rows is not None and (t.dim() == 0 or t.shape[0] != rows):
        raise ValueError("%s must have %d rows, not shape %s" % (name, rows, tuple(t.shape)))
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError("%s must have shape (n, %d), not %s" % (name, cols, tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _pos(x, name="x"):
    return _ptr(x, torch.float64, name, cols=3)


def _types(t, n):
    return _ptr(t, torch.int32, "types", rows=n)


def _hostbuf(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def table_sic():
    """2-species Si/C table (Si(C) set, Tersoff 1989 mixing) from the library."""
    t = np.zeros((2, 2, 2, NFIELD))
    _check(None, load_library().ters_table_sic(t.ctypes.data_as(ctypes.c_void_p)))
    return t


def table_element(which):
    """One-species table: 'Si(B)', 'Si(C)' or 'C'."""
    idx = {"Si(B)": 0, "Si(C)": 1, "C": 2}[which]
    t = np.zeros((1, 1, 1, NFIELD))
    _check(None, load_library().ters_table_element(idx, t.ctypes.data_as(ctypes.c_void_p)))
    return t


def _check(ctx, code):
    if code != 0:
        msg = load_library().ters_last_error(ctx).decode() if ctx else ""
        raise TersoffError(code, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Tersoff:
    """One library context on one GPU, with its parameter table and list."""

    def __init__(self, table, masses=None, device=0):
        self._L = load_library()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(None, self._L.ters_create(ctypes.byref(h), device, _stream()))
        self._h = h
        self.set_params(table, masses)
        self.skin = 0.0
        self.box = None

    def close(self):
        if getattr(self, "_h", None):
            self._L.ters_destroy(self._h)
            self._h = None

    def __del__(self):
        # during interpreter shutdown the HIP runtime may already be gone
        if _finalizing is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code):
        _check(self._h, code)

    def _bind_stream(self):
        self._L.ters_set_stream(self._h, _stream())

    def set_params(self, table, masses=None):
        t = np.ascontiguousarray(table, dtype=np.float64)
        nt = t.shape[0]
        assert t.shape == (nt, nt, nt, NFIELD), t.shape
        self.table = t
        self.ntypes = nt
        m = None if masses is None else np.ascontiguousarray(masses, dtype=np.float64)
        self._chk(self._L.ters_set_params(self._h, nt, t.ctypes.data_as(ctypes.c_void_p),
                                          None if m is None else m.ctypes.data_as(ctypes.c_void_p)))

    # -- neighbour list ---------------------------------------------------------
    def build_nlist(self, x, types, box, skin=0.0):
        self._bind_stream()
        b, bp = _hostbuf(box, np.float64)
        self._chk(self._L.ters_build_nlist(self._h, x.shape[0], _pos(x), _types(types, x.shape[0]), bp,
                                           float(skin)))
        self.skin = float(skin)
        self.box = b.copy()

    def needs_rebuild(self, x, flag=None):
        self._bind_stream()
        if flag is None:
            flag = torch.zeros(1, dtype=torch.int32, device=x.device)
        self._chk(self._L.ters_needs_rebuild(self._h, _pos(x), _ptr(flag, torch.int32, "flag")))
        return flag

    def nlist_stats(self):
        out = np.zeros(4, dtype=np.int64)
        self._chk(self._L.ters_nlist_stats(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return dict(n=int(out[0]), entries=int(out[1]), longest=int(out[2]), capacity=int(out[3]))

    def set_schedule(self, kernel=0, atoms=0, kmax=0):
        """kernel 1: workgroup schedule (atoms per workgroup <= 64, k_max);
        kernel 2: wavefront schedule (atoms per wavefront <= 32); kernel 3:
        thread per atom (forward only, atomic scatter); 0: default."""
        self._chk(self._L.ters_set_schedule(self._h, int(kernel), int(atoms), int(kmax)))

    def schedules(self):
        """Current kernel / atoms / force mode per precision."""
        out = {}
        for name, prec in (("fp64", FP64), ("mixed", MIXED), ("single", SINGLE)):
            v = np.zeros(3, dtype=np.int32)
            self._chk(self._L.ters_get_schedule(self._h, prec, v.ctypes.data_as(ctypes.c_void_p)))
            out[name] = {"kernel": int(v[0]), "atoms": int(v[1]), "force_mode": "gather" if v[2] else "atomic"}
        return out

    def set_filter(self, enabled=True):
        """Filter of in-cutoff pairs before the compute lanes (wavefront schedule);
        off only to measure it."""
        self._chk(self._L.ters_set_filter(self._h, 1 if enabled else 0))

    def set_force_mode(self, gather=True):
        """gather=True: owner-gather (deterministic, no atomics); False: FP64 atomics."""
        self._chk(self._L.ters_set_force_mode(self._h, 1 if gather else 0))

    def autotune(self, x, types, box, precision=FP64):
        self._bind_stream()
        b, bp = _hostbuf(box, np.float64)
        us = ctypes.c_double()
        self._chk(self._L.ters_autotune(self._h, x.shape[0], _pos(x), _types(types, x.shape[0]), bp, precision,
                                        ctypes.byref(us)))
        return us.value

    def profile_forward(self, x, types, box, precision=FP64, reps=20, with_gather=False):
        """Average force-kernel duration in microseconds (HIP events); with
        with_gather the owner-gather pass is included."""
        self._bind_stream()
        b, bp = _hostbuf(box, np.float64)
        us = ctypes.c_double()
        self._chk(self._L.ters_profile_forward(self._h, x.shape[0], _pos(x), _types(types, x.shape[0]), bp, precision,
                                               int(reps), int(bool(with_gather)), ctypes.byref(us)))
        return us.value

    # -- evaluation --------------------------------------------------------------
    def compute(self, x, types, box, precision=FP64, energy=True, forces=True, virial=True,
                per_atom=False, param_grad=False, out=None):
        """Energy [1], forces [n,3], virial [6], per-atom energy [n] and
        dE/dtable as float64 device tensors (a dict)."""
        self._bind_stream()
        n = x.shape[0]
        dev = x.device
        o = dict(out or {})
        flags = 0
        if energy:
            flags |= ENERGY
            o.setdefault("energy", torch.empty(1, dtype=torch.float64, device=dev))
        if forces:
            flags |= FORCES
            o.setdefault("forces", torch.empty((n, 3), dtype=torch.float64, device=dev))
        if virial:
            flags |= VIRIAL
            o.setdefault("virial", torch.empty(6, dtype=torch.float64, device=dev))
        if per_atom:
            flags |= PER_ATOM_E
            o.setdefault("e_atom", torch.empty(n, dtype=torch.float64, device=dev))
        if param_grad:
            flags |= PARAM_GRAD
            o.setdefault("param_grad", torch.zeros(self.table.shape, dtype=torch.float64, device=dev))
        b, bp = _hostbuf(box, np.float64)
        self._chk(self._L.ters_compute_ex(self._h, n, _pos(x), _types(types, n), bp, precision, flags,
                                          _ptr(o.get("energy"), name="energy", rows=1),
                                          _ptr(o.get("forces"), name="forces", rows=n, cols=3),
                                          _ptr(o.get("virial"), name="virial", rows=6),
                                          _ptr(o.get("e_atom"), name="e_atom", rows=n),
                                          _ptr(o.get("param_grad"), name="param_grad")))
        return o

    def compute_static(self, x, types, box, precision=FP64, out=None, per_atom=False):
        """ters_compute_static: list build and evaluation in one call with no
        device allocation inside the library (outputs as compute(); the
        caller may pass preallocated ones in `out`)."""
        self._bind_stream()
        n = x.shape[0]
        dev = x.device
        o = dict(out or {})
        o.setdefault("energy", torch.empty(1, dtype=torch.float64, device=dev))
        o.setdefault("forces", torch.empty((n, 3), dtype=torch.float64, device=dev))
        o.setdefault("virial", torch.empty(6, dtype=torch.float64, device=dev))
        flags = ENERGY | FORCES | VIRIAL
        if per_atom:
            flags |= PER_ATOM_E
            o.setdefault("e_atom", torch.empty(n, dtype=torch.float64, device=dev))
        b, bp = _hostbuf(box, np.float64)
        self._chk(self._L.ters_compute_static(self._h, n, _pos(x), _types(types, n), bp, precision,
                                              flags, _ptr(o["energy"], name="energy", rows=1),
                                              _ptr(o["forces"], name="forces", rows=n, cols=3),
                                              _ptr(o["virial"], name="virial", rows=6),
                                              _ptr(o.get("e_atom"), name="e_atom", rows=n)))
        return o

    def pair_compute(self, x, box, eps, sigma, rc, precision=FP64):
        """Truncated Lennard-Jones (the paper's Algorithm 1 over this context's
        list): energy [1], forces [n,3], virial [6] as float64 device tensors."""
        self._bind_stream()
        n = x.shape[0]
        dev = x.device
        o = {"energy": torch.empty(1, dtype=torch.float64, device=dev),
             "forces": torch.empty((n, 3), dtype=torch.float64, device=dev),
             "virial": torch.empty(6, dtype=torch.float64, device=dev)}
        b, bp = _hostbuf(box, np.float64)
        self._chk(self._L.ters_pair_compute(self._h, n, _pos(x), bp, float(eps), float(sigma),
                                            float(rc), precision, ENERGY | FORCES | VIRIAL,
                                            _ptr(o["energy"]), _ptr(o["forces"]), _ptr(o["virial"])))
        return o

    def backward(self, x, types, box, e_bar, f_bar, precision=FP64):
        """Vector-Jacobian product of (E, F) with cotangents (e_bar, f_bar):
        returns (x_grad [n,3], param_grad [nt,nt,nt,14])."""
        self._bind_stream()
        n = x.shape[0]
        xg = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        pg = torch.empty(self.table.shape, dtype=torch.float64, device=x.device)
        b, bp = _hostbuf(box, np.float64)
        fb = f_bar.contiguous()
        self._chk(self._L.ters_backward(self._h, n, _pos(x), _types(types, n), bp, precision,
                                        float(e_bar), _ptr(fb, name="f_bar", rows=n, cols=3),
                                        _ptr(xg), _ptr(pg)))
        return xg, pg

    def md_run(self, x, v, f, types, box, dt, nsteps, skin, precision=FP64, trace=None,
               use_graph=True):
        """Velocity Verlet in place on x, v, f; returns the energy trace."""
        self._bind_stream()
        if trace is None:
            trace = torch.empty(max(nsteps, 1), dtype=torch.float64, device=x.device)
        b, bp = _hostbuf(box, np.float64)
        n = x.shape[0]
        self._chk(self._L.ters_md_run(self._h, n, _pos(x), _pos(v, "v"), _pos(f, "f"), _types(types, n), bp,
                                      float(dt), int(nsteps), float(skin), precision,
                                      _ptr(trace, name="trace"),
                                      1 if use_graph else 0))
        return trace

    def md_run_timed(self, x, v, f, types, box, dt, nsteps, skin, precision=FP64, trace=None):
        """md_run launched step by step with HIP events around every force-kernel
        launch; returns (trace, average force-kernel microseconds)."""
        self._bind_stream()
        if trace is None:
            trace = torch.empty(max(nsteps, 1), dtype=torch.float64, device=x.device)
        b, bp = _hostbuf(box, np.float64)
        us = np.zeros(1, dtype=np.float64)
        n = x.shape[0]
        self._chk(self._L.ters_md_run_timed(self._h, n, _pos(x), _pos(v, "v"), _pos(f, "f"),
                                            _types(types, n), bp, float(dt), int(nsteps), float(skin),
                                            precision, _ptr(trace, name="trace"),
                                            us.ctypes.data_as(ctypes.c_void_p)))
        return trace, float(us[0])

    def sync(self):
        self._chk(self._L.ters_sync(self._h))

    def rebuilds(self):
        out = np.zeros(1, dtype=np.int64)
        self._chk(self._L.ters_md_rebuilds(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return int(out[0])


class BatchPlan:
    """Many independent configurations evaluated with one graph launch."""

    def __init__(self, model, natoms, boxes, precision=MIXED):
        self.model = model
        L = model._L
        self._L = L
        model._bind_stream()
        na = np.ascontiguousarray(natoms, dtype=np.int32)
        bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        self.nconf = na.size
        self.natoms = na
        self.offsets = np.concatenate([[0], np.cumsum(na)])
        h = ctypes.c_void_p()
        _check(model._h, L.ters_batch_plan(model._h, self.nconf, na.ctypes.data_as(ctypes.c_void_p),
                                           bx.ctypes.data_as(ctypes.c_void_p), precision, 0,
                                           ctypes.byref(h)))
        self._h = h

    def run(self, x, types, e=None, f=None, w=None, e_bar=None, f_bar=None, x_grad=None,
            param_grad=None):
        """Evaluate every configuration (ters_batch_run): energies e, forces f
        and virials w, any of them None; with f_bar (and e_bar, x_grad,
        param_grad) also the adjoint.  With f_bar given and e, f, w all None
        the graph runs the list build and the adjoint alone."""
        self.model._bind_stream()
        N = int(self.offsets[-1])
        _check(self.model._h, self._L.ters_batch_run(
            self._h, _ptr(x, name="x", rows=N, cols=3), _types(types, N), _ptr(e, name="e", rows=self.nconf),
            _ptr(f, name="f", rows=N, cols=3), _ptr(w, name="w", rows=self.nconf, cols=6),
            _ptr(e_bar, name="e_bar", rows=self.nconf), _ptr(f_bar, name="f_bar", rows=N, cols=3),
            _ptr(x_grad, name="x_grad", rows=N, cols=3), _ptr(param_grad, name="param_grad")))

    def schedule(self):
        out = np.zeros(6)
        _check(self.model._h, self._L.ters_plan_schedule(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return dict(atoms=int(out[0]), kernel=int(out[1]), us=float(out[2]),
                    adjoint_atoms=int(out[3]), adjoint_us=float(out[4]), workgroups=int(out[5]))

    def close(self):
        if getattr(self, "_h", None):
            self._L.ters_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        if _finalizing is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class TersoffEF(torch.autograd.Function):
    """(E, F) = Tersoff(x; table) with a hand-written adjoint.

    Forward and backward each build the neighbour list for their x, and the
    backward runs at the table of its own forward, so several frames (and
    parameter updates between steps) can share one model.

    forward(model, x, table, types, box, precision) -> (E [1], F [n,3])
    backward returns dL/dx and dL/dtable from one dual-number pass of the
    force kernel (zeta recomputed, no stored triplets)."""

    @staticmethod
    def _use(model, tab, x, types, box):
        """Make `tab` the model's table and build the list for x (with the
        model's skin): a fitting loop evaluates many frames, and the
        backward of one may run after the forward of another, so neither
        pass relies on a list built elsewhere."""
        if not np.array_equal(tab, model.table):
            model.set_params(tab)
        model.build_nlist(x, types, box, model.skin)

    @staticmethod
    def forward(ctx, model, x, table, types, box, precision=FP64):
        tab = table.detach().cpu().numpy().astype(np.float64)
        TersoffEF._use(model, tab, x.detach(), types, box)
        o = model.compute(x.detach(), types, box, precision, energy=True, forces=True, virial=False)
        ctx.model = model
        ctx.types = types
        ctx.box = np.asarray(box, dtype=np.float64)
        ctx.precision = precision
        ctx.table_device = table.device
        ctx.table = tab  # the adjoint runs at the parameters of this forward
        ctx.save_for_backward(x)
        return o["energy"], o["forces"]

    @staticmethod
    def backward(ctx, e_bar, f_bar):
        (x,) = ctx.saved_tensors
        eb = 0.0 if e_bar is None else float(e_bar.reshape(-1)[0].item())
        if f_bar is None:
            f_bar = torch.zeros_like(x)
        TersoffEF._use(ctx.model, ctx.table, x.detach(), ctx.types, ctx.box)
        xg, pg = ctx.model.backward(x.detach(), ctx.types, ctx.box, eb, f_bar.contiguous(),
                                    ctx.precision)
        return None, xg, pg.to(ctx.table_device), None, None, None
