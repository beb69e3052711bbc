"""ctypes binding of the C-ABI declared in include/nlte3d.h.

Argument marshalling only: every step of the method runs in the HIP library
``libnlte3d.so``.  ``load()`` raises if the library has not been built; there is no
fallback.  Host numpy arrays or torch device tensors may be passed as inputs; outputs
are returned as numpy arrays (or written into caller-provided torch tensors).
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlte3d.so")

OK, E_INVALID, E_OOM, E_DEVICE, E_DIVERGED = 0, -1, -2, -3, -4
W_NOT_CONVERGED, W_QUEUED = 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
MALI, FAS, FMG = 0, 1, 2
FP64, MIXED = 0, 1
SWEEP_AUTO, SWEEP_PLANE_STEP = 0, 1
RESTRICT_FULL, RESTRICT_HALF, RESTRICT_INJECT = 0, 1, 2
INTERP_TRILINEAR, INTERP_HERMITE = 0, 1
SC_BILINEAR, SC_HERMITE = 0, 1
INIT_ZERO_RAD, INIT_LTE, INIT_USER = 0, 1, 2

SYMBOLS = (
    "nlte_ctx_create", "nlte_ctx_destroy", "nlte_last_error", "nlte_version",
    "nlte_atom_create", "nlte_atom_destroy", "nlte_atmos_create", "nlte_atmos_destroy",
    "nlte_job_create", "nlte_job_run", "nlte_solve", "nlte_release", "nlte_batch_run",
    "nlte_get_populations", "nlte_set_populations", "nlte_get_source_function", "nlte_job_stats",
    "nlte_emergent_intensity", "nlte_emergent_intensity_noalloc", "nlte_emergent_continuum_intensity",
    "nlte_history",
    "nlte_formal_solution", "nlte_mali", "nlte_rate_solve", "nlte_residual", "nlte_vcycle",
    "nlte_restrict", "nlte_prolong", "nlte_voigt",
    "nlte_serve_config", "nlte_serve_batching", "nlte_estimate_footprint", "nlte_submit", "nlte_poll", "nlte_wait",
    "nlte_job_info",
)
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3


class NlteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nlte3d error {code}: {msg}")
        self.code = code


# ------------------------------------------------------------------ C structs
class LevelDesc(ct.Structure):
    _fields_ = [("E", ct.c_double), ("g", ct.c_double), ("stage", ct.c_int)]


class LineDesc(ct.Structure):
    _fields_ = [("lower", ct.c_int), ("upper", ct.c_int), ("A", ct.c_double),
                ("gamma_rad", ct.c_double), ("gamma_vdw", ct.c_double),
                ("nfreq", ct.c_int), ("q", ct.POINTER(ct.c_double))]


class ContDesc(ct.Structure):
    _fields_ = [("lower", ct.c_int), ("upper", ct.c_int), ("alpha0", ct.c_double)]


class CollDesc(ct.Structure):
    _fields_ = [("lower", ct.c_int), ("upper", ct.c_int), ("c_ul", ct.c_double),
                ("T_ref", ct.c_double), ("beta", ct.c_double)]


class AtomDesc(ct.Structure):
    _fields_ = [("nlevel", ct.c_int), ("nline", ct.c_int), ("ncont", ct.c_int), ("ncoll", ct.c_int),
                ("mass_amu", ct.c_double), ("xi", ct.c_double), ("epsilon", ct.c_double),
                ("levels", ct.POINTER(LevelDesc)), ("lines", ct.POINTER(LineDesc)),
                ("continua", ct.POINTER(ContDesc)), ("collisions", ct.POINTER(CollDesc)),
                ("ncont_nu", ct.c_int), ("cont_nu", ct.POINTER(ct.c_double))]


class AtmosDesc(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("dx", ct.c_double), ("dy", ct.c_double), ("z", ct.POINTER(ct.c_double)),
                ("T", ct.c_void_p), ("ne", ct.c_void_p), ("nH", ct.c_void_p), ("ntot", ct.c_void_p),
                ("vx", ct.c_void_p), ("vy", ct.c_void_p), ("vz", ct.c_void_p),
                ("chi_c", ct.c_void_p), ("nchi", ct.c_int), ("mem_kind", ct.c_int)]


class Params(ct.Structure):
    _fields_ = [("method", ct.c_int), ("precision", ct.c_int), ("nlev", ct.c_int),
                ("nu_fmg", ct.c_int), ("nu0", ct.c_int), ("nu1", ct.c_int), ("nu2", ct.c_int), ("nu3", ct.c_int),
                ("init", ct.c_int), ("init_pops", ct.POINTER(ct.c_double)),
                ("tol_C", ct.c_double), ("E_target", ct.c_double), ("max_iter", ct.c_int),
                ("repair_frac", ct.c_double), ("fallback_mali", ct.c_int),
                ("top_I", ct.POINTER(ct.c_double)), ("dirs_per_block", ct.c_int), ("timing", ct.c_int),
                ("graph", ct.c_int), ("sweep_kernel", ct.c_int), ("restriction", ct.c_int),
                ("coarse_atmos", ct.c_int), ("interpolation", ct.c_int), ("sc_interp", ct.c_int),
                ("diverge_cycles", ct.c_int), ("diverge_growth", ct.c_double)]


class Result(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iterations", ct.c_int), ("cycles", ct.c_int),
                ("C", ct.c_double), ("rho", ct.c_double), ("E_est", ct.c_double),
                ("repairs", ct.c_longlong), ("formal_solutions", ct.c_longlong * 8),
                ("fine_fs_equiv", ct.c_double), ("updates", ct.c_double),
                ("ms_total", ct.c_double), ("ms_setup", ct.c_double), ("ms_sweep", ct.c_double),
                ("ms_rates", ct.c_double), ("ms_transfer", ct.c_double), ("sweep_launches", ct.c_longlong),
                ("dirs_per_block", ct.c_int), ("sweep_kernel", ct.c_int), ("fallback", ct.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "formal_solutions"}
        d["formal_solutions"] = list(self.formal_solutions)
        return d


class JobInfo(ct.Structure):
    _fields_ = [("state", ct.c_int), ("status", ct.c_int), ("t_submit", ct.c_double), ("t_admit", ct.c_double),
                ("t_done", ct.c_double), ("footprint", ct.c_size_t), ("batch", ct.c_int), ("result", Result),
                ("error", ct.c_char * 256)]


_lib = None


def load(path=None):
    """Open the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run __graft_entry__.build() first")
    lib = ct.CDLL(path)
    P = ct.c_void_p
    I64 = ct.c_int64
    lib.nlte_ctx_create.argtypes = [ct.c_int, P, ct.c_size_t, ct.POINTER(P)]
    lib.nlte_ctx_destroy.argtypes = [P]
    lib.nlte_ctx_destroy.restype = None
    lib.nlte_last_error.argtypes = [P]
    lib.nlte_last_error.restype = ct.c_char_p
    lib.nlte_version.restype = ct.c_char_p
    lib.nlte_atom_create.argtypes = [P, ct.POINTER(AtomDesc), ct.POINTER(P)]
    lib.nlte_atom_destroy.argtypes = [P, P]
    lib.nlte_atom_destroy.restype = None
    lib.nlte_atmos_create.argtypes = [P, ct.POINTER(AtmosDesc), ct.POINTER(P)]
    lib.nlte_atmos_destroy.argtypes = [P, P]
    lib.nlte_atmos_destroy.restype = None
    lib.nlte_job_create.argtypes = [P, P, P, ct.POINTER(Params), ct.POINTER(I64)]
    lib.nlte_job_run.argtypes = [P, I64, ct.POINTER(Result)]
    lib.nlte_solve.argtypes = [P, P, P, ct.POINTER(Params), ct.POINTER(Result), ct.POINTER(I64)]
    lib.nlte_release.argtypes = [P, I64]
    lib.nlte_batch_run.argtypes = [P, ct.c_int, ct.POINTER(I64), ct.POINTER(Result)]
    lib.nlte_get_populations.argtypes = [P, I64, ct.c_int, P, ct.c_int]
    lib.nlte_set_populations.argtypes = [P, I64, ct.c_int, P, ct.c_int]
    lib.nlte_get_source_function.argtypes = [P, I64, P, ct.c_int]
    lib.nlte_emergent_intensity.argtypes = [P, I64, ct.c_int, P, P, ct.c_int]
    lib.nlte_emergent_intensity_noalloc.argtypes = [P, I64, ct.c_int, P, P]
    lib.nlte_emergent_continuum_intensity.argtypes = [P, I64, ct.c_int, P, P, ct.c_int]
    lib.nlte_history.argtypes = [P, I64, P, ct.c_int]
    lib.nlte_job_stats.argtypes = [P, I64, ct.POINTER(Result)]
    lib.nlte_formal_solution.argtypes = [P, I64, ct.c_int, P, P, ct.c_int]
    lib.nlte_mali.argtypes = [P, I64, ct.c_int, ct.c_int, ct.POINTER(ct.c_double)]
    lib.nlte_rate_solve.argtypes = [P, I64, ct.c_int, P, P, ct.c_int, ct.POINTER(ct.c_double)]
    lib.nlte_residual.argtypes = [P, I64, ct.c_int, P, ct.c_int]
    lib.nlte_vcycle.argtypes = [P, I64, ct.c_int, ct.c_int, ct.POINTER(ct.c_longlong)]
    lib.nlte_restrict.argtypes = [P, I64, ct.c_int, ct.c_int, P, P]
    lib.nlte_prolong.argtypes = [P, I64, ct.c_int, ct.c_int, P, P]
    lib.nlte_voigt.argtypes = [P, ct.c_int, ct.c_int, P, P, P]
    lib.nlte_serve_config.argtypes = [P, ct.c_int]
    lib.nlte_serve_batching.argtypes = [P, ct.c_int]
    lib.nlte_estimate_footprint.argtypes = [P, P, P, ct.POINTER(Params), ct.POINTER(ct.c_size_t)]
    lib.nlte_submit.argtypes = [P, P, P, ct.POINTER(Params), ct.POINTER(I64)]
    lib.nlte_poll.argtypes = [P, I64, ct.POINTER(ct.c_int)]
    lib.nlte_wait.argtypes = [P, I64, ct.c_int]
    lib.nlte_job_info.argtypes = [P, I64, ct.POINTER(JobInfo)]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class SolveParams:
    method: int = FAS
    precision: int = MIXED
    nlev: int = 3
    nu_fmg: int = 16
    nu0: int = 0
    nu1: int = 2
    nu2: int = 2
    nu3: int = 32
    init: int = INIT_ZERO_RAD
    tol_C: float = 0.0
    E_target: float = 1e-3
    max_iter: int = 100
    repair_frac: float = 0.1
    fallback_mali: int = 0
    dirs_per_block: int = 0
    timing: int = 0
    graph: int = 0
    sweep_kernel: int = 0
    restriction: int = 0       # RESTRICT_FULL / _HALF / _INJECT
    coarse_atmos: int = 0      # RESTRICT_FULL / _INJECT (or _HALF)
    interpolation: int = 0     # INTERP_TRILINEAR / _HERMITE
    sc_interp: int = 0         # SC_BILINEAR / SC_HERMITE
    diverge_cycles: int = 0    # consecutive growing cycles that count as divergence (0: 3, < 0: off)
    diverge_growth: float = 0.0   # growth factor of that test (0: 1)
    init_pops: np.ndarray | None = None
    top_I: np.ndarray | None = None
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self):
        p = Params()
        for k in ("method", "precision", "nlev", "nu_fmg", "nu0", "nu1", "nu2", "nu3", "init",
                  "max_iter", "fallback_mali", "dirs_per_block", "timing", "graph", "sweep_kernel",
                  "restriction", "coarse_atmos", "interpolation", "sc_interp", "diverge_cycles"):
            setattr(p, k, int(getattr(self, k)))
        for k in ("tol_C", "E_target", "repair_frac", "diverge_growth"):
            setattr(p, k, float(getattr(self, k)))
        self._keep = []
        if self.init_pops is not None:
            a = _f64(self.init_pops)
            self._keep.append(a)
            p.init_pops = a.ctypes.data_as(ct.POINTER(ct.c_double))
        if self.top_I is not None:
            a = _f64(self.top_I)
            self._keep.append(a)
            p.top_I = a.ctypes.data_as(ct.POINTER(ct.c_double))
        return p


class Context:
    """One device, one HIP stream (torch's current stream when torch is initialised)."""

    def __init__(self, device=0, stream=None, hbm_budget=0):
        self.lib = load()
        h = ct.c_void_p()
        st = ct.c_void_p(stream) if stream else None
        rc = self.lib.nlte_ctx_create(device, st, hbm_budget, ct.byref(h))
        if rc != OK:
            raise NlteError(rc, "context creation failed (no HIP device?)")
        self.h = h

    def close(self):
        if self.h:
            self.lib.nlte_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc):
        if rc < 0:
            raise NlteError(rc, self.lib.nlte_last_error(self.h).decode())
        return rc

    def voigt(self, precision, n, a_ptr, u_ptr, H_ptr):
        """H(a, u) of the sweeps' line profile at n points (device FP64 arrays)."""
        self.check(self.lib.nlte_voigt(self.h, precision, n, ct.c_void_p(a_ptr), ct.c_void_p(u_ptr),
                                       ct.c_void_p(H_ptr)))

    # ---- inputs
    def atom(self, atom):
        levels = (LevelDesc * len(atom["levels"]))(*[LevelDesc(l["E"], l["g"], l["stage"]) for l in atom["levels"]])
        qs = [_f64(ln["q"]) for ln in atom["lines"]]
        lines = (LineDesc * len(atom["lines"]))(*[
            LineDesc(ln["lower"], ln["upper"], ln["A"], ln["gamma_rad"], ln["gamma_vdw"], len(q),
                     q.ctypes.data_as(ct.POINTER(ct.c_double)))
            for ln, q in zip(atom["lines"], qs)])
        conts = (ContDesc * max(1, len(atom["continua"])))(*[ContDesc(c["lower"], c["upper"], c["alpha0"])
                                                             for c in atom["continua"]])
        colls = (CollDesc * max(1, len(atom["collisions"])))(*[
            CollDesc(c["lower"], c["upper"], c["c_ul"], c["T_ref"], c["beta"]) for c in atom["collisions"]])
        cnu = atom.get("continuum_nu")
        cnu = None if cnu is None else _f64(cnu)
        d = AtomDesc(len(atom["levels"]), len(atom["lines"]), len(atom["continua"]), len(atom["collisions"]),
                     atom["mass_amu"], atom["xi"], atom["epsilon"] or 0.0, levels, lines, conts, colls,
                     0 if cnu is None else cnu.size,
                     None if cnu is None else cnu.ctypes.data_as(ct.POINTER(ct.c_double)))
        h = ct.c_void_p()
        self.check(self.lib.nlte_atom_create(self.h, ct.byref(d), ct.byref(h)))
        return Handle(self, h, self.lib.nlte_atom_destroy)

    def atmos(self, atm):
        z = _f64(atm["z"])
        fields = {k: _f64(atm[k]) for k in ("T", "ne", "nH", "ntot", "vx", "vy", "vz")}
        chi = None if atm.get("chi_c") is None else _f64(atm["chi_c"])
        d = AtmosDesc(atm["nx"], atm["ny"], atm["nz"], atm["dx"], atm["dy"],
                      z.ctypes.data_as(ct.POINTER(ct.c_double)),
                      *[_ptr(fields[k]) for k in ("T", "ne", "nH", "ntot", "vx", "vy", "vz")],
                      _ptr(chi) if chi is not None else None, 0 if chi is None else chi.shape[0], MEM_HOST)
        h = ct.c_void_p()
        self.check(self.lib.nlte_atmos_create(self.h, ct.byref(d), ct.byref(h)))
        return Handle(self, h, self.lib.nlte_atmos_destroy)

    def job(self, atmos_h, atom_h, params: SolveParams):
        j = ct.c_int64()
        p = params.to_c()
        self.check(self.lib.nlte_job_create(self.h, atmos_h.h, atom_h.h, ct.byref(p), ct.byref(j)))
        return Job(self, j.value, params)

    def batch_run(self, jobs):
        """Run created jobs to their stop rules together (shared work-list sweeps); returns
        (status, [Result per job])."""
        ids = (ct.c_int64 * len(jobs))(*[j.id for j in jobs])
        res = (Result * len(jobs))()
        rc = self.check(self.lib.nlte_batch_run(self.h, len(jobs), ids, res))
        return rc, list(res)

    # ---- serving
    def serve_config(self, max_running):
        self.check(self.lib.nlte_serve_config(self.h, int(max_running)))

    def serve_batching(self, batch_max):
        self.check(self.lib.nlte_serve_batching(self.h, int(batch_max)))

    def footprint(self, atmos_h, atom_h, params: SolveParams):
        b = ct.c_size_t()
        p = params.to_c()
        self.check(self.lib.nlte_estimate_footprint(self.h, atmos_h.h, atom_h.h, ct.byref(p), ct.byref(b)))
        return b.value

    def submit(self, atmos_h, atom_h, params: SolveParams):
        """Queue a solve (returns at once); the handles must stay alive until it runs."""
        j = ct.c_int64()
        p = params.to_c()
        self.check(self.lib.nlte_submit(self.h, atmos_h.h, atom_h.h, ct.byref(p), ct.byref(j)))
        job = Job(self, j.value, params)
        job._inputs = (atmos_h, atom_h)
        return job


class Handle:
    def __init__(self, ctx, h, destroy):
        self.ctx, self.h, self._destroy = ctx, h, destroy

    def close(self):
        if self.h and self.ctx.h:
            self._destroy(self.ctx.h, self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Job:
    """A solve in progress: device-resident hierarchy and populations."""

    def __init__(self, ctx, jid, params):
        self.ctx, self.id, self.params = ctx, jid, params
        self.lib = ctx.lib
        self._shape_cache = {}

    def close(self):
        if self.id and self.ctx.h:
            self.lib.nlte_release(self.ctx.h, self.id)
        self.id = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def poll(self):
        st = ct.c_int()
        self.ctx.check(self.lib.nlte_poll(self.ctx.h, self.id, ct.byref(st)))
        return st.value

    def wait(self, timeout_ms=-1):
        return self.lib.nlte_wait(self.ctx.h, self.id, int(timeout_ms))

    def info(self):
        inf = JobInfo()
        self.ctx.check(self.lib.nlte_job_info(self.ctx.h, self.id, ct.byref(inf)))
        return inf

    def run(self):
        r = Result()
        rc = self.ctx.check(self.lib.nlte_job_run(self.ctx.h, self.id, ct.byref(r)))
        return rc, r

    def stats(self):
        """Counters and phase times accumulated so far (also over stage hooks)."""
        r = Result()
        self.ctx.check(self.lib.nlte_job_stats(self.ctx.h, self.id, ct.byref(r)))
        return r

    def populations(self, level, shape):
        out = np.empty(shape, dtype=np.float64)
        self.ctx.check(self.lib.nlte_get_populations(self.ctx.h, self.id, level, _ptr(out), MEM_HOST))
        return out

    def set_populations(self, level, n):
        a = _f64(n)
        self.ctx.check(self.lib.nlte_set_populations(self.ctx.h, self.id, level, _ptr(a), MEM_HOST))

    def source_function(self, shape):
        out = np.empty(shape, dtype=np.float64)
        self.ctx.check(self.lib.nlte_get_source_function(self.ctx.h, self.id, _ptr(out), MEM_HOST))
        return out

    def emergent(self, mus, nf, ny, nx):
        mus = _f64(np.atleast_2d(mus))
        out = np.empty((mus.shape[0], nf, ny, nx), dtype=np.float32)
        self.ctx.check(self.lib.nlte_emergent_intensity(self.ctx.h, self.id, mus.shape[0], _ptr(mus), _ptr(out),
                                                        MEM_HOST))
        return out

    def emergent_continuum(self, mus, nfc, ny, nx):
        mus = _f64(np.atleast_2d(mus))
        out = np.empty((mus.shape[0], nfc, ny, nx), dtype=np.float32)
        self.ctx.check(self.lib.nlte_emergent_continuum_intensity(self.ctx.h, self.id, mus.shape[0], _ptr(mus),
                                                                  _ptr(out), MEM_HOST))
        return out

    def history(self):
        n = self.lib.nlte_history(self.ctx.h, self.id, None, 0)
        out = np.empty(max(n, 0), dtype=np.float64)
        if n > 0:
            self.lib.nlte_history(self.ctx.h, self.id, _ptr(out), n)
        return out

    def formal_solution(self, level, shape):
        dt = np.float64 if self.params.precision == FP64 else np.float32
        j = np.empty(shape, dtype=dt)
        o = np.empty(shape, dtype=dt)
        self.ctx.check(self.lib.nlte_formal_solution(self.ctx.h, self.id, level, _ptr(j), _ptr(o), MEM_HOST))
        return j, o

    def mali(self, level, iters):
        c = ct.c_double()
        self.ctx.check(self.lib.nlte_mali(self.ctx.h, self.id, level, iters, ct.byref(c)))
        return c.value

    def rate_solve(self, level, jeff, oml):
        """One rate solve from given J-bar^eff and 1 - Lambda* (host arrays, rounded to the
        job's precision); returns the maximum relative change."""
        dt = np.float64 if self.params.precision == FP64 else np.float32
        j = np.ascontiguousarray(jeff, dtype=dt)
        o = np.ascontiguousarray(oml, dtype=dt)
        c = ct.c_double()
        self.ctx.check(self.lib.nlte_rate_solve(self.ctx.h, self.id, level, _ptr(j), _ptr(o), MEM_HOST,
                                                ct.byref(c)))
        return c.value

    def residual(self, level, shape):
        out = np.empty(shape, dtype=np.float64)
        self.ctx.check(self.lib.nlte_residual(self.ctx.h, self.id, level, _ptr(out), MEM_HOST))
        return out

    def vcycle(self, level, first=False):
        """One V-cycle on levels level..0; returns the job's repair count so far."""
        rep = ct.c_longlong()
        self.ctx.check(self.lib.nlte_vcycle(self.ctx.h, self.id, level, int(first), ct.byref(rep)))
        return rep.value

    def restrict(self, level, src_ptr, dst_ptr, nq):
        self.ctx.check(self.lib.nlte_restrict(self.ctx.h, self.id, level, nq, ct.c_void_p(src_ptr),
                                              ct.c_void_p(dst_ptr)))

    def prolong(self, level, src_ptr, dst_ptr, nq):
        self.ctx.check(self.lib.nlte_prolong(self.ctx.h, self.id, level, nq, ct.c_void_p(src_ptr),
                                             ct.c_void_p(dst_ptr)))
