"""FP64 CPU oracle of the two-fluid finite-volume update (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library never loads it
and the two share no code: this wrapper and ``oracle.c`` implement the update
independently from the paper (Eq. (1), Sec. 2.1-2.2; scheme of Sec. 3).

The compiled library ``_oracle.so`` is built by :func:`build` with gcc,
``-O2 -ffp-contract=off`` (no fused multiply-add, no fast-math) and OpenMP over
independent rows/columns.

Parity status of each function is recorded in the design notes: every entry
point here is pinned by the ``-m "not gpu"`` tests against closed forms, the
exact Riemann solution, Rankine-Hugoniot jumps, conservation and symmetry.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
SOURCE = _SRC
_LIB = os.path.join(_HERE, "_oracle.so")

TRANSMISSIVE = 0
PERIODIC = 1
VANLEER = 0
MINMOD = 1


GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", *GCC_FLAGS, "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_variant(src: str, out: str, extra=()) -> str:
    """Compile another copy of the oracle's source (a test's planted mistake,
    or extra flags such as sanitizers) into the shared library `out`; load it
    in a separate process by setting MESO_ORACLE_LIB=out."""
    cmd = ["gcc", *GCC_FLAGS, *extra, "-shared", "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("bc_xlo", C.c_int32), ("bc_xhi", C.c_int32), ("bc_ylo", C.c_int32),
                ("bc_yhi", C.c_int32), ("gamma1", C.c_double), ("pinf1", C.c_double),
                ("gamma2", C.c_double), ("pinf2", C.c_double), ("cfl", C.c_double),
                ("zeps", C.c_double), ("limiter", C.c_int32), ("eos2", C.c_int32),
                ("cc_gamma0", C.c_double), ("cc_A", C.c_double), ("cc_B", C.c_double),
                ("cc_C", C.c_double), ("cc_D", C.c_double), ("cc_rho0", C.c_double),
                ("reactive", C.c_int32), ("pad2_", C.c_int32), ("rx_C", C.c_double),
                ("rx_Ta", C.c_double), ("rx_Q", C.c_double), ("rx_cv2", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("MESO_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = C.CDLL(path)
        P = C.POINTER(_Problem)
        D = C.POINTER(C.c_double)
        I64 = C.POINTER(C.c_int64)
        lib.or_prim_to_cons.argtypes = [P, D, D]
        lib.or_cons_to_prim.argtypes = [P, D, D]
        lib.or_max_speed.argtypes = [P, D]
        lib.or_max_speed.restype = C.c_double
        lib.or_step.argtypes = [P, D, D, C.c_int64, C.c_double]
        lib.or_dt.argtypes = [P, D, C.c_double, C.c_double, D, D]
        lib.or_dt.restype = C.c_int
        lib.or_run.argtypes = [P, D, C.c_int64, C.c_int64, D, C.c_double, D]
        lib.or_run.restype = C.c_int64
        lib.or_step_cells.argtypes = [P, D, C.c_int64, C.c_double, I64, C.c_int64, D]
        lib.or_unit_cons_to_prim.argtypes = [P, D, D, D, D]
        lib.or_unit_limiter.argtypes = [C.c_double, C.c_double, C.c_int32]
        lib.or_unit_limiter.restype = C.c_double
        lib.or_unit_face_states.argtypes = [D, D, D, C.c_double, C.c_double, C.c_double,
                                            C.c_int32, D, D]
        lib.or_unit_hllc.argtypes = [P, D, D, D]
        lib.or_unit_sweep_line.argtypes = [P, C.c_int64, D, D, C.c_double]
        lib.or_num_threads.restype = C.c_int32
        lib.or_set_threads.argtypes = [C.c_int32]
        lib.or_y_averages.argtypes = [P, D, D, D, D]
        lib.or_liquid_temperature.argtypes = [P, C.c_double, C.c_double, C.c_double]
        lib.or_liquid_temperature.restype = C.c_double
        lib.or_unit_cc_reference.argtypes = [P, C.c_double, D]
        lib.or_integrals.argtypes = [P, D, D]
        lib.or_log_edges.argtypes = [C.c_double, C.c_double, C.c_int32, D]
        lib.or_log_histogram.argtypes = [P, D, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                         C.c_double, D]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Problem:
    """Grid, boundaries, materials and scheme options of one solve.

    Phase 1 is the gas (air, ideal gas: pinf1 = 0), phase 2 the liquid.
    """
    nx: int
    ny: int
    dx: float
    dy: float
    gamma1: float = 1.4
    pinf1: float = 0.0
    gamma2: float = 4.4
    pinf2: float = 6.0e8
    cfl: float = 0.4
    zeps: float = 1.0e-6
    limiter: int = VANLEER
    bc_xlo: int = TRANSMISSIVE
    bc_xhi: int = TRANSMISSIVE
    bc_ylo: int = TRANSMISSIVE
    bc_yhi: int = TRANSMISSIVE
    # liquid equation of state: 0 stiffened gas (gamma2, pinf2), 1 Cochran-Chan
    eos2: int = 0
    cc: tuple = (1.19, 0.819e9, 1.51e9, 4.53, 1.42, 1134.0)   # Gamma0, A, B, C, D, rho0
    # reactive liquid (7th plane z2 rho2 lambda): Arrhenius C [1/s], Ta [K], Q [J/kg]
    # (Table 3) and c_v,2 [J/(kg K)] (Table 1); requires eos2 == 1
    reactive: int = 0
    rx: tuple = (2.6e9, 11350.0, 4.46e6, 1714.0)

    @property
    def nplanes(self) -> int:
        return 7 if self.reactive else 6

    def _c(self) -> _Problem:
        return _Problem(self.nx, self.ny, self.dx, self.dy, self.bc_xlo, self.bc_xhi,
                        self.bc_ylo, self.bc_yhi, self.gamma1, self.pinf1, self.gamma2,
                        self.pinf2, self.cfl, self.zeps, self.limiter, self.eos2, *self.cc,
                        self.reactive, 0, *self.rx)


class Oracle:
    """Stateful FP64 solve on the CPU: U holds the 6 conserved planes."""

    def __init__(self, prob: Problem):
        self.prob = prob
        self._p = prob._c()
        self.U = np.zeros((prob.nplanes, prob.ny, prob.nx), dtype=np.float64)
        self.t = 0.0
        self.step = 0
        self.last_dt = 0.0

    # -- state -------------------------------------------------------------
    def set_primitive(self, prim: np.ndarray) -> None:
        """prim: (6, ny, nx) planes z1, rho1, rho2, u, v, p (+ lambda when reactive)."""
        prim = np.ascontiguousarray(prim, dtype=np.float64)
        assert prim.shape == self.U.shape
        _load().or_prim_to_cons(C.byref(self._p), _dp(prim), _dp(self.U))

    def set_conserved(self, U: np.ndarray) -> None:
        self.U[...] = U

    def primitive(self) -> dict:
        out = np.empty((self.prob.nplanes, self.prob.ny, self.prob.nx), dtype=np.float64)
        _load().or_cons_to_prim(C.byref(self._p), _dp(self.U), _dp(out))
        d = dict(rho=out[0], u=out[1], v=out[2], p=out[3], c=out[4], z1=out[5])
        if self.prob.reactive:
            d["lam"] = out[6]
        return d

    # -- time stepping -----------------------------------------------------
    def max_speed(self) -> float:
        return _load().or_max_speed(C.byref(self._p), _dp(self.U))

    def cfl_dt(self, t_end: float = 0.0):
        dt = C.c_double()
        tn = C.c_double()
        rc = _load().or_dt(C.byref(self._p), _dp(self.U), self.t, t_end, C.byref(dt),
                           C.byref(tn))
        if rc != 0:
            raise FloatingPointError("non-finite state or no positive signal speed")
        return dt.value, tn.value

    def step_dt(self, dt: float) -> None:
        """One step with a given dt."""
        tmp = np.empty_like(self.U)
        _load().or_step(C.byref(self._p), _dp(self.U), _dp(tmp), self.step, dt)
        self.step += 1
        self.t += dt
        self.last_dt = dt

    def run(self, nsteps: int, t_end: float = 0.0) -> int:
        t = C.c_double(self.t)
        ldt = C.c_double(self.last_dt)
        n = _load().or_run(C.byref(self._p), _dp(self.U), self.step, nsteps, C.byref(t),
                           t_end, C.byref(ldt))
        if n < 0:
            raise FloatingPointError("oracle: non-finite state")
        self.step += n
        self.t = t.value
        self.last_dt = ldt.value
        return int(n)

    # -- diagnostics (Sec. 4.2, Sec. 4.5) ---------------------------------
    def y_averages(self):
        nx = self.prob.nx
        p, r, u = (np.empty(nx) for _ in range(3))
        _load().or_y_averages(C.byref(self._p), _dp(self.U), _dp(p), _dp(r), _dp(u))
        return p, r, u

    def integrals(self) -> np.ndarray:
        out = np.empty(7)
        _load().or_integrals(C.byref(self._p), _dp(self.U), _dp(out))
        return out[:self.prob.nplanes]

    def log_histogram(self, field: int, lo: float, dn: float, nbins: int, m_ref: float):
        f = np.empty(nbins)
        _load().or_log_histogram(C.byref(self._p), _dp(self.U), field, lo, dn, nbins, m_ref,
                                 _dp(f))
        return f

    def step_cells(self, U: np.ndarray, step: int, dt: float, cells: np.ndarray) -> np.ndarray:
        """Post-step state at flat cell indices j*nx+i, from pre-step state U."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((self.prob.nplanes, cells.size), dtype=np.float64)
        _load().or_step_cells(C.byref(self._p), _dp(U), step, dt,
                              cells.ctypes.data_as(C.POINTER(C.c_int64)), cells.size, _dp(out))
        return out


# -- building blocks for unit pins -----------------------------------------
def unit_cons_to_prim(prob: Problem, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    w = np.empty(6)
    r = C.c_double()
    rc2 = C.c_double()
    _load().or_unit_cons_to_prim(C.byref(prob._c()), _dp(q), _dp(w), C.byref(r), C.byref(rc2))
    return w, r.value, rc2.value


def unit_limiter(a: float, b: float, limiter: int) -> float:
    return _load().or_unit_limiter(a, b, limiter)


def unit_face_states(wm, w0, wp, r, rc2, hl, limiter):
    wm, w0, wp = (np.ascontiguousarray(x, dtype=np.float64) for x in (wm, w0, wp))
    wl = np.empty(6)
    wh = np.empty(6)
    _load().or_unit_face_states(_dp(wm), _dp(w0), _dp(wp), r, rc2, hl, limiter, _dp(wl),
                                _dp(wh))
    return wl, wh


def unit_hllc(prob: Problem, wL, wR) -> np.ndarray:
    wL = np.ascontiguousarray(wL, dtype=np.float64)
    wR = np.ascontiguousarray(wR, dtype=np.float64)
    out = np.empty(8)
    _load().or_unit_hllc(C.byref(prob._c()), _dp(wL), _dp(wR), _dp(out))
    return out[:7]


def unit_sweep_line(prob: Problem, q: np.ndarray, lam: float) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.empty_like(q)
    _load().or_unit_sweep_line(C.byref(prob._c()), q.shape[1], _dp(q), _dp(out), lam)
    return out


def cc_reference(prob: Problem, rho: float):
    """(p_ref, e_ref, rho dp_ref/drho) of the Cochran-Chan liquid at rho."""
    out = np.empty(3)
    _load().or_unit_cc_reference(C.byref(prob._c()), rho, _dp(out))
    return out


def liquid_temperature(prob: Problem, rho2: float, p: float, cv2: float = 1714.0) -> float:
    return _load().or_liquid_temperature(C.byref(prob._c()), rho2, p, cv2)


def log_edges(lo: float, dn: float, nbins: int) -> np.ndarray:
    e = np.empty(nbins + 1)
    _load().or_log_edges(lo, dn, nbins, _dp(e))
    return e


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (n < 1: all
    processors); no result depends on it."""
    _load().or_set_threads(int(n))
