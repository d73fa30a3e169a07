"""Python binding of the C ABI in include/meso.h (argument marshalling only).

Every step of the solver runs in the HIP library ``libmeso.so``; this module
only converts arguments.  PyTorch supplies the device workspace (a uint8
tensor) and the HIP stream.  If the library is missing, or no HIP device is
present, construction raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmeso.so")

MF_OK = 0
STATUS = {0: "MF_OK", -1: "MF_E_INVALID_ARG", -2: "MF_E_OUT_OF_MEMORY",
          -3: "MF_E_NONFINITE_STATE", -4: "MF_E_CFL_VIOLATION", -5: "MF_E_DEVICE",
          -6: "MF_E_NOT_READY", -7: "MF_E_BUSY"}
PRECISION = {"fp64": 0, "fp32_fp64acc": 1, "mixed": 1, "fp32": 2, "fp64_fast": 3}
LIMITER = {"vanleer": 0, "minmod": 1}
BC = {"transmissive": 0, "periodic": 1}
FIELDS = {"z1rho1": 0, "z2rho2": 1, "rhou": 2, "rhov": 3, "rhoE": 4, "z1": 5,
          "rho": 6, "u": 7, "v": 8, "p": 9, "c": 10,
          # reactive solvers only
          "z2rho2lam": 11, "lam": 12, "T2": 13, "qdot": 14}

# every symbol the header declares
EXPORTS = ["mf_workspace_bytes", "mf_create", "mf_set_primitive", "mf_set_conserved",
           "mf_set_time", "mf_step", "mf_run_steps", "mf_run_to_time", "mf_sync",
           "mf_read_field", "mf_read_conserved", "mf_get_time", "mf_enable_timing",
           "mf_kernel_time", "mf_launch_info", "mf_y_averages", "mf_integrals",
           "mf_log_histogram", "mf_destroy", "mf_status_str", "mf_version",
           "mf_server_request_bytes", "mf_server_create", "mf_server_submit", "mf_server_tick",
           "mf_server_poll", "mf_server_finished", "mf_server_result", "mf_server_drain",
           "mf_server_get_stats",
           "mf_server_destroy", "mf_stream_copy", "mf_integrals_noalloc",
           "mf_record_averages", "mf_recorded_rows", "mf_record_integrals",
           "mf_record_histogram", "mf_recorded_counts"]


class MesoError(RuntimeError):
    def __init__(self, call: str, status: int):
        self.status = status
        super().__init__(f"{call} failed: {STATUS.get(status, status)}")


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("bc_xlo", C.c_int32), ("bc_xhi", C.c_int32), ("bc_ylo", C.c_int32),
                ("bc_yhi", C.c_int32)]


class Material(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reactive", C.c_int32), ("gamma", C.c_double),
                ("p_inf", C.c_double), ("gamma0", C.c_double), ("A", C.c_double),
                ("B", C.c_double), ("C", C.c_double), ("D", C.c_double), ("rho0", C.c_double),
                ("cv", C.c_double), ("arr_C", C.c_double), ("arr_Ta", C.c_double),
                ("heat_Q", C.c_double)]


EOS_STIFFENED, EOS_COCHRAN_CHAN = 0, 1


def stiffened(gamma: float, p_inf: float = 0.0) -> Material:
    """Stiffened gas p = (gamma - 1) rho e - gamma p_inf (air: p_inf = 0)."""
    return Material(EOS_STIFFENED, 0, float(gamma), float(p_inf), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0)


def cochran_chan(gamma0, A, B, C_, D, rho0, rx=None) -> Material:
    """Cochran-Chan liquid (Eqs. (2)-(4)); constants as in Table 1.  rx =
    (C [1/s], Ta [K], Q [J/kg], c_v [J/(kg K)]) makes it reactive (Eq. (6),
    Table 3; temperature of Eq. (5))."""
    m = Material(EOS_COCHRAN_CHAN, 0, 0.0, 0.0, float(gamma0), float(A), float(B),
                 float(C_), float(D), float(rho0), 0, 0, 0, 0)
    if rx is not None:
        m.reactive = 1
        m.arr_C, m.arr_Ta, m.heat_Q, m.cv = (float(v) for v in rx)
    return m


def materials_of(sc) -> "C.Array":
    """(gas, liquid) materials of a scenario."""
    if getattr(sc, "eos2", 0) == 1:
        liquid = cochran_chan(*sc.cc, rx=sc.rx if getattr(sc, "reactive", False) else None)
    else:
        liquid = stiffened(sc.gamma2, sc.pinf2)
    return (Material * 2)(stiffened(sc.gamma1, sc.pinf1), liquid)


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_slots", C.c_int32), ("precision", C.c_int32),
                ("limiter", C.c_int32), ("max_inflight", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("ticks", C.c_int64), ("cell_updates", C.c_int64), ("completed", C.c_int64),
                ("peak_bytes", C.c_int64), ("bytes_in_use", C.c_int64), ("active", C.c_int32),
                ("queued", C.c_int32), ("draining", C.c_int32), ("reserved", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("cfl", C.c_double), ("z_floor", C.c_double), ("limiter", C.c_int32),
                ("precision", C.c_int32), ("fused", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def load_library():
    """Load libmeso.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    I64 = C.POINTER(C.c_int64)
    I32 = C.POINTER(C.c_int32)
    sig = {
        "mf_workspace_bytes": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Material), C.c_int32]),
        "mf_create": (C.c_int32, [C.POINTER(Grid), C.POINTER(Material), C.POINTER(Options),
                                  P, C.c_size_t, P, C.POINTER(P)]),
        "mf_set_primitive": (C.c_int32, [P, D]),
        "mf_set_conserved": (C.c_int32, [P, D]),
        "mf_set_time": (C.c_int32, [P, C.c_double, C.c_int64]),
        "mf_step": (C.c_int32, [P, C.c_double]),
        "mf_run_steps": (C.c_int32, [P, C.c_int64]),
        "mf_run_to_time": (C.c_int32, [P, C.c_double, C.c_int64, I64]),
        "mf_sync": (C.c_int32, [P]),
        "mf_read_field": (C.c_int32, [P, C.c_int32, D, C.c_size_t]),
        "mf_read_conserved": (C.c_int32, [P, D, C.c_size_t]),
        "mf_get_time": (C.c_int32, [P, D, I64, D]),
        "mf_enable_timing": (C.c_int32, [P, C.c_int32]),
        "mf_kernel_time": (C.c_int32, [P, D, I64]),
        "mf_launch_info": (C.c_int32, [P, I64, I32, I32, I32]),
        "mf_y_averages": (C.c_int32, [P, D, D, D, C.c_size_t]),
        "mf_integrals": (C.c_int32, [P, D, C.c_size_t]),
        "mf_integrals_noalloc": (C.c_int32, [P, D, C.c_size_t]),
        "mf_record_averages": (C.c_int32, [P, P, C.c_int64]),
        "mf_recorded_rows": (C.c_int32, [P, I64]),
        "mf_record_integrals": (C.c_int32, [P, P, C.c_int64]),
        "mf_record_histogram": (C.c_int32, [P, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                            C.c_double, P, C.c_int64]),
        "mf_recorded_counts": (C.c_int32, [P, I64]),
        "mf_log_histogram": (C.c_int32, [P, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                         C.c_double, D]),
        "mf_destroy": (C.c_int32, [P]),
        "mf_status_str": (C.c_char_p, [C.c_int32]),
        "mf_server_request_bytes": (C.c_size_t, [C.POINTER(Grid), C.POINTER(Material),
                                                 C.c_int32]),
        "mf_server_create": (C.c_int32, [C.POINTER(ServerConfig), P, C.POINTER(P)]),
        "mf_server_submit": (C.c_int32, [P, C.POINTER(Grid), C.POINTER(Material),
                                         C.POINTER(Options), D, C.c_int64,
                                         C.POINTER(C.c_uint64)]),
        "mf_server_tick": (C.c_int32, [P, I32, I32]),
        "mf_server_poll": (C.c_int32, [P, C.c_uint64, I32]),
        "mf_server_finished": (C.c_int32, [P, C.POINTER(C.c_uint64), C.c_int32, I32]),
        "mf_server_result": (C.c_int32, [P, C.c_uint64, D, C.c_size_t, D, I64]),
        "mf_server_drain": (C.c_int32, [P]),
        "mf_server_get_stats": (C.c_int32, [P, C.POINTER(ServerStats)]),
        "mf_server_destroy": (C.c_int32, [P]),
        "mf_version": (C.c_char_p, []),
        "mf_stream_copy": (C.c_int32, [P, P, C.c_size_t, C.c_int32, C.c_int32, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _chk(call: str, st: int) -> None:
    if st != MF_OK:
        raise MesoError(call, st)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def stream_copy(src_ptr: int, dst_ptr: int, nbytes: int, variant: int = 3, workgroups: int = 0,
                stream: int = 0) -> None:
    """Enqueue the library's plain device copy of `nbytes` bytes (device
    pointers, e.g. ``tensor.data_ptr()``) on `stream` (a hipStream_t handle,
    e.g. ``torch.cuda.current_stream().cuda_stream``)."""
    _chk("mf_stream_copy", load_library().mf_stream_copy(
        C.c_void_p(src_ptr), C.c_void_p(dst_ptr), C.c_size_t(nbytes), int(variant),
        int(workgroups), C.c_void_p(stream)))


def make_grid(nx, ny, dx, dy, bc=("transmissive",) * 4) -> Grid:
    b = [BC[x] if isinstance(x, str) else int(x) for x in bc]
    return Grid(int(nx), int(ny), float(dx), float(dy), *b)


def workspace_bytes(nx, ny, dx=1.0, dy=1.0, precision="fp64", bc=("transmissive",) * 4,
                    mats=None) -> int:
    g = make_grid(nx, ny, dx, dy, bc)
    return int(load_library().mf_workspace_bytes(C.byref(g), mats, PRECISION[precision]))


class Solver:
    """One shock/bubble solve resident on the current HIP device."""

    def __init__(self, nx, ny, dx, dy, *, gamma1=1.4, pinf1=0.0, gamma2=4.4, pinf2=6.0e8,
                 cfl=0.4, z_floor=1e-6, limiter="vanleer", precision="fp64", fused=True,
                 bc=("transmissive",) * 4, workspace="torch", stream=None, liquid=None):
        import torch
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the solver runs only on the GPU")
        self.nx, self.ny = int(nx), int(ny)
        self.precision = precision
        self._lib = lib
        self._grid = make_grid(nx, ny, dx, dy, bc)
        mats = (Material * 2)(stiffened(gamma1, pinf1),
                              liquid if liquid is not None else stiffened(gamma2, pinf2))
        self.nplanes = 7 if mats[1].reactive else 6
        opt = Options(float(cfl), float(z_floor), LIMITER[limiter], PRECISION[precision],
                      1 if fused else 0, 0)
        nbytes = int(lib.mf_workspace_bytes(C.byref(self._grid), mats, PRECISION[precision]))
        if nbytes == 0:
            raise MesoError("mf_workspace_bytes", -1)
        self._ws = None
        ws_ptr = None
        if workspace == "torch":
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            ws_ptr = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _chk("mf_create", lib.mf_create(C.byref(self._grid), mats, C.byref(opt),
                                        ws_ptr, nbytes if ws_ptr else 0,
                                        C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self._h = h

    # ---------------------------------------------------------------- state
    @classmethod
    def from_scenario(cls, sc, precision="fp64", fused=True, **kw):
        s = cls(sc.nx, sc.ny, sc.dx, sc.dy, gamma1=sc.gamma1, pinf1=sc.pinf1, gamma2=sc.gamma2,
                pinf2=sc.pinf2, cfl=sc.cfl, z_floor=sc.zeps, limiter=sc.limiter,
                precision=precision, fused=fused, bc=sc.bc, liquid=materials_of(sc)[1], **kw)
        s.set_primitive(sc.prim)
        return s

    def set_primitive(self, prim: np.ndarray) -> None:
        prim = np.ascontiguousarray(prim, dtype=np.float64)
        assert prim.size == self.nplanes * self.nx * self.ny
        _chk("mf_set_primitive", self._lib.mf_set_primitive(self._h, _dptr(prim)))

    def set_conserved(self, U: np.ndarray) -> None:
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.size == self.nplanes * self.nx * self.ny
        _chk("mf_set_conserved", self._lib.mf_set_conserved(self._h, _dptr(U)))

    def set_time(self, t: float, step: int) -> None:
        _chk("mf_set_time", self._lib.mf_set_time(self._h, float(t), int(step)))

    # ------------------------------------------------------------ stepping
    def step(self, dt: float = 0.0) -> None:
        _chk("mf_step", self._lib.mf_step(self._h, float(dt)))

    def run_steps(self, n: int) -> None:
        _chk("mf_run_steps", self._lib.mf_run_steps(self._h, int(n)))

    def run_to_time(self, t_end: float, max_steps: int = 10 ** 9) -> int:
        taken = C.c_int64()
        _chk("mf_run_to_time", self._lib.mf_run_to_time(self._h, float(t_end), int(max_steps),
                                                         C.byref(taken)))
        return taken.value

    def sync(self) -> None:
        _chk("mf_sync", self._lib.mf_sync(self._h))

    # -------------------------------------------------------------- output
    def read_field(self, name) -> np.ndarray:
        f = FIELDS[name] if isinstance(name, str) else int(name)
        out = np.empty((self.ny, self.nx), dtype=np.float64)
        _chk("mf_read_field", self._lib.mf_read_field(self._h, f, _dptr(out), out.size))
        return out

    def read_conserved(self) -> np.ndarray:
        out = np.empty((self.nplanes, self.ny, self.nx), dtype=np.float64)
        _chk("mf_read_conserved", self._lib.mf_read_conserved(self._h, _dptr(out), out.size))
        return out

    def time(self):
        t = C.c_double()
        n = C.c_int64()
        dt = C.c_double()
        _chk("mf_get_time", self._lib.mf_get_time(self._h, C.byref(t), C.byref(n), C.byref(dt)))
        return t.value, n.value, dt.value

    # --------------------------------------------------------- diagnostics
    def y_averages(self):
        """(p_bar, rho_bar, u_bar) over y, one value per column (Sec. 4.2)."""
        p, r, u = (np.empty(self.nx) for _ in range(3))
        _chk("mf_y_averages", self._lib.mf_y_averages(self._h, _dptr(p), _dptr(r), _dptr(u),
                                                       self.nx))
        return p, r, u

    def integrals(self) -> np.ndarray:
        """Domain integrals of the conserved components and z1 (and the
        remaining reactant mass M_2,r of Eq. (10) for a reactive solver)."""
        out = np.empty(self.nplanes)
        _chk("mf_integrals", self._lib.mf_integrals(self._h, _dptr(out), self.nplanes))
        return out

    def log_histogram(self, field, lo: float, dn: float, nbins: int, m_ref: float):
        f = FIELDS[field] if isinstance(field, str) else int(field)
        out = np.empty(int(nbins))
        _chk("mf_log_histogram", self._lib.mf_log_histogram(self._h, f, float(lo), float(dn),
                                                             int(nbins), float(m_ref),
                                                             _dptr(out)))
        return out

    # -------------------------------------------------------------- timing
    def record_averages(self, rows_ptr: int, max_rows: int) -> None:
        """Record fused transverse averages into device memory at `rows_ptr`
        (e.g. ``torch.empty(max_rows, 3, nx, dtype=float64, device="cuda")
        .data_ptr()``); 0 stops recording."""
        _chk("mf_record_averages", self._lib.mf_record_averages(
            self._h, C.c_void_p(rows_ptr or None), int(max_rows)))

    def recorded_rows(self) -> int:
        n = C.c_int64()
        _chk("mf_recorded_rows", self._lib.mf_recorded_rows(self._h, C.byref(n)))
        return n.value

    def record_integrals(self, rows_ptr: int, max_rows: int) -> None:
        """Record fused domain integrals (rows of `nplanes` + 1 doubles: the
        values of `integrals()`, then the time of the state) into device
        memory at `rows_ptr`; 0 stops."""
        _chk("mf_record_integrals", self._lib.mf_record_integrals(
            self._h, C.c_void_p(rows_ptr or None), int(max_rows)))

    def record_histogram(self, field, lo: float, dn: float, nbins: int, m_ref: float,
                         rows_ptr: int, max_rows: int) -> None:
        """Record the fused mass-weighted PDF of `field` (rows of `nbins`
        doubles, as `log_histogram()`) into device memory at `rows_ptr`;
        rows_ptr 0 stops."""
        f = FIELDS[field] if isinstance(field, str) else int(field)
        _chk("mf_record_histogram", self._lib.mf_record_histogram(
            self._h, f, float(lo), float(dn), int(nbins), float(m_ref),
            C.c_void_p(rows_ptr or None), int(max_rows)))

    def recorded_counts(self):
        """Rows enqueued by the averages, integrals and histogram records."""
        n = (C.c_int64 * 3)()
        _chk("mf_recorded_counts", self._lib.mf_recorded_counts(self._h, n))
        return tuple(int(v) for v in n)

    def enable_timing(self, on: bool = True) -> None:
        _chk("mf_enable_timing", self._lib.mf_enable_timing(self._h, 1 if on else 0))

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_int64()
        _chk("mf_kernel_time", self._lib.mf_kernel_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def launch_info(self) -> dict:
        wg = C.c_int64()
        th, tw, tht = C.c_int32(), C.c_int32(), C.c_int32()
        _chk("mf_launch_info", self._lib.mf_launch_info(self._h, C.byref(wg), C.byref(th),
                                                         C.byref(tw), C.byref(tht)))
        return dict(workgroups=wg.value, threads=th.value, tile_w=tw.value, tile_h=tht.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.mf_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
