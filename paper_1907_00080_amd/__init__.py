"""Python binding of liblbib (MI355X LB-IB capillary solver).

Argument marshalling only: every step of the method runs in the HIP kernels
of liblbib.so, reached through its C ABI (include/lbib.h, lbib_batch.h).
PyTorch provides the device workspace and the HIP stream.  If the library
is not built, constructing a solver raises; there is no other code path.

    sim = Sim(workload, dtype="f32")    # workload: lattice + bodies description
    sim.step(1000)
    rho, ux, uy = sim.fields()
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbib.so")

LBIB_F32, LBIB_F64 = 0, 1
RBC_KINEMATIC, PARTICLE_SOFT, PARTICLE_RIGID = 0, 1, 2
STATUS = {0: "LBIB_OK", 1: "LBIB_EINVAL", 2: "LBIB_ESTATE", 3: "LBIB_EHIP",
          4: "LBIB_ENOSPACE", 5: "LBIB_EUNSTABLE"}
TILES = [(64, 4), (128, 2), (32, 8), (256, 1)]

# symbols the library exports (include/lbib.h and include/lbib_batch.h)
EXPORTS = [
    "lbib_abi_version", "lbib_status_string", "lbib_last_error", "lbib_create",
    "lbib_add_body", "lbib_set_receptors", "lbib_set_adhesion", "lbib_set_repulsion",
    "lbib_set_walls", "lbib_set_transfer",
    "lbib_init_fields",
    "lbib_workspace_query", "lbib_bind", "lbib_finalize_setup", "lbib_step",
    "lbib_set_watchdog", "lbib_set_graph_steps", "lbib_get_fields", "lbib_get_markers",
    "lbib_set_markers", "lbib_get_marker_forces", "lbib_num_ligands", "lbib_get_bonds",
    "lbib_set_bonds", "lbib_get_state", "lbib_set_state", "lbib_diagnostics",
    "lbib_get_step", "lbib_time_lattice_kernel", "lbib_set_kernel_timing",
    "lbib_get_kernel_timing", "lbib_destroy", "lbib_batch_create", "lbib_batch_size",
    "lbib_batch_get_fields", "lbib_batch_get_markers", "lbib_batch_get_bonds",
    "lbib_adjoint_workspace_query", "lbib_adjoint_bind", "lbib_adjoint_forward",
    "lbib_adjoint_backward", "lbib_set_body_params", "lbib_set_step_mode", "lbib_get_step_mode",
    "lbib_observe", "lbib_get_observations", "lbib_reset_observations",
    "lbib_set_cache_hints", "lbib_get_cache_hints", "lbib_set_lattice_launch", "lbib_get_lattice_launch",
    "lbib_set_streaming", "lbib_get_streaming", "lbib_set_watchdog_mass_tolerance",
    "lbib_get_fields_noalloc",
]

REGION_CFL, REGION_INTERMEDIATE, REGION_BULK = 0, 1, 2
TRANSFER_ROMA, TRANSFER_MLS = 0, 1
MLS_WEIGHTS = {"roma": 0, "cubic": 1, "gauss": 2}


class LatticeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("tau", ctypes.c_double), ("gx", ctypes.c_double),
                ("gy", ctypes.c_double), ("seed", ctypes.c_uint64), ("instance", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32)]


class BodyDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nv", ctypes.c_int32), ("ks", ctypes.c_double),
                ("kb", ctypes.c_double), ("ka", ctypes.c_double), ("p_ref", ctypes.c_double),
                ("density_ratio", ctypes.c_double), ("sigma", ctypes.c_double),
                ("ligand_stride", ctypes.c_int32)]


class AdhesionDesc(ctypes.Structure):
    _fields_ = [("y_cr", ctypes.c_double), ("y_eq", ctypes.c_double), ("kf0_dt", ctypes.c_double),
                ("kr0_dt", ctypes.c_double), ("sigma_ts_frac", ctypes.c_double),
                ("kbt", ctypes.c_double), ("freeze_topology", ctypes.c_int32)]


class BodyObs(ctypes.Structure):
    """lbib_body_obs: per-body observables (include/lbib.h)."""
    _fields_ = [("xc", ctypes.c_double), ("yc", ctypes.c_double), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("r_max", ctypes.c_double), ("u_x", ctypes.c_double),
                ("u_y", ctypes.c_double), ("u_x_sum", ctypes.c_double), ("u_y_sum", ctypes.c_double),
                ("region", ctypes.c_int32), ("n_bonds", ctypes.c_int32), ("n_bonds0", ctypes.c_int32),
                ("n_obs", ctypes.c_int32), ("step_obs", ctypes.c_int64)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass", ctypes.c_double), ("mom_x", ctypes.c_double),
                ("mom_y", ctypes.c_double), ("rho_min", ctypes.c_double), ("u_max", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("nbonds", ctypes.c_int32),
                ("bin_overflow", ctypes.c_int32), ("sync_timeouts", ctypes.c_int32)]


class LbibError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib: Optional[ctypes.CDLL] = None


def library() -> ctypes.CDLL:
    """Load liblbib.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblbib.so not found at {LIB_PATH}; build it with "
                          "python -m paper_1907_00080_amd.build")
    # torch ships its own HIP runtime; load it before the library so that the
    # process initialises HIP the way torch expects (loading the library
    # first leaves HIP without a device once torch starts)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "lbib_abi_version": (ctypes.c_uint32, []),
        "lbib_status_string": (ctypes.c_char_p, [I32]),
        "lbib_last_error": (ctypes.c_char_p, [P]),
        "lbib_create": (I32, [ctypes.POINTER(LatticeDesc), ctypes.POINTER(P)]),
        "lbib_add_body": (I32, [P, ctypes.POINTER(BodyDesc), dp, ip]),
        "lbib_set_receptors": (I32, [P, I32, dp, I32]),
        "lbib_set_adhesion": (I32, [P, ctypes.POINTER(AdhesionDesc)]),
        "lbib_set_repulsion": (I32, [P, D, D]),
        "lbib_set_walls": (I32, [P, I32, D, D]),
        "lbib_set_transfer": (I32, [P, I32, I32, D]),
        "lbib_init_fields": (I32, [P, dp, dp, dp]),
        "lbib_workspace_query": (I32, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "lbib_bind": (I32, [P, P, ctypes.c_size_t, P]),
        "lbib_finalize_setup": (I32, [P]),
        "lbib_step": (I32, [P, I64]),
        "lbib_set_watchdog": (I32, [P, I32]),
        "lbib_set_graph_steps": (I32, [P, I32]),
        "lbib_get_fields": (I32, [P, dp, dp, dp]),
        "lbib_get_fields_noalloc": (I32, [P, dp, dp, dp]),
        "lbib_get_markers": (I32, [P, I32, dp]),
        "lbib_set_markers": (I32, [P, I32, dp, dp]),
        "lbib_get_marker_forces": (I32, [P, I32, dp]),
        "lbib_num_ligands": (I32, [P, ip]),
        "lbib_get_bonds": (I32, [P, ip, ip]),
        "lbib_set_bonds": (I32, [P, ip]),
        "lbib_get_state": (I32, [P, P, ctypes.POINTER(ctypes.c_size_t)]),
        "lbib_set_state": (I32, [P, P, ctypes.c_size_t]),
        "lbib_diagnostics": (I32, [P, ctypes.POINTER(Diag)]),
        "lbib_observe": (I32, [P]),
        "lbib_get_observations": (I32, [P, ctypes.POINTER(BodyObs)]),
        "lbib_reset_observations": (I32, [P]),
        "lbib_get_step": (I32, [P, ctypes.POINTER(ctypes.c_int64)]),
        "lbib_time_lattice_kernel": (I32, [P, I32, ctypes.POINTER(ctypes.c_double)]),
        "lbib_set_kernel_timing": (I32, [P, I32]),
        "lbib_get_kernel_timing": (I32, [P, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
        "lbib_destroy": (I32, [P]),
        "lbib_batch_create": (I32, [ctypes.POINTER(P), I32, I32, I32, ctypes.POINTER(P)]),
        "lbib_batch_size": (I32, [P, ip]),
        "lbib_batch_get_fields": (I32, [P, I32, dp, dp, dp]),
        "lbib_batch_get_markers": (I32, [P, I32, I32, dp]),
        "lbib_batch_get_bonds": (I32, [P, I32, ip, ip]),
        "lbib_adjoint_workspace_query": (I32, [P, I64, I32, ctypes.POINTER(ctypes.c_size_t)]),
        "lbib_adjoint_bind": (I32, [P, P, ctypes.c_size_t, I64, I32]),
        "lbib_adjoint_forward": (I32, [P, ctypes.POINTER(ctypes.c_double), ip]),
        "lbib_adjoint_backward": (I32, [P, D, dp]),
        "lbib_set_body_params": (I32, [P, I32, D, D, D]),
        "lbib_set_step_mode": (I32, [P, I32]),
        "lbib_get_step_mode": (I32, [P, ip]),
        "lbib_set_cache_hints": (I32, [P, I32]),
        "lbib_set_lattice_launch": (I32, [P, I32]),
        "lbib_set_streaming": (I32, [P, I32]),
        "lbib_get_streaming": (I32, [P, ip]),
        "lbib_get_lattice_launch": (I32, [P, ip]),
        "lbib_set_watchdog_mass_tolerance": (I32, [P, D]),
        "lbib_get_cache_hints": (I32, [P, ip]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class _Ctx:
    """Owns one lbib_ctx plus its torch workspace."""

    def __init__(self):
        self.lib = library()
        self.h = ctypes.c_void_p()
        self.ws = None
        self.stream = None

    def check(self, st: int, handle=None):
        if st != 0:
            h = self.h if handle is None else handle
            msg = self.lib.lbib_last_error(h).decode()
            raise LbibError(st, msg)

    def bind(self, device, stream, streaming=None):
        import torch
        nb = ctypes.c_size_t()
        self.check(self.lib.lbib_workspace_query(self.h, ctypes.byref(nb)))
        dev = torch.device(device if device is not None else "cuda")
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        if stream is None:
            # a stream of our own (default priority): graph capture is not
            # possible on the legacy default stream
            stream = torch.cuda.Stream(device=dev)
            stream.wait_stream(torch.cuda.current_stream(dev))
        self.stream = stream
        self.check(self.lib.lbib_bind(self.h, ctypes.c_void_p(aligned), nb.value,
                                      ctypes.c_void_p(stream.cuda_stream)))
        if streaming is not None:
            self.check(self.lib.lbib_set_streaming(self.h, int(streaming)))
        self.check(self.lib.lbib_finalize_setup(self.h))
        self.workspace_bytes = nb.value

    # ----------------------------------------------------------- stepping (plain and batch)
    def step(self, n: int = 1):
        self.check(self.lib.lbib_step(self.h, int(n)))

    def set_graph_steps(self, n: int):
        self.check(self.lib.lbib_set_graph_steps(self.h, int(n)))

    def set_step_mode(self, mode: int):
        """0 automatic, 1 three kernels, 2 merged advance, 3 overlapped tiles."""
        self.check(self.lib.lbib_set_step_mode(self.h, int(mode)))

    @property
    def step_mode(self) -> int:
        m = ctypes.c_int32()
        self.check(self.lib.lbib_get_step_mode(self.h, ctypes.byref(m)))
        return m.value

    def set_watchdog(self, on: bool, mass_tolerance: Optional[float] = None):
        """Watchdog after every step call; optional relative mass-drift bound."""
        self.check(self.lib.lbib_set_watchdog(self.h, int(bool(on))))
        if mass_tolerance is not None:
            self.check(self.lib.lbib_set_watchdog_mass_tolerance(self.h, float(mass_tolerance)))

    def set_cache_hints(self, hints: int):
        """Lattice-kernel cache hints: -1 automatic, 0 plain, 1 non-temporal
        loads, 3 non-temporal loads and stores."""
        self.check(self.lib.lbib_set_cache_hints(self.h, int(hints)))

    @property
    def cache_hints(self) -> int:
        m = ctypes.c_int32()
        self.check(self.lib.lbib_get_cache_hints(self.h, ctypes.byref(m)))
        return m.value

    def set_lattice_launch(self, wgs_per_cu: int):
        """Lattice-kernel launch: 0 one workgroup per tile, 1/2/4/8 a
        persistent grid of that many workgroups per CU."""
        self.check(self.lib.lbib_set_lattice_launch(self.h, int(wgs_per_cu)))

    @property
    def lattice_launch(self) -> int:
        m = ctypes.c_int32()
        self.check(self.lib.lbib_get_lattice_launch(self.h, ctypes.byref(m)))
        return m.value

    def set_streaming(self, mode: int):
        """Population streaming: -1 automatic, 0 two buffers, 1 in place."""
        self.check(self.lib.lbib_set_streaming(self.h, int(mode)))

    @property
    def streaming(self) -> int:
        m = ctypes.c_int32()
        self.check(self.lib.lbib_get_streaming(self.h, ctypes.byref(m)))
        return m.value

    def time_lattice_kernel(self, reps: int = 20) -> float:
        """Mean duration (ms) of one fused lattice-kernel launch, HIP events."""
        ms = ctypes.c_double()
        self.check(self.lib.lbib_time_lattice_kernel(self.h, int(reps), ctypes.byref(ms)))
        return ms.value

    def set_kernel_timing(self, on: bool):
        self.check(self.lib.lbib_set_kernel_timing(self.h, int(bool(on))))

    def kernel_timing(self):
        """(mean ms of the in-step fused lattice kernel, launches) since timing was switched on."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self.check(self.lib.lbib_get_kernel_timing(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    @property
    def step_count(self) -> int:
        s = ctypes.c_int64()
        self.check(self.lib.lbib_get_step(self.h, ctypes.byref(s)))
        return s.value

    def diagnostics(self) -> dict:
        d = Diag()
        self.check(self.lib.lbib_diagnostics(self.h, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def n_bodies_total(self) -> int:
        # a Sim keeps one vertex count per body, a Batch one list per instance
        return sum(len(x) if isinstance(x, list) else 1 for x in getattr(self, "nv", []))

    def observe(self):
        """One observation of every body at the current step (on the device)."""
        self.check(self.lib.lbib_observe(self.h))

    def observations(self) -> list:
        """Per-body observation records (dicts, body order)."""
        n = self.n_bodies_total()
        if n == 0:
            return []
        arr = (BodyObs * n)()
        self.check(self.lib.lbib_get_observations(self.h, arr))
        return [{k: getattr(r, k) for k, _ in BodyObs._fields_} for r in arr]

    def reset_observations(self):
        self.check(self.lib.lbib_reset_observations(self.h))

    def close(self):
        if self.h:
            self.lib.lbib_destroy(self.h)
            self.h = ctypes.c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _create(lib, workload, dtype: int, tile) -> ctypes.c_void_p:
    """Create a set-up context from a workload description."""
    d = LatticeDesc(int(workload.nx), int(workload.ny), int(workload.periodic_y), dtype,
                    float(workload.tau), float(workload.gx), float(workload.gy),
                    int(workload.seed) & 0xFFFFFFFFFFFFFFFF, int(getattr(workload, "instance", 0)),
                    int(tile[0]), int(tile[1]))
    h = ctypes.c_void_p()
    st = lib.lbib_create(ctypes.byref(d), ctypes.byref(h))
    if st != 0:
        raise LbibError(st, lib.lbib_last_error(None).decode())

    def chk(s):
        if s != 0:
            msg = lib.lbib_last_error(h).decode()
            lib.lbib_destroy(h)
            raise LbibError(s, msg)

    for b in workload.bodies:
        xy = np.ascontiguousarray(b.xy, dtype=np.float64)
        bd = BodyDesc(int(b.kind), int(xy.shape[0]), float(b.ks), float(b.kb), float(b.ka),
                      float(b.p_ref), float(b.density_ratio), float(b.sigma), int(b.ligand_stride))
        bid = ctypes.c_int32()
        chk(lib.lbib_add_body(h, ctypes.byref(bd), _dptr(xy), ctypes.byref(bid)))
    for w in (0, 1):
        r = np.ascontiguousarray(workload.receptors[w], dtype=np.float64)
        chk(lib.lbib_set_receptors(h, w, _dptr(r) if r.size else None, int(r.size)))
    a = workload.adhesion
    ad = AdhesionDesc(float(a.y_cr), float(a.y_eq), float(a.kf0_dt), float(a.kr0_dt),
                      float(a.sigma_ts_frac), float(a.kbt), int(a.freeze_topology))
    chk(lib.lbib_set_adhesion(h, ctypes.byref(ad)))
    walls = getattr(workload, "walls", "bounce-back")
    if walls not in ("bounce-back", "zou-he"):
        lib.lbib_destroy(h)
        raise ValueError(f"walls must be 'bounce-back' or 'zou-he', got {walls!r}")
    u_lo, u_hi = (float(u) for u in getattr(workload, "u_wall", (0.0, 0.0)))
    if walls == "zou-he" and not workload.periodic_y:
        chk(lib.lbib_set_walls(h, 1, u_lo, u_hi))
    chk(lib.lbib_set_repulsion(h, float(getattr(workload, "repulsion", 0.0)),
                               float(getattr(workload, "repulsion_cutoff", 2.0))))
    transfer = getattr(workload, "transfer", "roma")
    weight = getattr(workload, "mls_weight", "cubic")
    if transfer not in ("roma", "mls") or weight not in MLS_WEIGHTS:
        lib.lbib_destroy(h)
        raise ValueError(f"transfer must be 'roma' or 'mls' and mls_weight one of "
                         f"{sorted(MLS_WEIGHTS)}, got {transfer!r}, {weight!r}")
    if transfer == "mls":
        chk(lib.lbib_set_transfer(h, TRANSFER_MLS, MLS_WEIGHTS[weight],
                                  float(getattr(workload, "mls_support", 1.3))))
    rho = None if workload.rho0 is None else np.ascontiguousarray(workload.rho0, dtype=np.float64)
    ux = uy = None
    if workload.u0 is not None:
        u0 = np.asarray(workload.u0, dtype=np.float64)
        ux = np.ascontiguousarray(u0[0])
        uy = np.ascontiguousarray(u0[1])
    chk(lib.lbib_init_fields(h, _dptr(rho), _dptr(ux), _dptr(uy)))
    return h


def _dtype_code(dtype) -> int:
    if dtype in ("f64", "float64", LBIB_F64):
        return LBIB_F64
    if dtype in ("f32", "float32", LBIB_F32):
        return LBIB_F32
    raise ValueError(f"dtype must be f32 or f64, got {dtype!r}")


class Sim(_Ctx):
    """One capillary lattice with its bodies, advanced on the GPU."""

    def __init__(self, workload, dtype=None, tile=(64, 4), device=None, stream=None,
                 graph_steps: int = 0, watchdog: bool = False, streaming: Optional[int] = None):
        super().__init__()
        code = _dtype_code(dtype if dtype is not None else getattr(workload, "dtype", "f32"))
        self.nx, self.ny = int(workload.nx), int(workload.ny)
        self.nv = [int(np.asarray(b.xy).shape[0]) for b in workload.bodies]
        self.dtype = code
        self.h = _create(self.lib, workload, code, tile)
        self.bind(device, stream, streaming)
        self.check(self.lib.lbib_set_graph_steps(self.h, int(graph_steps)))
        self.check(self.lib.lbib_set_watchdog(self.h, int(bool(watchdog))))
        n = ctypes.c_int32()
        self.check(self.lib.lbib_num_ligands(self.h, ctypes.byref(n)))
        self.n_ligands = n.value

    # ----------------------------------------------------------- readback
    def fields(self):
        N = self.nx * self.ny
        rho, ux, uy = (np.empty(N), np.empty(N), np.empty(N))
        self.check(self.lib.lbib_get_fields(self.h, _dptr(rho), _dptr(ux), _dptr(uy)))
        s = (self.ny, self.nx)
        return rho.reshape(s), ux.reshape(s), uy.reshape(s)

    def markers(self, body: int) -> np.ndarray:
        out = np.empty((self.nv[body], 2))
        self.check(self.lib.lbib_get_markers(self.h, int(body), _dptr(out)))
        return out

    def all_markers(self) -> np.ndarray:
        if not self.nv:
            return np.zeros((0, 2))
        return np.concatenate([self.markers(b) for b in range(len(self.nv))])

    def marker_forces(self, body: int) -> np.ndarray:
        out = np.empty((self.nv[body], 2))
        self.check(self.lib.lbib_get_marker_forces(self.h, int(body), _dptr(out)))
        return out

    def set_markers(self, body: int, xy, xy_prev=None):
        a = np.ascontiguousarray(xy, dtype=np.float64)
        b = None if xy_prev is None else np.ascontiguousarray(xy_prev, dtype=np.float64)
        self.check(self.lib.lbib_set_markers(self.h, int(body), _dptr(a), _dptr(b)))

    def bonds(self) -> np.ndarray:
        out = np.empty(max(self.n_ligands, 1), dtype=np.int32)
        nb = ctypes.c_int32()
        self.check(self.lib.lbib_get_bonds(self.h, _iptr(out), ctypes.byref(nb)))
        return out[: self.n_ligands].copy()

    def set_bonds(self, l2r):
        a = np.ascontiguousarray(l2r, dtype=np.int32)
        self.check(self.lib.lbib_set_bonds(self.h, _iptr(a)))

    def set_body_params(self, body: int, ks: float, kb: float, sigma: float):
        """Strain, bending and bond spring constants of one body."""
        self.check(self.lib.lbib_set_body_params(self.h, int(body), float(ks), float(kb),
                                                 float(sigma)))


    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        self.check(self.lib.lbib_get_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self.check(self.lib.lbib_get_state(self.h, buf, ctypes.byref(n)))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self.check(self.lib.lbib_set_state(self.h, buf, len(blob)))


class Batch(_Ctx):
    """Many independent capillary instances advanced together (parameter sweeps)."""

    def __init__(self, workloads: Sequence, dtype="f32", tile=(64, 4), device=None, stream=None,
                 graph_steps: int = 0, streaming: Optional[int] = None):
        super().__init__()
        code = _dtype_code(dtype)
        self.shapes = [(int(w.nx), int(w.ny)) for w in workloads]
        self.nv = [[int(np.asarray(b.xy).shape[0]) for b in w.bodies] for w in workloads]
        self.n_lig = [sum((int(np.asarray(b.xy).shape[0]) + b.ligand_stride - 1) // b.ligand_stride
                          for b in w.bodies if b.ligand_stride > 0) for w in workloads]
        singles = [_create(self.lib, w, code, tile) for w in workloads]
        try:
            arr = (ctypes.c_void_p * len(singles))(*[s.value for s in singles])
            h = ctypes.c_void_p()
            st = self.lib.lbib_batch_create(arr, len(singles), int(tile[0]), int(tile[1]),
                                            ctypes.byref(h))
            if st != 0:
                raise LbibError(st, self.lib.lbib_last_error(None).decode())
            self.h = h
        finally:
            for s in singles:
                self.lib.lbib_destroy(s)
        self.bind(device, stream, streaming)
        self.check(self.lib.lbib_set_graph_steps(self.h, int(graph_steps)))

    @property
    def n_instances(self) -> int:
        return len(self.shapes)

    @property
    def nodes(self) -> int:
        return sum(nx * ny for nx, ny in self.shapes)

    def fields(self, inst: int):
        nx, ny = self.shapes[inst]
        N = nx * ny
        rho, ux, uy = (np.empty(N), np.empty(N), np.empty(N))
        self.check(self.lib.lbib_batch_get_fields(self.h, int(inst), _dptr(rho), _dptr(ux), _dptr(uy)))
        return rho.reshape(ny, nx), ux.reshape(ny, nx), uy.reshape(ny, nx)

    def markers(self, inst: int, body: int) -> np.ndarray:
        out = np.empty((self.nv[inst][body], 2))
        self.check(self.lib.lbib_batch_get_markers(self.h, int(inst), int(body), _dptr(out)))
        return out

    def bonds(self, inst: int) -> np.ndarray:
        n = self.n_lig[inst]
        out = np.empty(max(n, 1), dtype=np.int32)
        nb = ctypes.c_int32()
        self.check(self.lib.lbib_batch_get_bonds(self.h, int(inst), _iptr(out), ctypes.byref(nb)))
        return out[:n].copy()

