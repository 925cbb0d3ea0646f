"""ctypes binding of libmpsim.so (C-ABI in include/mpsim.h).

Argument marshalling only: every step of the evolution runs in the HIP
library. PyTorch supplies the HIP stream and (optionally) its caching
allocator for the library's device buffers. If the library is missing this
module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpsim.so")

# torch bundles its own HIP runtime (same soname, libamdhip64.so.7); loading
# torch first makes the library bind to that runtime instead of starting a
# second one in the same process.
try:
    import torch  # noqa: F401
except ImportError:  # pure C-ABI use without torch
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError("libmpsim.so not built: run `python -m paper_2511_23438_amd.build` "
                      "(or __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------------------
MPS_OK, MPS_E_INVAL, MPS_E_NOMEM, MPS_E_DEVICE = 0, -1, -2, -3
MPS_E_NUMERIC, MPS_E_STATE, MPS_E_UNSUPPORTED = -4, -5, -6
PRECISION = {"fp64": 0, "c64": 1, "bf16x3": 2}
STATUS_NAME = {0: "MPS_OK", -1: "MPS_E_INVAL", -2: "MPS_E_NOMEM", -3: "MPS_E_DEVICE",
               -4: "MPS_E_NUMERIC", -5: "MPS_E_STATE", -6: "MPS_E_UNSUPPORTED"}


class MpsConfig(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("chi_max", C.c_int32),
                ("precision", C.c_int32), ("trotter_order", C.c_int32),
                ("schedule", C.c_int32), ("periodic", C.c_int32), ("eig_path", C.c_int32),
                ("J", C.c_double), ("h", C.c_double), ("dt", C.c_double),
                ("theta0", C.c_double), ("seed", C.c_uint64), ("layers", C.c_int32),
                ("model", C.c_int32), ("eig_batch", C.c_int32)]


class MpsObs(C.Structure):
    _fields_ = [("step", C.c_int32), ("eig_suspect", C.c_int32), ("z", C.c_double),
                ("z2", C.c_double), ("norm", C.c_double), ("fidelity", C.c_double),
                ("log_fidelity", C.c_double), ("z_rescaled", C.c_double),
                ("z2_rescaled", C.c_double), ("gamma", C.c_double), ("min_gap", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for (k, _) in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_int32)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class MpsAllocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


H = C.c_void_p
_sig = {
    "mps_init_product": (C.c_int, [C.POINTER(MpsConfig), C.POINTER(MpsAllocator), C.c_void_p,
                                   C.POINTER(H)]),
    "mps_apply_trotter_step": (C.c_int, [H, C.c_int32]),
    "mps_measure": (C.c_int, [H, C.c_double, C.POINTER(MpsObs)]),
    "mps_fidelity": (C.c_int, [H, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mps_free": (None, [H]),
    "mps_footprint_bytes": (C.c_int, [C.POINTER(MpsConfig), C.POINTER(C.c_size_t)]),
    "mps_schedule_dump": (C.c_int, [C.POINTER(MpsConfig), C.c_int32, C.POINTER(C.c_int32),
                                    C.c_int32, C.POINTER(C.c_int32)]),
    "mps_bond_dims": (C.c_int, [H, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    "mps_site_blocks": (C.c_int, [H, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    "mps_bond_spectrum": (C.c_int, [H, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                    C.POINTER(C.c_int32)]),
    "mps_get_site": (C.c_int, [H, C.c_int32, C.POINTER(C.c_double), C.c_int64,
                               C.POINTER(C.c_int32)]),
    "mps_set_state": (C.c_int, [H, C.POINTER(C.c_int32), C.POINTER(C.POINTER(C.c_double)),
                                C.c_int32]),
    "mps_apply_two_site": (C.c_int, [H, C.c_int32, C.c_int32, C.c_int32]),
    "mps_apply_two_site_toward": (C.c_int, [H, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "mps_apply_single_site": (C.c_int, [H, C.c_int32, C.c_int32]),
    "mps_truncation_log": (C.c_int, [H, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.c_int32, C.POINTER(C.c_int32)]),
    "mps_to_statevector": (C.c_int, [H, C.POINTER(C.c_double), C.c_int64]),
    "mps_apply_trotter_step_batched": (C.c_int, [C.POINTER(H), C.c_int32, C.c_int32]),
    "mps_sync": (C.c_int, [H]),
    "mps_set_progress": (C.c_int, [H, PROGRESS_FN, C.c_void_p]),
    "mps_profile": (C.c_int, [H, C.c_int32]),
    "mps_profile_min_work": (C.c_int, [H, C.c_double]),
    "mps_profile_read": (C.c_int, [H, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]),
    "mps_last_error": (C.c_char_p, [H]),
    "mps_measure_static": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]),
    "mps_debug_check_bounds": (C.c_int, [C.c_int32]),
    "mps_eigh_top": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                               C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.c_void_p]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class MpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAME.get(status, status), msg))
        self.status = status


def _check(st: int, handle=None) -> None:
    if st != MPS_OK:
        msg = _lib.mps_last_error(handle)
        raise MpsError(st, msg.decode() if msg else "")


def make_config(rows: int, cols: int, chi: int, J: float = -1.0, h: float = 2.0,
                dt: float = 0.25, theta0: float = math.pi / 18, order: int = 1,
                precision: str = "fp64", periodic: bool = True, seed: int = 0,
                schedule: int = 1, eig_path: int = 0, layers: int = 0,
                eig_batch: int = 0) -> MpsConfig:
    """rows x cols grid with half-row blocks, or with layers >= 2 the
    rows x cols x layers cube with one qubit per site (schedule 3 or 4).
    schedule: 1 block pairs with routed wrap pairs, 2 rotating rows, 3 route
    and return, 4 gate by gate (rank-2 operators and bond truncations).
    eig_batch: eigenvectors per band inverse-iteration launch (0: 1024)."""
    return MpsConfig(rows, cols, chi, PRECISION[precision], order, schedule,
                     1 if periodic else 0, eig_path, J, h, dt, theta0, seed, layers, 0,
                     eig_batch)


def make_xy_config(rows: int, cols: int, chi: int, g: float = 1.0,
                   dt: float = 0.05 * math.pi, tau: float = 0.06 * math.pi,
                   precision: str = "fp64", seed: int = 0, eig_path: int = 0) -> MpsConfig:
    """XY-model quench (model 1): rows x cols grid, open boundaries, one qubit
    per site, coupling g, step dt, start state of preparation time tau."""
    return MpsConfig(rows, cols, chi, PRECISION[precision], 2, 3, 0, eig_path, g, 0.0, dt,
                     tau, seed, 0, 1, 0)


def config_from_instance(inst, seed: int = 0) -> MpsConfig:
    return make_config(inst.rows, inst.cols, inst.chi, inst.J, inst.h, inst.dt,
                       inst.theta0, inst.order, inst.precision, True, seed,
                       getattr(inst, "schedule", 1), getattr(inst, "eig_path", 0), 0,
                       getattr(inst, "eig_batch", 0))


def footprint_bytes(cfg: MpsConfig) -> int:
    out = C.c_size_t(0)
    _check(_lib.mps_footprint_bytes(C.byref(cfg), C.byref(out)))
    return out.value


def schedule_dump(cfg: MpsConfig, nsteps: int = 1) -> np.ndarray:
    n = C.c_int32(0)
    _lib.mps_schedule_dump(C.byref(cfg), nsteps, None, 0, C.byref(n))
    buf = (C.c_int32 * max(n.value, 1))()
    _check(_lib.mps_schedule_dump(C.byref(cfg), nsteps, buf, n.value, C.byref(n)))
    return np.frombuffer(buf, dtype=np.int32, count=n.value).reshape(-1, 6).copy()


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self):
        import torch
        self.torch = torch
        self.dev = torch.cuda.current_device()

        def _alloc(ctx, nbytes, stream):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.dev,
                                                              int(stream or 0)))
            except Exception:
                return None

        def _free(ctx, ptr, stream):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = MpsAllocator(None, self._a, self._f)


def _current_stream() -> int:
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


class Simulation:
    """One block-MPS instance resident on the GPU (a handle of libmpsim)."""

    def __init__(self, cfg: MpsConfig, stream: Optional[int] = None,
                 torch_allocator: bool = True):
        self.cfg = cfg
        self.stream = _current_stream() if stream is None else int(stream)
        self._alloc = None
        ap = None
        if torch_allocator:
            try:
                import torch
                if torch.cuda.is_available():
                    self._alloc = _TorchAllocator()
                    ap = C.byref(self._alloc.struct)
            except ImportError:
                pass
        self.h = H()
        _check(_lib.mps_init_product(C.byref(cfg), ap, C.c_void_p(self.stream),
                                     C.byref(self.h)))
        if cfg.layers >= 2 or cfg.model == 1:      # cube or XY: one qubit per site
            self.n = cfg.rows * cfg.cols * max(cfg.layers, 1)
            self.N = self.n
        else:                    # grid: two half-row blocks per row
            self.n = cfg.rows * cfg.cols
            self.N = 2 * cfg.rows

    # -- core -------------------------------------------------------------
    def step(self, nsteps: int = 1) -> None:
        _check(_lib.mps_apply_trotter_step(self.h, nsteps), self.h)

    def measure(self, gamma: float = -1.0) -> dict:
        o = MpsObs()
        _check(_lib.mps_measure(self.h, gamma, C.byref(o)), self.h)
        return o.as_dict()

    def fidelity(self) -> tuple[float, float]:
        f, lf = C.c_double(), C.c_double()
        _check(_lib.mps_fidelity(self.h, C.byref(f), C.byref(lf)), self.h)
        return f.value, lf.value

    def sync(self) -> None:
        _check(_lib.mps_sync(self.h), self.h)

    def free(self) -> None:
        if self.h:
            _lib.mps_free(self.h)
            self.h = H()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def set_progress(self, fn) -> None:
        """fn(step, update, updates_per_step) after each two-site update is
        enqueued; None removes it."""
        if fn is None:
            self._progress = None
            _check(_lib.mps_set_progress(self.h, PROGRESS_FN(), None), self.h)
            return
        self._progress = PROGRESS_FN(lambda ctx, s, u, n: fn(s, u, n))
        _check(_lib.mps_set_progress(self.h, self._progress, None), self.h)

    # -- profiling ----------------------------------------------------------
    PROF = {"off": 0, "trd_hemv": 1, "gram": 2, "gemm": 3, "theta": 4}

    def profile(self, kind: str, min_work: float = 0.0) -> None:
        _check(_lib.mps_profile_min_work(self.h, float(min_work)), self.h)
        _check(_lib.mps_profile(self.h, self.PROF[kind]), self.h)

    def profile_read(self) -> tuple[float, int, float]:
        ms, n, w = C.c_double(), C.c_int64(), C.c_double()
        _check(_lib.mps_profile_read(self.h, C.byref(ms), C.byref(n), C.byref(w)), self.h)
        return ms.value, n.value, w.value

    # -- diagnostics --------------------------------------------------------
    def bond_dims(self) -> list[int]:
        buf = (C.c_int32 * (self.N + 1))()
        n = C.c_int32()
        _check(_lib.mps_bond_dims(self.h, buf, self.N + 1, C.byref(n)), self.h)
        return list(buf[:n.value])

    def site_blocks(self) -> list[int]:
        buf = (C.c_int32 * self.N)()
        n = C.c_int32()
        _check(_lib.mps_site_blocks(self.h, buf, self.N, C.byref(n)), self.h)
        return list(buf[:n.value])

    def bond_spectrum(self, bond: int) -> np.ndarray:
        cap = 8192
        buf = (C.c_double * cap)()
        n = C.c_int32()
        _check(_lib.mps_bond_spectrum(self.h, bond, buf, cap, C.byref(n)), self.h)
        return np.array(buf[:n.value])

    def get_site(self, p: int) -> np.ndarray:
        dims = (C.c_int32 * 3)()
        _lib.mps_get_site(self.h, p, None, 0, dims)
        n = dims[0] * dims[1] * dims[2]
        arr = np.zeros(2 * n, dtype=np.float64)
        _check(_lib.mps_get_site(self.h, p, arr.ctypes.data_as(C.POINTER(C.c_double)), n, dims),
               self.h)
        return arr.view(np.complex128).reshape(dims[0], dims[1], dims[2])

    def set_state(self, sites: Sequence[np.ndarray], centre: int) -> None:
        bonds = [1] + [int(a.shape[2]) for a in sites]
        bb = (C.c_int32 * len(bonds))(*bonds)
        keep = [np.ascontiguousarray(a, dtype=np.complex128).reshape(-1).view(np.float64)
                for a in sites]
        ptrs = (C.POINTER(C.c_double) * len(keep))(
            *[k.ctypes.data_as(C.POINTER(C.c_double)) for k in keep])
        _check(_lib.mps_set_state(self.h, bb, ptrs, centre), self.h)

    def apply_two_site(self, site: int, swap: bool, gate: bool, next_site: int = -1) -> None:
        """One two-site update; next_site is the step loop's hint for equal
        sides (a next update left of `site` keeps the centre on `site`)."""
        _check(_lib.mps_apply_two_site_toward(self.h, site, int(swap), int(gate), int(next_site)),
               self.h)

    def apply_single_site(self, site: int, variant: int) -> None:
        """The schedule's single-site gate (variant 0, 1 or 2) on one site."""
        _check(_lib.mps_apply_single_site(self.h, int(site), int(variant)), self.h)

    def truncation_log(self) -> tuple[np.ndarray, np.ndarray]:
        n = C.c_int32()
        _lib.mps_truncation_log(self.h, None, None, 0, C.byref(n))
        f = np.zeros(max(n.value, 1))
        g = np.zeros(max(n.value, 1))
        _check(_lib.mps_truncation_log(self.h, f.ctypes.data_as(C.POINTER(C.c_double)),
                                       g.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                       C.byref(n)), self.h)
        return f[:n.value], g[:n.value]

    def to_statevector(self) -> np.ndarray:
        ln = 1 << self.n
        arr = np.zeros(2 * ln, dtype=np.float64)
        _check(_lib.mps_to_statevector(self.h, arr.ctypes.data_as(C.POINTER(C.c_double)), ln),
               self.h)
        return arr.view(np.complex128)


def eigh_top(G: np.ndarray, q: int, eig_path: int = 1, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """mps_eigh_top: the q largest eigenvalues (descending) of the Hermitian
    n x n matrix G and their eigenvectors (n x q), by the library's
    truncation eigensolver (eig_path 1 one-stage, 2 two-stage)."""
    n = int(G.shape[0])
    g = np.asfortranarray(np.asarray(G, dtype=np.complex128)).reshape(-1, order="F").view(np.float64)
    g = np.ascontiguousarray(g)
    lam = np.zeros(q, dtype=np.float64)
    vecs = np.zeros((n, q), dtype=np.complex128)
    dp = C.POINTER(C.c_double)
    _check(_lib.mps_eigh_top(n, int(q), int(eig_path), int(seed), g.ctypes.data_as(dp),
                             lam.ctypes.data_as(dp), vecs.view(np.float64).ctypes.data_as(dp), None))
    return lam, vecs


def debug_check_bounds(enable: bool) -> None:
    """mps_debug_check_bounds: host-side operand extent checks before the
    library's GEMM, reflector, QR and eigensolver launches (process-wide)."""
    _check(_lib.mps_debug_check_bounds(1 if enable else 0))


def measure_static(bonds: Sequence[int], dims: Sequence[int], site_ptrs: Sequence[int],
                   stream: int, out_ptr: int) -> None:
    """mps_measure_static: the measurement of an MPS held in device memory
    (site_ptrs: device addresses of the row-major (b d) x b' complex128
    sites) with no allocation; out_ptr: device address of 3 doubles
    (<psi|psi>, <Z_tot>/n, <Z_tot^2>/n^2). Asynchronous on `stream`."""
    n = len(dims)
    bb = (C.c_int32 * (n + 1))(*[int(b) for b in bonds])
    dd = (C.c_int32 * n)(*[int(d) for d in dims])
    pp = (C.c_void_p * n)(*[int(p) for p in site_ptrs])
    _check(_lib.mps_measure_static(n, bb, dd, pp, C.c_void_p(int(stream)),
                                   C.c_void_p(int(out_ptr))))


def apply_batched(sims: Sequence[Simulation], nsteps: int = 1) -> None:
    arr = (H * len(sims))(*[s.h for s in sims])
    _check(_lib.mps_apply_trotter_step_batched(arr, len(sims), nsteps))
