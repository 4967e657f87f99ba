"""ctypes binding of the C-ABI library ``libsq_mi355x.so`` (include/sq.h).

Argument marshalling only: every step of the SQ path runs in the HIP
kernels behind the C ABI.  PyTorch provides the device memory (through the
library's allocator callback) and the stream.  If the library is missing the
binding raises -- there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SQ_LIB_PATH") or os.path.join(HERE, "libsq_mi355x.so")

SQ_OK, SQ_E_ARG, SQ_E_ALLOC, SQ_E_DEVICE, SQ_E_BOUNDS, SQ_E_NOCONV, SQ_E_STATE = range(7)
SQ_FP64, SQ_MIXED, SQ_MIXED_STRESS = 0, 1, 2
PRECISIONS = {"fp64": SQ_FP64, "mixed": SQ_MIXED, "mixed_stress": SQ_MIXED_STRESS}
SQ_MU_SOLVE, SQ_MU_FIXED = 0, 1
SQ_INJECT_NARROW, SQ_INJECT_MU_CAP = 1, 2
REC = 24

SPECIES_KEYS = ("v_amp", "v_sigma", "v_rcut", "p_sigma", "p_rcut", "gamma", "z_val")

# Names declared in include/sq.h (kept in step with the header; a CPU test
# checks both directions).
EXPORTS = ("sq_setup", "sq_density", "sq_energy", "sq_stress", "sq_stress_static", "sq_pressure", "sq_xc", "sq_nodes", "sq_bounds",
           "sq_moments", "sq_lanczos", "sq_cell_info", "sq_phase_times", "sq_status_str", "sq_last_error",
           "sq_destroy", "sq_probe_lds")
PHASES = ("lanczos", "bounds", "moments", "mu", "coeffs", "stress", "reduce")


class SqError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d)" % (message, status))
        self.status = status


class SqSpecies(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in SPECIES_KEYS]


class SqCell(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("fd_half_order", ctypes.c_int), ("n_atoms", ctypes.c_int),
                ("pos", ctypes.POINTER(ctypes.c_double)), ("species", ctypes.POINTER(ctypes.c_int)),
                ("n_species", ctypes.c_int), ("sp", ctypes.POINTER(SqSpecies)),
                ("n_electrons", ctypes.c_double), ("rcut", ctypes.c_double),
                ("npl", ctypes.c_int), ("kT", ctypes.c_double), ("mu_mode", ctypes.c_int),
                ("mu", ctypes.c_double), ("lanczos_steps", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class SqOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
                ("outputs_on_device", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("autotune", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("cheb_quad_points", ctypes.c_int), ("persistent", ctypes.c_int),
                ("inject", ctypes.c_int)]


_LIB = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is missing: build it with __graft_entry__.build()"
                           % LIB_PATH)
    # PyTorch's HIP runtime must be the process's only one: its libraries ask
    # for libamdhip64.so by an unversioned name, so if this library loaded the
    # system runtime first a second runtime would be loaded beside it and one
    # of the two would find no device.  Importing torch first makes this
    # library's libamdhip64.so.7 resolve to the runtime torch already holds.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.sq_setup.argtypes = [ctypes.POINTER(SqCell), ctypes.c_int, ctypes.POINTER(SqOptions),
                           ctypes.POINTER(ctypes.c_void_p)]
    L.sq_density.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
    L.sq_energy.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    L.sq_stress.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
    L.sq_stress_static.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
    L.sq_pressure.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
    L.sq_xc.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
    L.sq_nodes.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, ctypes.c_int64, dp]
    L.sq_bounds.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp]
    L.sq_moments.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, ctypes.c_int64, dp]
    L.sq_lanczos.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p, ctypes.c_int64, dp]
    L.sq_cell_info.argtypes = [ctypes.c_void_p, ctypes.c_int, i64p]
    L.sq_phase_times.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, i64p]
    L.sq_status_str.argtypes = [ctypes.c_int]
    L.sq_status_str.restype = ctypes.c_char_p
    L.sq_last_error.argtypes = [ctypes.c_void_p]
    L.sq_last_error.restype = ctypes.c_char_p
    L.sq_destroy.argtypes = [ctypes.c_void_p]
    L.sq_destroy.restype = None
    L.sq_probe_lds.argtypes = [ctypes.c_int, ctypes.c_void_p, dp, dp]
    L.sq_probe_lds.restype = ctypes.c_int
    for name in ("sq_setup", "sq_density", "sq_energy", "sq_stress", "sq_stress_static", "sq_pressure", "sq_xc",
                 "sq_nodes", "sq_bounds",
                 "sq_moments", "sq_lanczos", "sq_cell_info", "sq_phase_times"):
        getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


class _TorchAllocator:
    """Device memory for the plan from PyTorch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.blocks = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:   # out of memory: the library reports SQ_E_ALLOC
            return None
        p = t.data_ptr()
        self.blocks[p] = t
        return p

    def _free(self, ptr, ctx):
        self.blocks.pop(ptr, None)


def _cell_struct(cell: dict, keep: list) -> SqCell:
    pos = np.ascontiguousarray(cell["pos"], dtype=np.float64).reshape(-1, 3)
    sp_idx = np.ascontiguousarray(cell["species"], dtype=np.int32)
    sps = (SqSpecies * len(cell["species_params"]))()
    for i, s in enumerate(cell["species_params"]):
        for k in SPECIES_KEYS:
            setattr(sps[i], k, float(s[k]))
    keep.extend([pos, sp_idx, sps])
    c = SqCell()
    c.L = (ctypes.c_double * 3)(*[float(x) for x in cell["L"]])
    c.h = float(cell["h"])
    c.fd_half_order = int(cell["fd_half_order"])
    c.n_atoms = pos.shape[0]
    c.pos = _dp(pos)
    c.species = sp_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    c.n_species = len(cell["species_params"])
    c.sp = ctypes.cast(sps, ctypes.POINTER(SqSpecies))
    c.n_electrons = float(cell["n_electrons"])
    c.rcut = float(cell["rcut"])
    c.npl = int(cell["npl"])
    c.kT = float(cell["kT"])
    c.mu_mode = SQ_MU_FIXED if cell.get("mu_mode", "solve") == "fixed" else SQ_MU_SOLVE
    c.mu = float(cell.get("mu", 0.0))
    c.lanczos_steps = int(cell.get("lanczos_steps", 20))
    return c


class Plan:
    """One sq_plan over a list of cells (same-name methods as the C ABI)."""

    def __init__(self, cells: Sequence[dict], precision: str = "fp64", stream=None,
                 device: str = "cuda:0", use_torch_memory: bool = True, use_graph: bool = False,
                 autotune: bool = False, tune_cache: Optional[str] = None, cheb_quad_points: int = 0,
                 persistent: bool = False, inject: int = 0):
        import torch
        self.L = load()
        self.cells = list(cells)
        self.torch = torch
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._keep = []
        arr = (SqCell * len(self.cells))()
        for i, c in enumerate(self.cells):
            arr[i] = _cell_struct(c, self._keep)
        opt = SqOptions()
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % ", ".join(PRECISIONS))
        opt.precision = PRECISIONS[precision]
        opt.hip_stream = ctypes.c_void_p(stream.cuda_stream)
        self._alloc = _TorchAllocator(self.device) if use_torch_memory else None
        if self._alloc is not None:
            opt.dev_alloc = self._alloc.alloc_cb
            opt.dev_free = self._alloc.free_cb
        opt.outputs_on_device = 0
        opt.use_graph = int(bool(use_graph))
        opt.autotune = int(bool(autotune))
        self._tune_cache = tune_cache.encode() if tune_cache else None
        opt.tune_cache = self._tune_cache
        opt.cheb_quad_points = int(cheb_quad_points)
        opt.persistent = int(bool(persistent))
        opt.inject = int(inject)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.L.sq_setup(arr, len(self.cells), ctypes.byref(opt), ctypes.byref(handle))
        if st != SQ_OK:
            raise SqError(st, "sq_setup: " + self.L.sq_last_error(None).decode())
        self.h = handle
        self.info = []
        for i in range(len(self.cells)):
            inf = np.zeros(14, dtype=np.int64)
            self._check(self.L.sq_cell_info(self.h, i, _i64(inf)), "sq_cell_info")
            self.info.append(inf)

    # -- helpers -----------------------------------------------------------
    def _check(self, st, what):
        if st != SQ_OK:
            raise SqError(st, "%s: %s" % (what, self.L.sq_last_error(self.h).decode()))

    def _cells(self, cell):
        return list(range(len(self.cells))) if cell == -1 else [cell]

    def n_nodes(self, cell: int) -> int:
        return int(self.info[cell][0])

    # -- entry points --------------------------------------------------------
    def density(self, cell: int = -1):
        idx = self._cells(cell)
        rho = np.zeros(sum(self.n_nodes(i) for i in idx))
        mu = np.zeros(len(idx))
        self._check(self.L.sq_density(self.h, cell, _dp(rho), _dp(mu)), "sq_density")
        out, off = [], 0
        for i in idx:
            out.append(rho[off:off + self.n_nodes(i)])
            off += self.n_nodes(i)
        return out, mu

    def density_only(self, cell: int = -1):
        """sq_density without copying rho (timing); returns mu per cell."""
        mu = np.zeros(len(self._cells(cell)))
        self._check(self.L.sq_density(self.h, cell, None, _dp(mu)), "sq_density")
        return mu

    def energy(self, cell: int = -1) -> np.ndarray:
        e = np.zeros(len(self._cells(cell)))
        self._check(self.L.sq_energy(self.h, cell, _dp(e)), "sq_energy")
        return e

    def stress(self, cell: int = -1):
        n = len(self._cells(cell))
        sig = np.zeros(6 * n)
        parts = np.zeros(18 * n)
        self._check(self.L.sq_stress(self.h, cell, _dp(sig), _dp(parts)), "sq_stress")
        return sig.reshape(n, 6), parts.reshape(n, 18)

    def stress_static(self, cell: int = -1):
        """sq_stress_static: sq_stress with its sums in the library's static
        device scratch (no allocation)."""
        n = len(self._cells(cell))
        sig = np.zeros(6 * n)
        parts = np.zeros(18 * n)
        self._check(self.L.sq_stress_static(self.h, cell, _dp(sig), _dp(parts)), "sq_stress_static")
        return sig.reshape(n, 6), parts.reshape(n, 18)

    def pressure(self, cell: int = -1):
        """(p_direct, p_trace), one value per cell each."""
        n = len(self._cells(cell))
        pd = np.zeros(n)
        pt = np.zeros(n)
        self._check(self.L.sq_pressure(self.h, cell, _dp(pd), _dp(pt)), "sq_pressure")
        return pd, pt

    def xc(self, cell: int = -1):
        """(e_xc, sigma_xc), one value per cell each."""
        n = len(self._cells(cell))
        e = np.zeros(n)
        sg = np.zeros(n)
        self._check(self.L.sq_xc(self.h, cell, _dp(e), _dp(sg)), "sq_xc")
        return e, sg

    def nodes(self, cell: int, nodes: Iterable[int]) -> np.ndarray:
        nd = np.ascontiguousarray(np.asarray(list(nodes), dtype=np.int64))
        out = np.zeros((nd.shape[0], REC))
        self._check(self.L.sq_nodes(self.h, cell, _i64(nd), nd.shape[0], _dp(out)), "sq_nodes")
        return out

    def bounds(self, cell: int):
        n = self.n_nodes(cell)
        lo = np.zeros(n)
        hi = np.zeros(n)
        self._check(self.L.sq_bounds(self.h, cell, _dp(lo), _dp(hi)), "sq_bounds")
        return lo, hi

    def moments(self, cell: int, nodes: Iterable[int]) -> np.ndarray:
        nd = np.ascontiguousarray(np.asarray(list(nodes), dtype=np.int64))
        npl = int(self.info[cell][2])
        out = np.zeros((nd.shape[0], npl + 1))
        self._check(self.L.sq_moments(self.h, cell, _i64(nd), nd.shape[0], _dp(out)), "sq_moments")
        return out

    def lanczos(self, cell: int, nodes: Iterable[int]):
        """(steps, alpha [n, K], beta [n, K]) of the spectral-bound Lanczos."""
        nd = np.ascontiguousarray(np.asarray(list(nodes), dtype=np.int64))
        K = int(self.info[cell][9])   # the step count in effect (0 means 20)
        out = np.zeros((nd.shape[0], 2 * K + 1))
        self._check(self.L.sq_lanczos(self.h, cell, _i64(nd), nd.shape[0], _dp(out)), "sq_lanczos")
        return out[:, 0].astype(int), out[:, 1:K + 1], out[:, K + 1:]

    def phase_times(self, reset: bool = False) -> dict:
        ms = np.zeros(len(PHASES))
        n = np.zeros(len(PHASES), dtype=np.int64)
        self._check(self.L.sq_phase_times(self.h, int(reset), _dp(ms), _i64(n)), "sq_phase_times")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PHASES)}

    def close(self):
        if getattr(self, "h", None):
            self.L.sq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def probe_lds(bytes_per_lane: int = 8, stream=None):
    """Measured conflict-free LDS read bandwidth (TB/s, bytes/clk/CU) of the
    current device (include/sq_probe.h)."""
    import torch
    L = load()
    if stream is None:
        stream = torch.cuda.current_stream()
    tb = ctypes.c_double()
    bpc = ctypes.c_double()
    st = L.sq_probe_lds(int(bytes_per_lane), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(tb),
                        ctypes.byref(bpc))
    if st != 0:
        raise RuntimeError("sq_probe_lds failed with code %d" % st)
    return tb.value, bpc.value


def status_name(st: int) -> str:
    return load().sq_status_str(st).decode()
