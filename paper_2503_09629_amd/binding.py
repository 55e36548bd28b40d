"""ctypes binding of libsubcyc.so: the C-ABI under the same names.

Argument marshalling only.  Every step of the method runs in the library's
HIP kernels; PyTorch is used for the device arena and the stream.  Loading
fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsubcyc.so")

SC_OK, SC_E_ARG, SC_E_STATE, SC_E_NEST, SC_E_MEM, SC_E_HIP, SC_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
SC_RHS_WAVE, SC_RHS_Z4C = 0, 1
SC_FP64, SC_MIXED = 0, 1
SC_EXEC_PER_BLOCK, SC_EXEC_BATCHED, SC_EXEC_GRAPH = 0, 1, 2
SC_ARR_Y, SC_ARR_K1, SC_ARR_K2, SC_ARR_K3, SC_ARR_K4, SC_ARR_YN = range(6)
SC_FILL_Y1, SC_FILL_Y2, SC_FILL_Y3, SC_FILL_Y4, SC_FILL_END = 1, 2, 3, 4, 5
SC_ABI_VERSION = 3
SC_SUBCYCLED, SC_UNIFORM_DT, SC_BUFFER_ZONES = 0, 1, 2
SC_BC_FROZEN, SC_BC_RADIATIVE = 0, 1
SC_ID_STANDING_WAVE, SC_ID_GAUSSIAN_PULSES, SC_ID_BRILL_LINDQUIST, SC_ID_SPHERICAL_GAUSSIAN = 1, 2, 3, 4

EXPORTED = [
    "sc_config_default", "sc_create", "sc_destroy", "sc_last_error", "sc_build_hierarchy",
    "sc_get_counts", "sc_buffer_count", "sc_export_maps", "sc_device_bytes", "sc_bind_device_memory",
    "sc_set_initial_data", "sc_set_initial_data_analytic", "sc_phys_count", "sc_phys_points", "sc_set_phys_data",
    "sc_hamiltonian", "sc_error_norms", "sc_constraint_norm", "sc_advance", "sc_step_level", "sc_prolongate", "sc_fill_ghosts",
    "sc_restrict", "sc_read_back", "sc_read_rb", "sc_norms", "sc_norms_noalloc", "sc_check_finite",
    "sc_level_time", "sc_set_exec", "sc_poison_halos", "sc_autotune", "sc_tile_shape",
    "sc_set_tile_shape", "sc_profile_enable",
    "sc_profile_read", "sc_stats",
]


class ScConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("rhs", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("exec", ctypes.c_int32),
                ("nghost", ctypes.c_int32), ("time_stepping", ctypes.c_int32),
                ("ko_sigma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("z4c_kappa1", ctypes.c_double), ("z4c_kappa2", ctypes.c_double),
                ("z4c_eta_c", ctypes.c_double), ("z4c_eta_o", ctypes.c_double),
                ("z4c_eta_s", ctypes.c_double), ("fd_order", ctypes.c_int32),
                ("outer_bc", ctypes.c_int32)]


class ScBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int64 * 3), ("hi", ctypes.c_int64 * 3)]


class ScError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"subcyc error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        # PyTorch's HIP runtime must be the one in the process before the
        # library resolves libamdhip64.so.7, so that streams and device
        # pointers from torch are valid in the library.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIBPATH)
        P = ctypes.c_void_p
        i32, i64, f64, u64, sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_size_t)
        sig = {
            "sc_config_default": [P],
            "sc_create": [P, P, P],
            "sc_destroy": [P],
            "sc_build_hierarchy": [P, i32, P, f64, P, P, i32, P, P, u64, i32, i32],
            "sc_get_counts": [P, i32, P, P, P],
            "sc_buffer_count": [P, i32, P],
            "sc_export_maps": [P, P, P],
            "sc_device_bytes": [P, P],
            "sc_bind_device_memory": [P, P, sz],
            "sc_set_initial_data": [P, i32, i32, i32, P, i64],
            "sc_set_initial_data_analytic": [P, i32, P, i32, u64],
            "sc_phys_count": [P, i32, P],
            "sc_phys_points": [P, i32, P, i64],
            "sc_set_phys_data": [P, i32, i32, i32, P, i64],
            "sc_hamiltonian": [P, i32, i32, P, i64],
            "sc_error_norms": [P, i32, i32, i32, i32, P, i32, P],
            "sc_constraint_norm": [P, i32, f64, f64, P],
            "sc_advance": [P, i32],
            "sc_step_level": [P, i32, i32],
            "sc_prolongate": [P, i32],
            "sc_fill_ghosts": [P, i32, i32, i32],
            "sc_restrict": [P, i32],
            "sc_read_back": [P, i32, i32, i32, i32, P, i64],
            "sc_read_rb": [P, i32, i32, i32, i32, i32, P, i64],
            "sc_norms": [P, i32, i32, i32, i32, P],
            "sc_norms_noalloc": [P, i32, i32, i32, i32, P],
            "sc_check_finite": [P],
            "sc_level_time": [P, i32, P],
            "sc_set_exec": [P, i32],
            "sc_poison_halos": [P],
            "sc_autotune": [P, i32],
            "sc_tile_shape": [P, i32, P],
            "sc_set_tile_shape": [P, i32, i32, i32, i32, i32, i32, i32],
            "sc_profile_enable": [P, i32],
            "sc_profile_read": [P, P, P, P],
            "sc_stats": [P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.sc_last_error.argtypes = [P]
        L.sc_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Context:
    """One hierarchy evolved on one GPU stream.

    stream: a torch.cuda.Stream (a default-priority stream is created when
    None and a GPU is present; without a GPU only the host-side calls
    build / counts / export_maps are usable).
    """

    def __init__(self, sigma: float = 0.32, cfl: float = 0.25, exec: int = SC_EXEC_BATCHED,
                 precision: int = SC_FP64, stream=None, device: Optional[str] = None,
                 rhs: int = SC_RHS_WAVE, z4c: Optional[dict] = None,
                 time_stepping: int = SC_SUBCYCLED, fd_order: int = 4,
                 outer_bc: int = SC_BC_FROZEN, ko_order: int = 5):
        self.L = lib()
        cfg = ScConfig()
        self._check(self.L.sc_config_default(ctypes.byref(cfg)), None)
        cfg.time_stepping = time_stepping
        cfg.fd_order = fd_order
        # ghost width: 3 (fourth order), 4 (eighth order), 5 (eighth order with
        # the r = 8 dissipation, ko_order 9)
        cfg.nghost = (5 if ko_order == 9 else 4) if fd_order == 8 else 3
        cfg.outer_bc = outer_bc
        cfg.ko_sigma = sigma
        cfg.cfl = cfl
        cfg.exec = exec
        cfg.precision = precision
        cfg.rhs = rhs
        for k, v in (z4c or {}).items():
            setattr(cfg, "z4c_" + k, v)
        self.nvars = 22 if rhs == SC_RHS_Z4C else 2
        self.torch = None
        self.stream = stream
        handle = None
        if stream is None and device is not None:
            import torch
            self.torch = torch
            self.stream = torch.cuda.Stream(device=device)
        if self.stream is not None:
            handle = ctypes.c_void_p(self.stream.cuda_stream)
        ctx = ctypes.c_void_p()
        rc = self.L.sc_create(ctypes.byref(cfg), handle, ctypes.byref(ctx))
        if rc:
            raise ScError(rc, self.L.sc_last_error(None).decode())
        self.ctx = ctx
        self.arena = None
        self.nlevels = 0
        self.nmembers = 1

    def _check(self, rc, ctx="self"):
        if rc != SC_OK:
            c = self.ctx if ctx == "self" else ctx
            raise ScError(rc, self.L.sc_last_error(c).decode())

    def close(self):
        # sc_destroy waits for the context's queued kernels; only then may the
        # arena go back to torch's allocator
        if getattr(self, "ctx", None):
            self.L.sc_destroy(self.ctx)
            self.ctx = None
        if self.arena is not None and self.stream is not None:
            self.stream.synchronize()
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- hierarchy ------------------------------------------------------------
    def build(self, origin: Sequence[float], dx0: float, ncells0: Sequence[int],
              periodic: Sequence[bool], fine_boxes=(), nmembers: int = 1, block_seed: int = 1,
              min_block: int = 16, max_block: int = 48):
        self.nlevels = 1 + len(fine_boxes)
        self.nmembers = nmembers
        counts = (ctypes.c_int32 * max(1, len(fine_boxes)))(*[len(b) for b in fine_boxes])
        flat = [bx for lev in fine_boxes for bx in lev]
        boxes = (ScBox * max(1, len(flat)))()
        for i, (lo, hi) in enumerate(flat):
            boxes[i].lo[:] = list(lo)
            boxes[i].hi[:] = list(hi)
        o = (ctypes.c_double * 3)(*origin)
        n = (ctypes.c_int64 * 3)(*ncells0)
        p = (ctypes.c_int32 * 3)(*[int(bool(x)) for x in periodic])
        self._check(self.L.sc_build_hierarchy(self.ctx, nmembers, o, float(dx0), n, p,
                                              self.nlevels, counts, boxes,
                                              ctypes.c_uint64(block_seed), min_block, max_block))

    def build_spec(self, spec, **kw):
        """Build from a workloads.HierarchySpec-like object."""
        self.build(spec.origin, spec.dx0, spec.ncells0, spec.periodic, spec.fine_boxes,
                   nmembers=spec.nmembers, **kw)

    def counts(self, level: int):
        nb = ctypes.c_int32()
        no = ctypes.c_int64()
        nr = ctypes.c_int64()
        self._check(self.L.sc_get_counts(self.ctx, level, ctypes.byref(nb), ctypes.byref(no),
                                         ctypes.byref(nr)))
        return nb.value, no.value, nr.value

    def buffer_count(self, level: int) -> int:
        n = ctypes.c_int64()
        self._check(self.L.sc_buffer_count(self.ctx, level, ctypes.byref(n)))
        return n.value

    def export_maps(self) -> np.ndarray:
        n = ctypes.c_int64()
        self._check(self.L.sc_export_maps(self.ctx, None, ctypes.byref(n)))
        out = np.empty(n.value, dtype="<i8")
        self._check(self.L.sc_export_maps(self.ctx, _p(out), ctypes.byref(n)))
        return out

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        self._check(self.L.sc_device_bytes(self.ctx, ctypes.byref(n)))
        return n.value

    def bind(self):
        import torch
        self.torch = torch
        nbytes = self.device_bytes()
        dev = self.stream.device if self.stream is not None else "cuda"
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize(dev)
        ptr = buf.data_ptr()
        aligned = (ptr + 255) & ~255
        self.arena = buf
        self._check(self.L.sc_bind_device_memory(self.ctx, ctypes.c_void_p(aligned), nbytes))

    # -- data -------------------------------------------------------------------
    def set_initial_data(self, member: int, level: int, var: int, values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.L.sc_set_initial_data(self.ctx, member, level, var, _p(a), a.size))

    def set_initial_data_analytic(self, kind: int, params=(), seed: int = 0):
        p = np.ascontiguousarray(params, dtype=np.float64)
        self._check(self.L.sc_set_initial_data_analytic(
            self.ctx, kind, _p(p) if p.size else None, int(p.size), ctypes.c_uint64(seed)))

    def phys_points(self, level: int) -> np.ndarray:
        n = ctypes.c_int64()
        self._check(self.L.sc_phys_count(self.ctx, level, ctypes.byref(n)))
        out = np.empty((n.value, 3))
        if n.value:
            self._check(self.L.sc_phys_points(self.ctx, level, _p(out), n.value))
        return out

    def set_phys_data(self, member: int, level: int, var: int, values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        self._check(self.L.sc_set_phys_data(self.ctx, member, level, var, _p(a), a.size))

    def hamiltonian(self, member: int, level: int) -> np.ndarray:
        n = self.counts(level)[1]
        out = np.empty(n)
        self._check(self.L.sc_hamiltonian(self.ctx, member, level, _p(out), n))
        return out

    def read_back(self, member: int, level: int, var: int, array: int = SC_ARR_Y) -> np.ndarray:
        n = self.counts(level)[1]
        out = np.empty(n)
        self._check(self.L.sc_read_back(self.ctx, member, level, var, array, _p(out), n))
        return out

    def read_rb(self, member: int, level: int, which: int, substep: int, var: int) -> np.ndarray:
        n = self.counts(level)[2]
        out = np.empty(n)
        self._check(self.L.sc_read_rb(self.ctx, member, level, which, substep, var, _p(out), n))
        return out

    def norms(self, member: int, level: int, var: int, array: int = SC_ARR_Y):
        out = np.empty(3)
        self._check(self.L.sc_norms(self.ctx, member, level, var, array, _p(out)))
        return out

    def norms_noalloc(self, member: int, level: int, var: int, array: int = SC_ARR_Y):
        """sc_norms with the library's static workspace (no device allocation)."""
        out = np.empty(3)
        self._check(self.L.sc_norms_noalloc(self.ctx, member, level, var, array, _p(out)))
        return out

    def error_norms(self, member: int, level: int, var: int, kind: int, params):
        """(max |y - exact|, rms, non-finite count) against a closed form at time t."""
        p = np.ascontiguousarray(params, dtype=np.float64)
        out = np.empty(3)
        self._check(self.L.sc_error_norms(self.ctx, member, level, var, kind, _p(p), int(p.size),
                                          _p(out)))
        return out

    def constraint_norm(self, member: int = 0, rmax: float = 30.0, alpha_min: float = 0.3):
        """(composite L2 of H over r < rmax, alpha > alpha_min; max |H| there; non-finite count)."""
        out = np.empty(3)
        self._check(self.L.sc_constraint_norm(self.ctx, member, float(rmax), float(alpha_min),
                                              _p(out)))
        return out

    # -- evolution ----------------------------------------------------------------
    def advance(self, ncoarse: int = 1):
        self._check(self.L.sc_advance(self.ctx, ncoarse))

    def step_level(self, level: int, substep: int = 0):
        self._check(self.L.sc_step_level(self.ctx, level, substep))

    def prolongate(self, fine_level: int):
        self._check(self.L.sc_prolongate(self.ctx, fine_level))

    def fill_ghosts(self, level: int, which: int, substep: int):
        self._check(self.L.sc_fill_ghosts(self.ctx, level, which, substep))

    def restrict(self, fine_level: int):
        self._check(self.L.sc_restrict(self.ctx, fine_level))

    def check_finite(self) -> int:
        return self.L.sc_check_finite(self.ctx)

    def poison_halos(self):
        self._check(self.L.sc_poison_halos(self.ctx))

    def set_exec(self, mode: int):
        self._check(self.L.sc_set_exec(self.ctx, mode))

    def level_time(self, level: int) -> float:
        t = ctypes.c_double()
        self._check(self.L.sc_level_time(self.ctx, level, ctypes.byref(t)))
        return t.value

    def autotune(self, reps: int = 3):
        self._check(self.L.sc_autotune(self.ctx, reps))

    def tile_shape(self, level: int):
        out = (ctypes.c_int32 * 8)()
        self._check(self.L.sc_tile_shape(self.ctx, level, out))
        return dict(zip(("tx", "ty", "tz", "grid", "tiles", "depth", "slots", "threads"), list(out)))

    def set_tile_shape(self, level: int, tz: int, grid: int = 0, depth: int = 1, slots: int = 2,
                       threads: int = 256, tx: int = 0):
        self._check(self.L.sc_set_tile_shape(self.ctx, level, tz, grid, depth, slots, threads,
                                             tx))

    def profile_enable(self, on: bool = True):
        self._check(self.L.sc_profile_enable(self.ctx, int(bool(on))))

    def profile_read(self):
        """(launches, summed kernel ms, summed algorithmic bytes) since enable."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        b = ctypes.c_double()
        self._check(self.L.sc_profile_read(self.ctx, ctypes.byref(n), ctypes.byref(ms),
                                           ctypes.byref(b)))
        return n.value, ms.value, b.value

    def stats(self):
        u = ctypes.c_int64()
        n = ctypes.c_int64()
        self._check(self.L.sc_stats(self.ctx, ctypes.byref(u), ctypes.byref(n)))
        return u.value, n.value

    def synchronize(self):
        if self.stream is not None:
            self.stream.synchronize()
