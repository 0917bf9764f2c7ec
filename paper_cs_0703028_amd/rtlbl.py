"""Python binding of the C ABI in include/rtlbl.h (argument marshalling only).

Every computation runs in the HIP kernels of ``librtlbl.so``; this module only
converts numpy arrays and torch tensors to pointers and status codes to
exceptions.  PyTorch supplies device memory and streams.  torch is imported
before the library is loaded so that the library binds the same HIP runtime
as torch.

If ``librtlbl.so`` has not been built, importing this module raises
ImportError: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtlbl.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_ESTATE, RT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RT_NO_DEVICE = -1    # rt_create: a host-only handle (argument and call-order checks)
(KAPPA_PLAIN, KAPPA_COMPENSATED, KAPPA_SURROGATE, KAPPA_TABLE16, KAPPA_ADAPTIVE,
 KAPPA_ADAPTIVE_WINGS) = 0, 1, 2, 3, 4, 5
ADAPTIVE_GROUP = 8   # RT_ADAPTIVE_GROUP: cells sharing one line window
TALLY_F32, TALLY_F64 = 0, 1
BATCH_CHUNKED, BATCH_PERSISTENT = 0, 1  # rt_batch_tuning.mode
# rt_arith_op: name -> (code, operands read)
ARITH_OPS = {
    "copy": (0, 1), "add": (1, 2), "sub": (2, 2), "mul": (3, 2), "fma": (4, 3),
    "mul_add": (5, 3), "fma_err": (6, 2), "add_sub": (7, 3), "sub_sub": (8, 3),
    "div": (9, 2), "exp2": (10, 1), "log2": (11, 1), "rcp": (12, 1), "rsq": (13, 1),
    "sqrt": (14, 1),
}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_cs_0703028_amd.build`")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")


class RtStats(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "line_evals", "kappa_ms", "updates", "segments", "trace_ms", "march_ms", "rays",
        "march_launches", "batch_line_evals", "batch_updates", "batch_ms")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class RtCase(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("cell_m", C.c_double),
                ("T_K", C.c_void_p), ("x_h2o", C.c_void_p), ("p_atm", C.c_void_p),
                ("T_wall_K", C.c_double), ("seed", C.c_uint64), ("n_rays", C.c_uint64)]


class BatchTuning(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("chunk_points", "kappa_groups", "march_rays",
                                        "blocks_per_cu", "slots", "mode")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        return cls(**{n: int(d[n]) for n, _ in cls._fields_})


class SurrogateCfg(C.Structure):
    _fields_ = [("n_samples", C.c_int), ("T_K", C.c_void_p), ("x_h2o", C.c_void_p),
                ("p_atm", C.c_void_p), ("T_min", C.c_double), ("T_max", C.c_double),
                ("x_min", C.c_double), ("x_max", C.c_double), ("p_min", C.c_double),
                ("p_max", C.c_double), ("epochs", C.c_int), ("batch", C.c_int),
                ("lr", C.c_float), ("seed", C.c_uint64), ("check_cells", C.c_int),
                ("tolerance", C.c_double)]


class SurrogateStats(C.Structure):
    _fields_ = [("check_error", C.c_double), ("fallback_chunks", C.c_int),
                ("fallback_cells", C.c_int), ("n_chunks", C.c_int), ("infer_ms", C.c_double),
                ("check_ms", C.c_double), ("fallback_ms", C.c_double),
                ("train_loss", C.c_double), ("param_count", C.c_double),
                ("exact_chunks", C.c_int)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _load():
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.rt_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.rt_destroy.argtypes = [vp]
    L.rt_last_error.argtypes = [vp]
    L.rt_last_error.restype = C.c_char_p
    L.rt_setup_grid.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, _f64p, _f64p, _f64p,
                                C.c_double]
    L.rt_setup_lines.argtypes = [vp, C.c_int, _f64p, _f64p, _f64p, _f64p, vp, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.c_int]
    L.rt_required_pitch.argtypes = [vp]
    L.rt_required_pitch.restype = C.c_int64
    L.rt_march_chunk.argtypes = []
    L.rt_march_chunk.restype = C.c_int
    L.rt_compute_kappa.argtypes = [vp, C.c_int, vp, vp, C.c_int64]
    L.rt_set_line_tolerance.argtypes = [vp, C.c_double]
    L.rt_trace_rays.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int]
    L.rt_trace_rays_noalloc.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                        C.c_int]
    L.rt_trace_explicit.argtypes = [vp, C.c_int, _i64p, _i64p, C.c_double, C.c_int, vp]
    L.rt_tally.argtypes = [vp, vp, vp, vp]
    L.rt_reset_tally.argtypes = [vp]
    L.rt_debug_segments.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, _i32p,
                                    _i32p, _f32p, vp, vp]
    L.rt_get_stats.argtypes = [vp, C.POINTER(RtStats)]
    L.rt_batch_default_tuning.argtypes = [C.POINTER(BatchTuning)]
    L.rt_batch_workspace_size.argtypes = [vp, C.c_int, C.POINTER(RtCase), C.POINTER(BatchTuning),
                                          C.POINTER(C.c_int64)]
    L.rt_batch_prepare.argtypes = [vp, C.c_int, C.POINTER(RtCase), C.c_int,
                                   C.POINTER(BatchTuning), vp, C.c_int64]
    L.rt_batch_launch.argtypes = [vp]
    L.rt_batch_results.argtypes = [vp, vp, vp, vp]
    L.rt_batch_run.argtypes = [vp, C.c_int, C.POINTER(RtCase), C.c_int, vp, vp, vp, vp]
    L.rt_batch_autotune.argtypes = [vp, C.c_int, C.POINTER(RtCase), C.c_int, vp, C.c_int64,
                                    C.c_char_p, C.POINTER(BatchTuning)]
    L.rt_surrogate_train.argtypes = [vp, C.POINTER(SurrogateCfg), C.POINTER(C.c_double)]
    L.rt_surrogate_save.argtypes = [vp, C.c_char_p]
    L.rt_surrogate_load.argtypes = [vp, C.c_char_p]
    L.rt_surrogate_forward.argtypes = [vp, C.c_int, _f32p, _f32p]
    L.rt_surrogate_weights.argtypes = [vp, _f32p, C.c_int64]
    L.rt_surrogate_get_stats.argtypes = [vp, C.POINTER(SurrogateStats)]
    L.rt_surrogate_time_phases.argtypes = [vp, C.c_int]
    L.rt_arith_eval.argtypes = [vp, C.c_int, vp, vp, vp, vp, C.c_int64]
    L.rt_setup_gas.argtypes = [vp, C.c_int, vp, C.c_int, vp, vp, vp, vp, vp]
    for f in ("rt_surrogate_train", "rt_surrogate_save", "rt_surrogate_load",
              "rt_surrogate_forward", "rt_surrogate_weights", "rt_surrogate_get_stats",
              "rt_surrogate_time_phases"):
        getattr(L, f).restype = C.c_int
    for f in ("rt_create", "rt_destroy", "rt_setup_grid", "rt_setup_lines", "rt_compute_kappa",
              "rt_trace_rays", "rt_trace_rays_noalloc", "rt_trace_explicit", "rt_tally", "rt_reset_tally",
              "rt_debug_segments", "rt_get_stats", "rt_batch_default_tuning",
              "rt_batch_workspace_size", "rt_batch_prepare", "rt_batch_launch",
              "rt_batch_results", "rt_batch_autotune", "rt_arith_eval", "rt_setup_gas"):
        getattr(L, f).restype = C.c_int
    return L


lib = _load()
MARCH_CHUNK = int(lib.rt_march_chunk())  # nu points per march chunk


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


class Tracer:
    """One rt_ctx handle bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream: "torch.cuda.Stream | None" = None):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        s = lib.rt_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if s != RT_OK:
            raise RtError(s, lib.rt_last_error(None).decode())
        self._h = h
        self.grid = None
        self.lines = None
        self._tables = None

    @classmethod
    def host_only(cls) -> "Tracer":
        """A host-only handle (RT_NO_DEVICE): it checks arguments and the call
        order like a device handle and runs nothing on a device."""
        obj = cls.__new__(cls)
        obj.device = None
        obj.stream = None
        h = C.c_void_p()
        s = lib.rt_create(C.byref(h), RT_NO_DEVICE, None)
        if s != RT_OK:
            raise RtError(s, lib.rt_last_error(None).decode())
        obj._h = h
        obj.grid = None
        obj.lines = None
        obj._tables = None
        obj.gases = {}
        return obj

    # ------------------------------------------------------------ plumbing
    def _check(self, s):
        if s != RT_OK:
            raise RtError(s, lib.rt_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib.rt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------- the ABI
    def setup_grid(self, grid):
        n = grid.nx * grid.ny * grid.nz
        T, x, p = _f64(grid.T), _f64(grid.x), _f64(grid.p)
        if T.size != n or x.size != n or p.size != n:
            raise ValueError("grid arrays must have nx*ny*nz entries")
        self._check(lib.rt_setup_grid(self._h, grid.nx, grid.ny, grid.nz, grid.cell_m, T, x, p,
                                      grid.T_wall))
        self.grid = grid
        self.gases = {}   # the library drops further gases with a new grid

    def setup_lines(self, lines):
        n = len(lines.nu)
        E = None if lines.E_lower is None else _f64(lines.E_lower)
        self._check(lib.rt_setup_lines(self._h, n, _f64(lines.nu), _f64(lines.S),
                                       _f64(lines.gamma), _f64(lines.n_T), _ptr(E), lines.T_ref,
                                       lines.cutoff, lines.nu0, lines.dnu, lines.n_nu))
        self.lines = lines
        self.gases = {}

    def setup_gas(self, gas, g=None):
        """Further gas `gas` (1..3) from an inputs.Gas (mole fraction per cell
        and lines on the first gas's spectral grid); g=None removes it."""
        if g is None:
            self._check(lib.rt_setup_gas(self._h, gas, None, 0, None, None, None, None, None))
            self.gases.pop(gas, None)
            return
        L = g.lines
        n = len(L.nu)
        x = _f64(g.x)
        if x.size != self.grid.nx * self.grid.ny * self.grid.nz:
            raise ValueError("mole fractions must have nx*ny*nz entries")
        E = None if L.E_lower is None else _f64(L.E_lower)
        self._check(lib.rt_setup_gas(self._h, gas, _ptr(x), n, _ptr(_f64(L.nu)), _ptr(_f64(L.S)),
                                     _ptr(_f64(L.gamma)), _ptr(_f64(L.n_T)), _ptr(E)))
        self.gases[gas] = g

    def setup_workload(self, w):
        """setup_grid, setup_lines and every further gas of an inputs.Workload."""
        self.setup_grid(w.grid)
        self.setup_lines(w.lines)
        for k, g in enumerate(w.gases, start=1):
            self.setup_gas(k, g)

    def required_pitch(self) -> int:
        ld = lib.rt_required_pitch(self._h)
        if ld < 0:
            raise RtError(RT_ESTATE, "setup_lines first")
        return int(ld)

    def alloc_tables(self):
        """(kappa, planck) float32 device tensors [n_cells][ld] (caller owned)."""
        ld = self.required_pitch()
        n = self.grid.nx * self.grid.ny * self.grid.nz
        dev = torch.device("cuda", self.device)
        return (torch.empty((n, ld), dtype=torch.float32, device=dev),
                torch.empty((n, ld), dtype=torch.float32, device=dev))

    def set_line_tolerance(self, eps):
        """Tolerance of the adaptive line windows (KAPPA_ADAPTIVE), 0 < eps < 1."""
        self._check(lib.rt_set_line_tolerance(self._h, float(eps)))

    def compute_kappa(self, mode=KAPPA_PLAIN, kappa=None, planck=None):
        """Fills `kappa` (and `planck` when given) on the device.  With no
        kappa buffer, both tables are allocated here.  planck=None with a
        given kappa buffer means no Planck table (the plain march forms its
        Planck values in registers; the precision form needs the table)."""
        if kappa is None:
            kappa, planck = self.alloc_tables()
        for t in (kappa, planck):
            if t is None:
                continue
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
                raise ValueError("tables must be contiguous 2-D float32 device tensors")
        pp = C.c_void_p(planck.data_ptr()) if planck is not None else None
        self._check(lib.rt_compute_kappa(self._h, mode, C.c_void_p(kappa.data_ptr()), pp,
                                         kappa.shape[1]))
        self._tables = (kappa, planck)  # keep the caller's buffers alive
        return kappa, planck

    def trace_rays(self, seed, n_rays_total, begin=0, count=None, prec=TALLY_F32):
        if count is None:
            count = n_rays_total - begin
        self._check(lib.rt_trace_rays(self._h, seed, n_rays_total, begin, count, prec))

    def trace_rays_noalloc(self, seed, n_rays_total, begin=0, count=None, prec=TALLY_F32):
        """rt_trace_rays_noalloc: as trace_rays, with the library's static
        device scratch instead of any allocation."""
        if count is None:
            count = n_rays_total - begin
        self._check(lib.rt_trace_rays_noalloc(self._h, seed, n_rays_total, begin, count, prec))

    def trace_explicit(self, O, D, weight, prec=TALLY_F32, want_exit=False):
        O = np.ascontiguousarray(O, np.int64).reshape(-1, 3)
        D = np.ascontiguousarray(D, np.int64).reshape(-1, 3)
        n = O.shape[0]
        out = np.zeros((n, self.lines.n_nu), np.float64) if want_exit else None
        self._check(lib.rt_trace_explicit(self._h, n, O.ravel(), D.ravel(), weight, prec,
                                          _ptr(out)))
        return out

    def tally(self):
        n = self.grid.nx * self.grid.ny * self.grid.nz
        a = np.zeros(n, np.float64)
        e = np.zeros(n, np.float64)
        b = np.zeros(4, np.float64)
        self._check(lib.rt_tally(self._h, _ptr(a), _ptr(e), _ptr(b)))
        return a, e, b

    def reset_tally(self):
        self._check(lib.rt_reset_tally(self._h))

    def arith_eval(self, op, a, b=None, c=None):
        """rt_arith_eval on 1-D float32 device tensors of one length; returns
        the output tensor (computed on this handle's stream)."""
        code, k = ARITH_OPS[op]
        ins = [a, b, c][:k]
        for t in ins:
            if (t is None or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                    or t.numel() != a.numel()):
                raise ValueError("arith_eval operands: contiguous float32 device tensors of one length")
        out = torch.empty_like(a)
        ptrs = [C.c_void_p(t.data_ptr()) for t in ins] + [None] * (3 - k)
        self._check(lib.rt_arith_eval(self._h, code, *ptrs, C.c_void_p(out.data_ptr()), a.numel()))
        return out

    def debug_segments(self, seed, begin, count):
        g = self.grid
        ms = g.nx + g.ny + g.nz
        counts = np.zeros(count, np.int32)
        cells = np.full((count, ms), -1, np.int32)
        lens = np.zeros((count, ms), np.float32)
        O = np.zeros((count, 3), np.int64)
        D = np.zeros((count, 3), np.int64)
        self._check(lib.rt_debug_segments(self._h, seed, begin, count, ms, counts, cells.ravel(),
                                          lens.ravel(), _ptr(O), _ptr(D)))
        return counts, cells, lens, O, D

    def stats(self):
        s = RtStats()
        self._check(lib.rt_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    # -------------------------------------------------------- batched form
    @staticmethod
    def _cases(workloads):
        keep = []
        arr = (RtCase * len(workloads))()
        for k, w in enumerate(workloads):
            g = w.grid
            T, x, p = _f64(g.T), _f64(g.x), _f64(g.p)
            keep += [T, x, p]
            arr[k] = RtCase(g.nx, g.ny, g.nz, g.cell_m, T.ctypes.data, x.ctypes.data,
                            p.ctypes.data, g.T_wall, w.seed, w.n_rays)
        return arr, keep

    @staticmethod
    def default_tuning():
        t = BatchTuning()
        lib.rt_batch_default_tuning(C.byref(t))
        return t

    def batch_workspace_size(self, workloads, tuning=None):
        arr, keep = self._cases(workloads)
        n = C.c_int64()
        self._check(lib.rt_batch_workspace_size(self._h, len(workloads), arr,
                                                C.byref(tuning) if tuning else None, C.byref(n)))
        return int(n.value)

    def batch_prepare(self, workloads, kappa_mode=KAPPA_PLAIN, tuning=None, workspace=None):
        """Copies the cases into a device workspace (a uint8 tensor, allocated
        here if not given) and builds the launch graph; returns the workspace,
        which must stay alive while the batch is used."""
        nbytes = self.batch_workspace_size(workloads, tuning)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=torch.device("cuda", self.device))
        arr, keep = self._cases(workloads)
        self._check(lib.rt_batch_prepare(self._h, len(workloads), arr, kappa_mode,
                                         C.byref(tuning) if tuning else None,
                                         C.c_void_p(workspace.data_ptr()), workspace.numel()))
        self._batch = ([w.grid.n_cells for w in workloads], workspace)
        return workspace

    def batch_launch(self):
        self._check(lib.rt_batch_launch(self._h))

    def batch_results(self):
        """Per case: (absorbed [cells], emitted [cells], balance [4])."""
        sizes, _ = self._batch
        tot = int(sum(sizes))
        a = np.zeros(tot, np.float64)
        e = np.zeros(tot, np.float64)
        b = np.zeros((len(sizes), 4), np.float64)
        self._check(lib.rt_batch_results(self._h, _ptr(a), _ptr(e), _ptr(b)))
        out, off = [], 0
        for k, n in enumerate(sizes):
            out.append((a[off:off + n], e[off:off + n], b[k]))
            off += n
        return out

    def batch_run(self, workloads, kappa_mode=KAPPA_PLAIN, tuning=None):
        """The batched form in one call (the library allocates and frees the
        workspace).  Per case: (absorbed [cells], emitted [cells], balance [4])."""
        sizes = [w.grid.n_cells for w in workloads]
        tot = int(sum(sizes))
        a = np.zeros(tot, np.float64)
        e = np.zeros(tot, np.float64)
        b = np.zeros((len(sizes), 4), np.float64)
        arr, keep = self._cases(workloads)
        self._check(lib.rt_batch_run(self._h, len(workloads), arr, kappa_mode,
                                     C.byref(tuning) if tuning else None, _ptr(a), _ptr(e), _ptr(b)))
        out, off = [], 0
        for k, n in enumerate(sizes):
            out.append((a[off:off + n], e[off:off + n], b[k]))
            off += n
        return out

    def batch_autotune(self, workloads, kappa_mode=KAPPA_PLAIN, workspace=None, cache_path=None):
        best = BatchTuning()
        arr, keep = self._cases(workloads)
        self._check(lib.rt_batch_autotune(self._h, len(workloads), arr, kappa_mode,
                                          C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                          cache_path.encode() if cache_path else None,
                                          C.byref(best)))
        return best

    # -------------------------------------------------------- learned form
    MLP_DIMS = (4, 512, 512, 512, 256)

    def surrogate_train(self, T, x, p, box, epochs=10, batch=4096, lr=1e-3, seed=0,
                        check_cells=8, tolerance=1e-3):
        """Train the MLP on line-sum spectra of the gas states (T, x, p);
        box = (T_min, T_max, x_min, x_max, p_min, p_max).  Returns the final
        mean squared normalised error."""
        T, x, p = _f64(T), _f64(x), _f64(p)
        cfg = SurrogateCfg(len(T), T.ctypes.data, x.ctypes.data, p.ctypes.data, *box,
                           epochs, batch, lr, seed, check_cells, tolerance)
        loss = C.c_double()
        self._check(lib.rt_surrogate_train(self._h, C.byref(cfg), C.byref(loss)))
        return loss.value

    def surrogate_save(self, path):
        self._check(lib.rt_surrogate_save(self._h, path.encode()))

    def surrogate_load(self, path):
        self._check(lib.rt_surrogate_load(self._h, path.encode()))

    def surrogate_forward(self, inputs):
        inputs = np.ascontiguousarray(inputs, np.float32).reshape(-1, 4)
        out = np.zeros((inputs.shape[0], 256), np.float32)
        self._check(lib.rt_surrogate_forward(self._h, inputs.shape[0], inputs.ravel(),
                                             out.ravel()))
        return out

    def surrogate_weights(self):
        d = self.MLP_DIMS
        n = sum(d[i] * d[i + 1] + d[i + 1] for i in range(4))
        buf = np.zeros(n, np.float32)
        self._check(lib.rt_surrogate_weights(self._h, buf, n))
        out, off = [], 0
        for i in range(4):
            W = buf[off:off + d[i] * d[i + 1]].reshape(d[i], d[i + 1])
            off += d[i] * d[i + 1]
            b = buf[off:off + d[i + 1]]
            off += d[i + 1]
            out.append((W.copy(), b.copy()))
        return out

    def surrogate_time_phases(self, on=True):
        """Timing events between the inference phases (reported by
        surrogate_stats) on or off; off by default, since they cost each
        call several microseconds."""
        self._check(lib.rt_surrogate_time_phases(self._h, 1 if on else 0))

    def surrogate_stats(self):
        st = SurrogateStats()
        self._check(lib.rt_surrogate_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    # ------------------------------------------------------------- helpers
    def raw_status(self, name, *args):
        """Call an rt_* entry point and return its status (error-path tests)."""
        return getattr(lib, name)(self._h, *args)

    def last_error(self) -> str:
        return lib.rt_last_error(self._h).decode()

