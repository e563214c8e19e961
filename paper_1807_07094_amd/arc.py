"""ctypes binding of libarc (include/arc.h). Argument marshalling only: every step of the
ray-tracing and chemistry path runs in the HIP kernels of the library.

Device arrays are passed as torch CUDA tensors (their data pointers); host tables as
numpy arrays. The library must have been built (``python -m paper_1807_07094_amd.build``);
loading fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "libarc.so")
_lib = None

ARC_OK = 0
STATUS = {0: "ARC_OK", -1: "ARC_E_ARG", -2: "ARC_E_RANGE", -3: "ARC_E_NOMEM", -4: "ARC_E_DEVICE",
          -5: "ARC_E_OVERFLOW", -6: "ARC_E_QUEUE", -7: "ARC_E_UNSUPPORTED", -8: "ARC_E_MISMATCH"}
PREC = {"fp32_comp": 0, "fp32_plain": 1}
SCHED = {"plain": 0, "batched": 1, "batched_tuned": 2}
CORR = {"none": 0, "fc": 1, "conserving": 2, "fc_squared": 3}


class ArcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("cell_cm", C.c_double),
                ("y_he", C.c_double), ("n_h", C.c_void_p), ("x_hi", C.c_void_p), ("x_hei", C.c_void_p),
                ("x_heii", C.c_void_p), ("temp", C.c_void_p)]


class Sources(C.Structure):
    _fields_ = [("n", C.c_int32), ("pos", C.c_void_p), ("ndot", C.c_void_p), ("r_thin", C.c_void_p),
                ("r_thin_out", C.c_void_p)]


class Bins(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("frac", C.c_void_p), ("e_erg", C.c_void_p), ("sigma", C.c_void_p),
                ("e_thr", C.c_void_p)]


class TraceParams(C.Structure):
    _fields_ = [("level0", C.c_int32), ("max_level", C.c_int32), ("rays_per_cell", C.c_double),
                ("eps_term", C.c_double), ("precision", C.c_int32), ("schedule", C.c_int32),
                ("stream", C.c_void_p), ("tune_waves", C.c_int32), ("tune_blocks", C.c_int32),
                ("tune_refill", C.c_int32), ("tune_item_level", C.c_int32), ("tree_out", C.c_void_p),
                ("tree_cap", C.c_int64), ("u_j_override", C.c_double), ("graph", C.c_int32),
                ("correction", C.c_int32), ("spill_cap", C.c_int32), ("tune_stack", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("waves", C.c_int32), ("waves_per_cu", C.c_int32), ("refill", C.c_int32),
                ("item_delta", C.c_int32), ("ms_best", C.c_double), ("ms_default", C.c_double),
                ("candidates", C.c_int32), ("stack", C.c_int32)]


class Rates(C.Structure):
    _fields_ = [("gamma", C.c_void_p), ("heat", C.c_void_p)]


class Ledger(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed", C.c_double), ("escaped", C.c_double),
                ("crossings", C.c_uint64), ("rays", C.c_uint64), ("splits", C.c_uint64),
                ("terminated", C.c_uint64), ("escaped_rays", C.c_uint64), ("spills", C.c_uint64),
                ("tree_count", C.c_int64), ("u_j", C.c_double * 4), ("ms_trace", C.c_double),
                ("ms_total", C.c_double), ("ms_kernel", C.c_double), ("absorbed_thin", C.c_double),
                ("deposits", C.c_uint64), ("kernel_crossings", C.c_uint64), ("kernel_deposits", C.c_uint64)]


class ChemParams(C.Structure):
    _fields_ = [("isothermal", C.c_int32), ("rates", C.c_int32), ("collisional", C.c_int32),
                ("alpha_hii", C.c_double), ("eps", C.c_double), ("max_sub", C.c_int32), ("t_floor", C.c_double),
                ("mode", C.c_int32), ("stream", C.c_void_p), ("mlp", C.c_void_p), ("gate_tol", C.c_double),
                ("gate_min_count", C.c_int32), ("graph", C.c_int32)]


class ChemStats(C.Structure):
    _fields_ = [("cells", C.c_int64), ("sub_total", C.c_int64), ("sub_max", C.c_int32), ("capped", C.c_int64),
                ("ms", C.c_double), ("fallback", C.c_int64), ("ms_mlp", C.c_double)]


class TrainParams(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("seed", C.c_uint32),
                ("val_frac", C.c_double), ("stream", C.c_void_p), ("y_he", C.c_double), ("collisional", C.c_int32)]


class TrainReport(C.Structure):
    _fields_ = [("val_rmse_x", C.c_double), ("val_rmse_logt", C.c_double), ("val_max_err", C.c_double),
                ("n_train", C.c_int64), ("n_val", C.c_int64), ("bins_used", C.c_int64), ("ms", C.c_double)]

CHEM_MODE = {"plain": 0, "mlp_gated": 1, "mlp_only": 2}


def lib():
    """Load libarc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"libarc.so not built ({_LIB_PATH}); run python -m paper_1807_07094_amd.build")
        L = C.CDLL(_LIB_PATH)
        L.arc_create.restype = C.c_int32
        L.arc_create.argtypes = [C.c_int32, C.POINTER(C.c_void_p)]
        L.arc_destroy.restype = None
        L.arc_destroy.argtypes = [C.c_void_p]
        L.arc_last_error.restype = C.c_char_p
        L.arc_last_error.argtypes = [C.c_void_p]
        L.arc_trace.restype = C.c_int32
        L.arc_trace.argtypes = [C.c_void_p, C.POINTER(Grid), C.POINTER(Sources), C.POINTER(Bins), C.c_double,
                                C.POINTER(TraceParams), C.POINTER(Rates), C.POINTER(Ledger)]
        L.arc_autotune.restype = C.c_int32
        L.arc_autotune.argtypes = [C.c_void_p, C.POINTER(Grid), C.POINTER(Sources), C.POINTER(Bins), C.c_double,
                                   C.POINTER(TraceParams), C.POINTER(Rates), C.POINTER(TuneResult)]
        L.arc_get_field.restype = C.c_int32
        L.arc_get_field.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.arc_probe_requests.restype = C.c_int32
        L.arc_probe_requests.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_uint64, C.c_void_p,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.arc_healpix_dirs.restype = C.c_int32
        L.arc_healpix_dirs.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.arc_chem_step.restype = C.c_int32
        L.arc_chem_step.argtypes = [C.c_void_p, C.POINTER(Grid), C.POINTER(Rates), C.c_double,
                                    C.POINTER(ChemParams), C.POINTER(ChemStats)]
        L.arc_rt_timestep.restype = C.c_int32
        L.arc_rt_timestep.argtypes = [C.c_void_p, C.POINTER(Grid), C.POINTER(Rates), C.POINTER(Bins),
                                      C.POINTER(ChemParams), C.c_double, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.arc_rt_timestep_noalloc.restype = C.c_int32
        L.arc_rt_timestep_noalloc.argtypes = [C.c_void_p, C.POINTER(Grid), C.POINTER(Rates), C.POINTER(Bins),
                                              C.POINTER(ChemParams), C.c_double, C.c_void_p]
        L.arc_mlp_create.restype = C.c_int32
        L.arc_mlp_create.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
        L.arc_mlp_destroy.restype = None
        L.arc_mlp_destroy.argtypes = [C.c_void_p]
        L.arc_mlp_train.restype = C.c_int32
        L.arc_mlp_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.POINTER(TrainParams), C.POINTER(TrainReport)]
        L.arc_mlp_save.restype = C.c_int32
        L.arc_mlp_save.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]
        L.arc_mlp_load.restype = C.c_int32
        L.arc_mlp_load.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.arc_mlp_predict.restype = C.c_int32
        L.arc_mlp_predict.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("device arrays must be contiguous")
        return C.c_void_p(t.data_ptr())
    return t.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def device_grid(grid: dict, device="cuda"):
    """Copy a workload grid (numpy float32 arrays) to the device as torch tensors."""
    import torch

    out = {k: torch.from_numpy(np.ascontiguousarray(grid[k], np.float32)).to(device)
           for k in ("n_h", "x_hi", "x_hei", "x_heii", "temp") if k in grid}
    out["cell_cm"] = float(grid["cell_cm"])
    out["y_he"] = float(grid["y_he"])
    return out


def _grid(g) -> Grid:
    nz, ny, nx = g["n_h"].shape
    for k in ("n_h", "x_hi", "x_hei", "x_heii", "temp"):
        if k in g and tuple(g[k].shape) != (nz, ny, nx):
            raise ValueError(f"grid array {k} has shape {tuple(g[k].shape)}, expected {(nz, ny, nx)}")
    return Grid(nx, ny, nz, float(g["cell_cm"]), float(g["y_he"]), _ptr(g["n_h"]), _ptr(g["x_hi"]),
                _ptr(g["x_hei"]), _ptr(g["x_heii"]), _ptr(g.get("temp")))


class Context:
    """An arc_ctx: owns the library's device buffers on one GPU."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        rc = lib().arc_create(device, C.byref(h))
        if rc != ARC_OK:
            raise ArcError(rc, "arc_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().arc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != ARC_OK:
            raise ArcError(rc, lib().arc_last_error(self._h).decode())

    @staticmethod
    def _trace_args(grid, sources, bins, level0, rays_per_cell, max_level, eps_term, precision, schedule, stream,
                    tree, tune_waves, tune_blocks, tune_refill, tune_item_level, u_j_override, graph, correction=0,
                    spill_cap=0, tune_stack=0):
        g = _grid(grid)
        pos = np.ascontiguousarray(sources["pos"], np.float64).reshape(-1, 3)
        ndot = np.ascontiguousarray(sources["ndot"], np.float64).reshape(-1)
        # optically thin approximation (section 2.6): radii in, measured radii out (written in
        # place into sources["r_thin_out"], a float64 array of one entry per source)
        r_thin = sources.get("r_thin")
        r_thin = np.ascontiguousarray(r_thin, np.float64).reshape(-1) if r_thin is not None else None
        r_out = sources.get("r_thin_out")
        if r_thin is not None and r_thin.size != ndot.size:
            raise ValueError("r_thin needs one radius per source")
        if r_out is not None and (not isinstance(r_out, np.ndarray) or r_out.dtype != np.float64 or
                                  r_out.size != ndot.size or not r_out.flags.c_contiguous):
            raise ValueError("r_thin_out must be a contiguous float64 array with one entry per source")
        frac = np.ascontiguousarray(bins["frac"], np.float64)
        e = np.ascontiguousarray(bins["e_erg"], np.float64)
        sig = np.ascontiguousarray(bins["sigma"], np.float64).reshape(-1, 3)
        thr = np.ascontiguousarray(bins["e_thr"], np.float64)
        s = Sources(ndot.size, _ptr(pos), _ptr(ndot), _ptr(r_thin), _ptr(r_out))
        b = Bins(frac.size, _ptr(frac), _ptr(e), _ptr(sig), _ptr(thr))
        p = TraceParams(int(level0), int(max_level), float(rays_per_cell), float(eps_term),
                        PREC[precision] if isinstance(precision, str) else int(precision),
                        SCHED[schedule] if isinstance(schedule, str) else int(schedule), _stream(stream),
                        int(tune_waves), int(tune_blocks), int(tune_refill), int(tune_item_level), _ptr(tree),
                        int(tree.numel()) if tree is not None else 0, float(u_j_override), int(bool(graph)),
                        CORR[correction] if isinstance(correction, str) else int(correction), int(spill_cap),
                        int(tune_stack))
        # the host arrays must outlive the call: keep them with the structures
        return g, s, b, p, (pos, ndot, frac, e, sig, thr, r_thin, r_out)

    def trace(self, grid, sources: dict, bins: dict, dt: float, gamma, heat, level0=1, rays_per_cell=4.0,
              max_level=-1, eps_term=1e-6, precision="fp32_comp", schedule="batched", stream=None, tree=None,
              tune_waves=0, tune_blocks=0, tune_refill=0, tune_item_level=0, u_j_override=0.0, graph=False,
              correction="none", spill_cap=0, tune_stack=0) -> dict:
        """arc_trace. gamma/heat: device float32 tensors of shape [3, nz, ny, nx]. correction:
        "none", "fc", "conserving" or "fc_squared" (section 2.5). sources may carry "r_thin" and
        "r_thin_out" (section 2.6)."""
        g, s, b, p, _keep = self._trace_args(grid, sources, bins, level0, rays_per_cell, max_level, eps_term,
                                             precision, schedule, stream, tree, tune_waves, tune_blocks, tune_refill,
                                             tune_item_level, u_j_override, graph, correction, spill_cap,
                                             tune_stack)
        r = Rates(_ptr(gamma), _ptr(heat))
        led = Ledger()
        self._check(lib().arc_trace(self._h, C.byref(g), C.byref(s), C.byref(b), float(dt), C.byref(p),
                                    C.byref(r), C.byref(led)))
        out = {k: getattr(led, k) for k, _ in Ledger._fields_ if k != "u_j"}
        out["u_j"] = list(led.u_j)
        return out

    def autotune(self, grid, sources: dict, bins: dict, dt: float, gamma, heat, level0=1, rays_per_cell=4.0,
                 max_level=-1, eps_term=1e-6, precision="fp32_comp", stream=None) -> dict:
        """arc_autotune on these sources; the chosen shape is cached in the context for
        schedule="batched_tuned"."""
        g, s, b, p, _keep = self._trace_args(grid, sources, bins, level0, rays_per_cell, max_level, eps_term,
                                             precision, "batched", stream, None, 0, 0, 0, 0, 0.0, False)
        r = Rates(_ptr(gamma), _ptr(heat))
        res = TuneResult()
        self._check(lib().arc_autotune(self._h, C.byref(g), C.byref(s), C.byref(b), float(dt), C.byref(p),
                                       C.byref(r), C.byref(res)))
        return {k: getattr(res, k) for k, _ in TuneResult._fields_}

    def get_field(self, dst, stream=None):
        """arc_get_field into a device int64 tensor of nbins * ncell entries (3 * nbins * ncell
        after a trace with the conserving correction: the field, then the moved-photon field's
        low and high limbs)."""
        self._check(lib().arc_get_field(self._h, _ptr(dst), int(dst.numel()), _stream(stream)))
        return dst

    def probe_requests(self, items: int = 1 << 27, cells: int = 0, seed: int = 1, stream=None):
        """arc_probe_requests: (deposits/s, gathers/s) of random cells (among the first `cells`
        of the blocked layout, 0 = all) on the last trace's buffers (overwrites its field)."""
        d, g = C.c_double(0), C.c_double(0)
        self._check(lib().arc_probe_requests(self._h, int(items), int(cells), int(seed), _stream(stream), C.byref(d),
                                             C.byref(g)))
        return d.value, g.value

    def healpix_dirs(self, level: int, dst, stream=None):
        self._check(lib().arc_healpix_dirs(self._h, int(level), _ptr(dst), _stream(stream)))
        return dst

    def chem_step(self, grid, gamma, heat, dt: float, isothermal=0, rates=1, collisional=1, alpha_hii=2.59e-13,
                  eps=0.1, max_sub=100000, t_floor=1.0, mode="plain", stream=None, mlp=None, gate_tol=1e-3,
                  gate_min_count=16, graph=False) -> dict:
        g = _grid(grid)
        r = Rates(_ptr(gamma), _ptr(heat))
        p = ChemParams(int(isothermal), int(rates), int(collisional), float(alpha_hii), float(eps), int(max_sub),
                       float(t_floor), CHEM_MODE[mode] if isinstance(mode, str) else int(mode), _stream(stream),
                       mlp._h if mlp is not None else None, float(gate_tol), int(gate_min_count), int(bool(graph)))
        st = ChemStats()
        self._check(lib().arc_chem_step(self._h, C.byref(g), C.byref(r), float(dt), C.byref(p), C.byref(st)))
        return {k: getattr(st, k) for k, _ in ChemStats._fields_}

    def rt_timestep(self, grid, gamma, bins: dict, eps=0.1, rates=1, collisional=1, alpha_hii=2.59e-13,
                    stream=None):
        """arc_rt_timestep (section 2.9): (dt_n, dt_I) in seconds from the grid's state and the
        photoionisation rates gamma [3, nz, ny, nx] of the last trace."""
        g = _grid(grid)
        r = Rates(_ptr(gamma), 0)
        b, _keep = _bins_struct(bins)
        p = ChemParams(0, int(rates), int(collisional), float(alpha_hii), 0.1, 1, 1.0, 0, _stream(stream), None,
                       0.0, 0, 0)
        dn, di = C.c_double(0), C.c_double(0)
        self._check(lib().arc_rt_timestep(self._h, C.byref(g), C.byref(r), C.byref(b), C.byref(p), float(eps),
                                          C.byref(dn), C.byref(di)))
        return dn.value, di.value


    def rt_timestep_noalloc(self, grid, gamma, bins: dict, dt_out, eps=0.1, rates=1, collisional=1,
                            alpha_hii=2.59e-13, stream=None):
        """arc_rt_timestep_noalloc: (dt_n, dt_I) in seconds into the device float64 tensor
        dt_out[2], stream-ordered, without allocating or blocking."""
        if dt_out.dtype.itemsize != 8 or dt_out.numel() < 2:
            raise ValueError("dt_out must be a device float64 tensor of at least 2 entries")
        g = _grid(grid)
        r = Rates(_ptr(gamma), 0)
        b, _keep = _bins_struct(bins)
        p = ChemParams(0, int(rates), int(collisional), float(alpha_hii), 0.1, 1, 1.0, 0, _stream(stream), None,
                       0.0, 0, 0)
        self._check(lib().arc_rt_timestep_noalloc(self._h, C.byref(g), C.byref(r), C.byref(b), C.byref(p),
                                                  float(eps), _ptr(dt_out)))
        return dt_out


def _bins_struct(bins):
    frac = np.ascontiguousarray(bins["frac"], np.float64)
    e = np.ascontiguousarray(bins["e_erg"], np.float64)
    sig = np.ascontiguousarray(bins["sigma"], np.float64).reshape(-1, 3)
    thr = np.ascontiguousarray(bins["e_thr"], np.float64)
    return Bins(frac.size, _ptr(frac), _ptr(e), _ptr(sig), _ptr(thr)), (frac, e, sig, thr)


class MLP:
    """arc_mlp: the learned chemistry network (owned; release with close())."""

    def __init__(self, ctx: Context):
        h = C.c_void_p()
        rc = lib().arc_mlp_create(ctx._h, C.byref(h))
        if rc != ARC_OK:
            raise ArcError(rc, "arc_mlp_create failed")
        self._h = h
        self._ctx = ctx

    def close(self):
        if getattr(self, "_h", None):
            lib().arc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    N_IN = 8  # (n_H, x_HI, T, Gamma_HI, dt, h, x_HeII, x_HeI)

    def train(self, X, Y, epochs=8, batch=1024, lr=2e-3, seed=1, val_frac=0.1, stream=None, y_he=0.08,
              collisional=1) -> dict:
        """X: device float32 [m, 8] (n_H, x_HI, T, Gamma_HI, dt, h, x_HeII, x_HeI) with h the
        photoheating per H atom; Y: device float32 [m, 2] (x_HI', T'). y_he and collisional
        describe the samples' gas and solver."""
        if tuple(X.shape[1:]) != (self.N_IN,) or tuple(Y.shape) != (X.shape[0], 2):
            raise ValueError(f"expected X [m, {self.N_IN}] and Y [m, 2], got {tuple(X.shape)}, {tuple(Y.shape)}")
        p = TrainParams(int(epochs), int(batch), float(lr), int(seed), float(val_frac), _stream(stream),
                        float(y_he), int(collisional))
        rep = TrainReport()
        self._ctx._check(lib().arc_mlp_train(self._ctx._h, self._h, _ptr(X), _ptr(Y), int(X.shape[0]), C.byref(p),
                                             C.byref(rep)))
        return {k: getattr(rep, k) for k, _ in TrainReport._fields_}

    def predict(self, X, P, stream=None):
        if tuple(X.shape[1:]) != (self.N_IN,) or tuple(P.shape) != (X.shape[0], 2):
            raise ValueError(f"expected X [m, {self.N_IN}] and P [m, 2], got {tuple(X.shape)}, {tuple(P.shape)}")
        self._ctx._check(lib().arc_mlp_predict(self._ctx._h, self._h, _ptr(X), int(X.shape[0]), _ptr(P),
                                               _stream(stream)))
        return P

    def save(self) -> bytes:
        n = C.c_size_t(0)
        rc = lib().arc_mlp_save(self._h, None, C.byref(n))
        if rc != ARC_OK:
            raise ArcError(rc, "arc_mlp_save size query failed")
        buf = C.create_string_buffer(n.value)
        rc = lib().arc_mlp_save(self._h, buf, C.byref(n))
        if rc != ARC_OK:
            raise ArcError(rc, "arc_mlp_save failed")
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        rc = lib().arc_mlp_load(self._h, blob, len(blob))
        if rc != ARC_OK:
            raise ArcError(rc, "arc_mlp_load failed")
