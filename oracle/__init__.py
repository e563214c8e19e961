"""Plain FP64 CPU oracle for the ARC adaptive ray-tracing step (arXiv:1807.07094).

TEST INFRASTRUCTURE ONLY. This package is the yardstick the GPU library is checked
against. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the GPU library never does, and this package never imports
the GPU library. The arithmetic lives in ``arc_oracle.c`` (compiled with gcc); this
module only marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "arc_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libarc_oracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc into oracle/_build/libarc_oracle.so."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-fno-strict-aliasing", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("cell_cm", C.c_double), ("y_he", C.c_double),
                ("n_h", C.c_void_p), ("x_hi", C.c_void_p), ("x_hei", C.c_void_p), ("x_heii", C.c_void_p)]


class Sources(C.Structure):
    _fields_ = [("n", C.c_int32), ("pos", C.c_void_p), ("ndot", C.c_void_p), ("r_thin", C.c_void_p),
                ("r_thin_out", C.c_void_p)]


class Bins(C.Structure):
    _fields_ = [("nbins", C.c_int32), ("frac", C.c_void_p), ("e_erg", C.c_void_p),
                ("sigma", C.c_void_p), ("e_thr", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("level0", C.c_int32), ("max_level", C.c_int32), ("rays_per_cell", C.c_double),
                ("eps_term", C.c_double), ("correction", C.c_int32)]


class Ledger(C.Structure):
    _fields_ = [("emitted", C.c_double), ("absorbed_trace", C.c_double), ("escaped", C.c_double),
                ("crossings", C.c_uint64), ("rays", C.c_uint64), ("splits", C.c_uint64),
                ("terminated", C.c_uint64), ("escaped_rays", C.c_uint64), ("tree_count", C.c_int64),
                ("absorbed_thin", C.c_double)]


class ChemParams(C.Structure):
    _fields_ = [("isothermal", C.c_int32), ("rates", C.c_int32), ("collisional", C.c_int32),
                ("alpha_hii", C.c_double), ("eps", C.c_double), ("max_sub", C.c_int32),
                ("t_floor", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.orc_npix.restype = C.c_int64
        L.orc_npix.argtypes = [C.c_int32]
        L.orc_healpix_vec.restype = None
        L.orc_healpix_vec.argtypes = [C.c_int32, C.c_int64, C.c_void_p]
        L.orc_t_split.restype = C.c_double
        L.orc_t_split.argtypes = [C.c_double, C.c_int32]
        L.orc_auto_max_level.restype = C.c_int32
        L.orc_auto_max_level.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_double]
        L.orc_walk.restype = C.c_int64
        L.orc_walk.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                               C.c_double, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]
        L.orc_trace.restype = C.c_int32
        L.orc_trace.argtypes = [C.POINTER(Grid), C.POINTER(Sources), C.POINTER(Bins), C.POINTER(Params),
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Ledger)]
        L.orc_trace_mt.restype = C.c_int32
        L.orc_trace_mt.argtypes = [C.POINTER(Grid), C.POINTER(Sources), C.POINTER(Bins), C.POINTER(Params),
                                   C.c_void_p, C.c_int32, C.POINTER(Ledger)]
        L.orc_finalize.restype = None
        L.orc_finalize.argtypes = [C.POINTER(Grid), C.POINTER(Bins), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_double)]
        L.orc_chem.restype = None
        L.orc_chem.argtypes = [C.c_int64, C.c_double] + [C.c_void_p] * 7 + [C.c_double, C.POINTER(ChemParams)] + \
            [C.c_void_p] * 6
        L.orc_rate_coeffs.restype = None
        L.orc_rate_coeffs.argtypes = [C.c_double, C.c_void_p]
        L.orc_cooling_coeffs.restype = None
        L.orc_cooling_coeffs.argtypes = [C.c_double, C.c_void_p]
        L.orc_cooling.restype = C.c_double
        L.orc_cooling.argtypes = [C.c_double] * 7 + [C.c_int32]
        L.orc_timestep.restype = None
        L.orc_timestep.argtypes = [C.c_int64, C.c_double, C.c_double] + [C.c_void_p] * 6 + \
            [C.POINTER(ChemParams), C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------------
def npix(level: int) -> int:
    return int(lib().orc_npix(level))


def healpix_vec(level: int, pix) -> np.ndarray:
    """FP64 HEALPix nested pixel centres, shape [len(pix), 3]."""
    pix = np.atleast_1d(np.asarray(pix, dtype=np.int64))
    out = np.empty((pix.size, 3), np.float64)
    v = np.empty(3, np.float64)
    L = lib()
    for i, q in enumerate(pix):
        L.orc_healpix_vec(level, int(q), _p(v))
        out[i] = v
    return out


def t_split(rays_per_cell: float, level: int) -> float:
    return float(lib().orc_t_split(rays_per_cell, level))


def auto_max_level(shape, rays_per_cell: float) -> int:
    nz, ny, nx = shape
    return int(lib().orc_auto_max_level(nx, ny, nz, rays_per_cell))


def walk(shape, xs, d, t0=0.0, t_end=-1.0, cap=100000):
    """Cells and segment lengths of one ray; returns (cells, ds, how)."""
    nz, ny, nx = shape
    xs = _f64(xs)
    d = _f64(d)
    cells = np.empty(cap, np.int64)
    ds = np.empty(cap, np.float64)
    how = C.c_int32(0)
    n = lib().orc_walk(nx, ny, nz, _p(xs), _p(d), t0, t_end, _p(cells), _p(ds), cap, C.byref(how))
    if n > cap:
        raise ValueError("walk longer than cap")
    return cells[:n], ds[:n], how.value


def _grid(g, keep):
    n_h, x_hi, x_hei, x_heii = (_f32(g[k]) for k in ("n_h", "x_hi", "x_hei", "x_heii"))
    keep += [n_h, x_hi, x_hei, x_heii]
    nz, ny, nx = n_h.shape
    return Grid(nx, ny, nz, float(g["cell_cm"]), float(g["y_he"]), _p(n_h), _p(x_hi), _p(x_hei), _p(x_heii))


def _bins(b, keep):
    frac, e, sig, thr = _f64(b["frac"]), _f64(b["e_erg"]), _f64(b["sigma"]), _f64(b["e_thr"])
    keep += [frac, e, sig, thr]
    return Bins(frac.size, _p(frac), _p(e), _p(sig), _p(thr))


def trace(grid: dict, sources: dict, bins: dict, params: dict, tree_cap: int = 0, direct: bool = False):
    """Run the oracle tracer. Returns dict(J [nb,nz,ny,nx], ledger dict, tree, gdir, r_thin_out).
    sources may carry "r_thin" (optically thin radius per source, section 2.6); r_thin_out is
    each source's R_tau<0.1 measured by this trace."""
    keep = []
    g = _grid(grid, keep)
    b = _bins(bins, keep)
    pos = _f64(sources["pos"]).reshape(-1, 3)
    ndot = _f64(sources["ndot"]).reshape(-1)
    r_thin = sources.get("r_thin")
    r_thin = _f64(r_thin).reshape(-1) if r_thin is not None else None
    if r_thin is not None and r_thin.size != ndot.size:
        raise ValueError("r_thin needs one radius per source")
    r_out = np.empty(ndot.size, np.float64)
    keep += [pos, ndot, r_thin, r_out]
    s = Sources(ndot.size, _p(pos), _p(ndot), _p(r_thin), _p(r_out))
    p = Params(int(params["level0"]), int(params.get("max_level", -1)), float(params["rays_per_cell"]),
               float(params["eps_term"]), int(params.get("correction", 0)))
    shape = (g.nz, g.ny, g.nx)
    J = np.empty((b.nbins,) + shape, np.float64)
    gdir = np.empty((3,) + shape, np.float64) if direct else None
    tree = np.empty(max(tree_cap, 1), np.uint64) if tree_cap else None
    led = Ledger()
    rc = lib().orc_trace(C.byref(g), C.byref(s), C.byref(b), C.byref(p), _p(J), _p(gdir), _p(tree),
                         int(tree_cap), C.byref(led))
    if rc != 0:
        raise RuntimeError("orc_trace failed")
    ledger = {k: getattr(led, k) for k, _ in Ledger._fields_}
    out = {"J": J, "ledger": ledger, "gdir": gdir, "r_thin_out": r_out}
    if tree is not None:
        if led.tree_count > tree_cap:
            raise ValueError("tree_cap too small")
        out["tree"] = tree[: led.tree_count]
    return out


def trace_mt(grid: dict, sources: dict, bins: dict, params: dict, threads: int):
    """The oracle tracer with the sources split over host threads (one shared field, atomic
    additions). Returns dict(J, ledger, r_thin_out)."""
    keep = []
    g = _grid(grid, keep)
    b = _bins(bins, keep)
    pos = _f64(sources["pos"]).reshape(-1, 3)
    ndot = _f64(sources["ndot"]).reshape(-1)
    r_thin = sources.get("r_thin")
    r_thin = _f64(r_thin).reshape(-1) if r_thin is not None else None
    r_out = np.empty(ndot.size, np.float64)
    keep += [pos, ndot, r_thin, r_out]
    s = Sources(ndot.size, _p(pos), _p(ndot), _p(r_thin), _p(r_out))
    p = Params(int(params["level0"]), int(params.get("max_level", -1)), float(params["rays_per_cell"]),
               float(params["eps_term"]), int(params.get("correction", 0)))
    J = np.empty((b.nbins, g.nz, g.ny, g.nx), np.float64)
    led = Ledger()
    if lib().orc_trace_mt(C.byref(g), C.byref(s), C.byref(b), C.byref(p), _p(J), int(threads), C.byref(led)) != 0:
        raise RuntimeError("orc_trace_mt failed")
    return {"J": J, "ledger": {k: getattr(led, k) for k, _ in Ledger._fields_}, "r_thin_out": r_out}


def finalize(grid: dict, bins: dict, J: np.ndarray):
    """Rates from J: returns (gamma [3,...], heat [3,...], absorbed)."""
    keep = []
    g = _grid(grid, keep)
    b = _bins(bins, keep)
    J = _f64(J)
    shape = (g.nz, g.ny, g.nx)
    gamma = np.empty((3,) + shape, np.float64)
    heat = np.empty((3,) + shape, np.float64)
    absorbed = C.c_double(0)
    lib().orc_finalize(C.byref(g), C.byref(b), _p(J), _p(gamma), _p(heat), C.byref(absorbed))
    return gamma, heat, absorbed.value


def _chem_params(cp: dict):
    return ChemParams(int(cp.get("isothermal", 0)), int(cp.get("rates", 1)), int(cp.get("collisional", 1)),
                      float(cp.get("alpha_hii", 2.59e-13)), float(cp.get("eps", 0.1)),
                      int(cp.get("max_sub", 100000)), float(cp.get("t_floor", 1.0)))


def chem(grid: dict, state: dict, gamma, heat, dt: float, cp: dict):
    """Chemistry step. state has x_hi, x_hei, x_heii, temp (float32 arrays).
    Returns dict of float64 outputs plus nsub and flags."""
    n_h = _f32(grid["n_h"])
    xs = [_f32(state[k]) for k in ("x_hi", "x_hei", "x_heii", "temp")]
    gamma = _f64(gamma)
    heat = _f64(heat)
    n = n_h.size
    outs = [np.empty(n_h.shape, np.float64) for _ in range(4)]
    nsub = np.empty(n_h.shape, np.int32)
    flags = np.empty(n_h.shape, np.int32)
    p = _chem_params(cp)
    lib().orc_chem(n, float(grid["y_he"]), _p(n_h), *[_p(x) for x in xs], _p(gamma), _p(heat), float(dt),
                   C.byref(p), *[_p(o) for o in outs], _p(nsub), _p(flags))
    return {"x_hi": outs[0], "x_hei": outs[1], "x_heii": outs[2], "temp": outs[3], "nsub": nsub,
            "flags": flags}


def rate_coeffs(T: float) -> np.ndarray:
    out = np.empty(6, np.float64)
    lib().orc_rate_coeffs(float(T), _p(out))
    return out


def cooling_coeffs(T: float) -> np.ndarray:
    """[0] HII [1] HeII [2] HeIII recombination cooling, [3] HeII dielectronic cooling,
    [4] HI [5] HeII collisional excitation, [6] bremsstrahlung per Z^2 [erg cm^3 s^-1]."""
    out = np.empty(7, np.float64)
    lib().orc_cooling_coeffs(float(T), _p(out))
    return out


def cooling(T, ne, nhi, nhii, nhei, nheii, nheiii, collisional=1) -> float:
    """Cooling rate per volume [erg cm^-3 s^-1]."""
    return float(lib().orc_cooling(float(T), float(ne), float(nhi), float(nhii), float(nhei), float(nheii),
                                   float(nheiii), int(collisional)))


def timestep(grid: dict, state: dict, gamma, cp: dict, sigma0: float, eps: float):
    """Section 2.9 adaptive RT time step: returns (dt_n, dt_I) in seconds. gamma: [3, ...]
    or [...] photoionisation rates (the HI one is used)."""
    keep = []
    n_h = _f32(grid["n_h"])
    x_hi, x_hei, x_heii, temp = (_f32(state[k]) for k in ("x_hi", "x_hei", "x_heii", "temp"))
    g = np.ascontiguousarray(gamma, np.float64)
    ghi = np.ascontiguousarray(g.reshape(-1)[: n_h.size])
    keep += [n_h, x_hi, x_hei, x_heii, temp, ghi]
    p = _chem_params(cp)
    dn, di = C.c_double(0), C.c_double(0)
    lib().orc_timestep(n_h.size, float(grid["y_he"]), float(grid["cell_cm"]), _p(n_h), _p(x_hi), _p(x_hei),
                       _p(x_heii), _p(temp), _p(ghi), C.byref(p), float(sigma0), float(eps), C.byref(dn),
                       C.byref(di))
    return dn.value, di.value
