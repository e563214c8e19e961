"""Seeded synthetic inputs for the adaptive ray-tracing step.

This module only builds inputs: grids, source lists, frequency-bin tables and run
parameters. It holds none of the ray-tracing or chemistry arithmetic, and both the GPU
library's tests and the CPU oracle's tests draw their inputs from it.

Workloads (the shapes and value distributions of the paper's runs; every field is
synthetic, none of the comparison project's data is reproduced):

  c1  64^3 uniform hydrogen, the isothermal HII-region test of section 3 (Test 1):
      6.6 kpc box, n_H = 1e-3 cm^-3, T = 1e4 K, x_HII = 1.2e-3, one 13.6 eV source of
      5e48 photons/s at the box centre, root level 0, Phi = 4.
  lognormal(n, n_src, seed)  H + He (He/H = 0.08) on the cell size of the cosmic
      density-field test (Test 4: 0.5 h^-1 cMpc / 128 at z = 9), density
      n_H = 1e-3 exp(g - 1/2) with white-noise g, three bands with lower edges 13.6,
      24.6 and 54.4 eV averaged over a 1e5 K blackbody, power-law luminosities
      dN/dNdot ~ Ndot^-2 on [1e48, 1e51] photons/s.
  grf(n, n_src, seed)  as lognormal but with a Gaussian random field: white noise
      smoothed periodically by a Gaussian of 2 cells, unit variance, delta = 0.5 g,
      n_H = 1e-3 exp(delta - 0.125).

Random numbers: numpy Philox. Each quantity draws from its own key
(seed | tag << 64): tag 0 density (one key per z-slab so that slabs fill in parallel),
1 source cells, 2 luminosities, 3 sub-cell offsets. Source positions lie on a 2^-12
lattice inside their cell.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import functools
import math

import numpy as np

# Physical constants (CGS).
KPC_CM = 3.0856775814913673e21
EV_ERG = 1.602176634e-12
K_B = 1.380649e-16
MYR_S = 3.15576e13
KT_EV_PER_K = 8.617333262e-5

# Ionisation thresholds [eV]: HI, HeI, HeII.
E_THR_EV = (13.598, 24.587, 54.418)

LATTICE = 4096  # source positions are multiples of 1/LATTICE cells


# ----------------------------------------------------------------------------------
# Cross sections and frequency bins (inputs of the method, not part of it).
# ----------------------------------------------------------------------------------
def sigma_hydrogenic(e_ev: float, z: int) -> float:
    """Hydrogenic photoionisation cross section [cm^2] (Osterbrock & Ferland 2006,
    eq. 2.4) with threshold cross section 6.30e-18 / Z^2."""
    e1 = E_THR_EV[0] if z == 1 else E_THR_EV[2]
    if e_ev < e1:
        return 0.0
    eps = math.sqrt(e_ev / e1 - 1.0)
    a0 = 6.30e-18 / (z * z)
    if eps < 1e-8:
        return a0
    return a0 * (e1 / e_ev) ** 4 * math.exp(4.0 - 4.0 * math.atan(eps) / eps) / (1.0 - math.exp(-2.0 * math.pi / eps))


def sigma_hei(e_ev: float) -> float:
    """HeI ground-state photoionisation cross section [cm^2], analytic fit of
    Verner, Ferland, Korista & Yakovlev (1996, ApJ 465, 487), He I 1s parameters."""
    if e_ev < E_THR_EV[1]:
        return 0.0
    e0, s0, ya, p, yw, y0, y1 = 13.61, 949.2e-18, 1.469, 3.188, 2.039, 0.4434, 2.136
    x = e_ev / e0 - y0
    y = math.sqrt(x * x + y1 * y1)
    return s0 * ((x - 1.0) ** 2 + yw * yw) * y ** (0.5 * p - 5.5) * (1.0 + math.sqrt(y / ya)) ** (-p)


def sigma_species(e_ev: float):
    return (sigma_hydrogenic(e_ev, 1), sigma_hei(e_ev), sigma_hydrogenic(e_ev, 2))


def bins_monochromatic(e_ev: float = 13.6, sigma_hi: float = 6.30e-18) -> dict:
    """One bin at a single photon energy, hydrogen absorption only."""
    return {
        "frac": np.array([1.0]),
        "e_erg": np.array([e_ev * EV_ERG]),
        "sigma": np.array([[sigma_hi, 0.0, 0.0]]),
        "e_thr": np.array(E_THR_EV) * EV_ERG,
    }


@functools.lru_cache(maxsize=None)
def _blackbody_bands(t_bb: float, edges: tuple):
    from scipy import integrate

    kt = KT_EV_PER_K * t_bb

    def nphot(e):  # photon number spectrum of a blackbody, arbitrary normalisation
        x = e / kt
        return e * e / math.expm1(x) if x < 700 else 0.0

    lo_all = edges[0]
    total = integrate.quad(nphot, lo_all, np.inf, limit=200)[0]
    rows = []
    bounds = list(edges) + [np.inf]
    for i in range(len(edges)):
        lo, hi = bounds[i], bounds[i + 1]

        def q(f):
            return integrate.quad(lambda e: f(e) * nphot(e), lo, hi, limit=400)[0]

        n = q(lambda e: 1.0)
        rows.append((n / total, q(lambda e: e) / n, tuple(q(lambda e, s=s: sigma_species(e)[s]) / n for s in range(3))))
    return tuple(rows)


def bins_blackbody(t_bb: float = 1e5, edges=(13.6, 24.6, 54.4)) -> dict:
    """Bands with the given lower edges [eV] (the last extends to infinity); each band
    carries the photon-weighted mean energy and cross sections of a t_bb blackbody
    (section 2.2: one frequency per bin standing for the band-averaged cross section)."""
    rows = _blackbody_bands(float(t_bb), tuple(float(e) for e in edges))
    return {
        "frac": np.array([r[0] for r in rows]),
        "e_erg": np.array([r[1] for r in rows]) * EV_ERG,
        "sigma": np.array([r[2] for r in rows]),
        "e_thr": np.array(E_THR_EV) * EV_ERG,
    }


# ----------------------------------------------------------------------------------
# Workload container.
# ----------------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    grid: dict        # n_h, x_hi, x_hei, x_heii, temp (float32 [nz,ny,nx]); cell_cm, y_he
    sources: dict     # pos [n,3] float64 (lattice), ndot [n] float64
    bins: dict        # frac, e_erg, sigma [nb,3], e_thr [3]
    trace: dict       # level0, rays_per_cell, max_level, eps_term
    chem: dict        # isothermal, rates, collisional, alpha_hii, eps, max_sub, t_floor
    dt: float         # RT time step [s]

    @property
    def shape(self):
        return self.grid["n_h"].shape

    def state(self) -> dict:
        return {k: self.grid[k] for k in ("x_hi", "x_hei", "x_heii", "temp")}

    def subset(self, idx) -> "Workload":
        """The same grid with a subset of the sources."""
        idx = np.asarray(idx)
        src = {"pos": self.sources["pos"][idx], "ndot": self.sources["ndot"][idx]}
        return dataclasses.replace(self, name=f"{self.name}[subset {idx.size}]", sources=src)


def _key(seed: int, tag: int) -> int:
    return int(seed) | (int(tag) << 64)


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=_key(seed, tag)))


def white_noise(shape, seed: int, threads: int = 16) -> np.ndarray:
    """Standard normal float64 field; z-slab i draws from key (seed, tag 0, slab i)."""
    nz = shape[0]
    out = np.empty(shape, np.float64)
    slabs = min(64, nz)
    bounds = np.linspace(0, nz, slabs + 1).astype(int)

    def fill(i):
        g = np.random.Generator(np.random.Philox(key=_key(seed, 0) + (i << 96)))
        g.standard_normal(out=out[bounds[i]:bounds[i + 1]])

    with cf.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(fill, range(slabs)))
    return out


def _lattice_positions(cells_flat: np.ndarray, shape, seed: int) -> np.ndarray:
    nz, ny, nx = shape
    z, rem = np.divmod(cells_flat, ny * nx)
    y, x = np.divmod(rem, nx)
    k = _rng(seed, 3).integers(0, LATTICE, size=(cells_flat.size, 3))
    pos = np.stack([x, y, z], axis=1).astype(np.float64) + k / LATTICE
    return pos


def power_law_ndot(n: int, seed: int, lo=1e48, hi=1e51) -> np.ndarray:
    """dN/dNdot ~ Ndot^-2 on [lo, hi] by inverse CDF."""
    u = _rng(seed, 2).random(n)
    return 1.0 / (1.0 / lo - u * (1.0 / lo - 1.0 / hi))


def _initial_state(shape, y_he: float) -> dict:
    x_hii = 1.2e-3
    return {
        "x_hi": np.full(shape, 1.0 - x_hii, np.float32),
        "x_hei": np.full(shape, 1.0 - x_hii if y_he > 0 else 0.0, np.float32),
        "x_heii": np.full(shape, x_hii if y_he > 0 else 0.0, np.float32),
        "temp": np.full(shape, 1e4, np.float32),
    }


# Cell of the cosmic density-field test: 0.5 h^-1 comoving Mpc / 128 at z = 9, h = 0.7.
COSMIC_CELL_CM = 0.5 / 0.7 * 1000.0 * KPC_CM / 10.0 / 128.0


def c1(n: int = 64, box_kpc: float = 6.6, center=None, ndot: float = 5e48, level0: int = 0,
       eps_term: float = 1e-12, dt_myr: float = 1.0) -> Workload:
    shape = (n, n, n)
    grid = {"n_h": np.full(shape, 1e-3, np.float32), "cell_cm": box_kpc * KPC_CM / n, "y_he": 0.0}
    grid.update(_initial_state(shape, 0.0))
    pos = np.array([center if center is not None else (n / 2, n / 2, n / 2)], np.float64)
    return Workload(
        name=f"c1-{n}^3",
        grid=grid,
        sources={"pos": pos, "ndot": np.array([ndot])},
        bins=bins_monochromatic(13.6),
        trace={"level0": level0, "rays_per_cell": 4.0, "max_level": -1, "eps_term": eps_term},
        chem={"isothermal": 1, "rates": 0, "collisional": 0, "alpha_hii": 2.59e-13, "eps": 0.1,
              "max_sub": 100000, "t_floor": 1.0},
        dt=dt_myr * MYR_S,
    )


def _he_workload(name, n_h, n_src, seed, source_cells, dt_myr, level0, eps_term, cand=None) -> Workload:
    shape = n_h.shape
    y_he = 0.08
    ncell = n_h.size
    if source_cells == "uniform":
        cells = _rng(seed, 1).choice(ncell, size=n_src, replace=False)
    else:  # biased to the densest 1% of cells (cells at or above the 99th percentile)
        if cand is None:
            flat = n_h.reshape(-1)
            k = max(1, ncell // 100)
            thr = np.partition(flat, ncell - k)[ncell - k]
            cand = np.flatnonzero(flat >= thr)
        cells = cand[_rng(seed, 1).choice(cand.size, size=n_src, replace=False)]
    grid = {"n_h": n_h.astype(np.float32), "cell_cm": COSMIC_CELL_CM, "y_he": y_he}
    grid.update(_initial_state(shape, y_he))
    return Workload(
        name=name,
        grid=grid,
        sources={"pos": _lattice_positions(np.sort(cells), shape, seed), "ndot": power_law_ndot(n_src, seed)},
        bins=bins_blackbody(),
        trace={"level0": level0, "rays_per_cell": 4.0, "max_level": -1, "eps_term": eps_term},
        chem={"isothermal": 0, "rates": 1, "collisional": 1, "alpha_hii": 2.59e-13, "eps": 0.1,
              "max_sub": 100000, "t_floor": 1.0},
        dt=dt_myr * MYR_S,
    )


def lognormal(n: int, n_src: int, seed: int, source_cells: str = "top1", dt_myr: float = 0.1,
              level0: int = 1, eps_term: float = 1e-6, shape=None) -> Workload:
    shape = tuple(shape) if shape is not None else (n, n, n)
    g = white_noise(shape, seed)
    n_h = 1e-3 * np.exp(g - 0.5)
    return _he_workload(f"lognormal-{'x'.join(map(str, shape[::-1]))}-{n_src}src-s{seed}", n_h, n_src, seed,
                        source_cells, dt_myr, level0, eps_term)


def grf(n: int, n_src: int, seed: int, device=None, source_cells: str = "top1", dt_myr: float = 0.1,
        level0: int = 1, eps_term: float = 1e-6) -> Workload:
    """Gaussian-random-field density; the field arithmetic runs in FP64 with torch on
    `device` (the GPU for 1024^3), the noise comes from the seeded Philox streams."""
    import torch

    shape = (n, n, n)
    dev = torch.device(device) if device is not None else torch.device("cpu")
    f = torch.from_numpy(white_noise(shape, seed)).to(dev)
    fk = torch.fft.rfftn(f)
    del f
    for axis in range(3):
        k = (torch.fft.rfftfreq if axis == 2 else torch.fft.fftfreq)(n, device=dev, dtype=torch.float64)
        view = [1, 1, 1]
        view[axis] = -1
        fk *= torch.exp(-0.5 * (2 * math.pi * k * 2.0) ** 2).view(view)
    g = torch.fft.irfftn(fk, s=shape)
    del fk
    g -= g.mean()
    g /= g.std()
    n_h = (1e-3 * torch.exp(0.5 * g - 0.125)).to(torch.float32)
    del g
    cand = None
    if source_cells != "uniform":
        flat = n_h.reshape(-1)
        kk = max(1, flat.numel() // 100)
        thr = torch.topk(flat, kk, sorted=False).values.min()
        cand = torch.nonzero(flat >= thr).flatten().cpu().numpy()
    n_h_np = n_h.cpu().numpy()
    del n_h
    return _he_workload(f"grf-{n}^3-{n_src}src-s{seed}", n_h_np, n_src, seed, source_cells, dt_myr, level0, eps_term,
                        cand=cand)


def config(index: int, device=None) -> Workload:
    """The five benchmark configurations, smallest first."""
    if index == 0:
        return c1()
    if index == 1:
        return lognormal(128, 16, 2, source_cells="uniform")
    if index == 2:
        return lognormal(256, 1024, 3)
    if index == 3:
        return lognormal(512, 4096, 4)
    if index == 4:
        return grf(1024, 16384, 5, device=device)
    raise IndexError(index)
