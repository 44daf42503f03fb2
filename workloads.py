"""Seeded synthetic inputs shaped like the paper's TSV-array workloads.

This module holds input generation only: cell geometry and materials, the
cell-type map of an array, thermal load, boundary-condition choice, a smooth
background displacement field (a stand-in for the coarse chiplet solution the
paper uses for sub-modelling, Sec. 4.4 and 5.2, which is not available), and
a Poisson request stream.  It holds none of the method's arithmetic and is
the only module imported by both the oracle-side and the GPU-side code of
the tests and of the benchmark.

Units: micrometres, MPa, 1/K, K.  Material triples are (E, nu, alpha).
"""
import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

SI = (130.0e3, 0.28, 2.6e-6)      # silicon matrix
CU = (110.0e3, 0.35, 17.0e-6)     # copper via
SIO2 = (71.0e3, 0.16, 0.5e-6)     # dielectric liner
# Micro-bump layer (representative values; the paper fixes none for bumps).
UNDERFILL = (8.0e3, 0.30, 30.0e-6)
SNAG = (50.0e3, 0.36, 22.0e-6)    # SnAg solder


@dataclass(frozen=True)
class CellSpec:
    pitch_x: float = 15.0
    pitch_y: float = 15.0
    height: float = 50.0
    mesh: tuple = (16, 16, 32)            # hexes along x, y, z
    tsv_diameter: float = 5.0             # 0 => dummy (pure matrix) block
    liner_thickness: float = 0.0
    matrix: tuple = SI
    via: tuple = CU
    liner: tuple = SIO2
    interp: tuple = (4, 4, 4)             # Lagrange nodes per axis
    # "tsv": a via through the block with an optional liner around it.
    # "bump": a micro-bump block; tsv_diameter is the bump column's diameter,
    # `via` its solder, `liner` the metal of the pads at its two ends
    # (pad_thickness each) and `matrix` the underfill around it.
    structure: str = "tsv"
    pad_thickness: float = 0.0
    # Shear x += skew * y of the block: 0 for a 90-degree array; 1/sqrt(3)
    # with pitch_y = pitch_x sqrt(3)/2 for the rhombic block of a 120-degree
    # array (TSVs on a triangular lattice of spacing pitch_x).
    skew: float = 0.0

    def dummy(self):
        return replace(self, tsv_diameter=0.0, liner_thickness=0.0, pad_thickness=0.0)


@dataclass
class FourierField:
    """u(r) = sum_m w_m e_m cos(2 pi (a_m x/Lx + b_m y/Ly + c_m z/Lz) + phi_m).

    The weights sum to ``amplitude`` so |u| <= amplitude everywhere."""
    L: tuple
    k: np.ndarray          # (M, 3) integer wave numbers
    e: np.ndarray          # (M, 3) unit directions
    w: np.ndarray          # (M,) weights
    phi: np.ndarray        # (M,) phases

    def __call__(self, xyz):
        xyz = np.asarray(xyz, dtype=float)
        arg = 2.0 * np.pi * (xyz / np.asarray(self.L)[None, :]) @ self.k.T.astype(float)
        arg = arg + self.phi[None, :]
        return (np.cos(arg) * self.w[None, :]) @ self.e


def fourier_field(rng, L, modes=8, amplitude=0.1):
    ks = [(a, b, c) for a in range(3) for b in range(3) for c in range(3) if (a, b, c) != (0, 0, 0)]
    idx = rng.choice(len(ks), size=modes, replace=True)
    k = np.array([ks[i] for i in idx], dtype=np.int64)
    e = rng.normal(size=(modes, 3))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    w = rng.uniform(0.5, 1.0, size=modes)
    w *= amplitude / w.sum()
    phi = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    return FourierField(tuple(float(v) for v in L), k, e, w, phi)


@dataclass
class ArrayCase:
    """One global-stage problem: an N_x x N_y array of blocks of the given
    types (cell_type[cy * N_x + cx] indexes ``specs``)."""
    name: str
    specs: list
    nx_cells: int
    ny_cells: int
    cell_type: np.ndarray
    delta_T: float = -250.0
    clamp_bottom: bool = True
    clamp_top: bool = False
    field: Optional[FourierField] = None
    mixed: bool = False

    @property
    def n_cells(self):
        return self.nx_cells * self.ny_cells


def dummy_map(rng, n_cells, fraction):
    t = np.zeros(n_cells, dtype=np.uint8)
    k = int(round(fraction * n_cells))
    if k:
        t[rng.choice(n_cells, size=k, replace=False)] = 1
    return t


def case_c1():
    """2x2 array, 10x10x20 hexes, quadratic faces, bottom clamped."""
    spec = CellSpec(mesh=(10, 10, 20), interp=(3, 3, 3))
    return ArrayCase("2x2 TSV, 10x10x20 hex, quadratic", [spec], 2, 2,
                     np.zeros(4, dtype=np.uint8))


def case_c2(seed=0):
    """16x16 array, 16x16x32 hexes, cubic faces, diameter drawn from {4,5,6}."""
    rng = np.random.default_rng(seed)
    d = float(rng.choice([4.0, 5.0, 6.0]))
    spec = CellSpec(tsv_diameter=d)
    return ArrayCase(f"16x16 TSV d={d:g}, 16x16x32 hex, cubic", [spec], 16, 16,
                     np.zeros(256, dtype=np.uint8))


def case_c3(seed=0):
    """64x64 array with 10% dummy blocks, mixed precision."""
    rng = np.random.default_rng(seed)
    spec = CellSpec()
    return ArrayCase("64x64 TSV + 10% dummy, 16x16x32 hex, cubic", [spec, spec.dummy()], 64, 64,
                     dummy_map(rng, 4096, 0.10), mixed=True)


def case_c5(seed=0, n=200):
    """n x n array (200 x 200 by default), 20x20x40 hexes with a 0.5 um
    liner, Fourier field on all outer faces (smaller n: a sub-array of the
    same cell with a field of the same kind over its own extent)."""
    rng = np.random.default_rng(seed)
    spec = CellSpec(mesh=(20, 20, 40), liner_thickness=0.5)
    L = (n * spec.pitch_x, n * spec.pitch_y, spec.height)
    return ArrayCase(f"{n}x{n} TSV+liner, 20x20x40 hex, cubic, Fourier boundary", [spec], n, n,
                     np.zeros(n * n, dtype=np.uint8), clamp_bottom=False,
                     field=fourier_field(rng, L), mixed=True)


def bump_spec(**kw):
    """A micro-bump block: 40 x 40 x 20 um of underfill with a 25 um SnAg
    column and 3 um copper pads at both ends, 16 x 16 x 16 hexes, cubic faces."""
    base = dict(pitch_x=40.0, pitch_y=40.0, height=20.0, mesh=(16, 16, 16), tsv_diameter=25.0,
                matrix=UNDERFILL, via=SNAG, liner=CU, structure="bump", pad_thickness=3.0)
    base.update(kw)
    return CellSpec(**base)


def hex_spec(pitch=15.0, **kw):
    """Rhombic (60/120-degree) block of a 120-degree TSV array: TSVs on a
    triangular lattice of spacing `pitch`, 16 x 14 x 32 hexes (near-equal
    in-plane edges), cubic faces, the via of diameter 5 um at the centre."""
    base = dict(pitch_x=pitch, pitch_y=pitch * math.sqrt(3.0) / 2.0, skew=1.0 / math.sqrt(3.0),
                mesh=(16, 14, 32))
    base.update(kw)
    return CellSpec(**base)


def case_hex(seed=0, n=64, dummies=0.10):
    """n x n TSV array on a 120-degree lattice (rhombic blocks), bottom
    clamped, dT = -250 K, with a fraction of dummy blocks drawn from the seed."""
    rng = np.random.default_rng(seed)
    spec = hex_spec()
    return ArrayCase(f"{n}x{n} 120-degree TSV array, 16x14x32 hex, cubic, bottom clamped", [spec, spec.dummy()],
                     n, n, dummy_map(rng, n * n, dummies), mixed=True)


def case_bump(seed=0, n=100, missing=0.05):
    """n x n micro-bump layer between two clamped faces (substrate below, die
    above), cooled by 200 K after reflow; a fraction of sites without a bump
    (pure underfill blocks) drawn from the seed."""
    rng = np.random.default_rng(seed)
    spec = bump_spec()
    return ArrayCase(f"{n}x{n} micro-bump layer, 16x16x16 hex, cubic, both faces clamped", [spec, spec.dummy()],
                     n, n, dummy_map(rng, n * n, missing), delta_T=-200.0, clamp_bottom=True, clamp_top=True,
                     mixed=True)


def small_case(nx=3, ny=2, mesh=(4, 4, 6), interp=(3, 3, 3), dummies=True, seed=0, **kw):
    """A few-block array with a small cell mesh, for fast parity tests."""
    rng = np.random.default_rng(seed)
    spec = CellSpec(mesh=mesh, interp=interp, **kw)
    specs = [spec, spec.dummy()] if dummies else [spec]
    t = dummy_map(rng, nx * ny, 0.34) if dummies else np.zeros(nx * ny, dtype=np.uint8)
    return ArrayCase(f"{nx}x{ny} small", specs, nx, ny, t)


@dataclass
class Request:
    arrival_s: float
    N: int
    pitch: float
    delta_T: float
    seed: int


def request_stream(seed=0, n_requests=2000, rate_hz=200.0, n_min=4, n_max=48,
                   pitches=(10.0, 15.0, 20.0), dT_range=(-300.0, -150.0)):
    """Poisson arrivals; per request N ~ U{n_min..n_max}, pitch ~ U(pitches),
    dT ~ U[dT_range]; each request seeds its own 10% dummy placement."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        out.append(Request(float(t[i]), int(rng.integers(n_min, n_max + 1)),
                           float(rng.choice(pitches)), float(rng.uniform(*dT_range)),
                           int(rng.integers(0, 2 ** 31 - 1))))
    return out


def request_case(req, mesh=(16, 16, 32), interp=(4, 4, 4)):
    rng = np.random.default_rng(req.seed)
    spec = CellSpec(pitch_x=req.pitch, pitch_y=req.pitch, mesh=mesh, interp=interp)
    return ArrayCase(f"{req.N}x{req.N} p={req.pitch:g}", [spec, spec.dummy()], req.N, req.N,
                     dummy_map(rng, req.N * req.N, 0.10), delta_T=req.delta_T, mixed=True)
