"""Parity of the evaluation plane (mos_reconstruct_plane, the paper's
mid-height sample grid of Sec. 5.1) with the oracle's plain evaluation.

Tolerances: FP64 von Mises within 1e-9 of the largest value (as for the
centroid stress: the sampled stress is the same GEMM over a basis built at
other points); the mixed path (FP32 PCG + FP64 refinement, BF16-split MFMA
reconstruction) within 1e-3.
"""
import numpy as np
import pytest

import workloads as W
from oracle import array as oarray
from oracle import mor as omor
from oracle import plane as oplane

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mos():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos as m
    return m


@pytest.fixture(scope="module")
def ctx(mos):
    return mos.Context(0)


_oracle_cache = {}


def oracle_rom(spec):
    if spec not in _oracle_cache:
        _oracle_cache[spec] = omor.local_stage(spec)
    return _oracle_cache[spec]


def rel_max(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max()


def gpu_plane(mos, ctx, case, grid, mixed=False, roms=None):
    import torch
    if roms is None:
        roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in case.specs]
    sol = mos.mos_solve_array(ctx, roms, case.nx_cells, case.ny_cells, case.cell_type, case.delta_T,
                              clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top, mixed=mixed)
    vm = torch.full((case.n_cells, grid * grid), np.nan, dtype=torch.float32 if mixed else torch.float64,
                    device="cuda")
    mos.mos_reconstruct_plane(ctx, sol, grid, vm)
    return vm.cpu().numpy().astype(np.float64), sol, roms


def oracle_plane(case, grid):
    oroms = [oracle_rom(s) for s in case.specs]
    sp = case.specs[0]
    mesh = oarray.AbstractMesh(case.nx_cells, case.ny_cells, sp.interp, sp.pitch_x, sp.pitch_y, sp.height)
    dofs, vals = oarray.constrained_dofs(mesh, case.clamp_bottom, case.clamp_top)
    u = oarray.solve_mor(mesh, case.cell_type, oroms, case.delta_T, dofs, vals)
    return oplane.plane_von_mises(mesh, case.cell_type, oroms, u, case.delta_T, grid)


CASES = [
    # Two cell types with a liner; 49 points per cell (three full blocks of 16 and a ragged one).
    (W.small_case(nx=3, ny=2, mesh=(4, 4, 6), interp=(3, 3, 4), pitch_x=3.0, pitch_y=3.0, height=6.0,
                  tsv_diameter=1.6, liner_thickness=0.3), 7),
    # Every sample on an element face in x and y (4 elements, 2 samples).
    (W.small_case(nx=1, ny=1, mesh=(4, 4, 6), interp=(3, 3, 3), dummies=False, pitch_x=3.0, pitch_y=3.0,
                  height=6.0, tsv_diameter=1.6), 2),
    # Odd number of layers (the plane cuts a layer through its middle), ragged array.
    (W.small_case(nx=7, ny=5, mesh=(4, 4, 5), interp=(4, 4, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                  tsv_diameter=1.6, seed=3), 4),
    # The paper's 100 x 100 grid on the 2x2 array of 10x10x20 cells.
    (W.case_c1(), 100),
]


@pytest.mark.parametrize("case,grid", CASES, ids=["3x2_two_types_g7", "1x1_faces_g2", "7x5_odd_layers_g4",
                                                  "c1_g100"])
def test_plane_fp64_matches_oracle(mos, ctx, case, grid):
    print(f"[plane] {case.name} grid {grid}", flush=True)
    got, _, _ = gpu_plane(mos, ctx, case, grid)
    ref = oracle_plane(case, grid)
    assert got.shape == ref.shape
    assert rel_max(got, ref) < 1e-9
    assert oplane.normalized_mae(got, ref) < 1e-10


def test_plane_mixed_within_tolerance(mos, ctx):
    case = W.small_case(nx=6, ny=5, mesh=(4, 4, 6), interp=(3, 3, 4), pitch_x=3.0, pitch_y=3.0, height=6.0,
                        tsv_diameter=1.6, liner_thickness=0.3, seed=2)
    got, _, _ = gpu_plane(mos, ctx, case, 9, mixed=True)
    ref = oracle_plane(case, 9)
    assert rel_max(got, ref) < 1e-3


def test_odd_layers_matching_grid_equals_centroid_output(mos, ctx):
    # g = m_x = m_y with odd m_z: the samples are the centroids of the middle
    # layer, so the plane output equals mos_reconstruct's for that layer.
    import torch
    case = W.small_case(nx=4, ny=3, mesh=(4, 4, 5), interp=(3, 3, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                        tsv_diameter=1.6, seed=4)
    got, sol, roms = gpu_plane(mos, ctx, case, 4)
    vm = torch.empty((case.n_cells, 80), dtype=torch.float64, device="cuda")
    mos.mos_reconstruct(ctx, sol, vm=vm)
    layer = vm.cpu().numpy().reshape(case.n_cells, 5, 16)[:, 2, :]
    assert np.abs(got - layer).max() <= 1e-12 * np.abs(layer).max()


def test_grid_changes_and_bad_arguments(mos, ctx):
    import torch
    case = W.small_case(nx=3, ny=3, mesh=(4, 4, 6), interp=(3, 3, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                        tsv_diameter=1.6, seed=6)
    a, sol, roms = gpu_plane(mos, ctx, case, 3)
    b = torch.empty((case.n_cells, 25), dtype=torch.float64, device="cuda")
    mos.mos_reconstruct_plane(ctx, sol, 5, b)
    c = torch.empty((case.n_cells, 9), dtype=torch.float64, device="cuda")
    mos.mos_reconstruct_plane(ctx, sol, 3, c)
    assert np.array_equal(a, c.cpu().numpy())
    assert rel_max(b.cpu().numpy(), oracle_plane(case, 5)) < 1e-9
    # The library itself rejects grids outside [1, 256] (called through the
    # C ABI directly, past the binding's shape check).
    import ctypes
    for bad in (0, 257):
        st = mos.lib().mos_reconstruct_plane(ctx.ptr, sol.ptr, bad, ctypes.c_void_p(b.data_ptr()))
        assert st == mos.MOS_EINVAL


@pytest.mark.slow
def test_plane_c2_full_size(mos, ctx):
    # 16x16 array of 16x16x32 cells, cubic faces, the paper's 100 x 100 grid:
    # the oracle evaluates sampled cells from the GPU's FP64 solution; the
    # mixed path must agree with the FP64 path over every point.
    import torch
    case = W.case_c2(0)
    g = 100
    print(f"[plane] {case.name} grid {g}", flush=True)
    got, sol, roms = gpu_plane(mos, ctx, case, g)
    u, _, _ = mos.mos_get_solution(sol)
    oroms = [oracle_rom(s) for s in case.specs]
    sp = case.specs[0]
    mesh = oarray.AbstractMesh(case.nx_cells, case.ny_cells, sp.interp, sp.pitch_x, sp.pitch_y, sp.height)
    cells = np.array([0, 17, 100, 255])
    sub_t = case.cell_type[cells]
    # Oracle evaluation of the sampled cells only (their rows of the array).
    ref = np.stack([
        oplane.plane_von_mises(_OneCell(mesh, c), sub_t[i:i + 1], oroms, u, case.delta_T, g)[0]
        for i, c in enumerate(cells)])
    assert rel_max(got[cells], ref) < 1e-9
    got32, _, _ = gpu_plane(mos, ctx, case, g, mixed=True, roms=roms)
    err = rel_max(got32, got)
    nmae = oplane.normalized_mae(got32, got)
    print(f"[plane] mixed vs fp64 on the plane: max {err:.3e}, normalised MAE {nmae:.3e}", flush=True)
    assert err <= 1e-3


class _OneCell:
    """View of an abstract mesh restricted to one block (for the oracle's
    per-block evaluation of a sampled cell)."""

    def __init__(self, mesh, cell):
        self._dofs = mesh.cell_dofs()[cell:cell + 1]
        self.n_cells = 1

    def cell_dofs(self):
        return self._dofs
