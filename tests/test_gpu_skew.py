"""Skewed (parallelepiped) blocks on the GPU: the rhombic unit block of a
120-degree TSV array (Sec. 4.2 names 120-degree arrays; x += skew * y).  The
material map, CSR pattern, numbering and node coordinates bit for bit
against the oracle, K and b within 1e-13, the reduced model within
1e-11 / 1e-10; arrays with dummy blocks, clamped or carrying a Fourier field
on all outer faces, against the oracle's direct solve -- FP64 displacements
within 1e-10 and von Mises within 1e-9, mixed precision within 1e-3 --
including the 120-degree workload's 16x14x32 block; the evaluation plane
and ROMs of different skew in one array are refused."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import array as oarray
from oracle import fem as ofem
from oracle import mor as omor

pytestmark = pytest.mark.gpu

SMALL = W.CellSpec(pitch_x=3.0, pitch_y=3.0 * math.sqrt(3.0) / 2.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 4),
                   tsv_diameter=1.6, liner_thickness=0.3, skew=1.0 / math.sqrt(3.0))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos
    return mos, mos.Context(0), torch


def rel_max(a, b, floor=0.0):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


@pytest.mark.parametrize("spec", [SMALL, W.hex_spec(), W.CellSpec(pitch_x=3.0, pitch_y=2.5, height=6.0,
                                                                 mesh=(7, 5, 4), tsv_diameter=2.2, skew=-0.4)],
                         ids=["small_120", "hex_cell", "negative_skew"])
def test_skewed_cell_assembly(env, spec):
    mos, ctx, torch = env
    cell = mos.mos_build_cell(ctx, spec)
    indptr, indices, data, b, mat = mos.mos_cell_export(cell)
    K, b_ref, mats = ofem.assemble_cell(ofem.Cell(spec))
    np.testing.assert_array_equal(mat, mats)
    np.testing.assert_array_equal(indptr, K.indptr)
    np.testing.assert_array_equal(indices, K.indices)
    assert rel_max(data, K.data) < 1e-13
    assert rel_max(b, b_ref) < 1e-13


@pytest.mark.parametrize("spec", [SMALL, W.hex_spec()], ids=["small_120", "hex_cell"])
def test_skewed_reduction(env, spec):
    mos, ctx, torch = env
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
    phi, fT, Kr, br = mos.mos_rom_export(rom)
    ref = omor.local_stage(spec)
    assert rel_max(phi, ref.Phi) < 1e-11
    assert rel_max(fT, ref.fT, floor=1e-5) < 1e-11
    assert rel_max(Kr, ref.Kr) < 1e-10
    assert rel_max(br, ref.br) < 1e-10


def test_skewed_layout_matches_oracle(env):
    mos, ctx, torch = env
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, SMALL))
    coords, conn, indptr, indices = mos.mos_array_layout(ctx, 4, 3, rom, pattern=True)
    m = oarray.AbstractMesh(4, 3, SMALL.interp, SMALL.pitch_x, SMALL.pitch_y, SMALL.height, skew=SMALL.skew)
    assert np.array_equal(coords, m.coords)
    assert np.array_equal(conn, m.conn)
    ip, ix = m.csr_pattern()
    assert np.array_equal(indptr, ip) and np.array_equal(indices, ix)


def solve_and_compare(env, specs, nx, ny, t, dT, top=False, field=None):
    mos, ctx, torch = env
    s = specs[0]
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, x)) for x in specs]
    oroms = [omor.local_stage(x) for x in specs]
    mesh = oarray.AbstractMesh(nx, ny, s.interp, s.pitch_x, s.pitch_y, s.height, skew=s.skew)
    kw = dict(clamp_bottom=field is None, clamp_top=top)
    pd = pv = None
    od, ov = (), ()
    if field is not None:
        # Outer nodes by lattice position (the numbering is checked bit for
        # bit); values at each side's own coordinates.
        outer = np.nonzero(mesh.outer_node_mask())[0]
        coords, _, _, _ = mos.mos_array_layout(ctx, nx, ny, roms[0])
        pd = od = (3 * outer[:, None] + np.arange(3)[None, :]).ravel()
        pv = field(coords[outer]).ravel()
        ov = field(mesh.coords[outer]).ravel()
    dofs, vals = oarray.constrained_dofs(mesh, field is None, top, od, ov)
    u_ref = oarray.solve_mor(mesh, t, oroms, dT, dofs, vals)
    vm_ref = ofem.von_mises(oarray.reconstruct(mesh, t, oroms, u_ref, dT))
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    for mixed in (False, True):
        sol = mos.mos_solve_array(ctx, roms, nx, ny, t, dT, mixed=mixed, prescribed_dofs=pd, prescribed_values=pv,
                                  **kw)
        vm = torch.full((nx * ny, n_elem), float("nan"), dtype=torch.float32 if mixed else torch.float64,
                        device="cuda")
        mos.mos_reconstruct(ctx, sol, vm=vm)
        u, res, it = mos.mos_get_solution(sol)
        vm = vm.double().cpu().numpy()
        e_u, e_vm = rel_max(u, u_ref), rel_max(vm, vm_ref)
        print(f"[skew {nx}x{ny} {'mixed' if mixed else 'fp64'}] iters {it} u {e_u:.2e} vm {e_vm:.2e}", flush=True)
        if mixed:
            assert res <= 1e-10 and e_vm <= 1e-3
        else:
            assert res <= 1e-12 and e_u <= 1e-10 and e_vm <= 1e-9


@pytest.mark.parametrize("shape,top", [((3, 2), False), ((4, 3), True), ((7, 5), False)],
                         ids=["3x2-bottom", "4x3-both", "7x5-bottom"])
def test_skewed_array_matches_oracle(env, shape, top):
    nx, ny = shape
    rng = np.random.default_rng(nx * ny)
    solve_and_compare(env, [SMALL, SMALL.dummy()], nx, ny, W.dummy_map(rng, nx * ny, 0.3),
                      float(rng.uniform(-300.0, -150.0)), top)


def test_skewed_array_with_fourier_field_matches_oracle(env):
    rng = np.random.default_rng(11)
    field = W.fourier_field(rng, (4 * SMALL.pitch_x, 3 * SMALL.pitch_y, SMALL.height), amplitude=0.01)
    solve_and_compare(env, [SMALL, SMALL.dummy()], 4, 3, W.dummy_map(rng, 12, 0.25), -250.0, field=field)


def test_120_degree_workload_block_matches_oracle(env):
    rng = np.random.default_rng(4)
    spec = W.hex_spec()
    solve_and_compare(env, [spec, spec.dummy()], 4, 4, W.dummy_map(rng, 16, 0.2), -250.0)


def test_plane_and_mixed_skew_are_refused(env):
    mos, ctx, torch = env
    from dataclasses import replace
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, SMALL))
    sol = mos.mos_solve_array(ctx, [rom], 2, 2, np.zeros(4, dtype=np.uint8), -250.0)
    vm = torch.empty((4, 100), dtype=torch.float64, device="cuda")
    with pytest.raises(mos.MosError) as e:
        mos.mos_reconstruct_plane(ctx, sol, 10, vm)
    assert e.value.status == mos.MOS_EINVAL
    other = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, replace(SMALL, skew=0.0)))
    with pytest.raises(mos.MosError) as e:
        mos.mos_solve_array(ctx, [rom, other], 2, 2, np.array([0, 1, 0, 1], dtype=np.uint8), -250.0)
    assert e.value.status == mos.MOS_EINVAL
    with pytest.raises(mos.MosError) as e:
        mos.mos_build_cell(ctx, replace(SMALL, skew=float("nan")))
    assert e.value.status == mos.MOS_EINVAL
