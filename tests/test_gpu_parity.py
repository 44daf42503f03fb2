"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances:
* integer work (material map, CSR pattern, abstract-mesh numbering,
  connectivity, global sparsity): bit-exact;
* cell K and b: 1e-13 of the largest entry (sums of <= 8 element terms in a
  different order);
* Phi, f_T: 1e-11 of the largest entry, K_r, b_r: 1e-10 of the largest entry
  (two backward-stable direct solves of K_ff differ by about kappa(K_ff)
  * eps; K_r is a Galerkin projection, so its error is second order in the
  Phi error plus the local residual);
* FP64 displacements: 1e-10 relative in the max norm (the reduced system has
  kappa ~ 1e3, so K_r differences of 1e-13 move u by ~1e-10 at most);
* FP64 stress: 1e-9 of the largest von Mises value;
* mixed precision (FP32 PCG + FP64 refinement, bf16 reconstruction):
  1e-3 of the largest von Mises value.
"""
import numpy as np
import pytest

import workloads as W
from oracle import array as oarray
from oracle import fem as ofem
from oracle import mor as omor

pytestmark = pytest.mark.gpu

SPEC_SMALL = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 4),
                        tsv_diameter=1.6, liner_thickness=0.3)


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


def rel_max(a, b, floor=1e-300):
    """Max-norm difference relative to the reference's max norm (or `floor`
    when the reference is identically small)."""
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), floor)


@pytest.mark.parametrize("spec", [SPEC_SMALL, W.case_c1().specs[0],
                                  W.CellSpec(mesh=(16, 16, 32), tsv_diameter=6.0)],
                         ids=["small_liner", "c1_cell", "c2_cell_d6"])
def test_cell_assembly(mos, ctx, spec):
    cell = mos.mos_build_cell(ctx, spec)
    indptr, indices, data, b, mat = mos.mos_cell_export(cell)
    oc = ofem.Cell(spec)
    K, b_ref, mats = ofem.assemble_cell(oc)
    np.testing.assert_array_equal(mat, mats)
    np.testing.assert_array_equal(indptr, K.indptr)
    np.testing.assert_array_equal(indices, K.indices)
    assert rel_max(data, K.data) < 1e-13
    assert rel_max(b, b_ref) < 1e-13
    assert cell.query(mos.MOS_Q_FREE_DOFS) == 3 * (oc.mx - 1) * (oc.my - 1) * (oc.mz - 1)


@pytest.mark.parametrize("spec", [SPEC_SMALL, W.case_c1().specs[0], SPEC_SMALL.dummy(),
                                  # The benchmark cell: 28,611 DoFs, many band tiles, and
                                  # n + 1 = 169 right-hand sides (a ragged 16-column slab).
                                  W.CellSpec(mesh=(16, 16, 32), tsv_diameter=6.0),
                                  # One interior node: a single band tile and no off-diagonal ones.
                                  W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(2, 2, 2),
                                             interp=(3, 3, 3), tsv_diameter=1.6)],
                         ids=["small_liner", "c1_cell", "small_dummy", "c2_cell_d6", "one_tile"])
def test_reduction(mos, ctx, spec):
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
    phi, fT, Kr, br = mos.mos_rom_export(rom)
    ref = oracle_rom(spec)
    assert rom.query(mos.MOS_Q_N) == ref.n
    assert rel_max(phi, ref.Phi) < 1e-11
    # f_T is exactly 0 for a homogeneous block; its natural scale is the free
    # thermal displacement alpha * height per kelvin (~1e-5 um/K).
    assert rel_max(fT, ref.fT, floor=1e-5) < 1e-11
    assert rel_max(Kr, ref.Kr) < 1e-10
    assert rel_max(br, ref.br) < 1e-10
    assert np.array_equal(Kr, Kr.T)


@pytest.mark.parametrize("N,interp", [((3, 2), (3, 3, 4)), ((1, 1), (3, 3, 4)), ((5, 4), (4, 3, 3))])
def test_array_layout(mos, ctx, N, interp):
    spec = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=interp, tsv_diameter=1.6)
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
    coords, conn, indptr, indices = mos.mos_array_layout(ctx, N[0], N[1], rom, pattern=True)
    m = oarray.AbstractMesh(N[0], N[1], interp, 3.0, 3.0, 6.0)
    np.testing.assert_array_equal(conn, m.conn)
    np.testing.assert_array_equal(coords, m.coords)
    ip, ix = m.csr_pattern()
    np.testing.assert_array_equal(indptr, ip)
    np.testing.assert_array_equal(indices, ix)


def run_both(mos, ctx, case, mixed=False, vm_out=True, sigma=True):
    import torch
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in case.specs]
    sol = mos.mos_solve_array(ctx, roms, case.nx_cells, case.ny_cells, case.cell_type, case.delta_T,
                              clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top, mixed=mixed)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    dt = torch.float32 if mixed else torch.float64
    vm = torch.full((case.n_cells, n_elem), np.nan, dtype=dt, device="cuda") if vm_out else None
    s6 = torch.full((case.n_cells, n_elem, 6), np.nan, dtype=dt, device="cuda") if sigma else None
    mos.mos_reconstruct(ctx, sol, vm=vm, sigma6=s6)
    u, res, iters = mos.mos_get_solution(sol)
    oroms = [oracle_rom(s) for s in case.specs]
    sp = case.specs[0]
    mesh = oarray.AbstractMesh(case.nx_cells, case.ny_cells, sp.interp, sp.pitch_x, sp.pitch_y, sp.height)
    dofs, vals = oarray.constrained_dofs(mesh, case.clamp_bottom, case.clamp_top)
    u_ref = oarray.solve_mor(mesh, case.cell_type, oroms, case.delta_T, dofs, vals)
    sig_ref = oarray.reconstruct(mesh, case.cell_type, oroms, u_ref, case.delta_T)
    out = dict(u=u, u_ref=u_ref, res=res, iters=iters, sig_ref=sig_ref, vm_ref=ofem.von_mises(sig_ref))
    out["vm"] = vm.cpu().numpy().astype(np.float64) if vm_out else None
    out["sig"] = s6.cpu().numpy().astype(np.float64) if sigma else None
    return out


@pytest.mark.parametrize("case", [
    W.small_case(nx=3, ny=2, mesh=(4, 4, 6), interp=(3, 3, 4), pitch_x=3.0, pitch_y=3.0, height=6.0,
                 tsv_diameter=1.6, liner_thickness=0.3),
    W.small_case(nx=1, ny=1, mesh=(4, 4, 6), interp=(3, 3, 3), dummies=False, pitch_x=3.0, pitch_y=3.0,
                 height=6.0, tsv_diameter=1.6),
    W.small_case(nx=7, ny=5, mesh=(4, 4, 6), interp=(4, 4, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                 tsv_diameter=1.6, seed=3),
    W.case_c1(),
], ids=["3x2_two_types", "1x1", "7x5_ragged", "c1"])
def test_solve_and_reconstruct_fp64(mos, ctx, case):
    r = run_both(mos, ctx, case)
    assert r["res"] <= 1e-12
    assert rel_max(r["u"], r["u_ref"]) < 1e-10
    assert rel_max(r["vm"], r["vm_ref"]) < 1e-9
    assert rel_max(r["sig"], r["sig_ref"]) < 1e-9


def test_clamped_top_and_bottom(mos, ctx):
    case = W.small_case(nx=4, ny=3, mesh=(4, 4, 6), interp=(3, 3, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                        tsv_diameter=1.6, seed=5)
    case.clamp_top = True
    r = run_both(mos, ctx, case, sigma=False)
    assert rel_max(r["u"], r["u_ref"]) < 1e-10
    assert rel_max(r["vm"], r["vm_ref"]) < 1e-9


def test_mixed_precision_small(mos, ctx):
    case = W.small_case(nx=6, ny=5, mesh=(4, 4, 6), interp=(3, 3, 4), pitch_x=3.0, pitch_y=3.0, height=6.0,
                        tsv_diameter=1.6, liner_thickness=0.3, seed=2)
    r = run_both(mos, ctx, case, mixed=True)
    assert r["res"] <= 1e-10
    assert rel_max(r["u"], r["u_ref"]) < 1e-8
    assert rel_max(r["vm"], r["vm_ref"]) < 1e-3


def test_repeat_runs_are_bitwise_identical(mos, ctx):
    case = W.small_case(nx=5, ny=4, mesh=(4, 4, 6), interp=(3, 3, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                        tsv_diameter=1.6, seed=7)
    a = run_both(mos, ctx, case, sigma=False)
    b = run_both(mos, ctx, case, sigma=False)
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["vm"], b["vm"])


def test_error_codes(mos, ctx):
    spec = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 3), tsv_diameter=1.6)
    with pytest.raises(mos.MosError) as e:
        mos.mos_build_cell(ctx, W.CellSpec(mesh=(1, 4, 4)))
    assert e.value.status == mos.MOS_EINVAL
    with pytest.raises(mos.MosError) as e:
        mos.mos_build_cell(ctx, W.CellSpec(matrix=(130e3, 0.5, 2.6e-6)))
    assert e.value.status == mos.MOS_EINVAL
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
    with pytest.raises(mos.MosError) as e:
        mos.mos_solve_array(ctx, [rom], 2, 2, np.zeros(4), -250.0, clamp_bottom=False)
    assert e.value.status == mos.MOS_ESINGULAR
    with pytest.raises(mos.MosError) as e:
        mos.mos_solve_array(ctx, [rom], 2, 2, np.array([0, 1, 0, 0]), -250.0)
    assert e.value.status == mos.MOS_EINVAL
    with pytest.raises(mos.MosError) as e:
        mos.mos_solve_array(ctx, [rom], 3, 3, np.zeros(9), -250.0, max_iters=2)
    assert e.value.status == mos.MOS_ENOCONV
    with pytest.raises(mos.MosError) as e:
        mos.mos_solve_array(ctx, [rom], 2, 2, np.zeros(4), -250.0, prescribed_dofs=[10 ** 9],
                            prescribed_values=[0.0])
    assert e.value.status == mos.MOS_EINVAL
    other = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, W.CellSpec(pitch_x=4.0, pitch_y=3.0, height=6.0,
                                                                   mesh=(4, 4, 6), interp=(3, 3, 3))))
    with pytest.raises(mos.MosError) as e:
        mos.mos_solve_array(ctx, [rom, other], 2, 2, np.zeros(4), -250.0)
    assert e.value.status == mos.MOS_EINVAL


def test_zero_load_gives_zero_solution(mos, ctx):
    spec = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 3), tsv_diameter=1.6)
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
    sol = mos.mos_solve_array(ctx, [rom], 2, 3, np.zeros(6), 0.0)
    u, res, iters = mos.mos_get_solution(sol)
    assert np.all(u == 0.0) and iters == 0


@pytest.mark.parametrize("case,mixed", [
    (W.small_case(nx=3, ny=2, mesh=(4, 4, 6), interp=(3, 3, 4), pitch_x=3.0, pitch_y=3.0, height=6.0,
                  tsv_diameter=1.6, liner_thickness=0.3), False),
    (W.small_case(nx=7, ny=5, mesh=(4, 4, 6), interp=(4, 4, 3), pitch_x=3.0, pitch_y=3.0, height=6.0,
                  tsv_diameter=1.6, seed=3), False),
    (W.case_c1(), False),
    (W.small_case(nx=6, ny=5, mesh=(4, 4, 6), interp=(3, 3, 4), pitch_x=3.0, pitch_y=3.0, height=6.0,
                  tsv_diameter=1.6, liner_thickness=0.3, seed=2), True),
], ids=["3x2_two_types", "7x5_ragged", "c1", "6x5_mixed"])
def test_nodal_displacement(mos, ctx, case, mixed):
    # eq. 15 per cell, dT f_T + Phi u_cell, against the oracle's; 525 FE DoFs
    # per 4x4x6 cell leave a ragged last tile of 16 DoFs.
    import torch
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in case.specs]
    sol = mos.mos_solve_array(ctx, roms, case.nx_cells, case.ny_cells, case.cell_type, case.delta_T,
                              clamp_bottom=case.clamp_bottom, clamp_top=case.clamp_top, mixed=mixed)
    n_fe = roms[0].query(mos.MOS_Q_CELL_DOFS)
    out = torch.full((case.n_cells, n_fe), np.nan, dtype=torch.float64, device="cuda")
    mos.mos_reconstruct_displacement(ctx, sol, out)
    got = out.cpu().numpy()
    oroms = [oracle_rom(s) for s in case.specs]
    sp = case.specs[0]
    mesh = oarray.AbstractMesh(case.nx_cells, case.ny_cells, sp.interp, sp.pitch_x, sp.pitch_y, sp.height)
    dofs, vals = oarray.constrained_dofs(mesh, case.clamp_bottom, case.clamp_top)
    u_ref = oarray.solve_mor(mesh, case.cell_type, oroms, case.delta_T, dofs, vals)
    ref = np.stack([oarray.nodal_displacement(mesh, case.cell_type, oroms, u_ref, case.delta_T, c)
                    for c in range(case.n_cells)])
    assert np.isfinite(got).all()
    assert rel_max(got, ref) < (1e-8 if mixed else 1e-10)
    # The bottom face is clamped: its FE nodes carry exactly zero displacement.
    mz1 = (sp.mesh[0] + 1) * (sp.mesh[1] + 1)
    assert np.all(got[:, :3 * mz1] == 0.0)


@pytest.mark.parametrize("shape", [(5, 4), (16, 16)], ids=["5x4", "16x16"])
def test_bf16_reconstruction_kernels_agree_bitwise(shape):
    """The BF16-split reconstruction with two element blocks per workgroup
    and the one-block form compute the same products in the same order, so
    their outputs are bitwise equal (von Mises and the six components)."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos
    ctx = mos.Context(0)
    spec = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 7), interp=(4, 4, 4), tsv_diameter=1.6,
                      liner_thickness=0.3)
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in (spec, spec.dummy())]
    nx, ny = shape
    t = W.dummy_map(np.random.default_rng(4), nx * ny, 0.3)
    sol = mos.mos_solve_array(ctx, roms, nx, ny, t, -250.0, clamp_bottom=True, mixed=True)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    outs = []
    for v in ("1", "2"):
        os.environ["MOS_RECON_BF16"] = v
        try:
            vm = torch.full((nx * ny, n_elem), float("nan"), dtype=torch.float32, device="cuda")
            s6 = torch.full((nx * ny, n_elem, 6), float("nan"), dtype=torch.float32, device="cuda")
            mos.mos_reconstruct(ctx, sol, vm=vm, sigma6=s6)
            torch.cuda.synchronize()
            outs.append((vm.cpu().numpy(), s6.cpu().numpy()))
        finally:
            del os.environ["MOS_RECON_BF16"]
    assert np.isfinite(outs[0][0]).all() and np.isfinite(outs[1][1]).all()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("shape", [(5, 4), (16, 16)], ids=["5x4", "16x16"])
def test_fp64_reconstruction_kernels_agree_bitwise(shape):
    """The FP64 reconstruction with the cell operand streamed in
    double-buffered chunks and the form that requests a block's whole operand
    at once run the same MFMA chains, so their outputs are bitwise equal."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos
    ctx = mos.Context(0)
    spec = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 7), interp=(4, 4, 4), tsv_diameter=1.6,
                      liner_thickness=0.3)
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in (spec, spec.dummy())]
    nx, ny = shape
    t = W.dummy_map(np.random.default_rng(6), nx * ny, 0.3)
    sol = mos.mos_solve_array(ctx, roms, nx, ny, t, -250.0, clamp_bottom=True)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    outs = []
    for v in ("1", "2"):
        os.environ["MOS_RECON_F64"] = v
        try:
            vm = torch.full((nx * ny, n_elem), float("nan"), dtype=torch.float64, device="cuda")
            s6 = torch.full((nx * ny, n_elem, 6), float("nan"), dtype=torch.float64, device="cuda")
            mos.mos_reconstruct(ctx, sol, vm=vm, sigma6=s6)
            torch.cuda.synchronize()
            outs.append((vm.cpu().numpy(), s6.cpu().numpy()))
        finally:
            del os.environ["MOS_RECON_F64"]
    assert np.isfinite(outs[0][0]).all() and np.isfinite(outs[1][1]).all()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
