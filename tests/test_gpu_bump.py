"""Micro-bump blocks on the GPU (the method applied to a second repeated fine
structure, Sec. 4.1; micro-bump arrays are named in Sec. 1): the material map
and CSR pattern bit for bit against the oracle, K and b within 1e-13, the
reduced model (Phi, f_T, K_r, b_r) within 1e-11 / 1e-10, and layers of bumps
with empty sites, clamped at one or both faces, against the oracle's direct
solve -- FP64 displacements within 1e-10 and von Mises within 1e-9, mixed
precision within 1e-3 on von Mises -- including the benchmark's 16x16x16
bump block on a 5x4 layer.  Invalid bump descriptions are refused."""
import numpy as np
import pytest

import workloads as W
from oracle import array as oarray
from oracle import fem as ofem
from oracle import mor as omor

pytestmark = pytest.mark.gpu

SMALL = W.bump_spec(pitch_x=8.0, pitch_y=8.0, height=6.0, mesh=(6, 6, 6), tsv_diameter=5.0, pad_thickness=1.2,
                    interp=(3, 3, 4))


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


@pytest.mark.parametrize("spec", [SMALL, W.bump_spec(), SMALL.dummy()], ids=["small", "bench_cell", "empty_site"])
def test_bump_cell_assembly(env, spec):
    mos, ctx, torch = env
    cell = mos.mos_build_cell(ctx, spec)
    indptr, indices, data, b, mat = mos.mos_cell_export(cell)
    K, b_ref, mats = ofem.assemble_cell(ofem.Cell(spec))
    np.testing.assert_array_equal(mat, mats)
    np.testing.assert_array_equal(indptr, K.indptr)
    np.testing.assert_array_equal(indices, K.indices)
    assert rel_max(data, K.data) < 1e-13
    assert rel_max(b, b_ref) < 1e-13


@pytest.mark.parametrize("spec", [SMALL, W.bump_spec()], ids=["small", "bench_cell"])
def test_bump_reduction(env, spec):
    mos, ctx, torch = env
    rom = mos.mos_reduce(ctx, mos.mos_build_cell(ctx, spec))
    phi, fT, Kr, br = mos.mos_rom_export(rom)
    ref = omor.local_stage(spec)
    assert rom.query(mos.MOS_Q_N) == ref.n
    assert rel_max(phi, ref.Phi) < 1e-11
    assert rel_max(fT, ref.fT, floor=1e-5) < 1e-11
    assert rel_max(Kr, ref.Kr) < 1e-10
    assert rel_max(br, ref.br) < 1e-10


def oracle_solution(specs, nx, ny, t, dT, top):
    s = specs[0]
    roms = [omor.local_stage(x) for x in specs]
    mesh = oarray.AbstractMesh(nx, ny, s.interp, s.pitch_x, s.pitch_y, s.height)
    dofs, vals = oarray.constrained_dofs(mesh, True, top)
    u = oarray.solve_mor(mesh, t, roms, dT, dofs, vals)
    return u, ofem.von_mises(oarray.reconstruct(mesh, t, roms, u, dT))


@pytest.mark.parametrize("spec,shape,top", [(SMALL, (3, 2), False), (SMALL, (4, 3), True),
                                            (W.bump_spec(), (5, 4), True)],
                         ids=["small-3x2-bottom", "small-4x3-both", "bench_cell-5x4-both"])
def test_bump_layer_matches_oracle(env, spec, shape, top):
    mos, ctx, torch = env
    nx, ny = shape
    specs = [spec, spec.dummy()]
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in specs]
    rng = np.random.default_rng(nx * ny)
    t = W.dummy_map(rng, nx * ny, 0.25)
    dT = -200.0
    u_ref, vm_ref = oracle_solution(specs, nx, ny, t, dT, top)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    for mixed in (False, True):
        sol = mos.mos_solve_array(ctx, roms, nx, ny, t, dT, clamp_bottom=True, clamp_top=top, mixed=mixed)
        vm = torch.full((nx * ny, n_elem), float("nan"), dtype=torch.float32 if mixed else torch.float64,
                        device="cuda")
        mos.mos_reconstruct(ctx, sol, vm=vm)
        u, res, it = mos.mos_get_solution(sol)
        vm = vm.double().cpu().numpy()
        e_u, e_vm = rel_max(u, u_ref), rel_max(vm, vm_ref)
        print(f"[bump {shape} top={top} {'mixed' if mixed else 'fp64'}] iters {it} u {e_u:.2e} vm {e_vm:.2e}",
              flush=True)
        if mixed:
            assert res <= 1e-10 and e_vm <= 1e-3
        else:
            assert res <= 1e-12 and e_u <= 1e-10 and e_vm <= 1e-9


@pytest.mark.parametrize("bad", [dict(structure=7), dict(liner_thickness=0.5), dict(pad_thickness=3.0),
                                 dict(pad_thickness=-1.0), dict(structure="tsv", pad_thickness=1.0)],
                         ids=["unknown_structure", "bump_with_liner", "pads_fill_height", "negative_pad",
                              "tsv_with_pads"])
def test_invalid_bump_description_is_refused(env, bad):
    mos, ctx, torch = env
    from dataclasses import replace
    spec = replace(SMALL, **bad)
    with pytest.raises(mos.MosError) as e:
        mos.mos_build_cell(ctx, spec)
    assert e.value.status == mos.MOS_EINVAL
