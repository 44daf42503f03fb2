"""Stacked layers of blocks on the GPU (the abstract mesh of Sec. 4.3 with a
z index of blocks; each block's reduced model is unchanged): the library's
numbering and coordinates against the oracle's bit for bit, and the solve
and reconstruction of small stacks against the oracle's direct solve --
FP64 displacements within 1e-10 and von Mises within 1e-9, mixed precision
within 1e-3 on von Mises -- through mos_solve_array and through an engine
batch that mixes stacks with one-layer arrays (every problem's bits the same
alone and in the batch).  A two-level engine rejects a stacked array."""
import numpy as np
import pytest

import workloads as W
from oracle import array as oarray
from oracle import fem as ofem
from oracle import mor as omor

pytestmark = pytest.mark.gpu

SPEC = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 4), tsv_diameter=1.6,
                  liner_thickness=0.3)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos
    ctx = mos.Context(0)
    specs = [SPEC, SPEC.dummy()]
    roms = [mos.mos_reduce(ctx, mos.mos_build_cell(ctx, s)) for s in specs]
    oroms = [omor.local_stage(s) for s in specs]
    return mos, ctx, roms, oroms, torch


def oracle_solution(oroms, nx, ny, nz, t, dT, top=False):
    mesh = oarray.AbstractMesh(nx, ny, SPEC.interp, SPEC.pitch_x, SPEC.pitch_y, SPEC.height, nz_cells=nz)
    dofs, vals = oarray.constrained_dofs(mesh, True, top)
    u = oarray.solve_mor(mesh, t, oroms, dT, dofs, vals)
    vm = ofem.von_mises(oarray.reconstruct(mesh, t, oroms, u, dT))
    return u, vm


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 3), (1, 1, 4), (5, 3, 2)], ids=lambda s: "x".join(map(str, s)))
def test_layout_matches_oracle(env, shape):
    mos, ctx, roms, oroms, torch = env
    nx, ny, nz = shape
    coords, conn, indptr, indices = mos.mos_array_layout(ctx, nx, ny, roms[0], pattern=True, nz_cells=nz)
    mesh = oarray.AbstractMesh(nx, ny, SPEC.interp, SPEC.pitch_x, SPEC.pitch_y, SPEC.height, nz_cells=nz)
    assert coords.shape[0] == mesh.n_nodes
    assert np.array_equal(coords, mesh.coords)
    assert np.array_equal(conn, mesh.conn)
    ip, ix = mesh.csr_pattern()
    assert np.array_equal(indptr, ip) and np.array_equal(indices, ix)


@pytest.mark.parametrize("shape,top", [((2, 2, 2), False), ((3, 2, 3), True), ((1, 1, 4), False),
                                       ((4, 3, 2), False)], ids=["2x2x2", "3x2x3-top", "1x1x4", "4x3x2"])
def test_stacked_solve_matches_oracle(env, shape, top):
    mos, ctx, roms, oroms, torch = env
    nx, ny, nz = shape
    rng = np.random.default_rng(sum(shape))
    t = W.dummy_map(rng, nx * ny * nz, 0.3)
    dT = float(rng.uniform(-300.0, -150.0))
    u_ref, vm_ref = oracle_solution(oroms, nx, ny, nz, t, dT, top)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    for mixed in (False, True):
        sol = mos.mos_solve_array(ctx, roms, nx, ny, t, dT, clamp_bottom=True, clamp_top=top, mixed=mixed,
                                  nz_cells=nz)
        vm = torch.full((nx * ny * nz, n_elem), float("nan"), dtype=torch.float32 if mixed else torch.float64,
                        device="cuda")
        mos.mos_reconstruct(ctx, sol, vm=vm)
        u, res, it = mos.mos_get_solution(sol)
        vm = vm.double().cpu().numpy()
        e_u, e_vm = rel_max(u, u_ref), rel_max(vm, vm_ref)
        print(f"[stacked {shape} {'mixed' if mixed else 'fp64'}] iters {it} u {e_u:.2e} vm {e_vm:.2e}", flush=True)
        if mixed:
            assert res <= 1e-10 and e_vm <= 1e-3
        else:
            assert res <= 1e-12 and e_u <= 1e-10 and e_vm <= 1e-9


def run_engine(env, probs, mixed):
    mos, ctx, roms, oroms, torch = env
    eng = mos.Engine(ctx, roms, mixed=mixed, device_bytes=1 << 28, precond=0)
    n_elem = roms[0].query(mos.MOS_Q_CELL_ELEMS)
    outs = {}
    for i, (nx, ny, nz, t, dT) in enumerate(probs):
        coords, _, _, _ = mos.mos_array_layout(ctx, nx, ny, roms[0], nz_cells=nz)
        vm = torch.full((nx * ny * nz, n_elem), float("nan"), dtype=torch.float32 if mixed else torch.float64,
                        device="cuda")
        u = torch.full((3 * coords.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
        outs[eng.submit(nx, ny, t, dT, vm=vm, u=u, nz_cells=nz)] = (i, vm, u)
    done = {}
    rounds = 0
    while len(done) < len(probs):
        for tk in eng.progress(16):
            i, vm, u = outs[tk]
            st, rel, it, sw = eng.result(tk)
            done[i] = (st, rel, it, vm.double().cpu().numpy(), u.cpu().numpy())
        rounds += 1
        assert rounds < 5000
    eng.close()
    return [done[i] for i in range(len(probs))]


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_engine_batch_of_stacks_and_layers(env, mixed):
    mos, ctx, roms, oroms, torch = env
    rng = np.random.default_rng(5)
    probs = []
    for nx, ny, nz in ((3, 2, 2), (2, 2, 1), (4, 3, 3), (5, 1, 1), (2, 3, 2)):
        probs.append((nx, ny, nz, W.dummy_map(rng, nx * ny * nz, 0.3), float(rng.uniform(-300.0, -150.0))))
    mix = run_engine(env, probs, mixed)
    for (nx, ny, nz, t, dT), (st, rel, it, vm, u) in zip(probs, mix):
        assert st == 0
        u_ref, vm_ref = oracle_solution(oroms, nx, ny, nz, t, dT)
        if mixed:
            assert rel <= 1e-10 and rel_max(vm, vm_ref) <= 1e-3
        else:
            assert rel <= 1e-12 and rel_max(u, u_ref) <= 1e-10 and rel_max(vm, vm_ref) <= 1e-9
    for i in (0, 1, 2):
        alone = run_engine(env, [probs[i]], mixed)[0]
        assert alone[2] == mix[i][2]
        assert np.array_equal(alone[4], mix[i][4]), "reduced displacement differs"
        assert np.array_equal(alone[3], mix[i][3]), "von Mises differs"


def test_two_level_engine_rejects_a_stack(env):
    mos, ctx, roms, oroms, torch = env
    eng = mos.Engine(ctx, roms, device_bytes=1 << 26, precond=1)
    with pytest.raises(mos.MosError) as e:
        eng.submit(2, 2, np.zeros(8, dtype=np.uint8), -250.0, nz_cells=2)
    assert e.value.status == mos.MOS_EINVAL
    eng.close()
