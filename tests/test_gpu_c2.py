"""Parity at the 16x16 workload's own size (Sec. 4.3, eq. 20 and the
reconstruction that follows it): 16x16 arrays of 15x15x50 um cells meshed
16x16x32 with cubic face interpolation (n = 168), dT = -250 K, bottom clamped,
the via diameter drawn per run from {4, 5, 6} um (seeds 11, 1 and 0 draw 4, 5
and 6).

Each array's reduced system (22,668 DoFs) is small enough for the oracle's
direct solve, so every array is compared element by element:

* FP64 reduced displacements within 1e-10 of the oracle's (relative to its
  max norm) and FP64 centroid von Mises within 1e-9;
* the mixed-precision path (FP32 PCG with FP64 refinement, BF16-split
  reconstruction) within 1e-3 on von Mises;

both through ``mos_solve_array`` and through one engine batch that holds the
three arrays twice over, so the batched kernels run at n = 168 and at a
batch shape; and every array's bits are the same alone and in the batch.
"""
import numpy as np
import pytest

import workloads as W
from oracle import array as oarray
from oracle import fem as ofem
from oracle import mor as omor

pytestmark = pytest.mark.gpu

SEEDS = {4.0: 11, 5.0: 1, 6.0: 0}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_12690_amd import mos
    ctx = mos.Context(0)
    cases = {d: W.case_c2(s) for d, s in SEEDS.items()}
    for d, c in cases.items():
        assert c.specs[0].tsv_diameter == d
    roms = {d: mos.mos_reduce(ctx, mos.mos_build_cell(ctx, c.specs[0])) for d, c in cases.items()}
    return mos, ctx, torch, cases, roms


_ORACLE = {}


def oracle(case):
    """The oracle's direct solve and centroid von Mises of one array (local
    stage included; cached per diameter)."""
    d = case.specs[0].tsv_diameter
    if d not in _ORACLE:
        sp = case.specs[0]
        orom = omor.local_stage(sp)
        mesh = oarray.AbstractMesh(case.nx_cells, case.ny_cells, sp.interp, sp.pitch_x, sp.pitch_y, sp.height)
        dofs, vals = oarray.constrained_dofs(mesh, True, False)
        u = oarray.solve_mor(mesh, case.cell_type, [orom], case.delta_T, dofs, vals)
        vm = ofem.von_mises(oarray.reconstruct(mesh, case.cell_type, [orom], u, case.delta_T))
        _ORACLE[d] = (u, vm)
    return _ORACLE[d]


def rel_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.mark.parametrize("d", [4.0, 5.0, 6.0], ids=["d4", "d5", "d6"])
def test_solve_array_matches_oracle(env, d):
    mos, ctx, torch, cases, roms = env
    case = cases[d]
    u_ref, vm_ref = oracle(case)
    n_elem = roms[d].query(mos.MOS_Q_CELL_ELEMS)
    assert roms[d].query(mos.MOS_Q_N) == 168
    for mixed in (False, True):
        sol = mos.mos_solve_array(ctx, [roms[d]], case.nx_cells, case.ny_cells, case.cell_type, case.delta_T,
                                  clamp_bottom=True, mixed=mixed)
        vm = torch.full((case.n_cells, n_elem), float("nan"), dtype=torch.float32 if mixed else torch.float64,
                        device="cuda")
        mos.mos_reconstruct(ctx, sol, vm=vm)
        torch.cuda.synchronize()
        u, res, iters = mos.mos_get_solution(sol)
        vm = vm.double().cpu().numpy()
        e_u, e_vm = rel_max(u, u_ref), rel_max(vm, vm_ref)
        print(f"[c2 d={d:g} {'mixed' if mixed else 'fp64'}] iters {iters} residual {res:.2e} "
              f"u {e_u:.2e} vm {e_vm:.2e}", flush=True)
        if mixed:
            assert res <= 1e-10
            assert e_vm <= 1e-3
        else:
            assert res <= 1e-12
            assert e_u <= 1e-10
            assert e_vm <= 1e-9


def run_batch(env, ds, mixed):
    """One engine batch of the arrays of diameters `ds` (in that order);
    returns (status, residual, iterations, vm, u) per array."""
    mos, ctx, torch, cases, roms = env
    order = [4.0, 5.0, 6.0]
    eng = mos.Engine(ctx, [roms[d] for d in order], mixed=mixed, device_bytes=2 << 30)
    n_elem = roms[4.0].query(mos.MOS_Q_CELL_ELEMS)
    outs = {}
    for i, d in enumerate(ds):
        c = cases[d]
        t = np.full(c.n_cells, order.index(d), dtype=np.uint8)
        vm = torch.full((c.n_cells, n_elem), float("nan"), dtype=torch.float32 if mixed else torch.float64,
                        device="cuda")
        u = torch.full((22668,), float("nan"), dtype=torch.float64, device="cuda")
        outs[eng.submit(c.nx_cells, c.ny_cells, t, c.delta_T, vm=vm, u=u)] = (i, vm, u)
    done = {}
    rounds = 0
    while len(done) < len(ds):
        for tk in eng.progress(16):
            i, vm, u = outs[tk]
            st, rel, it, sw = eng.result(tk)
            torch.cuda.synchronize()
            done[i] = (st, rel, it, vm.double().cpu().numpy(), u.cpu().numpy())
        rounds += 1
        assert rounds < 2000
    eng.close()
    return [done[i] for i in range(len(ds))]


BATCH = [4.0, 5.0, 6.0, 6.0, 5.0, 4.0]


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_engine_batch_matches_oracle_and_alone(env, mixed):
    mos, ctx, torch, cases, roms = env
    mix = run_batch(env, BATCH, mixed)
    for d, (st, rel, it, vm, u) in zip(BATCH, mix):
        u_ref, vm_ref = oracle(cases[d])
        e_u, e_vm = rel_max(u, u_ref), rel_max(vm, vm_ref)
        print(f"[c2 batch d={d:g} {'mixed' if mixed else 'fp64'}] iters {it} residual {rel:.2e} "
              f"u {e_u:.2e} vm {e_vm:.2e}", flush=True)
        assert st == 0
        if mixed:
            assert rel <= 1e-10 and e_vm <= 1e-3
        else:
            assert rel <= 1e-12 and e_u <= 1e-10 and e_vm <= 1e-9
    # Equal inputs give equal bits wherever they sit in the batch, and the
    # same bits as a batch of one.
    for a, b in ((0, 5), (1, 4), (2, 3)):
        assert np.array_equal(mix[a][4], mix[b][4]) and np.array_equal(mix[a][3], mix[b][3])
    for i in (0, 1, 2):
        alone = run_batch(env, [BATCH[i]], mixed)[0]
        assert alone[2] == mix[i][2]
        assert np.array_equal(alone[4], mix[i][4]), "reduced displacement differs"
        assert np.array_equal(alone[3], mix[i][3]), "von Mises differs"
