"""Pins of the oracle's global stage (Sec. 4.3-4.4, eq. 20) and its full-FEM
comparison: numbering and sparsity against brute force, rigid null space,
closed-form thermal states, linearity, mirror symmetry.  CPU only."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import array, fem, mor


def spec_small(interp=(3, 3, 3), d=1.6, mesh=(4, 4, 6), **kw):
    return W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=mesh, interp=interp,
                      tsv_diameter=d, **kw)


@pytest.mark.parametrize("N,interp", [((2, 2), (3, 3, 3)), ((3, 2), (4, 3, 4)), ((4, 4), (4, 4, 4)),
                                      ((16, 16), (4, 4, 4)), ((2, 3), (2, 2, 2))])
def test_node_count_closed_form(N, interp):
    Nx, Ny = N
    nx, ny, nz = interp
    m = array.AbstractMesh(Nx, Ny, interp)
    X, Y = Nx * (nx - 1) + 1, Ny * (ny - 1) + 1
    assert m.n_nodes == X * Y * nz - Nx * Ny * (nx - 2) * (ny - 2) * (nz - 2)
    assert m.conn.shape == (Nx * Ny, mor.n_reduced(nx, ny, nz) // 3)
    # every node is used, ids are dense
    assert np.array_equal(np.unique(m.conn), np.arange(m.n_nodes))


def test_neighbouring_blocks_share_face_nodes():
    m = array.AbstractMesh(3, 2, (4, 3, 3))
    S = mor.surface_nodes(4, 3, 3)
    pos = {s: i for i, s in enumerate(S)}
    for cy in range(2):
        for cx in range(2):
            a, b = cy * 3 + cx, cy * 3 + cx + 1
            for (i, j, k) in S:
                if i == 3:
                    assert m.conn[a, pos[(3, j, k)]] == m.conn[b, pos[(0, j, k)]]
    # blocks that do not touch share nothing
    assert not set(m.conn[0]) & set(m.conn[2])
    # diagonal neighbours share exactly the vertical edge: n_z nodes
    assert len(set(m.conn[0]) & set(m.conn[4])) == 3


def test_pattern_equals_brute_force_pairs():
    m = array.AbstractMesh(3, 2, (3, 3, 3))
    indptr, idx = m.csr_pattern()
    pairs = set()
    for c in range(m.n_cells):
        d = [3 * int(nd) + k for nd in m.conn[c] for k in range(3)]
        pairs.update(itertools.product(d, d))
    rows = np.repeat(np.arange(m.n_dofs), np.diff(indptr))
    assert set(zip(rows.tolist(), idx.tolist())) == pairs
    assert len(pairs) == len(idx)
    for r in range(m.n_dofs):
        assert np.all(np.diff(idx[indptr[r]:indptr[r + 1]]) > 0)


@pytest.mark.parametrize("N", [4, 5])
def test_cubic_node_pair_count(N):
    # node-pair count of the cubic abstract mesh: 2640 N^2 + 480 N + 16,
    # counted by brute force on the node sets of overlapping blocks.
    m = array.AbstractMesh(N, N, (4, 4, 4))
    indptr, _ = m.csr_pattern()
    assert (indptr[-1]) == 9 * (2640 * N * N + 480 * N + 16)


@pytest.fixture(scope="module")
def roms_small():
    s = spec_small()
    return [mor.local_stage(s), mor.local_stage(s.dummy())]


def rigid(coords):
    out = [np.tile(t, len(coords)) for t in np.eye(3)]
    out += [np.cross(np.broadcast_to(w, coords.shape), coords - 1.0).ravel() for w in np.eye(3)]
    return np.array(out).T


def test_global_matrix_has_rigid_null_space_before_bcs(roms_small):
    m = array.AbstractMesh(3, 2, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.array([0, 1, 0, 0, 1, 1], dtype=np.uint8)
    A, b = array.assemble_global(m, t, roms_small, -250.0)
    R = rigid(m.coords)
    assert np.abs(A @ R).max() < 1e-9 * np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()


def test_assembly_equals_dense_scatter(roms_small):
    m = array.AbstractMesh(2, 2, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.array([1, 0, 0, 1], dtype=np.uint8)
    A, b = array.assemble_global(m, t, roms_small, -100.0)
    Ad = np.zeros((m.n_dofs, m.n_dofs))
    bd = np.zeros(m.n_dofs)
    for c in range(4):
        P = np.zeros((roms_small[0].n, m.n_dofs))
        for s in range(m.conn.shape[1]):
            for k in range(3):
                P[3 * s + k, 3 * m.conn[c, s] + k] = 1.0
        Ad += P.T @ roms_small[t[c]].Kr @ P
        bd += P.T @ (-100.0 * roms_small[t[c]].br)
    np.testing.assert_allclose(A.toarray(), Ad, rtol=1e-14, atol=1e-9)
    np.testing.assert_allclose(b, bd, rtol=1e-13, atol=1e-12)


def test_free_expansion_of_homogeneous_array_is_stress_free():
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    m = array.AbstractMesh(3, 2, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.zeros(6, dtype=np.uint8)
    # 3-2-1 support on reduced nodes
    n0 = m.node_id[0, 0, 0]
    n1 = m.node_id[0, 0, m.X - 1]
    n2 = m.node_id[0, m.Y - 1, 0]
    dofs = [3 * n0, 3 * n0 + 1, 3 * n0 + 2, 3 * n1 + 1, 3 * n1 + 2, 3 * n2 + 2]
    dT = -250.0
    u = array.solve_mor(m, t, [rom], dT, np.array(dofs), np.zeros(6))
    np.testing.assert_allclose(u.reshape(-1, 3), W.SI[2] * dT * m.coords, rtol=0, atol=1e-13)
    sig = array.reconstruct(m, t, [rom], u, dT)
    assert np.abs(sig).max() < 1e-8


def test_fully_clamped_homogeneous_array_is_hydrostatic():
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 2, (3, 3, 3), 3.0, 3.0, 6.0)
    outer = np.nonzero(m.outer_node_mask())[0]
    dofs = (3 * outer[:, None] + np.arange(3)).ravel()
    u = array.solve_mor(m, np.zeros(4, dtype=np.uint8), [rom], -250.0, dofs, np.zeros(dofs.size))
    assert np.abs(u).max() < 1e-14
    sig = array.reconstruct(m, np.zeros(4, dtype=np.uint8), [rom], u, -250.0)
    s0 = 130000.0 * 2.6e-6 * 250.0 / 0.44
    np.testing.assert_allclose(sig, np.broadcast_to([s0, s0, s0, 0, 0, 0], sig.shape), atol=1e-9)


def test_pcg_equals_dense_solve(roms_small):
    m = array.AbstractMesh(3, 3, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.array([0, 1, 0, 1, 0, 1, 0, 0, 1], dtype=np.uint8)
    A, b = array.assemble_global(m, t, roms_small, -250.0)
    dofs, vals = array.constrained_dofs(m, True, False)
    A2, b2 = array.lift(A, b, dofs, vals)
    assert m.n_dofs < 3000
    ref = np.linalg.solve(A2.toarray(), b2)
    x, it = array.pcg_jacobi(A2, b2, rtol=1e-14)
    assert it < 2000
    assert np.abs(x - ref).max() < 1e-11 * np.abs(ref).max()
    np.testing.assert_allclose(array.solve_direct(A2, b2), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_lifting_matches_row_replacement_form(roms_small):
    # Symmetric lifting has the same solution as eq. 13's row-replacement form.
    m = array.AbstractMesh(2, 1, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.array([0, 1], dtype=np.uint8)
    A, b = array.assemble_global(m, t, roms_small, -250.0)
    rng = np.random.default_rng(3)
    dofs, vals = array.constrained_dofs(m, True, False, [5, 40], rng.normal(size=2) * 0.01)
    A2, b2 = array.lift(A, b, dofs, vals)
    Ar = A.toarray()
    br = b.copy()
    Ar[dofs] = 0.0
    Ar[dofs, dofs] = 1.0
    br[dofs] = vals
    np.testing.assert_allclose(np.linalg.solve(A2.toarray(), b2), np.linalg.solve(Ar, br), atol=1e-12)


def test_solution_is_linear_in_delta_T(roms_small):
    m = array.AbstractMesh(3, 2, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.array([0, 1, 1, 0, 0, 1], dtype=np.uint8)
    dofs, vals = array.constrained_dofs(m, True, False)
    u250 = array.solve_mor(m, t, roms_small, -250.0, dofs, vals)
    u150 = array.solve_mor(m, t, roms_small, -150.0, dofs, vals)
    np.testing.assert_allclose(u150, 0.6 * u250, rtol=0, atol=1e-14 * np.abs(u250).max() * 10)


def test_mirror_symmetry_of_symmetric_array():
    s = spec_small(interp=(3, 3, 3), mesh=(4, 4, 6))
    rom = mor.local_stage(s)
    N = 3
    m = array.AbstractMesh(N, N, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.zeros(N * N, dtype=np.uint8)
    dofs, vals = array.constrained_dofs(m, True, False)
    u = array.solve_mor(m, t, [rom], -250.0, dofs, vals)
    sig = array.reconstruct(m, t, [rom], u, -250.0)          # (cells, elem, 6)
    mx, my, mz = s.mesh
    grid = sig.reshape(N, N, mz, my, mx, 6)                    # [cy, cx, ec, eb, ea, comp]
    grid = grid.transpose(2, 0, 3, 1, 4, 5).reshape(mz, N * my, N * mx, 6)  # [z, y, x, comp]
    tol = 1e-9 * np.abs(grid).max()
    fx = grid[:, :, ::-1, :]
    np.testing.assert_allclose(fx[..., [0, 1, 2, 4]], grid[..., [0, 1, 2, 4]], atol=tol)
    np.testing.assert_allclose(fx[..., [3, 5]], -grid[..., [3, 5]], atol=tol)
    fy = grid[:, ::-1, :, :]
    np.testing.assert_allclose(fy[..., [0, 1, 2, 5]], grid[..., [0, 1, 2, 5]], atol=tol)
    np.testing.assert_allclose(fy[..., [3, 4]], -grid[..., [3, 4]], atol=tol)
    tr = grid.transpose(0, 2, 1, 3)                            # x <-> y
    np.testing.assert_allclose(tr[..., 0], grid[..., 1], atol=tol)
    np.testing.assert_allclose(tr[..., 4], grid[..., 5], atol=tol)
    vm = fem.von_mises(grid)
    assert vm.max() > 10.0


def test_c1_mor_against_full_fem():
    """The 2x2 quadratic case against the full fine-mesh FEM: recorded, loosely
    bounded (every block of a 2x2 array touches the free boundary, where the
    paper notes the error concentrates)."""
    case = W.case_c1()
    spec = case.specs[0]
    rom = mor.local_stage(spec)
    m = array.AbstractMesh(2, 2, spec.interp, spec.pitch_x, spec.pitch_y, spec.height)
    dofs, vals = array.constrained_dofs(m, True, False)
    u = array.solve_mor(m, case.cell_type, [rom], case.delta_T, dofs, vals)
    sig = array.reconstruct(m, case.cell_type, [rom], u, case.delta_T)
    _, sf = array.FullArray([spec], case.cell_type, 2, 2).solve(case.delta_T, True, False)
    vm, vmf = fem.von_mises(sig), fem.von_mises(sf)
    mae = np.abs(vm - vmf).mean() / vmf.max()
    assert mae < 0.06
    assert 400.0 < vmf.max() < 700.0
