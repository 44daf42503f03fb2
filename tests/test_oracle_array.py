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


# ----------------------------------------------------------------------------
# Branches used as references by the GPU tests: the fine-mesh displacement of
# eq. 15, the clamped top face, and prescribed displacement on the outer faces
# of the full fine-mesh FEM (sub-modelling, Sec. 4.4).
# ----------------------------------------------------------------------------
def full_nodal(full, u_full, c):
    """Full-FEM displacement of block c at its own FE nodes, in the cell
    numbering (node (a, b, c) of the block, DoF 3 id + component)."""
    cx, cy = c % full.Nx, c // full.Nx
    C, B, A = np.meshgrid(np.arange(full.mz + 1), np.arange(full.my + 1), np.arange(full.mx + 1), indexing="ij")
    g = full.node_id(cx * full.mx + A.ravel(), cy * full.my + B.ravel(), C.ravel())
    return u_full.reshape(-1, 3)[g].ravel()


def test_nodal_displacement_of_free_expansion_is_alpha_dT_x():
    # Homogeneous array, 3-2-1 support at the origin: every fine node of every
    # block moves by alpha dT x (eq. 15 with Phi reproducing linear fields);
    # a block gathered at the wrong reduced DoFs would carry another offset.
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    m = array.AbstractMesh(3, 2, s.interp, 3.0, 3.0, 6.0)
    t = np.zeros(6, dtype=np.uint8)
    n0, n1, n2 = m.node_id[0, 0, 0], m.node_id[0, 0, m.X - 1], m.node_id[0, m.Y - 1, 0]
    dofs = np.array([3 * n0, 3 * n0 + 1, 3 * n0 + 2, 3 * n1 + 1, 3 * n1 + 2, 3 * n2 + 2])
    dT = -250.0
    u = array.solve_mor(m, t, [rom], dT, dofs, np.zeros(6))
    local = fem.Cell(s).node_coords()
    for c in range(m.n_cells):
        origin = np.array([3.0 * (c % 3), 3.0 * (c // 3), 0.0])
        nod = array.nodal_displacement(m, t, [rom], u, dT, c).reshape(-1, 3)
        np.testing.assert_allclose(nod, W.SI[2] * dT * (local + origin), rtol=0, atol=1e-13)


def test_nodal_displacement_equals_full_fem_under_static_condensation():
    # Lagrange nodes on every boundary FE node: MOR is static condensation,
    # so eq. 15 must give the full FEM's displacement at every fine node of
    # every block.  Via blocks have f_T != 0, so a dropped dT f_T term fails.
    s = spec_small(mesh=(4, 4, 4), interp=(5, 5, 5), d=1.6)
    specs = [s, s.dummy()]
    roms = [mor.local_stage(x) for x in specs]
    t = np.array([0, 1, 1, 0, 0, 0], dtype=np.uint8)
    m = array.AbstractMesh(3, 2, s.interp, 3.0, 3.0, 6.0)
    dT = -250.0
    dofs, vals = array.constrained_dofs(m, True, False)
    u = array.solve_mor(m, t, roms, dT, dofs, vals)
    full = array.FullArray(specs, t, 3, 2)
    uf, _ = full.solve(dT, True, False)
    scale = np.abs(uf).max()
    assert np.abs(dT * roms[0].fT).max() > 1e-3 * scale
    for c in range(m.n_cells):
        nod = array.nodal_displacement(m, t, roms, u, dT, c)
        np.testing.assert_allclose(nod, full_nodal(full, uf, c), rtol=0, atol=1e-11 * scale)


def test_clamp_top_constrains_exactly_the_top_lattice_plane():
    m = array.AbstractMesh(3, 2, (4, 3, 4), 3.0, 3.0, 6.0)
    want = set()
    for node in range(m.n_nodes):
        I, J, K = m.lattice[node]
        if K == m.nz - 1:
            assert m.coords[node, 2] == 6.0
            want.update(3 * node + k for k in range(3))
    dofs, vals = array.constrained_dofs(m, False, True)
    assert set(dofs.tolist()) == want and not np.any(vals)
    bottom, _ = array.constrained_dofs(m, True, False)
    both, _ = array.constrained_dofs(m, True, True)
    assert set(both.tolist()) == want | set(bottom.tolist())
    assert not want & set(bottom.tolist())


def test_top_and_bottom_clamped_array_is_mirror_symmetric_in_z():
    # Scenario 1 of the paper's evaluation clamps both faces: the all-TSV
    # array is then symmetric about z = h/2 (normal and xy stresses even,
    # yz and zx odd); with the bottom clamped alone it is not.
    s = spec_small(interp=(3, 3, 3), mesh=(4, 4, 6))
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 2, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.zeros(4, dtype=np.uint8)

    def grid(top):
        dofs, vals = array.constrained_dofs(m, True, top)
        u = array.solve_mor(m, t, [rom], -250.0, dofs, vals)
        return array.reconstruct(m, t, [rom], u, -250.0).reshape(4, 6, 4, 4, 6)   # [cell, z, y, x, comp]

    g = grid(True)
    tol = 1e-9 * np.abs(g).max()
    fz = g[:, ::-1]
    np.testing.assert_allclose(fz[..., [0, 1, 2, 3]], g[..., [0, 1, 2, 3]], atol=tol)
    np.testing.assert_allclose(fz[..., [4, 5]], -g[..., [4, 5]], atol=tol)
    g1 = grid(False)
    assert np.abs(g1[:, ::-1][..., 0] - g1[..., 0]).max() > 1e3 * tol


def linear_field(rng):
    a = rng.normal(size=3) * 0.05
    G = rng.normal(size=(3, 3)) * 1e-3
    return (lambda xyz: a[None, :] + np.asarray(xyz) @ G.T), G


def test_full_fem_reproduces_a_linear_field_on_the_outer_faces():
    # Patch test of the prescribed-field branch: a homogeneous array at dT = 0
    # with u = a + G x on all six outer faces is exactly that field inside,
    # with the constant stress D sym(G) in every element.
    s = spec_small(d=0.0)
    rng = np.random.default_rng(7)
    f, G = linear_field(rng)
    full = array.FullArray([s], np.zeros(6, dtype=np.uint8), 3, 2)
    u, sig = full.solve(0.0, False, False, field=f)
    np.testing.assert_allclose(u.reshape(-1, 3), f(full.node_coords()), rtol=0, atol=1e-13)
    eps = 0.5 * (G + G.T)
    voigt = np.array([eps[0, 0], eps[1, 1], eps[2, 2], 2 * eps[0, 1], 2 * eps[1, 2], 2 * eps[2, 0]])
    want = fem.elasticity_matrix(*W.SI[:2]) @ voigt
    np.testing.assert_allclose(sig, np.broadcast_to(want, sig.shape), rtol=0, atol=1e-9 * np.abs(want).max())


def test_mor_with_a_linear_field_on_the_outer_faces_is_exact():
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    rng = np.random.default_rng(8)
    f, _ = linear_field(rng)
    m = array.AbstractMesh(3, 2, s.interp, 3.0, 3.0, 6.0)
    t = np.zeros(6, dtype=np.uint8)
    outer = np.nonzero(m.outer_node_mask())[0]
    dofs = (3 * outer[:, None] + np.arange(3)).ravel()
    vals = f(m.coords[outer]).ravel()
    u = array.solve_mor(m, t, [rom], 0.0, dofs, vals)
    np.testing.assert_allclose(u.reshape(-1, 3), f(m.coords), rtol=0, atol=1e-13)
    local = fem.Cell(s).node_coords()
    for c in range(m.n_cells):
        origin = np.array([3.0 * (c % 3), 3.0 * (c // 3), 0.0])
        nod = array.nodal_displacement(m, t, [rom], u, 0.0, c).reshape(-1, 3)
        np.testing.assert_allclose(nod, f(local + origin), rtol=0, atol=1e-13)


def test_prescribed_field_mor_equals_full_fem_under_static_condensation():
    # Heterogeneous blocks, a smooth non-polynomial field on all six outer
    # faces and a thermal load: with Lagrange nodes on every boundary FE node
    # both sides see the same Dirichlet data, so they must agree exactly.
    s = spec_small(mesh=(4, 4, 4), interp=(5, 5, 5), d=1.6)
    specs = [s, s.dummy()]
    roms = [mor.local_stage(x) for x in specs]
    t = np.array([0, 1, 0, 0], dtype=np.uint8)
    m = array.AbstractMesh(2, 2, s.interp, 3.0, 3.0, 6.0)
    field = W.fourier_field(np.random.default_rng(3), (6.0, 6.0, 6.0), amplitude=0.05)
    outer = np.nonzero(m.outer_node_mask())[0]
    dofs = (3 * outer[:, None] + np.arange(3)).ravel()
    vals = field(m.coords[outer]).ravel()
    dT = -150.0
    u = array.solve_mor(m, t, roms, dT, dofs, vals)
    full = array.FullArray(specs, t, 2, 2)
    uf, sf = full.solve(dT, False, False, field=field)
    sig = array.reconstruct(m, t, roms, u, dT)
    np.testing.assert_allclose(sig, sf, rtol=0, atol=1e-9 * np.abs(sf).max())
    for c in range(m.n_cells):
        np.testing.assert_allclose(array.nodal_displacement(m, t, roms, u, dT, c), full_nodal(full, uf, c),
                                   rtol=0, atol=1e-11 * np.abs(uf).max())
