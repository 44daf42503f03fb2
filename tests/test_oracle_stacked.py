"""Pins of the oracle's stacked variant of the abstract mesh: N_z layers of
blocks stacked in z that share their horizontal faces (the abstract mesh of
Sec. 4.3 with a z index of blocks; the reduced model of each block is
unchanged).  Checked against brute-force numbering, exact static
condensation against the full fine-mesh FEM of the stack, closed-form
thermal states, the patch test, a taller single layer that is the same fine
mesh, and mirror symmetry.  CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import array, fem, mor


def spec_small(interp=(3, 3, 3), d=1.6, mesh=(4, 4, 6), **kw):
    return W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=mesh, interp=interp, tsv_diameter=d, **kw)


@pytest.mark.parametrize("N,interp", [((2, 2, 2), (3, 3, 3)), ((3, 2, 3), (4, 3, 4)), ((1, 1, 4), (2, 2, 2)),
                                      ((2, 3, 2), (4, 4, 4))])
def test_stacked_numbering_against_brute_force(N, interp):
    Nx, Ny, Nz = N
    nx, ny, nz = interp
    m = array.AbstractMesh(Nx, Ny, interp, nz_cells=Nz)
    X, Y, Z = Nx * (nx - 1) + 1, Ny * (ny - 1) + 1, Nz * (nz - 1) + 1
    # Lattice points that are nodes, by enumeration, ranked in (K, J, I) order.
    pts = [(I, J, K) for K in range(Z) for J in range(Y) for I in range(X)
           if I % (nx - 1) == 0 or J % (ny - 1) == 0 or K % (nz - 1) == 0]
    assert m.n_nodes == len(pts)
    assert np.array_equal(m.lattice, np.array(pts))
    # Closed form: N_z + 1 full planes and N_z (n_z - 2) planes of rows/columns.
    mid = (Ny + 1) * X + (Y - Ny - 1) * (Nx + 1)
    assert m.n_nodes == (Nz + 1) * X * Y + Nz * (nz - 2) * mid
    # Every block's surface node sits at its lattice point.
    rank = {p: i for i, p in enumerate(pts)}
    S = mor.surface_nodes(nx, ny, nz)
    for cz in range(Nz):
        for cy in range(Ny):
            for cx in range(Nx):
                c = (cz * Ny + cy) * Nx + cx
                for s, (i, j, k) in enumerate(S):
                    assert m.conn[c, s] == rank[(cx * (nx - 1) + i, cy * (ny - 1) + j, cz * (nz - 1) + k)]
    assert np.array_equal(np.unique(m.conn), np.arange(m.n_nodes))


def test_stacked_blocks_share_their_horizontal_face():
    m = array.AbstractMesh(2, 1, (4, 3, 3), nz_cells=3)
    S = mor.surface_nodes(4, 3, 3)
    pos = {s: i for i, s in enumerate(S)}
    for cz in range(2):
        for cx in range(2):
            lo, hi = cz * 2 + cx, (cz + 1) * 2 + cx
            for (i, j, k) in S:
                if k == 2:
                    assert m.conn[lo, pos[(i, j, 2)]] == m.conn[hi, pos[(i, j, 0)]]
    # Blocks two layers apart share nothing; a block and the one above its
    # x neighbour share the edge line of n_y nodes.
    assert not set(m.conn[0]) & set(m.conn[4])
    assert len(set(m.conn[0]) & set(m.conn[3])) == 3


def test_single_layer_is_the_unstacked_mesh():
    a = array.AbstractMesh(3, 2, (4, 3, 5), 3.0, 3.0, 6.0)
    b = array.AbstractMesh(3, 2, (4, 3, 5), 3.0, 3.0, 6.0, nz_cells=1)
    assert np.array_equal(a.conn, b.conn) and np.array_equal(a.coords, b.coords)


def full_nodal(full, u_full, c):
    """Full-FEM displacement at the fine nodes of block c of a stack, in the
    block's own node order."""
    cx = c % full.Nx
    cy = (c // full.Nx) % full.Ny
    cz = c // (full.Nx * full.Ny)
    C, B, A = np.meshgrid(np.arange(full.mz + 1), np.arange(full.my + 1), np.arange(full.mx + 1), indexing="ij")
    g = full.node_id(cx * full.mx + A.ravel(), cy * full.my + B.ravel(), cz * full.mz + C.ravel())
    return u_full.reshape(-1, 3)[g].ravel()


@pytest.mark.parametrize("top", [False, True], ids=["bottom", "top-and-bottom"])
def test_stack_mor_equals_full_fem_under_static_condensation(top):
    # Lagrange nodes on every boundary FE node: MOR of the stack is static
    # condensation of the full fine mesh of the stack, so displacements and
    # stresses agree exactly (a wrong layer offset, or blocks of one layer
    # numbered into another, would not).
    s = spec_small(mesh=(2, 2, 2), interp=(3, 3, 3), d=1.6)
    specs = [s, s.dummy()]
    roms = [mor.local_stage(x) for x in specs]
    t = np.array([0, 1, 1, 0, 0, 0, 1, 0], dtype=np.uint8)      # 2 x 2 x 2
    m = array.AbstractMesh(2, 2, s.interp, 3.0, 3.0, 6.0, nz_cells=2)
    dT = -250.0
    dofs, vals = array.constrained_dofs(m, True, top)
    u = array.solve_mor(m, t, roms, dT, dofs, vals)
    full = array.FullArray(specs, t, 2, 2, nz_cells=2)
    uf, sf = full.solve(dT, True, top)
    sig = array.reconstruct(m, t, roms, u, dT)
    np.testing.assert_allclose(sig, sf, rtol=0, atol=1e-9 * np.abs(sf).max())
    for c in range(m.n_cells):
        np.testing.assert_allclose(array.nodal_displacement(m, t, roms, u, dT, c), full_nodal(full, uf, c),
                                   rtol=0, atol=1e-11 * np.abs(uf).max())


def test_two_layers_are_one_taller_layer_of_the_same_fine_mesh():
    # A stack of two blocks of height h meshed m_z each is, element for
    # element, one block of height 2h meshed 2 m_z (the via is a prism, so
    # the material map does not depend on z): the full FEM must agree.
    s = spec_small(mesh=(4, 4, 3), d=1.6)
    tall = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=12.0, mesh=(4, 4, 6), interp=(3, 3, 3), tsv_diameter=1.6)
    t2 = np.zeros(2 * 2 * 2, dtype=np.uint8)
    t1 = np.zeros(2 * 2, dtype=np.uint8)
    ua, sa = array.FullArray([s], t2, 2, 2, nz_cells=2).solve(-250.0, True, False)
    ub, sb = array.FullArray([tall], t1, 2, 2).solve(-250.0, True, False)
    np.testing.assert_allclose(ua, ub, rtol=0, atol=1e-12 * np.abs(ub).max())
    # Block (cx, cy, cz)'s elements are the tall block's layers cz m_z ... .
    sb = sb.reshape(4, 6, 4, 4, 6)
    for cz in range(2):
        got = sa[cz * 4:(cz + 1) * 4].reshape(4, 3, 4, 4, 6)
        np.testing.assert_allclose(got, sb[:, cz * 3:(cz + 1) * 3], rtol=0, atol=1e-9 * np.abs(sb).max())


def test_free_expansion_of_a_homogeneous_stack_is_stress_free():
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 2, (3, 3, 3), 3.0, 3.0, 6.0, nz_cells=3)
    t = np.zeros(12, dtype=np.uint8)
    n0 = m.node_id[0, 0, 0]
    n1 = m.node_id[0, 0, m.X - 1]
    n2 = m.node_id[0, m.Y - 1, 0]
    dofs = np.array([3 * n0, 3 * n0 + 1, 3 * n0 + 2, 3 * n1 + 1, 3 * n1 + 2, 3 * n2 + 2])
    dT = -250.0
    u = array.solve_mor(m, t, [rom], dT, dofs, np.zeros(6))
    np.testing.assert_allclose(u.reshape(-1, 3), W.SI[2] * dT * m.coords, rtol=0, atol=1e-13)
    assert m.coords[:, 2].max() == 18.0
    sig = array.reconstruct(m, t, [rom], u, dT)
    assert np.abs(sig).max() < 1e-8


def test_fully_clamped_homogeneous_stack_is_hydrostatic():
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 1, (3, 3, 3), 3.0, 3.0, 6.0, nz_cells=2)
    outer = np.nonzero(m.outer_node_mask())[0]
    dofs = (3 * outer[:, None] + np.arange(3)).ravel()
    t = np.zeros(4, dtype=np.uint8)
    u = array.solve_mor(m, t, [rom], -250.0, dofs, np.zeros(dofs.size))
    # The nodes of the shared horizontal face inside the stack are free and
    # still do not move.
    assert (~m.outer_node_mask()).sum() > 0
    assert np.abs(u).max() < 1e-14
    sig = array.reconstruct(m, t, [rom], u, -250.0)
    s0 = 130000.0 * 2.6e-6 * 250.0 / 0.44
    np.testing.assert_allclose(sig, np.broadcast_to([s0, s0, s0, 0, 0, 0], sig.shape), atol=1e-9)


def test_linear_field_on_the_outer_faces_of_a_stack_is_exact():
    s = spec_small(d=0.0)
    rom = mor.local_stage(s)
    rng = np.random.default_rng(9)
    a = rng.normal(size=3) * 0.05
    G = rng.normal(size=(3, 3)) * 1e-3
    f = lambda xyz: a[None, :] + np.asarray(xyz) @ G.T       # noqa: E731
    m = array.AbstractMesh(2, 2, s.interp, 3.0, 3.0, 6.0, nz_cells=2)
    t = np.zeros(8, dtype=np.uint8)
    outer = np.nonzero(m.outer_node_mask())[0]
    dofs = (3 * outer[:, None] + np.arange(3)).ravel()
    u = array.solve_mor(m, t, [rom], 0.0, dofs, f(m.coords[outer]).ravel())
    np.testing.assert_allclose(u.reshape(-1, 3), f(m.coords), rtol=0, atol=1e-13)
    local = fem.Cell(s).node_coords()
    for c in range(m.n_cells):
        origin = np.array([3.0 * (c % 2), 3.0 * ((c // 2) % 2), 6.0 * (c // 4)])
        nod = array.nodal_displacement(m, t, [rom], u, 0.0, c).reshape(-1, 3)
        np.testing.assert_allclose(nod, f(local + origin), rtol=0, atol=1e-13)


def test_top_and_bottom_clamped_stack_is_mirror_symmetric_in_z():
    # Two layers of TSV blocks clamped at the bottom of the stack and at its
    # top: the stack is symmetric about its mid-height, the shared face, so
    # layer 1 is layer 0 reflected (normal and xy stresses even, yz and zx
    # odd).
    s = spec_small(interp=(3, 3, 3), mesh=(4, 4, 6))
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 2, (3, 3, 3), 3.0, 3.0, 6.0, nz_cells=2)
    t = np.zeros(8, dtype=np.uint8)
    dofs, vals = array.constrained_dofs(m, True, True)
    u = array.solve_mor(m, t, [rom], -250.0, dofs, vals)
    g = array.reconstruct(m, t, [rom], u, -250.0).reshape(2, 4, 6, 4, 4, 6)   # [cz, cell, z, y, x, comp]
    tol = 1e-9 * np.abs(g).max()
    fz = g[::-1, :, ::-1]
    np.testing.assert_allclose(fz[..., [0, 1, 2, 3]], g[..., [0, 1, 2, 3]], atol=tol)
    np.testing.assert_allclose(fz[..., [4, 5]], -g[..., [4, 5]], atol=tol)
    # A stack differs from one clamped layer: the shared face moves.
    shared = np.nonzero(m.lattice[:, 2] == 2)[0]
    assert np.abs(u.reshape(-1, 3)[shared]).max() > 1e-6
