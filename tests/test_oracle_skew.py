"""Pins of the oracle's skewed (parallelepiped) blocks, the rhombic unit block
of a 120-degree TSV array (Sec. 4.2 names 120-degree arrays; every point of
the block is sheared by x += skew * y, skew = 1/sqrt(3) with p_y = p sqrt(3)/2
for a triangular lattice of spacing p).  Checked against: the rectangular
block at skew 0, a closed form of the element energy of a uniform strain,
exact rational material classification, the lattice geometry, the patch
test, static condensation against the full fine-mesh FEM, free expansion and
point symmetry.  CPU only."""
import math
from dataclasses import replace
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import array, fem, mor


def small_skewed(skew=1.0 / math.sqrt(3.0), **kw):
    base = dict(pitch_x=3.0, pitch_y=3.0 * math.sqrt(3.0) / 2.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 3),
                tsv_diameter=1.6, skew=skew)
    base.update(kw)
    return W.CellSpec(**base)


def test_zero_skew_is_the_rectangular_block():
    a = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 3), tsv_diameter=1.6,
                   liner_thickness=0.3)
    b = replace(a, skew=0.0)
    ca, cb = fem.Cell(a), fem.Cell(b)
    assert np.array_equal(ca.node_coords(), cb.node_coords())
    assert np.array_equal(ca.node_coords(), ca.ref_coords())
    Ka, ba, ma = fem.assemble_cell(ca)
    Kb, bb, mb = fem.assemble_cell(cb)
    assert np.array_equal(ma, mb) and np.array_equal(Ka.data, Kb.data) and np.array_equal(ba, bb)
    assert np.array_equal(mor.local_stage(a).Kr, mor.local_stage(b).Kr)


@pytest.mark.parametrize("skew", [1.0 / math.sqrt(3.0), -0.4, 1.3])
def test_skewed_element_energy_of_a_uniform_strain(skew):
    # Nodal values u = G x (physical corners): the element is affine, so
    # B u_e is the constant strain sym(G) at every Gauss point and
    # u^T K u = V e^T D e, f . u = V beta tr(e), V = hx hy hz (a shear keeps
    # the volume).  A wrong Jacobian or inverse fails this.
    hx, hy, hz = 0.7, 0.55, 1.3
    X = fem.element_corners(hx, hy, hz, skew)
    rng = np.random.default_rng(3)
    G = rng.normal(size=(3, 3))
    u = (X @ G.T).ravel()
    E, nu, alpha = W.CU
    D = fem.elasticity_matrix(E, nu)
    beta = fem.thermal_coefficient(E, nu, alpha)
    Ke, fe = fem.hex8_element(X, D, beta)
    e = np.array([G[0, 0], G[1, 1], G[2, 2], G[0, 1] + G[1, 0], G[1, 2] + G[2, 1], G[2, 0] + G[0, 2]])
    V = hx * hy * hz
    assert u @ Ke @ u == pytest.approx(V * e @ D @ e, rel=1e-12)
    assert fe @ u == pytest.approx(V * beta * (e[0] + e[1] + e[2]), rel=1e-12)


def exact_map(px, py, skew, mesh, d):
    mx, my, mz = mesh
    px, py, skew, d = (Fraction(v) for v in (px, py, skew, d))
    out = []
    for ec in range(mz):
        for eb in range(my):
            dy = (eb + Fraction(1, 2)) * py / my - py / 2
            for ea in range(mx):
                dx = ((ea + Fraction(1, 2)) * px / mx - px / 2) + skew * dy
                r2 = dx * dx + dy * dy
                assert r2 != (d / 2) ** 2
                out.append(fem.VIA if r2 < (d / 2) ** 2 else fem.MATRIX)
    return np.array(out, dtype=np.uint8)


@pytest.mark.parametrize("skew,mesh,d", [(0.5, (8, 8, 2), 2.1), (-0.25, (10, 6, 2), 1.7), (0.75, (7, 9, 3), 2.3)])
def test_skewed_map_matches_exact_arithmetic(skew, mesh, d):
    spec = W.CellSpec(pitch_x=3.0, pitch_y=2.5, height=6.0, mesh=mesh, tsv_diameter=d, skew=skew)
    np.testing.assert_array_equal(fem.Cell(spec).material_map(), exact_map(3.0, 2.5, skew, mesh, d))


def test_rhombic_block_is_point_symmetric_and_tiles_a_triangular_lattice():
    spec = W.hex_spec()
    c = fem.Cell(spec)
    m = c.material_map().reshape(c.mz, c.my, c.mx)
    np.testing.assert_array_equal(m, m[:, ::-1, ::-1])         # 180 degrees about the via axis
    # Via axes of the blocks: the six nearest neighbours of a block are all
    # one pitch away (a triangular lattice), the next ones sqrt(3) pitches.
    axis = lambda cx, cy: np.array([cx * c.px + c.skew * cy * c.py + c.px / 2 + c.skew * c.py / 2,  # noqa: E731
                                    cy * c.py + c.py / 2])
    d = sorted(np.linalg.norm(axis(cx, cy) - axis(0, 0)) for cx in range(-2, 3) for cy in range(-2, 3)
               if (cx, cy) != (0, 0))
    np.testing.assert_allclose(d[:6], 15.0, rtol=1e-14)
    assert d[6] == pytest.approx(15.0 * math.sqrt(3.0), rel=1e-14)
    # The via is a disk of diameter 5 um in physical space: its element
    # count is the disk's share of the block, to the mesh's resolution.
    area = (m[0] == fem.VIA).sum() * (c.px / c.mx) * (c.py / c.my)
    assert area == pytest.approx(math.pi * 2.5 ** 2, rel=0.08)


def test_patch_test_on_a_skewed_array():
    # Homogeneous blocks, a linear field on all outer faces, dT = 0: affine
    # elements and Lagrange interpolation in the block's own coordinates
    # reproduce it exactly, on the full FEM and on the reduced model.
    s = small_skewed(tsv_diameter=0.0)
    rom = mor.local_stage(s)
    rng = np.random.default_rng(7)
    a = rng.normal(size=3) * 0.05
    G = rng.normal(size=(3, 3)) * 1e-3
    f = lambda xyz: a[None, :] + np.asarray(xyz) @ G.T          # noqa: E731
    m = array.AbstractMesh(2, 2, s.interp, s.pitch_x, s.pitch_y, s.height, skew=s.skew)
    t = np.zeros(4, dtype=np.uint8)
    outer = np.nonzero(m.outer_node_mask())[0]
    dofs = (3 * outer[:, None] + np.arange(3)).ravel()
    u = array.solve_mor(m, t, [rom], 0.0, dofs, f(m.coords[outer]).ravel())
    np.testing.assert_allclose(u.reshape(-1, 3), f(m.coords), rtol=0, atol=1e-13)
    local = fem.Cell(s).node_coords()
    for cidx in range(4):
        cx, cy = cidx % 2, cidx // 2
        origin = np.array([cx * s.pitch_x + s.skew * cy * s.pitch_y, cy * s.pitch_y, 0.0])
        nod = array.nodal_displacement(m, t, [rom], u, 0.0, cidx).reshape(-1, 3)
        np.testing.assert_allclose(nod, f(local + origin), rtol=0, atol=1e-13)
    full = array.FullArray([s], t, 2, 2)
    uf, _ = full.solve(0.0, False, False, field=f)
    np.testing.assert_allclose(uf.reshape(-1, 3), f(full.node_coords()), rtol=0, atol=1e-13)


def full_nodal(full, u_full, c):
    cx, cy = c % full.Nx, c // full.Nx
    C, B, A = np.meshgrid(np.arange(full.mz + 1), np.arange(full.my + 1), np.arange(full.mx + 1), indexing="ij")
    g = full.node_id(cx * full.mx + A.ravel(), cy * full.my + B.ravel(), C.ravel())
    return u_full.reshape(-1, 3)[g].ravel()


def test_skewed_mor_equals_full_fem_under_static_condensation():
    s = small_skewed(mesh=(2, 2, 2), interp=(3, 3, 3))
    specs = [s, s.dummy()]
    roms = [mor.local_stage(x) for x in specs]
    t = np.array([0, 1, 0, 0], dtype=np.uint8)
    m = array.AbstractMesh(2, 2, s.interp, s.pitch_x, s.pitch_y, s.height, skew=s.skew)
    dT = -250.0
    dofs, vals = array.constrained_dofs(m, True, False)
    u = array.solve_mor(m, t, roms, dT, dofs, vals)
    full = array.FullArray(specs, t, 2, 2)
    uf, sf = full.solve(dT, True, False)
    sig = array.reconstruct(m, t, roms, u, dT)
    np.testing.assert_allclose(sig, sf, rtol=0, atol=1e-9 * np.abs(sf).max())
    for c in range(m.n_cells):
        np.testing.assert_allclose(array.nodal_displacement(m, t, roms, u, dT, c), full_nodal(full, uf, c),
                                   rtol=0, atol=1e-11 * np.abs(uf).max())


def test_free_expansion_of_a_skewed_homogeneous_array_is_stress_free():
    s = small_skewed(tsv_diameter=0.0)
    rom = mor.local_stage(s)
    m = array.AbstractMesh(3, 2, s.interp, s.pitch_x, s.pitch_y, s.height, skew=s.skew)
    t = np.zeros(6, dtype=np.uint8)
    n0 = m.node_id[0, 0, 0]
    n1 = m.node_id[0, 0, m.X - 1]
    n2 = m.node_id[0, m.Y - 1, 0]
    dofs = np.array([3 * n0, 3 * n0 + 1, 3 * n0 + 2, 3 * n1 + 1, 3 * n1 + 2, 3 * n2 + 2])
    u = array.solve_mor(m, t, [rom], -250.0, dofs, np.zeros(6))
    np.testing.assert_allclose(u.reshape(-1, 3), W.SI[2] * -250.0 * m.coords, rtol=0, atol=1e-13)
    assert np.abs(array.reconstruct(m, t, [rom], u, -250.0)).max() < 1e-8
