"""Pins of the oracle's evaluation plane (Sec. 5.1 error metric): sample
geometry, exact reproduction of trilinear displacement fields at arbitrary
points, coincidence with centroid stress, the constrained-block thermal
state, mirror symmetry, and the normalised MAE on a hand example.  CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import array, fem, mor, plane


def spec_small(interp=(3, 3, 3), d=1.6, mesh=(4, 4, 6), **kw):
    return W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=mesh, interp=interp, tsv_diameter=d, **kw)


@pytest.mark.parametrize("mesh,g", [((4, 4, 6), 2), ((4, 4, 6), 7), ((3, 5, 5), 8), ((4, 4, 5), 4)])
def test_sample_points_lie_in_their_element(mesh, g):
    cell = fem.Cell(spec_small(mesh=mesh))
    elem, ref, xyz = plane.plane_points(cell, g)
    assert elem.shape == (g * g,)
    # Physical positions: grid-cell centres on the mid-height plane.
    i = np.arange(g * g) % g
    j = np.arange(g * g) // g
    np.testing.assert_allclose(xyz[:, 0], cell.px * (i + 0.5) / g, rtol=0, atol=1e-15)
    np.testing.assert_allclose(xyz[:, 1], cell.py * (j + 0.5) / g, rtol=0, atol=1e-15)
    assert np.all(xyz[:, 2] == cell.h / 2)
    # The reference coordinates map back to the point through the element's corners.
    ec = cell.element_coords()[elem]                       # (P, 8, 3)
    lo, hi = ec.min(axis=1), ec.max(axis=1)
    np.testing.assert_allclose(lo + (ref + 1.0) / 2.0 * (hi - lo), xyz, rtol=0, atol=1e-13)
    # Half-open boxes: a point on an element face belongs to the +side element.
    assert np.all(ref >= -1.0) and np.all(ref < 1.0)
    assert np.all(ref[:, 2] == (-1.0 if mesh[2] % 2 == 0 else 0.0))


def test_points_on_element_faces_go_to_the_plus_side():
    # 4 elements across, 2 samples: x = p/4 and 3p/4 are element faces.
    cell = fem.Cell(spec_small(mesh=(4, 4, 6)))
    elem, ref, _ = plane.plane_points(cell, 2)
    assert np.all(ref[:, :2] == -1.0)
    ea = elem % 4
    eb = (elem // 4) % 4
    ec = elem // 16
    assert list(ea) == [1, 3, 1, 3] and list(eb) == [1, 1, 3, 3] and np.all(ec == 3)


def _trilinear_field(rng):
    """Displacement components as random combinations of 1, x, y, z, xy, yz,
    zx, xyz, with their exact strains."""
    c = rng.standard_normal((3, 8))

    def u(X):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        mono = np.stack([np.ones_like(x), x, y, z, x * y, y * z, z * x, x * y * z], axis=1)
        return mono @ c.T                                   # (P, 3)

    def grad(X):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        one, zero = np.ones_like(x), np.zeros_like(x)
        dmx = np.stack([zero, one, zero, zero, y, zero, z, y * z], axis=1)
        dmy = np.stack([zero, zero, one, zero, x, z, zero, x * z], axis=1)
        dmz = np.stack([zero, zero, zero, one, zero, y, x, x * y], axis=1)
        return np.stack([dmx @ c.T, dmy @ c.T, dmz @ c.T], axis=2)   # G[p, comp, d/dx_k]

    return u, grad


@pytest.mark.parametrize("mesh,g", [((4, 4, 6), 7), ((3, 5, 5), 8), ((4, 4, 6), 2)])
def test_trilinear_fields_are_reproduced_at_every_sample(mesh, g):
    # Q1 elements interpolate trilinear fields exactly, so the sampled stress
    # must equal D eps of the field at the physical sample point.
    rng = np.random.default_rng(3)
    s = spec_small(mesh=mesh, d=0.0)                         # homogeneous matrix material
    cell = fem.Cell(s)
    mats = cell.material_map()
    u, grad = _trilinear_field(rng)
    nodal = u(cell.node_coords()).ravel()
    sig = plane.block_plane_stress(cell, mats, nodal, 0.0, g)
    _, _, xyz = plane.plane_points(cell, g)
    G = grad(xyz)
    eps = np.stack([G[:, 0, 0], G[:, 1, 1], G[:, 2, 2], G[:, 0, 1] + G[:, 1, 0], G[:, 1, 2] + G[:, 2, 1],
                    G[:, 2, 0] + G[:, 0, 2]], axis=1)
    D = fem.elasticity_matrix(*s.matrix[:2])
    want = eps @ D.T
    np.testing.assert_allclose(sig, want, rtol=0, atol=1e-11 * np.abs(want).max())


def test_odd_layers_with_matching_grid_sample_the_centroids():
    s = spec_small(mesh=(4, 4, 5))
    cell = fem.Cell(s)
    mats = cell.material_map()
    nodal = np.random.default_rng(5).standard_normal(cell.n_dofs)
    dT = -250.0
    sig = plane.block_plane_stress(cell, mats, nodal, dT, 4)
    cen = fem.centroid_stress(nodal, cell.element_dofs(), mats, cell.px / 4, cell.py / 4, cell.h / 5,
                              cell.materials, dT)
    layer = cen.reshape(5, 4, 4, 6)[2].reshape(16, 6)         # layer (m_z - 1) / 2, (eb, ea) order
    np.testing.assert_allclose(sig, layer, rtol=0, atol=1e-12 * np.abs(layer).max())


def test_constrained_homogeneous_block_is_hydrostatic_on_the_plane():
    # All boundary values zero in a homogeneous block: f_T = 0 (uniform beta
    # exerts no interior force), so sigma = -beta dT m at every sample point.
    s = spec_small(d=0.0, interp=(3, 3, 3))
    rom = mor.local_stage(s)
    m = array.AbstractMesh(1, 1, s.interp, 3.0, 3.0, 6.0)
    u = np.zeros(m.n_dofs)
    dT = -250.0
    sig = plane.plane_stress(m, np.zeros(1, dtype=np.uint8), [rom], u, dT, 5)
    E, nu, alpha = s.matrix
    want = -E * alpha * dT / (1 - 2 * nu)
    assert abs(want - 192.05) < 0.01
    np.testing.assert_allclose(sig[..., :3], want, rtol=1e-10)
    np.testing.assert_allclose(sig[..., 3:], 0.0, atol=1e-9 * want)


def test_plane_is_mirror_symmetric_on_a_symmetric_array():
    # Bottom-clamped all-TSV 3x3 array: the plane field is symmetric about
    # x = L/2 (sigma_xy, sigma_zx odd).  g = 8 puts no sample on an element
    # face, so mirrored samples use mirrored elements.
    s = spec_small(interp=(3, 3, 3), mesh=(4, 4, 6))
    rom = mor.local_stage(s)
    N, g = 3, 8
    m = array.AbstractMesh(N, N, (3, 3, 3), 3.0, 3.0, 6.0)
    t = np.zeros(N * N, dtype=np.uint8)
    dofs, vals = array.constrained_dofs(m, True, False)
    u = array.solve_mor(m, t, [rom], -250.0, dofs, vals)
    sig = plane.plane_stress(m, t, [rom], u, -250.0, g)      # (cells, g*g, 6)
    grid = sig.reshape(N, N, g, g, 6).transpose(0, 2, 1, 3, 4).reshape(N * g, N * g, 6)   # [y, x, comp]
    tol = 1e-9 * np.abs(grid).max()
    fx = grid[:, ::-1, :]
    np.testing.assert_allclose(fx[..., [0, 1, 2, 4]], grid[..., [0, 1, 2, 4]], atol=tol)
    np.testing.assert_allclose(fx[..., [3, 5]], -grid[..., [3, 5]], atol=tol)
    tr = grid.transpose(1, 0, 2)
    np.testing.assert_allclose(tr[..., 0], grid[..., 1], atol=tol)
    assert fem.von_mises(grid).max() > 10.0


def test_error_metrics_on_a_hand_example():
    vm = np.array([1.0, 2.0, 3.0, 4.0])
    ref = np.array([1.0, 2.0, 3.0, 5.0])
    assert plane.normalized_mae(vm, ref) == pytest.approx(0.25 / 5.0)
    assert plane.max_rel_error(vm, ref) == pytest.approx(1.0 / 5.0)


def test_full_fem_plane_agrees_with_mor_when_nodes_cover_the_boundary():
    # Lagrange nodes on every boundary FE node: MOR is static condensation,
    # so the reduced and the full plane fields coincide (pins the full-mesh
    # node gather of the plane evaluation against the reduced path).
    s = spec_small(mesh=(4, 4, 4), interp=(5, 5, 5))
    rom = mor.local_stage(s)
    t = np.array([0, 0, 0, 0], dtype=np.uint8)
    m = array.AbstractMesh(2, 2, s.interp, 3.0, 3.0, 6.0)
    dofs, vals = array.constrained_dofs(m, True, False)
    u = array.solve_mor(m, t, [rom], -250.0, dofs, vals)
    vm = plane.plane_von_mises(m, t, [rom], u, -250.0, 6)
    full = array.FullArray([s], t, 2, 2)
    uf, _ = full.solve(-250.0, True, False)
    vmf = plane.full_plane_von_mises(full, uf, -250.0, 6)
    assert plane.max_rel_error(vm, vmf) < 1e-9
