"""Pins of the oracle's local stage (Sec. 4.2, eq. 8-19) against the paper's
printed counts, closed forms, invariants and brute force.  CPU only."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import array, fem, mor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_spec(mesh=(4, 4, 6), interp=(3, 3, 3), d=1.6, t=0.0, **kw):
    return W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=mesh, interp=interp,
                      tsv_diameter=d, liner_thickness=t, **kw)


def test_eq16_matches_table3():
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_basis_counts.txt"), dtype=int)
    for nx, ny, nz, n in rows:
        assert mor.n_reduced(nx, ny, nz) == n
        assert 3 * len(mor.surface_nodes(nx, ny, nz)) == n


def test_surface_node_order():
    S = mor.surface_nodes(3, 3, 3)
    assert S[0] == (0, 0, 0) and S[-1] == (2, 2, 2)      # first and last entries of eq. 14
    assert (1, 1, 1) not in S and len(S) == 26
    keys = [(k, j, i) for i, j, k in S]
    assert keys == sorted(keys)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_lagrange_1d_cardinal_partition_and_reproduction(n):
    xs = mor.interp_points(15.0, n)
    for i in range(n):
        np.testing.assert_allclose(mor.lagrange_1d(xs, xs, i), np.eye(n)[i], atol=1e-15)
    x = np.linspace(0.0, 15.0, 37)
    basis = np.array([mor.lagrange_1d(x, xs, i) for i in range(n)])
    np.testing.assert_allclose(basis.sum(axis=0), 1.0, atol=1e-13)
    for deg in range(n):                                  # degree <= n-1 reproduced
        np.testing.assert_allclose(basis.T @ (xs / 15.0) ** deg, (x / 15.0) ** deg, atol=1e-12)
    err = np.abs(basis.T @ (xs / 15.0) ** n - (x / 15.0) ** n).max()
    assert err > 1e-4                                     # degree n is not


def test_interpolation_matrix_partition_and_face_conformity():
    spec = small_spec(mesh=(6, 4, 5), interp=(4, 3, 3))
    cell = fem.Cell(spec)
    L, bc_dofs, S = mor.interpolation_matrix(cell)
    for comp in range(3):
        np.testing.assert_allclose(L[comp::3, comp::3].sum(axis=1), 1.0, atol=1e-13)
        assert np.abs(L[comp::3, (comp + 1) % 3::3]).max() == 0.0
    W_ = L[0::3, 0::3]
    bnodes = bc_dofs[0::3] // 3
    row_of = {int(nd): r for r, nd in enumerate(bnodes)}
    nx, ny, nz = spec.interp
    # A node on face x = p depends only on Lagrange nodes with i = nx-1, and
    # with the same weights as its mirror on face x = 0 has on i = 0: the
    # traces of neighbouring blocks agree (conforming abstract mesh).
    for c in range(cell.mz + 1):
        for b in range(cell.my + 1):
            r_hi = W_[row_of[cell.node_id(cell.mx, b, c)]]
            r_lo = W_[row_of[cell.node_id(0, b, c)]]
            hi_cols = [s for s, (i, j, k) in enumerate(S) if i == nx - 1]
            lo_cols = [s for s, (i, j, k) in enumerate(S) if i == 0]
            assert np.abs(np.delete(r_hi, hi_cols)).max() == 0.0
            np.testing.assert_array_equal(r_hi[hi_cols], r_lo[lo_cols])


@pytest.fixture(scope="module")
def tsv_rom():
    return mor.local_stage(small_spec(mesh=(4, 4, 6), interp=(3, 3, 4), d=1.6, t=0.3))


def surface_coords(rom):
    c = rom.cell
    nx, ny, nz = c.spec.interp
    xs, ys, zs = mor.interp_points(c.px, nx), mor.interp_points(c.py, ny), mor.interp_points(c.h, nz)
    return np.array([[xs[i], ys[j], zs[k]] for i, j, k in rom.S])


def test_local_residual(tsv_rom):
    assert tsv_rom.local_residual < 1e-13
    assert tsv_rom.n == mor.n_reduced(3, 3, 4)


def test_basis_reproduces_rigid_motions_for_heterogeneous_cell(tsv_rom):
    P = surface_coords(tsv_rom)
    X = tsv_rom.cell.node_coords()
    for w in np.eye(3):
        t = w
        np.testing.assert_allclose(tsv_rom.Phi @ np.tile(t, len(P)), np.tile(t, len(X)), atol=1e-12)
        rot = lambda Y: np.cross(np.broadcast_to(w, Y.shape), Y - 1.0).ravel()
        np.testing.assert_allclose(tsv_rom.Phi @ rot(P), rot(X), atol=1e-11)


def test_basis_reproduces_linear_fields_for_homogeneous_cell():
    rom = mor.local_stage(small_spec(mesh=(4, 4, 6), interp=(2, 2, 2), d=0.0))
    P = surface_coords(rom)
    X = rom.cell.node_coords()
    G = np.array([[1.0, 0.2, -0.3], [0.4, -0.7, 0.1], [0.05, 0.3, 0.9]]) * 1e-3
    np.testing.assert_allclose(rom.Phi @ (P @ G.T).ravel(), (X @ G.T).ravel(), atol=1e-14)


def test_reduced_stiffness_spd_with_six_rigid_modes(tsv_rom):
    Kr = tsv_rom.Kr
    assert np.array_equal(Kr, Kr.T)
    ev = np.linalg.eigvalsh(Kr)
    assert np.all(ev > -1e-9 * ev[-1])
    assert int(np.sum(ev < 1e-9 * ev[-1])) == 6
    assert ev[6] > 1e-6 * ev[-1]


def test_reduced_stiffness_is_projected_schur_complement(tsv_rom):
    # K_r = L^T S L with S = K_bb - K_bf K_ff^{-1} K_fb, computed densely.
    K = tsv_rom.K.toarray()
    f, b = tsv_rom.free_dofs, tsv_rom.bc_dofs
    S = K[np.ix_(b, b)] - K[np.ix_(b, f)] @ np.linalg.solve(K[np.ix_(f, f)], K[np.ix_(f, b)])
    ref = tsv_rom.L.T @ S @ tsv_rom.L
    np.testing.assert_allclose(tsv_rom.Kr, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_thermal_basis_is_energy_orthogonal_to_phi(tsv_rom):
    # Phi^T K f_T = 0: f_T vanishes on the boundary and each f_i is discrete
    # harmonic inside, so the global system needs only eq. 18-19.
    v = tsv_rom.Phi.T @ (tsv_rom.K @ tsv_rom.fT)
    scale = np.abs(tsv_rom.Phi).max() * np.abs(tsv_rom.K @ tsv_rom.fT).sum()
    assert np.abs(v).max() < 1e-12 * scale
    assert np.abs(tsv_rom.fT[tsv_rom.bc_dofs]).max() == 0.0


def test_reduced_load_matches_dense_definition(tsv_rom):
    # b_r = Phi^T b with Phi from a dense solve of the lifted problem (eq. 13-15).
    K = tsv_rom.K.toarray()
    f, b = tsv_rom.free_dofs, tsv_rom.bc_dofs
    Xf = np.linalg.solve(K[np.ix_(f, f)], -K[np.ix_(f, b)] @ tsv_rom.L)
    Phi = np.zeros_like(tsv_rom.Phi)
    Phi[f], Phi[b] = Xf, tsv_rom.L
    np.testing.assert_allclose(tsv_rom.Phi, Phi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(tsv_rom.br, Phi.T @ tsv_rom.b, rtol=1e-12, atol=1e-14)


def mor_vs_full(spec, nx_cells, ny_cells, cell_type=None, dT=-250.0, dummy=False):
    specs = [spec, spec.dummy()] if dummy else [spec]
    if cell_type is None:
        cell_type = np.zeros(nx_cells * ny_cells, dtype=np.uint8)
    roms = [mor.local_stage(s) for s in specs]
    mesh = array.AbstractMesh(nx_cells, ny_cells, spec.interp, spec.pitch_x, spec.pitch_y, spec.height)
    dofs, vals = array.constrained_dofs(mesh, True, False)
    u = array.solve_mor(mesh, cell_type, roms, dT, dofs, vals)
    sig = array.reconstruct(mesh, cell_type, roms, u, dT)
    _, sig_full = array.FullArray(specs, cell_type, nx_cells, ny_cells).solve(dT, True, False)
    vm, vmf = fem.von_mises(sig), fem.von_mises(sig_full)
    return (np.abs(vm - vmf).max() / vmf.max(), np.abs(sig - sig_full).max() / np.abs(sig_full).max(),
            np.abs(vm - vmf).mean() / vmf.max())


def test_mor_equals_full_fem_when_nodes_cover_the_boundary():
    # Lagrange nodes on every boundary FE node => L is a selection and MOR is
    # static condensation, exact up to rounding.
    spec = small_spec(mesh=(4, 4, 4), interp=(5, 5, 5), d=1.6)
    e_vm, e_sig, _ = mor_vs_full(spec, 2, 2, np.array([0, 1, 1, 0], dtype=np.uint8), dummy=True)
    assert e_vm < 1e-10 and e_sig < 1e-10


def test_mor_error_falls_as_interpolation_order_rises():
    # Trend of Table 3: the normalised mean absolute von Mises error (the
    # paper's metric, Sec. 5.2) falls as (n_x, n_y, n_z) rises.
    mae, mx = [], []
    for k in (2, 3, 4, 5):
        spec = small_spec(mesh=(6, 6, 8), interp=(k, k, k), d=1.6)
        e_max, _, e_mae = mor_vs_full(spec, 2, 2)
        mae.append(e_mae)
        mx.append(e_max)
    assert mae[0] > mae[1] > mae[2] > mae[3]
    assert mae[3] < 0.25 * mae[0] and mx[3] < 0.5 * mx[0]
