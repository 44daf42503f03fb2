"""Pins of the oracle's finite-element layer (eq. 1-7) against closed forms,
invariants and exact arithmetic.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import fem

SI, CU, SIO2 = W.SI, W.CU, W.SIO2


def brick(hx=1.5, hy=1.5, hz=2.5):
    return (fem.HEX_CORNERS + 1.0) / 2.0 * np.array([hx, hy, hz])


def test_lame_closed_form_silicon():
    # Hand values for E = 130 GPa, nu = 0.28 from eq. 2:
    # lambda = 130000*0.28/(1.28*0.44) = 64630.68..., mu = 130000/2.56 = 50781.25
    lam, mu = fem.lame(*SI[:2])
    assert lam == pytest.approx(36400.0 / 0.5632, rel=1e-15)
    assert mu == pytest.approx(50781.25, rel=1e-15)
    # 3 lambda + 2 mu = E / (1 - 2 nu) (bulk relation)
    for E, nu, _ in (SI, CU, SIO2):
        l, m = fem.lame(E, nu)
        assert 3 * l + 2 * m == pytest.approx(E / (1 - 2 * nu), rel=1e-14)
    # Fully constrained silicon at dT = -250 K: sigma = -E alpha dT / (1 - 2 nu) = 192.045... MPa
    beta = fem.thermal_coefficient(*SI)
    assert -beta * -250.0 == pytest.approx(130000 * 2.6e-6 * 250 / 0.44, rel=1e-14)


def test_elasticity_matrix_responses():
    E, nu, _ = CU
    lam, mu = fem.lame(E, nu)
    D = fem.elasticity_matrix(E, nu)
    # hydrostatic strain e*1 -> (3 lambda + 2 mu) e * 1
    np.testing.assert_allclose(D @ (1e-3 * fem.M_VEC), (3 * lam + 2 * mu) * 1e-3 * fem.M_VEC, rtol=1e-14)
    # engineering shear gamma_xy -> tau = mu gamma
    g = np.zeros(6)
    g[3] = 2e-3
    np.testing.assert_allclose(D @ g, [0, 0, 0, mu * 2e-3, 0, 0], rtol=1e-14, atol=0)
    # uniaxial stress: strain (1, -nu, -nu)/E gives sigma_xx = 1, others 0
    s = D @ np.array([1 / E, -nu / E, -nu / E, 0, 0, 0])
    np.testing.assert_allclose(s, [1, 0, 0, 0, 0, 0], atol=1e-14)


def rigid_modes(coords):
    x, y, z = coords.T
    modes = []
    for t in np.eye(3):
        modes.append(np.tile(t, len(x)))
    for w in np.eye(3):
        disp = np.cross(np.broadcast_to(w, coords.shape), coords)
        modes.append(disp.ravel())
    return np.array(modes).T


def test_ke_symmetric_psd_with_rigid_null_space():
    c = brick()
    Ke, _ = fem.hex8_element(c, fem.elasticity_matrix(*CU[:2]), 1.0)
    np.testing.assert_allclose(Ke, Ke.T, rtol=0, atol=1e-9 * np.abs(Ke).max())
    ev = np.linalg.eigvalsh(Ke)
    scale = ev[-1]
    assert np.all(ev > -1e-12 * scale)
    assert np.sum(ev < 1e-10 * scale) == 6          # exactly the six rigid modes
    R = rigid_modes(c)
    assert np.abs(Ke @ R).max() < 1e-9 * scale


def test_ke_energy_of_uniform_strain_is_exact():
    # Q1 reproduces linear fields, so u = G x has energy V eps^T D eps exactly.
    hx, hy, hz = 1.5, 2.0, 3.5
    c = brick(hx, hy, hz)
    E, nu, _ = SI
    D = fem.elasticity_matrix(E, nu)
    Ke, _ = fem.hex8_element(c, D, 0.0)
    G = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.25, 0.7, 2.0]]) * 1e-3
    u = (c @ G.T).ravel()
    eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[0, 1] + G[1, 0], G[1, 2] + G[2, 1], G[2, 0] + G[0, 2]])
    assert u @ Ke @ u == pytest.approx(hx * hy * hz * eps @ D @ eps, rel=1e-12)


def test_ke_energy_of_bilinear_mode_matches_closed_form():
    # u_x = x y / (hx hy) on [0,hx]x[0,hy]x[0,hz]: eps_xx = y/(hx hy),
    # gamma_xy = x/(hx hy), so the exact energy is
    # (lambda+2mu) hx hz hy^3 / 3 / (hx hy)^2 + mu hy hz hx^3 / 3 / (hx hy)^2.
    # 2x2x2 Gauss integrates the trilinear element exactly; other rules do not.
    hx, hy, hz = 1.5, 2.0, 3.5
    c = brick(hx, hy, hz)
    E, nu, _ = CU
    lam, mu = fem.lame(E, nu)
    Ke, _ = fem.hex8_element(c, fem.elasticity_matrix(E, nu), 0.0)
    u = np.zeros((8, 3))
    u[:, 0] = c[:, 0] * c[:, 1] / (hx * hy)
    u = u.ravel()
    exact = ((lam + 2 * mu) * hx * hz * hy ** 3 / 3 + mu * hy * hz * hx ** 3 / 3) / (hx * hy) ** 2
    assert u @ Ke @ u == pytest.approx(exact, rel=1e-12)


def test_thermal_load_equals_force_of_stress_free_expansion():
    # fe = int B^T beta m = Ke (alpha x): the free thermal strain alpha*1 is
    # linear, and D (alpha m) = beta m.  Pins sign and magnitude of eq. 5.
    c = brick(1.0, 1.2, 0.8)
    E, nu, alpha = SIO2
    Ke, fe = fem.hex8_element(c, fem.elasticity_matrix(E, nu), fem.thermal_coefficient(E, nu, alpha))
    u_free = (alpha * c).ravel()
    np.testing.assert_allclose(fe, Ke @ u_free, rtol=1e-12, atol=1e-12 * np.abs(fe).max())
    # Each corner's load points outward with magnitude beta * (face areas)/4.
    beta = fem.thermal_coefficient(E, nu, alpha)
    areas = np.array([1.2 * 0.8, 1.0 * 0.8, 1.0 * 1.2]) / 4.0
    np.testing.assert_allclose(np.abs(fe.reshape(8, 3)), np.broadcast_to(beta * areas, (8, 3)), rtol=1e-12)
    np.testing.assert_array_equal(np.sign(fe.reshape(8, 3)), fem.HEX_CORNERS)


def cell_spec(mesh=(3, 3, 3), d=0.0, t=0.0, via=CU, liner=SIO2, **kw):
    return W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=4.5, mesh=mesh, tsv_diameter=d,
                      liner_thickness=t, via=via, liner=liner, **kw)


def solve_with_dirichlet(K, b, dofs, vals):
    n = K.shape[0]
    free = np.setdiff1d(np.arange(n), dofs)
    u = np.zeros(n)
    u[dofs] = vals
    Kd = K.toarray()
    u[free] = np.linalg.solve(Kd[np.ix_(free, free)], b[free] - Kd[np.ix_(free, dofs)] @ vals)
    return u


def test_patch_test_linear_trace_is_reproduced():
    spec = cell_spec(mesh=(3, 4, 3))
    cell = fem.Cell(spec)
    K, b, mats = fem.assemble_cell(cell)
    X = cell.node_coords()
    a0 = np.array([0.01, -0.02, 0.03])
    G = np.array([[2.0, 0.5, -1.0], [0.3, -1.0, 0.2], [0.6, 0.1, 1.5]]) * 1e-3
    exact = a0[None, :] + X @ G.T
    bn = np.nonzero(cell.boundary_node_mask())[0]
    dofs = (3 * bn[:, None] + np.arange(3)).ravel()
    u = solve_with_dirichlet(K, 0.0 * b, dofs, exact[bn].ravel())
    np.testing.assert_allclose(u.reshape(-1, 3), exact, rtol=0, atol=1e-12)
    sig = fem.centroid_stress(u, cell.element_dofs(), mats, cell.px / cell.mx,
                              cell.py / cell.my, cell.h / cell.mz, cell.materials, 0.0)
    eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[0, 1] + G[1, 0], G[1, 2] + G[2, 1], G[2, 0] + G[0, 2]])
    expect = fem.elasticity_matrix(*SI[:2]) @ eps
    np.testing.assert_allclose(sig, np.broadcast_to(expect, sig.shape), rtol=1e-10)


def test_fully_constrained_block_is_hydrostatic():
    spec = cell_spec(mesh=(3, 3, 4))
    cell = fem.Cell(spec)
    K, b, mats = fem.assemble_cell(cell)
    dT = -250.0
    bn = np.nonzero(cell.boundary_node_mask())[0]
    dofs = (3 * bn[:, None] + np.arange(3)).ravel()
    u = solve_with_dirichlet(K, dT * b, dofs, np.zeros(dofs.size))
    assert np.abs(u).max() < 1e-14
    sig = fem.centroid_stress(u, cell.element_dofs(), mats, cell.px / cell.mx, cell.py / cell.my,
                              cell.h / cell.mz, cell.materials, dT)
    # sigma = -E alpha dT / (1 - 2 nu) * 1 = +192.045... MPa for silicon
    s0 = 130000.0 * 2.6e-6 * 250.0 / 0.44
    np.testing.assert_allclose(sig, np.broadcast_to([s0, s0, s0, 0, 0, 0], sig.shape), rtol=1e-12, atol=1e-10)
    assert np.abs(fem.von_mises(sig)).max() < 1e-9


def three_two_one(cell):
    """Statically determinate support: node 0 fixed; node (mx,0,0) fixed in y,z;
    node (0,my,0) fixed in z."""
    n0 = cell.node_id(0, 0, 0)
    n1 = cell.node_id(cell.mx, 0, 0)
    n2 = cell.node_id(0, cell.my, 0)
    return np.array([3 * n0, 3 * n0 + 1, 3 * n0 + 2, 3 * n1 + 1, 3 * n1 + 2, 3 * n2 + 2])


@pytest.mark.parametrize("via", [SI, (CU[0], CU[1], SI[2])], ids=["homogeneous", "cu_with_si_alpha"])
def test_free_expansion_is_stress_free(via):
    # A body of uniform alpha expands freely: u = alpha dT (x - x0), sigma = 0,
    # whatever the elastic constants of its parts.
    spec = cell_spec(mesh=(4, 4, 3), d=1.6, t=0.5, via=via, liner=(SIO2[0], SIO2[1], SI[2]))
    cell = fem.Cell(spec)
    K, b, mats = fem.assemble_cell(cell)
    assert len(np.unique(mats)) == 3
    dT = -250.0
    dofs = three_two_one(cell)
    u = solve_with_dirichlet(K, dT * b, dofs, np.zeros(dofs.size))
    X = cell.node_coords()
    np.testing.assert_allclose(u.reshape(-1, 3), SI[2] * dT * X, rtol=0, atol=1e-13)
    sig = fem.centroid_stress(u, cell.element_dofs(), mats, cell.px / cell.mx, cell.py / cell.my,
                              cell.h / cell.mz, cell.materials, dT)
    assert np.abs(sig).max() < 1e-9


def test_mismatched_via_is_not_stress_free():
    # Negative control of the test above: with copper's own alpha there is stress.
    spec = cell_spec(mesh=(4, 4, 3), d=1.6)
    cell = fem.Cell(spec)
    K, b, mats = fem.assemble_cell(cell)
    u = solve_with_dirichlet(K, -250.0 * b, three_two_one(cell), np.zeros(6))
    sig = fem.centroid_stress(u, cell.element_dofs(), mats, cell.px / cell.mx, cell.py / cell.my,
                              cell.h / cell.mz, cell.materials, -250.0)
    assert np.abs(sig).max() > 10.0


def exact_material_count(p, m, d, t):
    """Count of via / liner elements per layer with exact rational arithmetic."""
    P, D, T = Fraction(p), Fraction(d), Fraction(t)
    via = liner = 0
    for eb in range(m):
        for ea in range(m):
            dx = (Fraction(2 * ea + 1, 2)) * P / m - P / 2
            dy = (Fraction(2 * eb + 1, 2)) * P / m - P / 2
            r2 = dx * dx + dy * dy
            if D > 0 and r2 < (D / 2) ** 2:
                via += 1
            elif D > 0 and r2 < (D / 2 + T) ** 2:
                liner += 1
    return via, liner


@pytest.mark.parametrize("p,m,d,t", [(15, 10, 5, 0), (15, 16, 4, 0), (15, 16, 5, 0), (15, 16, 6, 0),
                                      (10, 16, 5, 0), (20, 16, 5, 0), (15, 20, 5, 0.5)])
def test_material_map_matches_exact_rational_count(p, m, d, t):
    spec = W.CellSpec(pitch_x=p, pitch_y=p, mesh=(m, m, 2), tsv_diameter=d, liner_thickness=t)
    mats = fem.Cell(spec).material_map()
    layer = mats[: m * m]
    assert np.array_equal(layer, mats[m * m:])
    via, liner = exact_material_count(p, m, d, t)
    assert int(np.sum(layer == fem.VIA)) == via
    assert int(np.sum(layer == fem.LINER)) == liner
    # the via cross-section approximates pi d^2 / 4
    assert abs(via * (p / m) ** 2 - np.pi * d * d / 4) < 0.5 * np.pi * d * d / 4


def test_von_mises_special_cases():
    s = np.zeros(6)
    s[0] = -7.0
    assert fem.von_mises(s) == pytest.approx(7.0)                 # uniaxial -> |sigma|
    s = np.zeros(6)
    s[4] = 3.0
    assert fem.von_mises(s) == pytest.approx(3.0 * np.sqrt(3.0))  # pure shear -> sqrt(3)|tau|
    assert fem.von_mises(np.array([5.0, 5.0, 5.0, 0, 0, 0])) == pytest.approx(0.0, abs=1e-12)
