"""Pins of the oracle's micro-bump block (the method applied to another
repeated fine structure, Sec. 4.1; micro-bump arrays are named in Sec. 1):
a p x p x h block of underfill with a centred solder column of diameter d
and metal pads of thickness t_pad at both ends.  The material map is checked
against exact rational arithmetic, its symmetries, the reduced model against
the full fine-mesh FEM under static condensation, a z-mirror-symmetric
clamped layer, and free expansion with one common expansion coefficient.
CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import array, fem, mor


def exact_map(p, h, mesh, d, t_pad):
    """Material codes from exact rational centroids: no rounding anywhere."""
    mx, my, mz = mesh
    p, h, d, t_pad = (Fraction(v).limit_denominator(10**6) for v in (p, h, d, t_pad))
    out = []
    for ec in range(mz):
        zc = (ec + Fraction(1, 2)) * h / mz
        assert zc != t_pad and zc != h - t_pad, "tie on a pad face"
        pad = zc < t_pad or zc > h - t_pad
        for eb in range(my):
            dy = (eb + Fraction(1, 2)) * p / my - p / 2
            for ea in range(mx):
                dx = (ea + Fraction(1, 2)) * p / mx - p / 2
                r2 = dx * dx + dy * dy
                assert r2 != (d / 2) ** 2, "tie on the column's surface"
                out.append((fem.PAD if pad else fem.VIA) if r2 < (d / 2) ** 2 else fem.MATRIX)
    return np.array(out, dtype=np.uint8)


@pytest.mark.parametrize("kw", [dict(), dict(mesh=(10, 10, 12), tsv_diameter=17.0, pad_thickness=2.6),
                                dict(pitch_x=30.0, pitch_y=30.0, height=15.0, mesh=(12, 12, 8),
                                     tsv_diameter=21.0, pad_thickness=0.0),
                                dict(mesh=(9, 9, 7), tsv_diameter=30.0, pad_thickness=4.0)])
def test_bump_map_matches_exact_arithmetic(kw):
    spec = W.bump_spec(**kw)
    got = fem.Cell(spec).material_map()
    ref = exact_map(spec.pitch_x, spec.height, spec.mesh, spec.tsv_diameter, spec.pad_thickness)
    np.testing.assert_array_equal(got, ref)
    assert (got == fem.VIA).any() and (got == fem.MATRIX).any()
    assert (got == fem.PAD).any() == (spec.pad_thickness > 0.5 * spec.height / spec.mesh[2])


def test_bump_map_symmetries_and_counts():
    spec = W.bump_spec()
    c = fem.Cell(spec)
    m = c.material_map().reshape(c.mz, c.my, c.mx)
    # Mirror-symmetric in x, y and z, and symmetric under x <-> y.
    np.testing.assert_array_equal(m, m[::-1])
    np.testing.assert_array_equal(m, m[:, ::-1])
    np.testing.assert_array_equal(m, m[:, :, ::-1])
    np.testing.assert_array_equal(m, m.transpose(0, 2, 1))
    # Every layer has the same column cross-section; a layer is all pad or
    # all solder inside it, by its centroid height.
    column = m != fem.MATRIX
    assert all(np.array_equal(column[k], column[0]) for k in range(c.mz))
    zc = (np.arange(c.mz) + 0.5) * c.h / c.mz
    pad_layers = (zc < spec.pad_thickness) | (zc > c.h - spec.pad_thickness)
    for k in range(c.mz):
        assert set(np.unique(m[k][column[k]])) == {fem.PAD if pad_layers[k] else fem.VIA}
    assert pad_layers.sum() == 4      # 16 layers of 1.25 um, 3 um pads: two layers each end
    # A dummy site is pure underfill.
    assert (fem.Cell(spec.dummy()).material_map() == fem.MATRIX).all()


def small_bump(**kw):
    base = dict(pitch_x=8.0, pitch_y=8.0, height=6.0, mesh=(4, 4, 4), tsv_diameter=5.0, pad_thickness=1.0,
                interp=(5, 5, 5))
    base.update(kw)
    return W.bump_spec(**base)


def full_nodal(full, u_full, c):
    cx, cy = c % full.Nx, c // full.Nx
    C, B, A = np.meshgrid(np.arange(full.mz + 1), np.arange(full.my + 1), np.arange(full.mx + 1), indexing="ij")
    g = full.node_id(cx * full.mx + A.ravel(), cy * full.my + B.ravel(), C.ravel())
    return u_full.reshape(-1, 3)[g].ravel()


@pytest.mark.parametrize("top", [False, True], ids=["bottom", "top-and-bottom"])
def test_bump_layer_mor_equals_full_fem_under_static_condensation(top):
    # Lagrange nodes on every boundary FE node (interp = mesh + 1): MOR is
    # static condensation, exact to rounding, for a layer of bumps and
    # missing-bump sites.
    s = small_bump()
    specs = [s, s.dummy()]
    assert (fem.Cell(s).material_map() == fem.PAD).any()
    roms = [mor.local_stage(x) for x in specs]
    t = np.array([0, 1, 0, 0, 0, 1], dtype=np.uint8)          # 3 x 2
    m = array.AbstractMesh(3, 2, s.interp, s.pitch_x, s.pitch_y, s.height)
    dT = -200.0
    dofs, vals = array.constrained_dofs(m, True, top)
    u = array.solve_mor(m, t, roms, dT, dofs, vals)
    full = array.FullArray(specs, t, 3, 2)
    uf, sf = full.solve(dT, True, top)
    sig = array.reconstruct(m, t, roms, u, dT)
    np.testing.assert_allclose(sig, sf, rtol=0, atol=1e-9 * np.abs(sf).max())
    for c in range(m.n_cells):
        np.testing.assert_allclose(array.nodal_displacement(m, t, roms, u, dT, c), full_nodal(full, uf, c),
                                   rtol=0, atol=1e-11 * np.abs(uf).max())


def test_clamped_bump_layer_is_mirror_symmetric_in_z():
    # The block is symmetric about its mid-height and so is a layer clamped
    # at both faces: normal and xy stresses even in z, yz and zx odd.
    s = small_bump(interp=(3, 3, 3))
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 2, s.interp, s.pitch_x, s.pitch_y, s.height)
    t = np.zeros(4, dtype=np.uint8)
    dofs, vals = array.constrained_dofs(m, True, True)
    u = array.solve_mor(m, t, [rom], -200.0, dofs, vals)
    g = array.reconstruct(m, t, [rom], u, -200.0).reshape(4, 4, 4, 4, 6)   # [cell, z, y, x, comp]
    tol = 1e-9 * np.abs(g).max()
    fz = g[:, ::-1]
    np.testing.assert_allclose(fz[..., [0, 1, 2, 3]], g[..., [0, 1, 2, 3]], atol=tol)
    np.testing.assert_allclose(fz[..., [4, 5]], -g[..., [4, 5]], atol=tol)
    # The pads and the solder are loaded differently from the underfill.
    vm = fem.von_mises(g.reshape(-1, 6)).reshape(4, 4, 4, 4)
    mat = fem.Cell(s).material_map().reshape(4, 4, 4)
    assert abs(vm[0][mat == fem.VIA].mean() - vm[0][mat == fem.MATRIX].mean()) > 1.0


def test_free_expansion_with_one_common_alpha_is_stress_free():
    a = 20e-6
    s = small_bump(interp=(3, 3, 3), matrix=(8.0e3, 0.30, a), via=(50.0e3, 0.36, a), liner=(110.0e3, 0.35, a))
    rom = mor.local_stage(s)
    m = array.AbstractMesh(2, 2, s.interp, s.pitch_x, s.pitch_y, s.height)
    t = np.zeros(4, dtype=np.uint8)
    n0 = m.node_id[0, 0, 0]
    n1 = m.node_id[0, 0, m.X - 1]
    n2 = m.node_id[0, m.Y - 1, 0]
    dofs = np.array([3 * n0, 3 * n0 + 1, 3 * n0 + 2, 3 * n1 + 1, 3 * n1 + 2, 3 * n2 + 2])
    u = array.solve_mor(m, t, [rom], -200.0, dofs, np.zeros(6))
    np.testing.assert_allclose(u.reshape(-1, 3), a * -200.0 * m.coords, rtol=0, atol=1e-13)
    sig = array.reconstruct(m, t, [rom], u, -200.0)
    assert np.abs(sig).max() < 1e-8
