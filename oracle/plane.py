"""Oracle, part 4: the paper's evaluation of a stress field (Sec. 5.1, the
error metric of Tables 1-3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper samples von Mises stress on the mid-height plane of every block,
on a regular grid of 100 x 100 points per block, and reports the mean
absolute difference from the reference field divided by the reference
field's maximum.  Here:

1. Sample points.  Point (i, j) of a g x g grid sits at
   x = p_x (i + 1/2) / g, y = p_y (j + 1/2) / g, z = h / 2 inside its block
   (the grid's cell centres, so no point lies on a block's outer face).
2. Element lookup.  A point belongs to the fine element whose half-open box
   [x_a, x_{a+1}) x [y_b, y_{b+1}) x [z_c, z_{c+1}) holds it (so a point on
   an element face goes to the element on its +x / +y / +z side); the
   lookup is done in exact rational arithmetic.  With an even number of
   element layers the plane z = h/2 is the bottom face of layer m_z / 2
   (zeta = -1); with an odd number it cuts layer (m_z - 1) / 2 through the
   middle (zeta = 0).
3. Stress at the point (eq. 1): the nodal displacement of the block is
   dT f_T + Phi u_block (eq. 15); sigma = D B(xi, eta, zeta) u_e - beta dT m
   with B the trilinear element's strain-displacement matrix at the point's
   reference coordinates.
4. Metric: normalised MAE = mean |vm - vm_ref| / max |vm_ref| over all
   sampled points of all blocks (the paper's), and the max-norm relative
   error max |vm - vm_ref| / max |vm_ref|.
"""
from fractions import Fraction

import numpy as np

from . import fem


def plane_points(cell, g):
    """The g x g sample points of one block, point p = j g + i.

    Returns (elem (g*g,) element ids, ref (g*g, 3) reference coordinates
    (xi, eta, zeta), xyz (g*g, 3) physical coordinates)."""
    if cell.skew != 0.0:
        raise ValueError("the evaluation plane is defined for rectangular blocks (skew 0)")
    g = int(g)
    mx, my, mz = cell.mx, cell.my, cell.mz
    elem = np.zeros(g * g, dtype=np.int64)
    ref = np.zeros((g * g, 3))
    xyz = np.zeros((g * g, 3))
    # Position in element widths along each axis, exact.
    tz = Fraction(mz, 2)
    ec = tz.numerator // tz.denominator
    zeta = float(2 * (tz - ec) - 1)
    for j in range(g):
        ty = Fraction(my * (2 * j + 1), 2 * g)
        eb = ty.numerator // ty.denominator
        eta = float(2 * (ty - eb) - 1)
        for i in range(g):
            tx = Fraction(mx * (2 * i + 1), 2 * g)
            ea = tx.numerator // tx.denominator
            xi = float(2 * (tx - ea) - 1)
            p = j * g + i
            elem[p] = (ec * my + eb) * mx + ea
            ref[p] = (xi, eta, zeta)
            xyz[p] = (cell.px * (2 * i + 1) / (2 * g), cell.py * (2 * j + 1) / (2 * g), cell.h / 2.0)
    return elem, ref, xyz


def point_stress_operators(cell, mats, g):
    """Per sample point: the element DoFs (g*g, 24), D B at the point
    (g*g, 6, 24) and beta m (g*g, 6) of the element's material."""
    elem, ref, _ = plane_points(cell, g)
    hx, hy, hz = cell.px / cell.mx, cell.py / cell.my, cell.h / cell.mz
    coords = (fem.HEX_CORNERS + 1.0) / 2.0 * np.array([hx, hy, hz])
    edofs = cell.element_dofs()[elem]
    DB = np.zeros((len(elem), 6, 24))
    bm = np.zeros((len(elem), 6))
    for p in range(len(elem)):
        E, nu, alpha = cell.materials[int(mats[elem[p]])]
        dN_dx, _ = fem.hex8_physical_gradients(coords, *ref[p])
        DB[p] = fem.elasticity_matrix(E, nu) @ fem.strain_displacement(dN_dx)
        bm[p] = fem.thermal_coefficient(E, nu, alpha) * fem.M_VEC
    return edofs, DB, bm


def block_plane_stress(cell, mats, nodal, dT, g):
    """Stress (g*g, 6) on the mid-height plane of one block from its fine
    nodal displacement (n_dofs,) (eq. 1)."""
    edofs, DB, bm = point_stress_operators(cell, mats, g)
    return np.einsum("pij,pj->pi", DB, nodal[edofs]) - dT * bm


def plane_stress(mesh, cell_type, roms, u, dT, g, chunk=64):
    """Mid-height plane stress of every block of an array from the reduced
    solution u (eq. 15, then eq. 1 at the sample points).
    Returns sigma (n_cells, g*g, 6)."""
    dofs = mesh.cell_dofs()
    out = np.zeros((mesh.n_cells, g * g, 6))
    for t in np.unique(cell_type):
        rom = roms[int(t)]
        edofs, DB, bm = point_stress_operators(rom.cell, rom.mats, g)
        cells = np.nonzero(cell_type == t)[0]
        for s in range(0, len(cells), chunk):
            cs = cells[s:s + chunk]
            nodal = dT * rom.fT[:, None] + rom.Phi @ u[dofs[cs]].T          # (n_dofs, k)
            sig = np.einsum("pij,pjk->kpi", DB, nodal[edofs]) - dT * bm[None]
            out[cs] = sig
    return out


def plane_von_mises(mesh, cell_type, roms, u, dT, g):
    """Von Mises stress (n_cells, g*g) on the sample grid."""
    return fem.von_mises(plane_stress(mesh, cell_type, roms, u, dT, g))


def normalized_mae(vm, vm_ref):
    """The paper's error: mean |vm - vm_ref| over all points / max |vm_ref|."""
    vm = np.asarray(vm, dtype=float).ravel()
    vm_ref = np.asarray(vm_ref, dtype=float).ravel()
    return float(np.mean(np.abs(vm - vm_ref)) / np.max(np.abs(vm_ref)))


def max_rel_error(vm, vm_ref):
    """max |vm - vm_ref| / max |vm_ref| (the max-norm gate)."""
    vm = np.asarray(vm, dtype=float).ravel()
    vm_ref = np.asarray(vm_ref, dtype=float).ravel()
    return float(np.max(np.abs(vm - vm_ref)) / np.max(np.abs(vm_ref)))


def full_plane_von_mises(full, u, dT, g):
    """Von Mises (n_cells, g*g) on the sample grid of every block of a full
    fine-mesh solution (array.FullArray and its nodal u): each block's fine
    nodal displacement is read from the global mesh (block (cx, cy) local
    node (a, b, c) is global node (cx m_x + a, cy m_y + b, c)), then eq. 1 at
    the sample points as for a reduced solution."""
    out = np.zeros((full.Nx * full.Ny, g * g))
    c = np.arange(full.mz + 1)[:, None, None]
    b = np.arange(full.my + 1)[None, :, None]
    a = np.arange(full.mx + 1)[None, None, :]
    for cy in range(full.Ny):
        for cx in range(full.Nx):
            k = cy * full.Nx + cx
            cell = full.cells[int(full.cell_type[k])]
            # Local node ids run (c, b, a) with a fastest, as the broadcast below.
            glob = full.node_id(cx * full.mx + a, cy * full.my + b, c).ravel()
            nodal = u.reshape(-1, 3)[glob].ravel()
            out[k] = fem.von_mises(block_plane_stress(cell, cell.material_map(), nodal, dT, g))
    return out
