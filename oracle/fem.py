"""Oracle, part 1: linear thermo-elastic finite elements on one unit cell.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Units throughout: micrometres, MPa (= N/mm^2), 1/K and K.

What is computed, with the passage it follows:

* Lame parameters from E and nu (Sec. 3.1, eq. 2).
* Constitutive law sigma = lambda tr(eps) 1 + 2 mu eps - alpha(3 lambda + 2 mu)
  dT 1 and eps = sym grad u (Sec. 3.1, eq. 1).
* Weak form a(u, v) = L(v) with a the elastic energy product (eq. 4) and
  L(v) = int alpha(3 lambda + 2 mu) dT 1 : eps(v) (eq. 5); body force is zero
  and boundaries are clamped or free (Sec. 3.2).  Discretised with shape
  functions into A alpha = b (eq. 6-7).
* The unit block: a p x p x h silicon cuboid with a centred copper via of
  diameter d and an optional dielectric liner of thickness t (Sec. 4.2,
  Fig. 2).  The method applies to any repeated fine structure (Sec. 4.1); a
  micro-bump block (a solder column with metal pads at both ends, in
  underfill) is the second structure built here, read as stated in
  ``Cell.material_map``.

Readings where the paper is silent: the element is
the trilinear 8-node hexahedron with 2x2x2 Gauss quadrature; the mesh is a
structured m_x x m_y x m_z grid; an element belongs to the via if its
centroid lies strictly inside radius d/2 of the via axis, to the liner if
strictly inside d/2 + t, and to the matrix otherwise.
"""
import math

import numpy as np
import scipy.sparse as sp

# Material codes used by the cell material map.  A micro-bump block uses the
# same three slots: underfill (MATRIX), solder column (VIA), pads (LINER).
MATRIX, VIA, LINER = 0, 1, 2
PAD = LINER

# Voigt order of the strain and stress vectors; shears are engineering shears.
VOIGT = ("xx", "yy", "zz", "xy", "yz", "zx")
M_VEC = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])  # Voigt form of the unit tensor 1


def lame(E, nu):
    """Lame parameters (lambda, mu) from Young's modulus and Poisson ratio (eq. 2)."""
    lam = E * nu / (1.0 + nu) / (1.0 - 2.0 * nu)
    mu = E / 2.0 / (1.0 + nu)
    return lam, mu


def thermal_coefficient(E, nu, alpha):
    """alpha (3 lambda + 2 mu): the factor multiplying dT 1 in eq. 1."""
    lam, mu = lame(E, nu)
    return alpha * (3.0 * lam + 2.0 * mu)


def elasticity_matrix(E, nu):
    """6x6 matrix of lambda tr(eps) 1 + 2 mu eps (eq. 1) acting on the Voigt
    strain [exx, eyy, ezz, gxy, gyz, gzx] with engineering shears g = 2 eps."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    for i in range(3):
        D[i, i] = lam + 2.0 * mu
        D[3 + i, 3 + i] = mu
    return D


# ----------------------------------------------------------------------------
# Trilinear hexahedron
# ----------------------------------------------------------------------------
# Local node l = la + 2*lb + 4*lc sits at reference corner (2la-1, 2lb-1, 2lc-1).
HEX_CORNERS = np.array([[2 * (l & 1) - 1, 2 * ((l >> 1) & 1) - 1, 2 * ((l >> 2) & 1) - 1]
                        for l in range(8)], dtype=float)


def hex8_reference_gradients(xi, eta, zeta):
    """d N_l / d(xi, eta, zeta) of the eight trilinear shape functions
    N_l = (1 + xi_l xi)(1 + eta_l eta)(1 + zeta_l zeta) / 8.  Shape (8, 3)."""
    g = np.zeros((8, 3))
    for l in range(8):
        a, b, c = HEX_CORNERS[l]
        g[l, 0] = a * (1 + b * eta) * (1 + c * zeta) / 8.0
        g[l, 1] = b * (1 + a * xi) * (1 + c * zeta) / 8.0
        g[l, 2] = c * (1 + a * xi) * (1 + b * eta) / 8.0
    return g


def strain_displacement(dN_dx):
    """6 x 24 matrix B with eps_voigt = B u_e, u_e = [u0x,u0y,u0z,u1x,...]
    (eq. 1, third line, in Voigt form)."""
    B = np.zeros((6, 24))
    for l in range(8):
        dx, dy, dz = dN_dx[l]
        c = 3 * l
        B[0, c + 0] = dx
        B[1, c + 1] = dy
        B[2, c + 2] = dz
        B[3, c + 0] = dy
        B[3, c + 1] = dx
        B[4, c + 1] = dz
        B[4, c + 2] = dy
        B[5, c + 0] = dz
        B[5, c + 2] = dx
    return B


def hex8_physical_gradients(coords, xi, eta, zeta):
    """Shape-function gradients in physical coordinates and det J at a point."""
    dN = hex8_reference_gradients(xi, eta, zeta)
    J = dN.T @ coords                      # J[a, b] = sum_l dN_l/dxi_a * x_l,b
    detJ = np.linalg.det(J)
    dN_dx = np.linalg.solve(J, dN.T).T     # grad_x N = J^{-1} grad_xi N
    return dN_dx, detJ


def hex8_element(coords, D, beta):
    """Element stiffness Ke = int B^T D B and unit-dT thermal load
    fe = int B^T (beta m) for one hexahedron (eq. 4 and 5 restricted to the
    element), with 2x2x2 Gauss quadrature.  coords: (8, 3) in local order."""
    g = 1.0 / math.sqrt(3.0)
    Ke = np.zeros((24, 24))
    fe = np.zeros(24)
    for zeta in (-g, g):
        for eta in (-g, g):
            for xi in (-g, g):
                dN_dx, detJ = hex8_physical_gradients(coords, xi, eta, zeta)
                B = strain_displacement(dN_dx)
                Ke += B.T @ D @ B * detJ
                fe += B.T @ (beta * M_VEC) * detJ
    return Ke, fe


def centroid_B(coords):
    """B evaluated at the element centroid (xi = eta = zeta = 0)."""
    dN_dx, _ = hex8_physical_gradients(coords, 0.0, 0.0, 0.0)
    return strain_displacement(dN_dx)


def von_mises(sig):
    """Von Mises stress of Voigt stress rows [..., 6] = xx, yy, zz, xy, yz, zx."""
    sxx, syy, szz, sxy, syz, szx = (sig[..., i] for i in range(6))
    return np.sqrt(0.5 * ((sxx - syy) ** 2 + (syy - szz) ** 2 + (szz - sxx) ** 2)
                   + 3.0 * (sxy ** 2 + syz ** 2 + szx ** 2))


# ----------------------------------------------------------------------------
# Unit cell (Sec. 4.2, Fig. 2)
# ----------------------------------------------------------------------------
class Cell:
    """Structured hexahedral mesh of one unit block with its material map.

    ``spec`` is any object with attributes pitch_x, pitch_y, height, mesh
    (m_x, m_y, m_z), tsv_diameter, liner_thickness, matrix, via, liner (each
    an (E, nu, alpha) triple) and interp (n_x, n_y, n_z).

    Numbering: FE node (a, b, c) has id (c (m_y+1) + b)(m_x+1) + a, DoF
    3 id + component; element (ea, eb, ec) has id (ec m_y + eb) m_x + ea.
    """

    def __init__(self, spec):
        self.spec = spec
        self.px, self.py, self.h = float(spec.pitch_x), float(spec.pitch_y), float(spec.height)
        self.mx, self.my, self.mz = (int(v) for v in spec.mesh)
        self.materials = [tuple(spec.matrix), tuple(spec.via), tuple(spec.liner)]
        # x += skew * y: a parallelepiped block (skew = 1/sqrt(3) with
        # p_y = p sqrt(3)/2 is the rhombic block of a 120-degree array).
        self.skew = float(getattr(spec, "skew", 0.0))
        self.n_nodes = (self.mx + 1) * (self.my + 1) * (self.mz + 1)
        self.n_dofs = 3 * self.n_nodes
        self.n_elem = self.mx * self.my * self.mz

    def node_id(self, a, b, c):
        return (c * (self.my + 1) + b) * (self.mx + 1) + a

    def ref_coords(self):
        """(n_nodes, 3) reference coordinates; node (a,b,c) at
        (p_x a/m_x, p_y b/m_y, h c/m_z)."""
        a = np.arange(self.mx + 1)
        b = np.arange(self.my + 1)
        c = np.arange(self.mz + 1)
        C, B_, A = np.meshgrid(c, b, a, indexing="ij")
        x = self.px * A / self.mx
        y = self.py * B_ / self.my
        z = self.h * C / self.mz
        return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)

    def node_coords(self):
        """(n_nodes, 3) physical coordinates: the reference ones with
        x += skew * y."""
        X = self.ref_coords()
        X[:, 0] = X[:, 0] + self.skew * X[:, 1]
        return X

    def element_nodes(self):
        """(n_elem, 8) FE node ids of every element, local order la+2lb+4lc."""
        ea = np.arange(self.mx)
        eb = np.arange(self.my)
        ec = np.arange(self.mz)
        EC, EB, EA = np.meshgrid(ec, eb, ea, indexing="ij")
        EA, EB, EC = EA.ravel(), EB.ravel(), EC.ravel()
        nodes = np.zeros((self.n_elem, 8), dtype=np.int64)
        for l in range(8):
            la, lb, lc = l & 1, (l >> 1) & 1, (l >> 2) & 1
            nodes[:, l] = self.node_id(EA + la, EB + lb, EC + lc)
        return nodes

    def element_dofs(self):
        en = self.element_nodes()
        return (3 * en[:, :, None] + np.arange(3)[None, None, :]).reshape(self.n_elem, 24)

    def material_map(self):
        """Material code per element from the centroid's distance r to the
        block's vertical axis through its centre ((p_x/2, p_y/2), sheared like
        every point of a skewed block), strict comparisons of squared
        distances.  TSV block: via if r < d/2, liner if r < d/2 + t,
        matrix otherwise.  Micro-bump block (structure "bump"): inside the
        column (r < d/2) a pad if the centroid height z < t_pad or
        z > h - t_pad, solder otherwise; underfill outside."""
        d = float(self.spec.tsv_diameter)
        t = float(self.spec.liner_thickness)
        bump = getattr(self.spec, "structure", "tsv") == "bump"
        t_pad = float(getattr(self.spec, "pad_thickness", 0.0))
        out = np.full(self.n_elem, MATRIX, dtype=np.uint8)
        r_via2 = (d / 2.0) ** 2
        r_lin2 = (d / 2.0 + t) ** 2
        e = 0
        for ec in range(self.mz):
            zc = (ec + 0.5) * self.h / self.mz
            in_pad = zc < t_pad or zc > self.h - t_pad
            for eb in range(self.my):
                dy = (eb + 0.5) * self.py / self.my - self.py / 2.0
                for ea in range(self.mx):
                    # Offset from the axis through the block's centre (the
                    # centroid and the centre both sheared by skew * y).
                    dx = ((ea + 0.5) * self.px / self.mx - self.px / 2.0) + self.skew * dy
                    r2 = dx * dx + dy * dy
                    if bump:
                        if d > 0.0 and r2 < r_via2:
                            out[e] = PAD if in_pad else VIA
                    elif d > 0.0 and r2 < r_via2:
                        out[e] = VIA
                    elif d > 0.0 and r2 < r_lin2:
                        out[e] = LINER
                    e += 1
        return out

    def element_coords(self, e_nodes=None):
        X = self.node_coords()
        if e_nodes is None:
            e_nodes = self.element_nodes()
        return X[e_nodes]                           # (n_elem, 8, 3)

    def boundary_node_mask(self):
        """True for FE nodes on the surface of the block."""
        a = np.arange(self.mx + 1)
        b = np.arange(self.my + 1)
        c = np.arange(self.mz + 1)
        C, B_, A = np.meshgrid(c, b, a, indexing="ij")
        m = (A == 0) | (A == self.mx) | (B_ == 0) | (B_ == self.my) | (C == 0) | (C == self.mz)
        return m.ravel()


def assemble(n_dofs, elem_dofs, elem_mats, element_table):
    """Standard FE assembly (Sec. 3.2): K = sum_e P_e^T Ke P_e, b = sum_e P_e^T fe.

    element_table maps a material code to (Ke, fe) for the (identical) brick
    elements of a structured mesh.  Returns (K as CSR, b)."""
    rows, cols, vals = [], [], []
    b = np.zeros(n_dofs)
    for code, (Ke, fe) in element_table.items():
        sel = np.nonzero(elem_mats == code)[0]
        if sel.size == 0:
            continue
        dofs = elem_dofs[sel]                                   # (ne, 24)
        rows.append(np.repeat(dofs, 24, axis=1).ravel())
        cols.append(np.tile(dofs, (1, 24)).ravel())
        vals.append(np.broadcast_to(Ke.ravel(), (sel.size, 576)).ravel())
        np.add.at(b, dofs.ravel(), np.broadcast_to(fe, (sel.size, 24)).ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_dofs, n_dofs)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K, b


def element_corners(hx, hy, hz, skew=0.0):
    """Corner coordinates (local order) of one element of the structured
    grid: an hx x hy x hz brick, sheared by x += skew * y for a skewed block
    (a parallelepiped; skew 0 leaves the brick as it is)."""
    coords = (HEX_CORNERS + 1.0) / 2.0 * np.array([hx, hy, hz])
    coords[:, 0] = coords[:, 0] + skew * coords[:, 1]
    return coords


def brick_element_table(hx, hy, hz, materials, codes, skew=0.0):
    """(Ke, fe) for each material code of one element of the structured grid
    (an hx x hy x hz brick, sheared by `skew`)."""
    coords = element_corners(hx, hy, hz, skew)
    table = {}
    for code in codes:
        E, nu, alpha = materials[code]
        table[int(code)] = hex8_element(coords, elasticity_matrix(E, nu),
                                        thermal_coefficient(E, nu, alpha))
    return table


def assemble_cell(cell):
    """Stiffness K and unit-dT thermal load b of one unit block (eq. 11 with
    dT = 1).  Returns (K CSR, b, material map)."""
    mats = cell.material_map()
    table = brick_element_table(cell.px / cell.mx, cell.py / cell.my, cell.h / cell.mz,
                                cell.materials, np.unique(mats), cell.skew)
    K, b = assemble(cell.n_dofs, cell.element_dofs(), mats, table)
    return K, b, mats


def centroid_stress(u, elem_dofs, elem_mats, hx, hy, hz, materials, dT, skew=0.0):
    """sigma = D B0 u_e - alpha(3 lambda + 2 mu) dT m at the centroid of every
    element of the structured grid (hx x hy x hz bricks, sheared by `skew`)
    (eq. 1).  u may be (n_dofs,) or (n_dofs, k) for k displacement fields at
    once.  Returns (n_elem, 6) or (n_elem, 6, k)."""
    coords = element_corners(hx, hy, hz, skew)
    B0 = centroid_B(coords)
    single = u.ndim == 1
    U = u[:, None] if single else u
    out = np.zeros((len(elem_dofs), 6, U.shape[1]))
    for code in np.unique(elem_mats):
        E, nu, alpha = materials[int(code)]
        DB = elasticity_matrix(E, nu) @ B0
        beta = thermal_coefficient(E, nu, alpha)
        sel = np.nonzero(elem_mats == code)[0]
        ue = U[elem_dofs[sel]]                              # (ne, 24, k)
        out[sel] = np.einsum("ij,ejk->eik", DB, ue) - (beta * dT * M_VEC)[None, :, None]
    return out[:, :, 0] if single else out
