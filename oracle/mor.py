"""Oracle, part 2: the one-shot local stage of MORE-Stress (Sec. 4.2) and the
element matrices of the abstract cell element (Sec. 4.3, eq. 17-19).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order and notation:

1. Equally spaced Lagrange nodes (n_x, n_y, n_z) on the corners and surfaces
   of the block; 1D Lagrange polynomials (eq. 9) and their tensor product
   L_3D (eq. 8); the boundary displacement approximated per component by
   eq. 10; the number of retained nodal components n (eq. 16).
2. The Dirichlet problem of the block A_local alpha = dT b_local split into
   free and boundary DoFs (eq. 11-12); lifting gives
   A_ff alpha_f = dT b_f - A_f,bc u_bc (eq. 13).
3. Substituting u_bc = L u_nodes (eq. 14) and solving once per nodal
   component (dT = 0, that component 1, the others 0) gives f_i; solving with
   dT = 1 and all nodal values 0 gives f_T (eq. 15).  One factorisation of
   A_ff serves all n + 1 right-hand sides.
4. A_element = Phi^T A_local Phi (eq. 18) and b_element = Phi^T b_local
   (eq. 19, per unit dT), with Phi = [f_0 ... f_{n-1}] and the un-lifted
   A_local.

Readings of the paper: node coordinates x_i = p i / (n_x - 1); the
surface node set is ordered lexicographically in (k, j, i) with i fastest and
the reduced DoF is 3 s + component, which fixes eq. 14's vector order beyond
its first and last entries; eq. 14's "b_{local,}f" is b_{local,f}; eq. 18-19's
coefficient vectors are the basis functions' FE coefficients and A_local /
b_local are the un-lifted assembled matrix and vector; A_element is
symmetrised as (A + A^T)/2.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fem


def interp_points(length, n):
    """Equally spaced interpolation coordinates on [0, length], corners included."""
    return np.array([length * i / (n - 1) for i in range(n)], dtype=float)


def lagrange_1d(x, nodes, i):
    """L_1D(x; i) of eq. 9: prod_{j != i} (x - x_j) / (x_i - x_j)."""
    x = np.asarray(x, dtype=float)
    num = np.ones_like(x)
    den = 1.0
    for j in range(len(nodes)):
        if j == i:
            continue
        num = num * (x - nodes[j])
        den = den * (nodes[i] - nodes[j])
    return num / den


def n_reduced(nx, ny, nz):
    """Number of local basis functions f_i, eq. 16."""
    return (nx * ny * nz - (nx - 2) * (ny - 2) * (nz - 2)) * 3


def surface_nodes(nx, ny, nz):
    """Interpolation nodes (i, j, k) on the corners and surfaces of the block,
    in (k, j, i) lexicographic order with i fastest."""
    out = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if i in (0, nx - 1) or j in (0, ny - 1) or k in (0, nz - 1):
                    out.append((i, j, k))
    return out


def interpolation_matrix(cell):
    """Matrix L of eq. 14: rows are the boundary FE DoFs of the cell (ascending
    DoF order), columns the reduced DoFs 3 s + component; entry
    L_3D(r_node; i, j, k) (eq. 8) on matching components, 0 otherwise (eq. 10).

    Returns (L, bc_dofs, S) with S the surface node list."""
    nx, ny, nz = (int(v) for v in cell.spec.interp)
    S = surface_nodes(nx, ny, nz)
    xs = interp_points(cell.px, nx)
    ys = interp_points(cell.py, ny)
    zs = interp_points(cell.h, nz)
    # Interpolation in the block's reference coordinates (those of its
    # structured grid): for a skewed block the faces stay parameterised alike
    # on both blocks that share them.
    X = cell.ref_coords()
    bnodes = np.nonzero(cell.boundary_node_mask())[0]
    P = X[bnodes]
    W = np.zeros((len(bnodes), len(S)))
    for s, (i, j, k) in enumerate(S):
        W[:, s] = (lagrange_1d(P[:, 0], xs, i) * lagrange_1d(P[:, 1], ys, j)
                   * lagrange_1d(P[:, 2], zs, k))
    n = 3 * len(S)
    L = np.zeros((3 * len(bnodes), n))
    for comp in range(3):
        L[comp::3, comp::3] = W
    bc_dofs = (3 * bnodes[:, None] + np.arange(3)[None, :]).ravel()
    return L, bc_dofs, S


def _factor_and_solve(A, R):
    """Cholesky-factorise the SPD matrix A once (LAPACK banded, natural order)
    and solve for all columns of R."""
    A = A.tocoo()
    n = A.shape[0]
    low = A.row >= A.col
    bw = int((A.row - A.col)[low].max()) if n else 0
    if (bw + 1) * n * 8 > 2 ** 31:
        return spla.splu(A.tocsc()).solve(R)
    ab = np.zeros((bw + 1, n))
    np.add.at(ab, ((A.row - A.col)[low], A.col[low]), A.data[low])
    return sla.cho_solve_banded((sla.cholesky_banded(ab, lower=True), True), R)


class ReducedCell:
    """Output of the local stage for one cell type: the basis Phi (n_dofs x n),
    f_T (n_dofs), A_element = K_r (n x n), b_element per unit dT = b_r (n),
    plus the cell, its assembled K and b and the material map."""

    def __init__(self, cell, K, b, mats, Phi, fT, Kr, br, L, bc_dofs, free_dofs, S, residual):
        self.cell, self.K, self.b, self.mats = cell, K, b, mats
        self.Phi, self.fT, self.Kr, self.br = Phi, fT, Kr, br
        self.L, self.bc_dofs, self.free_dofs, self.S = L, bc_dofs, free_dofs, S
        self.local_residual = residual
        self.n = Phi.shape[1]


def local_stage(spec):
    """One-shot local stage for one cell type (Sec. 4.2, eq. 11-19)."""
    cell = fem.Cell(spec)
    K, b, mats = fem.assemble_cell(cell)                        # eq. 11-12
    L, bc_dofs, S = interpolation_matrix(cell)                  # eq. 8-10, 14
    n = L.shape[1]
    is_bc = np.zeros(cell.n_dofs, dtype=bool)
    is_bc[bc_dofs] = True
    free_dofs = np.nonzero(~is_bc)[0]
    K_ff = K[free_dofs][:, free_dofs].tocsc()
    K_fb = K[free_dofs][:, bc_dofs]
    # eq. 13-14: right-hand sides for the n unit nodal components (dT = 0)
    # and for the thermal load (dT = 1, zero nodal values).
    R = np.empty((len(free_dofs), n + 1))
    R[:, :n] = -(K_fb @ L)
    R[:, n] = b[free_dofs]
    Xf = _factor_and_solve(K_ff, R)                             # one factorisation
    residual = np.linalg.norm(K_ff @ Xf - R) / np.linalg.norm(R)
    # eq. 15: f_i and f_T on the whole cell.
    Phi = np.zeros((cell.n_dofs, n))
    Phi[free_dofs] = Xf[:, :n]
    Phi[bc_dofs] = L
    fT = np.zeros(cell.n_dofs)
    fT[free_dofs] = Xf[:, n]
    # eq. 18-19 with the un-lifted A_local and b_local.
    KPhi = K @ Phi
    Kr = Phi.T @ KPhi
    Kr = 0.5 * (Kr + Kr.T)
    br = Phi.T @ b
    return ReducedCell(cell, K, b, mats, Phi, fT, Kr, br, L, bc_dofs, free_dofs, S, residual)
