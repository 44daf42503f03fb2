"""Oracle, part 3: the global stage of MORE-Stress (Sec. 4.3-4.4) and the full
fine-mesh FEM of a whole TSV array to compare it with.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order:

1. Each unit block is an abstract element whose DoFs are its nodal
   displacement components; the array is an abstract mesh whose DoFs are all
   nodal components, shared between neighbouring blocks (Sec. 4.3).
2. Standard FE assembly of A_global and b_global from A_element and
   dT b_element of each block's type (Sec. 4.3; hybrid TSV/dummy arrays,
   Sec. 4.4).
3. Dirichlet data (clamped faces, or displacement values taken from a coarse
   model for sub-modelling) imposed by lifting (Sec. 4.2 eq. 13, Sec. 4.4).
4. Solve A_global u = b_global (eq. 20).
5. Per block, the displacement dT f_T + sum_i u_i f_i (eq. 15) and from it the
   strain and stress (eq. 1).

Readings of the paper: the abstract-mesh node at lattice point
(I, J, K) has id equal to its rank in (K, J, I) lexicographic order with I
fastest; block (cx, cy) has id cy N_x + cx and its surface node (i, j, k) sits
at (cx (n_x-1) + i, cy (n_y-1) + j, k); lifting is the symmetric form (rows
and columns of constrained DoFs replaced by identity, known values moved to
the right-hand side), which has the same solution as the row-only form of
eq. 13 and keeps the matrix symmetric; sums over blocks run in ascending
block id; stress is reported at element centroids.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from . import mor


class AbstractMesh:
    """Numbering of the abstract mesh of an N_x x N_y array of blocks with
    (n_x, n_y, n_z) interpolation nodes per block (Sec. 4.3).  With
    nz_cells = N_z > 1 the array holds N_z layers of blocks stacked in z that
    share their horizontal faces (a stacked variant of the same abstract
    mesh: block (cx, cy, cz) has id (cz N_y + cy) N_x + cx and its surface
    node (i, j, k) sits at lattice point (cx (n_x-1) + i, cy (n_y-1) + j,
    cz (n_z-1) + k))."""

    def __init__(self, nx_cells, ny_cells, interp, pitch_x=1.0, pitch_y=1.0, height=1.0, nz_cells=1, skew=0.0):
        self.Nx, self.Ny, self.Nz = int(nx_cells), int(ny_cells), int(nz_cells)
        self.nx, self.ny, self.nz = (int(v) for v in interp)
        self.X = self.Nx * (self.nx - 1) + 1
        self.Y = self.Ny * (self.ny - 1) + 1
        self.Z = self.Nz * (self.nz - 1) + 1
        K, J, I = np.meshgrid(np.arange(self.Z), np.arange(self.Y), np.arange(self.X), indexing="ij")
        is_node = ((I % (self.nx - 1) == 0) | (J % (self.ny - 1) == 0)
                   | (K % (self.nz - 1) == 0))
        self.node_id = np.full(is_node.shape, -1, dtype=np.int64)
        self.node_id[is_node] = np.arange(int(is_node.sum()))
        self.n_nodes = int(is_node.sum())
        self.n_dofs = 3 * self.n_nodes
        self.lattice = np.stack([I[is_node], J[is_node], K[is_node]], axis=1)   # (n_nodes, 3)
        self.coords = np.stack([pitch_x * self.lattice[:, 0] / (self.nx - 1),
                                pitch_y * self.lattice[:, 1] / (self.ny - 1),
                                height * self.lattice[:, 2] / (self.nz - 1)], axis=1)
        self.coords[:, 0] = self.coords[:, 0] + skew * self.coords[:, 1]     # skewed blocks
        S = mor.surface_nodes(self.nx, self.ny, self.nz)
        self.n_local = 3 * len(S)
        n_cells = self.Nx * self.Ny * self.Nz
        self.conn = np.zeros((n_cells, len(S)), dtype=np.int64)
        for cz in range(self.Nz):
            for cy in range(self.Ny):
                for cx in range(self.Nx):
                    c = (cz * self.Ny + cy) * self.Nx + cx
                    for s, (i, j, k) in enumerate(S):
                        self.conn[c, s] = self.node_id[cz * (self.nz - 1) + k, cy * (self.ny - 1) + j,
                                                       cx * (self.nx - 1) + i]

    @property
    def n_cells(self):
        return self.Nx * self.Ny * self.Nz

    def cell_dofs(self):
        """(n_cells, n) global DoF of each block DoF 3 s + component."""
        return (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(self.n_cells, -1)

    def outer_node_mask(self):
        """Nodes on the outer surface of the whole array (all six faces)."""
        I, J, K = self.lattice.T
        return ((I == 0) | (I == self.X - 1) | (J == 0) | (J == self.Y - 1)
                | (K == 0) | (K == self.Z - 1))

    def face_nodes(self, which):
        """Node ids on 'bottom' (K = 0) or 'top' (K = n_z - 1)."""
        K = self.lattice[:, 2]
        return np.nonzero(K == (0 if which == "bottom" else self.Z - 1))[0]

    def csr_pattern(self):
        """Union of the per-block dense n x n DoF blocks, columns sorted."""
        dofs = self.cell_dofs()
        n = dofs.shape[1]
        rows = np.repeat(dofs, n, axis=1).ravel()
        cols = np.tile(dofs, (1, n)).ravel()
        P = sp.coo_matrix((np.ones(rows.size, dtype=np.int8), (rows, cols)),
                          shape=(self.n_dofs, self.n_dofs)).tocsr()
        P.sort_indices()
        return P.indptr.astype(np.int64), P.indices.astype(np.int64)


def assemble_global(mesh, cell_type, roms, dT):
    """A_global = sum over blocks of A_element(type), b_global = dT sum of
    b_element(type) (Sec. 4.3, eq. 18-19; hybrid blocks Sec. 4.4)."""
    dofs = mesh.cell_dofs()
    n = dofs.shape[1]
    rows = np.repeat(dofs, n, axis=1).ravel()
    cols = np.tile(dofs, (1, n)).ravel()
    vals = np.concatenate([roms[int(t)].Kr.ravel() for t in cell_type])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(mesh.n_dofs, mesh.n_dofs)).tocsr()
    A.sum_duplicates()
    b = np.zeros(mesh.n_dofs)
    for c in range(mesh.n_cells):
        b[dofs[c]] += dT * roms[int(cell_type[c])].br
    return A, b


def constrained_dofs(mesh, clamp_bottom, clamp_top, prescribed_dofs=(), prescribed_values=()):
    """Constrained DoFs and their values: clamped faces get 0, then the
    explicit (DoF, value) list is applied (a later entry wins)."""
    g = {}
    for which, on in (("bottom", clamp_bottom), ("top", clamp_top)):
        if on:
            for node in mesh.face_nodes(which):
                for comp in range(3):
                    g[3 * int(node) + comp] = 0.0
    for d, v in zip(prescribed_dofs, prescribed_values):
        g[int(d)] = float(v)
    dofs = np.array(sorted(g), dtype=np.int64)
    vals = np.array([g[int(d)] for d in dofs], dtype=float)
    return dofs, vals


def lift(A, b, dofs, values):
    """Symmetric lifting: b_f -= A_f,c g; constrained rows and columns become
    identity with right-hand side g (same solution as eq. 13)."""
    n = A.shape[0]
    g = np.zeros(n)
    g[dofs] = values
    is_c = np.zeros(n)
    is_c[dofs] = 1.0
    b2 = b - A @ g
    b2[dofs] = values
    Mf = sp.diags(1.0 - is_c)
    A2 = (Mf @ A @ Mf + sp.diags(is_c)).tocsr()
    return A2, b2


def solve_direct(A, b):
    """Direct solve of an SPD system (eq. 20, eq. 13): LAPACK banded Cholesky
    in the natural order when the band is narrow, SuperLU otherwise."""
    return solve_spd(A, b)


def solve_spd(A, b):
    A = A.tocoo()
    n = A.shape[0]
    low = A.row >= A.col
    bw = int((A.row - A.col)[low].max()) if n else 0
    if (bw + 1) * n * 8 <= 2 ** 31 and n * bw * bw <= 2e11:
        ab = np.zeros((bw + 1, n))
        np.add.at(ab, ((A.row - A.col)[low], A.col[low]), A.data[low])
        return sla.cho_solve_banded((sla.cholesky_banded(ab, lower=True), True), b)
    return spla.splu(A.tocsc()).solve(b)


def pcg_jacobi(A, b, rtol=1e-14, max_iters=100000, x0=None):
    """Plain Jacobi-preconditioned conjugate gradients on the SPD system (the
    paper solves eq. 20 iteratively).  Stops when ||b - A x||_2 <= rtol ||b||_2
    computed from the recursively updated residual.  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    dinv = 1.0 / A.diagonal()
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for it in range(1, max_iters + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iters


def reconstruct(mesh, cell_type, roms, u, dT, chunk=256):
    """Per block: nodal displacement dT f_T + Phi u_block (eq. 15), then the
    centroid stress of every fine element (eq. 1).  Returns
    (sigma (n_cells, n_elem, 6), nodal displacement list per block if asked)."""
    dofs = mesh.cell_dofs()
    cell0 = roms[int(cell_type[0])].cell
    out = np.zeros((mesh.n_cells, cell0.n_elem, 6))
    for t in np.unique(cell_type):
        rom = roms[int(t)]
        cells = np.nonzero(cell_type == t)[0]
        edofs = rom.cell.element_dofs()
        for s in range(0, len(cells), chunk):
            cs = cells[s:s + chunk]
            U = u[dofs[cs]].T                                   # (n, k)
            nodal = dT * rom.fT[:, None] + rom.Phi @ U          # eq. 15
            sig = fem.centroid_stress(nodal, edofs, rom.mats,
                                      rom.cell.px / rom.cell.mx, rom.cell.py / rom.cell.my,
                                      rom.cell.h / rom.cell.mz, rom.cell.materials, dT, rom.cell.skew)
            out[cs] = np.transpose(sig, (2, 0, 1))
    return out


def nodal_displacement(mesh, cell_type, roms, u, dT, cell):
    """Fine-mesh displacement of one block, dT f_T + Phi u_block (eq. 15)."""
    rom = roms[int(cell_type[cell])]
    return dT * rom.fT + rom.Phi @ u[mesh.cell_dofs()[cell]]


def solve_mor(mesh, cell_type, roms, dT, bc_dofs, bc_values, direct=True, rtol=1e-14):
    """Global stage end to end: assemble, lift, solve eq. 20."""
    A, b = assemble_global(mesh, cell_type, roms, dT)
    A2, b2 = lift(A, b, bc_dofs, bc_values)
    if direct:
        return solve_direct(A2, b2)
    x, _ = pcg_jacobi(A2, b2, rtol=rtol)
    return x


# ----------------------------------------------------------------------------
# Full fine-mesh FEM of a whole array (the reference the MOR answer approximates)
# ----------------------------------------------------------------------------
class FullArray:
    """Fine hexahedral mesh of an N_x x N_y (x N_z stacked layers) array of
    blocks, every block meshed as in its own cell spec (all types share
    pitch, height and mesh)."""

    def __init__(self, specs, cell_type, nx_cells, ny_cells, nz_cells=1):
        self.specs = specs
        self.cell_type = np.asarray(cell_type)
        self.Nx, self.Ny, self.Nz = nx_cells, ny_cells, nz_cells
        self.cells = [fem.Cell(s) for s in specs]
        c0 = self.cells[0]
        self.mx, self.my, self.mz = c0.mx, c0.my, c0.mz
        self.px, self.py, self.h = c0.px, c0.py, c0.h
        self.skew = c0.skew
        self.GX, self.GY, self.GZ = self.Nx * self.mx, self.Ny * self.my, self.Nz * self.mz
        self.n_nodes = (self.GX + 1) * (self.GY + 1) * (self.GZ + 1)
        self.n_dofs = 3 * self.n_nodes

    def node_id(self, A, B, C):
        return (C * (self.GY + 1) + B) * (self.GX + 1) + A

    def node_coords(self):
        C, B, A = np.meshgrid(np.arange(self.GZ + 1), np.arange(self.GY + 1),
                              np.arange(self.GX + 1), indexing="ij")
        X = np.stack([(self.px * A / self.mx).ravel(), (self.py * B / self.my).ravel(),
                      (self.h * C / self.mz).ravel()], axis=1)
        X[:, 0] = X[:, 0] + self.skew * X[:, 1]
        return X

    def elements(self):
        """Per fine element: (8 node ids, block id, element id inside the block)."""
        EC, EB, EA = np.meshgrid(np.arange(self.GZ), np.arange(self.GY), np.arange(self.GX),
                                 indexing="ij")
        EA, EB, EC = EA.ravel(), EB.ravel(), EC.ravel()
        nodes = np.zeros((EA.size, 8), dtype=np.int64)
        for l in range(8):
            nodes[:, l] = self.node_id(EA + (l & 1), EB + ((l >> 1) & 1), EC + ((l >> 2) & 1))
        cell = ((EC // self.mz) * self.Ny + EB // self.my) * self.Nx + EA // self.mx
        local = ((EC % self.mz) * self.my + EB % self.my) * self.mx + EA % self.mx
        return nodes, cell, local

    def solve(self, dT, clamp_bottom, clamp_top, field=None):
        """Assemble, apply Dirichlet data (clamped faces; optionally a
        displacement field(x, y, z) -> (n, 3) on all six outer faces), solve.
        Returns (u, centroid stress per block (n_cells, n_elem_cell, 6))."""
        nodes, cell, local = self.elements()
        maps = [c.material_map() for c in self.cells]
        maps = np.stack(maps)                                   # (n_types, n_elem_cell)
        mats_of_elem = maps[self.cell_type[cell], local]
        type_of_elem = self.cell_type[cell]
        # A material key is (cell type, code); the element table holds each.
        key = type_of_elem.astype(np.int64) * 3 + mats_of_elem
        hx, hy, hz = self.px / self.mx, self.py / self.my, self.h / self.mz
        table = {}
        mat_list = {}
        for k in np.unique(key):
            t, code = divmod(int(k), 3)
            tri = self.cells[t].materials[code]
            table.update({int(k): fem.brick_element_table(hx, hy, hz, {0: tri}, [0], self.skew)[0]})
            mat_list[int(k)] = tri
        edofs = (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(len(nodes), 24)
        A, b = fem.assemble(self.n_dofs, edofs, key, table)
        b = dT * b
        X = self.node_coords()
        C = np.arange(self.n_nodes) // ((self.GX + 1) * (self.GY + 1))
        gval = np.full(self.n_dofs, np.nan)
        if field is not None:
            Ai = np.arange(self.n_nodes) % (self.GX + 1)
            Bi = (np.arange(self.n_nodes) // (self.GX + 1)) % (self.GY + 1)
            outer = np.nonzero((Ai == 0) | (Ai == self.GX) | (Bi == 0) | (Bi == self.GY)
                               | (C == 0) | (C == self.GZ))[0]
            vals = field(X[outer])
            for comp in range(3):
                gval[3 * outer + comp] = vals[:, comp]
        for on, level in ((clamp_bottom, 0), (clamp_top, self.GZ)):
            if on:
                nodes_c = np.nonzero(C == level)[0]
                for comp in range(3):
                    gval[3 * nodes_c + comp] = 0.0
        dofs = np.nonzero(~np.isnan(gval))[0]
        vals = gval[dofs]
        A2, b2 = lift(A, b, dofs, vals)
        u = solve_direct(A2, b2)
        # Centroid stress, per material key.
        sig = np.zeros((len(nodes), 6))
        B0 = fem.centroid_B(fem.element_corners(hx, hy, hz, self.skew))
        for k, (E, nu, alpha) in mat_list.items():
            sel = np.nonzero(key == k)[0]
            DB = fem.elasticity_matrix(E, nu) @ B0
            beta = fem.thermal_coefficient(E, nu, alpha)
            sig[sel] = u[edofs[sel]] @ DB.T - beta * dT * fem.M_VEC
        n_elem_cell = self.mx * self.my * self.mz
        out = np.zeros((self.Nx * self.Ny * self.Nz, n_elem_cell, 6))
        out[cell, local] = sig
        return u, out
