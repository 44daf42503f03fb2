"""Oracle, part 5: the condition estimate of the preconditioned reduced system
of eq. 20 that a conjugate-gradient solve yields as a by-product.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves eq. 20 iteratively and gives neither the preconditioner nor
the conditioning; the library reports an estimate of the latter from its own
CG steps.  What that estimate is, by definition: k steps of preconditioned CG
from x0 = 0 on A u = b with an SPD preconditioner M build the Krylov space
K_k(M^-1 A, M^-1 b).  Writing M^-1 = L L^T, the operator is similar to the
symmetric C = L^T A L, and the space to K_k(C, L^T b).  The Ritz values are
the eigenvalues of C restricted to that space (the Rayleigh-Ritz
projection); the estimate is the largest over the smallest.  They lie in
[lambda_min(C), lambda_max(C)], so the estimate never exceeds the true
condition number, and it reaches it only when b has weight on both extreme
eigenvectors (a load with a symmetry the extreme modes lack never excites
them).

Here the space is spanned explicitly: an orthonormal basis built by
applying C and orthogonalising each new vector against all earlier ones
(Gram-Schmidt, done twice so the basis stays orthonormal to rounding), then
the dense projection V^T C V and its eigenvalues (a library routine).

The library's preconditioners are not in the paper either (it names none);
the two it offers are written out here from their definitions, as dense
matrices for arrays small enough to hold A densely:

* Jacobi: M = diag(A).
* Two-level (additive): M^-1 = D^-1 + sum_a Z_a B_a^-1 Z_a^T with D the
  diagonal of A.  The array's blocks are grouped into aggregates of 2 x 2
  (along a row or column with an odd count, the last aggregate has one
  block).  A node of the abstract mesh belongs to one aggregate: the one
  whose node columns [2 a_x (n_x - 1), 2 (a_x + 1) (n_x - 1)) and rows hold
  it, the last aggregate also taking the array's closing column (row).
  Z_a holds the six rigid-body motions of the aggregate's nodes (three
  translations, three infinitesimal rotations about the aggregate's lower
  corner, in coordinates divided by the x pitch) on its free DoFs and zero
  elsewhere; B_a = Z_a^T A Z_a.  An aggregate whose B_a has no Cholesky
  factor keeps only the Jacobi term.
"""
import numpy as np
import scipy.linalg as sla


def krylov_basis(C, v0, k):
    """Orthonormal basis (columns) of K_k(C, v0) = span{v0, C v0, ...,
    C^(k-1) v0}.  Stops early when the space becomes invariant (the new
    direction vanishes against the scale of C v)."""
    V = [v0 / np.linalg.norm(v0)]
    for _ in range(k - 1):
        w = C @ V[-1]
        scale = np.linalg.norm(w)
        for _ in range(2):
            for u in V:
                w = w - (u @ w) * u
        nw = np.linalg.norm(w)
        if nw <= 1e-12 * scale:
            break
        V.append(w / nw)
    return np.array(V).T


def ritz_values(C, v0, k):
    """Eigenvalues (ascending) of the symmetric C restricted to K_k(C, v0)."""
    V = krylov_basis(C, v0, k)
    return np.linalg.eigvalsh(V.T @ (C @ V))


def preconditioned_cond(A, Minv, b, k):
    """Largest over smallest Ritz value of M^-1 A after k CG steps from
    x0 = 0 on A u = b: the Ritz values of C = L^T A L on K_k(C, L^T b),
    L the lower Cholesky factor of M^-1 (dense arrays)."""
    L = sla.cholesky(Minv, lower=True)
    C = L.T @ A @ L
    theta = ritz_values(C, L.T @ b, k)
    return theta[-1] / theta[0]


def jacobi_cond(A, b, k):
    """preconditioned_cond with M the diagonal of A (Jacobi)."""
    return preconditioned_cond(A, np.diag(1.0 / np.diag(A)), b, k)


def aggregate_of_nodes(mesh):
    """Aggregate id (a_y * n_aggregates_x + a_x) of every abstract-mesh node."""
    I, J = mesh.lattice[:, 0], mesh.lattice[:, 1]
    ax_n, ay_n = (mesh.Nx + 1) // 2, (mesh.Ny + 1) // 2
    ax = np.minimum(I // (2 * (mesh.nx - 1)), ax_n - 1)
    ay = np.minimum(J // (2 * (mesh.ny - 1)), ay_n - 1)
    return ay * ax_n + ax


def rigid_modes(mesh, nodes, corner, scale):
    """(3 len(nodes), 6): translations x, y, z and rotations about x, y, z
    through `corner`, coordinates divided by `scale`, in DoF order 3 node +
    component."""
    x, y, z = ((mesh.coords[nodes] - corner) / scale).T
    Z = np.zeros((3 * len(nodes), 6))
    for c in range(3):
        Z[c::3, c] = 1.0
    Z[1::3, 3], Z[2::3, 3] = -z, y           # about x
    Z[0::3, 4], Z[2::3, 4] = z, -x           # about y
    Z[0::3, 5], Z[1::3, 5] = -y, x           # about z
    return Z


def coarse_bases(mesh, free, pitch_x):
    """Z_a of every aggregate (ascending id) as (len(free), 6) arrays over
    the free DoFs `free` (sorted global DoF ids)."""
    agg = aggregate_of_nodes(mesh)
    pos = np.full(mesh.n_dofs, -1)
    pos[free] = np.arange(len(free))
    out = []
    for a in np.unique(agg):
        nodes = np.nonzero(agg == a)[0]
        Zn = rigid_modes(mesh, nodes, mesh.coords[nodes].min(axis=0), pitch_x)
        dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
        keep = pos[dofs] >= 0
        Z = np.zeros((len(free), 6))
        Z[pos[dofs[keep]]] = Zn[keep]
        out.append(Z)
    return out


def two_level_minv(mesh, A_ff, free, pitch_x):
    """Dense M^-1 = D^-1 + sum_a Z_a B_a^-1 Z_a^T over the free DoFs `free`
    of the reduced system A_ff."""
    minv = np.diag(1.0 / np.diag(A_ff))
    for Z in coarse_bases(mesh, free, pitch_x):
        B = Z.T @ A_ff @ Z
        try:
            Lb = np.linalg.cholesky(B)
        except np.linalg.LinAlgError:
            continue
        W = sla.solve_triangular(Lb, Z.T, lower=True)     # B^-1 = Lb^-T Lb^-1
        minv += W.T @ W
    return minv
