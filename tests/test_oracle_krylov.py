"""Pins of the oracle's condition estimate (Ritz values of the preconditioned
reduced system on the CG Krylov space): spectra fixed in closed form, a
start vector that misses eigenvectors, interlacing in k, the generalised
eigenproblem of (A, M), and the textbook identity between CG's step
coefficients and the Lanczos tridiagonal.  CPU only."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import krylov


def random_spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T, ev


def test_full_space_gives_the_spectrum():
    rng = np.random.default_rng(1)
    ev = np.sort(rng.uniform(0.5, 40.0, 30))
    C = np.diag(ev)
    theta = krylov.ritz_values(C, rng.standard_normal(30), 30)
    assert np.allclose(theta, ev, rtol=1e-9)


def test_one_step_is_a_rayleigh_quotient():
    rng = np.random.default_rng(2)
    A, _ = random_spd(20, rng)
    v = rng.standard_normal(20)
    theta = krylov.ritz_values(A, v, 1)
    assert theta.shape == (1,) and theta[0] == pytest.approx(v @ A @ v / (v @ v), rel=1e-12)
    assert krylov.jacobi_cond(A, v, 1) == 1.0


def test_unexcited_eigenvectors_stay_invisible():
    """A start vector with no weight on some eigenvectors: the Krylov space
    stays in the span of the others, the basis stops at their count, and the
    Ritz extremes are theirs however many steps are asked for."""
    ev = np.arange(1.0, 13.0)
    C = np.diag(ev)
    v = np.zeros(12)
    support = [2, 3, 5, 8]                     # eigenvalues 3, 4, 6, 9
    v[support] = [1.0, -2.0, 0.5, 1.5]
    V = krylov.krylov_basis(C, v, 12)
    assert V.shape == (12, 4)
    theta = krylov.ritz_values(C, v, 12)
    assert np.allclose(theta, ev[support], rtol=1e-12)


def test_extremes_interlace_in_k():
    rng = np.random.default_rng(3)
    A, ev = random_spd(40, rng, cond=1e4)
    v = rng.standard_normal(40)
    lo, hi = np.inf, -np.inf
    for k in range(1, 41):
        th = krylov.ritz_values(A, v, k)
        assert th[0] <= lo * (1 + 1e-12) and th[-1] >= hi * (1 - 1e-12)
        assert th[0] >= ev[0] * (1 - 1e-9) and th[-1] <= ev[-1] * (1 + 1e-9)
        lo, hi = th[0], th[-1]
    assert lo == pytest.approx(ev[0], rel=1e-8) and hi == pytest.approx(ev[-1], rel=1e-8)


@pytest.mark.parametrize("n", [7, 32])
def test_jacobi_on_the_1d_laplacian(n):
    """tridiag(-1, 2, -1): eigenvalues 2 - 2 cos(j pi / (n + 1)); Jacobi
    divides by 2, so the full-space ratio is cot^2(pi / (2 (n + 1)))."""
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    b = np.random.default_rng(n).standard_normal(n)
    assert krylov.jacobi_cond(A, b, n) == pytest.approx(1.0 / np.tan(np.pi / (2 * (n + 1))) ** 2, rel=1e-9)


def test_exact_preconditioner_gives_one():
    rng = np.random.default_rng(4)
    A, _ = random_spd(25, rng)
    b = rng.standard_normal(25)
    for k in (2, 10, 25):
        assert krylov.preconditioned_cond(A, np.linalg.inv(A), b, k) == pytest.approx(1.0, abs=1e-9)


def test_full_space_matches_the_generalised_eigenproblem():
    """k = n: the ratio of the extreme eigenvalues of A x = lambda M x."""
    rng = np.random.default_rng(5)
    A, _ = random_spd(24, rng, cond=1e3)
    B = rng.standard_normal((24, 24))
    M = B @ B.T + 24 * np.eye(24)
    ev = sla.eigh(A, M, eigvals_only=True)
    b = rng.standard_normal(24)
    assert krylov.preconditioned_cond(A, np.linalg.inv(M), b, 24) == pytest.approx(ev[-1] / ev[0], rel=1e-8)


def cg_tridiagonal(A, b, minv, k, rtol=0.0):
    """Up to k steps of CG from 0 preconditioned by minv (a diagonal as a
    vector, or a dense M^-1), fewer once ||r|| <= rtol ||b||; the Lanczos
    tridiagonal from its step lengths alpha_j and direction updates beta_j
    (diagonal 1/alpha_j + beta_(j-1)/alpha_(j-1), off-diagonal
    sqrt(beta_j)/alpha_j)."""
    prec = (lambda v: minv * v) if minv.ndim == 1 else (lambda v: minv @ v)
    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = r @ z
    al, be = [], []
    for _ in range(k):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        z = prec(r)
        rz1 = r @ z
        al.append(a)
        be.append(rz1 / rz)
        rz = rz1
        p = z + be[-1] * p
        if np.linalg.norm(r) <= rtol * np.linalg.norm(b):
            break
    m = len(al)
    T = np.diag([1.0 / al[j] + (be[j - 1] / al[j - 1] if j else 0.0) for j in range(m)])
    off = [np.sqrt(be[j]) / al[j] for j in range(m - 1)]
    return T + np.diag(off, 1) + np.diag(off, -1)


def cg_problem():
    rng = np.random.default_rng(6)
    A, _ = random_spd(60, rng, cond=1e3)
    A += np.diag(rng.uniform(0.0, 50.0, 60))        # a diagonal that is not constant
    return A, rng.standard_normal(60), 1.0 / np.diag(A)


@pytest.mark.parametrize("k", [3, 8, 12])
def test_cg_coefficients_give_the_ritz_values(k):
    """The identity between CG and Lanczos (e.g. Saad, Iterative Methods for
    Sparse Linear Systems, sec. 6.7.3): the tridiagonal built from CG's
    coefficients has the Ritz values of the Krylov space as eigenvalues --
    exactly while CG's residuals stay orthogonal (the first steps)."""
    A, b, dinv = cg_problem()
    theta_cg = np.linalg.eigvalsh(cg_tridiagonal(A, b, dinv, k))
    s = np.sqrt(dinv)
    theta = krylov.ritz_values(s[:, None] * A * s[None, :], s * b, k)
    assert np.allclose(theta_cg, theta, rtol=1e-8)
    assert theta_cg[-1] / theta_cg[0] == pytest.approx(krylov.jacobi_cond(A, b, k), rel=1e-8)


def test_converged_cg_gives_the_extremes():
    """Later, rounding spoils orthogonality and CG's tridiagonal gains extra
    copies of converged Ritz values, but once the solve has converged its
    extreme eigenvalues are the operator's: the ratio equals the oracle's."""
    A, b, dinv = cg_problem()
    T = cg_tridiagonal(A, b, dinv, 1000, rtol=1e-12)
    theta_cg = np.linalg.eigvalsh(T)
    assert theta_cg[-1] / theta_cg[0] == pytest.approx(krylov.jacobi_cond(A, b, T.shape[0]), rel=1e-8)


@pytest.mark.parametrize("k", [3, 8])
def test_cg_with_a_dense_preconditioner(k):
    """Before convergence, with a preconditioner that is not diagonal: the
    start vector and the similarity transform both matter."""
    A, b, _ = cg_problem()
    B = np.random.default_rng(7).standard_normal((60, 60))
    minv = np.linalg.inv(B @ B.T / 60 + np.diag(np.diag(A)))
    theta_cg = np.linalg.eigvalsh(cg_tridiagonal(A, b, minv, k))
    assert theta_cg[-1] / theta_cg[0] == pytest.approx(krylov.preconditioned_cond(A, minv, b, k), rel=1e-8)


# ---- the two-level preconditioner (written from its definition) ----------

import workloads as W                                     # noqa: E402
from oracle import array as oarray                        # noqa: E402
from oracle import mor as omor                            # noqa: E402

SPEC = W.CellSpec(pitch_x=3.0, pitch_y=2.5, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 3), tsv_diameter=1.4)


@pytest.mark.parametrize("N,interp,cols,rows", [
    # odd count: the last aggregate has one block and the closing column (row)
    ((3, 3), (3, 3, 3), [0, 0, 0, 0, 1, 1, 1], [0, 0, 0, 0, 1, 1, 1]),
    # even count: the last aggregate takes the closing column
    ((4, 1), (4, 3, 3), [0] * 6 + [1] * 7, [0, 0, 0]),
    ((1, 2), (3, 4, 3), [0, 0, 0], [0] * 7),
])
def test_aggregate_ownership_by_hand(N, interp, cols, rows):
    mesh = oarray.AbstractMesh(N[0], N[1], interp)
    agg = krylov.aggregate_of_nodes(mesh)
    ax_n = (N[0] + 1) // 2
    assert np.array_equal(agg % ax_n, np.array(cols)[mesh.lattice[:, 0]])
    assert np.array_equal(agg // ax_n, np.array(rows)[mesh.lattice[:, 1]])


def test_rigid_modes_are_rigid():
    """The six fields over a whole unclamped array are rigid motions: the
    assembled reduced matrix (eq. 20) annihilates them.  A wrong sign or a
    coordinate scaled per axis gives strain, and a nonzero product."""
    roms = [omor.local_stage(SPEC)]
    mesh = oarray.AbstractMesh(2, 2, SPEC.interp, SPEC.pitch_x, SPEC.pitch_y, SPEC.height)
    A, _ = oarray.assemble_global(mesh, np.zeros(4, dtype=np.uint8), roms, 0.0)
    nodes = np.arange(mesh.n_nodes)
    Z = krylov.rigid_modes(mesh, nodes, np.array([1.0, -2.0, 0.5]), SPEC.pitch_x)
    AZ = A @ Z
    assert np.abs(AZ).max() <= 1e-9 * np.abs(A).max() * np.abs(Z).max()
    assert np.linalg.matrix_rank(Z) == 6


def clamped_system(nx, ny, t):
    roms = [omor.local_stage(s) for s in (SPEC, SPEC.dummy())]
    mesh = oarray.AbstractMesh(nx, ny, SPEC.interp, SPEC.pitch_x, SPEC.pitch_y, SPEC.height)
    A, b = oarray.assemble_global(mesh, t, roms, -250.0)
    dofs, _ = oarray.constrained_dofs(mesh, True, False)
    free = np.setdiff1d(np.arange(A.shape[0]), dofs)
    return mesh, A[free][:, free].toarray(), np.asarray(b)[free], free


def test_coarse_bases_partition_the_free_dofs():
    mesh, A, b, free = clamped_system(3, 3, np.zeros(9, dtype=np.uint8))
    Zs = krylov.coarse_bases(mesh, free, SPEC.pitch_x)
    assert len(Zs) == 4
    comp = free % 3
    for c in range(3):
        cover = sum(Z[:, c] for Z in Zs)
        assert np.array_equal(cover, (comp == c).astype(float))
    for Z in Zs:
        P = Z @ np.linalg.solve(Z.T @ A @ Z, Z.T @ A)     # A-orthogonal projection on span Z_a
        assert np.allclose(P @ P, P, atol=1e-9) and np.allclose(P @ Z, Z, atol=1e-9)


def test_two_level_is_spd_and_better_than_jacobi():
    mesh, A, b, free = clamped_system(4, 3, W.dummy_map(np.random.default_rng(2), 12, 0.3))
    minv = krylov.two_level_minv(mesh, A, free, SPEC.pitch_x)
    assert np.array_equal(minv, minv.T)
    assert np.linalg.eigvalsh(minv)[0] > 0
    n = len(free)
    k2 = krylov.preconditioned_cond(A, minv, b, n)
    kj = krylov.jacobi_cond(A, b, n)
    assert 1.0 < k2 < 0.5 * kj
    # Disjoint supports (Z_a^T Z_b = 0 for a != b) leave each aggregate's
    # own term: Z_a^T (M^-1 - D^-1) A Z_a = Z_a^T Z_a B_a^-1 B_a = Z_a^T Z_a.
    coarse = minv - np.diag(1.0 / np.diag(A))
    for Z in krylov.coarse_bases(mesh, free, SPEC.pitch_x):
        assert np.allclose(Z.T @ coarse @ A @ Z, Z.T @ Z, rtol=1e-8, atol=1e-8 * np.abs(Z.T @ Z).max())
