"""CPU checks of the engine's host code that turns recorded PCG steps into the
condition estimate of the preconditioned reduced system (eq. 20): the
harness ``tests/host/mesh_check.cpp`` feeds it (alpha_j, beta_j) pairs in the
engine's record layout (beta_j = (r_j, z_j) / (r_(j-1), z_(j-1)), the update
that forms the j-th direction; beta_0 = 0) and prints what it returns, with
no GPU.  Checked against the oracle's Ritz ratio on the Krylov space (while
plain CG's residuals stay orthogonal), against LAPACK's eigenvalues of CG's
tridiagonal over the full 128-step record, and on degenerate records (fewer
than two steps, a non-positive or non-finite step, a negative update), also
under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import subprocess

import numpy as np
import pytest

from oracle import krylov

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")


def harness(sanitized=False):
    exe = os.path.join(HOST, "mesh_check_asan" if sanitized else "mesh_check")
    if not os.path.exists(exe):
        from paper_2411_12690_amd import build as b
        b.build_host_checks()
    return exe


def estimate(pairs, sanitized=False):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1") if sanitized else None
    text = f"{len(pairs)}\n" + "".join(f"{float(a)!r} {float(b)!r}\n" for a, b in pairs)
    p = subprocess.run([harness(sanitized), "lanczos"], input=text, capture_output=True, text=True, env=env,
                       timeout=60)
    assert p.returncode == 0, p.stdout + p.stderr
    kappa, steps = p.stdout.split()
    return float(kappa), int(steps)


def cg_record(A, b, dinv, k):
    """k steps of Jacobi-preconditioned CG from 0, as the engine records them."""
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    pairs, beta = [], 0.0
    for _ in range(k):
        q = A @ p
        a = rz / (p @ q)
        pairs.append((a, beta))
        x += a * p
        r -= a * q
        z = dinv * r
        rz1 = r @ z
        beta = rz1 / rz
        rz = rz1
        p = z + beta * p
    return pairs


def spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * np.geomspace(1.0, cond, n)) @ Q.T + np.diag(rng.uniform(0.0, 20.0, n))
    return A, rng.standard_normal(n)


@pytest.mark.parametrize("k", [2, 5, 9])
def test_matches_the_oracle_ritz_ratio(k):
    A, b = spd(80, 3)
    kappa, steps = estimate(cg_record(A, b, 1.0 / np.diag(A), k))
    assert steps == k
    assert kappa == pytest.approx(krylov.jacobi_cond(A, b, k), rel=1e-10)


def test_full_record_matches_lapack_on_the_tridiagonal():
    A, b = spd(300, 4, cond=1e4)
    pairs = cg_record(A, b, 1.0 / np.diag(A), 128)
    al = np.array([a for a, _ in pairs])
    be = np.array([bb for _, bb in pairs])
    diag = 1.0 / al + np.concatenate([[0.0], be[1:] / al[:-1]])
    off = np.sqrt(be[1:]) / al[:-1]
    ev = np.linalg.eigvalsh(np.diag(diag) + np.diag(off, 1) + np.diag(off, -1))
    kappa, steps = estimate(pairs)
    assert steps == 128
    assert kappa == pytest.approx(ev[-1] / ev[0], rel=1e-12)


@pytest.mark.parametrize("pairs", [
    [],
    [(0.5, 0.0)],
    [(0.5, 0.0), (0.0, 0.3)],
    [(0.5, 0.0), (-0.2, 0.3)],
    [(0.5, 0.0), (0.4, -0.1)],
    [(0.5, 0.0), (float("nan"), 0.3)],
    [(0.5, 0.0), (0.4, float("inf"))],
], ids=["empty", "one-step", "zero-step", "negative-step", "negative-update", "nan", "inf"])
def test_degenerate_records_give_no_estimate(pairs):
    assert estimate(pairs) == (0.0, 0)


def test_sanitized_build_agrees():
    A, b = spd(60, 5)
    pairs = cg_record(A, b, 1.0 / np.diag(A), 40)
    assert estimate(pairs, sanitized=True) == estimate(pairs)
    assert estimate([(0.5, 0.0)], sanitized=True) == (0.0, 0)
