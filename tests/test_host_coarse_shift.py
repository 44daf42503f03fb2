"""The identity behind the tabulated coarse matrices (two-level PCG
preconditioner): rigid-body modes about an aggregate corner are the
cell-local modes times a 6x6 shift T, so a cell's part of B_a = Z^T K_r Z
is T^T G T with G taken once in cell-local coordinates, for every cell
class (right / top face in the next aggregate), piece and offset.  Checked
on the oracle's reduced stiffness of a small cell.  CPU only."""
import numpy as np
import pytest

import workloads as W
from oracle import mor


@pytest.fixture(scope="module")
def cell():
    s = W.CellSpec(pitch_x=3.0, pitch_y=3.0, height=6.0, mesh=(4, 4, 6), interp=(3, 3, 4), tsv_diameter=1.6)
    return s, mor.local_stage(s), mor.surface_nodes(*s.interp)


def modes(spec, S, X0, Y0, cls, piece, bottom=True, top=False):
    """Rigid modes (translations; rotations z, x, y about the origin) on the
    cell's free DoFs of one piece, in coordinates scaled by the x pitch with
    the cell corner at (X0, Y0)."""
    nx, ny, nz = spec.interp
    h0, h1, h2 = 1.0 / (nx - 1), spec.pitch_y / spec.pitch_x / (ny - 1), spec.height / spec.pitch_x / (nz - 1)
    Z = np.zeros((3 * len(S), 6))
    for sn, (i, j, k) in enumerate(S):
        if (bottom and k == 0) or (top and k == nz - 1):
            continue
        p = (1 if (cls & 1) and i == nx - 1 else 0) + (2 if (cls & 2) and j == ny - 1 else 0)
        if p != piece:
            continue
        X, Y, Zc = X0 + i * h0, Y0 + j * h1, k * h2
        for ci in range(3):
            z = np.zeros(6)
            z[ci] = 1.0
            if ci == 0:
                z[3], z[5] = -Y, Zc
            elif ci == 1:
                z[3], z[4] = X, -Zc
            else:
                z[4], z[5] = Y, -X
            Z[3 * sn + ci] = z
    return Z


@pytest.mark.parametrize("top", [False, True])
def test_shifted_cell_terms_equal_the_direct_product(cell, top):
    spec, rom, S = cell
    K = rom.Kr
    for cls in range(4):
        for piece in range(4):
            Zc = modes(spec, S, 0.0, 0.0, cls, piece, top=top)
            G = Zc.T @ K @ Zc
            for X0, Y0 in ((-1.0, 0.0), (1.0, -1.0), (2.0, 1.0), (0.0, 0.0)):
                Za = modes(spec, S, X0, Y0, cls, piece, top=top)
                T = np.eye(6)
                T[0, 3], T[1, 3], T[2, 4], T[2, 5] = -Y0, X0, Y0, -X0
                np.testing.assert_allclose(Za, Zc @ T, rtol=0, atol=1e-14)
                direct = Za.T @ K @ Za
                scale = max(np.abs(direct).max(), 1e-300)
                assert np.abs(T.T @ G @ T - direct).max() <= 1e-12 * scale


def test_a_whole_free_cell_adds_nothing(cell):
    # Without constraints a cell held entirely by one aggregate contributes
    # Z^T K_r Z = 0: K_r annihilates the rigid modes (the reason the coarse
    # matrices are assembled from the constrained and split cells).
    spec, rom, S = cell
    Z = modes(spec, S, 0.0, 0.0, 0, 0, bottom=False)
    G = Z.T @ rom.Kr @ Z
    assert np.abs(G).max() <= 1e-9 * np.abs(rom.Kr).max()
