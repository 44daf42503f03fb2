// Host-side numbering of the abstract array mesh (Sec. 4.3): every unit block
// is an abstract element whose DoFs are its Lagrange surface nodes; blocks
// share the nodes of their common faces.  The numbering contract is stated in
// mos.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace mos {

// Closed form of the abstract-mesh numbering: the node id of lattice point
// (I, J, K) is its rank in (K, J, I) order among the lattice points that are
// nodes (I % (n_x-1) == 0, J % (n_y-1) == 0, or K on the bottom or top
// plane).  The bottom and top planes are full (X*Y nodes); an interior plane
// holds N_y+1 full rows of X nodes and Y-N_y-1 rows of N_x+1 nodes.
struct Lattice {
    int32_t Nx, Ny, nx, ny, nz;
    int64_t X, Y, Z, plane_full, plane_mid, n_nodes;
};

__host__ __device__ inline Lattice make_lattice(int Nx, int Ny, int nx, int ny, int nz) {
    Lattice L;
    L.Nx = Nx;
    L.Ny = Ny;
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.X = (int64_t)Nx * (nx - 1) + 1;
    L.Y = (int64_t)Ny * (ny - 1) + 1;
    L.Z = nz;
    L.plane_full = L.X * L.Y;
    L.plane_mid = (int64_t)(Ny + 1) * L.X + (L.Y - Ny - 1) * (int64_t)(Nx + 1);
    L.n_nodes = 2 * L.plane_full + (L.Z - 2) * L.plane_mid;
    return L;
}

// Node id of a lattice point that is a node (undefined otherwise).
__host__ __device__ inline int64_t node_id(const Lattice &L, int64_t I, int64_t J, int64_t K) {
    if (K == 0) return J * L.X + I;
    if (K == L.Z - 1) return L.plane_full + (L.Z - 2) * L.plane_mid + J * L.X + I;
    const int64_t full_before = (J + L.ny - 2) / (L.ny - 1);  // rows J' < J with J' % (n_y-1) == 0
    const int64_t base = L.plane_full + (K - 1) * L.plane_mid + full_before * L.X + (J - full_before) * (L.Nx + 1);
    return base + (J % (L.ny - 1) == 0 ? I : I / (L.nx - 1));
}

constexpr int MAX_TYPES = 8;
// Surface nodes per cell are bounded so a (slot, surface node) pair packs
// into one int32 as slot << INC_SHIFT | s.
constexpr int INC_SHIFT = 9;
constexpr int MAX_SURF = (1 << INC_SHIFT) - 1;

// Surface Lagrange nodes (i, j, k) of one block in (k, j, i) order, i fastest.
void surface_nodes(int nx, int ny, int nz, std::vector<int> &ijk);

struct ArrayMesh {
    int Nx = 0, Ny = 0, nx = 0, ny = 0, nz = 0, S = 0;
    int64_t X = 0, Y = 0, Z = 0, n_nodes = 0;
    Lattice lat{};
    std::vector<int> surf;         // 3*S
    std::vector<int32_t> conn;     // [Nx*Ny][S]
    void build(int Nx, int Ny, int nx, int ny, int nz);
};

}  // namespace mos
