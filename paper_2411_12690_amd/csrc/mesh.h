// Host-side numbering of the abstract array mesh (Sec. 4.3): every unit block
// is an abstract element whose DoFs are its Lagrange surface nodes; blocks
// share the nodes of their common faces.  The numbering contract is stated in
// mos.h.
#pragma once

#include <cstdint>
#include <vector>

namespace mos {

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
    std::vector<int32_t> node_of;  // lattice (K*Y + J)*X + I -> node id, -1 if none
    std::vector<int> surf;         // 3*S
    std::vector<int32_t> conn;     // [Nx*Ny][S]
    void build(int Nx, int Ny, int nx, int ny, int nz);
};

}  // namespace mos
