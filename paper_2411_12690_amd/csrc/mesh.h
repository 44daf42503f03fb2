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
// nodes (I % (n_x-1) == 0, J % (n_y-1) == 0, or K % (n_z-1) == 0).  An array
// of N_z stacked layers of blocks has Z = N_z (n_z-1) + 1 planes; the N_z + 1
// planes between layers (bottom and top included) are full (X*Y nodes), every
// other plane holds N_y+1 full rows of X nodes and Y-N_y-1 rows of N_x+1
// nodes.  One layer (N_z = 1) has only its bottom and top planes full.
struct Lattice {
    int32_t Nx, Ny, nx, ny, nz, Nz;
    int64_t X, Y, Z, plane_full, plane_mid, n_nodes;
};

__host__ __device__ inline Lattice make_lattice(int Nx, int Ny, int nx, int ny, int nz, int Nz = 1) {
    Lattice L;
    L.Nx = Nx;
    L.Ny = Ny;
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.Nz = Nz;
    L.X = (int64_t)Nx * (nx - 1) + 1;
    L.Y = (int64_t)Ny * (ny - 1) + 1;
    L.Z = (int64_t)Nz * (nz - 1) + 1;
    L.plane_full = L.X * L.Y;
    L.plane_mid = (int64_t)(Ny + 1) * L.X + (L.Y - Ny - 1) * (int64_t)(Nx + 1);
    L.n_nodes = (int64_t)(Nz + 1) * L.plane_full + (int64_t)Nz * (nz - 2) * L.plane_mid;
    return L;
}

// Node id of a lattice point that is a node (undefined otherwise).
__host__ __device__ inline int64_t node_id(const Lattice &L, int64_t I, int64_t J, int64_t K) {
    const int64_t sz = L.nz - 1;
    const int64_t fp = (K + sz - 1) / sz;  // full planes below K
    const int64_t base = fp * L.plane_full + (K - fp) * L.plane_mid;
    if (K % sz == 0) return base + J * L.X + I;
    const int64_t full_before = (J + L.ny - 2) / (L.ny - 1);  // rows J' < J with J' % (n_y-1) == 0
    return base + full_before * L.X + (J - full_before) * (L.Nx + 1) + (J % (L.ny - 1) == 0 ? I : I / (L.nx - 1));
}

// A box of the node lattice, wx x wy points per plane over Z planes, whose
// origin lies on a cell corner: its point (i, j, K) is a node when i is a
// multiple of sx, j a multiple of sy, or K a multiple of sz (Z - 1 is a
// multiple of sz: the box spans whole layers of blocks).  Nodes are ranked in
// (K, j, i) order.  The whole lattice is the box X x Y x Z; the closed form
// of node_id is this rank for it.
struct SubLattice {
    int32_t wx, wy, Z, sx, sy, sz;
    int32_t fc, fr;  // columns (i % sx == 0) and rows (j % sy == 0) of nodes present in every plane
    int64_t pf, pm;  // nodes of a full plane (K % sz == 0), and of any other plane
};

__host__ __device__ inline SubLattice make_sub(int wx, int wy, int Z, int sx, int sy, int sz) {
    SubLattice s;
    s.wx = wx;
    s.wy = wy;
    s.Z = Z;
    s.sx = sx;
    s.sy = sy;
    s.sz = sz;
    s.fc = (wx + sx - 1) / sx;
    s.fr = (wy + sy - 1) / sy;
    s.pf = (int64_t)wx * wy;
    s.pm = (int64_t)s.fr * wx + (int64_t)(wy - s.fr) * s.fc;
    return s;
}

__host__ __device__ inline int64_t sub_count(const SubLattice &s) {
    const int64_t nf = (s.Z - 1) / s.sz + 1;  // full planes
    return nf * s.pf + (s.Z - nf) * s.pm;
}

__host__ __device__ inline int64_t sub_encode(const SubLattice &s, int i, int j, int K) {
    const int64_t fp = (K + s.sz - 1) / s.sz;  // full planes below K
    const int64_t base = fp * s.pf + (K - fp) * s.pm;
    if (K % s.sz == 0) return base + (int64_t)j * s.wx + i;
    const int fb = (j + s.sy - 1) / s.sy;  // full rows below row j
    return base + (int64_t)fb * s.wx + (int64_t)(j - fb) * s.fc + (j % s.sy == 0 ? i : i / s.sx);
}

__host__ __device__ inline void sub_decode(const SubLattice &s, int64_t id, int &i, int &j, int &K) {
    // Layers of sz planes repeat: one full plane, then sz - 1 other planes;
    // the top full plane closes the box.
    const int64_t layer = s.pf + (int64_t)(s.sz - 1) * s.pm;
    const int nl = (s.Z - 1) / s.sz;
    int L = (int)(id / layer);
    if (L > nl) L = nl;
    int64_t t = id - (int64_t)L * layer;
    if (L == nl || t < s.pf) {
        K = L * s.sz;
        j = (int)(t / s.wx);
        i = (int)(t % s.wx);
        return;
    }
    t -= s.pf;
    K = L * s.sz + 1 + (int)(t / s.pm);
    t %= s.pm;
    // Rows repeat with period sy: one full row, then sy - 1 rows of fc nodes.
    const int64_t period = s.wx + (int64_t)(s.sy - 1) * s.fc;
    const int q = (int)(t / period);
    const int64_t u = t % period;
    if (u < s.wx) {
        j = q * s.sy;
        i = (int)u;
    } else {
        j = q * s.sy + 1 + (int)((u - s.wx) / s.fc);
        i = (int)((u - s.wx) % s.fc) * s.sx;
    }
}

__host__ __device__ inline SubLattice whole_lattice(const Lattice &L) {
    return make_sub((int)L.X, (int)L.Y, (int)L.Z, L.nx - 1, L.ny - 1, L.nz - 1);
}

// Internal node order of an array inside the solver: the array is cut into
// boxes of cx x cy cells (the last box of a row or column takes what is
// left, and the closing nodes of the array), and each box's nodes form one
// consecutive range, boxes in (gy, gx) order and nodes within a box in
// (K, j, i) order.  A node belongs to the box that holds it: boxes start on
// cell boundaries and end before the next box's first column or row.  One
// workgroup owns a box's DoFs, so the coarse correction of the
// preconditioner over the aggregates inside a box needs no other workgroup.
struct AggLayout {
    int32_t nax, nay, cx, cy, sx, sy, sz, Z;
    int32_t wxi, wxl, wyi, wyl;  // box widths of inner and last aggregates
    int64_t row;                 // nodes of a row of aggregates of inner height
};

__host__ __device__ inline AggLayout make_agg_layout(const Lattice &L, int cx, int cy) {
    AggLayout a;
    a.cx = cx;
    a.cy = cy;
    a.sx = L.nx - 1;
    a.sy = L.ny - 1;
    a.sz = L.nz - 1;
    a.Z = (int)L.Z;
    a.nax = (L.Nx + cx - 1) / cx;
    a.nay = (L.Ny + cy - 1) / cy;
    a.wxi = cx * a.sx;
    a.wyi = cy * a.sy;
    a.wxl = (L.Nx - cx * (a.nax - 1)) * a.sx + 1;
    a.wyl = (L.Ny - cy * (a.nay - 1)) * a.sy + 1;
    a.row = (int64_t)(a.nax - 1) * sub_count(make_sub(a.wxi, a.wyi, a.Z, a.sx, a.sy, a.sz)) +
            sub_count(make_sub(a.wxl, a.wyi, a.Z, a.sx, a.sy, a.sz));
    return a;
}

__host__ __device__ inline int agg_count(const AggLayout &a) { return a.nax * a.nay; }

// Box of aggregate (gx, gy).
__host__ __device__ inline SubLattice agg_box(const AggLayout &a, int gx, int gy) {
    return make_sub(gx == a.nax - 1 ? a.wxl : a.wxi, gy == a.nay - 1 ? a.wyl : a.wyi, a.Z, a.sx, a.sy, a.sz);
}

// First internal node of aggregate (gx, gy).
__host__ __device__ inline int64_t agg_first(const AggLayout &a, int gx, int gy) {
    const int wy = gy == a.nay - 1 ? a.wyl : a.wyi;
    return (int64_t)gy * a.row + (int64_t)gx * sub_count(make_sub(a.wxi, wy, a.Z, a.sx, a.sy, a.sz));
}

__host__ __device__ inline int agg_x(const AggLayout &a, int64_t I) {
    const int g = (int)(I / a.wxi);
    return g < a.nax - 1 ? g : a.nax - 1;
}
__host__ __device__ inline int agg_y(const AggLayout &a, int64_t J) {
    const int g = (int)(J / a.wyi);
    return g < a.nay - 1 ? g : a.nay - 1;
}

// Internal node id of lattice node (I, J, K).
__host__ __device__ inline int64_t agg_encode(const AggLayout &a, int64_t I, int64_t J, int K) {
    const int gx = agg_x(a, I), gy = agg_y(a, J);
    return agg_first(a, gx, gy) +
           sub_encode(agg_box(a, gx, gy), (int)(I - (int64_t)gx * a.wxi), (int)(J - (int64_t)gy * a.wyi), K);
}

// Lattice point (I, J, K) of internal node id.
__host__ __device__ inline void agg_decode(const AggLayout &a, int64_t id, int64_t &I, int64_t &J, int &K) {
    int gy = (int)(id / a.row);
    if (gy > a.nay - 1) gy = a.nay - 1;
    const int64_t rem = id - (int64_t)gy * a.row;
    const int wy = gy == a.nay - 1 ? a.wyl : a.wyi;
    const int64_t per = sub_count(make_sub(a.wxi, wy, a.Z, a.sx, a.sy, a.sz));
    int gx = (int)(rem / per);
    if (gx > a.nax - 1) gx = a.nax - 1;
    int i, j;
    sub_decode(agg_box(a, gx, gy), rem - (int64_t)gx * per, i, j, K);
    I = (int64_t)gx * a.wxi + i;
    J = (int64_t)gy * a.wyi + j;
}

constexpr int MAX_TYPES = 8;
// Surface nodes per cell are bounded so a (slot, surface node) pair packs
// into one int32 as slot << INC_SHIFT | s.
constexpr int INC_SHIFT = 9;
constexpr int MAX_SURF = (1 << INC_SHIFT) - 1;
// The same packing bounds the cell slots of one engine: slot << INC_SHIFT
// must stay below 2^31.
constexpr int64_t MAX_SLOTS = int64_t(1) << (31 - INC_SHIFT);

// Whether an engine of `slots` cell slots fits the incidence packing.
__host__ __device__ inline bool slots_fit(int64_t slots) { return slots >= 0 && slots <= MAX_SLOTS; }

// Surface Lagrange nodes (i, j, k) of one block in (k, j, i) order, i fastest.
void surface_nodes(int nx, int ny, int nz, std::vector<int> &ijk);

struct ArrayMesh {
    int Nx = 0, Ny = 0, Nz = 1, nx = 0, ny = 0, nz = 0, S = 0;
    int64_t X = 0, Y = 0, Z = 0, n_nodes = 0;
    Lattice lat{};
    std::vector<int> surf;         // 3*S
    std::vector<int32_t> conn;     // [Nx*Ny*Nz][S], block (cx, cy, cz) at (cz Ny + cy) Nx + cx
    void build(int Nx, int Ny, int nx, int ny, int nz, int Nz = 1);
};

}  // namespace mos
