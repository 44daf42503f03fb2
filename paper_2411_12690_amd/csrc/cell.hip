// Unit-cell FE assembly on the device (Sec. 3.2 and 4.2; eq. 1-7, 11-12).
//
// The block is a structured grid of identical bricks (identical
// parallelepipeds for a skewed block), so each material has one 24x24
// element stiffness and one 24-entry unit-dT load, built by k_element_tables
// with 2x2x2 Gauss quadrature from the closed form of B_l^T D B_m for an
// isotropic material:
//   lambda g_l[i] g_m[j] + mu g_l[j] g_m[i] + mu (g_l . g_m) delta_ij.
// Assembly is row-centric (one thread per matrix row gathers over the <= 8
// elements around its node), so it is deterministic and needs no atomics;
// the three small element tables sit in LDS.
#include "mos_internal.h"

#include <algorithm>
#include <cmath>

namespace mos {
namespace {

struct BrickGeom {
    int mx, my, mz;
    double px, py, h;
    double skew;  // x += skew * y (a parallelepiped block)
};

__device__ __forceinline__ void decode_node(int node, int mx, int my, int &a, int &b, int &c) {
    a = node % (mx + 1);
    int t = node / (mx + 1);
    b = t % (my + 1);
    c = t / (my + 1);
}

// Material code of each element from its centroid distance to the via axis
// (and, for a micro-bump block, its centroid height: pads at both ends of the
// column).  The products and sums are rounded separately (no contraction) so
// the comparisons are the plain IEEE evaluation of dx*dx + dy*dy and of
// (ec + 1/2) h / m_z.
__global__ void k_material_map(uint8_t *mat, BrickGeom g, double d, double t, int bump, double pad) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int n_elem = g.mx * g.my * g.mz;
    if (e >= n_elem) return;
    int ea = e % g.mx;
    int eb = (e / g.mx) % g.my;
    int ec = e / (g.mx * g.my);
    double dy = __dadd_rn(__ddiv_rn(__dmul_rn(eb + 0.5, g.py), (double)g.my), -(g.py / 2.0));
    // Offset from the axis through the block's centre; both points are
    // sheared by skew * y, so the x offset gains skew * dy.
    double dx = __dadd_rn(__dadd_rn(__ddiv_rn(__dmul_rn(ea + 0.5, g.px), (double)g.mx), -(g.px / 2.0)),
                          __dmul_rn(g.skew, dy));
    double r2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
    double rv = d / 2.0;
    double rl = rv + t;
    uint8_t code = 0;
    if (bump) {
        double zc = __ddiv_rn(__dmul_rn(ec + 0.5, g.h), (double)g.mz);
        bool in_pad = zc < pad || zc > __dadd_rn(g.h, -pad);
        if (d > 0.0 && r2 < __dmul_rn(rv, rv)) code = in_pad ? 2 : 1;
    } else if (d > 0.0 && r2 < __dmul_rn(rv, rv)) {
        code = 1;
    } else if (d > 0.0 && r2 < __dmul_rn(rl, rl)) {
        code = 2;
    }
    mat[e] = code;
}

// Gradient of trilinear shape function l (corner offsets la, lb, lc) of an
// hx x hy x hz brick sheared by x += skew * y, at reference point
// (xi, eta, zeta).  The map is affine with a constant Jacobian, whose inverse
// transpose leaves d/dx and d/dz as for the brick and gives
// d/dy = (brick d/dy) - skew d/dx; the volume (det J) is the brick's.
__device__ __forceinline__ void shape_grad(int l, double xi, double eta, double zeta, double hx,
                                           double hy, double hz, double skew, double g[3]) {
    double sa = (l & 1) ? 1.0 : -1.0;
    double sb = (l & 2) ? 1.0 : -1.0;
    double sc = (l & 4) ? 1.0 : -1.0;
    g[0] = sa * (1.0 + sb * eta) * (1.0 + sc * zeta) * 0.125 * (2.0 / hx);
    g[1] = sb * (1.0 + sa * xi) * (1.0 + sc * zeta) * 0.125 * (2.0 / hy) - skew * g[0];
    g[2] = sc * (1.0 + sa * xi) * (1.0 + sb * eta) * 0.125 * (2.0 / hz);
}

// One block per material; 576 stiffness entries + 24 load entries.
__global__ void k_element_tables(double *ke, double *fe, const double *mprop, double hx, double hy,
                                 double hz, double skew) {
    int m = blockIdx.x;
    double lam = mprop[3 * m + 0], mu = mprop[3 * m + 1], beta = mprop[3 * m + 2];
    const double gp = 0.57735026918962576451;  // 1/sqrt(3)
    double detJ = hx * hy * hz * 0.125;
    for (int idx = threadIdx.x; idx < 576 + 24; idx += blockDim.x) {
        double acc = 0.0;
        if (idx < 576) {
            int r = idx / 24, cidx = idx % 24;
            int l = r / 3, i = r % 3, mm = cidx / 3, j = cidx % 3;
            for (int q = 0; q < 8; ++q) {
                double xi = (q & 1) ? gp : -gp, eta = (q & 2) ? gp : -gp, zeta = (q & 4) ? gp : -gp;
                double gl[3], gm[3];
                shape_grad(l, xi, eta, zeta, hx, hy, hz, skew, gl);
                shape_grad(mm, xi, eta, zeta, hx, hy, hz, skew, gm);
                double dot = gl[0] * gm[0] + gl[1] * gm[1] + gl[2] * gm[2];
                double v = lam * gl[i] * gm[j] + mu * gl[j] * gm[i] + (i == j ? mu * dot : 0.0);
                acc += v * detJ;
            }
            ke[m * 576 + idx] = acc;
        } else {
            int r = idx - 576;
            int l = r / 3, i = r % 3;
            for (int q = 0; q < 8; ++q) {
                double xi = (q & 1) ? gp : -gp, eta = (q & 2) ? gp : -gp, zeta = (q & 4) ? gp : -gp;
                double gl[3];
                shape_grad(l, xi, eta, zeta, hx, hy, hz, skew, gl);
                acc += beta * gl[i] * detJ;
            }
            fe[m * 24 + r] = acc;
        }
    }
}

// Value of K(row = 3 n + ci, col = 3 n2 + cj) as the sum over the elements
// shared by nodes n = (a,b,c) and n2 = (a2,b2,c2).
__device__ __forceinline__ double pair_value(const double *s_ke, const uint8_t *mat, int mx, int my,
                                             int mz, int a, int b, int c, int ci, int a2, int b2,
                                             int c2, int cj) {
    double v = 0.0;
    int ec0 = max(max(c, c2) - 1, 0), ec1 = min(min(c, c2), mz - 1);
    int eb0 = max(max(b, b2) - 1, 0), eb1 = min(min(b, b2), my - 1);
    int ea0 = max(max(a, a2) - 1, 0), ea1 = min(min(a, a2), mx - 1);
    for (int ec = ec0; ec <= ec1; ++ec)
        for (int eb = eb0; eb <= eb1; ++eb)
            for (int ea = ea0; ea <= ea1; ++ea) {
                int e = (ec * my + eb) * mx + ea;
                int l = (a - ea) + 2 * (b - eb) + 4 * (c - ec);
                int l2 = (a2 - ea) + 2 * (b2 - eb) + 4 * (c2 - ec);
                v += s_ke[mat[e] * 576 + (3 * l + ci) * 24 + 3 * l2 + cj];
            }
    return v;
}

__global__ void k_csr_values(double *val, const int32_t *row_ptr, const double *ke,
                             const uint8_t *mat, int mx, int my, int mz, int n_dofs) {
    __shared__ double s_ke[3 * 576];
    for (int i = threadIdx.x; i < 3 * 576; i += blockDim.x) s_ke[i] = ke[i];
    __syncthreads();
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n_dofs) return;
    int node = row / 3, ci = row % 3;
    int a, b, c;
    decode_node(node, mx, my, a, b, c);
    int k = row_ptr[row];
    for (int dc = -1; dc <= 1; ++dc) {
        int c2 = c + dc;
        if (c2 < 0 || c2 > mz) continue;
        for (int db = -1; db <= 1; ++db) {
            int b2 = b + db;
            if (b2 < 0 || b2 > my) continue;
            for (int da = -1; da <= 1; ++da) {
                int a2 = a + da;
                if (a2 < 0 || a2 > mx) continue;
                for (int cj = 0; cj < 3; ++cj)
                    val[k++] = pair_value(s_ke, mat, mx, my, mz, a, b, c, ci, a2, b2, c2, cj);
            }
        }
    }
}

__global__ void k_load_vector(double *bvec, const double *fe, const uint8_t *mat, int mx, int my,
                              int mz, int n_dofs) {
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n_dofs) return;
    int node = row / 3, ci = row % 3;
    int a, b, c;
    decode_node(node, mx, my, a, b, c);
    double v = 0.0;
    for (int ec = max(c - 1, 0); ec <= min(c, mz - 1); ++ec)
        for (int eb = max(b - 1, 0); eb <= min(b, my - 1); ++eb)
            for (int ea = max(a - 1, 0); ea <= min(a, mx - 1); ++ea) {
                int e = (ec * my + eb) * mx + ea;
                int l = (a - ea) + 2 * (b - eb) + 4 * (c - ec);
                v += fe[mat[e] * 24 + 3 * l + ci];
            }
    bvec[row] = v;
}

__global__ void k_fill(double *p, size_t n, double v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Lower band of K_ff into column-major NB x NB tiles: tile (J, d) holds rows
// of block J+d and columns of block J.  Padding rows beyond n_free get a unit
// diagonal so the padded matrix stays SPD.
__global__ void k_band_fill(double *tiles, const int32_t *row_ptr, const int32_t *col,
                            const double *val, const int32_t *free_dof, const int32_t *dof_free,
                            int n_free, int n_pad, int W) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    int I = i / NB;
    if (i >= n_free) {
        tiles[((size_t)I * (W + 1)) * NB * NB + (i % NB) + (size_t)(i % NB) * NB] = 1.0;
        return;
    }
    int row = free_dof[i];
    for (int k = row_ptr[row]; k < row_ptr[row + 1]; ++k) {
        int j = dof_free[col[k]];
        if (j < 0 || j > i) continue;
        int J = j / NB;
        int d = I - J;
        tiles[((size_t)J * (W + 1) + d) * NB * NB + (i % NB) + (size_t)(j % NB) * NB] = val[k];
    }
}

}  // namespace

mos_status fill(mos_ctx ctx, double *p, size_t n, double v) {
    if (n == 0) return MOS_OK;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, ctx->stream, p, n, v);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

mos_status launch_cell_assembly(mos_cell c) {
    mos_ctx ctx = c->ctx;
    const mos_cell_desc &d = c->desc;
    const int mx = c->mx, my = c->my, mz = c->mz;
    c->n_nodes = (mx + 1) * (my + 1) * (mz + 1);
    c->n_dofs = 3 * c->n_nodes;
    c->n_elem = mx * my * mz;

    // ---- host: CSR pattern of the 27-node stencil, interior/boundary split
    std::vector<int32_t> row_ptr(c->n_dofs + 1);
    row_ptr[0] = 0;
    auto nid = [&](int a, int b, int cc) { return (cc * (my + 1) + b) * (mx + 1) + a; };
    for (int cc = 0; cc <= mz; ++cc)
        for (int b = 0; b <= my; ++b)
            for (int a = 0; a <= mx; ++a) {
                int na = 1 + (a > 0) + (a < mx), nb = 1 + (b > 0) + (b < my), nc = 1 + (cc > 0) + (cc < mz);
                int len = 3 * na * nb * nc;
                int node = nid(a, b, cc);
                for (int ci = 0; ci < 3; ++ci) row_ptr[3 * node + ci + 1] = len;
            }
    for (int i = 0; i < c->n_dofs; ++i) row_ptr[i + 1] += row_ptr[i];
    c->nnz = row_ptr[c->n_dofs];
    std::vector<int32_t> colv((size_t)c->nnz);
    std::vector<int32_t> dof_free(c->n_dofs, -1), free_dof, bnode;
    for (int cc = 0; cc <= mz; ++cc)
        for (int b = 0; b <= my; ++b)
            for (int a = 0; a <= mx; ++a) {
                int node = nid(a, b, cc);
                bool bnd = a == 0 || a == mx || b == 0 || b == my || cc == 0 || cc == mz;
                if (bnd) bnode.push_back(node);
                for (int ci = 0; ci < 3; ++ci) {
                    int k = row_ptr[3 * node + ci];
                    for (int dc = -1; dc <= 1; ++dc)
                        for (int db = -1; db <= 1; ++db)
                            for (int da = -1; da <= 1; ++da) {
                                int a2 = a + da, b2 = b + db, c2 = cc + dc;
                                if (a2 < 0 || a2 > mx || b2 < 0 || b2 > my || c2 < 0 || c2 > mz) continue;
                                for (int cj = 0; cj < 3; ++cj) colv[k++] = 3 * nid(a2, b2, c2) + cj;
                            }
                    if (!bnd) {
                        dof_free[3 * node + ci] = (int32_t)free_dof.size();
                        free_dof.push_back(3 * node + ci);
                    }
                }
            }
    c->n_free = (int)free_dof.size();
    c->n_bnodes = (int)bnode.size();
    int bw = 0;
    for (int i = 0; i < c->n_free; ++i) {
        int row = free_dof[i];
        for (int k = row_ptr[row]; k < row_ptr[row + 1]; ++k) {
            int j = dof_free[colv[k]];
            if (j >= 0 && j <= i) bw = std::max(bw, i - j);
        }
    }
    c->bw = bw;
    c->NT = ceil_div(c->n_free, NB);
    c->W = (bw + NB - 1) / NB;
    if (c->W >= c->NT) c->W = c->NT - 1;

    // ---- device allocations
    DeviceArena &m = c->mem;
    MOS_TRY(m.alloc_n(c->n_elem, &c->mat));
    MOS_TRY(m.alloc_n(3 * 576, &c->ke));
    MOS_TRY(m.alloc_n(3 * 24, &c->fe));
    MOS_TRY(m.alloc_n(9, &c->mprop));
    MOS_TRY(m.alloc_n(c->n_dofs + 1, &c->row_ptr));
    MOS_TRY(m.alloc_n(c->nnz, &c->col));
    MOS_TRY(m.alloc_n(c->nnz, &c->val));
    MOS_TRY(m.alloc_n(c->n_dofs, &c->b));
    MOS_TRY(m.alloc_n(std::max(c->n_free, 1), &c->free_dof));
    MOS_TRY(m.alloc_n(c->n_bnodes, &c->bnode));
    int32_t *dof_free_d = nullptr;
    MOS_TRY(m.alloc_n(c->n_dofs, &dof_free_d));
    size_t n_tiles = (size_t)c->NT * (c->W + 1);
    MOS_TRY(m.alloc_n(n_tiles * NB * NB, &c->tiles));

    double mprop[9];
    const mos_material *mats[3] = {&d.matrix, &d.via, &d.liner};
    for (int k = 0; k < 3; ++k) {
        double E = mats[k]->E, nu = mats[k]->nu, al = mats[k]->alpha;
        double lam = E * nu / (1.0 + nu) / (1.0 - 2.0 * nu);
        double mu = E / 2.0 / (1.0 + nu);
        mprop[3 * k + 0] = lam;
        mprop[3 * k + 1] = mu;
        mprop[3 * k + 2] = al * (3.0 * lam + 2.0 * mu);
    }
    hipStream_t st = ctx->stream;
    MOS_HIP(hipMemcpyAsync(c->mprop, mprop, sizeof(mprop), hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(c->row_ptr, row_ptr.data(), row_ptr.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(c->col, colv.data(), colv.size() * 4, hipMemcpyHostToDevice, st));
    if (c->n_free)
        MOS_HIP(hipMemcpyAsync(c->free_dof, free_dof.data(), free_dof.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(c->bnode, bnode.data(), bnode.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(dof_free_d, dof_free.data(), dof_free.size() * 4, hipMemcpyHostToDevice, st));

    BrickGeom g{mx, my, mz, d.pitch_x, d.pitch_y, d.height, d.skew};
    hipLaunchKernelGGL(k_material_map, dim3(ceil_div(c->n_elem, 256)), dim3(256), 0, st, c->mat, g,
                       d.tsv_diameter, d.liner_thickness, d.structure == MOS_CELL_BUMP ? 1 : 0, d.pad_thickness);
    MOS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_element_tables, dim3(3), dim3(256), 0, st, c->ke, c->fe, c->mprop,
                       d.pitch_x / mx, d.pitch_y / my, d.height / mz, d.skew);
    MOS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_csr_values, dim3(ceil_div(c->n_dofs, 256)), dim3(256), 0, st, c->val,
                       c->row_ptr, c->ke, c->mat, mx, my, mz, c->n_dofs);
    MOS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_load_vector, dim3(ceil_div(c->n_dofs, 256)), dim3(256), 0, st, c->b, c->fe,
                       c->mat, mx, my, mz, c->n_dofs);
    MOS_LAUNCH_CHECK();
    MOS_TRY(fill(ctx, c->tiles, n_tiles * NB * NB, 0.0));
    int n_pad = c->NT * NB;
    hipLaunchKernelGGL(k_band_fill, dim3(ceil_div(n_pad, 256)), dim3(256), 0, st, c->tiles, c->row_ptr,
                       c->col, c->val, c->free_dof, dof_free_d, c->n_free, n_pad, c->W);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

}  // namespace mos
