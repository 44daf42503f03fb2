// Local stage after assembly (Sec. 4.2-4.3, eq. 8-19):
//   1. Lagrange weights L of every boundary FE node (eq. 8-10) written as the
//      boundary rows of Phi;
//   2. right-hand sides [-K_f,bc L | b_f] of the n+1 lifted local problems
//      (eq. 13-15) and their solution with the banded Cholesky factor;
//   3. Galerkin projection P = [Phi f_T]^T [K Phi  b] with FP64 MFMA, from
//      which K_r = sym(Phi^T K Phi) (eq. 18), b_r = Phi^T b (eq. 19) and the
//      check f_T^T K Phi ~ 0;
//   4. the centroid stress basis Psi = D B0 Phi and the unit-dT thermal
//      stress sigma_T = D B0 f_T - beta 1 (eq. 1 at element centroids), laid
//      out as the A operand of the reconstruction GEMM.
#include "bf16.h"
#include "mos_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace mos {

mos_status fill(mos_ctx ctx, double *p, size_t n, double v);

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ void k_lagrange(double *phi, int ldp, const int32_t *bnode, int n_bnodes, const int32_t *surf,
                           int n_surf, int mx, int my, int mz, double px, double py, double h, int nx,
                           int ny, int nz) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_bnodes * n_surf) return;
    int r = idx / n_surf, s = idx % n_surf;
    int node = bnode[r];
    int a = node % (mx + 1), b = (node / (mx + 1)) % (my + 1), c = node / ((mx + 1) * (my + 1));
    double X[3] = {px * a / mx, py * b / my, h * c / mz};
    double len[3] = {px, py, h};
    int cnt[3] = {nx, ny, nz};
    int si = surf[3 * s + 0], sj = surf[3 * s + 1], sk = surf[3 * s + 2];
    int sel[3] = {si, sj, sk};
    double w = 1.0;
    for (int ax = 0; ax < 3; ++ax) {
        int n1 = cnt[ax] - 1;
        double xi = len[ax] * sel[ax] / n1;
        double num = 1.0, den = 1.0;
        for (int j = 0; j <= n1; ++j) {
            if (j == sel[ax]) continue;
            double xj = len[ax] * j / n1;
            num *= X[ax] - xj;
            den *= xi - xj;
        }
        w *= num / den;
    }
    for (int ci = 0; ci < 3; ++ci) phi[(size_t)(3 * node + ci) * ldp + 3 * s + ci] = w;
}

// One wave per row: lanes stride over the columns.
__global__ void k_rhs(const double *phi, int ldp, const int32_t *row_ptr, const int32_t *col,
                      const double *val, const double *b, const int32_t *free_dof, int n_free, int n_pad,
                      double *R, int ldr, int n) {
    int f = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x % 64;
    if (f >= n_pad) return;
    for (int q = lane; q < ldr; q += 64) {
        double v = 0.0;
        if (f < n_free) {
            int row = free_dof[f];
            if (q < n) {
                for (int k = row_ptr[row]; k < row_ptr[row + 1]; ++k) v -= val[k] * phi[(size_t)col[k] * ldp + q];
            } else if (q == n) {
                v = b[row];
            }
        }
        R[(size_t)f * ldr + q] = v;
    }
}

__global__ void k_scatter_solution(double *phi, int ldp, const double *R, int ldr, const int32_t *free_dof,
                                   int n_free, int n) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_free * (n + 1)) return;
    int f = idx / (n + 1), q = idx % (n + 1);
    phi[(size_t)free_dof[f] * ldp + q] = R[(size_t)f * ldr + q];
}

__global__ void k_spmm(const double *phi, int ldp, const int32_t *row_ptr, const int32_t *col,
                       const double *val, const double *b, double *Y, int n_dofs, int n) {
    int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x % 64;
    if (row >= n_dofs) return;
    for (int q = lane; q < ldp; q += 64) {
        double v = 0.0;
        if (q < n) {
            for (int k = row_ptr[row]; k < row_ptr[row + 1]; ++k) v += val[k] * phi[(size_t)col[k] * ldp + q];
        } else if (q == n) {
            v = b[row];
        }
        Y[(size_t)row * ldp + q] = v;
    }
}

// Split-K partial of P = A^T B for tall A, B (rows x ldp), one wave per 64x64
// output tile and row chunk, FP64 MFMA 16x16x4.  Lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; output register q of lane l is D[l/16 + 4q][l%16].
__global__ __launch_bounds__(64) void k_proj_partial(const double *A, const double *B, double *part,
                                                     int rows, int ldp, int NP, int chunk) {
    const int n_t = (NP + 63) / 64;
    const int ti = blockIdx.x / n_t, tj = blockIdx.x % n_t;
    const int ch = blockIdx.y;
    const int lane = threadIdx.x;
    const int i0 = ti * 64, j0 = tj * 64;
    const int rs = ch * chunk, re = min(rs + chunk, rows);
    d4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
    for (int r0 = rs; r0 < re; r0 += 4) {
        const int r = r0 + lane / 16;
        const bool rv = r < re;
        double a[4], bv[4];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) {
            int ci = i0 + 16 * bi + lane % 16;
            a[bi] = (rv && ci < ldp) ? A[(size_t)r * ldp + ci] : 0.0;
            int cj = j0 + 16 * bi + lane % 16;
            bv[bi] = (rv && cj < ldp) ? B[(size_t)r * ldp + cj] : 0.0;
        }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], bv[bj], acc[bi][bj], 0, 0, 0);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int i = i0 + 16 * bi + lane / 16 + 4 * q;   // FP64 MFMA output row
                int j = j0 + 16 * bj + lane % 16;
                if (i < NP && j < NP) part[((size_t)ch * NP + i) * NP + j] = acc[bi][bj][q];
            }
}

__global__ void k_proj_reduce(const double *part, double *P, int n_chunks, int NP, int n1) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * n1) return;
    int i = idx / n1, j = idx % n1;
    double s = 0.0;
    for (int ch = 0; ch < n_chunks; ++ch) s += part[((size_t)ch * NP + i) * NP + j];
    P[idx] = s;
}

__global__ void k_rom_finalize(const double *P, int n, int ldk, double *kr, double *kr_pad, float *kr32,
                               double *br) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ldk * ldk) return;
    int i = idx / ldk, j = idx % ldk;
    const int n1 = n + 1;
    double v = 0.0;
    if (i < n && j < n) {
        v = 0.5 * (P[i * n1 + j] + P[j * n1 + i]);
        kr[i * n + j] = v;
    }
    kr_pad[idx] = v;
    kr32[idx] = (float)v;
    if (j == 0 && i < n) br[i] = P[i * n1 + n];
}

// Centroid stress of column q of Phi (q < ldk; columns >= n are zero) or of
// f_T (q == ldk) for every element; D B0 applied in closed form.
__global__ void k_stress_basis(const double *phi, int ldp, const uint8_t *mat, const double *mprop, double *psi,
                               double *sig_t, int mx, int my, int mz, double hx, double hy, double hz,
                               double skew, int n, int ldk, int n_eblk) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_elem = mx * my * mz;
    if (idx >= n_eblk * 16 * (ldk + 1)) return;
    int q = idx % (ldk + 1), e = idx / (ldk + 1);
    int eb = e / 16, e16 = e % 16;
    double s[6] = {0, 0, 0, 0, 0, 0};
    int colq = q < ldk ? q : n;
    if (e < n_elem && (q == ldk || q < n)) {
        int ea = e % mx, ebb = (e / mx) % my, ec = e / (mx * my);
        double eps[6] = {0, 0, 0, 0, 0, 0};
        for (int l = 0; l < 8; ++l) {
            int a = ea + (l & 1), b = ebb + ((l >> 1) & 1), c = ec + ((l >> 2) & 1);
            int node = (c * (my + 1) + b) * (mx + 1) + a;
            double gx = ((l & 1) ? 1.0 : -1.0) / (4.0 * hx);
            // Sheared block (x += skew * y): d/dy loses skew d/dx.
            double gy = ((l & 2) ? 1.0 : -1.0) / (4.0 * hy) - skew * gx;
            double gz = ((l & 4) ? 1.0 : -1.0) / (4.0 * hz);
            double ux = phi[(size_t)(3 * node + 0) * ldp + colq];
            double uy = phi[(size_t)(3 * node + 1) * ldp + colq];
            double uz = phi[(size_t)(3 * node + 2) * ldp + colq];
            eps[0] += gx * ux;
            eps[1] += gy * uy;
            eps[2] += gz * uz;
            eps[3] += gy * ux + gx * uy;
            eps[4] += gz * uy + gy * uz;
            eps[5] += gz * ux + gx * uz;
        }
        int m = mat[e];
        double lam = mprop[3 * m + 0], mu = mprop[3 * m + 1], beta = mprop[3 * m + 2];
        double tr = eps[0] + eps[1] + eps[2];
        for (int k = 0; k < 3; ++k) s[k] = lam * tr + 2.0 * mu * eps[k];
        for (int k = 3; k < 6; ++k) s[k] = mu * eps[k];
        if (q == ldk)
            for (int k = 0; k < 3; ++k) s[k] -= beta;
    }
    if (q < ldk) {
        for (int k = 0; k < 6; ++k) psi[(((size_t)eb * 6 + k) * ldk + q) * 16 + e16] = s[k];
    } else if (e < n_elem) {
        for (int k = 0; k < 6; ++k) sig_t[(size_t)e * 6 + k] = s[k];
    }
}

// BF16 hi/lo split of Psi in the A-operand order of the 16x16x32 MFMA:
// [n_eblk][6][nks][64 lanes][8], lane l of k-step ks holding element
// 16 eb + l % 16 and columns 32 ks + 8 (l / 16) + 0..7 (zero past ldk).
__global__ void k_psi_split(const double *psi, int ldk, int nks, int64_t total, uint16_t *hi, uint16_t *lo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int v = (int)(idx % 8), lane = (int)((idx / 8) % 64), ks = (int)((idx / 512) % nks);
    const int64_t ebc = idx / (512 * (int64_t)nks);  // eb * 6 + component
    const int k = ks * 32 + 8 * (lane / 16) + v;
    const double x = k < ldk ? psi[((size_t)ebc * ldk + k) * 16 + lane % 16] : 0.0;
    uint16_t h, l;
    bf16_split(x, h, l);
    hi[idx] = h;
    lo[idx] = l;
}

// Stress of column q of Phi (q < ldk; columns >= n are zero) or of f_T
// (q == ldk) at the sample points of the mid-height plane (the paper's
// evaluation grid, Sec. 5.1): point p = j g + i at x = p_x (i + 1/2) / g,
// y = p_y (j + 1/2) / g, z = h / 2.  The point lies in the element whose
// half-open box holds it: along x that is a = floor(m_x (2i + 1) / (2g)) in
// integers (a point on an element face goes to the +x element) with
// reference coordinate xi = (m_x (2i + 1) - 2g a) / g - 1; along z the plane
// is the bottom face of layer m_z / 2 (zeta = -1) for even m_z and the
// middle of layer (m_z - 1) / 2 (zeta = 0) for odd m_z.  D B(xi, eta, zeta)
// of the trilinear element in closed form (eq. 1).  Same layout as the
// centroid basis with points in place of elements.
__global__ void k_plane_basis(const double *phi, int ldp, const uint8_t *mat, const double *mprop, double *psi,
                              double *sig_t, int mx, int my, int mz, double hx, double hy, double hz, int g, int n,
                              int ldk, int n_pblk) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_pblk * 16 * (ldk + 1)) return;
    const int q = (int)(idx % (ldk + 1)), p = (int)(idx / (ldk + 1));
    const int pb = p / 16, p16 = p % 16;
    double s[6] = {0, 0, 0, 0, 0, 0};
    const int colq = q < ldk ? q : n;
    if (p < g * g && (q == ldk || q < n)) {
        const int i = p % g, j = p / g;
        const int tx = mx * (2 * i + 1), ty = my * (2 * j + 1);
        const int ea = tx / (2 * g), eb = ty / (2 * g), ec = mz / 2;
        const double xi = (double)(tx - 2 * g * ea) / g - 1.0;
        const double eta = (double)(ty - 2 * g * eb) / g - 1.0;
        const double zeta = (mz % 2) ? 0.0 : -1.0;
        double eps[6] = {0, 0, 0, 0, 0, 0};
        for (int l = 0; l < 8; ++l) {
            const double sa = (l & 1) ? 1.0 : -1.0, sb = (l & 2) ? 1.0 : -1.0, sc = (l & 4) ? 1.0 : -1.0;
            const int node = ((ec + ((l >> 2) & 1)) * (my + 1) + eb + ((l >> 1) & 1)) * (mx + 1) + ea + (l & 1);
            // dN_l/dx = (2 / h_x) dN_l/dxi, N_l = (1 + sa xi)(1 + sb eta)(1 + sc zeta) / 8.
            const double gx = sa * (1.0 + sb * eta) * (1.0 + sc * zeta) / (4.0 * hx);
            const double gy = sb * (1.0 + sa * xi) * (1.0 + sc * zeta) / (4.0 * hy);
            const double gz = sc * (1.0 + sa * xi) * (1.0 + sb * eta) / (4.0 * hz);
            const double ux = phi[(size_t)(3 * node + 0) * ldp + colq];
            const double uy = phi[(size_t)(3 * node + 1) * ldp + colq];
            const double uz = phi[(size_t)(3 * node + 2) * ldp + colq];
            eps[0] += gx * ux;
            eps[1] += gy * uy;
            eps[2] += gz * uz;
            eps[3] += gy * ux + gx * uy;
            eps[4] += gz * uy + gy * uz;
            eps[5] += gz * ux + gx * uz;
        }
        const int m = mat[(ec * my + eb) * mx + ea];
        const double lam = mprop[3 * m + 0], mu = mprop[3 * m + 1], beta = mprop[3 * m + 2];
        const double tr = eps[0] + eps[1] + eps[2];
        for (int k = 0; k < 3; ++k) s[k] = lam * tr + 2.0 * mu * eps[k];
        for (int k = 3; k < 6; ++k) s[k] = mu * eps[k];
        if (q == ldk)
            for (int k = 0; k < 3; ++k) s[k] -= beta;
    }
    if (q < ldk) {
        for (int k = 0; k < 6; ++k) psi[(((size_t)pb * 6 + k) * ldk + q) * 16 + p16] = s[k];
    } else if (p < g * g) {
        for (int k = 0; k < 6; ++k) sig_t[(size_t)p * 6 + k] = s[k];
    }
}

}  // namespace

mos_status band_cholesky(mos_cell c, double *dinv, int *status_dev, int *not_spd);
mos_status band_solve(mos_cell c, const double *dinv, double *rhs, int ldr, int ncols);

mos_status reduce_cell(mos_cell c, mos_rom r) {
    mos_ctx ctx = c->ctx;
    hipStream_t st = ctx->stream;
    const mos_cell_desc &d = c->desc;
    const int nx = d.interp[0], ny = d.interp[1], nz = d.interp[2];
    std::vector<int32_t> surf;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1 || k == 0 || k == nz - 1) {
                    surf.push_back(i);
                    surf.push_back(j);
                    surf.push_back(k);
                }
    r->desc = d;
    r->mx = c->mx;
    r->my = c->my;
    r->mz = c->mz;
    r->n_dofs = c->n_dofs;
    r->n_elem = c->n_elem;
    r->n_surf = (int)surf.size() / 3;
    r->n = 3 * r->n_surf;
    const int n = r->n;
    r->ldp = (int)round_up(n + 1, 16);
    r->ldk = (int)round_up(n, 16);
    r->n_eblk = ceil_div(c->n_elem, 16);
    const int ldp = r->ldp, ldk = r->ldk;

    // Scratch owned by this call.
    DeviceArena tmp;
    tmp.ctx = ctx;
    struct Guard {
        DeviceArena &a;
        ~Guard() { a.release(); }
    } guard{tmp};
    int32_t *surf_d = nullptr;
    double *dinv = nullptr, *R = nullptr, *Y = nullptr, *part = nullptr, *P = nullptr;
    int *status_d = nullptr;
    const int n_pad = c->NT * NB;
    const int ldr = ldp;
    MOS_TRY(tmp.alloc_n(surf.size(), &surf_d));
    MOS_TRY(tmp.alloc_n((size_t)c->NT * NB * NB, &dinv));
    MOS_TRY(tmp.alloc_n((size_t)n_pad * ldr, &R));
    MOS_TRY(tmp.alloc_n(1, &status_d));

    DeviceArena &m = r->mem;
    MOS_TRY(m.alloc_n((size_t)c->n_dofs * ldp, &r->phi));
    MOS_TRY(m.alloc_n((size_t)n * n, &r->kr));
    MOS_TRY(m.alloc_n(n, &r->br));
    MOS_TRY(m.alloc_n((size_t)ldk * ldk, &r->kr_pad));
    MOS_TRY(m.alloc_n((size_t)ldk * ldk, &r->kr32_pad));
    MOS_TRY(m.alloc_n((size_t)r->n_eblk * 6 * ldk * 16, &r->psi));
    MOS_TRY(m.alloc_n((size_t)c->n_elem * 6, &r->sig_t));
    MOS_TRY(m.alloc_n(c->n_elem, &r->mat));
    MOS_TRY(m.alloc_n(9, &r->mprop));
    MOS_HIP(hipMemcpyAsync(r->mat, c->mat, c->n_elem, hipMemcpyDeviceToDevice, st));
    MOS_HIP(hipMemcpyAsync(r->mprop, c->mprop, 9 * sizeof(double), hipMemcpyDeviceToDevice, st));

    MOS_HIP(hipMemcpyAsync(surf_d, surf.data(), surf.size() * 4, hipMemcpyHostToDevice, st));
    MOS_TRY(fill(ctx, r->phi, (size_t)c->n_dofs * ldp, 0.0));
    hipLaunchKernelGGL(k_lagrange, dim3(ceil_div((int64_t)c->n_bnodes * r->n_surf, 256)), dim3(256), 0, st,
                       r->phi, ldp, c->bnode, c->n_bnodes, surf_d, r->n_surf, c->mx, c->my, c->mz, d.pitch_x,
                       d.pitch_y, d.height, nx, ny, nz);
    MOS_LAUNCH_CHECK();

    // Factor K_ff once.
    int not_spd = 0;
    MOS_TRY(band_cholesky(c, dinv, status_d, &not_spd));
    if (not_spd) {
        set_error("mos_reduce: interior stiffness K_ff is not positive definite (pivot %d)", not_spd - 1);
        return MOS_ESINGULAR;
    }
    // n + 1 right-hand sides and solves.
    hipLaunchKernelGGL(k_rhs, dim3(ceil_div(n_pad, 4)), dim3(256), 0, st, r->phi, ldp, c->row_ptr, c->col,
                       c->val, c->b, c->free_dof, c->n_free, n_pad, R, ldr, n);
    MOS_LAUNCH_CHECK();
    MOS_TRY(band_solve(c, dinv, R, ldr, n + 1));
    hipLaunchKernelGGL(k_scatter_solution, dim3(ceil_div((int64_t)c->n_free * (n + 1), 256)), dim3(256), 0, st,
                       r->phi, ldp, R, ldr, c->free_dof, c->n_free, n);
    MOS_LAUNCH_CHECK();

    // Projection.
    MOS_TRY(tmp.alloc_n((size_t)c->n_dofs * ldp, &Y));
    hipLaunchKernelGGL(k_spmm, dim3(ceil_div(c->n_dofs, 4)), dim3(256), 0, st, r->phi, ldp, c->row_ptr, c->col,
                       c->val, c->b, Y, c->n_dofs, n);
    MOS_LAUNCH_CHECK();
    const int NP = ldp;
    const int chunk = 512;
    const int n_chunks = ceil_div(c->n_dofs, chunk);
    const int n_t = ceil_div(NP, 64);
    MOS_TRY(tmp.alloc_n((size_t)n_chunks * NP * NP, &part));
    MOS_TRY(tmp.alloc_n((size_t)(n + 1) * (n + 1), &P));
    hipLaunchKernelGGL(k_proj_partial, dim3(n_t * n_t, n_chunks), dim3(64), 0, st, r->phi, Y, part, c->n_dofs,
                       ldp, NP, chunk);
    MOS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_proj_reduce, dim3(ceil_div((n + 1) * (n + 1), 256)), dim3(256), 0, st, part, P,
                       n_chunks, NP, n + 1);
    MOS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rom_finalize, dim3(ceil_div(ldk * ldk, 256)), dim3(256), 0, st, P, n, ldk, r->kr,
                       r->kr_pad, r->kr32_pad, r->br);
    MOS_LAUNCH_CHECK();

    // Stress basis.
    hipLaunchKernelGGL(k_stress_basis, dim3(ceil_div((int64_t)r->n_eblk * 16 * (ldk + 1), 256)), dim3(256), 0,
                       st, r->phi, ldp, c->mat, c->mprop, r->psi, r->sig_t, c->mx, c->my, c->mz,
                       d.pitch_x / c->mx, d.pitch_y / c->my, d.height / c->mz, d.skew, n, ldk, r->n_eblk);
    MOS_LAUNCH_CHECK();
    r->nks = ceil_div(ldk, 32);
    if (r->nks <= RECON_BF16_MAX_KS) {
        const int64_t total = (int64_t)r->n_eblk * 6 * r->nks * 512;
        MOS_TRY(m.alloc_n(total, &r->psi_hi));
        MOS_TRY(m.alloc_n(total, &r->psi_lo));
        hipLaunchKernelGGL(k_psi_split, dim3(ceil_div(total, 256)), dim3(256), 0, st, (const double *)r->psi, ldk,
                           r->nks, total, r->psi_hi, r->psi_lo);
        MOS_LAUNCH_CHECK();
    }

    // Health check of the projection: f_T^T K Phi should vanish (Phi^T K f_T = 0).
    std::vector<double> Ph((size_t)(n + 1) * (n + 1));
    MOS_HIP(hipMemcpyAsync(Ph.data(), P, Ph.size() * 8, hipMemcpyDeviceToHost, st));
    MOS_HIP(hipStreamSynchronize(st));
    double kmax = 0.0, omax = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) kmax = std::max(kmax, std::fabs(Ph[(size_t)i * (n + 1) + j]));
    for (int j = 0; j < n; ++j) omax = std::max(omax, std::fabs(Ph[(size_t)n * (n + 1) + j]));
    r->orth = kmax > 0 ? omax / kmax : 0.0;
    return MOS_OK;
}

mos_status plane_basis(mos_rom r, int grid) {
    if (grid < 1 || grid > PLANE_MAX_GRID) {
        set_error("plane grid %d outside [1, %d]", grid, PLANE_MAX_GRID);
        return MOS_EINVAL;
    }
    if (r->plane && r->plane_grid == grid) return MOS_OK;
    hipStream_t st = r->ctx->stream;
    if (r->plane) {
        // A different grid: the old basis may still be read by queued work.
        MOS_HIP(hipStreamSynchronize(st));
        r->plane->mem.release();
        delete r->plane;
        r->plane = nullptr;
        r->plane_grid = 0;
    }
    mos_rom_s *pl = new mos_rom_s();
    pl->ctx = r->ctx;
    pl->mem.ctx = r->ctx;
    pl->desc = r->desc;
    pl->mx = r->mx;
    pl->my = r->my;
    pl->mz = r->mz;
    pl->n = r->n;
    pl->n_surf = r->n_surf;
    pl->ldp = r->ldp;
    pl->ldk = r->ldk;
    pl->n_elem = grid * grid;
    pl->n_eblk = ceil_div(pl->n_elem, 16);
    pl->nks = r->nks;
    const int ldk = r->ldk;
    auto fail = [&](mos_status s) {
        pl->mem.release();
        delete pl;
        return s;
    };
    mos_status s = pl->mem.alloc_n((size_t)pl->n_eblk * 6 * ldk * 16, &pl->psi);
    if (s == MOS_OK) s = pl->mem.alloc_n((size_t)pl->n_elem * 6, &pl->sig_t);
    if (s != MOS_OK) return fail(s);
    const mos_cell_desc &d = r->desc;
    hipLaunchKernelGGL(k_plane_basis, dim3(ceil_div((int64_t)pl->n_eblk * 16 * (ldk + 1), 256)), dim3(256), 0, st,
                       r->phi, r->ldp, r->mat, r->mprop, pl->psi, pl->sig_t, r->mx, r->my, r->mz, d.pitch_x / r->mx,
                       d.pitch_y / r->my, d.height / r->mz, grid, r->n, ldk, pl->n_eblk);
    if (hipGetLastError() != hipSuccess) {
        set_error("k_plane_basis launch failed");
        return fail(MOS_EHIP);
    }
    if (pl->nks <= RECON_BF16_MAX_KS) {
        const int64_t total = (int64_t)pl->n_eblk * 6 * pl->nks * 512;
        s = pl->mem.alloc_n(total, &pl->psi_hi);
        if (s == MOS_OK) s = pl->mem.alloc_n(total, &pl->psi_lo);
        if (s != MOS_OK) return fail(s);
        hipLaunchKernelGGL(k_psi_split, dim3(ceil_div(total, 256)), dim3(256), 0, st, (const double *)pl->psi, ldk,
                           pl->nks, total, pl->psi_hi, pl->psi_lo);
        if (hipGetLastError() != hipSuccess) {
            set_error("k_psi_split launch failed");
            return fail(MOS_EHIP);
        }
    }
    r->plane = pl;
    r->plane_grid = grid;
    return MOS_OK;
}

}  // namespace mos
