// One Cholesky factorisation of the interior block K_ff of the unit cell and
// the n+1 triangular solves that follow it (Sec. 4.2: factor once, reuse for
// every local problem of eq. 14-15).
//
// K_ff in the natural interior ordering is banded (half bandwidth ~ one
// interior z-layer).  It is stored as a band of 64x64 column-major FP64 tiles,
// tile (J, d) holding rows of block J+d and columns of block J, d = 0..W.
// The factorisation is the right-looking tile algorithm: for each block
// column J, factor the diagonal tile (and form its inverse), solve the W
// tiles below it, then update the W(W+1)/2 trailing tiles.  The triangular
// solves use the stored diagonal inverses so every step is a small GEMM.
#include "mos_internal.h"

namespace mos {
namespace {

constexpr int LDS_LD = NB + 1;  // padded LDS row: conflict-free column walks

__device__ __forceinline__ double *tile_ptr(double *tiles, int J, int d, int W) {
    return tiles + ((size_t)J * (W + 1) + d) * NB * NB;
}

// acc[i][j] += sum_k A[ty+16i][k] * B[tx+16j][k] over k < NB (both in LDS,
// row-major with LDS_LD).
__device__ __forceinline__ void nt_tile_product(const double (*A)[LDS_LD], const double (*B)[LDS_LD],
                                                int tx, int ty, double acc[4][4]) {
    for (int k = 0; k < NB; ++k) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = A[ty + 16 * i][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = B[tx + 16 * j][k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
}

// Column-major global tile -> LDS [row][col].
__device__ __forceinline__ void load_tile(double (*S)[LDS_LD], const double *T) {
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) S[idx % NB][idx / NB] = T[idx];
}
// Column-major global tile -> LDS transposed: S[col][row].
__device__ __forceinline__ void load_tile_t(double (*S)[LDS_LD], const double *T) {
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) S[idx / NB][idx % NB] = T[idx];
}

// Diagonal tile: L_JJ (Cholesky) and X = L_JJ^{-1}.  The tile lives in
// registers during the factorisation: thread (i, w) of the 256 holds row i
// at columns w, w + 4, ..., w + 60.  Step k: the owner of (k, k) takes the
// square root, the owners of column k scale it and publish it in LDS, and
// every thread updates its own elements a_ij -= l_ik l_jk (j > k, i >= j).
__global__ __launch_bounds__(256) void k_potrf(double *tiles, double *dinv, int J, int W, int *status) {
    __shared__ double L[NB][LDS_LD];
    __shared__ double X[NB][LDS_LD];
    __shared__ double col[NB];
    __shared__ double diag;
    __shared__ double part_sum[4][NB];
    double *T = tile_ptr(tiles, J, 0, W);
    const int tid = threadIdx.x, i = tid % NB, w = tid / NB;
    double a[NB / 4];
#pragma unroll
    for (int m = 0; m < NB / 4; ++m) a[m] = T[(size_t)(w + 4 * m) * NB + i];
    for (int k = 0; k < NB; ++k) {
        const int wk = k % 4, mk = k / 4;
        if (w == wk && i == k) {
            double dkk = 0.0;
#pragma unroll
            for (int m = 0; m < NB / 4; ++m) dkk = m == mk ? a[m] : dkk;
            if (!(dkk > 0.0)) {
                atomicCAS(status, 0, 1 + J * NB + k);
                dkk = 1.0;
            }
            diag = sqrt(dkk);
        }
        __syncthreads();
        if (w == wk) {
            const double d = diag;
#pragma unroll
            for (int m = 0; m < NB / 4; ++m)
                if (m == mk) {
                    const double v = i == k ? d : (i > k ? a[m] / d : 0.0);
                    if (i >= k) a[m] = v;
                    col[i] = v;
                }
        }
        __syncthreads();
        const double ci = col[i];
#pragma unroll
        for (int m = 0; m < NB / 4; ++m) {
            const int j = w + 4 * m;
            if (j > k && i >= j) a[m] -= ci * col[j];
        }
    }
#pragma unroll
    for (int m = 0; m < NB / 4; ++m) L[i][w + 4 * m] = a[m];
    // X = L^{-1} by forward substitution on the identity, one row at a time
    // for all 64 columns at once: X[i][t] = (delta_it - sum_{k<i} L[i][k]
    // X[k][t]) / L[i][i].  Each dot product is split over four threads per
    // column (k = part, part + 4, ...) and the four partials summed in order.
    {
        const int t = i, part = w;
        for (int idx = tid; idx < NB * NB; idx += blockDim.x) X[idx / NB][idx % NB] = 0.0;
        __syncthreads();
        for (int r = 0; r < NB; ++r) {
            double sum = 0.0;
            for (int k = part; k < r; k += 4) sum += L[r][k] * X[k][t];
            part_sum[part][t] = sum;
            __syncthreads();
            if (part == 0) {
                const double sm = ((part_sum[0][t] + part_sum[1][t]) + part_sum[2][t]) + part_sum[3][t];
                X[r][t] = ((r == t ? 1.0 : 0.0) - sm) / L[r][r];
            }
            __syncthreads();
        }
    }
    double *D = dinv + (size_t)J * NB * NB;
    for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
        int r = idx % NB, c = idx / NB;
        T[idx] = r >= c ? L[r][c] : 0.0;
        D[idx] = r >= c ? X[r][c] : 0.0;
    }
}

// Tiles below the diagonal: T(J, d) := T(J, d) * L_JJ^{-T}.
__global__ __launch_bounds__(256) void k_trsm(double *tiles, const double *dinv, int J, int W, int NT) {
    __shared__ double A[NB][LDS_LD];
    __shared__ double B[NB][LDS_LD];
    int d = blockIdx.x + 1;
    if (J + d >= NT) return;
    double *T = tile_ptr(tiles, J, d, W);
    load_tile(A, T);
    load_tile(B, dinv + (size_t)J * NB * NB);
    __syncthreads();
    int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    nt_tile_product(A, B, tx, ty, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) T[(ty + 16 * i) + (tx + 16 * j) * NB] = acc[i][j];
}

// Trailing update: T(J+d2, d1-d2) -= T(J, d1) T(J, d2)^T for 1 <= d2 <= d1 <= W.
__global__ __launch_bounds__(256) void k_syrk(double *tiles, int J, int W, int NT) {
    __shared__ double A[NB][LDS_LD];
    __shared__ double B[NB][LDS_LD];
    int b = blockIdx.x, d1 = 1, d2 = 1;
    for (d1 = 1; d1 <= W; ++d1) {
        if (b < d1) {
            d2 = b + 1;
            break;
        }
        b -= d1;
    }
    if (J + d1 >= NT) return;
    load_tile(A, tile_ptr(tiles, J, d1, W));
    load_tile(B, tile_ptr(tiles, J, d2, W));
    __syncthreads();
    int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    nt_tile_product(A, B, tx, ty, acc);
    double *C = tile_ptr(tiles, J + d2, d1 - d2, W);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) C[(ty + 16 * i) + (tx + 16 * j) * NB] -= acc[i][j];
}

// Forward substitution step J, Y_J = L_JJ^{-1} (R_J - sum_d L(J, J-d) Y_{J-d}),
// in two launches.  k_fwd_part: one workgroup per (64 x 16 column slab of
// the row-major RHS, off-diagonal tile d = 1..W) forms L(J, J-d) Y_{J-d}
// into P[d-1]; k_fwd_fin: one workgroup per slab subtracts the P[d-1] from
// R_J in the order d = 1, 2, ... and applies the stored inverse of L_JJ.
// Spreading the W tile products over workgroups keeps the step from
// walking its tiles one after another.
__global__ __launch_bounds__(256) void k_fwd_part(const double *tiles, const double *R, double *P, int J, int W,
                                                  int ldr) {
    const int d = (int)blockIdx.y + 1;
    if (J - d < 0) return;
    __shared__ double L[NB][LDS_LD];
    __shared__ double Y[NB][17];
    const int col = threadIdx.x % 16, r0 = threadIdx.x / 16;
    const int c0 = blockIdx.x * 16;
    load_tile(L, tiles + ((size_t)(J - d) * (W + 1) + d) * NB * NB);
    for (int idx = threadIdx.x; idx < NB * 16; idx += blockDim.x)
        Y[idx / 16][idx % 16] = R[(size_t)((J - d) * NB + idx / 16) * ldr + c0 + idx % 16];
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < NB; ++k) {
        const double y = Y[k][col];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += L[r0 + 16 * i][k] * y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) P[((size_t)(d - 1) * NB + r0 + 16 * i) * ldr + c0 + col] = acc[i];
}

__global__ __launch_bounds__(256) void k_fwd_fin(const double *dinv, const double *P, double *R, int J, int W,
                                                 int ldr) {
    __shared__ double L[NB][LDS_LD];
    __shared__ double Y[NB][17];
    const int col = threadIdx.x % 16, r0 = threadIdx.x / 16;
    const int c0 = blockIdx.x * 16;
    load_tile(L, dinv + (size_t)J * NB * NB);
    double acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = R[(size_t)(J * NB + r0 + 16 * i) * ldr + c0 + col];
    for (int d = 1; d <= W && J - d >= 0; ++d)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] -= P[((size_t)(d - 1) * NB + r0 + 16 * i) * ldr + c0 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) Y[r0 + 16 * i][col] = acc[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + 16 * i;
        double s = 0.0;
        for (int k = 0; k <= r; ++k) s += L[r][k] * Y[k][col];
        R[(size_t)(J * NB + r) * ldr + c0 + col] = s;
    }
}

// Backward substitution step J, X_J = L_JJ^{-T} (Y_J - sum_d L(J+d, J)^T
// X_{J+d}), in the same two launches.
__global__ __launch_bounds__(256) void k_bwd_part(const double *tiles, const double *R, double *P, int J, int W,
                                                  int NT, int ldr) {
    const int d = (int)blockIdx.y + 1;
    if (J + d >= NT) return;
    __shared__ double L[NB][LDS_LD];
    __shared__ double Y[NB][17];
    const int col = threadIdx.x % 16, r0 = threadIdx.x / 16;
    const int c0 = blockIdx.x * 16;
    load_tile_t(L, tiles + ((size_t)J * (W + 1) + d) * NB * NB);
    for (int idx = threadIdx.x; idx < NB * 16; idx += blockDim.x)
        Y[idx / 16][idx % 16] = R[(size_t)((J + d) * NB + idx / 16) * ldr + c0 + idx % 16];
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < NB; ++k) {
        const double y = Y[k][col];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += L[r0 + 16 * i][k] * y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) P[((size_t)(d - 1) * NB + r0 + 16 * i) * ldr + c0 + col] = acc[i];
}

__global__ __launch_bounds__(256) void k_bwd_fin(const double *dinv, const double *P, double *R, int J, int W,
                                                 int NT, int ldr) {
    __shared__ double L[NB][LDS_LD];
    __shared__ double Y[NB][17];
    const int col = threadIdx.x % 16, r0 = threadIdx.x / 16;
    const int c0 = blockIdx.x * 16;
    load_tile_t(L, dinv + (size_t)J * NB * NB);
    double acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = R[(size_t)(J * NB + r0 + 16 * i) * ldr + c0 + col];
    for (int d = 1; d <= W && J + d < NT; ++d)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] -= P[((size_t)(d - 1) * NB + r0 + 16 * i) * ldr + c0 + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) Y[r0 + 16 * i][col] = acc[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + 16 * i;
        double s = 0.0;
        for (int k = r; k < NB; ++k) s += L[r][k] * Y[k][col];
        R[(size_t)(J * NB + r) * ldr + c0 + col] = s;
    }
}

}  // namespace

mos_status band_cholesky(mos_cell c, double *dinv, int *status_dev, int *not_spd) {
    hipStream_t st = c->ctx->stream;
    MOS_HIP(hipMemsetAsync(status_dev, 0, sizeof(int), st));
    const int W = c->W, NT = c->NT;
    for (int J = 0; J < NT; ++J) {
        hipLaunchKernelGGL(k_potrf, dim3(1), dim3(256), 0, st, c->tiles, dinv, J, W, status_dev);
        if (W > 0 && J + 1 < NT) {
            hipLaunchKernelGGL(k_trsm, dim3(W), dim3(256), 0, st, c->tiles, dinv, J, W, NT);
            hipLaunchKernelGGL(k_syrk, dim3(W * (W + 1) / 2), dim3(256), 0, st, c->tiles, J, W, NT);
        }
    }
    MOS_LAUNCH_CHECK();
    int *h = static_cast<int *>(c->ctx->pinned);
    MOS_HIP(hipMemcpyAsync(h, status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    MOS_HIP(hipStreamSynchronize(st));
    *not_spd = *h;
    return MOS_OK;
}

mos_status band_solve(mos_cell c, const double *dinv, double *rhs, int ldr, int ncols) {
    hipStream_t st = c->ctx->stream;
    const int W = c->W, NT = c->NT;
    const int blocks = ceil_div(ncols, 16);
    if (blocks * 16 > ldr) {
        set_error("band_solve: %d right-hand sides exceed the row stride %d", ncols, ldr);
        return MOS_EINVAL;
    }
    // Partial products of one step: [W][NB][ldr], reused by every step.
    DeviceArena tmp;
    tmp.ctx = c->ctx;
    struct Guard {
        DeviceArena &a;
        ~Guard() { a.release(); }
    } guard{tmp};
    double *P = nullptr;
    MOS_TRY(tmp.alloc_n((size_t)std::max(W, 1) * NB * ldr, &P));
    for (int J = 0; J < NT; ++J) {
        if (W > 0 && J > 0)
            hipLaunchKernelGGL(k_fwd_part, dim3(blocks, W), dim3(256), 0, st, (const double *)c->tiles,
                               (const double *)rhs, P, J, W, ldr);
        hipLaunchKernelGGL(k_fwd_fin, dim3(blocks), dim3(256), 0, st, dinv, (const double *)P, rhs, J, W, ldr);
    }
    for (int J = NT - 1; J >= 0; --J) {
        if (W > 0 && J + 1 < NT)
            hipLaunchKernelGGL(k_bwd_part, dim3(blocks, W), dim3(256), 0, st, (const double *)c->tiles,
                               (const double *)rhs, P, J, W, NT, ldr);
        hipLaunchKernelGGL(k_bwd_fin, dim3(blocks), dim3(256), 0, st, dinv, (const double *)P, rhs, J, W, NT, ldr);
    }
    MOS_LAUNCH_CHECK();
    return MOS_OK;  // releasing the scratch waits for the stream
}

}  // namespace mos
