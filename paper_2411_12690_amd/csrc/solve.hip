// Global stage (Sec. 4.3-4.4, eq. 20): the reduced system of the whole array
// is never assembled.  Its matrix-vector product is taken element by element:
// every cell's n x n stiffness K_r(type) multiplies the cell's gathered DoFs
// (one dense GEMM per cell type on MFMA, K_r shared by all cells of a type),
// and a node-centric pass sums the <= 4 cell contributions of every DoF in
// ascending cell order (deterministic, no atomics).  Constraints are lifted
// symmetrically.  Jacobi-PCG runs on the device with its scalars in device
// memory (no host round trip per iteration); the host only polls a status
// word between chunks of iterations.  The outer loop is iterative
// refinement on the FP64 true residual: with FP64 inner PCG it is a restart
// safeguard, with FP32 inner PCG it is the mixed-precision solver.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mesh.h"
#include "mos_internal.h"

namespace mos {

mos_status fill(mos_ctx ctx, double *p, size_t n, double v);

namespace {

struct TypeTable {
    const void *kr[MAX_TYPES];   // padded K_r (ldk x ldk), double or float
    const double *br[MAX_TYPES]; // b_r (n)
    int seg[MAX_TYPES + 1];      // slot ranges per type
    int n_types;
};

struct PcgState {
    double rho[2];   // r.z, double-buffered by iteration parity
    double pq;       // p.Ap of the current iteration
    double rr;       // r.r after the last update
    double tol2;     // stop when rr <= tol2
    int iter, done, max_iter, pad;
};

__device__ __forceinline__ int type_of_slot(const TypeTable &tt, int slot) {
    int t = 0;
    while (t + 1 < tt.n_types && slot >= tt.seg[t + 1]) ++t;
    return t;
}

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // Output register q of lane l holds row l/16 + 4q, column l%16.
    static __device__ __forceinline__ int row(int lane, int q) { return lane / 16 + 4 * q; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // Output register q of lane l holds row 4(l/16) + q, column l%16.
    static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane / 16) + q; }
};

// Y[k][slot] = sum_j K_r(type)[k][j] * v[gidx[j][slot]]: one wave per
// (16-row block, 16-slot block).  K_r is symmetric, so the A operand is read
// as K_r[j][k] which makes the 16 lanes of a row group read consecutive words.
template <class T>
__global__ __launch_bounds__(64) void k_cell_gemm(TypeTable tt, const T *v, const int32_t *gidx, T *Y, int ldk,
                                                  int n_pc, const PcgState *st) {
    if (st && st->done) return;
    typedef typename Mfma<T>::v4 v4;
    const int rb = blockIdx.x, pc0 = blockIdx.y * 16;
    const int lane = threadIdx.x;
    const T *kr = static_cast<const T *>(tt.kr[type_of_slot(tt, pc0)]);
    const int col = pc0 + lane % 16;
    v4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < ldk; k0 += 4) {
        const int kk = k0 + lane / 16;
        T a = kr[(size_t)kk * ldk + rb * 16 + lane % 16];
        int gi = gidx[(size_t)kk * n_pc + col];
        T b = gi >= 0 ? v[gi] : T(0);
        acc = Mfma<T>::op(a, b, acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Y[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * n_pc + col] = acc[q];
}

// Whether the solve has stopped, read once per block and shared, so every
// wave of a block takes the same early exit (another block may set the flag
// while this block runs).
__device__ __forceinline__ bool block_done(const PcgState *st) {
    __shared__ int flag;
    if (threadIdx.x == 0) flag = st->done;
    __syncthreads();
    return flag != 0;
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[16];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    const int w = threadIdx.x / 64, nw = blockDim.x / 64;
    __syncthreads();
    if (threadIdx.x % 64 == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += sh[i];
    return s;
}

// Sum of n partials in a fixed order, result in every thread of the block.
__device__ __forceinline__ double sum_partials(const double *part, int n) {
    double v = 0.0;
    if (threadIdx.x < 64)
        for (int i = threadIdx.x; i < n; i += 64) v += part[i];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    __shared__ double sh;
    __syncthreads();
    if (threadIdx.x == 0) sh = v;
    __syncthreads();
    return sh;
}

// q[d] = sum over the cells around d's node of Y[3s+ci][slot]; in mode 0 the
// lifted operator keeps constrained DoFs as identity (q = p there) and the
// block partial of p.q is written; mode 1 is the raw operator.
template <class T>
__global__ void k_assemble(const T *Y, const int32_t *inc, const uint8_t *cmask, const T *p, T *q, int64_t n_dofs,
                           int n_pc, int mode, double *part, const PcgState *st) {
    if (st && block_done(st)) return;
    double acc = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n_dofs; d += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = d / 3;
        const int ci = (int)(d % 3);
        T s = 0;
        for (int e = 0; e < 4; ++e) {
            int v = inc[node * 4 + e];
            if (v < 0) break;
            s += Y[(size_t)(3 * (v & MAX_SURF) + ci) * n_pc + (v >> INC_SHIFT)];
        }
        if (mode == 0) {
            T pv = p[d];
            T qv = cmask[d] ? pv : s;
            q[d] = qv;
            acc += (double)pv * (double)qv;
        } else {
            q[d] = s;
        }
    }
    if (mode == 0) {
        double b = block_sum(acc);
        if (threadIdx.x == 0) part[blockIdx.x] = b;
    }
}

template <class T>
__global__ void k_pcg_init(const T *rhs, T *x, T *r, T *z, T *p, const T *dinv, int64_t n, double *part_rz,
                           double *part_rr) {
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        T rv = rhs[i];
        T zv = dinv[i] * rv;
        x[i] = 0;
        r[i] = rv;
        z[i] = zv;
        p[i] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
    }
    double a = block_sum(rz);
    double b = block_sum(rr);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = a;
        part_rr[blockIdx.x] = b;
    }
}

__global__ void k_pcg_init2(const double *part_rz, const double *part_rr, int nparts, PcgState *st, double tol2,
                            int max_iter) {
    double rz = sum_partials(part_rz, nparts);
    double rr = sum_partials(part_rr, nparts);
    if (threadIdx.x == 0) {
        st->rho[0] = rz;
        st->rho[1] = 0.0;
        st->pq = 0.0;
        st->rr = rr;
        st->tol2 = tol2;
        st->iter = 0;
        st->max_iter = max_iter;
        st->done = (rr <= tol2) ? 1 : 0;
    }
}

template <class T>
__global__ void k_pcg_update1(T *x, T *r, T *z, const T *p, const T *q, const T *dinv, int64_t n,
                              const double *part_pq, int nparts, double *part_rz, double *part_rr, PcgState *st,
                              int parity) {
    if (block_done(st)) return;
    const double pq = sum_partials(part_pq, nparts);
    const double alpha = st->rho[parity] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->pq = pq;
    const T a = (T)alpha;
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += a * p[i];
        T rv = r[i] - a * q[i];
        r[i] = rv;
        T zv = dinv[i] * rv;
        z[i] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
    }
    double s1 = block_sum(rz);
    double s2 = block_sum(rr);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = s1;
        part_rr[blockIdx.x] = s2;
    }
}

template <class T>
__global__ void k_pcg_update2(T *p, const T *z, int64_t n, const double *part_rz, const double *part_rr, int nparts,
                              PcgState *st, int parity) {
    if (block_done(st)) return;
    const double rz = sum_partials(part_rz, nparts);
    const double rr = sum_partials(part_rr, nparts);
    const double beta = rz / st->rho[parity];
    const T b = (T)beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + b * p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho[parity ^ 1] = rz;
        st->rr = rr;
        st->iter += 1;
        if (!(st->pq > 0.0) || !isfinite(rz) || !isfinite(st->pq)) st->done = 2;
        else if (rr <= st->tol2) st->done = 1;
        else if (st->iter >= st->max_iter) st->done = 3;
    }
}

// b_raw[d] = dT * sum over the cells around d of b_r(type)[3s+ci].
__global__ void k_rhs_assemble(TypeTable tt, const int32_t *inc, double dT, double *b, int64_t n_dofs) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_dofs) return;
    const int64_t node = d / 3;
    const int ci = (int)(d % 3);
    double s = 0.0;
    for (int e = 0; e < 4; ++e) {
        int v = inc[node * 4 + e];
        if (v < 0) break;
        s += tt.br[type_of_slot(tt, v >> INC_SHIFT)][3 * (v & MAX_SURF) + ci];
    }
    b[d] = dT * s;
}

template <class T>
__global__ void k_diag(TypeTable tt, const int32_t *inc, const uint8_t *cmask, T *dinv, int64_t n_dofs, int ldk) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_dofs) return;
    const int64_t node = d / 3;
    const int ci = (int)(d % 3);
    double s = 0.0;
    for (int e = 0; e < 4; ++e) {
        int v = inc[node * 4 + e];
        if (v < 0) break;
        const int k = 3 * (v & MAX_SURF) + ci;
        s += static_cast<const double *>(tt.kr[type_of_slot(tt, v >> INC_SHIFT)])[(size_t)k * ldk + k];
    }
    dinv[d] = cmask[d] ? T(1) : T(1.0 / s);
}

// Lifted right-hand side: g on constrained DoFs, b - A g elsewhere; partial of its squared norm.
__global__ void k_lift(const double *b_raw, const double *ag, const double *g, const uint8_t *cmask, double *b_l,
                       int64_t n, double *part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = cmask[i] ? g[i] : b_raw[i] - ag[i];
        b_l[i] = v;
        acc += v * v;
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// True residual of the lifted system: 0 on constrained DoFs, b - A x on free.
__global__ void k_residual(const double *b_raw, const double *ax, const uint8_t *cmask, double *r, int64_t n,
                           double *part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = cmask[i] ? 0.0 : b_raw[i] - ax[i];
        r[i] = v;
        acc += v * v;
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_to(const double *part, int n, double *out) {
    double s = sum_partials(part, n);
    if (threadIdx.x == 0) *out = s;
}

template <class T>
__global__ void k_scale_to(const double *src, T *dst, double scale, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (T)(src[i] * scale);
}

template <class T>
__global__ void k_add_scaled(double *x, const T *d, double scale, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += scale * (double)d[i];
}

// ---------------------------------------------------------------------------
struct Workspace {
    int64_t n = 0;
    int n_pc = 0, ldk = 0, nblk = 0;
    TypeTable tt64{}, tt32{};
    int32_t *gidx = nullptr, *inc = nullptr;
    uint8_t *cmask = nullptr;
    double *g = nullptr, *b_raw = nullptr, *b_l = nullptr, *x = nullptr, *r64 = nullptr, *q64 = nullptr;
    double *Y64 = nullptr;
    double *part = nullptr, *part2 = nullptr, *part3 = nullptr, *scal = nullptr;
    PcgState *st = nullptr;
    // inner solver vectors (T = double or float)
    void *xi = nullptr, *ri = nullptr, *zi = nullptr, *pi = nullptr, *qi = nullptr, *di = nullptr, *rhs = nullptr,
         *Yi = nullptr;
};

template <class T>
mos_status apply_raw(hipStream_t st, const Workspace &w, const TypeTable &tt, const T *v, T *Y, T *out) {
    hipLaunchKernelGGL(k_cell_gemm<T>, dim3(w.ldk / 16, w.n_pc / 16), dim3(64), 0, st, tt, v, w.gidx, Y, w.ldk, w.n_pc,
                       (const PcgState *)nullptr);
    hipLaunchKernelGGL(k_assemble<T>, dim3(w.nblk), dim3(256), 0, st, Y, w.inc, w.cmask, v, out, w.n, w.n_pc, 1,
                       (double *)nullptr, (const PcgState *)nullptr);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

mos_status read_scalar(mos_ctx ctx, const double *dev, double *out) {
    double *h = static_cast<double *>(ctx->pinned);
    MOS_HIP(hipMemcpyAsync(h, dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    MOS_HIP(hipStreamSynchronize(ctx->stream));
    *out = *h;
    return MOS_OK;
}

// Jacobi-PCG on the lifted operator for rhs (type T), solution in w.xi.
template <class T>
mos_status pcg(mos_ctx ctx, Workspace &w, const TypeTable &tt, double rtol, int max_iter, int *iters, int *done) {
    hipStream_t st = ctx->stream;
    T *x = (T *)w.xi, *r = (T *)w.ri, *z = (T *)w.zi, *p = (T *)w.pi, *q = (T *)w.qi, *di = (T *)w.di,
      *rhs = (T *)w.rhs, *Y = (T *)w.Yi;
    hipLaunchKernelGGL(k_pcg_init<T>, dim3(w.nblk), dim3(256), 0, st, rhs, x, r, z, p, di, w.n, w.part2, w.part3);
    // tol2 relative to the rhs norm: computed in init2 from rr of r0 = rhs.
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, st, w.part3, w.nblk, w.scal);
    MOS_LAUNCH_CHECK();
    double rr0 = 0.0;
    MOS_TRY(read_scalar(ctx, w.scal, &rr0));
    hipLaunchKernelGGL(k_pcg_init2, dim3(1), dim3(64), 0, st, w.part2, w.part3, w.nblk, w.st, rtol * rtol * rr0,
                       max_iter);
    MOS_LAUNCH_CHECK();
    PcgState *hs = static_cast<PcgState *>(ctx->pinned);
    int it = 0, chunk = 8;
    while (true) {
        for (int j = 0; j < chunk; ++j, ++it) {
            const int par = it & 1;
            hipLaunchKernelGGL(k_cell_gemm<T>, dim3(w.ldk / 16, w.n_pc / 16), dim3(64), 0, st, tt, p, w.gidx, Y, w.ldk,
                               w.n_pc, w.st);
            hipLaunchKernelGGL(k_assemble<T>, dim3(w.nblk), dim3(256), 0, st, Y, w.inc, w.cmask, p, q, w.n, w.n_pc, 0,
                               w.part, w.st);
            hipLaunchKernelGGL(k_pcg_update1<T>, dim3(w.nblk), dim3(256), 0, st, x, r, z, p, q, di, w.n, w.part,
                               w.nblk, w.part2, w.part3, w.st, par);
            hipLaunchKernelGGL(k_pcg_update2<T>, dim3(w.nblk), dim3(256), 0, st, p, z, w.n, w.part2, w.part3, w.nblk,
                               w.st, par);
        }
        MOS_LAUNCH_CHECK();
        MOS_HIP(hipMemcpyAsync(hs, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, st));
        MOS_HIP(hipStreamSynchronize(st));
        if (hs->done) break;
        if (it > max_iter + 64) break;
        chunk = std::min(chunk * 2, 64);
    }
    *iters = hs->iter;
    *done = hs->done;
    return MOS_OK;
}

}  // namespace

mos_status solve_array(mos_ctx ctx, const mos_array_desc *d, const mos_rom *roms, int n_roms, mos_sol s) {
    hipStream_t st = ctx->stream;
    const mos_rom r0 = roms[0];
    const mos_cell_desc &cd = r0->desc;
    ArrayMesh m;
    m.build(d->nx_cells, d->ny_cells, cd.interp[0], cd.interp[1], cd.interp[2]);
    const int S = m.S, n = r0->n, ldk = r0->ldk;
    const int64_t n_cells = (int64_t)m.Nx * m.Ny;
    const int64_t n_dofs = 3 * m.n_nodes;
    if (n_dofs > (int64_t)INT32_MAX / 2) {
        set_error("array too large for 32-bit DoF indices");
        return MOS_EINVAL;
    }
    s->precision = d->precision;
    s->Nx = m.Nx;
    s->Ny = m.Ny;
    s->n_cells = (int)n_cells;
    s->n = n;
    s->n_surf = S;
    s->n_elem = r0->n_elem;
    s->ldk = ldk;
    s->n_eblk = r0->n_eblk;
    s->n_nodes = m.n_nodes;
    s->n_dofs = n_dofs;
    s->delta_T = d->delta_T;
    s->n_types = n_roms;
    s->roms.assign(roms, roms + n_roms);

    // Constraints.
    std::vector<double> g(n_dofs, 0.0);
    std::vector<uint8_t> cmask(n_dofs, 0);
    int64_t n_con = 0;
    for (int side = 0; side < 2; ++side) {
        uint32_t flag = side == 0 ? MOS_BC_CLAMP_BOTTOM : MOS_BC_CLAMP_TOP;
        if (!(d->bc_flags & flag)) continue;
        int64_t K = side == 0 ? 0 : m.Z - 1;
        for (int64_t J = 0; J < m.Y; ++J)
            for (int64_t I = 0; I < m.X; ++I) {
                int32_t id = m.node_of[(size_t)((K * m.Y + J) * m.X + I)];
                for (int ci = 0; ci < 3; ++ci) {
                    cmask[3 * (int64_t)id + ci] = 1;
                    g[3 * (int64_t)id + ci] = 0.0;
                }
            }
    }
    for (int64_t i = 0; i < d->n_prescribed; ++i) {
        int64_t dof = d->prescribed_dof[i];
        double v = d->prescribed_value[i];
        if (dof < 0 || dof >= n_dofs || !std::isfinite(v)) {
            set_error("prescribed entry %lld: DoF %lld outside [0, %lld) or value not finite", (long long)i,
                      (long long)dof, (long long)n_dofs);
            return MOS_EINVAL;
        }
        cmask[dof] = 1;
        g[dof] = v;
    }
    for (int64_t i = 0; i < n_dofs; ++i) n_con += cmask[i];
    if (n_con == 0) {
        set_error("array has no constrained DoF: the reduced stiffness is singular (rigid motions)");
        return MOS_ESINGULAR;
    }

    // Slots: cells grouped by type, each type segment padded to 16 slots.
    std::vector<int> count(n_roms, 0);
    for (int64_t c = 0; c < n_cells; ++c) count[d->cell_type[c]]++;
    s->seg.assign(n_roms + 1, 0);
    for (int t = 0; t < n_roms; ++t) s->seg[t + 1] = s->seg[t] + (int)round_up(count[t], 16);
    const int n_pc = std::max(s->seg[n_roms], 16);
    s->n_pc = n_pc;
    std::vector<int32_t> perm(n_pc, -1), slot_of((size_t)n_cells);
    {
        std::vector<int> next(s->seg.begin(), s->seg.end() - 1);
        for (int64_t c = 0; c < n_cells; ++c) {
            int sl = next[d->cell_type[c]]++;
            perm[sl] = (int32_t)c;
            slot_of[c] = sl;
        }
    }
    std::vector<int32_t> gidx((size_t)ldk * n_pc, -1);
    for (int sl = 0; sl < n_pc; ++sl) {
        int32_t c = perm[sl];
        if (c < 0) continue;
        for (int k = 0; k < n; ++k) gidx[(size_t)k * n_pc + sl] = 3 * m.conn[(size_t)c * S + k / 3] + k % 3;
    }
    std::vector<int32_t> inc((size_t)m.n_nodes * 4, -1);
    {
        std::vector<uint8_t> cnt((size_t)m.n_nodes, 0);
        for (int64_t c = 0; c < n_cells; ++c)
            for (int sidx = 0; sidx < S; ++sidx) {
                int32_t node = m.conn[(size_t)c * S + sidx];
                inc[(size_t)node * 4 + cnt[node]++] = (slot_of[c] << INC_SHIFT) | sidx;
            }
    }

    // Device buffers.
    Workspace w;
    w.n = n_dofs;
    w.n_pc = n_pc;
    w.ldk = ldk;
    w.nblk = (int)std::min<int64_t>(std::max<int64_t>(1, (n_dofs + 255) / 256), 1024);
    DeviceArena tmp;
    tmp.ctx = ctx;
    struct Guard {
        DeviceArena &a;
        ~Guard() { a.release(); }
    } guard{tmp};
    DeviceArena &mem = s->mem;
    MOS_TRY(mem.alloc_n(n_pc, &s->perm));
    MOS_TRY(mem.alloc_n((size_t)n_cells * S, &s->conn));
    MOS_TRY(mem.alloc_n(n_dofs, &s->u));
    MOS_TRY(mem.alloc_n((size_t)ldk * n_pc, &w.gidx));
    s->gidx = w.gidx;
    MOS_TRY(tmp.alloc_n((size_t)m.n_nodes * 4, &w.inc));
    MOS_TRY(tmp.alloc_n(n_dofs, &w.cmask));
    MOS_TRY(tmp.alloc_n(n_dofs, &w.g));
    MOS_TRY(tmp.alloc_n(n_dofs, &w.b_raw));
    MOS_TRY(tmp.alloc_n(n_dofs, &w.b_l));
    MOS_TRY(tmp.alloc_n(n_dofs, &w.r64));
    MOS_TRY(tmp.alloc_n(n_dofs, &w.q64));
    MOS_TRY(tmp.alloc_n((size_t)ldk * n_pc, &w.Y64));
    MOS_TRY(tmp.alloc_n(w.nblk, &w.part));
    MOS_TRY(tmp.alloc_n(w.nblk, &w.part2));
    MOS_TRY(tmp.alloc_n(w.nblk, &w.part3));
    MOS_TRY(tmp.alloc_n(4, &w.scal));
    MOS_TRY(tmp.alloc(sizeof(PcgState), (void **)&w.st));
    w.x = s->u;
    const bool mixed = d->precision == MOS_MIXED;
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.xi));
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.ri));
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.zi));
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.pi));
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.qi));
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.di));
    MOS_TRY(tmp.alloc(n_dofs * esz, &w.rhs));
    MOS_TRY(tmp.alloc((size_t)ldk * n_pc * esz, &w.Yi));

    MOS_HIP(hipMemcpyAsync(s->perm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(s->conn, m.conn.data(), m.conn.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(w.gidx, gidx.data(), gidx.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(w.inc, inc.data(), inc.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(w.cmask, cmask.data(), cmask.size(), hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(w.g, g.data(), g.size() * 8, hipMemcpyHostToDevice, st));
    // x0 = g on constrained DoFs, 0 elsewhere (g is already 0 off the constraints).
    MOS_HIP(hipMemcpyAsync(w.x, g.data(), g.size() * 8, hipMemcpyHostToDevice, st));

    w.tt64.n_types = w.tt32.n_types = n_roms;
    for (int t = 0; t <= n_roms; ++t) w.tt64.seg[t] = w.tt32.seg[t] = s->seg[t];
    for (int t = 0; t < n_roms; ++t) {
        w.tt64.kr[t] = roms[t]->kr_pad;
        w.tt32.kr[t] = roms[t]->kr32_pad;
        w.tt64.br[t] = w.tt32.br[t] = roms[t]->br;
    }

    // Right-hand side, lifting, Jacobi diagonal.
    hipLaunchKernelGGL(k_rhs_assemble, dim3(ceil_div(n_dofs, 256)), dim3(256), 0, st, w.tt64, w.inc, d->delta_T,
                       w.b_raw, n_dofs);
    MOS_LAUNCH_CHECK();
    MOS_TRY(apply_raw<double>(st, w, w.tt64, w.g, w.Y64, w.q64));
    hipLaunchKernelGGL(k_lift, dim3(w.nblk), dim3(256), 0, st, w.b_raw, w.q64, w.g, w.cmask, w.b_l, n_dofs, w.part);
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, st, w.part, w.nblk, w.scal);
    MOS_LAUNCH_CHECK();
    double bb = 0.0;
    MOS_TRY(read_scalar(ctx, w.scal, &bb));
    if (mixed)
        hipLaunchKernelGGL(k_diag<float>, dim3(ceil_div(n_dofs, 256)), dim3(256), 0, st, w.tt64, w.inc, w.cmask,
                           (float *)w.di, n_dofs, ldk);
    else
        hipLaunchKernelGGL(k_diag<double>, dim3(ceil_div(n_dofs, 256)), dim3(256), 0, st, w.tt64, w.inc, w.cmask,
                           (double *)w.di, n_dofs, ldk);
    MOS_LAUNCH_CHECK();

    const double rtol = d->rtol > 0 ? d->rtol : (mixed ? 1e-10 : 1e-12);
    const int max_iters = d->max_iters > 0 ? d->max_iters : 20000;
    const int max_refine = mixed ? 30 : 6;
    const double bnorm = std::sqrt(bb);
    int total_iters = 0, refines = 0;
    double rel = 0.0;
    while (true) {
        // True FP64 residual of the lifted system.
        MOS_TRY(apply_raw<double>(st, w, w.tt64, w.x, w.Y64, w.q64));
        hipLaunchKernelGGL(k_residual, dim3(w.nblk), dim3(256), 0, st, w.b_raw, w.q64, w.cmask, w.r64, n_dofs, w.part);
        hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, st, w.part, w.nblk, w.scal);
        MOS_LAUNCH_CHECK();
        double rr = 0.0;
        MOS_TRY(read_scalar(ctx, w.scal, &rr));
        rel = bnorm > 0 ? std::sqrt(rr) / bnorm : std::sqrt(rr);
        if (!std::isfinite(rel)) {
            set_error("non-finite residual in the global solve");
            return MOS_ENOCONV;
        }
        if (rel <= rtol || rr == 0.0) break;
        if (refines >= max_refine || total_iters >= max_iters) {
            set_error("global solve stopped at relative residual %.3e > rtol %.3e after %d iterations, %d sweeps", rel,
                      rtol, total_iters, refines);
            return MOS_ENOCONV;
        }
        const double rnorm = std::sqrt(rr);
        int iters = 0, done = 0;
        if (mixed) {
            hipLaunchKernelGGL(k_scale_to<float>, dim3(w.nblk), dim3(256), 0, st, w.r64, (float *)w.rhs, 1.0 / rnorm,
                               n_dofs);
            MOS_LAUNCH_CHECK();
            MOS_TRY(pcg<float>(ctx, w, w.tt32, 1e-5, max_iters - total_iters, &iters, &done));
            hipLaunchKernelGGL(k_add_scaled<float>, dim3(w.nblk), dim3(256), 0, st, w.x, (const float *)w.xi, rnorm,
                               n_dofs);
        } else {
            hipLaunchKernelGGL(k_scale_to<double>, dim3(w.nblk), dim3(256), 0, st, w.r64, (double *)w.rhs, 1.0,
                               n_dofs);
            MOS_LAUNCH_CHECK();
            double tol_in = std::max(0.1 * rtol * bnorm / rnorm, 1e-15);
            MOS_TRY(pcg<double>(ctx, w, w.tt64, tol_in, max_iters - total_iters, &iters, &done));
            hipLaunchKernelGGL(k_add_scaled<double>, dim3(w.nblk), dim3(256), 0, st, w.x, (const double *)w.xi, 1.0,
                               n_dofs);
        }
        MOS_LAUNCH_CHECK();
        total_iters += iters;
        refines++;
        if (done == 2) {
            set_error("PCG breakdown (p.Ap <= 0 or non-finite) after %d iterations", total_iters);
            return MOS_ENOCONV;
        }
    }
    s->rel_residual = rel;
    s->iters = total_iters;
    s->refines = refines;
    MOS_HIP(hipStreamSynchronize(st));
    return MOS_OK;
}

}  // namespace mos
