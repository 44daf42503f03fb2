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

// Scalars of the pipelined PCG.  The GEMM kernel of iteration i (block 0)
// reduces the dot-product partials, decides whether to stop, and publishes
// the step (alpha, beta) that the update kernel of the same iteration
// applies; gamma and alpha of iteration i are kept for iteration i+1.
struct PcgState {
    double gamma_prev, alpha_prev;  // of the last applied iteration
    double a_cur, b_cur;            // step of the current iteration
    double rr;                      // ||r||^2 at the last check
    int iter, done, pad0, pad1;
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

// Raw operator: q[d] = sum over the cells around d's node of Y[3s+ci][slot].
template <class T>
__global__ void k_assemble(const T *Y, const int32_t *inc, T *q, int64_t n_dofs, int n_pc) {
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n_dofs; d += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = d / 3;
        const int ci = (int)(d % 3);
        T s = 0;
        for (int e = 0; e < 4; ++e) {
            int v = inc[node * 4 + e];
            if (v < 0) break;
            s += Y[(size_t)(3 * (v & MAX_SURF) + ci) * n_pc + (v >> INC_SHIFT)];
        }
        q[d] = s;
    }
}

// Sum of the cell products around DoF d.
template <class T>
__device__ __forceinline__ T gather_sum(const T *Y, const int32_t *inc, int64_t d, int n_pc) {
    const int64_t node = d / 3;
    const int ci = (int)(d % 3);
    T s = 0;
    for (int e = 0; e < 4; ++e) {
        int v = inc[node * 4 + e];
        if (v < 0) break;
        s += Y[(size_t)(3 * (v & MAX_SURF) + ci) * n_pc + (v >> INC_SHIFT)];
    }
    return s;
}

// Copy DoF d's value into every cell slot that holds it (cell-major layout
// Mc[3s+ci][slot] read densely by the cell GEMM).
template <class T>
__device__ __forceinline__ void scatter_to_cells(T *Mc, const int32_t *inc, int64_t d, int n_pc, T v) {
    const int64_t node = d / 3;
    const int ci = (int)(d % 3);
    for (int e = 0; e < 4; ++e) {
        int iv = inc[node * 4 + e];
        if (iv < 0) break;
        Mc[(size_t)(3 * (iv & MAX_SURF) + ci) * n_pc + (iv >> INC_SHIFT)] = v;
    }
}

__device__ __forceinline__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double sh[3][16];
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m);
        b += __shfl_xor(b, m);
        c += __shfl_xor(c, m);
    }
    const int w = threadIdx.x / 64, nw = blockDim.x / 64;
    __syncthreads();
    if (threadIdx.x % 64 == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int i = 0; i < nw; ++i) {
        a += sh[0][i];
        b += sh[1][i];
        c += sh[2][i];
    }
}

// One wave: fixed-order sums of three partial arrays, result in every lane.
__device__ __forceinline__ void wave_sum3(const double *pa, const double *pb, const double *pc, int n, double &a,
                                          double &b, double &c) {
    a = b = c = 0.0;
    const int lane = threadIdx.x % 64;
    for (int i = lane; i < n; i += 64) {
        a += pa[i];
        b += pb[i];
        c += pc[i];
    }
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m);
        b += __shfl_xor(b, m);
        c += __shfl_xor(c, m);
    }
}

constexpr int GEMM_WAVES = 4;      // split-K ways of the cell GEMM
constexpr int GEMM_MAX_STEPS = 16; // k-steps of 4 whose loads are issued together

// Iteration `it` (it < 0: GEMM only), part 1.  Y[k][slot] = sum_j K_r(type)[k][j] Mc[j][slot] for
// one 16 x 16 output tile per workgroup, K split over four waves and summed
// in a fixed order through LDS; Mc is the cell-major copy of m = M^-1 w.
// One extra block turns the partial sums of (r,u), (w,u), (r,r) into the stop
// decision and the step (alpha, beta) of this iteration, in parallel with the
// GEMM tiles.
template <class T>
__global__ __launch_bounds__(256) void k_ppcg_gemm(TypeTable tt, const T *Mc, T *Y, int ldk, int n_pc, PcgState *st,
                                                   const double *pg, const double *pd, const double *pr, int nparts,
                                                   double tol2, int it, int max_iter) {
    typedef typename Mfma<T>::v4 v4;
    __shared__ v4 red[GEMM_WAVES - 1][64];
    __shared__ int done_flag;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if ((int)blockIdx.y == n_pc / 16) {
        // The extra block row: block 0 does the scalar work of the iteration.
        if (it < 0 || blockIdx.x != 0 || wave != 0) return;
        const double g_prev = st->gamma_prev, a_prev = st->alpha_prev;
        const int done = st->done;
        double gamma, delta, rr;
        wave_sum3(pg, pd, pr, nparts, gamma, delta, rr);
        if (lane == 0 && !done) {
            int stop = 0;
            double alpha = 0.0, beta = 0.0;
            if (rr <= tol2) {
                stop = 1;
            } else if (it >= max_iter) {
                stop = 3;
            } else {
                if (it == 0) {
                    alpha = gamma / delta;
                } else {
                    beta = gamma / g_prev;
                    alpha = gamma / (delta - beta * gamma / a_prev);
                }
                if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(beta)) stop = 2;
            }
            st->rr = rr;
            if (stop) {
                st->done = stop;
                st->iter = it;
            } else {
                st->a_cur = alpha;
                st->b_cur = beta;
                st->gamma_prev = gamma;
                st->alpha_prev = alpha;
                st->iter = it + 1;
            }
        }
        return;
    }
    const int rb = blockIdx.x, pc0 = blockIdx.y * 16;
    const T *kr = static_cast<const T *>(tt.kr[type_of_slot(tt, pc0)]);
    const int col = pc0 + lane % 16;
    const int steps = ldk / (4 * GEMM_WAVES);
    const int k_begin = wave * steps * 4;
    const T *ap = kr + (size_t)(k_begin + lane / 16) * ldk + rb * 16 + lane % 16;
    const T *bp = Mc + (size_t)(k_begin + lane / 16) * n_pc + col;
    T a[GEMM_MAX_STEPS], b[GEMM_MAX_STEPS];
    const int cnt0 = min(GEMM_MAX_STEPS, steps);
    // First operands are requested before the stop flag is known, so both
    // round trips overlap.
#pragma unroll
    for (int j = 0; j < GEMM_MAX_STEPS; ++j)
        if (j < cnt0) {
            a[j] = ap[(size_t)(4 * j) * ldk];
            b[j] = bp[(size_t)(4 * j) * n_pc];
        }
    if (threadIdx.x == 0) done_flag = st->done;
    __syncthreads();
    if (done_flag) return;
    v4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < GEMM_MAX_STEPS; ++j)
        if (j < cnt0) acc = Mfma<T>::op(a[j], b[j], acc);
    for (int s0 = GEMM_MAX_STEPS; s0 < steps; s0 += GEMM_MAX_STEPS) {
        const int cnt = min(GEMM_MAX_STEPS, steps - s0);
#pragma unroll
        for (int j = 0; j < GEMM_MAX_STEPS; ++j)
            if (j < cnt) {
                a[j] = ap[(size_t)(4 * (s0 + j)) * ldk];
                b[j] = bp[(size_t)(4 * (s0 + j)) * n_pc];
            }
#pragma unroll
        for (int j = 0; j < GEMM_MAX_STEPS; ++j)
            if (j < cnt) acc = Mfma<T>::op(a[j], b[j], acc);
    }
    if (wave > 0) red[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < GEMM_WAVES - 1; ++w) acc += red[w][lane];
#pragma unroll
        for (int q = 0; q < 4; ++q) Y[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * n_pc + col] = acc[q];
    }
}

// Pipelined PCG (one fused reduction per iteration), start, part 1:
// r = rhs, u = M^-1 r, x = z = q = s = p = 0, u copied to the cell layout.
template <class T>
__global__ void k_ppcg_start(const T *rhs, const T *dinv, const int32_t *inc, T *x, T *r, T *u, T *z, T *q, T *s,
                             T *p, T *Mc, int64_t n, int n_pc) {
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
        T rv = rhs[d];
        T uv = dinv[d] * rv;
        x[d] = 0;
        r[d] = rv;
        u[d] = uv;
        z[d] = 0;
        q[d] = 0;
        s[d] = 0;
        p[d] = 0;
        scatter_to_cells(Mc, inc, d, n_pc, uv);
    }
}

// Start, part 2: w = A u (lifted: 0 on constrained DoFs), m = M^-1 w in the
// cell layout, block partials of (r,u), (w,u), (r,r).
template <class T>
__global__ void k_ppcg_start2(const T *Y, const int32_t *inc, const uint8_t *cmask, const T *dinv, const T *r,
                              const T *u, T *w, T *m, T *Mc, int64_t n, int n_pc, double *pg, double *pd, double *pr,
                              PcgState *st) {
    double g = 0.0, dl = 0.0, rr = 0.0;
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
        T sum = gather_sum(Y, inc, d, n_pc);
        T wv = cmask[d] ? T(0) : sum;
        T mv = dinv[d] * wv;
        w[d] = wv;
        m[d] = mv;
        scatter_to_cells(Mc, inc, d, n_pc, mv);
        double rv = (double)r[d], uv = (double)u[d];
        g += rv * uv;
        dl += (double)wv * uv;
        rr += rv * rv;
    }
    block_sum3(g, dl, rr);
    if (threadIdx.x == 0) {
        pg[blockIdx.x] = g;
        pd[blockIdx.x] = dl;
        pr[blockIdx.x] = rr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = 0;
        st->done = 0;
        st->rr = 0.0;
    }
}

// Iteration `it`, part 2, per DoF: n = A m from the cell products, the eight
// recurrences with the step published by part 1, m = M^-1 w copied to the
// cell layout, and the block partials of the next (r,u), (w,u), (r,r).
template <class T>
__global__ void k_ppcg_step(const T *Y, const int32_t *inc, const uint8_t *cmask, const T *dinv, T *x, T *r, T *u,
                            T *w, T *z, T *q, T *s, T *p, T *m, T *Mc, int64_t n, int n_pc, double *pg, double *pd,
                            double *pr, const PcgState *st) {
    __shared__ int done_flag;
    __shared__ double step[2];
    const int64_t d0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // The incidence of the first DoF is requested before the flag barrier.
    int4 inc0 = make_int4(-1, -1, -1, -1);
    if (d0 < n) inc0 = reinterpret_cast<const int4 *>(inc)[d0 / 3];
    if (threadIdx.x == 0) {
        done_flag = st->done;
        step[0] = st->a_cur;
        step[1] = st->b_cur;
    }
    __syncthreads();
    if (done_flag) return;
    const T a = (T)step[0], b = (T)step[1];
    double g = 0.0, dl = 0.0, r2 = 0.0;
    for (int64_t d = d0; d < n; d += (int64_t)gridDim.x * blockDim.x) {
        const int ci = (int)(d % 3);
        int4 iv = d == d0 ? inc0 : reinterpret_cast<const int4 *>(inc)[d / 3];
        const int e4[4] = {iv.x, iv.y, iv.z, iv.w};
        T sum = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (e4[e] >= 0) sum += Y[(size_t)(3 * (e4[e] & MAX_SURF) + ci) * n_pc + (e4[e] >> INC_SHIFT)];
        T nv = cmask[d] ? T(0) : sum;
        T zv = nv + b * z[d];
        T qv = m[d] + b * q[d];
        T sv = w[d] + b * s[d];
        T pv = u[d] + b * p[d];
        x[d] += a * pv;
        T rv = r[d] - a * sv;
        T uv = u[d] - a * qv;
        T wv = w[d] - a * zv;
        T mv = dinv[d] * wv;
        z[d] = zv;
        q[d] = qv;
        s[d] = sv;
        p[d] = pv;
        r[d] = rv;
        u[d] = uv;
        w[d] = wv;
        m[d] = mv;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (e4[e] >= 0) Mc[(size_t)(3 * (e4[e] & MAX_SURF) + ci) * n_pc + (e4[e] >> INC_SHIFT)] = mv;
        g += (double)rv * (double)uv;
        dl += (double)wv * (double)uv;
        r2 += (double)rv * (double)rv;
    }
    block_sum3(g, dl, r2);
    if (threadIdx.x == 0) {
        pg[blockIdx.x] = g;
        pd[blockIdx.x] = dl;
        pr[blockIdx.x] = r2;
    }
}

__global__ void k_zero_words(uint32_t *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
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
    double *part = nullptr, *pg = nullptr, *pd = nullptr, *pr = nullptr, *scal = nullptr;
    PcgState *st = nullptr;
    // Inner solver (T = double or float): vectors and the cell-major copy.
    void *v[11] = {};     // x r u w z q s p m dinv rhs
    void *Mc = nullptr, *Yi = nullptr;
};

enum { VX, VR, VU, VW, VZ, VQ, VS, VP, VM, VDINV, VRHS, NVEC };

template <class T>
mos_status apply_raw(hipStream_t st, const Workspace &w, const TypeTable &tt, const T *v, T *Y, T *out) {
    hipLaunchKernelGGL(k_cell_gemm<T>, dim3(w.ldk / 16, w.n_pc / 16), dim3(64), 0, st, tt, v, w.gidx, Y, w.ldk, w.n_pc,
                       (const PcgState *)nullptr);
    hipLaunchKernelGGL(k_assemble<T>, dim3(w.nblk), dim3(256), 0, st, Y, w.inc, out, w.n, w.n_pc);
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

// Pipelined Jacobi-PCG on the lifted operator for the rhs in w.v[VRHS]
// (type T); the solution is left in w.v[VX].  Stops when the recursive
// residual satisfies ||r|| <= rtol ||rhs||.
template <class T>
mos_status pcg(mos_ctx ctx, Workspace &w, const TypeTable &tt, double rtol, int max_iter, int *iters, int *done) {
    hipStream_t st = ctx->stream;
    T *V[NVEC];
    for (int i = 0; i < NVEC; ++i) V[i] = static_cast<T *>(w.v[i]);
    T *Mc = static_cast<T *>(w.Mc), *Y = static_cast<T *>(w.Yi);
    const dim3 g_gemm(w.ldk / 16, w.n_pc / 16 + 1), g_vec(w.nblk), b_vec(256);
    hipLaunchKernelGGL(k_ppcg_start<T>, g_vec, b_vec, 0, st, V[VRHS], V[VDINV], w.inc, V[VX], V[VR], V[VU], V[VZ],
                       V[VQ], V[VS], V[VP], Mc, w.n, w.n_pc);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, (uint32_t *)w.st, sizeof(PcgState) / 4);
    // Y = K_r Mc(u) for w = A u: the GEMM alone (it = -1: no scalar work).
    hipLaunchKernelGGL(k_ppcg_gemm<T>, g_gemm, dim3(64 * GEMM_WAVES), 0, st, tt, Mc, Y, w.ldk, w.n_pc, w.st, w.pg,
                       w.pd, w.pr, 0, 0.0, -1, 0);
    hipLaunchKernelGGL(k_ppcg_start2<T>, g_vec, b_vec, 0, st, Y, w.inc, w.cmask, V[VDINV], V[VR], V[VU], V[VW], V[VM],
                       Mc, w.n, w.n_pc, w.pg, w.pd, w.pr, w.st);
    MOS_LAUNCH_CHECK();
    // tol2 is relative to ||rhs||^2 = the rr partials of the start kernel.
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(64), 0, st, w.pr, w.nblk, w.scal);
    MOS_LAUNCH_CHECK();
    double rr0 = 0.0;
    MOS_TRY(read_scalar(ctx, w.scal, &rr0));
    const double tol2 = rtol * rtol * rr0;
    PcgState *hs = static_cast<PcgState *>(ctx->pinned);
    int it = 0, chunk = 8;
    while (true) {
        for (int j = 0; j < chunk; ++j, ++it) {
            launch_timed(ctx, MOS_K_CELL_GEMM, k_ppcg_gemm<T>, g_gemm, dim3(64 * GEMM_WAVES), 0, st, tt,
                         (const T *)Mc, Y, w.ldk, w.n_pc, w.st, (const double *)w.pg, (const double *)w.pd,
                         (const double *)w.pr, w.nblk, tol2, it, max_iter);
            launch_timed(ctx, MOS_K_PCG_UPDATE, k_ppcg_step<T>, g_vec, b_vec, 0, st, (const T *)Y,
                         (const int32_t *)w.inc, (const uint8_t *)w.cmask, (const T *)V[VDINV], V[VX], V[VR], V[VU],
                         V[VW], V[VZ], V[VQ], V[VS], V[VP], V[VM], Mc, w.n, w.n_pc, w.pg, w.pd, w.pr,
                         (const PcgState *)w.st);
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
    MOS_TRY(tmp.alloc_n(w.nblk, &w.pg));
    MOS_TRY(tmp.alloc_n(w.nblk, &w.pd));
    MOS_TRY(tmp.alloc_n(w.nblk, &w.pr));
    MOS_TRY(tmp.alloc_n(4, &w.scal));
    MOS_TRY(tmp.alloc(sizeof(PcgState), (void **)&w.st));
    w.x = s->u;
    const bool mixed = d->precision == MOS_MIXED;
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    for (int i = 0; i < NVEC; ++i) MOS_TRY(tmp.alloc(n_dofs * esz, &w.v[i]));
    MOS_TRY(tmp.alloc((size_t)ldk * n_pc * esz, &w.Mc));
    MOS_TRY(tmp.alloc((size_t)ldk * n_pc * esz, &w.Yi));
    {
        size_t words = (size_t)ldk * n_pc * esz / 4;
        hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<size_t>((words + 255) / 256, 4096)), dim3(256), 0, st,
                           (uint32_t *)w.Mc, words);
        MOS_LAUNCH_CHECK();
    }

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
                           (float *)w.v[VDINV], n_dofs, ldk);
    else
        hipLaunchKernelGGL(k_diag<double>, dim3(ceil_div(n_dofs, 256)), dim3(256), 0, st, w.tt64, w.inc, w.cmask,
                           (double *)w.v[VDINV], n_dofs, ldk);
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
            hipLaunchKernelGGL(k_scale_to<float>, dim3(w.nblk), dim3(256), 0, st, w.r64, (float *)w.v[VRHS],
                               1.0 / rnorm, n_dofs);
            MOS_LAUNCH_CHECK();
            MOS_TRY(pcg<float>(ctx, w, w.tt32, 1e-4, max_iters - total_iters, &iters, &done));
            hipLaunchKernelGGL(k_add_scaled<float>, dim3(w.nblk), dim3(256), 0, st, w.x, (const float *)w.v[VX],
                               rnorm, n_dofs);
        } else {
            hipLaunchKernelGGL(k_scale_to<double>, dim3(w.nblk), dim3(256), 0, st, w.r64, (double *)w.v[VRHS], 1.0,
                               n_dofs);
            MOS_LAUNCH_CHECK();
            double tol_in = std::max(0.1 * rtol * bnorm / rnorm, 1e-15);
            MOS_TRY(pcg<double>(ctx, w, w.tt64, tol_in, max_iters - total_iters, &iters, &done));
            hipLaunchKernelGGL(k_add_scaled<double>, dim3(w.nblk), dim3(256), 0, st, w.x, (const double *)w.v[VX],
                               1.0, n_dofs);
        }
        MOS_LAUNCH_CHECK();
        total_iters += iters;
        refines++;
        // A breakdown after some progress only ends this correction sweep: the
        // iterate up to the last completed step is kept and the FP64 residual
        // of the next sweep decides.  Without progress the solve has failed.
        if (done == 2 && iters == 0) {
            set_error("PCG breakdown (p.Ap <= 0 or non-finite) at the start of sweep %d", refines);
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
