// Per-cell stress reconstruction (Sec. 4.3 last paragraph with eq. 1 and 15).
// For every cell c and fine element e of its type:
//   sigma(c, e) = dT sigma_T(e) + Psi(e) u_c,   Psi = D B0 Phi at the centroid,
// i.e. one GEMM per cell type, (6 n_elem x n) times (n x cells), with the
// thermal term and the von Mises norm fused into the epilogue.  The stress
// basis is stored so that one 16-row MFMA block is one stress component of
// 16 consecutive elements; each lane then holds all six components of its
// four (element, cell) outputs and forms von Mises in registers.  FP64 MFMA
// 16x16x4: lane l supplies A[l%16][l/16], B[l/16][l%16] and receives
// D[l/16 + 4q][l%16] in register q.
#include <cmath>

#include "mesh.h"
#include "mos_internal.h"

namespace mos {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct ReconTable {
    const double *psi[MAX_TYPES];
    const double *sig_t[MAX_TYPES];
    int seg[MAX_TYPES + 1];
    int n_types;
};

__device__ __forceinline__ int type_of_slot(const ReconTable &tt, int slot) {
    int t = 0;
    while (t + 1 < tt.n_types && slot >= tt.seg[t + 1]) ++t;
    return t;
}

// U[k][slot] = u[gidx[k][slot]] (0 for padding).
__global__ void k_gather_u(const double *u, const int32_t *gidx, double *U, int64_t total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int g = gidx[i];
    U[i] = g >= 0 ? u[g] : 0.0;
}

// One wave per (element block of 16, slot block of 16); four waves per
// workgroup share the element block so the Psi stream is reused from L1.
template <class OutT>
__global__ __launch_bounds__(256) void k_recon_f64(ReconTable tt, const double *U, const int32_t *perm, int n_pc,
                                                   int ldk, int n_elem, double dT, OutT *vm, OutT *sig6) {
    const int eb = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int sb = blockIdx.y * 4 + wave;
    const int pc0 = sb * 16;
    if (pc0 >= n_pc) return;
    const int t = type_of_slot(tt, pc0);
    const double *psi = tt.psi[t] + (size_t)eb * 6 * ldk * 16;
    d4 acc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < ldk; k0 += 4) {
        const int kk = k0 + lane / 16;
        const double b = U[(size_t)kk * n_pc + pc0 + lane % 16];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double a = psi[((size_t)k * ldk + kk) * 16 + lane % 16];
            acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
        }
    }
    const int cell = perm[pc0 + lane % 16];
    if (cell < 0) return;
    const double *st = tt.sig_t[t];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = eb * 16 + lane / 16 + 4 * q;   // FP64 MFMA output row
        if (e >= n_elem) continue;
        double s[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = acc[k][q] + dT * st[(size_t)e * 6 + k];
        const size_t o = (size_t)cell * n_elem + e;
        if (vm) {
            double a = s[0] - s[1], b = s[1] - s[2], c = s[2] - s[0];
            vm[o] = (OutT)sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
        }
        if (sig6)
#pragma unroll
            for (int k = 0; k < 6; ++k) sig6[o * 6 + k] = (OutT)s[k];
    }
}

}  // namespace

mos_status reconstruct(mos_ctx ctx, mos_sol s, uint32_t outputs, void *vm, void *sigma6) {
    hipStream_t st = ctx->stream;
    ReconTable tt{};
    tt.n_types = s->n_types;
    for (int t = 0; t <= s->n_types; ++t) tt.seg[t] = s->seg[t];
    for (int t = 0; t < s->n_types; ++t) {
        tt.psi[t] = s->roms[t]->psi;
        tt.sig_t[t] = s->roms[t]->sig_t;
    }
    DeviceArena tmp;
    tmp.ctx = ctx;
    struct Guard {
        DeviceArena &a;
        ~Guard() { a.release(); }
    } guard{tmp};
    double *U = nullptr;
    const int64_t total = (int64_t)s->ldk * s->n_pc;
    MOS_TRY(tmp.alloc_n(total, &U));
    hipLaunchKernelGGL(k_gather_u, dim3(ceil_div(total, 256)), dim3(256), 0, st, s->u, s->gidx, U, total);
    MOS_LAUNCH_CHECK();
    dim3 grid(s->n_eblk, ceil_div(s->n_pc / 16, 4));
    void *v = (outputs & MOS_OUT_VM) ? vm : nullptr;
    void *g = (outputs & MOS_OUT_SIGMA6) ? sigma6 : nullptr;
    if (s->precision == MOS_FP64)
        launch_timed(ctx, MOS_K_RECON, k_recon_f64<double>, grid, dim3(256), 0, st, tt, (const double *)U,
                     (const int32_t *)s->perm, s->n_pc, s->ldk, s->n_elem, s->delta_T, (double *)v, (double *)g);
    else
        launch_timed(ctx, MOS_K_RECON, k_recon_f64<float>, grid, dim3(256), 0, st, tt, (const double *)U,
                     (const int32_t *)s->perm, s->n_pc, s->ldk, s->n_elem, s->delta_T, (float *)v, (float *)g);
    MOS_LAUNCH_CHECK();
    MOS_HIP(hipStreamSynchronize(st));
    return MOS_OK;
}

}  // namespace mos
