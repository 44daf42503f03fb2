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
#include <cstdlib>
#include <mutex>

#include "bf16.h"
#include "gmem.h"
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

// LDS-staged form for bases up to ldk = 176: one workgroup of 8 waves per
// (element block of 16, slice of one type's slot blocks) stages that element
// block of Psi -- all six components, ldk k-rows of 16 elements, 135 KB at
// ldk = 176 -- in LDS once; each wave then streams slot blocks, holding u of
// 16 cells (ks MFMA k-steps) in registers and reading the A fragments from
// LDS, so Psi is read from memory once per workgroup instead of once per
// wave.  Same accumulation order as k_recon_f64.
template <class OutT, int KS, bool EXACT>
__global__ __launch_bounds__(512, 1) void k_recon_f64_lds(const double *psi, const double *sig_t, const double *U,
                                                          const int32_t *perm, int ld, const ReconJob *jobs,
                                                          int n_jobs, int total_sb, int chunk, int ks, int n_elem) {
    __shared__ double lds[6 * 4 * KS * 16];
    __shared__ double st_lds[16][6];
    if (EXACT) ks = KS;
    const int ldk = 4 * ks;
    const int eb = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int y0 = blockIdx.y * chunk, y1 = min(y0 + chunk, total_sb);
    {
        const double *g = psi + (size_t)eb * 6 * ldk * 16;
        for (int i = threadIdx.x; i < 6 * ldk * 16; i += 512) lds[i] = g[i];
        // sigma_T of the element block (rows past n_elem repeat the last; unused).
        if (threadIdx.x < 96) {
            const int e = min(eb * 16 + (int)threadIdx.x / 6, n_elem - 1);
            st_lds[threadIdx.x / 6][threadIdx.x % 6] = sig_t[(size_t)e * 6 + threadIdx.x % 6];
        }
    }
    __syncthreads();
    int j = 0;
    for (int f = y0 + wave; f < y1; f += 8) {
        // Flattened slot block f of the jobs -> its job (jobs in order of sb_off).
        while (j + 1 < n_jobs && f >= jobs[j + 1].sb_off) ++j;
        const ReconJob &J = jobs[j];
        const size_t pc0 = (size_t)(J.sb_first + (f - J.sb_off)) * 16;
        const double dT = J.dT;
        global_ptr<OutT> vm = to_global(static_cast<OutT *>(J.vm));
        global_ptr<OutT> sig6 = to_global(static_cast<OutT *>(J.sig6));
        // The block's cells, requested ahead of the MFMA chain.
        const int cell = perm[pc0 + lane % 16];
        const double *bp = U + (size_t)(lane / 16) * ld + pc0 + lane % 16;
        const double *ap = lds + (lane / 16) * 16 + lane % 16;
        d4 acc[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
        // u is streamed one k-step at a time (a few loads in flight through
        // the partial unroll); the six accumulators stay in registers.
        if (EXACT) {
            // All of the block's u requested at once (straight-line, so each
            // MFMA waits only for its own operand); the scheduling barriers
            // keep the LDS reads of Psi within a few k-steps of their use.
            double b[KS];
#pragma unroll
            for (int k = 0; k < KS; ++k) b[k] = bp[(size_t)(4 * k) * ld];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[(c * ldk + 4 * k) * 16], b[k], acc[c], 0, 0, 0);
                if (k % 2 == 1) __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            for (int k = 0; k < ks; ++k) {
                const double b = bp[(size_t)(4 * k) * ld];
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[(c * ldk + 4 * k) * 16], b, acc[c], 0, 0, 0);
            }
        }
        if (cell < 0) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = eb * 16 + lane / 16 + 4 * q;  // FP64 MFMA output row
            if (e >= n_elem) continue;
            double sv[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) sv[c] = acc[c][q] + dT * st_lds[lane / 16 + 4 * q][c];
            const size_t o = (size_t)cell * n_elem + e;
            if (vm) {
                double x = sv[0] - sv[1], y = sv[1] - sv[2], z = sv[2] - sv[0];
                vm[o] = (OutT)sqrt(0.5 * (x * x + y * y + z * z) + 3.0 * (sv[3] * sv[3] + sv[4] * sv[4] + sv[5] * sv[5]));
            }
            if (sig6)
#pragma unroll
                for (int c = 0; c < 6; ++c) sig6[o * 6 + c] = (OutT)sv[c];
        }
    }
}

// The same kernel with the cell operand streamed in chunks of KC k-steps,
// double-buffered across chunks and across a wave's slot blocks: the next
// chunk's loads (the next block's first chunk during the last one) are in
// flight while the current chunk's MFMAs run, so no block starts with an
// exposed round trip, and two chunks of u take the registers one whole
// block took (no spills).  Same products in the same order as
// k_recon_f64_lds, so the same bits.  The basis is stored with LDK columns
// and takes KS k-steps (4 KS <= LDK): a basis of 168 in the 176-column
// layout issues 42, not the 2 padding steps that only add zeros.
template <class OutT, int KS, int KC, int LDK = 4 * KS>
__global__ __launch_bounds__(512, 1) void k_recon_f64_pipe(const double *psi, const double *sig_t, const double *U,
                                                           const int32_t *perm, int ld, const ReconJob *jobs,
                                                           int n_jobs, int total_sb, int chunk, int n_elem) {
    static_assert(KS % KC == 0, "chunks must tile the k-steps");
    static_assert(4 * KS <= LDK, "the k-steps must fit the stored columns");
    constexpr int NCH = KS / KC;
    constexpr int ldk = LDK;
    __shared__ double lds[6 * ldk * 16];
    __shared__ double st_lds[16][6];
    const int eb = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int y0 = blockIdx.y * chunk, y1 = min(y0 + chunk, total_sb);
    {
        const double *g = psi + (size_t)eb * 6 * ldk * 16;
        for (int i = threadIdx.x; i < 6 * ldk * 16; i += 512) lds[i] = g[i];
        if (threadIdx.x < 96) {
            const int e = min(eb * 16 + (int)threadIdx.x / 6, n_elem - 1);
            st_lds[threadIdx.x / 6][threadIdx.x % 6] = sig_t[(size_t)e * 6 + threadIdx.x % 6];
        }
    }
    __syncthreads();
    int f = y0 + wave;
    if (f >= y1) return;
    int j = 0;
    // Operand column of flattened slot block f for this lane (job lookup
    // moves forward only).
    auto column = [&](int fb, int &jj) -> size_t {
        while (jj + 1 < n_jobs && fb >= jobs[jj + 1].sb_off) ++jj;
        const ReconJob &J = jobs[jj];
        return (size_t)(J.sb_first + (fb - J.sb_off)) * 16;
    };
    int jn = j;
    size_t pc0 = column(f, j);
    const double *ap = lds + (lane / 16) * 16 + lane % 16;
    double bc[KC], bn[KC];
    {
        const double *bp = U + (size_t)(lane / 16) * ld + pc0 + lane % 16;
#pragma unroll
        for (int k = 0; k < KC; ++k) bc[k] = bp[(size_t)(4 * k) * ld];
    }
    while (true) {
        const ReconJob &J = jobs[j];
        const double dT = J.dT;
        global_ptr<OutT> vm = to_global(static_cast<OutT *>(J.vm));
        global_ptr<OutT> sig6 = to_global(static_cast<OutT *>(J.sig6));
        const int cell = perm[pc0 + lane % 16];
        const int fn = f + 8;
        jn = j;
        const size_t pcn = fn < y1 ? column(fn, jn) : pc0;
        d4 acc[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            // Next chunk: this block's, or the next block's first (past the
            // wave's last block, the first chunk again; unused).
            const size_t col = ch + 1 < NCH ? pc0 : pcn;
            const int k0 = ch + 1 < NCH ? (ch + 1) * KC : 0;
            const double *bp = U + (size_t)(lane / 16) * ld + col + lane % 16;
#pragma unroll
            for (int k = 0; k < KC; ++k) bn[k] = bp[(size_t)(4 * (k0 + k)) * ld];
#pragma unroll
            for (int k = 0; k < KC; ++k) {
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[(c * ldk + 4 * (ch * KC + k)) * 16], bc[k],
                                                                 acc[c], 0, 0, 0);
                if (k % 2 == 1) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int k = 0; k < KC; ++k) bc[k] = bn[k];
        }
        if (cell >= 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = eb * 16 + lane / 16 + 4 * q;  // FP64 MFMA output row
                if (e >= n_elem) continue;
                double sv[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) sv[c] = acc[c][q] + dT * st_lds[lane / 16 + 4 * q][c];
                const size_t o = (size_t)cell * n_elem + e;
                if (vm) {
                    double x = sv[0] - sv[1], y = sv[1] - sv[2], z = sv[2] - sv[0];
                    vm[o] = (OutT)sqrt(0.5 * (x * x + y * y + z * z) +
                                       3.0 * (sv[3] * sv[3] + sv[4] * sv[4] + sv[5] * sv[5]));
                }
                if (sig6)
#pragma unroll
                    for (int c = 0; c < 6; ++c) sig6[o * 6 + c] = (OutT)sv[c];
            }
        }
        if (fn >= y1) break;
        f = fn;
        j = jn;
        pc0 = pcn;
    }
}

// Reduced-precision form of the same GEMM: BF16 operands, FP32 accumulation
// on the 16x16x32 MFMA.  Plain BF16 rounding of Psi and u loses too much to
// the cancellation inside Psi u, so both operands are split into hi + lo
// BF16 halves and three products are kept (hi*hi + hi*lo + lo*hi).
// Lane l supplies A[l%16][8(l/16)+v] and B[8(l/16)+v][l%16] (v = 0..7) and
// receives D[4(l/16)+q][l%16] in register q, so each lane ends with all six
// components of four consecutive elements of one cell.

// B fragments of a problem's slot blocks: Ub[sb][ks][lane] holds cell
// 16 sb + l%16, DoFs 32 ks + 8 (l/16) + 0..7, split into hi and lo.
// Job of flattened slot block v (jobs in ascending order of sb_off).
__device__ __forceinline__ const ReconJob &job_of(const ReconJob *jobs, int n_jobs, int v) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].sb_off <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return jobs[lo];
}

// BF16 hi/lo split of the cell operand of every flattened slot block of the
// jobs, in the MFMA B-fragment order (k-step, lane, 8 values).
__global__ void k_split_u(const double *U, int ld, const ReconJob *jobs, int n_jobs, int total, int ldk, int nks,
                          bf16x8 *ub_hi, bf16x8 *ub_lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)total * nks * 64) return;
    const int lane = (int)(i % 64), ks = (int)((i / 64) % nks);
    const int v = (int)(i / (64 * nks));
    const ReconJob &J = job_of(jobs, n_jobs, v);
    const size_t slot = (size_t)(J.sb_first + (v - J.sb_off)) * 16 + lane % 16;
    u16x8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = ks * 32 + 8 * (lane / 16) + q;
        const double x = k < ldk ? U[(size_t)k * ld + slot] : 0.0;
        uint16_t xh, xl;
        bf16_split(x, xh, xl);
        h[q] = xh;
        l[q] = xl;
    }
    ub_hi[i] = __builtin_bit_cast(bf16x8, h);
    ub_lo[i] = __builtin_bit_cast(bf16x8, l);
}

// One workgroup per (element block of 16, slice of one type's slot blocks).
// The workgroup stages its element block of Psi_hi and Psi_lo (6 components
// x nks k-steps x 1 KB each) and of sigma_T in LDS once; its four waves then
// stream the slice CB slot blocks at a time, each LDS fragment feeding 3 CB
// MFMAs.  A wave's blocks come in increasing order, so it finds their jobs
// by advancing one index, and it requests their jobs and cells before the
// MFMA chain so that those round trips overlap it.
template <int KSMAX, int CB>
__global__ __launch_bounds__(256, KSMAX <= 6 ? 2 : 1) void k_recon_bf16(const bf16x8 *psi_hi, const bf16x8 *psi_lo,
                                                       const double *sig_t, const bf16x8 *ub_hi,
                                                       const bf16x8 *ub_lo, const int32_t *perm,
                                                       const ReconJob *jobs, int n_jobs, int v_begin, int n_v,
                                                       int chunk, int nks, int n_elem) {
    __shared__ bf16x8 lds[2][6][KSMAX][64];
    __shared__ double st_lds[16][6];
    const int eb = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int y0 = v_begin + (int)blockIdx.y * chunk, y1 = min(y0 + chunk, v_begin + n_v);
    {
        const bf16x8 *gh = psi_hi + (size_t)eb * 6 * nks * 64;
        const bf16x8 *gl = psi_lo + (size_t)eb * 6 * nks * 64;
        for (int i = threadIdx.x; i < 6 * nks * 64; i += 256) {
            const int c = i / (nks * 64), r = i % (nks * 64);
            lds[0][c][r / 64][r % 64] = gh[i];
            lds[1][c][r / 64][r % 64] = gl[i];
        }
        if (threadIdx.x < 96) {
            const int e = min(eb * 16 + (int)threadIdx.x / 6, n_elem - 1);
            st_lds[threadIdx.x / 6][threadIdx.x % 6] = sig_t[(size_t)e * 6 + threadIdx.x % 6];
        }
    }
    __syncthreads();
    int j = 0;  // job of the wave's current block (blocks only move forward)
    for (int base = y0 + wave * CB; base < y1; base += 4 * CB) {
        // Jobs, outputs and cells of the CB blocks, requested ahead of the MFMAs.
        double dTv[CB];
        global_ptr<float> vmv[CB], s6v[CB];
        int cellv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int v = min(base + cb, y1 - 1);
            while (j + 1 < n_jobs && v >= jobs[j + 1].sb_off) ++j;
            const ReconJob &J = jobs[j];
            dTv[cb] = J.dT;
            vmv[cb] = to_global(static_cast<float *>(J.vm));
            s6v[cb] = to_global(static_cast<float *>(J.sig6));
            cellv[cb] = perm[(size_t)(J.sb_first + (v - J.sb_off)) * 16 + lane % 16];
        }
        f32x4 acc[CB][6];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[cb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            if (ks < nks) {
                bf16x8 bh[CB], bl[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    // Past the slice end: reread the last valid block, results unused.
                    const size_t f = ((size_t)min(base + cb, y1 - 1) * nks + ks) * 64 + lane;
                    bh[cb] = ub_hi[f];
                    bl[cb] = ub_lo[f];
                }
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const bf16x8 ah = lds[0][c][ks][lane], al = lds[1][c][ks][lane];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        acc[cb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], acc[cb][c], 0, 0, 0);
                        acc[cb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], acc[cb][c], 0, 0, 0);
                        acc[cb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], acc[cb][c], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if (base + cb >= y1) continue;
            const double dT = dTv[cb];
            global_ptr<float> vm = vmv[cb], sig6 = s6v[cb];
            const int cell = cellv[cb];
            if (cell < 0) continue;
            const int e0 = eb * 16 + 4 * (lane / 16);
            float vq[4], sq[4][6];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int c = 0; c < 6; ++c) sq[q][c] = acc[cb][c][q] + (float)(dT * st_lds[4 * (lane / 16) + q][c]);
                const float a = sq[q][0] - sq[q][1], b = sq[q][1] - sq[q][2], d = sq[q][2] - sq[q][0];
                vq[q] = sqrtf(0.5f * (a * a + b * b + d * d) +
                              3.0f * (sq[q][3] * sq[q][3] + sq[q][4] * sq[q][4] + sq[q][5] * sq[q][5]));
            }
            const size_t o = (size_t)cell * n_elem + e0;
            const bool whole = e0 + 3 < n_elem && o % 4 == 0;
            if (vm) {
                if (whole) {
                    *(global_ptr<f32x4>)(vm + o) = f32x4{vq[0], vq[1], vq[2], vq[3]};
                } else {
                    for (int q = 0; q < 4; ++q)
                        if (e0 + q < n_elem) vm[o + q] = vq[q];
                }
            }
            if (sig6) {
                if (whole) {
#pragma unroll
                    for (int jj = 0; jj < 6; ++jj)
                        *(global_ptr<f32x4>)(sig6 + o * 6 + 4 * jj) =
                            f32x4{sq[(4 * jj) / 6][(4 * jj) % 6], sq[(4 * jj + 1) / 6][(4 * jj + 1) % 6],
                                  sq[(4 * jj + 2) / 6][(4 * jj + 2) % 6], sq[(4 * jj + 3) / 6][(4 * jj + 3) % 6]};
                } else {
                    for (int q = 0; q < 4; ++q)
                        if (e0 + q < n_elem)
                            for (int c = 0; c < 6; ++c) sig6[(o + q) * 6 + c] = sq[q][c];
                }
            }
        }
    }
}

// Two element blocks per workgroup (32 elements, 144 KB of Psi hi and lo in
// LDS, one workgroup of eight waves per CU): each B fragment a wave loads
// feeds the MFMAs of both blocks, so the cell operand is read from L2 half
// as often per MFMA as with one block per workgroup.  Each wave streams CB
// slot blocks at a time, the next k-step's fragments requested while the
// current one's MFMAs run.  Products, their order and the epilogue are
// those of k_recon_bf16, so the results are bitwise the same.  EXACT: the
// basis takes all KSMAX k-steps, so no step's loads sit behind a run-time
// test (a load on one path only makes the next MFMA wait for every load
// issued after it, the next step's prefetch included).
template <int KSMAX, int CB, bool EXACT>
__global__ __launch_bounds__(512, 1) void k_recon_bf16_x2(const bf16x8 *psi_hi, const bf16x8 *psi_lo,
                                                          const double *sig_t, const bf16x8 *ub_hi,
                                                          const bf16x8 *ub_lo, const int32_t *perm,
                                                          const ReconJob *jobs, int n_jobs, int v_begin, int n_v,
                                                          int chunk, int nks, int n_elem, int n_eblk) {
    constexpr int NW = 8;
    if (EXACT) nks = KSMAX;
    __shared__ bf16x8 lds[2][2][6][KSMAX][64];
    __shared__ double st_lds[32][6];
    const int eb0 = 2 * (int)blockIdx.x;
    const int neb = min(2, n_eblk - eb0);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int y0 = v_begin + (int)blockIdx.y * chunk, y1 = min(y0 + chunk, v_begin + n_v);
    {
        const bf16x8 *gh = psi_hi + (size_t)eb0 * 6 * nks * 64;
        const bf16x8 *gl = psi_lo + (size_t)eb0 * 6 * nks * 64;
        const int per = 6 * nks * 64;
        for (int i = threadIdx.x; i < neb * per; i += 64 * NW) {
            const int b = i / per, c = (i % per) / (nks * 64), r = i % (nks * 64);
            lds[b][0][c][r / 64][r % 64] = gh[i];
            lds[b][1][c][r / 64][r % 64] = gl[i];
        }
        if (threadIdx.x < 192) {
            const int e = min(eb0 * 16 + (int)threadIdx.x / 6, n_elem - 1);
            st_lds[threadIdx.x / 6][threadIdx.x % 6] = sig_t[(size_t)e * 6 + threadIdx.x % 6];
        }
    }
    __syncthreads();
    int j = 0;  // job of the wave's current block (blocks only move forward)
    for (int base = y0 + wave * CB; base < y1; base += NW * CB) {
        double dTv[CB];
        global_ptr<float> vmv[CB], s6v[CB];
        int cellv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int v = min(base + cb, y1 - 1);
            while (j + 1 < n_jobs && v >= jobs[j + 1].sb_off) ++j;
            const ReconJob &J = jobs[j];
            dTv[cb] = J.dT;
            vmv[cb] = to_global(static_cast<float *>(J.vm));
            s6v[cb] = to_global(static_cast<float *>(J.sig6));
            cellv[cb] = perm[(size_t)(J.sb_first + (v - J.sb_off)) * 16 + lane % 16];
        }
        f32x4 acc[2][CB][6];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[b][cb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        // Past the slice end a wave rereads the last valid block (results unused).
        size_t fb[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) fb[cb] = (size_t)min(base + cb, y1 - 1) * nks * 64 + lane;
        bf16x8 bh[CB], bl[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            bh[cb] = ub_hi[fb[cb]];
            bl[cb] = ub_lo[fb[cb]];
        }
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            if (ks < nks) {
                bf16x8 nh[CB], nl[CB];
                if (ks + 1 < nks) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        nh[cb] = ub_hi[fb[cb] + (size_t)(ks + 1) * 64];
                        nl[cb] = ub_lo[fb[cb] + (size_t)(ks + 1) * 64];
                    }
                }
                // The next step's loads stay ahead of this step's MFMAs.
                if (EXACT) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        const bf16x8 ah = lds[b][0][c][ks][lane], al = lds[b][1][c][ks][lane];
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            acc[b][cb][c] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], acc[b][cb][c], 0, 0, 0);
                            acc[b][cb][c] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], acc[b][cb][c], 0, 0, 0);
                            acc[b][cb][c] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], acc[b][cb][c], 0, 0, 0);
                        }
                    }
                }
                if (ks + 1 < nks) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        bh[cb] = nh[cb];
                        bl[cb] = nl[cb];
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (b >= neb) continue;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if (base + cb >= y1) continue;
                const double dT = dTv[cb];
                global_ptr<float> vm = vmv[cb], sig6 = s6v[cb];
                const int cell = cellv[cb];
                if (cell < 0) continue;
                const int e0 = (eb0 + b) * 16 + 4 * (lane / 16);
                float vq[4], sq[4][6];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int c = 0; c < 6; ++c)
                        sq[q][c] = acc[b][cb][c][q] + (float)(dT * st_lds[b * 16 + 4 * (lane / 16) + q][c]);
                    const float x = sq[q][0] - sq[q][1], y = sq[q][1] - sq[q][2], d = sq[q][2] - sq[q][0];
                    vq[q] = sqrtf(0.5f * (x * x + y * y + d * d) +
                                  3.0f * (sq[q][3] * sq[q][3] + sq[q][4] * sq[q][4] + sq[q][5] * sq[q][5]));
                }
                const size_t o = (size_t)cell * n_elem + e0;
                const bool whole = e0 + 3 < n_elem && o % 4 == 0;
                if (vm) {
                    if (whole) {
                        *(global_ptr<f32x4>)(vm + o) = f32x4{vq[0], vq[1], vq[2], vq[3]};
                    } else {
                        for (int q = 0; q < 4; ++q)
                            if (e0 + q < n_elem) vm[o + q] = vq[q];
                    }
                }
                if (sig6) {
                    for (int q = 0; q < 4; ++q)
                        if (e0 + q < n_elem)
                            for (int c = 0; c < 6; ++c) sig6[(o + q) * 6 + c] = sq[q][c];
                }
            }
        }
    }
}

}  // namespace

int recon_f64_variant();
int recon_bf16_variant();

mos_status recon_f64_jobs(mos_ctx ctx, const mos_rom *roms, int n_types, const std::vector<ReconJob> *jobs,
                          ReconJob *dev_jobs, ReconJob *host_jobs, const double *U, int ld, const int32_t *perm,
                          bool fp32_out) {
    if (n_types < 1 || n_types > MAX_TYPES) return MOS_EINVAL;
    const mos_rom r = roms[0];
    const int ks = r->ldk / 4;
    if (ks > RECON_F64_LDS_KS) return MOS_EINVAL;
    hipStream_t st = ctx->stream;
    // One table upload for all types: type t's jobs at [first[t], first[t+1]).
    std::vector<int> first(n_types + 1, 0);
    for (int t = 0; t < n_types; ++t) first[t + 1] = first[t] + (int)jobs[t].size();
    if (first[n_types] == 0) return MOS_OK;
    for (int t = 0; t < n_types; ++t)
        for (size_t i = 0; i < jobs[t].size(); ++i) host_jobs[first[t] + i] = jobs[t][i];
    MOS_HIP(hipMemcpyAsync(dev_jobs, host_jobs, first[n_types] * sizeof(ReconJob), hipMemcpyHostToDevice, st));
    for (int t = 0; t < n_types; ++t) {
        const int nj = (int)jobs[t].size();
        if (nj == 0) continue;
        const int total = jobs[t].back().sb_off + jobs[t].back().n_sb;
        // Slices give >= ~512 workgroups (one per CU at a time: 135 KB of
        // LDS) while each slice still streams >= 16 slot blocks.
        const int ny = std::max(1, std::min(total / 16, ceil_div(512, r->n_eblk)));
        const int chunk = ceil_div(total, ny);
        const dim3 grid(r->n_eblk, ceil_div(total, chunk));
        const double *psi = roms[t]->psi, *sgt = roms[t]->sig_t;
        const ReconJob *dj = dev_jobs + first[t];
        // A basis of 168 (the benchmark cells) needs 42 of the 44 k-steps.
        const bool ks42 = ks == RECON_F64_LDS_KS && ceil_div(r->n, 4) == 42;
        if (ks42 && !fp32_out && recon_f64_variant() == 2)
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_pipe<double, 42, 6, 4 * RECON_F64_LDS_KS>, grid, dim3(512), 0,
                         st, psi, sgt, U, perm, ld, dj, nj, total, chunk, r->n_elem);
        else if (ks == RECON_F64_LDS_KS && !fp32_out && recon_f64_variant() == 2)
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_pipe<double, RECON_F64_LDS_KS, 11>, grid, dim3(512), 0, st,
                         psi, sgt, U, perm, ld, dj, nj, total, chunk, r->n_elem);
        else if (ks == RECON_F64_LDS_KS && fp32_out && recon_f64_variant() == 2)
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_pipe<float, RECON_F64_LDS_KS, 11>, grid, dim3(512), 0, st,
                         psi, sgt, U, perm, ld, dj, nj, total, chunk, r->n_elem);
        else if (ks == RECON_F64_LDS_KS && !fp32_out)
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_lds<double, RECON_F64_LDS_KS, true>, grid, dim3(512), 0, st, psi,
                         sgt, U, perm, ld, dj, nj, total, chunk, ks, r->n_elem);
        else if (!fp32_out)
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_lds<double, RECON_F64_LDS_KS, false>, grid, dim3(512), 0, st,
                         psi, sgt, U, perm, ld, dj, nj, total, chunk, ks, r->n_elem);
        else if (ks == RECON_F64_LDS_KS)
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_lds<float, RECON_F64_LDS_KS, true>, grid, dim3(512), 0, st, psi,
                         sgt, U, perm, ld, dj, nj, total, chunk, ks, r->n_elem);
        else
            launch_timed(ctx, MOS_K_RECON, k_recon_f64_lds<float, RECON_F64_LDS_KS, false>, grid, dim3(512), 0, st,
                         psi, sgt, U, perm, ld, dj, nj, total, chunk, ks, r->n_elem);
        MOS_LAUNCH_CHECK();
    }
    return MOS_OK;
}

int64_t recon_bf16_scratch(const mos_rom r, int n_sb) { return (int64_t)n_sb * r->nks * 64 * 2 * 16; }

// FP64 reconstruction kernel for bases of exactly 176 (44 k-steps): 2 = the
// chunked, double-buffered operand stream (default), 1 = the whole block's
// operand requested at once.  Both give the same bits; MOS_RECON_F64=1 in the
// environment at the time of the call selects the second (for comparisons).
int recon_f64_variant() {
    const char *e = std::getenv("MOS_RECON_F64");
    return (e && std::atoi(e) == 1) ? 1 : 2;
}

// BF16-split reconstruction kernel for bases up to 192 (nks <= 6): 2 = two
// element blocks per workgroup (default), 1 = one.  Both give the same bits;
// MOS_RECON_BF16=1 in the environment at the time of the call selects the
// second (for comparisons).
int recon_bf16_variant() {
    const char *e = std::getenv("MOS_RECON_BF16");
    return (e && std::atoi(e) == 1) ? 1 : 2;
}

mos_status recon_bf16_jobs(mos_ctx ctx, const mos_rom *roms, int n_types, const std::vector<ReconJob> *jobs,
                           ReconJob *dev_jobs, ReconJob *host_jobs, const double *U, int ld, const int32_t *perm,
                           void *split) {
    if (n_types < 1 || n_types > MAX_TYPES) return MOS_EINVAL;
    const mos_rom r = roms[0];
    for (int t = 0; t < n_types; ++t)
        if (!roms[t]->psi_hi || roms[t]->nks != r->nks || roms[t]->n_eblk != r->n_eblk) return MOS_EINVAL;
    hipStream_t st = ctx->stream;
    // One table for all types, flattened slot blocks numbered type-major:
    // type t's jobs at [first[t], first[t + 1]), its blocks at
    // [vbase[t], vbase[t + 1]).
    std::vector<int> first(n_types + 1, 0), vbase(n_types + 1, 0);
    for (int t = 0; t < n_types; ++t) {
        first[t + 1] = first[t] + (int)jobs[t].size();
        const int nt = jobs[t].empty() ? 0 : jobs[t].back().sb_off + jobs[t].back().n_sb;
        vbase[t + 1] = vbase[t] + nt;
    }
    const int total = vbase[n_types];
    if (total == 0) return MOS_OK;
    for (int t = 0; t < n_types; ++t)
        for (size_t i = 0; i < jobs[t].size(); ++i) {
            host_jobs[first[t] + i] = jobs[t][i];
            host_jobs[first[t] + i].sb_off += vbase[t];
        }
    MOS_HIP(hipMemcpyAsync(dev_jobs, host_jobs, first[n_types] * sizeof(ReconJob), hipMemcpyHostToDevice, st));
    bf16x8 *ub_hi = (bf16x8 *)split, *ub_lo = ub_hi + (size_t)total * r->nks * 64;
    const int64_t nfrag = (int64_t)total * r->nks * 64;
    hipLaunchKernelGGL(k_split_u, dim3(ceil_div(nfrag, 256)), dim3(256), 0, st, U, ld, (const ReconJob *)dev_jobs,
                       first[n_types], total, r->ldk, r->nks, ub_hi, ub_lo);
    MOS_LAUNCH_CHECK();
    for (int t = 0; t < n_types; ++t) {
        const int n_v = vbase[t + 1] - vbase[t];
        if (n_v <= 0) continue;
        // Slices of the type's blocks give >= ~2048 workgroups for large
        // batches while each slice still streams >= 32 slot blocks per
        // staged block of Psi.
        const int ny = std::max(1, std::min(n_v / 32, ceil_div(2048, r->n_eblk)));
        const int chunk = ceil_div(n_v, ny);
        const dim3 grid(r->n_eblk, ceil_div(n_v, chunk));
        const bf16x8 *ph = (const bf16x8 *)roms[t]->psi_hi, *pl = (const bf16x8 *)roms[t]->psi_lo;
        const ReconJob *dj = dev_jobs + first[t];
        const int nj = first[t + 1] - first[t];
        if (r->nks <= 6 && recon_bf16_variant() == 2) {
            // Two element blocks per workgroup, one workgroup per CU: slices
            // give >= ~512 workgroups while each still streams >= 32 blocks.
            const int nx2 = ceil_div(r->n_eblk, 2);
            const int ny2 = std::max(1, std::min(n_v / 32, ceil_div(512, nx2)));
            const int chunk2 = ceil_div(n_v, ny2);
            auto kern = r->nks == 6 ? k_recon_bf16_x2<6, 2, true> : k_recon_bf16_x2<6, 2, false>;
            launch_timed(ctx, MOS_K_RECON, kern, dim3(nx2, ceil_div(n_v, chunk2)), dim3(512), 0, st, ph, pl,
                         (const double *)roms[t]->sig_t, (const bf16x8 *)ub_hi, (const bf16x8 *)ub_lo, perm, dj, nj,
                         vbase[t], n_v, chunk2, r->nks, r->n_elem, r->n_eblk);
        } else if (r->nks <= 6)
            launch_timed(ctx, MOS_K_RECON, k_recon_bf16<6, 4>, grid, dim3(256), 0, st, ph, pl,
                         (const double *)roms[t]->sig_t, (const bf16x8 *)ub_hi, (const bf16x8 *)ub_lo, perm, dj, nj,
                         vbase[t], n_v, chunk, r->nks, r->n_elem);
        else
            launch_timed(ctx, MOS_K_RECON, k_recon_bf16<RECON_BF16_MAX_KS, 2>, grid, dim3(256), 0, st, ph, pl,
                         (const double *)roms[t]->sig_t, (const bf16x8 *)ub_hi, (const bf16x8 *)ub_lo, perm, dj, nj,
                         vbase[t], n_v, chunk, r->nks, r->n_elem);
        MOS_LAUNCH_CHECK();
    }
    return MOS_OK;
}

// Fine-mesh displacement of every cell (eq. 15): out[cell][d] = dT f_T[d] +
// sum_k Phi[d][k] u_cell[k] for the FE DoFs d of one cell type's block
// (f_T is column n of the stored Phi).  FP64 MFMA 16x16x4 with the cells as
// rows and the DoFs as columns, so the 16 lanes of a register's row hold 16
// consecutive DoFs of one cell (128-byte segments of the output).  Each wave
// owns a tile of 16 DoFs, keeps that tile of Phi (ldk columns, KS k-steps of
// 4; columns n..ldk-1 meet zero rows of U) in registers, and streams up to
// `chunk` slot blocks of the type's slots [s0, s0 + 16 n_sb).
// KS > 0: the wave's tile of Phi stays in registers (ks <= KS k-steps);
// KS == 0: any basis size, the tile read again for every slot block.
template <int KS>
__global__ __launch_bounds__(256) void k_nodal_u(const double *phi, int ldp, int n, int n_dofs, int ks,
                                                 const double *U, int n_pc, const int32_t *perm, int s0, int n_sb,
                                                 int chunk, double dT, double *out) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int d0 = (blockIdx.x * 4 + wave) * 16;
    if (d0 >= n_dofs) return;
    const int dcol = d0 + lane % 16;
    const bool dval = dcol < n_dofs;
    // B[k][dof] = Phi[dof][k]: lane l holds k = 4 s + l / 16 of DoF d0 + l % 16.
    constexpr int NB = KS > 0 ? KS : 1;
    double b[NB];
#pragma unroll
    for (int s = 0; s < NB; ++s)
        b[s] = (KS > 0 && s < ks && dval) ? phi[(size_t)dcol * ldp + 4 * s + lane / 16] : 0.0;
    const double *prow = phi + (size_t)(dval ? dcol : 0) * ldp + lane / 16;
    const double ft = dval ? dT * phi[(size_t)dcol * ldp + n] : 0.0;
    const int sb0 = blockIdx.y * chunk, sb1 = min(sb0 + chunk, n_sb);
    for (int sb = sb0; sb < sb1; ++sb) {
        const int pc0 = s0 + sb * 16;
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        if (KS > 0) {
#pragma unroll
            for (int s = 0; s < NB; ++s)
                if (s < ks) {
                    // A[cell][k] = U[k][slot]: lane l holds slot pc0 + l % 16, k = 4 s + l / 16.
                    const double a = U[(size_t)(4 * s + lane / 16) * n_pc + pc0 + lane % 16];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[s], acc, 0, 0, 0);
                }
        } else {
            for (int s = 0; s < ks; ++s) {
                const double a = U[(size_t)(4 * s + lane / 16) * n_pc + pc0 + lane % 16];
                const double bv = dval ? prow[4 * s] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cell = perm[pc0 + lane / 16 + 4 * q];   // output row of register q
            if (cell >= 0 && dval) out[(size_t)cell * n_dofs + dcol] = ft + acc[q];
        }
    }
}

// Scratch of the allocation-free reconstruction (mos_reconstruct_noalloc):
// the job table, the cell-major gather of u and, in the mixed path, its BF16
// split.  Each device holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives for the
// current device (noalloc_scratch_init), never through the symbol itself.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

mos_status noalloc_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device %d beyond the %d devices the scratch table holds", device, MAX_DEVICES);
        return MOS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return MOS_OK;
    void *p = nullptr;
    MOS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = p;
    return MOS_OK;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

namespace {
// Device bytes recon_with takes for its job table, the gather of u and (mixed)
// the BF16 split, each rounded to 256.
size_t recon_workspace(mos_sol s, const std::vector<mos_rom> &R, size_t *off_u, size_t *off_split) {
    const size_t jobs = round_up((int64_t)(MAX_TYPES * sizeof(ReconJob)), 256);
    const size_t u = round_up((int64_t)s->ldk * s->n_pc * (int64_t)sizeof(double), 256);
    const bool split = s->precision == MOS_MIXED && R[0]->psi_hi;
    const size_t b = split ? (size_t)round_up(recon_bf16_scratch(R[0], s->n_pc / 16), 256) : 0;
    *off_u = jobs;
    *off_split = jobs + u;
    return jobs + u + b;
}
}  // namespace

// The solution's cells through the stress bases R[t] (one per cell type:
// the centroid bases of the solution's ROMs, or their plane bases), which
// share ldk, n_eblk and n_elem (output points per cell).  Device scratch
// comes from `ws` (ws_bytes long, nothing allocated) when it is given, else
// from the context's allocator for the duration of the call.
static mos_status recon_with(mos_ctx ctx, mos_sol s, const std::vector<mos_rom> &R, void *v, void *g,
                             void *ws = nullptr, size_t ws_bytes = 0) {
    hipStream_t st = ctx->stream;
    const int n_eblk = R[0]->n_eblk, n_pts = R[0]->n_elem;
    ReconTable tt{};
    tt.n_types = s->n_types;
    for (int t = 0; t <= s->n_types; ++t) tt.seg[t] = s->seg[t];
    for (int t = 0; t < s->n_types; ++t) {
        tt.psi[t] = R[t]->psi;
        tt.sig_t[t] = R[t]->sig_t;
    }
    DeviceArena tmp;
    tmp.ctx = ctx;
    struct Guard {
        DeviceArena &a;
        ~Guard() { a.release(); }
    } guard{tmp};
    size_t off_u = 0, off_split = 0;
    const size_t need = recon_workspace(s, R, &off_u, &off_split);
    char *base = static_cast<char *>(ws);
    if (ws) {
        if (need > ws_bytes) {
            set_error("reconstruction of %d cell slots needs %zu bytes of scratch; the allocation-free entry point "
                      "holds %zu",
                      s->n_pc, need, ws_bytes);
            return MOS_EINVAL;
        }
    } else {
        void *p = nullptr;
        MOS_TRY(tmp.alloc(need, &p));
        base = static_cast<char *>(p);
    }
    ReconJob *dj = reinterpret_cast<ReconJob *>(base);
    double *U = reinterpret_cast<double *>(base + off_u);
    // Host copy of the job table: pinned memory of the context (the call
    // waits for the stream before it returns, so the buffer is free again).
    ReconJob *hj = reinterpret_cast<ReconJob *>(static_cast<char *>(ctx->pinned) + 2048);
    static_assert(MAX_TYPES * sizeof(ReconJob) <= 2048, "job table exceeds the pinned buffer");
    const int64_t total = (int64_t)s->ldk * s->n_pc;
    hipLaunchKernelGGL(k_gather_u, dim3(ceil_div(total, 256)), dim3(256), 0, st, s->u, s->gidx, U, total);
    MOS_LAUNCH_CHECK();
    dim3 grid(n_eblk, ceil_div(s->n_pc / 16, 4));
    if (s->precision == MOS_MIXED && R[0]->psi_hi) {
        std::vector<std::vector<ReconJob>> jobs(s->n_types);
        for (int t = 0; t < s->n_types; ++t) {
            const int nsb = (s->seg[t + 1] - s->seg[t]) / 16;
            if (nsb > 0) jobs[t].push_back(ReconJob{s->seg[t] / 16, 0, nsb, 0, s->delta_T, v, g});
        }
        MOS_TRY(recon_bf16_jobs(ctx, R.data(), s->n_types, jobs.data(), dj, hj, U, s->n_pc, s->perm,
                                base + off_split));
        MOS_HIP(hipStreamSynchronize(st));  // the host job table is reused by the next call
    } else if (s->ldk / 4 <= RECON_F64_LDS_KS) {
        std::vector<std::vector<ReconJob>> jobs(s->n_types);
        for (int t = 0; t < s->n_types; ++t) {
            const int nsb = (s->seg[t + 1] - s->seg[t]) / 16;
            if (nsb > 0) jobs[t].push_back(ReconJob{s->seg[t] / 16, 0, nsb, 0, s->delta_T, v, g});
        }
        MOS_TRY(recon_f64_jobs(ctx, R.data(), s->n_types, jobs.data(), dj, hj, U, s->n_pc, s->perm,
                               s->precision != MOS_FP64));
        MOS_HIP(hipStreamSynchronize(st));  // the host job table is reused by the next call
    } else if (s->precision == MOS_FP64)
        launch_timed(ctx, MOS_K_RECON, k_recon_f64<double>, grid, dim3(256), 0, st, tt, (const double *)U,
                     (const int32_t *)s->perm, s->n_pc, s->ldk, n_pts, s->delta_T, (double *)v, (double *)g);
    else
        launch_timed(ctx, MOS_K_RECON, k_recon_f64<float>, grid, dim3(256), 0, st, tt, (const double *)U,
                     (const int32_t *)s->perm, s->n_pc, s->ldk, n_pts, s->delta_T, (float *)v, (float *)g);
    MOS_LAUNCH_CHECK();
    MOS_HIP(hipStreamSynchronize(st));
    return MOS_OK;
}

mos_status reconstruct(mos_ctx ctx, mos_sol s, uint32_t outputs, void *vm, void *sigma6) {
    return recon_with(ctx, s, s->roms, (outputs & MOS_OUT_VM) ? vm : nullptr,
                      (outputs & MOS_OUT_SIGMA6) ? sigma6 : nullptr);
}

mos_status reconstruct_noalloc(mos_ctx ctx, mos_sol s, uint32_t outputs, void *vm, void *sigma6) {
    void *ws = noalloc_scratch(ctx->device);
    if (!ws) {
        set_error("the allocation-free scratch of device %d is not set up", ctx->device);
        return MOS_EHIP;
    }
    return recon_with(ctx, s, s->roms, (outputs & MOS_OUT_VM) ? vm : nullptr,
                      (outputs & MOS_OUT_SIGMA6) ? sigma6 : nullptr, ws, NOALLOC_SCRATCH_BYTES);
}

mos_status reconstruct_displacement(mos_ctx ctx, mos_sol s, double *u_nodal) {
    hipStream_t st = ctx->stream;
    const int ks = s->ldk / 4;
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
    for (int t = 0; t < s->n_types; ++t) {
        const mos_rom r = s->roms[t];
        const int n_sb = (s->seg[t + 1] - s->seg[t]) / 16;
        if (n_sb <= 0) continue;
        // Up to 8 slot blocks per wave, enough workgroups to fill the chip.
        const int n_dt = ceil_div(r->n_dofs, 64);
        const int chunk = std::max(1, std::min(8, n_sb * n_dt / 2048));
        const dim3 grid(n_dt, ceil_div(n_sb, chunk));
        if (ks <= RECON_F64_LDS_KS)
            hipLaunchKernelGGL(k_nodal_u<RECON_F64_LDS_KS>, grid, dim3(256), 0, st, (const double *)r->phi, r->ldp,
                               r->n, r->n_dofs, ks, (const double *)U, s->n_pc, (const int32_t *)s->perm, s->seg[t],
                               n_sb, chunk, s->delta_T, u_nodal);
        else
            hipLaunchKernelGGL(k_nodal_u<0>, grid, dim3(256), 0, st, (const double *)r->phi, r->ldp, r->n, r->n_dofs,
                               ks, (const double *)U, s->n_pc, (const int32_t *)s->perm, s->seg[t], n_sb, chunk,
                               s->delta_T, u_nodal);
        MOS_LAUNCH_CHECK();
    }
    MOS_HIP(hipStreamSynchronize(st));
    return MOS_OK;
}

mos_status reconstruct_plane(mos_ctx ctx, mos_sol s, int grid, void *vm) {
    std::vector<mos_rom> R(s->n_types);
    for (int t = 0; t < s->n_types; ++t) {
        MOS_TRY(plane_basis(s->roms[t], grid));
        R[t] = s->roms[t]->plane;
    }
    return recon_with(ctx, s, R, vm, nullptr);
}

}  // namespace mos
