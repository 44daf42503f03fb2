// Global stage for many arrays at once (Sec. 4.3-4.4, eq. 20).
//
// An engine owns capacity-sized device arenas.  Every admitted problem (one
// array: its own size, cell types, dT and constraints) gets a block-aligned
// range of DoFs (blocks of 256) and a range of cell slots (blocks of 16,
// one cell type per slot block) and keeps them for its lifetime.  The reduced
// operator is applied element by element: a per-slot-block GEMM with the
// shared K_r of the block's cell type (MFMA), then a node-centric sum over the
// <= 4 cells around each DoF in ascending cell order.  Pipelined Jacobi-PCG
// (one fused reduction per iteration) advances all iterating problems with
// two batch-wide launches per iteration; the extra blocks of the GEMM launch
// reduce each problem's dot-product partials in a fixed order and publish its
// step, so a problem's result does not depend on what else is in the batch.
// Between iteration chunks the host admits queued problems, checks the FP64
// true residual of problems whose inner solve stopped (iterative refinement:
// FP64 inner solves for MOS_FP64, FP32 for MOS_MIXED), restarts or retires
// them, and reconstructs finished ones.
#include <algorithm>
#include <cstring>
#include <cmath>
#include <deque>
#include <map>
#include <vector>

#include "engine.h"
#include "mesh.h"
#include "mos_internal.h"
#include "gmem.h"
#include "waitcnt.h"

namespace mos {
namespace {

constexpr int DB = 256;       // DoFs per DoF block
constexpr int N_XCD = 8;      // accelerator dies that workgroups are dealt to in turn
constexpr int DOF_ALIGN = 3 * DB;
// Two-level preconditioner: aggregates of AGG_C x AGG_C cells, boxes of
// at most BOX_CX x AGG_C cells (at most MAXA aggregates per box; narrower
// when a box of BOX_CX cells would exceed one workgroup's 1024 nodes).
constexpr int AGG_C = 2;
constexpr int BOX_CX = 6;
constexpr int MAXA = (BOX_CX + AGG_C - 1) / AGG_C;

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

// Fixed-order sums over partial[begin, end) of up to three arrays; every lane
// of the calling wave gets the result.
__device__ __forceinline__ void wave_sum3(const double *pa, const double *pb, const double *pc, int begin, int end,
                                          double &a, double &b, double &c) {
    a = b = c = 0.0;
    const int lane = threadIdx.x % 64;
    for (int i = begin + lane; i < end; i += 64) {
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

__device__ __forceinline__ bool selected(const ProbSel &S, int p) {
    return p >= 0 && ((S.bits[p >> 5] >> (p & 31)) & 1u);
}

// Scalars of iteration `it` of one problem, computed by one workgroup
// (Chronopoulos-Gear form of PCG: one fused reduction per iteration).
// Fixed-order sums -- each thread a fixed strided subset, then a fixed
// butterfly per wave and the waves in order -- of the problem's partials: gamma = (r,u) and rho = (r,r) per DoF block
// from the last update, delta = (u, A u) per (row block, slot block) tile
// from this iteration's cell GEMM.  Then the stop decision (1 converged,
// 2 breakdown, 3 iteration cap) or the step (alpha, beta).  Every workgroup
// that evaluates it for the same problem and iteration gets the same bits.
struct CgStep {
    int stop;
    double alpha, beta, gamma, rr, tol2;
};

constexpr int CG_LW = 256;  // logical width of the scalar reduction

// The step of iteration it from the sums (r,u), (r,r) and (u,A u): stop
// when (r,r) reaches the sweep's tolerance or the iteration cap, else alpha
// and beta of the Chronopoulos-Gear recurrence (breakdown stops with code 2).
__device__ CgStep cg_step(const ProbState &S, int it, double gamma, double rr, double delta) {
    CgStep o;
    o.gamma = gamma;
    o.rr = rr;
    o.tol2 = it == S.seg_start ? S.rtol2 * o.rr : S.tol2;
    o.stop = 0;
    o.alpha = o.beta = 0.0;
    if (o.rr <= o.tol2) {
        o.stop = 1;
    } else if (it - S.seg_start >= S.max_iter) {
        o.stop = 3;
    } else {
        if (it == 0) {
            o.alpha = o.gamma / delta;
        } else {
            const int pv = (it - 1) & 1;
            o.beta = o.gamma / S.hist_gamma[pv];
            o.alpha = o.gamma / (delta - o.beta * o.gamma / S.hist_alpha[pv]);
        }
        if (!(o.alpha > 0.0) || !isfinite(o.alpha) || !isfinite(o.beta)) o.stop = 2;
    }
    return o;
}

template <int NT>
__device__ CgStep cg_scalars_block(const ProbState &S, int it, const double *pg, const double *pr,
                                   const double *pdel, double (*red)[NT]) {
    static_assert(NT == CG_LW || 2 * NT == CG_LW, "one or two logical lanes per thread");
    // Logical lane L sums the partials L, L + CG_LW, ...; a thread holding
    // two lanes (t and t + NT) adds them as the first level of the tree
    // would, so the result has the same bits for either workgroup size.
    double g = 0.0, r = 0.0, dl = 0.0;
#pragma unroll
    for (int h = 0; h < CG_LW / NT; ++h) {
        const int L = threadIdx.x + h * NT;
        double gh = 0.0, rh = 0.0, dh = 0.0;
#pragma unroll 4
        for (int i = S.blk_begin + L; i < S.blk_end; i += CG_LW) {
            gh += pg[i];
            rh += pr[i];
        }
#pragma unroll 4
        for (int i = S.tile_begin + L; i < S.tile_end; i += CG_LW) dh += pdel[i];
        if (h == 0) {
            g = gh;
            r = rh;
            dl = dh;
        } else {
            g += gh;
            r += rh;
            dl += dh;
        }
    }
    red[0][threadIdx.x] = g;
    red[1][threadIdx.x] = r;
    red[2][threadIdx.x] = dl;
    __syncthreads();
    for (int m = NT / 2; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m)
            for (int j = 0; j < 3; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + m];
        __syncthreads();
    }
    CgStep o;
    o.gamma = red[0][0];
    o.rr = red[1][0];
    const double delta = red[2][0];
    o.tol2 = it == S.seg_start ? S.rtol2 * o.rr : S.tol2;
    o.stop = 0;
    o.alpha = o.beta = 0.0;
    if (o.rr <= o.tol2) {
        o.stop = 1;
    } else if (it - S.seg_start >= S.max_iter) {
        o.stop = 3;
    } else {
        if (it == 0) {
            o.alpha = o.gamma / delta;
        } else {
            const int pv = (it - 1) & 1;
            o.beta = o.gamma / S.hist_gamma[pv];
            o.alpha = o.gamma / (delta - o.beta * o.gamma / S.hist_alpha[pv]);
        }
        if (!(o.alpha > 0.0) || !isfinite(o.alpha) || !isfinite(o.beta)) o.stop = 2;
    }
    return o;
}

// Publish iteration `it`'s outcome (one writer per problem and iteration).
// Readers of the same launch only read the other history slot.  The steps
// of the problem's first sweep (up to LZ_MAX) also go to its row lz of the
// Lanczos record, (alpha, beta) per step.
__device__ __forceinline__ void cg_publish(ProbState &S, int it, const CgStep &o, double *lz) {
    S.rr = o.rr;
    if (it == S.seg_start) S.tol2 = o.tol2;
    if (o.stop) {
        S.done = o.stop;
    } else {
        S.a_cur = o.alpha;
        S.b_cur = o.beta;
        S.hist_gamma[it & 1] = o.gamma;
        S.hist_alpha[it & 1] = o.alpha;
        S.it = it + 1;
        if (lz && S.seg_start == 0 && it < LZ_MAX) {
            lz[2 * it] = o.alpha;
            lz[2 * it + 1] = o.beta;
        }
    }
}

// Row of problem pid in the Lanczos record (null: none kept).
__device__ __forceinline__ double *lz_row(double *lz, int pid) {
    return lz ? lz + (size_t)pid * LZ_MAX * 2 : nullptr;
}

// Separate scalar launch for problems too large to reduce in every update
// workgroup: one workgroup per problem, iteration launch ep[0] + j (the
// chunk's first epoch, set on the device, plus the launch's place in the
// chunk, so a captured chunk replays with the epochs of its replay).  The
// per-block partials are double-buffered by iteration parity: iteration it
// reads slot it & 1 (written by the previous update or the sweep start).
// Such a problem has tens of thousands of partials, so the workgroup is
// wide (CG_BIG lanes, each with several loads in flight); lane L sums
// partials L, L + CG_BIG, ..., then a butterfly per wave and the waves' sums
// in order.  Only problems above the fused size come here, so their scalars
// always take this order.
constexpr int CG_BIG = 1024;
__global__ __launch_bounds__(CG_BIG) void k_cg_scalars(ProbState *ps, const double *pg, const double *pr,
                                                       const double *pdel, const int *ep, int j, int cap_blk,
                                                       double *lz) {
    __shared__ double red[3][CG_BIG / 64];
    const int epoch = ep[0] + j;
    ProbState &S = ps[blockIdx.x];
    const int active = S.active, done = S.done, fused = S.fused;  // one round trip
    if (!((active != 0) & (done == 0) & (fused == 0))) return;     // uniform over the workgroup
    const int it = epoch - S.start_epoch;
    const size_t slot = (size_t)(it & 1) * cap_blk;
    const double *g = pg + slot, *r = pr + slot;
    const int t = threadIdx.x;
    double gs = 0.0, rs = 0.0, ds = 0.0;
#pragma unroll 8
    for (int i = S.blk_begin + t; i < S.blk_end; i += CG_BIG) {
        gs += g[i];
        rs += r[i];
    }
#pragma unroll 8
    for (int i = S.tile_begin + t; i < S.tile_end; i += CG_BIG) ds += pdel[i];
    for (int m = 32; m >= 1; m >>= 1) {
        gs += __shfl_xor(gs, m);
        rs += __shfl_xor(rs, m);
        ds += __shfl_xor(ds, m);
    }
    if (t % 64 == 0) {
        red[0][t / 64] = gs;
        red[1][t / 64] = rs;
        red[2][t / 64] = ds;
    }
    __syncthreads();
    if (t != 0) return;
    double sum[3];
    for (int q = 0; q < 3; ++q) {
        sum[q] = red[q][0];
        for (int w = 1; w < CG_BIG / 64; ++w) sum[q] += red[q][w];
    }
    cg_publish(S, it, cg_step(S, it, sum[0], sum[1], sum[2]), lz_row(lz, (int)blockIdx.x));
}

// (u, A u) over one 16x16 output tile: the tile's products times the cell
// operand at the same positions, summed over the wave in a fixed order
// (padding slots hold zeros in the cell layout, so they add nothing).
template <class T, class V4>
__device__ __forceinline__ double tile_dot(const V4 &acc, const T *Mc, int ld_slots, int rb, int col, int lane) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        t += (double)acc[q] * (double)Mc[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * ld_slots + col];
    for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m);
    return t;
}

constexpr int GEMM_WAVES = 4;       // split-K ways of the cell GEMM
constexpr int GEMM_MAX_STEPS = 16;  // k-steps of 4 whose loads are issued together

// Y[k][slot] = sum_j K_r[j][k] Mc[j][slot] for one 16 x 16 tile per workgroup
// (K_r symmetric), K split over four waves summed in a fixed order through
// LDS.  Slot blocks [sb_base, sb_base + n_sb); with gate 1 the tile is
// skipped unless its problem is iterating, with gate 2 unless its problem is
// in `sel`.  With pdel, the tile's (u, A u) partial goes to
// pdel[slot block * row blocks + row block].
template <class T>
__global__ __launch_bounds__(256) void k_bgemm(const void *const *kr_tab, const int32_t *sb_rom, const int32_t *sb_prob,
                                               const T *Mc, T *Y, int ldk, int ld_slots, int sb_base, int n_sb,
                                               int gate, const ProbState *ps, double *pdel, ProbSel sel) {
    typedef typename Mfma<T>::v4 v4;
    __shared__ v4 red[GEMM_WAVES - 1][64];
    __shared__ int skip;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int sb = sb_base + (int)blockIdx.y;
    const int rom = sb_rom[sb];
    const int rb = blockIdx.x, pc0 = sb * 16;
    const int col = pc0 + lane % 16;
    const int steps = ldk / (4 * GEMM_WAVES);
    const int k_begin = wave * steps * 4;
    if (threadIdx.x == 0) {
        int sk = rom < 0;
        if (!sk && gate == 1) {
            const ProbState &S = ps[sb_prob[sb]];
            sk = !S.active || S.done;
        } else if (!sk && gate == 2) {
            sk = !selected(sel, sb_prob[sb]);
        }
        skip = sk;
    }
    __syncthreads();
    if (skip) return;
    global_ptr<const T> kr = to_global(static_cast<const T *>(kr_tab[rom]));
    global_ptr<const T> ap = kr + (size_t)(k_begin + lane / 16) * ldk + rb * 16 + lane % 16;
    const T *bp = Mc + (size_t)(k_begin + lane / 16) * ld_slots + col;
    v4 acc = {0, 0, 0, 0};
    for (int s0 = 0; s0 < steps; s0 += GEMM_MAX_STEPS) {
        const int cnt = min(GEMM_MAX_STEPS, steps - s0);
        T a[GEMM_MAX_STEPS], b[GEMM_MAX_STEPS];
#pragma unroll
        for (int j = 0; j < GEMM_MAX_STEPS; ++j)
            if (j < cnt) {
                a[j] = ap[(size_t)(4 * (s0 + j)) * ldk];
                b[j] = bp[(size_t)(4 * (s0 + j)) * ld_slots];
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
        for (int q = 0; q < 4; ++q) Y[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * ld_slots + col] = acc[q];
        if (pdel) {
            const double t = tile_dot<T>(acc, Mc, ld_slots, rb, col, lane);
            if (lane == 0) pdel[(size_t)sb * (ldk / 16) + rb] = t;
        }
    }
}

// Live slot blocks of the run [s_begin, s_end) (at most 64): each lane
// checks one (in use, and iterating with gate 1 or selected with gate 2) and
// the wave's ballot gives the mask, bit i for slot block s_begin + i; every
// wave of a workgroup computes the same mask.  Lane i keeps that block's
// cell type in *rom_lane.  Two dependent loads for the whole run, instead
// of a chain of scalar loads before every block.
__device__ __forceinline__ uint64_t run_mask(const int32_t *sb_rom, const int32_t *sb_prob, const ProbState *ps,
                                            int gate, const ProbSel &sel, int sb_base, int s_begin, int s_end,
                                            int *rom_lane) {
    const int lane = threadIdx.x % 64;
    const int sl = s_begin + lane;
    bool live = false;
    int rom = -1;
    if (sl < s_end) {
        rom = sb_rom[sb_base + sl];
        const int owner = sb_prob[sb_base + sl];
        live = rom >= 0;
        if (live && gate == 1) {
            const ProbState &S = ps[owner];
            const int active = S.active, done = S.done;
            live = (active != 0) & (done == 0);
        } else if (live && gate == 2) {
            live = selected(sel, owner);
        }
    }
    *rom_lane = rom;
    return __ballot(live);
}

// First live slot block at or after sl given the run's mask (s_end if none).
__device__ __forceinline__ int next_in_mask(uint64_t mask, int s_begin, int s_end, int sl) {
    const int off = sl - s_begin;
    if (off >= 64) return s_end;
    const uint64_t m = mask & (~0ull << off);
    return m ? s_begin + __builtin_ctzll(m) : s_end;
}

// (u, A u) over one 16x16 output tile from operand values already loaded
// (t[q] = the cell operand at output position q of the lane).
template <class T, class V4>
__device__ __forceinline__ double tile_dot_vals(const V4 &acc, const T (&t)[4]) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) v += (double)acc[q] * (double)t[q];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// K_r-stationary variant: one wave per (16-row block of K_r, run of `spw`
// consecutive slot blocks).  The wave keeps its 16 rows of K_r (KS k-steps
// of 4) in registers, reloading them only when the cell type changes.  In
// FP64 the slot blocks of the run are software-pipelined: while the chain of
// KS MFMAs of one slot block runs, each k-step's operand register is
// refilled with the next live slot block's value right after its MFMA has
// read it, so the next block's loads are in flight during this block's
// arithmetic.  Each
// 16x16 output is one MFMA chain in k order, so results do not depend on
// spw.  With pdel, each tile's (u, A u) partial goes to
// pdel[slot block * row blocks + row block].  (Staging a row block of K_r
// in LDS for a whole workgroup was measured slower at every batch size: the
// extra barrier and serial staging cost more than the occupancy it frees.)
template <class T, int KS, bool EXACT, int KK = KS>
__global__ __launch_bounds__(256) void k_bgemm_rows(const void *const *kr_tab, const int32_t *sb_rom,
                                                    const int32_t *sb_prob, const T *Mc, T *Y, int ld_slots,
                                                    int sb_base, int n_sb, int spw, int gate, int ks,
                                                    const ProbState *ps, double *pdel, ProbSel sel) {
    typedef typename Mfma<T>::v4 v4;
    // KS bounds the k-steps held in registers; the basis uses ks <= KS of
    // them (ldk = 4 ks), and steps past ks are neither loaded nor issued.
    // EXACT instances (ks == KS) keep every operand offset an immediate,
    // and issue the first KK of them: a basis of 168 in the 176-row layout
    // needs 42 of 44 (the last two multiply zero padding of K_r and u).
    if (EXACT) ks = KS;
    const int kd = EXACT ? KK : ks;
    // FP64 pipelines the slot blocks and requests the epilogue operands
    // ahead of the chain.  FP32 (twice the MFMA rate, four waves per SIMD)
    // was measured faster issuing each block's loads after the previous
    // chain, as a plain loop.
    constexpr bool PIPELINE = sizeof(T) == 8, PREFETCH_T = PIPELINE;
    const int ldk = 4 * ks;
    const int nrb = ldk / 16;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int task = (int)blockIdx.x * 4 + wave;
    const int rb = task % nrb, run = task / nrb;
    const int s_begin = run * spw;
    if (s_begin >= n_sb) return;
    const int s_end = min(s_begin + spw, n_sb);
    // Live slot blocks of the run, decided once.
    int rom_lane;
    const uint64_t live = run_mask(sb_rom, sb_prob, ps, gate, sel, sb_base, s_begin, s_end, &rom_lane);
    auto next_live = [&](int sl) { return next_in_mask(live, s_begin, s_end, sl); };
    auto rom_of = [&](int sl) { return __builtin_amdgcn_readlane(rom_lane, sl - s_begin); };
    int sl = next_live(s_begin);
    if (sl >= s_end) return;
    // Per-type K_r bases up front, so a slot block's operand loads wait on
    // its type only, not on a second pointer load.
    global_ptr<const T> kr[MAX_TYPES];
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) kr[t] = to_global(static_cast<const T *>(kr_tab[t]));
    const T *lane_b = Mc + (size_t)(lane / 16) * ld_slots + lane % 16;
    T a[KS], b[KS];
    {
        const T *bp = lane_b + (size_t)(sb_base + sl) * 16;
#pragma unroll
        for (int k = 0; k < KS; ++k) b[k] = k < kd ? bp[(size_t)(4 * k) * ld_slots] : T(0);
    }
    int cur = -1;
    while (sl < s_end) {
        const int sb = sb_base + sl;
        const int rom = rom_of(sl);
        const int col = sb * 16 + lane % 16;
        // The epilogue's operand values, requested before this block's
        // chain (and before the next block's loads) so they are not waited
        // on behind them.
        // (Loaded whether or not partials are wanted: a load on one path
        // only would make the chain below wait for every later load.)
        T t[4] = {T(0), T(0), T(0), T(0)};
        if (PREFETCH_T) {
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] = Mc[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * ld_slots + col];
        }
        if (rom != cur) {
            global_ptr<const T> ap = kr[rom] + (size_t)(lane / 16) * ldk + rb * 16 + lane % 16;
#pragma unroll
            for (int k = 0; k < KS; ++k) a[k] = k < kd ? ap[(size_t)(4 * k) * ldk] : T(0);
            cur = rom;
            vm_wait_all();
        }
        const int nx = next_live(sl + 1);
        v4 acc = {0, 0, 0, 0};
        if (PIPELINE) {
            // The last block's chain re-reads its own operand, so every
            // pass takes this one path.
            const T *bn = lane_b + (size_t)(sb_base + (nx < s_end ? nx : sl)) * 16;
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (k < kd) {
                    acc = Mfma<T>::op(a[k], b[k], acc);
                    b[k] = bn[(size_t)(4 * k) * ld_slots];
                }
        } else {
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (k < kd) acc = Mfma<T>::op(a[k], b[k], acc);
            if (!PIPELINE && nx < s_end) {
                const T *bn = lane_b + (size_t)(sb_base + nx) * 16;
#pragma unroll
                for (int k = 0; k < KS; ++k) b[k] = k < kd ? bn[(size_t)(4 * k) * ld_slots] : T(0);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Y[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * ld_slots + col] = acc[q];
        if (pdel) {
            const double v = PREFETCH_T ? tile_dot_vals<T>(acc, t) : tile_dot<T>(acc, Mc, ld_slots, rb, col, lane);
            if (lane == 0) pdel[(size_t)sb * nrb + rb] = v;
        }
        sl = nx;
    }
}

// Operand-tile-stationary variant: one workgroup per run of `spw`
// consecutive slot blocks, one wave per 16-row block of K_r (64 nrb
// threads).  Each live slot block's operand tile (ldk rows x 16 cells) is
// read from HBM once per workgroup -- one 16-byte chunk or two per thread --
// and staged in LDS, double-buffered so the next tile's loads are in flight
// during this tile's MFMA chains; every row block reads it from there, and
// each wave keeps its K_r rows in registers (reloaded when the cell type
// changes).  The chains are the K_r-stationary variant's, in the same order,
// and the tile partials are the same sums, so the two give the same bits.
template <class T>
struct Chunk16;
template <>
struct Chunk16<double> {
    typedef double v __attribute__((ext_vector_type(2)));
};
template <>
struct Chunk16<float> {
    typedef float v __attribute__((ext_vector_type(4)));
};

template <class T, int KS, bool EXACT, int KK = KS>
__global__ __launch_bounds__(704) void k_bgemm_wg(const void *const *kr_tab, const int32_t *sb_rom,
                                                  const int32_t *sb_prob, const T *Mc, T *Y, int ld_slots,
                                                  int sb_base, int n_sb, int spw, int gate, int ks,
                                                  const ProbState *ps, double *pdel, ProbSel sel) {
    typedef typename Mfma<T>::v4 v4;
    typedef typename Chunk16<T>::v c16;
    constexpr int EPC = 16 / sizeof(T);  // elements per 16-byte chunk
    constexpr int CPR = 16 / EPC;        // chunks per tile row of 16 cells
    constexpr int CPT = 4 / EPC;         // chunks per thread: ldk CPR chunks over 64 nrb = 16 ks threads
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *tiles = reinterpret_cast<T *>(lds_raw);  // [2][ldk][16]
    if (EXACT) ks = KS;
    const int kd = EXACT ? KK : ks;  // k-steps that carry data (as in k_bgemm_rows)
    const int ldk = 4 * ks;
    const int nrb = ks / 4;
    const int nthr = 64 * nrb;
    const int tid = threadIdx.x, lane = tid % 64, rb = tid / 64;
    const int s_begin = (int)blockIdx.x * spw;
    if (s_begin >= n_sb) return;
    const int s_end = min(s_begin + spw, n_sb);
    // Live slot blocks of the run, decided once.
    int rom_lane;
    const uint64_t live = run_mask(sb_rom, sb_prob, ps, gate, sel, sb_base, s_begin, s_end, &rom_lane);
    auto next_live = [&](int sl) { return next_in_mask(live, s_begin, s_end, sl); };
    auto rom_of = [&](int sl) { return __builtin_amdgcn_readlane(rom_lane, sl - s_begin); };
    int sl = next_live(s_begin);
    if (sl >= s_end) return;
    // Tile chunk c of this thread: row c / CPR, cells (c % CPR) * EPC.
    c16 stage[CPT];
    auto fetch = [&](int slot_block) {
        const T *src = Mc + (size_t)slot_block * 16;
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int c = tid + i * nthr;
            stage[i] = *reinterpret_cast<const c16 *>(src + (size_t)(c / CPR) * ld_slots + (c % CPR) * EPC);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int c = tid + i * nthr;
            *reinterpret_cast<c16 *>(tiles + ((size_t)buf * ldk + c / CPR) * 16 + (c % CPR) * EPC) = stage[i];
        }
    };
    global_ptr<const T> kr[MAX_TYPES];
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) kr[t] = to_global(static_cast<const T *>(kr_tab[t]));
    T a[KS];
    int cur = -1;
    fetch(sb_base + sl);
    put(0);
    __syncthreads();
    int buf = 0;
    while (sl < s_end) {
        const int sb = sb_base + sl;
        const int rom = rom_of(sl);
        if (rom != cur) {
            global_ptr<const T> ap = kr[rom] + (size_t)(lane / 16) * ldk + rb * 16 + lane % 16;
#pragma unroll
            for (int k = 0; k < KS; ++k) a[k] = k < kd ? ap[(size_t)(4 * k) * ldk] : T(0);
            cur = rom;
            vm_wait_all();
        }
        // The next tile's loads are issued on every pass (the last one
        // re-reads this tile), so no path leaves them conditional and the
        // chain below never waits on them.
        const int nx = next_live(sl + 1);
        fetch(sb_base + (nx < s_end ? nx : sl));
        // Keep the loads ahead of the chain (the scheduler would otherwise
        // sink them next to their use in put()).
        __builtin_amdgcn_sched_barrier(0);
        const T *tb = tiles + (size_t)buf * ldk * 16;
        v4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < KS; ++k)
            if (k < kd) acc = Mfma<T>::op(a[k], tb[(4 * k + lane / 16) * 16 + lane % 16], acc);
        const int col = sb * 16 + lane % 16;
#pragma unroll
        for (int q = 0; q < 4; ++q) Y[(size_t)(rb * 16 + Mfma<T>::row(lane, q)) * ld_slots + col] = acc[q];
        if (pdel) {
            T t[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) t[q] = tb[(rb * 16 + Mfma<T>::row(lane, q)) * 16 + lane % 16];
            const double v = tile_dot_vals<T>(acc, t);
            if (lane == 0) pdel[(size_t)sb * nrb + rb] = v;
        }
        // The other buffer was last read before the previous barrier; this
        // one is not written again before the next barrier.
        if (nx < s_end) put(buf ^ 1);
        __syncthreads();
        buf ^= 1;
        sl = nx;
    }
}

// One K_r-stationary cell-GEMM launch over slot blocks [0, n_sb): operand
// path 0 streams the operand per wave from global memory (one wave per row
// block and run of spw slot blocks, four per workgroup), path 1 stages each
// operand tile in LDS (one workgroup of one wave per row block per run).
// Gate 1 skips slot blocks whose problem is not iterating, gate 2 those of
// problems not in sel.  The launch is sampled by the kernel timer under
// timed_id (0: never).
template <class T, int KS, bool EXACT, int KK = KS>
void launch_cell_gemm_ks(mos_ctx ctx, int timed_id, int path, int spw, hipStream_t st, const void *const *kr_tab,
                         const int32_t *sb_rom, const int32_t *sb_prob, const T *Mc, T *Y, int ld_slots, int n_sb,
                         int ks, const ProbState *ps, double *pdel, int gate, const ProbSel &sel) {
    const int nrb = ks / 4;
    if (path == 1) {
        const dim3 grid((unsigned)ceil_div(n_sb, spw));
        const size_t lds = 2 * (size_t)(4 * ks) * 16 * sizeof(T);
        launch_timed(ctx, timed_id, k_bgemm_wg<T, KS, EXACT, KK>, grid, dim3(64 * nrb), (uint32_t)lds, st, kr_tab,
                     sb_rom, sb_prob, Mc, Y, ld_slots, 0, n_sb, spw, gate, ks, ps, pdel, sel);
    } else {
        const dim3 grid((unsigned)ceil_div((int64_t)nrb * ceil_div(n_sb, spw), 4));
        launch_timed(ctx, timed_id, k_bgemm_rows<T, KS, EXACT, KK>, grid, dim3(256), 0, st, kr_tab, sb_rom, sb_prob,
                     Mc, Y, ld_slots, 0, n_sb, spw, gate, ks, ps, pdel, sel);
    }
}

// ks = ldk / 4 k-steps of the padded layout, of which the basis of n
// columns fills ceil(n / 4).
template <class T>
mos_status launch_cell_gemm(mos_ctx ctx, int timed_id, int path, int ks, int n, int spw, hipStream_t st,
                            const void *const *kr_tab, const int32_t *sb_rom, const int32_t *sb_prob, const T *Mc,
                            T *Y, int ld_slots, int n_sb, const ProbState *ps, double *pdel, int gate,
                            const ProbSel &sel) {
    if (ks == ROWS_MAX_KS && ceil_div(n, 4) == 42)
        launch_cell_gemm_ks<T, ROWS_MAX_KS, true, 42>(ctx, timed_id, path, spw, st, kr_tab, sb_rom, sb_prob, Mc, Y,
                                                      ld_slots, n_sb, ks, ps, pdel, gate, sel);
    else if (ks == 8)
        launch_cell_gemm_ks<T, 8, true>(ctx, timed_id, path, spw, st, kr_tab, sb_rom, sb_prob, Mc, Y, ld_slots,
                                        n_sb, ks, ps, pdel, gate, sel);
    else if (ks == 20)
        launch_cell_gemm_ks<T, 20, true>(ctx, timed_id, path, spw, st, kr_tab, sb_rom, sb_prob, Mc, Y, ld_slots,
                                         n_sb, ks, ps, pdel, gate, sel);
    else if (ks == ROWS_MAX_KS)
        launch_cell_gemm_ks<T, ROWS_MAX_KS, true>(ctx, timed_id, path, spw, st, kr_tab, sb_rom, sb_prob, Mc, Y,
                                                  ld_slots, n_sb, ks, ps, pdel, gate, sel);
    else if (ks < ROWS_MAX_KS)
        launch_cell_gemm_ks<T, ROWS_MAX_KS, false>(ctx, timed_id, path, spw, st, kr_tab, sb_rom, sb_prob, Mc, Y,
                                                   ld_slots, n_sb, ks, ps, pdel, gate, sel);
    else {
        set_error("no K_r-stationary GEMM for %d k-steps", ks);
        return MOS_EINVAL;
    }
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

// Incidence of DoF d: up to four packed (slot, surface node) of the cells
// around its node, ascending cell order, -1 padded.
__device__ __forceinline__ int4 incidence(const int32_t *inc, int64_t d) {
    return reinterpret_cast<const int4 *>(inc)[d / 3];
}

// Sum of a DoF's entries in the cell layout over the cells around its
// node.  Branch-free: an unused entry loads element 0 and is dropped by a
// select, so all four loads are in flight together instead of each waiting
// behind a branch.
template <class T>
__device__ __forceinline__ T cell_sum(const T *Y, int4 iv, int ci, int ld_slots) {
    const int e4[4] = {iv.x, iv.y, iv.z, iv.w};
    T v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const size_t i = (size_t)(3 * (e4[e] & MAX_SURF) + ci) * ld_slots + (e4[e] >> INC_SHIFT);
        v[e] = Y[e4[e] >= 0 ? i : 0];
    }
    T s = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s += e4[e] >= 0 ? v[e] : T(0);
    return s;
}

template <class T>
__device__ __forceinline__ void cell_scatter(T *Mc, int4 iv, int ci, int ld_slots, T v) {
    const int e4[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (e4[e] >= 0) Mc[(size_t)(3 * (e4[e] & MAX_SURF) + ci) * ld_slots + (e4[e] >> INC_SHIFT)] = v;
}

// The cells of a stacked array's layer above a node on a shared horizontal
// face (inc2, after those of the node's own layer in inc: ascending cell id),
// for the kernels that take them; -1 everywhere for one-layer arrays.
__device__ __forceinline__ int4 incidence2(const int32_t *inc2, int64_t d) {
    return inc2 ? reinterpret_cast<const int4 *>(inc2)[d / 3] : make_int4(-1, -1, -1, -1);
}

// Element at a 32-bit byte offset from a uniform base: lets the compiler
// address it as scalar base + one 32-bit offset register.
template <class T>
__device__ __forceinline__ T &at_byte(T *base, uint32_t off) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}
template <class T>
__device__ __forceinline__ const T &at_byte(const T *base, uint32_t off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// cell_sum / cell_scatter for cell layouts below 4 GiB (32-bit byte offsets).
template <class T>
__device__ __forceinline__ T cell_sum32(const T *Y, const int4 &iv, int ci, uint32_t ld_slots) {
    const int e4[4] = {iv.x, iv.y, iv.z, iv.w};
    T v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t o =
            ((uint32_t)(3 * (e4[e] & MAX_SURF) + ci) * ld_slots + (uint32_t)(e4[e] >> INC_SHIFT)) * (uint32_t)sizeof(T);
        v[e] = at_byte(Y, e4[e] >= 0 ? o : 0u);
    }
    T s = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s += e4[e] >= 0 ? v[e] : T(0);
    return s;
}

template <class T>
__device__ __forceinline__ void cell_scatter32(T *Mc, const int4 &iv, int ci, uint32_t ld_slots, T v) {
    const int e4[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (e4[e] >= 0)
            at_byte(Mc, ((uint32_t)(3 * (e4[e] & MAX_SURF) + ci) * ld_slots + (uint32_t)(e4[e] >> INC_SHIFT)) *
                            (uint32_t)sizeof(T)) = v;
}

// Owner and type tables of the listed problems' blocks back to -1, problems
// inactive; grid (any, problems).
__global__ __launch_bounds__(256) void k_release_list(PidList L, const ProbParams *pp, int32_t *blk_prob,
                                                      int32_t *sb_rom, int32_t *sb_prob, int4 *box_tab,
                                                      ProbState *ps) {
    const int p = L.pid[blockIdx.y];
    const ProbParams &P = pp[p];
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    for (int i = t0; i < P.n_blk; i += stride) blk_prob[P.blk_begin + i] = -1;
    if (P.box_begin >= 0)
        for (int i = t0; i < P.n_agg; i += stride) box_tab[P.box_begin + i] = make_int4(-1, -1, -1, -1);
    for (int i = t0; i < P.n_sb; i += stride) {
        sb_rom[P.sb_begin + i] = -1;
        sb_prob[P.sb_begin + i] = -1;
    }
    if (t0 == 0) ps[p].active = 0;
}

// Per-block (r,u) and (r,r) partials of an update workgroup of NT threads,
// DoF j NT + t of the block at thread t, slot j: each group of 64
// consecutive DoFs is summed by a butterfly over its wave's lanes, and the
// groups in DoF order -- the same bits for either workgroup size.
template <int NT>
__device__ __forceinline__ void block_partials(const double (&g)[DB / NT], const double (&r)[DB / NT], double &gs,
                                               double &rs) {
    constexpr int DPT = DB / NT, NG = DB / 64;
    __shared__ double sh[2][NG];
    const int w = threadIdx.x / 64;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        double a = g[j], b = r[j];
        for (int m = 32; m >= 1; m >>= 1) {
            a += __shfl_xor(a, m);
            b += __shfl_xor(b, m);
        }
        if (threadIdx.x % 64 == 0) {
            sh[0][j * (NT / 64) + w] = a;
            sh[1][j * (NT / 64) + w] = b;
        }
    }
    __syncthreads();
    gs = rs = 0.0;
    for (int i = 0; i < NG; ++i) {
        gs += sh[0][i];
        rs += sh[1][i];
    }
}

// Update workgroups of 256 threads (one DoF each) while every block of the
// launch fits on the chip at once; beyond that 128 threads with two DoFs
// each, so more blocks are resident and each thread has more loads in
// flight.  Both give the same bits.
constexpr int CG_WIDE_MAX_BLK = 2048;

// One iteration, per DoF block of every iterating problem, Chronopoulos-Gear
// form: with the published (alpha, beta) and w = A u assembled from the cell
// products (u = M^-1 r),
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
// then the next u = M^-1 r to the cell layout and the partials of the next
// (r,u) and (r,r).  Only x, r, p and s are stored.
template <class T, int NT>
__global__ __launch_bounds__(NT) void k_cgstep(const T *Y, const int32_t *inc, const int32_t *inc2,
                                               const uint8_t *cmask, const T *dinv, T *x, T *r, T *p, T *s, T *Mc,
                                               int ld_slots, const int32_t *blk_prob, ProbState *ps, double *pg,
                                               double *pr, const double *pdel, const int *ep, int j, int cap_blk,
                                               int n_blk, double *lz) {
    constexpr int DPT = DB / NT;
    __shared__ int go, it_sh;
    __shared__ double step[2];
    __shared__ double red[3][NT];
    // Workgroups are dealt to the XCDs in turn; DoF block `blk` is taken so
    // that each XCD gets one contiguous run of blocks, and the cell-layout
    // lines that neighbouring blocks gather from and scatter to meet in one
    // L2 instead of several.
    const int per = (n_blk + N_XCD - 1) / N_XCD;
    const int blk = (int)(blockIdx.x % N_XCD) * per + (int)(blockIdx.x / N_XCD);
    if (blk >= n_blk) return;
    const int64_t d0 = (int64_t)blk * DB + threadIdx.x;
    // Only the incidence is requested before the gate resolves: blocks of
    // problems that have stopped (converged, or between refinement sweeps)
    // must not spend bandwidth on their operands.
    int4 iv[DPT], iv2[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        iv[j] = incidence(inc, d0 + j * NT);
        iv2[j] = incidence2(inc2, d0 + j * NT);
    }
    const int pb = blk_prob[blk];
    if (threadIdx.x == 0) {
        int g = 0;
        if (pb >= 0) {
            // Every field read unconditionally (no short-circuit), so the
            // state arrives in one round trip rather than one per field.
            const ProbState &S = ps[pb];
            const int active = S.active, done = S.done, fused = S.fused, start = S.start_epoch;
            const double a_cur = S.a_cur, b_cur = S.b_cur;
            g = ((active != 0) & (done == 0)) ? 1 + (fused != 0) : 0;
            step[0] = a_cur;
            step[1] = b_cur;
            it_sh = ep[0] + j - start;
        }
        go = g;
    }
    __syncthreads();
    if (!go) return;
    // Per-block partials double-buffered by iteration parity: this
    // iteration reads slot it & 1 and writes slot (it + 1) & 1, so no block
    // overwrites a partial another block of the launch may still read.
    const int it = it_sh;
    const size_t rd_slot = (size_t)(it & 1) * cap_blk, wr_slot = (size_t)((it + 1) & 1) * cap_blk;
    if (go == 2) {
        // Small problem: every workgroup reduces its partials itself (same
        // bits in each); the problem's first workgroup publishes the state.
        ProbState &S = ps[pb];
        const CgStep o = cg_scalars_block<NT>(S, it, pg + rd_slot, pr + rd_slot, pdel, red);
        if (threadIdx.x == 0 && blk == S.blk_begin) cg_publish(S, it, o, lz_row(lz, pb));
        if (o.stop) return;
        if (threadIdx.x == 0) {
            step[0] = o.alpha;
            step[1] = o.beta;
        }
        __syncthreads();
    }
    const T a = (T)step[0], b = (T)step[1];
    // All operands of the thread's DoFs first (the arrays may alias as far
    // as the compiler knows, so loads are not moved past earlier stores).
    T dv[DPT], rd[DPT], pd0[DPT], sd[DPT], xd[DPT], wv[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int64_t d = d0 + j * NT;
        dv[j] = dinv[d];
        rd[j] = r[d];
        pd0[j] = p[d];
        sd[j] = s[d];
        xd[j] = x[d];
        T sum = cell_sum(Y, iv[j], (int)(d % 3), ld_slots);
        if (inc2) sum += cell_sum(Y, iv2[j], (int)(d % 3), ld_slots);
        wv[j] = cmask[d] ? T(0) : sum;
    }
    double g[DPT], r2[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int64_t d = d0 + j * NT;
        const T uv = dv[j] * rd[j];
        const T pv = uv + b * pd0[j];
        const T sv = wv[j] + b * sd[j];
        x[d] = xd[j] + a * pv;
        const T rv = rd[j] - a * sv;
        const T un = dv[j] * rv;
        p[d] = pv;
        s[d] = sv;
        r[d] = rv;
        cell_scatter(Mc, iv[j], (int)(d % 3), ld_slots, un);
        if (inc2) cell_scatter(Mc, iv2[j], (int)(d % 3), ld_slots, un);
        g[j] = (double)rv * (double)un;
        r2[j] = (double)rv * (double)rv;
    }
    double gs, rs;
    block_partials<NT>(g, r2, gs, rs);
    if (threadIdx.x == 0) {
        pg[wr_slot + blk] = gs;
        pr[wr_slot + blk] = rs;
    }
}

// ---- two-level preconditioner: Jacobi plus a coarse correction on aggregates ----
// M^-1 r = D^-1 r + sum over aggregates a of Z_a B_a^-1 Z_a^T r, with Z_a the
// six rigid-body modes of aggregate a (three translations, three rotations
// about its corner) on its free DoFs and zero elsewhere, and B_a = Z_a^T A Z_a.
// Aggregates are AGG_C x AGG_C cells; one workgroup owns a box of
// aggregates (the internal node order keeps a box's DoFs consecutive), so
// the restriction Z_a^T r, the 6x6 solve and the prolongation stay inside
// the workgroup.  Symmetric positive definite, so PCG stays valid.

// Rigid-body mode values at a node (coordinates X, Y, Zc from the
// aggregate's corner): restriction of the node's three components r, and
// prolongation of coefficients c onto them.
template <class T>
__device__ __forceinline__ void node_restrict(double X, double Y, double Zc, const T (&r)[3], const bool (&f)[3],
                                              double (&q)[6]) {
    const double r0 = f[0] ? (double)r[0] : 0.0, r1 = f[1] ? (double)r[1] : 0.0, r2 = f[2] ? (double)r[2] : 0.0;
    q[0] = r0;
    q[1] = r1;
    q[2] = r2;
    q[3] = X * r1 - Y * r0;
    q[4] = Y * r2 - Zc * r1;
    q[5] = Zc * r0 - X * r2;
}

__device__ __forceinline__ void node_prolong(double X, double Y, double Zc, const double *c, double (&u)[3]) {
    u[0] = c[0] - Y * c[3] + Zc * c[5];
    u[1] = c[1] + X * c[3] - Zc * c[4];
    u[2] = c[2] + Y * c[4] - X * c[5];
}

// Packed aggregate-local coordinates of a node: i | j << 8 | K << 16 |
// a << 24 | constrained components << 28 (a = aggregate within the box).
__device__ __forceinline__ void unpack_lc(uint32_t w, const double *h, double &X, double &Y, double &Zc, int &a,
                                          bool (&f)[3]) {
    // Physical coordinates of a skewed block: x += skew * y (h[3] = skew).
    Y = (double)((w >> 8) & 255u) * h[1];
    X = (double)(w & 255u) * h[0] + h[3] * Y;
    Zc = (double)((w >> 16) & 255u) * h[2];
    a = (int)((w >> 24) & 15u);
    for (int ci = 0; ci < 3; ++ci) f[ci] = ((w >> (28 + ci)) & 1u) == 0;
}

// Box b of problem P: its first node (index into the global node arrays),
// node count, and number of aggregates.
__device__ __forceinline__ void box_geometry(const ProbParams &P, int b, int64_t &first, int &nn, int &na) {
    const AggLayout &A = P.agg;
    const int gx = b % A.nax, gy = b / A.nax;
    first = P.d0 / 3 + agg_first(A, gx, gy);
    nn = (int)sub_count(agg_box(A, gx, gy));
    const int cells = gx == A.nax - 1 ? P.lat.Nx - A.cx * (A.nax - 1) : A.cx;
    na = (cells + AGG_C - 1) / AGG_C;
}

// Index in the inner vectors of DoF (node, ci) of problem P (node relative
// to the problem).  With boxes (two-level preconditioner) the inner vectors
// are component-major within each box -- component ci of the box's t-th node
// at 3 * first + ci * nn + t -- so a box workgroup with one node per thread
// reads and writes them in whole lines; otherwise 3 * node + ci.
__device__ __forceinline__ int64_t inner_index(const ProbParams &P, int64_t node, int ci) {
    if (P.box_begin < 0) return P.d0 + 3 * node + ci;
    const AggLayout &A = P.agg;
    int gy = (int)(node / A.row);
    if (gy > A.nay - 1) gy = A.nay - 1;
    const int64_t rem = node - (int64_t)gy * A.row;
    const int wy = gy == A.nay - 1 ? A.wyl : A.wyi;
    const int64_t per = sub_count(make_sub(A.wxi, wy, A.Z, A.sx, A.sy, A.sz));
    int gx = (int)(rem / per);
    if (gx > A.nax - 1) gx = A.nax - 1;
    const int64_t first = agg_first(A, gx, gy);
    const int64_t nn = sub_count(agg_box(A, gx, gy));
    return P.d0 + 3 * first + ci * nn + (node - first);
}

// Scalar step computed by one box workgroup of at least CG_LW threads
// (threads beyond CG_LW idle).  Every box workgroup of a problem sums its
// partials in the same order, so all get the same bits.
__device__ CgStep cg_scalars_wide(const ProbState &S, int it, const double *pg, const double *pr,
                                  const double *pdel, double (*red)[CG_LW]) {
    const int t = threadIdx.x;
    if (t < CG_LW) {
        // Lane t sums partials t, t + CG_LW, ...; a butterfly per wave; the
        // waves' sums in order (one barrier).
        double g = 0.0, r = 0.0, dl = 0.0;
#pragma unroll 4
        for (int i = S.blk_begin + t; i < S.blk_end; i += CG_LW) {
            g += pg[i];
            r += pr[i];
        }
#pragma unroll 4
        for (int i = S.tile_begin + t; i < S.tile_end; i += CG_LW) dl += pdel[i];
        for (int m = 32; m >= 1; m >>= 1) {
            g += __shfl_xor(g, m);
            r += __shfl_xor(r, m);
            dl += __shfl_xor(dl, m);
        }
        if (t % 64 == 0) {
            red[0][t / 64] = g;
            red[1][t / 64] = r;
            red[2][t / 64] = dl;
        }
    }
    __syncthreads();
    double sum[3];
    for (int j = 0; j < 3; ++j) {
        sum[j] = red[j][0];
        for (int w = 1; w < CG_LW / 64; ++w) sum[j] += red[j][w];
    }
    CgStep o;
    o.gamma = sum[0];
    o.rr = sum[1];
    const double delta = sum[2];
    o.tol2 = it == S.seg_start ? S.rtol2 * o.rr : S.tol2;
    o.stop = 0;
    o.alpha = o.beta = 0.0;
    if (o.rr <= o.tol2) {
        o.stop = 1;
    } else if (it - S.seg_start >= S.max_iter) {
        o.stop = 3;
    } else {
        if (it == 0) {
            o.alpha = o.gamma / delta;
        } else {
            const int pv = (it - 1) & 1;
            o.beta = o.gamma / S.hist_gamma[pv];
            o.alpha = o.gamma / (delta - o.beta * o.gamma / S.hist_alpha[pv]);
        }
        if (!(o.alpha > 0.0) || !isfinite(o.alpha) || !isfinite(o.beta)) o.stop = 2;
    }
    return o;
}

// LDS of a box workgroup (the per-node restriction terms are dynamic LDS,
// blockDim.x x 6 doubles).
struct BoxShared {
    double bi[MAXA][36];         // B^-1 of the box's aggregates
    double wsum[16][2];          // per-wave (r,D^-1 r) and (r,r)
    double cn[MAXA][6];          // coarse coefficients B^-1 q
    double en[MAXA];             // q . c per aggregate
    double cold[MAXA][6];        // coefficients of the current r (start of an iteration)
    int8_t tag[1024];            // aggregate of each thread's node, -1 if none
};

// Box data requested at the start of a box workgroup: B^-1 of its
// aggregates (and, for an iteration, the kept coefficients).
__device__ __forceinline__ void box_prefetch(BoxShared &sh, const double *binv, const double *cc, int bs, int na,
                                             bool coeffs) {
    const int t = threadIdx.x;
    if (t < na * 36) sh.bi[t / 36][t % 36] = binv[(size_t)bs * MAXA * 36 + t];
    if (coeffs && t < na * 6) sh.cold[t / 6][t % 6] = cc[(size_t)bs * MAXA * 6 + t];
}

// Second half of an update or sweep start, once the thread's node holds the
// new residual rv: restriction per aggregate (fixed order), coarse solve,
// u = D^-1 r + Z c to the cell layout, the box's (r,u) and (r,r) partials
// into slot `pslot` and the coefficients kept for the next iteration.
// B^-1 must be in sh.bi (box_prefetch, before a barrier).
template <class T>
__device__ __forceinline__ void box_coarse_finish(BoxShared &sh, double (*qn)[6], bool act, int nn, int na, int bs,
                                                  const int4 &iv, const T (&dv)[3], const T (&rv)[3],
                                                  const bool (&f)[3], double X, double Y, double Zc, int a, T *Mc,
                                                  int ld_slots, double *cc, double *pg, double *pr, size_t pslot) {
    const int t = threadIdx.x, lane = t % 64, w = t / 64, nw = blockDim.x / 64;
    double gd = 0.0, r2 = 0.0;
    double q[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        for (int ci = 0; ci < 3; ++ci) {
            gd += (double)rv[ci] * (double)(dv[ci] * rv[ci]);
            r2 += (double)rv[ci] * (double)rv[ci];
        }
        node_restrict(X, Y, Zc, rv, f, q);
    }
    for (int m = 0; m < 6; ++m) qn[t][m] = q[m];
    sh.tag[t] = act ? (int8_t)a : (int8_t)-1;
    for (int m = 32; m >= 1; m >>= 1) {
        gd += __shfl_xor(gd, m);
        r2 += __shfl_xor(r2, m);
    }
    if (lane == 0) {
        sh.wsum[w][0] = gd;
        sh.wsum[w][1] = r2;
    }
    __syncthreads();
    // Wave k < na sums aggregate k (lane L takes nodes L, L + 64, ...; the
    // butterfly leaves the sum in every lane) and solves its 6x6 system.
    if (w < na) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int l = lane; l < nn; l += 64)
            if (sh.tag[l] == w)
                for (int m = 0; m < 6; ++m) acc[m] += qn[l][m];
        for (int m = 0; m < 6; ++m)
            for (int k = 32; k >= 1; k >>= 1) acc[m] += __shfl_xor(acc[m], k);
        if (lane == 0) {
            double e = 0.0;
            for (int m = 0; m < 6; ++m) {
                double c = 0.0;
                for (int k = 0; k < 6; ++k) c += sh.bi[w][m * 6 + k] * acc[k];
                sh.cn[w][m] = c;
                e += acc[m] * c;
            }
            sh.en[w] = e;
        }
    }
    __syncthreads();
    if (act) {
        double uc[3];
        node_prolong(X, Y, Zc, sh.cn[a], uc);
        for (int ci = 0; ci < 3; ++ci) {
            const T un = dv[ci] * rv[ci] + (f[ci] ? (T)uc[ci] : T(0));
            cell_scatter32(Mc, iv, ci, (uint32_t)ld_slots, un);
        }
    }
    if (t < na * 6) cc[(size_t)bs * MAXA * 6 + t] = sh.cn[t / 6][t % 6];
    if (t == 0) {
        double g = 0.0, rr = 0.0;
        for (int i = 0; i < nw; ++i) {
            g += sh.wsum[i][0];
            rr += sh.wsum[i][1];
        }
        double e = 0.0;
        for (int ag = 0; ag < na; ++ag) e += sh.en[ag];
        pg[pslot + bs] = g + e;
        pr[pslot + bs] = rr;
    }
}

// One iteration of the two-level form, one workgroup per box (one thread
// per node, blockDim.x >= the box's nodes and >= CG_LW): as k_cgstep, with
// u = M^-1 r of the two-level preconditioner.  The current u is rebuilt
// from r and the coefficients kept by the previous step.
template <class T>
__global__ __launch_bounds__(1024) void k_cgstep2(const T *Y, const int32_t *inc, const uint8_t *cmask,
                                                  const T *dinv, const uint32_t *lc, T *x, T *r, T *p, T *s, T *Mc,
                                                  int ld_slots, const int4 *box_tab, const ProbParams *pp,
                                                  ProbState *ps, double *pg, double *pr, const double *pdel,
                                                  const double *binv, double *cc, const int *ep, int j,
                                                  int cap_blk, int n_box, double *lz) {
    // Dynamic LDS: the per-node restriction terms (blockDim.x x 6 doubles),
    // first used as the scalar step's reduction space (3 x CG_LW doubles).
    extern __shared__ double qn_dyn[];
    double(*qn)[6] = reinterpret_cast<double(*)[6]>(qn_dyn);
    double(*red)[CG_LW] = reinterpret_cast<double(*)[CG_LW]>(qn_dyn);
    __shared__ BoxShared sh;
    __shared__ int go, it_sh;
    __shared__ double step[2];
    const int per = (n_box + N_XCD - 1) / N_XCD;
    const int bs = (int)(blockIdx.x % N_XCD) * per + (int)(blockIdx.x / N_XCD);
    if (bs >= n_box) return;
    // The box's first node, node count, aggregates and owner, in one load.
    const int4 bt = box_tab[bs];
    const int pb = bt.w;
    if (pb < 0) return;
    const ProbParams &P = pp[pb];
    const int64_t first = bt.x;
    const int nn = bt.y, na = bt.z;
    const int t = threadIdx.x;
    const bool act = t < nn;
    // Uniform bases of the box and 32-bit lane offsets, so every vector
    // access shares one offset register.
    const int4 iv = act ? reinterpret_cast<const int4 *>(inc)[first + t] : make_int4(-1, -1, -1, -1);
    box_prefetch(sh, binv, cc, bs, na, true);
    if (t == 0) {
        const ProbState &S = ps[pb];
        const int active = S.active, done = S.done, fused = S.fused, start = S.start_epoch;
        const double a_cur = S.a_cur, b_cur = S.b_cur;
        const int g = ((active != 0) & (done == 0)) ? 1 + (fused != 0) : 0;
        step[0] = a_cur;
        step[1] = b_cur;
        it_sh = ep[0] + j - start;
        go = g;
    }
    __syncthreads();
    if (!go) return;
    const int it = it_sh;
    const size_t rd_slot = (size_t)(it & 1) * cap_blk, wr_slot = (size_t)((it + 1) & 1) * cap_blk;
    // The node's operands are requested before the scalar step (they do not
    // depend on alpha and beta), so their round trip overlaps the one for
    // the problem's partials.
    T dv[3] = {0, 0, 0}, rv[3] = {0, 0, 0};
    T rd[3] = {0, 0, 0}, pd0[3] = {0, 0, 0}, sd[3] = {0, 0, 0}, xd[3] = {0, 0, 0}, wv[3] = {0, 0, 0};
    bool f[3] = {false, false, false};
    uint32_t lw = 0;
    // Component-major within the box: component ci of node t at ci * nn + t.
    const int64_t vb = 3 * first;
    const T *db = dinv + vb;
    T *xb = x + vb, *rb = r + vb, *pbv = p + vb, *sb = s + vb;
    if (act) {
        lw = lc[first + t];
        for (int ci = 0; ci < 3; ++ci) {
            const uint32_t o = (uint32_t)(ci * nn + t) * (uint32_t)sizeof(T);
            dv[ci] = at_byte(db, o);
            rd[ci] = at_byte(rb, o);
            pd0[ci] = at_byte(pbv, o);
            sd[ci] = at_byte(sb, o);
            xd[ci] = at_byte(xb, o);
            wv[ci] = cell_sum32(Y, iv, ci, (uint32_t)ld_slots);
        }
    }
    if (go == 2) {
        ProbState &S = ps[pb];
        const CgStep o = cg_scalars_wide(S, it, pg + rd_slot, pr + rd_slot, pdel, red);
        if (t == 0 && bs == S.blk_begin) cg_publish(S, it, o, lz_row(lz, pb));
        if (o.stop) return;
        if (t == 0) {
            step[0] = o.alpha;
            step[1] = o.beta;
        }
        // Also ends every read of the reduction space before it holds
        // restriction terms.
        __syncthreads();
    }
    const T al = (T)step[0], be = (T)step[1];
    double X = 0.0, Yc = 0.0, Zc = 0.0;
    int a = 0;
    if (act) {
        unpack_lc(lw, P.h, X, Yc, Zc, a, f);
        for (int ci = 0; ci < 3; ++ci)
            if (!f[ci]) wv[ci] = T(0);
        double uc[3];
        node_prolong(X, Yc, Zc, sh.cold[a], uc);
        for (int ci = 0; ci < 3; ++ci) {
            const uint32_t o = (uint32_t)(ci * nn + t) * (uint32_t)sizeof(T);
            const T uv = dv[ci] * rd[ci] + (f[ci] ? (T)uc[ci] : T(0));
            const T pv = uv + be * pd0[ci];
            const T sv = wv[ci] + be * sd[ci];
            at_byte(xb, o) = xd[ci] + al * pv;
            rv[ci] = rd[ci] - al * sv;
            at_byte(pbv, o) = pv;
            at_byte(sb, o) = sv;
            at_byte(rb, o) = rv[ci];
        }
    }
    box_coarse_finish(sh, qn, act, nn, na, bs, iv, dv, rv, f, X, Yc, Zc, a, Mc, ld_slots, cc, pg, pr, wr_slot);
}

// Sweep start in the two-level form: r = scale_in * r64, x = 0, p and s
// cleared or rescaled, u = M^-1 r to the cell layout and the partials of the
// sweep's first iteration.
template <class T>
__global__ __launch_bounds__(1024) void k_cgstart2(ProbSel sel, const int4 *box_tab, const ProbParams *pp,
                                                   const SweepParams *sp, const ProbState *ps, const double *r64,
                                                   const T *dinv, const int32_t *inc, const uint8_t *cmask,
                                                   const uint32_t *lc, T *x, T *r, T *p, T *s, T *Mc, int ld_slots,
                                                   double *pg, double *pr, const double *binv, double *cc,
                                                   int cap_blk) {
    extern __shared__ double qn_dyn[];
    double(*qn)[6] = reinterpret_cast<double(*)[6]>(qn_dyn);
    __shared__ BoxShared sh;
    const int bs = blockIdx.x;
    const int4 bt = box_tab[bs];
    const int pb = bt.w;
    if (pb < 0 || !selected(sel, pb)) return;
    const ProbParams &P = pp[pb];
    const int64_t first = bt.x;
    const int nn = bt.y, na = bt.z;
    const int t = threadIdx.x;
    const bool act = t < nn;
    const int4 iv = act ? reinterpret_cast<const int4 *>(inc)[first + t] : make_int4(-1, -1, -1, -1);
    const SweepParams &W = sp[pb];
    box_prefetch(sh, binv, cc, bs, na, false);
    T dv[3] = {0, 0, 0}, rv[3] = {0, 0, 0};
    bool f[3] = {false, false, false};
    double X = 0.0, Yc = 0.0, Zc = 0.0;
    int a = 0;
    if (act) {
        unpack_lc(lc[first + t], P.h, X, Yc, Zc, a, f);
        const T c = (T)W.p_scale;
        for (int ci = 0; ci < 3; ++ci) {
            const int64_t v = 3 * first + ci * nn + t;  // component-major within the box
            dv[ci] = dinv[v];
            rv[ci] = (T)(r64[3 * (first + t) + ci] * W.scale_in);
            x[v] = 0;
            r[v] = rv[ci];
            if (W.cont) {
                p[v] *= c;
                s[v] *= c;
            } else {
                p[v] = 0;
                s[v] = 0;
            }
        }
    }
    box_coarse_finish(sh, qn, act, nn, na, bs, iv, dv, rv, f, X, Yc, Zc, a, Mc, ld_slots, cc, pg, pr,
                      (size_t)(ps[pb].it & 1) * cap_blk);
}

// Inverse of a symmetric positive definite 6x6 matrix G (row-major) into
// out, by Gauss-Jordan elimination without pivoting on the lanes of one
// wave (lane 6 i + j holds entry (i, j); lanes 36..63 idle along); all
// zeros when a pivot is not numerically positive, which leaves that
// aggregate without a coarse correction.
__device__ void spd_inverse6_wave(const double *G, double *out) {
    const int lane = threadIdx.x % 64;
    const int i = min(lane / 6, 5), j = lane % 6;
    double m = lane < 36 ? G[lane] : 0.0, v = lane < 36 && i == j ? 1.0 : 0.0;
    double dmax = 0.0;
    for (int k = 0; k < 6; ++k) dmax = fmax(dmax, G[k * 7]);
    bool ok = dmax > 0.0 && isfinite(dmax);
    for (int k = 0; k < 6; ++k) {
        const double piv = __shfl(m, k * 7);
        ok = ok && piv > 1e-12 * dmax;
        const double fac = __shfl(m, i * 6 + k);
        const double rm = __shfl(m, k * 6 + j) / piv, rv = __shfl(v, k * 6 + j) / piv;
        if (i == k) {
            m = rm;
            v = rv;
        } else {
            m -= fac * rm;
            v -= fac * rv;
        }
    }
    if (lane < 36) out[lane] = ok ? v : 0.0;
}

// B_a^-1 of every aggregate of the selected problems' boxes; grid (boxes,
// MAXA), one workgroup per aggregate.  B_a = sum over the cells touching
// the aggregate of Z_c^T K_r(type) Z_c, Z_c the aggregate's modes on the
// cell's DoFs that belong to it and are free.  K_r is read in FP32 (B only
// defines the preconditioner; any symmetric positive definite B keeps PCG
// converging to the same solution) with FP64 sums.  The touching cells (at
// most 3 x 3) are summed in a fixed order, then the 6x6 inverse.  One thread
// per reduced DoF of a cell: NTH >= n threads (256, or 512 for bases above
// 256).
template <int NTH>
__global__ __launch_bounds__(NTH) void k_coarse_setup(ProbSel sel, const int4 *box_tab, const ProbParams *pp,
                                                      const int32_t *cslot, const int32_t *sb_rom,
                                                      const void *const *kr32_tab, const uint8_t *cmask,
                                                      const int32_t *surf, int n, int ldk, double *binv,
                                                      const int32_t *agg_gen) {
    constexpr int NW = NTH / 64;
    const int bs = blockIdx.x, a = blockIdx.y;
    const int pb = box_tab[bs].w;
    if (pb < 0 || !selected(sel, pb)) return;
    const ProbParams &P = pp[pb];
    // Clamp-only problems take the table; problems with a prescribed list
    // take it for the aggregates k_coarse_agg_tab marked tabulated.
    if (P.tab_coarse == 1 || (P.tab_coarse == 2 && agg_gen[(size_t)bs * MAXA + a] == 0)) return;
    const AggLayout &A = P.agg;
    const int b = bs - P.box_begin, gx = b % A.nax, gy = b / A.nax;
    const int bx0 = gx * A.cx, bx1 = gx == A.nax - 1 ? P.lat.Nx : bx0 + A.cx;
    const int by0 = gy * A.cy, by1 = gy == A.nay - 1 ? P.lat.Ny : by0 + A.cy;
    const int na = (bx1 - bx0 + AGG_C - 1) / AGG_C;
    double *out = binv + ((size_t)bs * MAXA + a) * 36;
    const int t = threadIdx.x;
    if (a >= na) {
        if (t < 36) out[t] = 0.0;
        return;
    }
    const int ax0 = bx0 + a * AGG_C, ax1 = min(ax0 + AGG_C, bx1);
    const int cx0 = max(ax0 - 1, 0), cy0 = max(by0 - 1, 0);
    const int ncx = ax1 - cx0, ncells = ncx * (by1 - cy0);
    __shared__ double zl[NTH][6], G[21], wpart[NW][21];
    __shared__ int16_t list[NTH];
    __shared__ int wcnt[NW];
    __shared__ double Bfull[36];
    if (t < 21) G[t] = 0.0;
    const int sx = A.sx, sy = A.sy;
    const int w = t / 64, lane = t % 64;
    for (int ci_cell = 0; ci_cell < ncells; ++ci_cell) {
        const int cx = cx0 + ci_cell % ncx, cy = cy0 + ci_cell / ncx;
        const float *K = nullptr;
        {
            const int cell = cy * P.lat.Nx + cx;
            const int slot = cslot[(int64_t)P.sb_begin * 16 + cell];
            K = static_cast<const float *>(kr32_tab[sb_rom[slot / 16]]);
        }
        __syncthreads();
        bool mine = false;
        if (t < n) {
            const int sn = t / 3, ci = t % 3;
            const int64_t I = (int64_t)cx * sx + surf[3 * sn], J = (int64_t)cy * sy + surf[3 * sn + 1];
            const int Kz = surf[3 * sn + 2];
            bool in = agg_x(A, I) == gx && agg_y(A, J) == gy;
            const int ib = (int)(I - (int64_t)gx * A.wxi);
            const int ag = min(ib / (AGG_C * sx), na - 1);
            in = in && ag == a;
            const int64_t dd = P.d0 + 3 * agg_encode(A, I, J, Kz) + ci;
            in = in && cmask[dd] == 0;
            double z[6] = {0, 0, 0, 0, 0, 0};
            if (in) {
                const double Yc = (double)(J - (int64_t)gy * A.wyi) * P.h[1];
                const double X = (double)(ib - ag * AGG_C * sx) * P.h[0] + P.h[3] * Yc;
                const double Zc = (double)Kz * P.h[2];
                // Mode values at component ci (columns of Z).
                z[ci] = 1.0;
                if (ci == 0) {
                    z[3] = -Yc;
                    z[5] = Zc;
                } else if (ci == 1) {
                    z[3] = X;
                    z[4] = -Zc;
                } else {
                    z[4] = Yc;
                    z[5] = -X;
                }
            }
            for (int m = 0; m < 6; ++m) zl[t][m] = z[m];
            mine = in;
        }
        // The cell's DoFs in the aggregate, ascending, as a list (ballot per
        // wave, waves in order).
        const uint64_t bal = __ballot(mine);
        if (lane == 0) wcnt[w] = __popcll(bal);
        __syncthreads();
        int base = 0, nl = 0;
        for (int i = 0; i < NW; ++i) {
            base += i < w ? wcnt[i] : 0;
            nl += wcnt[i];
        }
        if (mine) list[base + __popcll(bal & ((1ull << lane) - 1))] = (int16_t)t;
        __syncthreads();
        // Row t of K_r Z over the listed columns (K_r symmetric: row l read
        // across threads), then the row's share of the symmetric Z^T K_r Z,
        // summed over the workgroup in a fixed order.
        double acc[6] = {0, 0, 0, 0, 0, 0};
        if (t < n) {
            // Sixteen rows' values requested at once (one register each),
            // then their products.
            for (int i0 = 0; i0 < nl; i0 += 16) {
                float kv[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int l = list[min(i0 + j, nl - 1)];
                    kv[j] = at_byte(K, (uint32_t)(l * ldk + t) * 4u);
                }
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (i0 + j < nl) {
                        const int l = list[i0 + j];
                        for (int m = 0; m < 6; ++m) acc[m] += (double)kv[j] * zl[l][m];
                    }
            }
        }
#pragma unroll 1
        for (int q = 0, m1 = 0, m2 = 0; q < 21; ++q) {
            double v = mine ? 0.5 * (zl[t][m1] * acc[m2] + zl[t][m2] * acc[m1]) : 0.0;
            for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k);
            if (lane == 0) wpart[w][q] = v;
            if (++m2 == 6) m2 = ++m1;
        }
        __syncthreads();
        if (t < 21) {
            double g = wpart[0][t];
            for (int i = 1; i < NW; ++i) g += wpart[i][t];
            G[t] += g;
        }
    }
    __syncthreads();
    if (t < 36) {
        // Full symmetric matrix from the 21 sums.
        const int i = t / 6, j = t % 6, lo = min(i, j), hi = max(i, j);
        Bfull[t] = G[lo * 6 - lo * (lo - 1) / 2 + (hi - lo)];
    }
    __syncthreads();
    if (t < 64) spd_inverse6_wave(Bfull, out);
}

// Tabulated coarse matrices for problems whose only constraints are clamped
// bottom / top faces.  Every cell of a type then has the same free DoFs,
// and its DoFs split into the same pieces wherever it sits, given its class
// (whether its right face, and its top face, belong to the next aggregate).
// Rigid modes in aggregate coordinates are the cell-local ones times a 6x6
// shift T (translations unchanged; the rotations about the aggregate corner
// gain the translations times the cell's offset), so a cell's part of B_a is
// T^T G T with G = Z^T K_r Z of the piece in cell-local coordinates.

// G[type][flags][class][piece][21] for one (type, class) per workgroup and
// clamp flags `flags`: row t of K_r Z over the cell's free DoFs of t's own
// piece (FP32 K_r, FP64 sums, sixteen rows' values in flight), the row's
// share of the symmetric 21 terms, then per piece the sums over the rows in
// a fixed order (waves in order).  NTH >= n threads.
struct TypeSpacing {
    double h[MAX_TYPES][4];  // coarse-coordinate node spacing per axis (x pitch = 1) and skew of each cell type
};
template <int NTH>
__global__ __launch_bounds__(NTH) void k_coarse_table(const void *const *kr32_tab, const int32_t *surf, int n,
                                                      int ldk, int nx, int ny, int nz, TypeSpacing hs, int flags,
                                                      double *ctab) {
    constexpr int NW = NTH / 64;
    const int type = blockIdx.x, cls = blockIdx.y, t = threadIdx.x, w = t / 64, lane = t % 64;
    const float *K = static_cast<const float *>(kr32_tab[type]);
    const double h0 = hs.h[type][0], h1 = hs.h[type][1], h2 = hs.h[type][2], skew = hs.h[type][3];
    __shared__ double zl[NTH][6];
    __shared__ int8_t pc[NTH];
    __shared__ double wpart[NW][4][21];
    int piece = -1;
    double z[6] = {0, 0, 0, 0, 0, 0};
    if (t < n) {
        const int sn = t / 3, ci = t % 3;
        const int i = surf[3 * sn], j = surf[3 * sn + 1], k = surf[3 * sn + 2];
        const bool fixed = ((flags & MOS_BC_CLAMP_BOTTOM) && k == 0) || ((flags & MOS_BC_CLAMP_TOP) && k == nz - 1);
        if (!fixed) {
            piece = ((cls & 1) && i == nx - 1 ? 1 : 0) + ((cls & 2) && j == ny - 1 ? 2 : 0);
            const double Y = j * h1, Zc = k * h2;
            const double X = i * h0 + skew * Y;
            z[ci] = 1.0;
            if (ci == 0) {
                z[3] = -Y;
                z[5] = Zc;
            } else if (ci == 1) {
                z[3] = X;
                z[4] = -Zc;
            } else {
                z[4] = Y;
                z[5] = -X;
            }
        }
    }
    for (int m = 0; m < 6; ++m) zl[t][m] = z[m];
    pc[t] = (int8_t)piece;
    __syncthreads();
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (piece >= 0) {
        for (int l0 = 0; l0 < n; l0 += 16) {
            float kv[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) kv[j] = K[(size_t)min(l0 + j, n - 1) * ldk + t];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int l = l0 + j;
                if (l < n && pc[l] == piece)
                    for (int m = 0; m < 6; ++m) acc[m] += (double)kv[j] * zl[l][m];
            }
        }
    }
    for (int p = 0; p < 4; ++p) {
#pragma unroll 1
        for (int q = 0, m1 = 0, m2 = 0; q < 21; ++q) {
            double v = piece == p ? 0.5 * (z[m1] * acc[m2] + z[m2] * acc[m1]) : 0.0;
            for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k);
            if (lane == 0) wpart[w][p][q] = v;
            if (++m2 == 6) m2 = ++m1;
        }
    }
    __syncthreads();
    if (t < 84) {
        const int p = t / 21, q = t % 21;
        double g = wpart[0][p][q];
        for (int i = 1; i < NW; ++i) g += wpart[i][p][q];
        ctab[((((size_t)type * 4 + flags) * 4 + cls) * 4 + p) * 21 + q] = g;
    }
}

// Aggregate column of lattice column I: box column times MAXA plus the
// aggregate within the box.
__device__ __forceinline__ int agg_column(const AggLayout &A, int Nx, int64_t I) {
    const int gx = agg_x(A, I);
    const int cells = gx == A.nax - 1 ? Nx - A.cx * (A.nax - 1) : A.cx;
    const int na = (cells + AGG_C - 1) / AGG_C;
    const int ib = (int)(I - (int64_t)gx * A.wxi);
    return gx * MAXA + min(ib / (AGG_C * A.sx), na - 1);
}

// B_a^-1 of every aggregate of the selected problems with tabulated coarse
// matrices; grid (boxes, MAXA), one wave per aggregate.  Lane q < 21 sums
// term q of T^T G T over the touching cells in (cy, cx) order, G the cell's
// table entry for its type, the problem's clamps, its class and the piece
// this aggregate holds (left / lower neighbours hold their right / top
// face), T its shift from the cell corner to the aggregate corner.
__global__ __launch_bounds__(64) void k_coarse_agg_tab(ProbSel sel, const int4 *box_tab, const ProbParams *pp,
                                                       const int32_t *cslot, const int32_t *sb_rom,
                                                       const double *ctab, const uint8_t *cmask,
                                                       const int32_t *surf, int n, double *binv,
                                                       int32_t *agg_gen) {
    const int bs = blockIdx.x, a = blockIdx.y;
    const int pb = box_tab[bs].w;
    if (pb < 0 || !selected(sel, pb)) return;
    const ProbParams &P = pp[pb];
    if (!P.tab_coarse) return;
    const AggLayout &A = P.agg;
    const int b = bs - P.box_begin, gx = b % A.nax, gy = b / A.nax;
    const int bx0 = gx * A.cx, bx1 = gx == A.nax - 1 ? P.lat.Nx : bx0 + A.cx;
    const int by0 = gy * A.cy, by1 = gy == A.nay - 1 ? P.lat.Ny : by0 + A.cy;
    const int na = (bx1 - bx0 + AGG_C - 1) / AGG_C;
    double *out = binv + ((size_t)bs * MAXA + a) * 36;
    const int t = threadIdx.x;
    if (a >= na) {
        if (t < 36) out[t] = 0.0;
        if (t == 0) agg_gen[(size_t)bs * MAXA + a] = 0;
        return;
    }
    const int ax0 = bx0 + a * AGG_C, ax1 = min(ax0 + AGG_C, bx1);
    const int Nx = P.lat.Nx, sx = A.sx, sy = A.sy;
    int flags = P.clamp & 3;
    if (P.tab_coarse == 2) {
        // Problems with a prescribed list: the table applies to this
        // aggregate when its DoFs in the touching cells are constrained
        // exactly on whole bottom / top planes (each plane all or none) and
        // nowhere else; otherwise the general kernel builds B_a.
        int c0 = 0, n0 = 0, cT = 0, nT = 0, cM = 0;
        for (int cy = max(by0 - 1, 0); cy < by1; ++cy)
            for (int cx = max(ax0 - 1, 0); cx < ax1; ++cx)
                for (int k = t; k < n; k += 64) {
                    const int sn = k / 3;
                    const int64_t I = (int64_t)cx * sx + surf[3 * sn], J = (int64_t)cy * sy + surf[3 * sn + 1];
                    const int Kz = surf[3 * sn + 2];
                    if (agg_column(A, Nx, I) != gx * MAXA + a || agg_y(A, J) != gy) continue;
                    const bool con = cmask[P.d0 + 3 * agg_encode(A, I, J, Kz) + k % 3] != 0;
                    if (Kz == 0) {
                        ++n0;
                        c0 += con;
                    } else if (Kz == A.Z - 1) {
                        ++nT;
                        cT += con;
                    } else {
                        cM += con;
                    }
                }
        for (int o = 32; o >= 1; o >>= 1) {
            c0 += __shfl_xor(c0, o);
            n0 += __shfl_xor(n0, o);
            cT += __shfl_xor(cT, o);
            nT += __shfl_xor(nT, o);
            cM += __shfl_xor(cM, o);
        }
        const bool ok = cM == 0 && (c0 == 0 || c0 == n0) && (cT == 0 || cT == nT);
        if (t == 0) agg_gen[(size_t)bs * MAXA + a] = ok ? 0 : 1;
        if (!ok) return;
        flags = (c0 > 0 ? MOS_BC_CLAMP_BOTTOM : 0) | (cT > 0 ? MOS_BC_CLAMP_TOP : 0);
    }
    __shared__ double Bfull[36];
    if (t < 21) {
        // Term q = (m1, m2), m1 <= m2, of the symmetric 6x6.
        int m1 = 0, r = t;
        while (r >= 6 - m1) {
            r -= 6 - m1;
            ++m1;
        }
        const int m2 = m1 + r;
        double g = 0.0;
        for (int cy = max(by0 - 1, 0); cy < by1; ++cy)
            for (int cx = max(ax0 - 1, 0); cx < ax1; ++cx) {
                const int cell = cy * Nx + cx;
                const int slot = cslot[(int64_t)P.sb_begin * 16 + cell];
                const int type = sb_rom[slot / 16];
                const int rx = agg_column(A, Nx, (int64_t)(cx + 1) * sx) != agg_column(A, Nx, (int64_t)cx * sx);
                const int ry = agg_y(A, (int64_t)(cy + 1) * sy) != agg_y(A, (int64_t)cy * sy);
                const int piece = (cx < ax0 ? 1 : 0) + (cy < by0 ? 2 : 0);
                const double *G = ctab + ((((size_t)type * 4 + flags) * 4 + (rx + 2 * ry)) * 4 + piece) * 21;
                // Offsets of the cell corner from the aggregate corner, in the
                // coarse coordinates (x pitch = 1).
                const double Y0 = (double)((cy - by0) * sy) * P.h[1];
                const double X0 = (double)((cx - ax0) * sx) * P.h[0] + P.h[3] * Y0;
                // Column m of T: (row, coefficient) pairs.
                int ri[2][3];
                double rc[2][3];
                int nr[2];
                const int mm[2] = {m1, m2};
                for (int u = 0; u < 2; ++u) {
                    const int m = mm[u];
                    ri[u][0] = m;
                    rc[u][0] = 1.0;
                    nr[u] = 1;
                    if (m == 3) {
                        ri[u][1] = 0;
                        rc[u][1] = -Y0;
                        ri[u][2] = 1;
                        rc[u][2] = X0;
                        nr[u] = 3;
                    } else if (m == 4) {
                        ri[u][1] = 2;
                        rc[u][1] = Y0;
                        nr[u] = 2;
                    } else if (m == 5) {
                        ri[u][1] = 2;
                        rc[u][1] = -X0;
                        nr[u] = 2;
                    }
                }
                double v = 0.0;
                for (int u = 0; u < nr[0]; ++u)
                    for (int w = 0; w < nr[1]; ++w) {
                        const int lo = min(ri[0][u], ri[1][w]), hi = max(ri[0][u], ri[1][w]);
                        v += rc[0][u] * rc[1][w] * G[lo * 6 - lo * (lo - 1) / 2 + (hi - lo)];
                    }
                g += v;
            }
        Bfull[m1 * 6 + m2] = g;
        Bfull[m2 * 6 + m1] = g;
    }
    __syncthreads();
    spd_inverse6_wave(Bfull, out);
}

// ---- batched per-problem phases (set-up, FP64 residual, sweep start/stop) ----
// Kernels over DoF blocks [0, high water) act on the blocks of selected
// problems only; per problem they do exactly what a single-problem launch
// would, so batching never changes a problem's results.

// Problem id of every DoF block and slot block of the listed problems.
__global__ void k_fill_owner(PidList L, const ProbParams *pp, int32_t *blk_prob, int32_t *sb_prob,
                             int4 *box_tab) {
    const int p = L.pid[blockIdx.x];
    const ProbParams &P = pp[p];
    for (int i = threadIdx.x; i < P.n_blk; i += blockDim.x) blk_prob[P.blk_begin + i] = p;
    for (int i = threadIdx.x; i < P.n_sb; i += blockDim.x) sb_prob[P.sb_begin + i] = p;
    if (P.box_begin >= 0)
        for (int i = threadIdx.x; i < P.n_agg; i += blockDim.x) {
            int64_t first;
            int nn, na;
            box_geometry(P, i, first, nn, na);
            box_tab[P.box_begin + i] = make_int4((int)first, nn, na, p);
        }
}

// Constrained DoFs: padding and, when clamped, the nodes of the bottom and
// top planes (value 0); the problem's incidence region doubles as the "last
// entry" table of its prescribed list, reset to -1.
__global__ void k_setup_dofs(ProbSel sel, const int32_t *blk_prob, const ProbParams *pp, uint8_t *cmask, double *g,
                             double *x64, int32_t *inc) {
    const int p = blk_prob[blockIdx.x];
    if (!selected(sel, p)) return;
    const ProbParams &P = pp[p];
    const int64_t d = (int64_t)blockIdx.x * DB + threadIdx.x, i = d - P.d0;
    bool c = i >= P.n_dofs;
    if (!c && P.clamp) {
        int64_t I, J;
        int K;
        agg_decode(P.agg, i / 3, I, J, K);
        c = ((P.clamp & MOS_BC_CLAMP_BOTTOM) && K == 0) || ((P.clamp & MOS_BC_CLAMP_TOP) && K == P.agg.Z - 1);
    }
    cmask[d] = c ? 1 : 0;
    g[d] = 0.0;
    x64[d] = 0.0;
    inc[P.d0 / 3 * 4 + i] = -1;
}

// Incidence entries of the selected problems' nodes reset to -1.
__global__ void k_clear_incidence(ProbSel sel, const int32_t *blk_prob, int32_t *inc, int32_t *inc2, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (selected(sel, blk_prob[(i / 4 * 3) / DB])) {
            inc[i] = -1;
            inc2[i] = -1;
        }
}

// Node -> (slot, surface node) incidence of the selected problems, entries
// in ascending cell id.  A node on a shared vertical face or edge belongs to
// 2 or 4 cells; the rank of cell (cx, cy) among them follows from which side
// of the face it lies.
__global__ void k_incidence_sel(ProbSel sel, const int32_t *sb_prob, const ProbParams *pp, const int32_t *perm,
                                int32_t *inc, int32_t *inc2, uint32_t *lc, int32_t *cslot, const uint8_t *cmask,
                                const int32_t *surf, int S, int64_t n_slots) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_slots * S) return;
    const int slot = (int)(idx / S), s = (int)(idx % S);
    const int p = sb_prob[slot / 16];
    if (!selected(sel, p)) return;
    const int32_t cell = perm[slot];
    if (cell < 0) return;
    const Lattice &L = pp[p].lat;
    const int cx = cell % L.Nx, cy = (cell / L.Nx) % L.Ny, cz = cell / (L.Nx * L.Ny);
    const int i = surf[3 * s], j = surf[3 * s + 1], k = surf[3 * s + 2];
    const AggLayout &A = pp[p].agg;
    const int64_t I = (int64_t)cx * (L.nx - 1) + i, J = (int64_t)cy * (L.ny - 1) + j;
    const int K = cz * (L.nz - 1) + k;
    const int64_t node = agg_encode(A, I, J, K);
    if (s == 0) cslot[(int64_t)pp[p].sb_begin * 16 + cell] = slot;
    if (pp[p].box_begin >= 0) {
        // Aggregate-local coordinates of the node (two-level preconditioner).
        const int gx = agg_x(A, I), gy = agg_y(A, J);
        const int cells = gx == A.nax - 1 ? L.Nx - A.cx * (A.nax - 1) : A.cx;
        const int na = (cells + AGG_C - 1) / AGG_C;
        const int ib = (int)(I - (int64_t)gx * A.wxi);
        const int ag = min(ib / (AGG_C * A.sx), na - 1);
        const uint32_t ia = (uint32_t)(ib - ag * AGG_C * A.sx), jb = (uint32_t)(J - (int64_t)gy * A.wyi);
        const int64_t dn = pp[p].d0 + 3 * node;
        const uint32_t cm = (cmask[dn] ? 1u : 0u) | (cmask[dn + 1] ? 2u : 0u) | (cmask[dn + 2] ? 4u : 0u);
        lc[pp[p].d0 / 3 + node] = ia | jb << 8 | (uint32_t)k << 16 | (uint32_t)ag << 24 | cm << 28;
    }
    const bool shx = (i == 0 && cx > 0) || (i == L.nx - 1 && cx < L.Nx - 1);
    const int ux = (i == 0 && cx > 0) ? 1 : 0;
    const int uy = (j == 0 && cy > 0) ? 1 : 0;
    // The bottom face of a block above the first layer is the top face of
    // the block below: that node's cells of this (upper) layer go to inc2.
    int32_t *dst = (k == 0 && cz > 0) ? inc2 : inc;
    dst[(pp[p].d0 / 3 + node) * 4 + uy * (shx ? 2 : 1) + ux] = (slot << INC_SHIFT) | s;
}

// b_raw = dT * sum over the cells around each DoF of b_r(type), and the
// Jacobi scaling 1 / sum of the K_r(type) diagonals (1 on constrained DoFs).
template <class T>
__global__ void k_rhs_diag(ProbSel sel, const int32_t *blk_prob, const ProbParams *pp,
                           const double *const *br_tab, const void *const *kr64_tab, const int32_t *sb_rom,
                           const int32_t *inc, const int32_t *inc2, const uint8_t *cmask, double *b, T *dinv,
                           int ldk) {
    const int p = blk_prob[blockIdx.x];
    if (!selected(sel, p)) return;
    const int64_t d = (int64_t)blockIdx.x * DB + threadIdx.x;
    const int4 iv = incidence(inc, d), iv2 = incidence2(inc2, d);
    const int e4[8] = {iv.x, iv.y, iv.z, iv.w, iv2.x, iv2.y, iv2.z, iv2.w};
    const int ci = (int)(d % 3);
    double sb = 0.0, sd = 0.0;
    for (int e = 0; e < 8; ++e)
        if (e4[e] >= 0) {
            const int rom = sb_rom[(e4[e] >> INC_SHIFT) / 16];
            const int k = 3 * (e4[e] & MAX_SURF) + ci;
            sb += br_tab[rom][k];
            sd += static_cast<const double *>(kr64_tab[rom])[(size_t)k * ldk + k];
        }
    b[d] = pp[p].dT * sb;
    const int64_t i = d - pp[p].d0;
    if (i < pp[p].n_dofs)
        dinv[inner_index(pp[p], i / 3, (int)(i % 3))] = (cmask[d] || sd == 0.0) ? T(1) : T(1.0 / sd);
    else if (pp[p].box_begin < 0)
        dinv[d] = T(1);
}

// FP64 vector of the selected problems to the cell-major layout.
__global__ void k_scatter_sel(ProbSel sel, const int32_t *blk_prob, const double *v, const int32_t *inc,
                              const int32_t *inc2, double *Mc, int ld_slots) {
    if (!selected(sel, blk_prob[blockIdx.x])) return;
    const int64_t d = (int64_t)blockIdx.x * DB + threadIdx.x;
    cell_scatter(Mc, incidence(inc, d), (int)(d % 3), ld_slots, v[d]);
    if (inc2) cell_scatter(Mc, incidence2(inc2, d), (int)(d % 3), ld_slots, v[d]);
}

// True residual of the lifted system r = b - A x (0 on constrained DoFs),
// A x assembled from the FP64 cell products, and per-block partials of
// ||r||^2 and, with `lift`, of ||b_l||^2 (b_l = g on constrained DoFs,
// b - A g elsewhere; at set-up x = g).
__global__ void k_residual_sel(ProbSel sel, const int32_t *blk_prob, const double *Y, const int32_t *inc,
                               const int32_t *inc2, const double *b_raw, const uint8_t *cmask, const double *g,
                               double *r, double *part_r, double *part_b, int lift, int ld_slots) {
    if (!selected(sel, blk_prob[blockIdx.x])) return;
    const int64_t d = (int64_t)blockIdx.x * DB + threadIdx.x;
    double ax = cell_sum(Y, incidence(inc, d), (int)(d % 3), ld_slots);
    if (inc2) ax += cell_sum(Y, incidence2(inc2, d), (int)(d % 3), ld_slots);
    const bool c = cmask[d];
    const double v = c ? 0.0 : b_raw[d] - ax;
    r[d] = v;
    double a = v * v, bl = 0.0, z = 0.0;
    if (lift) {
        const double w = c ? g[d] : v;
        bl = w * w;
    }
    block_sum3(a, bl, z);
    if (threadIdx.x == 0) {
        part_r[blockIdx.x] = a;
        if (lift) part_b[blockIdx.x] = bl;
    }
}

// dst[p] = fixed-order sum of the partials of problem p's DoF blocks, for
// each listed p (one block each); a second array with `part2`.
__global__ void k_reduce_list(PidList L, const ProbParams *pp, const double *part, double *dst, const double *part2,
                              double *dst2) {
    if (threadIdx.x >= 64) return;
    const int p = L.pid[blockIdx.x];
    const int b0 = pp[p].blk_begin, b1 = b0 + pp[p].n_blk;
    double a, b, c;
    wave_sum3(part, part2 ? part2 : part, part, b0, b1, a, b, c);
    if (threadIdx.x == 0) {
        dst[p] = a;
        if (part2) dst2[p] = b;
    }
}

// Sweep start, per listed problem: fresh scalar state.
__global__ void k_prob_start_list(PidList L, const ProbParams *pp, const SweepParams *sp, ProbState *ps, int epoch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int p = L.pid[i];
    ProbState &S = ps[p];
    if (sp[p].cont) {
        // Reliable update: the iteration goes on from where it stopped with
        // the true residual in place of the recursive one; the kept (r,u)
        // history follows the new scaling (alpha is scale-free).
        const double c2 = sp[p].p_scale * sp[p].p_scale;
        S.hist_gamma[0] *= c2;
        S.hist_gamma[1] *= c2;
    } else {
        S.hist_gamma[0] = S.hist_gamma[1] = S.hist_alpha[0] = S.hist_alpha[1] = 0.0;
        S.it = 0;
    }
    S.seg_start = S.it;
    S.start_epoch = epoch - S.it;
    S.a_cur = S.b_cur = S.rr = S.tol2 = 0.0;
    S.fused = pp[p].fused;
    S.rtol2 = sp[p].rtol2;
    S.done = 0;
    S.active = 1;
    S.max_iter = sp[p].max_iter;
    S.blk_begin = pp[p].part_begin;
    S.blk_end = pp[p].part_begin + pp[p].n_part;
    S.tile_begin = pp[p].sb_begin * pp[p].nrb;
    S.tile_end = (pp[p].sb_begin + pp[p].n_sb) * pp[p].nrb;
}

__global__ void k_prob_stop_list(PidList L, ProbState *ps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L.n) ps[L.pid[i]].active = 0;
}

// Sweep start: inner right-hand side r = scale_in * r64 (in T), x = p = s =
// 0, u = M^-1 r to the cell layout, partials of (r,u) and (r,r); the first
// iteration's cell GEMM then gives w = A u and (u, A u).
template <class T>
__global__ void k_cgstart_sel(ProbSel sel, const int32_t *blk_prob, const SweepParams *sp, const ProbState *ps,
                              const double *r64, const T *dinv, const int32_t *inc, const int32_t *inc2, T *x, T *r,
                              T *p, T *s, T *Mc, int ld_slots, double *pg, double *pr, int cap_blk) {
    const int pid = blk_prob[blockIdx.x];
    if (!selected(sel, pid)) return;
    const int64_t d = (int64_t)blockIdx.x * DB + threadIdx.x;
    const SweepParams &W = sp[pid];
    const T rv = (T)(r64[d] * W.scale_in);
    const T uv = dinv[d] * rv;
    x[d] = 0;
    r[d] = rv;
    if (W.cont) {
        const T c = (T)W.p_scale;
        p[d] *= c;
        s[d] *= c;
    } else {
        p[d] = 0;
        s[d] = 0;
    }
    cell_scatter(Mc, incidence(inc, d), (int)(d % 3), ld_slots, uv);
    if (inc2) cell_scatter(Mc, incidence2(inc2, d), (int)(d % 3), ld_slots, uv);
    double g = (double)rv * (double)uv, r2 = (double)rv * (double)rv, z = 0.0;
    block_sum3(g, r2, z);
    if (threadIdx.x == 0) {
        // Partials of the first iteration of the sweep, in its parity slot.
        const size_t slot = (size_t)(ps[pid].it & 1) * cap_blk;
        pg[slot + blockIdx.x] = g;
        pr[slot + blockIdx.x] = r2;
    }
}

// Zeros in the cell-layout columns of the selected problems' padding slots
// (no node refers to them, so nothing else ever writes them there).
__global__ void k_zero_padding(ProbSel sel, const int32_t *sb_prob, const int32_t *perm, uint8_t *Mc, int elem,
                               int ld_slots, int ldk, int64_t n_slots) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_slots * ldk) return;
    const int64_t slot = idx % n_slots;
    const int k = (int)(idx / n_slots);
    if (!selected(sel, sb_prob[slot / 16]) || perm[slot] >= 0) return;
    uint8_t *q = Mc + ((size_t)k * ld_slots + slot) * elem;
    if (elem == 8)
        *reinterpret_cast<double *>(q) = 0.0;
    else
        *reinterpret_cast<float *>(q) = 0.0f;
}

// x64 += sign * scale_out * dx on the selected problems (fold in a sweep's
// correction, or take it back).
template <class T>
__global__ void k_add_inner_sel(ProbSel sel, const int32_t *blk_prob, const ProbParams *pp, const SweepParams *sp,
                                double *x64, const T *dx, double sign) {
    const int pid = blk_prob[blockIdx.x];
    if (!selected(sel, pid)) return;
    const int64_t d = (int64_t)blockIdx.x * DB + threadIdx.x, i = d - pp[pid].d0;
    if (i < pp[pid].n_dofs) x64[d] += sign * sp[pid].scale_out * (double)dx[inner_index(pp[pid], i / 3, (int)(i % 3))];
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---- problem set-up on the device (numbering contract of the abstract mesh) ----

// Prescribed (DoF, value) list, a later entry overriding an earlier one: the
// largest entry index per DoF wins, then only that entry is applied.
// Last entry of the list for each DoF (a later entry overrides an earlier
// one).  Entries with a DoF outside [0, n_dofs) or a non-finite value are
// left out and raise *bad (lists checked on the host never hold one).
__global__ void k_prescribe_last(const int64_t *dof, const double *val, int64_t n, int64_t n_dofs, int32_t *last,
                                 int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t d = dof[i];
    if (d < 0 || d >= n_dofs || !isfinite(val[i])) {
        *bad = 1;
        return;
    }
    atomicMax(&last[d], (int32_t)i);
}

// DoF of the internal order for a DoF of the caller's order.
__device__ __forceinline__ int64_t internal_dof(const SubLattice &W, const AggLayout &A, int64_t dof) {
    int i, j, K;
    sub_decode(W, dof / 3, i, j, K);
    return 3 * agg_encode(A, i, j, K) + dof % 3;
}

// Prescribed values applied (the list holds DoFs of the caller's order).
__global__ void k_prescribe(const int64_t *dof, const double *val, int64_t n, int64_t n_dofs, const int32_t *last,
                            uint8_t *cmask, double *g, double *x64, int64_t d0, SubLattice W, AggLayout A) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || dof[i] < 0 || dof[i] >= n_dofs || last[dof[i]] != (int32_t)i) return;
    const int64_t d = d0 + internal_dof(W, A, dof[i]);
    cmask[d] = 1;
    g[d] = val[i];
    x64[d] = val[i];
}

// Solution in the caller's DoF order from the internal order.
__global__ void k_export_u(const double *x, double *u, int64_t n_dofs, SubLattice W, AggLayout A) {
    const int64_t dof = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (dof < n_dofs) u[dof] = x[internal_dof(W, A, dof)];
}

// Global DoF of cell DoF k in slot sl ([ldk][n_slots], -1 for padding).
__global__ void k_gather_index(int32_t *gidx, const int32_t *perm, int64_t n_slots, int ldk, int n,
                               const int32_t *surf, Lattice L) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)ldk * n_slots) return;
    const int k = (int)(idx / n_slots);
    const int64_t sl = idx % n_slots;
    const int32_t cell = perm[sl];
    if (cell < 0 || k >= n) {
        gidx[idx] = -1;
        return;
    }
    const int s = k / 3;
    const int cx = cell % L.Nx, cy = (cell / L.Nx) % L.Ny, cz = cell / (L.Nx * L.Ny);
    const int64_t node = node_id(L, (int64_t)cx * (L.nx - 1) + surf[3 * s], (int64_t)cy * (L.ny - 1) + surf[3 * s + 1],
                                 (int64_t)cz * (L.nz - 1) + surf[3 * s + 2]);
    gidx[idx] = (int32_t)(3 * node + k % 3);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

}  // namespace

// ---- first-fit range allocator ----
void RangeAlloc::init(int c) {
    cap = c;
    high = 0;
    free_.clear();
    if (c > 0) free_[0] = c;
}

int RangeAlloc::take(int n) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
        if (it->second >= n) {
            int b = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[b + n] = len - n;
            high = std::max(high, b + n);
            return b;
        }
    return -1;
}

void RangeAlloc::give(int b, int n) {
    auto it = free_.emplace(b, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_.erase(nx);
    }
    if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_.erase(it);
        }
    }
    // Allocated space is the complement of the free ranges.
    auto last = std::prev(free_.end());
    high = (last->first + last->second == cap) ? last->first : cap;
}

namespace {

// DoF blocks of a problem: its DoFs, and at least one block per aggregate
// (an aggregate's partials go to the slot of its block index); a multiple
// of 3 so every problem starts on a node boundary.
int problem_blocks(int64_t n_dofs, int n_agg) {
    return (int)std::max(round_up(n_dofs, DOF_ALIGN) / DB, round_up(n_agg, 3));
}

mos_status prepare_problem(mos_engine e, const mos_array_desc *d, EngineProblem *P) {
    const mos_cell_desc &cd = e->roms[0]->desc;
    const int Nz = d->nz_cells < 1 ? 1 : d->nz_cells;
    const Lattice L = make_lattice(d->nx_cells, d->ny_cells, cd.interp[0], cd.interp[1], cd.interp[2], Nz);
    P->lat = L;
    P->Nx = d->nx_cells;
    P->Ny = d->ny_cells;
    P->Nz = Nz;
    P->n_cells = (int64_t)P->Nx * P->Ny * Nz;
    P->n_nodes = L.n_nodes;
    P->n_dofs = 3 * L.n_nodes;
    P->dT = d->delta_T;
    const bool mixed = e->precision == MOS_MIXED;
    P->rtol = d->rtol > 0 ? d->rtol : (mixed ? 1e-10 : 1e-12);
    P->max_iters = d->max_iters > 0 ? d->max_iters : 20000;
    P->agg = make_agg_layout(L, e->box_cells[0], e->box_cells[1]);
    P->n_agg = agg_count(P->agg);
    P->n_blk = problem_blocks(P->n_dofs, P->n_agg);
    P->bc_flags = d->bc_flags & (MOS_BC_CLAMP_BOTTOM | MOS_BC_CLAMP_TOP);
    if (d->n_prescribed > INT32_MAX) {
        set_error("more than 2^31-1 prescribed entries");
        return MOS_EINVAL;
    }
    P->n_pres = d->n_prescribed;
    if (d->bc_flags & MOS_BC_LIST_ON_DEVICE) {
        // Device-resident list: read at set-up and checked there.
        P->dpdof = d->n_prescribed ? d->prescribed_dof : nullptr;
        P->dpval = d->n_prescribed ? d->prescribed_value : nullptr;
    } else {
        P->pdof.assign(d->prescribed_dof, d->prescribed_dof + d->n_prescribed);
        P->pval.assign(d->prescribed_value, d->prescribed_value + d->n_prescribed);
        for (int64_t i = 0; i < d->n_prescribed; ++i)
            if (P->pdof[i] < 0 || P->pdof[i] >= P->n_dofs || !std::isfinite(P->pval[i])) {
                set_error("prescribed entry %lld: DoF %lld outside [0, %lld) or value not finite", (long long)i,
                          (long long)P->pdof[i], (long long)P->n_dofs);
                return MOS_EINVAL;
            }
    }
    if (P->bc_flags == 0 && d->n_prescribed == 0) {
        set_error("array has no constrained DoF: the reduced stiffness is singular (rigid motions)");
        return MOS_ESINGULAR;
    }
    // Cells grouped by type, each type padded to 16 slots.
    const int n_roms = (int)e->roms.size();
    std::vector<int> count(n_roms, 0);
    for (int64_t c = 0; c < P->n_cells; ++c) count[d->cell_type[c]]++;
    P->seg.assign(n_roms + 1, 0);
    for (int t = 0; t < n_roms; ++t) P->seg[t + 1] = P->seg[t] + ceil_div(count[t], 16);
    P->n_sb = std::max(P->seg[n_roms], 1);
    P->perm.assign((size_t)P->n_sb * 16, -1);
    std::vector<int> next(n_roms);
    for (int t = 0; t < n_roms; ++t) next[t] = P->seg[t] * 16;
    // Within a type, slots follow the aggregates (cells of one aggregate in
    // neighbouring slots, its layers one after another), as the DoFs do: the
    // update's gathers and scatters for an aggregate then fall in a few cache
    // lines per cell-layout row.
    const AggLayout &A = P->agg;
    for (int gy = 0; gy < A.nay; ++gy)
        for (int gx = 0; gx < A.nax; ++gx) {
            const int cy1 = gy == A.nay - 1 ? P->Ny : (gy + 1) * A.cy;
            const int cx1 = gx == A.nax - 1 ? P->Nx : (gx + 1) * A.cx;
            for (int cz = 0; cz < Nz; ++cz)
                for (int cy = gy * A.cy; cy < cy1; ++cy)
                    for (int cx = gx * A.cx; cx < cx1; ++cx) {
                        const int64_t c = ((int64_t)cz * P->Ny + cy) * P->Nx + cx;
                        P->perm[next[d->cell_type[c]]++] = (int32_t)c;
                    }
        }
    P->sb_rom.assign(P->n_sb, -1);
    for (int t = 0; t < n_roms; ++t)
        for (int b = P->seg[t]; b < P->seg[t + 1]; ++b) P->sb_rom[b] = t;
    return MOS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Engine internals
// ---------------------------------------------------------------------------
namespace {

// Relative residual reduction asked of one FP32 inner solve.  FP32 PCG in
// this form tracks its true residual to below 1e-4 on these systems.  A
// target of 3e-4 per sweep reaches 1e-10 in three sweeps for two percent more
// iterations than 1e-2 (five sweeps), and was the fastest in time: each sweep
// costs an FP64 residual, a restart and a host decision.
constexpr double INNER_RTOL_F32 = 3e-4;

// Problems with at most this many partials (DoF blocks + GEMM tiles) have
// every update workgroup reduce them itself instead of a separate launch.
constexpr int64_t CG_FUSE_MAX = 8192;

// Problems taking part in one batched phase.
struct Batch {
    ProbSel sel{};
    PidList list{};
    void add(int p) {
        sel.bits[p >> 5] |= 1u << (p & 31);
        list.pid[list.n++] = (int16_t)p;
    }
    bool empty() const { return list.n == 0; }
};

// The host mirrors (pp_host, sb_rom_host, perm_host) may change only once
// the last span copy out of them has run.
mos_status mirror_wait(mos_engine e) {
    MOS_HIP(hipEventSynchronize(e->mirror_ev));
    return MOS_OK;
}

// FP64 true residual of the batch's problems into r64 and res2[p] (and, at
// set-up, ||b_l||^2 into bb2[p]), from x64 scattered to the cell layout --
// which is where the reconstruction later reads the solution.
mos_status residual_batch(mos_engine e, const Batch &B, bool lift) {
    hipStream_t st = e->ctx->stream;
    const int hw_blk = e->blk.high, hw_sb = e->sbs.high;
    hipLaunchKernelGGL(k_scatter_sel, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                       (const double *)e->x64, (const int32_t *)e->inc, (const int32_t *)(e->stacked ? e->inc2 : nullptr), e->Mc64, e->ld_slots);
    // The K_r-stationary variants share one FP64 product here (operand tiles
    // in LDS), so all of them give the same residual bits.
    if (e->gemm_rows)
        MOS_TRY(launch_cell_gemm<double>(e->ctx, 0, 1, e->ldk / 4, e->n, 1, st, (const void *const *)e->kr64_tab, e->sb_rom,
                                         e->sb_prob, (const double *)e->Mc64, e->Y64, e->ld_slots, hw_sb,
                                         (const ProbState *)e->ps, (double *)nullptr, 2, B.sel));
    else
        hipLaunchKernelGGL(k_bgemm<double>, dim3(e->ldk / 16, hw_sb), dim3(256), 0, st,
                           (const void *const *)e->kr64_tab, e->sb_rom, e->sb_prob, (const double *)e->Mc64, e->Y64,
                           e->ldk, e->ld_slots, 0, hw_sb, 2, (const ProbState *)e->ps, (double *)nullptr, B.sel);
    hipLaunchKernelGGL(k_residual_sel, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                       (const double *)e->Y64, (const int32_t *)e->inc, (const int32_t *)(e->stacked ? e->inc2 : nullptr), (const double *)e->b_raw,
                       (const uint8_t *)e->cmask, (const double *)e->g, e->r64, e->pr64, e->pd, lift ? 1 : 0,
                       e->ld_slots);
    hipLaunchKernelGGL(k_reduce_list, dim3(B.list.n), dim3(64), 0, st, B.list, (const ProbParams *)e->pp,
                       (const double *)e->pr64, e->res2, lift ? (const double *)e->pd : (const double *)nullptr,
                       e->bb2);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

// Device set-up of newly admitted problems (tables, constraints, incidence,
// load, Jacobi scaling) and their first residual.  The host sources
// (P->perm, P->sb_rom, P->pdof, P->pval, pp_host[p]) stay put until the
// problem is released.
mos_status setup_batch(mos_engine e, const std::vector<EngineProblem *> &adm, const Batch &B) {
    hipStream_t st = e->ctx->stream;
    MOS_TRY(mirror_wait(e));
    int sb_lo = INT32_MAX, sb_hi = 0;
    // From the first stacked array on, the Jacobi kernels also read the
    // incidence of the layer above (all -1 for one-layer arrays).
    for (EngineProblem *P : adm) e->stacked |= P->Nz > 1 ? 1 : 0;
    for (EngineProblem *P : adm) {
        ProbParams &H = e->pp_host[P->pid];
        const Lattice &L = P->lat;
        H.d0 = (int64_t)P->blk_begin * DB;
        H.n_dofs = P->n_dofs;
        H.nd_pad = (int64_t)P->n_blk * DB;
        H.clamp = (int32_t)P->bc_flags;
        H.agg = P->agg;
        H.n_agg = P->n_agg;
        H.box_begin = P->box_begin;
        H.part_begin = P->box_begin >= 0 ? P->box_begin : P->blk_begin;
        H.n_part = P->box_begin >= 0 ? P->n_agg : P->n_blk;
        {
            // Coordinates of the coarse modes: node spacing over the x pitch
            // of the problem's own cells (every cell of an array shares pitch
            // and height).
            const mos_cell_desc &cd = e->roms[P->sb_rom[0]]->desc;
            H.h[0] = 1.0 / (cd.interp[0] - 1);
            H.h[1] = cd.pitch_y / cd.pitch_x / (cd.interp[1] - 1);
            H.h[2] = cd.height / cd.pitch_x / (cd.interp[2] - 1);
            H.h[3] = cd.skew;
        }
        // Clamped faces only: every cell of a type has the same free DoFs, so
        // its coarse terms come from the per-type table.
        H.tab_coarse = !e->precond ? 0 : P->n_pres == 0 ? 1 : e->coarse_table ? 2 : 0;
        H.dT = P->dT;
        H.lat = L;
        H.blk_begin = P->blk_begin;
        H.n_blk = P->n_blk;
        H.sb_begin = P->sb_begin;
        H.n_sb = P->n_sb;
        H.nrb = e->ldk / 16;
        // Small problems reduce their scalars inside every update workgroup.
        H.fused = (int64_t)P->n_blk + (int64_t)P->n_sb * H.nrb <= CG_FUSE_MAX ? 1 : 0;
        std::memcpy(e->sb_rom_host + P->sb_begin, P->sb_rom.data(), P->n_sb * 4);
        std::memcpy(e->perm_host + (int64_t)P->sb_begin * 16, P->perm.data(), P->perm.size() * 4);
        sb_lo = std::min(sb_lo, P->sb_begin);
        sb_hi = std::max(sb_hi, P->sb_begin + P->n_sb);
    }
    // One copy per table for the whole batch: the spans may cover other
    // problems' ranges, whose mirror entries equal their device entries.
    const int hw_p = e->pids.high;
    MOS_HIP(hipMemcpyAsync(e->pp, e->pp_host, hw_p * sizeof(ProbParams), hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->sb_rom + sb_lo, e->sb_rom_host + sb_lo, (size_t)(sb_hi - sb_lo) * 4,
                           hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->perm + (int64_t)sb_lo * 16, e->perm_host + (int64_t)sb_lo * 16,
                           (size_t)(sb_hi - sb_lo) * 64, hipMemcpyHostToDevice, st));
    MOS_HIP(hipEventRecord(e->mirror_ev, st));
    const int hw_blk = e->blk.high, hw_sb = e->sbs.high;
    hipLaunchKernelGGL(k_fill_owner, dim3(B.list.n), dim3(256), 0, st, B.list, (const ProbParams *)e->pp, e->blk_prob,
                       e->sb_prob, e->box_tab);
    hipLaunchKernelGGL(k_setup_dofs, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                       (const ProbParams *)e->pp, e->cmask, e->g, e->x64, e->inc);
    for (EngineProblem *P : adm) {
        const int64_t np = P->n_pres;
        if (np == 0) continue;
        const int64_t d0 = (int64_t)P->blk_begin * DB;
        const int64_t *pdof = P->dpdof;
        const double *pval = P->dpval;
        if (!pdof) {
            // Host list: one device copy for the problem's lifetime.
            P->dev.ctx = e->ctx;
            int64_t *dd = nullptr;
            double *dv = nullptr;
            MOS_TRY(P->dev.alloc_n(np, &dd));
            MOS_TRY(P->dev.alloc_n(np, &dv));
            MOS_HIP(hipMemcpyAsync(dd, P->pdof.data(), np * 8, hipMemcpyHostToDevice, st));
            MOS_HIP(hipMemcpyAsync(dv, P->pval.data(), np * 8, hipMemcpyHostToDevice, st));
            pdof = dd;
            pval = dv;
        }
        int32_t *last = e->inc + d0 / 3 * 4;
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)(e->pres_bad + P->pid), (int64_t)1, 0u);
        hipLaunchKernelGGL(k_prescribe_last, dim3(ceil_div(np, 256)), dim3(256), 0, st, pdof, pval, np, P->n_dofs,
                           last, e->pres_bad + P->pid);
        hipLaunchKernelGGL(k_prescribe, dim3(ceil_div(np, 256)), dim3(256), 0, st, pdof, pval, np, P->n_dofs,
                           (const int32_t *)last, e->cmask, e->g, e->x64, d0, whole_lattice(P->lat), P->agg);
    }
    const int64_t n_inc = (int64_t)hw_blk * DB / 3 * 4;
    hipLaunchKernelGGL(k_clear_incidence, dim3((unsigned)std::min<int64_t>(ceil_div(n_inc, 256), 4096)), dim3(256),
                       0, st, B.sel, (const int32_t *)e->blk_prob, e->inc, e->inc2, n_inc);
    const int64_t n_slots = (int64_t)hw_sb * 16;
    hipLaunchKernelGGL(k_zero_padding, dim3(ceil_div(n_slots * e->ldk, 256)), dim3(256), 0, st, B.sel,
                       (const int32_t *)e->sb_prob, (const int32_t *)e->perm, (uint8_t *)e->Mc,
                       e->precision == MOS_MIXED ? 4 : 8, e->ld_slots, e->ldk, n_slots);
    hipLaunchKernelGGL(k_incidence_sel, dim3(ceil_div(n_slots * e->S, 256)), dim3(256), 0, st, B.sel,
                       (const int32_t *)e->sb_prob, (const ProbParams *)e->pp, (const int32_t *)e->perm, e->inc,
                       e->inc2, e->lc, e->cslot, (const uint8_t *)e->cmask, (const int32_t *)e->surf, e->S, n_slots);
    if (e->precision == MOS_MIXED)
        hipLaunchKernelGGL(k_rhs_diag<float>, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                           (const ProbParams *)e->pp, (const double *const *)e->br_tab,
                           (const void *const *)e->kr64_tab, (const int32_t *)e->sb_rom, (const int32_t *)e->inc,
                           (const int32_t *)(e->stacked ? e->inc2 : nullptr), (const uint8_t *)e->cmask, e->b_raw, (float *)e->v[VDINV], e->ldk);
    else
        hipLaunchKernelGGL(k_rhs_diag<double>, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                           (const ProbParams *)e->pp, (const double *const *)e->br_tab,
                           (const void *const *)e->kr64_tab, (const int32_t *)e->sb_rom, (const int32_t *)e->inc,
                           (const int32_t *)(e->stacked ? e->inc2 : nullptr), (const uint8_t *)e->cmask, e->b_raw, (double *)e->v[VDINV], e->ldk);
    if (e->precond) {
        bool any_tab = false, any_gen = false;
        for (EngineProblem *P : adm) {
            const ProbParams &H = e->pp_host[P->pid];
            any_tab |= H.tab_coarse != 0;
            any_gen |= H.tab_coarse != 1;
            // Clamp-only problems need the table of their flags; problems
            // with a prescribed list may use any of the four.
            for (int f = 0; f < 4; ++f) {
                const bool need = (H.tab_coarse == 1 && f == (H.clamp & 3)) || H.tab_coarse == 2;
                if (!need || ((e->ctab_built >> f) & 1)) continue;
                TypeSpacing hs{};
                for (size_t t = 0; t < e->roms.size(); ++t) {
                    const mos_cell_desc &cd = e->roms[t]->desc;
                    hs.h[t][0] = 1.0 / (cd.interp[0] - 1);
                    hs.h[t][1] = cd.pitch_y / cd.pitch_x / (cd.interp[1] - 1);
                    hs.h[t][2] = cd.height / cd.pitch_x / (cd.interp[2] - 1);
                    hs.h[t][3] = cd.skew;
                }
                const mos_cell_desc &c0 = e->roms[0]->desc;
                if (e->n <= 256)
                    hipLaunchKernelGGL(k_coarse_table<256>, dim3((unsigned)e->roms.size(), 4), dim3(256), 0, st,
                                       (const void *const *)e->kr32_tab, (const int32_t *)e->surf, e->n, e->ldk,
                                       c0.interp[0], c0.interp[1], c0.interp[2], hs, f, e->ctab);
                else
                    hipLaunchKernelGGL(k_coarse_table<512>, dim3((unsigned)e->roms.size(), 4), dim3(512), 0, st,
                                       (const void *const *)e->kr32_tab, (const int32_t *)e->surf, e->n, e->ldk,
                                       c0.interp[0], c0.interp[1], c0.interp[2], hs, f, e->ctab);
                e->ctab_built |= 1 << f;
            }
        }
        // The tabulated aggregates first: for problems with a prescribed list
        // they mark which aggregates the general kernel still has to build.
        if (any_tab)
            hipLaunchKernelGGL(k_coarse_agg_tab, dim3(e->boxes.high, MAXA), dim3(64), 0, st, B.sel,
                               (const int4 *)e->box_tab, (const ProbParams *)e->pp, (const int32_t *)e->cslot,
                               (const int32_t *)e->sb_rom, (const double *)e->ctab, (const uint8_t *)e->cmask,
                               (const int32_t *)e->surf, e->n, e->binv, e->agg_gen);
        if (any_gen) {
            if (e->n <= 256)
                hipLaunchKernelGGL(k_coarse_setup<256>, dim3(e->boxes.high, MAXA), dim3(256), 0, st, B.sel,
                                   (const int4 *)e->box_tab, (const ProbParams *)e->pp, (const int32_t *)e->cslot,
                                   (const int32_t *)e->sb_rom, (const void *const *)e->kr32_tab,
                                   (const uint8_t *)e->cmask, (const int32_t *)e->surf, e->n, e->ldk, e->binv,
                                   (const int32_t *)e->agg_gen);
            else
                hipLaunchKernelGGL(k_coarse_setup<512>, dim3(e->boxes.high, MAXA), dim3(512), 0, st, B.sel,
                                   (const int4 *)e->box_tab, (const ProbParams *)e->pp, (const int32_t *)e->cslot,
                                   (const int32_t *)e->sb_rom, (const void *const *)e->kr32_tab,
                                   (const uint8_t *)e->cmask, (const int32_t *)e->surf, e->n, e->ldk, e->binv,
                                   (const int32_t *)e->agg_gen);
        }
    }
    MOS_LAUNCH_CHECK();
    // At set-up x = g, so one product A g gives both ||b_l|| and the residual.
    return residual_batch(e, B, true);
}

// Inner solves of the batch's problems start from their FP64 residuals, with
// the sweep parameters already in sp_host.
template <class T>
mos_status start_batch(mos_engine e, const Batch &B) {
    hipStream_t st = e->ctx->stream;
    const int hw_blk = e->blk.high, hw_sb = e->sbs.high, hw_p = e->pids.high;
    T *V[NVEC];
    for (int i = 0; i < NVEC; ++i) V[i] = static_cast<T *>(e->v[i]);
    T *Mc = static_cast<T *>(e->Mc), *Y = static_cast<T *>(e->Yi);
    MOS_HIP(hipMemcpyAsync(e->sp, e->sp_host, hw_p * sizeof(SweepParams), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_prob_start_list, dim3(ceil_div(B.list.n, 64)), dim3(64), 0, st, B.list,
                       (const ProbParams *)e->pp, (const SweepParams *)e->sp, e->ps, e->epoch);
    if (e->precond)
        hipLaunchKernelGGL(k_cgstart2<T>, dim3(e->boxes.high), dim3(e->box_nt), e->box_nt * 6 * sizeof(double), st,
                           B.sel, (const int4 *)e->box_tab, (const ProbParams *)e->pp, (const SweepParams *)e->sp,
                           (const ProbState *)e->ps, (const double *)e->r64, (const T *)V[VDINV],
                           (const int32_t *)e->inc, (const uint8_t *)e->cmask, (const uint32_t *)e->lc, V[VX], V[VR],
                           V[VP], V[VS], Mc, e->ld_slots, e->pg, e->pr, (const double *)e->binv, e->cc,
                           e->cap_blk);
    else
        hipLaunchKernelGGL(k_cgstart_sel<T>, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                           (const SweepParams *)e->sp, (const ProbState *)e->ps, (const double *)e->r64,
                           (const T *)V[VDINV], (const int32_t *)e->inc, (const int32_t *)(e->stacked ? e->inc2 : nullptr), V[VX], V[VR], V[VP], V[VS],
                           Mc, e->ld_slots, e->pg, e->pr, e->cap_blk);
    MOS_LAUNCH_CHECK();
    (void)hw_sb;
    (void)Y;
    return MOS_OK;
}

// Fold the stopped inner solves' corrections into x64 (sign +1), or take a
// correction back (sign -1).
mos_status add_inner_batch(mos_engine e, const Batch &B, double sign) {
    hipStream_t st = e->ctx->stream;
    const int hw_blk = e->blk.high;
    if (e->precision == MOS_MIXED)
        hipLaunchKernelGGL(k_add_inner_sel<float>, dim3(hw_blk), dim3(DB), 0, st, B.sel, (const int32_t *)e->blk_prob,
                           (const ProbParams *)e->pp, (const SweepParams *)e->sp, e->x64, (const float *)e->v[VX],
                           sign);
    else
        hipLaunchKernelGGL(k_add_inner_sel<double>, dim3(hw_blk), dim3(DB), 0, st, B.sel,
                           (const int32_t *)e->blk_prob, (const ProbParams *)e->pp, (const SweepParams *)e->sp,
                           e->x64, (const double *)e->v[VX], sign);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

// After a residual: the relative residual decides; finish, fail, or set up
// the next sweep's parameters in sp_host (*start).  Refinement is kept
// monotone: a correction that raised the FP64 residual is taken back (one
// residual round trip of its own) and the next sweep gets half the
// iterations.
mos_status decide(mos_engine e, EngineProblem *P, double res2, double bb2, bool *start) {
    hipStream_t st = e->ctx->stream;
    *start = false;
    const bool mixed = e->precision == MOS_MIXED;
    if (P->sweep_cap == 0) P->sweep_cap = mixed ? 256 : P->max_iters;
    if (P->last_res2 >= 0.0 && !(res2 <= P->last_res2)) {
        Batch U;
        U.add(P->pid);
        MOS_TRY(add_inner_batch(e, U, -1.0));
        MOS_TRY(residual_batch(e, U, false));
        MOS_HIP(hipMemcpyAsync(e->host_scratch, e->res2 + P->pid, sizeof(double), hipMemcpyDeviceToHost, st));
        MOS_HIP(hipStreamSynchronize(st));
        res2 = e->host_scratch[0];
        P->sweep_cap = std::max(P->sweep_cap / 2, 8);
        P->undone++;
        P->can_continue = false;  // the solver state belonged to the rejected correction
    }
    P->last_res2 = res2;
    const double bnorm = std::sqrt(bb2), rnorm = std::sqrt(res2);
    P->rel = bnorm > 0 ? rnorm / bnorm : rnorm;
    if (!std::isfinite(P->rel)) {
        P->state = 3;
        P->status = MOS_ENOCONV;
        P->error = "non-finite residual in the global solve";
        return MOS_OK;
    }
    if (P->rel <= P->rtol || res2 == 0.0) {
        P->state = 2;
        return MOS_OK;
    }
    const int max_refine = mixed ? 40 : 8;
    if (P->sweeps >= max_refine || P->iters >= P->max_iters || P->undone > 8) {
        char buf[256];
        snprintf(buf, sizeof(buf), "global solve stopped at relative residual %.3e > rtol %.3e after %d iterations, %d sweeps",
                 P->rel, P->rtol, P->iters, P->sweeps);
        P->error = buf;
        P->state = 3;
        P->status = MOS_ENOCONV;
        return MOS_OK;
    }
    SweepParams &S = e->sp_host[P->pid];
    // Inner rhs = r / ||r|| (mixed) or r (FP64).
    S.scale_in = mixed ? 1.0 / rnorm : 1.0;
    S.scale_out = mixed ? rnorm : 1.0;
    // After a folded-in correction the inner iteration goes on with the
    // true residual (a reliable update) instead of starting over, keeping
    // its search direction rescaled to the new right-hand side.
    S.cont = P->can_continue ? 1 : 0;
    S.p_scale = P->can_continue ? S.scale_in / P->last_scale_in : 0.0;
    P->last_scale_in = S.scale_in;
    P->can_continue = true;
    double rtol_in;
    if (mixed) {
        // A fixed reduction per sweep; the last sweep asks for no more than
        // the remaining factor to the final target.
        rtol_in = std::min(0.5, std::max(INNER_RTOL_F32, P->rtol * bnorm / rnorm));
    } else {
        // FP64 inner solves aim at the final absolute target; the true
        // residual follows the recurrence closely, so one sweep usually ends
        // the solve (a short second one makes up any drift).
        rtol_in = std::min(0.5, std::max(P->rtol * bnorm / rnorm, 1e-15));
    }
    S.rtol2 = rtol_in * rtol_in;
    S.max_iter = std::min(P->sweep_cap, P->max_iters - P->iters);
    P->sweeps++;
    P->state = 1;
    *start = true;
    return MOS_OK;
}

// Decide every problem of a residual batch, then start the next sweep of
// those that continue, all in one batched start.
mos_status decide_and_start(mos_engine e, const std::vector<EngineProblem *> &probs) {
    hipStream_t st = e->ctx->stream;
    const int hw_p = e->pids.high;
    std::vector<double> r2(hw_p), b2(hw_p);
    std::vector<int32_t> bad(hw_p, 0);
    bool any_dev_list = false;
    for (EngineProblem *P : probs) any_dev_list |= P->dpdof != nullptr && P->last_res2 < 0.0;
    MOS_HIP(hipMemcpyAsync(r2.data(), e->res2, hw_p * 8, hipMemcpyDeviceToHost, st));
    MOS_HIP(hipMemcpyAsync(b2.data(), e->bb2, hw_p * 8, hipMemcpyDeviceToHost, st));
    if (any_dev_list) MOS_HIP(hipMemcpyAsync(bad.data(), e->pres_bad, hw_p * 4, hipMemcpyDeviceToHost, st));
    MOS_HIP(hipStreamSynchronize(st));
    Batch S;
    for (EngineProblem *P : probs) {
        if (P->dpdof && P->last_res2 < 0.0 && bad[P->pid]) {
            P->state = 3;
            P->status = MOS_EINVAL;
            P->error = "a device-resident prescribed entry has a DoF outside [0, n_dofs) or a non-finite value";
            continue;
        }
        bool start = false;
        MOS_TRY(decide(e, P, r2[P->pid], b2[P->pid], &start));
        if (start) S.add(P->pid);
    }
    if (S.empty()) return MOS_OK;
    return e->precision == MOS_MIXED ? start_batch<float>(e, S) : start_batch<double>(e, S);
}

}  // namespace

namespace {
int64_t largest_box(mos_engine e, bool *fits, int *width = nullptr);
}  // namespace

mos_status engine_alloc(mos_engine e, int64_t cap_dofs, int64_t cap_slots) {
    mos_ctx ctx = e->ctx;
    const bool mixed = e->precision == MOS_MIXED;
    const size_t w = mixed ? 4 : 8;
    const int ldk = e->ldk;
    const int64_t dofs = std::max<int64_t>(round_up(cap_dofs, DOF_ALIGN), DOF_ALIGN);
    const int64_t slots = std::max<int64_t>(round_up(cap_slots, 16), 16);
    if (!slots_fit(slots)) {
        set_error("%lld cell slots exceed the engine's limit of %lld (slot and surface node share one int32)",
                  (long long)slots, (long long)MAX_SLOTS);
        return MOS_EINVAL;
    }
    e->cap_blk = (int)(dofs / DB);
    e->cap_sb = (int)(slots / 16);
    e->ld_slots = (int)slots;
    DeviceArena &m = e->mem;
    for (int i = 0; i < NVEC; ++i) MOS_TRY(m.alloc(dofs * w, &e->v[i]));
    MOS_TRY(m.alloc((size_t)ldk * slots * w, &e->Mc));
    MOS_TRY(m.alloc((size_t)ldk * slots * w, &e->Yi));
    MOS_TRY(m.alloc_n((size_t)ldk * slots, &e->Mc64));
    MOS_TRY(m.alloc_n((size_t)ldk * slots, &e->Y64));
    MOS_TRY(m.alloc_n(dofs, &e->x64));
    MOS_TRY(m.alloc_n(dofs, &e->b_raw));
    MOS_TRY(m.alloc_n(dofs, &e->g));
    MOS_TRY(m.alloc_n(dofs, &e->r64));
    MOS_TRY(m.alloc_n(dofs, &e->cmask));
    MOS_TRY(m.alloc_n(dofs / 3 * 4, &e->inc));
    MOS_TRY(m.alloc_n(dofs / 3 * 4, &e->inc2));
    MOS_TRY(m.alloc_n(e->cap_blk, &e->blk_prob));
    MOS_TRY(m.alloc_n(2 * (size_t)e->cap_blk, &e->pg));  // two parity slots
    MOS_TRY(m.alloc_n(e->cap_blk, &e->pd));
    MOS_TRY(m.alloc_n(2 * (size_t)e->cap_blk, &e->pr));
    MOS_TRY(m.alloc_n(e->cap_blk, &e->pr64));
    MOS_TRY(m.alloc_n((size_t)e->cap_sb * (ldk / 16), &e->pdel));
    MOS_TRY(m.alloc_n(e->cap_sb, &e->sb_rom));
    MOS_TRY(m.alloc_n(e->cap_sb, &e->sb_prob));
    MOS_TRY(m.alloc_n(slots, &e->perm));
    MOS_TRY(m.alloc_n(dofs / 3, &e->lc));
    MOS_TRY(m.alloc_n(slots, &e->cslot));
    MOS_TRY(m.alloc_n(e->cap_blk, &e->box_tab));
    MOS_TRY(m.alloc_n((size_t)e->cap_blk * MAXA * 36, &e->binv));
    MOS_TRY(m.alloc_n((size_t)e->cap_blk * MAXA * 6, &e->cc));
    MOS_TRY(m.alloc_n((size_t)e->cap_blk * MAXA, &e->agg_gen));
    MOS_TRY(m.alloc_n((size_t)MAX_TYPES * 4 * 4 * 4 * 21, &e->ctab));
    MOS_TRY(m.alloc_n(MAX_PROBS, &e->ps));
    MOS_TRY(m.alloc_n(1, &e->epoch_dev));
    MOS_TRY(m.alloc_n(MAX_PROBS, &e->res2));
    MOS_TRY(m.alloc_n(MAX_PROBS, &e->bb2));
    MOS_TRY(m.alloc_n(MAX_PROBS, &e->pres_bad));
    if (hipHostMalloc((void **)&e->host_scratch, 8 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        e->host_scratch = nullptr;
        set_error("pinned host allocation failed");
        return MOS_ENOMEM;
    }
    if (e->precision == MOS_MIXED && e->roms[0]->psi_hi)
        MOS_TRY(m.alloc((size_t)recon_bf16_scratch(e->roms[0], e->cap_sb), &e->ub));
    std::vector<int> surf;
    surface_nodes(e->roms[0]->desc.interp[0], e->roms[0]->desc.interp[1], e->roms[0]->desc.interp[2], surf);
    e->S = (int)surf.size() / 3;
    MOS_TRY(m.alloc_n(surf.size(), &e->surf));
    MOS_TRY(m.alloc_n(MAX_PROBS, &e->pp));
    MOS_TRY(m.alloc_n(MAX_PROBS, &e->sp));
    if (hipHostMalloc((void **)&e->pp_host, MAX_PROBS * sizeof(ProbParams), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&e->sp_host, MAX_PROBS * sizeof(SweepParams), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("pinned host allocation failed");
        return MOS_ENOMEM;
    }
    std::memset((void *)e->sp_host, 0, MAX_PROBS * sizeof(SweepParams));
    if (hipHostMalloc((void **)&e->sb_rom_host, (size_t)e->cap_sb * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&e->perm_host, (size_t)slots * 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("pinned host allocation failed");
        return MOS_ENOMEM;
    }
    std::fill(e->sb_rom_host, e->sb_rom_host + e->cap_sb, -1);
    std::fill(e->perm_host, e->perm_host + slots, -1);
    if (hipHostMalloc((void **)&e->ps_host, MAX_PROBS * sizeof(ProbState), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("pinned host allocation failed");
        return MOS_ENOMEM;
    }
    // Written by the scalar step of each iteration (one thread, 16 bytes)
    // and read by the host once a problem's first sweep has stopped.
    if (hipHostMalloc((void **)&e->lz, (size_t)MAX_PROBS * LZ_MAX * 2 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        e->lz = nullptr;
        set_error("pinned host allocation failed");
        return MOS_ENOMEM;
    }
    MOS_HIP(hipEventCreateWithFlags(&e->mirror_ev, hipEventDisableTiming));
    MOS_HIP(hipEventRecord(e->mirror_ev, ctx->stream));
    MOS_TRY(m.alloc_n((size_t)MAX_PROBS * MAX_TYPES, &e->jobs));
    if (hipHostMalloc((void **)&e->jobs_host, (size_t)MAX_PROBS * MAX_TYPES * sizeof(ReconJob),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        e->jobs_host = nullptr;
        set_error("pinned host allocation failed");
        return MOS_ENOMEM;
    }
    MOS_TRY(m.alloc_n(MAX_TYPES, &e->kr64_tab));
    MOS_TRY(m.alloc_n(MAX_TYPES, &e->kr32_tab));
    MOS_TRY(m.alloc_n(MAX_TYPES, &e->br_tab));
    MOS_TRY(m.alloc_n(MAX_TYPES, &e->psi_tab));
    MOS_TRY(m.alloc_n(MAX_TYPES, &e->sigt_tab));
    hipStream_t st = ctx->stream;
    auto fill32 = [&](void *p, int64_t n, uint32_t v) {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                           (uint32_t *)p, n, v);
    };
    // Cell layouts must hold zeros in padding slots and rows.
    fill32(e->Mc, (int64_t)ldk * slots * w / 4, 0u);
    fill32(e->Mc64, (int64_t)ldk * slots * 2, 0u);
    // Kernels read the incidence of every block below the high-water mark
    // before they know whether the block is active, so it never holds
    // anything but -1 or a valid slot.
    fill32(e->inc, dofs / 3 * 4, 0xffffffffu);
    fill32(e->inc2, dofs / 3 * 4, 0xffffffffu);
    fill32(e->blk_prob, e->cap_blk, 0xffffffffu);
    fill32(e->sb_rom, e->cap_sb, 0xffffffffu);
    fill32(e->sb_prob, e->cap_sb, 0xffffffffu);  // -1: no owner (batched phases select by owner)
    fill32(e->perm, slots, 0xffffffffu);         // as its host mirror
    fill32(e->box_tab, (int64_t)e->cap_blk * 4, 0xffffffffu);
    fill32(e->ps, (int64_t)MAX_PROBS * sizeof(ProbState) / 4, 0u);
    MOS_LAUNCH_CHECK();
    std::vector<const void *> t64(MAX_TYPES, nullptr), t32(MAX_TYPES, nullptr), tb(MAX_TYPES, nullptr),
        tp(MAX_TYPES, nullptr), ts(MAX_TYPES, nullptr);
    for (size_t t = 0; t < e->roms.size(); ++t) {
        t64[t] = e->roms[t]->kr_pad;
        t32[t] = e->roms[t]->kr32_pad;
        tb[t] = e->roms[t]->br;
        tp[t] = e->roms[t]->psi;
        ts[t] = e->roms[t]->sig_t;
    }
    MOS_HIP(hipMemcpyAsync(e->kr64_tab, t64.data(), MAX_TYPES * 8, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->kr32_tab, t32.data(), MAX_TYPES * 8, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->br_tab, tb.data(), MAX_TYPES * 8, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->psi_tab, tp.data(), MAX_TYPES * 8, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->sigt_tab, ts.data(), MAX_TYPES * 8, hipMemcpyHostToDevice, st));
    MOS_HIP(hipMemcpyAsync(e->surf, surf.data(), surf.size() * 4, hipMemcpyHostToDevice, st));
    MOS_HIP(hipStreamSynchronize(st));
    // The GEMM variant is fixed per engine (never per batch), so a problem's
    // rounding does not depend on what else is in the batch.
    e->gemm_rows = ldk / 4 <= ROWS_MAX_KS;
    {
        bool fits = false;
        largest_box(e, &fits);
        MOS_TRY(engine_set_precond(e, e->precond && fits ? 1 : 0));
    }
    e->tuner.configure(e->gemm_paths, e->gemm_split);
    e->blk.init(e->cap_blk);
    e->sbs.init(e->cap_sb);
    e->pids.init(MAX_PROBS);
    e->boxes.init(e->cap_blk);
    return MOS_OK;
}

namespace {
// Box width (cells along x, a multiple of AGG_C up to BOX_CX: the widest
// whose corner box holds at most 1024 nodes), the nodes of that largest box
// (with the closing nodes), and whether the two-level kernels take it: one
// thread per node, a basis of at most 512 DoFs in the set-up, packed
// coordinates below 256.
int64_t largest_box(mos_engine e, bool *fits, int *width) {
    const mos_cell_desc &cd = e->roms[0]->desc;
    const int sx = cd.interp[0] - 1, sy = cd.interp[1] - 1, nz = cd.interp[2];
    int w = BOX_CX;
    int64_t max_nodes = sub_count(make_sub(w * sx + 1, AGG_C * sy + 1, nz, sx, sy, nz - 1));
    while (max_nodes > 1024 && w > AGG_C) {
        w -= AGG_C;
        max_nodes = sub_count(make_sub(w * sx + 1, AGG_C * sy + 1, nz, sx, sy, nz - 1));
    }
    if (width) *width = w;
    // The box kernels address the cell layouts with 32-bit byte offsets.
    const bool small_layout = e->ld_slots == 0 || (uint64_t)e->ldk * e->ld_slots * 8 < (1ull << 32);
    *fits = max_nodes <= 1024 && e->n <= 512 && AGG_C * sx < 256 && AGG_C * sy < 256 && nz < 256 && small_layout;
    return max_nodes;
}
}  // namespace

mos_status engine_set_precond(mos_engine e, int precond) {
    bool fits = false;
    int width = BOX_CX;
    const int64_t max_nodes = largest_box(e, &fits, &width);
    if (precond && !fits) {
        set_error("the two-level preconditioner needs boxes of at most 1024 nodes and a basis of at most 512");
        return MOS_EINVAL;
    }
    e->precond = precond;
    e->box_nt = (int)std::max<int64_t>(CG_LW, round_up(max_nodes, 64));
    // Jacobi alone keeps whole rows of cells per box (long rows of nodes
    // give the update's gathers the fewest cache lines per wave).
    e->box_cells[0] = precond ? width : 4096;
    e->box_cells[1] = AGG_C;
    return MOS_OK;
}

mos_status engine_check_desc(mos_engine e, const mos_array_desc *d) {
    if (!d || d->nx_cells < 1 || d->ny_cells < 1 || d->nz_cells < 0 ||
        (int64_t)d->nx_cells * d->ny_cells * (d->nz_cells < 1 ? 1 : d->nz_cells) > (1 << 22) || !d->cell_type) {
        set_error("array size must be >= 1x1 (x 1 layer) and <= 4M cells, with a cell_type map");
        return MOS_EINVAL;
    }
    if (d->nz_cells > 1 && e->precond) {
        set_error("stacked arrays take the Jacobi preconditioner: set MOS_OPT_PRECOND 0 before the first submission");
        return MOS_EINVAL;
    }
    if (!std::isfinite(d->delta_T) || d->n_prescribed < 0 ||
        (d->n_prescribed > 0 && (!d->prescribed_dof || !d->prescribed_value)) ||
        (d->bc_flags & ~(uint32_t)(MOS_BC_CLAMP_BOTTOM | MOS_BC_CLAMP_TOP | MOS_BC_LIST_ON_DEVICE)) ||
        d->precision != e->precision ||
        d->rtol < 0 || d->max_iters < 0) {
        set_error("invalid delta_T, constraints, precision (must match the engine), rtol or max_iters");
        return MOS_EINVAL;
    }
    const int64_t n_cells = (int64_t)d->nx_cells * d->ny_cells * (d->nz_cells < 1 ? 1 : d->nz_cells);
    int first = -1;
    for (int64_t c = 0; c < n_cells; ++c) {
        const int t = d->cell_type[c];
        if (t >= (int)e->roms.size()) {
            set_error("cell_type[%lld] = %d but only %d ROMs", (long long)c, t, (int)e->roms.size());
            return MOS_EINVAL;
        }
        if (first < 0) first = t;
        const mos_cell_desc &a = e->roms[first]->desc, &b = e->roms[t]->desc;
        if (a.pitch_x != b.pitch_x || a.pitch_y != b.pitch_y || a.height != b.height || a.skew != b.skew) {
            set_error("cells of one array use ROMs %d and %d of different pitch or height", first, t);
            return MOS_EINVAL;
        }
    }
    return MOS_OK;
}

mos_status engine_submit(mos_engine e, const mos_array_desc *d, void *vm, void *sig6, double *u_out,
                         int64_t *ticket) {
    MOS_TRY(engine_check_desc(e, d));
    EngineProblem *P = new (std::nothrow) EngineProblem();
    if (!P) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    mos_status s = prepare_problem(e, d, P);
    if (s != MOS_OK) {
        delete P;
        return s;
    }
    if (P->n_blk > e->cap_blk || P->n_sb > e->cap_sb) {
        set_error("problem needs %d DoF blocks and %d slot blocks; the engine holds %d and %d", P->n_blk, P->n_sb,
                  e->cap_blk, e->cap_sb);
        delete P;
        return MOS_EINVAL;
    }
    P->ticket = ++e->next_ticket;
    P->vm = vm;
    P->sig6 = sig6;
    P->u_out = u_out;
    e->queue.push_back(P);
    *ticket = P->ticket;
    return MOS_OK;
}

namespace {

mos_status reconstruct_problem(mos_engine e, EngineProblem *P);

// Release the listed problems: one launch returns their owner and type
// tables to -1 and marks them inactive (their device parameters are still
// in place when it runs); the host mirrors follow.
mos_status release_problems(mos_engine e, const std::vector<EngineProblem *> &probs) {
    if (probs.empty()) return MOS_OK;
    hipStream_t st = e->ctx->stream;
    Batch B;
    for (EngineProblem *P : probs) B.add(P->pid);
    hipLaunchKernelGGL(k_release_list, dim3(16, B.list.n), dim3(256), 0, st, B.list, (const ProbParams *)e->pp,
                       e->blk_prob, e->sb_rom, e->sb_prob, e->box_tab, e->ps);
    MOS_LAUNCH_CHECK();
    MOS_TRY(mirror_wait(e));
    for (EngineProblem *P : probs) {
        std::fill(e->sb_rom_host + P->sb_begin, e->sb_rom_host + P->sb_begin + P->n_sb, -1);
        std::fill(e->perm_host + (int64_t)P->sb_begin * 16, e->perm_host + (int64_t)(P->sb_begin + P->n_sb) * 16,
                  -1);
        P->dev.release();  // stream-ordered: later work on this stream may reuse it
        e->blk.give(P->blk_begin, P->n_blk);
        if (P->box_begin >= 0) e->boxes.give(P->box_begin, P->n_agg);
        e->sbs.give(P->sb_begin, P->n_sb);
        e->pids.give(P->pid, 1);
    }
    return MOS_OK;
}

}  // namespace

template <class T>
mos_status rows_step(mos_engine e, int ks, int hw_sb);

// The update launch of iteration j of the chunk over [0, hw_blk) DoF blocks.
template <class T>
void cgstep_launch(mos_engine e, int hw_blk, T *const *V, int j) {
    hipStream_t st = e->ctx->stream;
    if (e->precond) {
        const int hw_box = e->boxes.high;
        launch_timed(e->ctx, MOS_K_PCG_UPDATE, k_cgstep2<T>, dim3((unsigned)(ceil_div(hw_box, N_XCD) * N_XCD)),
                     dim3(e->box_nt), e->box_nt * 6 * sizeof(double), st, (const T *)e->Yi, (const int32_t *)e->inc,
                     (const uint8_t *)e->cmask, (const T *)V[VDINV], (const uint32_t *)e->lc, V[VX], V[VR], V[VP],
                     V[VS], (T *)e->Mc, e->ld_slots, (const int4 *)e->box_tab, (const ProbParams *)e->pp, e->ps,
                     e->pg, e->pr, (const double *)e->pdel, (const double *)e->binv, e->cc,
                     (const int *)e->epoch_dev, j, e->cap_blk, hw_box, e->lz);
        return;
    }
    const bool wide = e->update_width ? e->update_width == 256 : hw_blk <= CG_WIDE_MAX_BLK;
    const dim3 grid((unsigned)(ceil_div(hw_blk, N_XCD) * N_XCD));
    if (wide)
        launch_timed(e->ctx, MOS_K_PCG_UPDATE, k_cgstep<T, 256>, grid, dim3(256), 0, st, (const T *)e->Yi,
                     (const int32_t *)e->inc, (const int32_t *)(e->stacked ? e->inc2 : nullptr), (const uint8_t *)e->cmask, (const T *)V[VDINV], V[VX], V[VR], V[VP],
                     V[VS], (T *)e->Mc, e->ld_slots, (const int32_t *)e->blk_prob, e->ps, e->pg, e->pr,
                     (const double *)e->pdel, (const int *)e->epoch_dev, j, e->cap_blk, hw_blk, e->lz);
    else
        launch_timed(e->ctx, MOS_K_PCG_UPDATE, k_cgstep<T, 128>, grid, dim3(128), 0, st, (const T *)e->Yi,
                     (const int32_t *)e->inc, (const int32_t *)(e->stacked ? e->inc2 : nullptr), (const uint8_t *)e->cmask, (const T *)V[VDINV], V[VX], V[VR], V[VP],
                     V[VS], (T *)e->Mc, e->ld_slots, (const int32_t *)e->blk_prob, e->ps, e->pg, e->pr,
                     (const double *)e->pdel, (const int *)e->epoch_dev, j, e->cap_blk, hw_blk, e->lz);
}

// Read the tuning trials of the last chunk (the stream has been synchronised).
void tuner_collect(GemmTuner &T) {
    for (auto &pd : T.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pd.start, pd.stop) == hipSuccess) {
            GemmTuner::Bucket &B = T.buckets[pd.bucket];
            B.best[pd.cand] = std::min(B.best[pd.cand], ms);
            B.runs[pd.cand]++;
        } else {
            (void)hipGetLastError();
        }
        T.spare.push_back(pd.start);
        T.spare.push_back(pd.stop);
    }
    T.pending.clear();
    for (auto &kv : T.buckets) {
        GemmTuner::Bucket &B = kv.second;
        if (B.chosen > 0) continue;
        bool done = true;
        int best = 0;
        for (int c = 0; c < T.n_cand; ++c) {
            done &= B.runs[c] >= GemmTuner::REPS;
            if (B.best[c] < B.best[best]) best = c;
        }
        if (done) B.chosen = best + 1;
    }
}

void GemmTuner::configure(int paths, int fixed_spw) {
    n_cand = 0;
    for (int path = 0; path < 2; ++path) {
        if (!((paths >> path) & 1)) continue;
        if (fixed_spw > 0) {
            cand_path[n_cand] = path;
            cand_spw[n_cand++] = fixed_spw;
        } else {
            for (int k = 0; k < N_SPW; ++k) {
                if (SPW[k] == CHIP_SPLIT && path != 1) continue;
                cand_path[n_cand] = path;
                cand_spw[n_cand++] = SPW[k];
            }
        }
    }
    buckets.clear();
    for (const Pending &pd : pending) {
        spare.push_back(pd.start);
        spare.push_back(pd.stop);
    }
    pending.clear();
}

hipEvent_t tuner_event(GemmTuner &T) {
    if (!T.spare.empty()) {
        hipEvent_t ev = T.spare.back();
        T.spare.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return ev;
}

// One rows-GEMM launch of the iteration over [0, hw_sb) slot blocks, with
// the work split from the tuner (timed with events while it is a trial).
template <class T>
mos_status rows_step(mos_engine e, int ks, int hw_sb) {
    hipStream_t st = e->ctx->stream;
    GemmTuner &Tn = e->tuner;
    const void *const *tab = (const void *const *)(sizeof(T) == 4 ? e->kr32_tab : e->kr64_tab);
    auto launch = [&](int cand) {
        int spw = Tn.cand_spw[cand];
        if (spw == GemmTuner::CHIP_SPLIT) spw = std::min(64, std::max(1, ceil_div(hw_sb, e->ctx->n_cu)));
        return launch_cell_gemm<T>(e->ctx, MOS_K_CELL_GEMM, Tn.cand_path[cand], ks, e->n, spw, st, tab,
                                   e->sb_rom, e->sb_prob, (const T *)e->Mc, (T *)e->Yi, e->ld_slots, hw_sb,
                                   (const ProbState *)e->ps, e->pdel, 1, ProbSel{});
    };
    if (Tn.n_cand <= 1) return launch(0);
    int bucket = 0;
    while ((1 << bucket) < hw_sb) ++bucket;
    GemmTuner::Bucket &B = Tn.buckets[bucket];
    if (B.chosen > 0) return launch(B.chosen - 1);
    // Tuning round: every candidate still short of its trials runs on the
    // same operands, back to back, so all of them see the same set of
    // iterating problems (they write identical outputs); one untimed launch
    // first, so the first timed one does not wait for the host.
    MOS_TRY(launch(0));
    for (int k = 0; k < Tn.n_cand; ++k) {
        int queued = 0;
        for (const auto &pd : Tn.pending) queued += pd.bucket == bucket && pd.cand == k;
        if (B.runs[k] + queued >= GemmTuner::REPS) continue;
        hipEvent_t ev0 = tuner_event(Tn), ev1 = tuner_event(Tn);
        if (!ev0 || !ev1) {
            if (ev0) Tn.spare.push_back(ev0);
            if (ev1) Tn.spare.push_back(ev1);
            continue;
        }
        MOS_HIP(hipEventRecord(ev0, st));
        MOS_TRY(launch(k));
        MOS_HIP(hipEventRecord(ev1, st));
        Tn.pending.push_back({bucket, k, ev0, ev1});
    }
    return MOS_OK;
}


namespace {

// The launches of one chunk of iterations on e->ctx->stream: per iteration
// the cell GEMM (w = A u, (u, A u) tile partials), the scalar launch when a
// large problem iterates, and the vector update (which reduces small
// problems' scalars itself).  Iteration j reads its epoch as
// epoch_dev[0] + j.
mos_status issue_chunk(mos_engine e, int chunk, int hw_sb, int hw_blk, int hw_p, bool rows, int ks, bool any_large) {
    mos_ctx ctx = e->ctx;
    hipStream_t st = ctx->stream;
    const dim3 g_gemm(e->ldk / 16, hw_sb);
    for (int j = 0; j < chunk; ++j) {
        if (e->precision == MOS_MIXED) {
            float *V[NVEC];
            for (int i = 0; i < NVEC; ++i) V[i] = static_cast<float *>(e->v[i]);
            if (rows)
                MOS_TRY(rows_step<float>(e, ks, hw_sb));
            else
                launch_timed(ctx, MOS_K_CELL_GEMM, k_bgemm<float>, g_gemm, dim3(256), 0, st,
                             (const void *const *)e->kr32_tab, (const int32_t *)e->sb_rom,
                             (const int32_t *)e->sb_prob, (const float *)e->Mc, (float *)e->Yi, e->ldk, e->ld_slots,
                             0, hw_sb, 1, (const ProbState *)e->ps, e->pdel, ProbSel{});
            if (any_large)
                launch_timed(ctx, MOS_K_PCG_SCALARS, k_cg_scalars, dim3(hw_p), dim3(CG_BIG), 0, st, e->ps,
                             (const double *)e->pg, (const double *)e->pr, (const double *)e->pdel,
                             (const int *)e->epoch_dev, j, e->cap_blk, e->lz);
            cgstep_launch<float>(e, hw_blk, V, j);
        } else {
            double *V[NVEC];
            for (int i = 0; i < NVEC; ++i) V[i] = static_cast<double *>(e->v[i]);
            if (rows)
                MOS_TRY(rows_step<double>(e, ks, hw_sb));
            else
                launch_timed(ctx, MOS_K_CELL_GEMM, k_bgemm<double>, g_gemm, dim3(256), 0, st,
                             (const void *const *)e->kr64_tab, (const int32_t *)e->sb_rom,
                             (const int32_t *)e->sb_prob, (const double *)e->Mc, (double *)e->Yi, e->ldk,
                             e->ld_slots, 0, hw_sb, 1, (const ProbState *)e->ps, e->pdel, ProbSel{});
            if (any_large)
                launch_timed(ctx, MOS_K_PCG_SCALARS, k_cg_scalars, dim3(hw_p), dim3(CG_BIG), 0, st, e->ps,
                             (const double *)e->pg, (const double *)e->pr, (const double *)e->pdel,
                             (const int *)e->epoch_dev, j, e->cap_blk, e->lz);
            cgstep_launch<double>(e, hw_blk, V, j);
        }
    }
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

__global__ void k_set_epoch(int *ep, int value) {
    if (threadIdx.x == 0) ep[0] = value;
}

// One chunk: the chunk's first epoch to the device, then its launches --
// replayed from a captured graph when the engine's graph option is on and
// the chunk's launch sequence is fixed (no GEMM tuning trial, no kernel of
// the chunk under the kernel timer), otherwise issued directly.  The graph
// is captured on a private stream and launched on the context's stream; it
// is captured again whenever anything that shapes the launches changes.
mos_status run_chunk(mos_engine e, int chunk, int hw_sb, int hw_blk, int hw_p, bool rows, int ks, bool any_large) {
    mos_ctx ctx = e->ctx;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(k_set_epoch, dim3(1), dim3(64), 0, st, e->epoch_dev, e->epoch);
    MOS_LAUNCH_CHECK();
    int cand = 0;
    bool fixed = true;
    if (rows && e->tuner.n_cand > 1) {
        int bucket = 0;
        while ((1 << bucket) < hw_sb) ++bucket;
        auto it = e->tuner.buckets.find(bucket);
        fixed = it != e->tuner.buckets.end() && it->second.chosen > 0;
        cand = fixed ? it->second.chosen - 1 : -1;
    }
    const int tk = ctx->timed_kernel;
    const bool timed = tk == MOS_K_CELL_GEMM || tk == MOS_K_PCG_SCALARS || tk == MOS_K_PCG_UPDATE;
    if (!e->use_graph || !fixed || timed) {
        MOS_TRY(issue_chunk(e, chunk, hw_sb, hw_blk, hw_p, rows, ks, any_large));
        e->epoch += chunk;
        return MOS_OK;
    }
    const int key[GRAPH_KEY] = {chunk, hw_sb, hw_blk, hw_p, e->boxes.high, rows ? 1 : 0, cand, any_large ? 1 : 0,
                                e->precond, e->box_nt, e->update_width, e->stacked};
    if (!e->graph_exec || !std::equal(key, key + GRAPH_KEY, e->graph_key)) {
        if (e->graph_exec) {
            MOS_HIP(hipGraphExecDestroy(e->graph_exec));
            e->graph_exec = nullptr;
        }
        if (!e->cap_stream) MOS_HIP(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        ctx->stream = e->cap_stream;
        hipError_t be = hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal);
        mos_status s = be == hipSuccess ? issue_chunk(e, chunk, hw_sb, hw_blk, hw_p, rows, ks, any_large) : MOS_EHIP;
        hipError_t ce = be == hipSuccess ? hipStreamEndCapture(e->cap_stream, &g) : be;
        ctx->stream = st;
        if (s != MOS_OK || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            if (s == MOS_OK) set_error("graph capture of the iteration chunk failed: %s", hipGetErrorString(ce));
            return s != MOS_OK ? s : MOS_EHIP;
        }
        const hipError_t ie = hipGraphInstantiate(&e->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            e->graph_exec = nullptr;
            set_error("graph instantiation of the iteration chunk failed: %s", hipGetErrorString(ie));
            return MOS_EHIP;
        }
        std::copy(key, key + GRAPH_KEY, e->graph_key);
        ++e->graph_captures;
    }
    MOS_HIP(hipGraphLaunch(e->graph_exec, st));
    ++e->graph_replays;
    e->epoch += chunk;
    return MOS_OK;
}

}  // namespace

// One round: admit, iterate a chunk, check stopped problems, retire finished.
namespace {
// Move retired problems whose completion event has passed (all of them when
// `wait`) to the finished map and the completed list, in retirement order.
mos_status collect_retired(mos_engine e, std::vector<int64_t> *completed, bool wait) {
    while (!e->retiring.empty()) {
        mos_engine_s::Retiring &r = e->retiring.front();
        if (wait) {
            MOS_HIP(hipEventSynchronize(r.ev));
        } else {
            const hipError_t q = hipEventQuery(r.ev);
            if (q == hipErrorNotReady) break;
            MOS_HIP(q);
        }
        for (EngineProblem *P : r.probs) {
            e->finished[P->ticket] = P;
            if (completed) completed->push_back(P->ticket);
        }
        e->spare_events.push_back(r.ev);
        e->retiring.pop_front();
    }
    return MOS_OK;
}
}  // namespace

// Condition estimate of the preconditioned operator from k PCG steps:
// the Lanczos tridiagonal T of CG, T_jj = 1/alpha_j + beta_j/alpha_{j-1},
// T_{j-1,j} = sqrt(beta_j)/alpha_{j-1} (beta_0 = 0), has Ritz values inside
// the spectrum of M^-1 A that approach the ends of the part of it the
// right-hand side excites as the iteration goes on;
// their ratio is returned (0 when there are fewer than two steps or the
// record is not positive).  Both ends by bisection on the Sturm count (the
// number of negative pivots of T - x I is the number of eigenvalues below x).
double lanczos_cond(const double *lz, int k, int *steps) {
    *steps = 0;
    if (k < 2) return 0.0;
    std::vector<double> a(k), b(k, 0.0);  // diagonal, off-diagonal b[j] = T_{j-1,j}
    for (int j = 0; j < k; ++j) {
        const double al = lz[2 * j], be = lz[2 * j + 1];
        if (!(al > 0.0) || !(be >= 0.0) || !std::isfinite(al) || !std::isfinite(be)) return 0.0;
        a[j] = 1.0 / al + (j > 0 ? be / lz[2 * (j - 1)] : 0.0);
        if (j > 0) b[j] = std::sqrt(be) / lz[2 * (j - 1)];
    }
    double lo = a[0], hi = a[0];  // Gershgorin bounds
    for (int j = 0; j < k; ++j) {
        const double r = b[j] + (j + 1 < k ? b[j + 1] : 0.0);
        lo = std::min(lo, a[j] - r);
        hi = std::max(hi, a[j] + r);
    }
    auto below = [&](double x) {  // eigenvalues of T below x
        int c = 0;
        double d = 1.0;
        for (int j = 0; j < k; ++j) {
            d = (a[j] - x) - (j > 0 ? b[j] * b[j] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++c;
        }
        return c;
    };
    auto bisect = [&](int target) {  // smallest x with at least `target` eigenvalues below it
        double l = lo, h = hi;
        for (int it = 0; it < 200 && h - l > 1e-15 * std::max(std::fabs(l), std::fabs(h)); ++it) {
            const double m = 0.5 * (l + h);
            if (below(m) >= target)
                h = m;
            else
                l = m;
        }
        return 0.5 * (l + h);
    };
    const double lmin = bisect(1), lmax = bisect(k);
    if (!(lmin > 0.0)) return 0.0;
    *steps = k;
    return lmax / lmin;
}

mos_status engine_progress(mos_engine e, int chunk, std::vector<int64_t> *completed) {
    mos_ctx ctx = e->ctx;
    hipStream_t st = ctx->stream;
    MOS_TRY(collect_retired(e, completed, false));
    // 1. Admission in arrival order while the arenas have room.
    std::vector<EngineProblem *> admitted;
    while (!e->queue.empty()) {
        EngineProblem *P = e->queue.front();
        int pid = e->pids.take(1);
        if (pid < 0) break;
        int b = e->blk.take(P->n_blk);
        if (b < 0) {
            e->pids.give(pid, 1);
            break;
        }
        int sb = e->sbs.take(P->n_sb);
        if (sb < 0) {
            e->blk.give(b, P->n_blk);
            e->pids.give(pid, 1);
            break;
        }
        int bx = -1;
        if (e->precond) {
            bx = e->boxes.take(P->n_agg);
            if (bx < 0) {
                e->sbs.give(sb, P->n_sb);
                e->blk.give(b, P->n_blk);
                e->pids.give(pid, 1);
                break;
            }
        }
        P->pid = pid;
        P->blk_begin = b;
        P->sb_begin = sb;
        P->box_begin = bx;
        e->queue.pop_front();
        e->active.push_back(P);
        admitted.push_back(P);
    }
    // Device set-up of everything admitted, in one batch; its residuals
    // decide the first sweeps.
    if (!admitted.empty()) {
        Batch B;
        for (EngineProblem *P : admitted) B.add(P->pid);
        MOS_TRY(setup_batch(e, admitted, B));
        MOS_TRY(decide_and_start(e, admitted));
    }
    // 2. A chunk of iterations over everything that is iterating.
    bool any_iter = false;
    for (EngineProblem *P : e->active) any_iter |= P->state == 1;
    if (any_iter) {
        const int hw_sb = e->sbs.high, hw_blk = e->blk.high, hw_p = e->pids.high;
        // Cell GEMM variant is fixed per engine; the rows variant picks how
        // many slot blocks each wave streams from the batch size only (its
        // results do not depend on that choice).
        const int ks = e->ldk / 4;
        const bool rows = e->gemm_rows && ks <= ROWS_MAX_KS;
        bool any_large = false;
        for (EngineProblem *P : e->active)
            if (P->state == 1 && !e->pp_host[P->pid].fused) any_large = true;
        MOS_TRY(run_chunk(e, chunk, hw_sb, hw_blk, hw_p, rows, ks, any_large));
        MOS_LAUNCH_CHECK();
        // 3. Problems whose inner solve stopped: fold in the correction, FP64 residual.
        const ProbState *hs = e->ps_host;
        MOS_HIP(hipMemcpyAsync(e->ps_host, e->ps, hw_p * sizeof(ProbState), hipMemcpyDeviceToHost, st));
        MOS_HIP(hipStreamSynchronize(st));
        MOS_TRY(collect_retired(e, completed, false));
        tuner_collect(e->tuner);
        std::vector<EngineProblem *> stopped;
        Batch B;
        for (EngineProblem *P : e->active) {
            if (P->state != 1) continue;
            const ProbState &S = hs[P->pid];
            if (!S.done) continue;
            P->iters += S.it - S.seg_start;
            if (S.seg_start == 0 && !P->lz_kept && e->lz) {  // the estimate itself is formed on request
                const double *row = e->lz + (size_t)P->pid * LZ_MAX * 2;
                P->lz.assign(row, row + 2 * std::min(S.it, LZ_MAX));
                P->lz_kept = true;
            }
            if (S.done == 2) P->can_continue = false;  // breakdown: nothing to go on from
            if (S.done == 2 && S.it == S.seg_start) {
                P->state = 3;
                P->status = MOS_ENOCONV;
                P->error = "PCG breakdown (p.Ap <= 0 or non-finite) at the start of a sweep";
                continue;
            }
            stopped.push_back(P);
            B.add(P->pid);
        }
        if (!stopped.empty()) {
            MOS_TRY(add_inner_batch(e, B, 1.0));
            hipLaunchKernelGGL(k_prob_stop_list, dim3(ceil_div(B.list.n, 64)), dim3(64), 0, st, B.list, e->ps);
            MOS_TRY(residual_batch(e, B, false));
            MOS_TRY(decide_and_start(e, stopped));
        }
    }
    // 4. Retire finished problems (reconstruct into their buffers first).  The
    // reconstructions of every problem retiring now share one launch per
    // cell type (FP64, or BF16-split in the mixed engine), so each block of
    // the stress basis is staged once for all.
    const bool batch_f64 = e->precision == MOS_FP64 && e->ldk / 4 <= RECON_F64_LDS_KS;
    const bool batch_bf16 = e->precision == MOS_MIXED && e->ub;
    const bool batch_recon = batch_f64 || batch_bf16;
    if (batch_recon) {
        const int n_roms = (int)e->roms.size();
        std::vector<std::vector<ReconJob>> jobs(n_roms);
        for (EngineProblem *P : e->active) {
            if (P->state != 2 || !(P->vm || P->sig6)) continue;
            for (int t = 0; t < n_roms; ++t) {
                const int nsb = P->seg[t + 1] - P->seg[t];
                if (nsb <= 0) continue;
                const int off = jobs[t].empty() ? 0 : jobs[t].back().sb_off + jobs[t].back().n_sb;
                jobs[t].push_back(ReconJob{P->sb_begin + P->seg[t], off, nsb, 0, P->dT, P->vm, P->sig6});
            }
        }
        if (batch_f64)
            MOS_TRY(recon_f64_jobs(ctx, e->roms.data(), n_roms, jobs.data(), e->jobs, e->jobs_host,
                                   (const double *)e->Mc64, e->ld_slots, (const int32_t *)e->perm, false));
        else
            MOS_TRY(recon_bf16_jobs(ctx, e->roms.data(), n_roms, jobs.data(), e->jobs, e->jobs_host,
                                    (const double *)e->Mc64, e->ld_slots, (const int32_t *)e->perm, e->ub));
    }
    std::vector<EngineProblem *> keep, gone;
    for (EngineProblem *P : e->active) {
        if (P->state == 2 || P->state == 3) {
            if (P->state == 2 && (P->vm || P->sig6) && !batch_recon) MOS_TRY(reconstruct_problem(e, P));
            if (P->state == 2 && P->u_out)
                hipLaunchKernelGGL(k_export_u, dim3(ceil_div(P->n_dofs, 256)), dim3(256), 0, st,
                                   (const double *)(e->x64 + (int64_t)P->blk_begin * DB), P->u_out, P->n_dofs,
                                   whole_lattice(P->lat), P->agg);
            gone.push_back(P);
        } else {
            keep.push_back(P);
        }
    }
    e->active.swap(keep);
    MOS_TRY(release_problems(e, gone));
    if (!gone.empty()) {
        hipEvent_t ev = nullptr;
        if (!e->spare_events.empty()) {
            ev = e->spare_events.back();
            e->spare_events.pop_back();
        } else {
            MOS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        }
        e->retiring.push_back(mos_engine_s::Retiring{ev, {}});
        MOS_HIP(hipEventRecord(ev, st));
        e->retiring.back().probs = gone;
    }
    // With nothing left to iterate there is no later chunk to overlap with:
    // wait for the retirements here instead of on the caller's next call.
    return collect_retired(e, completed, e->active.empty() && e->queue.empty());
}

// ---------------------------------------------------------------------------
// Reconstruction of one engine problem (outputs in its caller buffers).
// ---------------------------------------------------------------------------
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// One wave per (element block of 16, slot block of 16) of the problem; the
// FP64 cell layout holds the scattered solution.
template <class OutT>
__global__ __launch_bounds__(256) void k_brecon(const double *const *psi_tab, const double *const *sigt_tab,
                                                const int32_t *sb_rom, const double *U, const int32_t *perm,
                                                int sb_begin, int n_sb, int ld_slots, int ldk, int n_elem, double dT,
                                                OutT *vm, OutT *sig6) {
    const int eb = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int sbl = blockIdx.y * 4 + wave;
    if (sbl >= n_sb) return;
    const int sb = sb_begin + sbl;
    const int rom = sb_rom[sb];
    if (rom < 0) return;
    const int pc0 = sb * 16;
    const double *psi = psi_tab[rom] + (size_t)eb * 6 * ldk * 16;
    d4 acc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < ldk; k0 += 4) {
        const int kk = k0 + lane / 16;
        const double b = U[(size_t)kk * ld_slots + pc0 + lane % 16];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double a = psi[((size_t)k * ldk + kk) * 16 + lane % 16];
            acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
        }
    }
    const int cell = perm[pc0 + lane % 16];
    if (cell < 0) return;
    const double *stt = sigt_tab[rom];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = eb * 16 + lane / 16 + 4 * q;  // FP64 MFMA output row
        if (e >= n_elem) continue;
        double s[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = acc[k][q] + dT * stt[(size_t)e * 6 + k];
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

mos_status reconstruct_problem(mos_engine e, EngineProblem *P) {
    hipStream_t st = e->ctx->stream;
    // The last residual check left the solution scattered in the FP64 cell layout.
    dim3 grid(e->n_eblk, ceil_div(P->n_sb, 4));
    if (e->precision == MOS_FP64)
        launch_timed(e->ctx, MOS_K_RECON, k_brecon<double>, grid, dim3(256), 0, st, (const double *const *)e->psi_tab,
                     (const double *const *)e->sigt_tab, (const int32_t *)e->sb_rom, (const double *)e->Mc64,
                     (const int32_t *)e->perm, P->sb_begin, P->n_sb, e->ld_slots, e->ldk, e->n_elem, P->dT,
                     (double *)P->vm, (double *)P->sig6);
    else
        launch_timed(e->ctx, MOS_K_RECON, k_brecon<float>, grid, dim3(256), 0, st, (const double *const *)e->psi_tab,
                     (const double *const *)e->sigt_tab, (const int32_t *)e->sb_rom, (const double *)e->Mc64,
                     (const int32_t *)e->perm, P->sb_begin, P->n_sb, e->ld_slots, e->ldk, e->n_elem, P->dT,
                     (float *)P->vm, (float *)P->sig6);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

}  // namespace

mos_status engine_gather_index(mos_engine e, const EngineProblem *P, const int32_t *perm, int32_t *gidx) {
    const int64_t n_slots = (int64_t)P->n_sb * 16;
    hipLaunchKernelGGL(k_gather_index, dim3(ceil_div((int64_t)e->ldk * n_slots, 256)), dim3(256), 0, e->ctx->stream,
                       gidx, perm, n_slots, e->ldk, e->n, (const int32_t *)e->surf, P->lat);
    MOS_LAUNCH_CHECK();
    return MOS_OK;
}

mos_status engine_problem_size(mos_engine e, const mos_array_desc *d, int64_t *dofs, int64_t *slots) {
    MOS_TRY(engine_check_desc(e, d));
    const mos_cell_desc &cd = e->roms[0]->desc;
    const int nx = cd.interp[0], ny = cd.interp[1], nz = cd.interp[2];
    const int Nz = d->nz_cells < 1 ? 1 : d->nz_cells;
    const Lattice L = make_lattice(d->nx_cells, d->ny_cells, nx, ny, nz, Nz);
    *dofs = (int64_t)problem_blocks(3 * L.n_nodes, agg_count(make_agg_layout(L, e->box_cells[0], e->box_cells[1]))) *
            DB;
    const int64_t n_cells = (int64_t)d->nx_cells * d->ny_cells * Nz;
    std::vector<int64_t> count(e->roms.size(), 0);
    for (int64_t c = 0; c < n_cells; ++c) count[d->cell_type[c]]++;
    int64_t sl = 0;
    for (int64_t cnt : count) sl += round_up(cnt, 16);
    *slots = std::max<int64_t>(sl, 16);
    return MOS_OK;
}

void engine_free(mos_engine e) {
    if (!e) return;
    for (EngineProblem *P : e->queue) delete P;
    for (EngineProblem *P : e->active) {
        P->dev.release();
        delete P;
    }
    for (auto &kv : e->finished) delete kv.second;
    for (auto &r : e->retiring) {
        (void)hipEventSynchronize(r.ev);
        (void)hipEventDestroy(r.ev);
        for (EngineProblem *P : r.probs) delete P;
    }
    for (hipEvent_t ev : e->spare_events) (void)hipEventDestroy(ev);
    e->retiring.clear();
    e->spare_events.clear();
    e->queue.clear();
    e->active.clear();
    e->finished.clear();
    for (auto &pd : e->tuner.pending) {
        (void)hipEventDestroy(pd.start);
        (void)hipEventDestroy(pd.stop);
    }
    for (hipEvent_t ev : e->tuner.spare) (void)hipEventDestroy(ev);
    e->tuner.pending.clear();
    e->tuner.spare.clear();
    e->mem.release();
    if (e->host_scratch) (void)hipHostFree(e->host_scratch);
    e->host_scratch = nullptr;
    if (e->jobs_host) (void)hipHostFree(e->jobs_host);
    e->jobs_host = nullptr;
    if (e->lz) (void)hipHostFree(e->lz);
    e->lz = nullptr;
    if (e->pp_host) (void)hipHostFree(e->pp_host);
    e->pp_host = nullptr;
    if (e->sp_host) (void)hipHostFree(e->sp_host);
    e->sp_host = nullptr;
    if (e->ps_host) (void)hipHostFree(e->ps_host);
    e->ps_host = nullptr;
    if (e->sb_rom_host) (void)hipHostFree(e->sb_rom_host);
    e->sb_rom_host = nullptr;
    if (e->perm_host) (void)hipHostFree(e->perm_host);
    e->perm_host = nullptr;
    if (e->mirror_ev) (void)hipEventDestroy(e->mirror_ev);
    e->mirror_ev = nullptr;
    if (e->graph_exec) (void)hipGraphExecDestroy(e->graph_exec);
    e->graph_exec = nullptr;
    if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
    e->cap_stream = nullptr;
}

}  // namespace mos
