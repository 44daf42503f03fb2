// Batched global-stage engine: types shared by engine.hip and api.cpp.
#pragma once

#include <cstdint>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "mesh.h"
#include "mos_internal.h"

namespace mos {

constexpr int MAX_PROBS = 1024;  // problems resident in one engine at a time
constexpr int LZ_MAX = 128;      // PCG steps of a problem's first sweep kept for its Lanczos estimate

// Per-problem PCG scalars in device memory.  Written by the problem's scalar
// wave (iteration launches) or by single-thread set-up kernels; read by the
// batch kernels and, between chunks, by the host.
struct ProbState {
    double hist_gamma[2], hist_alpha[2];  // (r,u) and step of iteration it, in slot it & 1
    double a_cur, b_cur;            // step of the current iteration (separate scalar launch)
    double rr;                      // ||r||^2 at the last check
    double tol2, rtol2;             // stop threshold and its relative form
    int it, done, active, max_iter; // iterations of this sweep; stop code; iterating; cap
    int blk_begin, blk_end;         // the problem's DoF blocks (partials of (r,u), (r,r))
    int tile_begin, tile_end;       // its cell-GEMM tiles (partials of (u, A u))
    int start_epoch, fused;         // iteration launch of iteration 0; scalars in the update
    int seg_start, pad;             // iteration at which this sweep began (tolerance and cap count from it)
};

// Inner PCG vectors (Chronopoulos-Gear form), in the inner precision.
enum { VX, VR, VP, VS, VDINV, NVEC };

struct EngineProblem;

// Selection of problems for a batched phase (bit p = problem id p), passed
// by value to the kernels of that phase.
struct ProbSel {
    uint32_t bits[MAX_PROBS / 32];
};
// The selected ids in ascending order, for per-problem work (reductions,
// state updates).
struct PidList {
    int32_t n;
    int16_t pid[MAX_PROBS];
};
// Static parameters of an admitted problem (device table by problem id).
struct ProbParams {
    int64_t d0, n_dofs, nd_pad;
    double dT;
    double h[4];                    // node spacing over pitch_x per axis (coarse-correction coordinates),
                                    // then the block's skew (x += skew * y)
    Lattice lat;
    AggLayout agg;                  // internal node order (boxes of cells)
    int32_t blk_begin, n_blk, sb_begin, n_sb, nrb, fused;
    int32_t clamp;                  // MOS_BC_CLAMP_* of the descriptor
    int32_t n_agg;                  // boxes of the internal node order
    int32_t box_begin;              // first box id (two-level preconditioner), else -1
    int32_t part_begin, n_part;     // the problem's (r,u), (r,r) partial slots: its boxes or DoF blocks
    int32_t tab_coarse;             // coarse matrices: 1 per-type table (clamped faces only), 2 table per
                                    // aggregate where its constraints are whole planes, else 0 general
};
// Parameters of a problem's current refinement sweep (device table by id).
struct SweepParams {
    double scale_in, scale_out, rtol2;
    double p_scale;                 // continuing sweeps: factor on the kept p, s (new over old scale_in)
    int32_t max_iter, cont;         // cap; 1 = keep the search direction of the previous sweep
};

// Largest number of 4-wide k-steps (ldk <= 176, basis size <= 176) the
// K_r-stationary GEMM keeps in registers; larger bases use the tile GEMM.
constexpr int ROWS_MAX_KS = 44;
// Entries of the launch shape a captured iteration chunk is valid for.
constexpr int GRAPH_KEY = 12;

// Online tuner of the rows GEMM's work split (slot blocks per wave).  The
// split only decides which wave computes which output tile -- every tile is
// still one wave's fixed-order MFMA chain -- so tuning never changes results.
// Per bucket of slot blocks (power of two of the high-water mark), tuning
// rounds run every candidate back to back within one iteration, on the same
// operands and the same set of iterating problems, each timed with stream
// events; after REPS rounds the fastest (minimum time) is used for that
// bucket for the life of the engine.
struct GemmTuner {
    // A candidate is an operand path of the K_r-stationary GEMM (0: operands
    // streamed per wave from global memory, 1: operand tile staged in LDS
    // per workgroup) and a work split (slot blocks per wave or workgroup).
    // All candidates compute the same MFMA chains, so the choice never
    // changes results.
    // A split of CHIP_SPLIT stands for the one that gives every compute
    // unit one workgroup (the LDS path runs one per CU): ceil(slot blocks /
    // CUs), so a launch fills the chip in a single even round.
    static constexpr int N_SPW = 7;
    static constexpr int CHIP_SPLIT = -1;
    static constexpr int SPW[N_SPW] = {1, 2, 4, 8, 16, 32, CHIP_SPLIT};
    static constexpr int MAX_CAND = 2 * N_SPW;
    static constexpr int REPS = 3;
    int n_cand = 0;
    int cand_path[MAX_CAND] = {}, cand_spw[MAX_CAND] = {};
    struct Bucket {
        float best[MAX_CAND];
        int runs[MAX_CAND];
        int chosen = 0;  // 0 while tuning, else 1 + the chosen candidate
        Bucket() {
            for (int c = 0; c < MAX_CAND; ++c) {
                best[c] = 1e30f;
                runs[c] = 0;
            }
        }
    };
    std::map<int, Bucket> buckets;
    struct Pending {
        int bucket, cand;
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    // Candidates from the allowed operand paths (bit 0 global, bit 1 LDS)
    // and a fixed split (> 0) or the tuned set; tuning starts over.
    void configure(int paths, int fixed_spw);
};

// First-fit allocator of block ranges (host side).
struct RangeAlloc {
    int cap = 0, high = 0;
    std::map<int, int> free_;  // begin -> length
    void init(int c);
    int take(int n);
    void give(int b, int n);
};

}  // namespace mos

struct mos_engine_s {
    uint32_t kind = 0x21474e45u;
    mos_ctx ctx = nullptr;
    bool held = false;  // holds ctx (returned to the caller)
    mos_precision precision = MOS_FP64;
    std::vector<mos_rom> roms;
    int ldk = 0, n = 0, n_elem = 0, n_eblk = 0;
    int cap_blk = 0, cap_sb = 0, ld_slots = 0;
    bool gemm_rows = false;                   // cell GEMM variant (fixed per engine)
    int gemm_paths = 3;                       // operand paths of the rows variant open to the tuner
    int gemm_split = 0;                       // fixed work split (0: tuned)
    int update_width = 0;                     // threads per update workgroup (0: by batch size)
    int precond = 1;                          // 0 Jacobi, 1 Jacobi + aggregate coarse correction
    int box_cells[2] = {6, 2};                // cells per box of the internal node order (x, y)
    int box_nt = 0;                           // threads per box workgroup (two-level update)
    mos::GemmTuner tuner;                     // operand path and work split of the rows variant
    mos::DeviceArena mem;
    // device arrays
    void *v[mos::NVEC] = {};                  // inner vectors (double or float)
    void *Mc = nullptr, *Yi = nullptr;        // inner cell layouts [ldk][ld_slots]
    double *Mc64 = nullptr, *Y64 = nullptr;   // FP64 cell layouts
    double *x64 = nullptr, *b_raw = nullptr, *g = nullptr, *r64 = nullptr;
    double *pdel = nullptr;                   // [cap_sb * ldk/16] per-tile (u, A u) partials
    uint8_t *cmask = nullptr;
    int32_t *inc = nullptr;                   // [dofs/3][4]
    int32_t *inc2 = nullptr;                  // [dofs/3][4]: cells of the layer above (stacked arrays), else -1
    int stacked = 0;                          // a stacked array has been admitted (Jacobi kernels read inc2)
    int32_t *blk_prob = nullptr;              // [cap_blk]
    double *pg = nullptr, *pd = nullptr, *pr = nullptr, *pr64 = nullptr;  // [cap_blk]
    int32_t *sb_rom = nullptr, *sb_prob = nullptr;  // [cap_sb]
    int32_t *perm = nullptr;                  // [ld_slots]
    // Two-level preconditioner: per node packed aggregate-local coordinates,
    // per problem cell -> slot, per box owner, B^-1 and kept coefficients.
    uint32_t *lc = nullptr;                   // [dofs/3]
    int32_t *cslot = nullptr;                 // [ld_slots], at sb_begin * 16 + cell
    int4 *box_tab = nullptr;                  // [cap_blk]: first node, nodes, aggregates, owner (-1 free)
    double *binv = nullptr;                   // [cap_blk][MAXA][36]
    double *cc = nullptr;                     // [cap_blk][MAXA][6]
    int32_t *agg_gen = nullptr;               // [cap_blk][MAXA]: 1 = B_a from the general kernel (prescribed lists)
    int coarse_table = 1;                     // problems with a prescribed list may take the table per aggregate
    // Per cell type, clamp flags, cell class (whether its right / top face
    // belongs to the next aggregate) and piece: the 21 terms of Z^T K_r Z
    // in cell-local coordinates; built per clamp-flag value on first use.
    double *ctab = nullptr;                   // [MAX_TYPES][4][4][4][21]
    int ctab_built = 0;                       // bit f: flags f tabulated
    // Pinned host mirrors of sb_rom and perm: set-up writes a problem's
    // tables here and copies one span per batch; release writes -1 back.
    // mirror_ev marks the last span copy, which must complete before the
    // host changes the mirrors again.
    int32_t *sb_rom_host = nullptr, *perm_host = nullptr;
    hipEvent_t mirror_ev = nullptr;
    mos::ProbState *ps = nullptr;             // [MAX_PROBS]
    mos::ProbState *ps_host = nullptr;        // pinned: states read back at the end of a chunk
    double *lz = nullptr;                     // pinned, written by the device: (alpha, beta) of the first
                                              // sweep's steps, [MAX_PROBS][LZ_MAX][2]
    double *res2 = nullptr, *bb2 = nullptr;   // [MAX_PROBS]
    int32_t *pres_bad = nullptr;              // [MAX_PROBS]: a device-resident prescribed list held a bad entry
    double *host_scratch = nullptr;           // pinned: a few doubles read back from the device
    void **kr64_tab = nullptr, **kr32_tab = nullptr;
    double **br_tab = nullptr, **psi_tab = nullptr, **sigt_tab = nullptr;
    void *ub = nullptr;  // BF16 split of a finished problem's cell block (mixed reconstruction)
    mos::ReconJob *jobs = nullptr, *jobs_host = nullptr;  // batched reconstruction table (device, pinned)
    mos::ProbParams *pp = nullptr, *pp_host = nullptr;    // per-problem parameters (device, pinned)
    int epoch = 0;                                        // PCG iteration launches issued so far
    int *epoch_dev = nullptr;  // [1] first epoch of the chunk in flight (iteration kernels add their place)
    // Graph replay of iteration chunks (MOS_OPT_GRAPH): the instantiated
    // chunk, the launch shape it was captured for, the private stream it is
    // captured on, and counts of captures and replays.
    int use_graph = 0;
    hipGraphExec_t graph_exec = nullptr;
    int graph_key[mos::GRAPH_KEY] = {};
    hipStream_t cap_stream = nullptr;
    int64_t graph_captures = 0, graph_replays = 0;
    mos::SweepParams *sp = nullptr, *sp_host = nullptr;   // per-sweep parameters (device, pinned)
    int32_t *surf = nullptr;  // [S][3] surface Lagrange nodes (i, j, k) of a cell, s order
    int S = 0;
    // host state
    mos::RangeAlloc blk, sbs, pids, boxes;
    int64_t next_ticket = 0;
    std::deque<mos::EngineProblem *> queue;
    std::vector<mos::EngineProblem *> active;
    std::map<int64_t, mos::EngineProblem *> finished;
    std::vector<int64_t> completed_unreported;
    // Problems retired by one progress call, behind an event recorded after
    // their reconstruction, export and release launches: they move to
    // `finished` (and are reported) only once that event has completed, so
    // a reported ticket's output buffers are written.
    struct Retiring {
        hipEvent_t ev;
        std::vector<mos::EngineProblem *> probs;
    };
    std::deque<Retiring> retiring;
    std::vector<hipEvent_t> spare_events;
};

namespace mos {

// Host description of one problem in an engine.
struct EngineProblem {
    int64_t ticket = 0;
    int pid = -1;
    int Nx = 0, Ny = 0, Nz = 1;   // blocks along x and y, stacked layers
    int64_t n_cells = 0, n_nodes = 0, n_dofs = 0;
    int blk_begin = 0, n_blk = 0;
    int sb_begin = 0, n_sb = 0;
    int box_begin = -1;           // first box id (two-level preconditioner)
    std::vector<int> seg;         // per ROM: first slot block within the problem (n_roms+1)
    std::vector<int32_t> perm;    // [n_sb*16] cell id per slot, -1 pad
    std::vector<int32_t> sb_rom;  // [n_sb] ROM of each slot block
    Lattice lat{};                // abstract-mesh numbering of the array
    AggLayout agg{};              // internal node order
    int n_agg = 0;
    uint32_t bc_flags = 0;        // MOS_BC_CLAMP_* of the descriptor
    std::vector<int64_t> pdof;    // prescribed (DoF, value) list as given (host lists)
    std::vector<double> pval;
    int64_t n_pres = 0;           // prescribed entries
    const int64_t *dpdof = nullptr;  // the caller's device list (MOS_BC_LIST_ON_DEVICE), else NULL
    const double *dpval = nullptr;
    mos::DeviceArena dev;         // device copy of the prescribed list
    double dT = 0.0, rtol = 0.0;
    int max_iters = 0, iters = 0, sweeps = 0;
    double rel = 1.0;
    std::vector<double> lz;  // (alpha_j, beta_j) of the first sweep's steps (at most LZ_MAX), kept when it ends
    bool lz_kept = false;
    double last_res2 = -1.0;      // FP64 residual before the last correction
    int sweep_cap = 0;            // inner iterations allowed per sweep
    int undone = 0;               // corrections undone because they raised the residual
    bool can_continue = false;    // the inner solver state belongs to the folded-in correction
    double last_scale_in = 0.0;   // scale_in of the last sweep
    int state = 0;                // 0 queued, 1 iterating, 2 converged, 3 failed
    mos_status status = MOS_OK;
    std::string error;
    void *vm = nullptr, *sig6 = nullptr;
    double *u_out = nullptr;
};

mos_status engine_alloc(mos_engine e, int64_t cap_dofs, int64_t cap_slots);
// Condition estimate from k recorded PCG steps (alpha_j, beta_j pairs):
// the ratio of the extreme eigenvalues of CG's Lanczos tridiagonal, *steps
// = k; 0 and 0 when k < 2 or the record is not positive.
double lanczos_cond(const double *lz, int k, int *steps);

// Preconditioner of problems admitted from now on (0 Jacobi, 1 Jacobi plus
// the aggregate coarse correction) and the internal node order it needs.
mos_status engine_set_precond(mos_engine e, int precond);
mos_status engine_submit(mos_engine e, const mos_array_desc *d, void *vm, void *sig6, double *u_out,
                         int64_t *ticket);
mos_status engine_progress(mos_engine e, int chunk, std::vector<int64_t> *completed);
void engine_free(mos_engine e);
// Gather index [ldk][n_sb*16] (global DoF of cell DoF k in each slot, -1
// for padding) of a retired problem, enqueued on the context stream; `perm`
// is the device copy of the problem's slot -> cell map.
mos_status engine_gather_index(mos_engine e, const EngineProblem *P, const int32_t *perm, int32_t *gidx);
// Capacity (DoFs, slots) one problem needs, for sizing an engine exactly.
mos_status engine_problem_size(mos_engine e, const mos_array_desc *d, int64_t *dofs, int64_t *slots);

}  // namespace mos
