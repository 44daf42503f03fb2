// Internal declarations of the MI355X MORE-Stress library: handle layouts,
// device-memory helpers, error reporting and the kernel launchers each
// translation unit provides.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "mos.h"

namespace mos {

void set_error(const char *fmt, ...);

#define MOS_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::mos::set_error("%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,  \
                             __LINE__);                                                 \
            return MOS_EHIP;                                                            \
        }                                                                               \
    } while (0)

#define MOS_LAUNCH_CHECK() MOS_HIP(hipGetLastError())

#define MOS_TRY(expr)                       \
    do {                                    \
        mos_status s_ = (expr);             \
        if (s_ != MOS_OK) return s_;        \
    } while (0)

enum : uint32_t { KIND_CELL = 0x4c4c4543u, KIND_ROM = 0x214d4f52u, KIND_SOL = 0x214c4f53u };

// Tile edge of the banded Cholesky factor (64 x 64 FP64 tiles).
constexpr int NB = 64;
// Largest number of 32-wide k-steps (basis size <= 384) for which the BF16
// reconstruction keeps one element block of Psi (hi and lo) in LDS.
constexpr int RECON_BF16_MAX_KS = 12;

// A set of device allocations released together.
struct DeviceArena {
    mos_ctx ctx = nullptr;
    std::vector<void *> ptrs;
    size_t bytes = 0;
    mos_status alloc(size_t n, void **out);
    template <class T>
    mos_status alloc_n(size_t count, T **out) {
        return alloc(count * sizeof(T), reinterpret_cast<void **>(out));
    }
    void release();
};

}  // namespace mos

struct mos_ctx_s {
    int device = 0;
    int n_cu = 256;  // compute units of the device
    hipStream_t stream = nullptr;
    mos_allocator alloc{};
    bool user_alloc = false;
    // Small pinned host buffer for status words read back from the device.
    void *pinned = nullptr;
    // Kernel timing (mos_timing_start / mos_timing_stop).
    int timed_kernel = 0;
    int timed_every = 1;          // time one launch in this many
    int64_t timed_seen = 0;       // launches of the timed kernel so far
    std::vector<hipEvent_t> ev;   // pairs (start, stop), reused
    size_t ev_used = 0;
    // Lifetime: handles returned to the caller (cells, ROMs, solutions,
    // engines) each hold the context; mos_ctx_destroy marks it closing and
    // the last of it and its handles to go releases it, so handles may be
    // freed before or after the context.
    std::mutex life;
    int live = 0;
    bool closing = false;
};

namespace mos {
// When this launch of kernel `id` is sampled for timing, returns true and the
// event pair the dispatch itself stamps (start and end of its execution).
bool timer_take(mos_ctx ctx, int id, hipEvent_t *e0, hipEvent_t *e1);

// Sampled launches go through hipExtLaunchKernelGGL so that they carry their
// own execution timestamps; the others are plain launches (which stream
// capture records as kernel nodes).
template <typename F, typename... Args>
inline void launch_timed(mos_ctx ctx, int id, F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t stream,
                         Args... args) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timer_take(ctx, id, &e0, &e1))
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
}
}  // namespace mos

struct mos_cell_s {
    uint32_t kind = mos::KIND_CELL;
    mos_ctx ctx = nullptr;
    bool held = false;  // holds ctx (returned to the caller)
    mos_cell_desc desc{};
    int mx = 0, my = 0, mz = 0;
    int n_nodes = 0, n_dofs = 0, n_elem = 0;
    int64_t nnz = 0;
    int n_free = 0, bw = 0;       // interior DoFs and half bandwidth of K_ff
    int NT = 0, W = 0;            // tiles along the band and sub-diagonal tile count
    int n_bnodes = 0;             // boundary FE nodes
    mos::DeviceArena mem;
    // device arrays
    uint8_t *mat = nullptr;       // [n_elem] material code
    double *ke = nullptr;         // [3][24][24] element stiffness per material
    double *fe = nullptr;         // [3][24] unit-dT element load per material
    double *mprop = nullptr;      // [3][3] (lambda, mu, beta) per material
    int32_t *row_ptr = nullptr;   // [n_dofs+1]
    int32_t *col = nullptr;       // [nnz]
    double *val = nullptr;        // [nnz]
    double *b = nullptr;          // [n_dofs]
    int32_t *free_dof = nullptr;  // [n_free] FE DoF of each interior DoF
    int32_t *bnode = nullptr;     // [n_bnodes] FE node id of each boundary node
    double *tiles = nullptr;      // [NT][W+1][NB*NB] band of K_ff, column-major tiles
};

struct mos_rom_s {
    uint32_t kind = mos::KIND_ROM;
    mos_ctx ctx = nullptr;
    bool held = false;  // holds ctx (returned to the caller)
    mos_cell_desc desc{};
    int mx = 0, my = 0, mz = 0, n_dofs = 0, n_elem = 0;
    int n = 0, n_surf = 0;
    int ldp = 0;                  // row stride of phi (>= n+1, multiple of 8)
    int ldk = 0;                  // n rounded up to 16 (padded K_r edge)
    int n_eblk = 0;               // element blocks of 16
    double orth = 0.0;            // max |f_T^T K Phi| / max |K_r|, a health check
    mos::DeviceArena mem;
    double *phi = nullptr;        // [n_dofs][ldp]; column n holds f_T
    double *kr = nullptr;         // [n][n]
    double *br = nullptr;         // [n]
    double *kr_pad = nullptr;     // [ldk][ldk] zero padded
    float *kr32_pad = nullptr;    // FP32 copy of kr_pad
    double *psi = nullptr;        // [n_eblk][6][ldk][16] centroid stress basis
    double *sig_t = nullptr;      // [n_elem][6] unit-dT thermal stress at centroids
    int nks = 0;                  // 32-wide k-steps of the BF16 reconstruction GEMM
    uint16_t *psi_hi = nullptr;   // BF16 split of psi in MFMA A-operand order
    uint16_t *psi_lo = nullptr;   //   [n_eblk][6][nks][64][8]; null if nks > RECON_BF16_MAX_KS
    uint8_t *mat = nullptr;       // [n_elem] material code per element (copy of the cell's)
    double *mprop = nullptr;      // [3][3] (lambda, mu, beta) per material
    // Stress basis at the sample points of the mid-height plane, built on
    // first use: a ROM of its own whose psi / sig_t / psi_hi / psi_lo hold
    // the points (n_elem = grid^2 points, n_eblk their blocks of 16) and
    // whose other arrays are null.  Owned by this ROM.
    mos_rom_s *plane = nullptr;
    int plane_grid = 0;
};

struct mos_sol_s {
    uint32_t kind = mos::KIND_SOL;
    mos_ctx ctx = nullptr;
    bool held = false;  // holds ctx (returned to the caller)
    mos_precision precision = MOS_FP64;
    int Nx = 0, Ny = 0, n_cells = 0;
    int n = 0, n_surf = 0, n_elem = 0, ldk = 0, n_eblk = 0;
    int64_t n_nodes = 0, n_dofs = 0;
    double delta_T = 0.0;
    double rel_residual = 0.0;
    int iters = 0, refines = 0;
    std::vector<double> lz;                  // (alpha_j, beta_j) of the first sweep's PCG steps
    int n_types = 0;
    int n_pc = 0;                            // padded permuted cell slots
    std::vector<int> seg;                    // [n_types+1] slot ranges per type (multiples of 16)
    std::vector<mos_rom> roms;               // per type, borrowed
    mos::DeviceArena mem;
    int32_t *perm = nullptr;                 // [n_pc] cell id per slot or -1
    int32_t *gidx = nullptr;                 // [ldk][n_pc] global DoF of cell DoF k in slot, -1 pad
    double *u = nullptr;                     // [n_dofs] solution
};

namespace mos {

// ---- kernel launchers (defined in the .hip files) ----
// cell.hip
mos_status launch_cell_assembly(mos_cell c);
mos_status fill(mos_ctx ctx, double *p, size_t n, double v);
// dense.hip
mos_status band_cholesky(mos_cell c, double *dinv, int *status_dev, int *not_spd);
mos_status band_solve(mos_cell c, const double *dinv, double *rhs, int ldr, int ncols);
// reduce.hip
mos_status reduce_cell(mos_cell c, mos_rom r);
// Stress basis of r at the grid x grid sample points of the mid-height plane
// (built once per grid size and kept in r->plane; MOS_EINVAL for a grid
// outside [1, PLANE_MAX_GRID]).
constexpr int PLANE_MAX_GRID = 256;
mos_status plane_basis(mos_rom r, int grid);
// recon.hip
mos_status reconstruct(mos_ctx ctx, mos_sol s, uint32_t outputs, void *vm, void *sigma6);
// The same reconstruction with its device scratch in the library's static
// per-device array (NOALLOC_SCRATCH_BYTES; MOS_EINVAL for a solution that
// needs more): no device allocation.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
mos_status reconstruct_noalloc(mos_ctx ctx, mos_sol s, uint32_t outputs, void *vm, void *sigma6);
// Address of that array on `device` (current when called), looked up once
// per device at context creation; noalloc_scratch gives it back (NULL before).
mos_status noalloc_scratch_init(int device);
void *noalloc_scratch(int device);
mos_status reconstruct_plane(mos_ctx ctx, mos_sol s, int grid, void *vm);
mos_status reconstruct_displacement(mos_ctx ctx, mos_sol s, double *u_nodal);
// FP64 MFMA reconstruction with one element block of Psi staged in LDS per
// workgroup, for bases with ldk / 4 <= RECON_F64_LDS_KS (else MOS_EINVAL).
// A job is one problem's run of slot blocks of one type in the cell-major
// block U ([ldk][ld]); jobs[t] lists type t's jobs, in order, with sb_off the
// running count of slot blocks before each.  All of a type's jobs share one
// launch, so Psi is staged once for all of them.  The job table goes through
// host_jobs (pinned or otherwise stable until the copy completes) to
// dev_jobs (room for every job).  Outputs are FP32 when fp32_out.
constexpr int RECON_F64_LDS_KS = 44;
struct ReconJob {
    int32_t sb_first, sb_off, n_sb, pad;
    double dT;
    void *vm, *sig6;
};
mos_status recon_f64_jobs(mos_ctx ctx, const mos_rom *roms, int n_types, const std::vector<ReconJob> *jobs,
                          ReconJob *dev_jobs, ReconJob *host_jobs, const double *U, int ld, const int32_t *perm,
                          bool fp32_out);
// BF16-split MFMA reconstruction (FP32 outputs) of the slot blocks listed
// by the jobs of each type (as for recon_f64_jobs: a job covers slot blocks
// [sb_first, sb_first + n_sb) of U, its outputs and dT, at sb_off within its
// type's flattened list).  Needs roms with psi_hi (nks <= RECON_BF16_MAX_KS),
// else MOS_EINVAL, and a device scratch of recon_bf16_scratch(rom, total
// slot blocks) bytes; the host table must outlive the upload.
int64_t recon_bf16_scratch(const mos_rom r, int n_sb);
mos_status recon_bf16_jobs(mos_ctx ctx, const mos_rom *roms, int n_types, const std::vector<ReconJob> *jobs,
                           ReconJob *dev_jobs, ReconJob *host_jobs, const double *U, int ld, const int32_t *perm,
                           void *split);

// ---- host helpers (api.cpp) ----
inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

}  // namespace mos
