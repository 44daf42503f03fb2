/*
 * mos.h - C ABI of the MI355X library for MORE-Stress, the model-order-reduced
 * thermal-stress solve of periodic TSV arrays (arXiv 2411.12690).
 *
 * The four stage calls follow the paper's problem statement:
 *   mos_build_cell   unit block -> fine FE system          (Sec. 3.2, 4.2; eq. 1-7, 11-12)
 *   mos_reduce       FE system -> reduced order model      (Sec. 4.2-4.3; eq. 8-19)
 *   mos_solve_array  ROMs + array layout -> reduced u      (Sec. 4.3-4.4; eq. 20)
 *   mos_reconstruct  reduced u -> per-cell stress          (Sec. 4.3, last paragraph; eq. 1, 15)
 *   mos_reconstruct_plane  von Mises on each cell's mid-height sample grid (Sec. 5.1)
 *   mos_reconstruct_displacement  fine-mesh displacement of every cell (eq. 15)
 *
 * Conventions
 *   Units: micrometres, MPa, 1/K, K.  Stress in MPa, displacement in um.
 *   Every call returns mos_status; on failure *out is set to NULL, nothing is
 *   written to caller buffers, and mos_last_error() (thread-local) describes
 *   the failure.  No C++ exception crosses this boundary.
 *   Handles are owned by the library and released with the matching *_free.
 *   Host input arrays are read during the call only (copied if kept).
 *   "device" pointers are HIP device addresses on the context's device;
 *   device work is enqueued on the context's stream.  Calls that return
 *   host data or status synchronise that stream.
 *   A context and its handles must be used from one host thread at a time.
 *
 * Numbering contracts (shared with any independent implementation)
 *   Cell FE node (a,b,c), 0<=a<=m_x etc., has id (c*(m_y+1)+b)*(m_x+1)+a and
 *   DoF 3*id+component.  Cell element (ea,eb,ec) has id (ec*m_y+eb)*m_x+ea.
 *   Lagrange surface node (i,j,k) of a cell (i in {0,n_x-1} or j in {0,n_y-1}
 *   or k in {0,n_z-1}) has local index s = its rank in (k,j,i) lexicographic
 *   order, i fastest; the reduced cell DoF is 3*s+component (eq. 14-16).
 *   The abstract array mesh of N_x x N_y blocks in N_z layers (N_z = 1 for
 *   one layer) has lattice X = N_x(n_x-1)+1, Y = N_y(n_y-1)+1,
 *   Z = N_z(n_z-1)+1; lattice point (I,J,K) is a node iff I%(n_x-1)==0 or
 *   J%(n_y-1)==0 or K%(n_z-1)==0; node id = rank in (K,J,I) order, I
 *   fastest; global DoF 3*id+component.  Cell (cx,cy,cz) has id
 *   (cz*N_y+cy)*N_x+cx and its surface node (i,j,k) is lattice point
 *   (cx(n_x-1)+i, cy(n_y-1)+j, cz(n_z-1)+k).
 */
#ifndef MOS_H
#define MOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MOS_OK = 0,
    MOS_EINVAL = -1,      /* invalid argument or incompatible handles */
    MOS_ENOMEM = -2,      /* device or host allocation failed */
    MOS_ENOCONV = -3,     /* iterative solve did not reach the tolerance */
    MOS_ESINGULAR = -4,   /* matrix not positive definite / no constraints */
    MOS_EHIP = -5,        /* HIP runtime error */
    MOS_EBUSY = -6        /* resource temporarily unavailable (serving) */
} mos_status;

typedef enum { MOS_FP64 = 0, MOS_MIXED = 1 } mos_precision;

typedef struct mos_ctx_s *mos_ctx;
typedef struct mos_cell_s *mos_cell;
typedef struct mos_rom_s *mos_rom;
typedef struct mos_sol_s *mos_sol;

/* Isotropic linear thermo-elastic material (eq. 1-2): E [MPa], nu [-], alpha [1/K]. */
typedef struct { double E, nu, alpha; } mos_material;

/* Repeated fine structure of a unit block (the method applies to any,
 * Sec. 4.1; TSVs and micro-bumps are the arrays Sec. 1 names). */
enum { MOS_CELL_TSV = 0, MOS_CELL_BUMP = 1 };

/* Unit block of Sec. 4.2 / Fig. 2: a pitch_x x pitch_y x height cuboid of
 * `matrix` with a centred via of diameter tsv_diameter (0 = dummy block,
 * Sec. 4.4) and a liner of liner_thickness around it, meshed as a structured
 * mesh[0] x mesh[1] x mesh[2] grid of trilinear hexahedra; an element takes
 * the via material if its centroid's distance r to the via axis satisfies
 * r < d/2, the liner if r < d/2 + t, else the matrix.  interp[] is the number
 * of equally spaced Lagrange nodes per axis (n_x, n_y, n_z) >= 2 (eq. 8-10).
 * structure MOS_CELL_BUMP makes it a micro-bump block instead: `matrix` is
 * the underfill, and a centred column of diameter tsv_diameter is solder
 * (`via`) except for pads of pad_thickness at its two ends (`liner`): an
 * element with r < d/2 is pad if its centroid height z satisfies
 * z < pad_thickness or z > height - pad_thickness, else solder.  A bump
 * block needs liner_thickness = 0 and 0 <= 2 pad_thickness < height; a TSV
 * block needs pad_thickness = 0 (MOS_EINVAL otherwise).  skew shears every
 * point of the block, x += skew * y (the grid, the via axis through the
 * block's centre, node coordinates), making it a parallelepiped: skew =
 * 1/sqrt(3) with pitch_y = pitch_x sqrt(3)/2 is the rhombic block of a
 * 120-degree array (Sec. 4.2), TSVs on a triangular lattice of spacing
 * pitch_x.  Interpolation and numbering stay in the block's reference
 * coordinates.  0 is the rectangular block; it must be finite and
 * |skew| <= 4. */
typedef struct {
    double pitch_x, pitch_y, height;
    int32_t mesh[3];
    double tsv_diameter, liner_thickness;
    mos_material matrix, via, liner;
    int32_t interp[3];
    int32_t structure;
    double pad_thickness;
    double skew;
} mos_cell_desc;

enum { MOS_BC_CLAMP_BOTTOM = 1, MOS_BC_CLAMP_TOP = 2, MOS_BC_LIST_ON_DEVICE = 4 };

/* One global-stage problem (Sec. 4.3-4.4).  cell_type[(cz*ny_cells+cy)*nx_cells+cx]
 * indexes the roms[] array passed with it (host memory).  nz_cells > 1 stacks
 * that many layers of blocks in z, sharing their horizontal faces (0 or 1:
 * one layer); stacked arrays take the Jacobi preconditioner
 * (MOS_OPT_PRECOND 0; mos_solve_array selects it by itself).  Constrained DoFs: the
 * clamped faces (value 0) and then the prescribed (global DoF, value) list,
 * a later entry overriding an earlier one; the system is lifted
 * symmetrically (Sec. 4.2 eq. 13 form, same solution).  rtol bounds the
 * FP64 true residual ||b - A u||_2 / ||b||_2 (0 selects 1e-12 for MOS_FP64,
 * 1e-10 for MOS_MIXED); max_iters bounds the total PCG iterations (0 selects
 * 20000).  The prescribed list is host memory, copied during the call,
 * unless bc_flags has MOS_BC_LIST_ON_DEVICE: then prescribed_dof and
 * prescribed_value are device arrays of the context's device (caller-owned,
 * read on the context's stream when the problem is set up, so they must stay
 * valid and unchanged until its ticket completes or mos_solve_array
 * returns), and their entries are checked on the device: a DoF outside
 * [0, n_dofs) or a non-finite value fails the problem with MOS_EINVAL
 * (the ticket's status, or mos_solve_array's return). */
typedef struct {
    int32_t nx_cells, ny_cells;
    const uint8_t *cell_type;
    double delta_T;
    uint32_t bc_flags;
    int64_t n_prescribed;
    const int64_t *prescribed_dof;
    const double *prescribed_value;
    mos_precision precision;
    double rtol;
    int32_t max_iters;
    int32_t nz_cells;
} mos_array_desc;

/* Optional device allocator (e.g. a framework's caching allocator).  NULL
 * members select hipMalloc / hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} mos_allocator;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  `alloc` may be NULL. */
mos_status mos_ctx_create(int device, void *hip_stream, const mos_allocator *alloc, mos_ctx *out);
/* Release the context.  Cells, ROMs, solutions and engines made from it may
 * be freed before or after this call, in any order: each holds the context,
 * and its stream, allocator and pinned memory are released when the last of
 * them (or this call, if none is left) goes.  After this call the context
 * must not be passed to any other entry point; the allocator's callbacks
 * must stay callable until the last handle is freed. */
void mos_ctx_destroy(mos_ctx ctx);

/* Sec. 3.2 and 4.2 (eq. 1-7, 11-12): mesh the unit block, assign materials,
 * and assemble on the device the FE stiffness K (CSR, 27-node stencil) and the
 * unit-dT thermal load b of the whole block, plus K_ff of the interior DoFs
 * in band form.  Errors: MOS_EINVAL for a non-positive size, a mesh axis
 * outside [2, 128], interp outside [2, 8], nu outside (-1, 0.5), E <= 0. */
mos_status mos_build_cell(mos_ctx ctx, const mos_cell_desc *desc, mos_cell *out);

/* Sec. 4.2-4.3 (eq. 8-19): Lagrange weights L of the boundary FE nodes, one
 * Cholesky factorisation of K_ff and n+1 solves giving Phi = [f_0..f_{n-1}]
 * and f_T, then A_element = K_r = sym(Phi^T K Phi), b_element = b_r =
 * Phi^T b, and the centroid stress basis used by mos_reconstruct.  The ROM
 * stays resident in device memory.  Errors: MOS_ESINGULAR if K_ff is not
 * positive definite.  The cell may be freed afterwards. */
mos_status mos_reduce(mos_ctx ctx, mos_cell cell, mos_rom *out);

/* Sec. 4.3-4.4 (eq. 20): assemble the reduced global system of the array
 * element by element, lift the constraints, and solve with Jacobi-PCG
 * (MOS_FP64: FP64 throughout; MOS_MIXED: FP32 PCG corrections inside FP64
 * iterative refinement on the true residual).  All roms must share pitch,
 * height, mesh and interp (MOS_EINVAL otherwise).  An array with no
 * constrained DoF is MOS_ESINGULAR; PCG breakdown or max_iters is
 * MOS_ENOCONV (the handle is still returned NULL). */
mos_status mos_solve_array(mos_ctx ctx, const mos_array_desc *desc, const mos_rom *roms,
                           int32_t n_roms, mos_sol *out);

enum { MOS_OUT_VM = 1, MOS_OUT_SIGMA6 = 2 };
/* Sec. 4.3 last paragraph with eq. 1 and 15: per cell c and fine element e,
 * sigma = dT sigma_T(e) + Psi(e) u_c with Psi = D B0 Phi at the element
 * centroid; von Mises from sigma.  vm: device array [n_cells][n_elem],
 * sigma6: device array [n_cells][n_elem][6] (xx,yy,zz,xy,yz,zx); element
 * order as in the numbering contract.  Element type is double for a
 * MOS_FP64 solution and float for MOS_MIXED.  Either pointer may be NULL
 * when its flag is not set. */
mos_status mos_reconstruct(mos_ctx ctx, mos_sol sol, uint32_t outputs, void *vm, void *sigma6);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * outputs of mos_reconstruct, bit for bit (same kernels, same order), with
 * its device scratch -- the job table, the cell-major gather of the
 * solution (8 ldk bytes per cell slot) and, for MOS_MIXED, its BF16 hi/lo
 * split (64 nks bytes per slot) -- taken from one static array of 32 MiB
 * per device that the library holds from the first mos_ctx_create on that
 * device until the process ends.  Nothing is allocated on the device.  A
 * solution whose scratch exceeds 32 MiB is rejected with MOS_EINVAL (with a
 * cubic basis: about 23,000 cells in FP64, 15,000 mixed).  All calls on one
 * device share the array and each leaves its contents behind (nothing in it
 * needs to start at zero): calls that overlap on one device (other threads,
 * or other contexts' streams) race.  Returns after the context's stream
 * has finished the call's work. */
mos_status mos_reconstruct_noalloc(mos_ctx ctx, mos_sol sol, uint32_t outputs, void *vm, void *sigma6);

/* Sec. 4.3 with eq. 15: the fine-mesh displacement of every cell,
 * u_cell = dT f_T + Phi u_r,cell over the cell's FE DoFs (DoF 3 node +
 * component, node and component order as in the cell numbering contract).
 * u_nodal: caller-owned device array of double [n_cells][n_fe_dofs]
 * (n_fe_dofs = mos_query(rom, MOS_Q_CELL_DOFS)), FP64 for either precision,
 * written on the context's stream (complete when the call returns).
 * Errors: MOS_EINVAL for a NULL u_nodal or a solution whose ROMs were
 * freed. */
mos_status mos_reconstruct_displacement(mos_ctx ctx, mos_sol sol, void *u_nodal);

/* The paper's evaluation plane (Sec. 5.1, error metric of Tables 1-3): von
 * Mises stress of every cell at grid x grid points of its mid-height plane,
 * sigma = dT sigma_T(p) + Psi(p) u_c with Psi(p) = D B(p) Phi at the point
 * (eq. 1 and 15).  Point p = j*grid + i of a cell sits at x = pitch_x (i +
 * 1/2) / grid, y = pitch_y (j + 1/2) / grid, z = height / 2 within the cell,
 * in the fine element whose half-open box [x_a, x_a+1) x [y_b, y_b+1) x
 * [z_c, z_c+1) holds it (points on an element face take the +x / +y / +z
 * element).  vm: caller-owned device array [n_cells][grid*grid], double for
 * a MOS_FP64 solution and float for MOS_MIXED, written on the context's
 * stream (complete when the call returns).  The first call for a ROM and
 * grid builds that ROM's plane stress basis (6 grid^2 x n, FP64, plus its
 * BF16 split) and keeps it with the ROM until mos_rom_free or a call with
 * another grid; a call with another grid first waits for the stream.  The
 * call modifies the ROM: calls that use the same ROM must not run
 * concurrently with it from other threads.
 * Errors: MOS_EINVAL for a NULL vm, a grid outside [1, 256], a solution
 * whose ROMs were freed, or skewed blocks (the plane is defined for
 * rectangular ones); MOS_ENOMEM if the basis does not fit. */
mos_status mos_reconstruct_plane(mos_ctx ctx, mos_sol sol, int32_t grid, void *vm);

/* Copy the reduced solution (n_global_dofs doubles) to host memory and report
 * the final relative true residual and total PCG iterations (any may be NULL). */
mos_status mos_get_solution(mos_sol sol, double *u_host, double *rel_residual, int32_t *iters);
/* Estimate of the condition number of the preconditioned operator M^-1 A
 * of the reduced system (eq. 20) that the PCG solved, from its own step
 * sizes: the steps alpha_j, beta_j of the first sweep (at most its first
 * 128) define the Lanczos tridiagonal of CG, whose extreme Ritz values lie
 * inside the spectrum of M^-1 A and approach the ends of the part of it
 * that the right-hand side excites (a load with no weight on an extreme
 * eigenvector never reaches that end), so *kappa is their ratio: a lower
 * bound, close once the sweep has converged on a generic load; *steps =
 * the steps used.  0 and 0 when the first sweep took fewer than two steps
 * (a zero load takes none), or when the engine could not allocate its
 * 2 MiB pinned host record of the steps (the solve itself is unaffected).  The mixed path reports its FP32 inner
 * solve's operator.  MOS_EINVAL for an invalid handle. */
mos_status mos_get_cond_estimate(mos_sol sol, double *kappa, int32_t *steps);

enum {
    MOS_Q_N = 1,            /* rom/cell: reduced DoFs per cell, n (eq. 16) */
    MOS_Q_CELL_DOFS = 2,    /* rom/cell: FE DoFs of the block */
    MOS_Q_CELL_ELEMS = 3,   /* rom/cell: fine elements of the block */
    MOS_Q_CELL_NNZ = 4,     /* cell: nonzeros of K */
    MOS_Q_FREE_DOFS = 5,    /* cell: interior DoFs */
    MOS_Q_BANDWIDTH = 6,    /* cell: half bandwidth of K_ff */
    MOS_Q_GLOBAL_DOFS = 7,  /* sol: reduced global DoFs */
    MOS_Q_ITERS = 8,        /* sol: total PCG iterations */
    MOS_Q_REFINES = 9,      /* sol: FP64 refinement sweeps */
    MOS_Q_DEVICE_BYTES = 10 /* any handle: device bytes it holds */
};
mos_status mos_query(const void *handle, int what, int64_t *value);

/* Parity exports (host buffers, caller-owned).  Cell: K as CSR over all FE
 * DoFs (row_ptr[n_dofs+1], col[nnz], val[nnz]), b[n_dofs], material code per
 * element (0 matrix, 1 via, 2 liner).  Any pointer may be NULL. */
mos_status mos_cell_export(mos_cell cell, int64_t *row_ptr, int32_t *col, double *val, double *b,
                           uint8_t *material);
/* ROM: Phi row-major [n_dofs][n], f_T[n_dofs], K_r row-major [n][n], b_r[n]. */
mos_status mos_rom_export(mos_rom rom, double *phi, double *f_T, double *K_r, double *b_r);

/* Abstract array mesh of nx_cells x ny_cells (x nz_cells stacked layers;
 * 0 or 1: one layer) blocks shaped like `rom` (numbering contract above).
 * n_nodes receives the node count; when the arrays are non-NULL:
 * coords[n_nodes][3] (um), conn[n_cells][n/3] node ids,
 * and the sparsity pattern of the assembled global matrix over DoFs
 * (union of per-cell dense blocks, columns ascending): row_ptr[3 n_nodes + 1]
 * and col[row_ptr[3 n_nodes]].  Call with col == NULL first to size it. */
mos_status mos_array_layout(mos_ctx ctx, int32_t nx_cells, int32_t ny_cells, int32_t nz_cells, mos_rom rom,
                            int64_t *n_nodes, double *coords, int32_t *conn, int64_t *row_ptr,
                            int32_t *col);

/* ---- Batched / served global stage ----------------------------------------
 * An engine keeps device arenas for many array problems that share one set
 * of ROMs (same cell mesh and interp; pitch and height may differ between
 * ROMs, but the cells of one array must agree on them) and one precision.  Problems
 * are submitted at any time, admitted in arrival order when their DoFs and
 * cell slots fit in the arenas (the device-memory budget), and advanced
 * together: every mos_engine_progress call admits what fits, runs
 * `iterations` PCG iterations of all admitted problems in shared launches,
 * refines / retires problems whose inner solve stopped, and reconstructs
 * retired problems into the buffers given at submission.  Per-problem
 * reductions are segmented and in a fixed order, so a problem's result is the
 * same alone or in any mix.  For callers that batch requests of different
 * sizes (continuous batching). */
typedef struct mos_engine_s *mos_engine;

/* device_bytes: arena budget; a problem larger than the arenas is rejected
 * with MOS_EINVAL at submission.  One engine addresses at most 4,194,304
 * cell slots (each cell type of a problem takes its cells rounded up to 16),
 * so a budget beyond that (about 45 GB in FP64) is used only up to it.
 * roms must outlive the engine. */
mos_status mos_engine_create(mos_ctx ctx, const mos_rom *roms, int32_t n_roms, mos_precision precision,
                             size_t device_bytes, mos_engine *out);
/* Queue one problem (desc->precision must equal the engine's).  vm / sigma6:
 * optional device outputs as for mos_reconstruct; u: optional device array of
 * the problem's reduced DoFs for the solution.  Buffers must stay valid until
 * the ticket completes. */
mos_status mos_engine_submit(mos_engine e, const mos_array_desc *desc, void *vm, void *sigma6, double *u,
                             int64_t *ticket);
/* One round of admission, `iterations` PCG iterations and retirement.
 * Tickets completed since the last call are written to completed[] (up to
 * max_completed; the rest are reported by the next call).  A ticket is
 * reported only once the device has finished writing its outputs
 * (reconstruction and u): a problem that retires while others still iterate
 * is reported by a later call (at the latest after the next chunk); when
 * nothing is left to iterate the call waits for the retirements itself. */
mos_status mos_engine_progress(mos_engine e, int32_t iterations, int64_t *completed, int32_t max_completed,
                               int32_t *n_completed);
/* Outcome of a completed ticket (status MOS_OK or the failure code), its
 * relative FP64 residual, PCG iterations and refinement sweeps; the ticket is
 * forgotten afterwards.  MOS_EBUSY if it has not completed. */
mos_status mos_engine_result(mos_engine e, int64_t ticket, int32_t *status, double *rel_residual, int32_t *iters,
                             int32_t *sweeps);
/* The condition estimate of mos_get_cond_estimate for a completed ticket,
 * taken before mos_engine_result forgets the ticket (MOS_EBUSY if it has
 * not completed or was already taken). */
mos_status mos_engine_cond_estimate(mos_engine e, int64_t ticket, double *kappa, int32_t *steps);
/* Engine options.  MOS_OPT_CELL_GEMM selects the cell-GEMM variant of the
 * PCG matvec (the per-type product K_r * u_cell of eq. 20 over all cells):
 * 1 = 16x16 output tiles with the contraction split over four waves (any
 * basis size); 2 = K_r-stationary rows: each wave holds 16 rows of K_r in
 * registers and streams consecutive 16-cell blocks of the operand from
 * global memory; 3 = the same chains, with each 16-cell operand tile read
 * once per workgroup (one wave per row block of K_r) and staged in LDS.
 * 2 and 3 apply to basis sizes up to 176 (interpolation up to 4 nodes per
 * axis); elsewhere they run 1.  0 (the default) = the K_r-stationary rows
 * where they apply, with the engine choosing between 2 and 3 online per
 * batch size, else 1.  2, 3 and 0 give the same bits; 1 can differ from
 * them in the last bits.  Set it before the first submission; results never
 * depend on the batch composition. */
/* MOS_OPT_GEMM_SPLIT sets how many consecutive 16-cell blocks one wave
 * (variant 2) or one workgroup (variant 3) of the K_r-stationary GEMM
 * streams: 0 (default) lets the engine tune it online per batch size (each
 * candidate in {1, 2, 4, 8, 16, 32}, for each operand path allowed, and for
 * variant 3 also ceil(blocks / compute units), one workgroup per unit, is
 * timed three times with stream events and the fastest kept); 1 <= k <= 64 fixes
 * it.  It only decides which wave computes which output tile, so results do
 * not depend on it; it may be changed at any time (tuning starts over). */
/* MOS_OPT_UPDATE_WIDTH sets the threads per workgroup of the PCG vector
 * update: 256 (one DoF each) or 128 (two DoFs each); 0 (default) takes 256
 * while the iterating DoF blocks fit on the chip at once and 128 beyond.
 * Both compute every sum in the same order, so results do not depend on it;
 * it may be changed at any time. */
/* MOS_OPT_PRECOND selects the PCG preconditioner of problems submitted
 * afterwards: 1 (the default where it applies) = Jacobi plus a coarse
 * correction on aggregates of 2x2 cells, M^-1 = D^-1 + sum_a Z_a B_a^-1 Z_a^T
 * with Z_a the aggregate's six rigid-body modes on its free DoFs and
 * B_a = Z_a^T A Z_a (symmetric positive definite, so PCG converges to the
 * same solution in fewer iterations); 0 = Jacobi alone.  1 needs cells of at
 * most 512 reduced DoFs and at most 1024 nodes in a box of 6x2 cells
 * (MOS_EINVAL otherwise; engines whose cells exceed this start with 0).
 * Set it before the first submission. */
/* MOS_OPT_GRAPH = 1 replays each chunk of PCG iterations (the launches of
 * mos_engine_progress's chunk: cell GEMM, scalar and update launches of
 * every iteration) from a HIP graph captured once per launch shape (batch
 * extents, chunk length, chosen GEMM split) instead of launching its
 * kernels one by one; 0 (default) launches them directly.  Chunks during a
 * GEMM tuning trial, or while mos_timing_start samples one of the chunk's
 * kernels, are launched directly either way.  The kernels and their
 * arguments are the same, so results do not depend on it; it may be
 * changed at any time. */
/* MOS_OPT_COARSE_TABLE (two-level preconditioner): 1 (default) builds each
 * aggregate's B_a from per-type tables of the cell terms wherever the
 * aggregate's constrained DoFs are whole bottom / top planes (always for
 * clamp-only problems; for problems with a prescribed list, every aggregate
 * whose cells carry no prescribed value off those planes), and from the
 * cells' K_r rows elsewhere; 0 builds every aggregate of problems with a
 * prescribed list from the K_r rows.  Both give the same B_a up to rounding
 * (only the preconditioner, never the converged solution); it applies to
 * problems submitted afterwards. */
enum { MOS_OPT_CELL_GEMM = 1, MOS_OPT_GEMM_SPLIT = 2, MOS_OPT_UPDATE_WIDTH = 3, MOS_OPT_PRECOND = 4,
       MOS_OPT_GRAPH = 5, MOS_OPT_COARSE_TABLE = 6 };
mos_status mos_engine_option(mos_engine e, int option, int64_t value);
/* Counts of iteration-chunk graph captures and replays so far (MOS_OPT_GRAPH;
 * either pointer may be NULL). */
mos_status mos_engine_graph_stats(mos_engine e, int64_t *captures, int64_t *replays);

/* Problems admitted and queued, and the arena capacities. */
mos_status mos_engine_stats(mos_engine e, int64_t *active, int64_t *queued, int64_t *capacity_dofs,
                            int64_t *capacity_slots);
void mos_engine_destroy(mos_engine e);

/* Kernel timing for measurement tools.  After mos_timing_start(ctx, k, every)
 * every `every`-th launch (every >= 1) of kernel k by this context is
 * bracketed by a pair of HIP events on the context stream; mos_timing_stop
 * synchronises the stream and returns the number of timed launches, their
 * summed duration in milliseconds and the number of launches of the kernel
 * seen since the start (timed or not), then stops timing.  One kernel at a
 * time. */
enum {
    MOS_K_CELL_GEMM = 1,    /* element-by-element K_r GEMM of the PCG matvec */
    MOS_K_PCG_SCALARS = 2,  /* per-problem fixed-order reductions and CG step */
    MOS_K_PCG_UPDATE = 3,   /* PCG vector updates and reductions */
    MOS_K_RECON = 4,        /* stress reconstruction GEMM + von Mises */
    MOS_K_COUNT = 5
};
mos_status mos_timing_start(mos_ctx ctx, int kernel, int every);
mos_status mos_timing_stop(mos_ctx ctx, int64_t *launches, double *total_ms, int64_t *seen);

void mos_cell_free(mos_cell cell);
void mos_rom_free(mos_rom rom);
void mos_sol_free(mos_sol sol);

/* Thread-local description of the last failure on this thread. */
const char *mos_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOS_H */
