// C ABI entry points: argument checking, handle lifetime, host-side
// numbering of the abstract array mesh (Sec. 4.3), and dispatch to the
// device stages.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"
#include "mesh.h"
#include "mos_internal.h"

namespace mos {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

mos_status DeviceArena::alloc(size_t n, void **out) {
    *out = nullptr;
    if (n == 0) n = 16;
    n = (size_t)round_up((int64_t)n, 256);
    void *p = nullptr;
    if (ctx->user_alloc) {
        p = ctx->alloc.alloc(n, ctx->alloc.user);
        if (!p) {
            set_error("device allocation of %zu bytes failed (user allocator)", n);
            return MOS_ENOMEM;
        }
    } else {
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
            return MOS_ENOMEM;
        }
    }
    ptrs.push_back(p);
    bytes += n;
    *out = p;
    return MOS_OK;
}

void DeviceArena::release() {
    if (!ctx) return;
    if (!ptrs.empty()) (void)hipStreamSynchronize(ctx->stream);
    for (void *p : ptrs) {
        if (ctx->user_alloc) ctx->alloc.free(p, ctx->alloc.user);
        else (void)hipFree(p);
    }
    ptrs.clear();
    bytes = 0;
}

bool timer_take(mos_ctx ctx, int id, hipEvent_t *e0, hipEvent_t *e1) {
    *e0 = *e1 = nullptr;
    if (!ctx || ctx->timed_kernel != id) return false;
    if (ctx->timed_seen++ % ctx->timed_every) return false;
    if (ctx->ev_used + 2 > ctx->ev.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        ctx->ev.push_back(a);
        ctx->ev.push_back(b);
    }
    *e0 = ctx->ev[ctx->ev_used];
    *e1 = ctx->ev[ctx->ev_used + 1];
    ctx->ev_used += 2;
    return true;
}

// ---------------------------------------------------------------------------
// Abstract array mesh (numbering contract in mos.h)
// ---------------------------------------------------------------------------
void surface_nodes(int nx, int ny, int nz, std::vector<int> &ijk) {
    ijk.clear();
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1 || k == 0 || k == nz - 1) {
                    ijk.push_back(i);
                    ijk.push_back(j);
                    ijk.push_back(k);
                }
}

void ArrayMesh::build(int Nx_, int Ny_, int nx_, int ny_, int nz_, int Nz_) {
    Nx = Nx_;
    Ny = Ny_;
    Nz = Nz_;
    nx = nx_;
    ny = ny_;
    nz = nz_;
    lat = make_lattice(Nx, Ny, nx, ny, nz, Nz);
    X = lat.X;
    Y = lat.Y;
    Z = lat.Z;
    n_nodes = lat.n_nodes;
    surface_nodes(nx, ny, nz, surf);
    S = (int)surf.size() / 3;
    conn.resize((size_t)Nx * Ny * Nz * S);
    for (int cz = 0; cz < Nz; ++cz)
        for (int cy = 0; cy < Ny; ++cy)
            for (int cx = 0; cx < Nx; ++cx) {
                const size_t c = ((size_t)cz * Ny + cy) * Nx + cx;
                for (int s = 0; s < S; ++s)
                    conn[c * S + s] = (int32_t)node_id(lat, (int64_t)cx * (nx - 1) + surf[3 * s],
                                                       (int64_t)cy * (ny - 1) + surf[3 * s + 1],
                                                       (int64_t)cz * (nz - 1) + surf[3 * s + 2]);
            }
}

}  // namespace mos

using namespace mos;

static bool valid_material(const mos_material &m) {
    return std::isfinite(m.E) && m.E > 0.0 && std::isfinite(m.nu) && m.nu > -1.0 && m.nu < 0.5 &&
           std::isfinite(m.alpha);
}

static mos_status check_cell_desc(const mos_cell_desc *d) {
    if (!d) {
        set_error("descriptor is NULL");
        return MOS_EINVAL;
    }
    if (!(d->pitch_x > 0 && d->pitch_y > 0 && d->height > 0) || !std::isfinite(d->pitch_x) ||
        !std::isfinite(d->pitch_y) || !std::isfinite(d->height)) {
        set_error("pitch and height must be positive and finite");
        return MOS_EINVAL;
    }
    for (int a = 0; a < 3; ++a) {
        if (d->mesh[a] < 2 || d->mesh[a] > 128) {
            set_error("mesh[%d] = %d outside [2, 128]", a, d->mesh[a]);
            return MOS_EINVAL;
        }
        if (d->interp[a] < 2 || d->interp[a] > 8) {
            set_error("interp[%d] = %d outside [2, 8]", a, d->interp[a]);
            return MOS_EINVAL;
        }
    }
    {
        int nx = d->interp[0], ny = d->interp[1], nz = d->interp[2];
        int S = nx * ny * nz - (nx - 2) * (ny - 2) * (nz - 2);
        if (S > MAX_SURF) {
            set_error("interp (%d,%d,%d) has %d surface nodes, more than %d", nx, ny, nz, S, MAX_SURF);
            return MOS_EINVAL;
        }
    }
    if (!(d->tsv_diameter >= 0) || !(d->liner_thickness >= 0) || !std::isfinite(d->tsv_diameter) ||
        !std::isfinite(d->liner_thickness)) {
        set_error("tsv_diameter and liner_thickness must be finite and >= 0");
        return MOS_EINVAL;
    }
    if (!std::isfinite(d->skew) || !(std::fabs(d->skew) <= 4.0)) {
        set_error("skew must be finite with |skew| <= 4");
        return MOS_EINVAL;
    }
    if (d->structure != MOS_CELL_TSV && d->structure != MOS_CELL_BUMP) {
        set_error("structure %d is neither MOS_CELL_TSV nor MOS_CELL_BUMP", d->structure);
        return MOS_EINVAL;
    }
    if (!std::isfinite(d->pad_thickness) || !(d->pad_thickness >= 0)) {
        set_error("pad_thickness must be finite and >= 0");
        return MOS_EINVAL;
    }
    if (d->structure == MOS_CELL_TSV && d->pad_thickness != 0) {
        set_error("a TSV block has no pads (pad_thickness must be 0)");
        return MOS_EINVAL;
    }
    if (d->structure == MOS_CELL_BUMP && (d->liner_thickness != 0 || !(2 * d->pad_thickness < d->height))) {
        set_error("a micro-bump block needs liner_thickness = 0 and 2 pad_thickness < height");
        return MOS_EINVAL;
    }
    if (!valid_material(d->matrix) || !valid_material(d->via) || !valid_material(d->liner)) {
        set_error("material needs E > 0, -1 < nu < 0.5 and finite alpha");
        return MOS_EINVAL;
    }
    int64_t dofs = 3LL * (d->mesh[0] + 1) * (d->mesh[1] + 1) * (d->mesh[2] + 1);
    if (dofs * 81 > (int64_t)INT32_MAX) {
        set_error("cell mesh too large for 32-bit sparse indices");
        return MOS_EINVAL;
    }
    return MOS_OK;
}

// Context lifetime (see mos_ctx_s::life): a handle returned to the caller
// holds its context until it is freed.
static void ctx_teardown(mos_ctx ctx) {
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    delete ctx;
}

static void ctx_hold(mos_ctx ctx) {
    std::lock_guard<std::mutex> g(ctx->life);
    ++ctx->live;
}

static void ctx_drop(mos_ctx ctx) {
    bool last;
    {
        std::lock_guard<std::mutex> g(ctx->life);
        last = --ctx->live == 0 && ctx->closing;
    }
    if (last) ctx_teardown(ctx);
}

extern "C" {

const char *mos_last_error(void) { return g_err; }

mos_status mos_ctx_create(int device, void *hip_stream, const mos_allocator *alloc, mos_ctx *out) {
    if (!out) {
        set_error("out is NULL");
        return MOS_EINVAL;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        set_error("no HIP device available (%s)", hipGetErrorString(e));
        return MOS_EHIP;
    }
    if (device < 0 || device >= n) {
        set_error("device %d out of range [0, %d)", device, n);
        return MOS_EINVAL;
    }
    if (alloc && ((alloc->alloc == nullptr) != (alloc->free == nullptr))) {
        set_error("allocator needs both alloc and free");
        return MOS_EINVAL;
    }
    MOS_HIP(hipSetDevice(device));
    MOS_TRY(noalloc_scratch_init(device));
    mos_ctx c = new (std::nothrow) mos_ctx_s();
    if (!c) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->n_cu = cus;
    else
        (void)hipGetLastError();
    if (alloc && alloc->alloc) {
        c->alloc = *alloc;
        c->user_alloc = true;
    }
    e = hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        set_error("hipHostMalloc failed: %s", hipGetErrorString(e));
        return MOS_ENOMEM;
    }
    *out = c;
    return MOS_OK;
}

void mos_ctx_destroy(mos_ctx ctx) {
    if (!ctx) return;
    bool now;
    {
        std::lock_guard<std::mutex> g(ctx->life);
        ctx->closing = true;
        now = ctx->live == 0;
    }
    if (now) ctx_teardown(ctx);
}

mos_status mos_timing_start(mos_ctx ctx, int kernel, int every) {
    if (!ctx || kernel < 1 || kernel >= MOS_K_COUNT || every < 1) {
        set_error("invalid context, kernel id or sampling interval");
        return MOS_EINVAL;
    }
    ctx->timed_kernel = kernel;
    ctx->timed_every = every;
    ctx->timed_seen = 0;
    ctx->ev_used = 0;
    return MOS_OK;
}

mos_status mos_timing_stop(mos_ctx ctx, int64_t *launches, double *total_ms, int64_t *seen) {
    if (!ctx) {
        set_error("invalid context");
        return MOS_EINVAL;
    }
    MOS_HIP(hipStreamSynchronize(ctx->stream));
    double total = 0.0;
    for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
        float ms = 0.0f;
        MOS_HIP(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
        total += ms;
    }
    if (launches) *launches = (int64_t)(ctx->ev_used / 2);
    if (total_ms) *total_ms = total;
    if (seen) *seen = ctx->timed_seen;
    ctx->timed_kernel = 0;
    ctx->ev_used = 0;
    return MOS_OK;
}

mos_status mos_build_cell(mos_ctx ctx, const mos_cell_desc *desc, mos_cell *out) {
    if (!out) {
        set_error("out is NULL");
        return MOS_EINVAL;
    }
    *out = nullptr;
    if (!ctx) {
        set_error("ctx is NULL");
        return MOS_EINVAL;
    }
    MOS_TRY(check_cell_desc(desc));
    MOS_HIP(hipSetDevice(ctx->device));
    mos_cell c = new (std::nothrow) mos_cell_s();
    if (!c) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    c->ctx = ctx;
    c->mem.ctx = ctx;
    c->desc = *desc;
    c->mx = desc->mesh[0];
    c->my = desc->mesh[1];
    c->mz = desc->mesh[2];
    mos_status s = launch_cell_assembly(c);
    if (s == MOS_OK) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            set_error("cell assembly failed: %s", hipGetErrorString(e));
            s = MOS_EHIP;
        }
    }
    if (s != MOS_OK) {
        mos_cell_free(c);
        return s;
    }
    ctx_hold(ctx);
    c->held = true;
    *out = c;
    return MOS_OK;
}

mos_status mos_reduce(mos_ctx ctx, mos_cell cell, mos_rom *out) {
    if (!out) {
        set_error("out is NULL");
        return MOS_EINVAL;
    }
    *out = nullptr;
    if (!ctx || !cell || cell->kind != KIND_CELL || cell->ctx != ctx) {
        set_error("invalid context or cell handle");
        return MOS_EINVAL;
    }
    if (cell->n_free == 0) {
        set_error("cell has no interior DoFs");
        return MOS_EINVAL;
    }
    MOS_HIP(hipSetDevice(ctx->device));
    mos_rom r = new (std::nothrow) mos_rom_s();
    if (!r) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    r->ctx = ctx;
    r->mem.ctx = ctx;
    mos_status s = reduce_cell(cell, r);
    if (s == MOS_OK) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) {
            set_error("reduction failed: %s", hipGetErrorString(e));
            s = MOS_EHIP;
        }
    }
    if (s != MOS_OK) {
        mos_rom_free(r);
        return s;
    }
    ctx_hold(ctx);
    r->held = true;
    *out = r;
    return MOS_OK;
}

// ROMs used together share the cell mesh and the interpolation order (same
// reduced size and stress basis shape); with same_block they must also share
// pitch and height (one array is made of one block geometry).
static mos_status check_roms(const mos_rom *roms, int32_t n_roms, bool same_block = true) {
    if (!roms || n_roms < 1 || n_roms > MAX_TYPES) {
        set_error("need 1..%d ROMs", MAX_TYPES);
        return MOS_EINVAL;
    }
    for (int t = 0; t < n_roms; ++t)
        if (!roms[t] || roms[t]->kind != KIND_ROM) {
            set_error("roms[%d] is not a ROM handle", t);
            return MOS_EINVAL;
        }
    const mos_cell_desc &a = roms[0]->desc;
    for (int t = 1; t < n_roms; ++t) {
        const mos_cell_desc &b = roms[t]->desc;
        bool same = true;
        for (int k = 0; k < 3; ++k) same = same && a.mesh[k] == b.mesh[k] && a.interp[k] == b.interp[k];
        if (same_block)
            same = same && a.pitch_x == b.pitch_x && a.pitch_y == b.pitch_y && a.height == b.height &&
                   a.skew == b.skew;
        if (!same) {
            set_error("roms[%d] differs from roms[0] in %s", t,
                      same_block ? "pitch, height, skew, mesh or interp" : "mesh or interp");
            return MOS_EINVAL;
        }
    }
    return MOS_OK;
}

static mos_engine new_engine(mos_ctx ctx, const mos_rom *roms, int32_t n_roms, mos_precision precision) {
    mos_engine e = new (std::nothrow) mos_engine_s();
    if (!e) return nullptr;
    e->ctx = ctx;
    e->mem.ctx = ctx;
    e->precision = precision;
    e->roms.assign(roms, roms + n_roms);
    e->ldk = roms[0]->ldk;
    e->n = roms[0]->n;
    e->n_elem = roms[0]->n_elem;
    e->n_eblk = roms[0]->n_eblk;
    return e;
}

mos_status mos_solve_array(mos_ctx ctx, const mos_array_desc *d, const mos_rom *roms, int32_t n_roms,
                           mos_sol *out) {
    if (!out) {
        set_error("out is NULL");
        return MOS_EINVAL;
    }
    *out = nullptr;
    if (!ctx || !d) {
        set_error("ctx or descriptor is NULL");
        return MOS_EINVAL;
    }
    MOS_TRY(check_roms(roms, n_roms));
    for (int t = 0; t < n_roms; ++t)
        if (roms[t]->ctx != ctx) {
            set_error("roms[%d] belongs to another context", t);
            return MOS_EINVAL;
        }
    if (d->precision != MOS_FP64 && d->precision != MOS_MIXED) {
        set_error("invalid precision");
        return MOS_EINVAL;
    }
    MOS_HIP(hipSetDevice(ctx->device));
    // A one-problem engine sized exactly for this array.
    mos_engine e = new_engine(ctx, roms, n_roms, d->precision);
    if (!e) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    struct EngineGuard {
        mos_engine e;
        ~EngineGuard() {
            engine_free(e);
            delete e;
        }
    } eg{e};
    // Stacked arrays take the Jacobi preconditioner.
    if (d->nz_cells > 1) MOS_TRY(engine_set_precond(e, 0));
    int64_t dofs = 0, slots = 0;
    MOS_TRY(engine_problem_size(e, d, &dofs, &slots));
    MOS_TRY(engine_alloc(e, dofs, slots));
    mos_sol s = new (std::nothrow) mos_sol_s();
    if (!s) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    s->ctx = ctx;
    s->mem.ctx = ctx;
    struct SolGuard {
        mos_sol s;
        bool keep = false;
        ~SolGuard() {
            if (!keep) mos_sol_free(s);
        }
    } sg{s};
    const mos_cell_desc &cd = roms[0]->desc;
    const Lattice lat = make_lattice(d->nx_cells, d->ny_cells, cd.interp[0], cd.interp[1], cd.interp[2],
                                     d->nz_cells < 1 ? 1 : d->nz_cells);
    MOS_TRY(s->mem.alloc_n(3 * lat.n_nodes, &s->u));
    int64_t ticket = 0;
    MOS_TRY(engine_submit(e, d, nullptr, nullptr, s->u, &ticket));
    std::vector<int64_t> done;
    while (e->finished.find(ticket) == e->finished.end()) MOS_TRY(engine_progress(e, 16, &done));
    EngineProblem *P = e->finished[ticket];
    if (P->status != MOS_OK) {
        set_error("%s", P->error.c_str());
        return P->status;
    }
    // The solution handle keeps what mos_reconstruct needs.
    s->precision = d->precision;
    s->Nx = P->Nx;
    s->Ny = P->Ny;
    s->n_cells = (int)P->n_cells;
    s->n = roms[0]->n;
    s->n_surf = roms[0]->n_surf;
    s->n_elem = roms[0]->n_elem;
    s->ldk = roms[0]->ldk;
    s->n_eblk = roms[0]->n_eblk;
    s->n_nodes = P->n_nodes;
    s->n_dofs = P->n_dofs;
    s->delta_T = d->delta_T;
    s->rel_residual = P->rel;
    s->iters = P->iters;
    s->refines = P->sweeps;
    s->lz = std::move(P->lz);
    s->n_types = n_roms;
    s->roms.assign(roms, roms + n_roms);
    s->seg.resize(n_roms + 1);
    for (int t = 0; t <= n_roms; ++t) s->seg[t] = P->seg[t] * 16;
    s->n_pc = P->n_sb * 16;
    MOS_TRY(s->mem.alloc_n(s->n_pc, &s->perm));
    MOS_TRY(s->mem.alloc_n((size_t)s->ldk * s->n_pc, &s->gidx));
    hipStream_t st = ctx->stream;
    MOS_HIP(hipMemcpyAsync(s->perm, P->perm.data(), P->perm.size() * 4, hipMemcpyHostToDevice, st));
    MOS_TRY(engine_gather_index(e, P, s->perm, s->gidx));
    MOS_HIP(hipStreamSynchronize(st));
    sg.keep = true;
    ctx_hold(ctx);
    s->held = true;
    *out = s;
    return MOS_OK;
}

mos_status mos_engine_create(mos_ctx ctx, const mos_rom *roms, int32_t n_roms, mos_precision precision,
                             size_t device_bytes, mos_engine *out) {
    if (!out) {
        set_error("out is NULL");
        return MOS_EINVAL;
    }
    *out = nullptr;
    if (!ctx || (precision != MOS_FP64 && precision != MOS_MIXED)) {
        set_error("invalid context or precision");
        return MOS_EINVAL;
    }
    MOS_TRY(check_roms(roms, n_roms, false));
    MOS_HIP(hipSetDevice(ctx->device));
    mos_engine e = new_engine(ctx, roms, n_roms, precision);
    if (!e) {
        set_error("out of host memory");
        return MOS_ENOMEM;
    }
    // Split the budget between DoF arrays and cell slots (~100 DoFs per cell).
    const double w = precision == MOS_MIXED ? 4.0 : 8.0;
    // Per DoF: vectors, FP64 vectors, constraint mask, incidence, packed
    // coordinates, block tables (partials, owners, coarse inverses and
    // coefficients of up to 4 aggregates per 256 DoFs).
    const double per_dof = 5 * w + 4 * 8 + 1 + 16.0 / 3 + 4.0 / 3 + 4 * 8.0 / 256 + 4.0 / 256 +
                           (4 * 42 * 8.0 + 4) / 256;
    const double per_slot = e->ldk * (2 * w + 16) + 8 + 8.0 / 16 + e->ldk / 16 * 8.0 / 16 +
                            (precision == MOS_MIXED ? (double)recon_bf16_scratch(roms[0], 1) / 16 : 0.0);
    const double units = (double)device_bytes / (100 * per_dof + per_slot);
    // A budget beyond what one engine can address is used only up to the
    // slot limit of the incidence packing (about 45 GB of FP64 arenas).
    const double units_cap = std::min(units, (double)MAX_SLOTS);
    const int64_t dofs = (int64_t)(units_cap * 100), slots = (int64_t)units_cap;
    if (dofs < 768 || slots < 16) {
        delete e;
        set_error("device budget of %zu bytes is too small for an engine", device_bytes);
        return MOS_EINVAL;
    }
    mos_status s = engine_alloc(e, dofs, slots);
    if (s != MOS_OK) {
        engine_free(e);
        delete e;
        return s;
    }
    ctx_hold(ctx);
    e->held = true;
    *out = e;
    return MOS_OK;
}

mos_status mos_engine_submit(mos_engine e, const mos_array_desc *desc, void *vm, void *sigma6, double *u,
                             int64_t *ticket) {
    if (!e || !desc || !ticket) {
        set_error("engine, descriptor or ticket is NULL");
        return MOS_EINVAL;
    }
    *ticket = 0;
    return engine_submit(e, desc, vm, sigma6, u, ticket);
}

mos_status mos_engine_progress(mos_engine e, int32_t iterations, int64_t *completed, int32_t max_completed,
                               int32_t *n_completed) {
    if (!e || iterations < 1 || max_completed < 0 || (max_completed > 0 && !completed)) {
        set_error("invalid engine or arguments");
        return MOS_EINVAL;
    }
    MOS_HIP(hipSetDevice(e->ctx->device));
    std::vector<int64_t> done;
    mos_status s = engine_progress(e, iterations, &done);
    e->completed_unreported.insert(e->completed_unreported.end(), done.begin(), done.end());
    int32_t k = 0;
    while (k < max_completed && k < (int32_t)e->completed_unreported.size()) {
        completed[k] = e->completed_unreported[k];
        ++k;
    }
    e->completed_unreported.erase(e->completed_unreported.begin(), e->completed_unreported.begin() + k);
    if (n_completed) *n_completed = k;
    return s;
}

mos_status mos_engine_result(mos_engine e, int64_t ticket, int32_t *status, double *rel_residual, int32_t *iters,
                             int32_t *sweeps) {
    if (!e) {
        set_error("invalid engine");
        return MOS_EINVAL;
    }
    auto it = e->finished.find(ticket);
    if (it == e->finished.end()) {
        set_error("ticket %lld has not completed", (long long)ticket);
        return MOS_EBUSY;
    }
    EngineProblem *P = it->second;
    if (status) *status = P->status;
    if (rel_residual) *rel_residual = P->rel;
    if (iters) *iters = P->iters;
    if (sweeps) *sweeps = P->sweeps;
    if (P->status != MOS_OK) set_error("%s", P->error.c_str());
    delete P;
    e->finished.erase(it);
    return MOS_OK;
}

mos_status mos_engine_cond_estimate(mos_engine e, int64_t ticket, double *kappa, int32_t *steps) {
    if (!e) {
        set_error("invalid engine");
        return MOS_EINVAL;
    }
    auto it = e->finished.find(ticket);
    if (it == e->finished.end()) {
        set_error("ticket %lld has not completed (or its result was already taken)", (long long)ticket);
        return MOS_EBUSY;
    }
    const std::vector<double> &lz = it->second->lz;
    int k = 0;
    const double kap = lanczos_cond(lz.data(), (int)(lz.size() / 2), &k);
    if (kappa) *kappa = kap;
    if (steps) *steps = k;
    return MOS_OK;
}

mos_status mos_engine_option(mos_engine e, int option, int64_t value) {
    if (!e) {
        set_error("invalid engine");
        return MOS_EINVAL;
    }
    if (option == MOS_OPT_CELL_GEMM && value >= 0 && value <= 3) {
        if (!e->active.empty() || !e->queue.empty()) {
            set_error("engine options must be set before the first submission");
            return MOS_EBUSY;
        }
        e->gemm_rows = value != 1 && e->ldk / 4 <= mos::ROWS_MAX_KS;
        e->gemm_paths = value == 2 ? 1 : value == 3 ? 2 : 3;
        e->tuner.configure(e->gemm_paths, e->gemm_split);
        return MOS_OK;
    }
    if (option == MOS_OPT_PRECOND && (value == 0 || value == 1)) {
        if (!e->active.empty() || !e->queue.empty()) {
            set_error("engine options must be set before the first submission");
            return MOS_EBUSY;
        }
        return engine_set_precond(e, (int)value);
    }
    if (option == MOS_OPT_UPDATE_WIDTH && (value == 0 || value == 128 || value == 256)) {
        e->update_width = (int)value;
        return MOS_OK;
    }
    if (option == MOS_OPT_COARSE_TABLE && (value == 0 || value == 1)) {
        e->coarse_table = (int)value;
        return MOS_OK;
    }
    if (option == MOS_OPT_GRAPH && (value == 0 || value == 1)) {
        e->use_graph = (int)value;
        return MOS_OK;
    }
    if (option == MOS_OPT_GEMM_SPLIT && value >= 0 && value <= 64) {
        e->gemm_split = (int)value;
        e->tuner.configure(e->gemm_paths, e->gemm_split);
        return MOS_OK;
    }
    set_error("unknown option %d or value %lld", option, (long long)value);
    return MOS_EINVAL;
}

mos_status mos_engine_graph_stats(mos_engine e, int64_t *captures, int64_t *replays) {
    if (!e) {
        set_error("invalid engine");
        return MOS_EINVAL;
    }
    if (captures) *captures = e->graph_captures;
    if (replays) *replays = e->graph_replays;
    return MOS_OK;
}

mos_status mos_engine_stats(mos_engine e, int64_t *active, int64_t *queued, int64_t *capacity_dofs,
                            int64_t *capacity_slots) {
    if (!e) {
        set_error("invalid engine");
        return MOS_EINVAL;
    }
    if (active) *active = (int64_t)e->active.size();
    if (queued) *queued = (int64_t)e->queue.size();
    if (capacity_dofs) *capacity_dofs = (int64_t)e->cap_blk * 256;
    if (capacity_slots) *capacity_slots = (int64_t)e->cap_sb * 16;
    return MOS_OK;
}

void mos_engine_destroy(mos_engine e) {
    if (!e) return;
    mos_ctx ctx = e->ctx;
    const bool held = e->held;
    engine_free(e);
    delete e;
    if (held) ctx_drop(ctx);
}

mos_status mos_reconstruct(mos_ctx ctx, mos_sol sol, uint32_t outputs, void *vm, void *sigma6) {
    if (!ctx || !sol || sol->kind != KIND_SOL || sol->ctx != ctx) {
        set_error("invalid context or solution handle");
        return MOS_EINVAL;
    }
    if ((outputs & ~(uint32_t)(MOS_OUT_VM | MOS_OUT_SIGMA6)) || outputs == 0 ||
        ((outputs & MOS_OUT_VM) && !vm) || ((outputs & MOS_OUT_SIGMA6) && !sigma6)) {
        set_error("outputs must select VM and/or SIGMA6 with non-NULL buffers");
        return MOS_EINVAL;
    }
    MOS_HIP(hipSetDevice(ctx->device));
    return reconstruct(ctx, sol, outputs, vm, sigma6);
}

mos_status mos_reconstruct_noalloc(mos_ctx ctx, mos_sol sol, uint32_t outputs, void *vm, void *sigma6) {
    if (!ctx || !sol || sol->kind != KIND_SOL || sol->ctx != ctx) {
        set_error("invalid context or solution handle");
        return MOS_EINVAL;
    }
    if ((outputs & ~(uint32_t)(MOS_OUT_VM | MOS_OUT_SIGMA6)) || outputs == 0 ||
        ((outputs & MOS_OUT_VM) && !vm) || ((outputs & MOS_OUT_SIGMA6) && !sigma6)) {
        set_error("outputs must select VM and/or SIGMA6 with non-NULL buffers");
        return MOS_EINVAL;
    }
    for (mos_rom r : sol->roms)
        if (!r || r->kind != KIND_ROM) {
            set_error("mos_reconstruct_noalloc: a ROM of this solution has been freed");
            return MOS_EINVAL;
        }
    MOS_HIP(hipSetDevice(ctx->device));
    return reconstruct_noalloc(ctx, sol, outputs, vm, sigma6);
}

mos_status mos_reconstruct_displacement(mos_ctx ctx, mos_sol sol, void *u_nodal) {
    if (!ctx || !sol || sol->kind != KIND_SOL || sol->ctx != ctx) {
        set_error("invalid context or solution handle");
        return MOS_EINVAL;
    }
    if (!u_nodal) {
        set_error("mos_reconstruct_displacement: u_nodal is NULL");
        return MOS_EINVAL;
    }
    for (mos_rom r : sol->roms)
        if (!r || r->kind != KIND_ROM) {
            set_error("mos_reconstruct_displacement: a ROM of this solution has been freed");
            return MOS_EINVAL;
        }
    MOS_HIP(hipSetDevice(ctx->device));
    return reconstruct_displacement(ctx, sol, static_cast<double *>(u_nodal));
}

mos_status mos_reconstruct_plane(mos_ctx ctx, mos_sol sol, int32_t grid, void *vm) {
    if (!ctx || !sol || sol->kind != KIND_SOL || sol->ctx != ctx) {
        set_error("invalid context or solution handle");
        return MOS_EINVAL;
    }
    if (!vm || grid < 1 || grid > PLANE_MAX_GRID) {
        set_error("mos_reconstruct_plane: need a non-NULL vm and a grid in [1, %d]", PLANE_MAX_GRID);
        return MOS_EINVAL;
    }
    for (mos_rom r : sol->roms) {
        if (!r || r->kind != KIND_ROM) {
            set_error("mos_reconstruct_plane: a ROM of this solution has been freed");
            return MOS_EINVAL;
        }
        if (r->desc.skew != 0.0) {
            set_error("mos_reconstruct_plane: the evaluation plane is defined for rectangular blocks (skew 0)");
            return MOS_EINVAL;
        }
    }
    MOS_HIP(hipSetDevice(ctx->device));
    return reconstruct_plane(ctx, sol, grid, vm);
}

mos_status mos_get_solution(mos_sol sol, double *u_host, double *rel_residual, int32_t *iters) {
    if (!sol || sol->kind != KIND_SOL) {
        set_error("invalid solution handle");
        return MOS_EINVAL;
    }
    if (u_host) {
        MOS_HIP(hipSetDevice(sol->ctx->device));
        MOS_HIP(hipMemcpyAsync(u_host, sol->u, sol->n_dofs * sizeof(double), hipMemcpyDeviceToHost,
                               sol->ctx->stream));
        MOS_HIP(hipStreamSynchronize(sol->ctx->stream));
    }
    if (rel_residual) *rel_residual = sol->rel_residual;
    if (iters) *iters = sol->iters;
    return MOS_OK;
}

mos_status mos_get_cond_estimate(mos_sol sol, double *kappa, int32_t *steps) {
    if (!sol || sol->kind != KIND_SOL) {
        set_error("invalid solution handle");
        return MOS_EINVAL;
    }
    int k = 0;
    const double kap = lanczos_cond(sol->lz.data(), (int)(sol->lz.size() / 2), &k);
    if (kappa) *kappa = kap;
    if (steps) *steps = k;
    return MOS_OK;
}

mos_status mos_query(const void *handle, int what, int64_t *value) {
    if (!handle || !value) {
        set_error("handle or value is NULL");
        return MOS_EINVAL;
    }
    uint32_t kind = *static_cast<const uint32_t *>(handle);
    if (kind == KIND_CELL) {
        const mos_cell_s *c = static_cast<const mos_cell_s *>(handle);
        int nx = c->desc.interp[0], ny = c->desc.interp[1], nz = c->desc.interp[2];
        switch (what) {
            case MOS_Q_N: *value = 3LL * (nx * ny * nz - (nx - 2) * (ny - 2) * (nz - 2)); return MOS_OK;
            case MOS_Q_CELL_DOFS: *value = c->n_dofs; return MOS_OK;
            case MOS_Q_CELL_ELEMS: *value = c->n_elem; return MOS_OK;
            case MOS_Q_CELL_NNZ: *value = c->nnz; return MOS_OK;
            case MOS_Q_FREE_DOFS: *value = c->n_free; return MOS_OK;
            case MOS_Q_BANDWIDTH: *value = c->bw; return MOS_OK;
            case MOS_Q_DEVICE_BYTES: *value = (int64_t)c->mem.bytes; return MOS_OK;
        }
    } else if (kind == KIND_ROM) {
        const mos_rom_s *r = static_cast<const mos_rom_s *>(handle);
        switch (what) {
            case MOS_Q_N: *value = r->n; return MOS_OK;
            case MOS_Q_CELL_DOFS: *value = r->n_dofs; return MOS_OK;
            case MOS_Q_CELL_ELEMS: *value = r->n_elem; return MOS_OK;
            case MOS_Q_DEVICE_BYTES: *value = (int64_t)r->mem.bytes; return MOS_OK;
        }
    } else if (kind == KIND_SOL) {
        const mos_sol_s *s = static_cast<const mos_sol_s *>(handle);
        switch (what) {
            case MOS_Q_GLOBAL_DOFS: *value = s->n_dofs; return MOS_OK;
            case MOS_Q_ITERS: *value = s->iters; return MOS_OK;
            case MOS_Q_REFINES: *value = s->refines; return MOS_OK;
            case MOS_Q_DEVICE_BYTES: *value = (int64_t)s->mem.bytes; return MOS_OK;
        }
    } else {
        set_error("unknown handle");
        return MOS_EINVAL;
    }
    set_error("query %d not defined for this handle", what);
    return MOS_EINVAL;
}

mos_status mos_cell_export(mos_cell c, int64_t *row_ptr, int32_t *col, double *val, double *b,
                           uint8_t *material) {
    if (!c || c->kind != KIND_CELL) {
        set_error("invalid cell handle");
        return MOS_EINVAL;
    }
    hipStream_t st = c->ctx->stream;
    MOS_HIP(hipSetDevice(c->ctx->device));
    if (row_ptr) {
        std::vector<int32_t> rp(c->n_dofs + 1);
        MOS_HIP(hipMemcpyAsync(rp.data(), c->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, st));
        MOS_HIP(hipStreamSynchronize(st));
        for (size_t i = 0; i < rp.size(); ++i) row_ptr[i] = rp[i];
    }
    if (col) MOS_HIP(hipMemcpyAsync(col, c->col, c->nnz * 4, hipMemcpyDeviceToHost, st));
    if (val) MOS_HIP(hipMemcpyAsync(val, c->val, c->nnz * 8, hipMemcpyDeviceToHost, st));
    if (b) MOS_HIP(hipMemcpyAsync(b, c->b, c->n_dofs * 8, hipMemcpyDeviceToHost, st));
    if (material) MOS_HIP(hipMemcpyAsync(material, c->mat, c->n_elem, hipMemcpyDeviceToHost, st));
    MOS_HIP(hipStreamSynchronize(st));
    return MOS_OK;
}

mos_status mos_rom_export(mos_rom r, double *phi, double *f_T, double *K_r, double *b_r) {
    if (!r || r->kind != KIND_ROM) {
        set_error("invalid ROM handle");
        return MOS_EINVAL;
    }
    hipStream_t st = r->ctx->stream;
    MOS_HIP(hipSetDevice(r->ctx->device));
    if (phi || f_T) {
        std::vector<double> h((size_t)r->n_dofs * r->ldp);
        MOS_HIP(hipMemcpyAsync(h.data(), r->phi, h.size() * 8, hipMemcpyDeviceToHost, st));
        MOS_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < r->n_dofs; ++i) {
            if (phi) std::memcpy(phi + (size_t)i * r->n, h.data() + (size_t)i * r->ldp, r->n * 8);
            if (f_T) f_T[i] = h[(size_t)i * r->ldp + r->n];
        }
    }
    if (K_r) MOS_HIP(hipMemcpyAsync(K_r, r->kr, (size_t)r->n * r->n * 8, hipMemcpyDeviceToHost, st));
    if (b_r) MOS_HIP(hipMemcpyAsync(b_r, r->br, r->n * 8, hipMemcpyDeviceToHost, st));
    MOS_HIP(hipStreamSynchronize(st));
    return MOS_OK;
}

mos_status mos_array_layout(mos_ctx ctx, int32_t nx_cells, int32_t ny_cells, int32_t nz_cells, mos_rom rom,
                            int64_t *n_nodes, double *coords, int32_t *conn, int64_t *row_ptr, int32_t *col) {
    const int32_t nz = nz_cells < 1 ? 1 : nz_cells;
    if (!ctx || !rom || rom->kind != KIND_ROM || !n_nodes || nx_cells < 1 || ny_cells < 1 ||
        (int64_t)nx_cells * ny_cells * nz > (1 << 22)) {
        set_error("invalid arguments to mos_array_layout");
        return MOS_EINVAL;
    }
    const mos_cell_desc &d = rom->desc;
    ArrayMesh m;
    m.build(nx_cells, ny_cells, d.interp[0], d.interp[1], d.interp[2], nz);
    *n_nodes = m.n_nodes;
    if (coords) {
        for (int64_t K = 0; K < m.Z; ++K)
            for (int64_t J = 0; J < m.Y; ++J)
                for (int64_t I = 0; I < m.X; ++I) {
                    if (!(I % (m.nx - 1) == 0 || J % (m.ny - 1) == 0 || K % (m.nz - 1) == 0)) continue;
                    const int64_t id = node_id(m.lat, I, J, K);
                    const double x = d.pitch_x * I / (m.nx - 1), y = d.pitch_y * J / (m.ny - 1);
                    const double sy = d.skew * y;  // its own statement: no fused multiply-add
                    coords[3 * (size_t)id + 0] = x + sy;
                    coords[3 * (size_t)id + 1] = y;
                    coords[3 * (size_t)id + 2] = d.height * K / (m.nz - 1);
                }
    }
    if (conn) std::memcpy(conn, m.conn.data(), m.conn.size() * sizeof(int32_t));
    if (row_ptr) {
        // Node-level pattern: union of the node sets of the cells around each node.
        std::vector<std::vector<int32_t>> cells_of((size_t)m.n_nodes);
        const int64_t nc = (int64_t)nx_cells * ny_cells * nz;
        for (int64_t c = 0; c < nc; ++c)
            for (int s = 0; s < m.S; ++s) cells_of[m.conn[(size_t)c * m.S + s]].push_back((int32_t)c);
        row_ptr[0] = 0;
        std::vector<int32_t> nb;
        for (int64_t node = 0; node < m.n_nodes; ++node) {
            nb.clear();
            for (int32_t c : cells_of[node])
                nb.insert(nb.end(), m.conn.begin() + (size_t)c * m.S, m.conn.begin() + (size_t)(c + 1) * m.S);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            for (int ci = 0; ci < 3; ++ci) {
                int64_t r = 3 * node + ci;
                row_ptr[r + 1] = row_ptr[r] + 3 * (int64_t)nb.size();
                if (col) {
                    int64_t k = row_ptr[r];
                    for (int32_t v : nb)
                        for (int cj = 0; cj < 3; ++cj) col[k++] = 3 * v + cj;
                }
            }
        }
    }
    return MOS_OK;
}

void mos_cell_free(mos_cell c) {
    if (!c || c->kind != KIND_CELL) return;
    mos_ctx ctx = c->ctx;
    const bool held = c->held;
    c->mem.release();
    c->kind = 0;
    delete c;
    if (held) ctx_drop(ctx);
}

void mos_rom_free(mos_rom r) {
    if (!r || r->kind != KIND_ROM) return;
    if (r->plane) {
        r->plane->mem.release();
        delete r->plane;
        r->plane = nullptr;
    }
    mos_ctx ctx = r->ctx;
    const bool held = r->held;
    r->mem.release();
    r->kind = 0;
    delete r;
    if (held) ctx_drop(ctx);
}

void mos_sol_free(mos_sol s) {
    if (!s || s->kind != KIND_SOL) return;
    mos_ctx ctx = s->ctx;
    const bool held = s->held;
    s->mem.release();
    s->kind = 0;
    delete s;
    if (held) ctx_drop(ctx);
}

}  // extern "C"
