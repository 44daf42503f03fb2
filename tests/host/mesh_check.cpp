// Host harness for the library's closed-form numbering (Sec. 4.3, abstract
// mesh of the array) and the host-side argument checks of the C ABI.  It
// runs without a GPU; the Python test compares what it prints with the
// oracle's brute-force numbering.
//
//   mesh_check mesh Nx Ny Nz nx ny nz cx cy
//       prints "n_nodes S bad" and then, for every lattice point that is a
//       node in (K, J, I) order, "I J K node_id internal_id", followed by the
//       connectivity of ArrayMesh (Nx*Ny*Nz rows of S node ids; Nz stacked
//       layers of blocks).  `bad` counts
//       failed round trips of the internal order (agg_decode of agg_encode,
//       and sub_decode of sub_encode within each box).
//   mesh_check abi
//       calls every C entry point with NULL or invalid arguments that are
//       rejected before any device work and prints "abi ok" when each
//       returns the documented status; also checks the engine's slot limit.
//   mesh_check lanczos
//       reads k and then k pairs (alpha_j, beta_j) of recorded PCG steps from
//       stdin and prints the library's condition estimate from them as
//       "kappa steps" (host code of the engine, no device work).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mesh.h"
#include "mos.h"

using namespace mos;

namespace mos {
double lanczos_cond(const double *lz, int k, int *steps);  // the engine's host code (engine.hip)
}

static int run_lanczos() {
    int k = 0;
    if (std::scanf("%d", &k) != 1 || k < 0 || k > 100000) return 2;
    std::vector<double> lz(2 * (size_t)k + 2, 0.0);
    for (int i = 0; i < 2 * k; ++i)
        if (std::scanf("%lf", &lz[i]) != 1) return 2;
    int steps = -1;
    const double kappa = lanczos_cond(lz.data(), k, &steps);
    std::printf("%.17g %d\n", kappa, steps);
    return 0;
}

static int fail(const char *what) {
    std::printf("FAIL %s\n", what);
    return 1;
}

static int run_mesh(int Nx, int Ny, int Nz, int nx, int ny, int nz, int cx, int cy) {
    const Lattice L = make_lattice(Nx, Ny, nx, ny, nz, Nz);
    const AggLayout A = make_agg_layout(L, cx, cy);
    ArrayMesh M;
    M.build(Nx, Ny, nx, ny, nz, Nz);
    int64_t bad = 0;
    // Every box's nodes in (K, j, i) order decode back to themselves.
    for (int gy = 0; gy < A.nay; ++gy)
        for (int gx = 0; gx < A.nax; ++gx) {
            const SubLattice B = agg_box(A, gx, gy);
            const int64_t cnt = sub_count(B);
            for (int64_t id = 0; id < cnt; ++id) {
                int i, j, K;
                sub_decode(B, id, i, j, K);
                if (i < 0 || i >= B.wx || j < 0 || j >= B.wy || K < 0 || K >= B.Z || sub_encode(B, i, j, K) != id)
                    ++bad;
            }
        }
    std::vector<char> line;
    std::printf("%lld %d %lld\n", (long long)L.n_nodes, M.S, (long long)bad);
    int64_t count = 0;
    for (int K = 0; K < (int)L.Z; ++K)
        for (int64_t J = 0; J < L.Y; ++J)
            for (int64_t I = 0; I < L.X; ++I) {
                const bool node = I % (nx - 1) == 0 || J % (ny - 1) == 0 || K % (nz - 1) == 0;
                if (!node) continue;
                ++count;
                const int64_t id = node_id(L, I, J, K);
                const int64_t in = agg_encode(A, I, J, K);
                int64_t I2, J2;
                int K2;
                agg_decode(A, in, I2, J2, K2);
                if (I2 != I || J2 != J || K2 != K) ++bad;
                std::printf("%lld %lld %d %lld %lld\n", (long long)I, (long long)J, K, (long long)id, (long long)in);
            }
    if (count != L.n_nodes) ++bad;
    for (int c = 0; c < Nx * Ny * Nz; ++c) {
        for (int s = 0; s < M.S; ++s) std::printf(s ? " %d" : "%d", M.conn[(size_t)c * M.S + s]);
        std::printf("\n");
    }
    std::printf("bad %lld\n", (long long)bad);
    return 0;
}

static int run_abi() {
    // Handles and outputs: NULL is rejected with MOS_EINVAL and an error text.
    if (mos_ctx_create(0, nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("ctx_create out NULL");
    if (std::strlen(mos_last_error()) == 0) return fail("error text");
    mos_cell cell = (mos_cell)0x1;
    if (mos_build_cell(nullptr, nullptr, &cell) != MOS_EINVAL || cell != nullptr) return fail("build_cell");
    mos_rom rom = (mos_rom)0x1;
    if (mos_reduce(nullptr, nullptr, &rom) != MOS_EINVAL || rom != nullptr) return fail("reduce");
    mos_sol sol = (mos_sol)0x1;
    if (mos_solve_array(nullptr, nullptr, nullptr, 0, &sol) != MOS_EINVAL || sol != nullptr) return fail("solve");
    mos_engine eng = (mos_engine)0x1;
    if (mos_engine_create(nullptr, nullptr, 0, MOS_FP64, 1 << 20, &eng) != MOS_EINVAL || eng != nullptr)
        return fail("engine_create");
    int64_t tk = 7;
    if (mos_engine_submit(nullptr, nullptr, nullptr, nullptr, nullptr, &tk) != MOS_EINVAL) return fail("submit");
    if (mos_engine_progress(nullptr, 16, nullptr, 0, nullptr) != MOS_EINVAL) return fail("progress");
    if (mos_engine_result(nullptr, 1, nullptr, nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("result");
    if (mos_engine_option(nullptr, MOS_OPT_GRAPH, 0) != MOS_EINVAL) return fail("option");
    if (mos_engine_stats(nullptr, nullptr, nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("stats");
    if (mos_reconstruct(nullptr, nullptr, MOS_OUT_VM, nullptr, nullptr) != MOS_EINVAL) return fail("reconstruct");
    if (mos_reconstruct_displacement(nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("displacement");
    if (mos_reconstruct_plane(nullptr, nullptr, 100, nullptr) != MOS_EINVAL) return fail("plane");
    if (mos_get_solution(nullptr, nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("get_solution");
    int64_t v = 0;
    if (mos_query(nullptr, MOS_Q_N, &v) != MOS_EINVAL) return fail("query");
    if (mos_cell_export(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("cell_export");
    if (mos_rom_export(nullptr, nullptr, nullptr, nullptr, nullptr) != MOS_EINVAL) return fail("rom_export");
    int64_t nn = 0;
    if (mos_array_layout(nullptr, 2, 2, 1, nullptr, &nn, nullptr, nullptr, nullptr, nullptr) != MOS_EINVAL)
        return fail("array_layout");
    if (mos_timing_start(nullptr, 1, 1) != MOS_EINVAL) return fail("timing_start");
    // Freeing NULL handles is a no-op.
    mos_cell_free(nullptr);
    mos_rom_free(nullptr);
    mos_sol_free(nullptr);
    mos_engine_destroy(nullptr);
    mos_ctx_destroy(nullptr);
    // The engine's slot limit: slot << INC_SHIFT | s must fit an int32.
    if (!slots_fit(MAX_SLOTS) || slots_fit(MAX_SLOTS + 1) || slots_fit(-1)) return fail("slot limit");
    if (((MAX_SLOTS - 1) << INC_SHIFT | MAX_SURF) != 0x7fffffffLL) return fail("slot packing");
    std::printf("abi ok\n");
    return 0;
}

int main(int argc, char **argv) {
    if (argc == 10 && std::strcmp(argv[1], "mesh") == 0) {
        int a[8];
        for (int i = 0; i < 8; ++i) a[i] = std::atoi(argv[2 + i]);
        return run_mesh(a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7]);
    }
    if (argc == 2 && std::strcmp(argv[1], "abi") == 0) return run_abi();
    if (argc == 2 && std::strcmp(argv[1], "lanczos") == 0) return run_lanczos();
    std::fprintf(stderr, "usage: mesh_check mesh Nx Ny Nz nx ny nz cx cy | mesh_check abi | mesh_check lanczos\n");
    return 2;
}
