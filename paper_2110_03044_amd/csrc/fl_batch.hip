// Batched problems: many independent meshes, scalar counts, limiters and time steps advanced
// by ONE kernel launch per Runge-Kutta stage, replayed from a HIP graph.  Problems on the face
// path (general cells, boundary faces, face distances) join the same graph with two more
// launches per stage for all of them: one over their faces, one over their cells.
//
// Each problem is described once in device memory (mesh slot tables, face velocity, buffers,
// limiter, dt).  The work table lists (problem, first cell) tiles of `tile` cells; a persistent
// grid of workgroups strides over the table, each workgroup processing one tile at a time with
// one thread per cell.  Tiles never span problems, so the problem descriptor, the limiter and
// the (pairs, scalars) specialisation chosen per tile are uniform within a workgroup: one kernel
// serves every problem.  Each cell runs the single-problem kernel's own routine (fl_device.h),
// so each problem's result equals its single-problem run bit for bit; so does each face-path
// problem's (the face and cell routines of fl_face_device.h).
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fl_device.h"
#include "fl_face_device.h"

struct BatchProblem {
    int64_t nc;
    int32_t P, S, lim, pad;
    double dt, area0, vol0;
    const uint32_t *sface;
    const int32_t *snbr, *sfar;
    const double *u, *area, *vol;
    double *th, *t1, *t2;
    const int32_t *halo_ptr, *halo;  // tile tables (LDS staging)
    const uint32_t *slot_local;
    // face path (face != 0): face records, side lists where general, cell face lists, inflow
    // values (nullable) and the flux buffer
    int32_t face, general, K, pad2;
    int64_t nf;
    const int4 *fc4;
    const int32_t *side_ptr, *side_cell, *cf_ptr, *cf_idx;
    const double *side_w, *inflow;
    double *phi;
};

struct BatchTile {
    int32_t prob, pad;
    int64_t c0;
};

namespace fl {
namespace bdev {

constexpr int kBlock = 256;

// One cell of one problem: the single-problem routine, specialised for the problem's pair and
// scalar counts (a uniform branch: a tile never spans problems).
__device__ __forceinline__ void batch_cell(const BatchProblem &pb, int64_t c, const double *ts,
                                           double a, double b, int mode, double *out) {
#define FL_BCELL(SS, PP)                                                                       \
    dev::fused_cell<SS, PP>(c, pb.nc, pb.sface, pb.snbr, pb.sfar, pb.u, pb.area, pb.area0,     \
                            pb.vol, pb.vol0, ts, pb.th, a, b, pb.dt, mode, pb.lim, out, 1.0)
#define FL_BCELL_S(PP)                      \
    switch (pb.S) {                         \
        case 1: FL_BCELL(1, PP); break;     \
        case 2: FL_BCELL(2, PP); break;     \
        case 3: FL_BCELL(3, PP); break;     \
        case 4: FL_BCELL(4, PP); break;     \
        case 5: FL_BCELL(5, PP); break;     \
        case 6: FL_BCELL(6, PP); break;     \
        case 7: FL_BCELL(7, PP); break;     \
        default: FL_BCELL(8, PP); break;    \
    }
    switch (pb.P) {
        case 1: FL_BCELL_S(1); break;
        case 2: FL_BCELL_S(2); break;
        default: FL_BCELL_S(3); break;
    }
#undef FL_BCELL_S
#undef FL_BCELL
}

// stage 0: theta -> t1 (Euler form); stage 1: (t1, theta) -> t2; stage 2: (t2, theta) -> theta.
// Forward Euler uses stage 0 only, followed by batch_copy_kernel (t1 -> theta).
__global__ __launch_bounds__(kBlock) void batch_stage_kernel(const BatchProblem *__restrict__ probs,
                                                             const BatchTile *__restrict__ tiles,
                                                             int64_t ntiles, int tile, int stage) {
    const double A[3] = {0.0, 0.75, 1.0 / 3.0};
    const double B[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile T = tiles[t];
        const BatchProblem &pb = probs[T.prob];
        const double *ts = stage == 0 ? pb.th : stage == 1 ? pb.t1 : pb.t2;
        double *out = stage == 0 ? pb.t1 : stage == 1 ? pb.t2 : pb.th;
        const int mode = stage == 0 ? MODE_EULER : MODE_RK;
        const int64_t c1 = min(T.c0 + (int64_t)tile, pb.nc);
        for (int64_t c = T.c0 + threadIdx.x; c < c1; c += blockDim.x)
            batch_cell(pb, c, ts, A[stage], B[stage], mode, out);
    }
}

// One tile of one problem, staged in LDS (tile index = first cell / kTileCells): the
// single-problem tile routine with the face terms read through the face index.
template <int S, int P>
__device__ __forceinline__ void batch_tile(const BatchProblem &pb, int64_t tile, double *lds,
                                           const double *ts, double a, double b, int mode,
                                           double *out) {
    // theta_n is not loaded ahead: the 4 VGPRs it needs would cost this kernel a wave per SIMD
    dev::fused_tile<S, P, false, false>(pb.nc, tile, lds, pb.halo_ptr, pb.halo, pb.slot_local,
                                        nullptr, pb.sface, pb.u, pb.area, pb.area0, pb.vol,
                                        pb.vol0, ts, pb.th, a, b, pb.dt, mode, pb.lim, out, 1.0);
}

// As batch_stage_kernel, with every tile's theta and halo staged in LDS (tiles of kTileCells
// cells, one thread per cell).  The barrier at the top of each tile keeps the previous tile's
// LDS reads ahead of the next staging; every thread of a workgroup walks the same tiles and takes
// the same (P, S) branch, so all reach every barrier.
// remap > 0 (the grid a multiple of 8 remap): the workgroups of one XCD take runs of remap
// consecutive tiles in every round (dev::block_id is a bijection of the workgroup index).
__global__ __launch_bounds__(kBlock) void batch_stage_lds_kernel(
    const BatchProblem *__restrict__ probs, const BatchTile *__restrict__ tiles, int64_t ntiles,
    int stage, int remap) {
    extern __shared__ double lds[];
    const double A[3] = {0.0, 0.75, 1.0 / 3.0};
    const double B[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int64_t t = dev::block_id(remap); t < ntiles; t += gridDim.x) {
        __syncthreads();
        const BatchTile T = tiles[t];
        const BatchProblem &pb = probs[T.prob];
        const double *ts = stage == 0 ? pb.th : stage == 1 ? pb.t1 : pb.t2;
        double *out = stage == 0 ? pb.t1 : stage == 1 ? pb.t2 : pb.th;
        const int mode = stage == 0 ? MODE_EULER : MODE_RK;
        const int64_t tile = T.c0 / kTileCells;
#define FL_BTILE(SS, PP) batch_tile<SS, PP>(pb, tile, lds, ts, A[stage], B[stage], mode, out)
#define FL_BTILE_S(PP)                     \
    switch (pb.S) {                        \
        case 1: FL_BTILE(1, PP); break;    \
        case 2: FL_BTILE(2, PP); break;    \
        case 3: FL_BTILE(3, PP); break;    \
        case 4: FL_BTILE(4, PP); break;    \
        case 5: FL_BTILE(5, PP); break;    \
        case 6: FL_BTILE(6, PP); break;    \
        case 7: FL_BTILE(7, PP); break;    \
        default: FL_BTILE(8, PP); break;   \
    }
        switch (pb.P) {
            case 1: FL_BTILE_S(1); break;
            case 2: FL_BTILE_S(2); break;
            default: FL_BTILE_S(3); break;
        }
#undef FL_BTILE_S
#undef FL_BTILE
    }
}

// Face-path problems, stage s (SSP-RK3: th -> t1, (t1, th) -> t2, (t2, th) -> th; forward
// Euler: th -> th in place, since a cell's update reads only its own theta and the fluxes were
// formed by the launch before): one launch over every such problem's faces, tiles of kBlock
// faces, then one over their cells.
__global__ __launch_bounds__(kBlock) void batch_face_kernel(const BatchProblem *__restrict__ probs,
                                                            const BatchTile *__restrict__ tiles,
                                                            int64_t ntiles, int stage) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile T = tiles[t];
        const BatchProblem &pb = probs[T.prob];
        const double *ts = stage == 0 ? pb.th : stage == 1 ? pb.t1 : pb.t2;
        const int64_t f = T.c0 + threadIdx.x;
        if (f >= pb.nf) continue;
#define FL_BFACE(SS)                                                                            \
    if (pb.general)                                                                             \
        dev::face_flux_general_one<SS>(f, pb.fc4, pb.side_ptr, pb.side_cell, pb.side_w, pb.u,   \
                                       ts, pb.area, pb.area0, pb.lim, pb.phi, 1.0, pb.inflow);  \
    else                                                                                        \
        dev::face_flux_one<SS>(f, pb.fc4, pb.u, ts, pb.area, pb.area0, pb.lim, pb.phi, 1.0)
        switch (pb.S) {
            case 1: FL_BFACE(1); break;
            case 2: FL_BFACE(2); break;
            case 3: FL_BFACE(3); break;
            case 4: FL_BFACE(4); break;
            case 5: FL_BFACE(5); break;
            case 6: FL_BFACE(6); break;
            case 7: FL_BFACE(7); break;
            default: FL_BFACE(8); break;
        }
#undef FL_BFACE
    }
}

__global__ __launch_bounds__(kBlock) void batch_face_cell_kernel(
    const BatchProblem *__restrict__ probs, const BatchTile *__restrict__ tiles, int64_t ntiles,
    int stage, int euler) {
    const double A[3] = {0.0, 0.75, 1.0 / 3.0};
    const double B[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile T = tiles[t];
        const BatchProblem &pb = probs[T.prob];
        const double *ts = stage == 0 ? pb.th : stage == 1 ? pb.t1 : pb.t2;
        double *out = stage == 0 ? (euler ? pb.th : pb.t1) : stage == 1 ? pb.t2 : pb.th;
        const int mode = stage == 0 ? MODE_EULER : MODE_RK;
        const int64_t c = T.c0 + threadIdx.x;
        if (c >= pb.nc) continue;
#define FL_BCU(SS)                                                                             \
    dev::cell_update_one<SS>(c, pb.K, pb.cf_ptr, pb.cf_idx, pb.phi, pb.vol, pb.vol0, ts, pb.th, \
                             A[stage], B[stage], pb.dt, mode, out)
        switch (pb.S) {
            case 1: FL_BCU(1); break;
            case 2: FL_BCU(2); break;
            case 3: FL_BCU(3); break;
            case 4: FL_BCU(4); break;
            case 5: FL_BCU(5); break;
            case 6: FL_BCU(6); break;
            case 7: FL_BCU(7); break;
            default: FL_BCU(8); break;
        }
#undef FL_BCU
    }
}

__global__ __launch_bounds__(kBlock) void batch_copy_kernel(const BatchProblem *__restrict__ probs,
                                                            const BatchTile *__restrict__ tiles,
                                                            int64_t ntiles, int tile) {
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile T = tiles[t];
        const BatchProblem &pb = probs[T.prob];
        const int64_t e0 = T.c0 * pb.S, e1 = min(T.c0 + (int64_t)tile, pb.nc) * pb.S;
        for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) pb.th[i] = pb.t1[i];
    }
}

}  // namespace bdev
}  // namespace fl

using namespace fl;

struct fl_batch {
    int device = -1;
    int scheme = FL_SSPRK3;
    int tile = 0;            // cells per tile (0 until tuned)
    bool lds = false;        // tiles staged in LDS (tile == kTileCells)
    size_t lds_bytes = 0;    // dynamic LDS of the staged kernel, 0 if not every mesh allows it
    int grid = 0;            // persistent grid size
    int remap = 0;           // XCD run length of the LDS-staged kernel's tile order (0: none)
    std::vector<BatchProblem> probs;
    std::vector<const fl_mesh *> meshes;
    BatchProblem *d_probs = nullptr;
    BatchTile *d_tiles = nullptr;
    int64_t ntiles = 0;
    // face-path problems: tiles of kBlock faces and of kBlock cells
    BatchTile *d_ftiles = nullptr, *d_ctiles = nullptr;
    int64_t nftiles = 0, nctiles = 0;
    int fgrid = 1, cgrid = 1;
    bool any_fused = false;
    std::vector<double *> owned;  // t1/t2 buffers
    hipStream_t cap = nullptr;    // capture stream (default priority)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool tuned_from_cache = false;  // the tile choice came from the on-disk cache
};

namespace {

fl_status hip_err(hipError_t e, const char *what) {
    return fail(FL_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Guard {
    int prev = -1;
    bool changed = false;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~Guard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

void drop_graph(fl_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Builds the tile table for a tile size and uploads it.
fl_status set_tile(fl_batch *b, int tile) {
    std::vector<BatchTile> tiles;
    for (size_t i = 0; i < b->probs.size(); ++i)
        if (!b->probs[i].face)
            for (int64_t c0 = 0; c0 < b->probs[i].nc; c0 += tile)
                tiles.push_back({(int32_t)i, 0, c0});
    tiles.push_back({0, 0, 0});  // (never read past ntiles; keeps the allocation non-empty)
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = nullptr;
    hipError_t e = hipMalloc((void **)&b->d_tiles, tiles.size() * sizeof(BatchTile));
    if (e != hipSuccess) return fail(FL_E_NOMEM, "batch tile table");
    e = hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_err(e, "batch tile table upload");
    b->ntiles = (int64_t)tiles.size() - 1;
    b->tile = tile;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    // persistent grid: a few workgroups per CU, never more than there are tiles
    b->grid = (int)std::min<int64_t>(b->ntiles, (int64_t)cus * 8);
    if (b->grid < 1) b->grid = 1;
    // XCD-aware tile order of the LDS-staged kernel, where the grid allows it
    const int m = xcd_remap();
    b->remap = (m >= 2 && b->grid % (8 * m) == 0) ? m : 0;
    drop_graph(b);
    return FL_OK;
}

// The face-path problems' work tables: tiles of kBlock faces and of kBlock cells.
fl_status face_tiles(fl_batch *b) {
    std::vector<BatchTile> ft, ct;
    for (size_t i = 0; i < b->probs.size(); ++i) {
        const BatchProblem &p = b->probs[i];
        if (!p.face) continue;
        for (int64_t f0 = 0; f0 < p.nf; f0 += bdev::kBlock) ft.push_back({(int32_t)i, 0, f0});
        for (int64_t c0 = 0; c0 < p.nc; c0 += bdev::kBlock) ct.push_back({(int32_t)i, 0, c0});
    }
    b->nftiles = (int64_t)ft.size();
    b->nctiles = (int64_t)ct.size();
    if (ft.empty()) return FL_OK;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    b->fgrid = (int)std::max<int64_t>(1, std::min<int64_t>(b->nftiles, (int64_t)cus * 8));
    b->cgrid = (int)std::max<int64_t>(1, std::min<int64_t>(b->nctiles, (int64_t)cus * 8));
    for (auto pr : {std::make_pair(&b->d_ftiles, &ft), std::make_pair(&b->d_ctiles, &ct)}) {
        const size_t n = pr.second->size() * sizeof(BatchTile);
        hipError_t e = hipMalloc((void **)pr.first, n);
        if (e != hipSuccess) return fail(FL_E_NOMEM, "batch face tile tables");
        e = hipMemcpy(*pr.first, pr.second->data(), n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_err(e, "batch face tile table upload");
    }
    return FL_OK;
}

hipError_t launch_stage(const fl_batch *b, int s, hipStream_t st) {
    if (b->ntiles == 0) return hipSuccess;
    if (b->lds)
        bdev::batch_stage_lds_kernel<<<b->grid, bdev::kBlock, b->lds_bytes, st>>>(
            b->d_probs, b->d_tiles, b->ntiles, s, b->remap);
    else
        bdev::batch_stage_kernel<<<b->grid, bdev::kBlock, 0, st>>>(b->d_probs, b->d_tiles,
                                                                  b->ntiles, b->tile, s);
    return hipGetLastError();
}

hipError_t enqueue_step(const fl_batch *b, hipStream_t st) {
    const int ns = b->scheme == FL_EULER ? 1 : 3;
    for (int s = 0; s < ns; ++s) {
        hipError_t e = launch_stage(b, s, st);
        if (e != hipSuccess) return e;
        if (b->nftiles > 0) {
            bdev::batch_face_kernel<<<b->fgrid, bdev::kBlock, 0, st>>>(b->d_probs, b->d_ftiles,
                                                                      b->nftiles, s);
            bdev::batch_face_cell_kernel<<<b->cgrid, bdev::kBlock, 0, st>>>(
                b->d_probs, b->d_ctiles, b->nctiles, s, b->scheme == FL_EULER ? 1 : 0);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    if (b->scheme == FL_EULER && b->ntiles > 0) {
        bdev::batch_copy_kernel<<<b->grid, bdev::kBlock, 0, st>>>(b->d_probs, b->d_tiles,
                                                                 b->ntiles, b->tile);
        return hipGetLastError();
    }
    return hipSuccess;
}

// Times the non-destructive first stage (theta -> t1) for each candidate: the LDS-staged kernel
// (tiles of kTileCells, where every mesh allows it), then the gather kernel at each tile size.
// Each candidate: 2 untimed launches, then the best of 3 timed runs of 3 launches each.
fl_status autotune(fl_batch *b, hipStream_t st) {
    static const int cand[] = {-1, 128, 256, 512, 1024, 2048, 4096};  // -1: LDS-staged
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FL_E_HIP, "hipEventCreate");
    float best = 1e30f;
    int best_tile = 256;
    for (int c : cand) {
        if (c < 0 && b->lds_bytes == 0) continue;
        fl_status s = set_tile(b, c < 0 ? kTileCells : c);
        if (s != FL_OK) return s;
        b->lds = c < 0;
        for (int rep = 0; rep < 2; ++rep) (void)launch_stage(b, 0, st);
        float cand_ms = 1e30f;
        for (int trial = 0; trial < 3; ++trial) {
            (void)hipEventRecord(e0, st);
            for (int rep = 0; rep < 3; ++rep) (void)launch_stage(b, 0, st);
            (void)hipEventRecord(e1, st);
            hipError_t e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipGetLastError();
            if (e != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return hip_err(e, "autotune");
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            cand_ms = std::min(cand_ms, ms);
        }
        if (cand_ms < best) {
            best = cand_ms;
            best_tile = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    fl_status s = set_tile(b, best_tile < 0 ? kTileCells : best_tile);
    b->lds = best_tile < 0;
    return s;
}

// On-disk cache of the autotuner's choice, so that a batch of the same shape on the same kind of
// GPU is not timed again: FL_TUNE_CACHE names the file ("" or "0": no cache); unset, the file is
// $XDG_CACHE_HOME/fluxlim/batch_tune.txt or $HOME/.cache/fluxlim/batch_tune.txt.  One line per
// shape: a 64-bit key (FNV-1a over the GPU's architecture name and CU count, the scheme, the
// XCD tile order, the LDS bytes and every problem's cell count, pairs, scalars and limiter), the
// tile size, and 1 if the tiles are staged in LDS.  A missing or unreadable file just means
// tuning; the choice never changes results (every tile size gives the same bits).
std::string tune_cache_path() {
    const char *env = std::getenv("FL_TUNE_CACHE");
    if (env) return (env[0] == 0 || std::strcmp(env, "0") == 0) ? std::string() : std::string(env);
    const char *xdg = std::getenv("XDG_CACHE_HOME");
    if (xdg && xdg[0]) return std::string(xdg) + "/fluxlim/batch_tune.txt";
    const char *home = std::getenv("HOME");
    if (home && home[0]) return std::string(home) + "/.cache/fluxlim/batch_tune.txt";
    return std::string();
}

struct Fnv {
    uint64_t h = 1469598103934665603ULL;
    void bytes(const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ULL;
    }
    template <class T>
    void add(T v) { bytes(&v, sizeof v); }
};

uint64_t tune_key(const fl_batch *b) {
    Fnv k;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) {
        k.bytes(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
        k.add<int32_t>(prop.multiProcessorCount);
    }
    k.add<int32_t>(b->scheme);
    k.add<int32_t>(xcd_remap());
    k.add<uint64_t>(b->lds_bytes);
    k.add<uint64_t>(b->probs.size());
    for (const BatchProblem &p : b->probs) {
        k.add<int64_t>(p.nc);
        k.add<int32_t>(p.P);
        k.add<int32_t>(p.S);
        k.add<int32_t>(p.lim);
    }
    return k.h;
}

bool tune_cache_read(const std::string &path, uint64_t key, int *tile, int *lds) {
    if (path.empty()) return false;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    unsigned long long k;
    int t, l;
    bool hit = false;
    // the last line for a key wins
    while (std::fscanf(f, "%llx %d %d", &k, &t, &l) == 3)
        if (k == key && t > 0 && t % 64 == 0 && (l == 0 || (l == 1 && t == kTileCells))) {
            *tile = t;
            *lds = l;
            hit = true;
        }
    std::fclose(f);
    return hit;
}

void tune_cache_write(const std::string &path, uint64_t key, int tile, int lds) {
    if (path.empty()) return;
    // create the parent directories (errors surface as fopen failing)
    for (size_t i = 1; i < path.size(); ++i)
        if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%016llx %d %d\n", (unsigned long long)key, tile, lds);
    std::fclose(f);
}

// Records one step on the private stream into a graph that fl_batch_step replays.
fl_status capture(fl_batch *b) {
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_err(e, "hipStreamBeginCapture");
    hipError_t le = enqueue_step(b, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess || e != hipSuccess) {
        drop_graph(b);
        return hip_err(le != hipSuccess ? le : e, "batch capture");
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return hip_err(e, "hipGraphInstantiate");
    }
    return FL_OK;
}

void destroy(fl_batch *b) {
    Guard g(b->device);
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (double *p : b->owned) (void)hipFree(p);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_ftiles) (void)hipFree(b->d_ftiles);
    if (b->d_ctiles) (void)hipFree(b->d_ctiles);
    delete b;
}

}  // namespace

extern "C" {

fl_status fl_batch_create(int n, fl_mesh *const *meshes, const int *limiter, const int *n_scalars,
                          const double *dt, int scheme, double *const *theta,
                          const double *const *u_f, int tile_cells, int device, fl_batch **out) {
    if (!out) return fail(FL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || !meshes || !limiter || !n_scalars || !dt || !theta || !u_f)
        return fail(FL_E_INVALID, "n must be positive and every array non-NULL");
    if (scheme != FL_EULER && scheme != FL_SSPRK3) return fail(FL_E_INVALID, "unknown scheme");
    if (tile_cells < 0 || (tile_cells > 0 && tile_cells % 64 != 0))
        return fail(FL_E_INVALID, "tile_cells must be 0 (autotune) or a positive multiple of 64");
    // host-only meshes have no device tables: reject them before anything is allocated
    if (device < 0) return fail(FL_E_NODEVICE, "a batch needs a device (device >= 0)");
    for (int i = 0; i < n; ++i)
        if (meshes[i] && meshes[i]->device < 0)
            return fail(FL_E_NODEVICE, "a batched problem's mesh is host-only (device = -1)");
    fl_batch *b = nullptr;
    try {
        b = new fl_batch();
    } catch (const std::bad_alloc &) {
        return fail(FL_E_NOMEM, "host allocation failed");
    }
    b->device = device;
    b->scheme = scheme;
    bool lds_all = true;
    size_t lds_max = 0;
    Guard g(device);
    for (int i = 0; i < n; ++i) {
        const fl_mesh *m = meshes[i];
        if (!m || m->device != device) {
            destroy(b);
            return fail(FL_E_INVALID, "every mesh must live on the batch's device");
        }
        const bool face = m->path != FL_PATH_FUSED || m->h.pairs < 1;
        if (face && m->inflow && m->inflow_S != n_scalars[i]) {
            destroy(b);
            return fail(FL_E_INVALID, "a problem's inflow values were set for another number of "
                                      "scalars");
        }
        if (limiter[i] < 0 || limiter[i] >= FL_NUM_LIMITERS || n_scalars[i] < 1 ||
            n_scalars[i] > FL_MAX_SCALARS || !theta[i] || !u_f[i] || !(dt[i] == dt[i])) {
            destroy(b);
            return fail(FL_E_INVALID, "bad limiter, scalar count, dt or pointer for a problem");
        }
        BatchProblem p{};
        p.nc = m->h.nc;
        p.P = face ? 0 : m->h.pairs;
        p.S = n_scalars[i];
        p.lim = limiter[i];
        p.dt = dt[i];
        p.area0 = m->h.area0;
        p.vol0 = m->h.vol0;
        p.sface = m->d_slot_face;
        p.snbr = m->d_slot_nbr;
        p.sfar = m->d_slot_far;
        p.u = u_f[i];
        p.area = m->d_area;
        p.vol = m->d_vol;
        p.th = theta[i];
        p.halo_ptr = m->d_halo_ptr;
        p.halo = m->d_halo;
        p.slot_local = m->d_slot_local;
        if (face) {
            p.face = 1;
            p.general = m->h.general ? 1 : 0;
            p.K = (int32_t)m->h.max_degree;
            p.nf = m->h.nf;
            p.fc4 = reinterpret_cast<const int4 *>(m->d_fc4);
            p.side_ptr = m->d_side_ptr;
            p.side_cell = m->d_side_cell;
            p.side_w = m->d_side_w;
            p.cf_ptr = m->d_cf_ptr;
            p.cf_idx = m->d_cf_idx;
            p.inflow = m->inflow;
            const size_t fbytes = std::max<size_t>((size_t)p.nf * p.S * sizeof(double), 8);
            if (hipMalloc((void **)&p.phi, fbytes) != hipSuccess) {
                destroy(b);
                return fail(FL_E_NOMEM, "batch flux buffers");
            }
            b->owned.push_back(p.phi);
        } else {
            b->any_fused = true;
            const size_t lds = lds_stage_bytes(m, p.S);
            lds_all = lds_all && lds > 0 && lds <= kMaxStageLds;
            lds_max = std::max(lds_max, lds);
        }
        const size_t bytes = (size_t)p.nc * p.S * sizeof(double);
        for (double **dst : {&p.t1, &p.t2}) {
            if (hipMalloc((void **)dst, bytes) != hipSuccess) {
                destroy(b);
                return fail(FL_E_NOMEM, "batch stage buffers");
            }
            b->owned.push_back(*dst);
        }
        b->probs.push_back(p);
        b->meshes.push_back(m);
    }
    b->lds_bytes = b->any_fused && lds_all ? lds_max : 0;
    hipError_t e = hipMalloc((void **)&b->d_probs, b->probs.size() * sizeof(BatchProblem));
    if (e == hipSuccess)
        e = hipMemcpy(b->d_probs, b->probs.data(), b->probs.size() * sizeof(BatchProblem),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreate(&b->cap);
    if (e != hipSuccess) {
        destroy(b);
        return hip_err(e, "batch setup");
    }
    fl_status s = face_tiles(b);
    if (s != FL_OK) {
        destroy(b);
        return s;
    }
    if (!b->any_fused) {
        // nothing for the autotuner: the fused tile table stays empty
        s = set_tile(b, kTileCells);
        b->lds = false;
    } else if (tile_cells > 0) {
        // a fixed tile of kTileCells cells runs staged in LDS where every mesh allows it
        s = set_tile(b, tile_cells);
        b->lds = tile_cells == kTileCells && b->lds_bytes > 0;
    } else {
        const std::string path = tune_cache_path();
        const uint64_t key = tune_key(b);
        int t = 0, l = 0;
        if (tune_cache_read(path, key, &t, &l) && (l == 0 || b->lds_bytes > 0)) {
            s = set_tile(b, t);
            b->lds = l == 1;
            b->tuned_from_cache = true;
        } else {
            // the candidates read theta: order them after the caller's earlier work
            hipError_t e = hipDeviceSynchronize();
            s = e == hipSuccess ? autotune(b, b->cap) : hip_err(e, "hipDeviceSynchronize");
            if (s == FL_OK) tune_cache_write(path, key, b->tile, b->lds ? 1 : 0);
        }
    }
    if (s == FL_OK) s = capture(b);
    if (s == FL_OK) {
        hipError_t e = hipStreamSynchronize(b->cap);
        if (e != hipSuccess) s = hip_err(e, "batch setup");
    }
    if (s != FL_OK) {
        destroy(b);
        return s;
    }
    *out = b;
    return FL_OK;
}

fl_status fl_batch_step(fl_batch *b, int n_steps, void *stream) {
    if (!b) return fail(FL_E_INVALID, "batch is NULL");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    if (!b->exec) return fail(FL_E_INVALID, "batch has no recorded step");
    Guard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    // replay the step recorded at creation on the caller's stream: no sync, no allocation
    for (int i = 0; i < n_steps; ++i) {
        hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
    }
    return FL_OK;
}

fl_status fl_batch_step_unbatched(fl_batch *b, int n_steps, void *stream) {
    if (!b) return fail(FL_E_INVALID, "batch is NULL");
    if (n_steps < 0) return fail(FL_E_INVALID, "n_steps must be >= 0");
    Guard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    for (int it = 0; it < n_steps; ++it)
        for (size_t i = 0; i < b->probs.size(); ++i) {
            const BatchProblem &p = b->probs[i];
            const fl_mesh *m = b->meshes[i];
            // the batch's per-cell work, one problem per launch: LDS-staged tiles when the
            // batch runs staged, the gather kernel otherwise
            auto one = [&](const double *ts, double a, double bb, int mode, double *out) {
                if (p.face) {  // the single-problem face path
                    hipError_t e = launch_face_flux(m, p.lim, p.S, ts, p.u, p.phi, st, 1.0);
                    return e != hipSuccess
                               ? e
                               : launch_cell_update(m, p.S, p.phi, ts, p.th, a, bb, p.dt, mode,
                                                    out, st);
                }
                return b->lds ? launch_fused_lds(m, p.lim, p.S, ts, p.th, nullptr, a, bb, p.dt,
                                                 mode, out, st, 1.0, p.u)
                              : launch_fused(m, p.lim, p.S, ts, p.th, p.u, a, bb, p.dt, mode,
                                             out, st);
            };
            hipError_t e;
            if (b->scheme == FL_EULER) {
                e = one(p.th, 0.0, 1.0, MODE_EULER, p.t1);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(p.th, p.t1, (size_t)p.nc * p.S * sizeof(double),
                                       hipMemcpyDeviceToDevice, st);
            } else {
                e = one(p.th, 0.0, 1.0, MODE_EULER, p.t1);
                if (e == hipSuccess) e = one(p.t1, 0.75, 0.25, MODE_RK, p.t2);
                if (e == hipSuccess) e = one(p.t2, 1.0 / 3.0, 2.0 / 3.0, MODE_RK, p.th);
            }
            if (e != hipSuccess) return hip_err(e, "unbatched launch");
        }
    return FL_OK;
}

fl_status fl_batch_tile(const fl_batch *b, int *tile_cells) {
    if (!b || !tile_cells) return fail(FL_E_INVALID, "NULL argument");
    *tile_cells = b->tile;
    return FL_OK;
}

fl_status fl_batch_lds(const fl_batch *b, int *lds_staged) {
    if (!b || !lds_staged) return fail(FL_E_INVALID, "NULL argument");
    *lds_staged = b->lds ? 1 : 0;
    return FL_OK;
}

fl_status fl_batch_tuned_from_cache(const fl_batch *b, int *from_cache) {
    if (!b || !from_cache) return fail(FL_E_INVALID, "NULL argument");
    *from_cache = b->tuned_from_cache ? 1 : 0;
    return FL_OK;
}

fl_status fl_batch_destroy(fl_batch *b) {
    if (b) destroy(b);
    return FL_OK;
}

}  // extern "C"
