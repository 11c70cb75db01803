// libddf, batched entry points: many independent lattices of uneven size and
// parameters advanced by one persistent launch per time step.
//
// Every instance keeps its own population planes in packed rows (rows of exactly nx
// nodes, planes rounded up to 64 elements; ddf_kernels.hpp) at a 256-byte aligned
// offset inside one f and one g buffer.  The tiles of all instances
// form one flat list; a fixed grid of workgroups walks it, each XCD taking one
// contiguous run of tiles (instances are laid out one after the other, so an XCD's
// L2 sees whole neighbourhoods).  Tile width and workgroups per CU are chosen by
// ddf_batch_autotune, which times the candidates on the actual instance mix and
// caches the choice per (storage, instance sizes).  Runs of K steps are captured once
// into a hipGraph (on an internal stream) and replayed on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/ddf_probe.h"
#include "ddf_kernels.hpp"

using namespace ddf;
using namespace ddf::host;

namespace {

template <class R>
struct InstDesc {
    Lat L;
    int64_t off;        // element offset of this instance's planes in f and g
    int64_t snap_off;   // element offset of its residual snapshot (3 * nx * ny)
    int bx_shift, by, tiles_x, ntiles;   // bx_shift < 0: flat tiles (see inst_node)
    Phys<R> P;
};

// Node of this thread in tile `tile` of an instance.  Rectangular tiles are
// 2^bx_shift x by nodes; flat tiles are kThreads consecutive nodes in row-major order,
// so an instance whose sides are not multiples of the tile leaves idle lanes only in
// its last tile.
template <class R>
__device__ __forceinline__ bool inst_node(const InstDesc<R> &D, int tile, int &x, int &y)
{
    if (D.bx_shift < 0) {
        // nx * ny <= 2^31, so the node index fits 32-bit unsigned arithmetic
        const uint32_t idx = (uint32_t)tile * kThreads + threadIdx.x;
        const uint32_t nx = (uint32_t)D.L.nx;
        if (idx >= nx * (uint32_t)D.L.ny) return false;
        const uint32_t yy = idx / nx;
        y = (int)yy;
        x = (int)(idx - yy * nx);
        return true;
    }
    return tile_node(tile, D.bx_shift, D.by, D.tiles_x, D.L.nx, D.L.ny, x, y);
}

struct TileRef {
    int inst;
    int tile;   // tile index inside the instance
};

template <class S, int SCALAR, bool ODD, bool NT>
__global__ __launch_bounds__(kThreads) void k_batch_step(S *__restrict__ f, S *__restrict__ g,
                                                         const InstDesc<typename Codec<S>::R> *__restrict__ inst,
                                                         const TileRef *__restrict__ tiles, const int ntiles,
                                                         const int64_t t)
{
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int t0 = (int)((int64_t)ntiles * xcd / 8), t1 = (int)((int64_t)ntiles * (xcd + 1) / 8);
    for (int k = t0 + local; k < t1; k += per) {
        const TileRef tr = tiles[k];
        const auto &D = inst[tr.inst];
        int x, y;
        if (inst_node(D, tr.tile, x, y))
            step_node<S, SCALAR, true, true, ODD, false, LY_ROW, NT>(f + D.off, g + D.off, D.L, D.P, x, y, t);
    }
}

// The batch step's memory accesses with the collision left out (the batch counterpart
// of ddf_pattern_probe): same tile list, XCD map and non-temporal policy; each value is
// stored with its top (sign) bit flipped where the step stores the opposite direction,
// which is the slot the step loaded as that direction (walls included).  Two launches of
// one parity restore the populations.
template <class S>
__device__ __forceinline__ S flip_top_bit(S v)
{
    if constexpr (sizeof(S) == 8) {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        u ^= (uint64_t)1 << 63;
        __builtin_memcpy(&v, &u, 8);
    } else if constexpr (sizeof(S) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u ^= 0x80000000u;
        __builtin_memcpy(&v, &u, 4);
    } else {
        uint16_t u;
        __builtin_memcpy(&u, &v, 2);
        u ^= 0x8000u;
        __builtin_memcpy(&v, &u, 2);
    }
    return v;
}

template <class S, bool ODD, bool NT>
__global__ __launch_bounds__(kThreads) void k_batch_pattern(S *__restrict__ f, S *__restrict__ g,
                                                            const InstDesc<typename Codec<S>::R> *__restrict__ inst,
                                                            const TileRef *__restrict__ tiles, const int ntiles)
{
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int t0 = (int)((int64_t)ntiles * xcd / 8), t1 = (int)((int64_t)ntiles * (xcd + 1) / 8);
    for (int k = t0 + local; k < t1; k += per) {
        const TileRef tr = tiles[k];
        const auto &D = inst[tr.inst];
        int x, y;
        if (!inst_node(D, tr.tile, x, y)) continue;
        S *fi = f + D.off, *gi = g + D.off;
        int pa[9];
        int64_t c[9];
        S vf[9], vg[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            c[a] = logical_cell<true, ODD, LY_ROW>(D.L, x, y, a, pa[a]);
            vf[a] = ld_pop<NT>(&elem<false>(fi, D.L, pa[a], c[a]));
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) vg[a] = ld_pop<NT>(&elem<false>(gi, D.L, pa[a], c[a]));
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            st_pop<NT>(&elem<false>(fi, D.L, pa[opp(a)], c[opp(a)]), flip_top_bit(vf[a]));
            st_pop<NT>(&elem<false>(gi, D.L, pa[opp(a)], c[opp(a)]), flip_top_bit(vg[a]));
        }
    }
}

// One workgroup per tile: FP64 partial statistics of the tile.
template <class S, bool ODD>
__global__ __launch_bounds__(kThreads) void k_batch_reduce(const S *__restrict__ f, const S *__restrict__ g,
                                                           const InstDesc<typename Codec<S>::R> *__restrict__ inst,
                                                           const TileRef *__restrict__ tiles,
                                                           typename Codec<S>::R *__restrict__ snap, const int snap_valid,
                                                           const int64_t t, double *__restrict__ partials)
{
    __shared__ double sh[RS_N][kThreads];
    const TileRef tr = tiles[blockIdx.x];
    const auto &D = inst[tr.inst];
    double v[RS_N];
    stats_identity(v);
    int x, y;
    if (inst_node(D, tr.tile, x, y))
        node_stats<S, true, ODD>(f + D.off, g + D.off, D.L, D.P, x, y, t, snap + D.snap_off, snap_valid, v);
    block_reduce_stats<kThreads>(sh, v, partials + (int64_t)blockIdx.x * RS_N);
}

// A tuning result applies to batches with the same storage, scalar collision model and
// instances of the same sizes and boundary kinds (periodic x, periodic y, body force).
struct TuneKey {
    int storage, scalar_model;
    std::vector<std::array<int, 5>> inst;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(storage, scalar_model, inst) < std::tie(o.storage, o.scalar_model, o.inst);
    }
};

// tuned (bx_max, blocks_per_cu, non-temporal even, non-temporal odd)
std::map<TuneKey, std::array<int, 4>> &tune_cache()
{
    static std::map<TuneKey, std::array<int, 4>> c;
    return c;
}

std::mutex &tune_mutex()
{
    static std::mutex m;
    return m;
}

const int kBxCandidates[] = {0, 64, 128, 256, 512};   // 0: flat tiles
const int kBpcCandidates[] = {0, 2, 4, 8};   // 0: one workgroup per tile

}  // namespace

struct ddf_batch {
    int n;
    std::vector<ddf_params> p;
    std::vector<PhysPair> P;
    std::vector<int64_t> off;        // element offsets of the instances' planes
    std::vector<int64_t> node_off;   // offsets in concatenated dense fields
    int64_t total_nodes;
    int storage, scalar_model;
    bool pulsatile;
    void *f, *g, *ws;
    // workspace carve-up
    void *d_inst;
    TileRef *d_tiles;        // all tiles (reductions)
    TileRef *d_step_tiles;   // tiles of the active instances (stepping)
    int nstep_tiles;
    int *d_first, *d_count;
    double *d_partials, *d_out;
    void *d_snap;
    int max_tiles;
    std::vector<unsigned char> active;   // instances whose tiles are in the step list
    // tiling
    int bx_max, bpc, ntiles, grid;
    int nt[2];             // non-temporal loads and stores in the even / odd step kernel
    std::vector<int> first, count;
    int num_cu;
    // state
    int64_t step, snap_step;
    bool snap_valid, initialised;
    // graph
    hipStream_t cap_stream;
    hipGraphExec_t graph_exec;
    hipGraphExec_t graph_red_exec;   // the same K steps followed by the reduction kernels
    int graph_steps;       // K (even); 0 = eager only
    int captured_steps;    // K of the instantiated graph, 0 = none
};

namespace {

size_t inst_desc_size(int storage) { return storage == DDF_F64 ? sizeof(InstDesc<double>) : sizeof(InstDesc<float>); }

int tiles_of(const ddf_params &p, int bx_max)
{
    if (bx_max == 0) return (int)(((int64_t)p.nx * p.ny + kThreads - 1) / kThreads);
    const Geom G = make_geom(p, bx_max);
    return G.ntiles;
}

struct Carve {
    size_t inst, tiles, first, count, partials, out, snap, total;
};

Carve carve(int n, const ddf_params *ps, int max_tiles, int64_t total_nodes)
{
    Carve c;
    size_t o = 0;
    c.inst = o; o += align256((size_t)n * inst_desc_size(ps[0].storage));
    c.tiles = o; o += 2 * align256((size_t)max_tiles * sizeof(TileRef));
    c.first = o; o += align256((size_t)n * sizeof(int));
    c.count = o; o += align256((size_t)n * sizeof(int));
    c.partials = o; o += align256((size_t)max_tiles * RS_N * sizeof(double));
    c.out = o; o += align256((size_t)n * RS_N * sizeof(double));
    c.snap = o; o += align256(3 * (size_t)total_nodes * (ps[0].storage == DDF_F64 ? 8 : 4));
    c.total = o;
    return c;
}

int max_tiles_of(int n, const ddf_params *ps)
{
    int best = 0;
    for (int bx : kBxCandidates) {
        int t = 0;
        for (int i = 0; i < n; ++i) t += tiles_of(ps[i], bx);
        best = std::max(best, t);
    }
    return best;
}

// Batch instances always keep packed rows.
ddf_params packed(ddf_params p)
{
    p.layout = DDF_LAYOUT_PACKED;
    return p;
}

int validate_batch(int n, const ddf_params *ps)
{
    if (n <= 0 || !ps) return fail(DDF_ERR_ARG, "batch needs n > 0 instances");
    for (int i = 0; i < n; ++i) {
        int rc = validate(&ps[i]);
        if (rc != DDF_OK) return fail(rc, "instance " + std::to_string(i) + ": " + error_slot());
        if (ps[i].storage != ps[0].storage) return fail(DDF_ERR_ARG, "all batch instances must share one storage type");
        const int m0 = ps[0].scalar_model == DDF_SCALAR_CASCADED ? DDF_SCALAR_CENTRAL : ps[0].scalar_model;
        const int mi = ps[i].scalar_model == DDF_SCALAR_CASCADED ? DDF_SCALAR_CENTRAL : ps[i].scalar_model;
        if (mi != m0) return fail(DDF_ERR_ARG, "all batch instances must share one scalar collision model");
        if (ps[i].layout == DDF_LAYOUT_ROW || ps[i].layout == DDF_LAYOUT_INTERLEAVED)
            return fail(DDF_ERR_UNSUPPORTED, "instance " + std::to_string(i) + ": batches keep packed rows "
                                             "(layout AUTO or PACKED)");
    }
    return DDF_OK;
}

template <class R>
void fill_desc(const ddf_batch *b, std::vector<InstDesc<R>> &d, std::vector<TileRef> &tl)
{
    d.resize(b->n);
    tl.clear();
    for (int i = 0; i < b->n; ++i) {
        const Geom G = make_geom(b->p[i], b->bx_max == 0 ? kThreads : b->bx_max);
        InstDesc<R> &D = d[i];
        std::memset(&D, 0, sizeof(D));
        D.L = G.L;
        D.off = b->off[i];
        D.snap_off = 3 * b->node_off[i];
        D.bx_shift = b->bx_max == 0 ? -1 : G.bx_shift;
        D.by = G.by;
        D.tiles_x = G.tiles_x;
        D.ntiles = tiles_of(b->p[i], b->bx_max);
        if constexpr (std::is_same<R, double>::value) D.P = b->P[i].d;
        else D.P = b->P[i].f;
        for (int k = 0; k < D.ntiles; ++k) tl.push_back(TileRef{i, k});
    }
}

// The host-side setters upload descriptors and tile lists on the private capture
// stream, which is not ordered after the caller's streams.  Their buffers may have been
// handed out by the caller's allocator while earlier work of the caller still writes
// that memory, and a replay of the old graph may still be reading the lists: wait for
// the whole device first.
int quiesce()
{
    DDF_HIP_TRY(hipDeviceSynchronize());
    return DDF_OK;
}

void drop_graph(ddf_batch *b)
{
    if (b->captured_steps) {
        (void)hipGraphExecDestroy(b->graph_exec);
        (void)hipGraphExecDestroy(b->graph_red_exec);
        b->captured_steps = 0;
    }
}

// Rebuilds descriptors and the tile list for (bx_max, bpc) and uploads them.
int apply_tiling(ddf_batch *b, int bx_max, int bpc, hipStream_t st)
{
    b->bx_max = bx_max;
    b->bpc = bpc;
    std::vector<TileRef> tl;
    std::vector<char> blob;
    if (b->storage == DDF_F64) {
        std::vector<InstDesc<double>> d;
        fill_desc(b, d, tl);
        blob.assign((const char *)d.data(), (const char *)d.data() + d.size() * sizeof(d[0]));
    } else {
        std::vector<InstDesc<float>> d;
        fill_desc(b, d, tl);
        blob.assign((const char *)d.data(), (const char *)d.data() + d.size() * sizeof(d[0]));
    }
    b->ntiles = (int)tl.size();
    if (b->ntiles > b->max_tiles) return fail(DDF_ERR_ARG, "tile list exceeds the workspace");
    b->first.assign(b->n, 0);
    b->count.assign(b->n, 0);
    for (int k = 0; k < b->ntiles; ++k) {
        if (b->count[tl[k].inst] == 0) b->first[tl[k].inst] = k;
        b->count[tl[k].inst]++;
    }
    DDF_HIP_TRY(hipMemcpyAsync(b->d_inst, blob.data(), blob.size(), hipMemcpyHostToDevice, st));
    std::vector<TileRef> act;
    for (const TileRef &t : tl)
        if (b->active[t.inst]) act.push_back(t);
    b->nstep_tiles = (int)act.size();
    DDF_HIP_TRY(hipMemcpyAsync(b->d_tiles, tl.data(), tl.size() * sizeof(TileRef), hipMemcpyHostToDevice, st));
    if (!act.empty())
        DDF_HIP_TRY(hipMemcpyAsync(b->d_step_tiles, act.data(), act.size() * sizeof(TileRef), hipMemcpyHostToDevice, st));
    DDF_HIP_TRY(hipMemcpyAsync(b->d_first, b->first.data(), b->n * sizeof(int), hipMemcpyHostToDevice, st));
    DDF_HIP_TRY(hipMemcpyAsync(b->d_count, b->count.data(), b->n * sizeof(int), hipMemcpyHostToDevice, st));
    DDF_HIP_TRY(hipStreamSynchronize(st));   // host vectors are released on return
    const int g = bpc == 0 ? b->nstep_tiles : bpc * b->num_cu;
    b->grid = std::max(8, (g + 7) / 8 * 8);
    drop_graph(b);
    return DDF_OK;
}

template <class S, int SC>
void launch_batch_step(ddf_batch *b, hipStream_t st, bool odd, int64_t t)
{
    using R = typename Codec<S>::R;
    const auto *inst = (const InstDesc<R> *)b->d_inst;
    if (b->nstep_tiles == 0) return;
#define DDF_BS(O_, N_)                                                                                              \
    hipLaunchKernelGGL((k_batch_step<S, SC, O_, N_>), dim3(b->grid), dim3(kThreads), 0, st, (S *)b->f, (S *)b->g, inst, \
                       b->d_step_tiles, b->nstep_tiles, t)
    if (odd) { if (b->nt[1]) DDF_BS(true, true); else DDF_BS(true, false); }
    else { if (b->nt[0]) DDF_BS(false, true); else DDF_BS(false, false); }
#undef DDF_BS
}

void launch_one_step(ddf_batch *b, hipStream_t st, int64_t step)
{
    const bool odd = (step & 1) != 0;
    with_storage(b->storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        switch (b->scalar_model) {
        case DDF_SCALAR_SRT: launch_batch_step<S, DDF_SCALAR_SRT>(b, st, odd, step); break;
        case DDF_SCALAR_CASCADED:
        case DDF_SCALAR_CENTRAL: launch_batch_step<S, DDF_SCALAR_CENTRAL>(b, st, odd, step); break;
        default: launch_batch_step<S, DDF_SCALAR_MRT>(b, st, odd, step);
        }
        return 0;
    });
}

// The reduction kernels of the current state: per-tile FP64 partials (against the
// residual snapshot when sv, which is then overwritten) and their per-instance sums in
// d_out.  t is the time index (it matters only for a time-dependent force).
void launch_reduce(ddf_batch *b, hipStream_t st, bool odd, int sv, int64_t t)
{
    with_storage(b->storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        using R = typename Codec<S>::R;
        const auto *inst = (const InstDesc<R> *)b->d_inst;
        if (odd)
            hipLaunchKernelGGL((k_batch_reduce<S, true>), dim3(b->ntiles), dim3(kThreads), 0, st, (const S *)b->f,
                               (const S *)b->g, inst, b->d_tiles, (R *)b->d_snap, sv, t, b->d_partials);
        else
            hipLaunchKernelGGL((k_batch_reduce<S, false>), dim3(b->ntiles), dim3(kThreads), 0, st, (const S *)b->f,
                               (const S *)b->g, inst, b->d_tiles, (R *)b->d_snap, sv, t, b->d_partials);
        return 0;
    });
    hipLaunchKernelGGL(k_reduce_rows<256>, dim3(b->n), dim3(256), 0, st, b->d_partials, b->d_first, b->d_count, 0,
                       b->d_out);
}

// Two graphs of K steps from an even step: the plain run, and the run followed by the
// reduction.  The captured reduction always compares with the snapshot; before the
// first reduction that comparison reads an unset snapshot, and the host reports no
// residual for it.  Graphs are used only where the step does not depend on time.
int capture_graph(ddf_batch *b)
{
    drop_graph(b);
    hipGraph_t graph;
    DDF_HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < b->graph_steps; ++k) launch_one_step(b, b->cap_stream, k);   // starts at an even step
    DDF_HIP_TRY(hipStreamEndCapture(b->cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(&b->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(DDF_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < b->graph_steps; ++k) launch_one_step(b, b->cap_stream, k);
        launch_reduce(b, b->cap_stream, false, 1, b->graph_steps);
        e = hipStreamEndCapture(b->cap_stream, &graph);
        if (e == hipSuccess) {
            e = hipGraphInstantiate(&b->graph_red_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
        }
    }
    if (e != hipSuccess) {   // the first graph is not kept without the second
        (void)hipGraphExecDestroy(b->graph_exec);
        return fail(DDF_ERR_HIP, std::string("capturing the step-and-reduce graph: ") + hipGetErrorString(e));
    }
    b->captured_steps = b->graph_steps;
    return DDF_OK;
}

// Copies the per-instance sums of the last reduction to the host and turns them into
// the DDF_STAT_* rows of out; the current state becomes the residual snapshot.
int finish_reduce(ddf_batch *b, double *out, hipStream_t st)
{
    std::vector<double> r((size_t)b->n * RS_N);
    DDF_HIP_TRY(hipMemcpyAsync(r.data(), b->d_out, r.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    DDF_HIP_TRY(hipStreamSynchronize(st));
    const double K = (double)(b->step - b->snap_step);
    bool bad = false;
    for (int i = 0; i < b->n; ++i) {
        const double *ri = &r[(size_t)i * RS_N];
        double *o = out + (size_t)i * DDF_NUM_STATS;
        o[DDF_STAT_MASS] = ri[RS_MASS];
        o[DDF_STAT_SCALAR] = ri[RS_SCALAR];
        o[DDF_STAT_RES_U] = (b->snap_valid && K > 0) ? std::sqrt(ri[RS_DU2]) / (K * std::sqrt(ri[RS_U2])) : NAN;
        o[DDF_STAT_RES_PHI] = (b->snap_valid && K > 0) ? std::sqrt(ri[RS_DPHI2]) / (K * std::sqrt(ri[RS_PHI2])) : NAN;
        o[DDF_STAT_NONFINITE] = ri[RS_NONFIN];
        o[DDF_STAT_STEPS] = b->snap_valid ? K : 0.0;
        o[DDF_STAT_UMAX] = ri[RS_UMAX];
        o[DDF_STAT_PHIMIN] = ri[RS_PHIMIN];
        bad |= ri[RS_NONFIN] > 0.0;
    }
    b->snap_valid = true;
    b->snap_step = b->step;
    if (bad) return fail(DDF_ERR_NONFINITE, "at least one instance holds non-finite values");
    return DDF_OK;
}

}  // namespace

extern "C" {

size_t ddf_batch_population_bytes(int32_t n, const ddf_params *ps)
{
    if (n <= 0 || !ps) return 0;
    size_t tot = 0;
    for (int i = 0; i < n; ++i) {
        const ddf_params q = packed(ps[i]);
        tot += population_bytes(&q);
    }
    return tot;
}

size_t ddf_batch_workspace_bytes(int32_t n, const ddf_params *ps)
{
    if (validate_batch(n, ps) != DDF_OK) return 0;
    int64_t nodes = 0;
    for (int i = 0; i < n; ++i) nodes += (int64_t)ps[i].nx * ps[i].ny;
    return carve(n, ps, max_tiles_of(n, ps), nodes).total;
}

int ddf_batch_create(int32_t n, const ddf_params *ps, void *pop_f, void *pop_g, void *workspace, ddf_batch **out)
{
    int rc = validate_batch(n, ps);
    if (rc != DDF_OK) return rc;
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (!pop_f || !pop_g || !workspace) return fail(DDF_ERR_ARG, "a device buffer is NULL");
    if (((uintptr_t)pop_f | (uintptr_t)pop_g | (uintptr_t)workspace) & 255)
        return fail(DDF_ERR_ARG, "device buffers must be 256-byte aligned");
    ddf_batch *b = new (std::nothrow) ddf_batch;
    if (!b) return fail(DDF_ERR_ARG, "out of host memory");
    b->n = n;
    b->p.assign(ps, ps + n);
    for (ddf_params &q : b->p) q = packed(q);
    b->storage = ps[0].storage;
    b->scalar_model = ps[0].scalar_model;
    b->pulsatile = false;
    int64_t off = 0, nodes = 0;
    const size_t s = storage_size(b->storage);
    for (int i = 0; i < n; ++i) {
        b->off.push_back(off);
        b->node_off.push_back(nodes);
        off += (int64_t)(population_bytes(&b->p[i]) / s);
        nodes += (int64_t)ps[i].nx * ps[i].ny;
        PhysPair pp;
        pp.d = make_phys<double>(ps[i]);
        pp.f = make_phys<float>(ps[i]);
        b->P.push_back(pp);
        if (ps[i].force_kind == DDF_FORCE_PULSATILE) b->pulsatile = true;
    }
    b->total_nodes = nodes;
    b->f = pop_f;
    b->g = pop_g;
    b->ws = workspace;
    b->max_tiles = max_tiles_of(n, ps);
    const Carve c = carve(n, ps, b->max_tiles, nodes);
    char *w = (char *)workspace;
    b->d_inst = w + c.inst;
    b->d_tiles = (TileRef *)(w + c.tiles);
    b->d_step_tiles = (TileRef *)(w + c.tiles + align256((size_t)b->max_tiles * sizeof(TileRef)));
    b->active.assign(n, 1);
    b->d_first = (int *)(w + c.first);
    b->d_count = (int *)(w + c.count);
    b->d_partials = (double *)(w + c.partials);
    b->d_out = (double *)(w + c.out);
    b->d_snap = w + c.snap;
    b->step = 0;
    b->snap_step = 0;
    b->snap_valid = false;
    b->initialised = false;
    b->captured_steps = 0;
    b->nt[0] = b->nt[1] = 0;
    // kernels take the time index as an argument, which a captured graph freezes: a
    // time-dependent force or stochastic rounding keys need eager launches
    b->graph_steps = (b->pulsatile || b->storage == DDF_BF16_SR) ? 0 : 100;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete b;
        return fail(DDF_ERR_HIP, "cannot query the device");
    }
    b->num_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(DDF_ERR_HIP, "cannot create the capture stream");
    }
    rc = quiesce();
    if (rc == DDF_OK) rc = apply_tiling(b, 0, 0, b->cap_stream);
    if (rc != DDF_OK) {
        (void)hipStreamDestroy(b->cap_stream);
        delete b;
        return rc;
    }
    *out = b;
    return DDF_OK;
}

void ddf_batch_destroy(ddf_batch *b)
{
    if (!b) return;
    (void)quiesce();
    drop_graph(b);
    (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

int32_t ddf_batch_size(const ddf_batch *b) { return b ? b->n : 0; }

int64_t ddf_batch_step_count(const ddf_batch *b) { return b ? b->step : -1; }

int ddf_batch_offsets(const ddf_batch *b, int32_t i, int64_t *pop_offset_bytes, int64_t *field_offset)
{
    if (!b || i < 0 || i >= b->n) return fail(DDF_ERR_ARG, "bad batch or instance index");
    if (pop_offset_bytes) *pop_offset_bytes = b->off[i] * (int64_t)storage_size(b->storage);
    if (field_offset) *field_offset = b->node_off[i];
    return DDF_OK;
}

int ddf_batch_init_equilibrium(ddf_batch *b, const double *rho, const double *ux, const double *uy, const double *phi,
                               void *stream)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (!rho || !ux || !uy || !phi) return fail(DDF_ERR_ARG, "a field pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    const size_t s = storage_size(b->storage);
    for (int i = 0; i < b->n; ++i) {
        const Geom G = make_geom(b->p[i]);
        const int64_t o = b->node_off[i];
        with_storage(b->storage, [&](auto *tag) {
            using S = std::remove_pointer_t<decltype(tag)>;
            hipLaunchKernelGGL((k_init<S>), dim3(grid_blocks(G)), dim3(kThreads), 0, st, (S *)((char *)b->f + b->off[i] * s),
                               (S *)((char *)b->g + b->off[i] * s), G, b->P[i].of<S>(), rho + o, ux + o, uy + o, phi + o);
            return 0;
        });
    }
    DDF_HIP_TRY(hipGetLastError());
    b->step = 0;
    b->snap_valid = false;
    b->initialised = true;
    return DDF_OK;
}

int ddf_batch_set_active(ddf_batch *b, const uint8_t *active)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (!active) return fail(DDF_ERR_ARG, "active is NULL");
    // an instance leaves and re-enters the step list in the natural slot order, so its
    // stored state stays readable as an even-step state while it is out
    if (b->step & 1) return fail(DDF_ERR_STATE, "set_active needs an even step count (natural slot order)");
    int rc = quiesce();
    if (rc != DDF_OK) return rc;
    for (int i = 0; i < b->n; ++i) b->active[i] = active[i] ? 1 : 0;
    return apply_tiling(b, b->bx_max, b->bpc, b->cap_stream);
}

int ddf_batch_init_instance(ddf_batch *b, int32_t i, const double *rho, const double *ux, const double *uy,
                            const double *phi, void *stream)
{
    if (!b || i < 0 || i >= b->n) return fail(DDF_ERR_ARG, "bad batch or instance index");
    if (!rho || !ux || !uy || !phi) return fail(DDF_ERR_ARG, "a field pointer is NULL");
    if (!b->initialised) return fail(DDF_ERR_STATE, "init_instance before ddf_batch_init_equilibrium");
    if (b->step & 1) return fail(DDF_ERR_STATE, "init_instance needs an even step count (natural slot order)");
    const size_t s = storage_size(b->storage);
    const Geom G = make_geom(b->p[i]);
    with_storage(b->storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL((k_init<S>), dim3(grid_blocks(G)), dim3(kThreads), 0, (hipStream_t)stream,
                           (S *)((char *)b->f + b->off[i] * s), (S *)((char *)b->g + b->off[i] * s), G,
                           b->P[i].of<S>(), rho, ux, uy, phi);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_batch_set_tiling(ddf_batch *b, int32_t bx_max, int32_t blocks_per_cu)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    bool ok = false;
    for (int c : kBxCandidates) ok |= (c == bx_max);
    if (!ok) return fail(DDF_ERR_ARG, "bx_max must be 0 (flat tiles), 64, 128, 256 or 512");
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(DDF_ERR_ARG, "blocks_per_cu must lie in [0, 64]");
    int rc = quiesce();
    if (rc != DDF_OK) return rc;
    return apply_tiling(b, bx_max, blocks_per_cu, b->cap_stream);
}

int ddf_batch_set_nontemporal(ddf_batch *b, int32_t even, int32_t odd)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if ((even != 0 && even != 1) || (odd != 0 && odd != 1)) return fail(DDF_ERR_ARG, "non-temporal flags are 0 or 1");
    if (b->captured_steps) {
        int rc = quiesce();
        if (rc != DDF_OK) return rc;
    }
    drop_graph(b);
    b->nt[0] = even;
    b->nt[1] = odd;
    return DDF_OK;
}

int ddf_batch_get_nontemporal(const ddf_batch *b, int32_t *even, int32_t *odd)
{
    if (!b || !even || !odd) return fail(DDF_ERR_ARG, "NULL argument");
    *even = b->nt[0];
    *odd = b->nt[1];
    return DDF_OK;
}

int ddf_batch_get_tiling(const ddf_batch *b, int32_t *bx_max, int32_t *blocks_per_cu, int32_t *ntiles, int32_t *grid)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (bx_max) *bx_max = b->bx_max;
    if (blocks_per_cu) *blocks_per_cu = b->bpc;
    if (ntiles) *ntiles = b->ntiles;
    if (grid) *grid = b->grid;
    return DDF_OK;
}

int ddf_batch_set_graph(ddf_batch *b, int32_t steps_per_graph)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (steps_per_graph < 0 || (steps_per_graph & 1)) return fail(DDF_ERR_ARG, "steps_per_graph must be even and >= 0");
    if (steps_per_graph > 0 && (b->pulsatile || b->storage == DDF_BF16_SR))
        return fail(DDF_ERR_UNSUPPORTED, "time-dependent forces and stochastic rounding step eagerly (no graph capture)");
    if (b->captured_steps) {
        int rc = quiesce();
        if (rc != DDF_OK) return rc;
    }
    drop_graph(b);
    b->graph_steps = steps_per_graph;
    return DDF_OK;
}

int ddf_batch_pattern_probe(ddf_batch *b, int32_t parity, void *stream)
{
    if (!b) return fail(DDF_ERR_ARG, "batch pattern probe: batch is NULL");
    if (parity != 0 && parity != 1) return fail(DDF_ERR_ARG, "batch pattern probe: parity must be 0 (even) or 1 (odd)");
    if (b->nstep_tiles == 0) return DDF_OK;
    hipStream_t st = (hipStream_t)stream;
    with_storage(b->storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        using R = typename Codec<S>::R;
        const auto *inst = (const InstDesc<R> *)b->d_inst;
#define DDF_BP(O_, N_)                                                                                              \
        hipLaunchKernelGGL((k_batch_pattern<S, O_, N_>), dim3(b->grid), dim3(kThreads), 0, st, (S *)b->f, (S *)b->g, inst, \
                           b->d_step_tiles, b->nstep_tiles)
        if (parity) { if (b->nt[1]) DDF_BP(true, true); else DDF_BP(true, false); }
        else { if (b->nt[0]) DDF_BP(false, true); else DDF_BP(false, false); }
#undef DDF_BP
        return 0;
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DDF_ERR_HIP, std::string("batch pattern probe launch: ") + hipGetErrorString(e));
    return DDF_OK;
}

int ddf_batch_step(ddf_batch *b, int64_t nsteps, void *stream)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (nsteps < 0) return fail(DDF_ERR_ARG, "nsteps < 0");
    if (!b->initialised) return fail(DDF_ERR_STATE, "step before init");
    hipStream_t st = (hipStream_t)stream;
    int64_t left = nsteps;
    if (b->graph_steps > 0 && left >= b->graph_steps + (b->step & 1)) {
        if (b->step & 1) {
            launch_one_step(b, st, b->step);
            b->step++;
            left--;
        }
        if (b->captured_steps != b->graph_steps) {
            int rc = capture_graph(b);
            if (rc != DDF_OK) return rc;
        }
        while (left >= b->graph_steps) {
            DDF_HIP_TRY(hipGraphLaunch(b->graph_exec, st));
            b->step += b->graph_steps;
            left -= b->graph_steps;
        }
    }
    for (; left > 0; --left) {
        launch_one_step(b, st, b->step);
        b->step++;
    }
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_batch_autotune(ddf_batch *b, int32_t steps_per_trial, int32_t *bx_max_out, int32_t *blocks_per_cu_out,
                       float *best_ms_per_step, void *stream)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (steps_per_trial < 2) return fail(DDF_ERR_ARG, "steps_per_trial must be >= 2");
    hipStream_t st = (hipStream_t)stream;
    // the tile lists are replaced below, which a replay of a captured graph may still read
    int qrc = quiesce();
    if (qrc != DDF_OK) return qrc;
    TuneKey key;
    key.storage = b->storage;
    key.scalar_model = b->scalar_model == DDF_SCALAR_CASCADED ? DDF_SCALAR_CENTRAL : b->scalar_model;
    for (int i = 0; i < b->n; ++i)
        key.inst.push_back({b->p[i].nx, b->p[i].ny, b->p[i].periodic_x ? 1 : 0, b->p[i].periodic_y ? 1 : 0,
                            b->p[i].force_kind});
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            b->nt[0] = it->second[2];
            b->nt[1] = it->second[3];
            int rc = apply_tiling(b, it->second[0], it->second[1], st);
            if (rc != DDF_OK) return rc;
            if (bx_max_out) *bx_max_out = b->bx_max;
            if (blocks_per_cu_out) *blocks_per_cu_out = b->bpc;
            if (best_ms_per_step) *best_ms_per_step = -1.0f;
            return DDF_OK;
        }
    }
    // Trial runs start from the rest state (all offsets zero) and leave the populations
    // clobbered: the caller initialises afterwards.
    const size_t s = storage_size(b->storage);
    size_t bytes = 0;
    for (int i = 0; i < b->n; ++i) bytes += population_bytes(&b->p[i]);
    DDF_HIP_TRY(hipMemsetAsync(b->f, 0, bytes, st));
    DDF_HIP_TRY(hipMemsetAsync(b->g, 0, bytes, st));
    (void)s;
    hipEvent_t e0, e1;
    DDF_HIP_TRY(hipEventCreate(&e0));
    DDF_HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    int best_bx = 512, best_bpc = 0, best_nt[2] = {0, 0};
    auto trial = [&](int bx, int bpc, int nte, int nto) -> int {
        b->nt[0] = nte;
        b->nt[1] = nto;
        int rc = apply_tiling(b, bx, bpc, st);
        if (rc != DDF_OK) return rc;
        launch_one_step(b, st, 0);
        launch_one_step(b, st, 1);
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < steps_per_trial; ++k) launch_one_step(b, st, k);
        (void)hipEventRecord(e1, st);
        DDF_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)steps_per_trial;
        if (ms < best) {
            best = ms;
            best_bx = bx;
            best_bpc = bpc;
            best_nt[0] = nte;
            best_nt[1] = nto;
        }
        return DDF_OK;
    };
    // tile shapes with plain accesses, then non-temporal accesses per parity on the best
    for (int bx : kBxCandidates)
        for (int bpc : kBpcCandidates) {
            int rc = trial(bx, bpc, 0, 0);
            if (rc != DDF_OK) return rc;
        }
    {
        const int bx = best_bx, bpc = best_bpc;
        for (const auto &nt : {std::array<int, 2>{1, 0}, std::array<int, 2>{0, 1}, std::array<int, 2>{1, 1}}) {
            int rc = trial(bx, bpc, nt[0], nt[1]);
            if (rc != DDF_OK) return rc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->nt[0] = best_nt[0];
    b->nt[1] = best_nt[1];
    int rc = apply_tiling(b, best_bx, best_bpc, st);
    if (rc != DDF_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        tune_cache()[key] = {best_bx, best_bpc, best_nt[0], best_nt[1]};
    }
    b->initialised = false;
    if (bx_max_out) *bx_max_out = best_bx;
    if (blocks_per_cu_out) *blocks_per_cu_out = best_bpc;
    if (best_ms_per_step) *best_ms_per_step = best;
    return DDF_OK;
}

}  // extern "C"

// Slot order of instance i's stored state: an inactive instance was taken out at an even
// step count and has not moved since.
static bool inst_odd(const ddf_batch *b, int i) { return b->active[i] && (b->step & 1) != 0; }

extern "C" {

int ddf_batch_reduce(ddf_batch *b, double *out, void *stream)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (!b->initialised) return fail(DDF_ERR_STATE, "reduce before init");
    hipStream_t st = (hipStream_t)stream;
    const bool odd = (b->step & 1) != 0;
    if (odd)
        for (int i = 0; i < b->n; ++i)
            if (!b->active[i]) return fail(DDF_ERR_STATE, "reduce at an odd step count while an instance is inactive");
    launch_reduce(b, st, odd, b->snap_valid ? 1 : 0, b->step);
    DDF_HIP_TRY(hipGetLastError());
    return finish_reduce(b, out, st);
}

int ddf_batch_step_reduce(ddf_batch *b, int64_t nsteps, double *out, void *stream)
{
    if (!b) return fail(DDF_ERR_ARG, "batch is NULL");
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (nsteps < 0) return fail(DDF_ERR_ARG, "nsteps < 0");
    if (!b->initialised) return fail(DDF_ERR_STATE, "step before init");
    hipStream_t st = (hipStream_t)stream;
    const int64_t K = b->graph_steps, lead = b->step & 1;
    if (K > 0 && nsteps >= K + lead && (nsteps - lead) % K == 0) {
        // the run ends on a whole replay: the last one carries the reduction
        int64_t left = nsteps;
        if (lead) {
            launch_one_step(b, st, b->step);
            b->step++;
            left--;
        }
        if (b->captured_steps != K) {
            int rc = capture_graph(b);
            if (rc != DDF_OK) return rc;
        }
        for (; left > K; left -= K, b->step += K) DDF_HIP_TRY(hipGraphLaunch(b->graph_exec, st));
        DDF_HIP_TRY(hipGraphLaunch(b->graph_red_exec, st));
        b->step += K;
        return finish_reduce(b, out, st);
    }
    int rc = ddf_batch_step(b, nsteps, stream);
    if (rc != DDF_OK) return rc;
    return ddf_batch_reduce(b, out, stream);
}

int ddf_batch_extract(ddf_batch *b, int32_t i, void *out, uint32_t mask, int32_t out_dtype, void *stream)
{
    if (!b || i < 0 || i >= b->n) return fail(DDF_ERR_ARG, "bad batch or instance index");
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (out_dtype != 0 && out_dtype != 1) return fail(DDF_ERR_ARG, "out_dtype must be 0 (double) or 1 (float)");
    if (!b->initialised) return fail(DDF_ERR_STATE, "extract before init");
    const size_t s = storage_size(b->storage);
    const Geom G = make_geom(b->p[i]);
    with_storage(b->storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        launch_extract<S>(G, b->P[i].of<S>(), has_walls(b->p[i]), inst_odd(b, i), (char *)b->f + b->off[i] * s,
                          (char *)b->g + b->off[i] * s, b->step, b->p[i].scalar_model, out, out_dtype, mask,
                          (hipStream_t)stream);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_batch_get_populations(ddf_batch *b, int32_t i, void *f, void *g, int32_t dtype, void *stream)
{
    if (!b || i < 0 || i >= b->n) return fail(DDF_ERR_ARG, "bad batch or instance index");
    if (!f || !g) return fail(DDF_ERR_ARG, "output pointer is NULL");
    if (dtype != 0 && dtype != 1) return fail(DDF_ERR_ARG, "dtype must be 0 (double) or 1 (raw)");
    if (!b->initialised) return fail(DDF_ERR_STATE, "get_populations before init");
    const size_t s = storage_size(b->storage);
    const Geom G = make_geom(b->p[i]);
    with_storage(b->storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        launch_get<S>(G, b->P[i].of<S>(), has_walls(b->p[i]), inst_odd(b, i), (char *)b->f + b->off[i] * s,
                      (char *)b->g + b->off[i] * s, f, g, dtype, (hipStream_t)stream);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

}  // extern "C"
