// libddf, single-lattice entry points: fused two-lattice DDF lattice Boltzmann step,
// local kinematics extraction and FP64 reductions for MI355X (gfx950), behind the
// C ABI declared in include/ddf.h.  Kernels and layout: ddf_kernels.hpp.
#include "ddf_handle.hpp"

using namespace ddf;
using namespace ddf::host;

namespace {

// Kernels take the time index as an argument, which a captured graph freezes: lattices
// whose step depends on it (a time-dependent force, stochastic rounding keys) run eagerly.
bool graph_capable(const ddf_params &p) { return p.force_kind != DDF_FORCE_PULSATILE && p.storage != DDF_BF16_SR; }

void drop_graph(ddf_handle *h)
{
    if (h->captured_steps) {
        (void)hipGraphExecDestroy(h->graph_exec);
        h->captured_steps = 0;
    }
}

int capture_graph(ddf_handle *h)
{
    drop_graph(h);
    if (!h->cap_stream) DDF_HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph;
    DDF_HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < h->graph_steps; ++k) launch_one(h, h->cap_stream, k);   // starts at an even step
    DDF_HIP_TRY(hipStreamEndCapture(h->cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(DDF_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h->captured_steps = h->graph_steps;
    return DDF_OK;
}

}  // namespace

extern "C" {

int64_t ddf_pitch(const ddf_params *p) { return p ? pitch_of(p) : 0; }

int64_t ddf_plane_stride(const ddf_params *p) { return p ? plane_of(p) : 0; }

size_t ddf_population_bytes(const ddf_params *p) { return p ? population_bytes(p) : 0; }

size_t ddf_workspace_bytes(const ddf_params *p)
{
    if (!p || validate(p) != DDF_OK) return 0;
    // reduction partials for the largest block count any tile width gives
    int blocks = 0;
    for (int bx : {64, 128, 256, 512}) blocks = std::max(blocks, grid_blocks(make_geom(*p, bx)));
    return snap_bytes(p) + align256((size_t)blocks * RS_N * sizeof(double)) + 256;
}

int ddf_set_tile_width(ddf_handle *h, int32_t bx_max)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (bx_max != 64 && bx_max != 128 && bx_max != 256 && bx_max != 512)
        return fail(DDF_ERR_ARG, "tile width must be 64, 128, 256 or 512");
    if (h->captured_steps) DDF_HIP_TRY(hipDeviceSynchronize());   // a replay may still be running
    drop_graph(h);
    h->tile_width = bx_max;
    const int qs = h->G.L.qs;
    h->G = make_geom(h->p, bx_max);
    h->G.L.qs = qs;
    h->nblocks = grid_blocks(h->G);
    return DDF_OK;
}

namespace {
// Whether every lane offset of the lattice's planes fits 32 bits as a byte count.
bool plane_fits_32(const ddf_handle *h)
{
    return (uint64_t)h->G.L.plane * (uint64_t)storage_size(h->p.storage) < (1ull << 32);
}

// Launch defaults of the step kernels, measured on the 8192^2 periodic field (with and
// without a body force) and an 8192^2 cavity (one MI355X).  Lattices whose two
// population arrays exceed the 256 MB Infinity Cache stream from HBM: there fewer
// resident workgroups per CU made the FP32 steps faster (one of the four possible:
// -6% on the periodic field; two with walls: -2.7% on the cavity, which one made 10%
// slower), FP64 (one: -4.4% to -5.3% with or without walls and force) and the periodic
// FP16 and BF16 steps (3 even, 2 odd, 64-bit offsets, -2.3% and -2.6%), while the FP16
// cavity step and the stochastic-rounding codec need every wavefront to hide their
// latency (the FP16 cavity step was 13% slower with caps).  Lattices held by the
// cache keep every wavefront.
//
// x-interleaved rows (non-temporal accesses, no gap between planes; every cap pair and
// both offset widths): on the 8192^2 field FP32 2 / 2 (6.2 TB/s), FP64 1 / 1 (6.4 TB/s),
// FP16 3 / 3 and BF16 3 / 0 with 64-bit offsets (6.0 and 6.1 TB/s), BF16 with
// stochastic rounding 3 / 0 (5.5 TB/s); on an 8192^2 cavity (measured with plane gaps)
// FP32 2 / 2 (6.1 TB/s), FP64 1 / 1 (4.8 TB/s) and the 16-bit formats 3 / 0 (5.6 TB/s).
void launch_defaults(ddf_handle *h)
{
    h->idx32 = plane_fits_32(h);
    h->wg_cap[0] = h->wg_cap[1] = 0;
    if (2 * population_bytes(&h->p) <= (size_t)256 << 20) return;
    if (h->G.L.qs) {
        static const int caps[5][2] = {{1, 1}, {2, 2}, {3, 3}, {3, 0}, {3, 0}};   // by ddf_storage
        const bool sixteen = h->p.storage == DDF_F16 || h->p.storage == DDF_BF16;
        const bool walls = has_walls(h->p);
        h->wg_cap[0] = caps[h->p.storage][0];
        h->wg_cap[1] = sixteen && walls ? 0 : caps[h->p.storage][1];
        if (sixteen && !walls) h->idx32 = false;
        return;
    }
    if (h->p.storage == DDF_F32) {
        h->wg_cap[0] = h->wg_cap[1] = has_walls(h->p) ? 2 : 1;
    } else if (h->p.storage == DDF_F64) {
        h->wg_cap[0] = h->wg_cap[1] = 1;
    } else if ((h->p.storage == DDF_F16 || h->p.storage == DDF_BF16) && !has_walls(h->p) &&
               h->p.force_kind == DDF_FORCE_NONE) {
        h->wg_cap[0] = 3;
        h->wg_cap[1] = 2;
        h->idx32 = false;
    }
}
}  // namespace

int ddf_set_address_width(ddf_handle *h, int32_t bits)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (bits != 32 && bits != 64) return fail(DDF_ERR_ARG, "address width must be 32 or 64");
    if (bits == 32 && !plane_fits_32(h))
        return fail(DDF_ERR_ARG, "a population plane of this lattice is 4 GiB or larger: 64-bit offsets only");
    if (h->captured_steps) DDF_HIP_TRY(hipDeviceSynchronize());   // a replay may still be running
    drop_graph(h);
    h->idx32 = bits == 32;
    return DDF_OK;
}

int32_t ddf_get_address_width(const ddf_handle *h) { return !h ? 0 : (h->idx32 ? 32 : 64); }

int ddf_set_workgroups_per_cu(ddf_handle *h, int32_t even, int32_t odd)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    for (int c : {even, odd})
        if (c < 0 || c > 3) return fail(DDF_ERR_ARG, "workgroups per CU must be 0 (no limit), 1, 2 or 3");
    if (h->captured_steps) DDF_HIP_TRY(hipDeviceSynchronize());   // a replay may still be running
    drop_graph(h);
    h->wg_cap[0] = even;
    h->wg_cap[1] = odd;
    return DDF_OK;
}

int ddf_get_workgroups_per_cu(const ddf_handle *h, int32_t *even, int32_t *odd)
{
    if (!h || !even || !odd) return fail(DDF_ERR_ARG, "NULL argument");
    *even = h->wg_cap[0];
    *odd = h->wg_cap[1];
    return DDF_OK;
}

int ddf_create(const ddf_params *p, void *pop_f, void *pop_g, void *workspace, ddf_handle **out)
{
    int rc = validate(p);
    if (rc != DDF_OK) return rc;
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (!pop_f || !pop_g || !workspace) return fail(DDF_ERR_ARG, "a device buffer is NULL");
    if (((uintptr_t)pop_f | (uintptr_t)pop_g | (uintptr_t)workspace) & 255)
        return fail(DDF_ERR_ARG, "device buffers must be 256-byte aligned");
    // Row layout: x-interleaved rows where the width allows them and the lattice streams
    // from HBM (AUTO), or as requested.
    int qs = interleave_shift(*p);
    if (p->layout == DDF_LAYOUT_INTERLEAVED && qs == 0)
        return fail(DDF_ERR_UNSUPPORTED, "x-interleaved rows need nx = 64 * 2^k with nx / 64 >= one 128-byte line "
                                         "of the storage type");
    if (p->layout == DDF_LAYOUT_ROW || p->layout == DDF_LAYOUT_PACKED ||
        (p->layout == DDF_LAYOUT_AUTO && 2 * population_bytes(p) <= (size_t)256 << 20))
        qs = 0;
    ddf_handle *h = new (std::nothrow) ddf_handle;
    if (!h) return fail(DDF_ERR_ARG, "out of host memory");
    h->p = *p;
    h->f = pop_f;
    h->g = pop_g;
    h->ws = workspace;
    // Lattices held by the 256 MB Infinity Cache step fastest with 512-wide tiles (1024^2
    // cavities: up to 3.9% against the HBM-streaming defaults below; never slower).
    h->tile_width = 2 * population_bytes(p) <= (size_t)256 << 20 ? 512 : default_tile_width(p->storage);
    h->G = make_geom(*p, h->tile_width);
    h->G.L.qs = qs;
    h->nblocks = grid_blocks(h->G);
    launch_defaults(h);
    h->step = 0;
    h->snap_step = 0;
    h->snap_valid = false;
    h->initialised = false;
    h->P.d = make_phys<double>(*p);
    h->P.f = make_phys<float>(*p);
    h->captured_steps = 0;
    h->graph_steps = graph_capable(*p) ? 100 : 0;
    h->cap_stream = nullptr;   // created at the first capture
    *out = h;
    return DDF_OK;
}

void ddf_destroy(ddf_handle *h)
{
    if (!h) return;
    if (h->captured_steps) (void)hipDeviceSynchronize();   // a replay may still be running
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
}

int ddf_set_graph(ddf_handle *h, int32_t steps_per_graph)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (steps_per_graph < 0 || (steps_per_graph & 1)) return fail(DDF_ERR_ARG, "steps_per_graph must be even and >= 0");
    if (steps_per_graph > 0 && !graph_capable(h->p))
        return fail(DDF_ERR_UNSUPPORTED, "time-dependent forces and stochastic rounding step eagerly (no graph capture)");
    if (h->captured_steps) DDF_HIP_TRY(hipDeviceSynchronize());
    drop_graph(h);
    h->graph_steps = steps_per_graph;
    return DDF_OK;
}

int32_t ddf_get_tile_width(const ddf_handle *h) { return h ? h->tile_width : 0; }

int32_t ddf_get_layout(const ddf_handle *h)
{
    if (!h) return 0;
    if (h->G.L.qs) return DDF_LAYOUT_INTERLEAVED;
    return h->p.layout == DDF_LAYOUT_PACKED ? DDF_LAYOUT_PACKED : DDF_LAYOUT_ROW;
}

int64_t ddf_step_count(const ddf_handle *h) { return h ? h->step : -1; }

const char *ddf_last_error(void) { return error_slot().c_str(); }

int ddf_init_equilibrium(ddf_handle *h, const double *rho, const double *ux, const double *uy, const double *phi,
                         void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!rho || !ux || !uy || !phi) return fail(DDF_ERR_ARG, "a field pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL((k_init<S>), dim3(h->nblocks), dim3(kThreads), 0, st, (S *)h->f, (S *)h->g, h->G,
                           h->P.of<S>(), rho, ux, uy, phi);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    h->step = 0;
    h->snap_valid = false;
    h->initialised = true;
    return DDF_OK;
}

int ddf_step(ddf_handle *h, int64_t nsteps, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (nsteps < 0) return fail(DDF_ERR_ARG, "nsteps < 0");
    if (!h->initialised) return fail(DDF_ERR_STATE, "step before init or set_populations");
    hipStream_t st = (hipStream_t)stream;
    int64_t left = nsteps;
    if (h->graph_steps > 0 && left >= h->graph_steps + (h->step & 1)) {
        if (h->step & 1) {   // replays start at an even step
            launch_one(h, st, h->step);
            h->step++;
            left--;
        }
        if (h->captured_steps != h->graph_steps) {
            int rc = capture_graph(h);
            if (rc != DDF_OK) return rc;
        }
        while (left >= h->graph_steps) {
            DDF_HIP_TRY(hipGraphLaunch(h->graph_exec, st));
            h->step += h->graph_steps;
            left -= h->graph_steps;
        }
    }
    for (; left > 0; --left) {
        launch_one(h, st, h->step);
        h->step++;
    }
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_extract(ddf_handle *h, void *out, uint32_t mask, int32_t out_dtype, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (out_dtype != 0 && out_dtype != 1) return fail(DDF_ERR_ARG, "out_dtype must be 0 (double) or 1 (float)");
    if (!h->initialised) return fail(DDF_ERR_STATE, "extract before init or set_populations");
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        launch_extract<S>(h->G, h->P.of<S>(), has_walls(h->p), (h->step & 1) != 0, h->f, h->g, h->step,
                          h->p.scalar_model, out, out_dtype, mask, (hipStream_t)stream);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_reduce(ddf_handle *h, double *out, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (!h->initialised) return fail(DDF_ERR_STATE, "reduce before init or set_populations");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)h->ws;
    void *snap = ws;
    double *partials = (double *)(ws + snap_bytes(&h->p));
    double *fin = (double *)((char *)partials + align256((size_t)h->nblocks * RS_N * sizeof(double)));
    const bool odd = (h->step & 1) != 0, w = has_walls(h->p);
    const int sv = h->snap_valid ? 1 : 0;
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        using R = typename Codec<S>::R;
#define DDF_REDUCE(W_, O_)                                                                                       \
    hipLaunchKernelGGL((k_reduce<S, W_, O_>), dim3(h->nblocks), dim3(kThreads), 0, st, (const S *)h->f,        \
                       (const S *)h->g, h->G, h->P.of<S>(), h->step, (R *)snap, sv, partials)
        if (w) { if (odd) DDF_REDUCE(true, true); else DDF_REDUCE(true, false); }
        else { if (odd) DDF_REDUCE(false, true); else DDF_REDUCE(false, false); }
#undef DDF_REDUCE
        return 0;
    });
    hipLaunchKernelGGL(k_reduce_rows<256>, dim3(1), dim3(256), 0, st, partials, (const int *)nullptr, (const int *)nullptr,
                       h->nblocks, fin);
    DDF_HIP_TRY(hipGetLastError());
    double r[RS_N];
    DDF_HIP_TRY(hipMemcpyAsync(r, fin, sizeof(r), hipMemcpyDeviceToHost, st));
    DDF_HIP_TRY(hipStreamSynchronize(st));
    const double K = (double)(h->step - h->snap_step);
    out[DDF_STAT_MASS] = r[RS_MASS];
    out[DDF_STAT_SCALAR] = r[RS_SCALAR];
    out[DDF_STAT_RES_U] = (h->snap_valid && K > 0) ? std::sqrt(r[RS_DU2]) / (K * std::sqrt(r[RS_U2])) : NAN;
    out[DDF_STAT_RES_PHI] = (h->snap_valid && K > 0) ? std::sqrt(r[RS_DPHI2]) / (K * std::sqrt(r[RS_PHI2])) : NAN;
    out[DDF_STAT_NONFINITE] = r[RS_NONFIN];
    out[DDF_STAT_STEPS] = h->snap_valid ? K : 0.0;
    out[DDF_STAT_UMAX] = r[RS_UMAX];
    out[DDF_STAT_PHIMIN] = r[RS_PHIMIN];
    h->snap_valid = true;
    h->snap_step = h->step;
    if (r[RS_NONFIN] > 0.0) return fail(DDF_ERR_NONFINITE, "state holds non-finite values");
    return DDF_OK;
}

int ddf_get_populations(ddf_handle *h, void *f, void *g, int32_t dtype, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!f || !g) return fail(DDF_ERR_ARG, "output pointer is NULL");
    if (dtype != 0 && dtype != 1) return fail(DDF_ERR_ARG, "dtype must be 0 (double) or 1 (raw)");
    if (!h->initialised) return fail(DDF_ERR_STATE, "get_populations before init or set_populations");
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        launch_get<S>(h->G, h->P.of<S>(), has_walls(h->p), (h->step & 1) != 0, h->f, h->g, f, g, dtype,
                      (hipStream_t)stream);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_set_populations(ddf_handle *h, const void *f, const void *g, int32_t dtype, int64_t step, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!f || !g) return fail(DDF_ERR_ARG, "input pointer is NULL");
    if (dtype != 0 && dtype != 1) return fail(DDF_ERR_ARG, "dtype must be 0 (double) or 1 (raw)");
    if (step < 0) return fail(DDF_ERR_ARG, "step < 0");
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        launch_set<S>(h->G, h->P.of<S>(), has_walls(h->p), (step & 1) != 0, h->f, h->g, f, g, dtype,
                      (hipStream_t)stream);
        return 0;
    });
    DDF_HIP_TRY(hipGetLastError());
    h->step = step;
    h->snap_valid = false;
    h->initialised = true;
    return DDF_OK;
}

}  // extern "C"
