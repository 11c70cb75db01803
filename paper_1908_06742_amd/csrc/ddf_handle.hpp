// State of one single-lattice handle of libddf and the step launchers shared by the
// translation units that instantiate the step kernels (one per row layout, compiled in
// parallel).
#pragma once

#include "ddf_kernels.hpp"

struct ddf_handle {
    ddf_params p;
    void *f, *g, *ws;
    ddf::Geom G;           // G.L.qs: x-interleaved rows (0 = row-major), fixed at create
    int tile_width;
    int nblocks;
    bool idx32;            // step kernels with 32-bit lane offsets (planes below 4 GiB)
    int wg_cap[2];         // resident step workgroups per CU, even / odd step (0 = no limit)
    int64_t step;
    int64_t snap_step;
    bool snap_valid;
    bool initialised;
    ddf::host::PhysPair P;
    // runs of graph_steps steps are captured once into a hipGraph on cap_stream and
    // replayed on the caller's stream
    hipStream_t cap_stream;
    hipGraphExec_t graph_exec;
    int graph_steps;       // even; 0 = always launch eagerly
    int captured_steps;    // steps of the instantiated graph, 0 = none
};

namespace ddf {
namespace host {

// Dynamic LDS that limits a 512-thread workgroup of a kernel using no LDS to `cap`
// resident workgroups per CU (0: no limit).  The CU's LDS size is read once.
inline int cap_lds_bytes(int cap)
{
    static const int lds_cu = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
            v = 0;
        return v;
    }();
    if (cap <= 0 || lds_cu <= 0) return 0;
    return (lds_cu / (cap + 1) + 512) / 512 * 512;   // cap of them fit, cap + 1 do not
}

// One step of time index t (its parity selects the streaming direction) with the
// kernels of row layout LY (instantiated in ddf_step_row.hip and ddf_step_il.hip).
template <int LY>
void launch_step_layout(ddf_handle *h, hipStream_t st, int64_t t);

inline void launch_one(ddf_handle *h, hipStream_t st, int64_t t)
{
    if (h->G.L.qs) launch_step_layout<LY_IL>(h, st, t);
    else launch_step_layout<LY_ROW>(h, st, t);
}

}  // namespace host
}  // namespace ddf
