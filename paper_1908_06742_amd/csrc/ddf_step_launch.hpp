// Step-kernel launchers of a single lattice for one row layout: dispatch on storage,
// scalar model, walls, body force, parity and lane-offset width.
#pragma once

#include "ddf_handle.hpp"

namespace ddf {
namespace host {

template <class S, int SC, bool W, bool FO, bool I32, int LY>
void launch_step_kernel(ddf_handle *h, hipStream_t st, bool odd, int64_t t)
{
    const auto &P = h->P.of<S>();
    const int lds = cap_lds_bytes(h->wg_cap[odd ? 1 : 0]);
    if (odd)
        hipLaunchKernelGGL((k_step<S, SC, W, FO, true, I32, LY>), dim3(h->nblocks), dim3(kThreads), lds, st, (S *)h->f,
                           (S *)h->g, h->G, P, t);
    else
        hipLaunchKernelGGL((k_step<S, SC, W, FO, false, I32, LY>), dim3(h->nblocks), dim3(kThreads), lds, st, (S *)h->f,
                           (S *)h->g, h->G, P, t);
}

template <class S, int SC, bool W, bool FO, int LY>
void launch_step_parity(ddf_handle *h, hipStream_t st, bool odd, int64_t t)
{
    if (h->idx32) launch_step_kernel<S, SC, W, FO, true, LY>(h, st, odd, t);
    else launch_step_kernel<S, SC, W, FO, false, LY>(h, st, odd, t);
}

template <class S, int SC, int LY>
void launch_step(ddf_handle *h, hipStream_t st, int64_t t)
{
    const bool odd = (t & 1) != 0;
    const bool w = has_walls(h->p);
    const bool fo = h->p.force_kind != DDF_FORCE_NONE;
    if (w) {
        if (fo) launch_step_parity<S, SC, true, true, LY>(h, st, odd, t);
        else launch_step_parity<S, SC, true, false, LY>(h, st, odd, t);
    } else {
        if (fo) launch_step_parity<S, SC, false, true, LY>(h, st, odd, t);
        else launch_step_parity<S, SC, false, false, LY>(h, st, odd, t);
    }
}

template <int LY>
void launch_step_layout(ddf_handle *h, hipStream_t st, int64_t t)
{
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        switch (h->p.scalar_model) {
        case DDF_SCALAR_SRT: launch_step<S, DDF_SCALAR_SRT, LY>(h, st, t); break;
        case DDF_SCALAR_CASCADED:
        case DDF_SCALAR_CENTRAL: launch_step<S, DDF_SCALAR_CENTRAL, LY>(h, st, t); break;
        default: launch_step<S, DDF_SCALAR_MRT, LY>(h, st, t);
        }
        return 0;
    });
}

}  // namespace host
}  // namespace ddf
