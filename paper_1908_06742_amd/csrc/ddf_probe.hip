// libddf HBM reference kernels (include/ddf_probe.h): a copy, a read-only and a
// write-only pass over a buffer, and the step's own access pattern without its
// arithmetic: the ceilings the bandwidth-bound step kernels are measured against.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ddf.h"
#include "../../include/ddf_probe.h"
#include "ddf_handle.hpp"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;

template <bool NT>
__device__ __forceinline__ f4 ld(const f4 *p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <bool NT>
__device__ __forceinline__ void st(f4 *p, f4 v)
{
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Workgroup b covers vectors [b * 256 U, (b + 1) * 256 U); thread t moves vectors
// b * 256 U + k * 256 + t for k < U, so every load and store instruction of a wavefront
// covers 1 KiB of consecutive bytes.  All loads of a thread are issued before its
// stores (copy) or before the reduction that keeps them alive (read).
template <int KIND, int U, bool NT>
__global__ __launch_bounds__(kProbeThreads) void k_probe(const f4 *__restrict__ src, f4 *__restrict__ dst,
                                                         const int64_t n4, const int keep)
{
    const int64_t base = (int64_t)blockIdx.x * (kProbeThreads * U) + threadIdx.x;
    if (KIND == DDF_PROBE_WRITE) {
        const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = base + (int64_t)k * kProbeThreads;
            if (i < n4) st<NT>(dst + i, z);
        }
        return;
    }
    f4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int64_t i = base + (int64_t)k * kProbeThreads;
        if (i < n4) v[k] = ld<NT>(src + i);
        else v[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    if (KIND == DDF_PROBE_COPY) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = base + (int64_t)k * kProbeThreads;
            if (i < n4) st<NT>(dst + i, v[k]);
        }
    } else {
        // the sum keeps the loads; the host passes keep = 0, so nothing is stored
        f4 acc = v[0];
#pragma unroll
        for (int k = 1; k < U; ++k) acc += v[k];
        if (keep) dst[base] = acc;
    }
}

template <int KIND, int U>
void launch_probe(bool nt, const void *src, void *dst, int64_t n4, hipStream_t st)
{
    const int64_t per = (int64_t)kProbeThreads * U;
    const dim3 grid((unsigned)((n4 + per - 1) / per));
    if (nt)
        hipLaunchKernelGGL((k_probe<KIND, U, true>), grid, dim3(kProbeThreads), 0, st, (const f4 *)src, (f4 *)dst, n4, 0);
    else
        hipLaunchKernelGGL((k_probe<KIND, U, false>), grid, dim3(kProbeThreads), 0, st, (const f4 *)src, (f4 *)dst, n4, 0);
}

template <int KIND>
void launch_kind(int unroll, bool nt, const void *src, void *dst, int64_t n4, hipStream_t st)
{
    switch (unroll) {
    case 1: launch_probe<KIND, 1>(nt, src, dst, n4, st); break;
    case 2: launch_probe<KIND, 2>(nt, src, dst, n4, st); break;
    case 4: launch_probe<KIND, 4>(nt, src, dst, n4, st); break;
    default: launch_probe<KIND, 8>(nt, src, dst, n4, st); break;
    }
}

// A stored population with its sign bit flipped (every storage format keeps the sign in
// its top bit): the probe stores values that differ from what it loaded, so no load or
// store can be dropped as a copy of a slot onto itself (the rest direction's would be).
__device__ __forceinline__ float flip_sign(float v) { return __uint_as_float(__float_as_uint(v) ^ 0x80000000u); }
__device__ __forceinline__ double flip_sign(double v)
{
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)0x8000000000000000ull);
}
__device__ __forceinline__ _Float16 flip_sign(_Float16 v) { return -v; }
__device__ __forceinline__ ddf::bf16 flip_sign(ddf::bf16 v) { return ddf::bf16{(uint16_t)(v.bits ^ 0x8000u)}; }
__device__ __forceinline__ ddf::bf16sr flip_sign(ddf::bf16sr v) { return ddf::bf16sr{(uint16_t)(v.bits ^ 0x8000u)}; }

// The step's memory accesses with the collision left out: every thread loads the nine
// stored populations of both lattices that the step of this parity loads for its node
// and stores each, sign flipped, where the step stores the population of the opposite
// direction, which is the slot the step loaded as that direction (the same tiles,
// tile-to-XCD map, lane offsets and non-temporal policy as the periodic step kernels).
// Within a node's slot set this swaps the pairs of opposite directions and negates
// them, so two launches of one parity restore the populations bit for bit.  Walls keep
// that form: a link that the step reflects is loaded from, and stored to, the node's
// own slots, exactly as the step does.
template <class S, bool WALLS, bool ODD, bool IDX32, int LY>
__global__ __launch_bounds__(ddf::kThreads) void k_pattern(S *__restrict__ f, S *__restrict__ g, const ddf::Geom G)
{
    using namespace ddf;
    constexpr bool NT = LY == LY_IL;
    const int tile = tile_of_block();
    if (tile >= G.ntiles) return;
    int m, y;
    if (!tile_node(tile, G.bx_shift, G.by, G.tiles_x, G.L.nx, G.L.ny, m, y)) return;
    const int x = x_of<LY>(G.L, m);
    int pa[9];
    int64_t c[9];
    S vf[9], vg[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        c[a] = logical_cell<WALLS, ODD, LY>(G.L, x, y, a, pa[a]);
        vf[a] = ld_pop<NT>(&elem<IDX32>(f, G.L, pa[a], c[a]));
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) vg[a] = ld_pop<NT>(&elem<IDX32>(g, G.L, pa[a], c[a]));
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        st_pop<NT>(&elem<IDX32>(f, G.L, pa[opp(a)], c[opp(a)]), flip_sign(vf[a]));
        st_pop<NT>(&elem<IDX32>(g, G.L, pa[opp(a)], c[opp(a)]), flip_sign(vg[a]));
    }
}

template <class S, bool WALLS, bool ODD, bool IDX32>
void launch_pattern(const ddf_handle *h, int lds, hipStream_t st)
{
    using namespace ddf;
    if (h->G.L.qs)
        hipLaunchKernelGGL((k_pattern<S, WALLS, ODD, IDX32, LY_IL>), dim3(h->nblocks), dim3(kThreads), lds, st,
                           (S *)h->f, (S *)h->g, h->G);
    else
        hipLaunchKernelGGL((k_pattern<S, WALLS, ODD, IDX32, LY_ROW>), dim3(h->nblocks), dim3(kThreads), lds, st,
                           (S *)h->f, (S *)h->g, h->G);
}

template <class S, bool WALLS>
void launch_pattern_parity(const ddf_handle *h, bool odd, int lds, hipStream_t st)
{
    if (odd) {
        if (h->idx32) launch_pattern<S, WALLS, true, true>(h, lds, st);
        else launch_pattern<S, WALLS, true, false>(h, lds, st);
    } else {
        if (h->idx32) launch_pattern<S, WALLS, false, true>(h, lds, st);
        else launch_pattern<S, WALLS, false, false>(h, lds, st);
    }
}

}  // namespace

extern "C" int ddf_bandwidth_probe(int32_t kind, int32_t unroll, int32_t nontemporal, const void *src, void *dst,
                                   size_t bytes, void *stream)
{
    using ddf::host::fail;
    if (kind != DDF_PROBE_COPY && kind != DDF_PROBE_READ && kind != DDF_PROBE_WRITE)
        return fail(DDF_ERR_ARG, "probe: kind must be DDF_PROBE_COPY, DDF_PROBE_READ or DDF_PROBE_WRITE");
    if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8)
        return fail(DDF_ERR_ARG, "probe: unroll must be 1, 2, 4 or 8");
    if (bytes == 0 || bytes % 16) return fail(DDF_ERR_ARG, "probe: bytes must be a positive multiple of 16");
    if (kind != DDF_PROBE_WRITE && !src) return fail(DDF_ERR_ARG, "probe: src is NULL");
    if (kind != DDF_PROBE_READ && !dst) return fail(DDF_ERR_ARG, "probe: dst is NULL");
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(DDF_ERR_ARG, "probe: buffers must be 16-byte aligned");
    const int64_t n4 = (int64_t)(bytes / 16);
    if (n4 / (kProbeThreads * unroll) >= ((int64_t)1 << 31)) return fail(DDF_ERR_ARG, "probe: buffer too large");
    if (kind == DDF_PROBE_COPY && src && dst) {
        const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
        if (a < b + bytes && b < a + bytes) return fail(DDF_ERR_ARG, "probe: src and dst overlap");
    }
    hipStream_t st = (hipStream_t)stream;
    const bool nt = nontemporal != 0;
    if (kind == DDF_PROBE_COPY) launch_kind<DDF_PROBE_COPY>(unroll, nt, src, dst, n4, st);
    else if (kind == DDF_PROBE_READ) launch_kind<DDF_PROBE_READ>(unroll, nt, src, dst, n4, st);
    else launch_kind<DDF_PROBE_WRITE>(unroll, nt, src, dst, n4, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DDF_ERR_HIP, std::string("probe launch: ") + hipGetErrorString(e));
    return DDF_OK;
}

extern "C" int ddf_pattern_probe(ddf_handle *h, int32_t parity, int32_t wg_per_cu, void *stream)
{
    using ddf::host::fail;
    if (!h) return fail(DDF_ERR_ARG, "pattern probe: handle is NULL");
    if (parity != 0 && parity != 1) return fail(DDF_ERR_ARG, "pattern probe: parity must be 0 (even) or 1 (odd)");
    if (wg_per_cu < 0 || wg_per_cu > 3)
        return fail(DDF_ERR_ARG, "pattern probe: workgroups per CU must be 0 (no limit), 1, 2 or 3");
    const int lds = ddf::host::cap_lds_bytes(wg_per_cu);
    hipStream_t st = (hipStream_t)stream;
    ddf::host::with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        if (ddf::host::has_walls(h->p)) launch_pattern_parity<S, true>(h, parity != 0, lds, st);
        else launch_pattern_parity<S, false>(h, parity != 0, lds, st);
        return 0;
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DDF_ERR_HIP, std::string("pattern probe launch: ") + hipGetErrorString(e));
    return DDF_OK;
}
