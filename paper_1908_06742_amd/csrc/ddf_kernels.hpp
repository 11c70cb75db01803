// Lattice geometry, AA-pattern addressing, the fused node update and the lattice
// kernels shared by the single-lattice and batched entry points of libddf.
//
// Data layout in HBM: each lattice is 9 planes (one per direction), each plane ny rows
// of `pitch` elements (pitch = nx rounded up to 64), so a wavefront reads or writes 64
// consecutive nodes of one direction: 256 B (FP32), 512 B (FP64), 128 B (FP16/BF16).
// Planes follow one another with no gap: a gap of 256 KiB + 256 B between large planes
// (so that the 18 streams a node touches do not start at the same offset of the HBM
// channel interleave) helped row-major rows by 2%, but with x-interleaved rows and
// non-temporal accesses the step ran faster without it (8192^2: FP32 2.7%, FP64 10%).
//
// Packed rows (the batch's layout) drop the row padding: pitch = nx, and each plane is
// rounded up to 64 elements so that every plane starts on a 128-byte line.  Flat tiles
// of consecutive nodes then read and write whole aligned lines in the even step, and
// no row ends inside a partly used line (a 256-instance batch of random widths: 5.3
// against 4.8 TB/s for padded rows).
//
// Large lattices whose width is 64 * 2^k (k >= 5 for 4-byte storage) may instead keep
// each row x-interleaved: memory column m of a row holds node x = (m mod Q) * 64 + m / Q
// with Q = nx / 64, i.e. the row is 64 sub-rows of Q nodes, 64 apart in x.  A wavefront
// then handles 64 nodes that are consecutive in memory and 64 apart in x, so their
// x +- 1 neighbours sit at the same lanes of the adjacent sub-row: every population
// access of both parities is a whole, aligned 128-byte line group, except at the
// sub-row wrap (one sub-row pair in 64).  With aligned accesses the step kernels also
// mark their loads and stores non-temporal (measured on the 8192^2 FP32 field: 6.0 TB/s
// against 5.6 TB/s for the row-major step).
//
// Streaming is the in-place AA pattern: an even step reads a node's own slots and
// writes its post-collision populations into the opposite slots of the same node; an
// odd step reads the slots its neighbours wrote and pushes its results into their
// natural slots.  Each step therefore reads and writes every population exactly once
// (36 s bytes per node-update for storage size s) with no second array.  Half-way walls
// are applied when the populations are written, in both parities, so that the reflected
// value (with the moving-wall or Dirichlet term of the node's own state) sits where the
// next step reads it.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

#include "../../include/ddf.h"
#include "ddf_device.hpp"

namespace ddf {

// Workgroup size of the lattice kernels (512 measured 1.5% faster than 256 on 8192^2).
constexpr int kThreads = 512;

// Geometry of one lattice.
struct Lat {
    int nx, ny;
    int pitch;          // elements per row
    int64_t plane;      // elements per direction plane
    int px, py;         // periodic flags
    int qs;             // x-interleaved rows: log2(nx / 64); 0 = row-major
    int kpitch;         // pitch and plane of padded row-major rows: the stochastic-rounding
    int64_t kplane;     // keys name slots by these, so every layout draws the same bits
};

// Row layouts, as template arguments: row-major, x-interleaved, or read from Lat::qs.
enum { LY_ROW = 0, LY_IL = 1, LY_ANY = 2 };

// Memory column of node x in its row, and the node of memory column m.
template <int LY>
__device__ __forceinline__ int col_of(const Lat &L, int x)
{
    if (LY == LY_ROW || (LY == LY_ANY && L.qs == 0)) return x;
    return ((x & 63) << L.qs) | (x >> 6);
}

template <int LY>
__device__ __forceinline__ int x_of(const Lat &L, int m)
{
    if (LY == LY_ROW || (LY == LY_ANY && L.qs == 0)) return m;
    return ((m & ((1 << L.qs) - 1)) << 6) | (m >> L.qs);
}

// One lattice tiled into workgroups of kThreads threads, bx = 1 << bx_shift wide.
struct Geom {
    Lat L;
    int bx_shift;
    int by;
    int tiles_x;
    int ntiles;
};

// Tile of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin by
// blockIdx; the remap gives each XCD one contiguous run of row-major tiles, so the
// neighbouring-row and partial-line traffic of the odd step stays in one L2.
__device__ __forceinline__ int tile_of_block()
{
    const int per = gridDim.x >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ bool tile_node(int tile, int bx_shift, int by, int tiles_x, int nx, int ny, int &x, int &y)
{
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int bx = 1 << bx_shift;
    x = (tx << bx_shift) + (threadIdx.x & (bx - 1));
    y = ty * by + (threadIdx.x >> bx_shift);
    return x < nx && y < ny;
}

// A row's padding slots [nx, pitch) are never read.  Lanes past the end of a row write
// zeros into those up to the end of the row's last 128-byte line, in every direction
// plane of both lattices, so that no line is left partly written: rows whose length is
// not a multiple of 64 nodes otherwise stepped markedly slower than their bytes (a
// 256-instance batch of random widths ran 17% below the same batch with widths
// rounded up).  Needs tiles at least 64 nodes wide (the last tile of a row then covers
// the line's remainder).
template <class S>
__device__ __forceinline__ bool pad_slot(const Lat &L, int x, int y)
{
    constexpr int line = 128 / (int)sizeof(S);
    const int end = min(L.pitch, (L.nx + line - 1) / line * line);
    return x >= L.nx && x < end && y < L.ny;
}

template <class S>
__device__ __forceinline__ void fill_pad(S *__restrict__ f, S *__restrict__ g, const Lat &L, int x, int y)
{
    const int64_t c = (int64_t)y * L.pitch + x;
    const S z{};
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f[a * L.plane + c] = z;
        g[a * L.plane + c] = z;
    }
}

// Node (x, y) of this thread: tiles cover memory columns, so consecutive lanes touch
// consecutive population slots in either row layout.
__device__ __forceinline__ bool node_of_thread(const Geom &G, int &x, int &y)
{
    const int t = tile_of_block();
    if (t >= G.ntiles) return false;
    int m;
    if (!tile_node(t, G.bx_shift, G.by, G.tiles_x, G.L.nx, G.L.ny, m, y)) return false;
    x = x_of<LY_ANY>(G.L, m);
    return true;
}

// Neighbour of (x, y) along (dx, dy) with periodic wrapping; returns the wall side
// crossed (DDF_SIDE_*) or -1 for a fluid node.  A corner link counts against the
// bottom/top wall.
template <bool WALLS>
__device__ __forceinline__ int neighbour(const Lat &L, int x, int y, int dx, int dy, int &tx, int &ty)
{
    tx = x + dx;
    ty = y + dy;
    if (!WALLS) {
        tx = tx < 0 ? tx + L.nx : (tx >= L.nx ? tx - L.nx : tx);
        ty = ty < 0 ? ty + L.ny : (ty >= L.ny ? ty - L.ny : ty);
        return -1;
    }
    if (L.px) tx = tx < 0 ? tx + L.nx : (tx >= L.nx ? tx - L.nx : tx);
    if (L.py) ty = ty < 0 ? ty + L.ny : (ty >= L.ny ? ty - L.ny : ty);
    if (ty < 0) return DDF_SIDE_BOTTOM;
    if (ty >= L.ny) return DDF_SIDE_TOP;
    if (tx < 0) return DDF_SIDE_LEFT;
    if (tx >= L.nx) return DDF_SIDE_RIGHT;
    return -1;
}

// Storage slot holding the logical pre-collision population a of node (x, y) at a
// step of parity ODD: natural slot after an even number of steps; after an odd number
// the population sits in the opposite slot of its source node, or (for a population
// reflected by a wall) in slot a of the node itself.  Returns the cell and sets the
// plane in *pa.
template <bool WALLS, bool ODD, int LY = LY_ANY>
__device__ __forceinline__ int64_t logical_cell(const Lat &L, int x, int y, int a, int &pa)
{
    const int64_t cell = (int64_t)y * L.pitch + col_of<LY>(L, x);
    pa = a;
    if (!ODD || a == 0) return cell;
    int sx, sy;
    const int w = neighbour<WALLS>(L, x, y, -ex(a), -ey(a), sx, sy);
    if (w >= 0) return cell;
    pa = opp(a);
    return (int64_t)sy * L.pitch + col_of<LY>(L, sx);
}

template <bool WALLS, bool ODD, int LY = LY_ANY>
__device__ __forceinline__ int64_t logical_slot(const Lat &L, int x, int y, int a)
{
    int pa;
    const int64_t cell = logical_cell<WALLS, ODD, LY>(L, x, y, a, pa);
    return (int64_t)pa * L.plane + cell;
}

// The lattice as padded row-major rows (slot indices that name stochastic-rounding keys).
__device__ __forceinline__ Lat key_lat(Lat L)
{
    L.pitch = L.kpitch;
    L.plane = L.kplane;
    L.qs = 0;
    return L;
}

// Element `cell` of direction plane `pa`.  With IDX32 (planes below 4 GiB) the lane's
// part of the address is a 32-bit byte offset from the plane's base; where the plane
// is the same for the whole wavefront (every slot of a periodic lattice) that base
// stays in scalar registers and the hardware adds the offset in its scalar-base
// addressing mode, so an address costs one vector register and one 32-bit
// multiply-add instead of two registers and 64-bit arithmetic.
template <bool IDX32, class S>
__device__ __forceinline__ S &elem(S *__restrict__ base, const Lat &L, int pa, int64_t cell)
{
    S *p = base + (int64_t)pa * L.plane;
    if (IDX32) return *(S *)((char *)p + (uint32_t)cell * (uint32_t)sizeof(S));
    return p[cell];
}

// Loads and stores of stored populations; NT marks them non-temporal (streamed: no
// reuse expected in the caches).
template <bool NT, class S>
__device__ __forceinline__ S ld_pop(const S *p)
{
    if constexpr (!NT) {
        return *p;
    } else if constexpr (std::is_same<S, bf16>::value || std::is_same<S, bf16sr>::value) {
        S r;
        r.bits = __builtin_nontemporal_load(&p->bits);
        return r;
    } else {
        return __builtin_nontemporal_load(p);
    }
}

template <bool NT, class S>
__device__ __forceinline__ void st_pop(S *p, S v)
{
    if constexpr (!NT) {
        *p = v;
    } else if constexpr (std::is_same<S, bf16>::value || std::is_same<S, bf16sr>::value) {
        __builtin_nontemporal_store(v.bits, &p->bits);
    } else {
        __builtin_nontemporal_store(v, p);
    }
}

template <class S, bool WALLS, bool ODD, bool IDX32 = false, int LY = LY_ANY, bool NT = false>
__device__ __forceinline__ void load_logical(const S *__restrict__ f, const Lat &L, int x, int y,
                                             typename Codec<S>::R inv_scale, typename Codec<S>::R v[9], int dc = 0)
{
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int pa;
        const int64_t c = logical_cell<WALLS, ODD, LY>(L, x, y, a, pa) + dc;
        v[a] = Codec<S>::dec(ld_pop<NT>(&elem<IDX32>(f, L, pa, c))) * inv_scale;
    }
}

// A zero the compiler cannot fold, produced only once all of v is available: added to
// later addresses, it holds their loads back until v's loads have returned.
template <class R>
__device__ __forceinline__ int zero_after(const R v[9])
{
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 9; ++a) s += (float)v[a];
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z) : "v"(s));
    return z;
}

// The periodic x-interleaved FP32 odd step issues the scalar lattice's loads only after
// the fluid's have returned: half as many loads in flight per wavefront, which the
// shifted accesses of that step serve faster (8192^2: 1.2% on the odd step; the even
// step and the other storage formats measured level or slower).
template <class S, bool WALLS, bool ODD, int LY>
constexpr bool kLoadsInTwoWaves = ODD && !WALLS && LY == LY_IL && std::is_same<S, float>::value;

// One time step of node (x, y): load both lattices, collide, stream with walls.
template <class S, int SCALAR, bool WALLS, bool FORCE, bool ODD, bool IDX32 = false, int LY = LY_ROW, bool NT = false>
__device__ __forceinline__ void step_node(S *__restrict__ f, S *__restrict__ g, const Lat &L,
                                          const Phys<typename Codec<S>::R> &P, int x, int y, int64_t t)
{
    using R = typename Codec<S>::R;
    R fv[9], gv[9];
    load_logical<S, WALLS, ODD, IDX32, LY, NT>(f, L, x, y, P.inv_scale, fv);
    int gz = 0;
    if constexpr (kLoadsInTwoWaves<S, WALLS, ODD, LY>) gz = zero_after(fv);
    load_logical<S, WALLS, ODD, IDX32, LY, NT>(g, L, x, y, P.inv_scale, gv, gz);

    R m[9], n[9];
    moments(fv, m);
    moments(gv, n);
    R Fx = (R)0, Fy = (R)0;
    if (FORCE) body_force(P, x, y, t, Fx, Fy);
    const Macro<R> M = macro(P, m, n, Fx, Fy);

    R fo[9], go[9];
    collide_fluid<R, FORCE>(P, M, m, Fx, Fy, fo);
    if (SCALAR == DDF_SCALAR_SRT) collide_scalar_srt(P, M, gv, go);
    else if (SCALAR == DDF_SCALAR_CENTRAL) collide_scalar_central(P, M, gv, go);
    else collide_scalar_mrt(P, M, n, go);

    const int64_t cell = (int64_t)y * L.pitch + col_of<LY>(L, x);
    // stochastic-rounding bits (codecs that round to nearest ignore them): keyed by the
    // step, the node and the direction, which every step writes exactly once each; the
    // key names the node by its coordinates, so both row layouts store the same bits
    const uint32_t salt = sr_step_salt(t);
    const int64_t key = 9 * ((int64_t)y * L.kpitch + x);
    // rest direction: same slot in both parities
    {
        const uint32_t h = sr_bits(key, salt);
        st_pop<NT>(&elem<IDX32>(f, L, 0, cell), Codec<S>::enc(fo[0] * P.scale, h));
        st_pop<NT>(&elem<IDX32>(g, L, 0, cell), Codec<S>::enc(go[0] * P.scale, h >> 16));
    }
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        int tx, ty;
        const int w = neighbour<WALLS>(L, x, y, ex(a), ey(a), tx, ty);
        R vf = fo[a], vg = go[a];
        int pa = opp(a);
        int64_t c = cell;
        if (WALLS && w >= 0) {
            // half-way bounce-back (with the moving-wall term) and anti-bounce-back
            // (Dirichlet scalar) land on the node itself, direction opp(a)
            vf = vf - M.rho * P.wall_f[w][a];
            if (P.wall_dirichlet[w]) vg = -vg + P.wall_g[w][a];
        } else if (ODD) {
            pa = a;
            c = (int64_t)ty * L.pitch + col_of<LY>(L, tx);
        }
        const uint32_t h = sr_bits(key + a, salt);
        st_pop<NT>(&elem<IDX32>(f, L, pa, c), Codec<S>::enc(vf * P.scale, h));
        st_pop<NT>(&elem<IDX32>(g, L, pa, c), Codec<S>::enc(vg * P.scale, h >> 16));
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// The fused step over one lattice.  LY_IL (x-interleaved rows, which have no padding)
// always runs with non-temporal loads and stores; LY_ROW never does.
template <class S, int SCALAR, bool WALLS, bool FORCE, bool ODD, bool IDX32, int LY>
__global__ __launch_bounds__(kThreads) void k_step(S *__restrict__ f, S *__restrict__ g, const Geom G,
                                                   const Phys<typename Codec<S>::R> P, const int64_t t)
{
    const int tile = tile_of_block();
    if (tile >= G.ntiles) return;
    int m, y;
    if (tile_node(tile, G.bx_shift, G.by, G.tiles_x, G.L.nx, G.L.ny, m, y))
        step_node<S, SCALAR, WALLS, FORCE, ODD, IDX32, LY, LY == LY_IL>(f, g, G.L, P, x_of<LY>(G.L, m), y, t);
    else if (LY == LY_ROW && G.bx_shift >= 6 && pad_slot<S>(G.L, m, y))
        fill_pad(f, g, G.L, m, y);
}

template <class S, bool WALLS, bool ODD, class O>
__global__ __launch_bounds__(kThreads) void k_extract(const S *__restrict__ f, const S *__restrict__ g, const Geom G,
                                                      const Phys<typename Codec<S>::R> P, const int64_t t,
                                                      const int scalar_model, O *__restrict__ out, const uint32_t mask)
{
    using R = typename Codec<S>::R;
    int x, y;
    if (!node_of_thread(G, x, y)) return;
    R fv[9], gv[9], m[9], n[9];
    load_logical<S, WALLS, ODD>(f, G.L, x, y, P.inv_scale, fv);
    load_logical<S, WALLS, ODD>(g, G.L, x, y, P.inv_scale, gv);
    moments(fv, m);
    moments(gv, n);
    R Fx = (R)0, Fy = (R)0;
    body_force(P, x, y, t, Fx, Fy);
    const Macro<R> M = macro(P, m, n, Fx, Fy);
    const Kin<R> K = kinematics(P, M, m, n, Fx, Fy, scalar_model);
    const R vals[DDF_NUM_OUTPUTS] = {M.rho, M.ux, M.uy, M.phi, K.Sxx, K.Syy, K.Sxy, K.wz,
                                     K.dxuy, K.dyux, K.dxphi, K.dyphi, K.Q, K.Rinv, K.Lx, K.Ly};
    const int64_t N = (int64_t)G.L.nx * G.L.ny;
    const int64_t c = (int64_t)y * G.L.nx + x;
#pragma unroll
    for (int k = 0; k < DDF_NUM_OUTPUTS; ++k)
        if (mask & (1u << k)) out[(int64_t)k * N + c] = (O)vals[k];
}

// Extraction over x-interleaved rows.  A workgroup takes 64 K consecutive nodes of one
// row (K = 2^KS = 32, or 16 for rows of 1024 nodes): memory columns k0 .. k0 + K - 1 of
// all 64 sub-rows, K / 8 nodes per thread, so each wavefront's population loads are runs
// of K consecutive slots (whole 128-byte lines in FP32).  The outputs are staged through
// LDS, four planes at a time, and stored in x order in runs of 64 K nodes.
template <class S, bool WALLS, bool ODD, class O, int KS>
__global__ __launch_bounds__(kThreads) void k_extract_il(const S *__restrict__ f, const S *__restrict__ g, const Lat L,
                                                         const Phys<typename Codec<S>::R> P, const int64_t t,
                                                         const int scalar_model, O *__restrict__ out, const uint32_t mask)
{
    using R = typename Codec<S>::R;
    constexpr int K = 1 << KS, NODES = 64 * K, NPT = NODES / kThreads;
    __shared__ O st[4][NODES];
    const int per_row = L.nx / NODES;
    const int y = blockIdx.x / per_row;
    const int X0 = (blockIdx.x - y * per_row) * NODES;
    O vals[NPT][DDF_NUM_OUTPUTS];
    int xl[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int i = j * kThreads + (int)threadIdx.x;
        const int sr = i >> KS, kk = i & (K - 1);   // sub-row, column within the run
        xl[j] = (kk << 6) + sr;                      // node x - X0
        const int x = X0 + xl[j];
        R fv[9], gv[9], m[9], n[9];
        load_logical<S, WALLS, ODD, false, LY_IL>(f, L, x, y, P.inv_scale, fv);
        load_logical<S, WALLS, ODD, false, LY_IL>(g, L, x, y, P.inv_scale, gv);
        moments(fv, m);
        moments(gv, n);
        R Fx = (R)0, Fy = (R)0;
        body_force(P, x, y, t, Fx, Fy);
        const Macro<R> M = macro(P, m, n, Fx, Fy);
        const Kin<R> Kn = kinematics(P, M, m, n, Fx, Fy, scalar_model);
        const R v[DDF_NUM_OUTPUTS] = {M.rho, M.ux, M.uy, M.phi, Kn.Sxx, Kn.Syy, Kn.Sxy, Kn.wz,
                                      Kn.dxuy, Kn.dyux, Kn.dxphi, Kn.dyphi, Kn.Q, Kn.Rinv, Kn.Lx, Kn.Ly};
#pragma unroll
        for (int k = 0; k < DDF_NUM_OUTPUTS; ++k) vals[j][k] = (O)v[k];
    }
    const int64_t N = (int64_t)L.nx * L.ny;
    const int64_t row = (int64_t)y * L.nx + X0;
#pragma unroll
    for (int grp = 0; grp < DDF_NUM_OUTPUTS / 4; ++grp) {
        if (!((mask >> (4 * grp)) & 15u)) continue;
#pragma unroll
        for (int j = 0; j < NPT; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) st[q][xl[j]] = vals[j][4 * grp + q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * grp + q;
            if (!(mask & (1u << k))) continue;
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int xi = j * kThreads + (int)threadIdx.x;
                out[(int64_t)k * N + row + xi] = st[q][xi];
            }
        }
        __syncthreads();
    }
}

template <class S>
__global__ __launch_bounds__(kThreads) void k_init(S *__restrict__ f, S *__restrict__ g, const Geom G,
                                                   const Phys<typename Codec<S>::R> P, const double *__restrict__ rho,
                                                   const double *__restrict__ ux, const double *__restrict__ uy,
                                                   const double *__restrict__ phi)
{
    using R = typename Codec<S>::R;
    int x, y;
    if (!node_of_thread(G, x, y)) return;
    const int64_t c = (int64_t)y * G.L.nx + x;
    Macro<R> M;
    M.rho = (R)rho[c];
    M.drho = (R)(rho[c] - (double)P.rho0);
    M.ux = (R)ux[c];
    M.uy = (R)uy[c];
    M.phi = (R)phi[c];
    M.dphi = (R)(phi[c] - (double)P.phi0);
    R Fx, Fy, e[9], n[9], fo[9], go[9];
    body_force(P, x, y, 0, Fx, Fy);
    fluid_eq(P, M, e);
    if (P.force_kind != 0) {
        R src[9];
        source(Fx, Fy, M.ux, M.uy, src);
#pragma unroll
        for (int k = 0; k < 9; ++k) e[k] -= (R)0.5 * src[k];
    }
    populations(e, fo);
    scalar_eq(P, M, n);
    populations(n, go);
    const int64_t node = (int64_t)y * G.L.kpitch + x;
    const int64_t cell = (int64_t)y * G.L.pitch + col_of<LY_ANY>(G.L, x);
    const uint32_t salt = sr_step_salt(-1);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int64_t s = (int64_t)a * G.L.plane + cell;
        const uint32_t h = sr_bits((int64_t)a * G.L.kplane + node, salt);   // same bits in every row layout
        f[s] = Codec<S>::enc(fo[a] * P.scale, h);
        g[s] = Codec<S>::enc(go[a] * P.scale, h >> 16);
    }
}

// Per-block FP64 partial sums; fixed tree order, so results are deterministic.
enum { RS_MASS = 0, RS_SCALAR, RS_DU2, RS_U2, RS_DPHI2, RS_PHI2, RS_NONFIN, RS_UMAX, RS_PHIMIN, RS_N };

template <int NT>
__device__ __forceinline__ void block_reduce_stats(double (*sh)[NT], double v[RS_N], double *out)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < RS_N; ++k) sh[k][tid] = v[k];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int k = 0; k < RS_UMAX; ++k) sh[k][tid] += sh[k][tid + s];
            sh[RS_UMAX][tid] = fmax(sh[RS_UMAX][tid], sh[RS_UMAX][tid + s]);
            sh[RS_PHIMIN][tid] = fmin(sh[RS_PHIMIN][tid], sh[RS_PHIMIN][tid + s]);
        }
        __syncthreads();
    }
    if (tid < RS_N) out[tid] = sh[tid][0];
}

// Statistics of node (x, y) into v; updates the residual snapshot.
template <class S, bool WALLS, bool ODD>
__device__ __forceinline__ void node_stats(const S *__restrict__ f, const S *__restrict__ g, const Lat &L,
                                           const Phys<typename Codec<S>::R> &P, int x, int y, int64_t t,
                                           typename Codec<S>::R *__restrict__ snap, int snap_valid, double v[RS_N])
{
    using R = typename Codec<S>::R;
    R fv[9], gv[9], m[9], n[9];
    load_logical<S, WALLS, ODD>(f, L, x, y, P.inv_scale, fv);
    load_logical<S, WALLS, ODD>(g, L, x, y, P.inv_scale, gv);
    moments(fv, m);
    moments(gv, n);
    R Fx = (R)0, Fy = (R)0;
    body_force(P, x, y, t, Fx, Fy);
    const Macro<R> M = macro(P, m, n, Fx, Fy);
    // the residual snapshot is private: kept in the populations' column order
    const int64_t N = (int64_t)L.nx * L.ny;
    const int64_t c = (int64_t)y * L.nx + col_of<LY_ANY>(L, x);
    const double ux = (double)M.ux, uy = (double)M.uy, phi = (double)M.phi;
    v[RS_MASS] = (double)P.rho0 + (double)M.drho;
    v[RS_SCALAR] = (double)P.phi0 + (double)M.dphi;
    v[RS_U2] = ux * ux + uy * uy;
    v[RS_PHI2] = phi * phi;
    if (snap_valid) {
        const double dux = ux - (double)snap[c], duy = uy - (double)snap[N + c], dp = phi - (double)snap[2 * N + c];
        v[RS_DU2] = dux * dux + duy * duy;
        v[RS_DPHI2] = dp * dp;
    }
    const bool fin = isfinite(v[RS_MASS]) && isfinite(ux) && isfinite(uy) && isfinite(phi);
    v[RS_NONFIN] = fin ? 0.0 : 1.0;
    v[RS_UMAX] = fin ? sqrt(v[RS_U2]) : 0.0;
    v[RS_PHIMIN] = fin ? phi : INFINITY;
    snap[c] = M.ux;
    snap[N + c] = M.uy;
    snap[2 * N + c] = M.phi;
}

__device__ __forceinline__ void stats_identity(double v[RS_N])
{
#pragma unroll
    for (int k = 0; k < RS_N; ++k) v[k] = 0.0;
    v[RS_PHIMIN] = INFINITY;
}

template <class S, bool WALLS, bool ODD>
__global__ __launch_bounds__(kThreads) void k_reduce(const S *__restrict__ f, const S *__restrict__ g, const Geom G,
                                                     const Phys<typename Codec<S>::R> P, const int64_t t,
                                                     typename Codec<S>::R *__restrict__ snap, const int snap_valid,
                                                     double *__restrict__ partials)
{
    __shared__ double sh[RS_N][kThreads];
    double v[RS_N];
    stats_identity(v);
    int x, y;
    if (node_of_thread(G, x, y)) node_stats<S, WALLS, ODD>(f, g, G.L, P, x, y, t, snap, snap_valid, v);
    block_reduce_stats<kThreads>(sh, v, partials + (int64_t)blockIdx.x * RS_N);
}

// Sums partials[first .. first + count) (RS_N doubles each) into out[RS_N]; one
// workgroup per output row (blockIdx.x), in a fixed order.
// Without row tables (first == NULL) there is one row of nb_single partials.
template <int NT>
__global__ __launch_bounds__(NT) void k_reduce_rows(const double *__restrict__ partials, const int *__restrict__ first,
                                                     const int *__restrict__ count, const int nb_single,
                                                     double *__restrict__ out)
{
    __shared__ double sh[RS_N][NT];
    const int row = blockIdx.x;
    const int b0 = first ? first[row] : 0;
    const int nb = first ? count[row] : nb_single;
    double v[RS_N];
    stats_identity(v);
    for (int b = threadIdx.x; b < nb; b += NT) {
        const double *p = partials + (int64_t)(b0 + b) * RS_N;
#pragma unroll
        for (int k = 0; k < RS_UMAX; ++k) v[k] += p[k];
        v[RS_UMAX] = fmax(v[RS_UMAX], p[RS_UMAX]);
        v[RS_PHIMIN] = fmin(v[RS_PHIMIN], p[RS_PHIMIN]);
    }
    block_reduce_stats<NT>(sh, v, out + (int64_t)row * RS_N);
}

// dtype 0: absolute FP64 values; dtype 1: raw stored elements.
template <class S, bool WALLS, bool ODD>
__global__ __launch_bounds__(kThreads) void k_get(const S *__restrict__ f, const S *__restrict__ g, const Geom G,
                                                  const Phys<typename Codec<S>::R> P, void *__restrict__ fo,
                                                  void *__restrict__ go, const int dtype)
{
    int x, y;
    if (!node_of_thread(G, x, y)) return;
    const int64_t N = (int64_t)G.L.nx * G.L.ny;
    const int64_t c = (int64_t)y * G.L.nx + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int64_t s = logical_slot<WALLS, ODD>(G.L, x, y, a);
        if (dtype == 0) {
            ((double *)fo)[a * N + c] = (double)Codec<S>::dec(f[s]) * (double)P.inv_scale + (double)P.rest_f[a] * (double)P.rho0;
            ((double *)go)[a * N + c] = (double)Codec<S>::dec(g[s]) * (double)P.inv_scale + (double)P.rest_g[a] * (double)P.phi0;
        } else {
            ((S *)fo)[a * N + c] = f[s];
            ((S *)go)[a * N + c] = g[s];
        }
    }
}

template <class S, bool WALLS, bool ODD>
__global__ __launch_bounds__(kThreads) void k_set(S *__restrict__ f, S *__restrict__ g, const Geom G,
                                                  const Phys<typename Codec<S>::R> P, const void *__restrict__ fi,
                                                  const void *__restrict__ gi, const int dtype)
{
    using R = typename Codec<S>::R;
    int x, y;
    if (!node_of_thread(G, x, y)) return;
    const int64_t N = (int64_t)G.L.nx * G.L.ny;
    const int64_t c = (int64_t)y * G.L.nx + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int64_t s = logical_slot<WALLS, ODD>(G.L, x, y, a);
        if (dtype == 0) {
            const double vf = ((const double *)fi)[a * N + c] - (double)P.rest_f[a] * (double)P.rho0;
            const double vg = ((const double *)gi)[a * N + c] - (double)P.rest_g[a] * (double)P.phi0;
            // keyed by the slot's index in padded row-major rows: the same bits in every layout
            const uint32_t h = sr_bits(logical_slot<WALLS, ODD, LY_ROW>(key_lat(G.L), x, y, a), sr_step_salt(-2));
            f[s] = Codec<S>::enc((R)(vf * (double)P.scale), h);
            g[s] = Codec<S>::enc((R)(vg * (double)P.scale), h >> 16);
        } else {
            f[s] = ((const S *)fi)[a * N + c];
            g[s] = ((const S *)gi)[a * N + c];
        }
    }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
namespace host {

inline std::string &error_slot()
{
    thread_local std::string s;
    return s;
}

inline int fail(int code, const std::string &msg)
{
    error_slot() = msg;
    return code;
}

#define DDF_HIP_TRY(expr)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return ::ddf::host::fail(DDF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_));        \
    } while (0)

// Row pitch in elements: nx rounded up to 64 (row-major and x-interleaved rows), or nx
// itself for packed rows.
inline int64_t row_pitch(int nx) { return ((int64_t)nx + 63) / 64 * 64; }
inline int64_t pitch_of(const ddf_params *p) { return p->layout == DDF_LAYOUT_PACKED ? p->nx : row_pitch(p->nx); }

inline size_t storage_size(int storage) { return storage == DDF_F64 ? 8 : (storage == DDF_F32 ? 4 : 2); }

// Single-lattice tile width by storage size (measured on the 8192^2 field: 128-wide
// tiles for 8- and 4-byte storage, 64-wide for 2-byte storage).
inline int default_tile_width(int storage) { return storage_size(storage) == 2 ? 64 : 128; }

// Elements per direction plane: pitch * ny rounded up to 64.
inline int64_t plane_with(const ddf_params *p, int64_t pitch) { return (pitch * p->ny + 63) / 64 * 64; }
inline int64_t plane_of(const ddf_params *p) { return plane_with(p, pitch_of(p)); }

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

inline size_t population_bytes(const ddf_params *p) { return align256(9 * (size_t)plane_of(p) * storage_size(p->storage)); }

// Host equilibria (absolute) used for wall terms and rest populations.
inline void host_feq(double rho, double ux, double uy, double c2, double out[9])
{
    const double ux2 = ux * ux, uy2 = uy * uy;
    double m[9] = {rho,
                   rho * ux,
                   rho * uy,
                   2.0 * c2 * rho + rho * (ux2 + uy2),
                   rho * (ux2 - uy2),
                   rho * ux * uy,
                   rho * uy * (c2 + ux2),
                   rho * ux * (c2 + uy2),
                   c2 * c2 * rho + rho * (c2 * (ux2 + uy2) + ux2 * uy2)};
    populations(m, out);
}

inline void host_geq(double phi, double ux, double uy, double c2, double b1, double b2, double out[9])
{
    const double ux2 = ux * ux, uy2 = uy * uy;
    double n[9] = {phi,
                   phi * ux,
                   phi * uy,
                   2.0 * c2 * phi + phi * (ux2 + uy2),
                   phi * (ux2 - uy2),
                   phi * ux * uy,
                   phi * uy * (b1 * c2 + ux2),
                   phi * ux * (b2 * c2 + uy2),
                   c2 * c2 * phi + phi * (c2 * (ux2 + uy2) + ux2 * uy2)};
    populations(n, out);
}

inline double storage_scale(const ddf_params &p)
{
    return p.pop_scale > 0.0 ? p.pop_scale : (p.storage == DDF_F16 ? 256.0 : 1.0);
}

template <class R>
Phys<R> make_phys(const ddf_params &p)
{
    const double scale = storage_scale(p);
    Phys<R> P;
    std::memset(&P, 0, sizeof(P));
    for (int k = 0; k < 9; ++k) {
        P.om[k] = (R)(k < 3 ? 0.0 : p.omega[k]);
        double w = k == 0 ? 0.0 : p.omega_phi[k];
        if (p.scalar_model == DDF_SCALAR_SRT && k > 0) w = p.omega_phi[1];
        P.omp[k] = (R)w;
    }
    P.b1 = (R)p.beta1;
    P.b2 = (R)p.beta2;
    P.c2 = (R)p.cs2;
    P.cp2 = (R)p.cs2_phi;
    P.rho0 = (R)p.rho0;
    P.phi0 = (R)p.phi0;
    P.scale = (R)scale;
    P.inv_scale = (R)(1.0 / scale);
    double rf[9], rg[9];
    host_feq(1.0, 0.0, 0.0, p.cs2, rf);
    host_geq(1.0, 0.0, 0.0, p.cs2_phi, p.beta1, p.beta2, rg);
    for (int a = 0; a < 9; ++a) {
        P.rest_f[a] = (R)rf[a];
        P.rest_g[a] = (R)rg[a];
    }
    for (int w = 0; w < 4; ++w) {
        double fe[9], ge[9];
        host_feq(1.0, p.wall_u[w][0], p.wall_u[w][1], p.cs2, fe);
        const bool dir = !std::isnan(p.wall_phi[w]);
        P.wall_dirichlet[w] = dir ? 1 : 0;
        if (dir) host_geq(p.wall_phi[w], p.wall_u[w][0], p.wall_u[w][1], p.cs2_phi, p.beta1, p.beta2, ge);
        for (int a = 0; a < 9; ++a) {
            P.wall_f[w][a] = (R)(fe[a] - fe[opp(a)]);
            P.wall_g[w][a] = dir ? (R)(ge[a] + ge[opp(a)] - 2.0 * p.phi0 * rg[a]) : (R)0;
        }
    }
    P.force_kind = p.force_kind;
    P.F0x = (R)p.force[0];
    P.F0y = (R)p.force[1];
    P.fk = (R)p.force_k;
    P.fom = (R)p.force_omega;
    P.phi_min = (R)p.phi_min;
    return P;
}

inline Lat make_lat(const ddf_params &p)
{
    Lat L;
    L.nx = p.nx;
    L.ny = p.ny;
    L.pitch = (int)pitch_of(&p);
    L.plane = plane_of(&p);
    L.px = p.periodic_x ? 1 : 0;
    L.py = p.periodic_y ? 1 : 0;
    L.qs = 0;   // row-major; a single lattice may switch to x-interleaved rows (interleave_shift)
    L.kpitch = (int)row_pitch(p.nx);
    L.kplane = plane_with(&p, L.kpitch);
    return L;
}

// Tile width: the smallest power of two >= nx, between 32 and bx_max.
inline int tile_shift(int nx, int bx_max)
{
    int bxs = 5;
    while ((1 << bxs) < nx && (1 << bxs) < bx_max) ++bxs;
    return bxs;
}

inline Geom make_geom(const ddf_params &p, int bx_max = kThreads)
{
    Geom G;
    G.L = make_lat(p);
    G.bx_shift = tile_shift(p.nx, bx_max);
    G.by = kThreads >> G.bx_shift;
    G.tiles_x = (p.nx + (1 << G.bx_shift) - 1) >> G.bx_shift;
    G.ntiles = G.tiles_x * ((p.ny + G.by - 1) / G.by);
    return G;
}

inline int grid_blocks(const Geom &G) { return (G.ntiles + 7) / 8 * 8; }

inline size_t snap_bytes(const ddf_params *p)
{
    const size_t r = p->storage == DDF_F64 ? 8 : 4;
    return align256(3 * (size_t)p->nx * p->ny * r);
}

inline int validate(const ddf_params *p)
{
    if (!p) return fail(DDF_ERR_ARG, "params is NULL");
    if (p->nx < 2 || p->ny < 2) return fail(DDF_ERR_ARG, "nx and ny must be >= 2");
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(DDF_ERR_ARG, "lattice larger than 2^31 nodes");
    if (p->storage < DDF_F64 || p->storage > DDF_BF16_SR) return fail(DDF_ERR_ARG, "unknown storage");
    if (p->scalar_model < DDF_SCALAR_MRT || p->scalar_model > DDF_SCALAR_CENTRAL)
        return fail(DDF_ERR_ARG, "unknown scalar model");
    if (p->force_kind < DDF_FORCE_NONE || p->force_kind > DDF_FORCE_PULSATILE)
        return fail(DDF_ERR_ARG, "unknown force kind");
    for (int k = 3; k < 9; ++k)
        if (!(p->omega[k] > 0.0 && p->omega[k] < 2.0)) return fail(DDF_ERR_ARG, "fluid rates omega3..8 must lie in (0, 2)");
    const int kmax = p->scalar_model == DDF_SCALAR_SRT ? 1 : 8;
    for (int k = 1; k <= kmax; ++k)
        if (!(p->omega_phi[k] > 0.0 && p->omega_phi[k] < 2.0))
            return fail(DDF_ERR_ARG, "scalar rates omega1..8^phi must lie in (0, 2)");
    if (!(std::fabs(p->beta1 - p->beta2) > 1e-12)) return fail(DDF_ERR_ARG, "beta1 == beta2: the vorticity relation is singular");
    if (!(p->cs2 > 0.0) || !(p->cs2_phi > 0.0)) return fail(DDF_ERR_ARG, "cs2 and cs2_phi must be positive");
    if (!(p->rho0 > 0.0)) return fail(DDF_ERR_ARG, "rho0 must be positive");
    if (p->layout < DDF_LAYOUT_AUTO || p->layout > DDF_LAYOUT_PACKED) return fail(DDF_ERR_ARG, "unknown layout");
    if (p->pop_scale < 0.0) return fail(DDF_ERR_ARG, "pop_scale must be >= 0");
    if (p->pop_scale > 0.0) {
        int e;
        if (std::frexp(p->pop_scale, &e) != 0.5) return fail(DDF_ERR_ARG, "pop_scale must be a power of two");
    }
    return DDF_OK;
}

inline bool has_walls(const ddf_params &p) { return !(p.periodic_x && p.periodic_y); }

// log2(nx / 64) when rows of this lattice can be x-interleaved (nx = 64 * 2^k, and a
// sub-row of nx / 64 nodes holds at least one 128-byte line of the storage type), else 0.
inline int interleave_shift(const ddf_params &p)
{
    const int64_t q = p.nx / 64, line = 128 / (int64_t)storage_size(p.storage);
    if (p.nx % 64 || q < line || (q & (q - 1))) return 0;
    int qs = 0;
    while (((int64_t)1 << qs) < q) ++qs;
    return qs;
}

// Calls fn with a null pointer of the storage element type.
template <class F>
int with_storage(int storage, F &&fn)
{
    switch (storage) {
    case DDF_F64: return fn((double *)nullptr);
    case DDF_F32: return fn((float *)nullptr);
    case DDF_F16: return fn((_Float16 *)nullptr);
    case DDF_BF16_SR: return fn((bf16sr *)nullptr);
    default: return fn((bf16 *)nullptr);
    }
}

// Stored-offset parameters of one lattice in both compute precisions.
struct PhysPair {
    Phys<double> d;
    Phys<float> f;
    template <class S>
    const Phys<typename Codec<S>::R> &of() const
    {
        if constexpr (std::is_same<typename Codec<S>::R, double>::value) return d;
        else return f;
    }
};

// Launchers of the per-lattice kernels (used for single lattices and for one instance of a batch).
template <class S>
void launch_extract(const Geom &G, const Phys<typename Codec<S>::R> &P, bool walls, bool odd, const void *f,
                    const void *g, int64_t t, int scalar_model, void *out, int out_dtype, uint32_t mask, hipStream_t st)
{
    const int nb = grid_blocks(G);
    auto go = [&](auto *otag) {
        using O = std::remove_pointer_t<decltype(otag)>;
        if (G.L.qs) {
            // 2048-node runs; rows of 1024 nodes (FP64 only) take 1024-node runs
            const int ks = G.L.nx % 2048 ? 4 : 5;
            const dim3 grid((unsigned)((int64_t)(G.L.nx >> (6 + ks)) * G.L.ny));
#define DDF_XI(W_, O_, KS_)                                                                                            \
    hipLaunchKernelGGL((k_extract_il<S, W_, O_, O, KS_>), grid, dim3(kThreads), 0, st, (const S *)f, (const S *)g, G.L, P, \
                       t, scalar_model, (O *)out, mask)
            if (ks == 5) {
                if (walls) { if (odd) DDF_XI(true, true, 5); else DDF_XI(true, false, 5); }
                else { if (odd) DDF_XI(false, true, 5); else DDF_XI(false, false, 5); }
            } else {
                if (walls) { if (odd) DDF_XI(true, true, 4); else DDF_XI(true, false, 4); }
                else { if (odd) DDF_XI(false, true, 4); else DDF_XI(false, false, 4); }
            }
#undef DDF_XI
            return;
        }
#define DDF_X(W_, O_)                                                                                          \
    hipLaunchKernelGGL((k_extract<S, W_, O_, O>), dim3(nb), dim3(kThreads), 0, st, (const S *)f, (const S *)g, G, P, t, \
                       scalar_model, (O *)out, mask)
        if (walls) { if (odd) DDF_X(true, true); else DDF_X(true, false); }
        else { if (odd) DDF_X(false, true); else DDF_X(false, false); }
#undef DDF_X
    };
    if (out_dtype == 0) go((double *)nullptr);
    else go((float *)nullptr);
}

template <class S>
void launch_get(const Geom &G, const Phys<typename Codec<S>::R> &P, bool walls, bool odd, const void *f, const void *g,
                void *fo, void *go, int dtype, hipStream_t st)
{
    const int nb = grid_blocks(G);
#define DDF_G(W_, O_) \
    hipLaunchKernelGGL((k_get<S, W_, O_>), dim3(nb), dim3(kThreads), 0, st, (const S *)f, (const S *)g, G, P, fo, go, dtype)
    if (walls) { if (odd) DDF_G(true, true); else DDF_G(true, false); }
    else { if (odd) DDF_G(false, true); else DDF_G(false, false); }
#undef DDF_G
}

template <class S>
void launch_set(const Geom &G, const Phys<typename Codec<S>::R> &P, bool walls, bool odd, void *f, void *g,
                const void *fi, const void *gi, int dtype, hipStream_t st)
{
    const int nb = grid_blocks(G);
#define DDF_S(W_, O_) \
    hipLaunchKernelGGL((k_set<S, W_, O_>), dim3(nb), dim3(kThreads), 0, st, (S *)f, (S *)g, G, P, fi, gi, dtype)
    if (walls) { if (odd) DDF_S(true, true); else DDF_S(true, false); }
    else { if (odd) DDF_S(false, true); else DDF_S(false, false); }
#undef DDF_S
}

}  // namespace host
}  // namespace ddf
