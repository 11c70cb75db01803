// libddf: fused two-lattice DDF lattice Boltzmann step, local kinematics extraction and
// FP64 reductions for MI355X (gfx950), behind the C ABI declared in include/ddf.h.
//
// Data layout in HBM: each lattice is 9 planes (one per direction), each plane ny rows
// of `pitch` elements (pitch = nx rounded up to 64), so a wavefront reads or writes 64
// consecutive nodes of one direction: 256 B (FP32), 512 B (FP64), 128 B (FP16/BF16).
// Large planes are separated by an extra 256 KiB + 256 B so that the 18 streams a
// node touches at one (x, y) do not start at the same offset of the HBM channel
// interleave (measured: +2% on 8192^2 FP32).
// Streaming is the in-place AA pattern: an even step reads a node's own slots and
// writes its post-collision populations into the opposite slots of the same node; an
// odd step reads the slots its neighbours wrote and pushes its results into their
// natural slots.  Each step therefore reads and writes every population exactly once
// (36 s bytes per node-update for storage size s) with no second array.  Half-way walls
// are applied when the populations are written, in both parities, so that the reflected
// value (with the moving-wall or Dirichlet term of the node's own state) sits where the
// next step reads it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>

#include "../../include/ddf.h"
#include "ddf_device.hpp"

using namespace ddf;

// Workgroup size of the lattice kernels (512 measured 1.5% faster than 256 on 8192^2).
constexpr int kThreads = 512;

// ---------------------------------------------------------------------------
// Geometry and tile mapping
// ---------------------------------------------------------------------------
struct Geom {
    int nx, ny;
    int pitch;          // elements per row
    int64_t plane;      // elements per direction plane (pitch * ny)
    int px, py;         // periodic flags
    int bx_shift;       // tile width = 1 << bx_shift
    int by;             // tile height (bx * by = kThreads)
    int tiles_x;
    int ntiles;
};

// Tile of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin by
// blockIdx; the remap gives each XCD one contiguous run of row-major tiles, so the
// neighbouring-row and partial-line traffic of the odd step stays in one L2.
__device__ __forceinline__ int tile_of_block(const Geom &G)
{
    const int per = gridDim.x >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ bool node_of_thread(const Geom &G, int &x, int &y)
{
    const int t = tile_of_block(G);
    if (t >= G.ntiles) return false;
    const int tx = t % G.tiles_x, ty = t / G.tiles_x;
    const int bx = 1 << G.bx_shift;
    x = (tx << G.bx_shift) + (threadIdx.x & (bx - 1));
    y = ty * G.by + (threadIdx.x >> G.bx_shift);
    return x < G.nx && y < G.ny;
}

// Neighbour of (x, y) along (dx, dy) with periodic wrapping; returns the wall side
// crossed (DDF_SIDE_*) or -1 for a fluid node.  A corner link counts against the
// bottom/top wall.
template <bool WALLS>
__device__ __forceinline__ int neighbour(const Geom &G, int x, int y, int dx, int dy, int &tx, int &ty)
{
    tx = x + dx;
    ty = y + dy;
    if (!WALLS) {
        tx = tx < 0 ? tx + G.nx : (tx >= G.nx ? tx - G.nx : tx);
        ty = ty < 0 ? ty + G.ny : (ty >= G.ny ? ty - G.ny : ty);
        return -1;
    }
    if (G.px) tx = tx < 0 ? tx + G.nx : (tx >= G.nx ? tx - G.nx : tx);
    if (G.py) ty = ty < 0 ? ty + G.ny : (ty >= G.ny ? ty - G.ny : ty);
    if (ty < 0) return DDF_SIDE_BOTTOM;
    if (ty >= G.ny) return DDF_SIDE_TOP;
    if (tx < 0) return DDF_SIDE_LEFT;
    if (tx >= G.nx) return DDF_SIDE_RIGHT;
    return -1;
}

// Storage slot holding the logical pre-collision population a of node (x, y) at a
// step of parity ODD: natural slot after an even number of steps; after an odd number
// the population sits in the opposite slot of its source node, or (for a population
// reflected by a wall) in slot a of the node itself.
template <bool WALLS, bool ODD>
__device__ __forceinline__ int64_t logical_slot(const Geom &G, int x, int y, int a)
{
    const int64_t cell = (int64_t)y * G.pitch + x;
    if (!ODD || a == 0) return (int64_t)a * G.plane + cell;
    int sx, sy;
    const int w = neighbour<WALLS>(G, x, y, -ex(a), -ey(a), sx, sy);
    if (w >= 0) return (int64_t)a * G.plane + cell;
    return (int64_t)opp(a) * G.plane + (int64_t)sy * G.pitch + sx;
}

template <class S, bool WALLS, bool ODD>
__device__ __forceinline__ void load_logical(const S *__restrict__ f, const Geom &G, int x, int y,
                                             typename Codec<S>::R inv_scale, typename Codec<S>::R v[9])
{
#pragma unroll
    for (int a = 0; a < 9; ++a) v[a] = Codec<S>::dec(f[logical_slot<WALLS, ODD>(G, x, y, a)]) * inv_scale;
}

// ---------------------------------------------------------------------------
// Step kernel
// ---------------------------------------------------------------------------
template <class S, int SCALAR, bool WALLS, bool FORCE, bool ODD>
__global__ __launch_bounds__(kThreads) void k_step(S *__restrict__ f, S *__restrict__ g, const Geom G,
                                              const Phys<typename Codec<S>::R> P, const int64_t t)
{
    using R = typename Codec<S>::R;
    int x, y;
    if (!node_of_thread(G, x, y)) return;

    R fv[9], gv[9];
    load_logical<S, WALLS, ODD>(f, G, x, y, P.inv_scale, fv);
    load_logical<S, WALLS, ODD>(g, G, x, y, P.inv_scale, gv);

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

    const int64_t cell = (int64_t)y * G.pitch + x;
    // rest direction: same slot in both parities
    f[cell] = Codec<S>::enc(fo[0] * P.scale);
    g[cell] = Codec<S>::enc(go[0] * P.scale);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        int tx, ty;
        const int w = neighbour<WALLS>(G, x, y, ex(a), ey(a), tx, ty);
        R vf = fo[a], vg = go[a];
        int64_t slot;
        if (WALLS && w >= 0) {
            // half-way bounce-back (with the moving-wall term) and anti-bounce-back
            // (Dirichlet scalar) land on the node itself, direction opp(a)
            vf = vf - M.rho * P.wall_f[w][a];
            if (P.wall_dirichlet[w]) vg = -vg + P.wall_g[w][a];
            slot = (int64_t)opp(a) * G.plane + cell;
        } else if (!ODD) {
            slot = (int64_t)opp(a) * G.plane + cell;
        } else {
            slot = (int64_t)a * G.plane + (int64_t)ty * G.pitch + tx;
        }
        f[slot] = Codec<S>::enc(vf * P.scale);
        g[slot] = Codec<S>::enc(vg * P.scale);
    }
}

// ---------------------------------------------------------------------------
// Extraction, initialisation, reductions, population access
// ---------------------------------------------------------------------------
template <class S, bool WALLS, bool ODD, class O>
__global__ __launch_bounds__(kThreads) void k_extract(const S *__restrict__ f, const S *__restrict__ g, const Geom G,
                                                 const Phys<typename Codec<S>::R> P, const int64_t t,
                                                 const int scalar_model, O *__restrict__ out, const uint32_t mask)
{
    using R = typename Codec<S>::R;
    int x, y;
    if (!node_of_thread(G, x, y)) return;
    R fv[9], gv[9], m[9], n[9];
    load_logical<S, WALLS, ODD>(f, G, x, y, P.inv_scale, fv);
    load_logical<S, WALLS, ODD>(g, G, x, y, P.inv_scale, gv);
    moments(fv, m);
    moments(gv, n);
    R Fx = (R)0, Fy = (R)0;
    body_force(P, x, y, t, Fx, Fy);
    const Macro<R> M = macro(P, m, n, Fx, Fy);
    const Kin<R> K = kinematics(P, M, m, n, Fx, Fy, scalar_model);
    const R vals[DDF_NUM_OUTPUTS] = {M.rho, M.ux, M.uy, M.phi, K.Sxx, K.Syy, K.Sxy, K.wz,
                                     K.dxuy, K.dyux, K.dxphi, K.dyphi, K.Q, K.Rinv, K.Lx, K.Ly};
    const int64_t N = (int64_t)G.nx * G.ny;
    const int64_t c = (int64_t)y * G.nx + x;
#pragma unroll
    for (int k = 0; k < DDF_NUM_OUTPUTS; ++k)
        if (mask & (1u << k)) out[(int64_t)k * N + c] = (O)vals[k];
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
    const int64_t c = (int64_t)y * G.nx + x;
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
    const int64_t cell = (int64_t)y * G.pitch + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f[(int64_t)a * G.plane + cell] = Codec<S>::enc(fo[a] * P.scale);
        g[(int64_t)a * G.plane + cell] = Codec<S>::enc(go[a] * P.scale);
    }
}

// Per-block FP64 partial sums; fixed tree order, so results are deterministic.
enum { RS_MASS = 0, RS_SCALAR, RS_DU2, RS_U2, RS_DPHI2, RS_PHI2, RS_NONFIN, RS_UMAX, RS_PHIMIN, RS_N };

template <class S, bool WALLS, bool ODD>
__global__ __launch_bounds__(kThreads) void k_reduce(const S *__restrict__ f, const S *__restrict__ g, const Geom G,
                                                const Phys<typename Codec<S>::R> P, const int64_t t,
                                                typename Codec<S>::R *__restrict__ snap, const int snap_valid,
                                                double *__restrict__ partials)
{
    using R = typename Codec<S>::R;
    __shared__ double sh[RS_N][kThreads];
    double v[RS_N] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    int x, y;
    if (node_of_thread(G, x, y)) {
        R fv[9], gv[9], m[9], n[9];
        load_logical<S, WALLS, ODD>(f, G, x, y, P.inv_scale, fv);
        load_logical<S, WALLS, ODD>(g, G, x, y, P.inv_scale, gv);
        moments(fv, m);
        moments(gv, n);
        R Fx = (R)0, Fy = (R)0;
        body_force(P, x, y, t, Fx, Fy);
        const Macro<R> M = macro(P, m, n, Fx, Fy);
        const int64_t N = (int64_t)G.nx * G.ny;
        const int64_t c = (int64_t)y * G.nx + x;
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
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < RS_N; ++k) sh[k][tid] = v[k];
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int k = 0; k < RS_UMAX; ++k) sh[k][tid] += sh[k][tid + s];
            sh[RS_UMAX][tid] = fmax(sh[RS_UMAX][tid], sh[RS_UMAX][tid + s]);
            sh[RS_PHIMIN][tid] = fmin(sh[RS_PHIMIN][tid], sh[RS_PHIMIN][tid + s]);
        }
        __syncthreads();
    }
    if (tid < RS_N) partials[(int64_t)blockIdx.x * RS_N + tid] = sh[tid][0];
}

__global__ __launch_bounds__(256) void k_reduce_final(const double *__restrict__ partials, const int nblocks,
                                                      double *__restrict__ out)
{
    __shared__ double sh[RS_N][256];
    const int tid = threadIdx.x;
    double v[RS_N] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    for (int b = tid; b < nblocks; b += 256) {
#pragma unroll
        for (int k = 0; k < RS_UMAX; ++k) v[k] += partials[(int64_t)b * RS_N + k];
        v[RS_UMAX] = fmax(v[RS_UMAX], partials[(int64_t)b * RS_N + RS_UMAX]);
        v[RS_PHIMIN] = fmin(v[RS_PHIMIN], partials[(int64_t)b * RS_N + RS_PHIMIN]);
    }
#pragma unroll
    for (int k = 0; k < RS_N; ++k) sh[k][tid] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
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

// dtype 0: absolute FP64 values; dtype 1: raw stored elements.
template <class S, bool WALLS, bool ODD>
__global__ __launch_bounds__(kThreads) void k_get(const S *__restrict__ f, const S *__restrict__ g, const Geom G,
                                             const Phys<typename Codec<S>::R> P, void *__restrict__ fo,
                                             void *__restrict__ go, const int dtype)
{
    int x, y;
    if (!node_of_thread(G, x, y)) return;
    const int64_t N = (int64_t)G.nx * G.ny;
    const int64_t c = (int64_t)y * G.nx + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int64_t s = logical_slot<WALLS, ODD>(G, x, y, a);
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
    const int64_t N = (int64_t)G.nx * G.ny;
    const int64_t c = (int64_t)y * G.nx + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int64_t s = logical_slot<WALLS, ODD>(G, x, y, a);
        if (dtype == 0) {
            const double vf = ((const double *)fi)[a * N + c] - (double)P.rest_f[a] * (double)P.rho0;
            const double vg = ((const double *)gi)[a * N + c] - (double)P.rest_g[a] * (double)P.phi0;
            f[s] = Codec<S>::enc((R)(vf * (double)P.scale));
            g[s] = Codec<S>::enc((R)(vg * (double)P.scale));
        } else {
            f[s] = ((const S *)fi)[a * N + c];
            g[s] = ((const S *)gi)[a * N + c];
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(DDF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

int64_t pitch_of(const ddf_params *p) { return ((int64_t)p->nx + 63) / 64 * 64; }

size_t storage_size(int storage) { return storage == DDF_F64 ? 8 : (storage == DDF_F32 ? 4 : 2); }

// Elements per direction plane: pitch * ny, plus 256 KiB + 256 B for planes of 16 MiB or more.
int64_t plane_of(const ddf_params *p)
{
    const int64_t s = (int64_t)storage_size(p->storage);
    const int64_t base = pitch_of(p) * p->ny;
    return base * s >= (16ll << 20) ? base + ((256ll << 10) + 256) / s : base;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Host equilibria (absolute) used for wall terms and rest populations.
void host_feq(double rho, double ux, double uy, double c2, double out[9])
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

void host_geq(double phi, double ux, double uy, double c2, double b1, double b2, double out[9])
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

template <class R>
Phys<R> make_phys(const ddf_params &p, double scale)
{
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

}  // namespace

struct ddf_handle {
    ddf_params p;
    void *f, *g, *ws;
    Geom G;
    int nblocks;
    int64_t step;
    int64_t snap_step;
    bool snap_valid;
    bool initialised;
    double scale;
    Phys<double> pd;
    Phys<float> pf;
};

namespace {

Geom make_geom(const ddf_params &p)
{
    Geom G;
    G.nx = p.nx;
    G.ny = p.ny;
    G.pitch = (int)pitch_of(&p);
    G.plane = plane_of(&p);
    G.px = p.periodic_x ? 1 : 0;
    G.py = p.periodic_y ? 1 : 0;
    // tile: as wide as the row allows (coalesced rows), kThreads threads
    int bxs = 9;
    while (bxs > 5 && (1 << (bxs - 1)) >= p.nx) --bxs;
    G.bx_shift = bxs;
    G.by = kThreads >> bxs;
    G.tiles_x = (p.nx + (1 << bxs) - 1) >> bxs;
    G.ntiles = G.tiles_x * ((p.ny + G.by - 1) / G.by);
    return G;
}

int grid_blocks(const Geom &G) { return (G.ntiles + 7) / 8 * 8; }

size_t snap_bytes(const ddf_params *p)
{
    const size_t r = p->storage == DDF_F64 ? 8 : 4;
    return align256(3 * (size_t)p->nx * p->ny * r);
}

int validate(const ddf_params *p)
{
    if (!p) return fail(DDF_ERR_ARG, "params is NULL");
    if (p->nx < 2 || p->ny < 2) return fail(DDF_ERR_ARG, "nx and ny must be >= 2");
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(DDF_ERR_ARG, "lattice larger than 2^31 nodes");
    if (p->storage < DDF_F64 || p->storage > DDF_BF16) return fail(DDF_ERR_ARG, "unknown storage");
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
    if (p->pop_scale < 0.0) return fail(DDF_ERR_ARG, "pop_scale must be >= 0");
    if (p->pop_scale > 0.0) {
        int e;
        if (std::frexp(p->pop_scale, &e) != 0.5) return fail(DDF_ERR_ARG, "pop_scale must be a power of two");
    }
    return DDF_OK;
}

bool has_walls(const ddf_params &p) { return !(p.periodic_x && p.periodic_y); }

// Dispatch helpers over (storage) x (walls) x (parity).
template <class F>
int with_storage(int storage, F &&fn)
{
    switch (storage) {
    case DDF_F64: return fn((double *)nullptr);
    case DDF_F32: return fn((float *)nullptr);
    case DDF_F16: return fn((_Float16 *)nullptr);
    default: return fn((bf16 *)nullptr);
    }
}

template <class S>
const Phys<typename Codec<S>::R> &phys_of(const ddf_handle *h);
template <> const Phys<double> &phys_of<double>(const ddf_handle *h) { return h->pd; }
template <> const Phys<float> &phys_of<float>(const ddf_handle *h) { return h->pf; }
template <> const Phys<float> &phys_of<_Float16>(const ddf_handle *h) { return h->pf; }
template <> const Phys<float> &phys_of<bf16>(const ddf_handle *h) { return h->pf; }

template <class S, int SC, bool W, bool FO>
void launch_step_parity(ddf_handle *h, hipStream_t st, bool odd)
{
    const int nb = grid_blocks(h->G);
    if (odd)
        hipLaunchKernelGGL((k_step<S, SC, W, FO, true>), dim3(nb), dim3(kThreads), 0, st, (S *)h->f, (S *)h->g, h->G,
                           phys_of<S>(h), h->step);
    else
        hipLaunchKernelGGL((k_step<S, SC, W, FO, false>), dim3(nb), dim3(kThreads), 0, st, (S *)h->f, (S *)h->g, h->G,
                           phys_of<S>(h), h->step);
}

template <class S, int SC>
void launch_step(ddf_handle *h, hipStream_t st)
{
    const bool odd = (h->step & 1) != 0;
    const bool w = has_walls(h->p);
    const bool fo = h->p.force_kind != DDF_FORCE_NONE;
    if (w) {
        if (fo) launch_step_parity<S, SC, true, true>(h, st, odd);
        else launch_step_parity<S, SC, true, false>(h, st, odd);
    } else {
        if (fo) launch_step_parity<S, SC, false, true>(h, st, odd);
        else launch_step_parity<S, SC, false, false>(h, st, odd);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int64_t ddf_pitch(const ddf_params *p) { return p ? pitch_of(p) : 0; }

int64_t ddf_plane_stride(const ddf_params *p) { return p ? plane_of(p) : 0; }

size_t ddf_population_bytes(const ddf_params *p)
{
    if (!p) return 0;
    return align256(9 * (size_t)plane_of(p) * storage_size(p->storage));
}

size_t ddf_workspace_bytes(const ddf_params *p)
{
    if (!p || validate(p) != DDF_OK) return 0;
    const Geom G = make_geom(*p);
    return snap_bytes(p) + align256((size_t)grid_blocks(G) * RS_N * sizeof(double)) + 256;
}

int ddf_create(const ddf_params *p, void *pop_f, void *pop_g, void *workspace, ddf_handle **out)
{
    int rc = validate(p);
    if (rc != DDF_OK) return rc;
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (!pop_f || !pop_g || !workspace) return fail(DDF_ERR_ARG, "a device buffer is NULL");
    if (((uintptr_t)pop_f | (uintptr_t)pop_g | (uintptr_t)workspace) & 255)
        return fail(DDF_ERR_ARG, "device buffers must be 256-byte aligned");
    ddf_handle *h = new (std::nothrow) ddf_handle;
    if (!h) return fail(DDF_ERR_ARG, "out of host memory");
    std::memset(h, 0, sizeof(*h));
    h->p = *p;
    h->f = pop_f;
    h->g = pop_g;
    h->ws = workspace;
    h->G = make_geom(*p);
    h->nblocks = grid_blocks(h->G);
    h->scale = p->pop_scale > 0.0 ? p->pop_scale : (p->storage == DDF_F16 ? 256.0 : 1.0);
    h->pd = make_phys<double>(*p, h->scale);
    h->pf = make_phys<float>(*p, h->scale);
    *out = h;
    return DDF_OK;
}

void ddf_destroy(ddf_handle *h) { delete h; }

int64_t ddf_step_count(const ddf_handle *h) { return h ? h->step : -1; }

const char *ddf_last_error(void) { return g_err.c_str(); }

int ddf_init_equilibrium(ddf_handle *h, const double *rho, const double *ux, const double *uy, const double *phi,
                         void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!rho || !ux || !uy || !phi) return fail(DDF_ERR_ARG, "a field pointer is NULL");
    hipStream_t st = (hipStream_t)stream;
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL((k_init<S>), dim3(h->nblocks), dim3(kThreads), 0, st, (S *)h->f, (S *)h->g, h->G, phys_of<S>(h),
                           rho, ux, uy, phi);
        return 0;
    });
    HIP_TRY(hipGetLastError());
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
    for (int64_t i = 0; i < nsteps; ++i) {
        with_storage(h->p.storage, [&](auto *tag) {
            using S = std::remove_pointer_t<decltype(tag)>;
            switch (h->p.scalar_model) {
            case DDF_SCALAR_SRT: launch_step<S, DDF_SCALAR_SRT>(h, st); break;
            case DDF_SCALAR_CASCADED:
            case DDF_SCALAR_CENTRAL: launch_step<S, DDF_SCALAR_CENTRAL>(h, st); break;
            default: launch_step<S, DDF_SCALAR_MRT>(h, st);
            }
            return 0;
        });
        h->step++;
    }
    HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_extract(ddf_handle *h, void *out, uint32_t mask, int32_t out_dtype, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!out) return fail(DDF_ERR_ARG, "out is NULL");
    if (out_dtype != 0 && out_dtype != 1) return fail(DDF_ERR_ARG, "out_dtype must be 0 (double) or 1 (float)");
    if (!h->initialised) return fail(DDF_ERR_STATE, "extract before init or set_populations");
    hipStream_t st = (hipStream_t)stream;
    const bool odd = (h->step & 1) != 0, w = has_walls(h->p);
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        auto go = [&](auto *otag) {
            using O = std::remove_pointer_t<decltype(otag)>;
#define DDF_EXTRACT(W_, O_)                                                                                      \
    hipLaunchKernelGGL((k_extract<S, W_, O_, O>), dim3(h->nblocks), dim3(kThreads), 0, st, (const S *)h->f,        \
                       (const S *)h->g, h->G, phys_of<S>(h), h->step, h->p.scalar_model, (O *)out, mask)
            if (w) { if (odd) DDF_EXTRACT(true, true); else DDF_EXTRACT(true, false); }
            else { if (odd) DDF_EXTRACT(false, true); else DDF_EXTRACT(false, false); }
#undef DDF_EXTRACT
        };
        if (out_dtype == 0) go((double *)nullptr);
        else go((float *)nullptr);
        return 0;
    });
    HIP_TRY(hipGetLastError());
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
    hipLaunchKernelGGL((k_reduce<S, W_, O_>), dim3(h->nblocks), dim3(kThreads), 0, st, (const S *)h->f,             \
                       (const S *)h->g, h->G, phys_of<S>(h), h->step, (R *)snap, sv, partials)
        if (w) { if (odd) DDF_REDUCE(true, true); else DDF_REDUCE(true, false); }
        else { if (odd) DDF_REDUCE(false, true); else DDF_REDUCE(false, false); }
#undef DDF_REDUCE
        return 0;
    });
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, partials, h->nblocks, fin);
    HIP_TRY(hipGetLastError());
    double r[RS_N];
    HIP_TRY(hipMemcpyAsync(r, fin, sizeof(r), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
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
    hipStream_t st = (hipStream_t)stream;
    const bool odd = (h->step & 1) != 0, w = has_walls(h->p);
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
#define DDF_GET(W_, O_)                                                                                          \
    hipLaunchKernelGGL((k_get<S, W_, O_>), dim3(h->nblocks), dim3(kThreads), 0, st, (const S *)h->f, (const S *)h->g, \
                       h->G, phys_of<S>(h), f, g, dtype)
        if (w) { if (odd) DDF_GET(true, true); else DDF_GET(true, false); }
        else { if (odd) DDF_GET(false, true); else DDF_GET(false, false); }
#undef DDF_GET
        return 0;
    });
    HIP_TRY(hipGetLastError());
    return DDF_OK;
}

int ddf_set_populations(ddf_handle *h, const void *f, const void *g, int32_t dtype, int64_t step, void *stream)
{
    if (!h) return fail(DDF_ERR_ARG, "handle is NULL");
    if (!f || !g) return fail(DDF_ERR_ARG, "input pointer is NULL");
    if (dtype != 0 && dtype != 1) return fail(DDF_ERR_ARG, "dtype must be 0 (double) or 1 (raw)");
    if (step < 0) return fail(DDF_ERR_ARG, "step < 0");
    hipStream_t st = (hipStream_t)stream;
    const bool odd = (step & 1) != 0, w = has_walls(h->p);
    with_storage(h->p.storage, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
#define DDF_SET(W_, O_)                                                                                          \
    hipLaunchKernelGGL((k_set<S, W_, O_>), dim3(h->nblocks), dim3(kThreads), 0, st, (S *)h->f, (S *)h->g, h->G,       \
                       phys_of<S>(h), f, g, dtype)
        if (w) { if (odd) DDF_SET(true, true); else DDF_SET(true, false); }
        else { if (odd) DDF_SET(false, true); else DDF_SET(false, false); }
#undef DDF_SET
        return 0;
    });
    HIP_TRY(hipGetLastError());
    h->step = step;
    h->snap_valid = false;
    h->initialised = true;
    return DDF_OK;
}

}  // extern "C"
