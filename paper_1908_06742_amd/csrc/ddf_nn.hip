// libddf, surrogate network kernels: the building blocks of a 2D U-Net on NHWC BF16
// activations with FP32 accumulation on the gfx950 matrix cores, its backward pass and
// an Adam step on FP32 master weights.  Declared in include/ddf_nn.h.
//
// 3x3 convolutions are implicit GEMMs: rows = output pixels, columns = output
// channels, reduction = 9 taps x input channels.  One wavefront owns a 32 x 32 output
// tile and issues v_mfma_f32_32x32x16_bf16 (A: 32 pixels x 16 channels of one tap,
// B: 16 channels x 32 output channels); lane l holds A[l % 32][8 (l / 32) + i] and
// B[8 (l / 32) + i][l % 32], i < 8, and receives C[8 (j / 4) + 4 (l / 32) + j % 4][l % 32],
// j < 16.  The data gradient is the same kernel on the output gradient with the taps
// flipped and the weight transposed; the weight gradient is a split-K GEMM over pixels
// whose FP32 partials are summed in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/ddf_nn.h"
#include "ddf_kernels.hpp"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

using ddf::host::fail;

__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *(const bf16x8 *)p; }
// Sixteen zero bytes in device memory.  A staging load whose pixel lies outside the image
// (or whose lane has nothing to stage) reads these instead of being skipped: with every
// load unconditional the compiler counts the loads still in flight exactly and waits for
// just the ones a write to LDS needs, where a skipped load (a branch) made it wait for all
// of them, the prefetched rows included.  The array is global memory (not const, which
// would place it in another address space and make the selected pointer a flat one); it
// is never written.
__device__ __align__(16) __bf16 kZero8[8] = {};

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

// out[p, oc0 + co] (= or +=) act(bias[co] + sum_{tap, ci} in[p + d(tap), ic0 + ci] w[tap][co][ci])
// WM x WN waves per workgroup, each a 32 x 32 tile.  Requirements (checked on the host):
// Cin % 16 == 0, Cout % (32 WN) == 0, npix % (32 WM) == 0, channel strides and offsets
// multiples of 8.
template <int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_conv3x3(const __bf16 *__restrict__ in, int N, int H, int W, int Cin,
                                                          int in_cs, int in_co, const __bf16 *__restrict__ wt,
                                                          const float *__restrict__ bias, __bf16 *__restrict__ out,
                                                          int Cout, int out_cs, int out_co, int relu, int accumulate,
                                                          const __bf16 *__restrict__ mask, int mask_cs, int mask_co)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int p0 = (blockIdx.x * WM + wm) * 32;
    const int co0 = (blockIdx.y * WN + wn) * 32;
    const int m = lane & 31, half = lane >> 5;
    // pixel of this lane's A row
    const int p = p0 + m;
    const int n = p / (H * W), rem = p - n * (H * W);
    const int y = rem / W, x = rem - y * W;
    f32x16 acc = {};
    const __bf16 *wrow = wt + (int64_t)(co0 + m) * Cin + 8 * half;
    for (int tap = 0; tap < 9; ++tap) {
        const int iy = y + tap / 3 - 1, ix = x + tap % 3 - 1;
        const bool ok = iy >= 0 && iy < H && ix >= 0 && ix < W;
        const int64_t aoff = ok ? ((int64_t)(n * H + iy) * W + ix) * in_cs + in_co + 8 * half : 0;
        const __bf16 *arow = in + aoff;
        const __bf16 *brow = wrow + (int64_t)tap * Cout * Cin;
        for (int c0 = 0; c0 < Cin; c0 += 16) {
            const bf16x8 a = ok ? load8(arow + c0) : zero8();
            const bf16x8 b = load8(brow + c0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
    }
    const int co = co0 + m;
    const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int pr = p0 + 8 * (j >> 2) + 4 * half + (j & 3);
        __bf16 *o = out + (int64_t)pr * out_cs + out_co + co;
        float v = acc[j] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        if (mask && !((float)mask[(int64_t)pr * mask_cs + mask_co + co] > 0.0f)) v = 0.0f;
        if (accumulate) v += (float)*o;
        *o = (__bf16)v;
    }
}

// Row-streaming convolution (same contract as k_conv3x3).  A workgroup of four
// wavefronts computes R consecutive output rows of PB consecutive pixels against WCO
// tiles of 32 output channels: wavefront w owns output-channel tile w mod WCO and, of
// every output row, the pixel tiles w / WCO, w / WCO + 4 / WCO, ...  Per 32-channel
// input chunk every wavefront holds the MFMA B operands of its tile's nine taps in
// registers (the 32 x 32 weight tile of each tap, 16-byte loads straight from global
// memory), and the R + 2 input rows the outputs read stream through a double-buffered
// LDS row (one pixel of halo on each side).  Each staged row feeds every output row it
// touches: one LDS read of an A operand (a pixel tile at one kernel column and channel
// half) feeds up to three MFMAs, one per kernel row, so LDS carries a third of an A
// operand and no B operand per MFMA.  The 16-byte global loads of the input row PD
// ahead (of this chunk or the next) are in flight during the current row's MFMAs, in PD
// register slots: with one wavefront per SIMD (the deep layers at batch 8 fill the chip
// once) a lead of one row left the loads' latency exposed (PD = 2 to 4: 5-25% faster on
// those layers).  Needs Cin % 32 == 0, W % PB == 0, H % R == 0, Cout % (32 WCO) == 0
// and (R + 2) % PD == 0; grid.y = Cout / (32 WCO).
template <int PB, int R, int WCO, int PD>
__global__ __launch_bounds__(256) void k_conv3x3_rows(const __bf16 *__restrict__ in, int N, int H, int W, int Cin,
                                                      int in_cs, int in_co, const __bf16 *__restrict__ wt,
                                                      const float *__restrict__ bias, __bf16 *__restrict__ out,
                                                      int Cout, int out_cs, int out_co, int relu, int accumulate,
                                                      const __bf16 *__restrict__ mask, int mask_cs, int mask_co)
{
    constexpr int WP = 4 / WCO;                  // wavefronts per output-channel tile
    constexpr int PMT = PB / 32;                 // pixel tiles per row
    constexpr int TW = PMT / WP;                 // pixel tiles per wavefront
    constexpr int NR = R + 2;                    // input rows per chunk
    static_assert(WP * WCO == 4 && TW >= 1 && PMT == WP * TW, "four wavefronts share the tiles evenly");
    static_assert(PD >= 1 && NR % PD == 0, "input rows are prefetched PD ahead in PD register slots");
    constexpr int RS = 40;                       // LDS row stride (32 channels + 8 of padding)
    __shared__ __attribute__((aligned(16))) __bf16 xs[2][PB + 2][RS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wc = wave % WCO, wp = wave / WCO;
    const int m = lane & 31, half = lane >> 5;
    const int segs = W / PB, bands = H / R;
    const int x0 = (int)(blockIdx.x % segs) * PB;
    const int64_t nb = blockIdx.x / segs;        // n * bands + band
    const int64_t img = nb / bands;              // n
    const int y0 = (int)(nb % bands) * R;
    const int co0 = (blockIdx.y * WCO + wc) * 32;
    f32x16 acc[R][TW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[r][t][j] = 0.0f;
    constexpr int XV = (PB + 2) * 4;             // 16-byte input vectors per staged row
    constexpr int NXV = (XV + 255) / 256;
    bf16x8 xr[PD][NXV];
    // input row y0 - 1 + j of chunk c0 into register slot d (zeros outside the image)
    auto fetch_row = [&](int d, int j, int c0) {
        const int yi = y0 - 1 + j;
        const bool row_ok = yi >= 0 && yi < H;
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = tid + 256 * i;
            const int c8 = v & 3, px = v >> 2, xx = x0 + px - 1;
            const bool ok = v < XV && row_ok && xx >= 0 && xx < W;
            xr[d][i] = load8(ok ? in + ((img * H + yi) * W + xx) * in_cs + in_co + c0 + 8 * c8 : kZero8);
        }
    };
    // B operands of a chunk: lane (m, half) holds output channel co0 + m, input channels
    // c0 + 16 k + 8 half .. + 7, for every tap and k
    bf16x8 bw[9][2];
    // the mask bits of this lane's outputs
    uint32_t mbits[R][TW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            mbits[r][t] = 0xffffu;
            if (mask) {
                const int pm = wp + WP * t;
                uint32_t b = 0;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int64_t pr = (img * H + y0 + r) * W + x0 + 32 * pm + 8 * (j >> 2) + 4 * half + (j & 3);
                    b |= ((float)mask[pr * mask_cs + mask_co + co0 + m] > 0.0f ? 1u : 0u) << j;
                }
                mbits[r][t] = b;
            }
        }
    const int nc = Cin / 32;
#pragma unroll
    for (int d = 0; d < PD; ++d) fetch_row(d, d, 0);
    for (int c = 0; c < nc; ++c) {
        const int c0 = 32 * c;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int k = 0; k < 2; ++k)
                bw[tap][k] = load8(wt + ((int64_t)tap * Cout + co0 + m) * Cin + c0 + 16 * k + 8 * half);
        // with R odd the chunk's last row was read from the buffer its first row is written to
        if ((R & 1) && c > 0) __syncthreads();
#pragma unroll
        for (int j = 0; j < NR; ++j) {           // input row y0 - 1 + j
            const int b = j & 1;
#pragma unroll
            for (int i = 0; i < NXV; ++i) {
                const int v = tid + 256 * i;
                if (v < XV) *(bf16x8 *)&xs[b][v >> 2][8 * (v & 3)] = xr[j % PD][i];
            }
            __syncthreads();
            // the input row PD ahead, of this chunk or of the next one
            if (j + PD < NR) fetch_row(j % PD, j + PD, c0);
            else if (c + 1 < nc) fetch_row(j % PD, j + PD - NR, c0 + 32);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int t = 0; t < TW; ++t) {
                        const int pm = wp + WP * t;
                        const bf16x8 a = *(const bf16x8 *)&xs[b][32 * pm + m + dx][16 * k + 8 * half];
#pragma unroll
                        for (int dy = 0; dy < 3; ++dy) {
                            const int yo = j - dy;   // the output row this input row meets with kernel row dy
                            if (yo < 0 || yo >= R) continue;
                            acc[yo][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw[3 * dy + dx][k], acc[yo][t], 0, 0, 0);
                        }
                    }
        }
    }
    const int co = co0 + m;
    const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TW; ++t) {
            const int pm = wp + WP * t;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t pr = (img * H + y0 + r) * W + x0 + 32 * pm + 8 * (j >> 2) + 4 * half + (j & 3);
                __bf16 *o = out + pr * out_cs + out_co + co;
                float v = acc[r][t][j] + bv;
                if (relu) v = fmaxf(v, 0.0f);
                if (!((mbits[r][t] >> j) & 1u)) v = 0.0f;
                if (accumulate) v += (float)*o;
                *o = (__bf16)v;
            }
        }
}

// LDS-staged convolution (same contract as k_conv3x3).  A workgroup of four wavefronts
// computes PB consecutive pixels of one image row against NCO tiles of 32 output
// channels.  The reduction runs over (kernel row dy, 32-channel chunk): per stage the
// input row y + dy with one pixel of halo on each side, and the weights of the row's
// three taps, are staged into LDS with 16-byte loads; then each wavefront applies the
// three taps (a dx shift moves whole pixels, so the 16-byte operand reads stay aligned)
// to its TPW output tiles.  Staged inputs feed 3 NCO MFMA tiles, staged weights PB / 32.
template <int PB, int NCO>
__global__ __launch_bounds__(256) void k_conv3x3_lds(const __bf16 *__restrict__ in, int N, int H, int W, int Cin,
                                                     int in_cs, int in_co, const __bf16 *__restrict__ wt,
                                                     const float *__restrict__ bias, __bf16 *__restrict__ out,
                                                     int Cout, int out_cs, int out_co, int relu, int accumulate,
                                                     const __bf16 *__restrict__ mask, int mask_cs, int mask_co)
{
    constexpr int PMT = PB / 32;                 // pixel tiles
    constexpr int TPW = PMT * NCO / 4;           // output tiles per wavefront
    static_assert(TPW >= 1 && PMT * NCO == 4 * TPW, "four wavefronts share the tiles evenly");
    constexpr int RS = 40;                       // LDS row stride (32 channels + 8 of padding)
    __shared__ __attribute__((aligned(16))) __bf16 xs[PB + 2][RS];
    __shared__ __attribute__((aligned(16))) __bf16 ws[3][32 * NCO][RS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 31, half = lane >> 5;
    const int segs = W / PB;
    const int64_t row = blockIdx.x / segs;       // n * H + y
    const int x0 = (int)(blockIdx.x % segs) * PB;
    const int y = (int)(row % H);
    const int co0 = blockIdx.y * 32 * NCO;
    f32x16 acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
    // Stages (kernel row dy, 32-channel chunk c0) in dy-major order.  Staging is
    // software-pipelined: the global loads of stage s + 1 are issued into registers before
    // the MFMAs of stage s and written to LDS after them.
    constexpr int XV = (PB + 2) * 4;             // 16-byte input vectors per stage
    constexpr int WV = 3 * 32 * NCO * 4;         // 16-byte weight vectors per stage
    constexpr int NXV = (XV + 255) / 256, NWV = (WV + 255) / 256;
    bf16x8 xr[NXV], wr[NWV];
    const int nc = Cin / 32, nst = 3 * nc;
    auto fetch = [&](int s) {
        const int dy = s / nc, c0 = 32 * (s - dy * nc);
        const int yy = y + dy - 1;
        const bool row_ok = yy >= 0 && yy < H;
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = tid + 256 * i;
            const int c8 = v & 3, px = v >> 2, xx = x0 + px - 1;
            const bool ok = v < XV && row_ok && xx >= 0 && xx < W;
            xr[i] = load8(ok ? in + ((row + dy - 1) * W + xx) * in_cs + in_co + c0 + 8 * c8 : kZero8);
        }
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const int v = tid + 256 * i;
            const int c8 = v & 3, q = v >> 2, co = q % (32 * NCO), dx = q / (32 * NCO);
            wr[i] = load8(v < WV ? wt + ((int64_t)(3 * dy + dx) * Cout + co0 + co) * Cin + c0 + 8 * c8 : kZero8);
        }
    };
    fetch(0);
    // The mask values of this lane's outputs, one bit each, loaded behind the first
    // stage's loads so that their latency is shared with it.
    uint32_t mbits[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        mbits[t] = 0xffffu;
        if (mask) {
            const int tile = wave * TPW + t, pm = tile % PMT, cn = tile / PMT;
            const int co = co0 + 32 * cn + m;
            uint32_t b = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t pr = row * W + x0 + 32 * pm + 8 * (j >> 2) + 4 * half + (j & 3);
                b |= ((float)mask[pr * mask_cs + mask_co + co] > 0.0f ? 1u : 0u) << j;
            }
            mbits[t] = b;
        }
    }
    for (int s = 0; s < nst; ++s) {
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = tid + 256 * i;
            if (v < XV) *(bf16x8 *)&xs[v >> 2][8 * (v & 3)] = xr[i];
        }
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const int v = tid + 256 * i;
            const int q = v >> 2;
            if (v < WV) *(bf16x8 *)&ws[q / (32 * NCO)][q % (32 * NCO)][8 * (v & 3)] = wr[i];
        }
        __syncthreads();
        if (s + 1 < nst) fetch(s + 1);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    const int tile = wave * TPW + t, pm = tile % PMT, cn = tile / PMT;
                    const bf16x8 a = *(const bf16x8 *)&xs[32 * pm + m + dx][16 * k + 8 * half];
                    const bf16x8 b = *(const bf16x8 *)&ws[dx][32 * cn + m][16 * k + 8 * half];
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int tile = wave * TPW + t, pm = tile % PMT, cn = tile / PMT;
        const int co = co0 + 32 * cn + m;
        const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int64_t pr = row * W + x0 + 32 * pm + 8 * (j >> 2) + 4 * half + (j & 3);
            __bf16 *o = out + pr * out_cs + out_co + co;
            float v = acc[t][j] + bv;
            if (relu) v = fmaxf(v, 0.0f);
            if (!((mbits[t] >> j) & 1u)) v = 0.0f;
            if (accumulate) v += (float)*o;
            *o = (__bf16)v;
        }
    }
}

// Split-K weight gradient: part[chunk][tap][co][ci] = sum over the chunk's pixels p of
// dout[p, co] * in[p + d(tap), ci].  One wavefront per (ci tile, co tile, tap, chunk).
__global__ __launch_bounds__(64) void k_conv3x3_wgrad(const __bf16 *__restrict__ in, int N, int H, int W, int Cin,
                                                      int in_cs, int in_co, const __bf16 *__restrict__ dout, int Cout,
                                                      int d_cs, int chunk, float *__restrict__ part)
{
    const int lane = threadIdx.x, m = lane & 31, half = lane >> 5;
    const int tiles_ci = Cin / 32;
    const int ci0 = (blockIdx.x % tiles_ci) * 32, co0 = (blockIdx.x / tiles_ci) * 32;
    const int tap = blockIdx.y, ck = blockIdx.z;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int npix = N * H * W;
    const int pbeg = ck * chunk, pend = min(npix, pbeg + chunk);
    f32x16 acc = {};
    for (int k0 = pbeg; k0 < pend; k0 += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int pk = k0 + 8 * half + i;
            const bool inr = pk < pend;
            // A[m = co][k = pixel]
            a[i] = inr ? dout[(int64_t)pk * d_cs + co0 + m] : (__bf16)0.0f;
            // B[k = pixel][n = ci]: input at the shifted pixel (zero outside)
            __bf16 bv = (__bf16)0.0f;
            if (inr) {
                const int n = pk / (H * W), rem = pk - n * (H * W);
                const int y = rem / W + dy, x = rem % W + dx;
                if (y >= 0 && y < H && x >= 0 && x < W)
                    bv = in[((int64_t)(n * H + y) * W + x) * in_cs + in_co + ci0 + m];
            }
            b[i] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    float *o = part + (((int64_t)ck * 9 + tap) * Cout) * Cin;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int co = co0 + 8 * (j >> 2) + 4 * half + (j & 3);
        o[(int64_t)co * Cin + ci0 + m] = acc[j];
    }
}

// MFMA operand of 8 consecutive pixels at one channel from a [pixel][channel] LDS tile,
// by two gfx950 transpose reads (ds_read_b64_tr_b16).  Within each 16-lane group, output
// lane t receives, in slot s, element t mod 4 of the 8-byte chunk addressed by group lane
// 4 s + t / 4.  So group lane i points at (pixel row + i / 4, channel + 4 (i mod 4)), and
// lane t gets 4 consecutive pixels of channel + t.  The caller passes the lane's address
// p = &tile[k0 + 8 (lane / 32) + (lane mod 16) / 4][32 tile + 16 ((lane / 16) mod 2) +
// 4 (lane mod 4)]; the second read starts 4 rows further.  The result is the MFMA layout:
// lane l holds rows m = l mod 32, k = 8 (l / 32) .. + 7.  The two halves are joined and
// reinterpreted as whole vectors: converting them element by element (bit-casting each
// short to __bf16) compiles, with this toolchain at -O3, to code that keeps only the first
// short of every pair.
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 tr_operand(const __bf16 *p, int row_stride)
{
    typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
    const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)p);
    const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(p + 4 * row_stride));
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

// LDS-staged weight gradient.  A sub-group of three wavefronts, one per kernel row
// (dy = -1, 0, 1), walks pixel blocks; a block is PB consecutive pixels of one image row.
// Per block it stages with 16-byte loads the output gradient dout[PB][32 CO_T] and the
// three input rows in[y-1 .. y+1][x0-1 .. x0+PB] (zero outside the image); then each
// wavefront contracts over the block's pixels for its three taps (dx = -1, 0, 1) and its
// CO_T x CI_T output tiles of 32 x 32, so each staged value feeds several MFMAs.  The
// contraction runs over pixels, which NHWC keeps strided: operands come out of the
// [pixel][channel] tiles by transpose reads (tr_operand); rows are padded by 8 elements.
// part[chunk * cstride + (tap Cout + co) Cin + ci] receives the chunk's sums
// (tap = 3 (dy + 1) + dx + 1).  The workgroups of the first input-channel
// tile also sum the staged output gradient over the chunk's pixels into
// bpart[chunk * cstride + co] (bias gradient), in a fixed order.
template <int PB, int CO_T, int CI_T>
__global__ __launch_bounds__(192) void k_wgrad_lds(const __bf16 *__restrict__ in, int N, int H, int W, int Cin,
                                                         int in_cs, int in_co, const __bf16 *__restrict__ dout, int Cout,
                                                         int d_cs, int blocks_per_chunk, float *__restrict__ part,
                                                         float *__restrict__ bpart, int64_t cstride)
{
    constexpr int XS = 32 * CI_T + 8;
    constexpr int DS = 32 * CO_T + 8;
    constexpr size_t XB = (size_t)3 * (PB + 2) * XS * 2, DB = (size_t)PB * DS * 2;
    __shared__ __attribute__((aligned(16))) unsigned char smem[XB + DB];
    __shared__ float bred[192][8];
    typedef __bf16 XRow[PB + 2][XS];
    typedef __bf16 DRow[DS];
    const int t = threadIdx.x, lane = t & 63, r = t >> 6;
    XRow *xs = (XRow *)smem;              // the three input rows
    DRow *ds = (DRow *)(smem + XB);       // and the output-gradient block
    const int m = lane & 31, half = lane >> 5;
    const int tiles_ci = Cin / (32 * CI_T);
    const int ci0 = (blockIdx.x % tiles_ci) * 32 * CI_T, co0 = (blockIdx.x / tiles_ci) * 32 * CO_T;
    const bool bias = bpart != nullptr && blockIdx.x % tiles_ci == 0;
    // transpose-read geometry (see tr_operand): pixel row and channel offsets of this lane
    const int tr_row = 8 * (lane >> 5) + ((lane & 15) >> 2);
    const int tr_col = 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
    float bsum[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) bsum[i] = 0.0f;
    const int ck = blockIdx.y;
    const int bpr = W / PB;
    const int64_t nblocks = (int64_t)N * H * bpr;
    const int64_t b0 = (int64_t)ck * blocks_per_chunk;
    const int64_t b1 = b0 + blocks_per_chunk < nblocks ? b0 + blocks_per_chunk : nblocks;
    f32x16 acc[3][CO_T][CI_T];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int a = 0; a < CO_T; ++a)
#pragma unroll
            for (int b = 0; b < CI_T; ++b)
#pragma unroll
                for (int j = 0; j < 16; ++j) acc[dx][a][b][j] = 0.0f;
    // Staging is software-pipelined: the global loads of the next block are issued into
    // registers before the MFMAs of the current block and written to LDS after them.
    constexpr int XV = 3 * (PB + 2) * 4 * CI_T;   // 16-byte input vectors per block
    constexpr int DV = PB * 4 * CO_T;             // 16-byte output-gradient vectors per block
    constexpr int NXV = (XV + 191) / 192, NDV = (DV + 191) / 192;
    bf16x8 xr[NXV], dr[NDV];
    auto fetch = [&](int64_t blk) {
        const bool ok = blk < b1;
        const int x0 = (int)(blk % bpr) * PB;
        const int64_t row = blk / bpr;   // n * H + y
        const int y = (int)(row % H);
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = t + 192 * i;
            const int c8 = v % (4 * CI_T), q = v / (4 * CI_T);
            const int px = q % (PB + 2), rr = q / (PB + 2);
            const int yy = y + rr - 1, xx = x0 + px - 1;
            const bool in_ok = ok && v < XV && yy >= 0 && yy < H && xx >= 0 && xx < W;
            xr[i] = load8(in_ok ? in + ((row + rr - 1) * W + xx) * in_cs + in_co + ci0 + 8 * c8 : kZero8);
        }
#pragma unroll
        for (int i = 0; i < NDV; ++i) {
            const int v = t + 192 * i;
            const int c8 = v % (4 * CO_T), px = v / (4 * CO_T);
            dr[i] = load8(ok && v < DV ? dout + (row * W + x0 + px) * d_cs + co0 + 8 * c8 : kZero8);
        }
    };
    if (b0 < b1) fetch(b0);
    for (int64_t blk = b0; blk < b1; ++blk) {
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = t + 192 * i;
            const int c8 = v % (4 * CI_T), q = v / (4 * CI_T);
            if (v < XV) *(bf16x8 *)&xs[q / (PB + 2)][q % (PB + 2)][8 * c8] = xr[i];
        }
        // 192 is a multiple of 4 CO_T: a thread keeps one group of 8 channels
#pragma unroll
        for (int i = 0; i < NDV; ++i) {
            const int v = t + 192 * i;
            const int c8 = v % (4 * CO_T), px = v / (4 * CO_T);
            if (v < DV) {
                *(bf16x8 *)&ds[px][8 * c8] = dr[i];
                if (bias) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) bsum[j] += (float)dr[i][j];
                }
            }
        }
        __syncthreads();
        if (blk + 1 < b1) fetch(blk + 1);
#pragma unroll
        for (int k0 = 0; k0 < PB; k0 += 16) {
            bf16x8 a[CO_T];
#pragma unroll
            for (int tt = 0; tt < CO_T; ++tt) a[tt] = tr_operand(&ds[k0 + tr_row][32 * tt + tr_col], DS);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
                for (int u = 0; u < CI_T; ++u) {
                    const bf16x8 b = tr_operand(&xs[r][k0 + tr_row + dx][32 * u + tr_col], XS);
#pragma unroll
                    for (int tt = 0; tt < CO_T; ++tt)
                        acc[dx][tt][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[tt], b, acc[dx][tt][u], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    if (bias) {
#pragma unroll
        for (int i = 0; i < 8; ++i) bred[t][i] = bsum[i];
        __syncthreads();
        if (t < 32 * CO_T) {
            const int c8 = t >> 3, i = t & 7;
            float s8 = 0.0f;
            for (int u = c8; u < 192; u += 4 * CO_T) s8 += bred[u][i];
            bpart[(int64_t)ck * cstride + co0 + 8 * c8 + i] = s8;
        }
    }
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        float *o = part + (int64_t)ck * cstride + ((int64_t)(3 * r + dx) * Cout) * Cin;
#pragma unroll
        for (int tt = 0; tt < CO_T; ++tt)
#pragma unroll
            for (int u = 0; u < CI_T; ++u)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int co = co0 + 32 * tt + 8 * (j >> 2) + 4 * half + (j & 3);
                    o[(int64_t)co * Cin + ci0 + 32 * u + m] = acc[dx][tt][u][j];
                }
    }
}

// Row-streaming weight gradient for one 32 x 32 (output channel, input channel) tile per
// workgroup.  dW[dy][dx][co][ci] = sum over output pixels q of dout[q][co] in[q + (dy, dx)][ci]
// is summed as sum over input pixels p of dout[p - (0, dx)][co] in[p + (dy, 0)][ci]: across
// the blocks of a row p covers [0, W) exactly, and the terms the substitution adds or drops
// have a zero factor (dout outside the image, or the convolution's zero padding).  The
// workgroup's four wavefronts walk a strip of output rows y0 .. y1-1 of one PB-pixel
// column; per row they stage the output-gradient row with a one-pixel halo and the next
// input row, which joins the two before it in a ring of three, so every input row is read
// from memory once per strip (plus two rows of halo).  Wavefront w takes the 16-pixel
// steps k0 = 16 (w + 4 i) of the row; per step it reads the three dx-shifted
// output-gradient operands and the three input rows' operands once and issues the nine tap
// products (A = output gradient, B = input, both by transpose reads).  The next row's loads
// are in flight during the current row's products, and the strip's first rows are requested
// together.  At the end the four wavefronts' sums are added in LDS in wavefront order, one
// kernel row (dy) at a time, and go to part[strip * cstride + (tap Cout + co) Cin + ci]; the
// workgroups of the first input-channel tile also write the strip's output-gradient sums to
// bpart (bias gradient).  The 1-D grid is split into eight contiguous ranges, one per XCD, so
// the workgroups of one strip (and its neighbours) share an L2.  Two workgroups of four
// wavefronts fit a CU (at most 256 registers per lane).
template <int PB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_wgrad_roll(
    const __bf16 *__restrict__ in, int N, int H, int W, int Cin, int in_cs, int in_co, const __bf16 *__restrict__ dout,
    int Cout, int d_cs, int rows_per_strip, float *__restrict__ part, float *__restrict__ bpart, int64_t cstride)
{
    static_assert(PB % 64 == 0, "four wavefronts of 16-pixel steps");
    constexpr int KPW = PB / 64;                       // steps per wavefront per row
    constexpr int RS = 40;                             // padded row stride (elements)
    constexpr int NDV = ((PB + 2) * 4 + 255) / 256;    // 16-byte output-gradient vectors per thread
    constexpr int NIV = (PB * 4 + 255) / 256;          // 16-byte input vectors per thread
    constexpr size_t STAGE = (size_t)(3 * PB + PB + 2) * RS * 2;
    constexpr size_t RED = (size_t)3 * 4 * 64 * 16 * 4;   // three taps x four wavefronts
    __shared__ __attribute__((aligned(16))) unsigned char smem[STAGE > RED ? STAGE : RED];
    __shared__ float bred[256][8];
    typedef __bf16 Row[RS];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63, m = lane & 31, half = lane >> 5;
    Row *is = (Row *)smem;         // input ring: slot s holds rows s PB .. s PB + PB - 1
    Row *ds = is + 3 * PB;         // output-gradient row, pixels x0 - 1 .. x0 + PB
    const int tiles_ci = Cin / 32, tiles = tiles_ci * (Cout / 32);
    const int bpr = W / PB, spc = (H + rows_per_strip - 1) / rows_per_strip;
    const int64_t total = (int64_t)tiles * N * bpr * spc;
    // XCD-contiguous order: block L runs on XCD L mod 8 and takes the (L / 8)-th item of
    // that XCD's range
    const int64_t L = blockIdx.x, q8 = total / 8, r8 = total % 8, x8 = L % 8;
    const int64_t item = x8 * q8 + (x8 < r8 ? x8 : r8) + L / 8;
    const int tile = (int)(item % tiles);
    const int64_t strip = item / tiles, col = strip / spc;
    const int ci0 = (tile % tiles_ci) * 32, co0 = (tile / tiles_ci) * 32;
    const bool bias = bpart != nullptr && tile % tiles_ci == 0;
    const int y0 = (int)(strip % spc) * rows_per_strip;
    const int y1 = y0 + rows_per_strip < H ? y0 + rows_per_strip : H;
    const int n = (int)(col / bpr), x0 = (int)(col % bpr) * PB;
    const int tr_row = 8 * (lane >> 5) + ((lane & 15) >> 2);
    const int tr_col = 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
    float bsum[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) bsum[i] = 0.0f;
    f32x16 acc[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[a][b][j] = 0.0f;
    bf16x8 dr[NDV], ir[NIV];
    // input row yy into v (zeros outside the image)
    auto fetch_in = [&](bf16x8 (&v)[NIV], int yy) {
#pragma unroll
        for (int i = 0; i < NIV; ++i) {
            const int e = t + 256 * i;
            const bool ok = e < PB * 4 && yy >= 0 && yy < H;
            v[i] = load8(ok ? in + (((int64_t)n * H + yy) * W + x0 + (e >> 2)) * in_cs + in_co + ci0 + 8 * (e & 3)
                            : kZero8);
        }
    };
    auto store_in = [&](const bf16x8 (&v)[NIV], int slot) {
#pragma unroll
        for (int i = 0; i < NIV; ++i) {
            const int e = t + 256 * i;
            if (e < PB * 4) *(bf16x8 *)&is[slot * PB + (e >> 2)][8 * (e & 3)] = v[i];
        }
    };
    // turn y: the output-gradient row y with its halo and the input row y + 1
    auto fetch = [&](int y) {
#pragma unroll
        for (int i = 0; i < NDV; ++i) {
            const int e = t + 256 * i;
            const int xx = x0 - 1 + (e >> 2);
            const bool ok = e < (PB + 2) * 4 && xx >= 0 && xx < W;
            dr[i] = load8(ok ? dout + (((int64_t)n * H + y) * W + xx) * d_cs + co0 + 8 * (e & 3) : kZero8);
        }
        fetch_in(ir, y + 1);
    };
    {   // prologue: input rows y0 - 1 and y0 into slots 0 and 1, the first turn's rows in flight
        bf16x8 p0[NIV], p1[NIV];
        fetch_in(p0, y0 - 1);
        fetch_in(p1, y0);
        fetch(y0);
        store_in(p0, 0);
        store_in(p1, 1);
    }
    for (int y = y0, k = 0; y < y1; ++y, ++k) {
        // rows y - 1, y, y + 1 sit in slots k, k + 1, k + 2 (mod 3)
        const int s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
#pragma unroll
        for (int i = 0; i < NDV; ++i) {
            const int e = t + 256 * i;
            if (e < (PB + 2) * 4) {
                *(bf16x8 *)&ds[e >> 2][8 * (e & 3)] = dr[i];
                if (bias && (e >> 2) >= 1 && (e >> 2) <= PB) {   // the halo belongs to other columns
#pragma unroll
                    for (int j = 0; j < 8; ++j) bsum[j] += (float)dr[i][j];
                }
            }
        }
        store_in(ir, s2);
        __syncthreads();
        if (y + 1 < y1) fetch(y + 1);
#pragma unroll
        for (int kk = 0; kk < KPW; ++kk) {
            const int k0 = 16 * (w + 4 * kk);
            bf16x8 a[3], b[3];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) a[dx] = tr_operand(&ds[k0 + 2 - dx + tr_row][tr_col], RS);
            b[0] = tr_operand(&is[s0 * PB + k0 + tr_row][tr_col], RS);
            b[1] = tr_operand(&is[s1 * PB + k0 + tr_row][tr_col], RS);
            b[2] = tr_operand(&is[s2 * PB + k0 + tr_row][tr_col], RS);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    acc[dy][dx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[dx], b[dy], acc[dy][dx], 0, 0, 0);
        }
        __syncthreads();
    }
    if (bias) {
#pragma unroll
        for (int i = 0; i < 8; ++i) bred[t][i] = bsum[i];
    }
    // the four wavefronts' sums, one kernel row at a time: wavefront u < 3 owns tap (dy, u)
    float *red = (float *)smem;   // [u][wavefront][j / 4][lane][4]
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        if (dy) __syncthreads();   // the previous row's owners have read red
#pragma unroll
        for (int u = 0; u < 3; ++u)
            if (u != w) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float4 v4 = {acc[dy][u][4 * q], acc[dy][u][4 * q + 1], acc[dy][u][4 * q + 2],
                                       acc[dy][u][4 * q + 3]};
                    *(float4 *)&red[(((u * 4 + w) * 4 + q) * 64 + lane) * 4] = v4;
                }
            }
        __syncthreads();
        if (w < 3) {
            f32x16 sum;
#pragma unroll
            for (int j = 0; j < 16; ++j) sum[j] = 0.0f;
#pragma unroll
            for (int w2 = 0; w2 < 4; ++w2) {
                if (w2 == w) {
#pragma unroll
                    for (int u = 0; u < 3; ++u)
                        if (u == w) {
#pragma unroll
                            for (int j = 0; j < 16; ++j) sum[j] += acc[dy][u][j];
                        }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float4 v4 = *(const float4 *)&red[(((w * 4 + w2) * 4 + q) * 64 + lane) * 4];
                        sum[4 * q] += v4.x;
                        sum[4 * q + 1] += v4.y;
                        sum[4 * q + 2] += v4.z;
                        sum[4 * q + 3] += v4.w;
                    }
                }
            }
            float *o = part + strip * cstride + ((int64_t)(3 * dy + w) * Cout) * Cin;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int co = co0 + 8 * (j >> 2) + 4 * half + (j & 3);
                o[(int64_t)co * Cin + ci0 + m] = sum[j];
            }
        }
    }
    if (bias) {
        __syncthreads();
        if (t < 32) {
            const int c8 = t >> 3, i = t & 7;
            float s8 = 0.0f;
            for (int u = c8; u < 256; u += 4) s8 += bred[u][i];
            bpart[strip * cstride + co0 + 8 * c8 + i] = s8;
        }
    }
}

// s[i] = sum_c part[c * stride + i] over c = 0 .. nchunk-1 for i < n, in a fixed order:
// a block of 256 threads covers 4 (256 / G) elements, as 256 / G groups of 4 consecutive
// elements (one 16-byte load) x G chunk groups; thread (e4, q) sums the chunks c = q,
// q + G, ... of its 4 elements in increasing c, then the G group sums of each element are
// added for q = 0 .. G-1.  s[i] goes to out[i] for i < na and to out_b[i - na] after
// (= or += with accumulate).  n, stride and na multiples of 4, part 16-byte aligned.
template <int G>
__global__ __launch_bounds__(256) void k_sum_chunks(const float *__restrict__ part, int64_t n, int64_t stride,
                                                    int nchunk, float *__restrict__ out, int64_t na,
                                                    float *__restrict__ out_b, int accumulate)
{
    constexpr int E4 = 256 / G;
    __shared__ float red[G][4 * E4 + 1];
    const int e4 = threadIdx.x % E4, q = threadIdx.x / E4;
    const int64_t i4 = ((int64_t)blockIdx.x * E4 + e4) * 4;
    float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (i4 < n) {
#pragma unroll 4
        for (int c = q; c < nchunk; c += G) {
            const float4 v = *(const float4 *)(part + (int64_t)c * stride + i4);
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
    }
    red[q][4 * e4] = s.x;
    red[q][4 * e4 + 1] = s.y;
    red[q][4 * e4 + 2] = s.z;
    red[q][4 * e4 + 3] = s.w;
    __syncthreads();
    const int e = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 4 * E4 + e;
    if (e < 4 * E4 && i < n) {
        float t = red[0][e];
#pragma unroll
        for (int k = 1; k < G; ++k) t += red[k][e];
        float *o = i < na ? out + i : out_b + (i - na);
        *o = accumulate ? *o + t : t;
    }
}

// Bias gradient partials: part[b][co] = sum of dout[p, co] over pixel block b (256 pixels).
__global__ __launch_bounds__(256) void k_bias_grad(const __bf16 *__restrict__ dout, int npix, int Cout, int d_cs,
                                                   float *__restrict__ part)
{
    const int co = threadIdx.x;
    if (co >= Cout) return;
    const int p0 = blockIdx.x * 256, p1 = min(npix, p0 + 256);
    float s = 0.0f;
    for (int p = p0; p < p1; ++p) s += (float)dout[(int64_t)p * d_cs + co];
    part[(int64_t)blockIdx.x * Cout + co] = s;
}

__global__ void k_relu_bwd(__bf16 *__restrict__ g, const __bf16 *__restrict__ act, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !((float)act[i] > 0.0f)) g[i] = (__bf16)0.0f;
}

// 2x2 average pooling and its adjoint (NHWC, C channels, contiguous).
// 2x2 average pooling of channels [ic0, ic0 + C) of in (channel stride in_cs) into out
// (C contiguous channels), and the adjoint into channels [dc0, dc0 + C) of din (stride
// d_cs; mask laid out as din).
__global__ void k_pool2(const __bf16 *__restrict__ in, int N, int H, int W, int C, int in_cs, int ic0,
                        __bf16 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int h = H / 2, w = W / 2;
    if (i >= (int64_t)N * h * w * C) return;
    const int c = i % C;
    const int64_t q = i / C;
    const int xo = q % w, yo = (q / w) % h, n = q / ((int64_t)w * h);
    const __bf16 *b = in + ((int64_t)(n * H + 2 * yo) * W + 2 * xo) * in_cs + ic0 + c;
    const float s = (float)b[0] + (float)b[in_cs] + (float)b[(int64_t)W * in_cs] + (float)b[(int64_t)W * in_cs + in_cs];
    out[i] = (__bf16)(0.25f * s);
}

__global__ void k_pool2_bwd(const __bf16 *__restrict__ dout, int N, int H, int W, int C, __bf16 *__restrict__ din,
                            int d_cs, int dc0, const __bf16 *__restrict__ mask, int accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * H * W * C) return;
    const int c = i % C;
    const int64_t q = i / C;
    const int x = q % W, y = (q / W) % H, n = q / ((int64_t)W * H);
    const int64_t e = q * d_cs + dc0 + c;
    float v = 0.25f * (float)dout[((int64_t)(n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
    if (mask && !((float)mask[e] > 0.0f)) v = 0.0f;
    din[e] = (__bf16)(accumulate ? (float)din[e] + v : v);
}

// Nearest-neighbour 2x upsampling of in (h x w) into channels [oc0, oc0 + C) of out
// (2h x 2w, channel stride out_cs), and the adjoint.
__global__ void k_up2(const __bf16 *__restrict__ in, int N, int h, int w, int C, __bf16 *__restrict__ out, int out_cs,
                      int oc0)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H = 2 * h, W = 2 * w;
    if (i >= (int64_t)N * H * W * C) return;
    const int c = i % C;
    const int64_t q = i / C;
    const int x = q % W, y = (q / W) % H, n = q / ((int64_t)W * H);
    out[q * out_cs + oc0 + c] = in[((int64_t)(n * h + y / 2) * w + x / 2) * C + c];
}

__global__ void k_up2_bwd(const __bf16 *__restrict__ dout, int N, int h, int w, int C, int d_cs, int dc0,
                          __bf16 *__restrict__ din)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * h * w * C) return;
    const int c = i % C;
    const int64_t q = i / C;
    const int x = q % w, y = (q / w) % h, n = q / ((int64_t)w * h);
    const int W = 2 * w;
    const int64_t b = ((int64_t)(n * 2 * h + 2 * y) * W + 2 * x);
    const float s = (float)dout[b * d_cs + dc0 + c] + (float)dout[(b + 1) * d_cs + dc0 + c] +
                    (float)dout[(b + W) * d_cs + dc0 + c] + (float)dout[(b + W + 1) * d_cs + dc0 + c];
    din[i] = (__bf16)s;
}

// dst[p, dc0 + c] (= or +=) src[p, sc0 + c], c < C: channel-slice copy (concatenation and its adjoint).
__global__ void k_slice(const __bf16 *__restrict__ src, int s_cs, int sc0, __bf16 *__restrict__ dst, int d_cs, int dc0,
                        int64_t npix, int C, int accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C) return;
    const int c = i % C;
    const int64_t p = i / C;
    const float v = (float)src[p * s_cs + sc0 + c];
    __bf16 *d = dst + p * d_cs + dc0 + c;
    *d = (__bf16)(accumulate ? (float)*d + v : v);
}

// 8-channel (16-byte) forms of the elementwise kernels above, used when every channel
// count, stride and offset is a multiple of 8 and the tensors are 16-byte aligned.
__device__ __forceinline__ void store8(__bf16 *p, const bf16x8 &v) { *(bf16x8 *)p = v; }

__global__ void k_relu_bwd8(__bf16 *__restrict__ g, const __bf16 *__restrict__ act, int64_t n8)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    bf16x8 gv = load8(g + 8 * i);
    const bf16x8 av = load8(act + 8 * i);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (!((float)av[k] > 0.0f)) gv[k] = (__bf16)0.0f;
    store8(g + 8 * i, gv);
}

// Row grid of the 8-channel resampling kernels: each block covers part of one pixel row
// (bpr blocks per row, `items` = row width x C / 8 threads' work per row), so the row,
// and with it the image and y, is uniform per block and a lane derives only its pixel and
// channel group, by a shift where C / 8 is a power of two (64-bit index division per lane
// made these kernels instruction-bound).
struct RowGrid {
    int bpr, items, C8, c8s;   // c8s = log2(C / 8), or -1
};

__device__ __forceinline__ bool row_item(const RowGrid &g, int &row, int &x, int &c)
{
    row = (int)blockIdx.x / g.bpr;
    const int j = ((int)blockIdx.x - row * g.bpr) * (int)blockDim.x + (int)threadIdx.x;
    if (j >= g.items) return false;
    x = g.c8s >= 0 ? j >> g.c8s : j / g.C8;
    c = 8 * (j - x * g.C8);
    return true;
}

// rows = N x h output rows of w pixels
__global__ void k_pool2_8(const __bf16 *__restrict__ in, const RowGrid g, int H, int W, int C, int in_cs, int ic0,
                          __bf16 *__restrict__ out)
{
    int row, xo, c;
    if (!row_item(g, row, xo, c)) return;
    const int h = H / 2, w = W / 2;
    const int n = row / h, yo = row - n * h;
    const __bf16 *b = in + ((int64_t)(n * H + 2 * yo) * W + 2 * xo) * in_cs + ic0 + c;
    const int64_t rs = (int64_t)W * in_cs;
    const bf16x8 a0 = load8(b), a1 = load8(b + in_cs), a2 = load8(b + rs), a3 = load8(b + rs + in_cs);
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (__bf16)(0.25f * ((float)a0[k] + (float)a1[k] + (float)a2[k] + (float)a3[k]));
    store8(out + ((int64_t)row * w + xo) * C + c, r);
}

// rows = N x H input rows of W pixels
__global__ void k_pool2_bwd8(const __bf16 *__restrict__ dout, const RowGrid g, int H, int W, int C,
                             __bf16 *__restrict__ din, int d_cs, int dc0, const __bf16 *__restrict__ mask, int accumulate)
{
    int row, x, c;
    if (!row_item(g, row, x, c)) return;
    const int n = row / H, y = row - n * H;
    const int64_t e = ((int64_t)row * W + x) * d_cs + dc0 + c;
    const bf16x8 d = load8(dout + ((int64_t)(n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
    bf16x8 r = accumulate ? load8(din + e) : zero8();
    const bf16x8 mk = mask ? load8(mask + e) : zero8();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float v = 0.25f * (float)d[k];
        if (mask && !((float)mk[k] > 0.0f)) v = 0.0f;
        r[k] = (__bf16)(accumulate ? (float)r[k] + v : v);
    }
    store8(din + e, r);
}

// rows = N x 2h output rows of 2w pixels
__global__ void k_up2_8(const __bf16 *__restrict__ in, const RowGrid g, int h, int w, int C, __bf16 *__restrict__ out,
                        int out_cs, int oc0)
{
    int row, x, c;
    if (!row_item(g, row, x, c)) return;
    const int H = 2 * h, W = 2 * w;
    const int n = row / H, y = row - n * H;
    store8(out + ((int64_t)row * W + x) * out_cs + oc0 + c, load8(in + ((int64_t)(n * h + y / 2) * w + x / 2) * C + c));
}

// rows = N x h output rows of w pixels
__global__ void k_up2_bwd8(const __bf16 *__restrict__ dout, const RowGrid g, int h, int w, int C, int d_cs, int dc0,
                           __bf16 *__restrict__ din)
{
    int row, x, c;
    if (!row_item(g, row, x, c)) return;
    const int n = row / h, y = row - n * h;
    const int W = 2 * w;
    const int64_t b = ((int64_t)(n * 2 * h + 2 * y) * W + 2 * x);
    const bf16x8 a0 = load8(dout + b * d_cs + dc0 + c), a1 = load8(dout + (b + 1) * d_cs + dc0 + c);
    const bf16x8 a2 = load8(dout + (b + W) * d_cs + dc0 + c), a3 = load8(dout + (b + W + 1) * d_cs + dc0 + c);
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (__bf16)((float)a0[k] + (float)a1[k] + (float)a2[k] + (float)a3[k]);
    store8(din + ((int64_t)row * w + x) * C + c, r);
}

__global__ void k_slice8(const __bf16 *__restrict__ src, int s_cs, int sc0, __bf16 *__restrict__ dst, int d_cs, int dc0,
                         int64_t npix, int C, int accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (i >= npix * C8) return;
    const int c = 8 * (int)(i % C8);
    const int64_t p = i / C8;
    const bf16x8 v = load8(src + p * s_cs + sc0 + c);
    __bf16 *d = dst + p * d_cs + dc0 + c;
    if (!accumulate) {
        store8(d, v);
        return;
    }
    bf16x8 r = load8(d);
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (__bf16)((float)r[k] + (float)v[k]);
    store8(d, r);
}

inline bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Weighted MSE over the first 4 channels of out (channel stride o_cs): per-block FP64
// partial of sum_c w_c (out_c - t_c)^2, and d out = 2 w_c (out_c - t_c) / npix (zero in
// the padding channels).
__global__ __launch_bounds__(256) void k_mse(const __bf16 *__restrict__ out, int o_cs, const float *__restrict__ target,
                                             int64_t npix, float w0, float w1, float w2, float w3,
                                             __bf16 *__restrict__ dout, double *__restrict__ part, int vec)
{
    __shared__ double sh[4];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc = 0.0;
    if (p < npix) {
        const float wc[4] = {w0, w1, w2, w3};
        if (vec) {   // 16-byte rows: the first vector carries the gradient, the rest zeros
            bf16x8 g = zero8();
            const bf16x8 o = load8(out + p * o_cs);
            const float4 t4 = *(const float4 *)(target + p * 4);
            const float tv[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float d = (float)o[c] - tv[c];
                acc += (double)wc[c] * (double)d * (double)d;
                g[c] = (__bf16)(2.0f * wc[c] * d / (float)npix);
            }
            store8(dout + p * o_cs, g);
            for (int c = 8; c < o_cs; c += 8) store8(dout + p * o_cs + c, zero8());
        } else {
            for (int c = 0; c < o_cs; ++c) {
                float g = 0.0f;
                if (c < 4) {
                    const float d = (float)out[p * o_cs + c] - target[p * 4 + c];
                    acc += (double)wc[c] * (double)d * (double)d;
                    g = 2.0f * wc[c] * d / (float)npix;
                }
                dout[p * o_cs + c] = (__bf16)g;
            }
        }
    }
    // fixed-order sums: a halving tree within each wavefront, then the four wavefront
    // sums in order
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) acc += __shfl_down(acc, s, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// out[0] = (sum of part[0 .. n)) / div: thread t sums part[t], part[t + 256], ... in order,
// then a fixed-order tree over the 256 thread sums (deterministic).
__global__ __launch_bounds__(256) void k_sum_f64(const double *__restrict__ part, int n, double div,
                                                 double *__restrict__ out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / div;
}

// Adam with bias correction on FP32 master weights.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2, float wd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] + wd * w[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP32 master weight w[9][Cout][Cin] -> BF16 forward copy wf[9][Cout_p][Cin_p] and the
// tap-flipped transpose for the data gradient wd[9][Cin_p][Cout_p] (zero padding).
__device__ __forceinline__ void cast_one(const float *__restrict__ w, int Cout, int Cin, int Cout_p, int Cin_p,
                                         __bf16 *__restrict__ wf, __bf16 *__restrict__ wd, int64_t i)
{
    const int ci = i % Cin_p;
    const int co = (i / Cin_p) % Cout_p;
    const int tap = i / ((int64_t)Cin_p * Cout_p);
    const float v = (co < Cout && ci < Cin) ? w[((int64_t)tap * Cout + co) * Cin + ci] : 0.0f;
    wf[i] = (__bf16)v;
    if (wd) wd[((int64_t)(8 - tap) * Cin_p + ci) * Cout_p + co] = (__bf16)v;
}

__global__ void k_cast_weights(const float *__restrict__ w, int Cout, int Cin, int Cout_p, int Cin_p,
                               __bf16 *__restrict__ wf, __bf16 *__restrict__ wd)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)9 * Cout_p * Cin_p) return;
    cast_one(w, Cout, Cin, Cout_p, Cin_p, wf, wd, i);
}

// Several layers in one launch: element i belongs to the layer k with start[k] <= i <
// start[k + 1] (start[k] = sum of 9 Cout_p Cin_p over the layers before k).
struct CastTable {
    ddf_nn_cast_layer l[DDF_NN_CAST_MAX_LAYERS];
    int64_t start[DDF_NN_CAST_MAX_LAYERS + 1];
    int n;
};

// Tiled form for layers whose padded channel counts are multiples of 32: one workgroup
// per (layer, tap, 32 output channels, 32 input channels) tile, which it reads and
// writes to wf along the input channels, then writes transposed to wd along the output
// channels through LDS, so both stores are coalesced (the per-element form scatters its
// wd stores Cout_p elements apart).  tstart[k] = start[k] / 1024.
__global__ __launch_bounds__(256) void k_cast_weight_tiles(const CastTable t)
{
    __shared__ float tile[32][33];
    const int64_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < t.n && b >= t.start[k + 1] / 1024) ++k;
    const ddf_nn_cast_layer &L = t.l[k];
    const int local = (int)(b - t.start[k] / 1024);
    const int nci = L.Cin_p / 32, nco = L.Cout_p / 32;
    const int cit = local % nci, cot = (local / nci) % nco, tap = local / (nci * nco);
    const int lane = threadIdx.x & 31, row = threadIdx.x >> 5;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int co = 32 * cot + row + 8 * r, ci = 32 * cit + lane;
        const float v = (co < L.Cout && ci < L.Cin) ? L.w[((int64_t)tap * L.Cout + co) * L.Cin + ci] : 0.0f;
        ((__bf16 *)L.wf)[((int64_t)tap * L.Cout_p + co) * L.Cin_p + ci] = (__bf16)v;
        tile[row + 8 * r][lane] = v;
    }
    if (!L.wd) return;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ci = 32 * cit + row + 8 * r, co = 32 * cot + lane;
        ((__bf16 *)L.wd)[((int64_t)(8 - tap) * L.Cin_p + ci) * L.Cout_p + co] = (__bf16)tile[lane][row + 8 * r];
    }
}

__global__ void k_cast_weights_multi(const CastTable t)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.start[t.n]) return;
    int k = 0;
    while (k + 1 < t.n && i >= t.start[k + 1]) ++k;
    const ddf_nn_cast_layer &L = t.l[k];
    cast_one(L.w, L.Cout, L.Cin, L.Cout_p, L.Cin_p, (__bf16 *)L.wf, (__bf16 *)L.wd, i - t.start[k]);
}

// Network input for lid-driven cavities: channel 0 wall mask (1 next to a fixed wall,
// 2 next to the lid), channel 1 (log Re - log Re_lo) / (log Re_hi - log Re_lo), channel
// 2 U / U_ref, channels 3..C-1 zero.  re, u: per-sample values.
__device__ __forceinline__ float cavity_channel(int c, int px, int py, int W, int H, float lre, float un)
{
    switch (c) {
    case 0: return py == H - 1 ? 2.0f : ((px == 0 || px == W - 1 || py == 0) ? 1.0f : 0.0f);   // lid 2, walls 1
    case 1: return lre;
    case 2: return un;
    // node coordinates in [0, 1]: the receptive field of the network is smaller than
    // the cavity, so position is an input rather than something inferred from walls
    case 3: return W > 1 ? (float)px / (float)(W - 1) : 0.0f;
    case 4: return H > 1 ? (float)py / (float)(H - 1) : 0.0f;
    default: return 0.0f;
    }
}

// One thread per (pixel, group of 8 channels) writing 16 bytes (C % 8 == 0, x 16-byte
// aligned), or per pixel with single stores (vec == 0).
__global__ void k_cavity_inputs(const float *__restrict__ re, const float *__restrict__ u, int N, int H, int W, int C,
                                float lre_lo, float lre_hi, float u_ref, __bf16 *__restrict__ x, int vec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int per = vec ? C / 8 : 1;
    if (i >= (int64_t)N * H * W * per) return;
    const int64_t pix = i / per;
    const int grp = (int)(i - pix * per);
    const int px = pix % W, py = (pix / W) % H, n = pix / ((int64_t)W * H);
    const float lre = (logf(re[n]) - lre_lo) / (lre_hi - lre_lo), un = u[n] / u_ref;
    if (vec) {
        bf16x8 v;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (__bf16)cavity_channel(8 * grp + k, px, py, W, H, lre, un);
        store8(x + pix * C + 8 * grp, v);
    } else {
        for (int c = 0; c < C; ++c) x[pix * C + c] = (__bf16)cavity_channel(c, px, py, W, H, lre, un);
    }
}

// The same on a grid of pixel rows (C % 8 == 0, x 16-byte aligned): each block takes its
// row (image, y) once, a lane its pixel and group of 8 channels by a shift, so no lane
// divides 64-bit indices.
__global__ void k_cavity_inputs8(const float *__restrict__ re, const float *__restrict__ u, const RowGrid g, int H,
                                 int W, int C, float lre_lo, float lre_hi, float u_ref, __bf16 *__restrict__ x)
{
    int row, px, c;
    if (!row_item(g, row, px, c)) return;
    const int n = row / H, py = row - n * H;
    const float lre = (logf(re[n]) - lre_lo) / (lre_hi - lre_lo), un = u[n] / u_ref;
    bf16x8 v;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (__bf16)cavity_channel(c + k, px, py, W, H, lre, un);
    store8(x + ((int64_t)row * W + px) * C + c, v);
}

// Normalised training targets from steady fields (dense FP64 [N][H][W] each):
// (u / U, v / U, (rho - 1) / U^2, phi).
__global__ void k_cavity_targets(const double *__restrict__ rho, const double *__restrict__ ux,
                                 const double *__restrict__ uy, const double *__restrict__ phi,
                                 const float *__restrict__ u, int N, int HW, float *__restrict__ t)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * HW) return;
    const float U = u[i / HW];
    t[i * 4 + 0] = (float)(ux[i] / U);
    t[i * 4 + 1] = (float)(uy[i] / U);
    t[i * 4 + 2] = (float)((rho[i] - 1.0) / ((double)U * U));
    t[i * 4 + 3] = (float)phi[i];
}

// Network output (channel stride o_cs) -> physical FP64 fields for a warm start.
__global__ void k_cavity_fields(const __bf16 *__restrict__ out, int o_cs, const float *__restrict__ u, int N, int HW,
                                double *__restrict__ rho, double *__restrict__ ux, double *__restrict__ uy,
                                double *__restrict__ phi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * HW) return;
    const double U = u[i / HW];
    const __bf16 *o = out + i * o_cs;
    ux[i] = U * (double)(float)o[0];
    uy[i] = U * (double)(float)o[1];
    rho[i] = 1.0 + U * U * (double)(float)o[2];
    phi[i] = (double)(float)o[3];
}

inline int blocks_for(int64_t n, int t = 256) { return (int)((n + t - 1) / t); }

// Row grid of `width` pixels x C channels per row (C a multiple of 8), 256-thread blocks.
inline RowGrid row_grid(int width, int C)
{
    RowGrid g;
    g.C8 = C / 8;
    g.items = width * g.C8;
    g.bpr = (g.items + 255) / 256;
    g.c8s = (g.C8 & (g.C8 - 1)) == 0 ? __builtin_ctz((unsigned)g.C8) : -1;
    return g;
}

// The row grid's block count and per-row indices fit in 32 bits.
inline bool row_grid_fits(int64_t rows, int64_t width, int64_t C)
{
    const int64_t items = width * (C / 8), bpr = (items + 255) / 256;
    return rows * bpr < ((int64_t)1 << 31) && bpr * 256 < ((int64_t)1 << 31);
}

// Fixed-order sum of nchunk partial vectors of n floats, stride apart (n, stride and na
// multiples of 4, 16-byte aligned); the first na sums go to out, the rest to out_b.
void sum_chunks(const float *part, int64_t n, int64_t stride, int nchunk, float *out, int64_t na, float *out_b,
                int accumulate, hipStream_t st)
{
    if (nchunk >= 128)
        hipLaunchKernelGGL(k_sum_chunks<32>, dim3(blocks_for(n, 32)), dim3(256), 0, st, part, n, stride, nchunk, out,
                           na, out_b, accumulate);
    else
        hipLaunchKernelGGL(k_sum_chunks<8>, dim3(blocks_for(n, 128)), dim3(256), 0, st, part, n, stride, nchunk, out,
                           na, out_b, accumulate);
}

constexpr int64_t kWgradWaves = 8192;    // target single-wave workgroups of the gather kernel
// LDS-staged weight gradient: split over pixels into about kWgradGroups three-wave
// workgroups, but with the split-K partials (written once, read once by the sum) held
// to kWgradPartFrac of the bytes the workgroups read.  Deep layers have few pixels and
// large 9 x Cout x Cin partials, so there the cap, not the fill target, sets the split.
#ifndef DDF_WGRAD_GROUPS
#define DDF_WGRAD_GROUPS 768
#endif
#ifndef DDF_WGRAD_PART_FRAC
#define DDF_WGRAD_PART_FRAC 1.0
#endif
constexpr int64_t kWgradGroups = DDF_WGRAD_GROUPS;
// row-streaming weight gradient: at most this many workgroups where strips of 8 or more
// rows allow it
constexpr int64_t kWgradRollBlocks = 512;
constexpr double kWgradPartFrac = DDF_WGRAD_PART_FRAC;

int check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DDF_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return DDF_OK;
}

}  // namespace

extern "C" {

int ddf_nn_conv3x3(const void *in, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t in_cs, int32_t in_co,
                   const void *wt, const float *bias, void *out, int32_t Cout, int32_t out_cs, int32_t out_co,
                   int32_t relu, int32_t accumulate, const void *mask, int32_t mask_cs, int32_t mask_co, void *stream)
{
    const int64_t npix = (int64_t)N * H * W;
    if (!in || !wt || !out || N <= 0 || H <= 0 || W <= 0) return fail(DDF_ERR_ARG, "conv3x3: bad tensor arguments");
    if (Cin % 16 || Cout % 32 || in_cs % 8 || in_co % 8 || out_cs < out_co + Cout || in_cs < in_co + Cin)
        return fail(DDF_ERR_ARG, "conv3x3: need Cin % 16 == 0, Cout % 32 == 0, 8-aligned channel strides and offsets");
    if (npix % 32) return fail(DDF_ERR_ARG, "conv3x3: N*H*W must be a multiple of 32");
    if (npix > (int64_t)1 << 30) return fail(DDF_ERR_ARG, "conv3x3: too many pixels");
    if (mask && (mask_co < 0 || mask_cs < mask_co + Cout))
        return fail(DDF_ERR_ARG, "conv3x3: the mask's channel stride and offset must cover the output channels");
    const __bf16 *mk = (const __bf16 *)mask;
    hipStream_t st = (hipStream_t)stream;
    const __bf16 *i = (const __bf16 *)in;
    const __bf16 *w = (const __bf16 *)wt;
    __bf16 *o = (__bf16 *)out;
    const bool lds = Cin % 32 == 0 && al16(in) && al16(wt);
#define DDF_CONV_LDS(PB, NCO)                                                                                      \
    hipLaunchKernelGGL((k_conv3x3_lds<PB, NCO>), dim3((unsigned)(npix / PB), (unsigned)(Cout / (32 * NCO))), dim3(256), \
                       0, st, i, N, H, W, Cin, in_cs, in_co, w, bias, o, Cout, out_cs, out_co, relu, accumulate, mk,       \
                       mask_cs, mask_co)
#define DDF_CONV_ROWS(PB, R, WCO, PD)                                                                              \
    do {                                                                                                          \
        hipLaunchKernelGGL((k_conv3x3_rows<PB, R, WCO, PD>), dim3((unsigned)(npix / ((PB) * (R))), (unsigned)(Cout / (32 * (WCO)))), \
                           dim3(256), 0, st, i, N, H, W, Cin, in_cs, in_co, w, bias, o, Cout, out_cs, out_co, relu,     \
                           accumulate, mk, mask_cs, mask_co);                                                        \
        return check_launch();                                                                                    \
    } while (0)
    // Row streaming where it beat the LDS-staged kernel on the surrogate's layers at batch 8
    // (forward and data gradient, 8 x 256^2 .. 8 x 32^2; the other shapes keep the LDS kernel):
    // 32 or 96 output channels at widths of 128 and more (1-8% faster; not with 64 input
    // channels); 64 or 192 output channels at those widths (10-26%); 128 or 384 output
    // channels from 128 or more input channels at width 64 (2-19%); 64 output channels at
    // width 64 (5%); 256 output channels at width 32 (10-15%).
    if (lds && W % 128 == 0 && H % 4 == 0) {
        if ((Cout == 32 || Cout == 96) && Cin != 64) DDF_CONV_ROWS(128, 4, 1, 2);
        if (Cout == 64 && Cin >= 128) DDF_CONV_ROWS(128, 4, 2, 2);
        if (Cout == 64 || Cout == 192) DDF_CONV_ROWS(64, 4, 2, 2);
    }
    if (lds && W == 64 && H % 2 == 0) {
        if (Cout % 128 == 0 && Cin >= 128) DDF_CONV_ROWS(64, 2, 4, 4);
        if (Cout == 64) DDF_CONV_ROWS(64, 2, 2, 4);
    }
    if (lds && W == 32 && H % 2 == 0 && Cout % 256 == 0) DDF_CONV_ROWS(32, 2, 4, 4);
#undef DDF_CONV_ROWS
    if (lds && W % 64 == 0 && Cout % 128 == 0) DDF_CONV_LDS(64, 4);
    else if (lds && W % 64 == 0 && Cout % 64 == 0) DDF_CONV_LDS(64, 2);
    else if (lds && W % 32 == 0 && Cout % 128 == 0) DDF_CONV_LDS(32, 4);
    else if (lds && W % 256 == 0 && Cin == 32 && Cout == 32) DDF_CONV_LDS(256, 1);
    else if (lds && W % 128 == 0) DDF_CONV_LDS(128, 1);
    else if (Cout % 64 == 0 && npix % 64 == 0)
        hipLaunchKernelGGL((k_conv3x3<2, 2>), dim3(npix / 64, Cout / 64), dim3(256), 0, st, i, N, H, W, Cin, in_cs,
                           in_co, w, bias, o, Cout, out_cs, out_co, relu, accumulate, mk, mask_cs, mask_co);
    else if (npix % 128 == 0)
        hipLaunchKernelGGL((k_conv3x3<4, 1>), dim3(npix / 128, Cout / 32), dim3(256), 0, st, i, N, H, W, Cin, in_cs,
                           in_co, w, bias, o, Cout, out_cs, out_co, relu, accumulate, mk, mask_cs, mask_co);
    else
        hipLaunchKernelGGL((k_conv3x3<1, 1>), dim3(npix / 32, Cout / 32), dim3(64), 0, st, i, N, H, W, Cin, in_cs,
                           in_co, w, bias, o, Cout, out_cs, out_co, relu, accumulate, mk, mask_cs, mask_co);
#undef DDF_CONV_LDS
    return check_launch();
}

}  // extern "C"

namespace {

// How ddf_nn_conv3x3_wgrad splits its work; the workspace size follows from it.
struct WgradPlan {
    bool roll;             // row-streaming kernel (rows of W % 64 == 0 pixels)
    bool lds;              // LDS-staged kernel (rows of W % 16 == 0 pixels)
    int pb, co_t, ci_t;    // pixel block, and the LDS-staged kernel's tile multiples
    int64_t nchunk;        // split-K chunks (partials): strips of the row-streaming kernel
    int64_t per_chunk;     // output rows (row-streaming kernel), pixel blocks (LDS-staged
                           // kernel) or pixels (gather kernel) per chunk
};

WgradPlan wgrad_plan(int N, int H, int W, int Cin, int Cout)
{
    WgradPlan P{};
    const int64_t npix = (int64_t)N * H * W;
    if (W % 64 == 0) {
        // Strips of 8, 16, 32, ... rows: the shortest that leave at most kWgradRollBlocks
        // workgroups (two per CU).  At batch 8 this is the fastest strip length measured
        // for every surrogate layer at widths 64 to 256 (32 -> 32 at 256^2: 8 rows, 512
        // workgroups; 384 -> 128 at 64^2: 64 rows, 384): more and shorter strips add
        // partials and per-strip start-up, fewer leave CUs idle.
        P.roll = true;
        P.pb = W % 128 == 0 ? 128 : 64;
        const int64_t tiles = (int64_t)(Cin / 32) * (Cout / 32), cols = (int64_t)N * (W / P.pb);
        int64_t rows = 8;
        while (rows < H && cols * ((H + rows - 1) / rows) * tiles > kWgradRollBlocks) rows *= 2;
        P.per_chunk = std::min<int64_t>(rows, H);
        P.nchunk = cols * ((H + P.per_chunk - 1) / P.per_chunk);
        return P;
    }
    P.pb = W % 32 == 0 ? 32 : (W % 16 == 0 ? 16 : 0);
    P.lds = P.pb > 0;
    if (P.lds) {
        // Two output-channel tiles per wavefront where there are pixels enough to fill the
        // chip from the pixel split alone; on small images (at most 32768 pixels) single
        // tiles win: more workgroups, and at 204 or fewer registers two wavefronts per
        // SIMD.  Two input-channel tiles (336 registers, one wavefront per
        // SIMD) measured slower at every layer size of the surrogate network.
        P.co_t = npix > 32768 && Cout % 64 == 0 ? 2 : 1;
        P.ci_t = 1;
        const int64_t groups = (int64_t)(Cin / (32 * P.ci_t)) * (Cout / (32 * P.co_t));
        const int64_t nblocks = npix / P.pb;
        // about kWgradGroups three-wavefront workgroups; half as many, with twice the pixels
        // each, where several channel tiles split a large image (64 -> 64 and 192 -> 64 at
        // 8 x 128^2 with 64-pixel blocks: 8-22% faster)
        const int64_t target = groups >= 2 && npix >= 131072 ? kWgradGroups / 2 : kWgradGroups;
        // bytes read: each workgroup stages its input-channel and output-channel slices
        const double reads = 2.0 * (double)npix *
                             ((double)Cin * (Cout / (32 * P.co_t)) + (double)Cout * (Cin / (32 * P.ci_t)));
        const double part_chunk = 4.0 * ((double)9 * Cout * Cin + Cout);
        const int64_t cap = std::max<int64_t>(1, (int64_t)std::min(kWgradPartFrac * reads / part_chunk, 1e15));
        int64_t nchunk = (target + groups - 1) / groups;
        nchunk = std::max<int64_t>(1, std::min<int64_t>({nchunk, cap, nblocks}));
        P.per_chunk = (nblocks + nchunk - 1) / nchunk;
        P.nchunk = (nblocks + P.per_chunk - 1) / P.per_chunk;
    } else {
        // gather kernel: about kWgradWaves single-wave workgroups, chunks of >= 256 pixels
        const int64_t tiles = (int64_t)std::max(1, Cin / 32) * std::max(1, Cout / 32);
        int64_t nchunk = (kWgradWaves + 9 * tiles - 1) / (9 * tiles);
        nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, (npix + 255) / 256));
        int64_t chunk = (npix + nchunk - 1) / nchunk;
        chunk = (chunk + 15) / 16 * 16;
        P.per_chunk = chunk;
        P.nchunk = (npix + chunk - 1) / chunk;
    }
    return P;
}

template <int PB>
int launch_wgrad_lds(const WgradPlan &P, const __bf16 *in, int N, int H, int W, int Cin, int in_cs, int in_co,
                     const __bf16 *dout, int Cout, int d_cs, float *part, float *bpart, int64_t cstride,
                     hipStream_t st)
{
    const dim3 grid((unsigned)((Cin / (32 * P.ci_t)) * (Cout / (32 * P.co_t))), (unsigned)P.nchunk);
    const int bpc = (int)P.per_chunk;
#define DDF_WGRAD_LAUNCH(CO, CI)                                                                              \
    hipLaunchKernelGGL((k_wgrad_lds<PB, CO, CI>), grid, dim3(192), 0, st, in, N, H, W, Cin, in_cs, in_co, dout, Cout, \
                       d_cs, bpc, part, bpart, cstride)
    if (P.co_t == 2) DDF_WGRAD_LAUNCH(2, 1);
    else DDF_WGRAD_LAUNCH(1, 1);
#undef DDF_WGRAD_LAUNCH
    return DDF_OK;
}

}  // namespace

extern "C" {

size_t ddf_nn_wgrad_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t *chunk_out)
{
    const int64_t npix = (int64_t)N * H * W;
    const WgradPlan P = wgrad_plan(N, H, W, Cin, Cout);
    if (chunk_out) *chunk_out = (int32_t)(P.roll || P.lds ? P.per_chunk * P.pb : P.per_chunk);
    const int64_t wsz = (int64_t)9 * Cout * Cin;
    if (P.roll || P.lds) return (size_t)(P.nchunk * (wsz + Cout)) * sizeof(float);
    const int64_t bsz = ((npix + 255) / 256) * Cout;
    return (size_t)std::max(P.nchunk * wsz, bsz) * sizeof(float);
}

int ddf_nn_conv3x3_wgrad(const void *in, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t in_cs, int32_t in_co,
                         const void *dout, int32_t Cout, int32_t d_cs, float *dw, float *db, int32_t accumulate,
                         void *workspace, void *stream)
{
    if (!in || !dout || !dw || !workspace) return fail(DDF_ERR_ARG, "wgrad: null pointer");
    if (N <= 0 || H <= 0 || W <= 0) return fail(DDF_ERR_ARG, "wgrad: bad shape");
    if (Cin % 32 || Cout % 32) return fail(DDF_ERR_ARG, "wgrad: Cin and Cout must be multiples of 32");
    if (Cout > 256) return fail(DDF_ERR_ARG, "wgrad: Cout must be at most 256");
    if (((uintptr_t)in | (uintptr_t)dout | (uintptr_t)workspace) & 15)
        return fail(DDF_ERR_ARG, "wgrad: tensors and workspace must be 16-byte aligned");
    if (in_cs % 8 || in_co % 8 || d_cs % 8 || in_cs < in_co + Cin || d_cs < Cout)
        return fail(DDF_ERR_ARG, "wgrad: channel strides and offsets must be multiples of 8 and cover the channels");
    hipStream_t st = (hipStream_t)stream;
    const WgradPlan P = wgrad_plan(N, H, W, Cin, Cout);
    const int64_t npix = (int64_t)N * H * W;
    float *part = (float *)workspace;
    const __bf16 *ib = (const __bf16 *)in, *db16 = (const __bf16 *)dout;
    const int64_t wsz = (int64_t)9 * Cout * Cin;
    if (P.roll) {
        // strip c holds its weight partials, then (with db) its bias partials
        const int64_t cs = wsz + (db ? Cout : 0);
        float *bpart = db ? part + wsz : nullptr;
        const dim3 grid((unsigned)(P.nchunk * (Cin / 32) * (Cout / 32)));
        const int rows = (int)P.per_chunk;
        if (P.pb == 128)
            hipLaunchKernelGGL(k_wgrad_roll<128>, grid, dim3(256), 0, st, ib, N, H, W, Cin, in_cs, in_co, db16, Cout, d_cs,
                               rows, part, bpart, cs);
        else
            hipLaunchKernelGGL(k_wgrad_roll<64>, grid, dim3(256), 0, st, ib, N, H, W, Cin, in_cs, in_co, db16, Cout, d_cs,
                               rows, part, bpart, cs);
        sum_chunks(part, cs, cs, (int)P.nchunk, dw, wsz, db, accumulate, st);
        return check_launch();
    }
    if (P.lds) {
        // chunk c holds its weight partials, then (with db) its bias partials
        const int64_t cs = wsz + (db ? Cout : 0);
        float *bpart = db ? part + wsz : nullptr;
        if (P.pb == 32) launch_wgrad_lds<32>(P, ib, N, H, W, Cin, in_cs, in_co, db16, Cout, d_cs, part, bpart, cs, st);
        else launch_wgrad_lds<16>(P, ib, N, H, W, Cin, in_cs, in_co, db16, Cout, d_cs, part, bpart, cs, st);
        sum_chunks(part, cs, cs, (int)P.nchunk, dw, wsz, db, accumulate, st);
        return check_launch();
    }
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3((Cin / 32) * (Cout / 32), 9, (unsigned)P.nchunk), dim3(64), 0, st, ib, N, H,
                       W, Cin, in_cs, in_co, db16, Cout, d_cs, (int)P.per_chunk, part);
    sum_chunks(part, wsz, wsz, (int)P.nchunk, dw, wsz, nullptr, accumulate, st);
    if (db) {
        const int nb = (int)((npix + 255) / 256);
        hipLaunchKernelGGL(k_bias_grad, dim3(nb), dim3(256), 0, st, db16, (int)npix, Cout, d_cs, part);
        sum_chunks(part, (int64_t)Cout, (int64_t)Cout, nb, db, (int64_t)Cout, nullptr, accumulate, st);
    }
    return check_launch();
}

int ddf_nn_relu_bwd(void *grad, const void *act, int64_t n, void *stream)
{
    if (!grad || !act) return fail(DDF_ERR_ARG, "relu_bwd: null pointer");
    if (n % 8 == 0 && al16(grad) && al16(act))
        hipLaunchKernelGGL(k_relu_bwd8, dim3(blocks_for(n / 8)), dim3(256), 0, (hipStream_t)stream, (__bf16 *)grad,
                           (const __bf16 *)act, n / 8);
    else
        hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, (__bf16 *)grad,
                           (const __bf16 *)act, n);
    return check_launch();
}

int ddf_nn_pool2(const void *in, int32_t N, int32_t H, int32_t W, int32_t C, int32_t in_cs, int32_t in_co, void *out,
                 void *stream)
{
    if (!in || !out || N <= 0 || H <= 0 || W <= 0 || C <= 0) return fail(DDF_ERR_ARG, "pool2: bad tensor arguments");
    if (H % 2 || W % 2) return fail(DDF_ERR_ARG, "pool2: H and W must be even");
    if (in_co < 0 || in_cs < in_co + C) return fail(DDF_ERR_ARG, "pool2: the channel stride must cover the channels");
    if (C % 8 == 0 && in_cs % 8 == 0 && in_co % 8 == 0 && al16(in) && al16(out) &&
        row_grid_fits((int64_t)N * (H / 2), W / 2, C)) {
        const RowGrid g = row_grid(W / 2, C);
        hipLaunchKernelGGL(k_pool2_8, dim3((unsigned)(N * (H / 2) * g.bpr)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)in, g, H, W, C, in_cs, in_co, (__bf16 *)out);
    }
    else
        hipLaunchKernelGGL(k_pool2, dim3(blocks_for((int64_t)N * H * W * C / 4)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)in, N, H, W, C, in_cs, in_co, (__bf16 *)out);
    return check_launch();
}

int ddf_nn_pool2_bwd(const void *dout, int32_t N, int32_t H, int32_t W, int32_t C, void *din, int32_t din_cs,
                     int32_t din_co, const void *mask, int32_t accumulate, void *stream)
{
    if (!dout || !din || N <= 0 || H <= 0 || W <= 0 || C <= 0) return fail(DDF_ERR_ARG, "pool2_bwd: bad tensor arguments");
    if (H % 2 || W % 2) return fail(DDF_ERR_ARG, "pool2_bwd: H and W must be even");
    if (din_co < 0 || din_cs < din_co + C) return fail(DDF_ERR_ARG, "pool2_bwd: the channel stride must cover the channels");
    const __bf16 *mk = (const __bf16 *)mask;
    if (C % 8 == 0 && din_cs % 8 == 0 && din_co % 8 == 0 && al16(dout) && al16(din) && (!mask || al16(mask)) &&
        row_grid_fits((int64_t)N * H, W, C)) {
        const RowGrid g = row_grid(W, C);
        hipLaunchKernelGGL(k_pool2_bwd8, dim3((unsigned)(N * H * g.bpr)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)dout, g, H, W, C, (__bf16 *)din, din_cs, din_co, mk, accumulate);
    }
    else
        hipLaunchKernelGGL(k_pool2_bwd, dim3(blocks_for((int64_t)N * H * W * C)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)dout, N, H, W, C, (__bf16 *)din, din_cs, din_co, mk, accumulate);
    return check_launch();
}

int ddf_nn_up2(const void *in, int32_t N, int32_t h, int32_t w, int32_t C, void *out, int32_t out_cs, int32_t out_co,
               void *stream)
{
    if (C % 8 == 0 && out_cs % 8 == 0 && out_co % 8 == 0 && al16(in) && al16(out) &&
        row_grid_fits((int64_t)N * 2 * h, 2 * (int64_t)w, C)) {
        const RowGrid g = row_grid(2 * w, C);
        hipLaunchKernelGGL(k_up2_8, dim3((unsigned)(N * 2 * h * g.bpr)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)in, g, h, w, C, (__bf16 *)out, out_cs, out_co);
    }
    else
        hipLaunchKernelGGL(k_up2, dim3(blocks_for((int64_t)N * 4 * h * w * C)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)in, N, h, w, C, (__bf16 *)out, out_cs, out_co);
    return check_launch();
}

int ddf_nn_up2_bwd(const void *dout, int32_t N, int32_t h, int32_t w, int32_t C, int32_t d_cs, int32_t d_co, void *din,
                   void *stream)
{
    if (C % 8 == 0 && d_cs % 8 == 0 && d_co % 8 == 0 && al16(dout) && al16(din) && row_grid_fits((int64_t)N * h, w, C)) {
        const RowGrid g = row_grid(w, C);
        hipLaunchKernelGGL(k_up2_bwd8, dim3((unsigned)(N * h * g.bpr)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)dout, g, h, w, C, d_cs, d_co, (__bf16 *)din);
    }
    else
        hipLaunchKernelGGL(k_up2_bwd, dim3(blocks_for((int64_t)N * h * w * C)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)dout, N, h, w, C, d_cs, d_co, (__bf16 *)din);
    return check_launch();
}

int ddf_nn_slice(const void *src, int32_t s_cs, int32_t s_co, void *dst, int32_t d_cs, int32_t d_co, int64_t npix,
                 int32_t C, int32_t accumulate, void *stream)
{
    if (C % 8 == 0 && s_cs % 8 == 0 && s_co % 8 == 0 && d_cs % 8 == 0 && d_co % 8 == 0 && al16(src) && al16(dst))
        hipLaunchKernelGGL(k_slice8, dim3(blocks_for(npix * C / 8)), dim3(256), 0, (hipStream_t)stream,
                           (const __bf16 *)src, s_cs, s_co, (__bf16 *)dst, d_cs, d_co, npix, C, accumulate);
    else
        hipLaunchKernelGGL(k_slice, dim3(blocks_for(npix * C)), dim3(256), 0, (hipStream_t)stream, (const __bf16 *)src,
                           s_cs, s_co, (__bf16 *)dst, d_cs, d_co, npix, C, accumulate);
    return check_launch();
}

size_t ddf_nn_mse_workspace_bytes(int64_t npix) { return (size_t)((npix + 255) / 256 + 1) * sizeof(double); }

int ddf_nn_mse(const void *out, int32_t o_cs, const float *target, int64_t npix, const float *weights4, void *dout,
               double *loss_dev, void *workspace, void *stream)
{
    if (o_cs < 4) return fail(DDF_ERR_ARG, "mse: at least 4 output channels");
    if (npix < 1 || npix > ((int64_t)1 << 40)) return fail(DDF_ERR_ARG, "mse: npix must be in [1, 2^40]");
    if (!out || !target || !weights4 || !dout || !loss_dev || !workspace) return fail(DDF_ERR_ARG, "mse: null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int nb = (int)((npix + 255) / 256);
    double *part = (double *)workspace;
    const int vec = o_cs % 8 == 0 && al16(out) && al16(dout) && al16(target);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, (const __bf16 *)out, o_cs, target, npix, weights4[0],
                       weights4[1], weights4[2], weights4[3], (__bf16 *)dout, part, vec);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, part, nb, (double)npix, loss_dev);
    return check_launch();
}

}  // extern "C"

// ddf_nn_mse_static keeps its partial sums in this file-scope device array instead of a
// caller workspace: one copy per GPU, held until the process ends.  In host code the
// name stands for a host-side shadow, so kernels get the device address that
// hipGetSymbolAddress returns for the current device (looked up once per device).
constexpr size_t kMseScratchBytes = (size_t)64 << 10;
static __device__ __align__(256) unsigned char scratch[kMseScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

int mse_scratch(void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    DDF_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DDF_ERR_UNSUPPORTED, "mse_static: device index beyond 63");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        DDF_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(DDF_ERR_HIP, "mse_static: no device address for the scratch array");
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return DDF_OK;
}

}  // namespace

extern "C" {

size_t ddf_nn_mse_static_max_pixels(void) { return (kMseScratchBytes / sizeof(double) - 1) * 256; }

int ddf_nn_mse_static(const void *out, int32_t o_cs, const float *target, int64_t npix, const float *weights4,
                      void *dout, double *loss_dev, void *stream)
{
    if (npix > (int64_t)ddf_nn_mse_static_max_pixels() || ddf_nn_mse_workspace_bytes(npix) > kMseScratchBytes)
        return fail(DDF_ERR_ARG, "mse_static: npix exceeds ddf_nn_mse_static_max_pixels() (" +
                                     std::to_string(ddf_nn_mse_static_max_pixels()) + ")");
    void *ws = nullptr;
    const int rc = mse_scratch(&ws);
    if (rc != DDF_OK) return rc;
    return ddf_nn_mse(out, o_cs, target, npix, weights4, dout, loss_dev, ws, stream);
}

int ddf_nn_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2, float eps,
                int64_t step, float weight_decay, void *stream)
{
    if (step < 1) return fail(DDF_ERR_ARG, "adam: step counts from 1");
    const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, n, lr, beta1, beta2,
                       eps, c1, c2, weight_decay);
    return check_launch();
}

int ddf_nn_cast_weights(const float *w, int32_t Cout, int32_t Cin, int32_t Cout_p, int32_t Cin_p, void *wf, void *wd,
                        void *stream)
{
    if (Cout_p < Cout || Cin_p < Cin) return fail(DDF_ERR_ARG, "cast_weights: padded sizes smaller than the real ones");
    hipLaunchKernelGGL(k_cast_weights, dim3(blocks_for((int64_t)9 * Cout_p * Cin_p)), dim3(256), 0, (hipStream_t)stream,
                       w, Cout, Cin, Cout_p, Cin_p, (__bf16 *)wf, (__bf16 *)wd);
    return check_launch();
}

int ddf_nn_cast_weights_multi(int32_t n, const ddf_nn_cast_layer *layers, void *stream)
{
    if (n < 1 || n > DDF_NN_CAST_MAX_LAYERS || !layers)
        return fail(DDF_ERR_ARG, "cast_weights_multi: need 1 to DDF_NN_CAST_MAX_LAYERS layers");
    CastTable t{};
    t.n = n;
    t.start[0] = 0;
    for (int k = 0; k < n; ++k) {
        const ddf_nn_cast_layer &L = layers[k];
        if (!L.w || !L.wf || L.Cout < 1 || L.Cin < 1 || L.Cout_p < L.Cout || L.Cin_p < L.Cin)
            return fail(DDF_ERR_ARG, "cast_weights_multi: layer " + std::to_string(k) +
                                         " has a null pointer or padded sizes smaller than the real ones");
        t.l[k] = L;
        t.start[k + 1] = t.start[k] + (int64_t)9 * L.Cout_p * L.Cin_p;
    }
    bool tiled = true;
    for (int k = 0; k < n; ++k) tiled = tiled && layers[k].Cout_p % 32 == 0 && layers[k].Cin_p % 32 == 0;
    if (tiled && t.start[n] / 1024 < ((int64_t)1 << 31))
        hipLaunchKernelGGL(k_cast_weight_tiles, dim3((unsigned)(t.start[n] / 1024)), dim3(256), 0,
                           (hipStream_t)stream, t);
    else
        hipLaunchKernelGGL(k_cast_weights_multi, dim3(blocks_for(t.start[n])), dim3(256), 0, (hipStream_t)stream, t);
    return check_launch();
}

int ddf_nn_cavity_inputs(const float *re, const float *u, int32_t N, int32_t H, int32_t W, int32_t C, float re_lo,
                         float re_hi, float u_ref, void *x, void *stream)
{
    if (C < 5) return fail(DDF_ERR_ARG, "cavity_inputs: at least 5 channels");
    if (N < 0 || H < 1 || W < 1) return fail(DDF_ERR_ARG, "cavity_inputs: bad shape");
    const int vec = C % 8 == 0 && al16(x);
    if (N == 0) return DDF_OK;
    if (vec && row_grid_fits((int64_t)N * H, W, C)) {
        const RowGrid g = row_grid(W, C);
        hipLaunchKernelGGL(k_cavity_inputs8, dim3((unsigned)(N * H * g.bpr)), dim3(256), 0, (hipStream_t)stream, re, u, g,
                           H, W, C, std::log(re_lo), std::log(re_hi), u_ref, (__bf16 *)x);
        return check_launch();
    }
    hipLaunchKernelGGL(k_cavity_inputs, dim3(blocks_for((int64_t)N * H * W * (vec ? C / 8 : 1))), dim3(256), 0,
                       (hipStream_t)stream, re, u, N, H, W, C, std::log(re_lo), std::log(re_hi), u_ref, (__bf16 *)x, vec);
    return check_launch();
}

int ddf_nn_cavity_targets(const double *rho, const double *ux, const double *uy, const double *phi, const float *u,
                          int32_t N, int32_t HW, float *t, void *stream)
{
    hipLaunchKernelGGL(k_cavity_targets, dim3(blocks_for((int64_t)N * HW)), dim3(256), 0, (hipStream_t)stream, rho, ux,
                       uy, phi, u, N, HW, t);
    return check_launch();
}

int ddf_nn_cavity_fields(const void *out, int32_t o_cs, const float *u, int32_t N, int32_t HW, double *rho, double *ux,
                         double *uy, double *phi, void *stream)
{
    hipLaunchKernelGGL(k_cavity_fields, dim3(blocks_for((int64_t)N * HW)), dim3(256), 0, (hipStream_t)stream,
                       (const __bf16 *)out, o_cs, u, N, HW, rho, ux, uy, phi);
    return check_launch();
}

}  // extern "C"
