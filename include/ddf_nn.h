/*
 * ddf_nn.h - C ABI of the surrogate-network kernels in libddf (MI355X, gfx950).
 *
 * The surrogate is a 2D U-Net that maps a lid-driven cavity's wall mask, Reynolds
 * number and lid speed to its steady fields (u, v, rho, phi); its prediction
 * warm-starts the lattice Boltzmann solver, which alone decides convergence.  It is
 * not part of the paper's method (arXiv:1908.06742); these entry points are the
 * building blocks its forward pass, backward pass and training step are made of.
 *
 * Conventions (in addition to those of ddf.h):
 *   - Activations are NHWC tensors of bf16 (2-byte) elements with a channel stride
 *     ("cs") that may exceed the channel count, so a call can read or write a channel
 *     slice starting at a channel offset ("co").  Channel strides and offsets are
 *     multiples of 8 and base pointers 16-byte aligned.
 *   - Convolution weights are FP32 masters w[9][Cout][Cin] (tap = 3 ky + kx, ky, kx in
 *     0..2, padding 1) cast by ddf_nn_cast_weights to bf16 copies; accumulation is FP32.
 *   - All calls are asynchronous on `stream`; none allocates memory.
 */
#ifndef DDF_NN_H
#define DDF_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out[p, out_co + co] = act(bias[co] + sum_{tap, ci} in[p + d(tap), in_co + ci] w[tap][co][ci])
 * (or += when accumulate).  wt: bf16 [9][Cout][Cin] from ddf_nn_cast_weights; bias may be
 * NULL; relu = 1 applies max(., 0).  Requires Cin % 16 == 0, Cout % 32 == 0,
 * N*H*W % 32 == 0.  With the tap-flipped transposed weight (the `wd` copy) and the
 * output gradient as input, the same call computes the data gradient.  mask (may be NULL,
 * bf16, mask_cs >= mask_co + Cout): the value for (p, co) is set to zero where
 * mask[p * mask_cs + mask_co + co] is not > 0, before it is added with accumulate.  With
 * the forward input of a layer whose input is a ReLU output as the mask, the data
 * gradient comes out multiplied by the ReLU's derivative (the ReLU adjoint is linear, so
 * each contribution to a gradient can be masked on its own). */
int ddf_nn_conv3x3(const void *in, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t in_cs, int32_t in_co,
                   const void *wt, const float *bias, void *out, int32_t Cout, int32_t out_cs, int32_t out_co,
                   int32_t relu, int32_t accumulate, const void *mask, int32_t mask_cs, int32_t mask_co,
                   void *stream);

/* Bytes of workspace ddf_nn_conv3x3_wgrad needs; *chunk receives its pixel chunk (pixels
 * per split-K partial). */
size_t ddf_nn_wgrad_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t Cout, int32_t *chunk);
/* dw[tap][co][ci] (= or +=) sum_p dout[p, co] in[p + d(tap), in_co + ci] in FP32, with
 * split-K partials summed in a fixed order (deterministic); db[co] (= or +=)
 * sum_p dout[p, co] if db is not NULL.  Requires Cin % 32 == 0, Cout % 32 == 0,
 * Cout <= 256, channel strides and offsets multiples of 8, and 16-byte aligned tensors
 * and workspace (else DDF_ERR_ARG).  Rows of W % 16 == 0 pixels take the LDS-staged
 * kernel, others a gather kernel. */
int ddf_nn_conv3x3_wgrad(const void *in, int32_t N, int32_t H, int32_t W, int32_t Cin, int32_t in_cs, int32_t in_co,
                         const void *dout, int32_t Cout, int32_t d_cs, float *dw, float *db, int32_t accumulate,
                         void *workspace, void *stream);

/* grad[i] = 0 where act[i] <= 0 (n contiguous elements). */
int ddf_nn_relu_bwd(void *grad, const void *act, int64_t n, void *stream);
/* 2x2 average pooling of channels [in_co, in_co + C) of in (channel stride in_cs) into out
 * (C contiguous channels), and its adjoint into channels [din_co, din_co + C) of din
 * (stride din_cs): din = or += dout / 4, each child's value set to zero where mask, laid
 * out as din, is not > 0 (mask may be NULL).  A skip connection's tensor can so live
 * inside the concatenation buffer that the decoder reads.  H and W even, strides covering
 * the channels (else DDF_ERR_ARG). */
int ddf_nn_pool2(const void *in, int32_t N, int32_t H, int32_t W, int32_t C, int32_t in_cs, int32_t in_co, void *out,
                 void *stream);
int ddf_nn_pool2_bwd(const void *dout, int32_t N, int32_t H, int32_t W, int32_t C, void *din, int32_t din_cs,
                     int32_t din_co, const void *mask, int32_t accumulate, void *stream);
/* Nearest 2x upsampling of in (h x w, C contiguous channels) into a channel slice of out,
 * and its adjoint (sum of the four children) from a channel slice of dout. */
int ddf_nn_up2(const void *in, int32_t N, int32_t h, int32_t w, int32_t C, void *out, int32_t out_cs, int32_t out_co,
               void *stream);
int ddf_nn_up2_bwd(const void *dout, int32_t N, int32_t h, int32_t w, int32_t C, int32_t d_cs, int32_t d_co, void *din,
                   void *stream);
/* dst[p, d_co + c] (= or +=) src[p, s_co + c] for c < C: concatenation and its adjoint. */
int ddf_nn_slice(const void *src, int32_t s_cs, int32_t s_co, void *dst, int32_t d_cs, int32_t d_co, int64_t npix,
                 int32_t C, int32_t accumulate, void *stream);

/* Weighted squared error per pixel of the first 4 channels of out against target
 * (FP32 [npix][4]): *loss_dev = (1/npix) sum_p sum_c w_c (out - t)^2 (FP64, device
 * memory) and its gradient dout = 2 w_c (out - t) / npix (zero in channels >= 4).
 * weights4: host array.  workspace: ddf_nn_mse_workspace_bytes(npix) bytes. */
size_t ddf_nn_mse_workspace_bytes(int64_t npix);
int ddf_nn_mse(const void *out, int32_t o_cs, const float *target, int64_t npix, const float *weights4, void *dout,
               double *loss_dev, void *workspace, void *stream);

/* ddf_nn_mse for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc): the same
 * kernels and results, with the partial sums in a fixed 64 KiB device array of the
 * library instead of a workspace, so npix is limited to ddf_nn_mse_static_max_pixels()
 * (2,096,896; DDF_ERR_ARG beyond).  The call allocates nothing; its first call on a
 * device looks the array up (hipGetSymbolAddress) with that device current.  Each GPU
 * has one such array, shared by every call on it: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be serialised by the
 * caller. */
size_t ddf_nn_mse_static_max_pixels(void);
int ddf_nn_mse_static(const void *out, int32_t o_cs, const float *target, int64_t npix, const float *weights4,
                      void *dout, double *loss_dev, void *stream);

/* Adam with bias correction (step counts from 1) and decoupled-free L2 weight decay
 * added to the gradient. */
int ddf_nn_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2, float eps,
                int64_t step, float weight_decay, void *stream);
/* FP32 w[9][Cout][Cin] -> bf16 wf[9][Cout_p][Cin_p] and (if wd) the tap-flipped transpose
 * wd[9][Cin_p][Cout_p] used for the data gradient; padding entries are zero. */
int ddf_nn_cast_weights(const float *w, int32_t Cout, int32_t Cin, int32_t Cout_p, int32_t Cin_p, void *wf, void *wd,
                        void *stream);
/* One layer of ddf_nn_cast_weights_multi: the arguments of ddf_nn_cast_weights (device
 * pointers; wd may be NULL). */
typedef struct {
    const float *w;
    void *wf;
    void *wd;
    int32_t Cout, Cin, Cout_p, Cin_p;
} ddf_nn_cast_layer;
#define DDF_NN_CAST_MAX_LAYERS 32
/* ddf_nn_cast_weights for n layers (1 <= n <= DDF_NN_CAST_MAX_LAYERS, else DDF_ERR_ARG) in
 * one launch: a network's casts after each optimizer step.  `layers` is a host array,
 * read during the call (passed to the kernel by value). */
int ddf_nn_cast_weights_multi(int32_t n, const ddf_nn_cast_layer *layers, void *stream);

/* Lid-driven cavity inputs [N][H][W][C], C >= 5: wall mask (1 next to a fixed wall, 2 next
 * to the lid at y = H - 1), (log Re - log re_lo) / (log re_hi - log re_lo), U / u_ref,
 * x / (W - 1), y / (H - 1), then zeros. */
int ddf_nn_cavity_inputs(const float *re, const float *u, int32_t N, int32_t H, int32_t W, int32_t C, float re_lo,
                         float re_hi, float u_ref, void *x, void *stream);
/* Targets [N][H][W][4] = (u / U, v / U, (rho - 1) / U^2, phi) from dense FP64 fields. */
int ddf_nn_cavity_targets(const double *rho, const double *ux, const double *uy, const double *phi, const float *u,
                          int32_t N, int32_t HW, float *t, void *stream);
/* Inverse map of a network output (channel stride o_cs) to FP64 fields for a warm start. */
int ddf_nn_cavity_fields(const void *out, int32_t o_cs, const float *u, int32_t N, int32_t HW, double *rho, double *ux,
                         double *uy, double *phi, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DDF_NN_H */
