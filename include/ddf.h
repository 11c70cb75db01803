/*
 * ddf.h - C ABI of libddf, the MI355X (gfx950) implementation of the
 * double-distribution-function lattice Boltzmann method with local vorticity
 * (Hajabdollahi & Premnath, arXiv:1908.06742).
 *
 * Two coupled D2Q9 lattices are advanced together:
 *   - a fluid lattice f with the MRT collision in the natural raw-moment basis and
 *     the trapezoidal body-force source (Sec. 2, eqs. MRT-LBEfluidmotion_transformed,
 *     eqmrawmoment, the sigma' source list, hydrodynamic_fields);
 *   - a passive-scalar lattice g with the MRT collision whose third-order
 *     off-diagonal equilibria carry the anisotropy beta1 != beta2 (Sec. 3,
 *     eqs. MRT-LBECDE, eqmrawmoment_CDE), or the SRT variant (App. B) or the
 *     central-moment variants (App. C, App. D).
 * The strain rate, spin, vorticity and scalar gradient are then extracted node by
 * node from the second-order non-equilibrium moments of both lattices (Sec. 4,
 * eqs. crossderivativeRHS1/2, offdiagvelderivativeresult1/2,
 * diagvelderivativeresult1/2, vorticityexpression).
 *
 * Conventions for every entry point:
 *   - All buffers are device memory allocated and owned by the caller; the library
 *     never frees them.  The handle owns host-side state only.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *     Calls are asynchronous on that stream except ddf_reduce, ddf_batch_reduce and
 *     ddf_batch_step_reduce, which synchronise it to return host values.
 *   - Return value: DDF_OK or a negative ddf_status.  No exception or abort crosses
 *     the ABI; ddf_last_error() returns a thread-local message for the last error.
 *   - Lattice units throughout (dx = dt = 1, Sec. 5).  Node (i, j) sits at x = i,
 *     y = j; half-way walls lie at x = -1/2, x = nx - 1/2, y = -1/2, y = ny - 1/2.
 *   - Dense field arrays are row-major [ny][nx] (x fastest).
 */
#ifndef DDF_H
#define DDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Population storage format.  Populations are stored as offsets from the rest
 * equilibrium, (f - f_eq(rho0, 0)) * pop_scale and (g - g_eq(phi0, 0)) * pop_scale;
 * F64 computes in double, the others in float.  F16 and BF16 round to nearest even.
 * BF16_SR stores bfloat16 with stochastic rounding: each stored population rounds up
 * with probability equal to the dropped fraction of an ulp, decided by a counter-based
 * hash of (slot, time step) whose two 16-bit halves serve the f and g lattices, so the
 * stored values are unbiased and a run is reproducible (also across a checkpoint
 * resume at the same step). */
typedef enum { DDF_F64 = 0, DDF_F32 = 1, DDF_F16 = 2, DDF_BF16 = 3, DDF_BF16_SR = 4 } ddf_storage;

typedef enum {
    DDF_OK = 0,
    DDF_ERR_ARG = -1,          /* invalid argument (message says which) */
    DDF_ERR_UNSUPPORTED = -2,  /* valid request the library does not support */
    DDF_ERR_HIP = -3,          /* a HIP runtime call failed */
    DDF_ERR_NONFINITE = -4,    /* the state holds NaN or Inf */
    DDF_ERR_STATE = -5         /* call out of order (e.g. step before init) */
} ddf_status;

enum { DDF_SIDE_LEFT = 0, DDF_SIDE_RIGHT = 1, DDF_SIDE_BOTTOM = 2, DDF_SIDE_TOP = 3 };

/* Body force F(x, t): none; uniform (force[0], force[1]); four-rolls mill of Sec. 5.2,
 * F = force[0] (sin k i sin k j, cos k i cos k j) with k = force_k; pulsatile of
 * Sec. 5.3, F = (force[0], force[1]) cos(force_omega t). */
enum { DDF_FORCE_NONE = 0, DDF_FORCE_UNIFORM = 1, DDF_FORCE_FOURROLL = 2, DDF_FORCE_PULSATILE = 3 };

/* Scalar collision: MRT (Sec. 3), SRT (App. B), cascaded (App. C), non-cascaded
 * central moments (App. D). */
enum { DDF_SCALAR_MRT = 0, DDF_SCALAR_SRT = 1, DDF_SCALAR_CASCADED = 2, DDF_SCALAR_CENTRAL = 3 };

/* Output planes of ddf_extract, in this order; bit k of the mask selects plane k.
 * A_ij = d_j u_i (Sec. 1); S_xy = N_xy / 2; Omega_xy = -wz / 2.  The planar
 * invariants Q, R and the Lamb vector L = omega x u are those of Sec. 1 with
 * omega = (0, 0, wz). */
enum {
    DDF_OUT_RHO = 0, DDF_OUT_UX, DDF_OUT_UY, DDF_OUT_PHI,
    DDF_OUT_SXX, DDF_OUT_SYY, DDF_OUT_SXY, DDF_OUT_WZ,
    DDF_OUT_DXUY, DDF_OUT_DYUX, DDF_OUT_DXPHI, DDF_OUT_DYPHI,
    DDF_OUT_Q, DDF_OUT_R, DDF_OUT_LX, DDF_OUT_LY,
    DDF_NUM_OUTPUTS
};

/* Row layout of the population planes.  Row-major: node x of a row at column x, rows
 * padded to a multiple of 64 elements.  x-interleaved: the row is 64 sub-rows of
 * Q = nx / 64 nodes, node x at column (x mod 64) Q + x / 64, so the 64 nodes of a
 * wavefront are consecutive in memory and their x +- 1 neighbours sit at the same lanes
 * of the adjacent sub-row (whole aligned cache lines in both streaming parities; the step
 * kernels then load and store non-temporally).  It needs nx = 64 * 2^k with nx / 64 at
 * least one 128-byte line of the storage type (nx >= 1024 in F64, 2048 in F32, 4096 in
 * 16-bit storage).  Packed: row-major rows of exactly nx elements with no padding, each
 * direction plane rounded up to 64 elements (so that planes start on a 128-byte line).
 * For a single lattice AUTO takes x-interleaved rows where the width allows them and the
 * two population arrays exceed 256 MB (they stream from HBM), else row-major; packed
 * rows only on request.  Batches always keep packed rows (AUTO or PACKED;
 * DDF_ERR_UNSUPPORTED for ROW and INTERLEAVED), which their flat tiles stream as whole
 * lines.  The layout is internal: every entry point reads and writes fields and
 * populations in the logical [ny][nx] order, and results are the same bit for bit in
 * every layout (stochastic rounding included; reduction sums up to their summation
 * order). */
enum { DDF_LAYOUT_AUTO = 0, DDF_LAYOUT_ROW = 1, DDF_LAYOUT_INTERLEAVED = 2, DDF_LAYOUT_PACKED = 3 };

/* Statistics returned by ddf_reduce (all from one FP64 pass over the state). */
enum {
    DDF_STAT_MASS = 0,        /* sum of rho */
    DDF_STAT_SCALAR,          /* sum of phi */
    DDF_STAT_RES_U,           /* |u^n - u^(n-K)|_2 / (K |u^n|_2), K = steps since the last reduce */
    DDF_STAT_RES_PHI,         /* same for phi */
    DDF_STAT_NONFINITE,       /* number of nodes with a non-finite rho, u or phi */
    DDF_STAT_STEPS,           /* K */
    DDF_STAT_UMAX,            /* max |u| */
    DDF_STAT_PHIMIN,          /* min phi */
    DDF_NUM_STATS
};

typedef struct {
    int32_t nx, ny;              /* nodes; nx, ny >= 2 */
    int32_t periodic_x;          /* 1 = periodic in x, 0 = half-way walls at x = -1/2, nx - 1/2 */
    int32_t periodic_y;          /* same in y */
    int32_t storage;             /* ddf_storage */
    int32_t scalar_model;        /* DDF_SCALAR_* */
    double omega[9];             /* fluid rates diag(0,0,0,w3..w8) (Sec. 2, eq. relaxationtimematrix_fluidmotion); [0..2] ignored */
    double omega_phi[9];         /* scalar rates diag(0,w1..w8) (Sec. 3, eq. relaxationtimematrix_CDE); [0] ignored.
                                    SRT uses omega_phi[1] for every population. */
    double beta1, beta2;         /* scalar-flux anisotropy; |beta1 - beta2| must exceed 1e-12 */
    double cs2, cs2_phi;         /* c_s^2 and c_sphi^2 (1/3 in the paper) */
    double wall_u[4][2];         /* wall velocity per side (DDF_SIDE_*); used where that side is a wall */
    double wall_phi[4];          /* Dirichlet scalar per side; NaN = zero-flux wall */
    int32_t force_kind;          /* DDF_FORCE_* */
    int32_t layout;              /* DDF_LAYOUT_*: row layout of the population planes (single lattices) */
    double force[2];
    double force_k;
    double force_omega;
    double rho0, phi0;           /* offset references of the population storage */
    double pop_scale;            /* power-of-two storage scale; 0 = library default (256 for F16, else 1) */
    double phi_min;              /* |phi| < phi_min: wz, dxuy, dyux, Q, R, L are NaN (the phi = 0 singularity of Sec. 4) */
} ddf_params;

typedef struct ddf_handle ddf_handle;

/* Row pitch in elements of every population plane: nx rounded up to 64, or nx for
 * DDF_LAYOUT_PACKED. */
int64_t ddf_pitch(const ddf_params *p);
/* Elements from one direction plane to the next: pitch * ny rounded up to 64. */
int64_t ddf_plane_stride(const ddf_params *p);
/* Bytes of one lattice's populations: 9 planes of ddf_plane_stride storage elements.
 * The caller allocates two such buffers (f and g). */
size_t ddf_population_bytes(const ddf_params *p);
/* Bytes of device workspace ddf_create needs (residual snapshot and reduction partials). */
size_t ddf_workspace_bytes(const ddf_params *p);

/* Validate p (tau > 1/2 equivalents: 0 < omega < 2 for omega3..8 and omega1^phi..8^phi,
 * beta1 != beta2, nx, ny >= 2, known storage/model/force/layout) and bind the caller's
 * buffers.  pop_f, pop_g: ddf_population_bytes(p) each; workspace:
 * ddf_workspace_bytes(p); all 256-byte aligned.  *out receives the handle.
 * DDF_ERR_UNSUPPORTED for DDF_LAYOUT_INTERLEAVED on a width that does not allow it. */
int ddf_create(const ddf_params *p, void *pop_f, void *pop_g, void *workspace, ddf_handle **out);
void ddf_destroy(ddf_handle *h);

/* Equilibrium initial state from dense FP64 device fields rho, ux, uy, phi
 * ([ny][nx] each): f = T^-1 (m_eq(rho, u) - S(F(x, 0), u) / 2), g = T^-1 n_eq(phi, u),
 * so that the velocity recovered with the half-force shift (Sec. 2,
 * eq. hydrodynamic_fields) equals u.  Resets the step counter to 0. */
int ddf_init_equilibrium(ddf_handle *h, const double *rho, const double *ux, const double *uy,
                         const double *phi, void *stream);

/* Advance nsteps >= 0 time steps.  Per step and node: the fluid populations are
 * collided in raw-moment space with the trapezoidal body-force source (Sec. 2,
 * eq. MRT-LBEfluidmotion_transformed with eqs. eqmrawmoment, relaxationtimematrix_fluidmotion
 * and the sigma' source list), the scalar populations with the anisotropic MRT
 * collision (Sec. 3, eq. MRT-LBECDE with eqs. eqmrawmoment_CDE, relaxationtimematrix_CDE),
 * or the SRT (App. B) or central-moment (App. C, App. D) variant selected by
 * scalar_model; both lattices are then streamed in place (the AA pattern: even steps
 * write a node's post-collision populations into its own opposite slots, odd steps into
 * the neighbours' natural slots), with half-way walls, moving walls and Dirichlet scalar
 * walls applied as the populations are written.  Asynchronous on `stream`;
 * DDF_ERR_STATE before ddf_init_equilibrium or ddf_set_populations. */
int ddf_step(ddf_handle *h, int64_t nsteps, void *stream);

/* Local kinematics of the current state (pre-collision populations at the current
 * step, Sec. 4) into out: DDF_NUM_OUTPUTS dense planes of ny * nx elements of type
 * out_dtype (0 = double, 1 = float); only planes whose bit is set in mask are written. */
int ddf_extract(ddf_handle *h, void *out, uint32_t mask, int32_t out_dtype, void *stream);

/* FP64 statistics of the current state into out[DDF_NUM_STATS] (host memory), and a
 * new residual snapshot.  Synchronises the stream.  Returns DDF_ERR_NONFINITE (with
 * out filled) when any node is non-finite. */
int ddf_reduce(ddf_handle *h, double *out, void *stream);

/* Logical populations of the current state, direction-major dense [9][ny][nx].
 * dtype 0: absolute values as double; dtype 1: the raw stored offsets in the storage
 * type (bitwise checkpoint). */
int ddf_get_populations(ddf_handle *h, void *f, void *g, int32_t dtype, void *stream);
/* Inverse of ddf_get_populations; the step counter becomes `step`. */
int ddf_set_populations(ddf_handle *h, const void *f, const void *g, int32_t dtype, int64_t step, void *stream);

/* Tile shape of every kernel of this lattice: tiles are min(bx_max, row length rounded
 * up to a power of two) nodes wide and 512 / width rows tall, one workgroup each
 * (bx_max = 64, 128, 256 or 512; DDF_ERR_ARG otherwise).  Results do not depend on it.
 * The default is 512 for lattices whose two population arrays fit in 256 MB, else 128
 * for 8- and 4-byte storage and 64 for 2-byte storage. */
int ddf_set_tile_width(ddf_handle *h, int32_t bx_max);
int32_t ddf_get_tile_width(const ddf_handle *h);
/* Width of the lane offsets of the step kernels: 32 (the default where a population
 * plane is below 4 GiB; DDF_ERR_ARG for a larger plane) or 64 (any size).  With 32 a
 * plane's base is shared by the wavefront and each address is one 32-bit byte offset,
 * which holds fewer registers per thread.  Results do not depend on it (bit for bit);
 * the call drops a captured graph like ddf_set_tile_width. */
int ddf_set_address_width(ddf_handle *h, int32_t bits);
int32_t ddf_get_address_width(const ddf_handle *h);
/* Resident step workgroups per CU for the even and the odd step: 0 (as many as the
 * registers allow, 4 for most kernels), 1, 2 or 3 (DDF_ERR_ARG otherwise), enforced by
 * reserving LDS the kernels do not use.  Defaults: lattices whose two population
 * arrays exceed 256 MB take 1 / 1 in FP64, 1 / 1 in FP32 (2 / 2 with walls), and 3 / 2
 * (with 64-bit offsets) in FP16 and BF16 (round to nearest) when they have neither walls
 * nor a body force; others 0 / 0.
 * Results do not depend on it; the call drops a captured graph. */
int ddf_set_workgroups_per_cu(ddf_handle *h, int32_t even, int32_t odd);
int ddf_get_workgroups_per_cu(const ddf_handle *h, int32_t *even, int32_t *odd);
/* ddf_step replays runs of steps_per_graph steps (even; default 100, 0 = always launch
 * eagerly) captured once into a hipGraph; the remainder and an odd start launch
 * eagerly.  Lattices with a time-dependent force or stochastic rounding always step
 * eagerly (their kernels take the time index as an argument): DDF_ERR_UNSUPPORTED for
 * steps_per_graph > 0.  Changing the tiling or the run length drops the captured graph
 * (after waiting for the device). */
int ddf_set_graph(ddf_handle *h, int32_t steps_per_graph);

/* DDF_LAYOUT_ROW, DDF_LAYOUT_INTERLEAVED or DDF_LAYOUT_PACKED: the layout ddf_create chose. */
int32_t ddf_get_layout(const ddf_handle *h);

int64_t ddf_step_count(const ddf_handle *h);
const char *ddf_last_error(void);

/* ---------------------------------------------------------------------------------
 * Batches: n independent lattices (own size, rates, walls, force) advanced together
 * by one persistent launch per time step.  All instances share one storage type and
 * one scalar collision model.  Instance i's populations (packed rows, DDF_LAYOUT_PACKED)
 * sit at a 256-byte aligned offset of one f and one g buffer (ddf_batch_offsets):
 * ddf_population_bytes of its parameters with layout PACKED; its dense fields sit at a
 * node offset of concatenated [ny_i][nx_i] arrays.  Runs of K steps (default 100,
 * ddf_batch_set_graph) are captured once into a hipGraph on an internal stream and
 * replayed on the caller's stream; batches with a time-dependent force step eagerly.
 * --------------------------------------------------------------------------------- */
typedef struct ddf_batch ddf_batch;

/* Bytes of the f (and of the g) buffer for n instances. */
size_t ddf_batch_population_bytes(int32_t n, const ddf_params *ps);
/* Bytes of device workspace (descriptors, tile list, reduction partials, snapshots). */
size_t ddf_batch_workspace_bytes(int32_t n, const ddf_params *ps);
/* Validate every instance as ddf_create does and bind the caller's buffers
 * (256-byte aligned).  Uploads the instance descriptors (synchronous).
 * ddf_batch_create, ddf_batch_set_tiling, ddf_batch_set_active, ddf_batch_set_graph
 * (when a graph is captured) and ddf_batch_destroy first wait for all work on the
 * device (hipDeviceSynchronize): the buffers may be memory the caller's allocator has
 * just recycled from tensors that queued work still writes, and a replay may still be
 * reading the lists they replace. */
int ddf_batch_create(int32_t n, const ddf_params *ps, void *pop_f, void *pop_g, void *workspace, ddf_batch **out);
void ddf_batch_destroy(ddf_batch *b);
int32_t ddf_batch_size(const ddf_batch *b);
int64_t ddf_batch_step_count(const ddf_batch *b);
/* Byte offset of instance i's planes in f and g; node offset of its dense fields. */
int ddf_batch_offsets(const ddf_batch *b, int32_t i, int64_t *pop_offset_bytes, int64_t *field_offset);
/* Equilibrium initial state of every instance from concatenated FP64 device fields
 * (same rule as ddf_init_equilibrium); resets the step counter. */
int ddf_batch_init_equilibrium(ddf_batch *b, const double *rho, const double *ux, const double *uy,
                               const double *phi, void *stream);
/* Tiling: tile width at most bx_max (64, 128, 256 or 512; 512 threads per tile), or
 * bx_max = 0 for flat tiles of 512 consecutive nodes in row-major order (instances whose
 * sides are not multiples of a tile then leave idle lanes only in their last tile; the
 * default at creation); and blocks_per_cu persistent workgroups per compute unit (0 =
 * one workgroup per tile).  Results do not depend on the tiling.  Invalidates the
 * captured graph. */
int ddf_batch_set_tiling(ddf_batch *b, int32_t bx_max, int32_t blocks_per_cu);
int ddf_batch_get_tiling(const ddf_batch *b, int32_t *bx_max, int32_t *blocks_per_cu, int32_t *ntiles, int32_t *grid);
/* Non-temporal (streaming) loads and stores in the even and in the odd step kernel (0 or
 * 1 each; default 0 / 0).  ddf_batch_autotune chooses them with the tiling.  Results do
 * not depend on them; the call drops a captured graph (after waiting for the device). */
int ddf_batch_set_nontemporal(ddf_batch *b, int32_t even, int32_t odd);
int ddf_batch_get_nontemporal(const ddf_batch *b, int32_t *even, int32_t *odd);
/* Times every (bx_max, blocks_per_cu) candidate (bx_max 0, 64, 128, 256 or 512) for
 * steps_per_trial steps on this instance mix, then non-temporal accesses in either
 * parity on the fastest, applies the best and caches it per (storage, scalar model,
 * instance sizes and boundary kinds) for the process.  The trials overwrite the populations: call it before
 * ddf_batch_init_equilibrium.  best_ms_per_step is -1 when the cache answered. */
int ddf_batch_autotune(ddf_batch *b, int32_t steps_per_trial, int32_t *bx_max, int32_t *blocks_per_cu,
                       float *best_ms_per_step, void *stream);
/* active[i] != 0 keeps instance i in the step list (all instances start active); inactive
 * instances keep their state and still appear in reductions (with a zero residual).
 * Needs an even step count (DDF_ERR_STATE otherwise): an inactive instance holds an
 * even-step state, so while one is inactive ddf_batch_reduce also needs an even step
 * count.  Rebuilds the list and invalidates the captured graph. */
int ddf_batch_set_active(ddf_batch *b, const uint8_t *active);
/* Re-initialise instance i alone at equilibrium from dense FP64 device fields of its
 * size (same rule as ddf_init_equilibrium); the batch step count must be even.  The
 * next ddf_batch_reduce measures instance i's residual against the state before the
 * re-initialisation, so take one reduction before reading its residual again. */
int ddf_batch_init_instance(ddf_batch *b, int32_t i, const double *rho, const double *ux, const double *uy,
                            const double *phi, void *stream);
/* Steps per captured graph (even; 0 = always launch eagerly). */
int ddf_batch_set_graph(ddf_batch *b, int32_t steps_per_graph);
int ddf_batch_step(ddf_batch *b, int64_t nsteps, void *stream);
/* Per-instance statistics into out[n][DDF_NUM_STATS] (host memory); synchronises.
 * Returns DDF_ERR_NONFINITE (with out filled) when any instance is non-finite; the
 * other instances' rows stay valid. */
int ddf_batch_reduce(ddf_batch *b, double *out, void *stream);
/* ddf_batch_step(b, nsteps) followed by ddf_batch_reduce(b, out): the same state and the
 * same statistics (bit for bit).  Where the run ends on a whole captured graph (graphs
 * on, and nsteps minus the one eager step that aligns an odd step count a multiple of
 * the steps per graph), the last replay carries the reduction kernels, so the K steps
 * and the reduction are one graph launch and the call only copies the statistics back.
 * Synchronises the stream. */
int ddf_batch_step_reduce(ddf_batch *b, int64_t nsteps, double *out, void *stream);
/* Same as ddf_extract / ddf_get_populations for instance i. */
int ddf_batch_extract(ddf_batch *b, int32_t i, void *out, uint32_t mask, int32_t out_dtype, void *stream);
int ddf_batch_get_populations(ddf_batch *b, int32_t i, void *f, void *g, int32_t dtype, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DDF_H */
