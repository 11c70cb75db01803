/*
 * ddf_probe.h - HBM reference kernels of libddf (MI355X, gfx950).
 *
 * Not part of the paper's method: these are the bandwidth ceilings the lattice
 * Boltzmann step kernels are measured against.  The step is bound by HBM bandwidth
 * (it reads and writes every population once per time step and does 1-2 flops per
 * byte), so its achieved GB/s is compared with the nominal HBM peak and with what a
 * plain stream reaches on the same device: a copy (each byte read once and written
 * once, like the step), a read-only and a write-only pass; and with the step's own
 * access pattern run without its arithmetic.
 *
 * Conventions: as in ddf.h (caller-owned device buffers, asynchronous on `stream`,
 * DDF_OK or a negative ddf_status, message in ddf_last_error()).
 */
#ifndef DDF_PROBE_H
#define DDF_PROBE_H

#include <stddef.h>
#include <stdint.h>

#include "ddf.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { DDF_PROBE_COPY = 0, DDF_PROBE_READ = 1, DDF_PROBE_WRITE = 2 };

/* One pass over `bytes` bytes (a positive multiple of 16; src and dst 16-byte aligned):
 *   DDF_PROBE_COPY : dst[i] = src[i]            (reads and writes `bytes`)
 *   DDF_PROBE_READ : reads src, writes nothing   (dst is not touched and may be NULL)
 *   DDF_PROBE_WRITE: dst[i] = 0                  (src is not read and may be NULL)
 * Each thread of a 256-thread workgroup moves `unroll` (1, 2, 4 or 8) 16-byte vectors
 * 4 KiB apart; nontemporal != 0 marks the loads and stores non-temporal.  src and dst
 * must not overlap.  DDF_ERR_ARG for anything else. */
int ddf_bandwidth_probe(int32_t kind, int32_t unroll, int32_t nontemporal, const void *src, void *dst, size_t bytes,
                        void *stream);

/* The memory accesses of one AA step of the given parity (0 even, 1 odd) over the
 * populations of handle h, without the collision: per node, the nine stored
 * populations of each lattice that the step of that parity loads are loaded, and each
 * is stored, sign bit flipped, where the step stores the population of the opposite
 * direction (in the in-place AA pattern that is the slot the step loaded as that
 * direction; the flip keeps the rest direction's copy onto itself a real store).  Same
 * tiles, tile-to-XCD map, row layout, lane offsets and non-temporal policy as the
 * handle's step kernels; wg_per_cu caps the resident workgroups per CU (0 = no cap, 1-3),
 * like ddf_set_workgroups_per_cu.  It swaps and negates opposite directions within each
 * node's slot set, so two calls of one parity leave the populations bit-identical; the step count
 * is not changed.  With walls, a link the step reflects is loaded from and stored to the
 * node's own slots, as in the step.  Runs on `stream`, which must be ordered after the
 * handle's earlier work.  DDF_ERR_ARG for a NULL handle, another parity or cap. */
int ddf_pattern_probe(ddf_handle *h, int32_t parity, int32_t wg_per_cu, void *stream);

/* The same for the batch b: one parity of its step's loads and stores over the tiles of
 * its active instances, with the collision left out (same tile list, XCD map and
 * non-temporal setting as ddf_batch_step; each value stored sign-flipped where the step
 * stores the opposite direction, walls included).  Two calls of one parity restore the
 * populations; the step count is not changed.  DDF_ERR_ARG for a NULL batch or another
 * parity. */
int ddf_batch_pattern_probe(ddf_batch *b, int32_t parity, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DDF_PROBE_H */
