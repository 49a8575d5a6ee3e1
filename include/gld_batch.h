/*
 * gld_batch.h -- C ABI of libgld's batched engine: many independent GLD
 * systems (uneven N, density, memory length and kernels) advanced together
 * on one GPU, every launch of a step covering all of them.
 *
 * Each system is the one gld.h describes (the integrator of eq.
 * (GLD_integrator), the dissipative force of eq. (dissipative_force2), the
 * colored noise of eq. (stochastic_force2) built as in Sec. II.C); the batch
 * changes how the work is launched, not what is computed: a system's results
 * are the same alone and in any batch, bit for bit (every sum of a system runs
 * in an order fixed by that system alone).
 *
 * Engine.  Per step: the memory convolution (streamed once per step), the
 * white-noise ring and the matrix-core filter bank (1/block of the next
 * block's outputs per step), the premixed Chebyshev inputs, the dissipative
 * pair product, the Clenshaw chain (as many launches as the longest chain of
 * the batch; shorter chains skip the first ones), the update, the cell list
 * and ELL pair lists at the new positions (rebuilt every step), all captured
 * in one HIP graph that is replayed every step.  The pair mat-vecs give each
 * particle 1, 2, 4 or 8 lanes by its system's mean neighbour count, with the
 * thresholds chosen by gld_batch_autotune.
 *
 * Limits per system: n <= 65535 (16-bit list indices), isotropic pair tensor,
 * noise_window 1, no caller-built filters; all systems of a batch share its
 * precision.
 *
 * Memory.  The caller provides one device workspace and a stream; systems are
 * placed in it by a first-fit allocator at gld_batch_add (GLD_ERR_OOM when
 * one does not fit) and their space is returned by gld_batch_remove.
 * Errors latched on the device are per system (gld_batch_read_state returns
 * them in gld_state.flags / flag_step); a system with an error keeps stepping
 * with the others until it is removed or a state is written.
 */
#ifndef GLD_BATCH_H
#define GLD_BATCH_H

#include "gld.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gld_batch gld_batch;

/* Lanes per particle of the batched pair mat-vec: a system whose mean
 * neighbour count is below lanes_threshold[0] takes 1 lane, below [1] 2,
 * below [2] 4, otherwise 8. */
typedef struct {
    int32_t lanes_threshold[3];
} gld_batch_schedule;

/* Device bytes of the batch's own tables for `capacity` systems (descriptors
 * and launch maps), to be added to the systems' footprints. */
gld_status gld_batch_base_size(int32_t capacity, size_t *bytes);

/* Create an empty batch of at most `capacity` systems in precision
 * `precision` (gld_precision) over the caller's workspace. */
gld_status gld_batch_create(int32_t precision, int32_t capacity, void *d_workspace, size_t workspace_bytes,
                            void *hip_stream, gld_batch **out);

/* Device bytes one system takes in a batch (its state, history ring, noise
 * buffers, pair lists).  Builds the system's noise construction for the
 * configuration r0 ([n][3]) on the host, as gld_batch_add does. */
gld_status gld_batch_footprint(const gld_batch *b, const gld_params *params, const double *r0, size_t *bytes);

/* Add systems at step 0 from (r0[i], v0[i]); the one-off noise constructions
 * run on host threads in parallel.  Each system is added on its own:
 * slots[i] receives its slot, or -1 if it could not be added, with its
 * status in status[i] (may be NULL): a parameter error, GLD_ERR_NOT_PD or
 * GLD_ERR_INTERVAL for its initial configuration, GLD_ERR_OOM when no slot
 * or no workspace piece is left.  Returns GLD_OK when every system was
 * added, else the status of the first that was not (gld_last_error names it). */
gld_status gld_batch_add(gld_batch *b, int32_t count, const gld_params *const *params, const double *const *r0,
                         const double *const *v0, int32_t *slots, int32_t *status);

/* Remove a system and return its workspace. */
gld_status gld_batch_remove(gld_batch *b, int32_t slot);

/* Enqueue n_steps steps of every system of the batch. */
gld_status gld_batch_step(gld_batch *b, int64_t n_steps);

/* Wait for the stream. */
gld_status gld_batch_sync(gld_batch *b);

/* Synchronise and copy one system's state (as gld_read_state). */
gld_status gld_batch_read_state(gld_batch *b, int32_t slot, gld_state *out);

/* Install a state of one system (as gld_write_state: r, v, step, optional
 * history); clears its latched error. */
gld_status gld_batch_write_state(gld_batch *b, int32_t slot, const gld_state *in);

/* Noise construction of one system (the fields gld_noise_info has for it). */
gld_status gld_batch_noise_parameters(const gld_batch *b, int32_t slot, gld_noise_info *out);

/* Choose the lane thresholds of the pair mat-vecs: each of
 * GLD_BATCH_CANDIDATES candidate schedules runs the batch's pair mat-vecs of
 * one step (the dissipative product and the whole chain) trial_steps times
 * on the current state, timed with HIP events (they rewrite only the chain's
 * work vectors, which every step recomputes), and the fastest is kept.
 * *chosen (may be NULL) receives it; ms_per_candidate (may be NULL, room for
 * GLD_BATCH_CANDIDATES) the measured time per pass of each candidate. */
#define GLD_BATCH_CANDIDATES 8
gld_status gld_batch_autotune(gld_batch *b, int32_t trial_steps, gld_batch_schedule *chosen,
                              double *ms_per_candidate);
gld_status gld_batch_set_schedule(gld_batch *b, const gld_batch_schedule *s);

/* Per-kernel timing, as gld_set_timing / gld_kernel_times for one system:
 * while enabled, gld_batch_step launches eagerly with a HIP event pair around
 * each kernel class (GLD_K_*: one pair per class and step, the count is the
 * number of such stretches); gld_batch_kernel_times synchronises and returns
 * the summed ms and counts since timing was enabled. */
gld_status gld_batch_set_timing(gld_batch *b, int enable);
gld_status gld_batch_kernel_times(gld_batch *b, double *ms_sum, int64_t *launches);

/* Systems, particles and total directed pairs of the batch (synchronises). */
gld_status gld_batch_stats(gld_batch *b, int32_t *systems, int64_t *particles, int64_t *pairs);

/* One system of the batch: its directed pairs in the current list and the
 * lanes per particle of its mat-vecs (1, 2, 4 or 8).  Synchronises. */
gld_status gld_batch_system_stats(gld_batch *b, int32_t slot, int64_t *pairs, int32_t *lanes);

/* Release the batch (the workspace stays the caller's).  Synchronises. */
gld_status gld_batch_destroy(gld_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* GLD_BATCH_H */
