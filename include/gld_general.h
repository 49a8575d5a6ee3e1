/*
 * gld_general.h -- the general memory model of GLD on one GPU (FP64).
 *
 * Jung, Hanke & Schmid, arXiv:1808.00270.  The system type of gld.h
 * expands the noise for a separable pair memory, where every per-frequency
 * correlation matrix is a function of one pair-weight matrix.  This system
 * type takes the general model of Sec. II:
 *
 *   - a tabulated pair kernel K^p_m(r_b) of any rank (gld_params.k_pair, or
 *     the separable k_pair_w x k_pair_g), linearly interpolated between the
 *     distance bins (Sec. III.A tabulates the kernels on a distance grid);
 *   - the distance-dependent self memory Delta K^s_m(r_b) of eq.
 *     (GLD_basic2) (gld_params.dk_self), with the pair memory's tensor form;
 *     its m = 0 term enters F^D' with each neighbour's weight on the
 *     particle's own velocity (eq. dissipative_force2); a and b of the
 *     integrator (eq. aa-bb) use the isotropic K^s_0 only;
 *   - the colored noise by Algorithm 1 on the GPU: every step, the real part
 *     of the length-(2 m_max - 1) DFT of the white-noise window (eq. FT),
 *     one Lanczos square root sqrt(K_hat_w) Re W_hat_w per frequency w with
 *     a matrix-free mat-vec over the pair list, the per-frequency
 *     correlation K_hat_w evaluated at the current distances (the time-scale
 *     separation of Sec. II.C), and F^R_n = (1/P)(x_0 + 2 sum_{w>=1} x_w),
 *     P = 2 m_max - 1.  The Lanczos process of frequency w stops when its
 *     iterate changes by at most noise_tol (relative, 2-norm), tested in the
 *     Krylov coordinates; a frequency starts testing two iterations below the
 *     count it needed at the previous step (the smallest Ritz value only
 *     falls with the iteration count, so a non-positive one is still found).
 *
 * Everything else is as in gld.h: the integrator of eq. (GLD_integrator)
 * with b in the position update, WCA conservative pair force, white noise
 * W_{i,c,t} from Philox4x32-10 (gld_white_noise), history before step 0
 * zero, kernels frozen below r_cut_min.  Pairs are found by an all-pairs
 * search every step (n <= GLD_GENERAL_MAX_N).
 *
 * Fields of gld_params used: n, box, dt, mass, kT, m_max, n_r, k_self,
 * k_pair or (k_pair_w, k_pair_g), dk_self, r0, dr, r_cut, r_cut_min,
 * pair_tensor, precision (must be GLD_FP64), wca_sigma, wca_eps, seed,
 * noise_tol (0: 1e-12), max_neighbors (0: automatic), noise_window (0 or
 * 1).  Ignored: lam_lo, lam_hi, check_interval, check_iters, verlet_skin,
 * noise_a, noise_b, noise_rank, noise_terms.
 *
 * Errors latched during stepping (gld_general_sync / read_state return them,
 * with the step in gld_state.flag_step): GLD_ERR_NOT_PD (a per-frequency
 * correlation matrix with a non-positive Rayleigh quotient or Ritz value),
 * GLD_ERR_NO_CONV (the Krylov dimension reached max_iters), GLD_ERR_CAPACITY
 * (more neighbours than the list holds), GLD_ERR_NONFINITE (a non-finite
 * velocity).  After a latched error the state is undefined until
 * gld_general_write_state.
 */
#ifndef GLD_GENERAL_H
#define GLD_GENERAL_H

#include <stddef.h>
#include <stdint.h>

#include "gld.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Largest particle count (all-pairs search) and Krylov dimension. */
#define GLD_GENERAL_MAX_N 32768
#define GLD_GENERAL_MAX_ITERS 128

typedef struct gld_general gld_general;

/* Device bytes of a general system with these parameters and Krylov cap
 * max_iters (0: 96).  The Lanczos bases take m_max * max_iters * 3n
 * doubles.  Host-only. */
gld_status gld_general_workspace_size(const gld_params *params, int32_t max_iters, size_t *bytes);

/* Create at step 0 from r0, v0 ([n][3], host) with zero history on the
 * caller's device workspace (d_workspace, at least gld_general_workspace_size
 * bytes, 256-byte aligned) and HIP stream.  Computes the per-frequency
 * spectra of the kernel tables on the device, the pair list and F^C_0, and
 * fills the white-noise window.  Synchronises.  The workspace stays the
 * caller's. */
gld_status gld_general_create(const gld_params *params, int32_t max_iters, const double *r0, const double *v0,
                              void *d_workspace, size_t workspace_bytes, void *hip_stream, gld_general **out);

/* Enqueue n_steps steps on the stream; returns without waiting. */
gld_status gld_general_step(gld_general *g, int64_t n_steps);

/* Wait for the stream; return the latched device status. */
gld_status gld_general_sync(gld_general *g);

/* Synchronise and copy the state to the host arrays of *out (gld_state of
 * gld.h; history [m_max-1][n][3]). */
gld_status gld_general_read_state(gld_general *g, gld_state *out);

/* Install r, v, step and the optional history (NULL: zero); rebuilds the
 * pair list, F^C and the white-noise window and clears latched errors.
 * Synchronises. */
gld_status gld_general_write_state(gld_general *g, const gld_state *in);

/* The per-frequency square roots of the last completed step:
 * out[w - w0][i][c] = x_w = sqrt(K_hat_w) Re W_hat_w for w0 <= w < w1, so
 * that F^R = (1/P)(x_0 + 2 sum_{w>=1} x_w).  Synchronises. */
gld_status gld_general_frequency_vectors(gld_general *g, int32_t w0, int32_t w1, double *out);

typedef struct {
    int32_t max_iters;      /* Krylov cap of the system                        */
    int32_t last_iters;     /* largest Krylov dimension used at the last step  */
    int64_t pairs;          /* directed pairs within r_cut at the current step */
    int32_t max_per_particle;
    int32_t capacity;       /* pair-list entries per particle                  */
    double tol;             /* Lanczos stopping tolerance                      */
} gld_general_info;

/* Synchronises. */
gld_status gld_general_get_info(gld_general *g, gld_general_info *out);

/* Per-kernel timing with HIP events on the system's stream, as gld.h's
 * gld_set_timing / gld_kernel_times, for the kernel classes below. */
enum {
    GLD_G_DISSIPATIVE = 0, /* F^D' over the pairs and the displacement ring    */
    GLD_G_DFT,             /* Re W_hat_w of the white-noise window             */
    GLD_G_LANCZOS,         /* per-frequency Lanczos square roots               */
    GLD_G_COMBINE,         /* F^R from the per-frequency vectors               */
    GLD_G_PAIRS,           /* all-pairs search, pair list and F^C              */
    GLD_G_UPDATE,          /* position / velocity updates, new white noise     */
    GLD_G_COUNT
};
gld_status gld_general_set_timing(gld_general *g, int enable);
gld_status gld_general_kernel_times(gld_general *g, double *ms_sum, int64_t *launches);

/* Release the handle.  Synchronises. */
gld_status gld_general_destroy(gld_general *g);

#ifdef __cplusplus
}
#endif

#endif /* GLD_GENERAL_H */
