/*
 * gld.h -- C ABI of the MI355X (gfx950) generalized Langevin dynamics (GLD)
 * time-step library, libgld.so.
 *
 * Method: G. Jung, M. Hanke, F. Schmid, "Generalized Langevin dynamics:
 * construction and numerical integration of non-Markovian particle-based
 * models", arXiv:1808.00270.  One call of gld_step advances N identical
 * particles in a periodic box by the G-JF type integrator of eq.
 * (GLD_integrator)/(aa-bb), with
 *   - the conservative pair force F^C (WCA pair potential),
 *   - the non-Markovian dissipative force F^D' of eq. (dissipative_force2):
 *     a memory convolution over the last m_max-1 displacement steps with the
 *     self kernel K^s_m and the pair kernel K^p_m(R_ij) evaluated at the
 *     current distances,
 *   - the colored random force F^R whose lag correlations obey the discrete
 *     fluctuation-dissipation relation eq. (stochastic_force2), i.e. the
 *     vector sum_s A_s W_{n+s} of eq. (noise_production) with the filter
 *     matrices A_s the per-frequency square roots of Sec. II.C.
 *
 * Memory and streams.  The library never allocates device memory.  The caller
 * provides one device workspace of at least gld_workspace_size() bytes and a
 * HIP stream (hipStream_t passed as void*); both must outlive the system.
 * All device work of a system is enqueued on that stream.
 *
 * Host arrays.  All host arrays are row-major, particle-major [n][3] doubles,
 * owned by the caller, read (or written) only during the call.
 *
 * Errors.  Every entry point returns a gld_status.  Errors found on the device
 * during gld_step (non-positive-definite noise correlation, non-finite state,
 * neighbour-list overflow, spectrum outside the noise interval) are latched
 * with their step index and returned by the next synchronising call
 * (gld_sync, gld_read_state).  After such an error the system is poisoned:
 * gld_step refuses to run until gld_write_state installs a new state.
 * gld_last_error() gives a thread-local message for the last failing call.
 */
#ifndef GLD_H
#define GLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GLD_OK = 0,
    GLD_ERR_INVALID_ARG = -1, /* bad parameter, size or pointer                       */
    GLD_ERR_NOT_PD = -2,      /* noise correlation matrix not positive definite        */
    GLD_ERR_NO_CONV = -3,     /* noise approximation did not reach the tolerance       */
    GLD_ERR_NONFINITE = -4,   /* NaN/Inf in positions or velocities                     */
    GLD_ERR_OOM = -5,         /* workspace too small                                   */
    GLD_ERR_DEVICE = -6,      /* HIP runtime error                                      */
    GLD_ERR_BOX = -7,         /* box too small for the cutoff (r_cut >= L/2)            */
    GLD_ERR_CAPACITY = -8,    /* more neighbours than max_neighbors                     */
    GLD_ERR_INTERVAL = -9     /* pair-matrix spectrum left the noise interval           */
} gld_status;

typedef enum { GLD_FP64 = 0, GLD_FP32_MIXED = 1 } gld_precision;

/* Largest distance grid of the pair weight w(r): the neighbour build keeps
 * the whole table in LDS. */
#define GLD_MAX_DISTANCE_BINS 1024

/* Most Lanczos iterations a spectrum check may run (gld_params.check_iters). */
#define GLD_MAX_CHECK_ITERS 200

/* Tensor structure of the pair memory (Sec. II.A): isotropic K^p 1, or only
 * the component parallel to the line of centres, K^p e e^T. */
typedef enum { GLD_PAIR_ISOTROPIC = 0, GLD_PAIR_PARALLEL = 1 } gld_pair_tensor;

/* System description.  Discrete kernels K_m are those of eq. (k-discrete);
 * the pair kernel is separable, K^p_m(r) = w(r) g_m, with w tabulated on the
 * uniform grid r_b = r0 + b dr (b = 0..n_r-1) and linearly interpolated, as
 * the paper tabulates its kernels on a distance grid (Sec. III.A); below
 * r_cut_min the kernel is frozen at its value at r_cut_min (Sec. III.B). */
typedef struct {
    int64_t n;                 /* particles, >= 1                                    */
    double box[3];             /* periodic box edges; each > 2 r_cut                 */
    double dt;                 /* time step                                          */
    double mass;               /* particle mass M                                    */
    double kT;                 /* k_B T (0 switches the random force off)             */
    int32_t m_max;             /* memory length: lags m = 0..m_max-1, 1..4096        */
    int32_t n_r;               /* distance grid points, 2..GLD_MAX_DISTANCE_BINS     */
    const double *k_self;      /* [m_max]  K^s_m                                     */
    const double *k_pair_g;    /* [m_max]  g_m (NULL: no pair memory)                */
    const double *k_pair_w;    /* [n_r]    w(r_b) (NULL: no pair memory)             */
    double r0, dr;             /* distance grid                                      */
    double r_cut;              /* pair cutoff (memory and neighbour list)            */
    double r_cut_min;          /* kernel frozen below this distance                  */
    int32_t pair_tensor;       /* gld_pair_tensor                                    */
    int32_t precision;         /* gld_precision                                      */
    double wca_sigma;          /* WCA conservative pair force; wca_eps = 0 disables  */
    double wca_eps;
    uint64_t seed;             /* Philox4x32-10 key of the white noise W             */
    double noise_tol;          /* relative rms accuracy of F^R (0: 4e-6 FP32_MIXED,
                                  whose forces are held to 1e-5; 1e-12 FP64)         */
    double lam_lo, lam_hi;     /* interval holding the spectrum of the pair-weight
                                  matrix P = [w(R_ij) T_ij]; both 0: chosen at
                                  create from the initial configuration              */
    int32_t max_neighbors;     /* pair-list capacity per particle (0: automatic)     */
    int32_t check_interval;    /* steps between spectrum (positive-definiteness)
                                  checks by Lanczos on P (0: 100, < 0: never)        */
    double verlet_skin;        /* >= 0.  0: the neighbour lists are rebuilt every
                                  step.  > 0: a list of candidates within
                                  r_cut + verlet_skin is rebuilt only once some
                                  particle has moved more than verlet_skin / 2 since
                                  the last build, and each step takes the pairs
                                  within r_cut from it (the same pairs; the order of
                                  the neighbour sums then depends on when the list
                                  was built, so a resumed run agrees with an
                                  uninterrupted one to rounding, not bit for bit) */
    int32_t noise_window;      /* W in [0, 16]; 0 and 1: the random force of every
                                  step at that step's positions (eq. stochastic_force2).
                                  W > 1: the variant Sec. II.C proposes (remarks after
                                  Algorithm 1) for positions that barely move over W
                                  steps: the random forces of W consecutive steps are
                                  computed together, all at the positions of the
                                  window's first step.  Windows start at the steps that
                                  are multiples of W; after gld_write_state at a step
                                  inside a window, the rest of that window uses the
                                  written positions.  The filter block of the noise
                                  plan (gld_noise_info.block) becomes the largest
                                  multiple of W it allows; W larger than the block the
                                  plan allows (64 / padded rank steps, so 8 and 4 for
                                  ranks 8 and 16) makes gld_create return
                                  GLD_ERR_INVALID_ARG.
                                  Ignored when kT = 0. */
    /* The general tables of eqs. (GLD_basic2) and (dissipative_force2) on the
     * same distance grid (Sec. III.A tabulates K^p(R, t) on a grid), row-major
     * [n_r][m_max]:
     *   k_pair   K^p_m(r_b); NULL: the separable form k_pair_w x k_pair_g.  A
     *            table of rank one (K^p_m(r) = w(r) g_m to 1e-13 of its
     *            largest entry) is taken in that separable form, scaled so
     *            that max_b |w(r_b)| = 1 (lam_lo, lam_hi refer to that w); a
     *            table of
     *            higher rank makes each per-frequency correlation a function
     *            of several pair matrices, which this system type does not
     *            expand: GLD_ERR_INVALID_ARG ("non-separable pair kernel").
     *   dk_self  Delta K^s_m(r_b), the distance-dependent part of the self
     *            memory; NULL or all zero: none.  Non-zero tables are not
     *            supported by this system type: GLD_ERR_INVALID_ARG. */
    const double *k_pair;
    const double *dk_self;
    /* Caller-built noise filters (the one-off noise coefficients of Sec. II.C,
     * e.g. from gld_build_noise_filters): noise_a [noise_rank][2 m_max - 1]
     * filter taps for the lags -(m_max-1)..m_max-1 and noise_b
     * [noise_terms][noise_rank] Chebyshev mixing weights, built for the
     * interval [lam_lo, lam_hi] of this struct (which must then be given,
     * lam_lo < lam_hi).  NULL: gld_create builds them (and a tight plan).
     * 1 <= noise_rank <= 32, 1 <= noise_terms <= 512; copied at create. */
    const double *noise_a;
    const double *noise_b;
    int32_t noise_rank;
    int32_t noise_terms;
    int32_t check_iters;       /* Lanczos iterations of each spectrum check
                                  (0: 40), at most GLD_MAX_CHECK_ITERS          */
    int32_t rebuild_period;    /* > 0 (with verlet_skin > 0): the candidate lists
                                  are also rebuilt at the positions of every step
                                  that is a multiple of it, so that the rebuilds
                                  keep a fixed cadence when the skin outlasts the
                                  period; 0: only the displacement test          */
} gld_params;

/* Snapshot of a system.  On read, every non-NULL array is filled; on write,
 * r and v are required, history is optional (NULL = zero history). */
typedef struct {
    double *r;        /* [n][3] positions, unwrapped                               */
    double *v;        /* [n][3] velocities                                         */
    double *f_c;      /* [n][3] F^C at the current positions (read only)           */
    double *f_d;      /* [n][3] F^D' of the last completed step (read only)        */
    double *f_r;      /* [n][3] F^R of the last completed step (read only)         */
    double *history;  /* [m_max-1][n][3] displacements dR_{n-m}, m = 1..m_max-1    */
    int64_t step;     /* time step index n of (r, v)                               */
    int32_t flags;    /* latched gld_status of the device checks (read only)       */
    int64_t flag_step;/* step at which the latched error occurred (read only)      */
} gld_state;

/* Parameters of the colored-noise construction chosen by the library. */
typedef struct {
    int32_t cheb_terms;     /* K: Chebyshev terms in the pair-weight matrix           */
    int32_t rank;           /* r: filters in the white-noise filter bank              */
    int32_t block;          /* steps of filter output produced per filter launch      */
    double lam_lo, lam_hi;  /* interval of the expansion                              */
    double lam_singular;    /* largest lambda where some frequency's K_hat is singular */
    double err_estimate;    /* estimated relative rms error of F^R                    */
    int32_t window_half;    /* h: the filters use the white noise at lags |t| <= h    */
    int32_t noise_window;   /* W: steps whose random forces are computed together    */
    int32_t cheb_terms_tight; /* K of the tight plan on [lam_lo, lam_hi_tight] (0: none).
                                 A step whose largest row sum of |w| (a bound on the
                                 spectrum of P) is at most lam_hi_tight uses it; the
                                 noise interval chosen at create only               */
    double lam_hi_tight;
    double lam_lo_tight;    /* lower end of the tight plan (closer to the spectrum
                               than lam_lo); a spectrum check whose smallest Ritz
                               value falls below it retires the tight plan       */
    int64_t tight_steps;    /* steps since create whose chain used the tight plan
                               (synchronises with the system's stream)               */
    int32_t list_index_bits; /* bits per staged index in the pair lists the mat-vecs
                               stream: 12 in a cell whose 27-cell stencil holds at
                               most 4096 particles, else 16; the largest over the
                               cells at the last list build (synchronises)          */
    double theta_min, theta_max; /* extreme Ritz values of the last spectrum check
                               (an upper bound on the smallest and a lower bound on
                               the largest eigenvalue of P; synchronises)           */
    int32_t tight_retired;  /* 1 once a check found theta_min below lam_lo_tight
                               (the wide plan until the next gld_write_state)       */
    int32_t filters_given;  /* 1: the filters came from gld_params.noise_a/b      */
    int32_t list_weight_bits; /* bits per pair weight in the lists of the cells with
                               12-bit indices, isotropic tensor: fixed point
                               relative to the largest |w| of the table, index
                               and weight in one word; 52 of 64 bits in FP64
                               (about 1e-16 of the largest weight); 20 of 32
                               bits in FP32_MIXED with a library-built noise
                               plan of tolerance at least 4e-6 (moves F^R by
                               about 1e-6 of its rms), else 32                    */
} gld_noise_info;

typedef struct gld_system gld_system;

/* Device bytes a system with these parameters needs.  Host-only. */
gld_status gld_workspace_size(const gld_params *params, size_t *bytes);

/* Create a system at step 0 from r0, v0 ([n][3]) with zero history.  Runs the
 * one-off FP64 construction of the noise filters (Sec. II.C: the Fourier
 * transforms of the kernels are precomputed under time-scale separation),
 * uploads the state, builds the neighbour list, computes F^C_0 and checks the
 * noise correlation for positive definiteness at t = 0 (Sec. II.B).
 * Synchronises the stream before returning.  *out receives the handle. */
gld_status gld_create(const gld_params *params, const double *r0, const double *v0,
                      void *d_workspace, size_t workspace_bytes, void *hip_stream,
                      gld_system **out);

/* Enqueue n_steps integrator steps on the system's stream; returns without
 * waiting.  A latched device error from an earlier step is returned here
 * only if it was already observed by a synchronising call. */
gld_status gld_step(gld_system *sys, int64_t n_steps);

/* Wait for the stream; return the latched device status. */
gld_status gld_sync(gld_system *sys);

/* Synchronise and copy the state to the host arrays of *out. */
gld_status gld_read_state(gld_system *sys, gld_state *out);

/* Install a state (r, v, step, optional history); recomputes the neighbour
 * list and F^C, clears latched errors and, with pair memory and noise,
 * measures the extreme Ritz values of the pair-weight matrix (the tight noise
 * plan needs the smallest; nothing is latched: the periodic spectrum check
 * judges the interval).  Synchronises. */
gld_status gld_write_state(gld_system *sys, const gld_state *in);

/* Noise-construction parameters of a system. */
gld_status gld_noise_parameters(const gld_system *sys, gld_noise_info *out);

/* Directed pairs (i, j), i != j, within r_cut in the current pair list (the
 * pairs every pair mat-vec of a step streams), and the most any particle
 * has.  Synchronises the system's stream. */
gld_status gld_list_stats(gld_system *sys, int64_t *pairs, int32_t *max_per_particle);

/* Use HIP graph replay for gld_step (default on).  */
gld_status gld_set_graph(gld_system *sys, int enable);

/* Per-kernel timing.  While enabled, gld_step launches eagerly and records a
 * HIP event pair around every kernel on the system's stream; gld_kernel_times
 * synchronises and returns, for each kernel class, the summed duration in ms
 * and the launch count since timing was enabled. */
enum {
    GLD_K_HISTORY = 0,  /* memory convolution over the displacement ring           */
    GLD_K_DISSIPATIVE,  /* pair contraction of F^D'                                */
    GLD_K_NOISE_FIR,    /* white-noise filter bank                                 */
    GLD_K_NOISE_SPMV,   /* Chebyshev pair mat-vec chain of F^R                     */
    GLD_K_UPDATE,       /* position and velocity updates                           */
    GLD_K_NEIGHBOR,     /* cell list, pair list and F^C                            */
    GLD_K_CHECK,        /* Lanczos spectrum check                                  */
    GLD_K_NOISE_SETUP,  /* the chain's plan choice, the premix of its terms'
                           filter combinations, its skipped terms and first term
                           (with timing on, GLD_K_NOISE_SPMV counts the terms that
                           stream the pair lists only)                             */
    GLD_K_COUNT
};
gld_status gld_set_timing(gld_system *sys, int enable);
gld_status gld_kernel_times(gld_system *sys, double *ms_sum, int64_t *launches);

/* Release the handle (the workspace stays the caller's). Synchronises. */
gld_status gld_destroy(gld_system *sys);

/* Bytes of the library's own static workspace (one per device). */
#define GLD_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: serving loops, harnesses that forbid it): gld_create with the
 * workspace taken from a static device array of GLD_STATIC_WORKSPACE_BYTES
 * that the library holds on each device it runs on until the process ends,
 * instead of a caller-provided one.  Same arguments, checks and result as
 * gld_create otherwise; allocates no device memory.  The current device
 * (hipGetDevice) owns the system, and hip_stream must belong to it.
 * Errors: GLD_ERR_OOM when gld_workspace_size() of these parameters exceeds
 * GLD_STATIC_WORKSPACE_BYTES; GLD_ERR_INVALID_ARG while another system created
 * by this call lives on the same device (one static workspace per device;
 * gld_destroy frees it for the next).  The array keeps the last system's
 * contents; creation clears what must start at zero.  Work of a static
 * system and of a later one on the same device must not overlap: gld_destroy
 * synchronises the stream before the array is reused. */
gld_status gld_create_static(const gld_params *params, const double *r0, const double *v0, void *hip_stream,
                             gld_system **out);

/* White noise exactly as the integrator draws it: out[t][i][c] = W_{i,c,t0+t}
 * for t < n_t, i < n, c < 3, on the device (d_out: n_t*n*3 doubles), and the
 * raw Philox4x32-10 words out4[t][i][4] (d_raw: n_t*n*4 uint32, may be NULL). */
gld_status gld_white_noise(uint64_t seed, int64_t n, int64_t t0, int64_t n_t,
                           double *d_out, uint32_t *d_raw, void *hip_stream);

/* Host only.  The one-off FP64 noise-filter construction (Sec. II.C, with the
 * Fourier transforms of the kernels precomputed) for the interval
 * [lam_lo, lam_hi] of the pair-weight matrix spectrum and relative rms
 * tolerance tol (0: the precision's default).  On success, *info holds K and
 * r, a_out[r][2 m_max - 1] the filter taps for lags -(m_max-1)..m_max-1 and
 * b_out[K][r] the Chebyshev mixing weights, so that
 *   F^R_n = sum_{k<K} T_k(alpha P + beta 1) sum_q b[k][q] sum_t a[q][t] W_{n+t},
 * alpha = 2/(hi-lo), beta = -(hi+lo)/(hi-lo).  Capacities: a_cap >= r (2 m_max - 1)
 * and b_cap >= K r doubles; too small -> GLD_ERR_INVALID_ARG. */
gld_status gld_build_noise_filters(const gld_params *params, double lam_lo, double lam_hi, double tol,
                                   double *a_out, size_t a_cap, double *b_out, size_t b_cap,
                                   gld_noise_info *info);

const char *gld_status_string(int status);
const char *gld_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GLD_H */
