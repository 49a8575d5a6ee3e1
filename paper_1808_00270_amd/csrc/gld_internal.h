// Internal declarations of libgld: host-side noise construction, device
// buffer layout and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gld.h"

namespace gld {

constexpr int kMaxCheb = 512;     // Chebyshev terms of the noise expansion
constexpr int kMaxRank = 32;      // filters in the white-noise filter bank
// default noise accuracy (relative rms of F^R): FP32-mixed forces are held to
// 1e-5, and the noise construction takes 4e-6 of it (the FP32 arithmetic of
// the chain, the history and the weights adds well under 1e-6); FP64 1e-12
constexpr double kNoiseTolMixed = 4e-6, kNoiseTolFp64 = 1e-12;
// largest magnitude of a fixed-point pair weight, 20 bits (FP32 lists) or
// 52 bits (FP64 lists), unsigned and signed
constexpr int kWeightQMax = (1 << 20) - 1, kWeightQMaxSigned = (1 << 19) - 1;
constexpr long long kWeightQMax64 = (1LL << 52) - 1, kWeightQMaxSigned64 = (1LL << 51) - 1;
constexpr int kCheckIters = 40;   // Lanczos iterations of a spectrum check (default)
constexpr int kMaxCheckIters = GLD_MAX_CHECK_ITERS;  // the most a system may ask for

// ---------------------------------------------------------------------------
// One-off FP64 construction of the colored-noise filters.
//
// For a separable pair memory K^p_m(r) = w(r) g_m and no distance dependent
// self memory, every per-frequency correlation matrix is
//     K_hat_w = S_w 1 + G_w P,   P = [w(R_ij) T_ij]  (zero diagonal blocks),
// with S_w, G_w the length-(2 m_max - 1) DFTs of kT a_m K^s_m / dt and
// kT a_m g_m / dt.  The noise of eq. (noise_production) is then
//     F_n = (1/P) sum_w' f_w(P) Re W_hat_w,   f_w(x) = sqrt(S_w + G_w x).
// Expanding f_w in Chebyshev polynomials on an interval [lo, hi] holding the
// spectrum of P and moving the frequency sum into the time domain gives
//     F_n = sum_k T_k(P~) v_k(n),   v_k(n) = sum_t C[k][t] W_{n+t},
// and the coefficient matrix C (K x (2 m_max - 1)) has a tiny numerical rank
// r, so C = B A with r time filters A and mixing weights B.
// ---------------------------------------------------------------------------
struct NoisePlan {
    int M = 0, P = 0;            // m_max, 2 m_max - 1
    int K = 0;                   // Chebyshev terms
    int r = 0;                   // filters
    double lo = 0, hi = 0;       // expansion interval
    double alpha = 0, beta = 0;  // P~ = alpha P + beta 1
    double sing_lo = 0, sing_hi = 0;  // nearest singular points (-inf/+inf if none)
    double err_cheb = 0, err_rank = 0, err_window = 0;
    int half = 0;                // filter window: lags |t| <= half
    std::vector<double> S, G;    // spectra [M]
    std::vector<double> Bmix;    // [K][r]
    std::vector<double> Afilt;   // [r][P], filter taps for lags t = -(M-1)..M-1 (zero beyond half)
    // Tight plan (Kt > 0): the expansion on [lo, hi_t], hi_t < hi, with the
    // same filters; a step whose row-sum bound of P stays below hi_t uses it
    int Kt = 0;
    double lo_t = 0, hi_t = 0, alpha_t = 0, beta_t = 0, err_cheb_t = 0;
    std::vector<double> Bmix_t;  // [Kt][r]
};

// Spectra and singular points only (no expansion).  Returns GLD_OK.
gld_status noise_spectra(const gld_params &p, NoisePlan &plan, std::string &err);
// Full construction on [lo, hi] with relative rms tolerance tol; with
// lo < hi_tight < hi also the tight plan on [max(lo, lo_tight), hi_tight]
// (one filter bank for both).  hi_tight NaN (the default): no tight plan.
gld_status noise_build(const gld_params &p, double lo, double hi, double tol, NoisePlan &plan,
                       std::string &err, double hi_tight = __builtin_nan(""), double lo_tight = -1e300);

// The thread-local message gld_last_error() returns.
void set_last_error(const std::string &msg);
// Parameter checks shared by every system type (gld_api.cpp).
gld_status validate_params(const gld_params *p);
// The same checks for the general system type: pair tables of any rank and
// a distance-dependent self memory are accepted.
gld_status validate_params_general(const gld_params *p);
// The general pair table as its separable form w x g (max |w| = 1), if it
// has rank one; `any` false for an all-zero table.
gld_status separable_pair_table(const gld_params *p, std::vector<double> &w, std::vector<double> &g, bool &any);
// The automatic noise interval [lo, hi] from the extreme Ritz values of the
// pair-weight matrix of a configuration and its largest row sum of |w|, and
// the tight plan's [lo_t, hi_t] (hi_t NaN: none).
void auto_interval(const gld_params &p, const NoisePlan &plan, double theta_min, double theta_max, double gmax,
                   double &lo, double &hi, double &hi_t, double &lo_t);

// ---------------------------------------------------------------------------
// Device-side system description passed to the launchers.
// ---------------------------------------------------------------------------
struct Dev {
    int64_t n = 0;
    int64_t S = 0;          // component stride (>= n, multiple of 64); vectors are [3][S]
    int nslots = 0;         // m_max - 1 ring slots
    int M = 0, P = 0;
    double box[3] = {0, 0, 0};
    double dt = 0, mass = 0, kT = 0, a = 0, b = 0;
    double r_cut = 0, r_cut_min = 0, r0 = 0, dr = 0;
    int n_r = 0;
    int parallel = 0;
    int fp64 = 0;
    int has_pair = 0;       // pair memory present
    double wca_sigma = 0, wca_eps = 0;
    uint64_t seed = 0;
    int cap = 0;            // neighbours per particle
    int capS = 0;           // candidates per particle (within r_cut + skin)
    double skin = 0;        // Verlet skin (0: rebuild every step)
    int rebuild_period = 0; // > 0: also rebuild at the positions of every multiple of it
    int nc[3] = {1, 1, 1};  // cell grid
    int noff[3] = {1, 1, 1};
    int offs[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    int ncell = 1;
    int fir_block = 1, fir_rcap = 8;
    int fir_half = 0;       // filter window half-width (lags |t| <= fir_half)
    int hist_block = 1;     // steps per block of the history convolution
    int wring_len = 1;      // slots of the white-noise ring
    double g0 = 0;
    double lam_hi = __builtin_huge_val();  // noise interval top, checked every step
    // Chebyshev chain with a tight plan (cheb_kt > 0): terms of the wide and
    // the tight plan, the row-sum bound below which the tight plan is used,
    // (alpha, beta) of the wide then the tight plan
    int cheb_kw = 0, cheb_kt = 0;
    float lam_tight = 0;
    double lam_lo_tight = -__builtin_huge_val();  // the tight plan needs the last check's smallest Ritz value
                                                  // at least this (-inf: no tight plan)
    double cheb_ab[4] = {0, 0, 0, 0};

    // state (double, [3][S])
    double *R = nullptr, *V = nullptr, *FC = nullptr, *FCn = nullptr, *Rw = nullptr;
    // work precision buffers (T = float or double), [3][S] unless noted
    void *ring = nullptr;   // [nslots][3][S]
    void *Dneg = nullptr, *Y = nullptr, *FD = nullptr, *FR = nullptr;
    void *cb[3] = {nullptr, nullptr, nullptr};  // T4 [S] Clenshaw vectors, sorted order
    void *U = nullptr;      // [2][fir_rows][3][S]: the outputs of two consecutive filter blocks
                            // (block b at (b mod 2)), rows (step in block) * rcap + filter
    void *wring = nullptr;  // [wring_len][3][S] white noise W_t, slot t mod wring_len
    void *Afilt = nullptr;  // [2 fir_half + 1][fir_rcap], tap-major
    void *Bmix = nullptr;   // [kMaxCheb][fir_rcap]
    void *ks = nullptr, *gm = nullptr;  // [M]
    void *hist_taps = nullptr;          // [hist_tap_rows][2]: (K^s_m, g_m), m = M-1 .. 1, zero-padded
    void *Uh = nullptr;                 // [2][kHistSplit][hist_block][2][3][S]: partial sums over the lags
                                        // m > j + HB of two consecutive history blocks (block b at b mod 2)
    double *wtab = nullptr;             // [n_r]
    void *nbl = nullptr;                // chunks of 8 staged-stencil indices, cell-blocked: cell at h0 with occ
                                        // particles holds [cap/8][occ] chunks from byte 16 h0 cap/8, each 8 x 16
                                        // bits, or 8 x 12 bits in 12 bytes where the stencil holds <= 4096
    void *nbw = nullptr;                // T pair weights (w, or w / R^2 for the parallel tensor), cell-blocked
                                        // [cap/4][occ][4] from row h0 cap/4
    // packed lists (isotropic tensor, library-built noise plan; FP32-mixed at
    // a noise tolerance >= the default): a narrow cell's entry is one word in
    // nbw, the 12-bit staged index in bits 0-11 and the weight in fixed point
    // above it, 20 bits of a 32-bit word (FP32) or 52 of a 64-bit one (FP64)
    // (q = round(w wq_scale), unsigned, or signed when the table has negative
    // values; w = q wq_inv); nbl is then unused for that cell
    int wpack = 0, wq_signed = 0;
    double wq_scale = 0.0, wq_inv = 0.0;
    void *stab = nullptr;               // int2 [ncell][28] stencil of each cell (first index, base)
    int maxc = 0;                       // candidates staged per round by the mat-vec
    void *snl = nullptr;                // uint16 [capS/8][n][8] candidate lists (staged indices, within r_cut + skin)
    int *snn = nullptr;                 // [n] candidate counts
    void *rb_s = nullptr;               // double4 [n] unwrapped positions at the last build, cell order
    void *relb = nullptr;               // double4 [n] positions relative to own cell at the last build
    int *nn = nullptr;                  // [n] neighbour counts (sorted order)
    void *pos_s = nullptr;              // double4 [n] wrapped positions, cell order
    void *reld = nullptr;               // double4 [n] current positions relative to the build-time cell, sorted
    void *relf = nullptr;               // float4 [n] the same rounded to float
    void *ys = nullptr;                 // T4 [S] dissipative input, sorted order
    void *us = nullptr;                 // T4 [fir_rcap][S] filter outputs of the step, sorted order
    // noise window (W > 1: the random forces of W steps computed together)
    int win = 1;
    void *usw = nullptr;                // T4 [W][r][S] filter outputs of the window's steps, sorted order
    void *cbw[3] = {nullptr, nullptr, nullptr};  // T4 [W][S] Clenshaw vectors of the window's chains
    void *FRw = nullptr;                // [W][3][S] random forces of the window's steps
    int *cell_id = nullptr, *cell_slot = nullptr, *cell_count = nullptr, *cell_start = nullptr;
    int *cell_tmp = nullptr, *cell_sorted = nullptr;
    // Lanczos check (T4 [S], sorted order)
    void *lq[3] = {nullptr, nullptr, nullptr};
    void *lw = nullptr;
    double *partial = nullptr;  // [2][kPartials]
    double *lab = nullptr;      // alpha[kMaxCheckIters], beta[kMaxCheckIters], result[4]
    int check_iters = kCheckIters;  // Lanczos iterations of a spectrum check
    // scalars
    long long *d_step = nullptr;
    int *d_flags = nullptr;     // [0] status, [1] unused
    long long *d_flag_step = nullptr;
    unsigned *d_rowmax = nullptr;  // max row sum of |w| (float bits)
    int *d_rebuild = nullptr;      // rebuild the cell order and candidate lists this step
    void *chain = nullptr;         // ChainStep [kMaxCheb]: the chain's terms as this step's plan sets them
    void *vk = nullptr;            // T4 [kMaxCheb][S]: v_k = sum_q B[k][q] u_q of the step, sorted order
    unsigned long long *d_tight = nullptr;  // steps whose chain used the tight plan
    int *d_retired = nullptr;      // a spectrum check found theta_min below the tight plan's lower end
};

constexpr int kPartials = 1024;

// Launchers (gld_kernels.hip).  All enqueue on `st` and return hipError_t.
hipError_t launch_neighbors(const Dev &d, hipStream_t st, double *fc_out);
// history convolution of the step: the block's product (launch_history_block)
// plus the step's own lags
hipError_t launch_history(const Dev &d, hipStream_t st);
// the lags m > j + HB of the steps n0 + j of a block, summed on the matrix
// cores: mode 0, the step's share of the next block's product (every step of
// a block computes 1/HB of it); mode 1, the whole product of the block holding
// the current step; mode 2, the whole product of the next block
hipError_t launch_history_block(const Dev &d, int mode, hipStream_t st);

hipError_t launch_dissipative(const Dev &d, hipStream_t st, bool reverse);
// filter bank, outputs of a block of `block` steps: mode 0, the step's share
// (1/block of the channels) of the next block's outputs; mode 1, the whole
// block holding the current step; mode 2, the whole next block
hipError_t launch_fir(const Dev &d, int mode, hipStream_t st);
// white-noise ring (block bf, window half h, n0 the start of the current
// step's block): mode 0 writes the slice the step adds, t = step + h + 2 bf - 1
// (one block ahead of the filter outputs it feeds); mode 1 fills the window of
// the current block, t = n0 - h .. n0 + bf - 1 + h; mode 2 the slices
// t = n0 + bf - h .. step + h + 2 bf - 2 (what the ring holds before the step
// in an uninterrupted run, for the next block's outputs)
hipError_t launch_white_ring(const Dev &d, int mode, hipStream_t st);
// filter block sizes for a padded rank (work precision), and the largest one
int fir_block_for(int fp64, int rcap);
int fir_rcap_for(int rank);
constexpr int kMaxFirBlock = 16;
// FP32 filter bank on the matrix cores: window steps per staged tap chunk; its
// taps are stored zero-padded, [bf - 1 + (2 half + 1) + kFirChunk + bf - 1][rcap]
constexpr int kFirChunk = 128;
inline size_t fir_padded_rows(int half, int bf) { return static_cast<size_t>(2 * half + 1 + kFirChunk + 2 * (bf - 1)); }
// steps per block of the history convolution: two filters (K^s, g) fill the
// 64 (FP32) or 32 (FP64) accumulator rows of the matrix-core product
constexpr int kHistBlock32 = 32, kHistBlock64 = 16;
// the history's block product is computed during the block before, in
// hist_block / kHistSplit channel slices times kHistSplit window splits
// (one per step; the step part adds the kHistSplit partial sums)
constexpr int kHistSplit = 4;
// accumulator rows of the filter bank's product (rows of one output block)
__host__ __device__ inline int fir_rows(int fp64) { return (void)fp64, 64; }
// steps between the launches that compute a share of the next filter block:
// the largest divisor of the block up to 5, so that the shares tile the
// block (a noise window makes the block any multiple of the window up to the
// largest block: 9, 14, 18 ...); the block's product is split into
// block / period shares
__host__ __device__ inline int fir_period(int bf)
{
    for (int p = 5; p > 1; --p)
        if (bf % p == 0) return p;
    return 1;
}
// the same for the history's block product (blocks of 32 or 16 steps)
constexpr int kHistPeriod = 4;
// rows of its zero-padded taps (the filter bank's layout, nslots taps)
inline size_t hist_tap_rows(int nslots, int hb) { return static_cast<size_t>(hb - 1 + nslots + kFirChunk + hb - 1); }
// out = a P x + b x + cz z + sum_q coef[q] us_q  (x, z, us: sorted T4; x, z may be null
// when a = b = 0 / cz = 0).  Written to out_sorted (T4) or, if that is null,
// scattered to out_orig ([3][S], original order) plus add_orig when given.
// reverse: the cells are taken in descending order.  The launches that stream
// the pair lists alternate the order, so that each starts on the lists the one
// before finished on, which are still in the caches.
hipError_t launch_spmv(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz,
                       const void *z, const void *coef, int r, void *out_sorted, void *out_orig,
                       const void *add_orig, bool reverse = false, int cheb_k = -1, bool premixed = false);
// the plan of this step's Chebyshev chain (tight or wide, from the row-sum
// bound the refresh left): the combination of each term, for the terms of
// launch_spmv that pass their index cheb_k
hipError_t launch_cheb_select(const Dev &d, hipStream_t st);
// v_k = sum_q B[k][q] u_q for the terms of the step's plan (the rows of the
// mixing table that k_cheb_select chose, or row k without a tight plan):
// the chain's terms then read one vector each instead of the r filter outputs
hipError_t launch_cheb_mix(const Dev &d, int r, int K, hipStream_t st);
// sorted copies of the dissipative input Y and of the r filter outputs of the step
hipError_t launch_permute(const Dev &d, hipStream_t st, int r);
// noise window: sorted copies of the r filter outputs of the W steps of the
// window holding the current step (into usw)
hipError_t launch_permute_window(const Dev &d, hipStream_t st, int r);
// noise window: launch_spmv over nv consecutive vectors (x, z, out_sorted: T4
// [nv][S]; us: T4 [nv][r][S]; out_orig: [nv][3][S]), the pair lists streamed
// once for every two vectors (isotropic tensor) or once per vector
hipError_t launch_spmv_window(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz,
                              const void *z, const void *coef, int r, const void *us, void *out_sorted,
                              void *out_orig, int nv, bool reverse, int cheb_k = -1);
// the chain's first pair term and the dissipative product through one stream
// of the pair lists (isotropic tensor): out = a P x + b x + cz z + v_k (the
// term cheb_k, premixed; to out_sorted, or to out_orig for k = 0) and
// F^D' = -P Y + Dneg (Y the sorted ys).  With a plan chosen on the device the
// launch takes the second product only where the plan makes cheb_k its first
// pair term; the host launches it for k = K - 2 of both plans.
hipError_t launch_spmv_dual(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz,
                            const void *z, void *out_sorted, void *out_orig, bool reverse, int cheb_k);
// noise window: FR = FRw[step mod W]
hipError_t launch_take_window(const Dev &d, hipStream_t st);
// largest mat-vec staging capacity (candidates) that fits the LDS of one work-group
int mv_max_staging(int fp64, int parallel);
hipError_t launch_update_r(const Dev &d, hipStream_t st);
hipError_t launch_update_v(const Dev &d, hipStream_t st);
hipError_t launch_step_advance(const Dev &d, hipStream_t st);
hipError_t launch_fill_zero_work(const Dev &d, void *p, int64_t count, hipStream_t st);
// Lanczos spectrum check on P; writes theta_min/max into d.lab[2*kMaxCheckIters + 0/1]
// and latches GLD_ERR_INTERVAL / GLD_ERR_NOT_PD against the given bounds.
hipError_t launch_spectrum_check(const Dev &d, hipStream_t st, int iters, double lo, double hi,
                                 double sing_lo, double sing_hi, long long salt);
hipError_t launch_white_noise(uint64_t seed, int64_t n, int64_t t0, int64_t nt, double *out,
                              uint32_t *raw, hipStream_t st);

}  // namespace gld
