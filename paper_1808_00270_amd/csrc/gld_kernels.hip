// Device kernels of the GLD time step for gfx950 (CDNA4, wave64).
//
// Paper: arXiv:1808.00270, Sec. II (eqs. GLD_integrator, aa-bb,
// dissipative_force2, stochastic_force2, noise_production) and Algorithm 1.
//
// Data layout in HBM (all vectors structure-of-arrays, component-major):
//   positions, velocities, F^C           double [3][S]
//   displacement ring (history)          T      [m_max-1][3][S]   slot-major
//   convolution outputs, F^D', F^R       T      [3][S]
//   white-noise ring                     T      [2 half + block][3][S]  slice t at t mod len
//   filter-bank outputs                  T      [block][rank][3][S]
//   neighbour lists (cell-sorted order)  uint16 [cap/8][occ][8] staged-stencil indices
//                                        T      [cap/4][occ][4] pair weights
//                                        (blocked by cell: occ particles of one cell)
// where the component stride S >= n is padded to a multiple of 64, so every
// component and every ring slot starts on a 256-byte boundary and the history
// stream is read with 16-byte (float4) or 32-byte (2 x double2) loads, a
// whole wave covering 1 KiB (2 KiB) per lag.  Padding entries stay zero.
//
// T is float in the FP32-mixed mode and double in the FP64 mode; positions,
// velocities and the conservative force are always double.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gld_internal.h"
#include "gld_device.h"

namespace gld {

namespace {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_zero_work(T *p, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// ---------------------------------------------------------------------------
// H3: memory convolution over the displacement ring
//   Dneg = -(1/dt) sum_{m=1}^{M-1} K^s_m dR_{n-m}
//   Y    = g_0 V + (1/dt) sum_{m=1}^{M-1} g_m dR_{n-m}
// in blocks of HB steps.  For step n = n0 + j of the block starting at n0,
// the lags m > j + HB reach only displacements from before the block before
// (t < n0 - HB); for all j at once these sums are one product (the filter
// bank's kernel on the matrix cores, ROLE 1):
//   Uh[j][0] = sum_{m=j+HB+1}^{M-1} K^s_m dR_{n0+j-m},  Uh[j][1] likewise with g_m,
// which the steps of the block before compute, each 1/HB of it (a slice of
// the channels and a split of the window, the splits' partial sums kept
// apart), so that every step does the same work and the ring is read once
// per block instead of once per step.  Each step then adds the splits and
// its lags m <= j + HB directly.  The sums are those of the definition,
// taken in another order.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double4;
};

template <typename T>
__device__ __forceinline__ typename Vec4<T>::type load4(const T *p)
{
    return *reinterpret_cast<const typename Vec4<T>::type *>(p);
}

// the step's part: 4 consecutive elements of the [3][S] vectors per thread
constexpr int kLagBatch = 4;  // ring loads in flight per thread
template <typename T>
__global__ __launch_bounds__(256) void k_history_step(const T *__restrict__ ring, const T *__restrict__ Uh,
                                                      int64_t n3, int nslots, int hb, const T *__restrict__ ks,
                                                      const T *__restrict__ gm,
                                                      const long long *__restrict__ d_step,
                                                      const double *__restrict__ V, T g0, T inv_dt,
                                                      T *__restrict__ Dneg, T *__restrict__ Y)
{
    const int64_t e0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
    if (e0 >= n3) return;
    const long long step = *d_step;
    const int j = static_cast<int>(step % hb);
    T d[4] = {T(0), T(0), T(0), T(0)}, h[4] = {T(0), T(0), T(0), T(0)};
    if (nslots > 0) {  // no history (m_max = 1): no block sums either
        // the kHistSplit partial sums of the block's product (parity of the block)
        const T *ub = Uh + ((step / hb) & 1) * kHistSplit * (2 * static_cast<int64_t>(hb)) * n3;
#pragma unroll
        for (int q = 0; q < kHistSplit; ++q) {
            const T *uq = ub + q * (2 * static_cast<int64_t>(hb)) * n3;
            const auto ud = load4<T>(uq + (2 * static_cast<int64_t>(j)) * n3 + e0);
            const auto uh = load4<T>(uq + (2 * static_cast<int64_t>(j) + 1) * n3 + e0);
            d[0] += ud.x;
            d[1] += ud.y;
            d[2] += ud.z;
            d[3] += ud.w;
            h[0] += uh.x;
            h[1] += uh.y;
            h[2] += uh.z;
            h[3] += uh.w;
        }
    }
    const int mm = min(j + hb, nslots);
    if (mm > 0) {
        // ring slot of step - m, walked down with a wrap from one remainder;
        // kLagBatch lags' loads in flight, their sums in the order of m
        int t = static_cast<int>((step - 1) % nslots);
        if (t < 0) t += nslots;
        auto lag = [&](const typename Vec4<T>::type &x, int m) __attribute__((always_inline)) {
            const T k = ks[m], q = gm[m];
            d[0] += k * x.x;
            d[1] += k * x.y;
            d[2] += k * x.z;
            d[3] += k * x.w;
            h[0] += q * x.x;
            h[1] += q * x.y;
            h[2] += q * x.z;
            h[3] += q * x.w;
        };
        int m = 1;
        for (; m + kLagBatch - 1 <= mm; m += kLagBatch) {
            int tt[kLagBatch];
            tt[0] = t;
#pragma unroll
            for (int u = 1; u < kLagBatch; ++u) tt[u] = tt[u - 1] == 0 ? nslots - 1 : tt[u - 1] - 1;
            typename Vec4<T>::type x[kLagBatch];
#pragma unroll
            for (int u = 0; u < kLagBatch; ++u) x[u] = load4<T>(ring + static_cast<int64_t>(tt[u]) * n3 + e0);
#pragma unroll
            for (int u = 0; u < kLagBatch; ++u) lag(x[u], m + u);
            t = tt[kLagBatch - 1] == 0 ? nslots - 1 : tt[kLagBatch - 1] - 1;
        }
        for (; m <= mm; ++m) {
            lag(load4<T>(ring + static_cast<int64_t>(t) * n3 + e0), m);
            t = t == 0 ? nslots - 1 : t - 1;
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t e = e0 + u;
        Dneg[e] = -d[u] * inv_dt;
        Y[e] = g0 * static_cast<T>(V[e]) + h[u] * inv_dt;
    }
}

template <typename T>
static hipError_t history_t(const Dev &d, hipStream_t st)
{
    const int64_t len = 3 * d.S;  // one slot; a multiple of 4 since S is a multiple of 64
    k_history_step<T><<<static_cast<unsigned>((len / 4 + 255) / 256), 256, 0, st>>>(
        static_cast<const T *>(d.ring), static_cast<const T *>(d.Uh), len, d.nslots, d.hist_block,
        static_cast<const T *>(d.ks), static_cast<const T *>(d.gm), d.d_step, d.V, static_cast<T>(d.g0),
        static_cast<T>(1.0 / d.dt), static_cast<T *>(d.Dneg), static_cast<T *>(d.Y));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// H5: white noise and the filter bank of eq. (noise_production).
//
// The white noise W_t of every particle is drawn once (Philox, Box-Muller)
// into a ring of the L = 2 half + BF most recent and upcoming steps, slot
// t mod L, [L][3][S]; each step adds the slice t = step + half + BF - 1.
// Every BF steps (when the device step counter is a multiple of BF) the
// filter bank streams the window t = n0-half .. n0+BF-1+half once and
// accumulates
//   u_q(n0 + b) = sum_{t=-half}^{half} A_q[t] W_{n0+b+t},  b < BF, q < RC
// (taps zero-padded to RC rows, window cut where the taps fall below the
// noise tolerance).  Output U[b][q][3][S].
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_white_ring(int64_t n, int64_t S, uint64_t seed, const long long *__restrict__ d_step, int mode,
                             int bf, int half, int len, T *__restrict__ W)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long cur = *d_step;
    const long long n0 = cur - cur % bf;
    const int y = blockIdx.y;
    long long t;
    if (mode == 0) {
        t = cur + half + 2 * bf - 1;
    } else if (mode == 1) {
        if (y >= 2 * half + bf) return;
        t = n0 - half + y;
    } else {
        t = n0 + bf - half + y;
        if (t > cur + half + 2 * bf - 2) return;
    }
    T w[3];
    BoxMuller<T>::gauss3(philox_at(seed, static_cast<uint32_t>(i), t, 0u), w);
    T *dst = W + static_cast<int64_t>(ring_slot(t, len)) * 3 * S;
    dst[i] = w[0];
    dst[S + i] = w[1];
    dst[2 * S + i] = w[2];
}


template <int ROLE>
__global__ __launch_bounds__(kFirMfmaThreads) void k_fir_mfma(int64_t n, int64_t S, int bf, int rc, int offset,
                                                              int span, int len, const float *__restrict__ A,
                                                              const float *__restrict__ W,
                                                              const long long *__restrict__ d_step,
                                                              float *__restrict__ U, FirPart part)
{
    fir_mfma_body<ROLE>(n, S, bf, rc, offset, span, len, A, W, d_step, U, part, blockIdx.x);
}

template <int ROLE, int RT>
__global__ __launch_bounds__(kFirMfmaThreads) void k_fir_mfma64(int64_t n, int64_t S, int bf, int rc, int offset,
                                                                int span, int len, const double *__restrict__ A,
                                                                const double *__restrict__ W,
                                                                const long long *__restrict__ d_step,
                                                                double *__restrict__ U, FirPart part)
{
    fir_mfma64_body<ROLE, RT>(n, S, bf, rc, offset, span, len, A, W, d_step, U, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// H6: G-JF type update, eq. (GLD_integrator) with the position coefficient b
// (App. A):  R' = R + dt b V + dt^2/(2M) b (F^C + F^D' + F^R);  dR -> ring.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_update_r(int64_t n3, double *__restrict__ R, const double *__restrict__ V,
                           const double *__restrict__ FC, const T *__restrict__ FD, const T *__restrict__ FR,
                           T *__restrict__ ring, int64_t S, int nslots, const long long *__restrict__ d_step,
                           double c_v, double c_f)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    const double f = FC[e] + static_cast<double>(FD[e]) + static_cast<double>(FR[e]);
    const double dR = c_v * V[e] + c_f * f;
    R[e] += dR;
    if (nslots > 0) {
        const int head = static_cast<int>(*d_step % nslots);
        ring[static_cast<int64_t>(head) * S + e] = static_cast<T>(dR);
    }
}

//   V' = a V + dt/(2M) (a F^C_n + F^C_{n+1}) + dt/M b (F^D' + F^R)
template <typename T>
__global__ void k_update_v(int64_t n3, const double *__restrict__ R, double *__restrict__ V, double *__restrict__ FC,
                           const double *__restrict__ FCn, const T *__restrict__ FD, const T *__restrict__ FR, double a,
                           double half_dt_m, double dtb_m, int *flags, long long *flag_step,
                           const long long *__restrict__ d_step)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    const double fcn = FCn[e];
    const double v = a * V[e] + half_dt_m * (a * FC[e] + fcn) +
                     dtb_m * (static_cast<double>(FD[e]) + static_cast<double>(FR[e]));
    V[e] = v;
    FC[e] = fcn;
    if (!isfinite(v) || !isfinite(R[e])) latch(flags, flag_step, GLD_ERR_NONFINITE, *d_step);
}

__global__ void k_step_advance(long long *d_step) { *d_step += 1; }

// ---------------------------------------------------------------------------
// Spectrum check: Lanczos on P (no reorthogonalisation, extreme Ritz values)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_lanczos_start(int64_t n, uint64_t seed, long long salt, T *__restrict__ q)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T z[3];
    BoxMuller<T>::gauss3(philox_at(seed, static_cast<uint32_t>(i), salt, 1u), z);
    q[4 * i] = z[0];
    q[4 * i + 1] = z[1];
    q[4 * i + 2] = z[2];
    q[4 * i + 3] = T(0);
}

// partial[block] = sum x*y over flat arrays of m entries
template <typename T>
__global__ __launch_bounds__(256) void k_dot(int64_t m, const T *__restrict__ x, const T *__restrict__ y,
                                             double *__restrict__ partial)
{
    __shared__ double sh[256];
    double s = 0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        s += static_cast<double>(x[e]) * static_cast<double>(y[e]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// out = sum(partial) (mode 0) or sqrt(sum) (mode 1)
__global__ __launch_bounds__(256) void k_dot_finish(const double *__restrict__ partial, int nb, double *out, int mode)
{
    __shared__ double sh[256];
    double s = 0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) s += partial[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = mode ? sqrt(sh[0]) : sh[0];
}

// The sum of nb partials in a fixed order (thread k takes k, k + 256, ...,
// then a tree), identical in every block that calls it.  sh: 256 doubles.
__device__ double sum_partials(const double *__restrict__ partial, int nb, double *sh)
{
    double s = 0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) s += partial[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One Lanczos step after the mat-vec w = P q, in two launches of nb blocks
// (the dot products' second stage folded into the next kernel):
//   orth_norm:  alpha = sum(partial_a) (q.w), w <- w - alpha q - beta_prev q_prev,
//               partial_b[block] = this block's part of |w|^2
//   scale_norm: beta = sqrt(sum(partial_b)), q_next = w / beta
// Block 0 stores alpha and beta.  Each partial sum is k_dot's (same grid,
// same stride, same tree) and each total k_dot_finish's, so the recurrence
// is the one the separate launches computed, bit for bit.
template <typename T>
__global__ __launch_bounds__(256) void k_lanczos_orth_norm(int64_t m, T *__restrict__ w, const T *__restrict__ q,
                                                          const T *__restrict__ qp, const double *__restrict__ partial_a,
                                                          int nb, double *alpha_out, const double *beta_prev,
                                                          double *__restrict__ partial_b)
{
    __shared__ double sh[256];
    const double alpha = sum_partials(partial_a, nb, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
    const T a = static_cast<T>(alpha);
    const T bp = beta_prev ? static_cast<T>(*beta_prev) : T(0);
    double s = 0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        T v = w[e] - a * q[e];
        if (beta_prev) v -= bp * qp[e];
        w[e] = v;
        s += static_cast<double>(v) * static_cast<double>(v);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial_b[blockIdx.x] = sh[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_lanczos_scale_norm(int64_t m, const T *__restrict__ w,
                                                           const double *__restrict__ partial_b, int nb,
                                                           double *beta_out, T *__restrict__ qn)
{
    __shared__ double sh[256];
    const double b = sqrt(sum_partials(partial_b, nb, sh));
    if (blockIdx.x == 0 && threadIdx.x == 0) *beta_out = b;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        qn[e] = b > 0 ? static_cast<T>(static_cast<double>(w[e]) / b) : T(0);
}

// q <- q / |q| using a precomputed norm
template <typename T>
__global__ void k_lanczos_normalize(int64_t m, T *__restrict__ q, const double *__restrict__ nrm)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m) return;
    q[e] = static_cast<T>(static_cast<double>(q[e]) / *nrm);
}

// Sturm count: number of eigenvalues of the tridiagonal (alpha, beta) below x
__device__ int sturm_count(const double *al, const double *be, int k, double x)
{
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
        const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
        d = al[i] - x - (i > 0 ? b2 / d : 0.0);
        if (d == 0.0) d = 1e-300;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// Extreme Ritz values of the tridiagonal (al, be) by multisection on one
// wave: each round the 64 lanes take the Sturm counts at 64 points inside the
// bracket and keep the sub-interval where the count first reaches the target
// (the bracket shrinks 65-fold per round, down to the rounding of the points).
// Checks them against the noise interval and the singular points:
// result[0] = theta_min, result[1] = theta_max.  A smallest Ritz value below
// lo_t (the tight plan's lower end) retires the tight plan for good (until a
// new state is written).
__device__ double ritz_extreme(const double *al, const double *be, int kk, double a, double b, int target)
{
    const int lane = threadIdx.x;
    for (int round = 0; round < 40; ++round) {
        const double x = a + (b - a) * (static_cast<double>(lane + 1) / 65.0);
        const bool hit = sturm_count(al, be, kk, x) >= target;
        const unsigned long long m = __ballot(hit);
        // first point at or past the target count (none: the last sub-interval)
        const int f = m ? __ffsll(static_cast<long long>(m)) - 1 : 64;
        const double na = f == 0 ? a : a + (b - a) * (static_cast<double>(f) / 65.0);
        const double nb = f == 64 ? b : a + (b - a) * (static_cast<double>(f + 1) / 65.0);
        if (!(nb - na < b - a)) break;  // no further progress in double precision
        a = na;
        b = nb;
    }
    return 0.5 * (a + b);
}

__global__ __launch_bounds__(64) void k_lanczos_judge(const double *al, const double *be, int k, double lo,
                                                      double hi, double sing_lo, double sing_hi, double lo_t,
                                                      double *result, int *flags, long long *flag_step,
                                                      const long long *d_step, int *retired)
{
    // the tridiagonal in LDS: every Sturm count of the multisection walks it
    __shared__ double sal[kMaxCheckIters], sbe[kMaxCheckIters];
    for (int i = threadIdx.x; i < k; i += 64) {
        sal[i] = al[i];
        sbe[i] = be[i];
    }
    __syncthreads();
    al = sal;
    be = sbe;
    // effective dimension: stop at the first (near) breakdown
    int kk = k;
    for (int i = 0; i < k - 1; ++i)
        if (!(be[i] > 1e-300)) { kk = i + 1; break; }
    double gl = 1e300, gh = -1e300;
    for (int i = 0; i < kk; ++i) {
        const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < kk - 1 ? fabs(be[i]) : 0.0);
        gl = fmin(gl, al[i] - r);
        gh = fmax(gh, al[i] + r);
    }
    const double tmin = ritz_extreme(al, be, kk, gl, gh, 1);
    const double tmax = ritz_extreme(al, be, kk, gl, gh, kk);
    if (threadIdx.x != 0) return;
    result[0] = tmin;
    result[1] = tmax;
    if (tmin < lo_t) *retired = 1;
    if (!(tmin > sing_lo) || !(tmax < sing_hi)) latch(flags, flag_step, GLD_ERR_NOT_PD, *d_step);
    else if (tmin < lo || tmax > hi) latch(flags, flag_step, GLD_ERR_INTERVAL, *d_step);
}

// ---------------------------------------------------------------------------
// white noise export
// ---------------------------------------------------------------------------
__global__ void k_white(uint64_t seed, int64_t n, long long t0, int64_t nt, double *out, uint32_t *raw)
{
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n * nt) return;
    const int64_t t = g / n, i = g - t * n;
    const U4 x = philox_at(seed, static_cast<uint32_t>(i), t0 + t, 0u);
    if (raw) {
        raw[4 * g] = x.x;
        raw[4 * g + 1] = x.y;
        raw[4 * g + 2] = x.z;
        raw[4 * g + 3] = x.w;
    }
    if (out) {
        double z[3];
        BoxMuller<double>::gauss3(x, z);
        out[3 * g] = z[0];
        out[3 * g + 1] = z[1];
        out[3 * g + 2] = z[2];
    }
}

inline unsigned blocks(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

template <typename T>
hipError_t spectrum_check_t(const Dev &d, hipStream_t st, int iters, double lo, double hi, double sing_lo,
                            double sing_hi, long long salt);

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
hipError_t launch_fill_zero_work(const Dev &d, void *p, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (d.fp64) k_zero_work<double><<<blocks(count, 256), 256, 0, st>>>(static_cast<double *>(p), count);
    else k_zero_work<float><<<blocks(count, 256), 256, 0, st>>>(static_cast<float *>(p), count);
    return hipGetLastError();
}


hipError_t launch_history(const Dev &d, hipStream_t st)
{
    return d.fp64 ? history_t<double>(d, st) : history_t<float>(d, st);
}

// padded ranks and, per work precision, the steps of one filter block:
// block * rcap <= 64 (FP32) or <= 32 (FP64), the accumulator rows of the
// filter bank's MFMA tiles
int fir_rcap_for(int rank)
{
    static const int caps[] = {4, 6, 8, 12, 16, 24, 32};
    for (int c : caps)
        if (rank <= c) return c;
    return 32;
}

int fir_block_for(int fp64, int rcap)
{
    // block * rcap <= 64 rows in both precisions (FP32: two 32-row MFMA
    // tiles; FP64: up to four 16-row tiles)
    (void)fp64;
    switch (rcap) {
    case 4: return 16;
    case 6: return 10;
    case 8: return 8;
    case 12: return 5;
    case 16: return 4;
    case 24: return 2;
    default: return 2;
    }
}

hipError_t launch_white_ring(const Dev &d, int mode, hipStream_t st)
{
    const unsigned gy = mode == 0 ? 1u : static_cast<unsigned>(2 * d.fir_half + 2 * d.fir_block);
    const dim3 grid(blocks(d.n, 256), gy);
    if (d.fp64)
        k_white_ring<double><<<grid, 256, 0, st>>>(d.n, d.S, d.seed, d.d_step, mode, d.fir_block, d.fir_half,
                                                    d.wring_len, static_cast<double *>(d.wring));
    else
        k_white_ring<float><<<grid, 256, 0, st>>>(d.n, d.S, d.seed, d.d_step, mode, d.fir_block, d.fir_half,
                                                   d.wring_len, static_cast<float *>(d.wring));
    return hipGetLastError();
}

hipError_t launch_fir(const Dev &d, int mode, hipStream_t st)
{
    // block * rcap <= 64 for every padded rank: the rows of the MFMA tiles
    // (FP64: four 16-row tiles above 32 rows, else two)
    const int64_t M = 3 * d.S;
    FirPart part;
    part.ustride = static_cast<int64_t>(fir_rows(d.fp64)) * M;
    part.ahead = mode == 1 ? 0 : 1;
    part.spread = mode == 0;
    part.period = fir_period(d.fir_block);
    part.nslice = mode == 0 ? d.fir_block / part.period : 1;
    part.cs = mode == 0 ? (M / part.nslice + 1 + kFirMfmaThreads - 1) / kFirMfmaThreads * kFirMfmaThreads : M;
    const unsigned grid = static_cast<unsigned>((part.cs + kFirMfmaThreads - 1) / kFirMfmaThreads);
    // window: t = n0 - half .. n0 + bf - 1 + half (2 half + 1 taps, bf outputs)
    const int span = 2 * d.fir_half + d.fir_block;
    if (d.fp64 && d.fir_block * d.fir_rcap > 32)
        k_fir_mfma64<0, 4><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.fir_block, d.fir_rcap, d.fir_half, span,
                                                             d.wring_len, static_cast<const double *>(d.Afilt),
                                                             static_cast<const double *>(d.wring), d.d_step,
                                                             static_cast<double *>(d.U), part);
    else if (d.fp64)
        k_fir_mfma64<0, 2><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.fir_block, d.fir_rcap, d.fir_half, span,
                                                             d.wring_len, static_cast<const double *>(d.Afilt),
                                                             static_cast<const double *>(d.wring), d.d_step,
                                                             static_cast<double *>(d.U), part);
    else
        k_fir_mfma<0><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.fir_block, d.fir_rcap, d.fir_half, span,
                                                        d.wring_len, static_cast<const float *>(d.Afilt),
                                                        static_cast<const float *>(d.wring), d.d_step,
                                                        static_cast<float *>(d.U), part);
    return hipGetLastError();
}

// noise window: the random force of the step is slot (step mod W) of the
// forces the window computed
template <typename T>
__global__ void k_take_window(int64_t len, const T *__restrict__ FRw, T *__restrict__ FR, int W,
                              const long long *__restrict__ d_step)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const int64_t slot = *d_step % W;
    FR[i] = FRw[slot * len + i];
}

hipError_t launch_take_window(const Dev &d, hipStream_t st)
{
    const int64_t len = 3 * d.S;
    if (d.fp64)
        k_take_window<double><<<blocks(len, 256), 256, 0, st>>>(len, static_cast<const double *>(d.FRw),
                                                                static_cast<double *>(d.FR), d.win, d.d_step);
    else
        k_take_window<float><<<blocks(len, 256), 256, 0, st>>>(len, static_cast<const float *>(d.FRw),
                                                               static_cast<float *>(d.FR), d.win, d.d_step);
    return hipGetLastError();
}

hipError_t launch_history_block(const Dev &d, int mode, hipStream_t st)
{
    if (d.nslots == 0) return hipSuccess;
    // the lags m > j + HB of step n0 + j of a block: the ring slices
    // t = n0 - (M - 1) .. n0 - HB - 1 (span nslots - HB) against the taps
    // (K^s_m, g_m), m = M - 1 .. 1, for the HB steps of the block
    const int64_t M = 3 * d.S;
    const int span = std::max(0, d.nslots - d.hist_block);
    FirPart part;
    part.ustride = static_cast<int64_t>(2 * d.hist_block) * M;
    part.ahead = mode == 1 ? 0 : 1;
    part.nsplit = kHistSplit;
    part.spread = mode == 0;
    part.period = kHistPeriod;
    part.nslice = mode == 0 ? d.hist_block / (kHistPeriod * kHistSplit) : 1;
    part.cs = mode == 0 ? (M / part.nslice + 1 + kFirMfmaThreads - 1) / kFirMfmaThreads * kFirMfmaThreads : M;
    const unsigned grid = static_cast<unsigned>((part.cs + kFirMfmaThreads - 1) / kFirMfmaThreads);
    for (int q = 0; q < (mode == 0 ? 1 : kHistSplit); ++q) {
        part.split = q;
        if (d.fp64)
            k_fir_mfma64<1, 2><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.hist_block, 2, d.nslots, span, d.nslots,
                                                              static_cast<const double *>(d.hist_taps),
                                                              static_cast<const double *>(d.ring), d.d_step,
                                                              static_cast<double *>(d.Uh), part);
        else
            k_fir_mfma<1><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.hist_block, 2, d.nslots, span, d.nslots,
                                                            static_cast<const float *>(d.hist_taps),
                                                            static_cast<const float *>(d.ring), d.d_step,
                                                            static_cast<float *>(d.Uh), part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_update_r(const Dev &d, hipStream_t st)
{
    const double c_v = d.dt * d.b, c_f = d.dt * d.dt / (2.0 * d.mass) * d.b;
    // element-wise over the whole padded [3][S] vectors (padding stays zero)
    const int64_t len = 3 * d.S;
    if (d.fp64)
        k_update_r<double><<<blocks(len, 256), 256, 0, st>>>(len, d.R, d.V, d.FC, (const double *)d.FD,
                                                              (const double *)d.FR, (double *)d.ring, 3 * d.S,
                                                              d.nslots, d.d_step, c_v, c_f);
    else
        k_update_r<float><<<blocks(len, 256), 256, 0, st>>>(len, d.R, d.V, d.FC, (const float *)d.FD,
                                                             (const float *)d.FR, (float *)d.ring, 3 * d.S,
                                                             d.nslots, d.d_step, c_v, c_f);
    return hipGetLastError();
}

hipError_t launch_update_v(const Dev &d, hipStream_t st)
{
    const int64_t len = 3 * d.S;
    const double half = d.dt / (2.0 * d.mass), dtb = d.dt / d.mass * d.b;
    if (d.fp64)
        k_update_v<double><<<blocks(len, 256), 256, 0, st>>>(len, d.R, d.V, d.FC, d.FCn, (const double *)d.FD,
                                                              (const double *)d.FR, d.a, half, dtb, d.d_flags,
                                                              d.d_flag_step, d.d_step);
    else
        k_update_v<float><<<blocks(len, 256), 256, 0, st>>>(len, d.R, d.V, d.FC, d.FCn, (const float *)d.FD,
                                                             (const float *)d.FR, d.a, half, dtb, d.d_flags,
                                                             d.d_flag_step, d.d_step);
    return hipGetLastError();
}

hipError_t launch_step_advance(const Dev &d, hipStream_t st)
{
    k_step_advance<<<1, 1, 0, st>>>(d.d_step);
    return hipGetLastError();
}

namespace {
template <typename T>
hipError_t spectrum_check_t(const Dev &d, hipStream_t st, int iters, double lo, double hi, double sing_lo,
                            double sing_hi, long long salt)
{
    const int64_t n = d.n, m = 4 * n;  // sorted T4 vectors, the 4th entry stays zero
    T *q[3] = {static_cast<T *>(d.lq[0]), static_cast<T *>(d.lq[1]), static_cast<T *>(d.lq[2])};
    T *w = static_cast<T *>(d.lw);
    double *al = d.lab, *be = d.lab + kMaxCheckIters, *res = d.lab + 2 * kMaxCheckIters;
    const unsigned nbd = static_cast<unsigned>(std::min<int64_t>(kPartials, blocks(m, 256)));
    const unsigned ne = blocks(m, 256);
    k_lanczos_start<T><<<blocks(n, 256), 256, 0, st>>>(n, d.seed, salt, q[0]);
    k_dot<T><<<nbd, 256, 0, st>>>(m, q[0], q[0], d.partial);
    k_dot_finish<<<1, 256, 0, st>>>(d.partial, nbd, res + 2, 1);
    k_lanczos_normalize<T><<<ne, 256, 0, st>>>(m, q[0], res + 2);
    iters = std::min(iters, kMaxCheckIters);
    for (int k = 0; k < iters; ++k) {
        T *qc = q[k % 3], *qp = q[(k + 2) % 3], *qn = q[(k + 1) % 3];
        hipError_t e = launch_spmv(d, st, 1.0, 0.0, qc, 0.0, nullptr, nullptr, 0, w, nullptr, nullptr);
        if (e != hipSuccess) return e;
        k_dot<T><<<nbd, 256, 0, st>>>(m, qc, w, d.partial);
        k_lanczos_orth_norm<T><<<nbd, 256, 0, st>>>(m, w, qc, qp, d.partial, nbd, al + k,
                                                    k > 0 ? be + k - 1 : nullptr, d.partial + kPartials);
        k_lanczos_scale_norm<T><<<nbd, 256, 0, st>>>(m, w, d.partial + kPartials, nbd, be + k, qn);
    }
    k_lanczos_judge<<<1, 64, 0, st>>>(al, be, iters, lo, hi, sing_lo, sing_hi, d.lam_lo_tight, res, d.d_flags,
                                      d.d_flag_step, d.d_step, d.d_retired);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_spectrum_check(const Dev &d, hipStream_t st, int iters, double lo, double hi, double sing_lo,
                                 double sing_hi, long long salt)
{
    return d.fp64 ? spectrum_check_t<double>(d, st, iters, lo, hi, sing_lo, sing_hi, salt)
                  : spectrum_check_t<float>(d, st, iters, lo, hi, sing_lo, sing_hi, salt);
}

hipError_t launch_white_noise(uint64_t seed, int64_t n, int64_t t0, int64_t nt, double *out, uint32_t *raw,
                              hipStream_t st)
{
    if (n * nt == 0) return hipSuccess;
    k_white<<<blocks(n * nt, 256), 256, 0, st>>>(seed, n, t0, nt, out, raw);
    return hipGetLastError();
}

}  // namespace gld
