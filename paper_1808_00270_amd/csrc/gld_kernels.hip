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

namespace gld {

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller.
// Counter (particle, step lo, step hi, stream), key (seed lo, seed hi).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        U4 o;
        o.x = hi1 ^ c.y ^ k0;
        o.y = lo1;
        o.z = hi0 ^ c.w ^ k1;
        o.w = lo0;
        c = o;
    }
    return c;
}

__device__ __forceinline__ U4 philox_at(uint64_t seed, uint32_t pid, long long t, uint32_t stream)
{
    const unsigned long long tu = static_cast<unsigned long long>(t);
    U4 c{pid, static_cast<uint32_t>(tu), static_cast<uint32_t>(tu >> 32), stream};
    return philox10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
}

template <typename T>
struct BoxMuller;

template <>
struct BoxMuller<double> {
    __device__ static void gauss3(U4 x, double z[3])
    {
        const double s = 1.0 / 4294967296.0;
        const double u0 = (static_cast<double>(x.x) + 0.5) * s, u1 = (static_cast<double>(x.y) + 0.5) * s;
        const double u2 = (static_cast<double>(x.z) + 0.5) * s, u3 = (static_cast<double>(x.w) + 0.5) * s;
        const double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
        double sa, ca, cb, sb;
        sincos(6.283185307179586476925286766559 * u1, &sa, &ca);
        sincos(6.283185307179586476925286766559 * u3, &sb, &cb);
        z[0] = ra * ca;
        z[1] = ra * sa;
        z[2] = rb * cb;
    }
};

template <>
struct BoxMuller<float> {
    __device__ static void gauss3(U4 x, float z[3])
    {
        // uniforms formed in double (exact), transcendental part in float
        const double s = 1.0 / 4294967296.0;
        const float u0 = static_cast<float>((static_cast<double>(x.x) + 0.5) * s);
        const float u1 = static_cast<float>((static_cast<double>(x.y) + 0.5) * s);
        const float u2 = static_cast<float>((static_cast<double>(x.z) + 0.5) * s);
        const float u3 = static_cast<float>((static_cast<double>(x.w) + 0.5) * s);
        const float ra = sqrtf(-2.0f * logf(u0)), rb = sqrtf(-2.0f * logf(u2));
        float sa, ca, sb, cb;
        sincosf(6.28318530717958647692f * u1, &sa, &ca);
        sincosf(6.28318530717958647692f * u3, &sb, &cb);
        z[0] = ra * ca;
        z[1] = ra * sa;
        z[2] = rb * cb;
    }
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void latch(int *flags, long long *flag_step, int code, long long step)
{
    if (atomicCAS(flags, 0, code) == 0) *flag_step = step;
}

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
// the lags m > j reach only displacements from before n0, which the ring
// already holds when the block starts; for all j at once these sums are one
// product (the filter bank's kernel on the matrix cores, ROLE 1):
//   Uh[j][0] = sum_{m=j+1}^{M-1} K^s_m dR_{n0+j-m},  Uh[j][1] likewise with g_m,
// which reads the ring once per block instead of once per step.  Each step
// then adds its lags m <= j (the block's own displacements) directly.  The
// sums are those of the definition, taken in another order.
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
        const auto ud = load4<T>(Uh + (2 * static_cast<int64_t>(j)) * n3 + e0);
        const auto uh = load4<T>(Uh + (2 * static_cast<int64_t>(j) + 1) * n3 + e0);
        d[0] = ud.x;
        d[1] = ud.y;
        d[2] = ud.z;
        d[3] = ud.w;
        h[0] = uh.x;
        h[1] = uh.y;
        h[2] = uh.z;
        h[3] = uh.w;
    }
    const int mm = min(j, nslots);
    for (int m = 1; m <= mm; ++m) {
        long long t = (step - m) % nslots;
        if (t < 0) t += nslots;
        const auto x = load4<T>(ring + t * n3 + e0);
        const T k = ks[m], q = gm[m];
        d[0] += k * x.x;
        d[1] += k * x.y;
        d[2] += k * x.z;
        d[3] += k * x.w;
        h[0] += q * x.x;
        h[1] += q * x.y;
        h[2] += q * x.z;
        h[3] += q * x.w;
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
__device__ __forceinline__ int ring_slot(long long t, int len)
{
    long long m = t % len;
    return static_cast<int>(m < 0 ? m + len : m);
}

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
        t = cur + half + bf - 1;
    } else if (mode == 1) {
        if (y >= len) return;
        t = n0 - half + y;
    } else {
        if (y >= cur - n0) return;
        t = n0 + half + bf + y;
    }
    T w[3];
    BoxMuller<T>::gauss3(philox_at(seed, static_cast<uint32_t>(i), t, 0u), w);
    T *dst = W + static_cast<int64_t>(ring_slot(t, len)) * 3 * S;
    dst[i] = w[0];
    dst[S + i] = w[1];
    dst[2 * S + i] = w[2];
}

// FP32 filter bank on the matrix cores.  For the block of steps starting at
// n0 the outputs are a product of two matrices:
//   U[b][q][m] = sum_k Ash[k][(b,q)] X[k][m],
//   X[k][m]    = W at window step k (ring slot of n0 - half + k), channel m
//                (m = component * S + particle), k < span = P + BF - 1,
//   Ash[k][(b,q)] = A[k - b][q] for 0 <= k - b < P, else 0.
// Each wave owns 64 channels and all BF*RC <= 64 rows (b,q): four 32x32
// accumulator tiles of v_mfma_f32_32x32x2f32, which takes two k per
// instruction (lanes 0-31 the first, 32-63 the second).  The channel operand
// is a 128-byte segment of one ring slice per half-wave; the tap operand
// comes from the taps staged in LDS in chunks of kFirChunk window steps.  The
// ring loads run two batches of kFirUnroll k-pairs ahead; past the window they
// read other (finite) ring slices, which meet zero taps.
// The taps come zero-padded (see kFirChunk): row t + bf - 1 holds A[t], so
// a chunk's rows are one contiguous copy.
typedef float fir_v16f __attribute__((ext_vector_type(16)));
constexpr int kFirMfmaThreads = 256;  // four waves, 256 channels
constexpr int kFirUnroll = 8;         // MFMA k-pairs per batch
constexpr int kFirStageIt = ((kFirChunk + kMaxFirBlock - 1) * kMaxRank / 2 + kFirMfmaThreads - 1) / kFirMfmaThreads;

template <int ROLE>
__global__ __launch_bounds__(kFirMfmaThreads) void k_fir_mfma(int64_t n, int64_t S, int bf, int rc, int offset,
                                                              int span, int len, const float *__restrict__ A,
                                                              const float *__restrict__ W,
                                                              const long long *__restrict__ d_step,
                                                              float *__restrict__ U, int force)
{
    __shared__ __align__(16) float taps[(kFirChunk + kMaxFirBlock - 1) * kMaxRank];
    const long long cur = *d_step;
    if (!force && cur % bf != 0) return;
    const long long n0 = cur - cur % bf;
    const int64_t M = 3 * S;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t m0 = (static_cast<int64_t>(blockIdx.x) * (kFirMfmaThreads / 64) + (tid >> 6)) * 64;
    const bool wlive = m0 < M;  // a wave past the channels only joins the staging
    const int hi = lane >> 5, lo = lane & 31;
    // this lane's tap rows i = 32 rt + lo, i.e. (b, q) = (i / rc, i % rc)
    // (rows past bf * rc read a valid tap and multiply it by 0, so the LDS
    // reads carry no branch)
    int trow[2];
    float tmul[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int i = 32 * rt + lo;
        const bool valid = i < bf * rc;
        tmul[rt] = valid ? 1.f : 0.f;
        trow[rt] = (bf - 1 - (valid ? i / rc : 0)) * rc + (valid ? i % rc : 0);
    }
    // channel columns of this lane (clamped for a dead wave: never stored)
    const int64_t c0 = wlive ? m0 + lo : lo;
    fir_v16f acc[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = fir_v16f{};
    // ring slot of this lane's window step k = 2 j + hi, and its channel c0
    // there (c1 = c0 + 32 follows at a fixed offset)
    int sl = ring_slot(n0 - offset + hi, len);
    const float *src = W + static_cast<int64_t>(sl) * M + c0;
    const int64_t wrap = static_cast<int64_t>(len) * M;
    // window step of the next load.  The history's taps reach past the span
    // (ROLE 1): its steps there count zero (the loads read other, finite
    // ring slices and are multiplied by 0, which keeps them unconditional);
    // the noise filters' taps are zero there already (ROLE 0)
    [[maybe_unused]] int kw = hi;
    float xa[kFirUnroll][2], xn[kFirUnroll][2], xm[kFirUnroll][2];
    auto load_batch = [&](float (&dst)[kFirUnroll][2]) {
#pragma unroll
        for (int u = 0; u < kFirUnroll; ++u) {
            if constexpr (ROLE == 1) {
                const float in = kw < span ? 1.f : 0.f;
                dst[u][0] = __builtin_nontemporal_load(src) * in;
                dst[u][1] = __builtin_nontemporal_load(src + 32) * in;
                kw += 2;
            } else {
                dst[u][0] = __builtin_nontemporal_load(src);
                dst[u][1] = __builtin_nontemporal_load(src + 32);
            }
            sl += 2;
            src += 2 * M;
            if constexpr (ROLE == 1) {
                while (sl >= len) {  // the history ring (m_max - 1 slices) can be shorter than 2
                    sl -= len;
                    src -= wrap;
                }
            } else if (sl >= len) {  // the white-noise ring holds at least 4 slices
                sl -= len;
                src -= wrap;
            }
        }
    };
    load_batch(xa);
    load_batch(xn);
    for (int k0 = 0; k0 < span; k0 += kFirChunk) {
        // taps of window steps [k0, k0 + kFirChunk) for every b: padded rows
        // k0 .. k0 + kFirChunk + bf - 2 (t = k0 - (bf - 1) ..), loaded before
        // the barrier that retires the previous chunk
        const int nel = (kFirChunk + bf - 1) * rc / 2;  // float2 (rc is even)
        const float2 *srcA = reinterpret_cast<const float2 *>(A + static_cast<int64_t>(k0) * rc);
        float2 tv[kFirStageIt];
#pragma unroll
        for (int j = 0; j < kFirStageIt; ++j) {
            const int e = tid + j * kFirMfmaThreads;
            tv[j] = e < nel ? srcA[e] : make_float2(0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kFirStageIt; ++j) {
            const int e = tid + j * kFirMfmaThreads;
            if (e < nel) reinterpret_cast<float2 *>(taps)[e] = tv[j];
        }
        __syncthreads();
#pragma unroll 1
        for (int kk = 0; kk < kFirChunk; kk += 2 * kFirUnroll) {
            load_batch(xm);  // two batches ahead
#pragma unroll
            for (int u = 0; u < kFirUnroll; ++u) {
                const int kl = kk + 2 * u + hi;  // window step k0 + kl of this lane
                float av[2];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) av[rt] = taps[kl * rc + trow[rt]] * tmul[rt];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rt], xa[u][ct], acc[rt][ct], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < kFirUnroll; ++u) {
                xa[u][0] = xn[u][0];
                xa[u][1] = xn[u][1];
                xn[u][0] = xm[u][0];
                xn[u][1] = xm[u][1];
            }
        }
    }
    if (!wlive) return;
    // accumulator element v of tile (rt, ct): row i = 32 rt + (v % 4) + 4 hi
    // + 8 (v / 4), channel m0 + 32 ct + lo
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const int64_t m = m0 + 32 * ct + lo;
        const int64_t p = m - (m >= S ? S : 0) - (m >= 2 * S ? S : 0);  // particle of channel m
        if (p >= n) continue;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 32 * rt + (v % 4) + 4 * hi + 8 * (v / 4);
                if (i < bf * rc) U[static_cast<int64_t>(i) * M + m] = acc[rt][ct][v];
            }
    }
}

// FP64 filter bank on the matrix cores, the same product with
// v_mfma_f64_16x16x4f64 (four k per instruction, lanes 16 g .. 16 g + 15
// taking k = g): each wave owns 64 channels (four 16-wide column tiles) and
// the bf * rc <= 32 rows (two 16-row tiles); accumulator element v of a tile
// is row 4 v + g, column lane % 16.  Taps are staged in chunks of
// kFirChunk64 window steps.
typedef double fir_v4d __attribute__((ext_vector_type(4)));
constexpr int kFirChunk64 = 64;
constexpr int kFirUnroll64 = 4;  // MFMA k-quads per batch
constexpr int kFirStageIt64 =
    ((kFirChunk64 + kMaxFirBlock - 1) * kMaxRank / 2 + kFirMfmaThreads - 1) / kFirMfmaThreads;

template <int ROLE>
__global__ __launch_bounds__(kFirMfmaThreads) void k_fir_mfma64(int64_t n, int64_t S, int bf, int rc, int offset,
                                                                int span, int len, const double *__restrict__ A,
                                                                const double *__restrict__ W,
                                                                const long long *__restrict__ d_step,
                                                                double *__restrict__ U, int force)
{
    __shared__ __align__(16) double taps[(kFirChunk64 + kMaxFirBlock - 1) * kMaxRank];
    const long long cur = *d_step;
    if (!force && cur % bf != 0) return;
    const long long n0 = cur - cur % bf;
    const int64_t M = 3 * S;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t m0 = (static_cast<int64_t>(blockIdx.x) * (kFirMfmaThreads / 64) + (tid >> 6)) * 64;
    const bool wlive = m0 < M;
    const int g = lane >> 4, lo = lane & 15;
    int trow[2];
    double tmul[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int i = 16 * rt + lo;
        const bool valid = i < bf * rc;
        tmul[rt] = valid ? 1.0 : 0.0;
        trow[rt] = (bf - 1 - (valid ? i / rc : 0)) * rc + (valid ? i % rc : 0);
    }
    const int64_t c0 = wlive ? m0 + lo : lo;
    fir_v4d acc[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = fir_v4d{};
    // ring slot of this lane's window step k = 4 j + g
    int sl = ring_slot(n0 - offset + g, len);
    const double *src = W + static_cast<int64_t>(sl) * M + c0;
    const int64_t wrap = static_cast<int64_t>(len) * M;
    // window step of the next load (ROLE 1, the history: past the span
    // multiplied by 0, as in the FP32 kernel)
    [[maybe_unused]] int kw = g;
    double xa[kFirUnroll64][4], xn[kFirUnroll64][4];
    auto load_batch = [&](double (&dst)[kFirUnroll64][4]) {
#pragma unroll
        for (int u = 0; u < kFirUnroll64; ++u) {
            if constexpr (ROLE == 1) {
                const double in = kw < span ? 1.0 : 0.0;
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) dst[u][ct] = __builtin_nontemporal_load(src + 16 * ct) * in;
                kw += 4;
            } else {
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) dst[u][ct] = __builtin_nontemporal_load(src + 16 * ct);
            }
            sl += 4;
            src += 4 * M;
            if constexpr (ROLE == 1) {
                while (sl >= len) {  // the history ring (m_max - 1 slices) can be shorter than 4
                    sl -= len;
                    src -= wrap;
                }
            } else if (sl >= len) {  // the white-noise ring holds at least 4 slices
                sl -= len;
                src -= wrap;
            }
        }
    };
    load_batch(xa);
    for (int k0 = 0; k0 < span; k0 += kFirChunk64) {
        const int nel = (kFirChunk64 + bf - 1) * rc / 2;  // double2 (rc is even)
        const double2 *srcA = reinterpret_cast<const double2 *>(A + static_cast<int64_t>(k0) * rc);
        double2 tv[kFirStageIt64];
#pragma unroll
        for (int j = 0; j < kFirStageIt64; ++j) {
            const int e = tid + j * kFirMfmaThreads;
            tv[j] = e < nel ? srcA[e] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kFirStageIt64; ++j) {
            const int e = tid + j * kFirMfmaThreads;
            if (e < nel) reinterpret_cast<double2 *>(taps)[e] = tv[j];
        }
        __syncthreads();
#pragma unroll 1
        for (int kk = 0; kk < kFirChunk64; kk += 4 * kFirUnroll64) {
            load_batch(xn);
#pragma unroll
            for (int u = 0; u < kFirUnroll64; ++u) {
                const int kl = kk + 4 * u + g;
                double av[2];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) av[rt] = taps[kl * rc + trow[rt]] * tmul[rt];
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], xa[u][ct], acc[rt][ct], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < kFirUnroll64; ++u)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) xa[u][ct] = xn[u][ct];
        }
    }
    if (!wlive) return;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int64_t m = m0 + 16 * ct + lo;
        const int64_t p = m - (m >= S ? S : 0) - (m >= 2 * S ? S : 0);
        if (p >= n) continue;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt + 4 * v + g;
                if (i < bf * rc) U[static_cast<int64_t>(i) * M + m] = acc[rt][ct][v];
            }
    }
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

// w <- w - alpha q - beta_prev q_prev   (beta_prev = 0 for the first step)
template <typename T>
__global__ void k_lanczos_orth(int64_t m, T *__restrict__ w, const T *__restrict__ q, const T *__restrict__ qp,
                               const double *__restrict__ alpha, const double *__restrict__ beta_prev)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m) return;
    T v = w[e] - static_cast<T>(*alpha) * q[e];
    if (beta_prev) v -= static_cast<T>(*beta_prev) * qp[e];
    w[e] = v;
}

// q_next = w / beta
template <typename T>
__global__ void k_lanczos_scale(int64_t m, const T *__restrict__ w, const double *__restrict__ beta,
                                T *__restrict__ qn)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const double b = *beta;
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

// Extreme Ritz values by bisection; checks them against the noise interval
// and the singular points; result[0] = theta_min, result[1] = theta_max.
__global__ void k_lanczos_judge(const double *al, const double *be, int k, double lo, double hi, double sing_lo,
                                double sing_hi, double *result, int *flags, long long *flag_step,
                                const long long *d_step)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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
    double a = gl, b = gh;
    for (int it = 0; it < 200; ++it) {  // smallest eigenvalue
        const double mid = 0.5 * (a + b);
        if (sturm_count(al, be, kk, mid) >= 1) b = mid; else a = mid;
    }
    const double tmin = 0.5 * (a + b);
    a = gl;
    b = gh;
    for (int it = 0; it < 200; ++it) {  // largest eigenvalue
        const double mid = 0.5 * (a + b);
        if (sturm_count(al, be, kk, mid) >= kk) b = mid; else a = mid;
    }
    const double tmax = 0.5 * (a + b);
    result[0] = tmin;
    result[1] = tmax;
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
    switch (rcap) {
    case 4: return fp64 ? 8 : 16;
    case 6: return fp64 ? 5 : 10;
    case 8: return fp64 ? 4 : 8;
    case 12: return fp64 ? 2 : 5;
    case 16: return fp64 ? 2 : 4;
    case 24: return fp64 ? 1 : 2;
    default: return fp64 ? 1 : 2;
    }
}

hipError_t launch_white_ring(const Dev &d, int mode, hipStream_t st)
{
    const unsigned gy = mode == 0 ? 1u : (mode == 1 ? static_cast<unsigned>(d.wring_len) : static_cast<unsigned>(d.fir_block));
    const dim3 grid(blocks(d.n, 256), gy);
    if (d.fp64)
        k_white_ring<double><<<grid, 256, 0, st>>>(d.n, d.S, d.seed, d.d_step, mode, d.fir_block, d.fir_half,
                                                    d.wring_len, static_cast<double *>(d.wring));
    else
        k_white_ring<float><<<grid, 256, 0, st>>>(d.n, d.S, d.seed, d.d_step, mode, d.fir_block, d.fir_half,
                                                   d.wring_len, static_cast<float *>(d.wring));
    return hipGetLastError();
}

hipError_t launch_fir(const Dev &d, int force, hipStream_t st)
{
    // block * rcap <= 64 (FP32) or <= 32 (FP64) for every padded rank: the
    // rows of one pair of MFMA tiles
    const int64_t M = 3 * d.S;
    const unsigned grid = static_cast<unsigned>((M + kFirMfmaThreads - 1) / kFirMfmaThreads);
    // window: t = n0 - half .. n0 + bf - 1 + half (2 half + 1 taps, bf outputs)
    const int span = 2 * d.fir_half + d.fir_block;
    if (d.fp64)
        k_fir_mfma64<0><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.fir_block, d.fir_rcap, d.fir_half, span,
                                                          d.wring_len, static_cast<const double *>(d.Afilt),
                                                          static_cast<const double *>(d.wring), d.d_step,
                                                          static_cast<double *>(d.U), force);
    else
        k_fir_mfma<0><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.fir_block, d.fir_rcap, d.fir_half, span,
                                                        d.wring_len, static_cast<const float *>(d.Afilt),
                                                        static_cast<const float *>(d.wring), d.d_step,
                                                        static_cast<float *>(d.U), force);
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

hipError_t launch_history_block(const Dev &d, int force, hipStream_t st)
{
    if (d.nslots == 0) return hipSuccess;
    // the M - 1 ring slices before the block (t = n0 - (M - 1) .. n0 - 1)
    // against the taps (K^s_m, g_m), m = M - 1 .. 1; HB steps of output
    const int64_t M = 3 * d.S;
    const unsigned grid = static_cast<unsigned>((M + kFirMfmaThreads - 1) / kFirMfmaThreads);
    if (d.fp64)
        k_fir_mfma64<1><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.hist_block, 2, d.nslots, d.nslots, d.nslots,
                                                          static_cast<const double *>(d.hist_taps),
                                                          static_cast<const double *>(d.ring), d.d_step,
                                                          static_cast<double *>(d.Uh), force);
    else
        k_fir_mfma<1><<<grid, kFirMfmaThreads, 0, st>>>(d.n, d.S, d.hist_block, 2, d.nslots, d.nslots, d.nslots,
                                                        static_cast<const float *>(d.hist_taps),
                                                        static_cast<const float *>(d.ring), d.d_step,
                                                        static_cast<float *>(d.Uh), force);
    return hipGetLastError();
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
    double *al = d.lab, *be = d.lab + kCheckIters, *res = d.lab + 2 * kCheckIters;
    const unsigned nbd = static_cast<unsigned>(std::min<int64_t>(kPartials, blocks(m, 256)));
    const unsigned ne = blocks(m, 256);
    k_lanczos_start<T><<<blocks(n, 256), 256, 0, st>>>(n, d.seed, salt, q[0]);
    k_dot<T><<<nbd, 256, 0, st>>>(m, q[0], q[0], d.partial);
    k_dot_finish<<<1, 256, 0, st>>>(d.partial, nbd, res + 2, 1);
    k_lanczos_normalize<T><<<ne, 256, 0, st>>>(m, q[0], res + 2);
    iters = std::min(iters, kCheckIters);
    for (int k = 0; k < iters; ++k) {
        T *qc = q[k % 3], *qp = q[(k + 2) % 3], *qn = q[(k + 1) % 3];
        hipError_t e = launch_spmv(d, st, 1.0, 0.0, qc, 0.0, nullptr, nullptr, 0, w, nullptr, nullptr);
        if (e != hipSuccess) return e;
        k_dot<T><<<nbd, 256, 0, st>>>(m, qc, w, d.partial);
        k_dot_finish<<<1, 256, 0, st>>>(d.partial, nbd, al + k, 0);
        k_lanczos_orth<T><<<ne, 256, 0, st>>>(m, w, qc, qp, al + k, k > 0 ? be + k - 1 : nullptr);
        k_dot<T><<<nbd, 256, 0, st>>>(m, w, w, d.partial);
        k_dot_finish<<<1, 256, 0, st>>>(d.partial, nbd, be + k, 1);
        k_lanczos_scale<T><<<ne, 256, 0, st>>>(m, w, be + k, qn);
    }
    k_lanczos_judge<<<1, 1, 0, st>>>(al, be, iters, lo, hi, sing_lo, sing_hi, res, d.d_flags, d.d_flag_step,
                                     d.d_step);
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
