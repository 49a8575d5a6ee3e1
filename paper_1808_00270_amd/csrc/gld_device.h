// Device code shared by the single-system kernels (gld_kernels.hip) and the
// batched ones (gld_batch.hip): the counter-based white noise and the
// matrix-core filter bank.  Internal to libgld.
#pragma once

#include <hip/hip_runtime.h>

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


__device__ __forceinline__ void latch(int *flags, long long *flag_step, int code, long long step)
{
    if (atomicCAS(flags, 0, code) == 0) *flag_step = step;
}

__device__ __forceinline__ int ring_slot(long long t, int len)
{
    long long m = t % len;
    return static_cast<int>(m < 0 ? m + len : m);
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
// Which part of a block's product one launch computes.  The block starts at
// n0 + ahead * bf (n0 the start of the block holding the current step).
// Not spread: all channels, the window chunks of split `split`.
// Spread over the block before (launched every step, working at the steps
// that are multiples of `period`, share i = (step mod bf) / period of
// bf / period): channels [c cs, (c + 1) cs) with c = i % nslice, and the
// window chunks of split q = i / nslice of nsplit, so that every `period`
// steps of a block compute the same share of the next block's product.  Outputs go
// to U + ((block parity) nsplit + q) ustride: two blocks' outputs alternate,
// and the nsplit partial sums over the window are added by the consumer.
struct FirPart {
    int ahead = 0, nslice = 1, nsplit = 1;
    int split = 0;   // not spread: the split this launch computes
    int spread = 0;  // spread: every `period` steps the share (i % nslice, i / nslice),
    int period = 1;  // i = (step mod bf) / period, with nslice nsplit = bf / period
    int64_t cs = 0, ustride = 0;
};

typedef float fir_v16f __attribute__((ext_vector_type(16)));
constexpr int kFirMfmaThreads = 256;  // four waves, 256 channels
constexpr int kFirUnroll = 8;         // MFMA k-pairs per batch
constexpr int kFirStageIt = ((kFirChunk + kMaxFirBlock - 1) * kMaxRank / 2 + kFirMfmaThreads - 1) / kFirMfmaThreads;

template <int ROLE>
__device__ __forceinline__ void fir_mfma_body(int64_t n, int64_t S, int bf, int rc, int offset, int span, int len,
                                              const float *__restrict__ A, const float *__restrict__ W,
                                              const long long *__restrict__ d_step, float *__restrict__ U,
                                              FirPart part, int64_t tile)
{
    __shared__ __align__(16) float taps[(kFirChunk + kMaxFirBlock - 1) * kMaxRank];
    const long long cur = *d_step;
    const int64_t M = 3 * S;
    const int tid = threadIdx.x, lane = tid & 63;
    // the block of steps computed, this launch's channels and window chunks,
    // and where its outputs go (see FirPart)
    const long long n0 = cur - cur % bf + part.ahead * bf;
    int cslice = 0, ksplit = part.split;
    if (part.spread) {
        if (cur % part.period != 0) return;  // the whole grid, before any barrier
        const int i = static_cast<int>(cur % bf) / part.period;
        cslice = i % part.nslice;
        ksplit = i / part.nslice;
    }
    const int nch = (span + kFirChunk - 1) / kFirChunk;
    const int kbeg = (ksplit * nch / part.nsplit) * kFirChunk, kend = ((ksplit + 1) * nch / part.nsplit) * kFirChunk;
    U += (((n0 / bf) & 1) * part.nsplit + ksplit) * part.ustride;
    const int64_t climit = min(M, (cslice + 1) * part.cs);
    const int64_t m0 = cslice * part.cs + (tile * (kFirMfmaThreads / 64) + (tid >> 6)) * 64;
    const bool wlive = m0 < climit;  // a wave past the channels only joins the staging
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
    int sl = ring_slot(n0 - offset + kbeg + hi, len);
    const float *src = W + static_cast<int64_t>(sl) * M + c0;
    const int64_t wrap = static_cast<int64_t>(len) * M;
    // window step of the next load.  The history's taps reach past the span
    // (ROLE 1): its steps there count zero (the loads read other, finite
    // ring slices and are multiplied by 0, which keeps them unconditional);
    // the noise filters' taps are zero there already (ROLE 0)
    [[maybe_unused]] int kw = kbeg + hi;
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
    for (int k0 = kbeg; k0 < kend; k0 += kFirChunk) {
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
// the bf * rc <= 16 RT rows (RT = 2 or 4 16-row tiles); accumulator element
// v of a tile is row 4 v + g, column lane % 16.  Taps are staged in chunks
// of kFirChunk64 window steps.
typedef double fir_v4d __attribute__((ext_vector_type(4)));
constexpr int kFirChunk64 = 64;
constexpr int kFirUnroll64 = 4;  // MFMA k-quads per batch
constexpr int kFirStageIt64 =
    ((kFirChunk64 + kMaxFirBlock - 1) * kMaxRank / 2 + kFirMfmaThreads - 1) / kFirMfmaThreads;

template <int ROLE, int RT>
__device__ __forceinline__ void fir_mfma64_body(int64_t n, int64_t S, int bf, int rc, int offset, int span, int len,
                                                const double *__restrict__ A, const double *__restrict__ W,
                                                const long long *__restrict__ d_step, double *__restrict__ U,
                                                FirPart part, int64_t tile)
{
    __shared__ __align__(16) double taps[(kFirChunk64 + kMaxFirBlock - 1) * kMaxRank];
    const long long cur = *d_step;
    const int64_t M = 3 * S;
    const int tid = threadIdx.x, lane = tid & 63;
    const long long n0 = cur - cur % bf + part.ahead * bf;
    int cslice = 0, ksplit = part.split;
    if (part.spread) {
        if (cur % part.period != 0) return;  // the whole grid, before any barrier
        const int i = static_cast<int>(cur % bf) / part.period;
        cslice = i % part.nslice;
        ksplit = i / part.nslice;
    }
    const int nch = (span + kFirChunk64 - 1) / kFirChunk64;
    const int kbeg = (ksplit * nch / part.nsplit) * kFirChunk64;
    const int kend = ((ksplit + 1) * nch / part.nsplit) * kFirChunk64;
    U += (((n0 / bf) & 1) * part.nsplit + ksplit) * part.ustride;
    const int64_t climit = min(M, (cslice + 1) * part.cs);
    const int64_t m0 = cslice * part.cs + (tile * (kFirMfmaThreads / 64) + (tid >> 6)) * 64;
    const bool wlive = m0 < climit;
    const int g = lane >> 4, lo = lane & 15;
    int trow[RT];
    double tmul[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int i = 16 * rt + lo;
        const bool valid = i < bf * rc;
        tmul[rt] = valid ? 1.0 : 0.0;
        trow[rt] = (bf - 1 - (valid ? i / rc : 0)) * rc + (valid ? i % rc : 0);
    }
    const int64_t c0 = wlive ? m0 + lo : lo;
    fir_v4d acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = fir_v4d{};
    // ring slot of this lane's window step k = 4 j + g
    int sl = ring_slot(n0 - offset + kbeg + g, len);
    const double *src = W + static_cast<int64_t>(sl) * M + c0;
    const int64_t wrap = static_cast<int64_t>(len) * M;
    // window step of the next load (ROLE 1, the history: past the span
    // multiplied by 0, as in the FP32 kernel)
    [[maybe_unused]] int kw = kbeg + g;
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
    for (int k0 = kbeg; k0 < kend; k0 += kFirChunk64) {
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
                double av[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) av[rt] = taps[kl * rc + trow[rt]] * tmul[rt];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
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
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt + 4 * v + g;
                if (i < bf * rc) U[static_cast<int64_t>(i) * M + m] = acc[rt][ct][v];
            }
    }
}

}  // namespace
}  // namespace gld
