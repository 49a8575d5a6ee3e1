// The general memory model (include/gld_general.h): tabulated pair kernels
// of any rank, the distance-dependent self memory Delta K^s, and the colored
// noise by Algorithm 1 (Lanczos per frequency) on the GPU.  FP64 throughout.
//
// Device layout (one system):
//   R, V, F^D, F^R          [n][3]
//   F^C                     two buffers [n][3]: current and next positions
//   displacement ring       [n][Hs][3], dR_t at slot t mod Hs, Hs = m_max - 1
//                           (a particle's lags are contiguous, so the lanes of
//                           a wave that split the lags read one segment)
//   pair list               capacity C per particle: j, the grid coordinate
//                           t = (max(r, r_cut_min) - r0) / dr clamped at 0
//                           (Sec. III.A grid, frozen below r_cut_min; bin
//                           b = min(floor t, n_r - 2), fraction t - b) and the
//                           unit vector e = (R_i - R_j) / r
//   kernel tables           K^p [n_r][m_max], Delta K^s [n_r][m_max], K^s [m_max]
//   spectra                 S_w [m_max], K^p_hat and Delta K^s_hat [m_max][n_r]
//                           (frequency-major: one Lanczos work-group reads one row)
//   white-noise ring        [P][n][3], W_t at slot t mod P, P = 2 m_max - 1
//   window transform        F_w(n) = sum_m W_{n+m} e^{-i theta w m}, theta = 2 pi / P,
//                           [m_max][n][3] real and imaginary parts
//   Lanczos                 bases [m_max][kmax][n][3], mat-vec scratch and
//                           the per-frequency results x_w [m_max][n][3]
//
// The window transform slides by one step exactly,
//   F_w(n+1) = e^{i theta w} (F_w(n) + (W_{n+M} - W_{n-M+1}) e^{i theta w (M-1)}),
// (P = 2M - 1, so e^{-i theta w M} = e^{i theta w (M-1)}), and is recomputed
// from the ring every kAnchor steps so that rounding cannot accumulate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "gld_device.h"
#include "gld_general.h"
#include "gld_internal.h"

namespace gld {
namespace gen {
namespace {

constexpr int kThreads = 256;
constexpr int kLzThreads = 1024;    // threads of a Lanczos work-group
constexpr int kLzLanes = 4;         // lanes per particle in its mat-vec
constexpr int kLzUnroll = 2;        // pair entries a lane has in flight
constexpr int kAnchor = 256;        // steps between full window transforms
constexpr int kDftOmega = 8;        // frequencies per thread of the full transform
constexpr int kDefaultIters = 96;
constexpr size_t kMaxLds = 160 * 1024;

struct GDev {
    int64_t n = 0, n3 = 0;
    int M = 0, P = 0, Hs = 1, NR = 0, C = 1, kmax = 0;
    int parallel = 0, has_dk = 0, noise_on = 0;
    double box[3] = {0, 0, 0};
    double dt = 0, mass = 0, kT = 0, r0 = 0, dr = 0, r_cut = 0, r_cut_min = 0;
    double wca_sigma = 0, wca_eps = 0, wca_rc = 0, tol = 0, a = 0, b = 0;
    uint64_t seed = 0;
    double *R = nullptr, *V = nullptr, *FD = nullptr, *FR = nullptr, *FC0 = nullptr, *FC1 = nullptr;
    double *hist = nullptr;
    int *pj = nullptr, *cnt = nullptr;
    double *pt = nullptr, *pe = nullptr;  // grid coordinate of the distance, unit vector
    double *kp = nullptr, *dk = nullptr, *ks = nullptr;
    double *shat = nullptr, *khT = nullptr, *dkhT = nullptr;
    double *cosP = nullptr, *tw = nullptr;  // tw: [4][M] cos, sin of theta w and of theta w (M-1)
    double *ring = nullptr, *delta = nullptr, *Fre = nullptr, *Fim = nullptr;
    double *KV = nullptr, *X = nullptr, *Vb = nullptr;
    int *kprev = nullptr;
    int *flags = nullptr;
    long long *flag_step = nullptr;
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a Lanczos work-group (kLzThreads lanes) in a fixed order; every
// thread gets the total.  red: kLzThreads / 64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kLzThreads / 64; ++k) s += red[k];
    return s;
}

// grid coordinate of a distance: r clamped to [r_cut_min, ...), t >= 0
__device__ __forceinline__ double grid_coord(const GDev &d, double r)
{
    if (r < d.r_cut_min) r = d.r_cut_min;
    const double t = (r - d.r0) / d.dr;
    return t < 0.0 ? 0.0 : t;
}

// bin b in [0, n_r - 2] and fraction f = t - b of a grid coordinate t >= 0
__device__ __forceinline__ void bin_of(const GDev &d, double t, int &b, double &f)
{
    int k = static_cast<int>(floor(t));
    if (k > d.NR - 2) k = d.NR - 2;
    if (k < 0) k = 0;
    b = k;
    f = t - static_cast<double>(k);
}

// y += k T x with T = 1 (isotropic) or e e^T (parallel)
__device__ __forceinline__ void tensor_add(bool par, const double e[3], double k, const double x[3], double y[3])
{
    if (!par) {
        y[0] += k * x[0];
        y[1] += k * x[1];
        y[2] += k * x[2];
    } else {
        const double s = k * (e[0] * x[0] + e[1] * x[1] + e[2] * x[2]);
        y[0] += s * e[0];
        y[1] += s * e[1];
        y[2] += s * e[2];
    }
}

// ---------------------------------------------------------------------------
// All-pairs search at positions R: pair list (in ascending j), F^C (WCA),
// capacity latch.  One wave per particle; its lanes test 64 candidates j at
// a time and the hits take consecutive list entries in j order (ballot and
// prefix count).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_pairs(GDev d, double *FC, long long step)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (i >= d.n) return;  // whole waves
    const double xi = d.R[3 * i], yi = d.R[3 * i + 1], zi = d.R[3 * i + 2];
    double f[3] = {0.0, 0.0, 0.0};
    int c = 0;  // hits so far (uniform over the wave)
    const int64_t base = i * d.C;
    for (int64_t j0 = 0; j0 < d.n; j0 += 64) {
        const int64_t j = j0 + lane;
        bool hit = false;
        double dx = 0.0, dy = 0.0, dz = 0.0, r = 0.0;
        if (j < d.n && j != i) {
            dx = xi - d.R[3 * j];
            dy = yi - d.R[3 * j + 1];
            dz = zi - d.R[3 * j + 2];
            dx -= d.box[0] * rint(dx / d.box[0]);
            dy -= d.box[1] * rint(dy / d.box[1]);
            dz -= d.box[2] * rint(dz / d.box[2]);
            r = sqrt(dx * dx + dy * dy + dz * dz);
            hit = r < d.r_cut;
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
            if (d.wca_eps != 0.0 && r < d.wca_rc) {
                const double s2 = (d.wca_sigma / r) * (d.wca_sigma / r);
                const double s6 = s2 * s2 * s2;
                const double fr = 24.0 * d.wca_eps * (2.0 * s6 * s6 - s6) / (r * r);
                f[0] += fr * dx;
                f[1] += fr * dy;
                f[2] += fr * dz;
            }
            const int k = c + __popcll(m & ((1ull << lane) - 1ull));
            if (k < d.C) {
                d.pj[base + k] = static_cast<int>(j);
                d.pt[base + k] = grid_coord(d, r);
                if (d.parallel) {
                    double *e = d.pe + 3 * (base + k);
                    e[0] = dx / r;
                    e[1] = dy / r;
                    e[2] = dz / r;
                }
            }
        }
        c += __popcll(m);
    }
    f[0] = wave_sum(f[0]);
    f[1] = wave_sum(f[1]);
    f[2] = wave_sum(f[2]);
    if (lane == 0) {
        FC[3 * i] = f[0];
        FC[3 * i + 1] = f[1];
        FC[3 * i + 2] = f[2];
        d.cnt[i] = c < d.C ? c : d.C;
        if (c > d.C) latch(d.flags, d.flag_step, GLD_ERR_CAPACITY, step);
    }
}

// ---------------------------------------------------------------------------
// F^D' of eq. (dissipative_force2), one wave per particle, lanes over lags:
//   F_i = - sum_{j} [K^p_0(R_ij) T V_j + Delta K^s_0(R_ij) T V_i]
//         - 1/dt sum_{m>=1} [sum_j K^p_m(R_ij) T dR_{j,n-m}
//                            + (K^s_m + sum_j Delta K^s_m(R_ij) T) dR_{i,n-m}]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_dissipative(GDev d, long long n)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (i >= d.n) return;
    const bool par = d.parallel != 0;
    const int M = d.M, Hs = d.Hs;
    const int np = d.cnt[i];
    const int64_t base = i * d.C;
    const double vi[3] = {d.V[3 * i], d.V[3 * i + 1], d.V[3 * i + 2]};
    double acc[3] = {0.0, 0.0, 0.0}, hs[3] = {0.0, 0.0, 0.0};
    const double *hi_ = d.hist + static_cast<int64_t>(i) * Hs * 3;
    for (int q = 0; q < np; ++q) {
        const int j = d.pj[base + q];
        int b;
        double f;
        bin_of(d, d.pt[base + q], b, f);
        double e[3] = {0.0, 0.0, 0.0};
        if (par) {
            e[0] = d.pe[3 * (base + q)];
            e[1] = d.pe[3 * (base + q) + 1];
            e[2] = d.pe[3 * (base + q) + 2];
        }
        const double *k0 = d.kp + static_cast<int64_t>(b) * M, *k1 = k0 + M;
        const double *q0 = d.has_dk ? d.dk + static_cast<int64_t>(b) * M : nullptr, *q1 = q0 ? q0 + M : nullptr;
        if (lane == 0) {
            const double vj[3] = {d.V[3 * j], d.V[3 * j + 1], d.V[3 * j + 2]};
            tensor_add(par, e, k0[0] * (1.0 - f) + k1[0] * f, vj, acc);
            if (q0) tensor_add(par, e, q0[0] * (1.0 - f) + q1[0] * f, vi, acc);
        }
        const double *hj = d.hist + static_cast<int64_t>(j) * Hs * 3;
        for (int m = 1 + lane; m < M; m += 64) {
            const int s = ring_slot(n - m, Hs);
            const double x[3] = {hj[3 * s], hj[3 * s + 1], hj[3 * s + 2]};
            tensor_add(par, e, k0[m] * (1.0 - f) + k1[m] * f, x, hs);
            if (q0) {
                const double xi[3] = {hi_[3 * s], hi_[3 * s + 1], hi_[3 * s + 2]};
                tensor_add(par, e, q0[m] * (1.0 - f) + q1[m] * f, xi, hs);
            }
        }
    }
    for (int m = 1 + lane; m < M; m += 64) {
        const int s = ring_slot(n - m, Hs);
        const double km = d.ks[m];
        hs[0] += km * hi_[3 * s];
        hs[1] += km * hi_[3 * s + 1];
        hs[2] += km * hi_[3 * s + 2];
    }
    hs[0] = wave_sum(hs[0]);
    hs[1] = wave_sum(hs[1]);
    hs[2] = wave_sum(hs[2]);
    if (lane == 0) {
        d.FD[3 * i] = -acc[0] - hs[0] / d.dt;
        d.FD[3 * i + 1] = -acc[1] - hs[1] / d.dt;
        d.FD[3 * i + 2] = -acc[2] - hs[2] / d.dt;
    }
}

// ---------------------------------------------------------------------------
// Spectra of the tables (eq. FT of the correlation sequences
// c_m = kT a_m K_m / dt, a_0 = 2, a_m = 1):
//   X_hat_w = c_0 + 2 sum_{m>=1} c_m cos(2 pi w m / P),
// rows b < n_r of K^p (which 0) and Delta K^s (which 1), row n_r the self
// kernel; written frequency-major.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_spectra(GDev d, int which)
{
    const int w = blockIdx.x * kThreads + threadIdx.x;
    const int b = blockIdx.y;  // 0..n_r (n_r: the self kernel, with which == 0)
    if (w >= d.M) return;
    const double *tab = b == d.NR ? d.ks : (which ? d.dk : d.kp) + static_cast<int64_t>(b) * d.M;
    const double sc = d.kT / d.dt;
    double s = sc * 2.0 * tab[0];
    int idx = 0;
    for (int m = 1; m < d.M; ++m) {
        idx += w;
        if (idx >= d.P) idx -= d.P;
        s += 2.0 * (sc * tab[m]) * d.cosP[idx];
    }
    if (b == d.NR) d.shat[w] = s;
    else (which ? d.dkhT : d.khT)[static_cast<int64_t>(w) * d.NR + b] = s;
}

// ---------------------------------------------------------------------------
// White noise.  Fill ring slots for t0 <= t < t0 + nt; and the per-step
// draw of W_{t} for t = n + M, which replaces W_{n-M+1} in the same slot and
// leaves the difference for the sliding transform.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_white_fill(GDev d, long long t0, int nt)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (k >= static_cast<int64_t>(nt) * d.n) return;
    const long long t = t0 + k / d.n;
    const int64_t i = k % d.n;
    double z[3];
    BoxMuller<double>::gauss3(philox_at(d.seed, static_cast<uint32_t>(i), t, 0u), z);
    double *o = d.ring + static_cast<int64_t>(ring_slot(t, d.P)) * d.n3 + 3 * i;
    o[0] = z[0];
    o[1] = z[1];
    o[2] = z[2];
}

__global__ __launch_bounds__(kThreads) void k_white_step(GDev d, long long t)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= d.n) return;
    double z[3];
    BoxMuller<double>::gauss3(philox_at(d.seed, static_cast<uint32_t>(i), t, 0u), z);
    double *o = d.ring + static_cast<int64_t>(ring_slot(t, d.P)) * d.n3 + 3 * i;
    for (int c = 0; c < 3; ++c) {
        d.delta[3 * i + c] = z[c] - o[c];
        o[c] = z[c];
    }
}

// Full window transform at step n: F_w(n) = sum_u W[u] e^{-i theta w ((u - n) mod P)},
// kDftOmega frequencies per thread (one ring read serves all of them).
__global__ __launch_bounds__(kThreads) void k_dft_full(GDev d, long long n)
{
    const int64_t I = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const int w0 = blockIdx.y * kDftOmega;
    if (I >= d.n3) return;
    const int P = d.P;
    const int sh = ring_slot(-n, P);  // (u - n) mod P = (u + sh) mod P
    int idx[kDftOmega], stp[kDftOmega];
    double re[kDftOmega], im[kDftOmega];
#pragma unroll
    for (int q = 0; q < kDftOmega; ++q) {
        const int w = w0 + q < d.M ? w0 + q : 0;
        stp[q] = w;
        idx[q] = static_cast<int>((static_cast<long long>(w) * sh) % P);
        re[q] = 0.0;
        im[q] = 0.0;
    }
    const double *sinP = d.cosP + P;  // sin(2 pi k / P) follows the cosine table
    for (int u = 0; u < P; ++u) {
        const double x = d.ring[static_cast<int64_t>(u) * d.n3 + I];
#pragma unroll
        for (int q = 0; q < kDftOmega; ++q) {
            re[q] += x * d.cosP[idx[q]];
            im[q] -= x * sinP[idx[q]];
            idx[q] += stp[q];
            if (idx[q] >= P) idx[q] -= P;
        }
    }
#pragma unroll
    for (int q = 0; q < kDftOmega; ++q) {
        const int w = w0 + q;
        if (w < d.M) {
            d.Fre[static_cast<int64_t>(w) * d.n3 + I] = re[q];
            d.Fim[static_cast<int64_t>(w) * d.n3 + I] = im[q];
        }
    }
}

// F_w(n+1) from F_w(n) and the new-minus-old white noise
__global__ __launch_bounds__(kThreads) void k_dft_slide(GDev d)
{
    const int64_t I = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const int w = blockIdx.y;
    if (I >= d.n3) return;
    const double c1 = d.tw[w], s1 = d.tw[d.M + w], c2 = d.tw[2 * d.M + w], s2 = d.tw[3 * d.M + w];
    const int64_t o = static_cast<int64_t>(w) * d.n3 + I;
    const double dl = d.delta[I];
    const double ar = d.Fre[o] + dl * c2, ai = d.Fim[o] + dl * s2;
    d.Fre[o] = c1 * ar - s1 * ai;
    d.Fim[o] = s1 * ar + c1 * ai;
}

// ---------------------------------------------------------------------------
// Algorithm 1, one frequency per work-group: x_w = sqrt(K_hat_w) b,
// b = Re W_hat_w.  Lanczos on the matrix-free mat-vec over the pair list,
//   (K_hat_w v)_i = S_w v_i + sum_j T_ij [K^p_hat_w(R_ij) v_j + Delta K^s_hat_w(R_ij) v_i],
// the square root of the tridiagonal projection H by its eigen-decomposition
// (implicit symmetric QR with Wilkinson shifts, Golub & Van Loan Sec. 8.3),
// y = sqrt(H) e_1, x = |b| V y.
// ---------------------------------------------------------------------------
struct LanczosLds {
    double *kh, *dkh, *al, *be, *dd, *ee, *y, *yo, *Q, *red;
    int *flag;
};

__device__ __forceinline__ LanczosLds carve_lds(double *base, int NR, int has_dk, int kmax)
{
    LanczosLds L;
    double *p = base;
    L.kh = p;
    p += NR;
    L.dkh = p;
    p += has_dk ? NR : 0;
    L.al = p;
    p += kmax;
    L.be = p;
    p += kmax;
    L.dd = p;
    p += kmax;
    L.ee = p;
    p += kmax;
    L.y = p;
    p += kmax;
    L.yo = p;
    p += kmax;
    L.red = p;
    p += kLzThreads / 64;
    L.flag = reinterpret_cast<int *>(p);
    p += 1;
    L.Q = p;
    return L;
}

size_t lanczos_lds_bytes(int NR, int has_dk, int kmax)
{
    return sizeof(double) * (static_cast<size_t>(NR) * (has_dk ? 2 : 1) + 6 * static_cast<size_t>(kmax) + kLzThreads / 64 +
                             1 + static_cast<size_t>(kmax) * kmax);
}

// y = K_hat_w x over this work-group's rows; returns this thread's part of
// x.y.  kLzLanes lanes per particle split its pairs (entries q = lane,
// lane + kLzLanes, ...) and sum them by a butterfly; the first adds S_w x_i.
__device__ double spmv(const GDev &d, const LanczosLds &L, double S, const double *x, double *y)
{
    const bool par = d.parallel != 0;
    const int sub = threadIdx.x % kLzLanes;
    double dot = 0.0;
    for (int64_t i = threadIdx.x / kLzLanes; i < d.n; i += kLzThreads / kLzLanes) {
        const double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        double acc[3] = {0.0, 0.0, 0.0};
        const int np = d.cnt[i];
        const int64_t base = i * d.C;
        // kLzUnroll of the lane's entries at a time: their list loads, then
        // their gathers, then their sums (several loads in flight per lane)
        for (int q0 = sub; q0 < np; q0 += kLzLanes * kLzUnroll) {
            int jj[kLzUnroll];
            double tt[kLzUnroll];
#pragma unroll
            for (int u = 0; u < kLzUnroll; ++u) {
                const int q = q0 + u * kLzLanes;
                jj[u] = q < np ? d.pj[base + q] : -1;
                tt[u] = q < np ? d.pt[base + q] : 0.0;
            }
            double xj[kLzUnroll][3];
#pragma unroll
            for (int u = 0; u < kLzUnroll; ++u) {
                const int j = jj[u] >= 0 ? jj[u] : 0;
                xj[u][0] = x[3 * j];
                xj[u][1] = x[3 * j + 1];
                xj[u][2] = x[3 * j + 2];
            }
#pragma unroll
            for (int u = 0; u < kLzUnroll; ++u) {
                if (jj[u] < 0) break;
                const int q = q0 + u * kLzLanes;
                int b;
                double f;
                bin_of(d, tt[u], b, f);
                double e[3] = {0.0, 0.0, 0.0};
                if (par) {
                    e[0] = d.pe[3 * (base + q)];
                    e[1] = d.pe[3 * (base + q) + 1];
                    e[2] = d.pe[3 * (base + q) + 2];
                }
                tensor_add(par, e, L.kh[b] * (1.0 - f) + L.kh[b + 1] * f, xj[u], acc);
                if (d.has_dk) tensor_add(par, e, L.dkh[b] * (1.0 - f) + L.dkh[b + 1] * f, xi, acc);
            }
        }
#pragma unroll
        for (int o = 1; o < kLzLanes; o <<= 1) {
            acc[0] += __shfl_xor(acc[0], o, kLzLanes);
            acc[1] += __shfl_xor(acc[1], o, kLzLanes);
            acc[2] += __shfl_xor(acc[2], o, kLzLanes);
        }
        if (sub == 0) {
            const double y0 = S * xi[0] + acc[0], y1 = S * xi[1] + acc[1], y2 = S * xi[2] + acc[2];
            y[3 * i] = y0;
            y[3 * i + 1] = y1;
            y[3 * i + 2] = y2;
            dot += xi[0] * y0 + xi[1] * y1 + xi[2] * y2;
        }
    }
    return dot;
}

// Eigen-decomposition of the kk x kk tridiagonal (dd, ee) by the first wave
// (every lane runs the same scalar recurrence; lane l rotates rows l, l + 64
// of Q), then y = Q diag(sqrt(theta)) Q^T e_1.  Returns 0, 1 for a
// non-positive eigenvalue, 2 if the sweeps do not converge.
__device__ int tridiag_sqrt_e1(const LanczosLds &L, int kk, int ld)
{
    const int lane = threadIdx.x & 63;
    double *d = L.dd, *e = L.ee, *Q = L.Q;
    for (int r = lane; r < kk; r += 64)
        for (int c = 0; c < kk; ++c) Q[r * ld + c] = r == c ? 1.0 : 0.0;
    const double eps = 2.220446049250313e-16;
    int hi = kk - 1, guard = 0;
    while (hi > 0) {
        if (++guard > 60 * kk + 100) return 2;
        const double tiny = eps * (fabs(d[hi - 1]) + fabs(d[hi]));
        if (fabs(e[hi - 1]) <= tiny) {
            if (lane == 0) e[hi - 1] = 0.0;
            __builtin_amdgcn_wave_barrier();
            --hi;
            continue;
        }
        // the unreduced block [lo, hi]
        int lo = hi - 1;
        while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
        // Wilkinson shift from the trailing 2 x 2 block
        const double dl = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double mu = d[hi] - eh * eh / (dl + copysign(sqrt(dl * dl + eh * eh), dl));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // Givens rotation G = [c s; -s c] zeroing z against x
            const double rr = sqrt(x * x + z * z);
            const double c = rr != 0.0 ? x / rr : 1.0, s = rr != 0.0 ? z / rr : 0.0;
            const double dk = d[k], ek = e[k], dk1 = d[k + 1];
            const double ekm = (k > lo) ? rr : 0.0;
            const double nd0 = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            const double nd1 = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            const double ne = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            double ek1 = 0.0, bulge = 0.0;
            if (k + 1 < hi) {
                ek1 = e[k + 1];
                bulge = s * ek1;
                ek1 = c * ek1;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                if (k > lo) e[k - 1] = ekm;
                d[k] = nd0;
                d[k + 1] = nd1;
                e[k] = ne;
                if (k + 1 < hi) e[k + 1] = ek1;
            }
            for (int r = lane; r < kk; r += 64) {
                const double a0 = Q[r * ld + k], a1 = Q[r * ld + k + 1];
                Q[r * ld + k] = c * a0 + s * a1;
                Q[r * ld + k + 1] = -s * a0 + c * a1;
            }
            __builtin_amdgcn_wave_barrier();
            x = ne;
            z = bulge;
        }
    }
    for (int q = 0; q < kk; ++q)
        if (!(d[q] > 0.0)) return 1;
    for (int r = lane; r < kk; r += 64) {
        double s = 0.0;
        for (int q = 0; q < kk; ++q) s += Q[r * ld + q] * sqrt(d[q]) * Q[q];
        L.y[r] = s;
    }
    __builtin_amdgcn_wave_barrier();
    return 0;
}

__global__ __launch_bounds__(kLzThreads) void k_lanczos(GDev d, long long step)
{
    extern __shared__ __align__(16) double glds[];
    const int w = blockIdx.x;
    const LanczosLds L = carve_lds(glds, d.NR, d.has_dk, d.kmax);
    const int ld = d.kmax;
    const int64_t n3 = d.n3;
    for (int b = threadIdx.x; b < d.NR; b += kLzThreads) {
        L.kh[b] = d.khT[static_cast<int64_t>(w) * d.NR + b];
        if (d.has_dk) L.dkh[b] = d.dkhT[static_cast<int64_t>(w) * d.NR + b];
    }
    const double S = d.shat[w];
    const double *bv = d.Fre + static_cast<int64_t>(w) * n3;
    double *Vb = d.Vb + static_cast<int64_t>(w) * d.kmax * n3;
    double *Kv = d.KV + static_cast<int64_t>(w) * n3;
    double *X = d.X + static_cast<int64_t>(w) * n3;
    double s = 0.0;
    for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) s += bv[I] * bv[I];
    const double nb = sqrt(block_sum(s, L.red));
    if (nb == 0.0) {
        for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) X[I] = 0.0;
        if (threadIdx.x == 0) d.kprev[w] = 1;
        return;
    }
    for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) Vb[I] = bv[I] / nb;
    __syncthreads();
    const double a0 = block_sum(spmv(d, L, S, Vb, Kv), L.red);
    int status = 0;
    int ko = 1;  // dimension of the last solved y (in L.yo)
    if (!(a0 > 0.0)) {
        status = GLD_ERR_NOT_PD;
    } else {
        if (threadIdx.x == 0) {
            L.al[0] = a0;
            L.yo[0] = sqrt(a0);
        }
        const int kstart = max(2, d.kprev[w] - 2);  // first dimension that is solved
        int k = 1;                                   // dimension of the basis
        for (;;) {
            if (k >= d.kmax) {
                status = GLD_ERR_NO_CONV;
                break;
            }
            __syncthreads();
            const double ak = L.al[k - 1], bk = k >= 2 ? L.be[k - 2] : 0.0;
            const double *vk = Vb + static_cast<int64_t>(k - 1) * n3;
            const double *vm = k >= 2 ? Vb + static_cast<int64_t>(k - 2) * n3 : nullptr;
            double *vn = Vb + static_cast<int64_t>(k) * n3;
            double rr = 0.0;
            for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) {
                double t = Kv[I] - ak * vk[I];
                if (vm) t -= bk * vm[I];
                vn[I] = t;
                rr += t * t;
            }
            const double beta = sqrt(block_sum(rr, L.red));
            if (beta <= 1e-14 * fabs(ak) || beta <= 1e-300) {
                // an invariant subspace: the dimension-k iterate is exact
                if (ko != k) {
                    if (threadIdx.x < 64) {
                        for (int q = threadIdx.x; q < k; q += 64) {
                            L.dd[q] = L.al[q];
                            if (q + 1 < k) L.ee[q] = L.be[q];
                        }
                        __builtin_amdgcn_wave_barrier();
                        const int rc = tridiag_sqrt_e1(L, k, ld);
                        if (threadIdx.x == 0) *L.flag = rc;
                        for (int q = threadIdx.x; q < k; q += 64) L.yo[q] = L.y[q];
                    }
                    __syncthreads();
                    const int rc = *L.flag;
                    if (rc) status = rc == 1 ? GLD_ERR_NOT_PD : GLD_ERR_NO_CONV;
                    ko = k;
                }
                break;
            }
            if (threadIdx.x == 0) L.be[k - 1] = beta;
            const double ib = 1.0 / beta;
            for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) vn[I] = vn[I] * ib;
            __syncthreads();
            const double ak1 = block_sum(spmv(d, L, S, vn, Kv), L.red);
            if (threadIdx.x == 0) L.al[k] = ak1;
            const int kk = k + 1;
            k = kk;
            if (kk < kstart) continue;
            __syncthreads();
            if (threadIdx.x < 64) {
                for (int q = threadIdx.x; q < kk; q += 64) {
                    L.dd[q] = L.al[q];
                    if (q + 1 < kk) L.ee[q] = L.be[q];
                }
                __builtin_amdgcn_wave_barrier();
                int rc = tridiag_sqrt_e1(L, kk, ld);
                int conv = 0;
                if (rc == 0 && ko == kk - 1) {
                    double df = 0.0, nx = 0.0;
                    for (int q = threadIdx.x; q < kk; q += 64) {
                        const double yq = L.y[q], oq = q < ko ? L.yo[q] : 0.0;
                        df += (yq - oq) * (yq - oq);
                        nx += yq * yq;
                    }
                    df = wave_sum(df);
                    nx = wave_sum(nx);
                    conv = sqrt(df) <= d.tol * sqrt(nx);
                }
                for (int q = threadIdx.x; q < kk; q += 64) L.yo[q] = L.y[q];
                if (threadIdx.x == 0) *L.flag = rc ? -rc : conv;
            }
            __syncthreads();
            const int fl = *L.flag;
            ko = kk;
            if (fl < 0) {
                status = fl == -1 ? GLD_ERR_NOT_PD : GLD_ERR_NO_CONV;
                break;
            }
            if (fl == 1) break;
        }
    }
    __syncthreads();
    if (status) {
        if (threadIdx.x == 0) latch(d.flags, d.flag_step, status, step);
        for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) X[I] = 0.0;
        if (threadIdx.x == 0) d.kprev[w] = 0;
        return;
    }
    for (int64_t I = threadIdx.x; I < n3; I += kLzThreads) {
        double acc = 0.0;
        for (int a = 0; a < ko; ++a) acc += Vb[static_cast<int64_t>(a) * n3 + I] * L.yo[a];
        X[I] = nb * acc;
    }
    if (threadIdx.x == 0) d.kprev[w] = ko;
}

// F^R_n = (1/P) (x_0 + 2 sum_{w>=1} x_w), summed over w in order
__global__ __launch_bounds__(kThreads) void k_combine(GDev d)
{
    const int64_t I = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (I >= d.n3) return;
    double s = 0.0;
    for (int w = 0; w < d.M; ++w) s += ((w == 0 ? 1.0 : 2.0) / d.P) * d.X[static_cast<int64_t>(w) * d.n3 + I];
    d.FR[I] = s;
}

// ---------------------------------------------------------------------------
// eq. (GLD_integrator): R_{n+1} = R + dt b V + dt^2/(2M) b (F^C + F^D + F^R),
// dR_n = R_{n+1} - R_n into the ring; then, with F^C at the new positions,
// V_{n+1} = a V + dt/(2M) (a F^C_n + F^C_{n+1}) + dt/M b (F^D + F^R).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_update_r(GDev d, const double *FC, long long n)
{
    const int64_t I = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (I >= d.n3) return;
    const double r = d.R[I];
    const double rn = r + d.dt * d.b * d.V[I] + d.dt * d.dt / (2.0 * d.mass) * d.b * (FC[I] + d.FD[I] + d.FR[I]);
    if (d.M > 1) {
        const int64_t i = I / 3, c = I % 3;
        d.hist[(i * d.Hs + ring_slot(n, d.Hs)) * 3 + c] = rn - r;
    }
    d.R[I] = rn;
}

__global__ __launch_bounds__(kThreads) void k_update_v(GDev d, const double *FCo, const double *FCn, long long n)
{
    const int64_t I = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (I >= d.n3) return;
    const double v = d.a * d.V[I] + d.dt / (2.0 * d.mass) * (d.a * FCo[I] + FCn[I]) +
                     d.dt / d.mass * d.b * (d.FD[I] + d.FR[I]);
    d.V[I] = v;
    if (!isfinite(v) || !isfinite(d.R[I])) latch(d.flags, d.flag_step, GLD_ERR_NONFINITE, n);
}

unsigned blocks(int64_t work) { return static_cast<unsigned>((work + kThreads - 1) / kThreads); }

}  // namespace
}  // namespace gen
}  // namespace gld

using gld::gen::GDev;

struct gld_general {
    GDev d;
    hipStream_t st = nullptr;
    int device = 0;
    int64_t step = 0;
    int cur = 0;  // which F^C buffer holds the current positions' forces
    size_t lds = 0;
    bool timing = false;
    struct Ev {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Ev> events;
    double ms[GLD_G_COUNT] = {};
    int64_t launches[GLD_G_COUNT] = {};
};

namespace {

gld_status gfail(gld_status st, const std::string &msg)
{
    gld::set_last_error(msg);
    return st;
}

gld_status hip_fail(hipError_t e, const char *what)
{
    return gfail(GLD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct Layout {
    size_t off = 0;
    char *base = nullptr;
    template <typename T>
    void take(T *&p, size_t count)
    {
        off = (off + 255) & ~static_cast<size_t>(255);
        p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
    }
};

int capacity_for(const gld_params *p)
{
    int64_t cap;
    if (p->max_neighbors > 0) {
        cap = p->max_neighbors;
    } else {
        const double vol = p->box[0] * p->box[1] * p->box[2];
        const double expect = static_cast<double>(p->n) / vol * (4.0 / 3.0) * M_PI * p->r_cut * p->r_cut * p->r_cut;
        cap = static_cast<int64_t>(1.5 * expect + 32);
    }
    cap = std::max<int64_t>(1, std::min<int64_t>(cap, std::max<int64_t>(1, p->n - 1)));
    return static_cast<int>(cap);
}

void plan(GDev &d, const gld_params *p, int kmax, bool has_dk, Layout &L)
{
    d.n = p->n;
    d.n3 = 3 * p->n;
    d.M = p->m_max;
    d.P = 2 * p->m_max - 1;
    d.Hs = std::max(1, p->m_max - 1);
    d.NR = p->n_r;
    d.C = capacity_for(p);
    d.kmax = kmax;
    d.has_dk = has_dk;
    d.noise_on = p->kT > 0;
    const size_t n3 = static_cast<size_t>(d.n3), M = d.M, NR = d.NR, N = d.n, C = d.C;
    L.take(d.R, n3);
    L.take(d.V, n3);
    L.take(d.FD, n3);
    L.take(d.FR, n3);
    L.take(d.FC0, n3);
    L.take(d.FC1, n3);
    L.take(d.hist, N * d.Hs * 3);
    L.take(d.pj, N * C);
    L.take(d.cnt, N);
    L.take(d.pt, N * C);
    L.take(d.pe, N * C * 3);
    L.take(d.kp, NR * M);
    if (has_dk) L.take(d.dk, NR * M);
    L.take(d.ks, M);
    L.take(d.flags, 4);
    L.take(d.flag_step, 1);
    if (d.noise_on) {
        L.take(d.shat, M);
        L.take(d.khT, M * NR);
        if (has_dk) L.take(d.dkhT, M * NR);
        L.take(d.cosP, 2 * static_cast<size_t>(d.P));
        L.take(d.tw, 4 * M);
        L.take(d.ring, static_cast<size_t>(d.P) * n3);
        L.take(d.delta, n3);
        L.take(d.Fre, M * n3);
        L.take(d.Fim, M * n3);
        L.take(d.KV, M * n3);
        L.take(d.X, M * n3);
        L.take(d.kprev, M);
        L.take(d.Vb, M * static_cast<size_t>(kmax) * n3);
    }
}

gld_status validate_general(const gld_params *p, int32_t max_iters, int &kmax, bool &has_dk,
                            std::vector<double> &kp_table)
{
    gld_status st = gld::validate_params_general(p);
    if (st != GLD_OK) return st;
    if (p->precision != GLD_FP64) return gfail(GLD_ERR_INVALID_ARG, "the general system computes in FP64 only");
    if (p->n > GLD_GENERAL_MAX_N) return gfail(GLD_ERR_INVALID_ARG, "n must be <= GLD_GENERAL_MAX_N");
    if (p->noise_window > 1) return gfail(GLD_ERR_INVALID_ARG, "the general system takes noise_window 0 or 1");
    if (max_iters < 0 || max_iters > GLD_GENERAL_MAX_ITERS || max_iters == 1)
        return gfail(GLD_ERR_INVALID_ARG, "max_iters must be 0 or in [2, GLD_GENERAL_MAX_ITERS]");
    kmax = max_iters ? max_iters : gld::gen::kDefaultIters;
    const size_t table = static_cast<size_t>(p->n_r) * p->m_max;
    kp_table.assign(table, 0.0);
    if (p->k_pair) {
        std::copy(p->k_pair, p->k_pair + table, kp_table.begin());
    } else if (p->k_pair_g) {
        for (int b = 0; b < p->n_r; ++b)
            for (int m = 0; m < p->m_max; ++m)
                kp_table[static_cast<size_t>(b) * p->m_max + m] = p->k_pair_w[b] * p->k_pair_g[m];
    }
    has_dk = false;
    if (p->dk_self)
        for (size_t i = 0; i < table; ++i)
            if (p->dk_self[i] != 0.0) has_dk = true;
    const size_t lds = gld::gen::lanczos_lds_bytes(p->n_r, has_dk, kmax);
    if (p->kT > 0 && lds > gld::gen::kMaxLds)
        return gfail(GLD_ERR_INVALID_ARG, "n_r and max_iters too large for the Lanczos work-group's LDS");
    return GLD_OK;
}

}  // namespace

namespace {

using namespace gld::gen;

// enqueue one kernel, bracketed by timing events when timing is on
template <typename F>
gld_status launch(gld_general *g, int cls, F &&f)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (g->timing) {
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return gfail(GLD_ERR_DEVICE, "hipEventCreate failed");
        (void)hipEventRecord(a, g->st);
    }
    f();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (g->timing) {
        (void)hipEventRecord(b, g->st);
        g->events.push_back({cls, a, b});
    }
    return GLD_OK;
}

// pair list and F^C at the positions in d.R, into F^C buffer `into`
gld_status enqueue_pairs(gld_general *g, int into, int64_t step)
{
    GDev &d = g->d;
    double *fc = into ? d.FC1 : d.FC0;
    return launch(g, GLD_G_PAIRS, [&] { k_pairs<<<blocks(d.n * 64), kThreads, 0, g->st>>>(d, fc, step); });
}

// the white-noise window of step n and its transform
gld_status enqueue_window(gld_general *g, int64_t n)
{
    GDev &d = g->d;
    if (!d.noise_on) return GLD_OK;
    const long long t0 = n - (d.M - 1);
    gld_status st = launch(g, GLD_G_UPDATE, [&] {
        k_white_fill<<<blocks(static_cast<int64_t>(d.P) * d.n), kThreads, 0, g->st>>>(d, t0, d.P);
    });
    if (st != GLD_OK) return st;
    dim3 grid(blocks(d.n3), (d.M + kDftOmega - 1) / kDftOmega);
    return launch(g, GLD_G_DFT, [&] { k_dft_full<<<grid, kThreads, 0, g->st>>>(d, n); });
}

gld_status enqueue_step(gld_general *g)
{
    GDev &d = g->d;
    const int64_t n = g->step;
    gld_status st;
    if ((st = launch(g, GLD_G_DISSIPATIVE, [&] {
             k_dissipative<<<blocks(d.n * 64), kThreads, 0, g->st>>>(d, n);
         })) != GLD_OK)
        return st;
    if (d.noise_on) {
        if ((st = launch(g, GLD_G_LANCZOS, [&] {
                 k_lanczos<<<d.M, kLzThreads, g->lds, g->st>>>(d, n);
             })) != GLD_OK)
            return st;
        if ((st = launch(g, GLD_G_COMBINE, [&] { k_combine<<<blocks(d.n3), kThreads, 0, g->st>>>(d); })) != GLD_OK)
            return st;
    }
    double *fco = g->cur ? d.FC1 : d.FC0, *fcn = g->cur ? d.FC0 : d.FC1;
    if ((st = launch(g, GLD_G_UPDATE, [&] { k_update_r<<<blocks(d.n3), kThreads, 0, g->st>>>(d, fco, n); })) != GLD_OK)
        return st;
    if ((st = enqueue_pairs(g, g->cur ^ 1, n + 1)) != GLD_OK) return st;
    if ((st = launch(g, GLD_G_UPDATE, [&] {
             k_update_v<<<blocks(d.n3), kThreads, 0, g->st>>>(d, fco, fcn, n);
         })) != GLD_OK)
        return st;
    if (d.noise_on) {
        if ((st = launch(g, GLD_G_UPDATE, [&] {
                 k_white_step<<<blocks(d.n), kThreads, 0, g->st>>>(d, n + d.M);
             })) != GLD_OK)
            return st;
        if ((n + 1) % kAnchor == 0) {
            dim3 grid(blocks(d.n3), (d.M + kDftOmega - 1) / kDftOmega);
            st = launch(g, GLD_G_DFT, [&] { k_dft_full<<<grid, kThreads, 0, g->st>>>(d, n + 1); });
        } else {
            dim3 grid(blocks(d.n3), d.M);
            st = launch(g, GLD_G_DFT, [&] { k_dft_slide<<<grid, kThreads, 0, g->st>>>(d); });
        }
        if (st != GLD_OK) return st;
    }
    g->cur ^= 1;
    g->step = n + 1;
    return GLD_OK;
}

gld_status read_flags(gld_general *g, int *flags, long long *fstep)
{
    hipError_t e = hipMemcpyAsync(flags, g->d.flags, sizeof(int), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipMemcpyAsync(fstep, g->d.flag_step, sizeof(long long), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "reading the status");
    return GLD_OK;
}

// install r, v, history (host, [m-1][n][3] or NULL) at step n
gld_status install(gld_general *g, const double *r, const double *v, const double *history, int64_t n)
{
    GDev &d = g->d;
    const size_t n3 = static_cast<size_t>(d.n3);
    for (size_t I = 0; I < n3; ++I)
        if (!std::isfinite(r[I]) || !std::isfinite(v[I])) return gfail(GLD_ERR_NONFINITE, "r or v not finite");
    std::vector<double> ring(static_cast<size_t>(d.n) * d.Hs * 3, 0.0);
    if (history && d.M > 1) {
        for (int m = 1; m < d.M; ++m) {
            const long long t = n - m;
            long long s = t % d.Hs;
            if (s < 0) s += d.Hs;
            for (int64_t i = 0; i < d.n; ++i)
                for (int c = 0; c < 3; ++c)
                    ring[(static_cast<size_t>(i) * d.Hs + s) * 3 + c] = history[((m - 1) * n3) + 3 * i + c];
        }
    }
    hipError_t e = hipMemcpyAsync(d.R, r, n3 * sizeof(double), hipMemcpyHostToDevice, g->st);
    if (e == hipSuccess) e = hipMemcpyAsync(d.V, v, n3 * sizeof(double), hipMemcpyHostToDevice, g->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.hist, ring.data(), ring.size() * sizeof(double), hipMemcpyHostToDevice, g->st);
    if (e == hipSuccess) e = hipMemsetAsync(d.FD, 0, n3 * sizeof(double), g->st);
    if (e == hipSuccess) e = hipMemsetAsync(d.FR, 0, n3 * sizeof(double), g->st);
    if (e == hipSuccess) e = hipMemsetAsync(d.flags, 0, 4 * sizeof(int), g->st);
    if (e == hipSuccess) e = hipMemsetAsync(d.flag_step, 0, sizeof(long long), g->st);
    if (e == hipSuccess && d.noise_on) e = hipMemsetAsync(d.kprev, 0, d.M * sizeof(int), g->st);
    if (e != hipSuccess) return hip_fail(e, "uploading the state");
    g->step = n;
    g->cur = 0;
    gld_status st = enqueue_pairs(g, 0, n);
    if (st == GLD_OK) st = enqueue_window(g, n);
    if (st != GLD_OK) return st;
    if ((e = hipStreamSynchronize(g->st)) != hipSuccess) return hip_fail(e, "installing the state");
    int fl = 0;
    long long fs = 0;
    if ((st = read_flags(g, &fl, &fs)) != GLD_OK) return st;
    if (fl) return gfail(static_cast<gld_status>(fl), "the state's pair list does not fit max_neighbors");
    return GLD_OK;
}

void drop_events(gld_general *g)
{
    for (auto &ev : g->events) {
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    g->events.clear();
}

}  // namespace

extern "C" {

gld_status gld_general_workspace_size(const gld_params *params, int32_t max_iters, size_t *bytes)
{
    if (!bytes) return gfail(GLD_ERR_INVALID_ARG, "bytes is NULL");
    int kmax = 0;
    bool has_dk = false;
    std::vector<double> table;
    gld_status st = validate_general(params, max_iters, kmax, has_dk, table);
    if (st != GLD_OK) return st;
    GDev d;
    Layout L;
    plan(d, params, kmax, has_dk, L);
    *bytes = (L.off + 255) & ~static_cast<size_t>(255);
    return GLD_OK;
}

gld_status gld_general_create(const gld_params *params, int32_t max_iters, const double *r0, const double *v0,
                              void *d_workspace, size_t workspace_bytes, void *hip_stream, gld_general **out)
{
    if (!out) return gfail(GLD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!r0 || !v0 || !d_workspace) return gfail(GLD_ERR_INVALID_ARG, "r0, v0 and the workspace are required");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return gfail(GLD_ERR_INVALID_ARG, "the workspace must be 256-byte aligned");
    int kmax = 0;
    bool has_dk = false;
    std::vector<double> kp;
    gld_status st = validate_general(params, max_iters, kmax, has_dk, kp);
    if (st != GLD_OK) return st;
    const gld_params &p = *params;
    auto *g = new gld_general();
    GDev &d = g->d;
    Layout L;
    L.base = static_cast<char *>(d_workspace);
    plan(d, params, kmax, has_dk, L);
    if (L.off > workspace_bytes) {
        delete g;
        return gfail(GLD_ERR_OOM, "workspace smaller than gld_general_workspace_size");
    }
    g->st = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&g->device);
    d.parallel = p.pair_tensor == GLD_PAIR_PARALLEL;
    for (int c = 0; c < 3; ++c) d.box[c] = p.box[c];
    d.dt = p.dt;
    d.mass = p.mass;
    d.kT = p.kT;
    d.r0 = p.r0;
    d.dr = p.dr;
    d.r_cut = p.r_cut;
    d.r_cut_min = p.r_cut_min;
    d.wca_sigma = p.wca_sigma;
    d.wca_eps = p.wca_eps;
    d.wca_rc = std::pow(2.0, 1.0 / 6.0) * p.wca_sigma;
    d.tol = p.noise_tol > 0 ? p.noise_tol : 1e-12;
    d.seed = p.seed;
    // eq. (aa-bb) with the isotropic K^s_0
    const double x = p.dt * p.k_self[0] / (2.0 * p.mass);
    d.b = 1.0 / (1.0 + x);
    d.a = d.b * (1.0 - x);
    g->lds = lanczos_lds_bytes(d.NR, d.has_dk, d.kmax);
    auto bail = [&](gld_status s) {
        delete g;
        return s;
    };
    const size_t M = d.M, NR = d.NR;
    hipError_t e = hipMemcpyAsync(d.kp, kp.data(), NR * M * sizeof(double), hipMemcpyHostToDevice, g->st);
    if (e == hipSuccess && has_dk)
        e = hipMemcpyAsync(d.dk, p.dk_self, NR * M * sizeof(double), hipMemcpyHostToDevice, g->st);
    if (e == hipSuccess) e = hipMemcpyAsync(d.ks, p.k_self, M * sizeof(double), hipMemcpyHostToDevice, g->st);
    std::vector<double> trig, tw;
    if (e == hipSuccess && d.noise_on) {
        // cos and sin of 2 pi k / P, and the sliding transform's twiddles
        const double two_pi = 6.283185307179586476925286766559;
        trig.resize(2 * static_cast<size_t>(d.P));
        for (int k = 0; k < d.P; ++k) {
            trig[k] = std::cos(two_pi * k / d.P);
            trig[d.P + k] = std::sin(two_pi * k / d.P);
        }
        tw.resize(4 * M);
        for (int w = 0; w < d.M; ++w) {
            const int k1 = w % d.P;
            const int k2 = static_cast<int>((static_cast<long long>(w) * (d.M - 1)) % d.P);
            tw[w] = trig[k1];
            tw[M + w] = trig[d.P + k1];
            tw[2 * M + w] = trig[k2];
            tw[3 * M + w] = trig[d.P + k2];
        }
        e = hipMemcpyAsync(d.cosP, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice, g->st);
        if (e == hipSuccess) e = hipMemcpyAsync(d.tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, g->st);
        if (e == hipSuccess) {
            k_spectra<<<dim3(blocks(d.M), d.NR + 1), kThreads, 0, g->st>>>(d, 0);
            if (has_dk) k_spectra<<<dim3(blocks(d.M), d.NR), kThreads, 0, g->st>>>(d, 1);
            e = hipGetLastError();
        }
        if (e == hipSuccess && g->lds > 65536)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lanczos),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(g->lds));
    }
    if (e != hipSuccess) return bail(hip_fail(e, "gld_general_create"));
    st = install(g, r0, v0, nullptr, 0);
    if (st != GLD_OK) return bail(st);
    *out = g;
    return GLD_OK;
}

gld_status gld_general_step(gld_general *g, int64_t n_steps)
{
    if (!g || n_steps < 0) return gfail(GLD_ERR_INVALID_ARG, "bad handle or step count");
    for (int64_t k = 0; k < n_steps; ++k) {
        gld_status st = enqueue_step(g);
        if (st != GLD_OK) return st;
    }
    return GLD_OK;
}

gld_status gld_general_sync(gld_general *g)
{
    if (!g) return gfail(GLD_ERR_INVALID_ARG, "bad handle");
    int fl = 0;
    long long fs = 0;
    gld_status st = read_flags(g, &fl, &fs);
    if (st != GLD_OK) return st;
    if (fl) return gfail(static_cast<gld_status>(fl), "latched during step " + std::to_string(fs));
    return GLD_OK;
}

gld_status gld_general_read_state(gld_general *g, gld_state *out)
{
    if (!g || !out) return gfail(GLD_ERR_INVALID_ARG, "bad handle or state");
    GDev &d = g->d;
    const size_t n3 = static_cast<size_t>(d.n3);
    int fl = 0;
    long long fs = 0;
    gld_status st = read_flags(g, &fl, &fs);
    if (st != GLD_OK) return st;
    hipError_t e = hipSuccess;
    auto get = [&](double *dst, const double *src) {
        if (dst && e == hipSuccess) e = hipMemcpyAsync(dst, src, n3 * sizeof(double), hipMemcpyDeviceToHost, g->st);
    };
    get(out->r, d.R);
    get(out->v, d.V);
    get(out->f_c, g->cur ? d.FC1 : d.FC0);
    get(out->f_d, d.FD);
    get(out->f_r, d.FR);
    std::vector<double> ring;
    if (out->history && d.M > 1) {
        ring.resize(static_cast<size_t>(d.n) * d.Hs * 3);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ring.data(), d.hist, ring.size() * sizeof(double), hipMemcpyDeviceToHost, g->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "gld_general_read_state");
    if (out->history && d.M > 1) {
        for (int m = 1; m < d.M; ++m) {
            long long s = (g->step - m) % d.Hs;
            if (s < 0) s += d.Hs;
            for (int64_t i = 0; i < d.n; ++i)
                for (int c = 0; c < 3; ++c)
                    out->history[(m - 1) * n3 + 3 * i + c] = ring[(static_cast<size_t>(i) * d.Hs + s) * 3 + c];
        }
    }
    out->step = g->step;
    out->flags = fl;
    out->flag_step = fs;
    if (fl) return gfail(static_cast<gld_status>(fl), "latched during step " + std::to_string(fs));
    return GLD_OK;
}

gld_status gld_general_write_state(gld_general *g, const gld_state *in)
{
    if (!g || !in || !in->r || !in->v) return gfail(GLD_ERR_INVALID_ARG, "bad handle or state (r, v required)");
    hipError_t e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "gld_general_write_state");
    return install(g, in->r, in->v, in->history, in->step);
}

gld_status gld_general_frequency_vectors(gld_general *g, int32_t w0, int32_t w1, double *out)
{
    if (!g || !out) return gfail(GLD_ERR_INVALID_ARG, "bad handle or output");
    GDev &d = g->d;
    if (!d.noise_on) return gfail(GLD_ERR_INVALID_ARG, "no noise (kT = 0)");
    if (w0 < 0 || w1 > d.M || w0 >= w1) return gfail(GLD_ERR_INVALID_ARG, "need 0 <= w0 < w1 <= m_max");
    const size_t bytes = static_cast<size_t>(w1 - w0) * d.n3 * sizeof(double);
    hipError_t e = hipMemcpyAsync(out, d.X + static_cast<int64_t>(w0) * d.n3, bytes, hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "gld_general_frequency_vectors");
    return GLD_OK;
}

gld_status gld_general_get_info(gld_general *g, gld_general_info *out)
{
    if (!g || !out) return gfail(GLD_ERR_INVALID_ARG, "bad handle or output");
    GDev &d = g->d;
    std::vector<int> cnt(d.n), kp(d.noise_on ? d.M : 0);
    hipError_t e = hipMemcpyAsync(cnt.data(), d.cnt, cnt.size() * sizeof(int), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess && d.noise_on)
        e = hipMemcpyAsync(kp.data(), d.kprev, kp.size() * sizeof(int), hipMemcpyDeviceToHost, g->st);
    if (e == hipSuccess) e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "gld_general_get_info");
    out->max_iters = d.kmax;
    out->last_iters = 0;
    for (int k : kp) out->last_iters = std::max(out->last_iters, k);
    out->pairs = 0;
    out->max_per_particle = 0;
    for (int c : cnt) {
        out->pairs += c;
        out->max_per_particle = std::max(out->max_per_particle, c);
    }
    out->capacity = d.C;
    out->tol = d.tol;
    return GLD_OK;
}

gld_status gld_general_set_timing(gld_general *g, int enable)
{
    if (!g) return gfail(GLD_ERR_INVALID_ARG, "bad handle");
    hipError_t e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "gld_general_set_timing");
    drop_events(g);
    g->timing = enable != 0;
    for (int k = 0; k < GLD_G_COUNT; ++k) {
        g->ms[k] = 0;
        g->launches[k] = 0;
    }
    return GLD_OK;
}

gld_status gld_general_kernel_times(gld_general *g, double *ms_sum, int64_t *launches)
{
    if (!g || !ms_sum || !launches) return gfail(GLD_ERR_INVALID_ARG, "bad handle or output");
    hipError_t e = hipStreamSynchronize(g->st);
    if (e != hipSuccess) return hip_fail(e, "gld_general_kernel_times");
    for (auto &ev : g->events) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
            g->ms[ev.cls] += ms;
            g->launches[ev.cls] += 1;
        }
    }
    drop_events(g);
    for (int k = 0; k < GLD_G_COUNT; ++k) {
        ms_sum[k] = g->ms[k];
        launches[k] = g->launches[k];
    }
    return GLD_OK;
}

gld_status gld_general_destroy(gld_general *g)
{
    if (!g) return GLD_OK;
    (void)hipStreamSynchronize(g->st);
    drop_events(g);
    delete g;
    return GLD_OK;
}

}  // extern "C"
