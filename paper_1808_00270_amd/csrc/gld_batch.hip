// Batched device kernels: many independent GLD systems advanced together.
//
// Paper: arXiv:1808.00270, Sec. II (eqs. GLD_integrator, aa-bb,
// dissipative_force2, stochastic_force2, noise_production).  The method per
// system is the one of the single-system kernels; what differs is the
// launch: every kernel below covers all systems of a batch at once through a
// flat block map (block -> system, first unit), reading each system's sizes,
// constants and buffers from its descriptor (BSys).  A system's results do
// not depend on the other systems of the batch: every sum runs in an order
// fixed by that system alone.
//
// Per system (N particles, stride S = roundup(N, 64)):
//   history ring     T  [m_max-1][3][S]  slot-major, streamed once per step
//   pair lists       ELL: uint16 index [cap][S], T weight [cap][S], column =
//                    particle (lane i of a wave reads entry k of particle i)
//   chain vectors    T4 [S] (x, y, z, 0) gathered from L2 by the mat-vecs
//   white noise      T  [2 h + 2 bf][3][S] ring, filter outputs [2][rows][3][S]
// The filter bank is the single-system matrix-core kernel (shared body),
// spread over the filter block: each step computes 1/bf of the next block.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gld_batch_dev.h"
#include "gld_device.h"

namespace gld {
namespace batch {

namespace {

template <typename T>
struct V4t;
template <>
struct V4t<float> {
    using t = float4;
};
template <>
struct V4t<double> {
    using t = double4;
};

__device__ __forceinline__ int wrap_slot(long long t, int len)
{
    long long m = t % len;
    return static_cast<int>(m < 0 ? m + len : m);
}

// ---------------------------------------------------------------------------
// H3: memory convolution, thread per particle, all lags (the definition's
// stream of the ring once per step):
//   Dneg = -(1/dt) sum_{m=1}^{M-1} K^s_m dR_{n-m},  Y = g_0 V + (1/dt) sum_m g_m dR_{n-m}
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_history(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n) return;
    const int64_t S = d.S, S3 = 3 * S;
    const T *ring = static_cast<const T *>(d.ring);
    const T *ks = static_cast<const T *>(d.ks), *gm = static_cast<const T *>(d.gm);
    const long long step = *d.step;
    T dx = T(0), dy = T(0), dz = T(0), hx = T(0), hy = T(0), hz = T(0);
    const int ns = d.nslots;
    if (ns > 0) {
        int slot = wrap_slot(step - 1, ns);
#pragma unroll 4
        for (int m = 1; m <= ns; ++m) {
            const T *r = ring + static_cast<int64_t>(slot) * S3 + i;
            const T x = r[0], y = r[S], z = r[2 * S];
            const T k = ks[m], g = gm[m];
            dx += k * x;
            dy += k * y;
            dz += k * z;
            hx += g * x;
            hy += g * y;
            hz += g * z;
            slot = slot == 0 ? ns - 1 : slot - 1;
        }
    }
    const T inv_dt = static_cast<T>(1.0 / d.dt), g0 = static_cast<T>(d.g0);
    T *Dn = static_cast<T *>(d.Dneg);
    Dn[i] = -dx * inv_dt;
    Dn[S + i] = -dy * inv_dt;
    Dn[2 * S + i] = -dz * inv_dt;
    typename V4t<T>::t y;
    y.x = g0 * static_cast<T>(d.V[i]) + hx * inv_dt;
    y.y = g0 * static_cast<T>(d.V[S + i]) + hy * inv_dt;
    y.z = g0 * static_cast<T>(d.V[2 * S + i]) + hz * inv_dt;
    y.w = T(0);
    static_cast<typename V4t<T>::t *>(d.y4)[d.cpos[i]] = y;
}

// ---------------------------------------------------------------------------
// H5a: white noise into each system's ring (the single-system modes:
// 0 the slice the step adds, t = step + h + 2 bf - 1; 1 the window of the
// current block; 2 the slices from the next block's window up to what an
// uninterrupted run holds before the step), blockIdx.y = slice
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_white(const BSys *__restrict__ sys, const BMap *__restrict__ map,
                                                     int mode)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n || !d.noise_on) return;
    const long long cur = *d.step;
    const int bf = d.bf, h = d.half;
    const long long n0 = cur - cur % bf;
    const int y = blockIdx.y;
    long long t;
    if (mode == 0) {
        if (y > 0) return;
        t = cur + h + 2 * bf - 1;
    } else if (mode == 1) {
        if (y >= 2 * h + bf) return;
        t = n0 - h + y;
    } else {
        t = n0 + bf - h + y;
        if (t > cur + h + 2 * bf - 2) return;
    }
    T w[3];
    BoxMuller<T>::gauss3(philox_at(d.seed, static_cast<uint32_t>(i), t, 0u), w);
    T *dst = static_cast<T *>(d.wring) + static_cast<int64_t>(wrap_slot(t, d.wlen)) * 3 * d.S;
    dst[i] = w[0];
    dst[d.S + i] = w[1];
    dst[2 * d.S + i] = w[2];
}

// ---------------------------------------------------------------------------
// H5a: the filter bank on the matrix cores, one tile of 256 channels per
// block: tiles[b] = (system, tile within the system's share).  mode 0: every
// fir_period(bf) steps a share of the next block; 1: the whole current block;
// 2: the whole next block.
// ---------------------------------------------------------------------------
__device__ __forceinline__ FirPart fir_part(const BSys &d, int mode, int64_t M)
{
    FirPart part;
    part.ahead = mode == 1 ? 0 : 1;
    part.spread = mode == 0;
    part.period = fir_period(d.bf);
    part.nslice = mode == 0 ? d.bf / part.period : 1;
    part.cs = mode == 0 ? (M / part.nslice + 1 + kThreads - 1) / kThreads * kThreads : M;
    return part;
}

__global__ __launch_bounds__(kFirMfmaThreads) void kb_fir32(const BSys *__restrict__ sys, const int2 *__restrict__ tiles,
                                                            int mode)
{
    const int2 tl = tiles[blockIdx.x];
    const BSys &d = sys[tl.x];
    const int64_t M = 3 * d.S;
    FirPart part = fir_part(d, mode, M);
    part.ustride = static_cast<int64_t>(fir_rows(0)) * M;
    fir_mfma_body<0>(d.n, d.S, d.bf, d.rcap, d.half, 2 * d.half + d.bf, d.wlen, static_cast<const float *>(d.Afilt),
                     static_cast<const float *>(d.wring), d.step, static_cast<float *>(d.U), part, tl.y);
}

__global__ __launch_bounds__(kFirMfmaThreads) void kb_fir64(const BSys *__restrict__ sys, const int2 *__restrict__ tiles,
                                                            int mode)
{
    const int2 tl = tiles[blockIdx.x];
    const BSys &d = sys[tl.x];
    const int64_t M = 3 * d.S;
    FirPart part = fir_part(d, mode, M);
    part.ustride = static_cast<int64_t>(fir_rows(1)) * M;
    // four row tiles: a launch covers every system, whose bf * rcap reach 64
    fir_mfma64_body<0, 4>(d.n, d.S, d.bf, d.rcap, d.half, 2 * d.half + d.bf, d.wlen,
                       static_cast<const double *>(d.Afilt), static_cast<const double *>(d.wring), d.step,
                       static_cast<double *>(d.U), part, tl.y);
}

// ---------------------------------------------------------------------------
// premixed chain inputs v_k = sum_q B[k][q] u_q (the filter outputs of the
// step, in the buffer of its block's parity), k < K of the system
// ---------------------------------------------------------------------------
template <typename T, int RMAX>
__global__ __launch_bounds__(kThreads) void kb_premix(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    using T4 = typename V4t<T>::t;
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n || !d.noise_on) return;
    const int64_t S = d.S, S3 = 3 * S;
    const long long cur = *d.step;
    const int rows = sizeof(T) == 8 ? fir_rows(1) : fir_rows(0);
    const T *u = static_cast<const T *>(d.U) + ((cur / d.bf) & 1) * rows * S3 +
                 static_cast<int64_t>(cur % d.bf) * d.rcap * S3;
    T ux[RMAX], uy[RMAX], uz[RMAX];
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
        ux[q] = uy[q] = uz[q] = T(0);
        if (q < d.rank) {
            const T *uq = u + q * S3 + i;
            ux[q] = uq[0];
            uy[q] = uq[S];
            uz[q] = uq[2 * S];
        }
    }
    const T *B = static_cast<const T *>(d.Bmix);
    T4 *vk = static_cast<T4 *>(d.vk);
    const int64_t p = d.cpos[i];  // the chain runs in cell order
    for (int k = 0; k < d.K; ++k) {
        const T *bk = B + static_cast<int64_t>(k) * d.rcap;
        T sx = T(0), sy = T(0), sz = T(0);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const T c = q < d.rank ? bk[q] : T(0);
            sx += c * ux[q];
            sy += c * uy[q];
            sz += c * uz[q];
        }
        T4 v;
        v.x = sx;
        v.y = sy;
        v.z = sz;
        v.w = T(0);
        vk[static_cast<int64_t>(k) * S + p] = v;
    }
}

// ---------------------------------------------------------------------------
// H4/H5b: pair mat-vec over the ELL lists, LANES lanes per particle (the
// lanes take every LANES-th neighbour; a fixed butterfly adds their sums):
//   k >= 0:  out = a P x + b x + cz z + v_k  with (a, b, cz) = terms[k],
//            x = cb[ix], z = cb[iz], out = cb[io] (T4), or F^R for k = 0
//   k = -1:  F^D' = -P y + Dneg  (y the history's Y)
// ---------------------------------------------------------------------------
constexpr int kSpmvUnroll = 8;  // list entries a lane of the mat-vec has in flight

template <typename T, int LANES>
__global__ __launch_bounds__(kThreads) void kb_spmv(const BSys *__restrict__ sys, const BMap *__restrict__ map, int k,
                                                    int ix, int iz, int io)
{
    using T4 = typename V4t<T>::t;
    const BMap mp = map[blockIdx.x];
    if (mp.sys < 0) return;  // padding of the XCD-ordered map
    const BSys &d = sys[mp.sys];
    if (k >= d.K && k >= 0) return;  // beyond this system's chain
    if (k >= 0 && !d.noise_on) return;
    const int sub = threadIdx.x % LANES;
    // p: a cell-order position (the vectors and lists are in cell order)
    const int64_t p = mp.first + threadIdx.x / LANES;
    const bool live = p < d.n;
    const int64_t S = d.S;
    const T4 *x = static_cast<const T4 *>(k < 0 ? d.y4 : d.cb[ix]);
    const BTerm tm = k >= 0 ? d.terms[k] : BTerm{-1.0, 0.0, 0.0};
    T ax = T(0), ay = T(0), az = T(0);
    if (live && tm.a != 0.0) {
        // lane sub reads entries sub, sub + LANES, ... of row p: in the
        // lane-interleaved lists a lane group's reads are LANES consecutive
        // entries, and a wave's 64 consecutive ones
        const int nn = d.nn[p];
        const uint16_t *li = d.nbl + p * LANES + sub;
        const T *lw = static_cast<const T *>(d.nbw) + p * LANES + sub;
        const int64_t row = S * LANES;
        int64_t o = 0;
        int q = sub;
        // kUnroll of the lane's entries at a time: their index and weight
        // loads, then their gathers, then the sums in entry order (several
        // loads in flight per lane; the same sums as one entry at a time)
        for (; q + (kSpmvUnroll - 1) * LANES < nn; q += kSpmvUnroll * LANES, o += kSpmvUnroll * row) {
            int jj[kSpmvUnroll];
            T ww[kSpmvUnroll];
#pragma unroll
            for (int u = 0; u < kSpmvUnroll; ++u) {
                jj[u] = li[o + u * row];
                ww[u] = lw[o + u * row];
            }
            T4 xx[kSpmvUnroll];
#pragma unroll
            for (int u = 0; u < kSpmvUnroll; ++u) xx[u] = x[jj[u]];
#pragma unroll
            for (int u = 0; u < kSpmvUnroll; ++u) {
                ax += ww[u] * xx[u].x;
                ay += ww[u] * xx[u].y;
                az += ww[u] * xx[u].z;
            }
        }
        for (; q < nn; q += LANES, o += row) {
            const int j = li[o];
            const T w = lw[o];
            const T4 xj = x[j];
            ax += w * xj.x;
            ay += w * xj.y;
            az += w * xj.z;
        }
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) {
        ax += __shfl_xor(ax, o, LANES);
        ay += __shfl_xor(ay, o, LANES);
        az += __shfl_xor(az, o, LANES);
    }
    if (!live || sub != 0) return;
    if (k < 0) {
        const int64_t i = d.cell_sorted[p];  // the particle, for the outputs in particle order
        const T *Dn = static_cast<const T *>(d.Dneg);
        T *FD = static_cast<T *>(d.FD);
        FD[i] = -ax + Dn[i];
        FD[S + i] = -ay + Dn[S + i];
        FD[2 * S + i] = -az + Dn[2 * S + i];
        return;
    }
    const T a = static_cast<T>(tm.a), b = static_cast<T>(tm.b), cz = static_cast<T>(tm.cz);
    const T4 vk = static_cast<const T4 *>(d.vk)[static_cast<int64_t>(k) * S + p];
    T ox = a * ax + vk.x, oy = a * ay + vk.y, oz = a * az + vk.z;
    if (b != T(0)) {
        const T4 xi = x[p];
        ox += b * xi.x;
        oy += b * xi.y;
        oz += b * xi.z;
    }
    if (cz != T(0)) {
        const T4 zi = static_cast<const T4 *>(d.cb[iz])[p];
        ox += cz * zi.x;
        oy += cz * zi.y;
        oz += cz * zi.z;
    }
    if (k == 0) {
        const int64_t i = d.cell_sorted[p];
        T *FR = static_cast<T *>(d.FR);
        FR[i] = ox;
        FR[S + i] = oy;
        FR[2 * S + i] = oz;
    } else {
        T4 o;
        o.x = ox;
        o.y = oy;
        o.z = oz;
        o.w = T(0);
        static_cast<T4 *>(d.cb[io])[p] = o;
    }
}

// ---------------------------------------------------------------------------
// H6: G-JF type update (eq. GLD_integrator with b in the position update)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void kb_update_r(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n) return;
    const int64_t S = d.S;
    const double c_v = d.dt * d.b, c_f = d.dt * d.dt / (2.0 * d.mass) * d.b;
    const T *FD = static_cast<const T *>(d.FD), *FR = static_cast<const T *>(d.FR);
    T *ring = static_cast<T *>(d.ring);
    const long long step = *d.step;
    const int64_t head = d.nslots > 0 ? (step % d.nslots) * 3 * S : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = c * S + i;
        const double f = d.FC[e] + static_cast<double>(FD[e]) + static_cast<double>(FR[e]);
        const double dR = c_v * d.V[e] + c_f * f;
        d.R[e] += dR;
        if (d.nslots > 0) ring[head + e] = static_cast<T>(dR);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_update_v(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n) return;
    const int64_t S = d.S;
    const double half = d.dt / (2.0 * d.mass), dtb = d.dt / d.mass * d.b;
    const T *FD = static_cast<const T *>(d.FD), *FR = static_cast<const T *>(d.FR);
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t e = c * S + i;
        const double fcn = d.FCn[e];
        const double v = d.a * d.V[e] + half * (d.a * d.FC[e] + fcn) +
                         dtb * (static_cast<double>(FD[e]) + static_cast<double>(FR[e]));
        d.V[e] = v;
        d.FC[e] = fcn;
        bad |= !isfinite(v) || !isfinite(d.R[e]);
    }
    if (bad) latch(d.flags, d.flag_step, GLD_ERR_NONFINITE, *d.step);
}

__global__ void kb_advance(const BSys *__restrict__ sys, int nsys)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys || sys[s].n == 0) return;
    *sys[s].step += 1;
}

// ---------------------------------------------------------------------------
// H1/H2: neighbour lists from a cell list, rebuilt every step.
// Cells of edge >= r_cut per axis; with fewer than three cells on an axis the
// stencil takes each neighbouring cell once (r_cut < L/2 makes the minimum
// image unique).  Within a cell, particles are ordered by index, so every
// list (and every sum over it) has an order fixed by the configuration.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void kb_cell_clear(const BSys *__restrict__ sys, const BMap *__restrict__ cmap)
{
    const BMap mp = cmap[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int c = mp.first + threadIdx.x;
    if (c < d.ncell) d.cell_count[c] = 0;
    if (c == 0) *d.rowmax = 0u;
}

__device__ __forceinline__ int cell_coord(double x, double L, int nc)
{
    int c = static_cast<int>(floor(x / L * nc));
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ __launch_bounds__(kThreads) void kb_cell_assign(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n) return;
    double p[3];
    int cc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double L = d.box[c];
        double x = d.R[c * d.S + i];
        x -= L * floor(x / L);
        if (x >= L) x -= L;  // rounding of x = -tiny
        p[c] = x;
        cc[c] = cell_coord(x, L, d.nc[c]);
    }
    const int cell = (cc[2] * d.nc[1] + cc[1]) * d.nc[0] + cc[0];
    d.Rw[i] = make_double4(p[0], p[1], p[2], 0.0);
    d.cell_id[i] = cell;
    d.cell_slot[i] = atomicAdd(&d.cell_count[cell], 1);
}

// exclusive scan of the cell counts, one block per system
__global__ __launch_bounds__(1024) void kb_cell_scan(const BSys *__restrict__ sys)
{
    const BSys &d = sys[blockIdx.x];
    if (d.n == 0) return;
    __shared__ int part[1024];
    const int nc = d.ncell, t = threadIdx.x;
    const int per = (nc + 1023) / 1024;
    const int b = t * per, e = min(nc, b + per);
    int s = 0;
    for (int c = b; c < e; ++c) s += d.cell_count[c];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? part[t - 1] : 0;
    for (int c = b; c < e; ++c) {
        d.cell_start[c] = run;
        run += d.cell_count[c];
    }
    if (t == 1023) d.cell_start[nc] = part[1023];
}

__global__ __launch_bounds__(kThreads) void kb_cell_scatter(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n) return;
    const int c = d.cell_id[i];
    d.cell_list[d.cell_start[c] + d.cell_slot[i]] = static_cast<int>(i);
}

// rank of a particle among its cell's particles by index: the cell order
__global__ __launch_bounds__(kThreads) void kb_cell_rank(const BSys *__restrict__ sys, const BMap *__restrict__ map)
{
    const BMap mp = map[blockIdx.x];
    const BSys &d = sys[mp.sys];
    const int64_t i = mp.first + threadIdx.x;
    if (i >= d.n) return;
    const int c = d.cell_id[i];
    const int b = d.cell_start[c], e = d.cell_start[c + 1];
    int r = 0;
    for (int q = b; q < e; ++q) r += d.cell_list[q] < i ? 1 : 0;
    d.cell_sorted[b + r] = static_cast<int>(i);
    d.cpos[i] = b + r;
    d.Rs[b + r] = d.Rw[i];
}

__device__ __forceinline__ double batch_weight(const BSys &d, double r)
{
    double rr = r < d.r_cut_min ? d.r_cut_min : r;
    const double t = fmax((rr - d.r0) / d.dr, 0.0);
    const double tb = fmin(floor(t), static_cast<double>(d.n_r - 2));
    const int b = static_cast<int>(fmax(tb, 0.0));
    const double f = t - b;
    return d.wtab[b] * (1.0 - f) + d.wtab[b + 1] * f;
}

// LANES lanes per particle take the candidates of each stencil cell in
// turns of LANES; the hits of a turn get consecutive list positions in
// candidate order (a ballot over the lane group), so the list is the same
// for any LANES and its order is fixed by the configuration
template <typename T, int LANES>
__global__ __launch_bounds__(kThreads) void kb_build(const BSys *__restrict__ sys, const BMap *__restrict__ map,
                                                     int into_fc)
{
    const BMap mp = map[blockIdx.x];
    if (mp.sys < 0) return;
    const BSys &d = sys[mp.sys];
    const int sub = threadIdx.x % LANES;
    const int64_t i = mp.first + threadIdx.x / LANES;
    const bool live = i < d.n;
    const int64_t S = d.S;
    const double4 pi = live ? d.Rw[i] : make_double4(0, 0, 0, 0);
    const int ci = live ? d.cell_id[i] : 0;
    const int cx = ci % d.nc[0], cy = (ci / d.nc[0]) % d.nc[1], cz = ci / (d.nc[0] * d.nc[1]);
    const double rc2 = d.r_cut * d.r_cut;
    // the particle's row and its neighbours' entries are cell-order positions
    const int64_t prow = live ? d.cpos[i] : 0;
    T *lw = static_cast<T *>(d.nbw) + prow * LANES;
    uint16_t *li = d.nbl + prow * LANES;
    const int64_t row = S * LANES;
    // lanes of this particle within the wave: bits [gbase, gbase + LANES)
    const int gbase = (threadIdx.x % 64) & ~(LANES - 1);
    const unsigned long long gmask = (LANES == 64 ? ~0ull : ((1ull << LANES) - 1)) << gbase;
    int cnt = 0;
    bool over = false;
    double fx = 0, fy = 0, fz = 0, rowsum = 0;
    for (int oz = 0; oz < d.noff[2]; ++oz)
        for (int oy = 0; oy < d.noff[1]; ++oy)
            for (int ox = 0; ox < d.noff[0]; ++ox) {
                // offsets -1, 0, +1 (three or more cells), else 0 and +1 or just 0
                const int dxo = d.noff[0] == 3 ? ox - 1 : ox, dyo = d.noff[1] == 3 ? oy - 1 : oy;
                const int dzo = d.noff[2] == 3 ? oz - 1 : oz;
                const int nx = (cx + dxo + d.nc[0]) % d.nc[0], ny = (cy + dyo + d.nc[1]) % d.nc[1];
                const int nz = (cz + dzo + d.nc[2]) % d.nc[2];
                const int cj = (nz * d.nc[1] + ny) * d.nc[0] + nx;
                const int b = live ? d.cell_start[cj] : 0, e = live ? d.cell_start[cj + 1] : 0;
                // the lanes of a group run the same number of turns
                for (int q0 = b; q0 < e; q0 += LANES) {
                    const int q = q0 + sub;
                    bool hit = false;
                    double w = 0;
                    if (q < e) {
                        // q: the candidate's cell-order position, the index the list stores
                        if (q != prow) {
                            const double4 pj = d.Rs[q];  // consecutive for the lanes of a group
                            double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
                            dx -= d.box[0] * rint(dx / d.box[0]);
                            dy -= d.box[1] * rint(dy / d.box[1]);
                            dz -= d.box[2] * rint(dz / d.box[2]);
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 < rc2) {
                                if (r2 < d.wca_rc2) {
                                    // WCA force on i: -dU/dr along (R_i - R_j) = -(dx, dy, dz)
                                    const double s2 = d.wca_s2 / r2, s6 = s2 * s2 * s2;
                                    const double fr = 24.0 * d.wca_eps * (2.0 * s6 * s6 - s6) / r2;
                                    fx -= fr * dx;
                                    fy -= fr * dy;
                                    fz -= fr * dz;
                                }
                                if (d.has_pair) {
                                    w = batch_weight(d, sqrt(r2));
                                    rowsum += fabs(w);
                                    hit = true;
                                }
                            }
                        }
                    }
                    const unsigned long long m = __ballot(hit) & gmask;
                    if (hit) {
                        const int pos = cnt + __popcll(m & ((1ull << (threadIdx.x % 64)) - 1) & gmask);
                        if (pos < d.cap) {
                            const int64_t o = static_cast<int64_t>(pos / LANES) * row + pos % LANES;
                            li[o] = static_cast<uint16_t>(q);
                            lw[o] = static_cast<T>(w);
                        } else {
                            over = true;
                        }
                    }
                    cnt += __popcll(m);
                }
            }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, LANES);
        fy += __shfl_xor(fy, o, LANES);
        fz += __shfl_xor(fz, o, LANES);
        rowsum += __shfl_xor(rowsum, o, LANES);
    }
    if (!live || sub != 0) {
        if (live && over) latch(d.flags, d.flag_step, GLD_ERR_CAPACITY, *d.step);
        return;
    }
    d.nn[prow] = min(cnt, d.cap);
    double *fc = into_fc ? d.FC : d.FCn;
    fc[i] = fx;
    fc[S + i] = fy;
    fc[2 * S + i] = fz;
    const long long step = *d.step;
    if (over || cnt > d.cap) latch(d.flags, d.flag_step, GLD_ERR_CAPACITY, step);
    if (rowsum > d.lam_hi) latch(d.flags, d.flag_step, GLD_ERR_INTERVAL, step);
    atomicMax(d.rowmax, __float_as_uint(static_cast<float>(rowsum)));
}

inline unsigned nb(int n) { return static_cast<unsigned>(n); }

}  // namespace

hipError_t b_history(int fp64, const BSys *sys, const BMap *map, int nblocks, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (fp64) kb_history<double><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    else kb_history<float><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    return hipGetLastError();
}

hipError_t b_white(int fp64, const BSys *sys, const BMap *map, int nblocks, int mode, int gy, hipStream_t st)
{
    if (nblocks <= 0 || gy <= 0) return hipSuccess;
    const dim3 grid(nb(nblocks), static_cast<unsigned>(gy));
    if (fp64) kb_white<double><<<grid, kThreads, 0, st>>>(sys, map, mode);
    else kb_white<float><<<grid, kThreads, 0, st>>>(sys, map, mode);
    return hipGetLastError();
}

hipError_t b_fir(int fp64, const BSys *sys, const int2 *tiles, int ntiles, int mode, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (fp64) kb_fir64<<<nb(ntiles), kFirMfmaThreads, 0, st>>>(sys, tiles, mode);
    else kb_fir32<<<nb(ntiles), kFirMfmaThreads, 0, st>>>(sys, tiles, mode);
    return hipGetLastError();
}

hipError_t b_premix(int fp64, int rmax, const BSys *sys, const BMap *map, int nblocks, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (fp64) {
        if (rmax <= 8) kb_premix<double, 8><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
        else if (rmax <= 16) kb_premix<double, 16><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
        else kb_premix<double, kMaxRank><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    } else {
        if (rmax <= 8) kb_premix<float, 8><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
        else if (rmax <= 16) kb_premix<float, 16><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
        else kb_premix<float, kMaxRank><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t spmv_t(int lanes, const BSys *sys, const BMap *map, int nblocks, int k, int ix, int iz, int io,
                         hipStream_t st)
{
    switch (lanes) {
    case 1: kb_spmv<T, 1><<<nb(nblocks), kThreads, 0, st>>>(sys, map, k, ix, iz, io); break;
    case 2: kb_spmv<T, 2><<<nb(nblocks), kThreads, 0, st>>>(sys, map, k, ix, iz, io); break;
    case 4: kb_spmv<T, 4><<<nb(nblocks), kThreads, 0, st>>>(sys, map, k, ix, iz, io); break;
    default: kb_spmv<T, 8><<<nb(nblocks), kThreads, 0, st>>>(sys, map, k, ix, iz, io); break;
    }
    return hipGetLastError();
}

hipError_t b_spmv(int fp64, int lanes, const BSys *sys, const BMap *map, int nblocks, int k, int ix, int iz, int io,
                  hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    return fp64 ? spmv_t<double>(lanes, sys, map, nblocks, k, ix, iz, io, st)
                : spmv_t<float>(lanes, sys, map, nblocks, k, ix, iz, io, st);
}

hipError_t b_update_r(int fp64, const BSys *sys, const BMap *map, int nblocks, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (fp64) kb_update_r<double><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    else kb_update_r<float><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    return hipGetLastError();
}

hipError_t b_update_v(int fp64, const BSys *sys, const BMap *map, int nblocks, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (fp64) kb_update_v<double><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    else kb_update_v<float><<<nb(nblocks), kThreads, 0, st>>>(sys, map);
    return hipGetLastError();
}

hipError_t b_advance(const BSys *sys, int nsys_total, hipStream_t st)
{
    if (nsys_total <= 0) return hipSuccess;
    kb_advance<<<static_cast<unsigned>((nsys_total + 63) / 64), 64, 0, st>>>(sys, nsys_total);
    return hipGetLastError();
}

template <typename T>
static void build_t(const BMap *const *smap, const int *ns, const BSys *sys, int into_fc, hipStream_t st)
{
    if (ns[0] > 0) kb_build<T, 1><<<nb(ns[0]), kThreads, 0, st>>>(sys, smap[0], into_fc);
    if (ns[1] > 0) kb_build<T, 2><<<nb(ns[1]), kThreads, 0, st>>>(sys, smap[1], into_fc);
    if (ns[2] > 0) kb_build<T, 4><<<nb(ns[2]), kThreads, 0, st>>>(sys, smap[2], into_fc);
    if (ns[3] > 0) kb_build<T, 8><<<nb(ns[3]), kThreads, 0, st>>>(sys, smap[3], into_fc);
}

hipError_t b_neighbors(int fp64, const BSys *sys, const BMap *pmap, int npblocks, const BMap *cmap, int ncblocks,
                       const BMap *const *smap, const int *nsblocks, int nsys_total, int into_fc, hipStream_t st)
{
    if (npblocks <= 0) return hipSuccess;
    kb_cell_clear<<<nb(ncblocks), kThreads, 0, st>>>(sys, cmap);
    kb_cell_assign<<<nb(npblocks), kThreads, 0, st>>>(sys, pmap);
    kb_cell_scan<<<nb(nsys_total), 1024, 0, st>>>(sys);
    kb_cell_scatter<<<nb(npblocks), kThreads, 0, st>>>(sys, pmap);
    kb_cell_rank<<<nb(npblocks), kThreads, 0, st>>>(sys, pmap);
    if (fp64) build_t<double>(smap, nsblocks, sys, into_fc, st);
    else build_t<float>(smap, nsblocks, sys, into_fc, st);
    return hipGetLastError();
}

}  // namespace batch
}  // namespace gld
