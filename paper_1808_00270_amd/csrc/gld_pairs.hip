// Pair work of the GLD step on gfx950: cell list, neighbour lists, the
// conservative force and the pair mat-vec y = P x with P = [w(R_ij) T_ij]
// (the pair part of eq. dissipative_force2 and the matrix of the colored
// noise, Sec. II.C).
//
// Design.  Particles are ordered by cell every step (cells of edge >= r_c,
// chosen so that a cell holds about one 128-lane work-group of particles).
// One work-group owns one cell and stages the input vector of the up to 27
// neighbour cells in LDS, chunk by chunk, so the ~260 neighbour gathers per
// particle hit LDS instead of L2.  Once per step the neighbour build stores,
// per particle, the 16-bit indices of its neighbours in that staged
// neighbourhood and the pair weights w(R_ij) (2 + 4 bytes per pair in FP32,
// read as 16-byte vectors, prefetched one group ahead); every mat-vec of the
// step then streams them once.  The parallel tensor form, which also needs
// the unit vectors, recomputes them from staged positions instead.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gld_internal.h"

namespace gld {

namespace {

constexpr int kPairThreads = 128;  // lanes per work-group (one cell)
constexpr int kBuildChunk = 1024;  // staged candidates per round, neighbour build
constexpr int kMaxStencil = 27;

inline unsigned blocks(int64_t n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

template <typename T>
struct V4;
template <>
struct V4<float> {
    using t = float4;
};
template <>
struct V4<double> {
    using t = double4;
};

__device__ __forceinline__ void latch(int *flags, long long *flag_step, int code, long long step)
{
    if (atomicCAS(flags, 0, code) == 0) *flag_step = step;
}

__device__ __forceinline__ double wrap_coord(double x, double L)
{
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0) y += L;
    return y;
}

// cell coordinate of a wrapped position, clamped to [0, nc-1] before the
// integer conversion (NaN or huge values stay in range)
__device__ __forceinline__ int cell_coord(double x, double L, int nc)
{
    const double q = fmin(fmax(floor(x / L * nc), 0.0), static_cast<double>(nc - 1));
    return static_cast<int>(q);
}

// linear interpolation on the distance grid; bin index clamped in floating
// point first (NaN maps to bin 0), so every table access is in range
template <typename T>
__device__ __forceinline__ T interp_w(const T *wt, int n_r, T r0, T inv_dr, T r, T rmin)
{
    if (r < rmin) r = rmin;
    const T t = fmax((r - r0) * inv_dr, T(0));
    const T tb = fmin(floor(t), static_cast<T>(n_r - 2));
    const int b = static_cast<int>(fmax(tb, T(0)));
    const T f = t - static_cast<T>(b);
    return wt[b] + f * (wt[b + 1] - wt[b]);
}

// ---------------------------------------------------------------------------
// cell list (deterministic order: by cell, then by particle id)
// ---------------------------------------------------------------------------
struct Geo {
    double L[3];
    int nc[3];
    int noff[3];
    int offs[3][3];
    double edge[3];  // L / nc
};

__global__ void k_zero(int *p, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_cell_assign(const double *__restrict__ R, int64_t S, int64_t n, Geo g, double *__restrict__ Rw,
                              int *__restrict__ cell_id, int *__restrict__ cell_slot, int *__restrict__ cell_count)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ci[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x = wrap_coord(R[c * S + i], g.L[c]);
        Rw[c * S + i] = x;
        ci[c] = cell_coord(x, g.L[c], g.nc[c]);
    }
    const int cid = (ci[2] * g.nc[1] + ci[1]) * g.nc[0] + ci[0];
    cell_id[i] = cid;
    cell_slot[i] = atomicAdd(&cell_count[cid], 1);
}

// exclusive scan of the cell counts by one work-group (chunked)
__global__ void k_cell_scan(const int *__restrict__ count, int *__restrict__ start, int ncell)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (ncell + nt - 1) / nt;
    const int b = tid * chunk, e = min(ncell, b + chunk);
    int s = 0;
    for (int k = b; k < e; ++k) s += count[k];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int k = b; k < e; ++k) {
        start[k] = run;
        run += count[k];
    }
    if (tid == nt - 1) start[ncell] = part[tid];
}

__global__ void k_cell_scatter(int64_t n, const int *__restrict__ cell_id, const int *__restrict__ cell_slot,
                               const int *__restrict__ start, int *__restrict__ tmp)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tmp[start[cell_id[i]] + cell_slot[i]] = static_cast<int>(i);
}

// rank within the cell by particle id; also the sorted copies of the wrapped
// positions: absolute (double4) and relative to the particle's own cell
// origin (float4 and double4, for staging)
__global__ void k_cell_order(int64_t n, int64_t S, Geo g, const int *__restrict__ cell_id,
                             const int *__restrict__ start, const int *__restrict__ tmp, int *__restrict__ sorted,
                             const double *__restrict__ Rw, double4 *__restrict__ pos_s,
                             float4 *__restrict__ relf, double4 *__restrict__ reld)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_id[i];
    const int b = start[c], e = start[c + 1];
    int rank = 0;
    for (int k = b; k < e; ++k) rank += tmp[k] < i;
    const int s = b + rank;
    sorted[s] = static_cast<int>(i);
    const double x = Rw[i], y = Rw[S + i], z = Rw[2 * S + i];
    pos_s[s] = make_double4(x, y, z, 0.0);
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    const double rx = x - cx * g.edge[0], ry = y - cy * g.edge[1], rz = z - cz * g.edge[2];
    relf[s] = make_float4(static_cast<float>(rx), static_cast<float>(ry), static_cast<float>(rz), 0.f);
    reld[s] = make_double4(rx, ry, rz, 0.0);
}

// ---------------------------------------------------------------------------
// the stencil of a home cell: up to 27 neighbour cells (offsets reduced to
// distinct values per axis for grids of 1 or 2 cells), their sorted ranges,
// the periodic image shift of each and the running base of the concatenation
// ---------------------------------------------------------------------------
struct Stencil {
    int n;
    int start[kMaxStencil];
    int base[kMaxStencil + 1];
    double shift[kMaxStencil][3];
    float offf[kMaxStencil][3];   // (neighbour cell origin + image shift - home origin), float
    double offd[kMaxStencil][3];  // the same in double
    double origin[3];
    int home;                     // entry of the home cell itself
};

// stencil entry holding staged index l (base[] ascending, n <= 27)
__device__ __forceinline__ int stencil_entry(const Stencil &st, int l)
{
    int lo = 0, hi = st.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st.base[mid] <= l) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ void make_stencil(const Geo &g, const int *__restrict__ cstart, int cid, Stencil &st)
{
    const int cx = cid % g.nc[0], cy = (cid / g.nc[0]) % g.nc[1], cz = cid / (g.nc[0] * g.nc[1]);
    st.origin[0] = cx * g.edge[0];
    st.origin[1] = cy * g.edge[1];
    st.origin[2] = cz * g.edge[2];
    int k = 0, base = 0;
    for (int a = 0; a < g.noff[2]; ++a)
        for (int b = 0; b < g.noff[1]; ++b)
            for (int e = 0; e < g.noff[0]; ++e) {
                const int u[3] = {cx + g.offs[0][e], cy + g.offs[1][b], cz + g.offs[2][a]};
                int w[3];
                const int hc[3] = {cx, cy, cz};
                for (int c = 0; c < 3; ++c) {
                    w[c] = (u[c] + g.nc[c]) % g.nc[c];
                    // image shift so the staged copy sits next to the home cell
                    st.shift[k][c] = (u[c] < 0) ? -g.L[c] : (u[c] >= g.nc[c] ? g.L[c] : 0.0);
                    // origin(w) + shift - origin(home) = (u - home) edge
                    st.offd[k][c] = (u[c] - hc[c]) * g.edge[c];
                    st.offf[k][c] = static_cast<float>(st.offd[k][c]);
                }
                const int nid = (w[2] * g.nc[1] + w[1]) * g.nc[0] + w[0];
                if (nid == cid && st.shift[k][0] == 0.0 && st.shift[k][1] == 0.0 && st.shift[k][2] == 0.0) st.home = k;
                st.start[k] = cstart[nid];
                st.base[k] = base;
                base += cstart[nid + 1] - cstart[nid];
                ++k;
            }
    st.n = k;
    st.base[k] = base;
}

// ---------------------------------------------------------------------------
// neighbour build: one work-group per cell.  Candidates are staged in LDS
// (positions relative to the home cell, periodic images applied, as float and
// double); the wave walks them in lockstep (broadcast reads, no memory
// traffic in the loop).  Per particle s (sorted order) it writes, column-major
// so that a wave's 64 consecutive particles touch one contiguous segment,
//   nbj[k][s]  sorted index of the k-th neighbour
//   nbw[k][s]  squared distance (turned into w(R_ij) by k_weights)
//   nbe[c][k][s]  separation vector (parallel tensor form only)
//   nn[s]      neighbour count,  fc[p] WCA force (FP64, original order)
// The pair decision is taken in FP64 in the FP64 mode and in FP32 otherwise
// (a pair within rounding of r_c has w ~ 0 either way); the force is FP64.
// ---------------------------------------------------------------------------
struct BuildArgs {
    Geo g;
    int64_t n, S;
    const int *cstart, *sorted;
    const double4 *reld_src;  // positions relative to their own cell, double
    int exact64, parallel;
    double rc2;
    int cap;
    double wca_rc2, wca_s2, wca_eps;
    int *nbj;
    void *nbw, *nbe;
    int *nn;
    double *fc;
    int *flags;
    long long *flag_step;
    const long long *d_step;
};

template <typename T>
__global__ __launch_bounds__(kPairThreads) void k_build(BuildArgs a)
{
    constexpr int CH = 1024;
    __shared__ Stencil st;
    __shared__ float4 relf[CH];
    __shared__ double4 reld[CH];
    __shared__ int sid[CH];
    const int cid = blockIdx.x;
    if (threadIdx.x == 0) make_stencil(a.g, a.cstart, cid, st);
    __syncthreads();
    const int h0 = a.cstart[cid], h1 = a.cstart[cid + 1];
    const int total = st.base[st.n];
    const float Lxf = static_cast<float>(a.g.L[0]), Lyf = static_cast<float>(a.g.L[1]), Lzf = static_cast<float>(a.g.L[2]);
    const bool mi0 = a.g.nc[0] < 3, mi1 = a.g.nc[1] < 3, mi2 = a.g.nc[2] < 3;
    const float rc2f = static_cast<float>(a.rc2);
    const int64_t plane = static_cast<int64_t>(a.cap) * a.n;
    T *nbw = static_cast<T *>(a.nbw);
    T *nbe = static_cast<T *>(a.nbe);
    for (int g0 = h0; g0 < h1; g0 += kPairThreads) {
        const int s = g0 + threadIdx.x;
        const bool live = s < h1;
        const int self_l = st.base[st.home] + (s - h0);
        const double4 xd = live ? a.reld_src[s] : make_double4(0, 0, 0, 0);
        const float xf0 = static_cast<float>(xd.x), xf1 = static_cast<float>(xd.y), xf2 = static_cast<float>(xd.z);
        int cnt = 0;
        double fx = 0, fy = 0, fz = 0;
        for (int c0 = 0; c0 < total; c0 += CH) {
            const int c1 = min(total, c0 + CH);
            __syncthreads();
            constexpr int per = CH / kPairThreads;
            double4 v[per];
            int sj[per];
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int l = c0 + static_cast<int>(threadIdx.x) + j * kPairThreads;
                if (l < c1) {
                    const int t = stencil_entry(st, l);
                    sj[j] = st.start[t] + (l - st.base[t]);
                    v[j] = a.reld_src[sj[j]];
                    v[j].x += st.offd[t][0];
                    v[j].y += st.offd[t][1];
                    v[j].z += st.offd[t][2];
                }
            }
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int l = static_cast<int>(threadIdx.x) + j * kPairThreads;
                if (c0 + l < c1) {
                    reld[l] = v[j];
                    relf[l] = make_float4(static_cast<float>(v[j].x), static_cast<float>(v[j].y),
                                          static_cast<float>(v[j].z), 0.f);
                    sid[l] = sj[j];
                }
            }
            __syncthreads();
            if (!live) continue;
            for (int l = c0; l < c1; ++l) {
                bool in;
                double r2, ex, ey, ez;
                if (a.exact64) {
                    const double4 q = reld[l - c0];
                    ex = xd.x - q.x;
                    ey = xd.y - q.y;
                    ez = xd.z - q.z;
                    if (mi0) ex -= a.g.L[0] * rint(ex / a.g.L[0]);
                    if (mi1) ey -= a.g.L[1] * rint(ey / a.g.L[1]);
                    if (mi2) ez -= a.g.L[2] * rint(ez / a.g.L[2]);
                    r2 = ex * ex + ey * ey + ez * ez;
                    in = r2 < a.rc2;
                } else {
                    const float4 q = relf[l - c0];
                    float dx = xf0 - q.x, dy = xf1 - q.y, dz = xf2 - q.z;
                    if (mi0) dx -= Lxf * rintf(dx / Lxf);
                    if (mi1) dy -= Lyf * rintf(dy / Lyf);
                    if (mi2) dz -= Lzf * rintf(dz / Lzf);
                    const float r2f = dx * dx + dy * dy + dz * dz;
                    in = r2f < rc2f;
                    r2 = r2f;
                    ex = dx;
                    ey = dy;
                    ez = dz;
                }
                if (!in || l == self_l) continue;
                if (r2 < a.wca_rc2 * 1.0001) {
                    // WCA force in FP64 from the staged double positions
                    const double4 q = reld[l - c0];
                    double gx = xd.x - q.x, gy = xd.y - q.y, gz = xd.z - q.z;
                    if (mi0) gx -= a.g.L[0] * rint(gx / a.g.L[0]);
                    if (mi1) gy -= a.g.L[1] * rint(gy / a.g.L[1]);
                    if (mi2) gz -= a.g.L[2] * rint(gz / a.g.L[2]);
                    const double rd2 = gx * gx + gy * gy + gz * gz;
                    if (rd2 < a.wca_rc2) {
                        const double s2 = a.wca_s2 / rd2, s6 = s2 * s2 * s2;
                        const double fr = 24.0 * a.wca_eps * (2.0 * s6 * s6 - s6) / rd2;
                        fx += fr * gx;
                        fy += fr * gy;
                        fz += fr * gz;
                    }
                }
                if (cnt < a.cap) {
                    const int64_t o = static_cast<int64_t>(cnt) * a.n + s;
                    a.nbj[o] = sid[l - c0];
                    nbw[o] = static_cast<T>(r2);
                    if (a.parallel) {
                        nbe[o] = static_cast<T>(ex);
                        nbe[plane + o] = static_cast<T>(ey);
                        nbe[2 * plane + o] = static_cast<T>(ez);
                    }
                }
                ++cnt;
            }
        }
        if (live) {
            const int p = a.sorted[s];
            if (cnt > a.cap) latch(a.flags, a.flag_step, GLD_ERR_CAPACITY, *a.d_step);
            a.nn[s] = min(cnt, a.cap);
            a.fc[p] = fx;
            a.fc[a.S + p] = fy;
            a.fc[2 * a.S + p] = fz;
        }
    }
}

__device__ __forceinline__ double interp_wd(const double *wt, int n_r, double r0, double dr, double r, double rmin)
{
    if (r < rmin) r = rmin;
    const double t = fmax((r - r0) / dr, 0.0);
    const double tb = fmin(floor(t), static_cast<double>(n_r - 2));
    const int b = static_cast<int>(fmax(tb, 0.0));
    const double f = t - b;
    return wt[b] * (1.0 - f) + wt[b + 1] * f;
}

// ---------------------------------------------------------------------------
// pair weights, lane-parallel over each particle's own list (lockstep k,
// coalesced): nbw <- w(sqrt(nbw)) (linear interpolation on the distance grid,
// frozen below r_cut_min), unit vectors for the parallel form, and the block
// Gershgorin check of the largest row sum of |w| (a bound on the spectral norm
// of P, ||T_ij|| = 1 for both tensor forms) against the noise interval.
// ---------------------------------------------------------------------------
template <typename T, bool PAR>
__global__ __launch_bounds__(256) void k_weights(int64_t n, int cap, const int *__restrict__ nn, T *__restrict__ nbw,
                                                 T *__restrict__ nbe, const double *__restrict__ wtab, int n_r,
                                                 double r0, double dr, double r_cut_min, double lam_hi,
                                                 unsigned *rowmax, int *flags, long long *flag_step,
                                                 const long long *d_step)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int cnt = nn[s];
    const int64_t plane = static_cast<int64_t>(cap) * n;
    const T tr0 = static_cast<T>(r0), inv_dr = static_cast<T>(1.0 / dr), rmin = static_cast<T>(r_cut_min);
    double rowsum = 0;
    for (int k = 0; k < cnt; ++k) {
        const int64_t o = static_cast<int64_t>(k) * n + s;
        const T r = sqrt(nbw[o]);
        T w;
        if (sizeof(T) == 8) {
            w = static_cast<T>(interp_wd(wtab, n_r, r0, dr, static_cast<double>(r), r_cut_min));
        } else {
            const T rr = r < rmin ? rmin : r;
            const T t = fmax((rr - tr0) * inv_dr, T(0));
            const T tb = fmin(floor(t), static_cast<T>(n_r - 2));
            const int b = static_cast<int>(fmax(tb, T(0)));
            const T f = t - static_cast<T>(b);
            const T w0 = static_cast<T>(wtab[b]), w1 = static_cast<T>(wtab[b + 1]);
            w = w0 + f * (w1 - w0);
        }
        nbw[o] = w;
        rowsum += fabs(static_cast<double>(w));
        if (PAR) {
            const T inv = T(1) / r;
            nbe[o] *= inv;
            nbe[plane + o] *= inv;
            nbe[2 * plane + o] *= inv;
        }
    }
    if (rowsum > lam_hi) {
        if (atomicCAS(flags, 0, GLD_ERR_INTERVAL) == 0) *flag_step = *d_step;
    }
    atomicMax(rowmax, __float_as_uint(static_cast<float>(rowsum)));
}

// ---------------------------------------------------------------------------
// sorted copies of the inputs of the pair mat-vecs:
//   ys[s]    = Y[p]                       (dissipative input)
//   us[q][s] = U[step % block][q][p]      (filter outputs of this step)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_permute(int64_t n, int64_t S, const int *__restrict__ sorted, const T *__restrict__ Y,
                          typename V4<T>::t *__restrict__ ys, const T *__restrict__ U, int r, int rcap, int block,
                          const long long *__restrict__ d_step, typename V4<T>::t *__restrict__ us)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int p = sorted[s];
    typename V4<T>::t v;
    v.x = Y[p];
    v.y = Y[S + p];
    v.z = Y[2 * S + p];
    v.w = T(0);
    ys[s] = v;
    if (r > 0) {
        const int bi = static_cast<int>(*d_step % block);
        const T *u = U + static_cast<int64_t>(bi) * rcap * 3 * S;
        for (int q = 0; q < r; ++q) {
            const T *uq = u + static_cast<int64_t>(q) * 3 * S;
            typename V4<T>::t o;
            o.x = uq[p];
            o.y = uq[S + p];
            o.z = uq[2 * S + p];
            o.w = T(0);
            us[static_cast<int64_t>(q) * S + s] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// pair mat-vec with fused combination, one thread per particle (sorted order):
//   out_s = a (P x)_s + b x_s + cz z_s + sum_q coef[q] us_q,s   (+ add[p])
// The k-th neighbour index and weight of 64 consecutive particles are one
// contiguous segment (column-major lists); x_j is gathered (cell order keeps
// a wave's neighbourhood in a few tens of KiB, i.e. in L1/L2).  x, z, us are
// sorted T4; out is sorted T4 or scattered to the original order [3][S]
// (out_orig), optionally plus add_orig[p].
// ---------------------------------------------------------------------------
struct MvArgs {
    int64_t n, S;
    const int *sorted;
    const int *nbj;
    const void *nbw, *nbe;
    const int *nn;
    int cap;
    double a, b, cz;
    const void *x, *z, *coef, *us, *add_orig;
    int r;
    void *out_sorted, *out_orig;
};

template <typename T, bool PAR>
__global__ __launch_bounds__(256) void k_mv(MvArgs A)
{
    using T4 = typename V4<T>::t;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= A.n) return;
    const T4 *__restrict__ x = static_cast<const T4 *>(A.x);
    const int *__restrict__ nbj = A.nbj;
    const T *__restrict__ nbw = static_cast<const T *>(A.nbw);
    const T *__restrict__ nbe = static_cast<const T *>(A.nbe);
    const int64_t n = A.n;
    T p0 = 0, p1 = 0, p2 = 0;
    if (A.a != 0.0) {
        const int cnt = A.nn[s];
        const int64_t plane = static_cast<int64_t>(A.cap) * n;
        int k = 0;
        // four independent gathers in flight per iteration
        for (; k + 3 < cnt; k += 4) {
            int j[4];
            T w[4];
            T4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t o = static_cast<int64_t>(k + u) * n + s;
                j[u] = nbj[o];
                w[u] = nbw[o];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = x[j[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (PAR) {
                    const int64_t o = static_cast<int64_t>(k + u) * n + s;
                    const T ex = nbe[o], ey = nbe[plane + o], ez = nbe[2 * plane + o];
                    const T sc = w[u] * (ex * v[u].x + ey * v[u].y + ez * v[u].z);
                    p0 += sc * ex;
                    p1 += sc * ey;
                    p2 += sc * ez;
                } else {
                    p0 += w[u] * v[u].x;
                    p1 += w[u] * v[u].y;
                    p2 += w[u] * v[u].z;
                }
            }
        }
        for (; k < cnt; ++k) {
            const int64_t o = static_cast<int64_t>(k) * n + s;
            const T w = nbw[o];
            const T4 v = x[nbj[o]];
            if (PAR) {
                const T ex = nbe[o], ey = nbe[plane + o], ez = nbe[2 * plane + o];
                const T sc = w * (ex * v.x + ey * v.y + ez * v.z);
                p0 += sc * ex;
                p1 += sc * ey;
                p2 += sc * ez;
            } else {
                p0 += w * v.x;
                p1 += w * v.y;
                p2 += w * v.z;
            }
        }
    }
    T o0 = static_cast<T>(A.a) * p0, o1 = static_cast<T>(A.a) * p1, o2 = static_cast<T>(A.a) * p2;
    if (A.b != 0.0) {
        const T4 xs = x[s];
        o0 += static_cast<T>(A.b) * xs.x;
        o1 += static_cast<T>(A.b) * xs.y;
        o2 += static_cast<T>(A.b) * xs.z;
    }
    if (A.cz != 0.0) {
        const T4 zs = static_cast<const T4 *>(A.z)[s];
        o0 += static_cast<T>(A.cz) * zs.x;
        o1 += static_cast<T>(A.cz) * zs.y;
        o2 += static_cast<T>(A.cz) * zs.z;
    }
    if (A.r > 0) {
        const T *coef = static_cast<const T *>(A.coef);
        const T4 *us = static_cast<const T4 *>(A.us);
        for (int q = 0; q < A.r; ++q) {
            const T c = coef[q];
            const T4 u = us[static_cast<int64_t>(q) * A.S + s];
            o0 += c * u.x;
            o1 += c * u.y;
            o2 += c * u.z;
        }
    }
    if (A.out_sorted) {
        T4 o;
        o.x = o0;
        o.y = o1;
        o.z = o2;
        o.w = T(0);
        static_cast<T4 *>(A.out_sorted)[s] = o;
    } else {
        const int p = A.sorted[s];
        T *out = static_cast<T *>(A.out_orig);
        if (A.add_orig) {
            const T *ad = static_cast<const T *>(A.add_orig);
            o0 += ad[p];
            o1 += ad[A.S + p];
            o2 += ad[2 * A.S + p];
        }
        out[p] = o0;
        out[A.S + p] = o1;
        out[2 * A.S + p] = o2;
    }
}

Geo make_geo(const Dev &d)
{
    Geo g{};
    for (int c = 0; c < 3; ++c) {
        g.L[c] = d.box[c];
        g.nc[c] = d.nc[c];
        g.noff[c] = d.noff[c];
        g.edge[c] = d.box[c] / d.nc[c];
        for (int k = 0; k < 3; ++k) g.offs[c][k] = d.offs[c][k];
    }
    return g;
}

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
hipError_t launch_zero_int(int *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_zero<<<blocks(n, 256), 256, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_neighbors(const Dev &d, hipStream_t st, double *fc_out)
{
    hipError_t e;
    if ((e = launch_zero_int(d.cell_count, d.ncell, st)) != hipSuccess) return e;
    if ((e = launch_zero_int(reinterpret_cast<int *>(d.d_rowmax), 1, st)) != hipSuccess) return e;
    const Geo g = make_geo(d);
    k_cell_assign<<<blocks(d.n, 256), 256, 0, st>>>(d.R, d.S, d.n, g, d.Rw, d.cell_id, d.cell_slot, d.cell_count);
    k_cell_scan<<<1, 1024, 0, st>>>(d.cell_count, d.cell_start, d.ncell);
    k_cell_scatter<<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.cell_id, d.cell_slot, d.cell_start, d.cell_tmp);
    k_cell_order<<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, g, d.cell_id, d.cell_start, d.cell_tmp, d.cell_sorted,
                                                   d.Rw, static_cast<double4 *>(d.pos_s),
                                                   static_cast<float4 *>(d.relf), static_cast<double4 *>(d.reld));
    BuildArgs a{};
    a.g = g;
    a.n = d.n;
    a.S = d.S;
    a.cstart = d.cell_start;
    a.sorted = d.cell_sorted;
    a.reld_src = static_cast<const double4 *>(d.reld);
    a.exact64 = d.fp64;
    a.parallel = d.parallel;
    a.rc2 = d.r_cut * d.r_cut;
    a.cap = d.cap;
    const double rw = std::pow(2.0, 1.0 / 6.0) * d.wca_sigma;
    a.wca_rc2 = d.wca_eps != 0.0 ? rw * rw : 0.0;
    a.wca_s2 = d.wca_sigma * d.wca_sigma;
    a.wca_eps = d.wca_eps;
    a.nbj = d.nbj;
    a.nbw = d.nbw;
    a.nbe = d.nbe;
    a.nn = d.nn;
    a.fc = fc_out;
    a.flags = d.d_flags;
    a.flag_step = d.d_flag_step;
    a.d_step = d.d_step;
    if (d.fp64) k_build<double><<<d.ncell, kPairThreads, 0, st>>>(a);
    else k_build<float><<<d.ncell, kPairThreads, 0, st>>>(a);
    const unsigned nb = blocks(d.n, 256);
    if (d.fp64) {
        if (d.parallel)
            k_weights<double, true><<<nb, 256, 0, st>>>(d.n, d.cap, d.nn, (double *)d.nbw, (double *)d.nbe, d.wtab,
                                                        d.n_r, d.r0, d.dr, d.r_cut_min, d.lam_hi, d.d_rowmax,
                                                        d.d_flags, d.d_flag_step, d.d_step);
        else
            k_weights<double, false><<<nb, 256, 0, st>>>(d.n, d.cap, d.nn, (double *)d.nbw, nullptr, d.wtab, d.n_r,
                                                         d.r0, d.dr, d.r_cut_min, d.lam_hi, d.d_rowmax, d.d_flags,
                                                         d.d_flag_step, d.d_step);
    } else {
        if (d.parallel)
            k_weights<float, true><<<nb, 256, 0, st>>>(d.n, d.cap, d.nn, (float *)d.nbw, (float *)d.nbe, d.wtab,
                                                       d.n_r, d.r0, d.dr, d.r_cut_min, d.lam_hi, d.d_rowmax,
                                                       d.d_flags, d.d_flag_step, d.d_step);
        else
            k_weights<float, false><<<nb, 256, 0, st>>>(d.n, d.cap, d.nn, (float *)d.nbw, nullptr, d.wtab, d.n_r,
                                                        d.r0, d.dr, d.r_cut_min, d.lam_hi, d.d_rowmax, d.d_flags,
                                                        d.d_flag_step, d.d_step);
    }
    return hipGetLastError();
}

hipError_t launch_permute(const Dev &d, hipStream_t st, int r)
{
    if (d.fp64)
        k_permute<double><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, d.cell_sorted, static_cast<const double *>(d.Y),
                                                            static_cast<double4 *>(d.ys),
                                                            static_cast<const double *>(d.U), r, d.fir_rcap,
                                                            d.fir_block, d.d_step, static_cast<double4 *>(d.us));
    else
        k_permute<float><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, d.cell_sorted, static_cast<const float *>(d.Y),
                                                           static_cast<float4 *>(d.ys), static_cast<const float *>(d.U),
                                                           r, d.fir_rcap, d.fir_block, d.d_step,
                                                           static_cast<float4 *>(d.us));
    return hipGetLastError();
}

hipError_t launch_spmv(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz, const void *z,
                       const void *coef, int r, void *out_sorted, void *out_orig, const void *add_orig)
{
    MvArgs A{};
    A.n = d.n;
    A.S = d.S;
    A.sorted = d.cell_sorted;
    A.nbj = d.nbj;
    A.nbw = d.nbw;
    A.nbe = d.nbe;
    A.nn = d.nn;
    A.cap = d.cap;
    A.a = d.has_pair ? a : 0.0;
    A.b = b;
    A.cz = cz;
    A.x = x;
    A.z = z;
    A.coef = coef;
    A.us = d.us;
    A.add_orig = add_orig;
    A.r = coef ? r : 0;
    A.out_sorted = out_sorted;
    A.out_orig = out_orig;
    const unsigned nb = blocks(d.n, 256);
    if (d.fp64) {
        if (d.parallel) k_mv<double, true><<<nb, 256, 0, st>>>(A);
        else k_mv<double, false><<<nb, 256, 0, st>>>(A);
    } else {
        if (d.parallel) k_mv<float, true><<<nb, 256, 0, st>>>(A);
        else k_mv<float, false><<<nb, 256, 0, st>>>(A);
    }
    return hipGetLastError();
}

hipError_t launch_dissipative(const Dev &d, hipStream_t st)
{
    // F^D' = -(P Y) + Dneg, scattered to the original order
    return launch_spmv(d, st, -1.0, 0.0, d.ys, 0.0, nullptr, nullptr, 0, nullptr, d.FD, d.Dneg);
}

}  // namespace gld
