// Pair work of the GLD step on gfx950: cell list, neighbour lists, the
// conservative force and the pair mat-vec y = P x with P = [w(R_ij) T_ij]
// (the pair part of eq. dissipative_force2 and the matrix of the colored
// noise, Sec. II.C).
//
// Design.  Particles are ordered by cell (cells of edge >= r_c + skin, about
// ninety particles each at the benchmark density).  The lists come in two
// stages.  Candidate lists hold, for every particle, the particles within
// r_c + skin as 16-bit indices into the concatenated candidate list of its
// cell's stencil (the up to 27 cells around it); they and the cell order are
// rebuilt only when some particle has moved more than skin/2 since the last
// build.  Every step the refresh filters the candidates to the pairs within
// r_c, in candidate order, with their final weights, and computes the WCA
// force and the Gershgorin bound of the noise interval.  Every mat-vec of the
// step (about forty: the dissipative force and the Chebyshev chain of the
// noise) then runs one work-group per cell: it stages the input vector of the
// stencil in LDS, and four lanes per particle stream the pair chunks (one
// 16-byte load brings 8 indices, another 4 weights; a wave's loads are one
// contiguous kilobyte) and gather from LDS.  The lists are 6 bytes per pair
// in FP32, so a mat-vec is bound by streaming them from HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "gld_internal.h"

namespace gld {

namespace {

constexpr int kPairThreads = 128;  // lanes per work-group of the neighbour build (one cell)
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

template <typename T>
struct V2;
template <>
struct V2<float> {
    using t = float2;
};
template <>
struct V2<double> {
    using t = double2;
};

// 16-byte loads marked non-temporal, for the candidate lists, which stream
// through L2 once per refresh: the hint keeps them from evicting the
// positions that the 27 work-groups of a cell's neighbourhood each stage.
// (The refresh's pair-list stores stay ordinary: their 16-byte pieces of a
// line arrive at different times and are merged in L2.  The mat-vec's loads
// of the pair lists stay ordinary too: its launches alternate the cell order
// so that each starts on the lists the one before read last, and with the
// hint that alternation measured no gain, without it 5% in FP64.)
template <typename V>
struct NtVec;
template <>
struct NtVec<uint4> {
    typedef unsigned t __attribute__((ext_vector_type(4)));
};
template <>
struct NtVec<float4> {
    typedef float t __attribute__((ext_vector_type(4)));
};
template <>
struct NtVec<double4> {
    typedef double t __attribute__((ext_vector_type(4)));
};
template <typename V>
__device__ __forceinline__ V stream_load(const V *p)
{
    const typename NtVec<V>::t v = __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<V>::t *>(p));
    V r;
    r.x = v.x;
    r.y = v.y;
    r.z = v.z;
    r.w = v.w;
    return r;
}
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

// The cell list and the candidate lists are rebuilt only when the device
// flag *gate is set (see k_disp_check); every kernel of the rebuild checks it
// first, so the same launch sequence serves every step of a graph.  The cell
// counts start at zero (the scan of the previous rebuild cleared them).
__global__ void k_cell_assign(const double *__restrict__ R, int64_t S, int64_t n, Geo g, double *__restrict__ Rw,
                              int *__restrict__ cell_id, int *__restrict__ cell_slot, int *__restrict__ cell_count,
                              const int *gate)
{
    if (*gate == 0) return;
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

// exclusive scan of the cell counts by one work-group (chunked); the counts
// are cleared behind it, so they start at zero at the next rebuild (the
// workspace starts zeroed)
__global__ void k_cell_scan(int *__restrict__ count, int *__restrict__ start, int ncell, const int *gate)
{
    if (*gate == 0) return;
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
        count[k] = 0;
    }
    if (tid == nt - 1) start[ncell] = part[tid];
}

__global__ void k_cell_scatter(int64_t n, const int *__restrict__ cell_id, const int *__restrict__ cell_slot,
                               const int *__restrict__ start, int *__restrict__ tmp, const int *gate)
{
    if (*gate == 0) return;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tmp[start[cell_id[i]] + cell_slot[i]] = static_cast<int>(i);
}

// rank within the cell by particle id; at the build, the sorted copies of
// the unwrapped positions (rb) and of the wrapped positions relative to the
// particle's own cell origin (relb); k_rel_update moves both every step
__global__ void k_cell_order(int64_t n, int64_t S, Geo g, const int *__restrict__ cell_id,
                             const int *__restrict__ start, const int *__restrict__ tmp, int *__restrict__ sorted,
                             const double *__restrict__ R, const double *__restrict__ Rw, double4 *__restrict__ rb,
                             double4 *__restrict__ relb, const int *gate)
{
    if (*gate == 0) return;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_id[i];
    const int b = start[c], e = start[c + 1];
    int rank = 0;
    for (int k = b; k < e; ++k) rank += tmp[k] < i;
    const int s = b + rank;
    sorted[s] = static_cast<int>(i);
    rb[s] = make_double4(R[i], R[S + i], R[2 * S + i], 0.0);
    const double x = Rw[i], y = Rw[S + i], z = Rw[2 * S + i];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    relb[s] = make_double4(x - cx * g.edge[0], y - cy * g.edge[1], z - cz * g.edge[2], 0.0);
}

// Every step, before the rebuild kernels: does some particle lie more than
// skin/2 from where it was at the last build?  Then the pairs within r_c may
// include one missing from the candidate list, and the lists are rebuilt.
__global__ void k_disp_check(int64_t n, int64_t S, const int *__restrict__ sorted, const double *__restrict__ R,
                             const double4 *__restrict__ rb, double thr2, int *gate, const long long *d_step,
                             int period)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    // a fixed cadence as well: the positions of every step that is a multiple of `period`
    if (period > 0 && s == 0 && (*d_step + 1) % period == 0) atomicOr(gate, 1);
    bool far = false;
    if (s < n) {
        const int p = sorted[s];
        const double4 b = rb[s];
        const double dx = R[p] - b.x, dy = R[S + p] - b.y, dz = R[2 * S + p] - b.z;
        far = !(dx * dx + dy * dy + dz * dz <= thr2);  // NaN counts as far
    }
    if (__any(far) && (threadIdx.x & 63) == 0) atomicOr(gate, 1);
}

// Every step, after the rebuild kernels: current positions in the cell order
// of the last build, relative to the build-time cell (relb + R - rb, from the
// unwrapped displacement, so crossing the box edge needs no care), as double
// and float, and wrapped absolute (WCA).  Clears the rebuild flag and the
// row-sum maximum that the refresh then takes.
__global__ void k_rel_update(int64_t n, int64_t S, Geo g, const int *__restrict__ sorted,
                             const double *__restrict__ R, const double4 *__restrict__ rb,
                             const double4 *__restrict__ relb, double4 *__restrict__ reld, float4 *__restrict__ relf,
                             double4 *__restrict__ pos_s, int *gate, unsigned *rowmax)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s == 0) {
        *gate = 0;
        *rowmax = 0u;
    }
    if (s >= n) return;
    const int p = sorted[s];
    const double x = R[p], y = R[S + p], z = R[2 * S + p];
    const double4 b = rb[s], q = relb[s];
    const double4 rel = make_double4(q.x + (x - b.x), q.y + (y - b.y), q.z + (z - b.z), 0.0);
    reld[s] = rel;
    relf[s] = make_float4(static_cast<float>(rel.x), static_cast<float>(rel.y), static_cast<float>(rel.z), 0.f);
    pos_s[s] = make_double4(wrap_coord(x, g.L[0]), wrap_coord(y, g.L[1]), wrap_coord(z, g.L[2]), 0.0);
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
// Neighbour lists.  Particle s (sorted order) with n_s neighbours holds in
// entry k the neighbour's position in the concatenated candidate list of the
// home cell's stencil (16 bits; the order in which the mat-vec stages them)
// and the pair weight, in chunks of 8 entries, blocked by cell: for the cell
// starting at sorted index h0 with occ particles, particle j = s - h0,
// C = cap/8,
//   nbl  uint16  entry (k, s) at ((h0 C + (k>>3) occ + j) 8 + (k&7)
//   nbw  T       entry (k, s) at ((2 h0 C + (k>>2) occ + j) 4 + (k&3)
// so that one lane fetches 8 indices, or 4 weights, with one 16-byte load
// (two for FP64 weights), a wave's consecutive particles read one
// contiguous segment, and a cell's lists are one contiguous stretch.  A cell
// whose stencil holds at most kNarrowStencil candidates stores its indices
// in 12 bits instead (narrow): chunk c of particle j is the 12-byte word
// triple at c occ + j from the cell's start (the same start as the wide
// form), entries 0..7 at bits 12 k of the 96.  The weight is w(R_ij) for the isotropic tensor and
// w(R_ij) / R_ij^2 for the parallel one, whose mat-vec rebuilds the
// separation d from staged positions (w e e^T x = (w / R^2) d (d . x)).
// Lists are padded to a multiple of 8 with zero weights (index of the
// particle itself).  The stencil of each cell is stored as well:
//   stab int2 [ncell][28]      (first sorted index, concatenation base) of
//                               each entry; entry nst holds (0, total)
// ---------------------------------------------------------------------------
constexpr int kStab = kMaxStencil + 1;
constexpr int kNarrowStencil = 4096;

// 8 staged indices (16-bit fields of a uint4) packed into 12-bit fields
__device__ __forceinline__ uint3 ids_pack12(uint4 w)
{
    const unsigned e0 = w.x & 0xffffu, e1 = w.x >> 16, e2 = w.y & 0xffffu, e3 = w.y >> 16;
    const unsigned e4 = w.z & 0xffffu, e5 = w.z >> 16, e6 = w.w & 0xffffu, e7 = w.w >> 16;
    uint3 v;
    v.x = e0 | (e1 << 12) | (e2 << 24);
    v.y = (e2 >> 8) | (e3 << 4) | (e4 << 16) | (e5 << 28);
    v.z = (e5 >> 4) | (e6 << 8) | (e7 << 20);
    return v;
}

// chunk k of a cell's index list, as loaded (narrow: w unused)
template <bool NARROW>
__device__ __forceinline__ uint4 ids_load(const void *cell, int64_t k)
{
    if constexpr (NARROW) {
        const uint3 v = static_cast<const uint3 *>(cell)[k];
        return make_uint4(v.x, v.y, v.z, 0u);
    } else {
        return static_cast<const uint4 *>(cell)[k];
    }
}

// Packed chunk (narrow cells of FP32 isotropic lists): 8 words, each the
// 12-bit staged index with the weight in 20-bit fixed point above it.
__device__ __forceinline__ uint32_t pack_entry(unsigned idx, float w, float scale, int sgn)
{
    int q = __float2int_rn(w * scale);
    q = sgn ? min(max(q, -kWeightQMaxSigned), kWeightQMaxSigned) : min(max(q, 0), kWeightQMax);
    return (idx & 0xfffu) | (static_cast<uint32_t>(q) << 12);
}

// FP64 lists: a 64-bit word, the index in bits 0-11, 52-bit weight above.
// q = qh 2^20 + ql (ql in [0, 2^20), all exact in double) gives the high
// word qh and the low word ql << 12 | idx without 64-bit integer steps
__device__ __forceinline__ uint64_t pack_entry64(unsigned idx, double w, double scale, int sgn)
{
    const double lim = sgn ? static_cast<double>(kWeightQMaxSigned64) : static_cast<double>(kWeightQMax64);
    const double q = fmin(fmax(rint(w * scale), sgn ? -lim : 0.0), lim);
    const double qh = floor(q * 0x1p-20);
    const unsigned ql = static_cast<unsigned>(fma(qh, -0x1p20, q));
    const unsigned hi = sgn ? static_cast<unsigned>(static_cast<int>(qh)) : static_cast<unsigned>(qh);
    return (static_cast<uint64_t>(hi) << 32) | ((ql << 12) | (idx & 0xfffu));
}

// the weight field of a 64-bit word: high word times 2^20 plus the low
// word's upper 20 bits (exact in double)
__device__ __forceinline__ double entry_q64(uint64_t e, int sgn)
{
    const unsigned hi = static_cast<unsigned>(e >> 32), lo = static_cast<unsigned>(e);
    const double h = sgn ? static_cast<double>(static_cast<int>(hi)) : static_cast<double>(hi);
    return fma(h, 0x1p20, static_cast<double>(lo >> 12));
}

__device__ __forceinline__ float entry_weight(uint32_t e, float inv, int sgn)
{
    const int q = sgn ? (static_cast<int>(e) >> 12) : static_cast<int>(e >> 12);
    return static_cast<float>(q) * inv;
}

// a packed FP32 chunk (words pa: entries 0-3, pb: 4-7) as 16-bit indices
// and weights (W4, the mat-vec's four-vector type, is a template parameter
// so that the FP64 instantiations, which never call it, still compile)
template <typename W4>
__device__ __forceinline__ void unpack_chunk(uint4 pa, uint4 pb, float inv, int sgn, uint4 &id, W4 &wa, W4 &wb)
{
    id = make_uint4((pa.x & 0xfffu) | ((pa.y & 0xfffu) << 16), (pa.z & 0xfffu) | ((pa.w & 0xfffu) << 16),
                    (pb.x & 0xfffu) | ((pb.y & 0xfffu) << 16), (pb.z & 0xfffu) | ((pb.w & 0xfffu) << 16));
    wa.x = entry_weight(pa.x, inv, sgn);
    wa.y = entry_weight(pa.y, inv, sgn);
    wa.z = entry_weight(pa.z, inv, sgn);
    wa.w = entry_weight(pa.w, inv, sgn);
    wb.x = entry_weight(pb.x, inv, sgn);
    wb.y = entry_weight(pb.y, inv, sgn);
    wb.z = entry_weight(pb.z, inv, sgn);
    wb.w = entry_weight(pb.w, inv, sgn);
}

// a packed FP64 chunk, its eight words held as the bits of two double4
// (entries 0-3, 4-7), as 16-bit indices and weights
template <typename W4>
__device__ __forceinline__ void unpack_chunk64(const W4 &ra, const W4 &rb, double inv, int sgn, uint4 &id, W4 &wa,
                                               W4 &wb)
{
    const uint64_t e[8] = {static_cast<uint64_t>(__double_as_longlong(ra.x)),
                           static_cast<uint64_t>(__double_as_longlong(ra.y)),
                           static_cast<uint64_t>(__double_as_longlong(ra.z)),
                           static_cast<uint64_t>(__double_as_longlong(ra.w)),
                           static_cast<uint64_t>(__double_as_longlong(rb.x)),
                           static_cast<uint64_t>(__double_as_longlong(rb.y)),
                           static_cast<uint64_t>(__double_as_longlong(rb.z)),
                           static_cast<uint64_t>(__double_as_longlong(rb.w))};
    const unsigned i[8] = {static_cast<unsigned>(e[0]) & 0xfffu, static_cast<unsigned>(e[1]) & 0xfffu,
                           static_cast<unsigned>(e[2]) & 0xfffu, static_cast<unsigned>(e[3]) & 0xfffu,
                           static_cast<unsigned>(e[4]) & 0xfffu, static_cast<unsigned>(e[5]) & 0xfffu,
                           static_cast<unsigned>(e[6]) & 0xfffu, static_cast<unsigned>(e[7]) & 0xfffu};
    id = make_uint4(i[0] | (i[1] << 16), i[2] | (i[3] << 16), i[4] | (i[5] << 16), i[6] | (i[7] << 16));
    wa.x = entry_q64(e[0], sgn) * inv;
    wa.y = entry_q64(e[1], sgn) * inv;
    wa.z = entry_q64(e[2], sgn) * inv;
    wa.w = entry_q64(e[3], sgn) * inv;
    wb.x = entry_q64(e[4], sgn) * inv;
    wb.y = entry_q64(e[5], sgn) * inv;
    wb.z = entry_q64(e[6], sgn) * inv;
    wb.w = entry_q64(e[7], sgn) * inv;
}

// staged index U (0..7, a compile-time constant) of a loaded chunk
template <bool NARROW, int U>
__device__ __forceinline__ unsigned id_at(uint4 id)
{
    static_assert(U >= 0 && U < 8, "eight entries per chunk");
    if constexpr (NARROW) {
        constexpr int b = 12 * U, wd = b / 32, sh = b % 32;
        const unsigned lo = wd == 0 ? id.x : (wd == 1 ? id.y : id.z);
        if constexpr (sh <= 20) {
            return (lo >> sh) & 0xfffu;
        } else {
            const unsigned hi = wd == 0 ? id.y : id.z;
            return ((lo >> sh) | (hi << (32 - sh))) & 0xfffu;
        }
    } else {
        const unsigned wv = U < 2 ? id.x : (U < 4 ? id.y : (U < 6 ? id.z : id.w));
        return (U & 1) ? (wv >> 16) : (wv & 0xffffu);
    }
}


struct BuildArgs {
    Geo g;
    int64_t n, S;
    int ncell;
    const int *cstart, *sorted;
    const double4 *reld_src;  // positions relative to their own (build-time) cell, double
    const float4 *relf_src;   // the same rounded to float (FP32 refresh)
    const double4 *pos_s;     // wrapped positions (WCA force in FP64)
    double rc2;               // r_cut^2
    double rcs2;              // (r_cut + skin)^2: candidate lists
    int cap, capS;            // pair list / candidate list capacity
    uint4 *snl;               // candidate lists: uint16 chunks of 8 staged indices, blocked by
                              // cell (the cell at h0 holds [capS/8][occ][8] from chunk h0 capS/8)
    int *snn;                 // candidate counts
    int nst;                  // stencil entries per cell
    int stage_n;              // stencil positions the refresh stages in LDS
    const int *cell_id;       // cell of each particle (original order)
    const int *gate;          // rebuild flag
    const double *wtab;       // w(r) on the distance grid
    int n_r;
    double r0, dr, r_cut_min, lam_hi;
    double wca_rc2, wca_s2, wca_eps;
    uint16_t *nbl;
    void *nbw;
    int wpack, wq_signed;     // packed lists (narrow cells, isotropic) and the weight's form
    double wq_scale;          // weight -> fixed point (FP64 lists)
    float wq_scale32;         // the same for FP32 lists
    int *nn;
    int2 *stab;
    const int2 *stab_c;
    double *fc;               // WCA force, [3][S] original order
    unsigned *rowmax;
    int *flags;
    long long *flag_step;
    const long long *d_step;
};

// w(r): linear interpolation on the distance grid, frozen below r_cut_min.
// tab2[b] = (w_b, w_{b+1}) in the work precision (FP32 entries are the FP64
// ones rounded), staged in LDS: one read per weight
template <typename T>
__device__ __forceinline__ T weight_of(const BuildArgs &a, const typename V2<T>::t *tab2, T r)
{
    if (sizeof(T) == 8) {
        double rr = static_cast<double>(r);
        if (rr < a.r_cut_min) rr = a.r_cut_min;
        const double t = fmax((rr - a.r0) / a.dr, 0.0);
        const double tb = fmin(floor(t), static_cast<double>(a.n_r - 2));
        const int b = static_cast<int>(fmax(tb, 0.0));
        const double f = t - b;
        const typename V2<T>::t e = tab2[b];
        return static_cast<T>(static_cast<double>(e.x) * (1.0 - f) + static_cast<double>(e.y) * f);
    }
    const T rmin = static_cast<T>(a.r_cut_min);
    const T rr = r < rmin ? rmin : r;
    const T t = fmax((rr - static_cast<T>(a.r0)) * static_cast<T>(1.0 / a.dr), T(0));
    const T tb = fmin(floor(t), static_cast<T>(a.n_r - 2));
    const int b = static_cast<int>(fmax(tb, T(0)));
    const T f = t - static_cast<T>(b);
    const typename V2<T>::t e = tab2[b];
    return e.x + f * (e.y - e.x);
}

// ---------------------------------------------------------------------------
// Neighbour lists in two stages.
//
// Build (only when the rebuild flag is set): one work-group per cell, one lane
// per particle.  Candidates are staged in LDS in chunks (positions relative to
// the home cell, periodic images applied, as float or double).  The wave walks
// them in lockstep with broadcast reads and only tests the distance against
// r_c + skin, appending the staged index of each hit to the lane's queue in
// LDS; the queues are drained with every lane busy into the candidate list
// (8-index chunks, one 16-byte store each).
//
// Refresh (every step): one work-group per cell stages the current positions
// of the stencil; each lane walks its particle's candidate list and keeps the
// pairs within r_c: the pair list with weights (the lists above), the WCA
// force, and the row sum of |w| (a bound on the spectral norm of P, ||T_ij|| =
// 1 for both tensor forms) against the top of the noise interval.  The
// distance is formed exactly as in the build, so with skin 0 the two agree
// pair for pair.  The pair decision is taken in FP64 in the FP64 mode and in
// FP32 otherwise (a pair within rounding of r_c has w ~ 0 either way); the WCA
// force is FP64 from the wrapped positions.
// ---------------------------------------------------------------------------
constexpr int kQueue = 48;                     // queued hits per lane
constexpr int kCheckBlock = 16;                // candidates tested between queue checks
constexpr int kDrainAt = kQueue - kCheckBlock;  // a queue this long is drained

// one candidate chunk being filled: 8 staged indices of 16 bits
struct IdxChunk {
    uint32_t i0 = 0, i1 = 0, i2 = 0, i3 = 0;
    __device__ __forceinline__ void put(int pos, uint32_t l)
    {
        const int sh = (pos & 1) * 16;
        const uint32_t keep = ~(0xffffu << sh), v = l << sh;
        const int w = pos >> 1;
        i0 = w == 0 ? (i0 & keep) | v : i0;
        i1 = w == 1 ? (i1 & keep) | v : i1;
        i2 = w == 2 ? (i2 & keep) | v : i2;
        i3 = w == 3 ? (i3 & keep) | v : i3;
    }
    // dst: the cell's candidate lists, chunk c of its particle j at c occ + j
    __device__ __forceinline__ void store(uint4 *dst, int chunk, int j, int occ) const
    {
        dst[static_cast<int64_t>(chunk) * occ + j] = make_uint4(i0, i1, i2, i3);
    }
};

// squared distance from the home particle to the staged candidate li, in the
// precision of the pair decision (FP64 data in the FP64 mode, FP32 otherwise);
// MI: some axis has fewer than 3 cells, so the minimum image is taken there
template <typename T, bool EXACT64, bool MI>
__device__ __forceinline__ T staged_r2(const double4 *reld, const float4 *relf, int li, const double4 &xd,
                                       const float (&xf)[3], const Geo &g, const bool (&mi)[3], const float (&Lf)[3])
{
    if (EXACT64) {
        const double4 q = reld[li];
        double ux = xd.x - q.x, uy = xd.y - q.y, uz = xd.z - q.z;
        if (MI && mi[0]) ux -= g.L[0] * rint(ux / g.L[0]);
        if (MI && mi[1]) uy -= g.L[1] * rint(uy / g.L[1]);
        if (MI && mi[2]) uz -= g.L[2] * rint(uz / g.L[2]);
        return static_cast<T>(ux * ux + uy * uy + uz * uz);
    } else {
        const float4 q = relf[li];
        float ux = xf[0] - q.x, uy = xf[1] - q.y, uz = xf[2] - q.z;
        if (MI && mi[0]) ux -= Lf[0] * rintf(ux / Lf[0]);
        if (MI && mi[1]) uy -= Lf[1] * rintf(uy / Lf[1]);
        if (MI && mi[2]) uz -= Lf[2] * rintf(uz / Lf[2]);
        return static_cast<T>(ux * ux + uy * uy + uz * uz);
    }
}

template <typename T, bool EXACT64, bool MI>
__global__ __launch_bounds__(kPairThreads) void k_build(BuildArgs a)
{
    if (*a.gate == 0) return;
    constexpr int CH = EXACT64 ? kBuildChunk / 2 : kBuildChunk;
    __shared__ Stencil st;
    // staged candidates; entries past the end of the stencil hold NaN
    // positions, which never pass the distance test
    __shared__ float4 relf[EXACT64 ? 1 : CH + 4];
    __shared__ double4 reld[EXACT64 ? CH + 4 : 1];
    __shared__ uint16_t queue[kQueue][kPairThreads];
    const int cid = blockIdx.x;
    const int tid = threadIdx.x;
    const double qnan = __builtin_nan("");
    if (tid < 4) {
        if (EXACT64) reld[CH + tid] = make_double4(qnan, qnan, qnan, 0.0);
        else relf[CH + tid] = make_float4(qnan, qnan, qnan, 0.f);
    }
    if (tid == 0) {
        make_stencil(a.g, a.cstart, cid, st);
        int2 *row = a.stab + static_cast<int64_t>(cid) * kStab;
        for (int k = 0; k < st.n; ++k) row[k] = make_int2(st.start[k], st.base[k]);
        row[st.n] = make_int2(0, st.base[st.n]);
    }
    __syncthreads();
    const int h0 = a.cstart[cid], h1 = a.cstart[cid + 1];
    uint4 *cl = a.snl + static_cast<int64_t>(h0) * (a.capS >> 3);  // this cell's candidate lists
    const int total = st.base[st.n];
    const bool store = total < 65536;  // staged indices and the end marker fit 16 bits
    const float Lf[3] = {static_cast<float>(a.g.L[0]), static_cast<float>(a.g.L[1]), static_cast<float>(a.g.L[2])};
    const bool mi[3] = {a.g.nc[0] < 3, a.g.nc[1] < 3, a.g.nc[2] < 3};
    const T rcs2 = static_cast<T>(a.rcs2);
    for (int g0 = h0; g0 < h1; g0 += kPairThreads) {
        const int s = g0 + tid;
        const bool live = s < h1;
        const int self_l = st.base[st.home] + (s - h0);
        const double4 xd = live ? a.reld_src[s] : make_double4(0, 0, 0, 0);
        const float xf[3] = {static_cast<float>(xd.x), static_cast<float>(xd.y), static_cast<float>(xd.z)};
        int cnt = 0, nq = 0;
        IdxChunk ck;
        for (int c0 = 0; c0 < total; c0 += CH) {
            const int c1 = min(total, c0 + CH);
            __syncthreads();
            constexpr int per = CH / kPairThreads;
            double4 v[per];
            int sj[per];
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int l = c0 + tid + j * kPairThreads;
                if (l < c1) {
                    const int t = stencil_entry(st, l);
                    sj[j] = st.start[t] + (l - st.base[t]);
                    v[j] = a.reld_src[sj[j]];
                    if (EXACT64) {
                        v[j].x += st.offd[t][0];
                        v[j].y += st.offd[t][1];
                        v[j].z += st.offd[t][2];
                    } else {
                        // position and image offset each rounded, then added
                        v[j].x = static_cast<float>(v[j].x) + st.offf[t][0];
                        v[j].y = static_cast<float>(v[j].y) + st.offf[t][1];
                        v[j].z = static_cast<float>(v[j].z) + st.offf[t][2];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < per; ++j) {
                const int l = tid + j * kPairThreads;
                if (c0 + l < c1) {
                    if (EXACT64) reld[l] = v[j];
                    else
                        relf[l] = make_float4(static_cast<float>(v[j].x), static_cast<float>(v[j].y),
                                              static_cast<float>(v[j].z), 0.f);
                } else if (EXACT64) {
                    reld[l] = make_double4(qnan, qnan, qnan, 0.0);
                } else {
                    relf[l] = make_float4(qnan, qnan, qnan, 0.f);
                }
            }
            __syncthreads();
            if (!live) continue;
            // lockstep distance test, four broadcast candidates per round,
            // appended without branches (a miss writes the next free slot and
            // does not advance); a queue is drained once one in the wave could
            // overflow in the next block, and at the end of the staged chunk.
            // Blocks start at multiples of 4 from c0, so a round only runs
            // past c1 into the NaN padding.
            const int self_li = self_l - c0;
            for (int b0 = c0;; b0 += kCheckBlock) {
                const int b1 = min(c1, b0 + kCheckBlock);
                for (int l0 = b0 - c0; l0 < b1 - c0; l0 += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int li = l0 + u;
                        const T r2 = staged_r2<T, EXACT64, MI>(reld, relf, li, xd, xf, a.g, mi, Lf);
                        const bool hit = r2 < rcs2 && li != self_li;
                        queue[nq][tid] = static_cast<uint16_t>(li);
                        nq += hit ? 1 : 0;
                    }
                }
                const bool last = b1 >= c1;
                if (last || __any(nq >= kDrainAt)) {
                    for (int e = 0; e < nq; ++e) {
                        if (store && cnt < a.capS) {
                            const int pos = cnt & 7;
                            ck.put(pos, static_cast<uint32_t>(c0 + queue[e][tid]));
                            if (pos == 7) ck.store(cl, cnt >> 3, s - h0, h1 - h0);
                        }
                        ++cnt;
                    }
                    nq = 0;
                }
                if (last) break;
            }
        }
        if (live) {
            const int kept = store ? min(cnt, a.capS) : 0;
            if (kept & 7) {
                // pad the last chunk with the end marker (index total: no
                // candidate)
                for (int pos = kept & 7; pos < 8; ++pos) ck.put(pos, static_cast<uint32_t>(total));
                ck.store(cl, kept >> 3, s - h0, h1 - h0);
            }
            if (cnt > a.capS || !store) latch(a.flags, a.flag_step, GLD_ERR_CAPACITY, *a.d_step);
            a.snn[s] = kept;
        }
    }
}

// Refresh, one work-group per cell (the cell order and stencils of the last
// build).  The current positions of the stencil's particles are staged in LDS
// with the image offset of their stencil entry, formed as in the build (FP32:
// position and offset each rounded, then added; FP64 exact), up to stage_n of
// them; a candidate past those is read from global memory.  Four lanes serve
// one particle: in round k lane q takes the k-th group of kPerLane candidates
// of its share (FP32: chunk 4k + q of 8 entries; FP64: half chunks of 4, which
// keeps the ring below small) and tests them against r_c.  The hits of a round
// get consecutive list positions in candidate order (a prefix sum over the
// quad), pass through a ring of kRing entries per particle in LDS and leave as
// whole 8-entry chunks, one per lane.  The pair list is thus the candidate
// list filtered in order, and with skin 0 the list a build at r_c would make.
// (The ring is written and read by the lanes of one wave, whose LDS accesses
// complete in issue order.)
constexpr int kRefreshThreads = 256;
constexpr int kRefreshGroup = kRefreshThreads / 4;  // particles per round of a work-group
constexpr size_t kRefreshLds = 80 * 1024;           // per work-group: two per CU
constexpr size_t kRefreshLds64 = 150 * 1024;        // FP64: one per CU

template <typename T>
struct RefreshShape;
template <>
struct RefreshShape<float> {
    static constexpr int kPerLane = 8;  // candidates per lane and round
    static constexpr int kRing = 64;    // ring entries per particle, >= 7 + 4 kPerLane
};
template <>
struct RefreshShape<double> {
    static constexpr int kPerLane = 4;
    static constexpr int kRing = 32;
};

// ring rows: 16-byte aligned, consecutive particles on different LDS banks
template <typename T>
constexpr int ring_idx_stride() { return RefreshShape<T>::kRing + 8; }
template <typename T>
constexpr int ring_w_stride() { return RefreshShape<T>::kRing + 4; }

// LDS of the refresh besides the staged positions (bytes, with slack)
template <typename T>
constexpr size_t refresh_fixed_lds()
{
    return 2 * sizeof(T) * GLD_MAX_DISTANCE_BINS + sizeof(uint16_t) * kRefreshGroup * ring_idx_stride<T>() +
           sizeof(T) * kRefreshGroup * ring_w_stride<T>() + sizeof(int) * 2 * kStab + sizeof(T) * 3 * kMaxStencil + 512;
}

// whole-chunk reads of the ring, which is written entry by entry: these
// types may alias the entries' types, so the compiler keeps the reads after
// the writes
typedef uint4 __attribute__((__may_alias__)) uint4_ring;
typedef float4 __attribute__((__may_alias__)) float4_ring;
typedef double4 __attribute__((__may_alias__)) double4_ring;
template <typename T>
struct RingV4;
template <>
struct RingV4<float> {
    using t = float4_ring;
};
template <>
struct RingV4<double> {
    using t = double4_ring;
};

// stencil entry holding staged index l (sb ascending over nst entries)
__device__ __forceinline__ int entry_of(const int *sb, int nst, int l)
{
    int lo = 0, hi = nst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sb[mid] <= l) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// current position of staged candidate l (stencil entry e) relative to the
// home cell, in the precision of the pair decision
template <typename T, bool EXACT64>
__device__ __forceinline__ typename V4<T>::t stencil_pos(const BuildArgs &a, const int *sst, const int *sb,
                                                         const T (*off)[3], int l, int e)
{
    const int t = sst[e] + (l - sb[e]);
    typename V4<T>::t p;
    if (EXACT64) {
        const double4 v = a.reld_src[t];
        p.x = static_cast<T>(v.x + static_cast<double>(off[e][0]));
        p.y = static_cast<T>(v.y + static_cast<double>(off[e][1]));
        p.z = static_cast<T>(v.z + static_cast<double>(off[e][2]));
    } else {
        const float4 v = a.relf_src[t];
        p.x = static_cast<T>(v.x + static_cast<float>(off[e][0]));
        p.y = static_cast<T>(v.y + static_cast<float>(off[e][1]));
        p.z = static_cast<T>(v.z + static_cast<float>(off[e][2]));
    }
    p.w = T(0);
    return p;
}

// the candidate indices of lane q in round k: kPerLane 16-bit entries in
// kPerLane/2 words; past the list, the end marker
template <typename T>
__device__ __forceinline__ void load_candidates(const uint4 *cl, int j, int occ, int k, int q, int nch, uint32_t fill,
                                                uint32_t (&w)[RefreshShape<T>::kPerLane / 2])
{
    if constexpr (RefreshShape<T>::kPerLane == 8) {
        const int c = 4 * k + q;
        uint4 v = make_uint4(fill, fill, fill, fill);
        if (c < nch) v = stream_load(&cl[static_cast<int64_t>(c) * occ + j]);
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    } else {
        const int h = 4 * k + q, c = h >> 1;
        uint2 v = make_uint2(fill, fill);
        if (c < nch) v = reinterpret_cast<const uint2 *>(cl)[(static_cast<int64_t>(c) * occ + j) * 2 + (h & 1)];
        w[0] = v.x;
        w[1] = v.y;
    }
}

// entry u (not a compile-time constant) of a lane's candidate words, by
// shifts of 64-bit halves (an indexed read would place the words in scratch)
template <int NW>
__device__ __forceinline__ int cand_at(const uint32_t (&w)[NW], int u)
{
    static_assert(NW == 2 || NW == 4, "two or four candidate words");
    const uint64_t lo = (static_cast<uint64_t>(w[1]) << 32) | w[0];
    uint64_t x = lo;
    if constexpr (NW == 4) {
        const uint64_t hi = (static_cast<uint64_t>(w[3]) << 32) | w[2];
        x = u < 4 ? lo : hi;
    }
    return static_cast<int>((x >> ((u & 3) * 16)) & 0xffffu);
}

// exclusive prefix sum of c over the four lanes of a quad (DPP quad
// permutes: lane q reads lane q-1, then lane q-2), and the quad's total
__device__ __forceinline__ int quad_scan(int c, int q, int &tot)
{
    int inc = c;
    int t = __builtin_amdgcn_update_dpp(0, inc, 0x90, 0xf, 0xf, false);  // quad_perm [0,0,1,2]
    inc += q >= 1 ? t : 0;
    t = __builtin_amdgcn_update_dpp(0, inc, 0x40, 0xf, 0xf, false);  // quad_perm [0,0,0,1]
    inc += q >= 2 ? t : 0;
    tot = __builtin_amdgcn_update_dpp(0, inc, 0xff, 0xf, 0xf, false);  // quad_perm [3,3,3,3]
    return inc - c;
}

template <typename T, bool EXACT64, bool PAR, bool MI>
__global__ __launch_bounds__(kRefreshThreads) void k_refresh(BuildArgs a)
{
    using T4 = typename V4<T>::t;
    using RV4 = typename RingV4<T>::t;
    constexpr int PL = RefreshShape<T>::kPerLane, RING = RefreshShape<T>::kRing;
    constexpr int RI = ring_idx_stride<T>(), RW = ring_w_stride<T>();
    extern __shared__ __align__(32) unsigned char rf_lds[];
    T4 *pos = reinterpret_cast<T4 *>(rf_lds);
    using T2 = typename V2<T>::t;
    __shared__ T2 tab2[GLD_MAX_DISTANCE_BINS];
    __shared__ __align__(16) uint16_t ring_i[kRefreshGroup * RI];
    __shared__ __align__(32) T ring_w[kRefreshGroup * RW];
    __shared__ int sst[kStab], sb[kStab];
    __shared__ T off[kMaxStencil][3];
    __shared__ unsigned blk_max;
    const int cid = blockIdx.x;
    const int h0 = a.cstart[cid], occ = a.cstart[cid + 1] - h0;
    if (occ <= 0) return;  // the whole work-group
    const int tid = threadIdx.x;
    const int nst = a.nst;
    for (int b = tid; b < a.n_r; b += kRefreshThreads) {
        T2 e;
        e.x = static_cast<T>(a.wtab[b]);
        e.y = static_cast<T>(a.wtab[min(b + 1, a.n_r - 1)]);
        tab2[b] = e;
    }
    if (tid <= nst) {
        const int2 e = a.stab_c[static_cast<int64_t>(cid) * kStab + tid];
        sst[tid] = e.x;
        sb[tid] = e.y;
    }
    if (tid < nst) {
        const int e0 = tid % a.g.noff[0], e1 = (tid / a.g.noff[0]) % a.g.noff[1];
        const int e2 = tid / (a.g.noff[0] * a.g.noff[1]);
        off[tid][0] = static_cast<T>(a.g.offs[0][e0] * a.g.edge[0]);
        off[tid][1] = static_cast<T>(a.g.offs[1][e1] * a.g.edge[1]);
        off[tid][2] = static_cast<T>(a.g.offs[2][e2] * a.g.edge[2]);
    }
    if (tid == 0) blk_max = 0u;
    __syncthreads();
    const int total = sb[nst];
    const int nstage = min(total, a.stage_n);
    // (one slot past the staged ones is read for candidates that are not
    // staged, and for the end marker)
    {
        // four positions per thread at a time: their searches and loads in
        // flight together, then the stores
        int l = tid;
        for (; l + 3 * kRefreshThreads < nstage; l += 4 * kRefreshThreads) {
            int e[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) e[u] = entry_of(sb, nst, l + u * kRefreshThreads);
            T4 p[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] = stencil_pos<T, EXACT64>(a, sst, sb, off, l + u * kRefreshThreads, e[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) pos[l + u * kRefreshThreads] = p[u];
        }
        for (; l < nstage; l += kRefreshThreads) pos[l] = stencil_pos<T, EXACT64>(a, sst, sb, off, l, entry_of(sb, nst, l));
    }
    if (tid == 0) pos[nstage] = T4{};
    __syncthreads();

    const int pl = tid >> 2, q = tid & 3;  // particle of the round, lane of the quad
    const T rc2 = static_cast<T>(a.rc2);
    const T wca_pre = static_cast<T>(a.wca_rc2 * 1.0001);
    const T Lw[3] = {static_cast<T>(a.g.L[0]), static_cast<T>(a.g.L[1]), static_cast<T>(a.g.L[2])};
    const bool mi[3] = {a.g.nc[0] < 3, a.g.nc[1] < 3, a.g.nc[2] < 3};
    const int capc = a.cap >> 3;
    const uint32_t fill = static_cast<uint32_t>(total) * 0x10001u;
    // the home cell is the stencil entry with zero offset on each axis
    const int home = ((a.g.noff[2] == 3 ? 1 : 0) * a.g.noff[1] + (a.g.noff[1] == 3 ? 1 : 0)) * a.g.noff[0] +
                     (a.g.noff[0] == 3 ? 1 : 0);
    uint16_t *ri = ring_i + pl * RI;
    T *rw = ring_w + pl * RW;
    // this cell's lists (cell-blocked: chunk c of the cell's particle j at
    // c occ + j, weight rows likewise)
    uint4 *nbl4 = reinterpret_cast<uint4 *>(a.nbl) + static_cast<int64_t>(h0) * capc;
    uint3 *nbl3 = reinterpret_cast<uint3 *>(nbl4);  // the same cell start, narrow form
    const bool narrow = total <= kNarrowStencil;
    const uint4 *cl = a.snl + static_cast<int64_t>(h0) * (a.capS >> 3);  // candidate lists, likewise
    T4 *nbw4 = static_cast<T4 *>(a.nbw) + static_cast<int64_t>(h0) * 2 * capc;
    uint4 *nbp4 = reinterpret_cast<uint4 *>(nbw4);  // packed chunks: two words of four entries
    const bool packed = !PAR && a.wpack && narrow;
    // chunk c of the cell's particle jj from the ring at base: indices and
    // weights, or the packed words
    auto put_chunk = [&](int c, int jj, int base) __attribute__((always_inline)) {
        const uint4 idv = *reinterpret_cast<const uint4_ring *>(ri + base);
        const RV4 w0 = *reinterpret_cast<const RV4 *>(rw + base), w1 = *reinterpret_cast<const RV4 *>(rw + base + 4);
        if constexpr (sizeof(T) == 8) {
            if (packed) {
                // eight 64-bit words in the weights' two double4 slots
                const double sc = a.wq_scale;
                const int sg = a.wq_signed;
                const unsigned ix[8] = {idv.x & 0xffffu, idv.x >> 16, idv.y & 0xffffu, idv.y >> 16,
                                        idv.z & 0xffffu, idv.z >> 16, idv.w & 0xffffu, idv.w >> 16};
                const double wv8[8] = {static_cast<double>(w0.x), static_cast<double>(w0.y), static_cast<double>(w0.z),
                                       static_cast<double>(w0.w), static_cast<double>(w1.x), static_cast<double>(w1.y),
                                       static_cast<double>(w1.z), static_cast<double>(w1.w)};
                T4 o0, o1;
                o0.x = __longlong_as_double(pack_entry64(ix[0], wv8[0], sc, sg));
                o0.y = __longlong_as_double(pack_entry64(ix[1], wv8[1], sc, sg));
                o0.z = __longlong_as_double(pack_entry64(ix[2], wv8[2], sc, sg));
                o0.w = __longlong_as_double(pack_entry64(ix[3], wv8[3], sc, sg));
                o1.x = __longlong_as_double(pack_entry64(ix[4], wv8[4], sc, sg));
                o1.y = __longlong_as_double(pack_entry64(ix[5], wv8[5], sc, sg));
                o1.z = __longlong_as_double(pack_entry64(ix[6], wv8[6], sc, sg));
                o1.w = __longlong_as_double(pack_entry64(ix[7], wv8[7], sc, sg));
                nbw4[(2 * c) * occ + jj] = o0;
                nbw4[(2 * c + 1) * occ + jj] = o1;
                return;
            }
        } else if (packed) {
            const float sc = a.wq_scale32;
            const int sg = a.wq_signed;
            nbp4[(2 * c) * occ + jj] = make_uint4(
                pack_entry(idv.x & 0xffffu, static_cast<float>(w0.x), sc, sg),
                pack_entry(idv.x >> 16, static_cast<float>(w0.y), sc, sg),
                pack_entry(idv.y & 0xffffu, static_cast<float>(w0.z), sc, sg),
                pack_entry(idv.y >> 16, static_cast<float>(w0.w), sc, sg));
            nbp4[(2 * c + 1) * occ + jj] = make_uint4(
                pack_entry(idv.z & 0xffffu, static_cast<float>(w1.x), sc, sg),
                pack_entry(idv.z >> 16, static_cast<float>(w1.y), sc, sg),
                pack_entry(idv.w & 0xffffu, static_cast<float>(w1.z), sc, sg),
                pack_entry(idv.w >> 16, static_cast<float>(w1.w), sc, sg));
            return;
        }
        if (narrow) nbl3[c * occ + jj] = ids_pack12(idv);
        else nbl4[c * occ + jj] = idv;
        nbw4[(2 * c) * occ + jj] = w0;
        nbw4[(2 * c + 1) * occ + jj] = w1;
    };
    for (int g0 = 0; g0 < occ; g0 += kRefreshGroup) {
        const bool live = g0 + pl < occ;
        const int64_t s = h0 + g0 + pl;
        T ox = 0, oy = 0, oz = 0;
        int ns = 0;
        if (live) {
            if (EXACT64) {
                const double4 v = a.reld_src[s];
                ox = static_cast<T>(v.x);
                oy = static_cast<T>(v.y);
                oz = static_cast<T>(v.z);
            } else {
                const float4 v = a.relf_src[s];
                ox = static_cast<T>(v.x);
                oy = static_cast<T>(v.y);
                oz = static_cast<T>(v.z);
            }
            ns = a.snn[s];
        }
        const int nch = (ns + 7) >> 3;
        const int nround = (ns + 4 * PL - 1) / (4 * PL);
        int cnt = 0;  // pairs so far (the same in the four lanes)
        T rowsum = 0;  // a bound checked with ample margin: work precision suffices
        double fx = 0, fy = 0, fz = 0;
        // pairs within the WCA range wait in a queue of four (16-bit staged
        // indices) and are evaluated together, in the order found, so that
        // their position loads are in flight at once
        uint32_t wq0 = 0, wq1 = 0;
        int wn = 0;
        const double4 xi = live ? a.pos_s[s] : make_double4(0, 0, 0, 0);
        auto wca_flush = [&]() __attribute__((always_inline)) {
            int sj[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int l = static_cast<int>(((k < 2 ? wq0 : wq1) >> ((k & 1) * 16)) & 0xffffu);
                const int e = entry_of(sb, nst, l);
                sj[k] = sst[e] + (l - sb[e]);
            }
            double4 xj[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < wn) xj[k] = a.pos_s[sj[k]];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= wn) break;
                // conservative WCA force in FP64 from the wrapped positions
                double gx = xi.x - xj[k].x, gy = xi.y - xj[k].y, gz = xi.z - xj[k].z;
                gx -= a.g.L[0] * rint(gx / a.g.L[0]);
                gy -= a.g.L[1] * rint(gy / a.g.L[1]);
                gz -= a.g.L[2] * rint(gz / a.g.L[2]);
                const double rd2 = gx * gx + gy * gy + gz * gz;
                if (rd2 < a.wca_rc2) {
                    const double s2 = a.wca_s2 / rd2, s6 = s2 * s2 * s2;
                    const double fr = 24.0 * a.wca_eps * (2.0 * s6 * s6 - s6) / rd2;
                    fx += fr * gx;
                    fy += fr * gy;
                    fz += fr * gz;
                }
            }
            wn = 0;
            wq0 = wq1 = 0;
        };
        uint32_t nxt[PL / 2];
        load_candidates<T>(cl, g0 + pl, occ, 0, q, nch, fill, nxt);
        for (int k = 0; k < nround; ++k) {
            uint32_t cur[PL / 2];
#pragma unroll
            for (int u = 0; u < PL / 2; ++u) cur[u] = nxt[u];
            if (k + 1 < nround) load_candidates<T>(cl, g0 + pl, occ, k + 1, q, nch, fill, nxt);
            // the round runs in phases of straight-line code (positions,
            // distances, weights, ring writes), so that the LDS reads of its
            // candidates are in flight together
            int lv[PL];
            T4 pv[PL];
            unsigned gmask = 0;  // candidates past the staged part of the stencil
#pragma unroll
            for (int u = 0; u < PL; ++u) {
                const int l = static_cast<int>((cur[u >> 1] >> ((u & 1) * 16)) & 0xffffu);
                lv[u] = l;
                pv[u] = pos[min(l, nstage)];
                gmask |= (l >= nstage && l < total) ? (1u << u) : 0u;
            }
            if (gmask) {
#pragma unroll
                for (int u = 0; u < PL; ++u)
                    if ((gmask >> u) & 1u)
                        pv[u] = stencil_pos<T, EXACT64>(a, sst, sb, off, lv[u], entry_of(sb, nst, lv[u]));
            }
            T r2v[PL];
            unsigned mask = 0;
#pragma unroll
            for (int u = 0; u < PL; ++u) {
                T ux = ox - pv[u].x, uy = oy - pv[u].y, uz = oz - pv[u].z;
                if (MI && mi[0]) ux -= Lw[0] * rint(ux / Lw[0]);
                if (MI && mi[1]) uy -= Lw[1] * rint(uy / Lw[1]);
                if (MI && mi[2]) uz -= Lw[2] * rint(uz / Lw[2]);
                const T r2 = ux * ux + uy * uy + uz * uz;
                r2v[u] = r2;
                mask |= (lv[u] < total && r2 < rc2) ? (1u << u) : 0u;
            }
            // list positions of this lane's hits: after those of the lanes
            // before it in the quad
            int tot;
            int at = cnt + quad_scan(__popc(mask), q, tot);
            // every candidate is weighed and written: a hit to its ring slot,
            // a miss to the lane's spare slot past the ring (FP32: hardware
            // square root, within one ulp)
            T wv[PL];
#pragma unroll
            for (int u = 0; u < PL; ++u) {
                const T r = sizeof(T) == 4 ? static_cast<T>(__builtin_amdgcn_sqrtf(static_cast<float>(r2v[u])))
                                           : sqrt(r2v[u]);
                wv[u] = weight_of<T>(a, tab2, r);
            }
            unsigned wmask = 0;  // hits within the WCA range
#pragma unroll
            for (int u = 0; u < PL; ++u) {
                const bool h = (mask >> u) & 1u;
                rowsum += h ? fabs(wv[u]) : T(0);
                const int slot = h ? (at & (RING - 1)) : RING + q;
                ri[slot] = static_cast<uint16_t>(lv[u]);
                rw[slot] = PAR ? wv[u] / r2v[u] : wv[u];
                at += h ? 1 : 0;
                wmask |= (h && r2v[u] < wca_pre) ? (1u << u) : 0u;
            }
            while (wmask) {
                const uint32_t l = static_cast<uint32_t>(cand_at(cur, __ffs(wmask) - 1));
                wmask &= wmask - 1;
                if (wn == 4) wca_flush();
                const int sh = (wn & 1) * 16;
                if (wn < 2) wq0 |= l << sh;
                else wq1 |= l << sh;
                ++wn;
            }
            // chunks completed this round, one per lane
            const int cnt1 = cnt + tot;
            const int fc = (cnt >> 3) + q;
            if (fc < (cnt1 >> 3) && fc < capc) put_chunk(fc, g0 + pl, (fc * 8) & (RING - 1));
            cnt = cnt1;
        }
        if (wn > 0) wca_flush();
        // quad sums (WCA force components in the order of the lanes' entries)
        for (int o = 1; o < 4; o <<= 1) {
            rowsum += __shfl_xor(rowsum, o);
            fx += __shfl_xor(fx, o);
            fy += __shfl_xor(fy, o);
            fz += __shfl_xor(fz, o);
        }
        if (live && q == 0) {
            const int kept = min(cnt, a.cap);
            if (kept & 7) {
                // pad the last chunk: zero weight, the particle itself
                const uint16_t self_l = static_cast<uint16_t>(sb[home] + (static_cast<int>(s) - sst[home]));
                for (int p = kept; p < ((kept + 7) & ~7); ++p) {
                    ri[p & (RING - 1)] = self_l;
                    rw[p & (RING - 1)] = T(0);
                }
                const int fl = kept >> 3;
                put_chunk(fl, g0 + pl, (fl * 8) & (RING - 1));
            }
            if (cnt > a.cap) latch(a.flags, a.flag_step, GLD_ERR_CAPACITY, *a.d_step);
            a.nn[s] = kept;
            const int p = a.sorted[s];
            a.fc[p] = fx;
            a.fc[a.S + p] = fy;
            a.fc[2 * a.S + p] = fz;
            if (static_cast<double>(rowsum) > a.lam_hi) latch(a.flags, a.flag_step, GLD_ERR_INTERVAL, *a.d_step);
            // row sums are >= 0, so their float bits order as unsigned
            // integers; one global atomic per work-group
            atomicMax(&blk_max, __float_as_uint(static_cast<float>(rowsum)));
        }
    }
    __syncthreads();
    if (tid == 0) atomicMax(a.rowmax, blk_max);
}

// ---------------------------------------------------------------------------
// sorted copies of the inputs of the pair mat-vecs:
//   ys[s]    = Y[p]                       (dissipative input)
//   us[q][s] = U[step % block][q][p]      (filter outputs of this step, in the
//                                          buffer of its block's parity)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_permute(int64_t n, int64_t S, const int *__restrict__ sorted, const T *__restrict__ Y,
                          typename V4<T>::t *__restrict__ ys, const T *__restrict__ U, int r, int rcap, int block,
                          int urows, const long long *__restrict__ d_step, typename V4<T>::t *__restrict__ us)
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
        const long long cur = *d_step;
        const int bi = static_cast<int>(cur % block);
        const T *u = U + ((cur / block) & 1) * urows * 3 * S + static_cast<int64_t>(bi) * rcap * 3 * S;
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
// pair mat-vec with fused combination, one work-group per cell:
//   out_s = a (P x)_s + b x_s + cz z_s + sum_q coef[q] us_q,s   (+ add[p])
// x is staged in LDS for the whole stencil (for the parallel tensor with the
// positions relative to the home cell, built exactly as in the neighbour
// build); L lanes per particle walk its chunks sub, sub + L, ... with the
// next chunk's loads in flight, and the L partial sums meet in LDS.  A
// stencil larger than the staging capacity is done in rounds, each lane
// taking the entries that fall into the staged range (the entries of a list
// ascend, so the summation order is the same).  x, z, us are sorted T4; out
// is sorted T4 or scattered to the original order [3][S] (out_orig),
// optionally plus add_orig[p].
// ---------------------------------------------------------------------------
// One term of the Chebyshev chain as the plan of the step sets it: the
// combination out = a P x + b x + cz z + sum_q B[row][q] u_q, or nothing
// (skip) for the terms beyond the chosen plan's K
struct ChainStep {
    double a, b, cz;
    int row;             // row of the mixing table (the tight plan's rows follow the wide plan's)
    unsigned char skip;  // a term beyond the plan's K
    unsigned char dual;  // the plan's first term that streams the pair lists (k = K - 2)
};
static_assert(sizeof(ChainStep) == 32, "the chain's device table holds 32 bytes per term");

struct MvArgs {
    int64_t n, S;
    const int *sorted, *cstart;
    const int2 *stab;
    int nst;    // stencil entries per cell
    int maxc;   // staged candidates per round
    int cap8;   // list chunks per particle (cap / 8)
    const uint4 *nbl;
    const void *nbw;
    int wpack, wq_signed;  // packed lists in the narrow cells (isotropic); signed weights
    double wq_inv;         // fixed point -> weight (FP64 lists)
    float wq_inv32;        // the same for FP32 lists
    const int *nn;
    const double4 *reld;  // parallel tensor: positions relative to their own cell
    Geo g;
    double a, b, cz;
    const void *x, *z, *coef, *us, *add_orig;
    int r;
    void *out_sorted, *out_orig;
    int rev;  // cells in descending order
    // a term of the Chebyshev chain whose plan is chosen on the device:
    // chain[cheb_k] holds a, b, cz and the row of coef (the mixing table,
    // rcap per row); null for every other mat-vec
    const ChainStep *chain;
    int cheb_k, rcap;
    int premix;  // us holds the term's v_k (coefficient 1, r = 1)
    // k_mvw's dual form: the second product -P y2 + dneg2 (y2 sorted T4),
    // scattered to fd2 ([3][S], original order)
    const void *y2, *dneg2;
    void *fd2;
};

// The staged input vector: for the isotropic mat-vec three planes x[], y[],
// z[] of stride maxc (3 values per candidate instead of 4: at N = 2e5, rho = 0.5 four FP32
// or two FP64 work-groups fit in a CU's LDS); for the parallel tensor
// (x, y, z, own x) per candidate
template <typename T, bool PAR>
constexpr bool mv_soa()
{
    return !PAR;
}

// FP32: x and y interleaved as (x, y) pairs in the first two planes' space
// (one 8-byte LDS read per staged entry instead of two; measured at N = 2e5,
// rho = 0.5: 52.5 -> 50.1 us per mat-vec; FP64 gained nothing from it)
template <typename T>
constexpr bool mv_xy()
{
    return sizeof(T) == 4;
}

constexpr int kStageDepth = 4;  // staged entries a thread of the mat-vec has in flight

template <typename T, bool SOA>
struct StageView {
    const typename V4<T>::t *aos;
    const T *soa;
    unsigned stride;
    __device__ __forceinline__ typename V4<T>::t get(unsigned l) const
    {
        if constexpr (SOA) {
            typename V4<T>::t v;
            if constexpr (mv_xy<T>()) {
                const typename V2<T>::t xy = reinterpret_cast<const typename V2<T>::t *>(soa)[l];
                v.x = xy.x;
                v.y = xy.y;
            } else {
                v.x = soa[l];
                v.y = soa[stride + l];
            }
            v.z = soa[2 * stride + l];
            v.w = T(0);
            return v;
        } else {
            return aos[l];
        }
    }
};

// LDS bytes of one work-group (the staging area is reused for the partial
// sums of BS lanes)
template <typename T, bool PAR, int BS>
constexpr size_t mv_lds_bytes(int maxc)
{
    using T4 = typename V4<T>::t;
    using T2 = typename V2<T>::t;
    const size_t stage = mv_soa<T, PAR>() ? static_cast<size_t>(maxc) * 3 * sizeof(T)
                                          : static_cast<size_t>(maxc) * sizeof(T4);
    const size_t part = static_cast<size_t>(BS) * sizeof(T4);
    return (stage > part ? stage : part) + (PAR ? static_cast<size_t>(maxc) * sizeof(T2) : 0);
}

// one chunk of 8 entries; CHECK: only entries with staged index in [c0, c0 + cn)
template <typename T, bool PAR, bool CHECK, bool MI, bool SOA, bool NARROW>
__device__ __forceinline__ void mv_chunk(const StageView<T, SOA> &xs, const typename V2<T>::t *pyz, uint4 id,
                                         const typename V4<T>::t &wa, const typename V4<T>::t &wb, const T (&own)[3],
                                         const T (&Lb)[3], const bool (&mi)[3], unsigned c0, unsigned cn, T &p0, T &p1,
                                         T &p2)
{
    using T4 = typename V4<T>::t;
    const unsigned li[8] = {id_at<NARROW, 0>(id), id_at<NARROW, 1>(id), id_at<NARROW, 2>(id),
                            id_at<NARROW, 3>(id), id_at<NARROW, 4>(id), id_at<NARROW, 5>(id),
                            id_at<NARROW, 6>(id), id_at<NARROW, 7>(id)};
    const T w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
    if constexpr (!CHECK && SOA && !PAR && !mv_xy<T>()) {
        // one plane at a time: eight staged values live instead of 24
        T acc[3] = {p0, p1, p2};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = xs.soa[q * xs.stride + li[u]];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[q] += w[u] * v[u];
        }
        p0 = acc[0];
        p1 = acc[1];
        p2 = acc[2];
    } else if constexpr (!CHECK && SOA && !PAR) {
        // (x, y) pairs four entries at a time, then the z plane: eight
        // staged values live (the FP32 kernel then needs 64 registers:
        // eight waves per SIMD), two LDS reads per entry instead of three;
        // each component's sum takes the entries in order
        using T2 = typename V2<T>::t;
        const T2 *xy = reinterpret_cast<const T2 *>(xs.soa);
#pragma unroll
        for (int h = 0; h < 8; h += 4) {
            T2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = xy[li[h + u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                p0 += w[h + u] * v[u].x;
                p1 += w[h + u] * v[u].y;
            }
        }
        T vz[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vz[u] = xs.soa[2 * xs.stride + li[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) p2 += w[u] * vz[u];
    } else if (!CHECK) {
        T4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = xs.get(li[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (PAR) {
                const typename V2<T>::t q = pyz[li[u]];
                T dx = own[0] - v[u].w, dy = own[1] - q.x, dz = own[2] - q.y;
                if (MI && mi[0]) dx -= Lb[0] * rint(dx / Lb[0]);
                if (MI && mi[1]) dy -= Lb[1] * rint(dy / Lb[1]);
                if (MI && mi[2]) dz -= Lb[2] * rint(dz / Lb[2]);
                const T sc = w[u] * (dx * v[u].x + dy * v[u].y + dz * v[u].z);
                p0 += sc * dx;
                p1 += sc * dy;
                p2 += sc * dz;
            } else {
                p0 += w[u] * v[u].x;
                p1 += w[u] * v[u].y;
                p2 += w[u] * v[u].z;
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned l = li[u] - c0;
            if (l >= cn) continue;
            const T4 v = xs.get(l);
            if (PAR) {
                const typename V2<T>::t q = pyz[l];
                T dx = own[0] - v.w, dy = own[1] - q.x, dz = own[2] - q.y;
                if (MI && mi[0]) dx -= Lb[0] * rint(dx / Lb[0]);
                if (MI && mi[1]) dy -= Lb[1] * rint(dy / Lb[1]);
                if (MI && mi[2]) dz -= Lb[2] * rint(dz / Lb[2]);
                const T sc = w[u] * (dx * v.x + dy * v.y + dz * v.z);
                p0 += sc * dx;
                p1 += sc * dy;
                p2 += sc * dz;
            } else {
                p0 += w[u] * v.x;
                p1 += w[u] * v.y;
                p2 += w[u] * v.z;
            }
        }
    }
}

// One packed chunk (FP32 isotropic, (x, y) pair staging): entry u of words
// pa (0-3), pb (4-7) holds staged index e & 0xfff and weight q = e >> 12
// (SGN: arithmetic shift) in units of the dequantisation step; the sums take
// q x, and the caller scales them by the step once (the same sums up to
// rounding, with three fewer instructions per entry).  CHECK: only entries
// with staged index in [c0, c0 + cn), read through the stage view.
template <bool SGN, bool CHECK>
__device__ __forceinline__ void mv_chunk_packed(const StageView<float, true> &xs, uint4 pa, uint4 pb, unsigned c0,
                                                unsigned cn, float &p0, float &p1, float &p2)
{
    const uint32_t e[8] = {pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w};
    unsigned li[8];
    float q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        li[u] = e[u] & 0xfffu;
        q[u] = SGN ? static_cast<float>(static_cast<int>(e[u]) >> 12) : static_cast<float>(e[u] >> 12);
    }
    if constexpr (!CHECK) {
        const float2 *xy = reinterpret_cast<const float2 *>(xs.soa);
        const float *zp = xs.soa + 2 * xs.stride;
#pragma unroll
        for (int h = 0; h < 8; h += 4) {
            float2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = xy[li[h + u]];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                p0 += q[h + u] * v[u].x;
                p1 += q[h + u] * v[u].y;
            }
        }
        float vz[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) vz[u] = zp[li[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) p2 += q[u] * vz[u];
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned l = li[u] - c0;
            if (l >= cn) continue;
            const float4 v = xs.get(l);
            p0 += q[u] * v.x;
            p1 += q[u] * v.y;
            p2 += q[u] * v.z;
        }
    }
}

// One packed FP64 chunk (isotropic, three planes): the eight 64-bit words
// held as the bits of ra (entries 0-3) and rb (4-7), index e & 0xfff and
// weight q = e >> 12 in units of the dequantisation step, as above.
template <bool SGN, bool CHECK>
__device__ __forceinline__ void mv_chunk_packed64(const StageView<double, true> &xs, const double4 &ra,
                                                  const double4 &rb, unsigned c0, unsigned cn, double &p0, double &p1,
                                                  double &p2)
{
    const uint64_t e[8] = {static_cast<uint64_t>(__double_as_longlong(ra.x)),
                           static_cast<uint64_t>(__double_as_longlong(ra.y)),
                           static_cast<uint64_t>(__double_as_longlong(ra.z)),
                           static_cast<uint64_t>(__double_as_longlong(ra.w)),
                           static_cast<uint64_t>(__double_as_longlong(rb.x)),
                           static_cast<uint64_t>(__double_as_longlong(rb.y)),
                           static_cast<uint64_t>(__double_as_longlong(rb.z)),
                           static_cast<uint64_t>(__double_as_longlong(rb.w))};
    unsigned li[8];
    double q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        li[u] = static_cast<unsigned>(e[u]) & 0xfffu;
        q[u] = entry_q64(e[u], SGN);
    }
    if constexpr (!CHECK) {
        double acc[3] = {p0, p1, p2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = xs.soa[d * xs.stride + li[u]];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[d] += q[u] * v[u];
        }
        p0 = acc[0];
        p1 = acc[1];
        p2 = acc[2];
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned l = li[u] - c0;
            if (l >= cn) continue;
            const double4 v = xs.get(l);
            p0 += q[u] * v.x;
            p1 += q[u] * v.y;
            p2 += q[u] * v.z;
        }
    }
}

// output of particle so (cell order): to the sorted vector, or to the
// original order with an optional addend
template <typename T>
__device__ __forceinline__ void mv_store(const MvArgs &A, int64_t so, T o0, T o1, T o2)
{
    using T4 = typename V4<T>::t;
    if (A.out_sorted) {
        T4 o;
        o.x = o0;
        o.y = o1;
        o.z = o2;
        o.w = T(0);
        static_cast<T4 *>(A.out_sorted)[so] = o;
    } else {
        const int p = A.sorted[so];
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

// FP32 isotropic: at most 80 registers, so that at least six waves per SIMD
// are resident (the kernel needs about 62: eight waves, four work-groups of
// 512, as the LDS of the planar staging allows at N = 2e5, rho = 0.5)
template <typename T, bool PAR>
constexpr int mv_min_waves()
{
    return (sizeof(T) == 4 && !PAR) ? 6 : 1;
}

template <typename T, bool PAR, bool MI, int BS, int L>
__global__ __launch_bounds__(BS, (mv_min_waves<T, PAR>())) void k_mv(MvArgs A)
{
    using T4 = typename V4<T>::t;
    using T2 = typename V2<T>::t;
    constexpr int PG = BS / L;  // particles per round
    extern __shared__ __align__(32) unsigned char mv_lds[];
    __shared__ int sst[kStab], sbase[kStab];
    double ca = A.a, cb = A.b, ccz = A.cz;
    const T *coefp = static_cast<const T *>(A.coef);
    if (A.chain) {
        // a term of the Chebyshev chain: its coefficients follow this step's plan
        const ChainStep cs = A.chain[A.cheb_k];
        if (cs.skip) return;
        ca = cs.a;
        cb = cs.b;
        ccz = cs.cz;
        coefp += static_cast<int64_t>(cs.row) * A.rcap;
    }
    const int cid = A.rev ? static_cast<int>(gridDim.x - 1 - blockIdx.x) : static_cast<int>(blockIdx.x);
    const int h0 = A.cstart[cid], occ = A.cstart[cid + 1] - h0;
    if (occ <= 0) return;
    const int tid = threadIdx.x;
    const int nst = A.nst;
    if (tid <= nst) {
        const int2 e = A.stab[static_cast<int64_t>(cid) * kStab + tid];
        sst[tid] = e.x;
        sbase[tid] = e.y;
    }
    constexpr bool SOA = mv_soa<T, PAR>();
    T4 *xs = reinterpret_cast<T4 *>(mv_lds);
    T *xsoa = reinterpret_cast<T *>(mv_lds);
    const unsigned sstride = static_cast<unsigned>(A.maxc);
    const StageView<T, SOA> view{xs, xsoa, sstride};
    T2 *pyz = reinterpret_cast<T2 *>(mv_lds + static_cast<size_t>(A.maxc > BS ? A.maxc : BS) * sizeof(T4));
    T4 *part = xs;  // reused once the gathers of a round are done
    const T4 *__restrict__ x = static_cast<const T4 *>(A.x);
    // this cell's lists (cell-blocked: chunk c of the cell's particle j at
    // c occ + j, weight rows likewise)
    const T4 *__restrict__ nbw4 = static_cast<const T4 *>(A.nbw) + static_cast<int64_t>(h0) * 2 * A.cap8;
    const uint4 *__restrict__ nbp4 = reinterpret_cast<const uint4 *>(nbw4);  // packed chunks
    const void *nbl = A.nbl + static_cast<int64_t>(h0) * A.cap8;  // either index form
    const bool pair = ca != 0.0;
    const T Lb[3] = {static_cast<T>(A.g.L[0]), static_cast<T>(A.g.L[1]), static_cast<T>(A.g.L[2])};
    const bool mi[3] = {A.g.nc[0] < 3, A.g.nc[1] < 3, A.g.nc[2] < 3};
    __syncthreads();
    const int total = __builtin_amdgcn_readfirstlane(sbase[nst]);
    const bool narrow = total <= kNarrowStencil;
    bool staged_all = false;
    for (int g0 = 0; g0 < occ; g0 += PG) {
        const int m = min(PG, occ - g0);
        const bool active = tid < m * L;
        const int sub = active ? tid / m : 0;
        const int pi = active ? tid - sub * m : 0;
        const int64_t s = h0 + g0 + pi;
        const int j = g0 + pi;  // particle of the cell
        const int nch = (active && pair) ? (A.nn[s] + 7) >> 3 : 0;
        T own[3] = {T(0), T(0), T(0)};
        if (PAR && active) {
            const double4 q = A.reld[s];
            own[0] = static_cast<T>(q.x);
            own[1] = static_cast<T>(q.y);
            own[2] = static_cast<T>(q.z);
        }
        T p0 = 0, p1 = 0, p2 = 0;
        // the pair sum, for either index form of the cell's lists
        // a staged input entry into the LDS layout of the view
        auto stage_put = [&](int at, const T4 &v) __attribute__((always_inline)) {
            if constexpr (SOA && mv_xy<T>()) {
                T2 xyv;
                xyv.x = v.x;
                xyv.y = v.y;
                reinterpret_cast<T2 *>(xsoa)[at] = xyv;
                xsoa[2 * sstride + at] = v.z;
            } else if constexpr (SOA) {
                xsoa[at] = v.x;
                xsoa[sstride + at] = v.y;
                xsoa[2 * sstride + at] = v.z;
            } else {
                xs[at] = v;
            }
        };
        // FM: the cell's list form, 0 wide (16-bit indices), 1 narrow (12-bit),
        // 2 and 3 packed (12-bit index and 20-bit weight per word, unsigned or
        // signed; its chunk's two words wait in id and id2 until the chunk is
        // used, and the sums are scaled by the weights' step at the end)
        auto pair_sum = [&](auto form) __attribute__((always_inline)) {
            constexpr int FM = decltype(form)::value;
            constexpr bool NR = FM == 1, PK = FM >= 2;
            auto load = [&](int c, uint4 &i1, uint4 &i2, T4 &w1, T4 &w2) __attribute__((always_inline)) {
                if constexpr (PK && sizeof(T) == 4) {
                    i1 = nbp4[(2 * c) * occ + j];
                    i2 = nbp4[(2 * c + 1) * occ + j];
                } else if constexpr (PK) {
                    // FP64: the chunk's eight words in the weights' slots
                    w1 = nbw4[(2 * c) * occ + j];
                    w2 = nbw4[(2 * c + 1) * occ + j];
                } else {
                    i1 = ids_load<NR>(nbl, c * occ + j);
                    w1 = nbw4[(2 * c) * occ + j];
                    w2 = nbw4[(2 * c + 1) * occ + j];
                }
            };
            // this lane's first chunk: its loads are in flight during the
            // staging below (a later staging round loads it again)
            uint4 id = make_uint4(0, 0, 0, 0), id2 = make_uint4(0, 0, 0, 0);
            T4 wa{}, wb{};
            if (sub < nch) load(sub, id, id2, wa, wb);
            for (int c0 = 0; c0 < total; c0 += A.maxc) {
                const int c1 = min(total, c0 + A.maxc);
                const bool single = c0 == 0 && c1 == total;
                if (!(single && staged_all)) {
                    __syncthreads();
                    // the stencil entry holding staged index l
                    auto source = [&](int l) __attribute__((always_inline)) {
                        int lo = 0, hi = nst - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (sbase[mid] <= l) lo = mid; else hi = mid - 1;
                        }
                        return lo;
                    };
                    if constexpr (!PAR) {
                        // kStageDepth entries per thread at a time: their
                        // searches and loads in flight together, then the
                        // stores
                        int l = c0 + tid;
                        for (; l + (kStageDepth - 1) * BS < c1; l += kStageDepth * BS) {
                            int t[kStageDepth];
#pragma unroll
                            for (int u = 0; u < kStageDepth; ++u) {
                                const int e = source(l + u * BS);
                                t[u] = sst[e] + (l + u * BS - sbase[e]);
                            }
                            T4 v[kStageDepth];
#pragma unroll
                            for (int u = 0; u < kStageDepth; ++u) v[u] = x[t[u]];
#pragma unroll
                            for (int u = 0; u < kStageDepth; ++u) stage_put(l + u * BS - c0, v[u]);
                        }
                        for (; l < c1; l += BS) {
                            const int e = source(l);
                            stage_put(l - c0, x[sst[e] + (l - sbase[e])]);
                        }
                    } else {
                        for (int l = c0 + tid; l < c1; l += BS) {
                            const int lo = source(l);
                            const int t = sst[lo] + (l - sbase[lo]);
                            T4 v = x[t];
                            const int e0 = lo % A.g.noff[0], e1 = (lo / A.g.noff[0]) % A.g.noff[1];
                            const int e2 = lo / (A.g.noff[0] * A.g.noff[1]);
                            const double4 q = A.reld[t];
                            // as in the neighbour lists: position and image offset
                            // each in the work precision, then added
                            v.w = static_cast<T>(q.x) + static_cast<T>(A.g.offs[0][e0] * A.g.edge[0]);
                            T2 yz;
                            yz.x = static_cast<T>(q.y) + static_cast<T>(A.g.offs[1][e1] * A.g.edge[1]);
                            yz.y = static_cast<T>(q.z) + static_cast<T>(A.g.offs[2][e2] * A.g.edge[2]);
                            pyz[l - c0] = yz;
                            stage_put(l - c0, v);
                        }
                    }
                    __syncthreads();
                    staged_all = single;
                }
                // this lane's chunks, the next one's loads in flight
                if (c0 > 0 && sub < nch) load(sub, id, id2, wa, wb);
                for (int ch = sub; ch < nch; ch += L) {
                    const uint4 cid8 = id, cid8b = id2;
                    const T4 cwa = wa, cwb = wb;
                    if (ch + L < nch) load(ch + L, id, id2, wa, wb);
                    if constexpr (PK && sizeof(T) == 4) {
                        if (single)
                            mv_chunk_packed<FM == 3, false>(view, cid8, cid8b, 0u, 0u, p0, p1, p2);
                        else
                            mv_chunk_packed<FM == 3, true>(view, cid8, cid8b, static_cast<unsigned>(c0),
                                                           static_cast<unsigned>(c1 - c0), p0, p1, p2);
                    } else if constexpr (PK) {
                        if (single)
                            mv_chunk_packed64<FM == 3, false>(view, cwa, cwb, 0u, 0u, p0, p1, p2);
                        else
                            mv_chunk_packed64<FM == 3, true>(view, cwa, cwb, static_cast<unsigned>(c0),
                                                             static_cast<unsigned>(c1 - c0), p0, p1, p2);
                    } else if (single) {
                        mv_chunk<T, PAR, false, MI, SOA, NR>(view, pyz, cid8, cwa, cwb, own, Lb, mi, 0u, 0u, p0, p1,
                                                             p2);
                    } else {
                        mv_chunk<T, PAR, true, MI, SOA, NR>(view, pyz, cid8, cwa, cwb, own, Lb, mi,
                                                            static_cast<unsigned>(c0), static_cast<unsigned>(c1 - c0),
                                                            p0, p1, p2);
                    }
                }
            }
            if constexpr (PK) {
                // the sums took the weights in units of their step
                const T inv = sizeof(T) == 4 ? static_cast<T>(A.wq_inv32) : static_cast<T>(A.wq_inv);
                p0 *= inv;
                p1 *= inv;
                p2 *= inv;
            }
        };
        if (pair) {
            if constexpr (!PAR) {
                if (narrow && A.wpack && A.wq_signed) pair_sum(std::integral_constant<int, 3>{});
                else if (narrow && A.wpack) pair_sum(std::integral_constant<int, 2>{});
                else if (narrow) pair_sum(std::integral_constant<int, 1>{});
                else pair_sum(std::integral_constant<int, 0>{});
            } else {
                if (narrow) pair_sum(std::integral_constant<int, 1>{});
                else pair_sum(std::integral_constant<int, 0>{});
            }
        }
        // the terms besides the pair sum, b x + cz z + sum_q c_q u_q, spread
        // over the L lanes of each particle (lane sub takes terms sub, sub + L,
        // ...: 0 is x, 1 is z, 2 + q is u_q), loaded right after the pair
        // loop and added to the lane's partial sum, so that their loads are
        // not left to the end of the work-group (measured at N = 2e5, rho = 0.5: FP64 138 ->
        // 128 us per mat-vec, FP32 68 -> 64 us with the planar staging)
        {
            T e0 = 0, e1 = 0, e2 = 0;
            if (active) {
                const int nterm = 2 + A.r;
                const T *coef = coefp;
                const T4 *us = static_cast<const T4 *>(A.us);
                const T4 *zv = static_cast<const T4 *>(A.z);
                for (int tt = sub; tt < nterm; tt += L) {
                    T cf = T(0);
                    T4 v{};
                    if (tt == 0) {
                        if (cb != 0.0) {
                            cf = static_cast<T>(cb);
                            v = x[s];
                        }
                    } else if (tt == 1) {
                        if (ccz != 0.0) {
                            cf = static_cast<T>(ccz);
                            v = zv[s];
                        }
                    } else {
                        cf = A.premix ? T(1) : coef[tt - 2];
                        v = us[static_cast<int64_t>(tt - 2) * A.S + s];
                    }
                    e0 += cf * v.x;
                    e1 += cf * v.y;
                    e2 += cf * v.z;
                }
            }
            // the L partial sums of each particle meet in LDS
            __syncthreads();
            if (active) {
                const T a = static_cast<T>(ca);
                T4 q;
                q.x = a * p0 + e0;
                q.y = a * p1 + e1;
                q.z = a * p2 + e2;
                q.w = T(0);
                part[sub * PG + pi] = q;
            }
            __syncthreads();
            staged_all = false;
            if (tid < m) {
                T o0 = 0, o1 = 0, o2 = 0;
#pragma unroll
                for (int u = 0; u < L; ++u) {
                    const T4 q = part[u * PG + tid];
                    o0 += q.x;
                    o1 += q.y;
                    o2 += q.z;
                }
                mv_store<T>(A, h0 + g0 + tid, o0, o1, o2);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Noise window (the variant of Sec. II.C that computes the random forces of
// W consecutive steps together, at the positions of the window's first step).
// Filter outputs of the W steps of the window holding the current step, in
// cell order: usw[(m r + q) S + s] = u_q(n0 + m) of the particle sorted[s],
// n0 = step - step mod W (W divides the filter block, so the W steps lie in
// the block whose outputs U holds).
template <typename T>
__global__ void k_permute_window(int64_t n, int64_t S, const int *__restrict__ sorted, const T *__restrict__ U,
                                 int r, int rcap, int block, int urows, int W, const long long *__restrict__ d_step,
                                 typename V4<T>::t *__restrict__ usw)
{
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int p = sorted[s];
    const long long n0 = *d_step - *d_step % W;
    U += ((n0 / block) & 1) * urows * 3 * S;
    for (int m = 0; m < W; ++m) {
        const int bi = static_cast<int>((n0 + m) % block);
        for (int q = 0; q < r; ++q) {
            const T *uq = U + (static_cast<int64_t>(bi) * rcap + q) * 3 * S;
            typename V4<T>::t o;
            o.x = uq[p];
            o.y = uq[S + p];
            o.z = uq[2 * S + p];
            o.w = T(0);
            usw[(static_cast<int64_t>(m) * r + q) * S + s] = o;
        }
    }
}

// NV right-hand sides through one stream of the pair lists (isotropic pair
// tensor): for v < NV,
//   out_v = a P x_v + b x_v + cz z_v + sum_q coef[q] us_{v,q},
// with x_v = x + v S, z_v = z + v S, us_{v,q} = us + (v r + q) S (sorted T4),
// out_v = out_sorted + v S (sorted T4) or out_orig + v 3 S ([3][S], original
// order).  The staging holds NV x 3 planes of maxc values; rounds, lanes and
// the spread epilogue are those of k_mv.  Each list chunk is read once for
// the NV vectors, so the list traffic per vector falls by NV.
// DUAL (NV = 2): vector 0 is a term of the step's chain (as k_mv computes
// it, premixed v_k included) and vector 1 the dissipative product
// F^D' = -P Y + Dneg (y2, dneg2, fd2), so that the chain's first pair term
// and P Y share one stream of the lists.  With a plan chosen on the device,
// the term takes the second product only where the plan marks it as its
// first pair term (ChainStep::dual), else it is the plain term.
template <typename T, int BS, int L, int NV, bool DUAL = false>
__global__ __launch_bounds__(BS) void k_mvw(MvArgs A)
{
    static_assert(!DUAL || NV == 2, "the dual form carries two vectors");
    using T4 = typename V4<T>::t;
    constexpr int PG = BS / L;
    extern __shared__ __align__(32) unsigned char mv_lds[];
    __shared__ int sst[kStab], sbase[kStab];
    double ca = A.a, cb = A.b, ccz = A.cz;
    const T *coefp = static_cast<const T *>(A.coef);
    bool dual = DUAL;
    if (A.chain) {
        // a term of the Chebyshev chains: its coefficients follow this step's plan
        const ChainStep cs = A.chain[A.cheb_k];
        if (cs.skip) return;
        ca = cs.a;
        cb = cs.b;
        ccz = cs.cz;
        coefp += static_cast<int64_t>(cs.row) * A.rcap;
        dual = DUAL && cs.dual != 0;
    }
    // vectors this launch carries; vector v's input
    const int nvl = DUAL ? (dual ? 2 : 1) : NV;
    const int cid = A.rev ? static_cast<int>(gridDim.x - 1 - blockIdx.x) : static_cast<int>(blockIdx.x);
    const int h0 = A.cstart[cid], occ = A.cstart[cid + 1] - h0;
    if (occ <= 0) return;
    const int tid = threadIdx.x;
    const int nst = A.nst;
    if (tid <= nst) {
        const int2 e = A.stab[static_cast<int64_t>(cid) * kStab + tid];
        sst[tid] = e.x;
        sbase[tid] = e.y;
    }
    T *xsoa = reinterpret_cast<T *>(mv_lds);   // [NV][3 maxc]: FP32 (x, y) pairs then z; FP64 three planes
    T4 *part = reinterpret_cast<T4 *>(mv_lds);  // [NV][BS], once the gathers of a round are done
    const unsigned ss = static_cast<unsigned>(A.maxc);
    const T4 *__restrict__ x = static_cast<const T4 *>(A.x);
    auto vin = [&](int v) -> const T4 * {
        return (DUAL && v == 1) ? static_cast<const T4 *>(A.y2) : x + static_cast<int64_t>(v) * A.S;
    };
    const T4 *__restrict__ nbw4 = static_cast<const T4 *>(A.nbw) + static_cast<int64_t>(h0) * 2 * A.cap8;
    const uint4 *__restrict__ nbp4 = reinterpret_cast<const uint4 *>(nbw4);  // packed chunks
    const void *nbl = A.nbl + static_cast<int64_t>(h0) * A.cap8;  // either index form
    const bool pair = ca != 0.0;
    __syncthreads();
    const int total = __builtin_amdgcn_readfirstlane(sbase[nst]);
    const bool narrow = total <= kNarrowStencil;
    bool staged_all = false;
    for (int g0 = 0; g0 < occ; g0 += PG) {
        const int m = min(PG, occ - g0);
        const bool active = tid < m * L;
        const int sub = active ? tid / m : 0;
        const int pi = active ? tid - sub * m : 0;
        const int64_t s = h0 + g0 + pi;
        const int j = g0 + pi;
        const int nch = (active && pair) ? (A.nn[s] + 7) >> 3 : 0;
        T p[NV][3];
#pragma unroll
        for (int v = 0; v < NV; ++v) p[v][0] = p[v][1] = p[v][2] = T(0);
        // the pair sums, for either index form of the cell's lists
        // FM: the cell's list form, as in k_mv (2 and 3: packed words,
        // unsigned and signed weights, in id, id2 or in FP64 in wa, wb; the
        // sums take the weights in units of their step and are scaled at the
        // end).  FP32 stages each vector as (x, y) pairs and a z plane.
        auto pair_sum = [&](auto form) __attribute__((always_inline)) {
            constexpr int FM = decltype(form)::value;
            constexpr bool NR = FM == 1, PK = FM >= 2;
            auto load = [&](int c, uint4 &i1, uint4 &i2, T4 &w1, T4 &w2) __attribute__((always_inline)) {
                if constexpr (PK && sizeof(T) == 4) {
                    i1 = nbp4[(2 * c) * occ + j];
                    i2 = nbp4[(2 * c + 1) * occ + j];
                } else if constexpr (PK) {
                    w1 = nbw4[(2 * c) * occ + j];
                    w2 = nbw4[(2 * c + 1) * occ + j];
                } else {
                    i1 = ids_load<NR>(nbl, c * occ + j);
                    w1 = nbw4[(2 * c) * occ + j];
                    w2 = nbw4[(2 * c + 1) * occ + j];
                }
            };
            for (int c0 = 0; c0 < total; c0 += A.maxc) {
                const int c1 = min(total, c0 + A.maxc);
                const bool single = c0 == 0 && c1 == total;
                if (!(single && staged_all)) {
                    __syncthreads();
                    // entries l + u BS (u < D) of the stage, their searches
                    // and loads in flight together, then the stores
                    auto stage = [&](int l, auto depth) __attribute__((always_inline)) {
                        constexpr int D = decltype(depth)::value;
                        int t[D];
#pragma unroll
                        for (int u = 0; u < D; ++u) {
                            const int e = entry_of(sbase, nst, l + u * BS);
                            t[u] = sst[e] + (l + u * BS - sbase[e]);
                        }
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            if (v >= nvl) break;
                            T4 q[D];
#pragma unroll
                            for (int u = 0; u < D; ++u) q[u] = vin(v)[t[u]];
#pragma unroll
                            for (int u = 0; u < D; ++u) {
                                const int at = l + u * BS - c0;
                                if constexpr (sizeof(T) == 4) {
                                    float2 xyv;
                                    xyv.x = q[u].x;
                                    xyv.y = q[u].y;
                                    reinterpret_cast<float2 *>(xsoa + 3 * v * ss)[at] = xyv;
                                    xsoa[(3 * v + 2) * ss + at] = q[u].z;
                                } else {
                                    xsoa[(3 * v + 0) * ss + at] = q[u].x;
                                    xsoa[(3 * v + 1) * ss + at] = q[u].y;
                                    xsoa[(3 * v + 2) * ss + at] = q[u].z;
                                }
                            }
                        }
                    };
                    int l = c0 + tid;
                    for (; l + (kStageDepth - 1) * BS < c1; l += kStageDepth * BS)
                        stage(l, std::integral_constant<int, kStageDepth>{});
                    for (; l < c1; l += BS) stage(l, std::integral_constant<int, 1>{});
                    __syncthreads();
                    staged_all = single;
                }
                uint4 id = make_uint4(0, 0, 0, 0), id2 = make_uint4(0, 0, 0, 0);
                T4 wa{}, wb{};
                if (sub < nch) load(sub, id, id2, wa, wb);
                const unsigned cn = static_cast<unsigned>(c1 - c0);
                for (int ch = sub; ch < nch; ch += L) {
                    const uint4 cid8 = id, cid8b = id2;
                    const T4 cwa = wa, cwb = wb;
                    if (ch + L < nch) load(ch + L, id, id2, wa, wb);
                    unsigned li[8];
                    T w[8];
                    if constexpr (PK && sizeof(T) == 4) {
                        const uint32_t ew[8] = {cid8.x, cid8.y, cid8.z, cid8.w, cid8b.x, cid8b.y, cid8b.z, cid8b.w};
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            li[u] = ew[u] & 0xfffu;
                            w[u] = FM == 3 ? static_cast<T>(static_cast<int>(ew[u]) >> 12)
                                           : static_cast<T>(ew[u] >> 12);
                        }
                    } else if constexpr (PK) {
                        const T ww[8] = {cwa.x, cwa.y, cwa.z, cwa.w, cwb.x, cwb.y, cwb.z, cwb.w};
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const uint64_t e = static_cast<uint64_t>(__double_as_longlong(static_cast<double>(ww[u])));
                            li[u] = static_cast<unsigned>(e) & 0xfffu;
                            w[u] = static_cast<T>(entry_q64(e, FM == 3));
                        }
                    } else {
                        const unsigned l8[8] = {id_at<NR, 0>(cid8), id_at<NR, 1>(cid8), id_at<NR, 2>(cid8),
                                                id_at<NR, 3>(cid8), id_at<NR, 4>(cid8), id_at<NR, 5>(cid8),
                                                id_at<NR, 6>(cid8), id_at<NR, 7>(cid8)};
                        const T w8[8] = {cwa.x, cwa.y, cwa.z, cwa.w, cwb.x, cwb.y, cwb.z, cwb.w};
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            li[u] = l8[u];
                            w[u] = w8[u];
                        }
                    }
                    unsigned lo8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        // a later round: entries outside the staged range count zero
                        lo8[u] = li[u] - static_cast<unsigned>(c0);
                        if (!single && lo8[u] >= cn) {
                            lo8[u] = 0;
                            w[u] = T(0);
                        }
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        if (v >= nvl) break;
                        if constexpr (sizeof(T) == 4) {
                            const float2 *xy = reinterpret_cast<const float2 *>(xsoa + 3 * v * ss);
#pragma unroll
                            for (int h = 0; h < 8; h += 4) {
                                float2 vv[4];
#pragma unroll
                                for (int u = 0; u < 4; ++u) vv[u] = xy[lo8[h + u]];
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    p[v][0] += w[h + u] * vv[u].x;
                                    p[v][1] += w[h + u] * vv[u].y;
                                }
                            }
                            T vz[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) vz[u] = xsoa[(3 * v + 2) * ss + lo8[u]];
#pragma unroll
                            for (int u = 0; u < 8; ++u) p[v][2] += w[u] * vz[u];
                        } else {
#pragma unroll
                            for (int q = 0; q < 3; ++q) {
                                T val[8];
#pragma unroll
                                for (int u = 0; u < 8; ++u) val[u] = xsoa[(3 * v + q) * ss + lo8[u]];
                                T acc = p[v][q];
#pragma unroll
                                for (int u = 0; u < 8; ++u) acc += w[u] * val[u];
                                p[v][q] = acc;
                            }
                        }
                    }
                }
            }
            if constexpr (PK) {
                // the sums took the weights in units of their step
                const T inv = sizeof(T) == 4 ? static_cast<T>(A.wq_inv32) : static_cast<T>(A.wq_inv);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (v >= nvl) break;
                    p[v][0] *= inv;
                    p[v][1] *= inv;
                    p[v][2] *= inv;
                }
            }
        };
        if (pair) {
            if (narrow && A.wpack && A.wq_signed) pair_sum(std::integral_constant<int, 3>{});
            else if (narrow && A.wpack) pair_sum(std::integral_constant<int, 2>{});
            else if (narrow) pair_sum(std::integral_constant<int, 1>{});
            else pair_sum(std::integral_constant<int, 0>{});
        }
        // b x_v + cz z_v + sum_q c_q u_{v,q}, spread over the L lanes of each
        // particle as in k_mv
        T e[NV][3];
#pragma unroll
        for (int v = 0; v < NV; ++v) e[v][0] = e[v][1] = e[v][2] = T(0);
        if (active) {
            const int nterm = 2 + A.r;
            const T *coef = coefp;
            const T4 *us = static_cast<const T4 *>(A.us);
            const T4 *zv = static_cast<const T4 *>(A.z);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (DUAL && v == 1) break;  // the dissipative product has no other terms
                for (int tt = sub; tt < nterm; tt += L) {
                    T cf = T(0);
                    T4 q{};
                    if (tt == 0) {
                        if (cb != 0.0) {
                            cf = static_cast<T>(cb);
                            q = x[static_cast<int64_t>(v) * A.S + s];
                        }
                    } else if (tt == 1) {
                        if (ccz != 0.0) {
                            cf = static_cast<T>(ccz);
                            q = zv[static_cast<int64_t>(v) * A.S + s];
                        }
                    } else {
                        cf = A.premix ? T(1) : coef[tt - 2];
                        q = us[(static_cast<int64_t>(v) * A.r + (tt - 2)) * A.S + s];
                    }
                    e[v][0] += cf * q.x;
                    e[v][1] += cf * q.y;
                    e[v][2] += cf * q.z;
                }
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (v >= nvl) break;
                const T a = (DUAL && v == 1) ? T(-1) : static_cast<T>(ca);
                T4 q;
                q.x = a * p[v][0] + e[v][0];
                q.y = a * p[v][1] + e[v][1];
                q.z = a * p[v][2] + e[v][2];
                q.w = T(0);
                part[v * BS + sub * PG + pi] = q;
            }
        }
        __syncthreads();
        staged_all = false;
        for (int k = tid; k < nvl * m; k += BS) {
            const int v = k / m, i = k - v * m;
            T o0 = 0, o1 = 0, o2 = 0;
#pragma unroll
            for (int u = 0; u < L; ++u) {
                const T4 q = part[v * BS + u * PG + i];
                o0 += q.x;
                o1 += q.y;
                o2 += q.z;
            }
            const int64_t so = h0 + g0 + i;
            if (DUAL && v == 1) {
                const int pp = A.sorted[so];
                const T *ad = static_cast<const T *>(A.dneg2);
                T *out = static_cast<T *>(A.fd2);
                out[pp] = o0 + ad[pp];
                out[A.S + pp] = o1 + ad[A.S + pp];
                out[2 * A.S + pp] = o2 + ad[2 * A.S + pp];
            } else if (A.out_sorted) {
                T4 o;
                o.x = o0;
                o.y = o1;
                o.z = o2;
                o.w = T(0);
                static_cast<T4 *>(A.out_sorted)[static_cast<int64_t>(v) * A.S + so] = o;
            } else {
                const int pp = A.sorted[so];
                T *out = static_cast<T *>(A.out_orig) + static_cast<int64_t>(v) * 3 * A.S;
                out[pp] = o0;
                out[A.S + pp] = o1;
                out[2 * A.S + pp] = o2;
            }
        }
    }
}

// The plan of this step's Chebyshev chain.  The refresh of the step before
// left the largest row sum of |w| (a Gershgorin bound on the spectrum of P,
// ||T_ij|| = 1) in rowmax; at most lam_t, the tight plan's interval holds the
// spectrum and its shorter expansion is used.  Term k of the chain (launched
// in the order k = Kw-1 .. 0) then gets its Clenshaw combination:
//   b_{Ka-1} = v_{Ka-1};  b_k = v_k + 2 P~ b_{k+1} - b_{k+2};  F = v_0 + P~ b_1 - b_2,
// with b_{Ka} = b_{Ka+1} = 0, P~ = alpha P + beta and Ka the chosen plan's K;
// the terms k >= Ka are skipped.
// The tight plan's lower end lies closer to the spectrum than the wide
// plan's: it also needs the smallest Ritz value of the last spectrum check
// (theta_min) at least lo_t; once a check finds it below, the retired flag
// stays set and every step takes the wide plan (until a new state is
// written), whose lower end the check guards as before.
struct ChainSel {
    int Kw, Kt;           // terms of the wide and the tight plan
    float lam_t;          // largest row-sum bound for the tight plan
    double lo_t;          // smallest Ritz value of the last check for the tight plan
    double aw, bw, at, bt;
};

__global__ void k_cheb_select(ChainSel c, const unsigned *__restrict__ rowmax, const double *__restrict__ theta,
                              const int *__restrict__ retired, ChainStep *__restrict__ out,
                              unsigned long long *__restrict__ tight_steps)
{
    const float g = __uint_as_float(*rowmax);
    const bool tight = c.Kt > 0 && g <= c.lam_t && theta[0] >= c.lo_t && *retired == 0;
    const int Ka = tight ? c.Kt : c.Kw;
    const double al = tight ? c.at : c.aw, be = tight ? c.bt : c.bw;
    for (int k = threadIdx.x; k < c.Kw; k += blockDim.x) {
        ChainStep e;
        e.row = (tight ? c.Kw : 0) + k;
        e.skip = k >= Ka ? 1 : 0;
        e.dual = k == Ka - 2 ? 1 : 0;
        if (k >= Ka - 1) {
            e.a = 0.0;
            e.b = 0.0;
            e.cz = 0.0;
        } else if (k >= 1) {
            e.a = 2.0 * al;
            e.b = 2.0 * be;
            e.cz = k == Ka - 2 ? 0.0 : -1.0;
        } else {
            e.a = al;
            e.b = be;
            e.cz = Ka == 2 ? 0.0 : -1.0;
        }
        out[k] = e;
    }
    if (threadIdx.x == 0 && tight) atomicAdd(tight_steps, 1ull);
}

// v_k = sum_q B[row_k][q] u_q for every term k < K of the chain (row_k and
// skip from the step's plan when there is a tight plan, else row k): one
// read of the r filter outputs per step; particle s in cell order
template <typename T, int RMAX>
__global__ void k_cheb_mix(int64_t n, int64_t S, int r, int rcap, int K, const T *__restrict__ B,
                           const ChainStep *__restrict__ chain, const typename V4<T>::t *__restrict__ us,
                           typename V4<T>::t *__restrict__ vk)
{
    using T4 = typename V4<T>::t;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    T ux[RMAX], uy[RMAX], uz[RMAX];  // the step's filter outputs of this particle (r <= RMAX)
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
        ux[q] = uy[q] = uz[q] = T(0);
        if (q < r) {
            const T4 u = us[static_cast<int64_t>(q) * S + s];
            ux[q] = u.x;
            uy[q] = u.y;
            uz[q] = u.z;
        }
    }
    for (int k = 0; k < K; ++k) {
        int row = k;
        if (chain) {
            if (chain[k].skip) continue;
            row = chain[k].row;
        }
        const T *b = B + static_cast<int64_t>(row) * rcap;  // rows are zero-padded to rcap >= RMAX's r
        T4 v;
        v.x = v.y = v.z = v.w = T(0);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const T c = q < r ? b[q] : T(0);
            v.x += c * ux[q];
            v.y += c * uy[q];
            v.z += c * uz[q];
        }
        vk[static_cast<int64_t>(k) * S + s] = v;
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

// launch shapes of the mat-vec: lanes per work-group, lanes per particle
constexpr int kMvThreads32 = 512, kMvLanes32 = 4;
constexpr int kMvThreads64 = 512, kMvLanes64 = 4;

template <typename T, bool PAR, bool MI, int BS, int L>
hipError_t launch_mv_t(const Dev &d, const MvArgs &A, hipStream_t st)
{
    const size_t shm = mv_lds_bytes<T, PAR, BS>(d.maxc);
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mv<T, PAR, MI, BS, L>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm));
        if (e != hipSuccess) return e;
    }
    k_mv<T, PAR, MI, BS, L><<<d.ncell, BS, shm, st>>>(A);
    return hipGetLastError();
}

template <typename T, bool EX>
hipError_t launch_build_t(const Dev &d, const BuildArgs &a, bool mi, hipStream_t st)
{
    if (mi) k_build<T, EX, true><<<d.ncell, kPairThreads, 0, st>>>(a);
    else k_build<T, EX, false><<<d.ncell, kPairThreads, 0, st>>>(a);
    return hipGetLastError();
}

template <typename T, bool EX, bool PAR, bool MI>
hipError_t refresh_k(const Dev &d, const BuildArgs &a, hipStream_t st)
{
    const size_t shm = static_cast<size_t>(a.stage_n + 1) * sizeof(typename V4<T>::t);
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_refresh<T, EX, PAR, MI>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm));
        if (e != hipSuccess) return e;
    }
    k_refresh<T, EX, PAR, MI><<<d.ncell, kRefreshThreads, shm, st>>>(a);
    return hipGetLastError();
}

template <typename T, bool EX>
hipError_t launch_refresh_t(const Dev &d, BuildArgs a, bool mi, hipStream_t st)
{
    // stage the expected stencil (the mat-vec's estimate) as far as the LDS
    // budget allows: two work-groups per CU in FP32; in FP64 (32 bytes per
    // position) one, which stages the whole stencil instead of half of it
    // and spares the rest the global path (N = 2e5, rho = 0.5: 0.91 ->
    // 0.83 ms of neighbour work per step)
    constexpr size_t per = sizeof(typename V4<T>::t);
    constexpr size_t budget = sizeof(T) == 8 ? kRefreshLds64 : kRefreshLds;
    const int room = static_cast<int>((budget - refresh_fixed_lds<T>()) / per) - 1;
    a.stage_n = std::max(0, std::min(d.maxc, room));
    if (d.parallel) return mi ? refresh_k<T, EX, true, true>(d, a, st) : refresh_k<T, EX, true, false>(d, a, st);
    return mi ? refresh_k<T, EX, false, true>(d, a, st) : refresh_k<T, EX, false, false>(d, a, st);
}

}  // namespace

// largest staging capacity (candidates) that fits one work-group's LDS
int mv_max_staging(int fp64, int parallel)
{
    const size_t budget = 160 * 1024 - 1024;
    size_t per;
    if (fp64) per = parallel ? sizeof(double4) + sizeof(double2) : 3 * sizeof(double);
    else per = parallel ? sizeof(float4) + sizeof(float2) : 3 * sizeof(float);
    return static_cast<int>(budget / per);
}

// ===========================================================================
// launchers
// ===========================================================================
hipError_t launch_neighbors(const Dev &d, hipStream_t st, double *fc_out)
{
    const Geo g = make_geo(d);
    const unsigned nb = blocks(d.n, 256);
    // rebuild the cell order and the candidate lists if some particle moved
    // more than skin/2 since the last build (or the host asked for it)
    const double half = 0.5 * d.skin;
    k_disp_check<<<nb, 256, 0, st>>>(d.n, d.S, d.cell_sorted, d.R, static_cast<const double4 *>(d.rb_s), half * half,
                                     d.d_rebuild, d.d_step, d.rebuild_period);
    k_cell_assign<<<nb, 256, 0, st>>>(d.R, d.S, d.n, g, d.Rw, d.cell_id, d.cell_slot, d.cell_count, d.d_rebuild);
    k_cell_scan<<<1, 1024, 0, st>>>(d.cell_count, d.cell_start, d.ncell, d.d_rebuild);
    k_cell_scatter<<<nb, 256, 0, st>>>(d.n, d.cell_id, d.cell_slot, d.cell_start, d.cell_tmp, d.d_rebuild);
    k_cell_order<<<nb, 256, 0, st>>>(d.n, d.S, g, d.cell_id, d.cell_start, d.cell_tmp, d.cell_sorted, d.R, d.Rw,
                                     static_cast<double4 *>(d.rb_s), static_cast<double4 *>(d.relb), d.d_rebuild);
    BuildArgs a{};
    a.g = g;
    a.ncell = d.ncell;
    a.n = d.n;
    a.S = d.S;
    a.cstart = d.cell_start;
    a.sorted = d.cell_sorted;
    a.reld_src = static_cast<const double4 *>(d.reld);
    a.relf_src = static_cast<const float4 *>(d.relf);
    a.pos_s = static_cast<const double4 *>(d.pos_s);
    a.rc2 = d.r_cut * d.r_cut;
    a.rcs2 = (d.r_cut + d.skin) * (d.r_cut + d.skin);
    a.cap = d.cap;
    a.capS = d.capS;
    a.snl = static_cast<uint4 *>(d.snl);
    a.snn = d.snn;
    a.nst = d.noff[0] * d.noff[1] * d.noff[2];
    a.cell_id = d.cell_id;
    a.gate = d.d_rebuild;
    a.wtab = d.wtab;
    a.n_r = d.n_r;
    a.r0 = d.r0;
    a.dr = d.dr;
    a.r_cut_min = d.r_cut_min;
    a.lam_hi = d.lam_hi;
    const double rw = std::pow(2.0, 1.0 / 6.0) * d.wca_sigma;
    a.wca_rc2 = d.wca_eps != 0.0 ? rw * rw : 0.0;
    a.wca_s2 = d.wca_sigma * d.wca_sigma;
    a.wca_eps = d.wca_eps;
    a.nbl = static_cast<uint16_t *>(d.nbl);
    a.nbw = d.nbw;
    a.wpack = d.wpack;
    a.wq_signed = d.wq_signed;
    a.wq_scale = d.wq_scale;
    a.wq_scale32 = static_cast<float>(d.wq_scale);
    a.nn = d.nn;
    a.stab = static_cast<int2 *>(d.stab);
    a.stab_c = static_cast<const int2 *>(d.stab);
    a.fc = fc_out;
    a.rowmax = d.d_rowmax;
    a.flags = d.d_flags;
    a.flag_step = d.d_flag_step;
    a.d_step = d.d_step;
    const bool mi = d.nc[0] < 3 || d.nc[1] < 3 || d.nc[2] < 3;
    hipError_t e;
    // the build stages the positions of the build itself (relb)
    BuildArgs ab = a;
    ab.reld_src = static_cast<const double4 *>(d.relb);
    if ((e = d.fp64 ? launch_build_t<double, true>(d, ab, mi, st) : launch_build_t<float, false>(d, ab, mi, st)) !=
        hipSuccess)
        return e;
    // current positions in the build's cell order; clears the rebuild flag
    k_rel_update<<<nb, 256, 0, st>>>(d.n, d.S, g, d.cell_sorted, d.R, static_cast<const double4 *>(d.rb_s),
                                     static_cast<const double4 *>(d.relb), static_cast<double4 *>(d.reld),
                                     static_cast<float4 *>(d.relf), static_cast<double4 *>(d.pos_s), d.d_rebuild,
                                     d.d_rowmax);
    return d.fp64 ? launch_refresh_t<double, true>(d, a, mi, st) : launch_refresh_t<float, false>(d, a, mi, st);
}

hipError_t launch_permute(const Dev &d, hipStream_t st, int r)
{
    if (d.fp64)
        k_permute<double><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, d.cell_sorted, static_cast<const double *>(d.Y),
                                                            static_cast<double4 *>(d.ys),
                                                            static_cast<const double *>(d.U), r, d.fir_rcap,
                                                            d.fir_block, fir_rows(1), d.d_step,
                                                            static_cast<double4 *>(d.us));
    else
        k_permute<float><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, d.cell_sorted, static_cast<const float *>(d.Y),
                                                           static_cast<float4 *>(d.ys), static_cast<const float *>(d.U),
                                                           r, d.fir_rcap, d.fir_block, fir_rows(0), d.d_step,
                                                           static_cast<float4 *>(d.us));
    return hipGetLastError();
}

MvArgs mv_args(const Dev &d, double a, double b, const void *x, double cz, const void *z, const void *coef, int r,
               const void *us, void *out_sorted, void *out_orig, const void *add_orig, bool reverse)
{
    MvArgs A{};
    A.rev = reverse ? 1 : 0;
    A.n = d.n;
    A.S = d.S;
    A.sorted = d.cell_sorted;
    A.cstart = d.cell_start;
    A.stab = static_cast<const int2 *>(d.stab);
    A.nst = d.noff[0] * d.noff[1] * d.noff[2];
    A.maxc = d.maxc;
    A.cap8 = d.cap >> 3;
    A.nbl = static_cast<const uint4 *>(d.nbl);
    A.nbw = d.nbw;
    A.wpack = d.wpack;
    A.wq_signed = d.wq_signed;
    A.wq_inv = d.wq_inv;
    A.wq_inv32 = static_cast<float>(d.wq_inv);
    A.nn = d.nn;
    A.reld = static_cast<const double4 *>(d.reld);
    A.g = make_geo(d);
    A.a = d.has_pair ? a : 0.0;
    A.b = b;
    A.cz = cz;
    A.x = x;
    A.z = z;
    A.coef = coef;
    A.us = us;
    A.add_orig = add_orig;
    A.r = coef ? r : 0;
    A.out_sorted = out_sorted;
    A.out_orig = out_orig;
    return A;
}

hipError_t launch_spmv(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz, const void *z,
                       const void *coef, int r, void *out_sorted, void *out_orig, const void *add_orig, bool reverse,
                       int cheb_k, bool premixed)
{
    MvArgs A = mv_args(d, a, b, x, cz, z, coef, r, d.us, out_sorted, out_orig, add_orig, reverse);
    if (cheb_k >= 0 && premixed) {
        // a term of the step's chain: its v_k is premixed (k_cheb_mix)
        A.us = static_cast<const char *>(d.vk) + static_cast<size_t>(cheb_k) * d.S * 4 * (d.fp64 ? 8 : 4);
        A.r = 1;
        A.premix = 1;
    }
    if (cheb_k >= 0 && d.cheb_kt > 0) {
        // the step's plan decides (k_cheb_select)
        A.chain = static_cast<const ChainStep *>(d.chain);
        A.cheb_k = cheb_k;
        A.rcap = d.fir_rcap;
        A.coef = d.Bmix;
    }
    const bool mi = d.nc[0] < 3 || d.nc[1] < 3 || d.nc[2] < 3;
    if (d.fp64) {
        if (d.parallel) {
            if (mi) return launch_mv_t<double, true, true, kMvThreads64, kMvLanes64>(d, A, st);
            return launch_mv_t<double, true, false, kMvThreads64, kMvLanes64>(d, A, st);
        }
        return launch_mv_t<double, false, false, kMvThreads64, kMvLanes64>(d, A, st);
    }
    if (d.parallel) {
        if (mi) return launch_mv_t<float, true, true, kMvThreads32, kMvLanes32>(d, A, st);
        return launch_mv_t<float, true, false, kMvThreads32, kMvLanes32>(d, A, st);
    }
    return launch_mv_t<float, false, false, kMvThreads32, kMvLanes32>(d, A, st);
}

// the staging capacity of the NV-vector mat-vec: what d.maxc asks for, at
// most what one work-group's LDS holds
template <typename T, int NV>
int mvw_staging(const Dev &d)
{
    // even, so that each vector's (x, y) pairs start 8-byte aligned: d.maxc
    // rounded up (at least 2), the LDS budget rounded down
    const size_t budget = 160 * 1024 - 1024;
    const size_t want = (static_cast<size_t>(std::max(d.maxc, 1)) + 1) & ~static_cast<size_t>(1);
    const size_t room = (budget / (NV * 3 * sizeof(T))) & ~static_cast<size_t>(1);
    return static_cast<int>(std::min(want, room));
}

template <typename T, int NV, bool DUAL = false>
hipError_t launch_mvw_t(const Dev &d, MvArgs A, hipStream_t st)
{
    constexpr int BS = sizeof(T) == 8 ? kMvThreads64 : kMvThreads32;
    constexpr int L = sizeof(T) == 8 ? kMvLanes64 : kMvLanes32;
    A.maxc = mvw_staging<T, NV>(d);
    if (A.maxc < 2) return hipErrorInvalidValue;  // the staging rounds advance by maxc
    const size_t stage = static_cast<size_t>(NV) * 3 * A.maxc * sizeof(T);
    const size_t part = static_cast<size_t>(NV) * BS * sizeof(typename V4<T>::t);
    const size_t shm = stage > part ? stage : part;
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mvw<T, BS, L, NV, DUAL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm));
        if (e != hipSuccess) return e;
    }
    k_mvw<T, BS, L, NV, DUAL><<<d.ncell, BS, shm, st>>>(A);
    return hipGetLastError();
}

hipError_t launch_spmv_dual(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz,
                            const void *z, void *out_sorted, void *out_orig, bool reverse, int cheb_k)
{
    if (d.parallel || !d.has_pair || !d.ys || !d.FD || !d.Dneg || !d.vk) return hipErrorInvalidValue;
    MvArgs A = mv_args(d, a, b, x, cz, z, nullptr, 1, d.us, out_sorted, out_orig, nullptr, reverse);
    // the term's premixed v_k (k_cheb_mix)
    A.us = static_cast<const char *>(d.vk) + static_cast<size_t>(cheb_k) * d.S * 4 * (d.fp64 ? 8 : 4);
    A.r = 1;
    A.premix = 1;
    if (d.cheb_kt > 0) {
        A.chain = static_cast<const ChainStep *>(d.chain);
        A.cheb_k = cheb_k;
        A.rcap = d.fir_rcap;
        A.coef = d.Bmix;
    }
    A.y2 = d.ys;
    A.dneg2 = d.Dneg;
    A.fd2 = d.FD;
    return d.fp64 ? launch_mvw_t<double, 2, true>(d, A, st) : launch_mvw_t<float, 2, true>(d, A, st);
}

hipError_t launch_spmv_window(const Dev &d, hipStream_t st, double a, double b, const void *x, double cz,
                              const void *z, const void *coef, int r, const void *us, void *out_sorted,
                              void *out_orig, int nv, bool reverse, int cheb_k)
{
    const size_t elt = d.fp64 ? 8 : 4;
    const size_t v4 = 4 * elt * static_cast<size_t>(d.S);  // one sorted T4 vector
    if (!d.parallel && nv == 2) {
        MvArgs A = mv_args(d, a, b, x, cz, z, coef, r, us, out_sorted, out_orig, nullptr, reverse);
        if (cheb_k >= 0 && d.cheb_kt > 0) {
            A.chain = static_cast<const ChainStep *>(d.chain);
            A.cheb_k = cheb_k;
            A.rcap = d.fir_rcap;
            A.coef = d.Bmix;
        }
        return d.fp64 ? launch_mvw_t<double, 2>(d, A, st) : launch_mvw_t<float, 2>(d, A, st);
    }
    // the parallel tensor (or a single vector): one mat-vec per vector
    auto at = [](const void *p, size_t off) -> const void * {
        return p ? static_cast<const void *>(static_cast<const char *>(p) + off) : nullptr;
    };
    for (int v = 0; v < nv; ++v) {
        Dev dv = d;
        dv.us = const_cast<void *>(at(us, static_cast<size_t>(v) * r * v4));
        void *os = out_sorted ? static_cast<char *>(out_sorted) + v * v4 : nullptr;
        void *oo = out_orig ? static_cast<char *>(out_orig) + static_cast<size_t>(v) * 3 * d.S * elt : nullptr;
        hipError_t e =
            launch_spmv(dv, st, a, b, at(x, v * v4), cz, at(z, v * v4), coef, r, os, oo, nullptr, reverse, cheb_k);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_cheb_select(const Dev &d, hipStream_t st)
{
    ChainSel c{};
    c.Kw = d.cheb_kw;
    c.Kt = d.cheb_kt;
    c.lam_t = d.lam_tight;
    c.lo_t = d.lam_lo_tight;
    c.aw = d.cheb_ab[0];
    c.bw = d.cheb_ab[1];
    c.at = d.cheb_ab[2];
    c.bt = d.cheb_ab[3];
    k_cheb_select<<<1, 64, 0, st>>>(c, d.d_rowmax, d.lab + 2 * kMaxCheckIters, d.d_retired,
                                    static_cast<ChainStep *>(d.chain), d.d_tight);
    return hipGetLastError();
}

template <typename T, int RMAX>
static hipError_t cheb_mix_t(const Dev &d, int r, int K, hipStream_t st)
{
    using T4 = typename V4<T>::t;
    const ChainStep *chain = d.cheb_kt > 0 ? static_cast<const ChainStep *>(d.chain) : nullptr;
    k_cheb_mix<T, RMAX><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, r, d.fir_rcap, K, static_cast<const T *>(d.Bmix),
                                                          chain, static_cast<const T4 *>(d.us),
                                                          static_cast<T4 *>(d.vk));
    return hipGetLastError();
}

hipError_t launch_cheb_mix(const Dev &d, int r, int K, hipStream_t st)
{
    if (d.fp64) {
        if (r <= 8) return cheb_mix_t<double, 8>(d, r, K, st);
        if (r <= 16) return cheb_mix_t<double, 16>(d, r, K, st);
        return cheb_mix_t<double, kMaxRank>(d, r, K, st);
    }
    if (r <= 8) return cheb_mix_t<float, 8>(d, r, K, st);
    if (r <= 16) return cheb_mix_t<float, 16>(d, r, K, st);
    return cheb_mix_t<float, kMaxRank>(d, r, K, st);
}

hipError_t launch_permute_window(const Dev &d, hipStream_t st, int r)
{
    if (d.fp64)
        k_permute_window<double><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, d.cell_sorted,
                                                                   static_cast<const double *>(d.U), r, d.fir_rcap,
                                                                   d.fir_block, fir_rows(1), d.win, d.d_step,
                                                                   static_cast<double4 *>(d.usw));
    else
        k_permute_window<float><<<blocks(d.n, 256), 256, 0, st>>>(d.n, d.S, d.cell_sorted,
                                                                  static_cast<const float *>(d.U), r, d.fir_rcap,
                                                                  d.fir_block, fir_rows(0), d.win, d.d_step,
                                                                  static_cast<float4 *>(d.usw));
    return hipGetLastError();
}

hipError_t launch_dissipative(const Dev &d, hipStream_t st, bool reverse)
{
    // F^D' = -(P Y) + Dneg, scattered to the original order
    return launch_spmv(d, st, -1.0, 0.0, d.ys, 0.0, nullptr, nullptr, 0, nullptr, d.FD, d.Dneg, reverse);
}

}  // namespace gld
