// Internal declarations of the batched engine (many independent GLD systems
// advanced together, every launch of a step covering all of them).  Not part
// of the public ABI; the C entry points are in include/gld_batch.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gld_internal.h"

namespace gld {
namespace batch {

// One Clenshaw term of a system's chain: out = a P x + b x + cz z + v_k.
struct BTerm {
    double a, b, cz;
};

// Device-resident description of one system of a batch (the per-system
// descriptor every batched kernel reads through its block map).
struct BSys {
    int64_t n, S;               // particles; component stride (multiple of 64)
    int nslots, M;              // history ring slots (m_max - 1), m_max
    int half, rank, rcap, K;    // noise: filter window, filters, padded filters, Chebyshev terms
    int bf, wlen, cap, n_r;     // filter block, white-noise ring slots, pair capacity, distance grid
    int nc[3], noff[3], ncell;  // cell grid (cells of edge >= r_cut), stencil offsets per axis
    int noise_on, has_pair;
    int lanes;                  // lanes per particle of the pair mat-vecs and the list build (1, 2, 4, 8);
                                // the pair lists are lane-interleaved: entry q of particle i at
                                // ((q / lanes) S + i) lanes + q % lanes
    double box[3];
    double dt, mass, kT, a, b, g0;
    double r_cut, r_cut_min, r0, dr, lam_hi;
    double wca_rc2, wca_s2, wca_eps;
    uint64_t seed;
    // state, double [3][S]
    double *R, *V, *FC, *FCn;
    double4 *Rw;                // wrapped positions [n]
    double4 *Rs;                // the same in cell order [n] (the list build reads candidates in order)
    // work precision T (float or double) buffers
    void *ring;                 // [nslots][3][S]
    void *Dneg, *FD, *FR;       // [3][S]
    void *wring;                // [wlen][3][S]
    void *U;                    // [2][fir_rows][3][S]
    void *Afilt;                // padded taps [fir_padded_rows][rcap]
    void *Bmix;                 // [K][rcap]
    void *ks, *gm;              // [M]
    // the mat-vec vectors are in the cell order of the last list build
    // (entry p holds particle cell_sorted[p]; particle i sits at cpos[i]),
    // so that the neighbours a particle gathers lie close together
    void *y4;                   // T4 [S]: dissipative input (cell order)
    void *cb[3];                // T4 [S]: Clenshaw vectors (cell order)
    void *vk;                   // T4 [K][S]: premixed chain inputs (cell order)
    double *wtab;               // [n_r]
    uint16_t *nbl;              // [cap / lanes][S][lanes] neighbours' cell-order positions, rows in
                                // cell order (cap a multiple of 8)
    void *nbw;                  // T, the same layout: pair weights w(R_ij)
    int *nn;                    // [S] neighbour counts, cell order
    int *cell_id, *cell_slot, *cell_count, *cell_start, *cell_list, *cell_sorted;
    int *cpos;                  // [S] cell-order position of each particle
    BTerm *terms;               // [K]
    long long *step;
    int *flags;
    long long *flag_step;
    unsigned *rowmax;
};

// block -> (system, first unit of the system) for the flat launches
struct BMap {
    int sys;
    int first;
};

constexpr int kThreads = 256;
// lanes per particle of the batched pair mat-vec
constexpr int kLaneChoices[4] = {1, 2, 4, 8};

// Launchers; all enqueue on st.  `map`/`nblocks` are the launch's flat block
// map over the systems it covers.
hipError_t b_history(int fp64, const BSys *sys, const BMap *map, int nblocks, hipStream_t st);
hipError_t b_white(int fp64, const BSys *sys, const BMap *map, int nblocks, int mode, int gy, hipStream_t st);
hipError_t b_fir(int fp64, const BSys *sys, const int2 *tiles, int ntiles, int mode, hipStream_t st);
hipError_t b_premix(int fp64, int rmax, const BSys *sys, const BMap *map, int nblocks, hipStream_t st);
// pair mat-vec of one chain term k (k >= 0; systems with k >= K skip), or the
// dissipative product (k = -1): x = cb[ix] (y4 for k = -1), z = cb[iz],
// out = cb[io] or, for k = 0, F^R ([3][S]), for k = -1, F^D' = -P y + Dneg
hipError_t b_spmv(int fp64, int lanes, const BSys *sys, const BMap *map, int nblocks, int k, int ix, int iz,
                  int io, hipStream_t st);
hipError_t b_update_r(int fp64, const BSys *sys, const BMap *map, int nblocks, hipStream_t st);
hipError_t b_update_v(int fp64, const BSys *sys, const BMap *map, int nblocks, hipStream_t st);
hipError_t b_advance(const BSys *sys, int nsys_total, hipStream_t st);
// neighbour list at the current positions (cells, pair lists, F^C into FCn
// (step) or FC (into_fc, set-up), row-sum check against lam_hi); the lists
// are built per lane class with the mat-vecs' maps smap[c] / nsblocks[c]
hipError_t b_neighbors(int fp64, const BSys *sys, const BMap *pmap, int npblocks, const BMap *cmap, int ncblocks,
                       const BMap *const *smap, const int *nsblocks, int nsys_total, int into_fc, hipStream_t st);

}  // namespace batch
}  // namespace gld
