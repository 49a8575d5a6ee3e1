// C ABI of the batched engine (include/gld_batch.h): systems placed in one
// workspace by a first-fit allocator, their one-off noise constructions on
// host threads, the flat launch maps, the per-step launch sequence (one HIP
// graph for the whole batch) and the mat-vec schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "gld.h"
#include "gld_batch.h"
#include "gld_batch_dev.h"
#include "gld_serve.h"
#include "gld_internal.h"

using gld::NoisePlan;
using gld::batch::BMap;
using gld::batch::BSys;
using gld::batch::BTerm;

namespace {

gld_status bfail(gld_status st, const std::string &msg)
{
    gld::set_last_error(msg);
    return st;
}

#define BHIP(expr)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return bfail(GLD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

#define BLAUNCH0(expr)                                                                                 \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return bfail(GLD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t up256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }
constexpr size_t kMapArena = size_t(16) << 20;  // launch maps of a batch (a few hundred KB at 256 systems)
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// First-fit allocator over [0, size) in 256-byte units.
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes
    void init(size_t bytes)
    {
        size = bytes & ~static_cast<size_t>(255);
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = up256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = up256(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

// Host-side description of one system: its parameters, noise construction
// and the layout of its workspace region.
struct Sys {
    bool used = false;
    gld_params p{};
    std::vector<double> k_self, g, w;
    NoisePlan plan;
    bool noise_on = false, has_pair = false;
    int64_t n = 0, S = 0;
    int rcap = 0, bf = 1, wlen = 4, cap = 1, nc[3] = {1, 1, 1}, noff[3] = {1, 1, 1}, ncell = 1;
    double mean_nbrs = 0, theta[2] = {0, 0};
    size_t off = 0, bytes = 0;
    BSys d{};  // device descriptor (pointers into the workspace)
};

struct Built {
    gld_status st = GLD_OK;
    std::string err;
};

}  // namespace

struct gld_batch {
    int fp64 = 0;
    int capacity = 0;
    char *base = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    Pool pool;              // the systems' regions (offsets from base)
    Pool mpool;             // launch maps (offsets from mbase)
    char *mbase = nullptr;
    std::vector<Sys> sys;
    BSys *d_sys = nullptr;  // [capacity] at the front of the workspace
    size_t front = 0;       // bytes of the descriptor table
    // launch maps (one allocation, rebuilt when the batch changes)
    size_t map_off = 0, map_bytes = 0;
    BMap *pmap = nullptr, *cmap = nullptr, *smap[4] = {nullptr, nullptr, nullptr, nullptr};
    int2 *tiles = nullptr;
    int np = 0, nc = 0, ns[4] = {0, 0, 0, 0}, ntiles = 0;
    int kmax = 0, rmax = 0, any_noise = 0;
    gld_batch_schedule sched{{24, 64, 160}};
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // per-kernel timing (eager launches with an event pair per kernel class)
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<std::pair<int, size_t>> pending;  // (class, index of the start event)
    double ms[GLD_K_COUNT] = {0};
    int64_t cnt[GLD_K_COUNT] = {0};
};

namespace {

// ---------------------------------------------------------------------------
// host set-up of one system
// ---------------------------------------------------------------------------

// Extreme Ritz values of the pair-weight matrix W = [w(R_ij)] at r (the
// spectrum of P = W (x) 1_3 for the isotropic tensor) by 60 Lanczos steps,
// its largest row sum of |w|, and the mean neighbour count.
void host_spectrum(const gld_params &p, const double *r, double theta[2], double &gmax, double &mean_nbrs)
{
    const int64_t n = p.n;
    // cell list, cells of edge >= r_cut
    int nc[3];
    for (int c = 0; c < 3; ++c) nc[c] = std::max(1, static_cast<int>(std::floor(p.box[c] / p.r_cut)));
    const int ncell = nc[0] * nc[1] * nc[2];
    std::vector<std::vector<int64_t>> cells(ncell);
    std::vector<double> rw(3 * n);
    auto cell_of = [&](const double *x) {
        int cc[3];
        for (int c = 0; c < 3; ++c) cc[c] = std::min(nc[c] - 1, std::max(0, static_cast<int>(std::floor(x[c] / p.box[c] * nc[c]))));
        return (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
    };
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) {
            double x = r[3 * i + c];
            x -= p.box[c] * std::floor(x / p.box[c]);
            if (x >= p.box[c]) x -= p.box[c];
            rw[3 * i + c] = x;
        }
        cells[cell_of(&rw[3 * i])].push_back(i);
    }
    auto weight = [&](double rr) {
        if (rr < p.r_cut_min) rr = p.r_cut_min;
        const double t = std::max((rr - p.r0) / p.dr, 0.0);
        const int b = static_cast<int>(std::max(std::min(std::floor(t), static_cast<double>(p.n_r - 2)), 0.0));
        const double f = t - b;
        return p.k_pair_w[b] * (1.0 - f) + p.k_pair_w[b + 1] * f;
    };
    std::vector<int64_t> start(n + 1, 0), nbr;
    std::vector<double> wv;
    const double rc2 = p.r_cut * p.r_cut;
    gmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int ci = cell_of(&rw[3 * i]);
        const int cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
        double rs = 0;
        const int no[3] = {std::min(nc[0], 3), std::min(nc[1], 3), std::min(nc[2], 3)};
        for (int oz = 0; oz < no[2]; ++oz)
            for (int oy = 0; oy < no[1]; ++oy)
                for (int ox = 0; ox < no[0]; ++ox) {
                    const int dx = no[0] == 3 ? ox - 1 : ox, dy = no[1] == 3 ? oy - 1 : oy, dz = no[2] == 3 ? oz - 1 : oz;
                    const int cj = (((cz + dz + nc[2]) % nc[2]) * nc[1] + (cy + dy + nc[1]) % nc[1]) * nc[0] +
                                   (cx + dx + nc[0]) % nc[0];
                    for (int64_t j : cells[cj]) {
                        if (j == i) continue;
                        double d2 = 0;
                        for (int c = 0; c < 3; ++c) {
                            double x = rw[3 * j + c] - rw[3 * i + c];
                            x -= p.box[c] * std::nearbyint(x / p.box[c]);
                            d2 += x * x;
                        }
                        if (d2 >= rc2) continue;
                        const double wij = weight(std::sqrt(d2));
                        nbr.push_back(j);
                        wv.push_back(wij);
                        rs += std::fabs(wij);
                    }
                }
        start[i + 1] = static_cast<int64_t>(nbr.size());
        gmax = std::max(gmax, rs);
    }
    mean_nbrs = n > 0 ? static_cast<double>(nbr.size()) / n : 0.0;
    // Lanczos on W (FP64, random start, no reorthogonalisation)
    const int iters = static_cast<int>(std::min<int64_t>(60, n));
    std::vector<double> q(n), qp(n, 0.0), wq(n), al, be;
    std::mt19937_64 rng(p.seed ^ 0x5eed5eedULL);
    std::normal_distribution<double> nd(0.0, 1.0);
    double nq = 0;
    for (auto &x : q) { x = nd(rng); nq += x * x; }
    nq = std::sqrt(nq);
    for (auto &x : q) x /= nq;
    double bprev = 0;
    for (int k = 0; k < iters; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            double s = 0;
            for (int64_t e = start[i]; e < start[i + 1]; ++e) s += wv[e] * q[nbr[e]];
            wq[i] = s;
        }
        double a = 0;
        for (int64_t i = 0; i < n; ++i) a += q[i] * wq[i];
        double b2 = 0;
        for (int64_t i = 0; i < n; ++i) {
            wq[i] -= a * q[i] + bprev * qp[i];
            b2 += wq[i] * wq[i];
        }
        al.push_back(a);
        const double b = std::sqrt(b2);
        be.push_back(b);
        if (!(b > 1e-300)) break;
        for (int64_t i = 0; i < n; ++i) {
            qp[i] = q[i];
            q[i] = wq[i] / b;
        }
        bprev = b;
    }
    // extreme eigenvalues of the tridiagonal by bisection on Sturm counts
    const int kk = static_cast<int>(al.size());
    auto count_below = [&](double x) {
        int c = 0;
        double dd = 1.0;
        for (int i = 0; i < kk; ++i) {
            dd = al[i] - x - (i > 0 ? be[i - 1] * be[i - 1] / dd : 0.0);
            if (dd == 0.0) dd = 1e-300;
            if (dd < 0) ++c;
        }
        return c;
    };
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < kk; ++i) {
        const double rr = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i < kk - 1 ? std::fabs(be[i]) : 0.0);
        lo = std::min(lo, al[i] - rr);
        hi = std::max(hi, al[i] + rr);
    }
    for (int which = 0; which < 2; ++which) {
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (count_below(mid) >= (which == 0 ? 1 : kk)) b = mid;
            else a = mid;
        }
        theta[which] = 0.5 * (a + b);
    }
    if (kk == 0) theta[0] = theta[1] = 0.0;
}

// Parameters, noise construction and workspace layout of one system (no
// device work): fills y and its region size.
Built build_system(int fp64, const gld_params *params, const double *r0, Sys &y)
{
    Built out;
    gld_status st = gld::validate_params(params);
    if (st != GLD_OK) {
        out.st = st;
        out.err = gld_last_error();
        return out;
    }
    auto err = [&](gld_status s, const std::string &m) {
        out.st = s;
        out.err = m;
        return out;
    };
    if ((params->precision == GLD_FP64) != (fp64 != 0)) return err(GLD_ERR_INVALID_ARG, "precision differs from the batch's");
    if (params->n > 65535) return err(GLD_ERR_INVALID_ARG, "a batched system holds at most 65535 particles");
    if (params->pair_tensor != GLD_PAIR_ISOTROPIC) return err(GLD_ERR_INVALID_ARG, "batched systems use the isotropic pair tensor");
    if (params->noise_window > 1) return err(GLD_ERR_INVALID_ARG, "batched systems use noise_window 1");
    if (params->noise_a) return err(GLD_ERR_INVALID_ARG, "batched systems build their own noise filters");
    if (!r0) return err(GLD_ERR_INVALID_ARG, "NULL positions");
    y.p = *params;
    y.k_self.assign(params->k_self, params->k_self + params->m_max);
    bool pair = params->k_pair_g != nullptr;
    if (params->k_pair) {
        if ((st = gld::separable_pair_table(params, y.w, y.g, pair)) != GLD_OK) return err(st, gld_last_error());
    } else if (pair) {
        y.g.assign(params->k_pair_g, params->k_pair_g + params->m_max);
        y.w.assign(params->k_pair_w, params->k_pair_w + params->n_r);
    }
    y.p.k_self = y.k_self.data();
    y.p.k_pair_g = pair ? y.g.data() : nullptr;
    y.p.k_pair_w = pair ? y.w.data() : nullptr;
    y.p.k_pair = nullptr;
    y.p.dk_self = nullptr;
    y.has_pair = pair;
    y.noise_on = params->kT > 0;
    y.n = params->n;
    y.S = round_up(params->n, 64);
    const gld_params &p = y.p;
    // noise construction, interval from this configuration
    double gmax = 0;
    y.mean_nbrs = 0;
    if (pair) host_spectrum(p, r0, y.theta, gmax, y.mean_nbrs);
    if (y.noise_on) {
        std::string e;
        if ((st = gld::noise_spectra(p, y.plan, e)) != GLD_OK) return err(st, e);
        const double tol = p.noise_tol > 0 ? p.noise_tol : (fp64 ? gld::kNoiseTolFp64 : gld::kNoiseTolMixed);
        double lo = p.lam_lo, hi = p.lam_hi;
        if (!(hi > lo)) {
            if (!pair) {
                lo = -1.0;
                hi = 1.0;
            } else {
                if (!(y.theta[0] > y.plan.sing_lo) || !(y.theta[1] < y.plan.sing_hi))
                    return err(GLD_ERR_NOT_PD, "initial configuration: pair-matrix spectrum reaches a singular point "
                                               "of the noise correlation: not positive definite");
                double hi_t, lo_t;
                gld::auto_interval(p, y.plan, y.theta[0], y.theta[1], gmax, lo, hi, hi_t, lo_t);
            }
        }
        if (pair && (y.theta[0] < lo || y.theta[1] > hi))
            return err(GLD_ERR_INTERVAL, "initial configuration: pair-matrix spectrum outside the noise interval");
        if ((st = gld::noise_build(p, lo, hi, tol, y.plan, e)) != GLD_OK) return err(st, e);
        y.rcap = gld::fir_rcap_for(y.plan.r);
        y.bf = gld::fir_block_for(fp64, y.rcap);
        y.wlen = std::max(4, 2 * y.plan.half + 2 * y.bf);
    }
    // geometry: pair capacity and cells
    const double vol = p.box[0] * p.box[1] * p.box[2];
    if (p.max_neighbors > 0) {
        y.cap = p.max_neighbors;
    } else {
        const double expect = static_cast<double>(p.n) / vol * (4.0 / 3.0) * M_PI * p.r_cut * p.r_cut * p.r_cut;
        y.cap = static_cast<int>(round_up(static_cast<int64_t>(1.5 * std::max(expect, y.mean_nbrs) + 32), 8));
    }
    y.cap = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(y.cap, std::max<int64_t>(1, p.n - 1))));
    y.ncell = 1;
    for (int c = 0; c < 3; ++c) {
        y.nc[c] = std::max(1, static_cast<int>(std::floor(p.box[c] / p.r_cut)));
        y.noff[c] = std::min(y.nc[c], 3);
        y.ncell *= y.nc[c];
    }
    // region size
    const size_t elt = fp64 ? 8 : 4, S = static_cast<size_t>(y.S), vec = 3 * S;
    const int M = p.m_max, nslots = std::max(0, M - 1);
    const int K = y.noise_on ? y.plan.K : 0;
    size_t sz = 0;
    auto take = [&](size_t b) { sz = up256(sz) + b; };
    for (int k = 0; k < 4; ++k) take(vec * 8);  // R V FC FCn
    take(S * 32);                                // Rw
    take(S * 32);                                // Rs
    take(static_cast<size_t>(nslots) * vec * elt);
    for (int k = 0; k < 3; ++k) take(vec * elt);  // Dneg FD FR
    if (y.noise_on) {
        take(static_cast<size_t>(y.wlen) * vec * elt);
        take(2 * static_cast<size_t>(gld::fir_rows(fp64)) * vec * elt);
        take(gld::fir_padded_rows(y.plan.half, y.bf) * y.rcap * elt);
        take(static_cast<size_t>(K) * y.rcap * elt);
        take(static_cast<size_t>(K) * 4 * S * elt);  // vk
        take(static_cast<size_t>(K) * sizeof(BTerm));
    }
    take(static_cast<size_t>(M) * elt);  // ks
    take(static_cast<size_t>(M) * elt);  // gm
    for (int k = 0; k < 4; ++k) take(4 * S * elt);  // y4 cb0-2
    take(static_cast<size_t>(p.n_r) * 8);
    take(static_cast<size_t>(y.cap) * S * 2);
    take(static_cast<size_t>(y.cap) * S * elt);
    take(S * 4);                        // nn
    for (int k = 0; k < 5; ++k) take(S * 4);  // cell id, slot, list, sorted, cpos
    take(static_cast<size_t>(y.ncell) * 4);
    take(static_cast<size_t>(y.ncell + 1) * 4);
    for (int k = 0; k < 4; ++k) take(8);  // step flags flag_step rowmax
    y.bytes = up256(sz) + 256;
    return out;
}

// Pointers of a system's descriptor in its region (base = workspace + off).
void carve_system(int fp64, Sys &y, char *base)
{
    const size_t elt = fp64 ? 8 : 4, S = static_cast<size_t>(y.S), vec = 3 * S;
    const gld_params &p = y.p;
    const int M = p.m_max, nslots = std::max(0, M - 1);
    const int K = y.noise_on ? y.plan.K : 0;
    size_t off = 0;
    auto take = [&](size_t b) -> char * {
        off = up256(off);
        char *r = base + off;
        off += b;
        return r;
    };
    BSys &d = y.d;
    d = BSys{};
    d.R = reinterpret_cast<double *>(take(vec * 8));
    d.V = reinterpret_cast<double *>(take(vec * 8));
    d.FC = reinterpret_cast<double *>(take(vec * 8));
    d.FCn = reinterpret_cast<double *>(take(vec * 8));
    d.Rw = reinterpret_cast<double4 *>(take(S * 32));
    d.Rs = reinterpret_cast<double4 *>(take(S * 32));
    d.ring = take(static_cast<size_t>(nslots) * vec * elt);
    d.Dneg = take(vec * elt);
    d.FD = take(vec * elt);
    d.FR = take(vec * elt);
    if (y.noise_on) {
        d.wring = take(static_cast<size_t>(y.wlen) * vec * elt);
        d.U = take(2 * static_cast<size_t>(gld::fir_rows(fp64)) * vec * elt);
        d.Afilt = take(gld::fir_padded_rows(y.plan.half, y.bf) * y.rcap * elt);
        d.Bmix = take(static_cast<size_t>(K) * y.rcap * elt);
        d.vk = take(static_cast<size_t>(K) * 4 * S * elt);
        d.terms = reinterpret_cast<BTerm *>(take(static_cast<size_t>(K) * sizeof(BTerm)));
    }
    d.ks = take(static_cast<size_t>(M) * elt);
    d.gm = take(static_cast<size_t>(M) * elt);
    d.y4 = take(4 * S * elt);
    for (auto &c : d.cb) c = take(4 * S * elt);
    d.wtab = reinterpret_cast<double *>(take(static_cast<size_t>(p.n_r) * 8));
    d.nbl = reinterpret_cast<uint16_t *>(take(static_cast<size_t>(y.cap) * S * 2));
    d.nbw = take(static_cast<size_t>(y.cap) * S * elt);
    d.nn = reinterpret_cast<int *>(take(S * 4));
    d.cell_id = reinterpret_cast<int *>(take(S * 4));
    d.cell_slot = reinterpret_cast<int *>(take(S * 4));
    d.cell_list = reinterpret_cast<int *>(take(S * 4));
    d.cell_sorted = reinterpret_cast<int *>(take(S * 4));
    d.cpos = reinterpret_cast<int *>(take(S * 4));
    d.cell_count = reinterpret_cast<int *>(take(static_cast<size_t>(y.ncell) * 4));
    d.cell_start = reinterpret_cast<int *>(take(static_cast<size_t>(y.ncell + 1) * 4));
    d.step = reinterpret_cast<long long *>(take(8));
    d.flags = reinterpret_cast<int *>(take(8));
    d.flag_step = reinterpret_cast<long long *>(take(8));
    d.rowmax = reinterpret_cast<unsigned *>(take(8));
    // scalars
    d.n = y.n;
    d.S = y.S;
    d.nslots = nslots;
    d.M = M;
    d.half = y.noise_on ? y.plan.half : 0;
    d.rank = y.noise_on ? y.plan.r : 0;
    d.rcap = y.rcap;
    d.K = K;
    d.bf = y.bf;
    d.wlen = y.wlen;
    d.cap = y.cap;
    d.n_r = p.n_r;
    for (int c = 0; c < 3; ++c) {
        d.nc[c] = y.nc[c];
        d.noff[c] = y.noff[c];
        d.box[c] = p.box[c];
    }
    d.ncell = y.ncell;
    d.noise_on = y.noise_on ? 1 : 0;
    d.has_pair = y.has_pair ? 1 : 0;
    d.dt = p.dt;
    d.mass = p.mass;
    d.kT = p.kT;
    const double x = p.dt * p.k_self[0] / (2.0 * p.mass);  // eq. (aa-bb), isotropic K^s_0
    d.b = 1.0 / (1.0 + x);
    d.a = d.b * (1.0 - x);
    d.g0 = y.has_pair ? p.k_pair_g[0] : 0.0;
    d.r_cut = p.r_cut;
    d.r_cut_min = p.r_cut_min;
    d.r0 = p.r0;
    d.dr = p.dr;
    d.lam_hi = (y.noise_on && y.has_pair) ? y.plan.hi : std::numeric_limits<double>::infinity();
    const double rw = std::pow(2.0, 1.0 / 6.0) * p.wca_sigma;
    d.wca_rc2 = p.wca_eps != 0.0 ? rw * rw : 0.0;
    d.wca_s2 = p.wca_sigma * p.wca_sigma;
    d.wca_eps = p.wca_eps;
    d.seed = p.seed;
}

template <typename T>
std::vector<T> to_work(const std::vector<double> &v)
{
    return std::vector<T>(v.begin(), v.end());
}

gld_status put(hipStream_t st, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return GLD_OK;
    BHIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return GLD_OK;
}

// host [n][3] -> device [3][S] of T
template <typename T>
gld_status put_vec(hipStream_t st, int64_t n, int64_t S, void *dst, const double *src, std::vector<T> &stage)
{
    stage.assign(3 * S, T(0));
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) stage[c * S + i] = static_cast<T>(src[3 * i + c]);
    BHIP(hipMemcpyAsync(dst, stage.data(), stage.size() * sizeof(T), hipMemcpyHostToDevice, st));
    BHIP(hipStreamSynchronize(st));
    return GLD_OK;
}

template <typename T>
gld_status get_vec(hipStream_t st, int64_t n, int64_t S, double *dst, const void *src)
{
    std::vector<T> h(3 * S);
    BHIP(hipMemcpyAsync(h.data(), src, h.size() * sizeof(T), hipMemcpyDeviceToHost, st));
    BHIP(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) dst[3 * i + c] = static_cast<double>(h[c * S + i]);
    return GLD_OK;
}

// the tables of a system (taps, mixing weights, chain terms, kernels, w)
template <typename T>
gld_status upload_tables(gld_batch *b, Sys &y)
{
    hipStream_t st = b->st;
    const BSys &d = y.d;
    const gld_params &p = y.p;
    std::vector<T> ks = to_work<T>(y.k_self), gm(p.m_max, T(0));
    if (y.has_pair)
        for (int m = 0; m < p.m_max; ++m) gm[m] = static_cast<T>(y.g[m]);
    std::vector<double> wt(p.n_r, 0.0);
    if (y.has_pair) wt = y.w;
    gld_status s;
    if ((s = put(st, d.ks, ks.data(), ks.size() * sizeof(T))) != GLD_OK) return s;
    if ((s = put(st, d.gm, gm.data(), gm.size() * sizeof(T))) != GLD_OK) return s;
    if ((s = put(st, d.wtab, wt.data(), wt.size() * 8)) != GLD_OK) return s;
    std::vector<T> A, B;
    std::vector<BTerm> terms;
    if (y.noise_on) {
        const NoisePlan &pl = y.plan;
        const int front = y.bf - 1, Pw = 2 * pl.half + 1;
        A.assign(gld::fir_padded_rows(pl.half, y.bf) * y.rcap, T(0));
        for (int q = 0; q < pl.r; ++q)
            for (int t = 0; t < Pw; ++t)
                A[static_cast<size_t>(t + front) * y.rcap + q] =
                    static_cast<T>(pl.Afilt[static_cast<size_t>(q) * pl.P + (pl.M - 1 - pl.half) + t]);
        B.assign(static_cast<size_t>(pl.K) * y.rcap, T(0));
        for (int k = 0; k < pl.K; ++k)
            for (int q = 0; q < pl.r; ++q) B[static_cast<size_t>(k) * y.rcap + q] = static_cast<T>(pl.Bmix[static_cast<size_t>(k) * pl.r + q]);
        // Clenshaw: b_{K-1} = v_{K-1}; b_k = v_k + 2 P~ b_{k+1} - b_{k+2}; F = v_0 + P~ b_1 - b_2
        const int K = pl.K;
        terms.resize(K);
        for (int k = 0; k < K; ++k) {
            if (k == K - 1) terms[k] = BTerm{0.0, 0.0, 0.0};
            else if (k >= 1) terms[k] = BTerm{2.0 * pl.alpha, 2.0 * pl.beta, k == K - 2 ? 0.0 : -1.0};
            else terms[k] = BTerm{pl.alpha, pl.beta, K == 2 ? 0.0 : -1.0};
        }
        if ((s = put(st, d.Afilt, A.data(), A.size() * sizeof(T))) != GLD_OK) return s;
        if ((s = put(st, d.Bmix, B.data(), B.size() * sizeof(T))) != GLD_OK) return s;
        if ((s = put(st, d.terms, terms.data(), terms.size() * sizeof(BTerm))) != GLD_OK) return s;
    }
    BHIP(hipStreamSynchronize(st));  // the staging vectors go out of scope
    return GLD_OK;
}

// ---------------------------------------------------------------------------
// launch maps
// ---------------------------------------------------------------------------
int lanes_for(const gld_batch_schedule &s, double mean_nbrs)
{
    if (mean_nbrs < s.lanes_threshold[0]) return 1;
    if (mean_nbrs < s.lanes_threshold[1]) return 2;
    if (mean_nbrs < s.lanes_threshold[2]) return 4;
    return 8;
}

int lane_class(int lanes) { return lanes == 1 ? 0 : (lanes == 2 ? 1 : (lanes == 4 ? 2 : 3)); }

// particle maps (blocks of `per` particles) of the given systems
void part_map(const gld_batch *b, const std::vector<int> &which, int per, std::vector<BMap> &out)
{
    for (int s : which) {
        const int64_t n = b->sys[s].n;
        for (int64_t f = 0; f < n; f += per) out.push_back(BMap{s, static_cast<int>(f)});
    }
}

// filter-bank tiles: mode 0, the step's share (1/bf of the channels); else the whole product
void fir_tiles(const gld_batch *b, const std::vector<int> &which, int mode, std::vector<int2> &out)
{
    for (int s : which) {
        const Sys &y = b->sys[s];
        if (!y.noise_on) continue;
        const int64_t M = 3 * y.S;
        const int nslice = y.bf / gld::fir_period(y.bf);
        const int64_t cs = mode == 0 ? (M / nslice + 1 + 255) / 256 * 256 : M;
        const int nt = static_cast<int>((cs + 255) / 256);
        for (int t = 0; t < nt; ++t) out.push_back(int2{s, t});
    }
}

struct HostMaps {
    std::vector<BMap> p, c, sl[4];
    std::vector<int2> t;
};

// The blocks of the pair mat-vecs and list builds of one lane class, in an
// XCD-aware order: the GPU hands work-group b to XCD b mod 8, so each system
// is given to one XCD (largest pair work first, to the least loaded XCD) and
// its blocks are placed at indices of that residue; the input vectors its
// mat-vecs gather then stay in that XCD's L2.  Shorter XCD lists are padded
// with empty blocks (sys -1).
void xcd_map(const gld_batch *b, const std::vector<int> &cls, int per, std::vector<BMap> &out)
{
    constexpr int kXcd = 8;
    std::vector<int> order(cls);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        const double wx = b->sys[x].n * (1.0 + b->sys[x].mean_nbrs), wy = b->sys[y].n * (1.0 + b->sys[y].mean_nbrs);
        return wx > wy || (wx == wy && x < y);
    });
    std::vector<std::vector<BMap>> bins(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (int s : order) {
        const int x = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        const int64_t n = b->sys[s].n;
        for (int64_t f = 0; f < n; f += per) bins[x].push_back(BMap{s, static_cast<int>(f)});
        load[x] += b->sys[s].n * (1.0 + b->sys[s].mean_nbrs);
    }
    size_t longest = 0;
    for (auto &v : bins) longest = std::max(longest, v.size());
    for (size_t j = 0; j < longest; ++j)
        for (int x = 0; x < kXcd; ++x) out.push_back(j < bins[x].size() ? bins[x][j] : BMap{-1, 0});
}

void make_maps(const gld_batch *b, const std::vector<int> &which, HostMaps &h, int fir_mode)
{
    part_map(b, which, gld::batch::kThreads, h.p);
    for (int s : which) {
        const int nc = b->sys[s].ncell;
        for (int f = 0; f < nc; f += gld::batch::kThreads) h.c.push_back(BMap{s, f});
    }
    for (int k = 0; k < 4; ++k) {
        std::vector<int> cls;
        for (int s : which)
            if (lane_class(lanes_for(b->sched, b->sys[s].mean_nbrs)) == k) cls.push_back(s);
        xcd_map(b, cls, gld::batch::kThreads / gld::batch::kLaneChoices[k], h.sl[k]);
    }
    fir_tiles(b, which, fir_mode, h.t);
}

// one allocation holding the maps; returns its offset/bytes
gld_status upload_maps(gld_batch *b, const HostMaps &h, size_t &off, size_t &bytes, BMap *&pm, BMap *&cm,
                       BMap *(&sm)[4], int2 *&tl)
{
    size_t sz = up256(h.p.size() * sizeof(BMap)) + up256(h.c.size() * sizeof(BMap)) + up256(h.t.size() * sizeof(int2));
    for (auto &v : h.sl) sz += up256(v.size() * sizeof(BMap));
    sz += 256;
    if (!b->mpool.alloc(sz, off)) return bfail(GLD_ERR_OOM, "no room left for the batch's launch maps");
    bytes = sz;
    char *base = b->mbase + off;
    size_t o = 0;
    auto place = [&](const void *src, size_t n) -> char * {
        char *r = base + o;
        if (n) (void)hipMemcpyAsync(r, src, n, hipMemcpyHostToDevice, b->st);
        o += up256(n);
        return r;
    };
    pm = reinterpret_cast<BMap *>(place(h.p.data(), h.p.size() * sizeof(BMap)));
    cm = reinterpret_cast<BMap *>(place(h.c.data(), h.c.size() * sizeof(BMap)));
    for (int k = 0; k < 4; ++k) sm[k] = reinterpret_cast<BMap *>(place(h.sl[k].data(), h.sl[k].size() * sizeof(BMap)));
    tl = reinterpret_cast<int2 *>(place(h.t.data(), h.t.size() * sizeof(int2)));
    BHIP(hipStreamSynchronize(b->st));
    return GLD_OK;
}

std::vector<int> active(const gld_batch *b)
{
    std::vector<int> a;
    for (int s = 0; s < b->capacity; ++s)
        if (b->sys[s].used) a.push_back(s);
    return a;
}

void drop_graph(gld_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

// the batch's maps and chain length after a change of its systems or schedule
gld_status rebuild(gld_batch *b)
{
    drop_graph(b);
    if (b->map_bytes) b->mpool.release(b->map_off, b->map_bytes);
    b->map_bytes = 0;
    HostMaps h;
    const std::vector<int> a = active(b);
    make_maps(b, a, h, 0);
    gld_status s = upload_maps(b, h, b->map_off, b->map_bytes, b->pmap, b->cmap, b->smap, b->tiles);
    if (s != GLD_OK) return s;
    b->np = static_cast<int>(h.p.size());
    b->nc = static_cast<int>(h.c.size());
    for (int k = 0; k < 4; ++k) b->ns[k] = static_cast<int>(h.sl[k].size());
    b->ntiles = static_cast<int>(h.t.size());
    b->kmax = 0;
    b->rmax = 1;
    b->any_noise = 0;
    bool relayout = false;
    for (int s2 : a) {
        Sys &y = b->sys[s2];
        const int lanes = lanes_for(b->sched, y.mean_nbrs);
        if (lanes != y.d.lanes) {
            y.d.lanes = lanes;
            BHIP(hipMemcpyAsync(b->d_sys + s2, &y.d, sizeof(BSys), hipMemcpyHostToDevice, b->st));
            relayout = true;
        }
        if (!y.noise_on) continue;
        b->any_noise = 1;
        b->kmax = std::max(b->kmax, y.plan.K);
        b->rmax = std::max(b->rmax, y.plan.r);
    }
    if (relayout) {
        // the pair lists of the current positions again, in the new lane
        // layout (F^C into the scratch FCn, as in a step)
        const BMap *sm[4] = {b->smap[0], b->smap[1], b->smap[2], b->smap[3]};
        BLAUNCH0(gld::batch::b_neighbors(b->fp64, b->d_sys, b->pmap, b->np, b->cmap, b->nc, sm, b->ns, b->capacity, 0,
                                         b->st));
        BHIP(hipStreamSynchronize(b->st));
    }
    b->dirty = false;
    return GLD_OK;
}

// ---------------------------------------------------------------------------
// the step
// ---------------------------------------------------------------------------
#define BLAUNCH(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return bfail(GLD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// event pair around a stretch of launches of one kernel class (timing mode)
struct Timed {
    gld_batch *b;
    int cls;
    size_t ix = 0;
    Timed(gld_batch *bb, int c) : b(bb), cls(c)
    {
        if (!b->timing) return;
        ix = b->ev.size();
        for (int k = 0; k < 2; ++k) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            b->ev.push_back(e);
        }
        (void)hipEventRecord(b->ev[ix], b->st);
    }
    ~Timed()
    {
        if (!b->timing) return;
        (void)hipEventRecord(b->ev[ix + 1], b->st);
        b->pending.emplace_back(cls, ix);
    }
};

// the pair mat-vecs of one step: the dissipative product and the chain
gld_status enqueue_pairs(gld_batch *b)
{
    using namespace gld::batch;
    const int f = b->fp64;
    {
        Timed t(b, GLD_K_DISSIPATIVE);
        for (int c = 0; c < 4; ++c)
            BLAUNCH(b_spmv(f, kLaneChoices[c], b->d_sys, b->smap[c], b->ns[c], -1, 0, 0, 0, b->st));
    }
    if (!b->any_noise) return GLD_OK;
    Timed t(b, GLD_K_NOISE_SPMV);
    int prev1 = -1, prev2 = -1;
    for (int k = b->kmax - 1; k >= 0; --k) {
        int out = 0;
        while (out == prev1 || out == prev2) ++out;
        const int ix = prev1 < 0 ? 0 : prev1, iz = prev2 < 0 ? 0 : prev2;
        for (int c = 0; c < 4; ++c)
            BLAUNCH(b_spmv(f, kLaneChoices[c], b->d_sys, b->smap[c], b->ns[c], k, ix, iz, k > 0 ? out : 0, b->st));
        prev2 = prev1;
        prev1 = out;
    }
    return GLD_OK;
}

gld_status enqueue_step(gld_batch *b)
{
    using namespace gld::batch;
    const int f = b->fp64;
    hipStream_t st = b->st;
    {
        Timed t(b, GLD_K_HISTORY);
        BLAUNCH(b_history(f, b->d_sys, b->pmap, b->np, st));
    }
    if (b->any_noise) {
        {
            Timed t(b, GLD_K_NOISE_FIR);
            BLAUNCH(b_white(f, b->d_sys, b->pmap, b->np, 0, 1, st));
            BLAUNCH(b_fir(f, b->d_sys, b->tiles, b->ntiles, 0, st));
        }
        Timed t(b, GLD_K_NOISE_SETUP);
        BLAUNCH(b_premix(f, b->rmax, b->d_sys, b->pmap, b->np, st));
    }
    gld_status s = enqueue_pairs(b);
    if (s != GLD_OK) return s;
    {
        Timed t(b, GLD_K_UPDATE);
        BLAUNCH(b_update_r(f, b->d_sys, b->pmap, b->np, st));
    }
    {
        Timed t(b, GLD_K_NEIGHBOR);
        const BMap *sm[4] = {b->smap[0], b->smap[1], b->smap[2], b->smap[3]};
        BLAUNCH(b_neighbors(f, b->d_sys, b->pmap, b->np, b->cmap, b->nc, sm, b->ns, b->capacity, 0, st));
    }
    Timed t(b, GLD_K_UPDATE);
    BLAUNCH(b_update_v(f, b->d_sys, b->pmap, b->np, st));
    BLAUNCH(b_advance(b->d_sys, b->capacity, st));
    return GLD_OK;
}

// Device set-up of the systems `which` at their current step (after their
// state is on the device): F^C and the pair lists, the white-noise ring and
// the filter outputs of the current and the next block.
gld_status prime(gld_batch *b, const std::vector<int> &which)
{
    using namespace gld::batch;
    HostMaps h, h2;
    make_maps(b, which, h, 1);
    size_t off = 0, bytes = 0;
    BMap *pm, *cm, *sm[4];
    int2 *tl;
    gld_status s = upload_maps(b, h, off, bytes, pm, cm, sm, tl);
    if (s != GLD_OK) return s;
    const int f = b->fp64;
    hipStream_t st = b->st;
    const int np = static_cast<int>(h.p.size()), nt = static_cast<int>(h.t.size());
    int gy = 1;
    for (int w : which)
        if (b->sys[w].noise_on) gy = std::max(gy, 2 * b->sys[w].plan.half + 2 * b->sys[w].bf);
    const BMap *smp[4] = {sm[0], sm[1], sm[2], sm[3]};
    int nsp[4];
    for (int k = 0; k < 4; ++k) nsp[k] = static_cast<int>(h.sl[k].size());
    BLAUNCH(b_neighbors(f, b->d_sys, pm, np, cm, static_cast<int>(h.c.size()), smp, nsp, b->capacity, 1, st));
    BLAUNCH(b_white(f, b->d_sys, pm, np, 1, gy, st));
    BLAUNCH(b_fir(f, b->d_sys, tl, nt, 1, st));
    BLAUNCH(b_white(f, b->d_sys, pm, np, 2, gy, st));
    // the next block's outputs once past a block's first step (whose own
    // white-noise slice completes that block's window)
    std::vector<int> mid;
    for (int w : which) {
        const Sys &y = b->sys[w];
        long long stp = 0;
        BHIP(hipMemcpyAsync(&stp, y.d.step, 8, hipMemcpyDeviceToHost, st));
        BHIP(hipStreamSynchronize(st));
        if (y.noise_on && stp % y.bf != 0) mid.push_back(w);
    }
    if (!mid.empty()) {
        fir_tiles(b, mid, 2, h2.t);
        size_t o2 = 0, b2 = 0;
        BMap *pm2, *cm2, *sm2[4];
        int2 *tl2;
        if ((s = upload_maps(b, h2, o2, b2, pm2, cm2, sm2, tl2)) != GLD_OK) {
            b->mpool.release(off, bytes);
            return s;
        }
        BLAUNCH(b_fir(f, b->d_sys, tl2, static_cast<int>(h2.t.size()), 2, st));
        BHIP(hipStreamSynchronize(st));
        b->mpool.release(o2, b2);
    }
    BHIP(hipStreamSynchronize(st));
    b->mpool.release(off, bytes);
    return GLD_OK;
}

// Install a prepared system in slot s at workspace offset off (state at
// step 0 from r0, v0; zero history); the caller primes it.
gld_status place(gld_batch *b, Sys &&src, size_t off, int s, const double *r0, const double *v0)
{
    gld_status st;
    Sys &y = b->sys[s];
    y = std::move(src);
    // the copies of the tables now live in y: re-point the parameters
    y.p.k_self = y.k_self.data();
    y.p.k_pair_g = y.has_pair ? y.g.data() : nullptr;
    y.p.k_pair_w = y.has_pair ? y.w.data() : nullptr;
    y.off = off;
    y.used = true;
    char *base = b->base + y.off;
    BHIP(hipMemsetAsync(base, 0, y.bytes, b->st));
    carve_system(b->fp64, y, base);
    y.d.lanes = lanes_for(b->sched, y.mean_nbrs);
    if ((st = b->fp64 ? upload_tables<double>(b, y) : upload_tables<float>(b, y)) != GLD_OK) return st;
    std::vector<double> dstage;
    if ((st = put_vec<double>(b->st, y.n, y.S, y.d.R, r0, dstage)) != GLD_OK) return st;
    if ((st = put_vec<double>(b->st, y.n, y.S, y.d.V, v0, dstage)) != GLD_OK) return st;
    BHIP(hipMemcpyAsync(b->d_sys + s, &y.d, sizeof(BSys), hipMemcpyHostToDevice, b->st));
    BHIP(hipStreamSynchronize(b->st));
    return GLD_OK;
}

gld_status read_flags_of(gld_batch *b, const Sys &y, int &flags, long long &fstep)
{
    int fl[2] = {0, 0};
    BHIP(hipStreamSynchronize(b->st));
    BHIP(hipMemcpy(fl, y.d.flags, sizeof(fl), hipMemcpyDeviceToHost));
    BHIP(hipMemcpy(&fstep, y.d.flag_step, sizeof(fstep), hipMemcpyDeviceToHost));
    flags = fl[0];
    return GLD_OK;
}

}  // namespace

extern "C" {

gld_status gld_batch_base_size(int32_t capacity, size_t *bytes)
{
    if (capacity < 1 || capacity > (1 << 20) || !bytes) return bfail(GLD_ERR_INVALID_ARG, "capacity must be in [1, 2^20]");
    // descriptors and the arena of the launch maps
    *bytes = up256(static_cast<size_t>(capacity) * sizeof(BSys)) + kMapArena;
    return GLD_OK;
}

gld_status gld_batch_create(int32_t precision, int32_t capacity, void *d_workspace, size_t workspace_bytes,
                            void *hip_stream, gld_batch **out)
{
    if (!out || !d_workspace) return bfail(GLD_ERR_INVALID_ARG, "NULL argument");
    if (precision != GLD_FP64 && precision != GLD_FP32_MIXED) return bfail(GLD_ERR_INVALID_ARG, "unknown precision");
    size_t base_need = 0;
    gld_status st = gld_batch_base_size(capacity, &base_need);
    if (st != GLD_OK) return st;
    if (workspace_bytes < base_need + 256) return bfail(GLD_ERR_OOM, "workspace smaller than the batch's own tables");
    gld_batch *b = new gld_batch();
    b->fp64 = precision == GLD_FP64;
    b->capacity = capacity;
    char *base = static_cast<char *>(d_workspace);
    const size_t skew = (256 - (reinterpret_cast<uintptr_t>(base) & 255)) & 255;
    b->base = base + skew;
    b->bytes = workspace_bytes - skew;
    b->st = static_cast<hipStream_t>(hip_stream);
    b->sys.resize(capacity);
    b->front = up256(static_cast<size_t>(capacity) * sizeof(BSys));
    b->d_sys = reinterpret_cast<BSys *>(b->base);
    // [descriptors][map arena][systems' pool]
    b->mbase = b->base + b->front;
    b->mpool.init(kMapArena);
    b->pool.init(b->bytes - b->front - kMapArena);
    b->base += b->front + kMapArena;
    if (hipMemsetAsync(b->d_sys, 0, b->front, b->st) != hipSuccess || hipStreamSynchronize(b->st) != hipSuccess) {
        delete b;
        return bfail(GLD_ERR_DEVICE, "descriptor table clear failed");
    }
    *out = b;
    return GLD_OK;
}

gld_status gld_batch_footprint(const gld_batch *b, const gld_params *params, const double *r0, size_t *bytes)
{
    if (!b || !params || !bytes) return bfail(GLD_ERR_INVALID_ARG, "NULL argument");
    Sys y;
    Built r = build_system(b->fp64, params, r0, y);
    if (r.st != GLD_OK) return bfail(r.st, r.err);
    *bytes = y.bytes;
    return GLD_OK;
}

gld_status gld_batch_add(gld_batch *b, int32_t count, const gld_params *const *params, const double *const *r0,
                         const double *const *v0, int32_t *slots, int32_t *status)
{
    if (!b || count < 0 || (count > 0 && (!params || !r0 || !v0 || !slots)))
        return bfail(GLD_ERR_INVALID_ARG, "NULL argument");
    if (count == 0) return GLD_OK;
    std::vector<Built> res(count);
    std::vector<Sys> ys(count);
    for (int i = 0; i < count; ++i) {
        slots[i] = -1;
        if (!params[i] || !r0[i] || !v0[i]) {
            res[i] = Built{GLD_ERR_INVALID_ARG, "NULL system argument"};
            continue;
        }
        for (int64_t e = 0; e < 3 * params[i]->n; ++e)
            if (!std::isfinite(r0[i][e]) || !std::isfinite(v0[i][e])) {
                res[i] = Built{GLD_ERR_NONFINITE, "initial state not finite"};
                break;
            }
    }
    // host constructions on parallel threads
    // host threads: OMP_NUM_THREADS when set (the host's share of cores), else
    // the hardware's, at most 16
    int hw = static_cast<int>(std::thread::hardware_concurrency());
    if (const char *e = std::getenv("OMP_NUM_THREADS")) hw = std::max(1, std::atoi(e));
    const int nth = std::max(1, std::min({count, hw, 16}));
    {
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                for (int i = t; i < count; i += nth)
                    if (res[i].st == GLD_OK) res[i] = build_system(b->fp64, params[i], r0[i], ys[i]);
            });
        for (auto &x : th) x.join();
    }
    gld_status first = GLD_OK;
    std::string first_msg;
    std::vector<int> placed;
    int next_slot = 0;
    for (int i = 0; i < count; ++i) {
        gld_status st = res[i].st;
        std::string msg = res[i].err;
        size_t off = 0;
        if (st == GLD_OK) {
            while (next_slot < b->capacity && b->sys[next_slot].used) ++next_slot;
            if (next_slot >= b->capacity) {
                st = GLD_ERR_OOM;
                msg = "no free system slot in the batch";
            } else if (!b->pool.alloc(ys[i].bytes, off)) {
                st = GLD_ERR_OOM;
                msg = "needs " + std::to_string(ys[i].bytes) + " workspace bytes; the largest free piece holds " +
                      std::to_string(b->pool.largest());
            }
        }
        if (status) status[i] = st;
        if (st != GLD_OK) {
            if (first == GLD_OK) {
                first = st;
                first_msg = "system " + std::to_string(i) + ": " + msg;
            }
            continue;
        }
        const int s = next_slot;
        if ((st = place(b, std::move(ys[i]), off, s, r0[i], v0[i])) != GLD_OK) return st;
        slots[i] = s;
        placed.push_back(s);
    }
    if (!placed.empty()) {
        gld_status st = prime(b, placed);
        if (st != GLD_OK) return st;
        b->dirty = true;
    }
    if (first != GLD_OK) return bfail(first, first_msg);
    return GLD_OK;
}

gld_status gld_batch_remove(gld_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->capacity || !b->sys[slot].used) return bfail(GLD_ERR_INVALID_ARG, "no such system");
    BHIP(hipStreamSynchronize(b->st));
    Sys &y = b->sys[slot];
    b->pool.release(y.off, y.bytes);
    y = Sys{};
    const BSys zero{};
    BHIP(hipMemcpyAsync(b->d_sys + slot, &zero, sizeof(BSys), hipMemcpyHostToDevice, b->st));
    BHIP(hipStreamSynchronize(b->st));
    b->dirty = true;
    return GLD_OK;
}

gld_status gld_batch_step(gld_batch *b, int64_t n_steps)
{
    if (!b || n_steps < 0) return bfail(GLD_ERR_INVALID_ARG, "bad batch or step count");
    gld_status st;
    if (b->dirty && (st = rebuild(b)) != GLD_OK) return st;
    if (b->np == 0 || n_steps == 0) return GLD_OK;
    if (!b->gexec && b->st) {
        BHIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeRelaxed));
        st = enqueue_step(b);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->st, &g);
        if (st != GLD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return bfail(GLD_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        b->graph = g;
        BHIP(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    }
    for (int64_t k = 0; k < n_steps; ++k) {
        if (b->gexec && !b->timing) BHIP(hipGraphLaunch(b->gexec, b->st));
        else if ((st = enqueue_step(b)) != GLD_OK) return st;
    }
    return GLD_OK;
}

gld_status gld_batch_set_timing(gld_batch *b, int enable)
{
    if (!b) return bfail(GLD_ERR_INVALID_ARG, "NULL batch");
    BHIP(hipStreamSynchronize(b->st));
    for (auto e : b->ev) (void)hipEventDestroy(e);
    b->ev.clear();
    b->pending.clear();
    for (int k = 0; k < GLD_K_COUNT; ++k) {
        b->ms[k] = 0;
        b->cnt[k] = 0;
    }
    b->timing = enable != 0;
    return GLD_OK;
}

gld_status gld_batch_kernel_times(gld_batch *b, double *ms_sum, int64_t *launches)
{
    if (!b || !ms_sum || !launches) return bfail(GLD_ERR_INVALID_ARG, "NULL argument");
    BHIP(hipStreamSynchronize(b->st));
    for (auto &[cls, ix] : b->pending) {
        float ms = 0;
        BHIP(hipEventElapsedTime(&ms, b->ev[ix], b->ev[ix + 1]));
        b->ms[cls] += ms;
        b->cnt[cls] += 1;
    }
    b->pending.clear();
    for (int k = 0; k < GLD_K_COUNT; ++k) {
        ms_sum[k] = b->ms[k];
        launches[k] = b->cnt[k];
    }
    return GLD_OK;
}

gld_status gld_batch_sync(gld_batch *b)
{
    if (!b) return bfail(GLD_ERR_INVALID_ARG, "NULL batch");
    BHIP(hipStreamSynchronize(b->st));
    return GLD_OK;
}

gld_status gld_batch_read_state(gld_batch *b, int32_t slot, gld_state *o)
{
    if (!b || !o || slot < 0 || slot >= b->capacity || !b->sys[slot].used)
        return bfail(GLD_ERR_INVALID_ARG, "no such system");
    const Sys &y = b->sys[slot];
    const BSys &d = y.d;
    gld_status st;
    BHIP(hipStreamSynchronize(b->st));
    auto work = [&](double *dst, const void *src) {
        return b->fp64 ? get_vec<double>(b->st, y.n, y.S, dst, src) : get_vec<float>(b->st, y.n, y.S, dst, src);
    };
    if (o->r && (st = get_vec<double>(b->st, y.n, y.S, o->r, d.R)) != GLD_OK) return st;
    if (o->v && (st = get_vec<double>(b->st, y.n, y.S, o->v, d.V)) != GLD_OK) return st;
    if (o->f_c && (st = get_vec<double>(b->st, y.n, y.S, o->f_c, d.FC)) != GLD_OK) return st;
    if (o->f_d && (st = work(o->f_d, d.FD)) != GLD_OK) return st;
    if (o->f_r && (st = work(o->f_r, d.FR)) != GLD_OK) return st;
    long long stp = 0;
    BHIP(hipMemcpy(&stp, d.step, 8, hipMemcpyDeviceToHost));
    if (o->history && d.nslots > 0) {
        const size_t elt = b->fp64 ? 8 : 4;
        for (int m = 1; m <= d.nslots; ++m) {
            const int sl = static_cast<int>(((stp - m) % d.nslots + d.nslots) % d.nslots);
            const void *src = static_cast<const char *>(d.ring) + static_cast<size_t>(sl) * 3 * d.S * elt;
            if ((st = work(o->history + static_cast<size_t>(m - 1) * y.n * 3, src)) != GLD_OK) return st;
        }
    }
    o->step = stp;
    int flags = 0;
    long long fstep = 0;
    if ((st = read_flags_of(b, y, flags, fstep)) != GLD_OK) return st;
    o->flags = flags;
    o->flag_step = fstep;
    return GLD_OK;
}

gld_status gld_batch_write_state(gld_batch *b, int32_t slot, const gld_state *in)
{
    if (!b || !in || !in->r || !in->v || slot < 0 || slot >= b->capacity || !b->sys[slot].used)
        return bfail(GLD_ERR_INVALID_ARG, "no such system or NULL state");
    if (in->step < 0) return bfail(GLD_ERR_INVALID_ARG, "step must be >= 0");
    Sys &y = b->sys[slot];
    const BSys &d = y.d;
    for (int64_t e = 0; e < 3 * y.n; ++e)
        if (!std::isfinite(in->r[e]) || !std::isfinite(in->v[e])) return bfail(GLD_ERR_NONFINITE, "state not finite");
    // the written configuration against the noise interval and the singular
    // points (Sec. II.B), on the host
    if (y.noise_on && y.has_pair) {
        double th[2], gm = 0, mn = 0;
        host_spectrum(y.p, in->r, th, gm, mn);
        if (!(th[0] > y.plan.sing_lo) || !(th[1] < y.plan.sing_hi))
            return bfail(GLD_ERR_NOT_PD, "written configuration: pair-matrix spectrum reaches a singular point");
        if (th[0] < y.plan.lo || th[1] > y.plan.hi || gm > y.plan.hi)
            return bfail(GLD_ERR_INTERVAL, "written configuration: pair-matrix spectrum outside the noise interval");
    }
    BHIP(hipStreamSynchronize(b->st));
    gld_status st;
    std::vector<double> dstage;
    if ((st = put_vec<double>(b->st, y.n, y.S, d.R, in->r, dstage)) != GLD_OK) return st;
    if ((st = put_vec<double>(b->st, y.n, y.S, d.V, in->v, dstage)) != GLD_OK) return st;
    const long long stp = in->step;
    BHIP(hipMemcpyAsync(d.step, &stp, 8, hipMemcpyHostToDevice, b->st));
    const size_t elt = b->fp64 ? 8 : 4;
    if (d.nslots > 0) {
        if (in->history) {
            for (int m = 1; m <= d.nslots; ++m) {
                const int sl = static_cast<int>(((stp - m) % d.nslots + d.nslots) % d.nslots);
                void *dst = static_cast<char *>(d.ring) + static_cast<size_t>(sl) * 3 * d.S * elt;
                const double *src = in->history + static_cast<size_t>(m - 1) * y.n * 3;
                if (b->fp64) {
                    std::vector<double> stg;
                    if ((st = put_vec<double>(b->st, y.n, y.S, dst, src, stg)) != GLD_OK) return st;
                } else {
                    std::vector<float> stg;
                    if ((st = put_vec<float>(b->st, y.n, y.S, dst, src, stg)) != GLD_OK) return st;
                }
            }
        } else {
            BHIP(hipMemsetAsync(d.ring, 0, static_cast<size_t>(d.nslots) * 3 * d.S * elt, b->st));
        }
    }
    BHIP(hipMemsetAsync(d.FD, 0, 3 * d.S * elt, b->st));
    BHIP(hipMemsetAsync(d.FR, 0, 3 * d.S * elt, b->st));
    BHIP(hipMemsetAsync(d.flags, 0, 8, b->st));
    BHIP(hipMemsetAsync(d.flag_step, 0, 8, b->st));
    BHIP(hipStreamSynchronize(b->st));
    return prime(b, std::vector<int>{slot});
}

gld_status gld_batch_noise_parameters(const gld_batch *b, int32_t slot, gld_noise_info *o)
{
    if (!b || !o || slot < 0 || slot >= b->capacity || !b->sys[slot].used)
        return bfail(GLD_ERR_INVALID_ARG, "no such system");
    const Sys &y = b->sys[slot];
    std::memset(o, 0, sizeof(*o));
    o->cheb_terms = y.noise_on ? y.plan.K : 0;
    o->rank = y.noise_on ? y.plan.r : 0;
    o->block = y.bf;
    o->lam_lo = y.plan.lo;
    o->lam_hi = y.plan.hi;
    o->lam_singular = y.plan.sing_lo;
    o->err_estimate = y.plan.err_cheb + y.plan.err_rank + y.plan.err_window;
    o->window_half = y.noise_on ? y.plan.half : 0;
    o->noise_window = 1;
    o->list_index_bits = 16;
    o->list_weight_bits = b->fp64 ? 64 : 32;
    o->theta_min = y.theta[0];
    o->theta_max = y.theta[1];
    return GLD_OK;
}

gld_status gld_batch_set_schedule(gld_batch *b, const gld_batch_schedule *s)
{
    if (!b || !s) return bfail(GLD_ERR_INVALID_ARG, "NULL argument");
    b->sched = *s;
    b->dirty = true;
    return GLD_OK;
}

gld_status gld_batch_autotune(gld_batch *b, int32_t trial_steps, gld_batch_schedule *chosen, double *ms_per_candidate)
{
    if (!b || trial_steps < 1) return bfail(GLD_ERR_INVALID_ARG, "bad batch or trial count");
    static const gld_batch_schedule cand[GLD_BATCH_CANDIDATES] = {
        {{1 << 30, 1 << 30, 1 << 30}},  // one lane per particle everywhere
        {{0, 1 << 30, 1 << 30}},        // two
        {{0, 0, 1 << 30}},              // four
        {{0, 0, 0}},                    // eight
        {{8, 32, 96}},
        {{16, 48, 128}},
        {{24, 64, 160}},
        {{32, 96, 256}},
    };
    gld_status st;
    // keep F^D' and F^R of the last step: the trial passes rewrite them
    const std::vector<int> a = active(b);
    const size_t elt = b->fp64 ? 8 : 4;
    size_t keep_bytes = 0;
    for (int s : a) keep_bytes += up256(2 * 3 * b->sys[s].S * elt);
    size_t keep_off = 0;
    if (keep_bytes && !b->pool.alloc(keep_bytes, keep_off)) return bfail(GLD_ERR_OOM, "no workspace left to autotune");
    {
        size_t o = keep_off;
        for (int s : a) {
            const BSys &d = b->sys[s].d;
            const size_t v = 3 * d.S * elt;
            BHIP(hipMemcpyAsync(b->base + o, d.FD, v, hipMemcpyDeviceToDevice, b->st));
            BHIP(hipMemcpyAsync(b->base + o + v, d.FR, v, hipMemcpyDeviceToDevice, b->st));
            o += up256(2 * v);
        }
    }
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    double best = 1e300;
    int besti = 0;
    for (int c = 0; c < GLD_BATCH_CANDIDATES; ++c) {
        b->sched = cand[c];
        if ((st = rebuild(b)) != GLD_OK) return st;
        if ((st = enqueue_pairs(b)) != GLD_OK) return st;  // warm-up pass
        BHIP(hipEventRecord(e0, b->st));
        for (int t = 0; t < trial_steps; ++t)
            if ((st = enqueue_pairs(b)) != GLD_OK) return st;
        BHIP(hipEventRecord(e1, b->st));
        BHIP(hipEventSynchronize(e1));
        float ms = 0;
        BHIP(hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / trial_steps;
        if (ms_per_candidate) ms_per_candidate[c] = per;
        if (per < best) {
            best = per;
            besti = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        size_t o = keep_off;
        for (int s : a) {
            const BSys &d = b->sys[s].d;
            const size_t v = 3 * d.S * elt;
            BHIP(hipMemcpyAsync(d.FD, b->base + o, v, hipMemcpyDeviceToDevice, b->st));
            BHIP(hipMemcpyAsync(d.FR, b->base + o + v, v, hipMemcpyDeviceToDevice, b->st));
            o += up256(2 * v);
        }
        BHIP(hipStreamSynchronize(b->st));
    }
    if (keep_bytes) b->pool.release(keep_off, keep_bytes);
    b->sched = cand[besti];
    b->dirty = true;
    if (chosen) *chosen = cand[besti];
    return GLD_OK;
}

gld_status gld_batch_stats(gld_batch *b, int32_t *systems, int64_t *particles, int64_t *pairs)
{
    if (!b) return bfail(GLD_ERR_INVALID_ARG, "NULL batch");
    BHIP(hipStreamSynchronize(b->st));
    int32_t ns = 0;
    int64_t np = 0, pr = 0;
    for (int s : active(b)) {
        const Sys &y = b->sys[s];
        ++ns;
        np += y.n;
        if (pairs) {
            std::vector<int> nn(static_cast<size_t>(y.n));
            BHIP(hipMemcpy(nn.data(), y.d.nn, nn.size() * sizeof(int), hipMemcpyDeviceToHost));
            for (int v : nn) pr += v;
        }
    }
    if (systems) *systems = ns;
    if (particles) *particles = np;
    if (pairs) *pairs = pr;
    return GLD_OK;
}

gld_status gld_batch_system_stats(gld_batch *b, int32_t slot, int64_t *pairs, int32_t *lanes)
{
    if (!b || slot < 0 || slot >= b->capacity || !b->sys[slot].used)
        return bfail(GLD_ERR_INVALID_ARG, "no such system");
    BHIP(hipStreamSynchronize(b->st));
    const Sys &y = b->sys[slot];
    if (pairs) {
        std::vector<int> nn(static_cast<size_t>(y.n));
        BHIP(hipMemcpy(nn.data(), y.d.nn, nn.size() * sizeof(int), hipMemcpyDeviceToHost));
        int64_t pr = 0;
        for (int v : nn) pr += v;
        *pairs = pr;
    }
    if (lanes) *lanes = y.d.lanes;
    return GLD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Continuous-batching server over one batch.
// ---------------------------------------------------------------------------
namespace {

struct Request {
    int64_t id = 0;
    double arrival = 0, admitted = -1, done = -1;
    int64_t steps = 0, left = 0;
    int slot = -1;
    gld_status status = GLD_OK;
    Sys prepared;
    std::vector<double> r0, v0;
    // the final state
    std::vector<double> r, v, f_c, f_d, f_r;
    int64_t step_end = 0;
    int32_t flags = 0;
    int64_t flag_step = 0;
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct gld_server {
    gld_batch *b = nullptr;
    int chunk = 50;
    std::vector<Request> req;
    double t_start = 0, t_end = 0;
    int64_t batch_steps = 0;
};

namespace {

gld_status finish(gld_server *sv, Request &q, double t)
{
    gld_batch *b = sv->b;
    const int64_t n3 = 3 * q.prepared.n;
    q.r.assign(n3, 0.0);
    q.v.assign(n3, 0.0);
    q.f_c.assign(n3, 0.0);
    q.f_d.assign(n3, 0.0);
    q.f_r.assign(n3, 0.0);
    gld_state st{};
    st.r = q.r.data();
    st.v = q.v.data();
    st.f_c = q.f_c.data();
    st.f_d = q.f_d.data();
    st.f_r = q.f_r.data();
    gld_status e = gld_batch_read_state(b, q.slot, &st);
    if (e != GLD_OK) return e;
    q.step_end = st.step;
    q.flags = st.flags;
    q.flag_step = st.flag_step;
    if ((e = gld_batch_remove(b, q.slot)) != GLD_OK) return e;
    q.slot = -1;
    q.done = t;
    return GLD_OK;
}

}  // namespace

extern "C" {

gld_status gld_server_create(int32_t precision, int32_t max_systems, void *d_workspace, size_t workspace_bytes,
                             void *hip_stream, int32_t chunk_steps, const gld_batch_schedule *schedule,
                             gld_server **out)
{
    if (!out || chunk_steps < 1) return bfail(GLD_ERR_INVALID_ARG, "NULL argument or chunk_steps < 1");
    gld_batch *b = nullptr;
    gld_status st = gld_batch_create(precision, max_systems, d_workspace, workspace_bytes, hip_stream, &b);
    if (st != GLD_OK) return st;
    if (schedule) b->sched = *schedule;
    gld_server *sv = new gld_server();
    sv->b = b;
    sv->chunk = chunk_steps;
    *out = sv;
    return GLD_OK;
}

gld_status gld_server_submit(gld_server *sv, const gld_params *params, const double *r0, const double *v0,
                             int64_t steps, double arrival_s, int64_t *id, size_t *footprint)
{
    if (!sv || !params || !r0 || !v0 || steps < 1 || !(arrival_s >= 0)) return bfail(GLD_ERR_INVALID_ARG, "bad request");
    Request q;
    q.id = static_cast<int64_t>(sv->req.size());
    q.arrival = arrival_s;
    q.steps = q.left = steps;
    // the one-off host construction (noise filters, interval) happens here,
    // before the request's arrival; admission then only places it
    Built r = build_system(sv->b->fp64, params, r0, q.prepared);
    if (r.st != GLD_OK) return bfail(r.st, r.err);
    q.r0.assign(r0, r0 + 3 * params->n);
    q.v0.assign(v0, v0 + 3 * params->n);
    if (id) *id = q.id;
    if (footprint) *footprint = q.prepared.bytes;
    sv->req.push_back(std::move(q));
    return GLD_OK;
}

gld_status gld_server_run(gld_server *sv)
{
    if (!sv) return bfail(GLD_ERR_INVALID_ARG, "NULL server");
    gld_batch *b = sv->b;
    std::vector<int> order(sv->req.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sv->req[x].arrival < sv->req[y].arrival; });
    size_t head = 0;  // next request to admit, in arrival order
    std::vector<int> act;
    const double t0 = now_s();
    sv->t_start = t0;
    gld_status st;
    size_t finished = 0;
    while (finished < sv->req.size()) {
        double t = now_s() - t0;
        // admission, first come first served, while a slot and a workspace
        // piece of the request's footprint are free
        std::vector<int> placed;
        while (head < order.size()) {
            Request &q = sv->req[order[head]];
            if (q.arrival > t) break;
            int slot = -1;
            for (int s = 0; s < b->capacity; ++s)
                if (!b->sys[s].used) { slot = s; break; }
            size_t off = 0;
            if (slot < 0 || !b->pool.alloc(q.prepared.bytes, off)) break;
            const size_t bytes = q.prepared.bytes;
            Sys copy = q.prepared;  // keep the prepared system for an alone run of the same request
            if ((st = place(b, std::move(copy), off, slot, q.r0.data(), q.v0.data())) != GLD_OK) return st;
            (void)bytes;
            q.slot = slot;
            placed.push_back(order[head]);
            act.push_back(order[head]);
            ++head;
        }
        if (!placed.empty()) {
            std::vector<int> slots;
            for (int i : placed) slots.push_back(sv->req[i].slot);
            if ((st = prime(b, slots)) != GLD_OK) return st;
            b->dirty = true;
            t = now_s() - t0;
            for (int i : placed) sv->req[i].admitted = t;
        }
        if (act.empty()) {
            if (head >= order.size()) break;
            const double wait = sv->req[order[head]].arrival - (now_s() - t0);
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            continue;
        }
        // advance every admitted request together by the next chunk
        int64_t k = sv->chunk;
        for (int i : act) k = std::min(k, sv->req[i].left);
        if ((st = gld_batch_step(b, k)) != GLD_OK) return st;
        BHIP(hipStreamSynchronize(b->st));
        sv->batch_steps += k;
        t = now_s() - t0;
        std::vector<int> still;
        for (int i : act) {
            Request &q = sv->req[i];
            q.left -= k;
            if (q.left == 0) {
                if ((st = finish(sv, q, t)) != GLD_OK) return st;
                ++finished;
            } else {
                still.push_back(i);
            }
        }
        act.swap(still);
    }
    sv->t_end = now_s() - t0;
    return GLD_OK;
}

gld_status gld_server_request(const gld_server *sv, int64_t id, gld_request_info *info, gld_state *out)
{
    if (!sv || id < 0 || id >= static_cast<int64_t>(sv->req.size())) return bfail(GLD_ERR_INVALID_ARG, "no such request");
    const Request &q = sv->req[id];
    if (info) {
        info->id = q.id;
        info->n = q.prepared.n;
        info->m_max = q.prepared.p.m_max;
        info->steps = q.steps;
        info->footprint = q.prepared.bytes;
        info->arrival_s = q.arrival;
        info->admitted_s = q.admitted;
        info->done_s = q.done;
        info->status = q.done >= 0 ? (q.flags ? q.flags : GLD_OK) : GLD_ERR_INVALID_ARG;
    }
    if (out) {
        if (q.done < 0) return bfail(GLD_ERR_INVALID_ARG, "request not completed");
        const size_t n3 = q.r.size();
        auto cp = [&](double *dst, const std::vector<double> &src) {
            if (dst) std::copy(src.begin(), src.end(), dst);
        };
        (void)n3;
        cp(out->r, q.r);
        cp(out->v, q.v);
        cp(out->f_c, q.f_c);
        cp(out->f_d, q.f_d);
        cp(out->f_r, q.f_r);
        out->step = q.step_end;
        out->flags = q.flags;
        out->flag_step = q.flag_step;
    }
    return GLD_OK;
}

gld_status gld_server_stats(const gld_server *sv, double *makespan_s, int64_t *batch_steps)
{
    if (!sv) return bfail(GLD_ERR_INVALID_ARG, "NULL server");
    if (makespan_s) *makespan_s = sv->t_end;
    if (batch_steps) *batch_steps = sv->batch_steps;
    return GLD_OK;
}

gld_status gld_server_destroy(gld_server *sv)
{
    if (!sv) return GLD_OK;
    gld_status st = gld_batch_destroy(sv->b);
    delete sv;
    return st;
}

gld_status gld_batch_destroy(gld_batch *b)
{
    if (!b) return GLD_OK;
    if (b->st) (void)hipStreamSynchronize(b->st);
    drop_graph(b);
    for (auto e : b->ev) (void)hipEventDestroy(e);
    delete b;
    return GLD_OK;
}

}  // extern "C"
