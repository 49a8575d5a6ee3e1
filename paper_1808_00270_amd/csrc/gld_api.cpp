// C ABI of libgld (see include/gld.h): validation, workspace layout, the
// one-off setup, the per-step launch sequence (replayed as a HIP graph) and
// state transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gld.h"
#include "gld_internal.h"

using gld::Dev;
using gld::NoisePlan;

namespace {

thread_local std::string g_last_error;

gld_status fail(gld_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(GLD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

struct Layout {
    size_t off = 0;
    char *base = nullptr;
    template <typename P>
    void take(P *&ptr, size_t bytes)
    {
        off = (off + 255) & ~static_cast<size_t>(255);
        ptr = base ? reinterpret_cast<P *>(base + off) : nullptr;
        off += bytes;
    }
};

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

bool finite_all(const double *p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

gld_status separable_form(const gld_params *p, std::vector<double> &w, std::vector<double> &g, bool &any);

// general: the checks of the general system type (gld_general.h), which
// takes pair tables of any rank and a distance-dependent self memory
gld_status validate(const gld_params *p, bool general = false)
{
    if (!p) return fail(GLD_ERR_INVALID_ARG, "params is NULL");
    if (p->n < 1 || p->n > (int64_t(1) << 30)) return fail(GLD_ERR_INVALID_ARG, "n must be in [1, 2^30]");
    if (p->m_max < 1 || p->m_max > 4096) return fail(GLD_ERR_INVALID_ARG, "m_max must be in [1, 4096]");
    if (p->n_r < 2 || p->n_r > GLD_MAX_DISTANCE_BINS)
        return fail(GLD_ERR_INVALID_ARG, "n_r must be in [2, GLD_MAX_DISTANCE_BINS]");
    if (!(p->dt > 0) || !(p->mass > 0) || !(p->kT >= 0) || !std::isfinite(p->kT))
        return fail(GLD_ERR_INVALID_ARG, "dt, mass must be > 0 and kT >= 0");
    if (!p->k_self || !finite_all(p->k_self, p->m_max)) return fail(GLD_ERR_INVALID_ARG, "k_self missing or not finite");
    if ((p->k_pair_g == nullptr) != (p->k_pair_w == nullptr))
        return fail(GLD_ERR_INVALID_ARG, "k_pair_g and k_pair_w must both be given or both NULL");
    if (p->k_pair_g && (!finite_all(p->k_pair_g, p->m_max) || !finite_all(p->k_pair_w, p->n_r)))
        return fail(GLD_ERR_INVALID_ARG, "pair kernel tables not finite");
    if (!(p->dr > 0) || !std::isfinite(p->r0)) return fail(GLD_ERR_INVALID_ARG, "dr must be > 0");
    if (!(p->r_cut > 0)) return fail(GLD_ERR_INVALID_ARG, "r_cut must be > 0");
    for (int c = 0; c < 3; ++c) {
        if (!(p->box[c] > 0) || !std::isfinite(p->box[c])) return fail(GLD_ERR_INVALID_ARG, "box edges must be > 0");
        if (!(p->r_cut < 0.5 * p->box[c]))
            return fail(GLD_ERR_BOX, "r_cut must be smaller than half of every box edge (minimum image)");
    }
    if (p->pair_tensor != GLD_PAIR_ISOTROPIC && p->pair_tensor != GLD_PAIR_PARALLEL)
        return fail(GLD_ERR_INVALID_ARG, "unknown pair_tensor");
    if (p->precision != GLD_FP64 && p->precision != GLD_FP32_MIXED)
        return fail(GLD_ERR_INVALID_ARG, "unknown precision");
    if (p->wca_eps != 0.0 && !(std::pow(2.0, 1.0 / 6.0) * p->wca_sigma <= p->r_cut))
        return fail(GLD_ERR_INVALID_ARG, "the WCA range 2^(1/6) sigma must not exceed r_cut");
    if (p->noise_tol < 0 || p->noise_tol >= 1) return fail(GLD_ERR_INVALID_ARG, "noise_tol must be in [0, 1)");
    if (p->max_neighbors < 0) return fail(GLD_ERR_INVALID_ARG, "max_neighbors must be >= 0");
    if (!(p->verlet_skin >= 0) || !std::isfinite(p->verlet_skin))
        return fail(GLD_ERR_INVALID_ARG, "verlet_skin must be finite and >= 0");
    if (p->noise_window < 0 || p->noise_window > gld::kMaxFirBlock)
        return fail(GLD_ERR_INVALID_ARG, "noise_window must be in [0, " + std::to_string(gld::kMaxFirBlock) + "]");
    if (p->rebuild_period < 0) return fail(GLD_ERR_INVALID_ARG, "rebuild_period must be >= 0");
    if (p->check_iters < 0 || p->check_iters > GLD_MAX_CHECK_ITERS)
        return fail(GLD_ERR_INVALID_ARG, "check_iters must be in [0, GLD_MAX_CHECK_ITERS]");
    const size_t table = static_cast<size_t>(p->n_r) * p->m_max;
    if (p->k_pair) {
        if (p->k_pair_g || p->k_pair_w)
            return fail(GLD_ERR_INVALID_ARG, "give either the general table k_pair or its separable form k_pair_w, k_pair_g");
        if (!finite_all(p->k_pair, static_cast<int64_t>(table))) return fail(GLD_ERR_INVALID_ARG, "k_pair not finite");
        if (!general) {
            std::vector<double> w, g;
            bool any = false;
            gld_status st = separable_form(p, w, g, any);
            if (st != GLD_OK) return st;
        }
    }
    if (p->dk_self) {
        if (!finite_all(p->dk_self, static_cast<int64_t>(table))) return fail(GLD_ERR_INVALID_ARG, "dk_self not finite");
        for (size_t i = 0; i < table && !general; ++i)
            if (p->dk_self[i] != 0.0)
                return fail(GLD_ERR_INVALID_ARG, "distance-dependent self memory (dk_self): not supported by this "
                                                 "system type (the general system of gld_general.h takes it)");
    }
    if ((p->noise_a == nullptr) != (p->noise_b == nullptr))
        return fail(GLD_ERR_INVALID_ARG, "noise_a and noise_b must both be given or both NULL");
    if (p->noise_a) {
        if (p->noise_rank < 1 || p->noise_rank > gld::kMaxRank || p->noise_terms < 1 || p->noise_terms > gld::kMaxCheb)
            return fail(GLD_ERR_INVALID_ARG, "noise_rank must be in [1, 32] and noise_terms in [1, 512]");
        if (!(p->lam_hi > p->lam_lo))
            return fail(GLD_ERR_INVALID_ARG, "caller-built noise filters need their interval lam_lo < lam_hi");
        if (!finite_all(p->noise_a, static_cast<int64_t>(p->noise_rank) * (2 * p->m_max - 1)) ||
            !finite_all(p->noise_b, static_cast<int64_t>(p->noise_terms) * p->noise_rank))
            return fail(GLD_ERR_INVALID_ARG, "noise filters not finite");
    }
    return GLD_OK;
}

// The general pair table as its separable form, when it has one: with the
// largest entry at (b*, m*), w_b = K[b][m*] / K[b*][m*] (so max |w| = 1, the
// scale in which the noise interval of P = [w(R_ij) T_ij] is given) and
// g_m = K[b*][m]; the table is taken as separable when every entry agrees
// with w_b g_m to 1e-13 of the largest.  An all-zero table means no pair
// memory.
gld_status separable_form(const gld_params *p, std::vector<double> &w, std::vector<double> &g, bool &any)
{
    const int nr = p->n_r, M = p->m_max;
    const double *K = p->k_pair;
    size_t at = 0;
    double big = 0;
    for (size_t i = 0; i < static_cast<size_t>(nr) * M; ++i)
        if (std::fabs(K[i]) > big) { big = std::fabs(K[i]); at = i; }
    any = big > 0;
    if (!any) return GLD_OK;
    const int bs = static_cast<int>(at / M), ms = static_cast<int>(at % M);
    w.assign(nr, 0.0);
    g.assign(M, 0.0);
    for (int b = 0; b < nr; ++b) w[b] = K[static_cast<size_t>(b) * M + ms] / K[at];
    for (int m = 0; m < M; ++m) g[m] = K[static_cast<size_t>(bs) * M + m];
    double worst = 0;
    for (int b = 0; b < nr; ++b)
        for (int m = 0; m < M; ++m) worst = std::max(worst, std::fabs(K[static_cast<size_t>(b) * M + m] - w[b] * g[m]));
    if (worst > 1e-13 * big)
        return fail(GLD_ERR_INVALID_ARG, "non-separable pair kernel table (rank > 1; largest deviation from the "
                                         "rank-one form " + std::to_string(worst / big) + " of its largest entry): "
                                         "not supported by this system type (the general system of gld_general.h "
                                         "takes it)");
    return GLD_OK;
}

struct Geometry {
    int64_t S = 0;
    int cap = 0;
    int capS = 0;  // candidates within r_cut + skin
    int nc[3] = {1, 1, 1};
    int ncell = 1;
    bool fp64 = false, parallel = false;
    int firw = 64;
    int maxc = 1;  // candidates the mat-vec stages per round
    int win = 1;   // noise window W
};

Geometry geometry(const gld_params *p)
{
    Geometry g;
    g.S = round_up(p->n, 64);
    g.fp64 = p->precision == GLD_FP64;
    g.parallel = p->pair_tensor == GLD_PAIR_PARALLEL;
    g.firw = gld::fir_rows(g.fp64);  // the rows of a filter block's outputs
    g.win = p->kT > 0 ? std::max(1, p->noise_window) : 1;
    const double vol = p->box[0] * p->box[1] * p->box[2];
    if (p->max_neighbors > 0) {
        g.cap = p->max_neighbors;
    } else {
        const double expect = static_cast<double>(p->n) / vol * (4.0 / 3.0) * M_PI * p->r_cut * p->r_cut * p->r_cut;
        g.cap = static_cast<int>(round_up(static_cast<int64_t>(1.5 * expect + 32), 32));
    }
    g.cap = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g.cap, p->n - 1)));
    g.cap = static_cast<int>(round_up(g.cap, 8));  // lists are stored in chunks of 8 entries
    // candidate lists within r_cut + skin: the pair capacity scaled by volume
    const double grow = std::pow((p->r_cut + p->verlet_skin) / p->r_cut, 3.0);
    g.capS = static_cast<int>(round_up(static_cast<int64_t>(std::ceil(g.cap * grow)), 8));
    // Cells of edge >= r_cut; a work-group of 128 lanes owns one cell, so aim
    // for about 96 particles per cell (larger cells are always valid).
    const double target = 96.0;
    int64_t cells = 1;
    for (int c = 0; c < 3; ++c) {
        // cells of edge >= r_cut + skin hold every candidate in the 27-cell stencil
        const int by_cut = std::max(1, static_cast<int>(std::floor(p->box[c] / (p->r_cut + p->verlet_skin))));
        const double frac = p->box[c] / std::cbrt(vol);
        const int by_occ = std::max(1, static_cast<int>(std::lround(std::cbrt(p->n / target) * frac)));
        g.nc[c] = std::min(by_cut, by_occ);
        cells *= g.nc[c];
    }
    g.ncell = static_cast<int>(cells);
    // The mat-vec stages the candidates of a cell's stencil in LDS: room for
    // 15 % over the mean (larger stencils are staged in rounds), at most what
    // one work-group's LDS holds.
    int nst = 1;
    for (int c = 0; c < 3; ++c) nst *= std::min(g.nc[c], 3);
    const double occ = static_cast<double>(p->n) / cells;
    int64_t want = round_up(static_cast<int64_t>(1.15 * nst * occ + 64), 64);
    want = std::min<int64_t>(want, p->n);
    g.maxc = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, gld::mv_max_staging(g.fp64, g.parallel))));
    return g;
}

// Carve the workspace.  With base == nullptr only the size is computed.
size_t carve(const gld_params *p, const Geometry &g, char *base, Dev &d)
{
    Layout L;
    L.base = base;
    const size_t elt = g.fp64 ? 8 : 4;
    const int64_t S = g.S, n = p->n, vec = 3 * S;
    const int nslots = std::max(0, p->m_max - 1);
    const int P = 2 * p->m_max - 1;
    L.take(d.R, vec * 8);
    L.take(d.V, vec * 8);
    L.take(d.FC, vec * 8);
    L.take(d.FCn, vec * 8);
    L.take(d.Rw, vec * 8);
    L.take(d.ring, static_cast<size_t>(nslots) * vec * elt);
    L.take(d.Dneg, vec * elt);
    L.take(d.Y, vec * elt);
    L.take(d.FD, vec * elt);
    L.take(d.FR, vec * elt);
    const size_t v4 = 4 * static_cast<size_t>(S) * elt;  // one sorted T4 vector
    for (auto &b : d.cb) L.take(b, v4);
    for (auto &b : d.lq) L.take(b, v4);
    L.take(d.lw, v4);
    L.take(d.ys, v4);
    L.take(d.us, static_cast<size_t>(gld::kMaxRank) * v4);
    if (g.win > 1) {
        // W r <= block rcap <= firw vectors of filter outputs
        L.take(d.usw, static_cast<size_t>(g.firw) * v4);
        for (auto &b : d.cbw) L.take(b, static_cast<size_t>(g.win) * v4);
        L.take(d.FRw, static_cast<size_t>(g.win) * vec * elt);
    }
    L.take(d.pos_s, static_cast<size_t>(n) * 32);
    L.take(d.reld, static_cast<size_t>(n) * 32);  // both modes: the neighbour build decides in FP64 data
    L.take(d.relf, static_cast<size_t>(n) * 16);
    L.take(d.rb_s, static_cast<size_t>(n) * 32);
    L.take(d.relb, static_cast<size_t>(n) * 32);
    L.take(d.snl, static_cast<size_t>(g.capS) * n * 2);
    L.take(d.snn, n * 4);
    L.take(d.U, 2 * static_cast<size_t>(g.firw) * vec * elt);
    // white-noise ring: at most the full filter window plus two of the largest blocks
    if (p->kT > 0)
        L.take(d.wring, static_cast<size_t>(std::max(0, 2 * (p->m_max - 1)) + 2 * gld::kMaxFirBlock) * vec * elt);
    L.take(d.Afilt, static_cast<size_t>(gld::kMaxRank) * gld::fir_padded_rows(p->m_max - 1, gld::kMaxFirBlock) * elt);
    L.take(d.Bmix, static_cast<size_t>(gld::kMaxCheb) * gld::kMaxRank * elt);
    L.take(d.ks, static_cast<size_t>(p->m_max) * elt);
    if (nslots > 0) {
        const int hb = g.fp64 ? gld::kHistBlock64 : gld::kHistBlock32;
        L.take(d.hist_taps, gld::hist_tap_rows(nslots, hb) * 2 * elt);
        L.take(d.Uh, 2 * static_cast<size_t>(gld::kHistSplit) * hb * 2 * vec * elt);
    }
    L.take(d.gm, static_cast<size_t>(p->m_max) * elt);
    L.take(d.wtab, static_cast<size_t>(p->n_r) * 8);
    L.take(d.nbl, static_cast<size_t>(g.cap) * n * 2);
    L.take(d.nbw, static_cast<size_t>(g.cap) * n * elt);
    L.take(d.stab, static_cast<size_t>(g.ncell) * 28 * 8);
    L.take(d.nn, n * 4);
    L.take(d.cell_id, n * 4);
    L.take(d.cell_slot, n * 4);
    L.take(d.cell_tmp, n * 4);
    L.take(d.cell_sorted, n * 4);
    L.take(d.cell_count, static_cast<size_t>(g.ncell) * 4);
    L.take(d.cell_start, static_cast<size_t>(g.ncell + 1) * 4);
    L.take(d.partial, 2 * gld::kPartials * 8);  // two stages of the check's dot products
    L.take(d.lab, (2 * gld::kMaxCheckIters + 4) * 8);
    L.take(d.d_step, 8);
    L.take(d.d_flags, 8);
    L.take(d.d_flag_step, 8);
    L.take(d.d_rowmax, 8);
    L.take(d.d_rebuild, 8);
    L.take(d.chain, static_cast<size_t>(gld::kMaxCheb) * 32);  // ChainStep
    if (p->kT > 0) L.take(d.vk, static_cast<size_t>(gld::kMaxCheb) * v4);
    L.take(d.d_tight, 8);
    L.take(d.d_retired, 8);
    return L.off + 256;
}

}  // namespace

namespace gld {

gld_status validate_params(const gld_params *p) { return validate(p); }
gld_status validate_params_general(const gld_params *p) { return validate(p, true); }

void set_last_error(const std::string &msg) { g_last_error = msg; }

gld_status separable_pair_table(const gld_params *p, std::vector<double> &w, std::vector<double> &g, bool &any)
{
    return separable_form(p, w, g, any);
}

void auto_interval(const gld_params &p, const NoisePlan &plan, double theta_min, double theta_max, double gmax,
                   double &lo, double &hi, double &hi_t, double &lo_t)
{
    // lower end a quarter of the way from the smallest Ritz value to the
    // singular point: the expansion's cost grows as that gap closes, while
    // the smallest eigenvalue of P is set by the short-range structure and
    // moves by a few percent of the gap as a lattice start melts (N = 2e5,
    // rho = 0.5: -0.810 -> -0.797 over 1000 steps, gap 1.05); a 40-step
    // Lanczos run's smallest Ritz value sits 0.009 - 0.016 above the smallest
    // eigenvalue in rho = 0.5 liquids of N = 500 - 4000, against a margin of
    // 0.26 here (0.13 for the tight plan); the periodic Lanczos check latches
    // GLD_ERR_INTERVAL if it ever crosses
    const double span = std::max(1.0, theta_max - theta_min);
    lo = std::isfinite(plan.sing_lo) ? theta_min - 0.25 * (theta_min - plan.sing_lo) : theta_min - 0.5 * span;
    // the largest row sum of |w| bounds lambda_max at every step; leave room
    // for it to grow as the configuration evolves: 8 standard deviations above
    // the mean row sum of an ideal gas at this density (mean rho int w dV,
    // variance rho int w^2 dV; a liquid fluctuates less), and at least 1.2
    // times the initial bound plus 0.5 (a lattice start at N = 2e5, rho = 0.5:
    // 26.6, its liquid 29.2 - 30.5 over 1000 steps)
    double mu = 0, var = 0;
    const double rho = static_cast<double>(p.n) / (p.box[0] * p.box[1] * p.box[2]);
    for (int b = 0; b + 1 < p.n_r; ++b) {
        // trapezoid over the grid, inside the cutoff
        const double ra = p.r0 + b * p.dr, rb = ra + p.dr;
        if (ra >= p.r_cut) break;
        const double wa = std::fabs(p.k_pair_w[b]), wb = std::fabs(p.k_pair_w[b + 1]);
        mu += 0.5 * p.dr * (ra * ra * wa + rb * rb * wb);
        var += 0.5 * p.dr * (ra * ra * wa * wa + rb * rb * wb * wb);
    }
    mu *= 4.0 * M_PI * rho;
    var *= 4.0 * M_PI * rho;
    const double observed = 1.2 * std::max(gmax, theta_max) + 0.5;
    hi = std::max(observed, mu + 8.0 * std::sqrt(var));
    if (std::isfinite(plan.sing_hi)) hi = std::min(hi, theta_max + 0.5 * (plan.sing_hi - theta_max));
    // A second, tight plan on [lo, observed] for the steps whose row-sum bound
    // stays below it (the liquid's bound settles well below the ideal-gas
    // margin: near 30 against 48 at N = 2e5, rho = 0.5); the device picks the
    // plan at every step, so the tight one is used only where its interval
    // provably holds the spectrum.
    hi_t = observed < hi ? observed : std::numeric_limits<double>::quiet_NaN();
    // its lower end an eighth of the way to the singular point (the wide
    // plan's a quarter); a spectrum check whose smallest Ritz value drops
    // below it retires it until the next written state
    lo_t = std::isfinite(plan.sing_lo) ? theta_min - 0.125 * (theta_min - plan.sing_lo) : lo;
}

}  // namespace gld

struct gld_system {
    gld_params p{};
    std::vector<double> k_self, g, w;
    std::vector<double> noise_a, noise_b;  // caller-built noise filters (copies)
    Geometry geo;
    Dev d;
    NoisePlan plan;
    hipStream_t st = nullptr;
    int64_t step = 0;
    int noise_on = 0;
    int check_interval = 100;
    bool graph_on = true;
    // one graph per step of the noise window (one in all unless W > 1)
    bool graph_ready[gld::kMaxFirBlock] = {};
    hipGraph_t graph[gld::kMaxFirBlock] = {};
    hipGraphExec_t gexec[gld::kMaxFirBlock] = {};
    bool win_valid = false;  // the window buffers hold the current window
    bool timing = false;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    // (class, index of the start event, launches between the two events)
    std::vector<std::tuple<int, size_t, int>> pending;
    double ms[GLD_K_COUNT] = {0};
    int64_t cnt[GLD_K_COUNT] = {0};
    double theta[2] = {0, 0};
    gld_status latched = GLD_OK;
    bool filters_given = false;
    int static_device = -1;  // >= 0: the workspace is that device's static array
};

namespace {

// host [n][3] doubles -> device [3][S] of type T (staging through a host buffer)
template <typename T>
gld_status upload_vec(gld_system *s, void *dst, const double *src)
{
    const int64_t n = s->p.n, S = s->geo.S;
    std::vector<T> h(3 * S, T(0));
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) h[c * S + i] = static_cast<T>(src[3 * i + c]);
    HIP_TRY(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    return GLD_OK;
}

template <typename T>
gld_status download_vec(gld_system *s, double *dst, const void *src)
{
    const int64_t n = s->p.n, S = s->geo.S;
    std::vector<T> h(3 * S);
    HIP_TRY(hipMemcpyAsync(h.data(), src, h.size() * sizeof(T), hipMemcpyDeviceToHost, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) dst[3 * i + c] = static_cast<double>(h[c * S + i]);
    return GLD_OK;
}

gld_status upload_work_vec(gld_system *s, void *dst, const double *src)
{
    return s->geo.fp64 ? upload_vec<double>(s, dst, src) : upload_vec<float>(s, dst, src);
}

gld_status download_work_vec(gld_system *s, double *dst, const void *src)
{
    return s->geo.fp64 ? download_vec<double>(s, dst, src) : download_vec<float>(s, dst, src);
}

template <typename T>
gld_status upload_table(gld_system *s, void *dst, const double *src, size_t n)
{
    std::vector<T> h(src, src + n);
    HIP_TRY(hipMemcpyAsync(dst, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    return GLD_OK;
}

gld_status upload_work_table(gld_system *s, void *dst, const double *src, size_t n)
{
    return s->geo.fp64 ? upload_table<double>(s, dst, src, n) : upload_table<float>(s, dst, src, n);
}

gld_status read_flags(gld_system *s)
{
    int flags[2] = {0, 0};
    long long fstep = 0;
    HIP_TRY(hipStreamSynchronize(s->st));
    HIP_TRY(hipMemcpy(flags, s->d.d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&fstep, s->d.d_flag_step, sizeof(fstep), hipMemcpyDeviceToHost));
    if (flags[0] != 0 && s->latched == GLD_OK) {
        s->latched = static_cast<gld_status>(flags[0]);
        g_last_error = std::string("device check failed at step ") + std::to_string(fstep) + ": " +
                       gld_status_string(flags[0]);
    }
    return s->latched;
}

// -- timing helpers ----------------------------------------------------------
// force: record even while per-launch events are paused
gld_status ev_begin(gld_system *s, size_t &idx, bool force = false)
{
    if (!s->timing && !force) return GLD_OK;
    while (s->pool.size() < s->pool_used + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        s->pool.push_back(e);
    }
    idx = s->pool_used;
    s->pool_used += 2;
    HIP_TRY(hipEventRecord(s->pool[idx], s->st));
    return GLD_OK;
}

gld_status ev_end(gld_system *s, int cls, size_t idx, int launches = 1, bool force = false)
{
    if (!s->timing && !force) return GLD_OK;
    HIP_TRY(hipEventRecord(s->pool[idx + 1], s->st));
    s->pending.emplace_back(cls, idx, launches);
    return GLD_OK;
}

// per-launch events off for a stretch timed as a whole (restored on every
// way out of the scope)
struct TimingPause {
    gld_system *s;
    bool was;
    explicit TimingPause(gld_system *sys) : s(sys), was(sys->timing) { s->timing = false; }
    ~TimingPause() { s->timing = was; }
};

#define LAUNCH(cls, expr)                                  \
    do {                                                   \
        size_t ix_ = 0;                                    \
        gld_status s_ = ev_begin(s, ix_);                  \
        if (s_ != GLD_OK) return s_;                       \
        HIP_TRY(expr);                                     \
        if ((s_ = ev_end(s, cls, ix_)) != GLD_OK) return s_; \
    } while (0)

// Noise window of W > 1 steps (the variant the remarks after Algorithm 1 of
// Sec. II.C propose when the positions barely move over W steps): the random
// forces of the W steps of the window holding the current step, all at the
// current positions, into FRw.  One Clenshaw chain per step of the window;
// the chains of two steps share each stream of the pair lists.
gld_status enqueue_window(gld_system *s)
{
    const Dev &d = s->d;
    hipStream_t st = s->st;
    const NoisePlan &pl = s->plan;
    const int W = d.win;
    const size_t elt = s->geo.fp64 ? 8 : 4;
    const size_t v4 = 4 * elt * static_cast<size_t>(d.S);
    const int rc = d.fir_rcap;
    auto coef = [&](int k) {
        return static_cast<const void *>(static_cast<const char *>(d.Bmix) + static_cast<size_t>(k) * rc * elt);
    };
    LAUNCH(GLD_K_NOISE_SPMV, gld::launch_permute_window(d, st, pl.r));
    // the chains are timed as a whole, as in the single-step chain
    size_t ix_chain = 0;
    gld_status ts = ev_begin(s, ix_chain);
    if (ts != GLD_OK) return ts;
    int launches = 0;
    {
        const TimingPause pause(s);
        // the plan of the window's positions (tight or wide), as for one step
        if (d.cheb_kt > 0) LAUNCH(GLD_K_NOISE_SPMV, gld::launch_cheb_select(d, st));
        bool rev = true;  // the cell order alternates from launch to launch
        for (int m0 = 0; m0 < W; m0 += 2) {
            const int nv = std::min(2, W - m0);
            const void *us = static_cast<const char *>(d.usw) + static_cast<size_t>(m0) * pl.r * v4;
            auto buf = [&](int i) -> void * { return i < 0 ? nullptr : static_cast<char *>(d.cbw[i]) + m0 * v4; };
            void *fr = static_cast<char *>(d.FRw) + static_cast<size_t>(m0) * 3 * d.S * elt;
            int prev1 = -1, prev2 = -1;
            for (int k = pl.K - 1; k >= 1; --k) {
                int out = 0;
                while (out == prev1 || out == prev2) ++out;
                if (prev1 < 0) {
                    LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv_window(d, st, 0.0, 0.0, nullptr, 0.0, nullptr, coef(k),
                                                                     pl.r, us, buf(out), nullptr, nv, false, k));
                } else {
                    rev = !rev;
                    LAUNCH(GLD_K_NOISE_SPMV,
                           gld::launch_spmv_window(d, st, 2.0 * pl.alpha, 2.0 * pl.beta, buf(prev1),
                                                   prev2 >= 0 ? -1.0 : 0.0, buf(prev2), coef(k), pl.r, us, buf(out),
                                                   nullptr, nv, rev, k));
                }
                ++launches;
                prev2 = prev1;
                prev1 = out;
            }
            if (prev1 >= 0) {
                rev = !rev;
                LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv_window(d, st, pl.alpha, pl.beta, buf(prev1),
                                                                 prev2 >= 0 ? -1.0 : 0.0, buf(prev2), coef(0), pl.r,
                                                                 us, nullptr, fr, nv, rev, 0));
            } else {
                LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv_window(d, st, 0.0, 0.0, nullptr, 0.0, nullptr, coef(0),
                                                                 pl.r, us, nullptr, fr, nv, false, 0));
            }
            ++launches;
        }
    }
    if ((ts = ev_end(s, GLD_K_NOISE_SPMV, ix_chain, launches)) != GLD_OK) return ts;
    return GLD_OK;
}

// One integrator step, eq. (GLD_integrator).  Every launch reads the step
// index from device memory, so the same sequence is replayed for any step;
// with a noise window the sequence of the window's first step (slot 0) also
// computes the window's random forces.
gld_status enqueue_step(gld_system *s, int slot)
{
    const Dev &d = s->d;
    hipStream_t st = s->st;
    const NoisePlan &pl = s->plan;
    LAUNCH(GLD_K_HISTORY, gld::launch_history_block(d, 0, st));
    LAUNCH(GLD_K_HISTORY, gld::launch_history(d, st));
    if (s->noise_on) {
        LAUNCH(GLD_K_NOISE_FIR, gld::launch_white_ring(d, 0, st));
        LAUNCH(GLD_K_NOISE_FIR, gld::launch_fir(d, 0, st));
    }
    LAUNCH(GLD_K_DISSIPATIVE, gld::launch_permute(d, st, (s->noise_on && d.win == 1) ? pl.r : 0));
    // With the per-step chain (isotropic pair tensor), the dissipative
    // product P Y rides on the chain's first pair term (one stream of the
    // lists for both); otherwise it streams the lists alone, here.
    const bool fuse = s->noise_on && d.win == 1 && !d.parallel && d.has_pair && pl.K >= 2 &&
                      (d.cheb_kt == 0 || d.cheb_kt >= 2);
    // the refresh of the step before wrote the pair lists in ascending cell
    // order; the mat-vecs that stream them alternate the order from here on,
    // the first one descending
    bool rev = !fuse;
    if (!fuse) LAUNCH(GLD_K_DISSIPATIVE, gld::launch_dissipative(d, st, rev));
    // the chain terms that may be the step's first pair term (k = K - 2 of
    // the wide and of the tight plan): with fusion they carry P Y
    auto first_pair = [&](int k) { return fuse && (k == pl.K - 2 || (d.cheb_kt > 0 && k == d.cheb_kt - 2)); };
    if (s->noise_on && d.win > 1) {
        if (slot == 0) {
            gld_status ws = enqueue_window(s);
            if (ws != GLD_OK) return ws;
        }
        LAUNCH(GLD_K_NOISE_SPMV, gld::launch_take_window(d, st));
    } else if (s->noise_on) {
        const size_t elt = s->geo.fp64 ? 8 : 4;
        const int rc = d.fir_rcap;
        auto coef = [&](int k) {
            return static_cast<const void *>(static_cast<const char *>(d.Bmix) + static_cast<size_t>(k) * rc * elt);
        };
        // Clenshaw: b_k = v_k + 2 P~ b_{k+1} - b_{k+2};  F = v_0 + P~ b_1 - b_2,
        // v_k = sum_q B[k][q] u_q, P~ = alpha P + beta 1
        // Timing: the terms that stream the pair lists (k <= Ka - 2, Ka the K
        // of the step's plan) run back to back between one event pair (an
        // event pair per launch would add the event gaps to each of them);
        // the plan choice, the skipped terms and the first term between
        // another (noise_setup).  The host knows the step's plan only once
        // the step before has run: timing mode synchronises here to read it.
        const bool timing_on = s->timing;
        int Ka = pl.K;
        if (timing_on && d.cheb_kt > 0) {
            HIP_TRY(hipStreamSynchronize(st));
            unsigned bits = 0;
            double theta_min = 0;
            int retired = 0;
            HIP_TRY(hipMemcpy(&bits, d.d_rowmax, sizeof(bits), hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(&theta_min, d.lab + 2 * gld::kMaxCheckIters, sizeof(double), hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(&retired, d.d_retired, sizeof(int), hipMemcpyDeviceToHost));
            float g = 0;
            std::memcpy(&g, &bits, sizeof(g));
            if (g <= d.lam_tight && theta_min >= d.lam_lo_tight && retired == 0) Ka = pl.Kt;  // as k_cheb_select
        }
        size_t ix = 0;
        gld_status ts = ev_begin(s, ix);
        if (ts != GLD_OK) return ts;
        int setup = 0;
        bool in_pairs = false;
        auto to_pairs = [&](int k) -> gld_status {
            // before term k: the first term that streams the lists opens the second event pair
            if (!timing_on || in_pairs || k > Ka - 2) return GLD_OK;
            in_pairs = true;
            gld_status e = ev_end(s, GLD_K_NOISE_SETUP, ix, setup, true);
            return e != GLD_OK ? e : ev_begin(s, ix, true);
        };
        {
            const TimingPause pause(s);
            if (d.cheb_kt > 0) {
                LAUNCH(GLD_K_NOISE_SETUP, gld::launch_cheb_select(d, st));
                ++setup;
            }
            LAUNCH(GLD_K_NOISE_SETUP, gld::launch_cheb_mix(d, pl.r, pl.K, st));
            ++setup;
            // term k of the chain passes its index: with a tight plan the
            // step's plan (k_cheb_select) sets its combination, and the terms
            // beyond the tight plan's K return at once
            void *prev1 = nullptr, *prev2 = nullptr;
            for (int k = pl.K - 1; k >= 1; --k) {
                if ((ts = to_pairs(k)) != GLD_OK) return ts;
                void *out = nullptr;
                for (void *c : d.cb)
                    if (c != prev1 && c != prev2) { out = c; break; }
                if (!prev1) {
                    LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv(d, st, 0.0, 0.0, nullptr, 0.0, nullptr, coef(k), pl.r,
                                                              out, nullptr, nullptr, false, k, true));
                } else if (first_pair(k)) {
                    rev = !rev;
                    LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv_dual(d, st, 2.0 * pl.alpha, 2.0 * pl.beta, prev1,
                                                                   prev2 ? -1.0 : 0.0, prev2, out, nullptr, rev, k));
                } else {
                    rev = !rev;
                    LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv(d, st, 2.0 * pl.alpha, 2.0 * pl.beta, prev1,
                                                              prev2 ? -1.0 : 0.0, prev2, coef(k), pl.r, out, nullptr,
                                                              nullptr, rev, k, true));
                }
                if (!in_pairs) ++setup;
                prev2 = prev1;
                prev1 = out;
            }
            if ((ts = to_pairs(0)) != GLD_OK) return ts;
            if (prev1 && first_pair(0)) {
                LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv_dual(d, st, pl.alpha, pl.beta, prev1, prev2 ? -1.0 : 0.0,
                                                               prev2, nullptr, d.FR, !rev, 0));
            } else if (prev1) {
                LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv(d, st, pl.alpha, pl.beta, prev1, prev2 ? -1.0 : 0.0, prev2,
                                                          coef(0), pl.r, nullptr, d.FR, nullptr, !rev, 0, true));
            } else {
                LAUNCH(GLD_K_NOISE_SPMV, gld::launch_spmv(d, st, 0.0, 0.0, nullptr, 0.0, nullptr, coef(0), pl.r,
                                                          nullptr, d.FR, nullptr, false, 0, true));
            }
            if (!in_pairs) ++setup;
        }
        if ((ts = ev_end(s, in_pairs ? GLD_K_NOISE_SPMV : GLD_K_NOISE_SETUP, ix, in_pairs ? Ka - 1 : setup)) !=
            GLD_OK)
            return ts;
    }
    LAUNCH(GLD_K_UPDATE, gld::launch_update_r(d, st));
    LAUNCH(GLD_K_NEIGHBOR, gld::launch_neighbors(d, st, d.FCn));
    LAUNCH(GLD_K_UPDATE, gld::launch_update_v(d, st));
    HIP_TRY(gld::launch_step_advance(d, st));
    return GLD_OK;
}

gld_status enqueue_check(gld_system *s)
{
    const NoisePlan &pl = s->plan;
    LAUNCH(GLD_K_CHECK, gld::launch_spectrum_check(s->d, s->st, s->d.check_iters, pl.lo, pl.hi, pl.sing_lo,
                                                     pl.sing_hi, s->step + 0x5eed));
    return GLD_OK;
}

void drop_graph(gld_system *s)
{
    for (int k = 0; k < gld::kMaxFirBlock; ++k) {
        if (s->gexec[k]) (void)hipGraphExecDestroy(s->gexec[k]);
        if (s->graph[k]) (void)hipGraphDestroy(s->graph[k]);
        s->gexec[k] = nullptr;
        s->graph[k] = nullptr;
        s->graph_ready[k] = false;
    }
}

gld_status build_graph(gld_system *s, int slot)
{
    HIP_TRY(hipStreamBeginCapture(s->st, hipStreamCaptureModeRelaxed));
    gld_status st = enqueue_step(s, slot);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s->st, &g);
    if (st != GLD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(GLD_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    s->graph[slot] = g;
    HIP_TRY(hipGraphInstantiate(&s->gexec[slot], g, nullptr, nullptr, 0));
    s->graph_ready[slot] = true;
    return GLD_OK;
}

gld_status set_step(gld_system *s, int64_t step)
{
    long long v = step;
    HIP_TRY(hipMemcpyAsync(s->d.d_step, &v, sizeof(v), hipMemcpyHostToDevice, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    s->step = step;
    return GLD_OK;
}

gld_status clear_flags(gld_system *s)
{
    HIP_TRY(hipMemsetAsync(s->d.d_flags, 0, 8, s->st));
    HIP_TRY(hipMemsetAsync(s->d.d_flag_step, 0, 8, s->st));
    HIP_TRY(hipMemsetAsync(s->d.d_retired, 0, 8, s->st));
    HIP_TRY(hipStreamSynchronize(s->st));
    s->latched = GLD_OK;
    return GLD_OK;
}

gld_status run_check_now(gld_system *s, double lo, double hi, double slo, double shi, double theta[2],
                         float *rowmax)
{
    HIP_TRY(gld::launch_spectrum_check(s->d, s->st, s->d.check_iters, lo, hi, slo, shi, s->step + 0x5eed));
    HIP_TRY(hipStreamSynchronize(s->st));
    double res[2];
    HIP_TRY(hipMemcpy(res, s->d.lab + 2 * gld::kMaxCheckIters, sizeof(res), hipMemcpyDeviceToHost));
    theta[0] = res[0];
    theta[1] = res[1];
    if (rowmax) {
        unsigned bits = 0;
        HIP_TRY(hipMemcpy(&bits, s->d.d_rowmax, sizeof(bits), hipMemcpyDeviceToHost));
        std::memcpy(rowmax, &bits, sizeof(float));
    }
    return GLD_OK;
}

gld_status install_plan(gld_system *s);

gld_status setup_noise(gld_system *s)
{
    const gld_params &p = s->p;
    Dev &d = s->d;
    s->noise_on = p.kT > 0;
    if (!s->noise_on) return GLD_OK;
    std::string err;
    gld_status st = gld::noise_spectra(p, s->plan, err);
    if (st != GLD_OK) return fail(st, err);
    const double tol = p.noise_tol > 0 ? p.noise_tol : (s->geo.fp64 ? gld::kNoiseTolFp64 : gld::kNoiseTolMixed);
    double lo = p.lam_lo, hi = p.lam_hi;
    if (p.noise_a) {
        // the caller's filters for [lam_lo, lam_hi]: the interval must stay
        // clear of the singular points, as for a plan built here
        NoisePlan &pl = s->plan;
        if (!(lo > pl.sing_lo) || !(hi < pl.sing_hi))
            return fail(GLD_ERR_NOT_PD, "the interval of the given noise filters reaches a singular point of the "
                                        "noise correlation (" + std::to_string(pl.sing_lo) + ", " +
                                        std::to_string(pl.sing_hi) + ")");
        pl.K = p.noise_terms;
        pl.r = p.noise_rank;
        pl.lo = lo;
        pl.hi = hi;
        pl.alpha = 2.0 / (hi - lo);
        pl.beta = -(hi + lo) / (hi - lo);
        pl.Afilt.assign(p.noise_a, p.noise_a + static_cast<size_t>(pl.r) * pl.P);
        pl.Bmix.assign(p.noise_b, p.noise_b + static_cast<size_t>(pl.K) * pl.r);
        // the filter window: the largest lag with a non-zero tap
        pl.half = 0;
        for (int q = 0; q < pl.r; ++q)
            for (int t = 0; t < pl.P; ++t)
                if (pl.Afilt[static_cast<size_t>(q) * pl.P + t] != 0.0) pl.half = std::max(pl.half, std::abs(t - (pl.M - 1)));
        pl.err_cheb = pl.err_rank = pl.err_window = 0.0;  // unknown: the caller's construction
        pl.Kt = 0;
        pl.Bmix_t.clear();
        s->filters_given = true;
        return install_plan(s);
    }
    double hi_t = std::numeric_limits<double>::quiet_NaN(), lo_t = -1e300;  // tight plan (automatic interval only)
    const bool has_pair = d.has_pair;
    if (!(hi > lo)) {
        if (!has_pair) {
            lo = -1.0;
            hi = 1.0;
        } else {
            double th[2];
            float gmax = 0;
            const double inf = std::numeric_limits<double>::infinity();
            if ((st = run_check_now(s, -inf, inf, -inf, inf, th, &gmax)) != GLD_OK) return st;
            if (!(th[0] > s->plan.sing_lo) || !(th[1] < s->plan.sing_hi))
                return fail(GLD_ERR_NOT_PD, "initial configuration: pair-matrix spectrum [" + std::to_string(th[0]) +
                                                ", " + std::to_string(th[1]) + "] reaches a singular point of the "
                                                "noise correlation (" + std::to_string(s->plan.sing_lo) + ", " +
                                                std::to_string(s->plan.sing_hi) + "): not positive definite");
            gld::auto_interval(p, s->plan, th[0], th[1], gmax, lo, hi, hi_t, lo_t);
        }
    }
    st = gld::noise_build(p, lo, hi, tol, s->plan, err, hi_t, lo_t);
    if (st != GLD_OK) return fail(st, err);
    if (s->plan.K + s->plan.Kt > gld::kMaxCheb) s->plan.Kt = 0;  // the mixing table holds both plans' rows
    return install_plan(s);
}

// the device side of a noise plan: filter block and ring sizes, the padded
// taps and mixing weights, the chain's parameters
gld_status install_plan(gld_system *s)
{
    Dev &d = s->d;
    const bool has_pair = d.has_pair;
    gld_status st;
    const NoisePlan &pl = s->plan;
    d.fir_rcap = gld::fir_rcap_for(pl.r);
    d.fir_block = gld::fir_block_for(s->geo.fp64, d.fir_rcap);
    d.fir_half = pl.half;
    // a noise window lies inside one filter block: the block becomes the
    // largest multiple of W that the filter bank allows
    d.win = s->geo.win;
    if (d.win > d.fir_block)
        return fail(GLD_ERR_INVALID_ARG, "noise_window " + std::to_string(d.win) + " exceeds the filter block " +
                                             std::to_string(d.fir_block) + " that this noise plan allows");
    d.fir_block -= d.fir_block % d.win;
    // the ring holds the window of the next block's outputs while the steps
    // of the current block add the slices one block further ahead:
    // 2 half + 2 block - 1 slices (the filter bank steps through the ring 2
    // (FP32) or 4 (FP64) slices at a time and wraps once per step: at least 4)
    d.wring_len = std::max(4, 2 * pl.half + 2 * d.fir_block);
    // filter taps of the window, tap-major [2 half + 1][rcap] (columns beyond
    // r zero) with block - 1 zero rows before and kFirChunk + block - 1 after
    // (the matrix-core filter bank copies whole chunks of rows); and mixing
    // weights [K][rcap]
    const int Pw = 2 * pl.half + 1;
    const int front = d.fir_block - 1;
    const size_t rows = gld::fir_padded_rows(pl.half, d.fir_block);
    std::vector<double> A(static_cast<size_t>(d.fir_rcap) * rows, 0.0), B(static_cast<size_t>(pl.K) * d.fir_rcap, 0.0);
    for (int q = 0; q < pl.r; ++q)
        for (int t = 0; t < Pw; ++t)
            A[static_cast<size_t>(t + front) * d.fir_rcap + q] =
                pl.Afilt[static_cast<size_t>(q) * pl.P + (pl.M - 1 - pl.half) + t];
    B.resize(static_cast<size_t>(pl.K + pl.Kt) * d.fir_rcap, 0.0);  // the tight plan's rows follow
    for (int k = 0; k < pl.K; ++k)
        for (int q = 0; q < pl.r; ++q) B[static_cast<size_t>(k) * d.fir_rcap + q] = pl.Bmix[static_cast<size_t>(k) * pl.r + q];
    for (int k = 0; k < pl.Kt; ++k)
        for (int q = 0; q < pl.r; ++q)
            B[static_cast<size_t>(pl.K + k) * d.fir_rcap + q] = pl.Bmix_t[static_cast<size_t>(k) * pl.r + q];
    d.cheb_kw = pl.K;
    d.cheb_kt = pl.Kt;
    // a margin for the rounding of the row sums (float)
    d.lam_tight = pl.Kt > 0 ? static_cast<float>(pl.hi_t * (1.0 - 1e-5)) : 0.0f;
    d.lam_lo_tight = pl.Kt > 0 ? pl.lo_t : -std::numeric_limits<double>::infinity();
    // the measurement that set the interval judged nothing: the tight plan starts unretired
    HIP_TRY(hipMemsetAsync(d.d_retired, 0, 8, s->st));
    d.cheb_ab[0] = pl.alpha;
    d.cheb_ab[1] = pl.beta;
    d.cheb_ab[2] = pl.alpha_t;
    d.cheb_ab[3] = pl.beta_t;
    HIP_TRY(hipMemsetAsync(d.d_tight, 0, 8, s->st));
    if ((st = upload_work_table(s, d.Afilt, A.data(), A.size())) != GLD_OK) return st;
    if ((st = upload_work_table(s, d.Bmix, B.data(), B.size())) != GLD_OK) return st;
    if (has_pair) d.lam_hi = pl.hi;  // from now on every pair build checks the bound
    return GLD_OK;
}

// white-noise ring and filter outputs for the current step (at creation and
// after a state is installed): the window of the current block and its
// filter outputs; then the slices the ring holds before this step in an
// uninterrupted run and, past the block's first step (whose own slice
// completes that window), the next block's outputs, which the block's
// earlier steps would have computed
gld_status prime_noise(gld_system *s)
{
    s->win_valid = false;
    if (!s->noise_on) return GLD_OK;
    HIP_TRY(gld::launch_white_ring(s->d, 1, s->st));
    HIP_TRY(gld::launch_fir(s->d, 1, s->st));
    HIP_TRY(gld::launch_white_ring(s->d, 2, s->st));
    if (s->step % s->d.fir_block != 0) HIP_TRY(gld::launch_fir(s->d, 2, s->st));
    return GLD_OK;
}

gld_status refresh_forces(gld_system *s)
{
    // a new configuration: rebuild the cell order and candidate lists
    static const int one = 1;
    HIP_TRY(hipMemcpyAsync(s->d.d_rebuild, &one, sizeof(int), hipMemcpyHostToDevice, s->st));
    HIP_TRY(gld::launch_neighbors(s->d, s->st, s->d.FC));
    HIP_TRY(hipStreamSynchronize(s->st));
    return GLD_OK;
}

// The workspace of gld_create_static: one file-scope device array per GPU,
// which each device holds until the process ends.  Host code never uses the
// array's name as an address (on the host it is a stand-in): the device
// address is looked up once per device with hipGetSymbolAddress and kept.
// One system at a time may live in a device's array.
static __device__ __align__(256) unsigned char scratch[GLD_STATIC_WORKSPACE_BYTES];

struct StaticSlot {
    bool resolved = false;
    void *ptr = nullptr;  // device address of this device's copy of scratch
    bool in_use = false;
};
std::mutex g_static_mu;
std::vector<StaticSlot> g_static;

gld_status acquire_static(int &dev, void *&base)
{
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (static_cast<int>(g_static.size()) <= dev) g_static.resize(dev + 1);
    StaticSlot &sl = g_static[dev];
    if (!sl.resolved) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return fail(GLD_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        sl.ptr = ptr;
        sl.resolved = true;
    }
    if (sl.in_use)
        return fail(GLD_ERR_INVALID_ARG, "the static workspace of device " + std::to_string(dev) +
                                             " holds a live system (gld_destroy it first)");
    sl.in_use = true;
    base = sl.ptr;
    return GLD_OK;
}

void release_static(int dev)
{
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (dev >= 0 && dev < static_cast<int>(g_static.size())) g_static[dev].in_use = false;
}

}  // namespace

extern "C" {

const char *gld_status_string(int status)
{
    switch (status) {
    case GLD_OK: return "ok";
    case GLD_ERR_INVALID_ARG: return "invalid argument";
    case GLD_ERR_NOT_PD: return "noise correlation not positive definite";
    case GLD_ERR_NO_CONV: return "noise approximation did not converge";
    case GLD_ERR_NONFINITE: return "non-finite state";
    case GLD_ERR_OOM: return "workspace too small";
    case GLD_ERR_DEVICE: return "HIP runtime error";
    case GLD_ERR_BOX: return "box too small for the cutoff";
    case GLD_ERR_CAPACITY: return "neighbour list capacity exceeded";
    case GLD_ERR_INTERVAL: return "pair-matrix spectrum outside the noise interval";
    default: return "unknown status";
    }
}

const char *gld_last_error(void) { return g_last_error.c_str(); }

gld_status gld_workspace_size(const gld_params *params, size_t *bytes)
{
    gld_status st = validate(params);
    if (st != GLD_OK) return st;
    if (!bytes) return fail(GLD_ERR_INVALID_ARG, "bytes is NULL");
    Dev d;
    *bytes = carve(params, geometry(params), nullptr, d);
    return GLD_OK;
}

gld_status gld_create(const gld_params *params, const double *r0, const double *v0, void *d_workspace,
                      size_t workspace_bytes, void *hip_stream, gld_system **out)
{
    gld_status st = validate(params);
    if (st != GLD_OK) return st;
    if (!r0 || !v0 || !out || !d_workspace) return fail(GLD_ERR_INVALID_ARG, "NULL pointer argument");
    if (!finite_all(r0, 3 * params->n) || !finite_all(v0, 3 * params->n))
        return fail(GLD_ERR_NONFINITE, "initial state not finite");
    *out = nullptr;
    gld_system *s = new gld_system();
    s->p = *params;
    s->k_self.assign(params->k_self, params->k_self + params->m_max);
    bool pair = params->k_pair_g != nullptr;
    if (params->k_pair) {
        if ((st = separable_form(params, s->w, s->g, pair)) != GLD_OK) {
            delete s;
            return st;
        }
    } else if (pair) {
        s->g.assign(params->k_pair_g, params->k_pair_g + params->m_max);
        s->w.assign(params->k_pair_w, params->k_pair_w + params->n_r);
    }
    s->p.k_self = s->k_self.data();
    s->p.k_pair_g = pair ? s->g.data() : nullptr;
    s->p.k_pair_w = pair ? s->w.data() : nullptr;
    s->p.k_pair = nullptr;
    s->p.dk_self = nullptr;
    if (params->noise_a) {
        s->noise_a.assign(params->noise_a, params->noise_a + static_cast<size_t>(params->noise_rank) * (2 * params->m_max - 1));
        s->noise_b.assign(params->noise_b, params->noise_b + static_cast<size_t>(params->noise_terms) * params->noise_rank);
        s->p.noise_a = s->noise_a.data();
        s->p.noise_b = s->noise_b.data();
    }
    s->geo = geometry(&s->p);
    s->st = static_cast<hipStream_t>(hip_stream);
    s->check_interval = params->check_interval == 0 ? 100 : params->check_interval;
    s->graph_on = s->st != nullptr;  // the legacy null stream cannot be captured
    Dev &d = s->d;
    const size_t need = carve(&s->p, s->geo, static_cast<char *>(d_workspace), d);
    if (workspace_bytes < need) {
        delete s;
        return fail(GLD_ERR_OOM, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " + std::to_string(need));
    }
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) {
        // re-carve from the next 256-byte boundary (the size includes that slack)
        char *b = static_cast<char *>(d_workspace);
        b += 256 - (reinterpret_cast<uintptr_t>(b) & 255);
        carve(&s->p, s->geo, b, d);
    }
    const gld_params &p = s->p;
    d.n = p.n;
    d.S = s->geo.S;
    d.nslots = std::max(0, p.m_max - 1);
    d.M = p.m_max;
    d.P = 2 * p.m_max - 1;
    for (int c = 0; c < 3; ++c) d.box[c] = p.box[c];
    d.dt = p.dt;
    d.mass = p.mass;
    d.kT = p.kT;
    const double x = p.dt * p.k_self[0] / (2.0 * p.mass);  // eq. (aa-bb), isotropic K^s_0
    d.b = 1.0 / (1.0 + x);
    d.a = d.b * (1.0 - x);
    d.r_cut = p.r_cut;
    d.r_cut_min = p.r_cut_min;
    d.r0 = p.r0;
    d.dr = p.dr;
    d.n_r = p.n_r;
    d.parallel = s->geo.parallel;
    d.fp64 = s->geo.fp64;
    d.has_pair = p.k_pair_g != nullptr;
    d.wca_sigma = p.wca_sigma;
    d.wca_eps = p.wca_eps;
    d.seed = p.seed;
    d.cap = s->geo.cap;
    d.maxc = s->geo.maxc;
    d.capS = s->geo.capS;
    d.skin = p.verlet_skin;
    d.rebuild_period = p.rebuild_period;
    d.ncell = s->geo.ncell;
    for (int c = 0; c < 3; ++c) {
        d.nc[c] = s->geo.nc[c];
        if (d.nc[c] == 1) { d.noff[c] = 1; d.offs[c][0] = 0; }
        else if (d.nc[c] == 2) { d.noff[c] = 2; d.offs[c][0] = 0; d.offs[c][1] = 1; }
        else { d.noff[c] = 3; d.offs[c][0] = -1; d.offs[c][1] = 0; d.offs[c][2] = 1; }
    }
    d.g0 = d.has_pair ? p.k_pair_g[0] : 0.0;
    d.check_iters = p.check_iters > 0 ? p.check_iters : gld::kCheckIters;
    {
        // packed pair lists (isotropic tensor): in FP64 always (52 bits:
        // about 1e-16 of the largest weight); in FP32-mixed where a noise plan
        // built here leaves room for 20-bit weights (their rounding moves F^R
        // by about 1e-6 of its rms), not with caller-built filters, whose
        // accuracy the library does not know
        const double tol = p.noise_tol > 0 ? p.noise_tol : (d.fp64 ? gld::kNoiseTolFp64 : gld::kNoiseTolMixed);
        double wmax = 0.0, wmin = 0.0;
        for (int b = 0; d.has_pair && b < p.n_r; ++b) {
            wmax = std::max(wmax, std::fabs(p.k_pair_w[b]));
            wmin = std::min(wmin, p.k_pair_w[b]);
        }
        d.wpack = (!d.parallel && d.has_pair && wmax > 0 &&
                   (d.fp64 || (p.kT > 0 && !p.noise_a && tol >= gld::kNoiseTolMixed))) ? 1 : 0;
        if (d.wpack) {
            d.wq_signed = wmin < 0 ? 1 : 0;
            const double qmax = d.fp64 ? static_cast<double>(d.wq_signed ? gld::kWeightQMaxSigned64 : gld::kWeightQMax64)
                                       : (d.wq_signed ? gld::kWeightQMaxSigned : gld::kWeightQMax);
            d.wq_scale = qmax / wmax;
            d.wq_inv = wmax / qmax;
        }
    }

    auto bail = [&](gld_status e) {
        if (s->st) (void)hipStreamSynchronize(s->st);
        delete s;
        return e;
    };
    if (hipMemsetAsync(d_workspace, 0, need, s->st) != hipSuccess) return bail(fail(GLD_ERR_DEVICE, "workspace clear failed"));
    std::vector<double> zero_w(p.n_r, 0.0);
    std::vector<double> zero_g(p.m_max, 0.0);
    if (hipMemcpyAsync(d.wtab, d.has_pair ? p.k_pair_w : zero_w.data(), p.n_r * sizeof(double), hipMemcpyHostToDevice,
                       s->st) != hipSuccess)
        return bail(fail(GLD_ERR_DEVICE, "upload failed"));
    if ((st = upload_work_table(s, d.ks, p.k_self, p.m_max)) != GLD_OK) return bail(st);
    if ((st = upload_work_table(s, d.gm, d.has_pair ? p.k_pair_g : zero_g.data(), p.m_max)) != GLD_OK) return bail(st);
    d.hist_block = s->geo.fp64 ? gld::kHistBlock64 : gld::kHistBlock32;
    if (d.nslots > 0) {
        // taps of the blocked history convolution: row t + hb - 1 holds
        // (K^s_m, g_m) for the lag m = M - 1 - t
        const int hb = d.hist_block;
        std::vector<double> A(gld::hist_tap_rows(d.nslots, hb) * 2, 0.0);
        for (int t = 0; t < d.nslots; ++t) {
            const int m = d.nslots - t;
            A[static_cast<size_t>(t + hb - 1) * 2] = p.k_self[m];
            A[static_cast<size_t>(t + hb - 1) * 2 + 1] = d.has_pair ? p.k_pair_g[m] : 0.0;
        }
        if ((st = upload_work_table(s, d.hist_taps, A.data(), A.size())) != GLD_OK) return bail(st);
    }
    if ((st = upload_vec<double>(s, d.R, r0)) != GLD_OK) return bail(st);
    if ((st = upload_vec<double>(s, d.V, v0)) != GLD_OK) return bail(st);
    if ((st = set_step(s, 0)) != GLD_OK) return bail(st);
    if ((st = refresh_forces(s)) != GLD_OK) return bail(st);
    if ((st = read_flags(s)) != GLD_OK) return bail(st);
    if ((st = setup_noise(s)) != GLD_OK) return bail(st);
    if ((st = prime_noise(s)) != GLD_OK) return bail(st);
    if (s->noise_on && d.has_pair) {
        // positive definiteness at t = 0 on the chosen interval (Sec. II.B)
        float gm = 0;
        if ((st = run_check_now(s, s->plan.lo, s->plan.hi, s->plan.sing_lo, s->plan.sing_hi, s->theta, &gm)) != GLD_OK)
            return bail(st);
        if ((st = read_flags(s)) != GLD_OK) return bail(st);
    }
    *out = s;
    return GLD_OK;
}

gld_status gld_step(gld_system *s, int64_t n_steps)
{
    if (!s || n_steps < 0) return fail(GLD_ERR_INVALID_ARG, "bad system or step count");
    if (s->latched != GLD_OK) return fail(s->latched, std::string("system is poisoned: ") + gld_status_string(s->latched));
    gld_status st;
    const bool use_graph = s->graph_on && !s->timing;
    const int W = s->d.win;
    if (use_graph)
        for (int64_t k = 0; k < std::min<int64_t>(n_steps, W); ++k) {
            const int sl = static_cast<int>((s->step + k) % W);
            if (!s->graph_ready[sl] && (st = build_graph(s, sl)) != GLD_OK) return st;
        }
    for (int64_t k = 0; k < n_steps; ++k) {
        if (s->noise_on && s->d.has_pair && s->check_interval > 0 && s->step > 0 && s->step % s->check_interval == 0)
            if ((st = enqueue_check(s)) != GLD_OK) return st;
        const int slot = static_cast<int>(s->step % W);
        // a state installed mid-window: the rest of that window at the
        // installed positions
        if (slot != 0 && !s->win_valid && (st = enqueue_window(s)) != GLD_OK) return st;
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(s->gexec[slot], s->st));
        } else if ((st = enqueue_step(s, slot)) != GLD_OK) {
            return st;
        }
        s->win_valid = true;
        ++s->step;
    }
    return GLD_OK;
}

gld_status gld_sync(gld_system *s)
{
    if (!s) return fail(GLD_ERR_INVALID_ARG, "NULL system");
    return read_flags(s);
}

gld_status gld_read_state(gld_system *s, gld_state *o)
{
    if (!s || !o) return fail(GLD_ERR_INVALID_ARG, "NULL argument");
    gld_status flag = read_flags(s);
    if (flag == GLD_ERR_DEVICE) return flag;
    gld_status st;
    const Dev &d = s->d;
    if (o->r && (st = download_vec<double>(s, o->r, d.R)) != GLD_OK) return st;
    if (o->v && (st = download_vec<double>(s, o->v, d.V)) != GLD_OK) return st;
    if (o->f_c && (st = download_vec<double>(s, o->f_c, d.FC)) != GLD_OK) return st;
    if (o->f_d && (st = download_work_vec(s, o->f_d, d.FD)) != GLD_OK) return st;
    if (o->f_r && (st = download_work_vec(s, o->f_r, d.FR)) != GLD_OK) return st;
    if (o->history && d.nslots > 0) {
        const size_t elt = s->geo.fp64 ? 8 : 4;
        const int64_t n = s->p.n;
        for (int m = 1; m <= d.nslots; ++m) {
            int slot = static_cast<int>(((s->step - m) % d.nslots + d.nslots) % d.nslots);
            const void *src = static_cast<const char *>(d.ring) + static_cast<size_t>(slot) * 3 * d.S * elt;
            if ((st = download_work_vec(s, o->history + static_cast<size_t>(m - 1) * n * 3, src)) != GLD_OK) return st;
        }
    }
    o->step = s->step;
    int flags[2] = {0, 0};
    long long fstep = 0;
    HIP_TRY(hipMemcpy(flags, d.d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&fstep, d.d_flag_step, sizeof(fstep), hipMemcpyDeviceToHost));
    o->flags = flags[0];
    o->flag_step = fstep;
    return flag;
}

gld_status gld_write_state(gld_system *s, const gld_state *in)
{
    if (!s || !in || !in->r || !in->v) return fail(GLD_ERR_INVALID_ARG, "NULL argument");
    if (in->step < 0 || in->step > (int64_t(1) << 60)) return fail(GLD_ERR_INVALID_ARG, "step must be in [0, 2^60]");
    if (!finite_all(in->r, 3 * s->p.n) || !finite_all(in->v, 3 * s->p.n))
        return fail(GLD_ERR_NONFINITE, "state not finite");
    HIP_TRY(hipStreamSynchronize(s->st));
    gld_status st;
    Dev &d = s->d;
    if ((st = upload_vec<double>(s, d.R, in->r)) != GLD_OK) return st;
    if ((st = upload_vec<double>(s, d.V, in->v)) != GLD_OK) return st;
    if ((st = set_step(s, in->step)) != GLD_OK) return st;
    const size_t elt = s->geo.fp64 ? 8 : 4;
    if (d.nslots > 0) {
        const int64_t n = s->p.n;
        if (in->history) {
            if (!finite_all(in->history, static_cast<int64_t>(d.nslots) * 3 * n))
                return fail(GLD_ERR_NONFINITE, "history not finite");
            for (int m = 1; m <= d.nslots; ++m) {
                int slot = static_cast<int>(((in->step - m) % d.nslots + d.nslots) % d.nslots);
                void *dst = static_cast<char *>(d.ring) + static_cast<size_t>(slot) * 3 * d.S * elt;
                if ((st = upload_work_vec(s, dst, in->history + static_cast<size_t>(m - 1) * n * 3)) != GLD_OK) return st;
            }
        } else {
            HIP_TRY(hipMemsetAsync(d.ring, 0, static_cast<size_t>(d.nslots) * 3 * d.S * elt, s->st));
        }
    }
    HIP_TRY(hipMemsetAsync(d.FD, 0, 3 * d.S * elt, s->st));
    HIP_TRY(hipMemsetAsync(d.FR, 0, 3 * d.S * elt, s->st));
    if ((st = clear_flags(s)) != GLD_OK) return st;
    if ((st = refresh_forces(s)) != GLD_OK) return st;
    if ((st = prime_noise(s)) != GLD_OK) return st;
    // the history's block products of the block holding this step and of the
    // next one (the steps of this block would have computed the latter)
    HIP_TRY(gld::launch_history_block(s->d, 1, s->st));
    HIP_TRY(gld::launch_history_block(s->d, 2, s->st));
    // the installed configuration against the noise interval and the
    // singular points, as at creation (Sec. II.B: positive definiteness is
    // checked on the fly); its smallest Ritz value also decides whether the
    // tight plan may be used.  A failure latches GLD_ERR_INTERVAL or
    // GLD_ERR_NOT_PD at the written step, returned here.
    if (s->noise_on && s->d.has_pair) {
        double th[2];
        if ((st = run_check_now(s, s->plan.lo, s->plan.hi, s->plan.sing_lo, s->plan.sing_hi, th, nullptr)) != GLD_OK)
            return st;
    }
    return read_flags(s);
}

gld_status gld_noise_parameters(const gld_system *s, gld_noise_info *o)
{
    if (!s || !o) return fail(GLD_ERR_INVALID_ARG, "NULL argument");
    o->cheb_terms = s->noise_on ? s->plan.K : 0;
    o->rank = s->noise_on ? s->plan.r : 0;
    o->block = s->d.fir_block;
    o->lam_lo = s->plan.lo;
    o->lam_hi = s->plan.hi;
    o->lam_singular = s->plan.sing_lo;
    o->err_estimate = s->plan.err_cheb + s->plan.err_rank + s->plan.err_window;
    o->window_half = s->noise_on ? s->plan.half : 0;
    o->noise_window = s->d.win;
    o->cheb_terms_tight = s->noise_on ? s->plan.Kt : 0;
    o->lam_hi_tight = s->noise_on ? s->plan.hi_t : 0.0;
    o->lam_lo_tight = s->noise_on ? s->plan.lo_t : 0.0;
    o->tight_steps = 0;
    if (s->noise_on && s->d.d_tight) {
        unsigned long long n = 0;
        HIP_TRY(hipStreamSynchronize(s->st));
        HIP_TRY(hipMemcpy(&n, s->d.d_tight, sizeof(n), hipMemcpyDeviceToHost));
        o->tight_steps = static_cast<int64_t>(n);
    }
    // entry nst of each cell's stencil row holds (0, total)
    std::vector<int2> stab(static_cast<size_t>(s->d.ncell) * 28);
    HIP_TRY(hipStreamSynchronize(s->st));
    HIP_TRY(hipMemcpy(stab.data(), s->d.stab, stab.size() * sizeof(int2), hipMemcpyDeviceToHost));
    int most = 0;
    const int nst = s->d.noff[0] * s->d.noff[1] * s->d.noff[2];
    for (int c = 0; c < s->d.ncell; ++c) most = std::max(most, stab[static_cast<size_t>(c) * 28 + nst].y);
    o->list_index_bits = most <= 4096 ? 12 : 16;
    double th[2] = {0, 0};
    int retired = 0;
    HIP_TRY(hipMemcpy(th, s->d.lab + 2 * gld::kMaxCheckIters, sizeof(th), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&retired, s->d.d_retired, sizeof(int), hipMemcpyDeviceToHost));
    o->theta_min = th[0];
    o->theta_max = th[1];
    o->tight_retired = retired;
    o->filters_given = s->filters_given ? 1 : 0;
    o->list_weight_bits = s->d.wpack ? (s->d.fp64 ? 52 : 20) : (s->d.fp64 ? 64 : 32);
    return GLD_OK;
}

gld_status gld_list_stats(gld_system *s, int64_t *pairs, int32_t *max_per_particle)
{
    if (!s || !pairs) return fail(GLD_ERR_INVALID_ARG, "NULL argument");
    std::vector<int> nn(static_cast<size_t>(s->p.n));
    HIP_TRY(hipStreamSynchronize(s->st));
    HIP_TRY(hipMemcpy(nn.data(), s->d.nn, nn.size() * sizeof(int), hipMemcpyDeviceToHost));
    int64_t tot = 0;
    int most = 0;
    for (int v : nn) {
        tot += v;
        most = std::max(most, v);
    }
    *pairs = tot;
    if (max_per_particle) *max_per_particle = most;
    return GLD_OK;
}

gld_status gld_set_graph(gld_system *s, int enable)
{
    if (!s) return fail(GLD_ERR_INVALID_ARG, "NULL system");
    s->graph_on = enable && s->st != nullptr;
    return GLD_OK;
}

gld_status gld_set_timing(gld_system *s, int enable)
{
    if (!s) return fail(GLD_ERR_INVALID_ARG, "NULL system");
    HIP_TRY(hipStreamSynchronize(s->st));
    s->timing = enable != 0;
    s->pending.clear();
    s->pool_used = 0;
    for (int k = 0; k < GLD_K_COUNT; ++k) {
        s->ms[k] = 0;
        s->cnt[k] = 0;
    }
    return GLD_OK;
}

gld_status gld_kernel_times(gld_system *s, double *ms_sum, int64_t *launches)
{
    if (!s || !ms_sum || !launches) return fail(GLD_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(hipStreamSynchronize(s->st));
    for (auto &[cls, idx, n] : s->pending) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, s->pool[idx], s->pool[idx + 1]));
        s->ms[cls] += ms;
        s->cnt[cls] += n;
    }
    s->pending.clear();
    s->pool_used = 0;
    for (int k = 0; k < GLD_K_COUNT; ++k) {
        ms_sum[k] = s->ms[k];
        launches[k] = s->cnt[k];
    }
    return GLD_OK;
}

gld_status gld_destroy(gld_system *s)
{
    if (!s) return GLD_OK;
    if (s->st) (void)hipStreamSynchronize(s->st);
    else (void)hipDeviceSynchronize();
    drop_graph(s);
    for (auto e : s->pool) (void)hipEventDestroy(e);
    if (s->static_device >= 0) release_static(s->static_device);
    delete s;
    return GLD_OK;
}

gld_status gld_create_static(const gld_params *params, const double *r0, const double *v0, void *hip_stream,
                             gld_system **out)
{
    gld_status st = validate(params);
    if (st != GLD_OK) return st;
    if (!out) return fail(GLD_ERR_INVALID_ARG, "NULL pointer argument");
    *out = nullptr;
    size_t need = 0;
    {
        Dev d;
        need = carve(params, geometry(params), nullptr, d);
    }
    if (need > GLD_STATIC_WORKSPACE_BYTES)
        return fail(GLD_ERR_OOM, "system needs " + std::to_string(need) + " workspace bytes; the static workspace "
                                 "holds GLD_STATIC_WORKSPACE_BYTES = " + std::to_string(GLD_STATIC_WORKSPACE_BYTES));
    int dev = 0;
    void *base = nullptr;
    if ((st = acquire_static(dev, base)) != GLD_OK) return st;
    st = gld_create(params, r0, v0, base, GLD_STATIC_WORKSPACE_BYTES, hip_stream, out);
    if (st != GLD_OK) {
        release_static(dev);
        return st;
    }
    (*out)->static_device = dev;
    return GLD_OK;
}

gld_status gld_build_noise_filters(const gld_params *params, double lam_lo, double lam_hi, double tol, double *a_out,
                                   size_t a_cap, double *b_out, size_t b_cap, gld_noise_info *info)
{
    gld_status st = validate(params);
    if (st != GLD_OK) return st;
    if (!a_out || !b_out || !info) return fail(GLD_ERR_INVALID_ARG, "NULL argument");
    if (!(params->kT > 0)) return fail(GLD_ERR_INVALID_ARG, "kT must be > 0 for a noise construction");
    if (tol <= 0) tol = params->precision == GLD_FP64 ? gld::kNoiseTolFp64 : gld::kNoiseTolMixed;
    NoisePlan plan;
    std::string err;
    gld_params q = *params;
    std::vector<double> wv, gv;
    if (params->k_pair) {
        bool any = false;
        if ((st = separable_form(params, wv, gv, any)) != GLD_OK) return st;
        q.k_pair_w = any ? wv.data() : nullptr;
        q.k_pair_g = any ? gv.data() : nullptr;
        q.k_pair = nullptr;
    }
    st = gld::noise_build(q, lam_lo, lam_hi, tol, plan, err);
    if (st != GLD_OK) return fail(st, err);
    if (a_cap < plan.Afilt.size() || b_cap < plan.Bmix.size())
        return fail(GLD_ERR_INVALID_ARG, "output capacity too small");
    std::copy(plan.Afilt.begin(), plan.Afilt.end(), a_out);
    std::copy(plan.Bmix.begin(), plan.Bmix.end(), b_out);
    info->cheb_terms = plan.K;
    info->rank = plan.r;
    info->block = 0;
    info->lam_lo = plan.lo;
    info->lam_hi = plan.hi;
    info->lam_singular = plan.sing_lo;
    info->err_estimate = plan.err_cheb + plan.err_rank + plan.err_window;
    info->window_half = plan.half;
    info->noise_window = std::max(1, params->noise_window);
    info->cheb_terms_tight = 0;
    info->lam_hi_tight = 0.0;
    info->lam_lo_tight = 0.0;
    info->tight_steps = 0;
    info->list_index_bits = 0;
    info->theta_min = info->theta_max = 0.0;
    info->tight_retired = 0;
    info->filters_given = 0;
    info->list_weight_bits = 0;
    return GLD_OK;
}

gld_status gld_white_noise(uint64_t seed, int64_t n, int64_t t0, int64_t n_t, double *d_out, uint32_t *d_raw,
                           void *hip_stream)
{
    if (n < 0 || n_t < 0 || n > (int64_t(1) << 32)) return fail(GLD_ERR_INVALID_ARG, "bad sizes");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(gld::launch_white_noise(seed, n, t0, n_t, d_out, d_raw, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GLD_OK;
}

}  // extern "C"
