// One-off FP64 construction of the colored-noise filters (host side).
//
// Paper: Sec. II.C.  The random force F_n must have lag covariances
// kT a_m K_m / dt (eq. stochastic_force2, a_0 = 2, a_m = 1), and is produced
// as F_n = sum_s A_s W_{n+s} (eq. noise_production) with the A_s defined per
// frequency as the square roots of the DFT of the correlation matrices
// (eq. FT, Algorithm 1).  With time-scale separation the kernel transforms
// are precomputed once (Sec. II.C, remarks after Algorithm 1); this file is
// that precomputation.  Instead of a Lanczos run per frequency and per step,
// the square-root function of every frequency is expanded in one common
// Chebyshev basis of the pair-weight matrix P, which turns the per-step work
// into a small white-noise filter bank plus a short chain of pair mat-vecs.
#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "gld_internal.h"

namespace gld {

namespace {

// cos(2 pi w m / P) with the phase reduced exactly in integers
inline double cos_phase(long long w, long long m, long long P)
{
    long long ph = (w * m) % P;
    if (ph < 0) ph += P;
    return std::cos(6.283185307179586476925286766559 * static_cast<double>(ph) / static_cast<double>(P));
}

// One-sided Jacobi (Hestenes) SVD of X (rows x cols, column-major columns):
// on return the columns of X are U_q sigma_q and V (cols x cols, row-major)
// holds the right singular vectors, so X_in = X_out V^T.
void hestenes_svd(int rows, int cols, std::vector<double> &X, std::vector<double> &V)
{
    V.assign(static_cast<size_t>(cols) * cols, 0.0);
    for (int i = 0; i < cols; ++i) V[static_cast<size_t>(i) * cols + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < cols - 1; ++p)
            for (int q = p + 1; q < cols; ++q) {
                double *xp = &X[static_cast<size_t>(p) * rows];
                double *xq = &X[static_cast<size_t>(q) * rows];
                double a = 0, b = 0, g = 0;
                for (int i = 0; i < rows; ++i) {
                    a += xp[i] * xp[i];
                    b += xq[i] * xq[i];
                    g += xp[i] * xq[i];
                }
                if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
                rotated = true;
                const double zeta = (b - a) / (2.0 * g);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < rows; ++i) {
                    const double u = xp[i], v = xq[i];
                    xp[i] = c * u - s * v;
                    xq[i] = s * u + c * v;
                }
                for (int i = 0; i < cols; ++i) {
                    double &vp = V[static_cast<size_t>(i) * cols + p];
                    double &vq = V[static_cast<size_t>(i) * cols + q];
                    const double u = vp, v = vq;
                    vp = c * u - s * v;
                    vq = s * u + c * v;
                }
            }
        if (!rotated) break;
    }
}

}  // namespace

gld_status noise_spectra(const gld_params &p, NoisePlan &plan, std::string &err)
{
    const int M = p.m_max;
    const int P = 2 * M - 1;
    plan.M = M;
    plan.P = P;
    plan.S.assign(M, 0.0);
    plan.G.assign(M, 0.0);
    const bool has_pair = p.k_pair_g && p.k_pair_w;
    std::vector<double> cs(M), cg(M, 0.0);
    for (int m = 0; m < M; ++m) {
        const double am = (m == 0) ? 2.0 : 1.0;
        cs[m] = p.kT * am * p.k_self[m] / p.dt;
        if (has_pair) cg[m] = p.kT * am * p.k_pair_g[m] / p.dt;
    }
    for (int w = 0; w < M; ++w) {
        double s = cs[0], g = cg[0];
        for (int m = 1; m < M; ++m) {
            const double c = cos_phase(w, m, P);
            s += 2.0 * cs[m] * c;
            g += 2.0 * cg[m] * c;
        }
        plan.S[w] = s;
        plan.G[w] = g;
    }
    double lo = -std::numeric_limits<double>::infinity();
    double hi = std::numeric_limits<double>::infinity();
    for (int w = 0; w < M; ++w) {
        const double s = plan.S[w], g = plan.G[w];
        if (g > 0) lo = std::max(lo, -s / g);
        if (g < 0) hi = std::min(hi, s / (-g));
        if (g == 0 && !(s > 0) && p.kT > 0) {
            err = "self noise spectrum is not positive at frequency " + std::to_string(w);
            return GLD_ERR_NOT_PD;
        }
    }
    plan.sing_lo = lo;
    plan.sing_hi = hi;
    return GLD_OK;
}

namespace {

// Chebyshev coefficients c_k(w) of f_w(x) = sqrt(S_w + G_w x) on [lo, hi],
// truncated after the smallest K whose tail error is within tol/2, and the
// time-domain rows X[k][t] = (1/P) sum_{w=-(M-1)}^{M-1} c_k(|w|) cos(2 pi w t / P),
// t = -(M-1)..M-1 (P entries per row).
gld_status cheb_rows(const NoisePlan &plan, double lo, double hi, double tol, double sig, int &K, double &err_cheb,
                     std::vector<double> &X, std::string &err)
{
    const int M = plan.M, P = plan.P;
    const int Kc = kMaxCheb;
    const int nq = 2 * Kc;
    std::vector<double> costab(static_cast<size_t>(Kc) * nq), lam(nq);
    for (int j = 0; j < nq; ++j) {
        const double th = M_PI * (j + 0.5) / nq;
        lam[j] = 0.5 * (hi - lo) * std::cos(th) + 0.5 * (hi + lo);
        for (int k = 0; k < Kc; ++k) costab[static_cast<size_t>(k) * nq + j] = std::cos(k * th);
    }
    std::vector<double> c(static_cast<size_t>(Kc) * M);  // c[k][w]
    std::vector<double> fv(nq);
    for (int w = 0; w < M; ++w) {
        double fmax = 0;
        for (int j = 0; j < nq; ++j) {
            fv[j] = std::sqrt(plan.S[w] + plan.G[w] * lam[j]);
            fmax = std::max(fmax, std::fabs(fv[j]));
        }
        // coefficients below the round-off floor of the quadrature sum carry
        // no information (the true ones decay geometrically below it)
        const double floor_w = 64.0 * std::numeric_limits<double>::epsilon() * fmax;
        for (int k = 0; k < Kc; ++k) {
            const double *ct = &costab[static_cast<size_t>(k) * nq];
            double s = 0;
            for (int j = 0; j < nq; ++j) s += fv[j] * ct[j];
            s = (k == 0 ? 1.0 : 2.0) * s / nq;
            c[static_cast<size_t>(k) * M + w] = std::fabs(s) < floor_w ? 0.0 : s;
        }
    }
    // relative rms error of truncating after K terms:
    //   sum_w wt_w (sum_{k>=K} |c_k(w)|)^2 / sum_w wt_w S_w,  wt = 1 (w=0), 2
    std::vector<double> tail(M, 0.0);
    K = Kc;
    err_cheb = 0;
    for (int k = Kc - 1; k >= 0; --k) {
        double e2 = 0;
        for (int w = 0; w < M; ++w) e2 += (w == 0 ? 1.0 : 2.0) * tail[w] * tail[w];
        const double e = std::sqrt(e2 / sig);
        if (e > 0.5 * tol) break;
        K = k + 1;
        err_cheb = e;
        for (int w = 0; w < M; ++w) tail[w] += std::fabs(c[static_cast<size_t>(k) * M + w]);
    }
    // K: smallest count whose tail error is within tol/2.  K = kMaxCheb means
    // even the last coefficient is too large: the interval is too close to a
    // singular point for this tolerance.
    if (K >= Kc - 8) {
        err = "Chebyshev expansion of the noise does not reach the tolerance within " + std::to_string(Kc) +
              " terms (interval too close to a singular point)";
        return GLD_ERR_NO_CONV;
    }
    std::vector<double> cosm(static_cast<size_t>(M) * M);
    for (int w = 0; w < M; ++w)
        for (int t = 0; t < M; ++t) cosm[static_cast<size_t>(w) * M + t] = cos_phase(w, t, P);
    X.assign(static_cast<size_t>(K) * P, 0.0);
    for (int k = 0; k < K; ++k) {
        const double *ck = &c[static_cast<size_t>(k) * M];
        for (int t = 0; t < M; ++t) {
            double s = ck[0];
            for (int w = 1; w < M; ++w) s += 2.0 * ck[w] * cosm[static_cast<size_t>(w) * M + t];
            s /= P;
            X[static_cast<size_t>(k) * P + (M - 1) + t] = s;
            X[static_cast<size_t>(k) * P + (M - 1) - t] = s;
        }
    }
    return GLD_OK;
}

}  // namespace

gld_status noise_build(const gld_params &p, double lo, double hi, double tol, NoisePlan &plan,
                       std::string &err, double hi_tight, double lo_tight)
{
    gld_status st = noise_spectra(p, plan, err);
    if (st != GLD_OK) return st;
    const int M = plan.M, P = plan.P;
    if (!(hi > lo)) {
        err = "noise interval must satisfy lam_hi > lam_lo";
        return GLD_ERR_INVALID_ARG;
    }
    plan.lo = lo;
    plan.hi = hi;
    plan.alpha = 2.0 / (hi - lo);
    plan.beta = -(hi + lo) / (hi - lo);
    // positive definiteness of every K_hat_w on the interval (linear in lambda)
    for (int w = 0; w < M; ++w) {
        const double a = plan.S[w] + plan.G[w] * lo, b = plan.S[w] + plan.G[w] * hi;
        if (!(a > 0) || !(b > 0)) {
            err = "noise correlation not positive definite on [" + std::to_string(lo) + ", " +
                  std::to_string(hi) + "] at frequency " + std::to_string(w) +
                  " (singular points " + std::to_string(plan.sing_lo) + ", " + std::to_string(plan.sing_hi) + ")";
            return GLD_ERR_NOT_PD;
        }
    }
    double sig = 0;
    for (int w = 0; w < M; ++w) sig += (w == 0 ? 1.0 : 2.0) * plan.S[w];
    if (!(sig > 0)) {
        err = "zero self noise power";
        return GLD_ERR_NOT_PD;
    }
    int K = 0;
    double err_cheb = 0;
    std::vector<double> X;  // rows of the plan on [lo, hi], then those of the tight plan
    if ((st = cheb_rows(plan, lo, hi, tol, sig, K, err_cheb, X, err)) != GLD_OK) return st;
    int Kt = 0;
    double err_t = 0;
    const double lo_t = std::max(lo, lo_tight);
    if (hi_tight > lo_t && hi_tight < hi) {
        std::vector<double> Xt;
        if ((st = cheb_rows(plan, lo_t, hi_tight, tol, sig, Kt, err_t, Xt, err)) != GLD_OK) return st;
        if (Kt < K) X.insert(X.end(), Xt.begin(), Xt.end());
        else Kt = 0;  // no saving
    }
    const int Ka = K + Kt;
    // one filter bank for both plans: the leading singular vectors of the
    // stacked rows; X = C^T as Ka columns of length P
    std::vector<double> Vr;
    hestenes_svd(P, Ka, X, Vr);
    std::vector<int> order(Ka);
    std::vector<double> sv(Ka);
    for (int q = 0; q < Ka; ++q) {
        double s = 0;
        for (int i = 0; i < P; ++i) s += X[static_cast<size_t>(q) * P + i] * X[static_cast<size_t>(q) * P + i];
        sv[q] = std::sqrt(s);
        order[q] = q;
    }
    std::sort(order.begin(), order.end(), [&](int a, int b) { return sv[a] > sv[b]; });
    // Truncation error of the rank-r filter bank.  Along an eigenvector of P
    // with eigenvalue x the error is sum_t (dC^T tau)_t xi_t, xi_t iid N(0,1),
    // tau_k = T_k(x~), |tau|^2 <= K; hence its rms relative to the signal
    // (variance c0 = sig / P per component) is at most
    //     sqrt(K) ||dC||_2 / sqrt(c0),  ||dC||_2 = sigma_{r+1}
    // (for either plan: its rows are part of the stacked matrix, and K >= Kt).
    // Error budget: Chebyshev tail tol/2, rank tol/4, filter window tol/4.
    // Smallest r with the rank bound within tol/4:
    const double c0 = sig / P;
    int r = Ka;
    for (int q = Ka - 1; q >= 1; --q) {
        if (std::sqrt(static_cast<double>(K) / c0) * sv[order[q]] > 0.25 * tol) break;  // keep order[q]
        r = q;
    }
    const double dropped_max = r < Ka ? sv[order[r]] : 0.0;
    if (r > kMaxRank) {
        err = "noise filter bank needs rank " + std::to_string(r) + " > " + std::to_string(kMaxRank);
        return GLD_ERR_NO_CONV;
    }
    plan.K = K;
    plan.r = r;
    plan.err_cheb = err_cheb;
    plan.err_rank = std::sqrt(static_cast<double>(K) / c0) * dropped_max;
    plan.Kt = Kt;
    plan.lo_t = Kt > 0 ? lo_t : 0.0;
    plan.hi_t = Kt > 0 ? hi_tight : 0.0;
    plan.alpha_t = Kt > 0 ? 2.0 / (hi_tight - lo_t) : 0.0;
    plan.beta_t = Kt > 0 ? -(hi_tight + lo_t) / (hi_tight - lo_t) : 0.0;
    plan.err_cheb_t = err_t;
    plan.Bmix.assign(static_cast<size_t>(K) * r, 0.0);
    plan.Bmix_t.assign(static_cast<size_t>(Kt) * r, 0.0);
    plan.Afilt.assign(static_cast<size_t>(r) * P, 0.0);
    for (int qq = 0; qq < r; ++qq) {
        const int q = order[qq];
        const double s = sv[q];
        for (int k = 0; k < K; ++k) plan.Bmix[static_cast<size_t>(k) * r + qq] = Vr[static_cast<size_t>(k) * Ka + q] * s;
        for (int k = 0; k < Kt; ++k)
            plan.Bmix_t[static_cast<size_t>(k) * r + qq] = Vr[static_cast<size_t>(K + k) * Ka + q] * s;
        for (int t = 0; t < P; ++t)
            plan.Afilt[static_cast<size_t>(qq) * P + t] = (s > 0) ? X[static_cast<size_t>(q) * P + t] / s : 0.0;
    }
    // Filter window.  The taps decay with the memory; dropping the lags
    // |t| > h changes C = B A by dC (its columns |t| > h), with the same
    // bound as above: sqrt(K) ||dC||_F / sqrt(c0) <= tol/4, the columns of
    // both plans counted together.  Smallest h:
    std::vector<double> col2(P, 0.0);  // squared column norms of B A
    for (int t = 0; t < P; ++t) {
        double acc = 0;
        for (int k = 0; k < Ka; ++k) {
            const double *brow = k < K ? &plan.Bmix[static_cast<size_t>(k) * r] : &plan.Bmix_t[static_cast<size_t>(k - K) * r];
            double v = 0;
            for (int q = 0; q < r; ++q) v += brow[q] * plan.Afilt[static_cast<size_t>(q) * P + t];
            acc += v * v;
        }
        col2[t] = acc;
    }
    int h = M - 1;
    double dropped2 = 0;
    while (h > 0) {
        const double add = col2[(M - 1) - h] + col2[(M - 1) + h];
        if (std::sqrt(static_cast<double>(K) * (dropped2 + add) / c0) > 0.25 * tol) break;
        dropped2 += add;
        --h;
    }
    plan.half = h;
    plan.err_window = std::sqrt(static_cast<double>(K) * dropped2 / c0);
    for (int q = 0; q < r; ++q)
        for (int t = 0; t < P; ++t)
            if (std::abs(t - (M - 1)) > h) plan.Afilt[static_cast<size_t>(q) * P + t] = 0.0;
    return GLD_OK;
}
}  // namespace gld
