// SRJ schedule planner (host, C++).
//
// Optimal weights.  The scheme minimises max over kappa in [km, kM] of
// log Gamma(kappa) = sum_i beta_i log|1 - w_i kappa| (Sec. 3.1, Eq. Gamma) over the weights
// w and the fractions beta (sum 1).  At the optimum log Gamma has P + 1 equal maxima: at
// km, at one interior point kappa_j between each pair of zeros 1/w_j < 1/w_{j+1}, and at
// kM (Sec. 3.2, Eq. equMax).  This planner solves the first-order (KKT) conditions of
// that minimax problem directly:
//   * beta from the P - 1 stationarity conditions of Eq. partialG at the interior kappa_j
//     plus sum beta = 1 (a P x P linear solve);
//   * multipliers lambda_0..lambda_P >= 0 on the P + 1 active maxima with
//     sum_j lambda_j kappa_j / (1 - w_i kappa_j) = 0 for every i (stationarity in w), whose
//     solution is the partial-fraction residue
//     lambda_j ~ prod_i (w_i - 1/kappa_j) / prod_{l != j} (1/kappa_l - 1/kappa_j);
//   * equations: the P equal-maxima conditions and stationarity in beta,
//     sum_j lambda_j log|1 - w_i kappa_j| equal for all i (P - 1 conditions).
// Unknowns are the 2P - 1 values (w, kappa_1..kappa_{P-1}), as in the reduced system of
// Sec. 3.5; they are parametrised so that every weight stays inside (1/kM, 1/km) and every
// kappa_j inside (1/w_j, 1/w_{j+1}).  The system is solved in extended precision by damped
// Newton (Levenberg-Marquardt as fallback), growing the number of levels at a moderate
// resolution and then continuing in log km to the target (Sec. 3.3: starting values from
// solved neighbours).
//
// Integer counts: q_i = floor(beta_i / beta_1) (Sec. 4.3).
//
// Step order: the paper asks only that the large over-relaxations be spread over the
// cycle (Sec. 5.1).  Two orders are offered: "even spread" (the r-th use of weight i at
// (r + 1/2) / q_i of the cycle) and "balanced greedy", which keeps the partial product
// of the cycle close to the geometric path towards the full cycle factor in every mode;
// the latter bounds the transient amplification of rounding errors far better.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace srj {

using ld = long double;

static const double kPi = 3.14159265358979323846;

static double grid_kappa(int ndim, const int64_t* n, const double* wt, bool lowest)
{
    double s = 0.0;
    for (int i = 0; i < ndim; ++i) {
        const double a = kPi / (2.0 * (double)(n[i] + 1));
        const double v = lowest ? std::sin(a) : std::cos(a);
        const double axis = (!wt || i == 0) ? 1.0 : wt[i - 1];
        s = s + (wt ? axis * (v * v) : v * v);
    }
    return wt ? (4.0 * s) / wt[2] : (2.0 / (double)ndim) * s;
}

double grid_kappa_min(int ndim, const int64_t* n, const double* wt) { return grid_kappa(ndim, n, wt, true); }

double grid_kappa_max(int ndim, const int64_t* n, const double* wt) { return grid_kappa(ndim, n, wt, false); }

double neumann_kappa_min(int ndim, const int64_t* n, const double* wt)
{
    double m = 0.0;
    for (int i = 0; i < ndim; ++i) {
        const double v = std::sin(kPi / (2.0 * (double)n[i]));
        const double axis = (!wt || i == 0) ? 1.0 : wt[i - 1];
        const double t = axis * (v * v);
        if (i == 0 || t < m) m = t;
    }
    return wt ? (4.0 * m) / wt[2] : (2.0 / (double)ndim) * m;
}

double neumann_kappa_max(int ndim, const int64_t* n, const double* wt)
{
    double s = 0.0;
    for (int i = 0; i < ndim; ++i) {
        const double v = std::cos(kPi / (2.0 * (double)n[i]));
        const double axis = (!wt || i == 0) ? 1.0 : wt[i - 1];
        s = s + (wt ? axis * (v * v) : v * v);
    }
    return wt ? (4.0 * s) / wt[2] : (2.0 / (double)ndim) * s;
}

// ----------------------------------------------------------------- the system

namespace {

struct Sys {
    int P;
    ld km, kM, a, c;  // interval and its logs
};

inline ld sigm(ld x) { return 1.0L / (1.0L + expl(-x)); }

inline ld log_abs_one_minus(ld w, ld k)
{
    ld x = w * k;
    return (fabsl(x) < 0.5L) ? log1pl(-x) : logl(fabsl(1.0L - x));
}

void unpack(const Sys& s, const ld* z, ld* w, ld* kap)
{
    ld lw[SRJ_PLAN_MAXP];
    for (int i = 0; i < s.P; ++i) {
        lw[i] = -(s.a + sigm(z[i]) * (s.c - s.a));
        w[i] = expl(lw[i]);
    }
    for (int j = 0; j + 1 < s.P; ++j) kap[j] = expl(-lw[j] + sigm(z[s.P + j]) * (lw[j] - lw[j + 1]));
}

void pack(const Sys& s, const ld* w, const ld* kap, ld* z)
{
    ld lw[SRJ_PLAN_MAXP];
    for (int i = 0; i < s.P; ++i) {
        lw[i] = logl(w[i]);
        ld t = (-lw[i] - s.a) / (s.c - s.a);
        z[i] = logl(t / (1.0L - t));
    }
    for (int j = 0; j + 1 < s.P; ++j) {
        ld th = (logl(kap[j]) + lw[j]) / (lw[j] - lw[j + 1]);
        z[s.P + j] = logl(th / (1.0L - th));
    }
}

// Gaussian elimination with partial pivoting; A is n x n row-major, b is overwritten.
bool linsolve(int n, ld* A, ld* b)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabsl(A[i * n + k]) > fabsl(A[p * n + k])) p = i;
        if (!(fabsl(A[p * n + k]) > 0.0L)) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
            std::swap(b[k], b[p]);
        }
        for (int i = k + 1; i < n; ++i) {
            ld f = A[i * n + k] / A[k * n + k];
            if (f == 0.0L) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        ld v = b[k];
        for (int j = k + 1; j < n; ++j) v -= A[k * n + j] * b[j];
        b[k] = v / A[k * n + k];
    }
    return true;
}

struct Eval {
    ld w[SRJ_PLAN_MAXP], kap[SRJ_PLAN_MAXP], beta[SRJ_PLAN_MAXP], lam[SRJ_PLAN_MAXP + 1];
};

// F has 2P - 1 entries.  Returns false if the evaluation is not finite.
bool residual(const Sys& s, const ld* z, ld* F, Eval* ev)
{
    const int P = s.P;
    unpack(s, z, ev->w, ev->kap);
    const ld* w = ev->w;
    // beta: stationarity of log Gamma at each interior kappa_j, and sum beta = 1
    ld A[SRJ_PLAN_MAXP * SRJ_PLAN_MAXP], rhs[SRJ_PLAN_MAXP];
    for (int j = 0; j + 1 < P; ++j) {
        for (int i = 0; i < P; ++i) A[j * P + i] = w[i] / (1.0L - ev->kap[j] * w[i]);
        rhs[j] = 0.0L;
    }
    for (int i = 0; i < P; ++i) A[(P - 1) * P + i] = 1.0L;
    rhs[P - 1] = 1.0L;
    if (!linsolve(P, A, rhs)) return false;
    for (int i = 0; i < P; ++i) ev->beta[i] = rhs[i];
    ld K[SRJ_PLAN_MAXP + 1];
    K[0] = s.km;
    for (int j = 0; j + 1 < P; ++j) K[j + 1] = ev->kap[j];
    K[P] = s.kM;
    auto lg = [&](ld k) {
        ld v = 0.0L;
        for (int i = 0; i < P; ++i) v += ev->beta[i] * log_abs_one_minus(w[i], k);
        return v;
    };
    ld g0 = lg(K[0]);
    if (!std::isfinite((double)g0) || g0 == 0.0L) return false;
    for (int i = 1; i <= P; ++i) F[i - 1] = (lg(K[i]) - g0) / fabsl(g0);
    // multipliers on the active maxima (partial-fraction residues), in log magnitude
    ld logm[SRJ_PLAN_MAXP + 1];
    int sgn[SRJ_PLAN_MAXP + 1];
    ld mx = -std::numeric_limits<ld>::infinity();
    for (int j = 0; j <= P; ++j) {
        ld lm = 0.0L;
        int sg = 1;
        ld ij = 1.0L / K[j];
        for (int i = 0; i < P; ++i) {
            ld d = w[i] - ij;
            if (d < 0) sg = -sg;
            lm += logl(fabsl(d));
        }
        for (int l = 0; l <= P; ++l) {
            if (l == j) continue;
            ld d = 1.0L / K[l] - ij;
            if (d < 0) sg = -sg;
            lm -= logl(fabsl(d));
        }
        logm[j] = lm;
        sgn[j] = sg;
        mx = std::max(mx, lm);
    }
    ld tot = 0.0L;
    for (int j = 0; j <= P; ++j) {
        ev->lam[j] = sgn[j] * expl(logm[j] - mx);
        tot += ev->lam[j];
    }
    if (tot == 0.0L) return false;
    for (int j = 0; j <= P; ++j) ev->lam[j] /= tot;
    for (int i = 0; i + 1 < P; ++i) {
        ld v = 0.0L;
        for (int j = 0; j <= P; ++j)
            v += ev->lam[j] * (log_abs_one_minus(w[i], K[j]) - log_abs_one_minus(w[P - 1], K[j]));
        F[P + i] = v;
    }
    for (int i = 0; i < 2 * P - 1; ++i)
        if (!std::isfinite((double)F[i])) return false;
    return true;
}

ld maxabs(int n, const ld* v)
{
    ld m = 0.0L;
    for (int i = 0; i < n; ++i) m = std::max(m, fabsl(v[i]));
    return m;
}

// Trust region of both solvers: no unknown moves by more than 1 per step (the unknowns are
// logits of positions inside their intervals; a longer step can swap the order of weights
// and land near another, spurious root).
inline void clamp_step(int n, ld* d)
{
    const ld m = maxabs(n, d);
    if (m > 1.0L)
        for (int i = 0; i < n; ++i) d[i] /= m;
}

// Levenberg-Marquardt on F(z) = 0 with a forward-difference Jacobian.
bool levmar(const Sys& s, ld* z, ld tol, int maxit)
{
    const int n = 2 * s.P - 1;
    ld F[2 * SRJ_PLAN_MAXP], Ft[2 * SRJ_PLAN_MAXP], zt[2 * SRJ_PLAN_MAXP];
    ld J[(2 * SRJ_PLAN_MAXP) * (2 * SRJ_PLAN_MAXP)];
    Eval ev;
    if (!residual(s, z, F, &ev)) return false;
    ld f = 0.0L;
    for (int i = 0; i < n; ++i) f += F[i] * F[i];
    ld mu = 1e-3L;
    for (int it = 0; it < maxit; ++it) {
        if (maxabs(n, F) < tol) return true;
        for (int k = 0; k < n; ++k) {
            std::memcpy(zt, z, sizeof(ld) * n);
            ld hk = 1e-9L * (1.0L + fabsl(z[k]));
            zt[k] += hk;
            if (!residual(s, zt, Ft, &ev)) {
                zt[k] = z[k] - hk;
                if (!residual(s, zt, Ft, &ev)) return false;
                hk = -hk;
            }
            for (int i = 0; i < n; ++i) J[i * n + k] = (Ft[i] - F[i]) / hk;
        }
        ld JtJ[(2 * SRJ_PLAN_MAXP) * (2 * SRJ_PLAN_MAXP)], JtF[2 * SRJ_PLAN_MAXP];
        for (int a = 0; a < n; ++a) {
            ld v = 0.0L;
            for (int i = 0; i < n; ++i) v += J[i * n + a] * F[i];
            JtF[a] = v;
            for (int b = 0; b < n; ++b) {
                ld u = 0.0L;
                for (int i = 0; i < n; ++i) u += J[i * n + a] * J[i * n + b];
                JtJ[a * n + b] = u;
            }
        }
        bool accepted = false;
        for (int tries = 0; tries < 40; ++tries) {
            ld M[(2 * SRJ_PLAN_MAXP) * (2 * SRJ_PLAN_MAXP)], d[2 * SRJ_PLAN_MAXP];
            std::memcpy(M, JtJ, sizeof(ld) * n * n);
            for (int a = 0; a < n; ++a) {
                M[a * n + a] += mu * std::max(JtJ[a * n + a], (ld)1e-30L);
                d[a] = -JtF[a];
            }
            if (linsolve(n, M, d)) {
                clamp_step(n, d);
                for (int a = 0; a < n; ++a) zt[a] = z[a] + d[a];
                if (residual(s, zt, Ft, &ev)) {
                    ld ft = 0.0L;
                    for (int i = 0; i < n; ++i) ft += Ft[i] * Ft[i];
                    if (ft < f) {
                        std::memcpy(z, zt, sizeof(ld) * n);
                        std::memcpy(F, Ft, sizeof(ld) * n);
                        f = ft;
                        mu = std::max(mu * 0.1L, (ld)1e-18L);
                        accepted = true;
                        break;
                    }
                }
            }
            mu *= 10.0L;
            if (mu > 1e25L) break;
        }
        if (!accepted) return maxabs(n, F) < tol;
    }
    return maxabs(n, F) < tol;
}

// Damped Newton (backtracking on ||F||^2) with a forward-difference Jacobian.
bool newton(const Sys& s, ld* z, ld tol, int maxit)
{
    const int n = 2 * s.P - 1;
    ld F[2 * SRJ_PLAN_MAXP], Ft[2 * SRJ_PLAN_MAXP], zt[2 * SRJ_PLAN_MAXP];
    ld J[(2 * SRJ_PLAN_MAXP) * (2 * SRJ_PLAN_MAXP)];
    Eval ev;
    if (!residual(s, z, F, &ev)) return false;
    ld f = 0.0L;
    for (int i = 0; i < n; ++i) f += F[i] * F[i];
    for (int it = 0; it < maxit; ++it) {
        if (maxabs(n, F) < tol) return true;
        for (int k = 0; k < n; ++k) {
            std::memcpy(zt, z, sizeof(ld) * n);
            ld hk = 1e-9L * (1.0L + fabsl(z[k]));
            zt[k] += hk;
            if (!residual(s, zt, Ft, &ev)) return false;
            for (int i = 0; i < n; ++i) J[i * n + k] = (Ft[i] - F[i]) / hk;
        }
        ld d[2 * SRJ_PLAN_MAXP];
        for (int i = 0; i < n; ++i) d[i] = -F[i];
        if (!linsolve(n, J, d)) return false;
        clamp_step(n, d);
        ld lam = 1.0L; bool acc = false;
        for (int ls = 0; ls < 30; ++ls) {
            for (int a = 0; a < n; ++a) zt[a] = z[a] + lam * d[a];
            if (residual(s, zt, Ft, &ev)) {
                ld ft = 0.0L; for (int i = 0; i < n; ++i) ft += Ft[i] * Ft[i];
                if (ft < (1.0L - 1e-4L * lam) * f) { std::memcpy(z, zt, sizeof(ld)*n); std::memcpy(F, Ft, sizeof(ld)*n); f = ft; acc = true; break; }
            }
            lam *= 0.5L;
        }
        if (!acc) return false;
    }
    return maxabs(n, F) < tol;
}

bool valid(const Sys& s, const ld* z, Eval* ev)
{
    ld F[2 * SRJ_PLAN_MAXP];
    if (!residual(s, z, F, ev)) return false;
    if (maxabs(2 * s.P - 1, F) > 1e-11L) return false;
    for (int i = 0; i < s.P; ++i)
        if (!(ev->beta[i] > 0.0L)) return false;
    for (int j = 0; j <= s.P; ++j)
        if (!(ev->lam[j] > 0.0L)) return false;
    for (int i = 0; i + 1 < s.P; ++i)
        if (!(ev->w[i] > ev->w[i + 1])) return false;
    return true;
}

// Position of 1/w inside [log km, log kM], in [0, 1].
void tpos(const ld* w, int P, ld km, ld kM, ld* t)
{
    for (int i = 0; i < P; ++i) t[i] = (logl(1.0L / w[i]) - logl(km)) / (logl(kM) - logl(km));
}

void from_t(const ld* t, int P, ld km, ld kM, ld* w)
{
    for (int i = 0; i < P; ++i) w[i] = 1.0L / expl(logl(km) + t[i] * (logl(kM) - logl(km)));
}

void kappa_guess(const ld* w, int P, ld* kap)
{
    for (int j = 0; j + 1 < P; ++j) {
        ld a = logl(1.0L / w[j]), b = logl(1.0L / w[j + 1]);
        kap[j] = expl(a + (b - a) / 3.0L);
    }
}

bool solve_from_weights(Sys& s, const ld* wguess, ld* z, Eval* ev)
{
    ld kap[SRJ_PLAN_MAXP];
    kappa_guess(wguess, s.P, kap);
    pack(s, wguess, kap, z);
    // the solvers aim at 1e-14; at extreme intervals the evaluation's own rounding can sit
    // just above that, so acceptance is decided by valid() (residual below 1e-11, positive
    // fractions and multipliers, descending weights) at whatever point they reached
    if (!newton(s, z, 1e-14L, 200)) levmar(s, z, 1e-14L, 300);
    return valid(s, z, ev);
}

}  // namespace

// Carry a solved P-level system from s.km to target by continuation in log km (the unknowns
// are positions relative to the interval, so the previous solution is the starting point at
// the next km); steps are halved on failure, and more than 40 consecutive halvings give up.
static bool continue_to(Sys& s, ld* z, Eval* ev, ld target)
{
    const int P = s.P;
    ld cur = logl(s.km), tgt = logl(target);
    int nst = std::max(1, (int)ceill(fabsl(tgt - cur) / 0.25L));
    ld step = (tgt - cur) / nst;
    int fails = 0;
    ld zs[2 * SRJ_PLAN_MAXP];
    while (fabsl(tgt - cur) > 1e-15L) {
        ld nxt = cur + step;
        if ((step > 0 && nxt > tgt) || (step < 0 && nxt < tgt)) nxt = tgt;
        Sys s2 = s;
        s2.km = expl(nxt);
        if (nxt == tgt) s2.km = target;
        s2.a = logl(s2.km);
        std::memcpy(zs, z, sizeof(ld) * (2 * P - 1));
        Eval ev2;
        if (!newton(s2, zs, 1e-14L, 60)) levmar(s2, zs, 1e-14L, 100);
        if (!valid(s2, zs, &ev2)) {
            step *= 0.5L;
            if (++fails > 40) return false;
            continue;
        }
        fails = 0;
        std::memcpy(z, zs, sizeof(ld) * (2 * P - 1));
        *ev = ev2;
        s = s2;
        cur = nxt;
    }
    return true;
}

bool optimal_schedule(int P, double km_d, double kM_d, Optimum* out, std::string* err)
{
    if (P < 1 || P > SRJ_PLAN_MAXP) {
        if (err) *err = "levels must be in [1, " + std::to_string(SRJ_PLAN_MAXP) + "]";
        return false;
    }
    if (!(km_d > 0.0) || !(kM_d > km_d)) {
        if (err) *err = "need 0 < kappa_min < kappa_max";
        return false;
    }
    const ld km = km_d, kM = kM_d;
    if (P == 1) {
        out->w = {(double)(2.0L / (km + kM))};
        out->beta = {1.0};
        out->kappa.clear();
        return true;
    }
    const ld pi = 3.14159265358979323846264338327950288L;
    // grow levels at a moderate resolution (N = 100 of Eq. boundaries), or at N = 2000 when
    // more than 12 are wanted (few levels fit a coarse interval: Sec. 4.2 reports the same
    // limit); the 2-level solution is carried there by continuation
    const ld kb = powl(sinl(pi / 200.0L), 2);
    const ld kseed = P > 12 ? powl(sinl(pi / 4000.0L), 2) : kb;
    Sys s;
    s.kM = kM;
    s.c = logl(kM);
    s.km = kb;
    s.a = logl(kb);
    s.P = 2;
    ld z[2 * SRJ_PLAN_MAXP];
    Eval ev;
    ld w0[SRJ_PLAN_MAXP] = {0.0795L / kb, 0.968L};
    if (!solve_from_weights(s, w0, z, &ev)) {
        if (err) *err = "optimiser failed for 2 levels at the seed resolution";
        return false;
    }
    if (kseed != kb && !continue_to(s, z, &ev, kseed)) {
        if (err) *err = "continuation to the seed resolution failed";
        return false;
    }
    // log w_1 and log(w_P - 1/2) of the levels solved so far, for the extrapolated guess
    std::vector<ld> hist_first{logl(ev.w[0])}, hist_last{logl(ev.w[1] - 0.5L)};
    auto extrapolate = [](const std::vector<ld>& v) {
        const size_t m = v.size();
        if (m == 1) return v[0];
        if (m == 2) return 2.0L * v[1] - v[0];
        return v[m - 3] - 3.0L * v[m - 2] + 3.0L * v[m - 1];  // parabola through the last three
    };
    for (int p = 3; p <= P; ++p) {
        ld t[SRJ_PLAN_MAXP], t2[SRJ_PLAN_MAXP], wg[SRJ_PLAN_MAXP];
        tpos(ev.w, p - 1, s.km, kM, t);
        // first guess: the (p-1)-level shape resampled at p points, both ends pulled outwards
        for (int i = 0; i < p; ++i) {
            ld x = (ld)i / (ld)(p - 1) * (ld)(p - 2);
            int i0 = std::min((int)floorl(x), p - 3);
            ld fr = x - i0;
            t2[i] = t[i0] * (1.0L - fr) + t[i0 + 1] * fr;
        }
        ld f = powl((ld)(p - 1) / (ld)p, 2);
        t2[0] = t[0] * f;
        t2[p - 1] = 1.0L - (1.0L - t[p - 2]) * f;
        from_t(t2, p, s.km, kM, wg);
        Sys sp = s;
        sp.P = p;
        ld zp[2 * SRJ_PLAN_MAXP];
        Eval evp;
        bool ok = solve_from_weights(sp, wg, zp, &evp);
        if (!ok) {
            // second guess (Sec. 3.3): both end weights extrapolated in P from the levels
            // solved so far, inverse weights spread logarithmically between them
            const ld w1 = std::min(expl(extrapolate(hist_first)), 0.999L / s.km);
            const ld wP = 0.5L + expl(extrapolate(hist_last));
            for (int i = 0; i < p; ++i) wg[i] = expl(logl(w1) + (ld)i / (ld)(p - 1) * (logl(wP) - logl(w1)));
            ok = solve_from_weights(sp, wg, zp, &evp);
        }
        if (!ok) {
            if (err) *err = "optimiser failed while adding level " + std::to_string(p);
            return false;
        }
        s = sp;
        std::memcpy(z, zp, sizeof(z));
        ev = evp;
        hist_first.push_back(logl(ev.w[0]));
        hist_last.push_back(logl(ev.w[p - 1] - 0.5L));
    }
    if (!continue_to(s, z, &ev, km)) {
        if (err) *err = "continuation to the target kappa_min failed";
        return false;
    }
    out->w.assign(P, 0.0);
    out->beta.assign(P, 0.0);
    out->kappa.assign(P - 1, 0.0);
    for (int i = 0; i < P; ++i) {
        out->w[i] = (double)ev.w[i];
        out->beta[i] = (double)ev.beta[i];
    }
    for (int j = 0; j + 1 < P; ++j) out->kappa[j] = (double)ev.kap[j];
    return true;
}

std::vector<int64_t> floor_counts(const std::vector<double>& beta)
{
    std::vector<int64_t> q(beta.size());
    for (size_t i = 0; i < beta.size(); ++i) q[i] = (int64_t)std::floor(beta[i] / beta[0]);
    return q;
}

static std::vector<double> log_grid(double km, double kM, int G);

std::vector<int64_t> round_counts(const std::vector<double>& beta, int mode, const double* w, double km,
                                  double kM)
{
    const int P = (int)beta.size();
    std::vector<int64_t> fl(P), ce(P);
    for (int i = 0; i < P; ++i) {
        const double r = beta[i] / beta[0];
        fl[i] = (int64_t)std::floor(r);
        ce[i] = (int64_t)std::ceil(r);
    }
    fl[0] = ce[0] = 1;
    if (mode == 0) return fl;
    if (mode == 2) return ce;
    if (mode == 1) {
        std::vector<int64_t> q(P);
        for (int i = 0; i < P; ++i) q[i] = (int64_t)std::floor(beta[i] / beta[0] + 0.5);
        q[0] = 1;
        return q;
    }
    if (mode != 3 || P > 12 || !w || !(km > 0) || !(kM > km)) return {};
    // levels whose ratio is an integer have one choice; the others two
    std::vector<int> free_lv;
    for (int i = 1; i < P; ++i)
        if (ce[i] != fl[i]) free_lv.push_back(i);
    const int G = 4096;
    std::vector<double> grid = log_grid(km, kM, G);
    std::vector<double> L((size_t)P * G);
    for (int i = 0; i < P; ++i)
        for (int g = 0; g < G; ++g) L[(size_t)i * G + g] = std::log(std::fabs(1.0 - w[i] * grid[g]));
    std::vector<int64_t> best = fl, q(P);
    double best_rate = std::numeric_limits<double>::infinity();
    int best_ceils = P + 1;
    const uint32_t ncomb = 1u << free_lv.size();
    for (uint32_t mask = 0; mask < ncomb; ++mask) {
        q = fl;
        int ceils = 0;
        for (size_t b = 0; b < free_lv.size(); ++b)
            if (mask & (1u << b)) {
                q[free_lv[b]] = ce[free_lv[b]];
                ++ceils;
            }
        int64_t M = 0;
        for (int i = 0; i < P; ++i) M += q[i];
        double mx = -std::numeric_limits<double>::infinity();
        for (int g = 0; g < G; ++g) {
            double v = 0.0;
            for (int i = 0; i < P; ++i) v += (double)q[i] * L[(size_t)i * G + g];
            mx = std::max(mx, v);
        }
        const double rate = mx / (double)M;  // log of the per-step factor
        if (rate < best_rate || (rate == best_rate && ceils < best_ceils)) {
            best_rate = rate;
            best_ceils = ceils;
            best = q;
        }
    }
    return best;
}

// ------------------------------------------------------------------- ordering

static std::vector<double> log_grid(double km, double kM, int G)
{
    std::vector<double> g(G);
    double a = std::log(km), c = std::log(kM);
    for (int i = 0; i < G; ++i) g[i] = std::exp(a + (double)i * (c - a) / (double)(G - 1));
    g[0] = km;
    g[G - 1] = kM;
    return g;
}

std::vector<int32_t> order_steps(int P, const double* w, const int64_t* q, double km, double kM,
                                 int ordering)
{
    int64_t M = 0;
    for (int i = 0; i < P; ++i) M += q[i];
    std::vector<int32_t> seq;
    seq.reserve((size_t)M);
    if (ordering == 1) {
        // r-th use of weight i at (2r+1) / (2 q_i); exact rational comparison, ties to lower i
        struct Item { int64_t num, den; int32_t i; };
        std::vector<Item> it;
        it.reserve((size_t)M);
        for (int i = 0; i < P; ++i)
            for (int64_t r = 0; r < q[i]; ++r) it.push_back({2 * r + 1, 2 * q[i], i});
        std::sort(it.begin(), it.end(), [](const Item& x, const Item& y) {
            __int128 l = (__int128)x.num * y.den, r = (__int128)y.num * x.den;
            if (l != r) return l < r;
            return x.i < y.i;
        });
        for (auto& x : it) seq.push_back(x.i);
        return seq;
    }
    const int G = 4096;
    std::vector<double> grid = log_grid(km, kM, G);
    std::vector<double> L((size_t)P * G), T(G, 0.0), s(G, 0.0), target(G);
    for (int i = 0; i < P; ++i)
        for (int g = 0; g < G; ++g) L[(size_t)i * G + g] = std::log(std::fabs(1.0 - w[i] * grid[g]));
    for (int i = 0; i < P; ++i)
        for (int g = 0; g < G; ++g) T[g] = T[g] + (double)q[i] * L[(size_t)i * G + g];
    std::vector<int64_t> rem(q, q + P);
    for (int64_t k = 1; k <= M; ++k) {
        for (int g = 0; g < G; ++g) target[g] = ((double)k * T[g]) / (double)M;
        double best = 0.0;
        int besti = -1;
        for (int i = 0; i < P; ++i) {
            if (rem[i] == 0) continue;
            const double* Li = &L[(size_t)i * G];
            double e = 0.0;
            for (int g = 0; g < G; ++g) {
                double v = std::fabs((s[g] + Li[g]) - target[g]);
                if (v > e) e = v;
            }
            if (besti < 0 || e < best) {
                best = e;
                besti = i;
            }
        }
        const double* Lb = &L[(size_t)besti * G];
        for (int g = 0; g < G; ++g) s[g] = s[g] + Lb[g];
        rem[besti] -= 1;
        seq.push_back(besti);
    }
    return seq;
}

double gamma_q_max(int P, const double* w, const int64_t* q, double km, double kM)
{
    const int G = 16384;
    std::vector<double> grid = log_grid(km, kM, G);
    int64_t M = 0;
    for (int i = 0; i < P; ++i) M += q[i];
    double mx = -std::numeric_limits<double>::infinity();
    for (int g = 0; g < G; ++g) {
        double v = 0.0;
        for (int i = 0; i < P; ++i) v += (double)q[i] * std::log(std::fabs(1.0 - w[i] * grid[g]));
        mx = std::max(mx, v);
    }
    return std::exp(mx / (double)M);
}

void partial_peaks(int P, const double* w, const std::vector<int32_t>& seq, double km, double kM,
                   double* prefix_log10, double* suffix_log10)
{
    const int G = 4096;
    std::vector<double> grid = log_grid(km, kM, G);
    std::vector<double> L((size_t)P * G), T(G, 0.0), s(G, 0.0);
    for (int i = 0; i < P; ++i)
        for (int g = 0; g < G; ++g) L[(size_t)i * G + g] = std::log(std::fabs(1.0 - w[i] * grid[g]));
    for (int32_t i : seq)
        for (int g = 0; g < G; ++g) T[g] += L[(size_t)i * G + g];
    double pre = 0.0, suf = 0.0;
    for (int32_t i : seq) {
        for (int g = 0; g < G; ++g) {
            s[g] += L[(size_t)i * G + g];
            pre = std::max(pre, s[g]);
            suf = std::max(suf, T[g] - s[g]);
        }
    }
    *prefix_log10 = pre / std::log(10.0);
    *suffix_log10 = suf / std::log(10.0);
}

}  // namespace srj
