"""Optimal SRJ schedules from the paper's Sec. 3-4 -- oracle side (test infrastructure).

Notation follows the paper: weights w_1 > ... > w_P (Sec. 2), fractions beta_i with
sum 1, counts q_i, cycle length M = sum q_i, spectral interval [kappa_m, kappa_M]
(Eq. boundaries, kappa_M = 2), per-iteration amplification
Gamma(kappa) = prod |1 - w_i kappa|^beta_i (Eq. Gamma).

The optimum is the solution of the reduced system S(w, kappa) of Sec. 3.5:
  unknowns   w_1..w_P and the interior maxima kappa_1..kappa_{P-1};
  beta       from Theorem 2 (Eq. betai), which makes every kappa_i a stationary point
             of log Gamma (Eq. partialG) and gives sum beta = 1;
  equations  Gamma(kappa_0) = Gamma(kappa_i), i = 1..P with kappa_0 = kappa_m and
             kappa_P = kappa_M (Eq. equMax), and
             d log Gamma(kappa_0) / d beta_j = 0, j = 1..P-1 (Eq. partialbeta), whose
             dw/dbeta comes from Theorem 1 (Eq. ancVar) through the closed-form inverse
             of Lemma 1.
Starting values follow Sec. 3.3 and Sec. 3.5: inverse weights spread logarithmically
between 1/w_1 and 1/w_P (the ends extrapolated in P with a parabola through the last
solved levels), kappa_i one third of the way from 1/w_i to 1/w_{i+1} (taken in
log kappa, see the readings list), and continuation in kappa_m from solved neighbours.
The rows of Table 1 at N = 500 seed the levels P = 2..5.

The integer counts are q_i = floor(beta_i / beta_1) (Sec. 4.3).  The order of the M
steps inside a cycle is not fixed by the paper beyond "spread the large weights evenly"
(Sec. 5.1); two orders are provided (even spread, and a balanced greedy order).
"""
import math

import numpy as np
from scipy.optimize import root

KAPPA_M = 2.0  # Eq. boundaries: the upper end of the spectral interval

# Table 1 rows at N = 500 (P = 2..5), the paper's printed weights, used only as
# starting points of the solve.
TABLE1_N500 = {
    2: [1923.36, 0.992522],
    3: [17673.1, 107.432, 0.927487],
    4: [41329.0, 1177.71, 25.2645, 0.831242],
    5: [56698.8, 3776.87, 183.430, 9.01057, 0.737910],
}
SEED_N = 500.0


# ------------------------------------------------------------- spectral interval

def kappa_min_neumann(N, d=2):
    """kappa_m^(d) = (2/d) sin^2(pi / (2N))  (Eq. boundaries1D3D)."""
    return (2.0 / d) * math.sin(math.pi / (2.0 * N)) ** 2


def kappa_min_dirichlet(n_interior, h=None):
    """(2/d) sum_i sin^2(pi / (2 N_i)) with N_i = n_i + 1 zones (Eq. effectiveNDirichlet).

    With one spacing per axis, h = (h_x, h_y[, h_z]) in the order of n_interior, the
    equation multiplied through by h_x^2 has axis weights a = (1, h_x^2/h_y^2, h_x^2/h_z^2)
    and diagonal dg = 2 sum a_i; the smallest symbol is then 4 sum_i a_i sin^2(..) / dg."""
    d = len(n_interior)
    if h is None:
        return (2.0 / d) * sum(math.sin(math.pi / (2.0 * (n + 1))) ** 2 for n in n_interior)
    from .sweeps import axis_weights

    wy, wz, dg = axis_weights(h, d)
    a = (1.0, float(wy), float(wz))
    s = 0.0
    for i, n in enumerate(n_interior):
        s = s + a[i] * (math.sin(math.pi / (2.0 * (n + 1))) ** 2)
    return (4.0 * s) / float(dg)


def n_eff(zones):
    """N_eff^(2) of Eq. effectiveNDirichlet from the zone counts N_i."""
    d = len(zones)
    s = math.sqrt((2.0 / d) * sum(math.sin(math.pi / (2.0 * N)) ** 2 for N in zones))
    return math.pi / (2.0 * math.asin(s))


# ------------------------------------------------------------ Gamma and theorems

def log_gamma(w, beta, kappa):
    """log Gamma(kappa) = sum beta_i log|1 - w_i kappa|  (Eq. Gamma)."""
    w = np.asarray(w, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    return float(np.sum(beta * np.log(np.abs(1.0 - w * kappa))))


def beta_theorem2(w, kap):
    """beta_i = prod_{k=1}^{P-1} prod_{l != i} (1 - kappa_k w_i) w_l / (w_l - w_i)  (Eq. betai)."""
    P = len(w)
    beta = np.empty(P)
    for i in range(P):
        v = 1.0
        for kk in kap:
            v *= 1.0 - kk * w[i]
        for l in range(P):
            if l != i:
                v *= w[l] / (w[l] - w[i])
        beta[i] = v
    return beta


def lemma1_A(w, beta, k1P):
    """a_ij = kappa_i beta_j / (1 - kappa_i w_j), rows kappa_1..kappa_P (kappa_P = kappa_M)."""
    P = len(w)
    return np.array([[k1P[i] * beta[j] / (1.0 - k1P[i] * w[j]) for j in range(P)] for i in range(P)])


def lemma1_A_inverse(w, beta, k1P):
    """Closed-form inverse of Lemma 1 (Eq. lemmaM); rows index w, columns index kappa."""
    P = len(w)
    At = np.empty((P, P))
    for i in range(P):
        for j in range(P):
            v = (1.0 - k1P[j] * w[i]) / (beta[i] * k1P[j])
            for k in range(P):
                if k != j:
                    v *= (1.0 - k1P[k] * w[i]) / (k1P[k] - k1P[j])
            for l in range(P):
                if l != i:
                    v *= (1.0 - k1P[j] * w[l]) / (w[l] - w[i])
            At[i, j] = v
    return At


def dw_dbeta_theorem1(w, beta, k1P):
    """D[i, q] = d w_i / d beta_q, q = 1..P-1 (Eq. ancVar): A^-1 applied to
    f_j = log|(1 - kappa_j w_q) / (1 - kappa_j w_P)|."""
    P = len(w)
    At = lemma1_A_inverse(w, beta, k1P)
    D = np.empty((P, P - 1))
    for q in range(P - 1):
        f = np.log(np.abs((1.0 - k1P * w[q]) / (1.0 - k1P * w[P - 1])))
        D[:, q] = At @ f
    return D


# ------------------------------------------------------------------ the system

def _unpack(z, P, km, kM):
    # w_i = 1 / kappa at fraction t_i of [log km, log kM]; kappa_i at fraction th_i of
    # [log 1/w_i, log 1/w_{i+1}] -- a change of variables that keeps every unknown in
    # its interval (Sec. 3.5: kappa_i lies between 1/w_i and 1/w_{i+1}).
    a, c = math.log(km), math.log(kM)
    t = 1.0 / (1.0 + np.exp(-z[:P]))
    lw = -(a + t * (c - a))
    th = 1.0 / (1.0 + np.exp(-z[P:]))
    kap = np.exp(-lw[:-1] + th * (lw[:-1] - lw[1:]))
    return np.exp(lw), kap


def _pack(w, kap, km, kM):
    a, c = math.log(km), math.log(kM)
    lw = np.log(w)
    t = (-lw - a) / (c - a)
    th = (np.log(kap) + lw[:-1]) / (lw[:-1] - lw[1:])
    return np.concatenate([np.log(t / (1.0 - t)), np.log(th / (1.0 - th))])


def system(w, kap, km, kM=KAPPA_M):
    """Residuals of Eq. equMax (P) and Eq. partialbeta (P-1), both divided by |log Gamma(km)|."""
    P = len(w)
    beta = beta_theorem2(w, kap)
    k1P = np.concatenate([kap, [kM]])
    g0 = log_gamma(w, beta, km)
    e1 = np.array([log_gamma(w, beta, k) - g0 for k in k1P])
    D = dw_dbeta_theorem1(w, beta, k1P)
    e2 = np.empty(P - 1)
    for q in range(P - 1):
        e2[q] = (math.log(abs(1.0 - w[q] * km)) - math.log(abs(1.0 - w[P - 1] * km))
                 - float(np.sum(beta * km / (1.0 - w * km) * D[:, q])))
    return np.concatenate([e1, e2]) / abs(g0)


def _kappa_guess(w):
    lw = np.log(1.0 / w)
    return np.exp(lw[:-1] + (lw[1:] - lw[:-1]) / 3.0)


def solve_system(P, km, w_guess, kM=KAPPA_M):
    """Solve S(w, kappa) = 0 from a weight guess; returns (ok, w, beta, kappa, |residual|)."""
    w_guess = np.asarray(w_guess, dtype=np.float64)
    z0 = _pack(w_guess, _kappa_guess(w_guess), km, kM)

    def F(z):
        w, kap = _unpack(z, P, km, kM)
        return system(w, kap, km, kM)

    with np.errstate(all="ignore"):
        sol = root(F, z0, method="hybr", options=dict(xtol=1e-14, maxfev=200000))
        w, kap = _unpack(sol.x, P, km, kM)
        beta = beta_theorem2(w, kap)
        res = float(np.max(np.abs(sol.fun)))
    ok = (np.isfinite(res) and res < 1e-8 and bool(np.all(beta > 0))
          and bool(np.all(np.diff(w) < 0)))
    return ok, w, beta, kap, res


def _extrapolate(vals):
    """Next value of a sequence in P: parabola through the last (up to) 4 (Sec. 3.3)."""
    x = np.arange(len(vals), dtype=np.float64)
    m = min(len(vals), 4)
    deg = min(2, m - 1)
    c = np.polyfit(x[-m:], np.asarray(vals[-m:]), deg)
    return float(np.polyval(c, len(vals)))


def optimal(P, km, kM=KAPPA_M):
    """Optimal (w, beta, kappa_1..kappa_{P-1}) for P levels on [km, kM].

    Levels are added one at a time at the seed resolution N = 500 and the solution is
    then carried to km by continuation in log km.  Raises RuntimeError if a step fails.
    """
    if P < 1:
        raise ValueError("P >= 1")
    if P == 1:
        # one weight: the minimax of |1 - w kappa| on [km, kM] is w = 2 / (km + kM)
        return dict(w=np.array([2.0 / (km + kM)]), beta=np.array([1.0]), kappa=np.zeros(0))
    kb = kappa_min_neumann(SEED_N)
    sols = []
    for p in range(2, P + 1):
        if p in TABLE1_N500:
            w0 = np.array(TABLE1_N500[p])
        else:
            l1 = _extrapolate([math.log(s[0]) for s in sols])
            lP = _extrapolate([math.log(s[-1] - 0.5) for s in sols])
            w1 = min(math.exp(l1), 0.999 / kb)
            wP = 0.5 + math.exp(lP)
            w0 = np.exp(np.linspace(math.log(w1), math.log(wP), p))
        ok, w, beta, kap, res = solve_system(p, kb, w0, kM)
        if not ok:
            raise RuntimeError(f"level growth failed at P={p} (residual {res:.3g})")
        sols.append(w)
    cur, tgt = math.log(kb), math.log(km)
    nst = max(1, math.ceil(abs(tgt - cur) / 0.25))
    step = (tgt - cur) / nst
    fails = 0
    while abs(tgt - cur) > 1e-15:
        nxt = cur + step
        if (step > 0 and nxt > tgt) or (step < 0 and nxt < tgt):
            nxt = tgt
        frac = (np.log(1.0 / w) - cur) / (math.log(kM) - cur)
        wg = 1.0 / np.exp(nxt + frac * (math.log(kM) - nxt))
        ok, w2, b2, k2, res = solve_system(P, math.exp(nxt), wg, kM)
        if not ok:
            step /= 2.0
            fails += 1
            if fails > 40:
                raise RuntimeError("continuation in kappa_m failed")
            continue
        w, beta, kap, cur = w2, b2, k2, nxt
    return dict(w=w, beta=beta, kappa=kap)


def rho(w, beta):
    """Convergence performance index rho = sum w_i beta_i  (Eq. rho)."""
    return float(np.sum(np.asarray(w) * np.asarray(beta)))


def q_floor(beta):
    """q_i = floor(beta_i / beta_1)  (Sec. 4.3)."""
    beta = np.asarray(beta, dtype=np.float64)
    return np.floor(beta / beta[0]).astype(np.int64)


def q_counts(beta, mode, w=None, km=None, kM=KAPPA_M, G=4096):
    """Integer counts from the fractions (Sec. 4.3; the paper tries floor, rounding to the
    nearest integer, ceiling and per-level mixtures of them).  q_1 = 1 always.
      mode 0: floor(beta_i / beta_1);  1: nearest integer (floor(x + 1/2));  2: ceiling;
      3: every combination of floor and ceiling per level (levels whose ratio is an integer
         have one choice), keeping the one with the smallest per-step factor
         max over the log-spaced grid of [km, kM] of sum_i q_i log|1 - w_i k| / M; exact
         ties to fewer ceilings, then to the earlier combination in binary order (level 2
         the lowest bit).  An exhaustive search, for P <= 12."""
    beta = np.asarray(beta, dtype=np.float64)
    r = beta / beta[0]
    fl = np.floor(r).astype(np.int64)
    ce = np.ceil(r).astype(np.int64)
    fl[0] = ce[0] = 1
    if mode == 0:
        return fl
    if mode == 2:
        return ce
    if mode == 1:
        q = np.floor(r + 0.5).astype(np.int64)
        q[0] = 1
        return q
    if mode != 3:
        raise ValueError("mode must be 0..3")
    free = [i for i in range(1, len(r)) if ce[i] != fl[i]]
    grid = balanced_grid(km, kM, G)
    L = [[math.log(abs(1.0 - float(w[i]) * k)) for k in grid] for i in range(len(r))]
    best, best_rate, best_ceils = fl, None, None
    for mask in range(1 << len(free)):
        q = fl.copy()
        for b, lv in enumerate(free):
            if mask & (1 << b):
                q[lv] = ce[lv]
        ceils = bin(mask).count("1")
        M = int(np.sum(q))
        mx = max(sum(float(q[i]) * L[i][g] for i in range(len(r))) for g in range(len(grid)))
        rate = mx / M
        if best_rate is None or rate < best_rate or (rate == best_rate and ceils < best_ceils):
            best, best_rate, best_ceils = q, rate, ceils
    return best


def gamma_q_max(w, q, kappa_grid):
    """max over kappa of |prod (1 - w_i kappa)^q_i|^(1/M): the integer scheme's Gamma
    (Sec. 4.3 requires it below 1)."""
    M = int(np.sum(q))
    lg = np.zeros_like(np.asarray(kappa_grid, dtype=np.float64))
    for wi, qi in zip(w, q):
        lg = lg + int(qi) * np.log(np.abs(1.0 - wi * np.asarray(kappa_grid)))
    return float(np.exp(np.max(lg) / M))


# -------------------------------------------------------------------- orderings

def order_even(q):
    """Even spread (Sec. 5.1): the r-th use of weight i sits at (r + 1/2) / q_i of the
    cycle; positions sorted, ties to the larger weight.  Exact rational comparisons."""
    items = []
    for i, qi in enumerate(q):
        for r in range(int(qi)):
            items.append((2 * r + 1, 2 * int(qi), i))
    import functools

    def cmp(a, b):
        lhs = a[0] * b[1]
        rhs = b[0] * a[1]
        if lhs != rhs:
            return -1 if lhs < rhs else 1
        return -1 if a[2] < b[2] else (1 if a[2] > b[2] else 0)

    items.sort(key=functools.cmp_to_key(cmp))
    return np.array([it[2] for it in items], dtype=np.int32)


def balanced_grid(km, kM=KAPPA_M, G=4096):
    """G points evenly spaced in log kappa over [km, kM], ends set exactly."""
    a, c = math.log(km), math.log(kM)
    grid = [math.exp(a + g * (c - a) / (G - 1)) for g in range(G)]
    grid[0] = km
    grid[-1] = kM
    return grid


def order_balanced(w, q, km, kM=KAPPA_M, G=4096):
    """Balanced greedy order of the M steps.

    With L_i(kappa) = log|1 - w_i kappa| on the grid and T = sum_i q_i L_i, step k picks,
    among weights with uses left, the one minimising max_kappa |(s + L_i) - k T / M|,
    where s is the sum of the L of the steps already taken (ties to the larger weight).
    The partial products of the cycle then stay close to the straight path from 1 to the
    full cycle factor in every mode.  The ordering is an engineering choice the paper leaves
    open; pinned by a three-level example worked by hand on a two-point grid, and by being a
    permutation with the right counts whose full cycle factor does not depend on the order.
    """
    grid = balanced_grid(km, kM, G)
    P = len(w)
    L = np.array([[math.log(abs(1.0 - float(w[i]) * k)) for k in grid] for i in range(P)])
    T = np.zeros(G)
    for i in range(P):
        T = T + float(q[i]) * L[i]
    M = int(np.sum(q))
    rem = np.array(q, dtype=np.int64).copy()
    s = np.zeros(G)
    seq = np.empty(M, dtype=np.int32)
    for k in range(1, M + 1):
        target = (float(k) * T) / float(M)
        best, besti = None, -1
        for i in range(P):
            if rem[i] == 0:
                continue
            e = float(np.max(np.abs((s + L[i]) - target)))
            if best is None or e < best:
                best, besti = e, i
        s = s + L[besti]
        rem[besti] -= 1
        seq[k - 1] = besti
    return seq


def partial_peaks(w, seq, km, kM=KAPPA_M, G=4096):
    """log10 of the largest prefix and suffix partial products over the grid."""
    grid = np.array(balanced_grid(km, kM, G))
    L = np.log(np.abs(1.0 - np.asarray(w)[:, None] * grid[None, :]))
    s = np.zeros_like(grid)
    T = np.sum(L[np.asarray(seq)], axis=0)
    pre, suf = 0.0, 0.0
    for i in seq:
        s = s + L[i]
        pre = max(pre, float(np.max(s)))
        suf = max(suf, float(np.max(T - s)))
    return pre / math.log(10.0), suf / math.log(10.0)


def weight_sequence(w, seq):
    return np.asarray(w, dtype=np.float64)[np.asarray(seq)]
