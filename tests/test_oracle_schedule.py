"""Pins of the oracle's schedule optimiser (Sec. 3-4) against the paper's printed tables,
the worked example of Sec. 5.1, the lemma/theorem identities and brute-force checks."""
import math
import os

import numpy as np
import pytest

from oracle import schedule as S

# Printed Table 1 rows that are measurably off the optimum of the stated problem: our
# solution has a strictly lower max Gamma for each of them (checked below), and the
# P = 4, N = 450 row does not even have equal maxima.  Listed in the design notes.
OFF_OPTIMUM_ROWS = {(4, 150), (4, 250), (4, 400), (4, 450), (4, 500)}
# Rows whose printed point lies close to the optimum but further from it than 6-digit
# rounding explains (about 3e-6 relative for the other rows): the oracle's point solves the
# optimality system in 30-digit arithmetic and the printed one does not (see
# test_near_rows_optimality_in_extended_precision); compared at the stated tolerance.
NEAR_OPTIMUM_ROWS = {(4, 100): 1e-3, (5, 100): 1.5e-4}


def read_table1(golden_dir):
    rows = []
    for line in open(os.path.join(golden_dir, "table1.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        a = line.split("|")
        P, N = map(int, a[0].split())
        rows.append((P, N, np.array(list(map(float, a[1].split()))),
                     np.array(list(map(float, a[2].split()))), float(a[3])))
    return rows


def read_worked(golden_dir):
    d = {}
    for line in open(os.path.join(golden_dir, "worked_example.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            d[k] = v
    return d


def max_log_gamma(w, beta, km, npts=200001):
    g = np.exp(np.linspace(math.log(km), math.log(S.KAPPA_M), npts))
    beta = np.asarray(beta) / np.sum(beta)
    return float(np.max(np.sum(beta[:, None] * np.log(np.abs(1 - np.asarray(w)[:, None] * g[None, :])),
                               axis=0)))


def test_table1_rows(golden_dir):
    for P, N, w, beta, rho in read_table1(golden_dir):
        km = S.kappa_min_neumann(N)
        o = S.optimal(P, km)
        ours = max_log_gamma(o["w"], o["beta"], km)
        printed = max_log_gamma(w, beta, km)
        assert ours <= printed + 1e-12, (P, N)
        if (P, N) in OFF_OPTIMUM_ROWS:
            continue
        tol = NEAR_OPTIMUM_ROWS.get((P, N), 3e-5)
        np.testing.assert_allclose(o["w"], w, rtol=tol, err_msg=f"P={P} N={N}")
        np.testing.assert_allclose(o["beta"], beta, rtol=tol, err_msg=f"P={P} N={N}")
        assert abs(S.rho(o["w"], o["beta"]) - rho) <= 0.0051, (P, N)


def test_worked_example_P10_N550(golden_dir):
    d = read_worked(golden_dir)
    P, N = int(d["P"][0]), float(d["N"][0])
    o = S.optimal(P, S.kappa_min_neumann(N))
    q = S.q_floor(o["beta"])
    assert list(q) == [int(x) for x in d["q"]]
    assert int(np.sum(q)) == int(d["M"][0])
    head = [float(x) for x in d["omega_head"]]
    for mine, printed in zip(o["w"][:3], head):
        assert float(f"{mine:.6g}") == printed
    assert round(S.rho(o["w"], o["beta"]), 2) == float(d["rho"][0])


def test_effective_resolution_example(golden_dir):
    d = read_worked(golden_dir)
    zones = [int(x) for x in d["neff_zones"]]
    assert round(S.n_eff(zones), 2) == float(d["neff"][0])


def _random_interlaced(P, rng):
    iw = np.sort(np.exp(rng.uniform(math.log(1e-4), math.log(1.9), P)))
    w = 1.0 / iw
    kap = np.exp(np.log(iw[:-1]) + rng.uniform(0.1, 0.9, P - 1) * (np.log(iw[1:]) - np.log(iw[:-1])))
    return w, kap


@pytest.mark.parametrize("P", [2, 3, 5, 8])
def test_theorem2_identities(P):
    rng = np.random.default_rng(P)
    for _ in range(5):
        w, kap = _random_interlaced(P, rng)
        beta = S.beta_theorem2(w, kap)
        assert math.isclose(float(np.sum(beta)), 1.0, rel_tol=1e-11)
        for k in kap:  # Eq. partialG at every interior kappa
            terms = beta * w / (1 - k * w)
            assert abs(np.sum(terms)) <= 1e-10 * np.sum(np.abs(terms))


@pytest.mark.parametrize("P", [2, 4, 7])
def test_lemma1_inverse_and_theorem1(P):
    rng = np.random.default_rng(10 + P)
    w, kap = _random_interlaced(P, rng)
    beta = S.beta_theorem2(w, kap)
    k1P = np.concatenate([kap, [S.KAPPA_M]])
    A = S.lemma1_A(w, beta, k1P)
    At = S.lemma1_A_inverse(w, beta, k1P)
    np.testing.assert_allclose(At @ A, np.eye(P), atol=1e-9)
    D = S.dw_dbeta_theorem1(w, beta, k1P)
    for q in range(P - 1):
        f = np.log(np.abs((1 - k1P * w[q]) / (1 - k1P * w[P - 1])))
        np.testing.assert_allclose(D[:, q], np.linalg.solve(A, f), rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("P,N", [(3, 200), (6, 256), (8, 362.75), (10, 2897.0)])
def test_equal_maxima_and_local_optimality_brute_force(P, N):
    km = S.kappa_min_neumann(N)
    o = S.optimal(P, km)
    w, beta = o["w"], o["beta"]
    lg0 = S.log_gamma(w, beta, km)
    # equal maxima: the dense grid never exceeds Gamma(km), and every solver maximum equals it
    assert max_log_gamma(w, beta, km, 400001) <= lg0 * (1 - 1e-9)
    for k in list(o["kappa"]) + [S.KAPPA_M]:
        assert math.isclose(S.log_gamma(w, beta, k), lg0, rel_tol=1e-8)
    # no random small move of (w, beta) lowers the maximum to first order
    rng = np.random.default_rng(1)
    grid = np.exp(np.linspace(math.log(km), math.log(2.0), 100001))
    grid = np.unique(np.concatenate([grid, o["kappa"], [km, 2.0]]))
    base = np.max(np.sum(beta[:, None] * np.log(np.abs(1 - w[:, None] * grid[None, :])), axis=0))
    eps = 1e-6
    for _ in range(30):
        dw = rng.standard_normal(P)
        db = rng.standard_normal(P)
        db -= db.mean()
        w2 = w * np.exp(eps * dw)
        b2 = beta + eps * db * beta
        b2 /= b2.sum()
        v = np.max(np.sum(b2[:, None] * np.log(np.abs(1 - w2[:, None] * grid[None, :])), axis=0))
        assert v >= base - 1e-9 * abs(base)


def test_kappa_min_dirichlet_matches_spectrum():
    from oracle import spectral
    for shape in [(7, 9), (5, 6, 4), (64, 64)]:
        km = S.kappa_min_dirichlet(shape)
        assert math.isclose(km, float(np.min(spectral.kappas(shape))), rel_tol=1e-12)
        assert math.isclose(S.kappa_min_neumann(S.n_eff([n + 1 for n in shape])), km, rel_tol=1e-12)


def test_orderings_are_permutations_and_balanced_is_tighter():
    km = S.kappa_min_neumann(550)
    o = S.optimal(10, km)
    q = S.q_floor(o["beta"])
    for seq in (S.order_even(q), S.order_balanced(o["w"], q, km)):
        assert np.array_equal(np.bincount(seq, minlength=len(q)), q)
    even = S.partial_peaks(o["w"], S.order_even(q), km)
    bal = S.partial_peaks(o["w"], S.order_balanced(o["w"], q, km), km)
    assert bal[0] <= even[0] and bal[0] < 3.0


def test_even_order_positions_exact():
    seq = S.order_even([1, 2, 4])
    # positions: w1 at 1/2; w2 at 1/4, 3/4; w3 at 1/8, 3/8, 5/8, 7/8 ; tie 1/2 none
    assert list(seq) == [2, 1, 2, 0, 2, 1, 2]


def test_integer_scheme_stays_convergent():
    for P, N in [(2, 46.0), (8, 362.75), (10, 2897.0)]:
        km = S.kappa_min_neumann(N)
        o = S.optimal(P, km)
        q = S.q_floor(o["beta"])
        g = np.exp(np.linspace(math.log(km), math.log(2.0), 100001))
        assert S.gamma_q_max(o["w"], q, g) < 1.0


def test_balanced_order_hand_worked():
    """Balanced greedy order on a two-point grid {0.5, 2}, worked by hand.

    w = (3, 1, 0.6), q = (1, 2, 3), M = 6.  L_i = (ln|1 - 0.5 w_i|, ln|1 - 2 w_i|):
      L_1 = (ln 0.5, ln 5) = (-0.693147, 1.609438)
      L_2 = (ln 0.5, ln 1) = (-0.693147, 0)
      L_3 = (ln 0.7, ln 0.2) = (-0.356675, -1.609438)
    T = L_1 + 2 L_2 + 3 L_3 = (-3.149466, -3.218876); the step-k target is (k/6) T.
    Step k takes the weight with uses left minimising max over the grid of |s + L_i - (k/6) T|:
      k=1 target (-0.524911, -0.536479): i=1 -> 2.145917, i=2 -> 0.536479, i=3 -> 1.072959: take 2
      k=2 target (-1.049822, -1.072959), s = L_2: i=1 -> 2.682397, i=2 -> 1.072959,
          i=3 -> 0.536479: take 3
      k=3 target (-1.574733, -1.609438): i=1 -> 1.609438, i=2 -> 0.168236, i=3 -> 1.609438: take 2
      k=4 target (-2.099644, -2.145917) (weight 2 used up): i=1 -> 2.145917, i=3 -> 1.072959: take 3
      k=5 target (-2.624555, -2.682397): i=1 -> 1.072959, i=3 -> 2.145917: take 1
      k=6: only weight 3 is left.
    Taking the target one step early, the largest instead of the smallest maximum, or the
    signed instead of the absolute deviation each changes the sequence.
    """
    seq = S.order_balanced([3.0, 1.0, 0.6], [1, 2, 3], 0.5, 2.0, G=2)
    assert list(seq) == [1, 2, 1, 2, 0, 2]


def _mp_optimality(w, beta, km, kM=2.0):
    """Equal-maxima spread and first-order minimax residual of log Gamma (Eq. Gamma) at a
    point (w, beta), in 30-digit arithmetic, independent of the oracle's solver.

    The local maxima of log Gamma on [km, kM] are km, kM and one stationary point between
    each pair of consecutive poles 1/w_i (Sec. 3.2).  At a minimax optimum all P + 1 maxima
    are equal (Eq. equMax), and no move of (w, beta) with sum beta fixed lowers all of them
    at once: some convex combination mu of their gradients is parallel to the gradient of
    sum beta.  The residual of that linear system (least squares, mu summing to 1) is
    returned with the spread and the largest maximum."""
    import mpmath as mp

    mp.mp.dps = 30
    w = [mp.mpf(float(x)) for x in w]
    b = [mp.mpf(float(x)) for x in beta]
    tot = mp.fsum(b)
    b = [x / tot for x in b]
    P = len(w)
    lg = lambda k: mp.fsum(bi * mp.log(abs(1 - wi * k)) for wi, bi in zip(w, b))
    dlg = lambda k: mp.fsum(-bi * wi / (1 - wi * k) for wi, bi in zip(w, b))
    ks = [mp.mpf(float(km))]
    for i in range(P - 1):
        lo, hi = (1 / w[i]) * (1 + mp.mpf("1e-20")), (1 / w[i + 1]) * (1 - mp.mpf("1e-20"))
        ks.append(mp.findroot(dlg, (lo, hi), solver="anderson"))
    ks.append(mp.mpf(kM))
    vals = [lg(k) for k in ks]
    spread = (max(vals) - min(vals)) / abs(vals[0])
    A = mp.zeros(2 * P + 1, P + 2)
    rhs = mp.zeros(2 * P + 1, 1)
    for j, k in enumerate(ks):
        for i in range(P):
            A[i, j] = b[i] * (-k) / (1 - w[i] * k)
            A[P + i, j] = mp.log(abs(1 - w[i] * k))
    for i in range(P):
        A[P + i, P + 1] = -1
        A[2 * P, i] = 1
    A[2 * P, P] = 1
    rhs[2 * P] = 1
    x = mp.lu_solve(A.T * A, A.T * rhs)
    res = mp.norm(A * x - rhs) / mp.norm(A)
    mu = [x[j] for j in range(P + 1)]
    return float(spread), float(res), float(max(vals)), [float(m) for m in mu]


@pytest.mark.parametrize("P,N", [(4, 100), (5, 100)])
def test_near_rows_optimality_in_extended_precision(golden_dir, P, N):
    """Which point solves the optimality system of Sec. 3.2 for the two near rows: the
    oracle's (spread of the maxima and the first-order residual at 30-digit rounding level,
    multipliers positive).  The printed point has a higher maximum of Gamma and lies further
    from it than its 6 printed digits explain (the regular rows agree to about 3e-6)."""
    row = [r for r in read_table1(golden_dir) if r[0] == P and r[1] == N][0]
    km = S.kappa_min_neumann(N)
    o = S.optimal(P, km)
    sp_o, res_o, max_o, mu_o = _mp_optimality(o["w"], o["beta"], km)
    sp_p, res_p, max_p, _ = _mp_optimality(row[2], row[3], km)
    assert sp_o < 1e-11 and res_o < 1e-16 and min(mu_o) > 0, (sp_o, res_o, mu_o)
    assert max_p > max_o * (1 - 5e-5), (max_p, max_o)
    assert res_p > 1e5 * res_o and sp_p > 1e3 * sp_o
    assert float(np.max(np.abs(o["w"] / row[2] - 1.0))) > 2e-5


def test_regular_row_optimality_in_extended_precision(golden_dir):
    """A row reproduced to 3e-5: the oracle's point solves the system to 30-digit rounding
    level too, and the printed point's maximum is higher only by its 6-digit rounding."""
    row = [r for r in read_table1(golden_dir) if r[0] == 5 and r[1] == 200][0]
    km = S.kappa_min_neumann(200)
    o = S.optimal(5, km)
    sp_o, res_o, max_o, mu_o = _mp_optimality(o["w"], o["beta"], km)
    _, _, max_p, _ = _mp_optimality(row[2], row[3], km)
    assert sp_o < 1e-11 and res_o < 1e-16 and min(mu_o) > 0
    assert max_o <= max_p <= max_o * (1 - 1e-3)


def test_q_counts_simple_modes():
    """Sec. 4.3's conversions on fractions worked by hand: ratios 1, 3.49, 7.51, 88."""
    beta = [0.01, 0.0349, 0.0751, 0.88]
    assert list(S.q_counts(beta, 0)) == [1, 3, 7, 88]
    assert list(S.q_counts(beta, 1)) == [1, 3, 8, 88]
    assert list(S.q_counts(beta, 2)) == [1, 4, 8, 88]
    assert list(S.q_counts(beta, 0)) == list(S.q_floor(beta))


def test_q_counts_best_combination_is_the_exhaustive_minimum():
    """Mode 3 against an independent exhaustive search (numpy over a dense grid): no other
    floor/ceiling combination has a smaller per-step factor, and its factor is at most
    floor's, ceiling's and nearest's."""
    import itertools

    km = S.kappa_min_neumann(256)
    o = S.optimal(5, km)
    w, beta = o["w"], o["beta"]
    best = S.q_counts(beta, 3, w, km)
    grid = np.exp(np.linspace(math.log(km), math.log(2.0), 4096))
    grid[0], grid[-1] = km, 2.0
    L = np.log(np.abs(1.0 - np.asarray(w)[:, None] * grid[None, :]))

    def rate(q):
        q = np.asarray(q, dtype=np.float64)
        return float(np.max(q @ L)) / float(np.sum(q))

    r = beta / beta[0]
    choices = [[1]] + [sorted({int(math.floor(x)), int(math.ceil(x))}) for x in r[1:]]
    rates = {qs: rate(qs) for qs in itertools.product(*choices)}
    assert rate(best) <= min(rates.values()) * (1 - 1e-12) or math.isclose(rate(best), min(rates.values()),
                                                                              rel_tol=1e-12)
    for mode in (0, 1, 2):
        assert rate(best) <= rate(S.q_counts(beta, mode)) + 1e-15


@pytest.mark.parametrize("P,N", [(15, 64), (14, 4096)])
def test_p14_p15_oracle_rows_solve_the_system(golden_dir, P, N):
    """The oracle's P = 14 / 15 schemes (Tables 2-3 resolutions) satisfy the optimality
    system of Sec. 3.2 in 30-digit arithmetic, with a lower maximum of Gamma than the printed
    row; its rho exceeds the printed one by less than 1%."""
    rows = []
    for line in open(os.path.join(golden_dir, "table2_3.txt")):
        if line.strip() and not line.startswith("#"):
            a = line.split("|")
            if tuple(map(int, a[0].split())) == (P, N):
                rows.append((np.array(list(map(float, a[1].split()))), np.array(list(map(float, a[2].split()))),
                             float(a[3])))
    w_p, b_p, rho_p = rows[0]
    km = S.kappa_min_neumann(N)
    o = S.optimal(P, km)
    sp, res, mx, mu = _mp_optimality(o["w"], o["beta"], km)
    assert sp < 1e-10 and res < 1e-16 and min(mu) > 0, (sp, res, mu)
    assert mx <= _mp_optimality(w_p, b_p, km)[2]
    assert rho_p <= S.rho(o["w"], o["beta"]) <= 1.01 * rho_p
