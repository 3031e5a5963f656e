// Host-side SRJ schedule planner: optimal weights (Sec. 3), integer counts (Sec. 4.3) and
// the order of the steps inside one cycle (Sec. 5.1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#define SRJ_PLAN_MAXP 16

namespace srj {

struct Optimum {
    std::vector<double> w;      // descending weights w_1 > ... > w_P
    std::vector<double> beta;   // fractions, sum 1
    std::vector<double> kappa;  // interior maxima of Gamma (P - 1)
};

// Smallest Jacobi symbol of the Dirichlet grid: (2/d) sum_i sin^2(pi / (2 (n_i + 1))) with
// equal spacings (wt = null); with axis weights wt = {wy, wz, dg} (the equation multiplied
// through by h_x^2) it is 4 (s_x + wy s_y [+ wz s_z]) / dg, s_i = sin^2(pi / (2 (n_i + 1))).
double grid_kappa_min(int ndim, const int64_t* n, const double* wt = nullptr);
// Largest Jacobi symbol of the Dirichlet grid: the same with cos^2.
double grid_kappa_max(int ndim, const int64_t* n, const double* wt = nullptr);
// The same for a cell-centred grid of n_i cells with homogeneous Neumann boundaries (Sec. 3.1,
// Eq. boundaries1D3D): symbols 4 sum_i a_i sin^2(k_i pi / (2 n_i)) / dg, k_i = 0..n_i - 1; the
// smallest nonzero one is 4 min_i a_i sin^2(pi / (2 n_i)) / dg ((2/d) sin^2(pi / 2N) with
// equal spacings), the largest 4 sum_i a_i cos^2(pi / (2 n_i)) / dg.
double neumann_kappa_min(int ndim, const int64_t* n, const double* wt = nullptr);
double neumann_kappa_max(int ndim, const int64_t* n, const double* wt = nullptr);

// Minimax-optimal P-level scheme on [km, kM]; false (with a message) if the solve fails.
bool optimal_schedule(int P, double km, double kM, Optimum* out, std::string* err);

// q_i = floor(beta_i / beta_1).
std::vector<int64_t> floor_counts(const std::vector<double>& beta);

// Integer counts from the fractions (Sec. 4.3): mode 0 floor, 1 nearest integer, 2 ceiling
// of beta_i / beta_1 (q_1 = 1 in every mode), 3 floor or ceiling per level, whichever
// combination gives the smallest max over [km, kM] of |prod (1 - w_i k)^q_i|^(1/M) (P <= 12;
// ties to the combination with more floors, then to the lower levels' floors).  Returns an
// empty vector for a bad mode.
std::vector<int64_t> round_counts(const std::vector<double>& beta, int mode, const double* w, double km,
                                  double kM);

// Order of the M steps: balanced greedy (0) or even spread (1).
std::vector<int32_t> order_steps(int P, const double* w, const int64_t* q, double km, double kM,
                                 int ordering);

// max over a log-spaced grid of [km, kM] of |prod (1 - w_i k)^q_i|^(1/M).
double gamma_q_max(int P, const double* w, const int64_t* q, double km, double kM);

// log10 of the largest prefix / suffix partial product of an ordered cycle over [km, kM].
void partial_peaks(int P, const double* w, const std::vector<int32_t>& seq, double km, double kM,
                   double* prefix_log10, double* suffix_log10);

}  // namespace srj
