// Schedule of a plan (Sec. 2-4) from an srj_schedule request, shared by single-grid plans and
// batches: weights and fractions (optimised or explicit), integer counts, the order of the M
// steps, and the checks of the integer scheme on the grid's own spectrum.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/srj.h"

namespace srj {

struct SchedOut {
    int P = 0;
    double omega[SRJ_MAX_LEVELS] = {0};
    double beta[SRJ_MAX_LEVELS] = {0};
    int64_t q[SRJ_MAX_LEVELS] = {0};
    int64_t M = 0;
    std::vector<int32_t> seq;
    double kappa_min = 0, kappa_max = 0, rho = 0, gamma_q = 0, pre = 0, suf = 0;
};

// The spectrum the schedule is built and checked on.
enum SpecKind {
    SPEC_DIRICHLET = 0,  // Poisson operator, Dirichlet ring: the grid's exact symbols
    SPEC_NEUMANN = 1,    // Poisson operator, homogeneous Neumann (cell-centred) boundaries
    SPEC_OPERATOR = 2,   // a user's operator: [kappa_min as requested, 2] (Eq. boundaries' kappa_M)
};

// ndim, n: the grid; wt: its axis weights {wy, wz, dg} (null: equal spacings).  With
// peaks = false the prefix / suffix peaks are not computed.
srj_status make_schedule(int ndim, const int64_t* n, const double* wt, const srj_schedule* sc, bool peaks,
                         SchedOut* out, std::string* err, SpecKind kind = SPEC_DIRICHLET);

}  // namespace srj
