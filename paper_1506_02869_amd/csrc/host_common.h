// Host-side helpers shared by the single-scenario engine and the batched
// engine: scenario validation, rollout scalars, per-aircraft parameter rows,
// the tempering schedule and the 1-D wind-covariance factors.
#pragma once

#include <string>
#include <vector>

#include "engine.h"
#include "smc_mpc.h"

namespace smc {
namespace host {

// Number of wind samples of iteration J before the scale kappa (Sec. "Wind
// Model" schedule): floor(3 + 5 exp(0.05 J)).
double sample_schedule(int J);

// Lower Cholesky factor of the 1-D squared-exponential Gram matrix on n
// evenly spaced nodes of [lo, hi] plus the nugget (FP64); false if not
// positive definite.
bool axis_factor(int n, double lo, double hi, double ell, double nugget, std::vector<double>& Lo);

// Factors of the exponential covariance (Sec. "Wind Model", eq. cov):
// Lh = chol(R_h + nugget I) over the nx ny horizontal nodes p = ix ny + iy,
// R_h[p][q] = exp(-beta |xy_p - xy_q|) (Euclidean), and Lz = chol(R_z +
// nugget I), R_z[a][b] = exp(-gamma |z_a - z_b|); nodes evenly spaced over
// the box as for axis_factor.  FP64, row-major; false if not positive
// definite.
bool exp_factors(int nx, int ny, int nz, const double box[3], double beta, double gamma,
                 double nugget, std::vector<double>& Lh, std::vector<double>& Lz);

// Checks one scenario; on failure returns the status and sets msg.
smc_status validate_scenario(const smc_scenario* s, std::string& msg);

// Rollout scalars of a scenario (H = horizon_max, P = n_particles).
void fill_rollout_params(const smc_scenario* s, RolloutParams& rp);

// Constants of the world-per-lane rollout (both precisions) from the
// scalars already in rp.
void fill_rollout_consts(RolloutParams& rp);

// Per-aircraft parameter rows [N][kAcR] of the world-per-lane rollout.
void fill_acR(const smc_scenario* s, std::vector<double>& t);

}  // namespace host
}  // namespace smc
