// Host-side launch sequences of the device kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mvn {

// Lower triangle of the padded ld x ld matrix A (row-major) from the caller's
// Sigma (row stride lds) or from locations with the Matern kernel; rows and
// columns n..ld-1 become the identity.  Also clears *info.
hipError_t launch_build_matrix(int n, int ld, const double* sigma, int lds, const double* locs,
                               double sigma2, double beta, double nu, double nugget, double* A,
                               int* info, hipStream_t st);

// In-place right-looking tiled Cholesky of the padded matrix; *info gets the
// 1-based index of the first non-positive pivot.  Upper triangle zeroed.
hipError_t launch_cholesky_f64(int ld, int tile, double* A, int* info, hipStream_t st);

struct SweepArgs {
  const double* L;
  int ld;
  int n;
  const double* at;        // centred lower limits (padded to ld)
  const double* bt;        // centred upper limits
  const uint64_t* lattice; // A_i, n entries
  uint64_t seed;           // shift D_{s,i} = SplitMix64 output s*n + i from this state
  int N, S, periodize;
  double* yscr;            // per-workgroup scratch, grid x ld x 128 doubles
  double* ell;             // N*S per-sample log-products
  int grid;                // persistent workgroups
};

// Setup of one probability call: centred limits and the invalid-limit flag.
hipError_t launch_prob_setup(int n, int ld, const double* a, const double* b, const double* mu,
                             double* at, double* bt, int* bad, hipStream_t st);

hipError_t launch_sweep_f64(const SweepArgs& a, hipStream_t st);

// log-sum-exp over samples, per shift and overall, into out[4 + S].
hipError_t launch_reduce(const double* ell, int N, int S, double* part, const int* info_factor,
                         const int* bad_limits, double* out, hipStream_t st);

int sweep_tile_cols();

}  // namespace mvn
