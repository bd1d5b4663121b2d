// Internal declarations shared by the HIP kernels and the host driver of libfld.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace fld {

// cgs constants
constexpr double kC = 2.99792458e10;
constexpr double kSigmaSB = 5.670374419e-5;
constexpr double kARad = 4.0 * kSigmaSB / kC;

// Tiling of the 2D stencil kernels: 256 threads as 64 x 4, each thread owns
// 4 rows of a 64 x 16 cell tile.  Wave64: one wavefront = one 64-cell row.
constexpr int TBX = 64;
constexpr int TBY = 4;
constexpr int TRows = 16;
constexpr int kThreads = TBX * TBY;
constexpr int k1DBlocksMax = 2048;   // grid size cap of the 1D streaming kernels

enum { BC_REFLECT = 0, BC_DIRICHLET_FACE = 1, BC_DIRICHLET_GHOST = 2, BC_FLUX_IN = 3, BC_FREE_STREAM = 4, BC_AXIS = 5,
       BC_MILNE = 6 };
enum { LIM_LP = 0, LIM_MINERBO = 1, LIM_DIFFUSION = 2 };

// Separable grid metrics, FP64, device arrays.
//   dV(i,j)      = vx[i] * vy[j]
//   dS_x(f,j)    = sx[f] * vy[j]        x/r face f between cells f-1 and f
//   dS_y(i,f)    = ax[i] * sy[f]        y/theta face f between rows f-1 and f
//   centre-to-face distances: x: hxL[f], hxR[f]; y: (hyL[f], hyR[f]) * arc[i]
struct Metrics {
    int nx, ny;
    const double *vx, *vy, *sx, *sy, *ax, *hxL, *hxR, *hyL, *hyR, *arc;
};

struct BCDev {
    int kind[4];
    double value[4];
};

// Device-resident solver state of one solve (one context).
struct Scalars {
    double rz_old;      // r.z of the previous iteration (scaled to the current residual scale)
    double rz_cur;      // r.z of this iteration (summed by k_spmv from the last sweep's partials)
    double alpha, beta;
    double pscale;      // factor applied to p at the next p-update (residual rescaling)
    double rr;          // inner residual norm^2 (recurrence)
    double rr_ref;      // inner residual norm^2 at the last reliable update
    double gamma;       // current residual scale: r_inner = r / gamma, gamma = ||r||_2
    double corr;        // gamma / mu: E += corr * x_inner
    double corr_apply;  // the correction the last true-residual check evaluated E with
    double rho_last;    // last true relative residual (selected norm)
    double sums[4];     // true residual: ||r/dV||^2, ||S r||^2, ||rhs/dV||^2, ||S rhs||^2
    double rel_row, rel_scaled, rel_sel;
    double eps;         // target relative residual
    double best;        // smallest true relative residual seen in this solve
    double delta2;      // reliable-update threshold (squared)
    double inner_tol2;  // FP32-only: stop when rr <= inner_tol2
    int iter, done, pending, status;
    int max_iter, norm, reliable, nchecks;
    int stall;          // true-residual checks without progress
    int restart;        // next p-update starts a new search direction
    int demote;         // a new true residual waits to be demoted
    int apply;          // a check happened: E += corr_apply x_inner and the demotion are due
};

enum {
    ST_OK = 0, ST_ENOCONV = 4, ST_EBREAKDOWN = 5, ST_ENONFINITE = 6
};

}  // namespace fld
