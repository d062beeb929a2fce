// LOBPCG driver (k_lobpcg.hip): device block operations, host Rayleigh-Ritz.
#pragma once

#include <functional>

#include "sait_internal.h"

namespace sait {

// Y = Op(X) for n x k row-major device blocks on stream s.
using BlockOp = std::function<void(const double *X, double *Y, hipStream_t s)>;

// Smallest admissible Cholesky pivot L_jj^2 of the unit-diagonal scaled
// S^T S: kPivotP for [X, W, P] (below it the step drops P), kPivotMin for
// [X, W] and the start block (below it the basis counts as numerically
// dependent).  The Rayleigh-Ritz values lose about as many digits as the
// basis condition number has: with [X, W, P] pivots near 1e-10 a clustered
// spectrum's Ritz values drifted below the smallest eigenvalue and the
// iteration diverged; near convergence W is small and noisy, and the
// stricter bound on [X, W] would stop the iteration one step short.
constexpr double kPivotMin = 1e-14;
constexpr double kPivotP = 1e-8;

class Lobpcg {
  public:
    Lobpcg();
    Lobpcg(const Lobpcg &) = delete;
    Lobpcg &operator=(const Lobpcg &) = delete;
    ~Lobpcg();
    // X: n x k device block (start block in, Ritz vectors out); lambda: host
    // (k); history: host (maxit + 1) or null.  Returns a status code.
    int run(Allocator *a, int64_t n, int k, double *X, const BlockOp &applyA, const BlockOp &applyT,
            const sait_eig_opts &o, double *lambda, double *history, sait_eig_info *info, hipStream_t s);

  private:
    struct Bufs;
    Bufs *b_;
};

}  // namespace sait
