// LOBPCG driver (k_lobpcg.hip): device block operations, host Rayleigh-Ritz.
#pragma once

#include <functional>

#include "sait_internal.h"

namespace sait {

// Y = Op(X) for n x k row-major device blocks on stream s.
using BlockOp = std::function<void(const double *X, double *Y, hipStream_t s)>;

// Smallest admissible Cholesky pivot L_jj^2 of the unit-diagonal scaled
// S^T S; below it the trial basis counts as numerically dependent.
constexpr double kPivotMin = 1e-14;

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
