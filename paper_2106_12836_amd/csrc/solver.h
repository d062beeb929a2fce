// Device-resident restarted (F)GMRES state and its host driver.
#pragma once

#include "sait_internal.h"

namespace sait {

// Lives in device memory; the array pointers point into one device buffer.
struct GmresDev {
    double *Hraw, *R;   // (restart+1) x restart, column-major: Arnoldi Hessenberg, and after the rotations
    double *Gam;        // restart x restart, column-major (FGMRES): z~_j = sum_i Gam_ij z_i; null for GMRES
    double *cs, *sn, *g, *y, *yh, *s1, *s1n, *ca, *cg;
    double *red;        // 2 restart + 2 reduced inner products of the current step
    double nb, beta, est, rinv, eor, rtol;
    int restart, maxit, iters, jc, done;
};

// Operators of one solve: A (FP64) and the preconditioner: SAIT z = M2 (M1 v)
// (default), s Jacobi sweeps on L then U, the exact solves with L then U,
// or none.
struct Ops {
    const DevCsr *A = nullptr, *M1 = nullptr, *M2 = nullptr;
    int lanesA = 8, lanes1 = 8, lanes2 = 8;
    int precision = SAIT_F64;
    int prec_kind = SAIT_PREC_SAIT;
    int sweeps = 1;
    const JacobiFactor *JL = nullptr, *JU = nullptr;
    const LevelFactor *EL = nullptr, *EU = nullptr;
};

// Device state of a PCG solve.
struct PcgDev {
    double nb, rz, alpha, beta, relres, rtol, true_rr;
    int iters, maxit, done, breakdown;
};

class Solver {
  public:
    Solver() = default;
    Solver(const Solver &) = delete;
    Solver &operator=(const Solver &) = delete;
    ~Solver();
    int solve(Allocator *a, const Ops &ops, const double *b, double *x, const sait_solve_opts &o,
              sait_solve_info *info, hipStream_t s);
    // Preconditioned conjugate gradients (o.method == SAIT_METHOD_PCG).
    int pcg(Allocator *a, const Ops &ops, const double *b, double *x, const sait_solve_opts &o,
            sait_solve_info *info, hipStream_t s);
    // z = M r with the preconditioner of ops (r and z distinct, n doubles).
    void apply_prec(const Ops &ops, const double *in, double *out, hipStream_t s);

  private:
    void ensure(Allocator *a, int64_t n, int restart, bool flexible, int precision);
    void ensure_prec_tmp(Allocator *a, int64_t n, int precision);
    static void fill_info(sait_solve_info *info, int iters, int restarts, int status, double est, double relres);

    int64_t n_ = -1, ldv_ = 0;
    int restart_ = 0;
    bool flex_ = false;
    DevBuf V_, Z_, zt_, ut_, y32_, arr_, st_, part_;
    DevBuf pt1_, pt2_;                      // preconditioner scratch (Jacobi sweeps, exact solves)
    DevBuf pr_, pz_, pp_, pq_, pst_, ppart_;  // PCG vectors, state, partial sums
    int64_t pn_ = -1;
    void *mailbox_ = nullptr;
};

// Operators of a batched solve: block-diagonal A and its SAIT factors (FP64,
// sliced-ELL copies prepared) and the first row of every system.
struct BatchedOps {
    const DevCsr *A = nullptr, *ML = nullptr, *MU = nullptr;
    std::vector<int64_t> sys_ptr;
};

// One persistent cooperative launch solving every (system, right-hand side)
// pair with its own restarted right-preconditioned GMRES (k_batched.hip).
class BatchedSolver {
  public:
    BatchedSolver();
    BatchedSolver(const BatchedSolver &) = delete;
    BatchedSolver &operator=(const BatchedSolver &) = delete;
    ~BatchedSolver();
    // R <= 8 right-hand sides, b and x row-major n x ld (device)
    int solve(Allocator *a, const BatchedOps &ops, const double *b, double *x, int R, int64_t ld,
              const sait_solve_opts &o, sait_solve_info *info, hipStream_t s);

  private:
    struct Impl;
    Impl *impl_;
};

// dst[r*ldd] = src[r*lds] for r < n.
void copy_strided(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, hipStream_t s);

// Streaming device copy (bandwidth reference), bytes a multiple of 16.
void copy_bytes(const void *src, void *dst, size_t bytes, hipStream_t s);

// grad[p] = -lambda[row p] * x[col p] over the stored entries of A.
void grad_values(const DevCsr &A, const double *lambda, const double *x, double *grad, hipStream_t s);

}  // namespace sait
