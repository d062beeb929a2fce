// The comparison preconditioners of the paper's experiments (Sec. 4):
//  * s Jacobi sweeps on each triangular factor (Sec. 4, comparison with the
//    Jacobi iteration): from y = 0, y_i <- (r_i - sum_{j != i} T_ij y_j) / T_ii
//    over the previous iterate -- the truncated series SAIT_Thr(0, s - 1)
//    evaluated without forming it;
//  * the exact triangular solves of the ILU factors (forward / backward
//    substitution), level-scheduled: rows whose dependencies are all in
//    earlier levels are solved together, one launch per level.
// Each row is computed in the CSR column order with separately rounded
// products and differences, as the substitution is written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "sait_internal.h"

namespace sait {

namespace {

constexpr int kNT = 256;

__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// y = r / d (one Jacobi sweep from y = 0)
__global__ void k_div(int64_t n, const double *__restrict__ r, const double *__restrict__ d, double *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = r[i] / d[i];
}

// x_i = (b_i - sum_{j != i} T_ij x_j) / T_ii for the rows of one level
__global__ void k_level_rows(int nrows, const int *__restrict__ rows, const int *__restrict__ rp,
                             const int *__restrict__ ci, const double *__restrict__ v, const double *__restrict__ b,
                             double *__restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int i = rows[t];
    double acc = b[i], d = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int c = ci[p];
        if (c == i) {
            d = v[p];
        } else {
#pragma clang fp contract(off)
            acc = acc - mul_rn(v[p], x[c]);
        }
    }
    x[i] = acc / d;
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kNT - 1) / kNT, 8192)); }

}  // namespace

void build_jacobi(Allocator *a, const HostCsr &T, JacobiFactor &J, hipStream_t s) {
    HostCsr N;
    N.n = T.n;
    N.rp.assign(T.n + 1, 0);
    std::vector<double> d(T.n, 0.0);
    N.ci.reserve(T.ci.size());
    N.v.reserve(T.v.size());
    for (int64_t i = 0; i < T.n; ++i) {
        for (int32_t p = T.rp[i]; p < T.rp[i + 1]; ++p) {
            if (T.ci[p] == i) {
                d[i] = T.v[p];
            } else {
                N.ci.push_back(T.ci[p]);
                N.v.push_back(T.v[p]);
            }
        }
        if (d[i] == 0.0) fail(SAIT_E_ZERO_PIVOT, "Jacobi preconditioner: zero diagonal entry");
        N.rp[i + 1] = (int32_t)N.ci.size();
    }
    upload_csr(a, N, J.N, s);
    prepare_sell(a, J.N, s);
    J.d.alloc(a, sizeof(double) * (size_t)std::max<int64_t>(T.n, 1));
    if (T.n) SAIT_HIP(hipMemcpyAsync(J.d.as<void>(), d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice, s));
    SAIT_HIP(hipStreamSynchronize(s));
}

void jacobi_apply(const JacobiFactor &J, int sweeps, const double *r, double *y, double *tmp, hipStream_t s) {
    const int64_t n = J.N.n;
    if (n == 0) return;
    if (sweeps < 1) fail(SAIT_E_INVALID, "Jacobi sweeps must be >= 1");
    // ping-pong between y and tmp so that the last sweep writes y
    double *buf[2] = {y, tmp};
    int cur = (sweeps % 2 == 1) ? 0 : 1;
    hipLaunchKernelGGL(k_div, dim3(grid_for(n)), dim3(kNT), 0, s, n, r, J.d.as<double>(), buf[cur]);
    SAIT_LAUNCH_CHECK();
    for (int k = 1; k < sweeps; ++k) {
        jacobi_sweep(J.N, J.d.as<double>(), r, buf[cur], buf[cur ^ 1], s);
        cur ^= 1;
    }
}

void build_levels(Allocator *a, const HostCsr &T, bool lower, LevelFactor &F, hipStream_t s) {
    const int64_t n = T.n;
    std::vector<int> level(n, 0);
    int nlev = 0;
    for (int64_t t = 0; t < n; ++t) {
        const int64_t i = lower ? t : n - 1 - t;
        int lv = 0;
        bool has_diag = false;
        for (int32_t p = T.rp[i]; p < T.rp[i + 1]; ++p) {
            const int64_t c = T.ci[p];
            if (c == i) {
                has_diag = T.v[p] != 0.0;
            } else {
                if (lower ? c > i : c < i) fail(SAIT_E_INVALID, "triangular solve: entry on the wrong side of the diagonal");
                lv = std::max(lv, level[c] + 1);
            }
        }
        if (!has_diag) fail(SAIT_E_ZERO_PIVOT, "triangular solve: missing or zero diagonal entry");
        level[i] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    F.level_ptr.assign(nlev + 1, 0);
    for (int64_t i = 0; i < n; ++i) F.level_ptr[level[i] + 1]++;
    for (int l = 0; l < nlev; ++l) F.level_ptr[l + 1] += F.level_ptr[l];
    std::vector<int> rows(std::max<int64_t>(n, 1));
    std::vector<int> fill(F.level_ptr.begin(), F.level_ptr.end() - (nlev > 0 ? 1 : 0));
    for (int64_t i = 0; i < n; ++i) rows[fill[level[i]]++] = (int)i;
    upload_csr(a, T, F.T, s);
    F.rows.alloc(a, sizeof(int) * rows.size());
    SAIT_HIP(hipMemcpyAsync(F.rows.as<void>(), rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, s));
    SAIT_HIP(hipStreamSynchronize(s));
}

void level_solve(const LevelFactor &F, const double *b, double *x, hipStream_t s) {
    const int nlev = (int)F.level_ptr.size() - 1;
    for (int l = 0; l < nlev; ++l) {
        const int r0 = F.level_ptr[l], cnt = F.level_ptr[l + 1] - r0;
        hipLaunchKernelGGL(k_level_rows, dim3((cnt + kNT - 1) / kNT), dim3(kNT), 0, s, cnt, F.rows.as<int>() + r0,
                           F.T.rp.as<int>(), F.T.ci.as<int>(), F.T.v.as<double>(), b, x);
    }
    SAIT_LAUNCH_CHECK();
}

}  // namespace sait
