// Fine-grained parallel ILU on the device (Chow and Patel, SIAM J. Sci.
// Comput. 37 (2015), the parallel ILU construction cited in the paper's
// introduction), synchronous form.  On the pattern S of E (A's values,
// explicit zeros at fill) the factors are the fixed point of
//     u_ij = a_ij - sum_{k < i} l_ik u_kj               (i <= j)
//     l_ij = (a_ij - sum_{k < j} l_ik u_kj) / u_jj      (i > j)
// over k with (i,k), (k,j) in S.  One sweep recomputes every entry -- one
// thread each -- from the previous sweep's L and U (double-buffered), the
// products subtracted in increasing k with separate roundings; the start
// is l_ij = a_ij / a_jj, u_ij = a_ij.  Deterministic: the factors after s
// sweeps are the same on every run.  For a symmetric A the incomplete
// Cholesky form keeps only U, with l_ki = u_ik / u_ii throughout:
//     u_ij = a_ij - sum_{k < i} (u_ki / u_kk) u_kj,
// so the factors stay symmetric after every sweep (the unsymmetric sweeps
// divide by the previous sweep's pivots and do not).  The pattern split and
// the factors stay
// on the device; a level-k pattern comes from the host's symbolic phase.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "sait_internal.h"

namespace sait {

namespace {

__device__ __forceinline__ double pmul(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double psub(double a, double b) {
#pragma clang fp contract(off)
    return a - b;
}

// Position of column j in the sorted row [b, e) of ci, or -1.
__device__ __forceinline__ int find_col(const int *ci, int b, int e, int j) {
    while (b < e) {
        const int m = (b + e) >> 1;
        const int c = ci[m];
        if (c == j) return m;
        if (c < j) b = m + 1;
        else e = m;
    }
    return -1;
}

struct Pattern {
    const int *lrp, *lci, *lrow;  // strictly lower part, CSR, row of every entry
    const double *la;             // a_ij on the lower part
    const int *urp, *uci, *urow;  // upper part with the diagonal
    const double *ua;
    int nl, nu;
};

// Start values; err |= 1 on a non-finite one when no sweep follows.
__global__ void k_parilu_start(Pattern p, double *__restrict__ l, double *__restrict__ u, int check,
                               int *__restrict__ err) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double out = 0.0;
    if (t < p.nl) {
        const int j = p.lci[t];
        out = p.la[t] / p.ua[p.urp[j]];
        l[t] = out;
    } else if (t < p.nl + p.nu) {
        out = p.ua[t - p.nl];
        u[t - p.nl] = out;
    }
    if (check && !isfinite(out)) atomicOr(err, 1);
}

// One synchronous sweep: (l0, u0) -> (l1, u1).  err |= 1 on a non-finite
// entry in the last sweep.
__global__ void k_parilu_sweep(Pattern p, const double *__restrict__ l0, const double *__restrict__ u0,
                               double *__restrict__ l1, double *__restrict__ u1, int check, int *__restrict__ err) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.nl + p.nu) return;
    const bool lower = t < p.nl;
    const int e = lower ? t : t - p.nl;
    const int i = lower ? p.lrow[e] : p.urow[e];
    const int j = lower ? p.lci[e] : p.uci[e];
    double acc = lower ? p.la[e] : p.ua[e];
    const int kb = p.lrp[i], ke = p.lrp[i + 1];
    for (int q = kb; q < ke; ++q) {
        const int k = p.lci[q];
        if (lower && k >= j) break;  // k < min(i, j)
        const int f = find_col(p.uci, p.urp[k], p.urp[k + 1], j);
        if (f >= 0) acc = psub(acc, pmul(l0[q], u0[f]));
    }
    double out;
    if (lower) {
        out = acc / u0[p.urp[j]];
        l1[e] = out;
    } else {
        out = acc;
        u1[e] = out;
    }
    if (check && !isfinite(out)) atomicOr(err, 1);
}

// Row i's strictly lower and upper counts; err |= 1 without a nonzero
// diagonal.
__global__ void k_pl_count(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                           int64_t *__restrict__ lcnt, int64_t *__restrict__ ucnt, int *__restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int nl = 0, nu = 0;
    bool diag = false;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
        const int j = ci[q];
        if (j < i) ++nl;
        else ++nu;
        if (j == i) diag = v[q] != 0.0;
    }
    lcnt[i] = nl;
    ucnt[i] = nu;
    if (!diag) atomicOr(err, 1);
}

// Split row i of E into its strictly lower and upper parts (the row order
// of both is E's, i.e. ascending columns).
__global__ void k_pl_split(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                           const int64_t *__restrict__ lptr, const int64_t *__restrict__ uptr, int *__restrict__ lrp,
                           int *__restrict__ urp, int *__restrict__ lci, double *__restrict__ la,
                           int *__restrict__ lrow, int *__restrict__ uci, double *__restrict__ ua,
                           int *__restrict__ urow) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    lrp[i] = (int)lptr[i];
    urp[i] = (int)uptr[i];
    if (i == n) return;
    int a = (int)lptr[i], b = (int)uptr[i];
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
        const int j = ci[q];
        if (j < i) {
            lci[a] = j;
            la[a] = v[q];
            lrow[a] = i;
            ++a;
        } else {
            uci[b] = j;
            ua[b] = v[q];
            urow[b] = i;
            ++b;
        }
    }
}

// L with its unit diagonal after the row's strictly lower entries.
__global__ void k_pl_assemble_l(int n, const int *__restrict__ lrp, const int *__restrict__ lci,
                                const double *__restrict__ lv, int *__restrict__ Lrp, int *__restrict__ Lci,
                                double *__restrict__ Lv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    Lrp[i] = lrp[i] + i;
    if (i == n) return;
    int o = lrp[i] + i;
    for (int q = lrp[i]; q < lrp[i + 1]; ++q, ++o) {
        Lci[o] = lci[q];
        Lv[o] = lv[q];
    }
    Lci[o] = i;
    Lv[o] = 1.0;
}

// Symmetric form: cpos[q] = position of (k, i) in U for the strictly lower
// entry q = (i, k); err |= 2 when the pattern is not structurally symmetric.
__global__ void k_pc_map(int nl, const int *__restrict__ lci, const int *__restrict__ lrow,
                         const int *__restrict__ urp, const int *__restrict__ uci, int *__restrict__ cpos,
                         int *__restrict__ err) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nl) return;
    const int k = lci[q], i = lrow[q];
    const int f = find_col(uci, urp[k], urp[k + 1], i);
    cpos[q] = f < 0 ? urp[k] : f;
    if (f < 0) atomicOr(err, 2);
}

__device__ __forceinline__ double pdiv(double a, double b) { return a / b; }

// One synchronous sweep of the symmetric form over the U entries:
//   u_ij = a_ij - sum_{k < i} fl(fl(u_ki / u_kk) u_kj),  k ascending.
__global__ void k_paric_sweep(Pattern p, const int *__restrict__ cpos, const double *__restrict__ u0,
                              double *__restrict__ u1, int check, int *__restrict__ err) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.nu) return;
    const int i = p.urow[e], j = p.uci[e];
    double acc = p.ua[e];
    for (int q = p.lrp[i]; q < p.lrp[i + 1]; ++q) {
        const int k = p.lci[q];
        const int f = find_col(p.uci, p.urp[k], p.urp[k + 1], j);
        if (f >= 0) acc = psub(acc, pmul(pdiv(u0[cpos[q]], u0[p.urp[k]]), u0[f]));
    }
    u1[e] = acc;
    if (check && !isfinite(acc)) atomicOr(err, 1);
}

// L of the symmetric form: l_ik = u_ki / u_kk, then the unit diagonal.
__global__ void k_pc_assemble_l(int n, const int *__restrict__ lrp, const int *__restrict__ lci,
                                const int *__restrict__ cpos, const int *__restrict__ urp,
                                const double *__restrict__ u, int *__restrict__ Lrp, int *__restrict__ Lci,
                                double *__restrict__ Lv, int *__restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    Lrp[i] = lrp[i] + i;
    if (i == n) return;
    int o = lrp[i] + i;
    for (int q = lrp[i]; q < lrp[i + 1]; ++q, ++o) {
        const int k = lci[q];
        const double l = pdiv(u[cpos[q]], u[urp[k]]);
        Lci[o] = k;
        Lv[o] = l;
        if (!isfinite(l)) atomicOr(err, 1);
    }
    Lci[o] = i;
    Lv[o] = 1.0;
}

}  // namespace

void parilu_device(Allocator *a, const DevCsr &E, int sweeps, bool symmetric, DevCsr &L, DevCsr &U,
                   hipStream_t s) {
    if (sweeps < 0) fail(SAIT_E_INVALID, "ParILU: sweeps must be >= 0");
    const int n = (int)E.n;
    const int rgrid = std::max(1, (n + 256) / 256);
    DevBuf lcnt, ucnt, lptr, uptr, err;
    lcnt.alloc(a, (size_t)std::max(n, 1) * sizeof(int64_t));
    ucnt.alloc(a, (size_t)std::max(n, 1) * sizeof(int64_t));
    lptr.alloc(a, (size_t)(n + 1) * sizeof(int64_t));
    uptr.alloc(a, (size_t)(n + 1) * sizeof(int64_t));
    err.alloc(a, sizeof(int));
    SAIT_HIP(hipMemsetAsync(err.as<void>(), 0, sizeof(int), s));
    hipLaunchKernelGGL(k_pl_count, dim3(rgrid), dim3(256), 0, s, n, E.rp.as<int>(), E.ci.as<int>(), E.v.as<double>(),
                       lcnt.as<int64_t>(), ucnt.as<int64_t>(), err.as<int>());
    SAIT_LAUNCH_CHECK();
    scan_exclusive_i64(a, lcnt.as<int64_t>(), lptr.as<int64_t>(), n, s);
    scan_exclusive_i64(a, ucnt.as<int64_t>(), uptr.as<int64_t>(), n, s);
    int64_t nl = 0, nu = 0;
    int herr = 0;
    SAIT_HIP(hipMemcpyAsync(&nl, lptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipMemcpyAsync(&nu, uptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (herr) fail(SAIT_E_ZERO_PIVOT, "ParILU: zero or missing diagonal entry");
    if (nl + nu + n > INT32_MAX) fail(SAIT_E_INVALID, "ParILU: more than 2^31-1 entries");
    DevBuf dlrp, dlci, dlrow, dla, durow, bl[2], bu[2];
    U.n = n;
    U.nnz = nu;
    U.precision = SAIT_F64;
    dlrp.alloc(a, (size_t)(n + 1) * sizeof(int));
    U.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
    dlci.alloc(a, (size_t)std::max<int64_t>(nl, 1) * sizeof(int));
    dlrow.alloc(a, (size_t)std::max<int64_t>(nl, 1) * sizeof(int));
    dla.alloc(a, (size_t)std::max<int64_t>(nl, 1) * sizeof(double));
    U.ci.alloc(a, (size_t)std::max<int64_t>(nu, 1) * sizeof(int));
    durow.alloc(a, (size_t)std::max<int64_t>(nu, 1) * sizeof(int));
    DevBuf dua;
    dua.alloc(a, (size_t)std::max<int64_t>(nu, 1) * sizeof(double));
    for (int b = 0; b < 2; ++b) {
        bl[b].alloc(a, (size_t)std::max<int64_t>(nl, 1) * sizeof(double));
        bu[b].alloc(a, (size_t)std::max<int64_t>(nu, 1) * sizeof(double));
    }
    hipLaunchKernelGGL(k_pl_split, dim3(rgrid), dim3(256), 0, s, n, E.rp.as<int>(), E.ci.as<int>(), E.v.as<double>(),
                       lptr.as<int64_t>(), uptr.as<int64_t>(), dlrp.as<int>(), U.rp.as<int>(), dlci.as<int>(),
                       dla.as<double>(), dlrow.as<int>(), U.ci.as<int>(), dua.as<double>(), durow.as<int>());
    SAIT_LAUNCH_CHECK();
    Pattern p;
    p.lrp = dlrp.as<int>();
    p.lci = dlci.as<int>();
    p.lrow = dlrow.as<int>();
    p.la = dla.as<double>();
    p.urp = U.rp.as<int>();
    p.uci = U.ci.as<int>();
    p.urow = durow.as<int>();
    p.ua = dua.as<double>();
    p.nl = (int)nl;
    p.nu = (int)nu;
    const int grid = (int)std::max<int64_t>(1, (nl + nu + 255) / 256);
    if (symmetric) {
        // U only; L follows from the final U
        DevBuf cpos;
        cpos.alloc(a, (size_t)std::max<int64_t>(nl, 1) * sizeof(int));
        hipLaunchKernelGGL(k_pc_map, dim3((int)std::max<int64_t>(1, (nl + 255) / 256)), dim3(256), 0, s, (int)nl,
                           dlci.as<int>(), dlrow.as<int>(), U.rp.as<int>(), U.ci.as<int>(), cpos.as<int>(),
                           err.as<int>());
        SAIT_LAUNCH_CHECK();
        SAIT_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipStreamSynchronize(s));
        if (herr & 2) fail(SAIT_E_INVALID, "ParIC: the pattern is not structurally symmetric");
        SAIT_HIP(hipMemcpyAsync(bu[0].as<void>(), dua.as<void>(), (size_t)nu * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
        const int ugrid = (int)std::max<int64_t>(1, (nu + 255) / 256);
        int cur = 0;
        for (int sw = 0; sw < sweeps; ++sw) {
            hipLaunchKernelGGL(k_paric_sweep, dim3(ugrid), dim3(256), 0, s, p, cpos.as<int>(), bu[cur].as<double>(),
                               bu[cur ^ 1].as<double>(), (int)(sw + 1 == sweeps), err.as<int>());
            SAIT_LAUNCH_CHECK();
            cur ^= 1;
        }
        L.n = n;
        L.nnz = nl + n;
        L.precision = SAIT_F64;
        L.vs.reset();
        L.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
        L.ci.alloc(a, (size_t)std::max<int64_t>(nl + n, 1) * sizeof(int));
        L.v.alloc(a, (size_t)std::max<int64_t>(nl + n, 1) * sizeof(double));
        hipLaunchKernelGGL(k_pc_assemble_l, dim3(rgrid), dim3(256), 0, s, n, dlrp.as<int>(), dlci.as<int>(),
                           cpos.as<int>(), U.rp.as<int>(), bu[cur].as<double>(), L.rp.as<int>(), L.ci.as<int>(),
                           L.v.as<double>(), err.as<int>());
        SAIT_LAUNCH_CHECK();
        U.v = std::move(bu[cur]);
        U.vs.reset();
        SAIT_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipStreamSynchronize(s));
        if (herr) fail(SAIT_E_NONFINITE, "ParIC: the sweeps produced a non-finite factor entry");
        return;
    }
    hipLaunchKernelGGL(k_parilu_start, dim3(grid), dim3(256), 0, s, p, bl[0].as<double>(), bu[0].as<double>(),
                       (int)(sweeps == 0), err.as<int>());
    SAIT_LAUNCH_CHECK();
    int cur = 0;
    for (int sw = 0; sw < sweeps; ++sw) {
        hipLaunchKernelGGL(k_parilu_sweep, dim3(grid), dim3(256), 0, s, p, bl[cur].as<double>(), bu[cur].as<double>(),
                           bl[cur ^ 1].as<double>(), bu[cur ^ 1].as<double>(), (int)(sw + 1 == sweeps),
                           err.as<int>());
        SAIT_LAUNCH_CHECK();
        cur ^= 1;
    }
    // U takes the final value buffer; L gets its unit diagonal
    U.v = std::move(bu[cur]);
    U.vs.reset();
    L.n = n;
    L.nnz = nl + n;
    L.precision = SAIT_F64;
    L.vs.reset();
    L.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
    L.ci.alloc(a, (size_t)std::max<int64_t>(nl + n, 1) * sizeof(int));
    L.v.alloc(a, (size_t)std::max<int64_t>(nl + n, 1) * sizeof(double));
    hipLaunchKernelGGL(k_pl_assemble_l, dim3(rgrid), dim3(256), 0, s, n, dlrp.as<int>(), dlci.as<int>(),
                       bl[cur].as<double>(), L.rp.as<int>(), L.ci.as<int>(), L.v.as<double>());
    SAIT_LAUNCH_CHECK();
    SAIT_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (herr) fail(SAIT_E_NONFINITE, "ParILU: the sweeps produced a non-finite factor entry");
}

}  // namespace sait
