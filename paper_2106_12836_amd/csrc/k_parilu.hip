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
// sweeps are the same on every run.  The symbolic pattern stays on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

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

}  // namespace

void parilu_device(Allocator *a, const HostCsr &E, int sweeps, HostCsr &L, HostCsr &U, hipStream_t s) {
    if (sweeps < 0) fail(SAIT_E_INVALID, "ParILU: sweeps must be >= 0");
    const int64_t n = E.n;
    // host: split the pattern, check the diagonal
    std::vector<int32_t> lrp(n + 1, 0), urp(n + 1, 0), lci, uci, lrow, urow;
    std::vector<double> la, ua;
    lci.reserve(E.nnz());
    uci.reserve(E.nnz());
    for (int64_t i = 0; i < n; ++i) {
        bool diag = false;
        for (int32_t q = E.rp[i]; q < E.rp[i + 1]; ++q) {
            const int32_t j = E.ci[q];
            if (j < i) {
                lci.push_back(j);
                la.push_back(E.v[q]);
                lrow.push_back((int32_t)i);
            } else {
                if (j == i) diag = E.v[q] != 0.0;
                uci.push_back(j);
                ua.push_back(E.v[q]);
                urow.push_back((int32_t)i);
            }
        }
        if (!diag) fail(SAIT_E_ZERO_PIVOT, "ParILU: zero or missing diagonal entry");
        lrp[i + 1] = (int32_t)lci.size();
        urp[i + 1] = (int32_t)uci.size();
    }
    const int64_t nl = (int64_t)lci.size(), nu = (int64_t)uci.size();
    if (nl + nu > INT32_MAX) fail(SAIT_E_INVALID, "ParILU: more than 2^31-1 entries");
    auto up = [&](DevBuf &d, const void *src, size_t bytes) {
        d.alloc(a, std::max<size_t>(bytes, 16));
        if (bytes) SAIT_HIP(hipMemcpyAsync(d.as<void>(), src, bytes, hipMemcpyHostToDevice, s));
    };
    DevBuf dlrp, dlci, dlrow, dla, durp, duci, durow, dua, bl[2], bu[2], err;
    up(dlrp, lrp.data(), (n + 1) * sizeof(int32_t));
    up(dlci, lci.data(), nl * sizeof(int32_t));
    up(dlrow, lrow.data(), nl * sizeof(int32_t));
    up(dla, la.data(), nl * sizeof(double));
    up(durp, urp.data(), (n + 1) * sizeof(int32_t));
    up(duci, uci.data(), nu * sizeof(int32_t));
    up(durow, urow.data(), nu * sizeof(int32_t));
    up(dua, ua.data(), nu * sizeof(double));
    for (int b = 0; b < 2; ++b) {
        bl[b].alloc(a, std::max<size_t>(nl * sizeof(double), 16));
        bu[b].alloc(a, std::max<size_t>(nu * sizeof(double), 16));
    }
    err.alloc(a, sizeof(int));
    SAIT_HIP(hipMemsetAsync(err.as<void>(), 0, sizeof(int), s));
    Pattern p;
    p.lrp = dlrp.as<int>();
    p.lci = dlci.as<int>();
    p.lrow = dlrow.as<int>();
    p.la = dla.as<double>();
    p.urp = durp.as<int>();
    p.uci = duci.as<int>();
    p.urow = durow.as<int>();
    p.ua = dua.as<double>();
    p.nl = (int)nl;
    p.nu = (int)nu;
    const int grid = (int)std::max<int64_t>(1, (nl + nu + 255) / 256);
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
    std::vector<double> lv(nl), uv(nu);
    if (nl) SAIT_HIP(hipMemcpyAsync(lv.data(), bl[cur].as<void>(), nl * sizeof(double), hipMemcpyDeviceToHost, s));
    if (nu) SAIT_HIP(hipMemcpyAsync(uv.data(), bu[cur].as<void>(), nu * sizeof(double), hipMemcpyDeviceToHost, s));
    int herr = 0;
    SAIT_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (herr) fail(SAIT_E_NONFINITE, "ParILU: the sweeps produced a non-finite factor entry");
    // L with its unit diagonal (after the row's strictly lower entries), U
    L = HostCsr{};
    U = HostCsr{};
    L.n = U.n = n;
    L.rp.assign(n + 1, 0);
    L.ci.reserve(nl + n);
    L.v.reserve(nl + n);
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t e = lrp[i]; e < lrp[i + 1]; ++e) {
            L.ci.push_back(lci[e]);
            L.v.push_back(lv[e]);
        }
        L.ci.push_back((int32_t)i);
        L.v.push_back(1.0);
        L.rp[i + 1] = (int32_t)L.ci.size();
    }
    U.rp = std::move(urp);
    U.ci = std::move(uci);
    U.v = std::move(uv);
}

}  // namespace sait
