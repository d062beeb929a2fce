// CSR sparse matrix-vector and matrix-block products: the SAIT apply
// x = M_U (M_L y) of Sec. 3.1 and the operator products A z of the Krylov
// solver.  Bandwidth-bound (about 0.17 flop per byte in FP64): the design
// goals are streaming the column/value arrays with full-width coalesced
// loads and keeping the gathered vector entries in the XCD's L2.
//
//  * LPR lanes of a wavefront share a row (LPR in 1..64); each lane strides
//    the row by LPR, products accumulate in registers, the LPR partial sums
//    are combined with cross-lane shuffles.
//  * Storage types: FP64 values with FP64 accumulation, or binary32 /
//    bfloat16 values with binary32 accumulation (the input vector is
//    rounded to binary32 on load).
//  * XCD-aware block order: MI355X dispatches consecutive workgroups
//    round-robin over its 8 XCDs, each with a private L2.  Blocks are
//    renumbered so every XCD walks one contiguous slab of rows; the
//    gathered vector window of a banded matrix then stays in one L2.
//  * Blocks of right-hand sides (row-major n x k, leading dimension ld):
//    each row group accumulates KT columns at once, so matrix entries are
//    read once per KT columns.
#include <hip/hip_runtime.h>

#include "sait_internal.h"
#include "solver.h"

namespace sait {

namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

__device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned nb) {
    const unsigned per = nb / kXcds, rem = nb % kXcds;
    const unsigned x = bid % kXcds, k = bid / kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

struct Bf16 {
    unsigned short bits;
};

template <class A, class V> __device__ __forceinline__ A to_acc(V v);
template <> __device__ __forceinline__ double to_acc<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float to_acc<float, double>(double v) { return __double2float_rn(v); }
template <> __device__ __forceinline__ float to_acc<float, float>(float v) { return v; }
template <> __device__ __forceinline__ float to_acc<float, Bf16>(Bf16 v) { return __uint_as_float(((unsigned)v.bits) << 16); }

template <class V> __device__ __forceinline__ V ld_stream(const V *p) { return __builtin_nontemporal_load(p); }
template <> __device__ __forceinline__ Bf16 ld_stream<Bf16>(const Bf16 *p) {
    Bf16 r;
    r.bits = __builtin_nontemporal_load(&p->bits);
    return r;
}

template <class A, int W> __device__ __forceinline__ A group_sum(A x) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, W);
    return x;
}

// y[row] = sum_p v[p] * x[ci[p]]   (or b[row] - that, RESID)
template <int LPR, class VT, class XT, class AT, class YT, bool RESID>
__global__ __launch_bounds__(kBlock) void k_spmv(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const VT *__restrict__ v, const XT *__restrict__ x,
                                                 YT *__restrict__ y, const double *__restrict__ b) {
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int row = (int)(((int64_t)blk * kBlock + threadIdx.x) / LPR);
    const int lane = threadIdx.x & (LPR - 1);
    if (row >= n) return;
    const int e = rp[row + 1];
    AT acc = 0;
    for (int p = rp[row] + lane; p < e; p += LPR) {
        const int c = ld_stream(ci + p);
        acc = fma(to_acc<AT>(ld_stream(v + p)), to_acc<AT>(x[c]), acc);
    }
    acc = group_sum<AT, LPR>(acc);
    if (lane == 0) {
        if constexpr (RESID) y[row] = (YT)(b[row] - (double)acc);
        else y[row] = (YT)acc;
    }
}

// Block of KT right-hand sides (columns k0 .. k0+KT-1 selected by blockIdx.y).
template <int LPR, int KT, class VT, class XT, class AT, class YT>
__global__ __launch_bounds__(kBlock) void k_spmm(int n, int nrhs, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const VT *__restrict__ v, const XT *__restrict__ x, int64_t ldx,
                                                 YT *__restrict__ y, int64_t ldy) {
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int row = (int)(((int64_t)blk * kBlock + threadIdx.x) / LPR);
    const int lane = threadIdx.x & (LPR - 1);
    const int k0 = blockIdx.y * KT;
    if (row >= n) return;
    const int e = rp[row + 1];
    AT acc[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) acc[k] = 0;
    const bool full = k0 + KT <= nrhs;
    for (int p = rp[row] + lane; p < e; p += LPR) {
        const int c = ld_stream(ci + p);
        const AT a = to_acc<AT>(ld_stream(v + p));
        const XT *xr = x + (int64_t)c * ldx + k0;
        if (full) {
#pragma unroll
            for (int k = 0; k < KT; ++k) acc[k] = fma(a, to_acc<AT>(xr[k]), acc[k]);
        } else {
#pragma unroll
            for (int k = 0; k < KT; ++k)
                if (k0 + k < nrhs) acc[k] = fma(a, to_acc<AT>(xr[k]), acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < KT; ++k) acc[k] = group_sum<AT, LPR>(acc[k]);
    if (lane == 0) {
        YT *yr = y + (int64_t)row * ldy + k0;
#pragma unroll
        for (int k = 0; k < KT; ++k)
            if (k0 + k < nrhs) yr[k] = (YT)acc[k];
    }
}

template <int LPR, class VT, class XT, class AT, class YT>
void launch_one(const DevCsr &M, const void *x, void *y, hipStream_t s, const double *b) {
    const int n = (int)M.n;
    const unsigned rows_per_block = kBlock / LPR;
    const unsigned nb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
    if (nb == 0) return;
    const VT *vals = static_cast<const VT *>(M.stored());
    if (b)
        hipLaunchKernelGGL((k_spmv<LPR, VT, XT, AT, YT, true>), dim3(nb), dim3(kBlock), 0, s, n, M.rp.as<int>(),
                           M.ci.as<int>(), vals, static_cast<const XT *>(x), static_cast<YT *>(y), b);
    else
        hipLaunchKernelGGL((k_spmv<LPR, VT, XT, AT, YT, false>), dim3(nb), dim3(kBlock), 0, s, n, M.rp.as<int>(),
                           M.ci.as<int>(), vals, static_cast<const XT *>(x), static_cast<YT *>(y), nullptr);
    SAIT_LAUNCH_CHECK();
}

template <int LPR, int KT, class VT, class XT, class AT, class YT>
void launch_block(const DevCsr &M, const void *x, int64_t ldx, void *y, int64_t ldy, int nrhs, hipStream_t s) {
    const int n = (int)M.n;
    const unsigned rows_per_block = kBlock / LPR;
    const unsigned nb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
    if (nb == 0) return;
    const VT *vals = static_cast<const VT *>(M.stored());
    hipLaunchKernelGGL((k_spmm<LPR, KT, VT, XT, AT, YT>), dim3(nb, (nrhs + KT - 1) / KT), dim3(kBlock), 0, s, n, nrhs,
                       M.rp.as<int>(), M.ci.as<int>(), vals, static_cast<const XT *>(x), ldx, static_cast<YT *>(y), ldy);
    SAIT_LAUNCH_CHECK();
}

template <class VT, class XT, class AT, class YT>
void dispatch_lanes(const DevCsr &M, const void *x, void *y, int nrhs, int64_t ldx, int64_t ldy, int lanes,
                    hipStream_t s, const double *b) {
    if (nrhs == 1 && ldx == 1 && ldy == 1) {
        switch (lanes) {
        case 1: return launch_one<1, VT, XT, AT, YT>(M, x, y, s, b);
        case 2: return launch_one<2, VT, XT, AT, YT>(M, x, y, s, b);
        case 4: return launch_one<4, VT, XT, AT, YT>(M, x, y, s, b);
        case 8: return launch_one<8, VT, XT, AT, YT>(M, x, y, s, b);
        case 16: return launch_one<16, VT, XT, AT, YT>(M, x, y, s, b);
        case 32: return launch_one<32, VT, XT, AT, YT>(M, x, y, s, b);
        case 64: return launch_one<64, VT, XT, AT, YT>(M, x, y, s, b);
        default: fail(SAIT_E_INVALID, "lanes per row must be a power of two in 1..64");
        }
    }
    if (b) fail(SAIT_E_INVALID, "residual form is single right-hand side only");
    // blocks of right-hand sides: 8 columns per pass (fewer when nrhs is small)
    switch (lanes) {
    case 1: return nrhs >= 8 ? launch_block<1, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                             : launch_block<1, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 2: return nrhs >= 8 ? launch_block<2, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                             : launch_block<2, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 4: return nrhs >= 8 ? launch_block<4, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                             : launch_block<4, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 8: return nrhs >= 8 ? launch_block<8, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                             : launch_block<8, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 16: return nrhs >= 8 ? launch_block<16, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                              : launch_block<16, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 32: return nrhs >= 8 ? launch_block<32, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                              : launch_block<32, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 64: return nrhs >= 8 ? launch_block<64, 8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s)
                              : launch_block<64, 4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    default: fail(SAIT_E_INVALID, "lanes per row must be a power of two in 1..64");
    }
}

// Adjoint gradient on the pattern of A: g[p] = -(lambda_i * x_j), 16 lanes per row.
__global__ __launch_bounds__(kBlock) void k_grad(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                 const double *__restrict__ lam, const double *__restrict__ x,
                                                 double *__restrict__ g) {
    const int row = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 4);
    const int lane = threadIdx.x & 15;
    if (row >= n) return;
    const double li = lam[row];
    for (int p = rp[row] + lane; p < rp[row + 1]; p += 16) g[p] = -(li * x[ci[p]]);
}

}  // namespace

void grad_values(const DevCsr &A, const double *lambda, const double *x, double *grad, hipStream_t s) {
    const int n = (int)A.n;
    if (n == 0) return;
    const unsigned nb = (unsigned)(((int64_t)n * 16 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_grad, dim3(nb), dim3(kBlock), 0, s, n, A.rp.as<int>(), A.ci.as<int>(), lambda, x, grad);
    SAIT_LAUNCH_CHECK();
}

int default_lanes(const DevCsr &M) {
    const double avg = M.n ? (double)M.nnz / (double)M.n : 1.0;
    int l = 1;
    while (l < 64 && l < avg) l <<= 1;
    return l;
}

void spmv(const DevCsr &M, const void *x, XKind xk, void *y, YKind yk, int nrhs, int64_t ldx, int64_t ldy, int lanes,
          hipStream_t s, const double *resid_b) {
    if (M.n == 0 || nrhs == 0) return;
    if (M.precision == SAIT_F64) {
        if (xk != XKind::F64 || yk != YKind::F64) fail(SAIT_E_INVALID, "FP64 factor needs FP64 vectors");
        return dispatch_lanes<double, double, double, double>(M, x, y, nrhs, ldx, ldy, lanes, s, resid_b);
    }
    if (resid_b) fail(SAIT_E_INVALID, "residual form needs FP64 values");
    if (M.precision == SAIT_F32) {
        if (xk == XKind::F64 && yk == YKind::F32)
            return dispatch_lanes<float, double, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F64)
            return dispatch_lanes<float, float, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F32)
            return dispatch_lanes<float, float, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F64 && yk == YKind::F64)
            return dispatch_lanes<float, double, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
    }
    if (M.precision == SAIT_BF16) {
        if (xk == XKind::F64 && yk == YKind::F32)
            return dispatch_lanes<Bf16, double, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F64)
            return dispatch_lanes<Bf16, float, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F32)
            return dispatch_lanes<Bf16, float, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F64 && yk == YKind::F64)
            return dispatch_lanes<Bf16, double, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
    }
    fail(SAIT_E_INVALID, "unsupported precision / vector type combination");
}

}  // namespace sait
