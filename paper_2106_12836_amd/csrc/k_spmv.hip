// Sparse matrix-vector and matrix-block products: the SAIT apply
// x = M_U (M_L y) of Sec. 3.1 and the operator products A z of the Krylov
// solver.  Bandwidth-bound (about 0.17 flop per byte in FP64): the design
// goals are streaming the index/value arrays with wide coalesced loads,
// keeping enough bytes in flight per CU, and keeping the gathered vector
// entries in the XCD's L2.
//
// Kernels (selected per matrix by the autotuner, see sait_autotune):
//  * Sliced ELL (default for stencil-like factors): a copy of the CSR
//    matrix in slices of 64 rows = one wavefront; a lane owns a row and walks
//    it in column order, 4 entries per 16-byte index load, two groups of 4
//    per pipeline stage, with the next stage's index/value loads issued
//    before the current stage's gathers are consumed.  Entry k of 64
//    consecutive rows is contiguous, so for banded factors the x gathers of a
//    wavefront are nearly contiguous too.
//  * LDS-staged CSR (for irregular row lengths, where slicing would pad): a
//    workgroup streams a row-aligned chunk of up to 2040 / 4088 entries with
//    16-byte loads, writes the rounded products to LDS and each thread sums
//    one row in column order.
//  * Wavefront CSR: LPR lanes per row with a shuffle reduction; also the
//    kernel for blocks of right-hand sides (KT columns per pass).
// The sliced-ELL and LDS-staged kernels round every product and every sum
// separately and add in column order: their result is exactly the
// row-by-row sum sum_p v_p x_{c_p} evaluated left to right.
//
// XCD-aware block order: MI355X dispatches consecutive workgroups
// round-robin over its 8 XCDs, each with a private L2.  Workgroups are
// renumbered so that every XCD walks one contiguous slab of rows; the
// gathered window of a banded matrix then stays in one L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

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

// Separately rounded product and sum: the multiplies created here carry no
// contraction permission, so they are never fused into an FMA with the add.
__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ float mul_rn(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double add_rn(double a, double b) {
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ float add_rn(float a, float b) {
#pragma clang fp contract(off)
    return a + b;
}

// The four entries of one lane in one 4-entry group of a slice (grp = the
// group's first element): 16-byte (8-byte for bfloat16) aligned vector
// loads, streamed past the caches.  FP64 groups are stored as two planes --
// entries 0-1 of the 64 lanes, then entries 2-3 -- so each of the two loads
// of a wavefront reads 1 KiB contiguously; binary32 and bfloat16 groups hold
// a lane's four entries together.
typedef int i4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned short u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_idx4(const int *p, int (&o)[4]) {
    const i4v a = __builtin_nontemporal_load(reinterpret_cast<const i4v *>(p));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}
// Four consecutive CSR entries starting at a multiple of 4.
__device__ __forceinline__ void load_csr4(const double *p, double (&o)[4]) {
    const d2v a = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    const d2v b = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p + 2));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
__device__ __forceinline__ void load_csr4(const float *p, float (&o)[4]) {
    const f4v a = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}
__device__ __forceinline__ void load_csr4(const Bf16 *p, float (&o)[4]) {
    const u4v a = __builtin_nontemporal_load(reinterpret_cast<const u4v *>(p));
    o[0] = __uint_as_float(((unsigned)a.x) << 16);
    o[1] = __uint_as_float(((unsigned)a.y) << 16);
    o[2] = __uint_as_float(((unsigned)a.z) << 16);
    o[3] = __uint_as_float(((unsigned)a.w) << 16);
}

__device__ __forceinline__ void load_quad(const double *grp, int l, double (&o)[4]) {
    const d2v a = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(grp + 2 * l));
    const d2v b = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(grp + 128 + 2 * l));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}
__device__ __forceinline__ void load_quad(const float *grp, int l, float (&o)[4]) {
    const f4v a = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(grp + 4 * l));
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}
__device__ __forceinline__ void load_quad(const Bf16 *grp, int l, float (&o)[4]) {
    const u4v a = __builtin_nontemporal_load(reinterpret_cast<const u4v *>(grp + 4 * l));
    o[0] = __uint_as_float(((unsigned)a.x) << 16);
    o[1] = __uint_as_float(((unsigned)a.y) << 16);
    o[2] = __uint_as_float(((unsigned)a.z) << 16);
    o[3] = __uint_as_float(((unsigned)a.w) << 16);
}

// The row result goes out with a streaming (nontemporal) store: it is read
// once, by the next kernel, and keeping it out of the caches leaves them to
// the gathered vector (measured on the C3 factors: FP64 apply 190 against
// 195 us, FP32 140 against 144 us, BF16 122 against 125 us).
template <bool RESID, class YT, class AT>
__device__ __forceinline__ void store_row(YT *y, const double *b, int row, AT acc) {
    if constexpr (RESID) __builtin_nontemporal_store((YT)(b[row] - (double)acc), y + row);
    else __builtin_nontemporal_store((YT)acc, y + row);
}

// ---------------------------------------------------------------------------
// Sliced ELL, one row per lane (layout in DevCsr: entry k of row 64 s + l at
// sell_ptr[s] + (k / 4) * 256 + 4 l + k % 4).
// ---------------------------------------------------------------------------
template <int U, class VT, class XT, class AT, class YT, bool RESID>
__global__ __launch_bounds__(kBlock) void k_spmv_sell(int n, int nslices, const int64_t *__restrict__ sptr,
                                                      const int *__restrict__ rp, const int *__restrict__ sci,
                                                      const VT *__restrict__ sv, const XT *__restrict__ x,
                                                      YT *__restrict__ y, const double *__restrict__ b) {
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = (int)blk * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (s >= nslices) return;
    const int row = s * 64 + l;
    const int len = row < n ? rp[row + 1] - rp[row] : 0;
    const int64_t base = sptr[s];
    const int ngroups = (int)((sptr[s + 1] - base) >> 8);
    AT acc = 0;
    int cols[2][U][4];
    AT vals[2][U][4];
    auto load_set = [&](int g0, int slot) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (g0 + u < ngroups) {
                const int64_t grp = base + (int64_t)(g0 + u) * 256;
                load_idx4(sci + grp + 4 * l, cols[slot][u]);
                load_quad(sv + grp, l, vals[slot][u]);
            }
        }
    };
    auto use_set = [&](int g0, int slot) {
        AT xs[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                xs[u][j] = ((g0 + u) * 4 + j < len) ? to_acc<AT>(x[cols[slot][u][j]]) : AT(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((g0 + u) * 4 + j < len) acc = add_rn(acc, mul_rn(vals[slot][u][j], xs[u][j]));
    };
    // two stages of U groups: the loads of stage g0+U are issued before the
    // gathers of stage g0 are consumed
    if (ngroups > 0) load_set(0, 0);
    for (int g0 = 0; g0 < ngroups; g0 += 2 * U) {
        if (g0 + U < ngroups) load_set(g0 + U, 1);
        use_set(g0, 0);
        if (g0 + U >= ngroups) break;
        if (g0 + 2 * U < ngroups) load_set(g0 + 2 * U, 0);
        use_set(g0 + U, 1);
    }
    if (row < n) store_row<RESID>(y, b, row, acc);
}

// Sliced ELL, one row per lane, K right-hand sides (x: n x ldx, y: n x ldy,
// row-major): each stored entry multiplies the K contiguous x values of its
// column.  Per right-hand side the products are added in column order with
// separate roundings, as in k_spmv_sell, so every column of y equals the
// one-vector product bit for bit.  Stages of U groups: the gathers of a
// stage are issued together, and the next stage's indices and values are
// loaded before they are consumed.
template <int K, int U, class VT, class XT, class AT, class YT>
__global__ __launch_bounds__(kBlock) void k_spmm_sell(int n, int nslices, const int64_t *__restrict__ sptr,
                                                      const int *__restrict__ rp, const int *__restrict__ sci,
                                                      const VT *__restrict__ sv, const XT *__restrict__ x,
                                                      int64_t ldx, YT *__restrict__ y, int64_t ldy) {
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = (int)blk * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (s >= nslices) return;
    const int row = s * 64 + l;
    const int len = row < n ? rp[row + 1] - rp[row] : 0;
    const int64_t base = sptr[s];
    const int ngroups = (int)((sptr[s + 1] - base) >> 8);
    AT acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = AT(0);
    int cols[2][U][4];
    AT vals[2][U][4];
    auto load = [&](int g0, int slot) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (g0 + u < ngroups) {
                const int64_t grp = base + (int64_t)(g0 + u) * 256;
                load_idx4(sci + grp + 4 * l, cols[slot][u]);
                load_quad(sv + grp, l, vals[slot][u]);
            }
    };
    auto use = [&](int g0, int slot) {
        AT xs[U][4][K];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool on = (g0 + u) * 4 + j < len;
                const XT *xr = x + (int64_t)(on ? cols[slot][u][j] : 0) * ldx;
#pragma unroll
                for (int k = 0; k < K; ++k) xs[u][j][k] = on ? to_acc<AT>(xr[k]) : AT(0);
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((g0 + u) * 4 + j < len)
#pragma unroll
                    for (int k = 0; k < K; ++k) acc[k] = add_rn(acc[k], mul_rn(vals[slot][u][j], xs[u][j][k]));
    };
    if (ngroups > 0) load(0, 0);
    for (int g0 = 0, slot = 0; g0 < ngroups; g0 += U, slot ^= 1) {
        if (g0 + U < ngroups) load(g0 + U, slot ^ 1);
        use(g0, slot);
    }
    if (row < n)
#pragma unroll
        for (int k = 0; k < K; ++k) y[(int64_t)row * ldy + k] = (YT)acc[k];
}

// Slice widths: 64 * (longest row of the slice rounded up to 4).
__global__ void k_sell_width(int n, int nslices, const int *__restrict__ rp, int64_t *__restrict__ cnt) {
    const int s = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int l = threadIdx.x & 63;
    if (s >= nslices) return;
    const int row = s * 64 + l;
    int len = row < n ? rp[row + 1] - rp[row] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
    if (l == 0) cnt[s] = (int64_t)64 * ((len + 3) & ~3);
}

// Position of entry k of lane l's row in the value array of a group that
// starts at grp (see load_quad).
template <class VT> __device__ __forceinline__ int64_t sell_value_index(int64_t grp, int l, int k) {
    if constexpr (sizeof(VT) == 8) return grp + ((k >> 1) & 1) * 128 + 2 * l + (k & 1);
    else return grp + 4 * l + (k & 3);
}

template <class VT>
__global__ void k_sell_fill(int n, const int *__restrict__ rp, const int *__restrict__ ci, const VT *__restrict__ v,
                            const int64_t *__restrict__ sptr, int *__restrict__ sci, VT *__restrict__ sv) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = row >> 6;
    if (s * 64 >= n) return;
    const int l = (int)(row & 63);
    const int64_t base = sptr[s];
    const int width = (int)((sptr[s + 1] - base) >> 6);
    const int b0 = row < n ? rp[row] : 0;
    const int len = row < n ? rp[row + 1] - b0 : 0;
    for (int k = 0; k < width; ++k) {
        const int64_t grp = base + (int64_t)(k >> 2) * 256;
        const int64_t off = grp + 4 * l + (k & 3);
        const int64_t voff = sell_value_index<VT>(grp, l, k);
        if (k < len) {
            sci[off] = ci[b0 + k];
            sv[voff] = v[b0 + k];
        } else {
            sci[off] = 0;
            sv[voff] = VT{};
        }
    }
}

// ---------------------------------------------------------------------------
// LDS-staged CSR.  Row block [brow[blk], brow[blk+1]): at most 256 rows and
// one chunk of CAP entries, or a single longer row processed chunk by chunk.
// ---------------------------------------------------------------------------
// The aligned quads covering any CAP consecutive entries number at most
// (CAP + 6) / 4 <= Q * kBlock.
template <int Q> constexpr int stream_cap() { return Q * kBlock * 4 - 8; }
constexpr int kStreamRows = kBlock;

template <int Q, class VT, class XT, class AT, class YT, bool RESID>
__global__ __launch_bounds__(kBlock) void k_spmv_stream(const int *__restrict__ brow, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, const VT *__restrict__ v,
                                                        const XT *__restrict__ x, YT *__restrict__ y,
                                                        const double *__restrict__ b) {
    constexpr int CAP = stream_cap<Q>();
    __shared__ AT prod[CAP];
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int r0 = brow[blk], r1 = brow[blk + 1];
    const int e0 = rp[r0], e1 = rp[r1];
    const int row = r0 + t;
    const bool has_row = row < r1;
    int rs = 0, re = 0;
    if (has_row) {
        rs = rp[row];
        re = rp[row + 1];
    }
    AT acc = 0;
    for (int c0 = e0; c0 < e1; c0 += CAP) {
        const int cnt = min(CAP, e1 - c0);
        const int c1 = c0 + cnt;
        const int a0 = c0 & ~3;
        int cols[Q][4];
        AT vals[Q][4];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int base = a0 + 4 * (k * kBlock + t);
            if (base < c1) {
                load_idx4(ci + base, cols[k]);
                load_csr4(v + base, vals[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int base = a0 + 4 * (k * kBlock + t);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = base + j;
                if (e >= c0 && e < c1) prod[e - c0] = mul_rn(vals[k][j], to_acc<AT>(x[cols[k][j]]));
            }
        }
        __syncthreads();
        if (has_row) {
            const int lo = max(rs, c0), hi = min(re, c1);
            for (int q = lo; q < hi; ++q) acc = add_rn(acc, prod[q - c0]);
        }
        __syncthreads();
    }
    if (has_row) store_row<RESID>(y, b, row, acc);
}

// ---------------------------------------------------------------------------
// Wavefront CSR: LPR lanes per row, shuffle reduction (FMA accumulation).
// ---------------------------------------------------------------------------
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
    if (lane == 0) store_row<RESID>(y, b, row, acc);
}

// Block of KT right-hand sides (columns k0 .. k0+KT-1 selected by blockIdx.y).
template <int K, class VT, class XT, class AT, class YT>
void launch_spmm_sell(const DevCsr &M, const void *x, int64_t ldx, void *y, int64_t ldy, hipStream_t s) {
    if (M.nslices <= 0 || M.sell_ptr.empty()) fail(SAIT_E_INVALID, "sliced-ELL SpMM needs the sliced copy");
    constexpr int per_block = kBlock / 64;
    // one group per stage: with two (8 K gathers in flight) the K = 4 FP64
    // form needs 132 VGPRs and ran 95 us against 84 us on a 20-entry-per-row
    // factor at n = 10^6 (lower occupancy)
    constexpr int U = 1;
    const dim3 grid((unsigned)((M.nslices + per_block - 1) / per_block));
    hipLaunchKernelGGL((k_spmm_sell<K, U, VT, XT, AT, YT>), grid, dim3(kBlock), 0, s, (int)M.n, (int)M.nslices,
                       M.sell_ptr.as<int64_t>(), M.rp.as<int>(), M.sell_ci.as<int>(), M.sell_v.as<VT>(),
                       static_cast<const XT *>(x), ldx, static_cast<YT *>(y), ldy);
    SAIT_LAUNCH_CHECK();
}

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

// Plain streaming copy, 16 bytes per lane per step (bandwidth reference).
__global__ __launch_bounds__(kBlock) void k_copy16(int64_t n16, const i4v *__restrict__ src, i4v *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int LPR, class VT, class XT, class AT, class YT>
void launch_one(const DevCsr &M, const void *x, void *y, hipStream_t s, const double *b) {
    const int n = (int)M.n;
    const unsigned rows_per_block = kBlock / LPR;
    const unsigned nb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
    const VT *vals = static_cast<const VT *>(M.stored());
    if (b)
        hipLaunchKernelGGL((k_spmv<LPR, VT, XT, AT, YT, true>), dim3(nb), dim3(kBlock), 0, s, n, M.rp.as<int>(),
                           M.ci.as<int>(), vals, static_cast<const XT *>(x), static_cast<YT *>(y), b);
    else
        hipLaunchKernelGGL((k_spmv<LPR, VT, XT, AT, YT, false>), dim3(nb), dim3(kBlock), 0, s, n, M.rp.as<int>(),
                           M.ci.as<int>(), vals, static_cast<const XT *>(x), static_cast<YT *>(y), nullptr);
    SAIT_LAUNCH_CHECK();
}

template <int Q, class VT, class XT, class AT, class YT>
void launch_stream(const DevCsr &M, int slot, const void *x, void *y, hipStream_t s, const double *b) {
    if (M.nblk[slot] <= 0 || M.brow[slot].empty()) fail(SAIT_E_INVALID, "LDS-staged SpMV needs prepared row blocks");
    const VT *vals = static_cast<const VT *>(M.stored());
    const dim3 grid((unsigned)M.nblk[slot]);
    if (b)
        hipLaunchKernelGGL((k_spmv_stream<Q, VT, XT, AT, YT, true>), grid, dim3(kBlock), 0, s, M.brow[slot].as<int>(),
                           M.rp.as<int>(), M.ci.as<int>(), vals, static_cast<const XT *>(x), static_cast<YT *>(y), b);
    else
        hipLaunchKernelGGL((k_spmv_stream<Q, VT, XT, AT, YT, false>), grid, dim3(kBlock), 0, s, M.brow[slot].as<int>(),
                           M.rp.as<int>(), M.ci.as<int>(), vals, static_cast<const XT *>(x), static_cast<YT *>(y),
                           nullptr);
    SAIT_LAUNCH_CHECK();
}

template <int U, class VT, class XT, class AT, class YT>
void launch_sell(const DevCsr &M, const void *x, void *y, hipStream_t s, const double *b) {
    if (M.nslices <= 0 || M.sell_ptr.empty()) fail(SAIT_E_INVALID, "sliced-ELL SpMV needs the sliced copy");
    constexpr int per_block = kBlock / 64;
    const dim3 grid((unsigned)((M.nslices + per_block - 1) / per_block));
    auto *sv = M.sell_v.as<VT>();
    if (b)
        hipLaunchKernelGGL((k_spmv_sell<U, VT, XT, AT, YT, true>), grid, dim3(kBlock), 0, s, (int)M.n,
                           (int)M.nslices, M.sell_ptr.as<int64_t>(), M.rp.as<int>(), M.sell_ci.as<int>(), sv,
                           static_cast<const XT *>(x), static_cast<YT *>(y), b);
    else
        hipLaunchKernelGGL((k_spmv_sell<U, VT, XT, AT, YT, false>), grid, dim3(kBlock), 0, s, (int)M.n,
                           (int)M.nslices, M.sell_ptr.as<int64_t>(), M.rp.as<int>(), M.sell_ci.as<int>(), sv,
                           static_cast<const XT *>(x), static_cast<YT *>(y), nullptr);
    SAIT_LAUNCH_CHECK();
}

template <int LPR, int KT, class VT, class XT, class AT, class YT>
void launch_block(const DevCsr &M, const void *x, int64_t ldx, void *y, int64_t ldy, int nrhs, hipStream_t s) {
    const int n = (int)M.n;
    const unsigned rows_per_block = kBlock / LPR;
    const unsigned nb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
    const VT *vals = static_cast<const VT *>(M.stored());
    hipLaunchKernelGGL((k_spmm<LPR, KT, VT, XT, AT, YT>), dim3(nb, (nrhs + KT - 1) / KT), dim3(kBlock), 0, s, n, nrhs,
                       M.rp.as<int>(), M.ci.as<int>(), vals, static_cast<const XT *>(x), ldx, static_cast<YT *>(y), ldy);
    SAIT_LAUNCH_CHECK();
}

template <int KT, class VT, class XT, class AT, class YT>
void dispatch_block(const DevCsr &M, const void *x, int64_t ldx, void *y, int64_t ldy, int nrhs, int lanes,
                    hipStream_t s) {
    switch (lanes) {
    case 1: return launch_block<1, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 2: return launch_block<2, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 4: return launch_block<4, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 8: return launch_block<8, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 16: return launch_block<16, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 32: return launch_block<32, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    case 64: return launch_block<64, KT, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, s);
    default: fail(SAIT_E_INVALID, "lanes per row must be a power of two in 1..64");
    }
}

template <class VT, class XT, class AT, class YT>
void dispatch(const DevCsr &M, const void *x, void *y, int nrhs, int64_t ldx, int64_t ldy, int shape, hipStream_t s,
              const double *b) {
    if (nrhs == 1 && ldx == 1 && ldy == 1) {
        switch (shape) {
        case kSell: return launch_sell<2, VT, XT, AT, YT>(M, x, y, s, b);
        case kSell1: return launch_sell<1, VT, XT, AT, YT>(M, x, y, s, b);
        case kStream8: return launch_stream<2, VT, XT, AT, YT>(M, 0, x, y, s, b);
        case kStream: return launch_stream<4, VT, XT, AT, YT>(M, 1, x, y, s, b);
        case 1: return launch_one<1, VT, XT, AT, YT>(M, x, y, s, b);
        case 2: return launch_one<2, VT, XT, AT, YT>(M, x, y, s, b);
        case 4: return launch_one<4, VT, XT, AT, YT>(M, x, y, s, b);
        case 8: return launch_one<8, VT, XT, AT, YT>(M, x, y, s, b);
        case 16: return launch_one<16, VT, XT, AT, YT>(M, x, y, s, b);
        case 32: return launch_one<32, VT, XT, AT, YT>(M, x, y, s, b);
        case 64: return launch_one<64, VT, XT, AT, YT>(M, x, y, s, b);
        default: fail(SAIT_E_INVALID, "unknown apply shape");
        }
    }
    if (b) fail(SAIT_E_INVALID, "residual form is single right-hand side only");
    if (shape < 0 && M.nslices > 0) {
        // sliced-ELL blocks of 2..5 or 8 right-hand sides (for blocks the
        // gathers outweigh the slice padding, so also where the one-vector
        // product uses the LDS-staged kernel)
        switch (nrhs) {
        case 2: return launch_spmm_sell<2, VT, XT, AT, YT>(M, x, ldx, y, ldy, s);
        case 3: return launch_spmm_sell<3, VT, XT, AT, YT>(M, x, ldx, y, ldy, s);
        case 4: return launch_spmm_sell<4, VT, XT, AT, YT>(M, x, ldx, y, ldy, s);
        case 5: return launch_spmm_sell<5, VT, XT, AT, YT>(M, x, ldx, y, ldy, s);
        case 8: return launch_spmm_sell<8, VT, XT, AT, YT>(M, x, ldx, y, ldy, s);
        default: break;
        }
    }
    if (shape < 0) shape = 8;  // other blocks of right-hand sides use the wavefront kernel
    if (nrhs >= 8) dispatch_block<8, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, shape, s);
    else dispatch_block<4, VT, XT, AT, YT>(M, x, ldx, y, ldy, nrhs, shape, s);
}

// One Jacobi sweep for a triangular system T y = r on the sliced-ELL copy of
// N, the off-diagonal part of T, and its diagonal d:
//   ynew_i = (r_i - sum_j N_ij yold_j) / d_i,
// the products subtracted from r_i one by one in column order with separate
// roundings (one row per lane, two groups of 4 entries per stage).
__global__ __launch_bounds__(kBlock) void k_jacobi_sell(int n, int nslices, const int64_t *__restrict__ sptr,
                                                        const int *__restrict__ rp, const int *__restrict__ sci,
                                                        const double *__restrict__ sv, const double *__restrict__ d,
                                                        const double *__restrict__ r, const double *__restrict__ yold,
                                                        double *__restrict__ ynew) {
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int s = (int)blk * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (s >= nslices) return;
    const int row = s * 64 + l;
    const int len = row < n ? rp[row + 1] - rp[row] : 0;
    const int64_t base = sptr[s];
    const int ngroups = (int)((sptr[s + 1] - base) >> 8);
    double acc = row < n ? r[row] : 0.0;
    int cols[2][4];
    double vals[2][4];
    if (ngroups > 0) {
        load_idx4(sci + base + 4 * l, cols[0]);
        load_quad(sv + base, l, vals[0]);
    }
    for (int g = 0; g < ngroups; ++g) {
        const int cur = g & 1;
        if (g + 1 < ngroups) {
            const int64_t grp = base + (int64_t)(g + 1) * 256;
            load_idx4(sci + grp + 4 * l, cols[cur ^ 1]);
            load_quad(sv + grp, l, vals[cur ^ 1]);
        }
        double xs[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xs[j] = (g * 4 + j < len) ? yold[cols[cur][j]] : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (g * 4 + j < len) {
#pragma clang fp contract(off)
                acc = acc - mul_rn(vals[cur][j], xs[j]);
            }
    }
    if (row < n) ynew[row] = acc / d[row];
}

}  // namespace

bool valid_shape(int shape) {
    return shape == kSell || shape == kSell1 || shape == kStream8 || shape == kStream ||
           (shape >= 1 && shape <= 64 && (shape & (shape - 1)) == 0);
}

void copy_bytes(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return;
    const int64_t blocks = std::min<int64_t>((n16 + kBlock - 1) / kBlock, 256 * 32);
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kBlock), 0, s, n16, static_cast<const i4v *>(src),
                       static_cast<i4v *>(dst));
    SAIT_LAUNCH_CHECK();
}

void grad_values(const DevCsr &A, const double *lambda, const double *x, double *grad, hipStream_t s) {
    const int n = (int)A.n;
    if (n == 0) return;
    const unsigned nb = (unsigned)(((int64_t)n * 16 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_grad, dim3(nb), dim3(kBlock), 0, s, n, A.rp.as<int>(), A.ci.as<int>(), lambda, x, grad);
    SAIT_LAUNCH_CHECK();
}

void prepare_stream(Allocator *a, DevCsr &M, hipStream_t s) {
    const int64_t n = M.n;
    std::vector<int> rp(n + 1);
    SAIT_HIP(hipMemcpyAsync(rp.data(), M.rp.as<void>(), (n + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    const int caps[2] = {stream_cap<2>(), stream_cap<4>()};
    for (int slot = 0; slot < 2; ++slot) {
        std::vector<int> brow;
        brow.reserve(n / 64 + 2);
        brow.push_back(0);
        int64_t start = 0, cnt = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t len = rp[i + 1] - rp[i];
            if (i > start && (i - start == kStreamRows || cnt + len > caps[slot])) {
                brow.push_back((int)i);
                start = i;
                cnt = 0;
            }
            cnt += len;
        }
        if (n > 0) brow.push_back((int)n);
        M.nblk[slot] = (int64_t)brow.size() - 1;
        M.brow[slot].alloc(a, brow.size() * sizeof(int));
        SAIT_HIP(hipMemcpyAsync(M.brow[slot].as<void>(), brow.data(), brow.size() * sizeof(int),
                                hipMemcpyHostToDevice, s));
        SAIT_HIP(hipStreamSynchronize(s));
    }
}

void prepare_sell(Allocator *a, DevCsr &M, hipStream_t s) {
    const int64_t n = M.n;
    M.nslices = (n + 63) / 64;
    if (n == 0) return;
    DevBuf cnt;
    cnt.alloc(a, (size_t)M.nslices * sizeof(int64_t));
    M.sell_ptr.alloc(a, (size_t)(M.nslices + 1) * sizeof(int64_t));
    hipLaunchKernelGGL(k_sell_width, dim3((unsigned)((M.nslices * 64 + 255) / 256)), dim3(256), 0, s, (int)n,
                       (int)M.nslices, M.rp.as<int>(), cnt.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    scan_exclusive_i64(a, cnt.as<int64_t>(), M.sell_ptr.as<int64_t>(), M.nslices, s);
    int64_t total = 0;
    SAIT_HIP(hipMemcpyAsync(&total, M.sell_ptr.as<int64_t>() + M.nslices, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    M.sell_nnz = total;
    M.sell_ci.alloc(a, (size_t)std::max<int64_t>(total, 1) * sizeof(int));
    const unsigned grid = (unsigned)((M.nslices * 64 + 255) / 256);
    if (M.precision == SAIT_F64) {
        M.sell_v.alloc(a, (size_t)std::max<int64_t>(total, 1) * sizeof(double));
        hipLaunchKernelGGL(k_sell_fill<double>, dim3(grid), dim3(256), 0, s, (int)n, M.rp.as<int>(), M.ci.as<int>(),
                           M.v.as<double>(), M.sell_ptr.as<int64_t>(), M.sell_ci.as<int>(), M.sell_v.as<double>());
    } else if (M.precision == SAIT_F32) {
        M.sell_v.alloc(a, (size_t)std::max<int64_t>(total, 1) * sizeof(float));
        hipLaunchKernelGGL(k_sell_fill<float>, dim3(grid), dim3(256), 0, s, (int)n, M.rp.as<int>(), M.ci.as<int>(),
                           M.vs.as<float>(), M.sell_ptr.as<int64_t>(), M.sell_ci.as<int>(), M.sell_v.as<float>());
    } else {
        M.sell_v.alloc(a, (size_t)std::max<int64_t>(total, 1) * sizeof(Bf16));
        hipLaunchKernelGGL(k_sell_fill<Bf16>, dim3(grid), dim3(256), 0, s, (int)n, M.rp.as<int>(), M.ci.as<int>(),
                           M.vs.as<Bf16>(), M.sell_ptr.as<int64_t>(), M.sell_ci.as<int>(), M.sell_v.as<Bf16>());
    }
    SAIT_LAUNCH_CHECK();
    SAIT_HIP(hipStreamSynchronize(s));
}

int default_lanes(const DevCsr &M) {
    // sliced ELL unless slicing pads more than 1/8 of the entries
    if (M.nslices > 0 && M.sell_nnz > 0 && M.sell_nnz <= M.nnz + M.nnz / 8) return kSell;
    if (M.nblk[0] > 0) return kStream8;
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
        return dispatch<double, double, double, double>(M, x, y, nrhs, ldx, ldy, lanes, s, resid_b);
    }
    if (resid_b) fail(SAIT_E_INVALID, "residual form needs FP64 values");
    if (M.precision == SAIT_F32) {
        if (xk == XKind::F64 && yk == YKind::F32)
            return dispatch<float, double, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F64)
            return dispatch<float, float, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F32)
            return dispatch<float, float, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F64 && yk == YKind::F64)
            return dispatch<float, double, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
    }
    if (M.precision == SAIT_BF16) {
        if (xk == XKind::F64 && yk == YKind::F32)
            return dispatch<Bf16, double, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F64)
            return dispatch<Bf16, float, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F32 && yk == YKind::F32)
            return dispatch<Bf16, float, float, float>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
        if (xk == XKind::F64 && yk == YKind::F64)
            return dispatch<Bf16, double, float, double>(M, x, y, nrhs, ldx, ldy, lanes, s, nullptr);
    }
    fail(SAIT_E_INVALID, "unsupported precision / vector type combination");
}


void jacobi_sweep(const DevCsr &N, const double *d, const double *r, const double *yold, double *ynew, hipStream_t s) {
    if (N.n == 0) return;
    if (N.precision != SAIT_F64 || N.nslices <= 0) fail(SAIT_E_INVALID, "jacobi_sweep needs an FP64 sliced-ELL matrix");
    const int grid = (int)((N.nslices + kBlock / 64 - 1) / (kBlock / 64));
    hipLaunchKernelGGL(k_jacobi_sell, dim3(grid), dim3(kBlock), 0, s, (int)N.n, (int)N.nslices,
                       N.sell_ptr.as<int64_t>(), N.rp.as<int>(), N.sell_ci.as<int>(), N.sell_v.as<double>(), d, r,
                       yold, ynew);
    SAIT_LAUNCH_CHECK();
}

}  // namespace sait
