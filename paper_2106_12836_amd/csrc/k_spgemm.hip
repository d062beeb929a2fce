// SAIT construction on the device (Sec. 2-3: Alg. 1-3, Eq. Recursive).
//
// For a triangular T with diagonal D:
//   split:   T~ = I - D^-1 T   (strictly triangular: its diagonal is not
//            stored), dinv_i = fl(1/d_i), T~_ij = -(dinv_i * T_ij)
//   passes:  M <- drop(T~ M + I), m times (Horner / Qin Jiushao form),
//            or M <- drop(M T~ + I) (right-multiplied: used for the upper
//            factor, so that a symmetric A gives M_U = M_L^T D^-1),
//            drop = keep |W_ij| > tau (Alg. 2), or keep pattern S (Alg. 3),
//            optional cap: diagonal + (cap-1) largest |W_ij| per row
//   scale:   M <- M D^-1 (column j times dinv_j), then cast to the storage
//            precision (FP64, binary32 RNE, bfloat16 RNE of the binary32).
//
// One Horner pass is a row-wise SpGEMM W = X Y + I with (X, Y) = (T~, M),
// or (M, T~) for the right-multiplied recursion.  Row i of W gathers the
// candidate products X_il * Y_lj for every l in row i of X (l ascending)
// plus the unit diagonal; candidates are keyed (column j, position) and sorted by a
// bitonic network in LDS, equal columns are then summed in key order --
// i.e. in increasing l, the order of a Gustavson accumulator -- with
// explicitly rounded multiply and add.  The drop rule, the cap and the
// compaction into sorted CSR are fused into the same kernel.  Rows are
// binned by candidate count: a 64-lane workgroup with 64- or 256-entry LDS
// buffers, a 256-lane workgroup with 2048 entries, and a global-memory
// fallback for anything larger.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sait_internal.h"

namespace sait {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;

// Separately rounded product and sum (never contracted into an FMA).
__device__ __forceinline__ double dmul(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double dadd(double a, double b) {
#pragma clang fp contract(off)
    return a + b;
}

// ---------------------------------------------------------------------------
// Jacobi split: dinv and T~ (row i of T~ = row i of T without its diagonal).
// ---------------------------------------------------------------------------
__global__ void k_split(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                        const double *__restrict__ v, int *__restrict__ trp, int *__restrict__ tci,
                        double *__restrict__ tv, double *__restrict__ dinv, int *__restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        trp[n] = rp[n] - n;
        return;
    }
    const int b = rp[i], e = rp[i + 1];
    double d = 0.0;
    int found = 0;
    for (int p = b; p < e; ++p)
        if (ci[p] == i) {
            d = v[p];
            found = 1;
        }
    trp[i] = b - i;
    if (!found || d == 0.0 || !isfinite(d)) {
        // the build stops on err; write nothing else (without a diagonal the
        // row would not fit its slot of T~)
        atomicOr(err, 1);
        dinv[i] = 1.0;
        return;
    }
    const double di = 1.0 / d;
    dinv[i] = di;
    int o = b - i;
    for (int p = b; p < e; ++p) {
        if (ci[p] == i) continue;
        tci[o] = ci[p];
        tv[o] = -dmul(di, v[p]);
        ++o;
    }
}

// Size of row i of X Y + I: its candidate count 1 + sum over l in X_i of
// |Y_l|, but at least |X_i| + 1, the length of the row's segment table (a
// row of Y may be empty: T~ has no entries in the last row of U).
__global__ void k_count(int n, const int *__restrict__ trp, const int *__restrict__ tci,
                        const int *__restrict__ mrp, int64_t *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t c = 1;
    for (int p = trp[i]; p < trp[i + 1]; ++p) {
        const int l = tci[p];
        c += mrp[l + 1] - mrp[l];
    }
    const int64_t seg = (int64_t)(trp[i + 1] - trp[i]) + 1;
    cnt[i] = c > seg ? c : seg;
}

// Tier of a row by candidate count.
constexpr int kTierCap0 = 64, kTierCap1 = 256, kTierCap2 = 2048;
// Slots are claimed per block (LDS counters, then one global atomic per tier
// and block), so the global counters see gridDim.x updates, not n.
__global__ void k_classify(int n, const int64_t *__restrict__ cnt, int *__restrict__ tier_n,
                           int *__restrict__ lists) {
    __shared__ int lcount[4], lbase[4];
    if (threadIdx.x < 4) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int t = 0, slot = 0;
    if (i < n) {
        const int64_t c = cnt[i];
        t = c <= kTierCap0 ? 0 : c <= kTierCap1 ? 1 : c <= kTierCap2 ? 2 : 3;
        slot = atomicAdd(&lcount[t], 1);
    }
    __syncthreads();
    if (threadIdx.x < 4 && lcount[threadIdx.x]) lbase[threadIdx.x] = atomicAdd(&tier_n[threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
    if (i < n) lists[(int64_t)t * n + lbase[t] + slot] = i;
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 (three phases: block totals, scan of totals,
// per-block scan with offset).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ int64_t block_scan_excl(int64_t x, int64_t *sh, int64_t *total) {
    // Hillis-Steele inclusive scan in LDS, converted to exclusive.
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        int64_t y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    const int64_t incl = sh[t];
    if (total) *total = sh[NT - 1];
    __syncthreads();
    return incl - x;
}

__global__ void k_scan_partials(const int64_t *__restrict__ in, int64_t n, int64_t *__restrict__ part) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_scan_excl<kScanBlock>(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void k_scan_top(int64_t *__restrict__ part, int64_t nb) {
    __shared__ int64_t sh[kScanBlock];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t x = i < nb ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_scan_excl<kScanBlock>(x, sh, &tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

__global__ void k_scan_final(const int64_t *__restrict__ in, int64_t n, const int64_t *__restrict__ part,
                             int64_t *__restrict__ out) {
    __shared__ int64_t sh[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock * kScanItems + (int64_t)threadIdx.x * kScanItems;
    int64_t loc[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        loc[k] = i < n ? in[i] : 0;
        s += loc[k];
    }
    int64_t ex = block_scan_excl<kScanBlock>(s, sh, nullptr) + part[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += loc[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        // total lives in part[gridDim.x]
        out[n] = part[gridDim.x];
    }
}

// ---------------------------------------------------------------------------
// One row of W = X Y + I with drop / cap / compaction.
// key/val/kf/seg point at LDS (tiers 0-2) or at global scratch (tier 3),
// sized by the row's bound from k_count.
// ---------------------------------------------------------------------------
struct PassArgs {
    const int *trp, *tci;   // X
    const double *tv;
    const int *mrp, *mci;   // Y
    const double *mv;
    double tau;
    int cap;
    const int *srp, *sci;   // pattern mask (nullptr: threshold rule)
    const int64_t *cand_ptr;
    int *out_ci;
    double *out_v;
    int *nk;
};

template <int NT>
__device__ __forceinline__ int block_scan_excl_i32(int x, int *sh, int *total) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        int y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    const int incl = sh[t];
    if (total) *total = sh[NT - 1];
    __syncthreads();
    return incl - x;
}

__device__ __forceinline__ bool in_pattern(const int *sci, int b, int e, int col) {
    while (b < e) {
        const int mid = (b + e) >> 1;
        const int c = sci[mid];
        if (c == col) return true;
        if (c < col) b = mid + 1;
        else e = mid;
    }
    return false;
}

__device__ __forceinline__ int next_pow2(int c) {
    int p = 1;
    while (p < c) p <<= 1;
    return p;
}

template <int NT>
__device__ void pass_row(const PassArgs &a, int i, unsigned long long *key, double *val, unsigned char *kf,
                         int *seg, int *shi) {
    const int tid = threadIdx.x;
    const int tb = a.trp[i];
    const int S = a.trp[i + 1] - tb;
    int C;  // candidates: the products plus the identity
    // 1. segment lengths -> exclusive offsets (seg[0..S], seg[S] = C-1)
    {
        const int E = (S + NT - 1) / NT;
        const int s0 = tid * E;
        int local = 0;
        for (int s = s0; s < s0 + E && s < S; ++s) {
            const int l = a.tci[tb + s];
            const int len = a.mrp[l + 1] - a.mrp[l];
            seg[s] = len;
            local += len;
        }
        int products;
        int ex = block_scan_excl_i32<NT>(local, shi, &products);
        C = products + 1;
        for (int s = s0; s < s0 + E && s < S; ++s) {
            const int len = seg[s];
            seg[s] = ex;
            ex += len;
        }
        if (tid == 0) seg[S] = C - 1;
        __syncthreads();
    }
    const int P = next_pow2(C);
    // 2. candidates: key = (column << 32) | candidate index; val[index] = product
    for (int c = tid; c < C - 1; c += NT) {
        int lo = 0, hi = S;  // largest s with seg[s] <= c
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (seg[mid] <= c) lo = mid;
            else hi = mid;
        }
        const int l = a.tci[tb + lo];
        const int q = a.mrp[l] + (c - seg[lo]);
        key[c] = ((unsigned long long)(unsigned)a.mci[q] << 32) | (unsigned)c;
        val[c] = dmul(a.tv[tb + lo], a.mv[q]);
    }
    if (tid == 0) {
        key[C - 1] = ((unsigned long long)(unsigned)i << 32) | (unsigned)(C - 1);
        val[C - 1] = 1.0;
    }
    for (int c = C + tid; c < P; c += NT) key[c] = ~0ull;
    __syncthreads();
    // 3. bitonic sort of key[0..P)
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int lj = __ffs(j) - 1;
            for (int t = tid; t < (P >> 1); t += NT) {
                const int lo_i = ((t >> lj) << (lj + 1)) | (t & (j - 1));
                const int hi_i = lo_i + j;
                const unsigned long long x = key[lo_i], y = key[hi_i];
                const bool up = (lo_i & k) == 0;
                if ((x > y) == up) {
                    key[lo_i] = y;
                    key[hi_i] = x;
                }
            }
            __syncthreads();
        }
    }
    // 4. sum each run of equal columns in key order (l ascending); the head's
    //    slot of val receives the sum.
    for (int q = tid; q < C; q += NT) {
        const unsigned col = (unsigned)(key[q] >> 32);
        if (q > 0 && (unsigned)(key[q - 1] >> 32) == col) continue;
        double s = 0.0;
        int t = q;
        do {
            s = dadd(s, val[(unsigned)key[t]]);
            ++t;
        } while (t < C && (unsigned)(key[t] >> 32) == col);
        val[(unsigned)key[q]] = s;
    }
    __syncthreads();
    // 5. keep flags (bit 0), counted per thread over a contiguous chunk
    const int E = (C + NT - 1) / NT;
    const int q0 = tid * E;
    int kept_off = 0;
    for (int q = q0; q < q0 + E && q < C; ++q) {
        const unsigned col = (unsigned)(key[q] >> 32);
        const bool head = q == 0 || (unsigned)(key[q - 1] >> 32) != col;
        unsigned char f = 0;
        if (head) {
            if ((int)col == i) f = 1;
            else {
                const double w = val[(unsigned)key[q]];
                const bool keep = a.srp ? (w != 0.0 && in_pattern(a.sci, a.srp[i], a.srp[i + 1], (int)col))
                                        : (fabs(w) > a.tau);
                f = keep ? 1 : 0;
                kept_off += f;
            }
        }
        kf[q] = f;
    }
    // 6. optional cap: keep diagonal + (cap-1) largest |w| (ties: smaller column)
    if (a.cap > 0) {
        int total_off;
        block_scan_excl_i32<NT>(kept_off, shi, &total_off);  // includes a barrier
        if (total_off > a.cap - 1) {
            for (int q = tid; q < C; q += NT) {
                if (!(kf[q] & 1)) continue;
                const unsigned col = (unsigned)(key[q] >> 32);
                if ((int)col == i) {
                    kf[q] |= 2;
                    continue;
                }
                const double w = fabs(val[(unsigned)key[q]]);
                int rank = 0;
                for (int t = 0; t < C && rank < a.cap - 1; ++t) {
                    if (!(kf[t] & 1) || t == q) continue;
                    const unsigned ct = (unsigned)(key[t] >> 32);
                    if ((int)ct == i) continue;
                    const double wt = fabs(val[(unsigned)key[t]]);
                    if (wt > w || (wt == w && ct < col)) ++rank;
                }
                if (rank < a.cap - 1) kf[q] |= 2;
            }
            __syncthreads();
            for (int q = tid; q < C; q += NT) kf[q] = (kf[q] >> 1) & 1;
            __syncthreads();
        }
    } else {
        __syncthreads();
    }
    // 7. compaction in column order
    int mine = 0;
    for (int q = q0; q < q0 + E && q < C; ++q) mine += kf[q] & 1;
    int total;
    int pos = block_scan_excl_i32<NT>(mine, shi, &total);
    const int64_t base = a.cand_ptr[i];
    for (int q = q0; q < q0 + E && q < C; ++q) {
        if (!(kf[q] & 1)) continue;
        a.out_ci[base + pos] = (int)(key[q] >> 32);
        a.out_v[base + pos] = val[(unsigned)key[q]];
        ++pos;
    }
    if (tid == 0) a.nk[i] = total;
}

template <int NT, int CAP>
__global__ __launch_bounds__(NT) void k_pass_lds(PassArgs a, const int *__restrict__ rows, const int64_t *__restrict__ cnt) {
    __shared__ unsigned long long key[CAP];
    __shared__ double val[CAP];
    __shared__ unsigned char kf[CAP];
    __shared__ int seg[CAP + 1];
    __shared__ int shi[NT];
    (void)cnt;
    pass_row<NT>(a, rows[blockIdx.x], key, val, kf, seg, shi);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_pass_global(PassArgs a, const int *__restrict__ rows,
                                                    const int64_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ soff, unsigned char *scratch) {
    __shared__ int shi[NT];
    const int r = blockIdx.x;
    const int i = rows[r];
    const int C = (int)cnt[i];  // the row's bound: the layout the host sized
    const int P = next_pow2(C);
    unsigned char *base = scratch + soff[r];
    unsigned long long *key = reinterpret_cast<unsigned long long *>(base);
    double *val = reinterpret_cast<double *>(base + (size_t)P * 8);
    int *seg = reinterpret_cast<int *>(base + (size_t)P * 16);
    unsigned char *kf = base + (size_t)P * 16 + (size_t)(C + 1) * 4;
    pass_row<NT>(a, i, key, val, kf, seg, shi);
}

// Identity M_0 = I.
__global__ void k_identity(int n, int *__restrict__ rp, int *__restrict__ ci, double *__restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    rp[i] = i;
    if (i < n) {
        ci[i] = i;
        v[i] = 1.0;
    }
}

__global__ void k_rowptr_i32(int n, const int64_t *__restrict__ p64, int *__restrict__ p32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) p32[i] = (int)p64[i];
}

__global__ void k_i32_to_i64(int n, const int *__restrict__ in, int64_t *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// Gather each row's kept entries from its candidate slot into the final CSR;
// optionally scale by dinv[col] (final pass) -- 16 lanes per row.
__global__ void k_compact(int n, const int64_t *__restrict__ cand_ptr, const int *__restrict__ rp_new,
                          const int *__restrict__ in_ci, const double *__restrict__ in_v, int *__restrict__ out_ci,
                          double *__restrict__ out_v, const double *__restrict__ dinv) {
    const int g = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int lane = threadIdx.x & 15;
    if (g >= n) return;
    const int64_t src = cand_ptr[g];
    const int dst = rp_new[g];
    const int len = rp_new[g + 1] - dst;
    for (int t = lane; t < len; t += 16) {
        const int c = in_ci[src + t];
        double x = in_v[src + t];
        if (dinv) x = dmul(x, dinv[c]);
        out_ci[dst + t] = c;
        out_v[dst + t] = x;
    }
}

__global__ void k_cast_f32(int64_t nnz, const double *__restrict__ v, float *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) o[i] = __double2float_rn(v[i]);
}

__global__ void k_cast_bf16(int64_t nnz, const double *__restrict__ v, unsigned short *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nnz) o[i] = bf16_rne(__double2float_rn(v[i]));
}

// Transpose: count per column, scan, scatter (atomic slots), sort each row.
__global__ void k_tcount(int64_t nnz, const int *__restrict__ ci, int *__restrict__ colcnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) atomicAdd(&colcnt[ci[p]], 1);
}

__global__ void k_tscatter(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                           const int64_t *__restrict__ trp, int *__restrict__ fill, int *__restrict__ tci,
                           double *__restrict__ tv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const int slot = atomicAdd(&fill[j], 1);
        tci[trp[j] + slot] = i;
        tv[trp[j] + slot] = v[p];
    }
}

// Insertion sort of each (short) row by column; one thread per row.
__global__ void k_rowsort(int n, const int *__restrict__ rp, int *__restrict__ ci, double *__restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = rp[i], e = rp[i + 1];
    for (int p = b + 1; p < e; ++p) {
        const int c = ci[p];
        const double x = v[p];
        int q = p - 1;
        while (q >= b && ci[q] > c) {
            ci[q + 1] = ci[q];
            v[q + 1] = v[q];
            --q;
        }
        ci[q + 1] = c;
        v[q + 1] = x;
    }
}

__global__ void k_iota_f64(int64_t nnz, double *__restrict__ v) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) v[p] = (double)p;
}

__global__ void k_f64_to_i32(int64_t nnz, const double *__restrict__ v, int *__restrict__ o) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) o[p] = (int)v[p];
}

__global__ void k_gather_f64(int64_t nnz, const int *__restrict__ perm, const double *__restrict__ src,
                             double *__restrict__ dst) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) dst[p] = src[perm[p]];
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

// ===========================================================================
// Host orchestration
// ===========================================================================

void scan_exclusive_i64(Allocator *a, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    const int64_t per = (int64_t)kScanBlock * kScanItems;
    const int64_t nb = std::max<int64_t>(1, (n + per - 1) / per);
    DevBuf part;
    part.alloc(a, (size_t)(nb + 1) * sizeof(int64_t));
    hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, part.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s, part.as<int64_t>(), nb);
    SAIT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, part.as<int64_t>(), out);
    SAIT_LAUNCH_CHECK();
    SAIT_HIP(hipStreamSynchronize(s));  // `part` is released on return
}

void upload_csr(Allocator *a, const HostCsr &h, DevCsr &d, hipStream_t s) {
    d.n = h.n;
    d.nnz = h.nnz();
    d.precision = SAIT_F64;
    d.rp.alloc(a, (size_t)(h.n + 1) * sizeof(int));
    d.ci.alloc(a, (size_t)std::max<int64_t>(d.nnz, 1) * sizeof(int));
    d.v.alloc(a, (size_t)std::max<int64_t>(d.nnz, 1) * sizeof(double));
    SAIT_HIP(hipMemcpyAsync(d.rp.as<void>(), h.rp.data(), (h.n + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    if (d.nnz) {
        SAIT_HIP(hipMemcpyAsync(d.ci.as<void>(), h.ci.data(), d.nnz * sizeof(int), hipMemcpyHostToDevice, s));
        SAIT_HIP(hipMemcpyAsync(d.v.as<void>(), h.v.data(), d.nnz * sizeof(double), hipMemcpyHostToDevice, s));
    }
    SAIT_HIP(hipStreamSynchronize(s));
}

void download_csr(const DevCsr &d, HostCsr &h, hipStream_t s) {
    h.n = d.n;
    h.rp.resize(d.n + 1);
    h.ci.resize(d.nnz);
    h.v.resize(d.nnz);
    SAIT_HIP(hipMemcpyAsync(h.rp.data(), d.rp.as<void>(), (d.n + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    if (d.nnz) {
        SAIT_HIP(hipMemcpyAsync(h.ci.data(), d.ci.as<void>(), d.nnz * sizeof(int), hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipMemcpyAsync(h.v.data(), d.v.as<void>(), d.nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    SAIT_HIP(hipStreamSynchronize(s));
}

void cast_values(Allocator *a, DevCsr &M, int precision, hipStream_t s) {
    M.precision = precision;
    const int64_t nnz = std::max<int64_t>(M.nnz, 1);
    if (precision == SAIT_F64) {
        M.vs.reset();
        return;
    }
    if (precision == SAIT_F32) {
        M.vs.alloc(a, nnz * sizeof(float));
        if (M.nnz) hipLaunchKernelGGL(k_cast_f32, dim3(blocks_for(M.nnz, 256)), dim3(256), 0, s, M.nnz, M.v.as<double>(), M.vs.as<float>());
    } else if (precision == SAIT_BF16) {
        M.vs.alloc(a, nnz * sizeof(unsigned short));
        if (M.nnz) hipLaunchKernelGGL(k_cast_bf16, dim3(blocks_for(M.nnz, 256)), dim3(256), 0, s, M.nnz, M.v.as<double>(), M.vs.as<unsigned short>());
    } else {
        fail(SAIT_E_INVALID, "unknown storage precision");
    }
    SAIT_LAUNCH_CHECK();
}

namespace {

// Split T into dinv and T~ (device).
struct Split {
    DevBuf trp, tci, tv, dinv;
};

void do_split(Allocator *a, const DevCsr &T, Split &sp, hipStream_t s) {
    const int n = (int)T.n;
    sp.trp.alloc(a, (size_t)(n + 1) * sizeof(int));
    sp.tci.alloc(a, (size_t)std::max<int64_t>(T.nnz - n, 1) * sizeof(int));
    sp.tv.alloc(a, (size_t)std::max<int64_t>(T.nnz - n, 1) * sizeof(double));
    sp.dinv.alloc(a, (size_t)std::max(n, 1) * sizeof(double));
    DevBuf err;
    err.alloc(a, sizeof(int));
    SAIT_HIP(hipMemsetAsync(err.as<void>(), 0, sizeof(int), s));
    hipLaunchKernelGGL(k_split, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n, T.rp.as<int>(), T.ci.as<int>(),
                       T.v.as<double>(), sp.trp.as<int>(), sp.tci.as<int>(), sp.tv.as<double>(), sp.dinv.as<double>(),
                       err.as<int>());
    SAIT_LAUNCH_CHECK();
    int herr = 0;
    SAIT_HIP(hipMemcpyAsync(&herr, err.as<void>(), sizeof(int), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (herr) fail(SAIT_E_ZERO_PIVOT, "SAIT: triangular factor has a zero, missing or non-finite diagonal entry");
}

// One pass: Mnext = drop(T~ Mprev + I), or drop(Mprev T~ + I) if right; if
// dinv != nullptr the result is also scaled by D^-1 (final pass).
void one_pass(Allocator *a, int n, const Split &sp, const DevCsr &Mprev, bool right, double tau, int cap,
              const int *srp, const int *sci, const double *final_dinv, DevCsr &Mnext, hipStream_t s) {
    DevBuf cnt, cptr, lists, tier_n, nk, nk64, rp64;
    cnt.alloc(a, (size_t)std::max(n, 1) * sizeof(int64_t));
    cptr.alloc(a, (size_t)(n + 1) * sizeof(int64_t));
    // operands of W = X Y + I
    const int *xrp = right ? Mprev.rp.as<int>() : sp.trp.as<int>();
    const int *xci = right ? Mprev.ci.as<int>() : sp.tci.as<int>();
    const double *xv = right ? Mprev.v.as<double>() : sp.tv.as<double>();
    const int *yrp = right ? sp.trp.as<int>() : Mprev.rp.as<int>();
    const int *yci = right ? sp.tci.as<int>() : Mprev.ci.as<int>();
    const double *yv = right ? sp.tv.as<double>() : Mprev.v.as<double>();
    hipLaunchKernelGGL(k_count, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, xrp, xci, yrp, cnt.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    scan_exclusive_i64(a, cnt.as<int64_t>(), cptr.as<int64_t>(), n, s);
    int64_t total = 0;
    SAIT_HIP(hipMemcpyAsync(&total, cptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    lists.alloc(a, (size_t)4 * std::max(n, 1) * sizeof(int));
    tier_n.alloc(a, 4 * sizeof(int));
    SAIT_HIP(hipMemsetAsync(tier_n.as<void>(), 0, 4 * sizeof(int), s));
    hipLaunchKernelGGL(k_classify, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, cnt.as<int64_t>(), tier_n.as<int>(),
                       lists.as<int>());
    SAIT_LAUNCH_CHECK();
    int tn[4];
    SAIT_HIP(hipMemcpyAsync(tn, tier_n.as<void>(), sizeof(tn), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));

    DevBuf oci, ov;
    oci.alloc(a, (size_t)std::max<int64_t>(total, 1) * sizeof(int));
    ov.alloc(a, (size_t)std::max<int64_t>(total, 1) * sizeof(double));
    nk.alloc(a, (size_t)std::max(n, 1) * sizeof(int));

    PassArgs pa;
    pa.trp = xrp;
    pa.tci = xci;
    pa.tv = xv;
    pa.mrp = yrp;
    pa.mci = yci;
    pa.mv = yv;
    pa.tau = tau;
    pa.cap = cap;
    pa.srp = srp;
    pa.sci = sci;
    pa.cand_ptr = cptr.as<int64_t>();
    pa.out_ci = oci.as<int>();
    pa.out_v = ov.as<double>();
    pa.nk = nk.as<int>();
    const int *L = lists.as<int>();
    if (tn[0]) hipLaunchKernelGGL((k_pass_lds<64, kTierCap0>), dim3(tn[0]), dim3(64), 0, s, pa, L, cnt.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    if (tn[1]) hipLaunchKernelGGL((k_pass_lds<64, kTierCap1>), dim3(tn[1]), dim3(64), 0, s, pa, L + (size_t)n, cnt.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    if (tn[2]) hipLaunchKernelGGL((k_pass_lds<256, kTierCap2>), dim3(tn[2]), dim3(256), 0, s, pa, L + (size_t)2 * n, cnt.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    DevBuf scratch, soff;
    if (tn[3]) {
        // per-row scratch: P keys + P values + (C+1) segment offsets + P flags
        std::vector<int> rows(tn[3]);
        std::vector<int64_t> c64(n);
        SAIT_HIP(hipMemcpyAsync(rows.data(), L + (size_t)3 * n, tn[3] * sizeof(int), hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipMemcpyAsync(c64.data(), cnt.as<void>(), (size_t)n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> off(tn[3] + 1, 0);
        for (int r = 0; r < tn[3]; ++r) {
            const int64_t C = c64[rows[r]];
            if (C >= (int64_t)1 << 30) fail(SAIT_E_INVALID, "SAIT: a row of T~ M has more than 2^30 candidate products");
            int64_t P = 1;
            while (P < C) P <<= 1;
            const int64_t bytes = P * 17 + (C + 1) * 4;
            off[r + 1] = off[r] + ((bytes + 15) / 16) * 16;
        }
        scratch.alloc(a, (size_t)off[tn[3]]);
        soff.alloc(a, (size_t)(tn[3] + 1) * sizeof(int64_t));
        SAIT_HIP(hipMemcpyAsync(soff.as<void>(), off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_pass_global<256>, dim3(tn[3]), dim3(256), 0, s, pa, L + (size_t)3 * n, cnt.as<int64_t>(),
                           soff.as<int64_t>(), scratch.as<unsigned char>());
        SAIT_LAUNCH_CHECK();
    }
    // row pointers of the result
    nk64.alloc(a, (size_t)std::max(n, 1) * sizeof(int64_t));
    rp64.alloc(a, (size_t)(n + 1) * sizeof(int64_t));
    hipLaunchKernelGGL(k_i32_to_i64, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, nk.as<int>(), nk64.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    scan_exclusive_i64(a, nk64.as<int64_t>(), rp64.as<int64_t>(), n, s);
    int64_t nnz = 0;
    SAIT_HIP(hipMemcpyAsync(&nnz, rp64.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (nnz > INT32_MAX) fail(SAIT_E_INVALID, "SAIT: factor exceeds 2^31-1 stored entries");
    Mnext.n = n;
    Mnext.nnz = nnz;
    Mnext.precision = SAIT_F64;
    Mnext.vs.reset();
    Mnext.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
    Mnext.ci.alloc(a, (size_t)std::max<int64_t>(nnz, 1) * sizeof(int));
    Mnext.v.alloc(a, (size_t)std::max<int64_t>(nnz, 1) * sizeof(double));
    hipLaunchKernelGGL(k_rowptr_i32, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n, rp64.as<int64_t>(), Mnext.rp.as<int>());
    SAIT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_compact, dim3(blocks_for((int64_t)n * 16, 256)), dim3(256), 0, s, n, cptr.as<int64_t>(),
                       Mnext.rp.as<int>(), oci.as<int>(), ov.as<double>(), Mnext.ci.as<int>(), Mnext.v.as<double>(),
                       final_dinv);
    SAIT_LAUNCH_CHECK();
    SAIT_HIP(hipStreamSynchronize(s));
}

void make_identity(Allocator *a, int n, DevCsr &M, hipStream_t s) {
    M.n = n;
    M.nnz = n;
    M.precision = SAIT_F64;
    M.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
    M.ci.alloc(a, (size_t)std::max(n, 1) * sizeof(int));
    M.v.alloc(a, (size_t)std::max(n, 1) * sizeof(double));
    hipLaunchKernelGGL(k_identity, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n, M.rp.as<int>(), M.ci.as<int>(),
                       M.v.as<double>());
    SAIT_LAUNCH_CHECK();
}

// Scale columns by dinv (used when m == 0 or when the last pass is not fused).
__global__ void k_scale_cols(int64_t nnz, const int *__restrict__ ci, double *__restrict__ v, const double *__restrict__ dinv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) v[p] = dmul(v[p], dinv[ci[p]]);
}

}  // namespace

void build_sait_factor(Allocator *a, const DevCsr &T, const SaitParams &p, DevCsr &M, hipStream_t s) {
    if (!(p.tau >= 0.0 && p.tau < 1.0)) fail(SAIT_E_INVALID, "SAIT: tau must satisfy 0 <= tau < 1");
    if (p.m < 0) fail(SAIT_E_INVALID, "SAIT: m must be >= 0");
    if (p.cap < 0) fail(SAIT_E_INVALID, "SAIT: max_nnz_row must be >= 0");
    const int n = (int)T.n;
    Split sp;
    do_split(a, T, sp, s);
    DevCsr cur;
    make_identity(a, n, cur, s);
    DevBuf srp, sci;
    const int p_unrestricted = p.pattern_p >= 0 ? p.pattern_p : 0;
    const int total = p_unrestricted + p.m;
    int done = 0;
    // Alg. 3: p passes without dropping (keep numerical nonzeros), pattern S
    for (int k = 0; k < p_unrestricted; ++k, ++done) {
        DevCsr nxt;
        const bool last = done + 1 == total;
        one_pass(a, n, sp, cur, p.right, 0.0, 0, nullptr, nullptr, last ? sp.dinv.as<double>() : nullptr, nxt, s);
        cur = std::move(nxt);
    }
    const int *S_rp = nullptr, *S_ci = nullptr;
    DevCsr S;
    if (p.pattern_p >= 0) {
        if (total == p_unrestricted && total > 0) {
            // m == 0: the result is already final (scaled in the last pass)
        } else {
            S.n = cur.n;
            S.nnz = cur.nnz;
            S.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
            S.ci.alloc(a, (size_t)std::max<int64_t>(cur.nnz, 1) * sizeof(int));
            SAIT_HIP(hipMemcpyAsync(S.rp.as<void>(), cur.rp.as<void>(), (n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
            if (cur.nnz)
                SAIT_HIP(hipMemcpyAsync(S.ci.as<void>(), cur.ci.as<void>(), cur.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
            S_rp = S.rp.as<int>();
            S_ci = S.ci.as<int>();
        }
    }
    // Alg. 2 / Alg. 3 dropping passes
    for (int k = 0; k < p.m; ++k, ++done) {
        DevCsr nxt;
        const bool last = done + 1 == total;
        one_pass(a, n, sp, cur, p.right, p.tau, p.pattern_p >= 0 ? 0 : p.cap, S_rp, S_ci,
                 last ? sp.dinv.as<double>() : nullptr, nxt, s);
        cur = std::move(nxt);
    }
    if (total == 0 && n > 0) {
        // M = I D^-1
        hipLaunchKernelGGL(k_scale_cols, dim3(blocks_for(cur.nnz, 256)), dim3(256), 0, s, cur.nnz, cur.ci.as<int>(),
                           cur.v.as<double>(), sp.dinv.as<double>());
        SAIT_LAUNCH_CHECK();
    }
    cast_values(a, cur, p.precision, s);
    SAIT_HIP(hipStreamSynchronize(s));
    M = std::move(cur);
}

void sait_single_pass(Allocator *a, const DevCsr &T, const DevCsr &Mprev, bool right, double tau, int cap,
                      DevCsr &Mnext, hipStream_t s) {
    if (!(tau >= 0.0 && tau < 1.0)) fail(SAIT_E_INVALID, "SAIT: tau must satisfy 0 <= tau < 1");
    if (cap < 0) fail(SAIT_E_INVALID, "SAIT: max_nnz_row must be >= 0");
    Split sp;
    do_split(a, T, sp, s);
    one_pass(a, (int)T.n, sp, Mprev, right, tau, cap, nullptr, nullptr, nullptr, Mnext, s);
}

void transpose_csr(Allocator *a, const DevCsr &M, DevCsr &Mt, hipStream_t s) {
    const int n = (int)M.n;
    DevBuf colcnt, c64, trp64, fill;
    colcnt.alloc(a, (size_t)std::max(n, 1) * sizeof(int));
    SAIT_HIP(hipMemsetAsync(colcnt.as<void>(), 0, (size_t)std::max(n, 1) * sizeof(int), s));
    if (M.nnz) hipLaunchKernelGGL(k_tcount, dim3(blocks_for(M.nnz, 256)), dim3(256), 0, s, M.nnz, M.ci.as<int>(), colcnt.as<int>());
    SAIT_LAUNCH_CHECK();
    c64.alloc(a, (size_t)std::max(n, 1) * sizeof(int64_t));
    trp64.alloc(a, (size_t)(n + 1) * sizeof(int64_t));
    hipLaunchKernelGGL(k_i32_to_i64, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, colcnt.as<int>(), c64.as<int64_t>());
    SAIT_LAUNCH_CHECK();
    scan_exclusive_i64(a, c64.as<int64_t>(), trp64.as<int64_t>(), n, s);
    fill.alloc(a, (size_t)std::max(n, 1) * sizeof(int));
    SAIT_HIP(hipMemsetAsync(fill.as<void>(), 0, (size_t)std::max(n, 1) * sizeof(int), s));
    Mt.n = n;
    Mt.nnz = M.nnz;
    Mt.precision = SAIT_F64;
    Mt.vs.reset();
    Mt.rp.alloc(a, (size_t)(n + 1) * sizeof(int));
    Mt.ci.alloc(a, (size_t)std::max<int64_t>(M.nnz, 1) * sizeof(int));
    Mt.v.alloc(a, (size_t)std::max<int64_t>(M.nnz, 1) * sizeof(double));
    hipLaunchKernelGGL(k_tscatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, M.rp.as<int>(), M.ci.as<int>(),
                       M.v.as<double>(), trp64.as<int64_t>(), fill.as<int>(), Mt.ci.as<int>(), Mt.v.as<double>());
    SAIT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rowptr_i32, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n, trp64.as<int64_t>(), Mt.rp.as<int>());
    SAIT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rowsort, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, Mt.rp.as<int>(), Mt.ci.as<int>(), Mt.v.as<double>());
    SAIT_LAUNCH_CHECK();
    SAIT_HIP(hipStreamSynchronize(s));
}

void transpose_perm(Allocator *a, const DevCsr &M, DevBuf &perm, hipStream_t s) {
    DevCsr idx, idxT;
    idx.n = M.n;
    idx.nnz = M.nnz;
    idx.rp.alloc(a, (size_t)(M.n + 1) * sizeof(int));
    idx.ci.alloc(a, (size_t)std::max<int64_t>(M.nnz, 1) * sizeof(int));
    idx.v.alloc(a, (size_t)std::max<int64_t>(M.nnz, 1) * sizeof(double));
    SAIT_HIP(hipMemcpyAsync(idx.rp.as<void>(), M.rp.as<void>(), (M.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (M.nnz) {
        SAIT_HIP(hipMemcpyAsync(idx.ci.as<void>(), M.ci.as<void>(), M.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_iota_f64, dim3(blocks_for(M.nnz, 256)), dim3(256), 0, s, M.nnz, idx.v.as<double>());
        SAIT_LAUNCH_CHECK();
    }
    transpose_csr(a, idx, idxT, s);
    perm.alloc(a, (size_t)std::max<int64_t>(M.nnz, 1) * sizeof(int));
    if (M.nnz) {
        hipLaunchKernelGGL(k_f64_to_i32, dim3(blocks_for(M.nnz, 256)), dim3(256), 0, s, M.nnz, idxT.v.as<double>(),
                           perm.as<int>());
        SAIT_LAUNCH_CHECK();
    }
    SAIT_HIP(hipStreamSynchronize(s));
}

void gather_values(int64_t nnz, const int *perm, const double *src, double *dst, hipStream_t s) {
    if (!nnz) return;
    hipLaunchKernelGGL(k_gather_f64, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, perm, src, dst);
    SAIT_LAUNCH_CHECK();
}

}  // namespace sait
