// Batched SAIT-preconditioned GMRES in one persistent launch.
//
// A is the block-diagonal concatenation of nsys independent systems
// (sys_ptr), each with R right-hand sides (row-major n x ld blocks).  Every
// (system, right-hand side) pair runs its own restarted right-preconditioned
// GMRES(k) -- the same sequence of operations as a separate solve: Arnoldi
// steps until its residual estimate meets rtol, a breakdown, maxit or k
// steps, then x += M (V y), the true residual, and a restart or exit.  The
// pairs advance in lockstep through one cooperative launch whose phases are
// separated by grid barriers:
//   apply (two SpMMs, R columns per lane-row on the sliced-ELL factors),
//   A z, segmented inner products per pair, classical Gram-Schmidt update
//   with the DGKS re-orthogonalisation test, per-pair Givens rotation and
//   convergence flags, normalisation; at a cycle end the per-pair triangular
//   solve, V y, the preconditioner, the x update and the true residual.
// Pairs that stop early wait for the cycle end; converged pairs drop out,
// and rows of systems without a participating pair are skipped.  Reductions
// are deterministic: per-unit partial sums (units are row ranges inside one
// system), summed in unit order.
//
// The grid barrier spins with a bounded count; if it is ever exceeded the
// kernel raises an abort flag that every block checks, so the launch always
// terminates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "sait_internal.h"
#include "solver.h"

namespace sait {

namespace {

constexpr int kNT = 256;
constexpr int kRT = 8;          // right-hand sides per pass (R <= 8)
constexpr int kUnitRows = 4096;  // rows per reduction unit
constexpr int kMaxRestart = 64;
constexpr unsigned long long kSpinLimit = 1ull << 25;  // about 2 s of s_sleep(2) polling

struct SellView {
    int nslices;
    const int64_t *sptr;
    const int *rp, *sci;
    const double *sv;
};

struct BatchArgs {
    int n, nsys, R, k, maxit, nunits, npairs;
    double rtol;
    const int64_t *sys_ptr;  // nsys + 1
    SellView A, ML, MU;
    const int *slice_sys;    // system of the first row of every 64-row slice
    const int *unit_sys;     // nunits
    const int64_t *unit_row; // nunits + 1
    const int *sys_unit;     // nsys + 1
    const double *b;
    double *x;
    int64_t ld;              // leading dimension of b and x
    double *V;               // (k+1) blocks of n*R
    double *T, *Z, *U;       // n*R each
    double *part;            // nunits * (k+2) * R
    // per pair
    int *active, *cyc, *jc, *iters, *restarts, *status, *reorth;
    double *nb, *beta, *est, *inv, *wpre2;
    double *H, *cs, *sn, *g, *y, *h1, *h2;
    unsigned char *sysmask;  // per system: bit q = pair (s, q) takes part in the current phase
    int *ctrl;               // [0] pairs in cycle, [1] pairs needing re-orthogonalisation, [2] active pairs
    unsigned *bar_count, *bar_gen;
    int *abort;
};

// ---------------------------------------------------------------------------
// Grid barrier (all workgroups are co-resident: cooperative launch).
// ---------------------------------------------------------------------------
__device__ bool grid_barrier(const BatchArgs &a) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __shared__ int bad;
    if (threadIdx.x == 0) {
        bad = 0;
        const unsigned gen = __hip_atomic_load(a.bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(a.bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(a.bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a.bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while (__hip_atomic_load(a.bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        bad = __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return bad == 0;
}

__device__ __forceinline__ int ld_ctrl(const BatchArgs &a, int i) {
    return __hip_atomic_load(a.ctrl + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double mul_rn(double p, double q) {
#pragma clang fp contract(off)
    return p * q;
}
__device__ __forceinline__ double add_rn(double p, double q) {
#pragma clang fp contract(off)
    return p + q;
}

// ---------------------------------------------------------------------------
// SpMM on a sliced-ELL matrix: out[row*R + q] = sum_k v x[col*ldx + q]
// (or b[row*ldb + q] - that), for the rows of systems whose mask is nonzero.
// One wavefront per 64-row slice, lane = row, column order, separately
// rounded products and sums.
// ---------------------------------------------------------------------------
__device__ void phase_spmm(const BatchArgs &a, const SellView &M, const double *xin, int64_t ldx, double *out,
                           int64_t ldo, const double *bres, int64_t ldb) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int R = a.R;
    for (int s = blockIdx.x * (kNT / 64) + wave; s < M.nslices; s += gridDim.x * (kNT / 64)) {
        const int row = s * 64 + l;
        bool act = false;
        int len = 0;
        if (row < a.n) {
            int sy = a.slice_sys[s];
            while (row >= a.sys_ptr[sy + 1]) ++sy;
            act = a.sysmask[sy] != 0;
            if (act) len = M.rp[row + 1] - M.rp[row];
        }
        if (__ballot(act) == 0) continue;
        const int64_t base = M.sptr[s];
        const int ngroups = (int)((M.sptr[s + 1] - base) >> 8);
        double acc[kRT];
#pragma unroll
        for (int q = 0; q < kRT; ++q) acc[q] = 0.0;
        for (int gi = 0; gi < ngroups; ++gi) {
            const int64_t off = base + (int64_t)gi * 256 + 4 * l;
            int cols[4];
            double vals[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cols[j] = M.sci[off + j];
                vals[j] = M.sv[off + j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (gi * 4 + j < len) {
                    const double *xr = xin + (int64_t)cols[j] * ldx;
#pragma unroll
                    for (int q = 0; q < kRT; ++q)
                        if (q < R) acc[q] = add_rn(acc[q], mul_rn(vals[j], xr[q]));
                }
            }
        }
        if (act) {
#pragma unroll
            for (int q = 0; q < kRT; ++q)
                if (q < R) {
                    if (bres) out[(int64_t)row * ldo + q] = bres[(int64_t)row * ldb + q] - acc[q];
                    else out[(int64_t)row * ldo + q] = acc[q];
                }
        }
    }
}

// Block sum of R values per thread -> sh[q] (valid after the call).
__device__ void block_sum_r(double (&v)[kRT], double *sh) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kRT; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((threadIdx.x & 63) == 0) sh[w * kRT + q] = x;
    }
    __syncthreads();
    if (threadIdx.x < kRT) {
        const int q = threadIdx.x;
        sh[4 * kRT + q] = (sh[q] + sh[kRT + q]) + (sh[2 * kRT + q] + sh[3 * kRT + q]);
    }
    __syncthreads();
}

// Partial inner products of the unit's rows: part[u][i][q] = sum_r V_i[r][q] w[r][q]
// for i < nv, and (with_norm) part[u][nv][q] = sum_r w[r][q]^2, for pairs
// whose flag (cyc or reorth) is set.
__device__ void phase_dots(const BatchArgs &a, int nv, const double *w, bool with_norm, const int *flag,
                           double *sh) {
    const int R = a.R;
    const int stride = a.k + 2;
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        if (a.sysmask[s] == 0) continue;
        const int64_t r0 = a.unit_row[u], r1 = a.unit_row[u + 1];
        for (int i = 0; i <= (with_norm ? nv : nv - 1); ++i) {
            const double *vi = i < nv ? a.V + (int64_t)i * a.n * R : w;
            double acc[kRT];
#pragma unroll
            for (int q = 0; q < kRT; ++q) acc[q] = 0.0;
            for (int64_t r = r0 + threadIdx.x; r < r1; r += kNT) {
#pragma unroll
                for (int q = 0; q < kRT; ++q)
                    if (q < R) acc[q] = fma(vi[r * R + q], w[r * R + q], acc[q]);
            }
            block_sum_r(acc, sh);
            if (threadIdx.x < R) {
                const int q = threadIdx.x;
                if (flag[s * R + q]) a.part[((int64_t)u * stride + i) * R + q] = sh[4 * kRT + q];
            }
        }
    }
    (void)stride;
}

// Sum the unit partials of index first+i (i < count) for every flagged pair
// into out[p*ldo + i].
__device__ void phase_reduce(const BatchArgs &a, int first, int count, const int *flag, double *out, int ldo) {
    const int R = a.R;
    const int stride = a.k + 2;
    const int total = a.npairs * count;
    for (int t = blockIdx.x * kNT + threadIdx.x; t < total; t += gridDim.x * kNT) {
        const int p = t / count, i = t % count;
        if (!flag[p]) continue;
        const int s = p / R, q = p % R;
        double acc = 0.0;
        for (int u = a.sys_unit[s]; u < a.sys_unit[s + 1]; ++u) acc += a.part[((int64_t)u * stride + first + i) * R + q];
        out[(int64_t)p * ldo + i] = acc;
    }
}

// w -= sum_{i < nv} h[p][i] V_i for flagged pairs, and per-unit partial ||w||^2
// into part[u][0][q].
__device__ void phase_update(const BatchArgs &a, int nv, double *w, const int *flag, const double *h, int ldh,
                             double *sh) {
    const int R = a.R;
    const int stride = a.k + 2;
    __shared__ double hs[kRT * (kMaxRestart + 1)];
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        if (a.sysmask[s] == 0) continue;
        __syncthreads();
        for (int t = threadIdx.x; t < R * nv; t += kNT) {
            const int q = t / nv, i = t % nv;
            const int p = s * R + q;
            hs[q * (kMaxRestart + 1) + i] = flag[p] ? h[(int64_t)p * ldh + i] : 0.0;
        }
        __syncthreads();
        const int64_t r0 = a.unit_row[u], r1 = a.unit_row[u + 1];
        double acc[kRT];
#pragma unroll
        for (int q = 0; q < kRT; ++q) acc[q] = 0.0;
        for (int64_t r = r0 + threadIdx.x; r < r1; r += kNT) {
#pragma unroll
            for (int q = 0; q < kRT; ++q) {
                if (q < R && flag[s * R + q]) {
                    double xv = w[r * R + q];
                    for (int i = 0; i < nv; ++i) xv = fma(-hs[q * (kMaxRestart + 1) + i], a.V[((int64_t)i * a.n + r) * R + q], xv);
                    w[r * R + q] = xv;
                    acc[q] = fma(xv, xv, acc[q]);
                }
            }
        }
        block_sum_r(acc, sh);
        if (threadIdx.x < R) {
            const int q = threadIdx.x;
            if (flag[s * R + q]) a.part[((int64_t)u * stride) * R + q] = sh[4 * kRT + q];
        }
    }
}

// Per-pair Givens update of column j (= jc) with h1 (+ h2), Arnoldi norm hn.
__device__ void pair_finalize(const BatchArgs &a, int p, double hn, bool use_h2) {
    const int k = a.k;
    const int j = a.jc[p];
    double *H = a.H + ((int64_t)p * k + j) * (k + 1);
    double *h1 = a.h1 + (int64_t)p * (k + 2);
    double *h2 = a.h2 + (int64_t)p * (k + 2);
    double *cs = a.cs + (int64_t)p * k, *sn = a.sn + (int64_t)p * k;
    double *g = a.g + (int64_t)p * (k + 1);
    for (int i = 0; i <= j; ++i) H[i] = use_h2 ? h1[i] + h2[i] : h1[i];
    H[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double x0 = H[i], x1 = H[i + 1];
        H[i] = cs[i] * x0 + sn[i] * x1;
        H[i + 1] = -sn[i] * x0 + cs[i] * x1;
    }
    const double x0 = H[j], x1 = H[j + 1];
    const double den = hypot(x0, x1);
    double c = 1.0, sgn = 0.0;
    if (den != 0.0) {
        c = x0 / den;
        sgn = x1 / den;
    }
    cs[j] = c;
    sn[j] = sgn;
    H[j] = den;
    H[j + 1] = 0.0;
    g[j + 1] = -sgn * g[j];
    g[j] = c * g[j];
    a.jc[p] = j + 1;
    a.iters[p] += 1;
    a.est[p] = fabs(g[j + 1]) / a.nb[p];
    a.inv[p] = hn != 0.0 ? 1.0 / hn : 0.0;
    const bool stop = a.est[p] <= a.rtol || a.iters[p] >= a.maxit || hn == 0.0 || a.jc[p] >= k;
    if (stop) a.cyc[p] = 0;
}

// Build the per-system participation mask from a per-pair flag.
__device__ void phase_mask(const BatchArgs &a, const int *flag) {
    const int R = a.R;
    for (int s = blockIdx.x * kNT + threadIdx.x; s < a.nsys; s += gridDim.x * kNT) {
        unsigned m = 0;
        for (int q = 0; q < R; ++q)
            if (flag[s * R + q]) m |= 1u << q;
        a.sysmask[s] = (unsigned char)m;
    }
}

__device__ __forceinline__ bool first_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

// f(t, p) for every element t = row*R + q of the rows of system-unit blocks,
// p = the pair (system, q); one workgroup per unit, grid-strided.
template <class F> __device__ void for_elems(const BatchArgs &a, F f) {
    const int R = a.R;
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        const int64_t e0 = a.unit_row[u] * R, e1 = a.unit_row[u + 1] * R;
        for (int64_t t = e0 + threadIdx.x; t < e1; t += kNT) f(t, s * R + (int)(t % R));
    }
}

// ---------------------------------------------------------------------------
// The persistent kernel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT) void k_batched_gmres(BatchArgs a) {
    __shared__ double sh[5 * kRT];
    const int R = a.R;
    const int nR = a.n * R;
    const int gtid = blockIdx.x * kNT + threadIdx.x;
    const int gsz = gridDim.x * kNT;
    double *V0 = a.V;

    // ---- ||b|| per pair (V0 <- b) ----
    for (int t = gtid; t < nR; t += gsz) V0[t] = a.b[(int64_t)(t / R) * a.ld + t % R];
    for (int p = gtid; p < a.npairs; p += gsz) a.active[p] = 1;
    if (!grid_barrier(a)) return;
    phase_mask(a, a.active);
    if (!grid_barrier(a)) return;
    phase_dots(a, 0, V0, true, a.active, sh);
    if (!grid_barrier(a)) return;
    phase_reduce(a, 0, 1, a.active, a.nb, 1);
    if (!grid_barrier(a)) return;
    for (int p = gtid; p < a.npairs; p += gsz) {
        a.nb[p] = sqrt(a.nb[p]);
        a.iters[p] = 0;
        a.restarts[p] = 0;
        a.status[p] = SAIT_OK;
        a.est[p] = 0.0;
        a.beta[p] = 0.0;
        if (a.nb[p] == 0.0) a.active[p] = 0;  // b = 0: x = 0 below
    }
    if (!grid_barrier(a)) return;
    for_elems(a, [&](int64_t t, int p) {
        if (a.nb[p] == 0.0) a.x[(t / R) * a.ld + t % R] = 0.0;
    });
    if (!grid_barrier(a)) return;

    for (;;) {
        // ---- true residual r = b - A x into V0 for active pairs ----
        phase_mask(a, a.active);
        if (!grid_barrier(a)) return;
        phase_spmm(a, a.A, a.x, a.ld, V0, R, a.b, a.ld);
        if (!grid_barrier(a)) return;
        phase_dots(a, 0, V0, true, a.active, sh);
        if (!grid_barrier(a)) return;
        phase_reduce(a, 0, 1, a.active, a.beta, 1);
        if (first_thread()) {
            __hip_atomic_store(a.ctrl + 0, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!grid_barrier(a)) return;
        // ---- cycle start / exit decisions ----
        for (int p = gtid; p < a.npairs; p += gsz) {
            a.cyc[p] = 0;
            a.jc[p] = 0;
            if (!a.active[p]) continue;
            const double beta = sqrt(a.beta[p]);
            a.beta[p] = beta;
            const double rel = beta / a.nb[p];
            if (rel <= a.rtol) {
                a.active[p] = 0;
                a.status[p] = SAIT_OK;
            } else if (a.iters[p] >= a.maxit) {
                a.active[p] = 0;
                a.status[p] = SAIT_NOT_CONVERGED;
            } else {
                a.cyc[p] = 1;
                double *g = a.g + (int64_t)p * (a.k + 1);
                g[0] = beta;
                for (int i = 1; i <= a.k; ++i) g[i] = 0.0;
                a.inv[p] = 1.0 / beta;
                __hip_atomic_fetch_add(a.ctrl + 0, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (!grid_barrier(a)) return;
        if (ld_ctrl(a, 0) == 0) break;  // every pair converged or hit maxit
        phase_mask(a, a.cyc);
        for_elems(a, [&](int64_t t, int p) {
            if (a.cyc[p]) V0[t] *= a.inv[p];
        });
        if (!grid_barrier(a)) return;
        // ---- Arnoldi steps ----
        for (int j = 0; j < a.k; ++j) {
            double *vj = a.V + (int64_t)j * nR;
            double *w = a.V + (int64_t)(j + 1) * nR;
            phase_spmm(a, a.ML, vj, R, a.T, R, nullptr, 0);
            if (!grid_barrier(a)) return;
            phase_spmm(a, a.MU, a.T, R, a.Z, R, nullptr, 0);
            if (!grid_barrier(a)) return;
            phase_spmm(a, a.A, a.Z, R, w, R, nullptr, 0);
            if (!grid_barrier(a)) return;
            phase_dots(a, j + 1, w, true, a.cyc, sh);
            if (!grid_barrier(a)) return;
            phase_reduce(a, 0, j + 1, a.cyc, a.h1, a.k + 2);
            phase_reduce(a, j + 1, 1, a.cyc, a.wpre2, 1);  // ||w||^2 before the update
            if (!grid_barrier(a)) return;
            phase_update(a, j + 1, w, a.cyc, a.h1, a.k + 2, sh);
            if (first_thread()) __hip_atomic_store(a.ctrl + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!grid_barrier(a)) return;
            // norms after the update (partials at index 0), DGKS decision / finalize
            for (int p = gtid; p < a.npairs; p += gsz) {
                a.reorth[p] = 0;
                if (!a.cyc[p]) continue;
                const int s = p / R, q = p % R;
                double hn2 = 0.0;
                for (int u = a.sys_unit[s]; u < a.sys_unit[s + 1]; ++u) hn2 += a.part[((int64_t)u * (a.k + 2)) * R + q];
                if (hn2 < 0.5 * a.wpre2[p]) {
                    a.reorth[p] = 1;
                    __hip_atomic_fetch_add(a.ctrl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    pair_finalize(a, p, sqrt(hn2), false);
                }
            }
            if (!grid_barrier(a)) return;
            if (ld_ctrl(a, 1) > 0) {
                phase_mask(a, a.reorth);
                if (!grid_barrier(a)) return;
                phase_dots(a, j + 1, w, false, a.reorth, sh);
                if (!grid_barrier(a)) return;
                phase_reduce(a, 0, j + 1, a.reorth, a.h2, a.k + 2);
                if (!grid_barrier(a)) return;
                phase_update(a, j + 1, w, a.reorth, a.h2, a.k + 2, sh);
                if (!grid_barrier(a)) return;
                for (int p = gtid; p < a.npairs; p += gsz) {
                    if (!a.reorth[p]) continue;
                    const int s = p / R, q = p % R;
                    double hn2 = 0.0;
                    for (int u = a.sys_unit[s]; u < a.sys_unit[s + 1]; ++u) hn2 += a.part[((int64_t)u * (a.k + 2)) * R + q];
                    pair_finalize(a, p, sqrt(hn2), true);
                }
                if (!grid_barrier(a)) return;
            }
            // normalise v_{j+1} for pairs still in the cycle; count them
            if (first_thread()) __hip_atomic_store(a.ctrl + 0, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!grid_barrier(a)) return;
            for_elems(a, [&](int64_t t, int p) {
                if (a.cyc[p]) w[t] *= a.inv[p];
            });
            for (int p = gtid; p < a.npairs; p += gsz)
                if (a.cyc[p]) __hip_atomic_fetch_add(a.ctrl + 0, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            phase_mask(a, a.cyc);
            if (!grid_barrier(a)) return;
            if (ld_ctrl(a, 0) == 0) break;
        }
        // ---- cycle end: y = R^-1 g, U = V y, x += M U (pairs with jc > 0) ----
        for (int p = gtid; p < a.npairs; p += gsz) {
            const int jc = a.jc[p];
            a.cyc[p] = jc > 0 ? 1 : 0;
            const int k = a.k;
            const double *H = a.H + (int64_t)p * k * (k + 1);
            const double *g = a.g + (int64_t)p * (k + 1);
            double *y = a.y + (int64_t)p * k;
            for (int i = jc - 1; i >= 0; --i) {
                double sacc = g[i];
                for (int t = i + 1; t < jc; ++t) sacc -= H[(int64_t)t * (k + 1) + i] * y[t];
                const double d = H[(int64_t)i * (k + 1) + i];
                y[i] = d != 0.0 ? sacc / d : 0.0;
            }
            if (jc > 0) a.restarts[p] += 1;
        }
        if (!grid_barrier(a)) return;
        phase_mask(a, a.cyc);
        for_elems(a, [&](int64_t t, int p) {
            const int jc = a.jc[p];
            double acc = 0.0;
            const double *y = a.y + (int64_t)p * a.k;
            for (int i = 0; i < jc; ++i) acc = fma(y[i], a.V[(int64_t)i * nR + t], acc);
            a.U[t] = acc;
        });
        if (!grid_barrier(a)) return;
        phase_spmm(a, a.ML, a.U, R, a.T, R, nullptr, 0);
        if (!grid_barrier(a)) return;
        phase_spmm(a, a.MU, a.T, R, a.Z, R, nullptr, 0);
        if (!grid_barrier(a)) return;
        for_elems(a, [&](int64_t t, int p) {
            if (a.cyc[p]) a.x[(t / R) * a.ld + t % R] += a.Z[t];
        });
        if (!grid_barrier(a)) return;
    }
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================

struct BatchedSolver::Impl {
    DevBuf V, T, Z, U, part, pairs_i, pairs_d, ctrl, sysmask, units_s, units_r, sys_unit, sysptr, slsys;
    int64_t n = -1;
    int k = 0, R = 0, nunits = 0, npairs = 0;
};

BatchedSolver::BatchedSolver() : impl_(new Impl) {}
BatchedSolver::~BatchedSolver() { delete impl_; }

int BatchedSolver::solve(Allocator *al, const BatchedOps &ops, const double *b, double *x, int R, int64_t ld,
                         const sait_solve_opts &o, sait_solve_info *info, hipStream_t s) {
    const int64_t n = ops.A->n;
    const int nsys = (int)ops.sys_ptr.size() - 1;
    const int k = o.restart;
    if (R < 1 || R > kRT) fail(SAIT_E_INVALID, "batched solve supports 1..8 right-hand sides per call");
    if (k < 1 || k > kMaxRestart) fail(SAIT_E_INVALID, "batched solve supports restart lengths 1..64");
    if (o.maxit < 0 || !(o.rtol >= 0.0)) fail(SAIT_E_INVALID, "maxit must be >= 0 and rtol >= 0");
    if (o.flexible) fail(SAIT_E_INVALID, "the batched solve runs right-preconditioned GMRES (flexible = 0)");
    for (const DevCsr *M : {ops.A, ops.ML, ops.MU})
        if (M->precision != SAIT_F64 || M->nslices <= 0) fail(SAIT_E_INVALID, "batched solve needs FP64 factors");
    if (n * R >= INT32_MAX) fail(SAIT_E_INVALID, "batched solve: n * nrhs exceeds int32 indexing");
    Impl &I = *impl_;
    const int npairs = nsys * R;
    // reduction units: row ranges of at most kUnitRows inside one system
    std::vector<int> usys, sunit(nsys + 1, 0);
    std::vector<int64_t> urow;
    for (int sy = 0; sy < nsys; ++sy) {
        sunit[sy] = (int)usys.size();
        for (int64_t r = ops.sys_ptr[sy]; r < ops.sys_ptr[sy + 1]; r += kUnitRows) {
            usys.push_back(sy);
            urow.push_back(r);
        }
    }
    sunit[nsys] = (int)usys.size();
    urow.push_back(n);
    const int nunits = (int)usys.size();
    const int64_t nsl = (n + 63) / 64;
    std::vector<int> slsys(std::max<int64_t>(nsl, 1), 0);
    for (int64_t sl = 0, sy = 0; sl < nsl; ++sl) {
        while (sl * 64 >= ops.sys_ptr[sy + 1]) ++sy;
        slsys[sl] = (int)sy;
    }
    if (I.n != n || I.k != k || I.R != R || I.nunits != nunits) {
        I.V.alloc(al, sizeof(double) * (size_t)n * R * (k + 1));
        I.T.alloc(al, sizeof(double) * (size_t)n * R);
        I.Z.alloc(al, sizeof(double) * (size_t)n * R);
        I.U.alloc(al, sizeof(double) * (size_t)n * R);
        I.part.alloc(al, sizeof(double) * (size_t)nunits * (k + 2) * R);
        I.pairs_i.alloc(al, sizeof(int) * (size_t)npairs * 7);
        I.pairs_d.alloc(al, sizeof(double) * (size_t)npairs * (5 + (size_t)k * (k + 1) + 2 * k + (k + 1) + k + 2 * (k + 2)));
        I.ctrl.alloc(al, 64);
        I.sysmask.alloc(al, (size_t)nsys);
        I.units_s.alloc(al, sizeof(int) * (size_t)nunits);
        I.units_r.alloc(al, sizeof(int64_t) * (size_t)(nunits + 1));
        I.sys_unit.alloc(al, sizeof(int) * (size_t)(nsys + 1));
        I.sysptr.alloc(al, sizeof(int64_t) * (size_t)(nsys + 1));
        I.slsys.alloc(al, sizeof(int) * slsys.size());
        I.n = n;
        I.k = k;
        I.R = R;
        I.nunits = nunits;
        I.npairs = npairs;
    }
    SAIT_HIP(hipMemcpyAsync(I.units_s.as<void>(), usys.data(), sizeof(int) * usys.size(), hipMemcpyHostToDevice, s));
    SAIT_HIP(hipMemcpyAsync(I.units_r.as<void>(), urow.data(), sizeof(int64_t) * urow.size(), hipMemcpyHostToDevice, s));
    SAIT_HIP(hipMemcpyAsync(I.sys_unit.as<void>(), sunit.data(), sizeof(int) * sunit.size(), hipMemcpyHostToDevice, s));
    SAIT_HIP(hipMemcpyAsync(I.sysptr.as<void>(), ops.sys_ptr.data(), sizeof(int64_t) * ops.sys_ptr.size(),
                            hipMemcpyHostToDevice, s));
    SAIT_HIP(hipMemcpyAsync(I.slsys.as<void>(), slsys.data(), sizeof(int) * slsys.size(), hipMemcpyHostToDevice, s));
    SAIT_HIP(hipMemsetAsync(I.ctrl.as<void>(), 0, 64, s));
    SAIT_HIP(hipMemsetAsync(I.part.as<void>(), 0, sizeof(double) * (size_t)nunits * (k + 2) * R, s));

    BatchArgs a{};
    a.n = (int)n;
    a.nsys = nsys;
    a.R = R;
    a.k = k;
    a.maxit = o.maxit;
    a.rtol = o.rtol;
    a.nunits = nunits;
    a.npairs = npairs;
    a.sys_ptr = I.sysptr.as<int64_t>();
    auto view = [](const DevCsr *M) {
        SellView v;
        v.nslices = (int)M->nslices;
        v.sptr = M->sell_ptr.as<int64_t>();
        v.rp = M->rp.as<int>();
        v.sci = M->sell_ci.as<int>();
        v.sv = M->sell_v.as<double>();
        return v;
    };
    a.A = view(ops.A);
    a.ML = view(ops.ML);
    a.MU = view(ops.MU);
    a.slice_sys = I.slsys.as<int>();
    a.unit_sys = I.units_s.as<int>();
    a.unit_row = I.units_r.as<int64_t>();
    a.sys_unit = I.sys_unit.as<int>();
    a.b = b;
    a.x = x;
    a.ld = ld;
    a.V = I.V.as<double>();
    a.T = I.T.as<double>();
    a.Z = I.Z.as<double>();
    a.U = I.U.as<double>();
    a.part = I.part.as<double>();
    int *pi = I.pairs_i.as<int>();
    a.active = pi;
    a.cyc = pi + npairs;
    a.jc = pi + 2 * npairs;
    a.iters = pi + 3 * npairs;
    a.restarts = pi + 4 * npairs;
    a.status = pi + 5 * npairs;
    a.reorth = pi + 6 * npairs;
    double *pd = I.pairs_d.as<double>();
    a.nb = pd;
    a.beta = pd + npairs;
    a.est = pd + 2 * (size_t)npairs;
    a.inv = pd + 3 * (size_t)npairs;
    a.wpre2 = pd + 4 * (size_t)npairs;
    double *q = pd + 5 * (size_t)npairs;
    a.H = q;
    q += (size_t)npairs * k * (k + 1);
    a.cs = q;
    q += (size_t)npairs * k;
    a.sn = q;
    q += (size_t)npairs * k;
    a.g = q;
    q += (size_t)npairs * (k + 1);
    a.y = q;
    q += (size_t)npairs * k;
    a.h1 = q;
    q += (size_t)npairs * (k + 2);
    a.h2 = q;
    a.sysmask = I.sysmask.as<unsigned char>();
    int *ctrl = I.ctrl.as<int>();
    a.ctrl = ctrl;
    a.bar_count = reinterpret_cast<unsigned *>(ctrl + 4);
    a.bar_gen = reinterpret_cast<unsigned *>(ctrl + 5);
    a.abort = ctrl + 6;

    // co-resident grid
    int dev = 0, cus = 0, per_cu = 0;
    SAIT_HIP(hipGetDevice(&dev));
    SAIT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SAIT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched_gmres, kNT, 0));
    if (per_cu < 1) fail(SAIT_E_DEVICE, "batched solve kernel does not fit on a CU");
    const int grid = std::max(1, std::min(per_cu, 4) * cus);
    void *args[] = {&a};
    SAIT_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_batched_gmres), dim3(grid), dim3(kNT), args,
                                        0, s));
    std::vector<int> hi(7 * (size_t)npairs);
    std::vector<double> hd(5 * (size_t)npairs);
    int hctrl[8];
    SAIT_HIP(hipMemcpyAsync(hi.data(), pi, sizeof(int) * hi.size(), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipMemcpyAsync(hd.data(), pd, sizeof(double) * hd.size(), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipMemcpyAsync(hctrl, ctrl, sizeof(hctrl), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (hctrl[6]) fail(SAIT_E_DEVICE, "batched solve: grid barrier watchdog expired");
    int status = SAIT_OK;
    for (int p = 0; p < npairs; ++p) {
        const int st = hi[5 * (size_t)npairs + p];
        if (st != SAIT_OK) status = SAIT_NOT_CONVERGED;
        if (info) {
            info[p].iterations = hi[3 * (size_t)npairs + p];
            info[p].restarts = hi[4 * (size_t)npairs + p];
            info[p].status = st;
            info[p].est_relres = hd[2 * (size_t)npairs + p];
            const double nb = hd[p];
            info[p].true_relres = nb > 0.0 ? hd[(size_t)npairs + p] / nb : 0.0;
        }
    }
    return status;
}

}  // namespace sait
