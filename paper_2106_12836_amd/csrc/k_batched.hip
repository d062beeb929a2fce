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
// and rows of systems without a participating pair are skipped.  Inside the
// kernel every vector is n x RP (RP = R rounded up to a power of two), so one
// thread owns one (row, right-hand side) element and each vector phase
// streams contiguous memory.  Reductions are deterministic: per-unit partial
// sums in a fixed order (units are row ranges inside one system), then a
// fixed wave butterfly over the units of a system.
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

constexpr int kNT = 512;         // one 8-wave workgroup per CU
constexpr int kWaves = kNT / 64;
constexpr int kBarGroups = 16;   // first level of the grid barrier's arrival tree
constexpr int kRT = 8;           // right-hand sides per launch (R <= 8)
constexpr int kUnitRows = 2048;  // rows per reduction unit
constexpr int kMaxRestart = 64;
constexpr size_t kCtrlBytes = 4 * (128 + 32 * kBarGroups);
constexpr int kChunk = 16;       // basis vectors per sweep of the inner-product phase
constexpr int kSlots = 2 * kChunk + 2;  // partial sums per sweep: V.u, V.z, u.u, u.z
constexpr int kRounds = (2 * kMaxRestart + 2 + 63) / 64;  // per-lane registers of one pair's partials
constexpr int kXcdSlices = 64;   // sliced-ELL slices per XCD chunk of the SpMM phase

struct SellView {
    int nslices;
    const int64_t *sptr;
    const int *rp, *sci;
    const double *sv;
};

// Internal vectors (V blocks, T, Z, U, X, B) are n x RP row-major with RP the
// next power of two >= R; column q >= R is padding that stays zero.
struct BatchArgs {
    int n, nsys, R, k, maxit, nunits, npairs;
    double rtol;
    uint64_t wait_ticks;     // barrier watchdog, in ticks of the constant-rate wall clock
    const int64_t *sys_ptr;  // nsys + 1
    SellView A, ML, MU;
    const int *slice_sys;    // systems of the first and last row of every 64-row slice: [2 s], [2 s + 1]
    const int *unit_sys;     // nunits
    const int64_t *unit_row; // nunits + 1
    const int *sys_unit;     // nsys + 1
    const double *b;         // user right-hand sides (n x ld, R columns)
    double *x;               // user solution (n x ld, R columns)
    int64_t ld;
    double *V;               // (k+1) blocks of n*RP
    double *T, *Z, *W, *U, *X, *B;  // U aliases W (used only at a cycle end)
    double *part;            // nunits * (2k+2) * R
    // per pair
    int *active, *cyc, *jc, *iters, *restarts, *status;
    double *nb, *beta, *est, *rinv, *eor;
    double *Hraw, *Rr;       // k x (k+1) per pair: Arnoldi Hessenberg columns, and after the rotations
    double *cs, *sn, *g, *y, *s1, *ca, *cg;
    unsigned char *sysmask;  // per system: bit q = pair (s, q) takes part in the current phase
    unsigned char *slice_on; // per 64-row slice: some system in it has a participating pair
    int *ctrl;               // [0] some pair is (still) in the cycle
    unsigned *bar_count, *bar_gen, *bar_sub;  // bar_sub: kBarGroups counters, 128 bytes apart
    int *abort;
};

// ---------------------------------------------------------------------------
// Grid barrier (all workgroups are co-resident: cooperative launch).  One
// thread per workgroup arrives, first on the counter of its group
// (blockIdx % kBarGroups), the last of a group on the root counter, the last
// group bumps the generation that the others poll.  Each arrival is a release
// (it also orders the earlier read of the generation), each last arriver
// acquires before passing the count on, and the counters are reset before the
// releasing increment that follows them.  A wait longer than wait_ticks of
// the wall clock raises the abort flag; every workgroup then leaves the
// kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool grid_barrier(const BatchArgs &a) {
    __shared__ int bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(a.bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int grp = blockIdx.x % kBarGroups;
        const unsigned gsize = gridDim.x / kBarGroups + (grp < (int)(gridDim.x % kBarGroups) ? 1u : 0u);
        const unsigned ngroups = gridDim.x < (unsigned)kBarGroups ? gridDim.x : (unsigned)kBarGroups;
        unsigned *sc = a.bar_sub + 32 * grp;
        bool last = false;
        if (__hip_atomic_fetch_add(sc, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(sc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(a.bar_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == ngroups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(a.bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(a.bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                last = true;
            }
        }
        if (!last) {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(a.bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                if (wall_clock64() - t0 > a.wait_ticks) {
                    __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        bad = __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return bad == 0;
}

// Raise control flag i if cond holds for any lane of the wavefront (one store
// per wavefront).
__device__ __forceinline__ void raise_ctrl(const BatchArgs &a, int i, bool cond) {
    const unsigned long long m = __ballot(cond);
    if (m != 0 && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1)
        __hip_atomic_store(a.ctrl + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

__device__ __forceinline__ bool pair_on(const BatchArgs &a, const int *flag, int s, int q) {
    return q < a.R && flag[s * a.R + q] != 0;
}

// Fixed-order sum of sh[w * stride] over the kWaves wavefronts.
__device__ __forceinline__ double sum_waves(const double *sh, int stride) {
    double t = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t += sh[w * stride];
    return t;
}

// Sum over the lanes of a wavefront that share lane % RP.
template <int RP> __device__ __forceinline__ double wave_sum_by_col(double x) {
#pragma unroll
    for (int off = 32; off >= RP; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Column indices and values of lane l's entries in the 4-entry group that
// starts at grp (a multiple of 256: 16-byte aligned).  Indices: the lane's
// four together; FP64 values: two planes, entries 0-1 of the 64 lanes then
// entries 2-3.  Streamed once, so loaded non-temporally.
__device__ __forceinline__ void load_group(const SellView &M, int64_t grp, int l, int (&cols)[4],
                                           double (&vals)[4]) {
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const i32x4 c = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(M.sci + grp + 4 * l));
    const f64x2 v0 = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(M.sv + grp + 2 * l));
    const f64x2 v1 = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(M.sv + grp + 128 + 2 * l));
    cols[0] = c.x;
    cols[1] = c.y;
    cols[2] = c.z;
    cols[3] = c.w;
    vals[0] = v0.x;
    vals[1] = v0.y;
    vals[2] = v1.x;
    vals[3] = v1.y;
}

// ---------------------------------------------------------------------------
// SpMM on a sliced-ELL matrix: out[row][q] = sum_k v x[col][q]  (or
// bres[row][q] - that) for the rows of the slices flagged active.  One
// wavefront per 64-row slice, lane = row, entries in column order, separately
// rounded products and sums.  Slices go to XCDs in contiguous chunks of
// kXcdSlices so that the gathered neighbour rows stay in one XCD's L2.
// ---------------------------------------------------------------------------
template <int RP>
__device__ __forceinline__ void phase_spmm(const BatchArgs &a, const SellView &M, const double *xin, double *out,
                           const double *bres) {
    const int l = threadIdx.x & 63;
    const int xcd = blockIdx.x & 7;
    const int wx = (blockIdx.x >> 3) * kWaves + (threadIdx.x >> 6);  // wave rank inside the XCD
    const int wpx = (gridDim.x >> 3) * kWaves;                        // waves per XCD
    const int nchunks = (M.nslices + kXcdSlices - 1) / kXcdSlices;
    for (int it = wx;; it += wpx) {
        const int c = xcd + 8 * (it / kXcdSlices);
        if (c >= nchunks) break;
        const int s = c * kXcdSlices + it % kXcdSlices;
        if (s >= M.nslices) continue;
        if (a.slice_on[s] == 0) continue;
        // Every row of an active slice is computed: rows of systems without
        // a participating pair only read and write their own system's rows,
        // which no participating pair uses.
        const int row = s * 64 + l;
        const bool inb = row < a.n;
        const int len = inb ? M.rp[row + 1] - M.rp[row] : 0;
        const int64_t base = M.sptr[s];
        const int ngroups = (int)((M.sptr[s + 1] - base) >> 8);
        double acc[RP];
#pragma unroll
        for (int q = 0; q < RP; ++q) acc[q] = 0.0;
        // software pipeline: the indices and values of group gi + 1 are in
        // flight while the rows of x for group gi are gathered
        int cols[4] = {0, 0, 0, 0};
        double vals[4] = {0.0, 0.0, 0.0, 0.0};
        if (ngroups > 0) load_group(M, base, l, cols, vals);
        for (int gi = 0; gi < ngroups; ++gi) {
            int nc[4] = {0, 0, 0, 0};
            double nv[4] = {0.0, 0.0, 0.0, 0.0};
            if (gi + 1 < ngroups) load_group(M, base + (int64_t)(gi + 1) * 256, l, nc, nv);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (gi * 4 + j < len) {
                    const double *xr = xin + (int64_t)cols[j] * RP;
                    double xv[RP];
                    if constexpr (RP == 1) {
                        xv[0] = xr[0];
                    } else {
#pragma unroll
                        for (int q = 0; q < RP; q += 2) {
                            const double2 t = *reinterpret_cast<const double2 *>(xr + q);
                            xv[q] = t.x;
                            xv[q + 1] = t.y;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < RP; ++q) acc[q] = add_rn(acc[q], mul_rn(vals[j], xv[q]));
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cols[j] = nc[j];
                vals[j] = nv[j];
            }
        }
        if (inb) {
            double *o = out + (int64_t)row * RP;
            if (bres) {
                const double *br = bres + (int64_t)row * RP;
#pragma unroll
                for (int q = 0; q < RP; ++q) acc[q] = br[q] - acc[q];
            }
            if constexpr (RP == 1) {
                o[0] = acc[0];
            } else {
#pragma unroll
                for (int q = 0; q < RP; q += 2) *reinterpret_cast<double2 *>(o + q) = make_double2(acc[q], acc[q + 1]);
            }
        }
    }
}

// One sweep of the inner-product phase over the unit's elements owned by
// this thread: C basis vectors (vp), u, z, and u.u, u.z on the first sweep.
template <int RP, int C>
__device__ __forceinline__ void dots_sweep(const double *const (&vp)[kChunk], const double *uvec, const double *zvec,
                                           int64_t e0, int64_t e1, bool first, double (&av)[kChunk],
                                           double (&bv)[kChunk], double &cu, double &du) {
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kNT) {
        const double ue = uvec[e];
        const double ze = zvec ? zvec[e] : 0.0;
        if (first) {
            cu = fma(ue, ue, cu);
            du = fma(ue, ze, du);
        }
        double qv[C > 0 ? C : 1];
#pragma unroll
        for (int c = 0; c < C; ++c) qv[c] = vp[c][e];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            av[c] = fma(qv[c], ue, av[c]);
            bv[c] = fma(qv[c], ze, bv[c]);
        }
    }
}

// Per-unit partial inner products for the pairs whose flag is set, stored
// in part[u][idx][q]:
//   idx = i       (i < nq): V_i . u
//   idx = k + i   (i < nq): V_i . z      (z != nullptr)
//   idx = 2k              : u . u
//   idx = 2k + 1          : u . z      (z != nullptr)
// One workgroup per unit; each thread owns the elements
// e = threadIdx.x (mod kNT) of the unit, all of column q = threadIdx.x % RP.
// The basis is swept kChunk vectors at a time.
template <int RP>
__device__ __forceinline__ void phase_dots(const BatchArgs &a, int nq, const double *uvec, const double *zvec,
                                           const int *flag, double *sh) {
    const int k = a.k, P = 2 * k + 2;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nRP = (int64_t)a.n * RP;
    const int nch = nq > 0 ? (nq + kChunk - 1) / kChunk : 1;
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        if (a.sysmask[s] == 0) continue;
        const int64_t e0 = a.unit_row[u] * RP, e1 = a.unit_row[u + 1] * RP;
        for (int ch = 0; ch < nch; ++ch) {
            const int i0 = ch * kChunk;
            // this sweep covers basis vectors i0 .. i0 + cnt - 1; the count is
            // rounded up to a multiple of 4 with the last vector repeated, so
            // every load of a sweep is unconditional
            const int cnt = nq - i0 < kChunk ? nq - i0 : kChunk;
            const double *vp[kChunk];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) vp[c] = a.V + (int64_t)(i0 + c < nq ? i0 + c : (nq > 0 ? nq - 1 : 0)) * nRP;
            double av[kChunk], bv[kChunk], cu = 0.0, du = 0.0;
#pragma unroll
            for (int c = 0; c < kChunk; ++c) av[c] = bv[c] = 0.0;
            switch (cnt <= 0 ? 0 : (cnt + 3) >> 2) {
            case 0: dots_sweep<RP, 0>(vp, uvec, zvec, e0, e1, ch == 0, av, bv, cu, du); break;
            case 1: dots_sweep<RP, 4>(vp, uvec, zvec, e0, e1, ch == 0, av, bv, cu, du); break;
            case 2: dots_sweep<RP, 8>(vp, uvec, zvec, e0, e1, ch == 0, av, bv, cu, du); break;
            case 3: dots_sweep<RP, 12>(vp, uvec, zvec, e0, e1, ch == 0, av, bv, cu, du); break;
            default: dots_sweep<RP, 16>(vp, uvec, zvec, e0, e1, ch == 0, av, bv, cu, du); break;
            }
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) {
                const double v = sl < kChunk ? av[sl] : sl < 2 * kChunk ? bv[sl - kChunk] : sl == 2 * kChunk ? cu : du;
                const double t = wave_sum_by_col<RP>(v);
                if (l < RP) sh[(wv * kSlots + sl) * RP + l] = t;
            }
            __syncthreads();
            if (threadIdx.x < kSlots * RP) {
                const int sl = threadIdx.x / RP, q = threadIdx.x % RP;
                int idx;
                bool valid;
                if (sl < kChunk) {
                    idx = i0 + sl;
                    valid = idx < nq;
                } else if (sl < 2 * kChunk) {
                    idx = k + i0 + sl - kChunk;
                    valid = zvec != nullptr && i0 + sl - kChunk < nq;
                } else {
                    idx = sl == 2 * kChunk ? 2 * k : 2 * k + 1;
                    valid = ch == 0 && (sl == 2 * kChunk || zvec != nullptr);
                }
                if (valid && pair_on(a, flag, s, q))
                    a.part[((int64_t)u * P + idx) * a.R + q] = sum_waves(sh + sl * RP + q, kSlots * RP);
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Value held by lane idx % 64 in round idx / 64 of a per-lane array.
__device__ __forceinline__ double lane_get(const double (&r)[kRounds], int idx) {
    const int src = idx & 63;
    double v = 0.0;
#pragma unroll
    for (int rd = 0; rd < kRounds; ++rd) {
        const double t = __shfl(r[rd], src, 64);
        if ((idx >> 6) == rd) v = t;
    }
    return v;
}

// Sum over the units of system s of partial idx of pair (s, q): lanes take
// units, then a fixed butterfly (every lane gets the sum).
__device__ __forceinline__ double pair_sum_lanes(const BatchArgs &a, int s, int q, int idx) {
    const int P = 2 * a.k + 2;
    double acc = 0.0;
    for (int u = a.sys_unit[s] + (int)(threadIdx.x & 63); u < a.sys_unit[s + 1]; u += 64)
        acc += a.part[((int64_t)u * P + idx) * a.R + q];
    return wave_sum(acc);
}

// Same sum, computed serially in unit order by one lane.
__device__ __forceinline__ double pair_sum_serial(const BatchArgs &a, int s, int q, int idx) {
    const int P = 2 * a.k + 2;
    const int u1 = a.sys_unit[s + 1];
    const int64_t step = (int64_t)P * a.R;
    const double *pp = a.part + (int64_t)idx * a.R + q;
    double acc = 0.0;
    int u = a.sys_unit[s];
    for (; u + 4 <= u1; u += 4) {
        double t[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) t[c] = pp[(int64_t)(u + c) * step];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc += t[c];
    }
    for (; u < u1; ++u) acc += pp[(int64_t)u * step];
    return acc;
}

// ||b|| per pair (one wavefront per pair) and the per-pair initial state.
__device__ __forceinline__ void phase_init_pairs(const BatchArgs &a) {
    const int l = threadIdx.x & 63;
    const int gw = blockIdx.x * kWaves + (threadIdx.x >> 6), nw = gridDim.x * kWaves;
    for (int p = gw; p < a.npairs; p += nw) {
        const double nb = sqrt(pair_sum_lanes(a, p / a.R, p % a.R, 2 * a.k));
        if (l == 0) {
            a.nb[p] = nb;
            a.iters[p] = 0;
            a.restarts[p] = 0;
            a.status[p] = SAIT_OK;
            a.est[p] = 0.0;
            a.beta[p] = 0.0;
            if (nb == 0.0) a.active[p] = 0;  // b = 0: x = 0
        }
    }
}

// Cycle start (one wavefront per pair): beta = ||b - A x||, exit tests, g.
__device__ __forceinline__ void phase_cycle_start(const BatchArgs &a) {
    const int l = threadIdx.x & 63;
    const int k = a.k;
    const int gw = blockIdx.x * kWaves + (threadIdx.x >> 6), nw = gridDim.x * kWaves;
    for (int p = gw; p < a.npairs; p += nw) {
        bool start = false;
        if (a.active[p]) {
            const double beta = sqrt(pair_sum_lanes(a, p / a.R, p % a.R, 2 * k));
            if (beta / a.nb[p] <= a.rtol) {
                if (l == 0) {
                    a.active[p] = 0;
                    a.status[p] = SAIT_OK;
                }
            } else if (a.iters[p] >= a.maxit) {
                if (l == 0) {
                    a.active[p] = 0;
                    a.status[p] = SAIT_NOT_CONVERGED;
                }
            } else {
                start = true;
                double *g = a.g + (int64_t)p * (k + 1);
                for (int i = l; i <= k; i += 64) g[i] = i == 0 ? beta : 0.0;
            }
            if (l == 0) a.beta[p] = beta;
        }
        if (l == 0) {
            a.cyc[p] = start ? 1 : 0;
            a.jc[p] = 0;
        }
        raise_ctrl(a, 0, start && l == 0);
    }
}

// Step j of the delayed classical Gram-Schmidt Arnoldi process, per pair in
// the cycle (one wavefront per pair).  Inputs: the partials of phase_dots
// with u = u_j (the once-projected, unnormalised candidate for basis vector
// j, held in V_j) and z = A M u_j.  With a = Q^T u, b = Q^T z (Q = V_0..V_{j-1}),
// c = u.u, d = u.z:
//   rho = ||u - Q a|| = sqrt(c - a.a)          (rho = beta at j = 0)
//   column j-1 of the Hessenberg matrix: s1 + a over rows < j, rho at row j,
//   then its Givens rotation, the residual estimate and the stop tests;
//   e = q_j . z = (d - a.b) / rho,
//   s1 of column j = ([b; e] - H a) / rho, from the Arnoldi relation
//   A M Q = Q_j H, and the update coefficients of phase_update.
// At j = k only column k-1 is completed.
__device__ __forceinline__ void phase_finalize(const BatchArgs &a, int j) {
    const int l = threadIdx.x & 63;
    const int k = a.k, R = a.R, K1 = k + 1;
    const bool full = j < k;
    const int gw = blockIdx.x * kWaves + (threadIdx.x >> 6), nw = gridDim.x * kWaves;
    for (int p = gw; p < a.npairs; p += nw) {
        if (!a.cyc[p]) continue;
        const int s = p / R, q = p % R;
        double r[kRounds];
#pragma unroll
        for (int rd = 0; rd < kRounds; ++rd) {
            const int idx = l + 64 * rd;
            const bool need = idx < j || (full && idx >= k && idx < k + j) || (idx == 2 * k && j > 0) ||
                              (full && idx == 2 * k + 1);
            r[rd] = need ? pair_sum_serial(a, s, q, idx) : 0.0;
        }
        const double ai = l < j ? r[0] : 0.0;
        double rho = a.beta[p];
        double hcol = 0.0;  // column j-1, row l (rows < j)
        bool stop = false;
        if (j > 0) {
            const double r2 = lane_get(r, 2 * k) - wave_sum(ai * ai);
            rho = r2 > 0.0 ? sqrt(r2) : 0.0;
            const double *s1 = a.s1 + (int64_t)p * K1;
            hcol = l < j ? s1[l] + ai : 0.0;
            double *Hc = a.Hraw + ((int64_t)p * k + (j - 1)) * K1;
            if (l < j) Hc[l] = hcol;
            if (l == 0) Hc[j] = rho;
            // previous rotations applied to the column (all lanes carry the scalars)
            const double *cs = a.cs + (int64_t)p * k, *sn = a.sn + (int64_t)p * k;
            const double csl = l < j - 1 ? cs[l] : 0.0, snl = l < j - 1 ? sn[l] : 0.0;
            double carry = __shfl(hcol, 0, 64), mine = 0.0;
            for (int i = 0; i < j - 1; ++i) {
                const double hn = __shfl(hcol, i + 1, 64);
                const double ci = __shfl(csl, i, 64), si = __shfl(snl, i, 64);
                const double top = ci * carry + si * hn;
                carry = -si * carry + ci * hn;
                if (l == i) mine = top;
            }
            const double den = hypot(carry, rho);
            double c0 = 1.0, s0 = 0.0;
            if (den != 0.0) {
                c0 = carry / den;
                s0 = rho / den;
            }
            double *g = a.g + (int64_t)p * K1;
            const double gj = g[j - 1];
            const int it = a.iters[p] + 1;
            const double est = fabs(s0 * gj) / a.nb[p];
            double *Rc = a.Rr + ((int64_t)p * k + (j - 1)) * K1;
            if (l < j - 1) Rc[l] = mine;
            if (l == 0) {
                Rc[j - 1] = den;
                a.cs[(int64_t)p * k + j - 1] = c0;
                a.sn[(int64_t)p * k + j - 1] = s0;
                g[j] = -s0 * gj;
                g[j - 1] = c0 * gj;
                a.jc[p] = j;
                a.iters[p] = it;
                a.est[p] = est;
            }
            stop = est <= a.rtol || it >= a.maxit || rho == 0.0 || !full;
        }
        if (stop) {
            if (l == 0) a.cyc[p] = 0;
            continue;
        }
        // update coefficients of step j
        const double bt = lane_get(r, k + (l < j ? l : 0));
        const double bi = l < j ? bt : 0.0;
        const double d = lane_get(r, 2 * k + 1);
        const double e = (d - wave_sum(ai * bi)) / rho;
        const double eor = e / rho;
        double ha = 0.0;  // (H a) at row l; columns < j-1 from memory, j-1 from registers
        for (int m0 = 0; m0 < j; m0 += 8) {
            double hv[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int m = m0 + c;
                hv[c] = (m < j - 1 && l <= m + 1) ? a.Hraw[((int64_t)p * k + m) * K1 + l] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int m = m0 + c;
                const double am = __shfl(ai, m & 63, 64);
                const double hm = m == j - 1 ? (l < j ? hcol : (l == j ? rho : 0.0)) : hv[c];
                if (m < j) ha = fma(hm, am, ha);
            }
        }
        const double bz = l < j ? bi : (l == j ? e : 0.0);
        if (l <= j) a.s1[(int64_t)p * K1 + l] = (bz - ha) / rho;
        if (l < j) {
            a.ca[(int64_t)p * k + l] = ai;
            a.cg[(int64_t)p * k + l] = bi - eor * ai;
        }
        if (l == 0) {
            a.rinv[p] = 1.0 / rho;
            a.eor[p] = eor;
        }
        raise_ctrl(a, 0, l == 0);
    }
}

// Update of step j for the pairs still in the cycle:
//   V_j     <- (u - sum_i ca_i V_i) / rho                  (basis vector q_j)
//   V_{j+1} <- (z - (e/rho) u - sum_i cg_i V_i) / rho      (candidate u_{j+1})
// with u = V_j, z = W, i < j; one pass over the basis.
template <int RP> __device__ __forceinline__ void phase_update(const BatchArgs &a, int j, double *hs) {
    const int q = threadIdx.x & (RP - 1);
    const int k = a.k, R = a.R;
    const int64_t nRP = (int64_t)a.n * RP;
    double *uv = a.V + (int64_t)j * nRP, *un = a.V + (int64_t)(j + 1) * nRP;
    constexpr int H = kMaxRestart + 1;
    __shared__ double sc[2 * kRT];
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        bool any = false;
        for (int qq = 0; qq < R; ++qq) any |= a.cyc[s * R + qq] != 0;
        if (!any) continue;
        __syncthreads();
        for (int t = threadIdx.x; t < RP * j; t += kNT) {
            const int qq = t / j, i = t % j;
            const bool on = pair_on(a, a.cyc, s, qq);
            const int64_t pi = (int64_t)(s * R + qq) * k + i;
            hs[qq * H + i] = on ? a.ca[pi] : 0.0;
            hs[(RP + qq) * H + i] = on ? a.cg[pi] : 0.0;
        }
        if (threadIdx.x < RP) {
            const int qq = threadIdx.x;
            const bool on = pair_on(a, a.cyc, s, qq);
            sc[qq] = on ? a.rinv[s * R + qq] : 0.0;
            sc[RP + qq] = on ? a.eor[s * R + qq] : 0.0;
        }
        __syncthreads();
        if (!pair_on(a, a.cyc, s, q)) continue;
        const double *ha = hs + q * H, *hg = hs + (RP + q) * H;
        const double ri = sc[q], eo = sc[RP + q];
        const int64_t e0 = a.unit_row[u] * RP, e1 = a.unit_row[u + 1] * RP;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kNT) {
            const double ue = uv[e], ze = a.W[e];
            double sa = 0.0, sg = 0.0;
            int i = 0;
            for (; i + 16 <= j; i += 16) {
                double vv[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) vv[c] = a.V[(int64_t)(i + c) * nRP + e];
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    sa = fma(ha[i + c], vv[c], sa);
                    sg = fma(hg[i + c], vv[c], sg);
                }
            }
            for (; i + 4 <= j; i += 4) {
                double vv[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) vv[c] = a.V[(int64_t)(i + c) * nRP + e];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    sa = fma(ha[i + c], vv[c], sa);
                    sg = fma(hg[i + c], vv[c], sg);
                }
            }
            for (; i < j; ++i) {
                const double vv = a.V[(int64_t)i * nRP + e];
                sa = fma(ha[i], vv, sa);
                sg = fma(hg[i], vv, sg);
            }
            uv[e] = (ue - sa) * ri;
            un[e] = (ze - eo * ue - sg) * ri;
        }
    }
}

// Cycle end (one wavefront per pair): y = R^-1 g over the jc completed
// columns by column-oriented back substitution; cyc = (jc > 0).
__device__ __forceinline__ void phase_hsolve(const BatchArgs &a) {
    const int l = threadIdx.x & 63;
    const int k = a.k, K1 = k + 1;
    const int gw = blockIdx.x * kWaves + (threadIdx.x >> 6), nw = gridDim.x * kWaves;
    for (int p = gw; p < a.npairs; p += nw) {
        const int jc = a.jc[p];
        if (jc > 0) {
            const double *Rp = a.Rr + (int64_t)p * k * K1;
            double rhs = l < jc ? a.g[(int64_t)p * K1 + l] : 0.0, mine = 0.0;
            for (int i = jc - 1; i >= 0; --i) {
                const double rii = Rp[(int64_t)i * K1 + i];
                const double yi = rii != 0.0 ? __shfl(rhs, i, 64) / rii : 0.0;
                if (l == i) mine = yi;
                if (l < i) rhs = fma(-Rp[(int64_t)i * K1 + l], yi, rhs);
            }
            if (l < jc) a.y[(int64_t)p * k + l] = mine;
        }
        if (l == 0) {
            a.cyc[p] = jc > 0 ? 1 : 0;
            if (jc > 0) a.restarts[p] += 1;
        }
    }
}

// U = sum_{i < jc[p]} y[p][i] V_i on the rows of masked systems (0 for pairs
// outside the cycle and for padding columns).
template <int RP> __device__ __forceinline__ void phase_combine(const BatchArgs &a, double *hs) {
    const int q = threadIdx.x & (RP - 1);
    const int64_t nRP = (int64_t)a.n * RP;
    constexpr int H = kMaxRestart + 1;
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        if (a.sysmask[s] == 0) continue;
        __syncthreads();
        for (int t = threadIdx.x; t < RP * a.k; t += kNT) {
            const int qq = t / a.k, i = t % a.k;
            const int p = s * a.R + qq;
            hs[qq * H + i] = (pair_on(a, a.cyc, s, qq) && i < a.jc[p]) ? a.y[(int64_t)p * a.k + i] : 0.0;
        }
        __syncthreads();
        const int jc = pair_on(a, a.cyc, s, q) ? a.jc[s * a.R + q] : 0;
        const double *yq = hs + q * H;
        const int64_t e0 = a.unit_row[u] * RP, e1 = a.unit_row[u + 1] * RP;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kNT) {
            double acc = 0.0;
            int i = 0;
            for (; i + 8 <= jc; i += 8) {
                double vv[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) vv[c] = a.V[(int64_t)(i + c) * nRP + e];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc = fma(yq[i + c], vv[c], acc);
            }
            for (; i < jc; ++i) acc = fma(yq[i], a.V[(int64_t)i * nRP + e], acc);
            a.U[e] = acc;
        }
    }
}

// Build the per-system participation mask and the per-slice activity flag
// from a per-pair flag.
__device__ __forceinline__ void phase_mask(const BatchArgs &a, const int *flag) {
    const int R = a.R;
    for (int s = blockIdx.x * kNT + threadIdx.x; s < a.nsys; s += gridDim.x * kNT) {
        unsigned m = 0;
        for (int q = 0; q < R; ++q)
            if (flag[s * R + q]) m |= 1u << q;
        a.sysmask[s] = (unsigned char)m;
    }
    for (int sl = blockIdx.x * kNT + threadIdx.x; sl < a.A.nslices; sl += gridDim.x * kNT) {
        bool on = false;
        for (int sy = a.slice_sys[2 * sl]; sy <= a.slice_sys[2 * sl + 1] && !on; ++sy)
            for (int q = 0; q < R; ++q) on |= flag[sy * R + q] != 0;
        a.slice_on[sl] = on ? 1 : 0;
    }
}

__device__ __forceinline__ bool first_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }

// f(e, p) for every element e = row*RP + q (q < R) of the unit blocks of
// systems with a nonzero mask; p = the pair (system, q).
template <int RP, class F> __device__ __forceinline__ void for_elems(const BatchArgs &a, F f) {
    const int q = threadIdx.x & (RP - 1);
    if (q >= a.R) return;
    for (int u = blockIdx.x; u < a.nunits; u += gridDim.x) {
        const int s = a.unit_sys[u];
        if (a.sysmask[s] == 0) continue;
        const int p = s * a.R + q;
        const int64_t e0 = a.unit_row[u] * RP, e1 = a.unit_row[u + 1] * RP;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kNT) f(e, p);
    }
}

// ---------------------------------------------------------------------------
// The persistent kernel.
// ---------------------------------------------------------------------------
template <int RP> __global__ __launch_bounds__(kNT, 1) void k_batched_gmres(BatchArgs a) {
    __shared__ double sh[kWaves * kSlots * RP];
    __shared__ double hs[2 * kRT * (kMaxRestart + 1)];
    const int R = a.R, k = a.k;
    const int64_t nRP = (int64_t)a.n * RP;
    const int gtid = blockIdx.x * kNT + threadIdx.x;
    const int gsz = gridDim.x * kNT;
    double *V0 = a.V;

    // ---- internal copies of b and x0 (padding columns zero), ||b|| per pair ----
    for (int64_t t = gtid; t < nRP; t += gsz) {
        const int64_t r = t / RP;
        const int q = (int)(t % RP);
        a.B[t] = q < R ? a.b[r * a.ld + q] : 0.0;
        a.X[t] = q < R ? a.x[r * a.ld + q] : 0.0;
    }
    for (int p = gtid; p < a.npairs; p += gsz) a.active[p] = 1;
    if (!grid_barrier(a)) return;
    phase_mask(a, a.active);
    if (!grid_barrier(a)) return;
    phase_dots<RP>(a, 0, a.B, nullptr, a.active, sh);
    if (!grid_barrier(a)) return;
    phase_init_pairs(a);
    if (!grid_barrier(a)) return;
    for_elems<RP>(a, [&](int64_t e, int p) {
        if (a.nb[p] == 0.0) a.X[e] = 0.0;
    });
    if (!grid_barrier(a)) return;

    for (;;) {
        // ---- true residual u_0 = b - A x into V_0 for active pairs ----
        phase_mask(a, a.active);
        if (!grid_barrier(a)) return;
        phase_spmm<RP>(a, a.A, a.X, V0, a.B);
        if (!grid_barrier(a)) return;
        phase_dots<RP>(a, 0, V0, nullptr, a.active, sh);
        if (first_thread()) __hip_atomic_store(a.ctrl + 0, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!grid_barrier(a)) return;
        phase_cycle_start(a);
        if (!grid_barrier(a)) return;
        if (ld_ctrl(a, 0) == 0) break;  // every pair converged or hit maxit
        phase_mask(a, a.cyc);
        if (!grid_barrier(a)) return;
        // ---- Arnoldi steps; step k only completes column k-1 ----
        for (int j = 0; j <= k; ++j) {
            double *uj = a.V + (int64_t)j * nRP;
            const bool full = j < k;
            if (full) {
                phase_spmm<RP>(a, a.ML, uj, a.T, nullptr);
                if (!grid_barrier(a)) return;
                phase_spmm<RP>(a, a.MU, a.T, a.Z, nullptr);
                if (!grid_barrier(a)) return;
                phase_spmm<RP>(a, a.A, a.Z, a.W, nullptr);
                if (!grid_barrier(a)) return;
            }
            phase_dots<RP>(a, j, uj, full ? a.W : nullptr, a.cyc, sh);
            if (first_thread()) __hip_atomic_store(a.ctrl + 0, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!grid_barrier(a)) return;
            phase_finalize(a, j);
            if (!grid_barrier(a)) return;
            if (ld_ctrl(a, 0) == 0) break;
            phase_update<RP>(a, j, hs);
            phase_mask(a, a.cyc);
            if (!grid_barrier(a)) return;
        }
        // ---- cycle end: y = R^-1 g, U = V y, x += M U (pairs with jc > 0) ----
        phase_hsolve(a);
        if (!grid_barrier(a)) return;
        phase_mask(a, a.cyc);
        if (!grid_barrier(a)) return;
        phase_combine<RP>(a, hs);
        if (!grid_barrier(a)) return;
        phase_spmm<RP>(a, a.ML, a.U, a.T, nullptr);
        if (!grid_barrier(a)) return;
        phase_spmm<RP>(a, a.MU, a.T, a.Z, nullptr);
        if (!grid_barrier(a)) return;
        for_elems<RP>(a, [&](int64_t e, int p) {
            if (a.cyc[p]) a.X[e] += a.Z[e];
        });
        if (!grid_barrier(a)) return;
    }
    // ---- copy the iterate out ----
    for (int64_t t = gtid; t < nRP; t += gsz) {
        const int q = (int)(t % RP);
        if (q < R) a.x[(t / RP) * a.ld + q] = a.X[t];
    }
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================

constexpr int kPairInts = 6;  // active, cyc, jc, iters, restarts, status
// Doubles per pair: nb, beta, est, rinv, eor; Hraw, Rr; cs, sn, g, y, s1, ca, cg.
static size_t pair_doubles(int k) { return 5 + 2 * (size_t)k * (k + 1) + 7 * (size_t)k + 2; }

struct BatchedSolver::Impl {
    DevBuf V, T, Z, W, X, B, part, pairs_i, pairs_d, ctrl, sysmask, slice_on, units_s, units_r, sys_unit, sysptr, slsys;
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
    const int RP = R == 1 ? 1 : R == 2 ? 2 : R <= 4 ? 4 : 8;  // padded columns of the internal vectors
    if (n * RP >= INT32_MAX) fail(SAIT_E_INVALID, "batched solve: n * nrhs exceeds int32 indexing");
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
    std::vector<int> slsys(2 * std::max<int64_t>(nsl, 1), 0);
    for (int64_t sl = 0, sy = 0; sl < nsl; ++sl) {
        while (sl * 64 >= ops.sys_ptr[sy + 1]) ++sy;
        int64_t sz = sy;
        const int64_t last = std::min<int64_t>(sl * 64 + 63, n - 1);
        while (last >= ops.sys_ptr[sz + 1]) ++sz;
        slsys[2 * sl] = (int)sy;
        slsys[2 * sl + 1] = (int)sz;
    }
    if (I.n != n || I.k != k || I.R != R || I.nunits != nunits) {
        const size_t vec = sizeof(double) * (size_t)n * RP;
        I.V.alloc(al, vec * (k + 1));
        I.T.alloc(al, vec);
        I.Z.alloc(al, vec);
        I.W.alloc(al, vec);
        I.X.alloc(al, vec);
        I.B.alloc(al, vec);
        I.part.alloc(al, sizeof(double) * (size_t)nunits * (2 * k + 2) * R);
        I.pairs_i.alloc(al, sizeof(int) * (size_t)npairs * kPairInts);
        I.pairs_d.alloc(al, sizeof(double) * (size_t)npairs * pair_doubles(k));
        I.ctrl.alloc(al, kCtrlBytes);
        I.sysmask.alloc(al, (size_t)nsys);
        I.slice_on.alloc(al, (size_t)std::max<int64_t>(nsl, 1));
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
    SAIT_HIP(hipMemsetAsync(I.ctrl.as<void>(), 0, kCtrlBytes, s));
    SAIT_HIP(hipMemsetAsync(I.part.as<void>(), 0, sizeof(double) * (size_t)nunits * (2 * k + 2) * R, s));

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
    a.W = I.W.as<double>();
    a.U = a.W;
    a.X = I.X.as<double>();
    a.B = I.B.as<double>();
    a.part = I.part.as<double>();
    int *pi = I.pairs_i.as<int>();
    a.active = pi;
    a.cyc = pi + npairs;
    a.jc = pi + 2 * npairs;
    a.iters = pi + 3 * npairs;
    a.restarts = pi + 4 * npairs;
    a.status = pi + 5 * npairs;
    double *pd = I.pairs_d.as<double>();
    a.nb = pd;
    a.beta = pd + npairs;
    a.est = pd + 2 * (size_t)npairs;
    a.rinv = pd + 3 * (size_t)npairs;
    a.eor = pd + 4 * (size_t)npairs;
    double *q = pd + 5 * (size_t)npairs;
    auto take = [&](size_t per_pair) {
        double *r = q;
        q += (size_t)npairs * per_pair;
        return r;
    };
    a.Hraw = take((size_t)k * (k + 1));
    a.Rr = take((size_t)k * (k + 1));
    a.cs = take(k);
    a.sn = take(k);
    a.g = take(k + 1);
    a.y = take(k);
    a.s1 = take(k + 1);
    a.ca = take(k);
    a.cg = take(k);
    a.sysmask = I.sysmask.as<unsigned char>();
    a.slice_on = I.slice_on.as<unsigned char>();
    int *ctrl = I.ctrl.as<int>();
    a.ctrl = ctrl;
    // control words: flags at 0..1, barrier root at 32, generation at 64,
    // abort at 96, group counters from 128 on (each in its own 128-byte line)
    a.bar_count = reinterpret_cast<unsigned *>(ctrl + 32);
    a.bar_gen = reinterpret_cast<unsigned *>(ctrl + 64);
    a.abort = ctrl + 96;
    a.bar_sub = reinterpret_cast<unsigned *>(ctrl + 128);

    // co-resident grid: one workgroup per CU
    int dev = 0, cus = 0, per_cu = 0, clock_khz = 0;
    SAIT_HIP(hipGetDevice(&dev));
    SAIT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    SAIT_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
    a.wait_ticks = (uint64_t)std::max(clock_khz, 1) * 1000ull * 10ull;  // 10 s
    const void *kern = RP == 1   ? reinterpret_cast<const void *>(k_batched_gmres<1>)
                       : RP == 2 ? reinterpret_cast<const void *>(k_batched_gmres<2>)
                       : RP == 4 ? reinterpret_cast<const void *>(k_batched_gmres<4>)
                                 : reinterpret_cast<const void *>(k_batched_gmres<8>);
    SAIT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNT, 0));
    // The SpMM phase deals slices to the 8 XCDs (block b runs on XCD b % 8):
    // the grid is a multiple of 8 workgroups, all co-resident.
    const int grid = cus & ~7;
    if (per_cu < 1) fail(SAIT_E_DEVICE, "batched solve kernel does not fit on a CU");
    if (grid < 8) fail(SAIT_E_DEVICE, "batched solve kernel does not fit 8 co-resident workgroups");
    void *args[] = {&a};
    SAIT_HIP(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kNT), args, 0, s));
    std::vector<int> hi(kPairInts * (size_t)npairs);
    std::vector<double> hd(5 * (size_t)npairs);
    int hctrl[128];
    SAIT_HIP(hipMemcpyAsync(hi.data(), pi, sizeof(int) * hi.size(), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipMemcpyAsync(hd.data(), pd, sizeof(double) * hd.size(), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipMemcpyAsync(hctrl, ctrl, sizeof(hctrl), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (hctrl[96]) fail(SAIT_E_DEVICE, "batched solve: grid barrier watchdog expired");
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
