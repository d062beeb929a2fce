// Restarted right-preconditioned GMRES(k) / FGMRES(k) on the device, the
// iterative method the SAIT preconditioner is applied inside (Sec. 3.1,
// Sec. 3.2 Eq. runtime: each iteration is one preconditioner application
// comp(M_L, M_U) plus "othercomp": an operator product, inner products and
// vector updates).
//
// Everything is FP64 and stays on the device: the Krylov basis V (and the
// preconditioned vectors for FGMRES), the inner products, the Hessenberg
// matrix with its Givens rotations and the true residual.  The Arnoldi
// process is classical Gram-Schmidt with delayed re-orthogonalisation
// (dcgs2_finalize): one step is
//   z = M u_j, w = A z                    (SAIT apply, any storage precision)
//   one pass: V^T u, V^T w, u.u, u.w      (k_dots2, per-block partials)
//   one block: sums, column j-1 of H and the coefficients (k_dots2_fin)
//   one pass: q_j and u_{j+1}             (k_update2)
// Reductions are deterministic: each block writes a partial and a one-block
// kernel sums the partials in a fixed order.  A second launch costs less
// than an atomic ticket taken by every block of the pass (the ticket's
// agent-scope release writes back each XCD's L2 once per block: measured
// 15.8 against 8.5 us for a 2-vector pass over 2^21 rows in 512 blocks).  Every
// Krylov kernel of an Arnoldi step starts by reading the `done` flag; the
// preconditioner and operator products do not, so each of the (at most
// three) steps enqueued after convergence still costs those products.  The
// host keeps a few steps queued ahead and polls a pinned, device-written
// mailbox to stop enqueueing.  The host synchronises once per restart cycle, to read the
// true residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "sait_internal.h"
#include "solver.h"

namespace sait {

namespace {

constexpr int kNT = 256;

struct Mailbox {
    int done;
    int iters;
    double est;
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Sum of x over the block (fixed order); result valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double *sh) {
    x = wave_sum(x);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// Sum of part[0 .. B) in a fixed order (one block; the result is valid in
// thread 0): thread t adds the partials t, t + kNT, ... in turn, then the
// block sum.
__device__ double sum_partials(const double *part, int B, double *sh) {
    double s = 0.0;
    for (int b = threadIdx.x; b < B; b += kNT) s += part[b];
    return block_sum(s, sh);
}

struct Rows {
    int64_t lo, hi;
};
__device__ __forceinline__ Rows block_rows(int64_t n, int B) {
    const int64_t chunk = ((n + B - 1) / B + kNT - 1) / kNT * kNT;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    return {lo, lo + chunk < n ? lo + chunk : n};
}

// One Arnoldi step in delayed classical Gram-Schmidt form.  V_j holds u_j,
// the once-projected (unnormalised) candidate for basis vector j; z = M u_j
// and w = A z are in hand.  One pass over the basis gives
//   a = Q^T u, b = Q^T w (Q = V_0 .. V_{j-1}), c = u.u, d = u.w,
// then (one block):
//   rho = ||u - Q a|| = sqrt(c - a.a)                 (beta at j = 0)
//   column j-1 of the Hessenberg matrix: s1 + a over rows < j, rho at row j,
//   its Givens rotation, the residual estimate and the stop decision;
//   e = q_j . w = (d - a.b) / rho, and from the Arnoldi relation
//   A M Q = Q_j H the first projection of column j, s1 = ([b; e] - H a) / rho;
// and the update pass writes
//   q_j = (u - Q a) / rho,   u_{j+1} = (w - (e/rho) u - Q (b - (e/rho) a)) / rho.
// FGMRES keeps z~_j = M u_j: with z_j the vectors that satisfy A Z = Q_{j+1} H,
// z~_j = sum_{i<j} a_i z_i + rho z_j, i.e. Z~ = Z Gamma with Gamma upper
// triangular (column j: a, rho), so the cycle's update is x += Z~ (Gamma^-1 y).
// Step j = k only completes column k-1.
__device__ void dcgs2_finalize(GmresDev *st, int j, bool full, Mailbox *mb, double *sh) {
    const int k = st->restart, K1 = k + 1;
    const double *red = st->red;
    const double c = red[2 * k], d = red[2 * k + 1];
    __shared__ double rho_s, e_s;
    __shared__ int stop_s;
    // a.a and a.b over the block (fixed order)
    double aa = 0.0, ab = 0.0;
    for (int i = threadIdx.x; i < j; i += kNT) {
        aa = fma(red[i], red[i], aa);
        if (full) ab = fma(red[i], red[k + i], ab);
    }
    aa = block_sum(aa, sh);
    ab = block_sum(ab, sh);
    if (threadIdx.x == 0) {
        double rho = st->beta;
        if (j > 0) {
            const double r2 = c - aa;
            rho = r2 > 0.0 ? sqrt(r2) : 0.0;
        }
        rho_s = rho;
        e_s = (full && rho != 0.0) ? (d - ab) / rho : 0.0;
        stop_s = 0;
    }
    __syncthreads();
    const double rho = rho_s;
    if (j > 0) {
        double *Hc = st->Hraw + (size_t)(j - 1) * K1;
        double *Rc = st->R + (size_t)(j - 1) * K1;
        for (int i = threadIdx.x; i < j; i += kNT) Hc[i] = st->s1[i] + red[i];
        if (threadIdx.x == 0) Hc[j] = rho;
        __syncthreads();
        // previous rotations applied to the column, 64 rows at a time through
        // LDS (the rotation chain itself is sequential: thread 0)
        __shared__ double cs_s[64], sn_s[64], col_s[65];
        double carry = 0.0;
        for (int i0 = 0; i0 + 1 < j || i0 == 0; i0 += 64) {
            const int m = (j - 1 - i0) < 64 ? (j - 1 - i0) : 64;  // rotations i0 .. i0+m-1
            if (threadIdx.x < 64) {
                const int i = i0 + threadIdx.x;
                cs_s[threadIdx.x] = threadIdx.x < m ? st->cs[i] : 0.0;
                sn_s[threadIdx.x] = threadIdx.x < m ? st->sn[i] : 0.0;
                col_s[threadIdx.x + 1] = (threadIdx.x < m) ? Hc[i + 1] : 0.0;
            }
            if (threadIdx.x == 0) col_s[0] = i0 == 0 ? Hc[0] : carry;
            __syncthreads();
            if (threadIdx.x == 0) {
                double c0 = col_s[0];
                for (int t = 0; t < m; ++t) {
                    const double x1 = col_s[t + 1];
                    col_s[t] = cs_s[t] * c0 + sn_s[t] * x1;
                    c0 = -sn_s[t] * c0 + cs_s[t] * x1;
                }
                carry = c0;
                col_s[64] = c0;
            }
            __syncthreads();
            if (threadIdx.x < m) Rc[i0 + threadIdx.x] = col_s[threadIdx.x];
            carry = col_s[64];
            __syncthreads();
            if (m < 64) break;
        }
        if (threadIdx.x == 0) {
            const double x0 = j == 1 ? Hc[0] : carry, x1 = rho;
            const double den = hypot(x0, x1);
            double cc = 1.0, ss = 0.0;
            if (den != 0.0) {
                cc = x0 / den;
                ss = x1 / den;
            }
            st->cs[j - 1] = cc;
            st->sn[j - 1] = ss;
            Rc[j - 1] = den;
            Rc[j] = 0.0;
            st->g[j] = -ss * st->g[j - 1];
            st->g[j - 1] = cc * st->g[j - 1];
            st->jc = j;
            st->iters += 1;
            st->est = fabs(st->g[j]) / st->nb;
            const bool stop = st->est <= st->rtol || st->iters >= st->maxit || rho == 0.0 || !full;
            stop_s = stop ? 1 : 0;
            st->done = stop_s;
            if (mb) {
                mb->est = st->est;
                mb->iters = st->iters;
                __threadfence_system();
                __hip_atomic_store(&mb->done, st->done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
        if (stop_s) return;
    }
    // coefficients of step j (j < k here)
    const double e = e_s, eor = e / rho;
    for (int i = threadIdx.x; i <= j; i += kNT) {
        // (H a)_i over the completed columns m < j (column m has rows <= m+1);
        // the column loads are issued 8 at a time
        double ha = 0.0;
        for (int m0 = (i > 0 ? i - 1 : 0); m0 < j; m0 += 8) {
            double hv[8], av[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int m = m0 + c;
                hv[c] = m < j ? st->Hraw[(size_t)m * K1 + i] : 0.0;
                av[c] = m < j ? red[m] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) ha = fma(hv[c], av[c], ha);
        }
        const double bz = i < j ? red[k + i] : e;
        st->s1n[i] = (bz - ha) / rho;
    }
    for (int i = threadIdx.x; i < j; i += kNT) {
        st->ca[i] = red[i];
        st->cg[i] = red[k + i] - eor * red[i];
    }
    if (st->Gam) {
        double *Gc = st->Gam + (size_t)j * k;
        for (int i = threadIdx.x; i < j; i += kNT) Gc[i] = red[i];
        if (threadIdx.x == 0) Gc[j] = rho;
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += kNT) st->s1[i] = st->s1n[i];
    if (threadIdx.x == 0) {
        st->rinv = 1.0 / rho;
        st->eor = eor;
    }
}

// One sweep of the inner-product pass over rows [lo, hi) of this thread,
// two rows per iteration (all their loads issued together): C basis
// vectors (vp), u, w (may be null), and u.u, u.w on the first sweep.  The
// basis vectors are read once per pass with streaming (nontemporal) loads,
// which leaves the caches to u and w, read again by every group of 8
// (and by the update pass); C3 FGMRES(40): 69.0 -> 67.5 ms in FP64.
template <int C>
__device__ __forceinline__ void dots_rows(const double *const (&vp)[8], const double *u, const double *w, int64_t lo,
                                          int64_t hi, bool first, double (&av)[8], double (&bv)[8], double &cu,
                                          double &du) {
    for (int64_t r0 = lo + threadIdx.x; r0 < hi; r0 += 2 * kNT) {
        double ue[2], we[2], qv[2][C > 0 ? C : 1];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int64_t r = r0 + t * kNT;
            const bool ok = r < hi;
            ue[t] = ok ? u[r] : 0.0;
            we[t] = (ok && w) ? w[r] : 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) qv[t][c] = ok ? __builtin_nontemporal_load(vp[c] + r) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (first) {
                cu = fma(ue[t], ue[t], cu);
                du = fma(ue[t], we[t], du);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                av[c] = fma(qv[t][c], ue[t], av[c]);
                bv[c] = fma(qv[t][c], we[t], bv[c]);
            }
        }
    }
}

// Partial inner products of one Arnoldi step (nq = j basis vectors, u = V_j,
// w = A M u_j or null at the closing step), per block into part[idx * B +
// block] with idx = i (V_i.u), k + i (V_i.w), 2k (u.u), 2k + 1 (u.w).
__global__ __launch_bounds__(kNT) void k_dots2(int64_t n, const double *__restrict__ V, int64_t ldv, int nq,
                                               const double *__restrict__ u, const double *__restrict__ w,
                                               const GmresDev *st, double *part) {
    constexpr int kSl = 18;
    __shared__ double sh[4 * kSl];
    if (st->done) return;
    const int k = st->restart;
    const int B = gridDim.x;
    const Rows Rw = block_rows(n, B);
    const int nch = nq > 0 ? (nq + 7) / 8 : 1;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int ch = 0; ch < nch; ++ch) {
        const int i0 = ch * 8;
        const int cnt = nq - i0 < 8 ? nq - i0 : 8;
        const double *vp[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) vp[c] = V + (int64_t)(i0 + c < nq ? i0 + c : (nq > 0 ? nq - 1 : 0)) * ldv;
        double av[8], bv[8], cu = 0.0, du = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) av[c] = bv[c] = 0.0;
        switch (cnt <= 0 ? 0 : (cnt + 3) >> 2) {
        case 0: dots_rows<0>(vp, u, w, Rw.lo, Rw.hi, ch == 0, av, bv, cu, du); break;
        case 1: dots_rows<4>(vp, u, w, Rw.lo, Rw.hi, ch == 0, av, bv, cu, du); break;
        default: dots_rows<8>(vp, u, w, Rw.lo, Rw.hi, ch == 0, av, bv, cu, du); break;
        }
#pragma unroll
        for (int sl = 0; sl < kSl; ++sl) {
            const double v = sl < 8 ? av[sl] : sl < 16 ? bv[sl - 8] : sl == 16 ? cu : du;
            const double t = wave_sum(v);
            if (lane == 0) sh[wv * kSl + sl] = t;
        }
        __syncthreads();
        if (threadIdx.x < kSl) {
            const int sl = threadIdx.x;
            int idx = -1;
            if (sl < 8) {
                if (i0 + sl < nq) idx = i0 + sl;
            } else if (sl < 16) {
                if (w && i0 + sl - 8 < nq) idx = k + i0 + sl - 8;
            } else if (ch == 0 && (sl == 16 || w)) {
                idx = sl == 16 ? 2 * k : 2 * k + 1;
            }
            if (idx >= 0)
                part[(size_t)idx * B + blockIdx.x] = (sh[sl] + sh[kSl + sl]) + (sh[2 * kSl + sl] + sh[3 * kSl + sl]);
        }
        __syncthreads();
    }
}

// The sums of k_dots2's partials over its B blocks (in block order) and
// dcgs2_finalize; one block.  full: w was present (not the closing step).
__global__ __launch_bounds__(kNT) void k_dots2_fin(int nq, int full, int B, GmresDev *st, const double *part,
                                                   Mailbox *mb) {
    __shared__ double sh[8];
    if (st->done) return;
    const int k = st->restart;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // each wavefront reduces 4 values at a time: lanes take blocks (all loads
    // of the 4 values in flight together), then a fixed butterfly per value
    const int nvals = 2 * nq + 2;
    auto value_index = [&](int v) {
        if (v < nq) return v;
        if (v < 2 * nq) return k + v - nq;
        return v == 2 * nq ? 2 * k : 2 * k + 1;
    };
    for (int v0 = 4 * wv; v0 < nvals; v0 += 4 * (kNT / 64)) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b0 = 0; b0 < B; b0 += 8 * 64) {
            double x[4][8];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int idx = v0 + g < nvals ? value_index(v0 + g) : 0;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int b = b0 + c * 64 + lane;
                    x[g][c] = b < B ? part[(size_t)idx * B + b] : 0.0;
                }
            }
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int c = 0; c < 8; ++c) t[g] += x[g][c];
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const double tv = wave_sum(t[g]);
            if (lane == 0 && v0 + g < nvals) {
                const int idx = value_index(v0 + g);
                if (full || !(idx == 2 * k + 1 || (idx >= k && idx < 2 * k))) st->red[idx] = tv;
            }
        }
    }
    if (!full && threadIdx.x == 0) st->red[2 * k + 1] = 0.0;
    __syncthreads();
    dcgs2_finalize(st, nq, full != 0, mb, sh);
}

// Update of step j (skipped once the cycle is done):
//   V_j <- (u - sum_i ca_i V_i) / rho,   V_{j+1} <- (w - (e/rho) u - sum_i cg_i V_i) / rho
// with u = V_j, w = V_{j+1} on entry, i < j; coefficients staged 64 at a time.
__global__ __launch_bounds__(kNT) void k_update2(int64_t n, double *__restrict__ V, int64_t ldv, int j,
                                                 const GmresDev *st) {
    __shared__ double ca[64], cg[64];
    if (st->done) return;
    const double ri = st->rinv, eo = st->eor;
    double *uv = V + (int64_t)j * ldv, *wv = V + (int64_t)(j + 1) * ldv;
    const int B = gridDim.x;
    const Rows Rw = block_rows(n, B);
    const int nch = j > 0 ? (j + 63) / 64 : 1;
    for (int ch = 0; ch < nch; ++ch) {
        const int i0 = ch * 64;
        const int m = j - i0 < 64 ? j - i0 : 64;
        __syncthreads();
        if (threadIdx.x < 64) {
            ca[threadIdx.x] = threadIdx.x < m ? st->ca[i0 + threadIdx.x] : 0.0;
            cg[threadIdx.x] = threadIdx.x < m ? st->cg[i0 + threadIdx.x] : 0.0;
        }
        __syncthreads();
        const bool first = ch == 0, last = ch == nch - 1;
        const double *Q = V + (int64_t)i0 * ldv;
        for (int64_t r = Rw.lo + threadIdx.x; r < Rw.hi; r += kNT) {
            const double ue = uv[r];
            double we = wv[r];
            if (first) we = fma(-eo, ue, we);
            double sa = 0.0, sg = 0.0;
            int i = 0;
            for (; i + 8 <= m; i += 8) {
                double q[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) q[c] = __builtin_nontemporal_load(Q + (int64_t)(i + c) * ldv + r);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    sa = fma(ca[i + c], q[c], sa);
                    sg = fma(cg[i + c], q[c], sg);
                }
            }
            for (; i < m; ++i) {
                const double q = Q[(int64_t)i * ldv + r];
                sa = fma(ca[i], q, sa);
                sg = fma(cg[i], q, sg);
            }
            if (last) {
                uv[r] = (ue - sa) * ri;
                wv[r] = (we - sg) * ri;
            } else {
                uv[r] = ue - sa;
                wv[r] = we - sg;
            }
        }
    }
}

// Partials of ||r||^2 per block (k_cycle_norm_fin sums them).
__global__ __launch_bounds__(kNT) void k_cycle_norm(int64_t n, const double *__restrict__ r, double *part) {
    __shared__ double sh[4];
    const Rows R = block_rows(n, gridDim.x);
    double a = 0;
    for (int64_t i = R.lo + threadIdx.x; i < R.hi; i += kNT) a = fma(r[i], r[i], a);
    const double s = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ||r|| from the B partials (one block).  mode 0: r = b (sets ||b||);
// mode 1: r is the residual in V[0]: beta, g = beta e_1, jc = 0, done
// unless more iterations are needed.
__global__ __launch_bounds__(kNT) void k_cycle_norm_fin(int B, GmresDev *st, int mode, const double *part,
                                                        Mailbox *mb) {
    __shared__ double sh[4];
    const double ss = sum_partials(part, B, sh);
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(ss);
    if (mode == 0) {
        st->nb = nrm;
        return;
    }
    st->beta = nrm;
    st->g[0] = nrm;
    for (int i = 1; i <= st->restart; ++i) st->g[i] = 0.0;
    st->jc = 0;
    const bool ok = st->nb == 0.0 || nrm / st->nb <= st->rtol;
    st->done = (ok || st->iters >= st->maxit) ? 1 : 0;
    if (mb) {
        mb->iters = st->iters;
        __threadfence_system();
        __hip_atomic_store(&mb->done, st->done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Column-oriented back substitution T u = rhs for an upper triangular T
// (column i at T + i * ldt) over n rows; rhs in LDS, solution into u.
__device__ void back_substitute(const double *T, int64_t ldt, int n, double *rhs, double *u) {
    for (int i = n - 1; i >= 0; --i) {
        const double d = T[(int64_t)i * ldt + i];
        const double ui = d != 0.0 ? rhs[i] / d : 0.0;
        for (int t = threadIdx.x; t < i; t += blockDim.x) rhs[t] = fma(-T[(int64_t)i * ldt + t], ui, rhs[t]);
        if (threadIdx.x == 0) u[i] = ui;
        __syncthreads();
    }
}

// y = R^-1 g over the jc completed steps; for FGMRES also yh = Gamma^-1 y
// (one block).
__global__ __launch_bounds__(kNT) void k_hsolve(GmresDev *st) {
    __shared__ double rhs[1024];
    const int k = st->restart, jc = st->jc;
    for (int t = threadIdx.x; t < jc; t += kNT) rhs[t] = st->g[t];
    __syncthreads();
    back_substitute(st->R, k + 1, jc, rhs, st->y);
    if (!st->Gam) return;
    for (int t = threadIdx.x; t < jc; t += kNT) rhs[t] = st->y[t];
    __syncthreads();
    back_substitute(st->Gam, k, jc, rhs, st->yh);
}

// out (+)= sum_{i < jc} c_i B_i with c = y (GMRES) or yh (FGMRES)
__global__ void k_combine(int64_t n, const double *__restrict__ Bv, int64_t ldb, const GmresDev *st,
                          double *__restrict__ out, int accumulate) {
    __shared__ double ys[64];
    const int jc = st->jc;
    const double *yc = st->Gam ? st->yh : st->y;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r - threadIdx.x < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int i0 = 0; i0 < jc; i0 += 64) {
            const int m = jc - i0 < 64 ? jc - i0 : 64;
            __syncthreads();
            if (threadIdx.x < m) ys[threadIdx.x] = yc[i0 + threadIdx.x];
            __syncthreads();
            if (r < n)
                for (int i = 0; i < m; ++i) acc = fma(ys[i], Bv[(int64_t)(i0 + i) * ldb + r], acc);
        }
        if (r < n) out[r] = accumulate ? out[r] + acc : acc;
    }
}

__global__ void k_axpy_inplace(int64_t n, double *__restrict__ x, const double *__restrict__ z) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        x[r] += z[r];
}

__global__ void k_copy_strided(int64_t n, const double *__restrict__ src, int64_t lds, double *__restrict__ dst,
                               int64_t ldd) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        dst[r * ldd] = src[r * lds];
}

__global__ void k_init_state(GmresDev *st, int restart, int maxit, double rtol) {
    st->restart = restart;
    st->maxit = maxit;
    st->rtol = rtol;
    st->iters = 0;
    st->done = 0;
    st->jc = 0;
    st->nb = 0.0;
}

// ---------------------------------------------------------------------------
// Preconditioned conjugate gradients (textbook form; the solver of the
// paper's experiments, Sec. 4):
//   r = b - A x, z = M r, p = z; per iteration q = A p,
//   alpha = (r, z) / (p, q), x += alpha p, r -= alpha q, stop once
//   ||r|| / ||b|| <= rtol, z = M r, beta = (r, z)_new / (r, z)_old,
//   p = z + beta p.
// Each PCG kernel reads `done` first (the preconditioner and operator
// products do not); the reductions are per-block partials summed in block
// order by a one-block kernel (k_pcg_fin).
// ---------------------------------------------------------------------------

// Partial sums of x.y (and u.w if u) of the block's rows into part[0 / 1][blk].
// check_done: skip once the iteration has stopped.
__global__ __launch_bounds__(kNT) void k_pcg_dots(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ u, const double *__restrict__ w,
                                                  const PcgDev *st, int check_done, double *part) {
    __shared__ double sh[4];
    if (check_done && st->done) return;
    const int B = gridDim.x;
    const Rows R = block_rows(n, B);
    double a = 0.0, c = 0.0;
    for (int64_t r = R.lo + threadIdx.x; r < R.hi; r += kNT) {
        a = fma(x[r], y[r], a);
        if (u) c = fma(u[r], w[r], c);
    }
    a = block_sum(a, sh);
    if (u) c = block_sum(c, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        if (u) part[B + blockIdx.x] = c;
    }
}

// p = z (first) or p = z + beta p
__global__ void k_pcg_dir(int64_t n, const double *__restrict__ z, double *__restrict__ p, const PcgDev *st,
                          int first) {
    if (st->done) return;
    const double beta = first ? 0.0 : st->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = first ? z[i] : fma(beta, p[i], z[i]);
}

// x += alpha p, r -= alpha q, partials of ||r||^2
__global__ __launch_bounds__(kNT) void k_pcg_xr(int64_t n, const double *__restrict__ p, const double *__restrict__ q,
                                                double *__restrict__ x, double *__restrict__ r, const PcgDev *st,
                                                double *part) {
    __shared__ double sh[4];
    if (st->done) return;
    const double alpha = st->alpha;
    const Rows R = block_rows(n, gridDim.x);
    double a = 0.0;
    for (int64_t i = R.lo + threadIdx.x; i < R.hi; i += kNT) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        a = fma(ri, ri, a);
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

enum PcgStep : int { kPcgStart, kPcgRz, kPcgRzFirst, kPcgAlpha, kPcgXr, kPcgTrue };

__device__ void pcg_post(Mailbox *mb, int done, const PcgDev *st, bool progress) {
    if (!mb) return;
    if (progress) {
        mb->iters = st->iters;
        mb->est = st->relres;
    }
    __threadfence_system();
    __hip_atomic_store(&mb->done, done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The scalar part of a PCG step from the B partials of the preceding pass
// (one block, sums in block order):
//   kPcgStart: ||b|| and ||r0|| (done when b = 0 or already converged)
//   kPcgRz / kPcgRzFirst: (r, z); beta = rz_new / rz except on the first call
//   kPcgAlpha: alpha = (r, z) / (p, q); (p, q) = 0 ends the iteration
//   kPcgXr: ||r||: count the iteration, decide convergence
//   kPcgTrue: ||b - A x||^2 into true_rr
__global__ __launch_bounds__(kNT) void k_pcg_fin(int step, int B, PcgDev *st, const double *part, Mailbox *mb) {
    __shared__ double sh[4];
    if ((step == kPcgRz || step == kPcgRzFirst || step == kPcgAlpha || step == kPcgXr) && st->done) return;
    const double t0 = sum_partials(part, B, sh);
    const double t1 = step == kPcgStart ? sum_partials(part + B, B, sh) : 0.0;
    if (threadIdx.x != 0) return;
    switch (step) {
    case kPcgStart:
        st->nb = sqrt(t0);
        st->relres = st->nb > 0.0 ? sqrt(t1) / st->nb : 0.0;
        st->iters = 0;
        st->breakdown = 0;
        st->done = (st->nb == 0.0 || st->relres <= st->rtol || st->maxit == 0) ? 1 : 0;
        if (mb) mb->iters = 0;
        pcg_post(mb, st->done, st, false);
        return;
    case kPcgRz:
        st->beta = t0 / st->rz;
        st->rz = t0;
        return;
    case kPcgRzFirst:
        st->rz = t0;
        return;
    case kPcgAlpha:
        if (t0 == 0.0) {
            st->breakdown = 1;
            st->done = 1;
            pcg_post(mb, 1, st, false);
            return;
        }
        st->alpha = st->rz / t0;
        return;
    case kPcgXr:
        st->iters += 1;
        st->relres = sqrt(t0) / st->nb;
        st->done = (st->relres <= st->rtol || st->iters >= st->maxit) ? 1 : 0;
        pcg_post(mb, st->done, st, true);
        return;
    case kPcgTrue:
        st->true_rr = t0;
        return;
    default:
        return;
    }
}

__global__ void k_pcg_init(PcgDev *st, int maxit, double rtol) {
    st->maxit = maxit;
    st->rtol = rtol;
    st->done = 0;
    st->iters = 0;
    st->breakdown = 0;
}

// Grid of the inner-product passes: up to 512 blocks of >= 2048 rows.
int reduce_blocks(int64_t n) {
    const int64_t b = (n + 2047) / 2048;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 512));
}

// Grid of the update pass (no reduction): up to 4096 blocks of >= 512 rows.
int update_blocks(int64_t n) {
    const int64_t b = (n + 511) / 512;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

int stream_blocks(int64_t n) {
    const int64_t b = (n + 1023) / 1024;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace

// ===========================================================================
// Host driver
// ===========================================================================

Solver::~Solver() {
    if (mailbox_) (void)hipHostFree(mailbox_);
}

void Solver::ensure(Allocator *a, int64_t n, int restart, bool flexible, int precision) {
    // 512-byte aligned vectors, consecutive ones 2 KiB off a multiple of the
    // rounded length: with n a power of two the basis vectors would otherwise
    // start at the same address bits and the streams of one pass would meet
    // in the same memory channels (measured: 3.9 vs 4.6 TB/s for a 34-vector pass)
    const int64_t ld = (n + 63) / 64 * 64 + 256;
    const bool need = n != n_ || restart != restart_ || flexible != flex_ || (precision != SAIT_F64 && y32_.empty());
    if (!need) return;
    n_ = n;
    restart_ = restart;
    flex_ = flexible;
    ldv_ = ld;
    const int64_t nn = std::max<int64_t>(ld, 64);
    V_.alloc(a, (size_t)nn * (restart + 1) * sizeof(double));
    if (flexible) Z_.alloc(a, (size_t)nn * restart * sizeof(double));
    else Z_.reset();
    zt_.alloc(a, (size_t)nn * sizeof(double));
    ut_.alloc(a, (size_t)nn * sizeof(double));
    if (precision != SAIT_F64) y32_.alloc(a, (size_t)nn * sizeof(float));
    else y32_.reset();
    const size_t kk = (size_t)restart, hsz = (kk + 1) * kk;
    arr_.alloc(a, sizeof(double) * (2 * hsz + (flexible ? kk * kk : 0) + 9 * (kk + 2) + 2 * kk + 2));
    st_.alloc(a, sizeof(GmresDev));
    part_.alloc(a, sizeof(double) * (size_t)512 * (2 * kk + 2));
    if (!mailbox_) SAIT_HIP(hipHostMalloc(&mailbox_, 256, hipHostMallocMapped));
    // bind the array pointers inside the device state
    GmresDev h{};
    double *base = arr_.as<double>();
    auto take = [&](size_t cnt) {
        double *r = base;
        base += cnt;
        return r;
    };
    h.Hraw = take(hsz);
    h.R = take(hsz);
    h.Gam = flexible ? take(kk * kk) : nullptr;
    h.cs = take(kk + 2);
    h.sn = take(kk + 2);
    h.g = take(kk + 2);
    h.y = take(kk + 2);
    h.yh = take(kk + 2);
    h.s1 = take(kk + 2);
    h.s1n = take(kk + 2);
    h.ca = take(kk + 2);
    h.cg = take(kk + 2);
    h.red = take(2 * kk + 2);
    SAIT_HIP(hipMemcpy(st_.as<void>(), &h, sizeof(h), hipMemcpyHostToDevice));
}

void Solver::ensure_prec_tmp(Allocator *a, int64_t n, int precision) {
    const size_t nn = (size_t)std::max<int64_t>(n, 64);
    if (zt_.bytes() < nn * sizeof(double)) zt_.alloc(a, nn * sizeof(double));
    if (pt1_.bytes() < nn * sizeof(double)) pt1_.alloc(a, nn * sizeof(double));
    if (precision != SAIT_F64 && y32_.bytes() < nn * sizeof(float)) y32_.alloc(a, nn * sizeof(float));
}

void Solver::apply_prec(const Ops &ops, const double *in, double *out, hipStream_t s) {
    const int64_t n = ops.A->n;
    switch (ops.prec_kind) {
    case SAIT_PREC_SAIT:
        if (ops.precision == SAIT_F64) {
            spmv(*ops.M1, in, XKind::F64, zt_.as<double>(), YKind::F64, 1, 1, 1, ops.lanes1, s);
            spmv(*ops.M2, zt_.as<double>(), XKind::F64, out, YKind::F64, 1, 1, 1, ops.lanes2, s);
        } else {
            spmv(*ops.M1, in, XKind::F64, y32_.as<float>(), YKind::F32, 1, 1, 1, ops.lanes1, s);
            spmv(*ops.M2, y32_.as<float>(), XKind::F32, out, YKind::F64, 1, 1, 1, ops.lanes2, s);
        }
        return;
    case SAIT_PREC_JACOBI:
        jacobi_apply(*ops.JL, ops.sweeps, in, zt_.as<double>(), pt1_.as<double>(), s);
        jacobi_apply(*ops.JU, ops.sweeps, zt_.as<double>(), out, pt1_.as<double>(), s);
        return;
    case SAIT_PREC_EXACT:
        level_solve(*ops.EL, in, zt_.as<double>(), s);
        level_solve(*ops.EU, zt_.as<double>(), out, s);
        return;
    case SAIT_PREC_NONE:
        if (n) SAIT_HIP(hipMemcpyAsync(out, in, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
        return;
    default:
        fail(SAIT_E_INVALID, "unknown preconditioner kind");
    }
}

int Solver::pcg(Allocator *a, const Ops &ops, const double *b, double *x, const sait_solve_opts &o,
                sait_solve_info *info, hipStream_t s) {
    const int64_t n = ops.A->n;
    if (o.maxit < 0) fail(SAIT_E_INVALID, "maxit must be >= 0");
    if (!(o.rtol >= 0.0)) fail(SAIT_E_INVALID, "rtol must be >= 0");
    ensure_prec_tmp(a, n, ops.precision);
    if (pn_ != n) {
        const size_t nn = (size_t)std::max<int64_t>(n, 64) * sizeof(double);
        pr_.alloc(a, nn);
        pz_.alloc(a, nn);
        pp_.alloc(a, nn);
        pq_.alloc(a, nn);
        pst_.alloc(a, sizeof(PcgDev));
        ppart_.alloc(a, sizeof(double) * 2 * 1024);
        if (!mailbox_) SAIT_HIP(hipHostMalloc(&mailbox_, 256, hipHostMallocMapped));
        pn_ = n;
    }
    PcgDev *st = pst_.as<PcgDev>();
    Mailbox *mbh = reinterpret_cast<Mailbox *>(mailbox_);
    Mailbox *mbd = nullptr;
    SAIT_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&mbd), mailbox_, 0));
    double *r = pr_.as<double>(), *z = pz_.as<double>(), *p = pp_.as<double>(), *q = pq_.as<double>();
    double *part = ppart_.as<double>();
    const int RB = std::min(reduce_blocks(n), 1024);
    // a reduction: RB partial sums, then the scalar step on one block
    auto reduce = [&](int step, const double *x1, const double *y1, const double *u1, const double *w1,
                      int check_done, Mailbox *mb) {
        hipLaunchKernelGGL(k_pcg_dots, dim3(RB), dim3(kNT), 0, s, n, x1, y1, u1, w1, st, check_done, part);
        hipLaunchKernelGGL(k_pcg_fin, dim3(1), dim3(kNT), 0, s, step, RB, st, part, mb);
    };
    const int SB = stream_blocks(n);

    hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(1), 0, s, st, o.maxit, o.rtol);
    spmv(*ops.A, x, XKind::F64, r, YKind::F64, 1, 1, 1, ops.lanesA, s, b);  // r = b - A x
    reduce(kPcgStart, b, b, r, r, 0, mbd);
    SAIT_LAUNCH_CHECK();
    PcgDev hs{};
    SAIT_HIP(hipMemcpyAsync(&hs, st, sizeof(PcgDev), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    if (hs.nb == 0.0) {
        if (n) SAIT_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
        SAIT_HIP(hipStreamSynchronize(s));
        fill_info(info, 0, 0, SAIT_OK, 0.0, 0.0);
        return SAIT_OK;
    }
    if (!hs.done) {
        apply_prec(ops, r, z, s);
        reduce(kPcgRzFirst, r, z, nullptr, nullptr, 1, nullptr);
        hipLaunchKernelGGL(k_pcg_dir, dim3(SB), dim3(256), 0, s, n, z, p, st, 1);
        SAIT_LAUNCH_CHECK();
        // iterations, a few queued ahead of the polled mailbox
        constexpr int kAhead = 3;
        hipEvent_t ev[kAhead + 1];
        for (auto &e : ev) SAIT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        bool stop = false;
        for (int it = 0; it < o.maxit && !stop; ++it) {
            spmv(*ops.A, p, XKind::F64, q, YKind::F64, 1, 1, 1, ops.lanesA, s);
            reduce(kPcgAlpha, p, q, nullptr, nullptr, 1, mbd);
            hipLaunchKernelGGL(k_pcg_xr, dim3(RB), dim3(kNT), 0, s, n, p, q, x, r, st, part);
            hipLaunchKernelGGL(k_pcg_fin, dim3(1), dim3(kNT), 0, s, (int)kPcgXr, RB, st, part, mbd);
            apply_prec(ops, r, z, s);
            reduce(kPcgRz, r, z, nullptr, nullptr, 1, nullptr);
            hipLaunchKernelGGL(k_pcg_dir, dim3(SB), dim3(256), 0, s, n, z, p, st, 0);
            SAIT_LAUNCH_CHECK();
            SAIT_HIP(hipEventRecord(ev[it % (kAhead + 1)], s));
            if (it >= kAhead) {
                SAIT_HIP(hipEventSynchronize(ev[(it - kAhead) % (kAhead + 1)]));
                if (__hip_atomic_load(&mbh->done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)) stop = true;
            }
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
    // true residual
    spmv(*ops.A, x, XKind::F64, q, YKind::F64, 1, 1, 1, ops.lanesA, s, b);
    reduce(kPcgTrue, q, q, nullptr, nullptr, 0, nullptr);
    SAIT_LAUNCH_CHECK();
    SAIT_HIP(hipMemcpyAsync(&hs, st, sizeof(PcgDev), hipMemcpyDeviceToHost, s));
    SAIT_HIP(hipStreamSynchronize(s));
    const double true_rel = sqrt(hs.true_rr) / hs.nb;
    const int status = (hs.relres <= o.rtol && !hs.breakdown) ? SAIT_OK : SAIT_NOT_CONVERGED;
    fill_info(info, hs.iters, 0, status, hs.relres, true_rel);
    return status;
}

int Solver::solve(Allocator *a, const Ops &ops, const double *b, double *x, const sait_solve_opts &o,
                  sait_solve_info *info, hipStream_t s) {
    const int64_t n = ops.A->n;
    const int k = o.restart;
    if (k < 1 || k > 1000) fail(SAIT_E_INVALID, "restart must be in 1..1000");
    if (o.maxit < 0) fail(SAIT_E_INVALID, "maxit must be >= 0");
    if (!(o.rtol >= 0.0)) fail(SAIT_E_INVALID, "rtol must be >= 0");
    ensure(a, n, k, o.flexible != 0, ops.precision);
    ensure_prec_tmp(a, n, ops.precision);
    GmresDev *st = st_.as<GmresDev>();
    Mailbox *mbh = reinterpret_cast<Mailbox *>(mailbox_);
    Mailbox *mbd = nullptr;
    SAIT_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&mbd), mailbox_, 0));
    double *V = V_.as<double>();
    double *part = part_.as<double>();
    const int RB = reduce_blocks(n);
    const int SB = stream_blocks(n);
    const int UB = update_blocks(n);

    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, k, o.maxit, o.rtol);
    SAIT_LAUNCH_CHECK();
    // ||b||
    hipLaunchKernelGGL(k_cycle_norm, dim3(RB), dim3(kNT), 0, s, n, b, part);
    hipLaunchKernelGGL(k_cycle_norm_fin, dim3(1), dim3(kNT), 0, s, RB, st, 0, part, (Mailbox *)nullptr);
    SAIT_LAUNCH_CHECK();
    GmresDev hs{};
    int restarts = 0;
    int status = SAIT_OK;
    for (;;) {
        // r = b - A x  -> V[0], beta, cycle reset
        spmv(*ops.A, x, XKind::F64, V, YKind::F64, 1, 1, 1, ops.lanesA, s, b);
        hipLaunchKernelGGL(k_cycle_norm, dim3(RB), dim3(kNT), 0, s, n, V, part);
        hipLaunchKernelGGL(k_cycle_norm_fin, dim3(1), dim3(kNT), 0, s, RB, st, 1, part, mbd);
        SAIT_LAUNCH_CHECK();
        SAIT_HIP(hipMemcpyAsync(&hs, st, sizeof(GmresDev), hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipStreamSynchronize(s));
        const double relres = hs.nb == 0.0 ? 0.0 : hs.beta / hs.nb;
        if (hs.nb == 0.0) {
            // b = 0: x = 0 is the solution
            SAIT_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
            SAIT_HIP(hipStreamSynchronize(s));
            fill_info(info, 0, 0, SAIT_OK, 0.0, 0.0);
            return SAIT_OK;
        }
        if (relres <= o.rtol) {
            fill_info(info, hs.iters, restarts, SAIT_OK, hs.est, relres);
            return SAIT_OK;
        }
        if (hs.iters >= o.maxit) {
            fill_info(info, hs.iters, restarts, SAIT_NOT_CONVERGED, hs.est, relres);
            status = SAIT_NOT_CONVERGED;
            return status;
        }
        // Arnoldi steps (step k closes column k-1), a few queued ahead of the
        // polled mailbox
        constexpr int kAhead = 3;
        hipEvent_t ev[kAhead + 1];
        for (auto &e : ev) SAIT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        int enq = 0;
        bool stop = false;
        for (int j = 0; j <= k && !stop; ++j) {
            double *uj = V + (int64_t)j * ldv_;
            double *w = j < k ? V + (int64_t)(j + 1) * ldv_ : nullptr;
            if (j < k) {
                double *zj = o.flexible ? Z_.as<double>() + (int64_t)j * ldv_ : ut_.as<double>();
                apply_prec(ops, uj, zj, s);
                spmv(*ops.A, zj, XKind::F64, w, YKind::F64, 1, 1, 1, ops.lanesA, s);
            }
            hipLaunchKernelGGL(k_dots2, dim3(RB), dim3(kNT), 0, s, n, V, ldv_, j, uj, w, st, part);
            hipLaunchKernelGGL(k_dots2_fin, dim3(1), dim3(kNT), 0, s, j, (int)(w != nullptr), RB, st, part, mbd);
            if (j < k) hipLaunchKernelGGL(k_update2, dim3(UB), dim3(kNT), 0, s, n, V, ldv_, j, st);
            SAIT_LAUNCH_CHECK();
            SAIT_HIP(hipEventRecord(ev[j % (kAhead + 1)], s));
            ++enq;
            if (enq > kAhead) {
                // wait for the step enqueued kAhead steps ago, then read the mailbox
                SAIT_HIP(hipEventSynchronize(ev[(j - kAhead) % (kAhead + 1)]));
                if (__hip_atomic_load(&mbh->done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)) stop = true;
            }
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        // x update
        hipLaunchKernelGGL(k_hsolve, dim3(1), dim3(kNT), 0, s, st);
        SAIT_LAUNCH_CHECK();
        if (o.flexible) {
            hipLaunchKernelGGL(k_combine, dim3(SB), dim3(256), 0, s, n, Z_.as<double>(), ldv_, st, x, 1);
        } else {
            hipLaunchKernelGGL(k_combine, dim3(SB), dim3(256), 0, s, n, V, ldv_, st, ut_.as<double>(), 0);
            apply_prec(ops, ut_.as<double>(), V + (int64_t)k * ldv_, s);  // V[k] is free scratch here
            hipLaunchKernelGGL(k_axpy_inplace, dim3(SB), dim3(256), 0, s, n, x, V + (int64_t)k * ldv_);
        }
        SAIT_LAUNCH_CHECK();
        ++restarts;
    }
}

void Solver::fill_info(sait_solve_info *info, int iters, int restarts, int status, double est, double relres) {
    if (!info) return;
    info->iterations = iters;
    info->restarts = restarts;
    info->status = status;
    info->est_relres = est;
    info->true_relres = relres;
}

void copy_strided(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_strided, dim3(stream_blocks(n)), dim3(256), 0, s, n, src, lds, dst, ldd);
    SAIT_LAUNCH_CHECK();
}

}  // namespace sait
