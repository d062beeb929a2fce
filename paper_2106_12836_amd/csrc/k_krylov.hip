// Restarted right-preconditioned GMRES(k) / FGMRES(k) on the device, the
// iterative method the SAIT preconditioner is applied inside (Sec. 3.1,
// Sec. 3.2 Eq. runtime: each iteration is one preconditioner application
// comp(M_L, M_U) plus "othercomp": an operator product, inner products and
// vector updates).
//
// Everything is FP64 and stays on the device: the Krylov basis V (and Z
// for FGMRES), the inner products, the Hessenberg matrix with its Givens
// rotations and the true residual.  One Arnoldi step is
//   z_j = M v_j                      (SAIT apply, any storage precision)
//   w   = A z_j                      (written straight into V[j+1])
//   h   = V_j^T w,  w -= V_j h        classical Gram-Schmidt
//   (repeated once if ||w_new|| < ||w_old|| / sqrt(2): the DGKS test)
//   h_{j+1,j} = ||w||, Givens update of the least-squares residual
//   v_{j+1} = w / h_{j+1,j}
// Reductions are deterministic: each block writes a partial, the last block
// to finish (atomic ticket) sums the partials in a fixed order.  Every
// kernel of an Arnoldi step starts by reading the `done` flag, so steps
// enqueued after convergence cost only a launch; the host keeps a few steps
// queued ahead and polls a pinned, device-written mailbox to stop
// enqueueing.  The host synchronises once per restart cycle, to read the
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

__device__ __forceinline__ bool last_block(unsigned *counter) {
    __shared__ int am_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        am_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    return am_last != 0;
}

__device__ __forceinline__ double ld_acq(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reduce part[i*B + b] over b for i < count into out[i] (last block only).
__device__ void reduce_partials(const double *part, int B, int count, double *out, double *sh) {
    for (int i = 0; i < count; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < B; b += kNT) s += ld_acq(part + (size_t)i * B + b);
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[i] = s;
    }
}

struct Rows {
    int64_t lo, hi;
};
__device__ __forceinline__ Rows block_rows(int64_t n, int B) {
    const int64_t chunk = ((n + B - 1) / B + kNT - 1) / kNT * kNT;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    return {lo, lo + chunk < n ? lo + chunk : n};
}

// Givens update of column j and the convergence decision (one thread).
__device__ void finalize_step(GmresDev *st, double hn, bool use_h2, Mailbox *mb) {
    const int k = st->restart;
    const int j = st->jc;
    double *H = st->H + (size_t)j * (k + 1);  // column j, (k+1) entries
    for (int i = 0; i <= j; ++i) H[i] = use_h2 ? st->h1[i] + st->h2[i] : st->h1[i];
    H[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = H[i], b = H[i + 1];
        H[i] = st->cs[i] * a + st->sn[i] * b;
        H[i + 1] = -st->sn[i] * a + st->cs[i] * b;
    }
    const double a = H[j], b = H[j + 1];
    const double den = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (den != 0.0) {
        c = a / den;
        s = b / den;
    }
    st->cs[j] = c;
    st->sn[j] = s;
    H[j] = den;
    H[j + 1] = 0.0;
    st->g[j + 1] = -s * st->g[j];
    st->g[j] = c * st->g[j];
    st->jc = j + 1;
    st->iters += 1;
    st->est = fabs(st->g[j + 1]) / st->nb;
    st->inv_hn = hn != 0.0 ? 1.0 / hn : 0.0;
    const bool stop = st->est <= st->rtol || st->iters >= st->maxit || hn == 0.0 || st->jc >= k;
    st->done = stop ? 1 : 0;
    if (mb) {
        mb->est = st->est;
        mb->iters = st->iters;
        __threadfence_system();
        __hip_atomic_store(&mb->done, st->done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// h[i] = V_i . w for i < nv (grouped by 4), optionally also w . w.
__global__ __launch_bounds__(kNT) void k_dots(int64_t n, const double *__restrict__ V, int64_t ldv, int nv,
                                              const double *__restrict__ w, GmresDev *st, int phase, double *part,
                                              unsigned *counter) {
    __shared__ double sh[4];
    if (st->done) return;
    if (phase == 2 && !st->reorth) return;
    const int B = gridDim.x;
    const Rows R = block_rows(n, B);
    for (int i0 = 0; i0 < nv; i0 += 4) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        const double *v0 = V + (int64_t)i0 * ldv;
        const int m = nv - i0;
        for (int64_t r = R.lo + threadIdx.x; r < R.hi; r += kNT) {
            const double x = w[r];
            a0 = fma(v0[r], x, a0);
            if (m > 1) a1 = fma(v0[ldv + r], x, a1);
            if (m > 2) a2 = fma(v0[2 * ldv + r], x, a2);
            if (m > 3) a3 = fma(v0[3 * ldv + r], x, a3);
        }
        const double s0 = block_sum(a0, sh);
        const double s1 = m > 1 ? block_sum(a1, sh) : 0.0;
        const double s2 = m > 2 ? block_sum(a2, sh) : 0.0;
        const double s3 = m > 3 ? block_sum(a3, sh) : 0.0;
        if (threadIdx.x == 0) {
            part[(size_t)i0 * B + blockIdx.x] = s0;
            if (m > 1) part[(size_t)(i0 + 1) * B + blockIdx.x] = s1;
            if (m > 2) part[(size_t)(i0 + 2) * B + blockIdx.x] = s2;
            if (m > 3) part[(size_t)(i0 + 3) * B + blockIdx.x] = s3;
        }
    }
    const bool with_norm = phase == 1;
    if (with_norm) {
        double a = 0;
        for (int64_t r = R.lo + threadIdx.x; r < R.hi; r += kNT) a = fma(w[r], w[r], a);
        const double s = block_sum(a, sh);
        if (threadIdx.x == 0) part[(size_t)nv * B + blockIdx.x] = s;
    }
    if (!last_block(counter)) return;
    double *out = phase == 1 ? st->h1 : st->h2;
    reduce_partials(part, B, nv, out, sh);
    if (with_norm) reduce_partials(part + (size_t)nv * B, B, 1, &st->wpre2, sh);
    if (threadIdx.x == 0) *counter = 0;
}

// w -= sum_i h_i V_i for i < nv, then ||w||^2; last block decides
// reorthogonalisation (phase 1) or finalises the step.
__global__ __launch_bounds__(kNT) void k_update(int64_t n, const double *__restrict__ V, int64_t ldv, int nv,
                                                double *__restrict__ w, GmresDev *st, int phase, double *part,
                                                unsigned *counter, Mailbox *mb) {
    __shared__ double sh[4];
    __shared__ double hs[64];
    if (st->done) return;
    if (phase == 2 && !st->reorth) return;
    const double *h = phase == 1 ? st->h1 : st->h2;
    const int B = gridDim.x;
    const Rows R = block_rows(n, B);
    double nrm = 0;
    for (int i0 = 0; i0 < nv; i0 += 64) {
        const int m = nv - i0 < 64 ? nv - i0 : 64;
        __syncthreads();
        if (threadIdx.x < m) hs[threadIdx.x] = h[i0 + threadIdx.x];
        __syncthreads();
        const bool final_chunk = i0 + 64 >= nv;
        for (int64_t r = R.lo + threadIdx.x; r < R.hi; r += kNT) {
            double x = w[r];
            const double *vp = V + (int64_t)i0 * ldv + r;
            for (int i = 0; i < m; ++i) x = fma(-hs[i], vp[(int64_t)i * ldv], x);
            w[r] = x;
            if (final_chunk) nrm = fma(x, x, nrm);
        }
    }
    const double s = block_sum(nrm, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (!last_block(counter)) return;
    double hn2 = 0;
    reduce_partials(part, B, 1, &hn2, sh);
    if (threadIdx.x == 0) {
        *counter = 0;
        if (phase == 1 && hn2 < 0.5 * st->wpre2) {
            st->reorth = 1;  // DGKS: too much cancellation, orthogonalise again
        } else {
            finalize_step(st, sqrt(hn2), phase == 2, mb);
            st->reorth = 0;
        }
    }
}

// V[j+1] = w * (1/h_{j+1,j})  (in place; skipped once the cycle is done)
__global__ void k_normalize(int64_t n, double *__restrict__ w, const GmresDev *st) {
    if (st->done) return;
    const double s = st->inv_hn;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        w[r] *= s;
}

// ||r||^2 of the residual in V[0]; the last block starts a cycle:
// beta, g = beta e_1, jc = 0, done unless more iterations are needed.
// mode 0: r = b (computes ||b||); mode 1: cycle start.
__global__ __launch_bounds__(kNT) void k_cycle_norm(int64_t n, const double *__restrict__ r, GmresDev *st, int mode,
                                                    double *part, unsigned *counter, Mailbox *mb) {
    __shared__ double sh[4];
    const int B = gridDim.x;
    const Rows R = block_rows(n, B);
    double a = 0;
    for (int64_t i = R.lo + threadIdx.x; i < R.hi; i += kNT) a = fma(r[i], r[i], a);
    const double s = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (!last_block(counter)) return;
    double ss = 0;
    reduce_partials(part, B, 1, &ss, sh);
    if (threadIdx.x == 0) {
        *counter = 0;
        const double nrm = sqrt(ss);
        if (mode == 0) {
            st->nb = nrm;
        } else {
            st->beta = nrm;
            st->g[0] = nrm;
            for (int i = 1; i <= st->restart; ++i) st->g[i] = 0.0;
            st->jc = 0;
            st->reorth = 0;
            st->inv_hn = nrm != 0.0 ? 1.0 / nrm : 0.0;
            const bool ok = st->nb == 0.0 || nrm / st->nb <= st->rtol;
            st->done = (ok || st->iters >= st->maxit) ? 1 : 0;
            if (mb) {
                mb->iters = st->iters;
                __threadfence_system();
                __hip_atomic_store(&mb->done, st->done, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

// y = R^-1 g over the jc completed steps (single block, sequential).
__global__ void k_hsolve(GmresDev *st) {
    if (threadIdx.x != 0) return;
    const int k = st->restart, jc = st->jc;
    for (int i = jc - 1; i >= 0; --i) {
        double s = st->g[i];
        for (int t = i + 1; t < jc; ++t) s -= st->H[(size_t)t * (k + 1) + i] * st->y[t];
        const double d = st->H[(size_t)i * (k + 1) + i];
        st->y[i] = d != 0.0 ? s / d : 0.0;
    }
}

// out (+)= sum_{i < jc} y_i B_i
__global__ void k_combine(int64_t n, const double *__restrict__ Bv, int64_t ldb, const GmresDev *st,
                          double *__restrict__ out, int accumulate) {
    __shared__ double ys[64];
    const int jc = st->jc;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r - threadIdx.x < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int i0 = 0; i0 < jc; i0 += 64) {
            const int m = jc - i0 < 64 ? jc - i0 : 64;
            __syncthreads();
            if (threadIdx.x < m) ys[threadIdx.x] = st->y[i0 + threadIdx.x];
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
    st->reorth = 0;
    st->nb = 0.0;
}

int reduce_blocks(int64_t n) {
    const int64_t b = (n + 2047) / 2048;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
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
    const int64_t ld = (n + 63) / 64 * 64;  // 512-byte aligned vectors
    const bool need = n != n_ || restart != restart_ || (flexible && Z_.empty()) || (precision != SAIT_F64 && y32_.empty());
    if (!need) return;
    n_ = n;
    restart_ = restart;
    ldv_ = ld;
    const int64_t nn = std::max<int64_t>(ld, 64);
    V_.alloc(a, (size_t)nn * (restart + 1) * sizeof(double));
    if (flexible) Z_.alloc(a, (size_t)nn * restart * sizeof(double));
    else Z_.reset();
    zt_.alloc(a, (size_t)nn * sizeof(double));
    ut_.alloc(a, (size_t)nn * sizeof(double));
    if (precision != SAIT_F64) y32_.alloc(a, (size_t)nn * sizeof(float));
    else y32_.reset();
    arr_.alloc(a, sizeof(double) * ((size_t)(restart + 1) * restart + 6 * (restart + 2)));
    st_.alloc(a, sizeof(GmresDev));
    part_.alloc(a, sizeof(double) * (size_t)1024 * (restart + 3));
    counters_.alloc(a, 4 * sizeof(unsigned));
    SAIT_HIP(hipMemset(counters_.as<void>(), 0, 4 * sizeof(unsigned)));
    if (!mailbox_) SAIT_HIP(hipHostMalloc(&mailbox_, 256, hipHostMallocMapped));
    // bind the array pointers inside the device state
    GmresDev h{};
    double *base = arr_.as<double>();
    h.H = base;
    base += (size_t)(restart + 1) * restart;
    h.cs = base;
    base += restart + 2;
    h.sn = base;
    base += restart + 2;
    h.g = base;
    base += restart + 2;
    h.y = base;
    base += restart + 2;
    h.h1 = base;
    base += restart + 2;
    h.h2 = base;
    SAIT_HIP(hipMemcpy(st_.as<void>(), &h, sizeof(h), hipMemcpyHostToDevice));
}

void Solver::apply_prec(const Ops &ops, const double *in, double *out, hipStream_t s) {
    if (ops.precision == SAIT_F64) {
        spmv(*ops.M1, in, XKind::F64, zt_.as<double>(), YKind::F64, 1, 1, 1, ops.lanes1, s);
        spmv(*ops.M2, zt_.as<double>(), XKind::F64, out, YKind::F64, 1, 1, 1, ops.lanes2, s);
    } else {
        spmv(*ops.M1, in, XKind::F64, y32_.as<float>(), YKind::F32, 1, 1, 1, ops.lanes1, s);
        spmv(*ops.M2, y32_.as<float>(), XKind::F32, out, YKind::F64, 1, 1, 1, ops.lanes2, s);
    }
}

int Solver::solve(Allocator *a, const Ops &ops, const double *b, double *x, const sait_solve_opts &o,
                  sait_solve_info *info, hipStream_t s) {
    const int64_t n = ops.A->n;
    const int k = o.restart;
    if (k < 1 || k > 1000) fail(SAIT_E_INVALID, "restart must be in 1..1000");
    if (o.maxit < 0) fail(SAIT_E_INVALID, "maxit must be >= 0");
    if (!(o.rtol >= 0.0)) fail(SAIT_E_INVALID, "rtol must be >= 0");
    ensure(a, n, k, o.flexible != 0, ops.precision);
    GmresDev *st = st_.as<GmresDev>();
    Mailbox *mbh = reinterpret_cast<Mailbox *>(mailbox_);
    Mailbox *mbd = nullptr;
    SAIT_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&mbd), mailbox_, 0));
    double *V = V_.as<double>();
    double *part = part_.as<double>();
    unsigned *cnt = counters_.as<unsigned>();
    const int RB = reduce_blocks(n);
    const int SB = stream_blocks(n);

    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, k, o.maxit, o.rtol);
    SAIT_LAUNCH_CHECK();
    // ||b||
    hipLaunchKernelGGL(k_cycle_norm, dim3(RB), dim3(kNT), 0, s, n, b, st, 0, part, cnt, (Mailbox *)nullptr);
    SAIT_LAUNCH_CHECK();
    GmresDev hs{};
    int restarts = 0;
    int status = SAIT_OK;
    for (;;) {
        // r = b - A x  -> V[0], beta, cycle reset
        spmv(*ops.A, x, XKind::F64, V, YKind::F64, 1, 1, 1, ops.lanesA, s, b);
        hipLaunchKernelGGL(k_cycle_norm, dim3(RB), dim3(kNT), 0, s, n, V, st, 1, part, cnt, mbd);
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
        hipLaunchKernelGGL(k_normalize, dim3(SB), dim3(256), 0, s, n, V, st);
        SAIT_LAUNCH_CHECK();
        // Arnoldi steps, a few queued ahead of the polled mailbox
        constexpr int kAhead = 3;
        hipEvent_t ev[kAhead + 1];
        for (auto &e : ev) SAIT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        int enq = 0;
        bool stop = false;
        for (int j = 0; j < k && !stop; ++j) {
            double *vj = V + (int64_t)j * ldv_;
            double *w = V + (int64_t)(j + 1) * ldv_;
            double *zj = o.flexible ? Z_.as<double>() + (int64_t)j * ldv_ : ut_.as<double>();
            apply_prec(ops, vj, zj, s);
            spmv(*ops.A, zj, XKind::F64, w, YKind::F64, 1, 1, 1, ops.lanesA, s);
            hipLaunchKernelGGL(k_dots, dim3(RB), dim3(kNT), 0, s, n, V, ldv_, j + 1, w, st, 1, part, cnt);
            hipLaunchKernelGGL(k_update, dim3(RB), dim3(kNT), 0, s, n, V, ldv_, j + 1, w, st, 1, part, cnt + 1, mbd);
            hipLaunchKernelGGL(k_dots, dim3(RB), dim3(kNT), 0, s, n, V, ldv_, j + 1, w, st, 2, part, cnt);
            hipLaunchKernelGGL(k_update, dim3(RB), dim3(kNT), 0, s, n, V, ldv_, j + 1, w, st, 2, part, cnt + 1, mbd);
            hipLaunchKernelGGL(k_normalize, dim3(SB), dim3(256), 0, s, n, w, st);
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
        hipLaunchKernelGGL(k_hsolve, dim3(1), dim3(64), 0, s, st);
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
