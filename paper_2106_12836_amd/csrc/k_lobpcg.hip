// LOBPCG for the k <= 5 smallest eigenpairs of a symmetric positive definite
// A with the SAIT preconditioner applied to the whole residual block (the
// eigenvalue experiment of Sec. 4: the preconditioning step is two sparse
// matrix-matrix products).  Knyazev's locally optimal block preconditioned
// conjugate gradient:
//
//   R = A X - X diag(theta);  W = T R;  S = [X, W, P];
//   Rayleigh-Ritz on span(S) -> theta, coefficients c (3k x k);
//   X <- S c,  P <- [W, P] c_(W,P)   (A X, A P carried along)
//
// Device work per step: the preconditioner and A W (block SpMM, row-major
// n x k blocks), one Gram pass, one update pass.  The Gram matrices
// S^T (A S) and S^T S are a dense contraction over n of at most 15 columns:
// each wavefront accumulates them with v_mfma_f64_16x16x4f64 (four rows per
// instruction; lane l supplies S[r0 + l/16][l%16] as both operands' element
// and receives G[4v + l/16][l%16] in register v).  The Rayleigh-Ritz problem
// of order <= 15 is solved on the host (Cholesky of the unit-diagonal scaled
// S^T S, cyclic Jacobi on the reduced matrix) from one readback per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lobpcg.h"

namespace sait {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGramThreads = 256;  // 4 wavefronts
constexpr int kGramTile = 256;     // one 16 x 16 FP64 tile
constexpr int kUpdThreads = 256;
constexpr int kMaxBlock = 5;       // 3k <= 15 columns fit one tile

struct GramArgs {
    const double *s[3], *as[3];  // blocks X, W, P and A X, A W, A P (n x k row-major)
    int64_t n, quads;             // quads = ceil(n / 4)
    int k, nb;                    // block width, blocks in the basis (1..3)
};

// Partial Gram tiles of the rows one workgroup covers: part[blk][0..255] =
// S^T (A S), part[blk][256..511] = S^T S (16 x 16, row-major, zero padded).
__global__ __launch_bounds__(kGramThreads) void k_gram(GramArgs a, double *__restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 15, kk = lane >> 4;
    const int b = c / a.k, j = c - b * a.k;
    const bool on = b < a.nb;
    const double *S = on ? a.s[b] : nullptr;
    const double *AS = on ? a.as[b] : nullptr;
    v4d ga0 = {0, 0, 0, 0}, gb0 = {0, 0, 0, 0}, ga1 = {0, 0, 0, 0}, gb1 = {0, 0, 0, 0};
    // every wavefront takes a contiguous range of quads (whole cache lines),
    // two quads per iteration into alternating accumulators
    const int64_t waves = (int64_t)gridDim.x * (kGramThreads / 64);
    const int64_t chunk = (a.quads + waves - 1) / waves;
    const int64_t q0 = ((int64_t)blockIdx.x * (kGramThreads / 64) + wave) * chunk;
    const int64_t q1 = q0 + chunk < a.quads ? q0 + chunk : a.quads;
    int64_t q = q0;
    for (; q + 1 < q1; q += 2) {
        const int64_t r0 = q * 4 + kk, r1 = r0 + 4;
        double s0 = 0.0, t0 = 0.0, s1 = 0.0, t1 = 0.0;
        if (on) {
            if (r0 < a.n) {
                s0 = S[r0 * a.k + j];
                t0 = AS[r0 * a.k + j];
            }
            if (r1 < a.n) {
                s1 = S[r1 * a.k + j];
                t1 = AS[r1 * a.k + j];
            }
        }
        ga0 = __builtin_amdgcn_mfma_f64_16x16x4f64(s0, t0, ga0, 0, 0, 0);
        gb0 = __builtin_amdgcn_mfma_f64_16x16x4f64(s0, s0, gb0, 0, 0, 0);
        ga1 = __builtin_amdgcn_mfma_f64_16x16x4f64(s1, t1, ga1, 0, 0, 0);
        gb1 = __builtin_amdgcn_mfma_f64_16x16x4f64(s1, s1, gb1, 0, 0, 0);
    }
    if (q < q1) {
        const int64_t r0 = q * 4 + kk;
        double s0 = 0.0, t0 = 0.0;
        if (on && r0 < a.n) {
            s0 = S[r0 * a.k + j];
            t0 = AS[r0 * a.k + j];
        }
        ga0 = __builtin_amdgcn_mfma_f64_16x16x4f64(s0, t0, ga0, 0, 0, 0);
        gb0 = __builtin_amdgcn_mfma_f64_16x16x4f64(s0, s0, gb0, 0, 0, 0);
    }
    __shared__ double red[kGramThreads / 64][2 * kGramTile];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int e = (4 * v + kk) * 16 + c;
        red[wave][e] = ga0[v] + ga1[v];
        red[wave][kGramTile + e] = gb0[v] + gb1[v];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * kGramTile; e += kGramThreads) {
        double t = red[0][e];
#pragma unroll
        for (int w = 1; w < kGramThreads / 64; ++w) t += red[w][e];
        part[(int64_t)blockIdx.x * 2 * kGramTile + e] = t;
    }
}

// Both reductions of a step in one launch: workgroup e < wa writes
// oa[e] = sum over p < na of pa[p * wa + e] (the Gram tiles), workgroup
// wa + e writes ob[e] = sum over p < nb of pb[p * wb + e] (the residual
// norms of the previous update); each sum in a fixed tree order
// (deterministic).
__global__ __launch_bounds__(256) void k_sum_two(const double *__restrict__ pa, int na, int wa,
                                                 double *__restrict__ oa, const double *__restrict__ pb, int nb,
                                                 int wb, double *__restrict__ ob) {
    __shared__ double sh[256];
    const bool first = (int)blockIdx.x < wa;
    const int e = first ? (int)blockIdx.x : (int)blockIdx.x - wa;
    const double *part = first ? pa : pb;
    const int nparts = first ? na : nb, width = first ? wa : wb;
    double t = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 256) t += part[(int64_t)p * width + e];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) (first ? oa : ob)[e] = sh[0];
}

struct UpdArgs {
    double *x, *ax, *w, *aw, *p, *ap, *r;  // n x K row-major blocks, 16-byte aligned
    const double *coef;                     // (NB K) x K, row-major
    const double *theta;                    // K Ritz values
    int64_t n;
};

typedef double d2v __attribute__((ext_vector_type(2)));

// One row of a block: 16-byte accesses when K is even.
template <int K> __device__ __forceinline__ void load_row(const double *p, double (&o)[K]) {
    if constexpr (K % 2 == 0) {
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const d2v v = *reinterpret_cast<const d2v *>(p + 2 * i);
            o[2 * i] = v.x;
            o[2 * i + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) o[i] = p[i];
    }
}
template <int K> __device__ __forceinline__ void store_row(double *p, const double (&o)[K]) {
    if constexpr (K % 2 == 0) {
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            d2v v;
            v.x = o[2 * i];
            v.y = o[2 * i + 1];
            *reinterpret_cast<d2v *>(p + 2 * i) = v;
        }
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) p[i] = o[i];
    }
}

// X <- S c, A X <- (A S) c, P <- [W, P] c_(W,P), A P likewise (NB >= 2),
// R = A X - X diag(theta); per-workgroup partial sums of R_j^2 (wavefront
// shuffles, then the four wavefronts in a fixed order).
template <int K, int NB>
__global__ __launch_bounds__(kUpdThreads) void k_lob_update(UpdArgs a, double *__restrict__ part) {
    const int64_t row = (int64_t)blockIdx.x * kUpdThreads + threadIdx.x;
    double r2[K];
#pragma unroll
    for (int j = 0; j < K; ++j) r2[j] = 0.0;
    if (row < a.n) {
        double s[NB][K], t[NB][K];
        load_row<K>(a.x + row * K, s[0]);
        load_row<K>(a.ax + row * K, t[0]);
        if constexpr (NB > 1) {
            load_row<K>(a.w + row * K, s[1]);
            load_row<K>(a.aw + row * K, t[1]);
        }
        if constexpr (NB > 2) {
            load_row<K>(a.p + row * K, s[2]);
            load_row<K>(a.ap + row * K, t[2]);
        }
        double xn[K], axn[K], pn[K], apn[K], rn[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            double px = 0.0, pa = 0.0;
#pragma unroll
            for (int b = 1; b < NB; ++b)
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    const double cf = a.coef[(b * K + c) * K + j];
                    px = fma(s[b][c], cf, px);
                    pa = fma(t[b][c], cf, pa);
                }
            double xx = px, xa = pa;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const double cf = a.coef[c * K + j];
                xx = fma(s[0][c], cf, xx);
                xa = fma(t[0][c], cf, xa);
            }
            xn[j] = xx;
            axn[j] = xa;
            pn[j] = px;
            apn[j] = pa;
            rn[j] = xa - a.theta[j] * xx;
            r2[j] = rn[j] * rn[j];
        }
        store_row<K>(a.x + row * K, xn);
        store_row<K>(a.ax + row * K, axn);
        store_row<K>(a.r + row * K, rn);
        if constexpr (NB > 1) {
            store_row<K>(a.p + row * K, pn);
            store_row<K>(a.ap + row * K, apn);
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) r2[j] += __shfl_xor(r2[j], off, 64);
    __shared__ double sh[kUpdThreads / 64][K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < K; ++j) sh[wave][j] = r2[j];
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double t = sh[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kUpdThreads / 64; ++w) t += sh[w][threadIdx.x];
        part[(int64_t)blockIdx.x * K + threadIdx.x] = t;
    }
}

template <int K>
void launch_update(const UpdArgs &a, int nb, double *part, int grid, hipStream_t s) {
    if (nb == 1) hipLaunchKernelGGL((k_lob_update<K, 1>), dim3(grid), dim3(kUpdThreads), 0, s, a, part);
    else if (nb == 2) hipLaunchKernelGGL((k_lob_update<K, 2>), dim3(grid), dim3(kUpdThreads), 0, s, a, part);
    else hipLaunchKernelGGL((k_lob_update<K, 3>), dim3(grid), dim3(kUpdThreads), 0, s, a, part);
    SAIT_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Host: Rayleigh-Ritz of order m <= 15.
// ---------------------------------------------------------------------------

// Cyclic Jacobi eigen-decomposition of the symmetric m x m matrix C (row-
// major, overwritten): eigenvalues ascending in w, eigenvectors in the
// columns of V.
void jacobi_eigen(int m, std::vector<double> &C, std::vector<double> &w, std::vector<double> &V) {
    V.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
    double fro = 0.0;
    for (double x : C) fro += x * x;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) off += C[(size_t)p * m + q] * C[(size_t)p * m + q];
        if (off <= 1e-32 * fro || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = C[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = C[(size_t)p * m + p], aqq = C[(size_t)q * m + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
                for (int i = 0; i < m; ++i) {  // columns p, q
                    const double cip = C[(size_t)i * m + p], ciq = C[(size_t)i * m + q];
                    C[(size_t)i * m + p] = cs * cip - sn * ciq;
                    C[(size_t)i * m + q] = sn * cip + cs * ciq;
                }
                for (int i = 0; i < m; ++i) {  // rows p, q
                    const double cpi = C[(size_t)p * m + i], cqi = C[(size_t)q * m + i];
                    C[(size_t)p * m + i] = cs * cpi - sn * cqi;
                    C[(size_t)q * m + i] = sn * cpi + cs * cqi;
                }
                for (int i = 0; i < m; ++i) {
                    const double vip = V[(size_t)i * m + p], viq = V[(size_t)i * m + q];
                    V[(size_t)i * m + p] = cs * vip - sn * viq;
                    V[(size_t)i * m + q] = sn * vip + cs * viq;
                }
            }
    }
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return C[(size_t)a * m + a] < C[(size_t)b * m + b]; });
    std::vector<double> Vs((size_t)m * m);
    w.resize(m);
    for (int jj = 0; jj < m; ++jj) {
        w[jj] = C[(size_t)order[jj] * m + order[jj]];
        for (int i = 0; i < m; ++i) Vs[(size_t)i * m + jj] = V[(size_t)i * m + order[jj]];
    }
    V.swap(Vs);
}

// k smallest Ritz pairs of (GA, GB) (m x m, leading block of 16 x 16
// tiles): theta[k], coef (m x k row-major).  false if the unit-diagonal
// scaled GB has a Cholesky pivot <= pivot_min.
bool rayleigh_ritz(int m, int k, const double *GA16, const double *GB16, std::vector<double> &theta,
                   std::vector<double> &coef, double pivot_min) {
    std::vector<double> d(m), A((size_t)m * m), B((size_t)m * m), L((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) {
        const double g = GB16[i * 16 + i];
        if (!(g > 0.0)) return false;
        d[i] = 1.0 / std::sqrt(g);
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            A[(size_t)i * m + j] = 0.5 * (GA16[i * 16 + j] + GA16[j * 16 + i]) * d[i] * d[j];
            B[(size_t)i * m + j] = GB16[i * 16 + j] * d[i] * d[j];
        }
    for (int j = 0; j < m; ++j) {  // B = L L^T
        double s = B[(size_t)j * m + j];
        for (int q = 0; q < j; ++q) s -= L[(size_t)j * m + q] * L[(size_t)j * m + q];
        if (!(s > pivot_min)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double t = B[(size_t)i * m + j];
            for (int q = 0; q < j; ++q) t -= L[(size_t)i * m + q] * L[(size_t)j * m + q];
            L[(size_t)i * m + j] = t / ljj;
        }
    }
    // Y = L^-1 A (columns by forward substitution), C = L^-1 Y^T = L^-1 A L^-T
    std::vector<double> Y((size_t)m * m), Cm((size_t)m * m);
    auto fwd = [&](const std::vector<double> &Rhs, std::vector<double> &Out) {
        for (int col = 0; col < m; ++col)
            for (int i = 0; i < m; ++i) {
                double t = Rhs[(size_t)i * m + col];
                for (int q = 0; q < i; ++q) t -= L[(size_t)i * m + q] * Out[(size_t)q * m + col];
                Out[(size_t)i * m + col] = t / L[(size_t)i * m + i];
            }
    };
    fwd(A, Y);
    std::vector<double> Yt((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Yt[(size_t)i * m + j] = Y[(size_t)j * m + i];
    fwd(Yt, Cm);
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j) {
            const double avg = 0.5 * (Cm[(size_t)i * m + j] + Cm[(size_t)j * m + i]);
            Cm[(size_t)i * m + j] = Cm[(size_t)j * m + i] = avg;
        }
    std::vector<double> w, V;
    jacobi_eigen(m, Cm, w, V);
    // coef = D L^-T V[:, :k]  (back substitution with L^T)
    theta.assign(w.begin(), w.begin() + k);
    coef.assign((size_t)m * k, 0.0);
    for (int col = 0; col < k; ++col)
        for (int i = m - 1; i >= 0; --i) {
            double t = V[(size_t)i * m + col];
            for (int q = i + 1; q < m; ++q) t -= L[(size_t)q * m + i] * coef[(size_t)q * k + col];
            coef[(size_t)i * k + col] = t / L[(size_t)i * m + i];
        }
    for (int i = 0; i < m; ++i)
        for (int col = 0; col < k; ++col) coef[(size_t)i * k + col] *= d[i];
    return true;
}

int gram_grid(int64_t quads) {
    const int64_t waves = (quads + 7) / 8;  // about 8 quads per wavefront
    return (int)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 1024));
}

}  // namespace

struct Lobpcg::Bufs {
    DevBuf x, ax, w, aw, p, ap, r, gpart, upart, small;  // x: aligned working copy of X
    double *host = nullptr;  // pinned: 2 tiles + K norms
    ~Bufs() {
        if (host) (void)hipHostFree(host);
    }
};

Lobpcg::Lobpcg() : b_(new Bufs) {}
Lobpcg::~Lobpcg() { delete b_; }

int Lobpcg::run(Allocator *alloc, int64_t n, int k, double *X, const BlockOp &applyA, const BlockOp &applyT,
                const sait_eig_opts &o, double *lambda, double *history, sait_eig_info *info, hipStream_t s) {
    if (k < 1 || k > kMaxBlock) fail(SAIT_E_INVALID, "LOBPCG block size must be 1..5");
    if (n < 3 * (int64_t)k) fail(SAIT_E_INVALID, "LOBPCG needs n >= 3 k");
    if (o.maxit < 0) fail(SAIT_E_INVALID, "maxit must be >= 0");
    if (!(o.tol >= 0.0)) fail(SAIT_E_INVALID, "tol must be >= 0");
    if (!X || !lambda) fail(SAIT_E_INVALID, "null X or lambda");
    const size_t blk = (size_t)n * k * sizeof(double);
    Bufs &B = *b_;
    for (DevBuf *d : {&B.x, &B.ax, &B.w, &B.aw, &B.p, &B.ap, &B.r})
        if (d->bytes() < blk) d->alloc(alloc, blk);
    double *Xi = B.x.as<double>();
    const int64_t quads = (n + 3) / 4;
    const int ggrid = gram_grid(quads);
    const int ugrid = (int)((n + kUpdThreads - 1) / kUpdThreads);
    if (B.gpart.bytes() < (size_t)ggrid * 2 * kGramTile * sizeof(double))
        B.gpart.alloc(alloc, (size_t)ggrid * 2 * kGramTile * sizeof(double));
    if (B.upart.bytes() < (size_t)ugrid * kMaxBlock * sizeof(double))
        B.upart.alloc(alloc, (size_t)ugrid * kMaxBlock * sizeof(double));
    // device and pinned host layout: two tiles, K squared norms, (3K) x K
    // coefficients, K Ritz values
    const size_t small = (2 * kGramTile + kMaxBlock + 3 * kMaxBlock * kMaxBlock + kMaxBlock) * sizeof(double);
    if (B.small.bytes() < small) B.small.alloc(alloc, small);
    if (!B.host) SAIT_HIP(hipHostMalloc((void **)&B.host, small, hipHostMallocDefault));
    double *dG = B.small.as<double>();          // 512: the two tiles
    double *dnorm = dG + 2 * kGramTile;         // K squared residual norms
    double *dcoef = dnorm + kMaxBlock;          // (3K) x K coefficients
    double *dtheta = dcoef + 3 * kMaxBlock * kMaxBlock;
    double *h = B.host;

    auto gram = [&](int nb, bool with_norms) {
        GramArgs g{};
        g.s[0] = Xi;
        g.s[1] = B.w.as<double>();
        g.s[2] = B.p.as<double>();
        g.as[0] = B.ax.as<double>();
        g.as[1] = B.aw.as<double>();
        g.as[2] = B.ap.as<double>();
        g.n = n;
        g.quads = quads;
        g.k = k;
        g.nb = nb;
        hipLaunchKernelGGL(k_gram, dim3(ggrid), dim3(kGramThreads), 0, s, g, B.gpart.as<double>());
        SAIT_LAUNCH_CHECK();
        // the norms of the last update's residual are reduced in the same launch
        const int wb = with_norms ? k : 0;
        hipLaunchKernelGGL(k_sum_two, dim3(2 * kGramTile + wb), dim3(256), 0, s, B.gpart.as<double>(), ggrid,
                           2 * kGramTile, dG, B.upart.as<double>(), ugrid, k, dnorm);
        SAIT_LAUNCH_CHECK();
    };
    auto readback = [&](bool with_norms) {
        const size_t bytes = (2 * kGramTile + (with_norms ? k : 0)) * sizeof(double);
        SAIT_HIP(hipMemcpyAsync(h, dG, bytes, hipMemcpyDeviceToHost, s));
        SAIT_HIP(hipStreamSynchronize(s));
    };
    auto update = [&](int nb, const std::vector<double> &theta, const std::vector<double> &coef) {
        // coefficients and Ritz values staged in pinned memory (the next
        // readback's synchronisation orders its reuse after this copy)
        double *hc = h + (dcoef - dG);
        std::copy(coef.begin(), coef.end(), hc);
        std::copy(theta.begin(), theta.end(), hc + (dtheta - dcoef));
        SAIT_HIP(hipMemcpyAsync(dcoef, hc, (size_t)((dtheta - dcoef) + k) * sizeof(double), hipMemcpyHostToDevice, s));
        UpdArgs u{};
        u.x = Xi;
        u.ax = B.ax.as<double>();
        u.w = B.w.as<double>();
        u.aw = B.aw.as<double>();
        u.p = B.p.as<double>();
        u.ap = B.ap.as<double>();
        u.r = B.r.as<double>();
        u.coef = dcoef;
        u.theta = dtheta;
        u.n = n;
        switch (k) {
        case 1: launch_update<1>(u, nb, B.upart.as<double>(), ugrid, s); break;
        case 2: launch_update<2>(u, nb, B.upart.as<double>(), ugrid, s); break;
        case 3: launch_update<3>(u, nb, B.upart.as<double>(), ugrid, s); break;
        case 4: launch_update<4>(u, nb, B.upart.as<double>(), ugrid, s); break;
        default: launch_update<5>(u, nb, B.upart.as<double>(), ugrid, s); break;
        }
    };

    // Rayleigh-Ritz on span(X0)
    SAIT_HIP(hipMemcpyAsync(Xi, X, blk, hipMemcpyDeviceToDevice, s));
    applyA(Xi, B.ax.as<double>(), s);
    gram(1, false);
    readback(false);
    std::vector<double> theta, coef;
    if (!rayleigh_ritz(k, k, h, h + kGramTile, theta, coef, kPivotMin))
        fail(SAIT_E_INVALID, "LOBPCG: the start block is numerically rank deficient");
    update(1, theta, coef);

    int status = 1, it = 0, p_drops = 0;
    bool has_p = false;
    double relres = 0.0;
    for (it = 0;; ++it) {
        applyT(B.r.as<double>(), B.w.as<double>(), s);
        applyA(B.w.as<double>(), B.aw.as<double>(), s);
        const int nb = has_p ? 3 : 2;
        gram(nb, true);
        readback(true);
        relres = 0.0;
        for (int j = 0; j < k; ++j)
            relres = std::max(relres, std::sqrt(std::max(h[2 * kGramTile + j], 0.0)) / std::fabs(theta[j]));
        if (history) history[it] = relres;
        if (relres <= o.tol) {
            status = 0;
            break;
        }
        if (it == o.maxit) break;
        // the [X, W] pencil is the leading 2k x 2k part of the [X, W, P] tiles
        int use = nb;
        bool ok = rayleigh_ritz(use * k, k, h, h + kGramTile, theta, coef, use == 3 ? kPivotP : kPivotMin);
        if (!ok && use == 3) {
            ++p_drops;
            use = 2;
            ok = rayleigh_ritz(use * k, k, h, h + kGramTile, theta, coef, kPivotMin);
        }
        if (!ok) {
            status = 2;
            break;
        }
        update(use, theta, coef);
        has_p = true;
    }
    SAIT_HIP(hipMemcpyAsync(X, Xi, blk, hipMemcpyDeviceToDevice, s));
    SAIT_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) lambda[j] = theta[j];
    if (info) {
        info->iterations = it;
        info->status = status == 0 ? SAIT_OK : status == 1 ? SAIT_NOT_CONVERGED : SAIT_BREAKDOWN;
        info->p_drops = p_drops;
        info->relres = relres;
    }
    return status == 0 ? SAIT_OK : status == 1 ? SAIT_NOT_CONVERGED : SAIT_BREAKDOWN;
}

}  // namespace sait
