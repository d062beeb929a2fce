// Host incomplete factorisations feeding SAIT (Sec. 3.1: L, U of an ILU
// preconditioner are the triangular matrices SAIT approximates).
//
//  * ILU(0): "level-0 ILU" (Sec. 4) -- Gaussian elimination restricted to
//    the pattern of A, row-wise (IKJ) order, Doolittle form (unit lower L,
//    stored with its diagonal so that D_L = I in the Jacobi split).
//  * ILUT(tau, p): Saad's dual-threshold incomplete LU (Iterative Methods
//    for Sparse Linear Systems, 2nd ed., Sec. 10.4): tau_i = tau*||a_i||_2,
//    multipliers below tau_i are dropped during elimination, and after it
//    every off-diagonal below tau_i is dropped and only the p largest of
//    each of the L and U parts are kept (ties to the smaller column).
//
// Compiled with -ffp-contract=off: a - l*u is a rounded product followed by
// a rounded difference.  Parallel ILU is outside the paper's scope (its
// introduction names it as the first, separate problem); it runs on the host.
#include <algorithm>
#include <cmath>
#include <functional>
#include <limits>
#include <queue>

#include "sait_internal.h"

namespace sait {

void validate_csr(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const char *what) {
    if (n < 0) fail(SAIT_E_INVALID, std::string(what) + ": negative n");
    if (n > INT32_MAX - 1) fail(SAIT_E_INVALID, std::string(what) + ": n exceeds int32 indexing");
    if (!rp) fail(SAIT_E_INVALID, std::string(what) + ": null row_ptr");
    if (rp[0] != 0) fail(SAIT_E_INVALID, std::string(what) + ": row_ptr[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) fail(SAIT_E_INVALID, std::string(what) + ": row_ptr decreases at row " + std::to_string(i));
    int64_t nnz = rp[n];
    if (nnz > 0 && !ci) fail(SAIT_E_INVALID, std::string(what) + ": null col_idx");
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n)
                fail(SAIT_E_INVALID, std::string(what) + ": column out of range in row " + std::to_string(i));
            if (p > rp[i] && ci[p] <= ci[p - 1])
                fail(SAIT_E_INVALID, std::string(what) + ": columns not sorted/unique in row " + std::to_string(i));
        }
    }
    if (v)
        for (int64_t p = 0; p < nnz; ++p)
            if (!std::isfinite(v[p])) fail(SAIT_E_NONFINITE, std::string(what) + ": non-finite value");
}

// ---------------------------------------------------------------------------
// ILU(0).  For row i and each k < i present in row i (ascending):
//   l_ik = a_ik / u_kk ;  a_ij -= l_ik * u_kj  for j > k present in both rows.
// Matches between row i and row k are found by walking both sorted rows.
// ---------------------------------------------------------------------------
void host_ilu0(const HostCsr &A, HostCsr &L, HostCsr &U) {
    const int64_t n = A.n;
    const int32_t *rp = A.rp.data();
    const int32_t *ci = A.ci.data();
    std::vector<double> a(A.v);
    std::vector<int64_t> diag(n);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *b = ci + rp[i], *e = ci + rp[i + 1];
        const int32_t *d = std::lower_bound(b, e, (int32_t)i);
        if (d == e || *d != i) fail(SAIT_E_ZERO_PIVOT, "ILU(0): missing diagonal in row " + std::to_string(i));
        diag[i] = d - ci;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rp[i]; p < diag[i]; ++p) {
            const int64_t k = ci[p];
            a[p] = a[p] / a[diag[k]];
            const double lik = a[p];
            // walk row k (entries after its diagonal) against row i (entries after p)
            int64_t q = diag[k] + 1, qe = rp[k + 1];
            int64_t t = p + 1, te = rp[i + 1];
            while (q < qe && t < te) {
                if (ci[q] < ci[t]) ++q;
                else if (ci[q] > ci[t]) ++t;
                else {
                    a[t] = a[t] - lik * a[q];
                    ++q;
                    ++t;
                }
            }
        }
        const double piv = a[diag[i]];
        if (piv == 0.0) fail(SAIT_E_ZERO_PIVOT, "ILU(0): zero pivot in row " + std::to_string(i));
        if (!std::isfinite(piv)) fail(SAIT_E_NONFINITE, "ILU(0): non-finite pivot in row " + std::to_string(i));
    }
    L.n = U.n = n;
    L.rp.assign(n + 1, 0);
    U.rp.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        L.rp[i + 1] = L.rp[i] + (int32_t)(diag[i] - rp[i]) + 1;
        U.rp[i + 1] = U.rp[i] + (int32_t)(rp[i + 1] - diag[i]);
    }
    L.ci.resize(L.rp[n]);
    L.v.resize(L.rp[n]);
    U.ci.resize(U.rp[n]);
    U.v.resize(U.rp[n]);
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = L.rp[i];
        for (int64_t p = rp[i]; p < diag[i]; ++p, ++o) {
            L.ci[o] = ci[p];
            L.v[o] = a[p];
        }
        L.ci[o] = (int32_t)i;
        L.v[o] = 1.0;
        o = U.rp[i];
        for (int64_t p = diag[i]; p < rp[i + 1]; ++p, ++o) {
            U.ci[o] = ci[p];
            U.v[o] = a[p];
        }
    }
}

// ---------------------------------------------------------------------------
// ILUT(tau, p).
// ---------------------------------------------------------------------------
namespace {
struct Cand {
    int32_t col;
    double val;
};
// Larger magnitude first; equal magnitudes: smaller column first.
inline bool bigger(const Cand &x, const Cand &y) {
    const double ax = std::fabs(x.val), ay = std::fabs(y.val);
    if (ax != ay) return ax > ay;
    return x.col < y.col;
}
void keep_largest(std::vector<Cand> &c, int p) {
    if ((int64_t)c.size() > p) {
        std::nth_element(c.begin(), c.begin() + p, c.end(), bigger);
        c.resize(p);
    }
    std::sort(c.begin(), c.end(), [](const Cand &x, const Cand &y) { return x.col < y.col; });
}
}  // namespace

void host_ilut(const HostCsr &A, double tau, int fill, HostCsr &L, HostCsr &U) {
    if (!(tau >= 0.0) || fill < 0) fail(SAIT_E_INVALID, "ILUT: need tau >= 0 and fill >= 0");
    const int64_t n = A.n;
    std::vector<double> w(n, 0.0);
    std::vector<char> in(n, 0);
    std::vector<int32_t> touched;
    std::vector<double> udiag(n);
    std::vector<Cand> lo, up;
    L = HostCsr();
    U = HostCsr();
    L.n = U.n = n;
    L.rp.assign(1, 0);
    U.rp.assign(1, 0);
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> pending;
    for (int64_t i = 0; i < n; ++i) {
        double ss = 0.0;
        touched.clear();
        for (int64_t q = A.rp[i]; q < A.rp[i + 1]; ++q) {
            const int32_t j = A.ci[q];
            w[j] = A.v[q];
            in[j] = 1;
            touched.push_back(j);
            if (j < i) pending.push(j);
            ss = ss + A.v[q] * A.v[q];
        }
        const double tol = tau * std::sqrt(ss);
        while (!pending.empty()) {
            const int32_t k = pending.top();
            pending.pop();
            if (w[k] == 0.0) continue;
            w[k] = w[k] / udiag[k];
            if (std::fabs(w[k]) < tol) {
                w[k] = 0.0;
                continue;
            }
            const double lk = w[k];
            for (int64_t q = U.rp[k] + 1; q < U.rp[k + 1]; ++q) {  // off-diagonals of row k of U
                const int32_t j = U.ci[q];
                if (!in[j]) {
                    in[j] = 1;
                    w[j] = 0.0;
                    touched.push_back(j);
                    if (j < i) pending.push(j);
                }
                w[j] = w[j] - lk * U.v[q];
            }
        }
        lo.clear();
        up.clear();
        for (int32_t j : touched) {
            const double x = w[j];
            if (j == i || x == 0.0 || std::fabs(x) < tol) continue;
            (j < i ? lo : up).push_back({j, x});
        }
        keep_largest(lo, fill);
        keep_largest(up, fill);
        const double d = in[i] ? w[i] : 0.0;
        if (d == 0.0) fail(SAIT_E_ZERO_PIVOT, "ILUT: zero pivot in row " + std::to_string(i));
        if (!std::isfinite(d)) fail(SAIT_E_NONFINITE, "ILUT: non-finite pivot in row " + std::to_string(i));
        udiag[i] = d;
        for (const Cand &c : lo) {
            L.ci.push_back(c.col);
            L.v.push_back(c.val);
        }
        L.ci.push_back((int32_t)i);
        L.v.push_back(1.0);
        L.rp.push_back((int32_t)L.ci.size());
        U.ci.push_back((int32_t)i);
        U.v.push_back(d);
        for (const Cand &c : up) {
            U.ci.push_back(c.col);
            U.v.push_back(c.val);
        }
        U.rp.push_back((int32_t)U.ci.size());
        for (int32_t j : touched) {
            w[j] = 0.0;
            in[j] = 0;
        }
    }
}


// ILU(p) by levels of fill ("level-1 ILU", Sec. 4): the level of an entry
// of A is 0; eliminating (i, k), k < i in increasing order, reaches (i, j)
// for every j > k of row k of U at level lev(i,k) + lev(k,j) + 1; positions
// reached at a level <= p form the pattern, and the factors are the ILU(0)
// elimination over it (A's values there, zeros at the fill positions).
void host_iluk_pattern(const HostCsr &A, int level, HostCsr &E) {
    if (level < 0) fail(SAIT_E_INVALID, "ILU(k): level must be >= 0");
    const int64_t n = A.n;
    constexpr int kNone = std::numeric_limits<int>::max();
    std::vector<int> lev(n, kNone);
    std::vector<int32_t> upos(n + 1, 0);   // U-part (columns > row) levels of finished rows
    std::vector<int32_t> ucol;
    std::vector<int> ulev;
    E = HostCsr{};                           // A on the level-p pattern
    E.n = n;
    E.rp.assign(n + 1, 0);
    std::vector<int32_t> row;
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> pending;
    for (int64_t i = 0; i < n; ++i) {
        row.clear();
        for (int32_t q = A.rp[i]; q < A.rp[i + 1]; ++q) {
            const int32_t j = A.ci[q];
            lev[j] = 0;
            row.push_back(j);
            if (j < i) pending.push(j);
        }
        while (!pending.empty()) {
            const int32_t k = pending.top();
            pending.pop();
            const int lk = lev[k];
            for (int32_t q = upos[k]; q < upos[k + 1]; ++q) {
                const int32_t j = ucol[q];
                const int reach = lk + ulev[q] + 1;
                if (reach > level) continue;
                if (lev[j] == kNone) {
                    lev[j] = reach;
                    row.push_back(j);
                    if (j < i) pending.push(j);
                } else if (reach < lev[j]) {
                    lev[j] = reach;
                }
            }
        }
        std::sort(row.begin(), row.end());
        size_t qa = A.rp[i];
        for (const int32_t j : row) {
            E.ci.push_back(j);
            // A's value where A has the entry (both lists sorted), 0 at fill
            while (qa < (size_t)A.rp[i + 1] && A.ci[qa] < j) ++qa;
            E.v.push_back((qa < (size_t)A.rp[i + 1] && A.ci[qa] == j) ? A.v[qa] : 0.0);
            if (j > i) {
                ucol.push_back(j);
                ulev.push_back(lev[j]);
            }
            lev[j] = kNone;
        }
        E.rp[i + 1] = (int32_t)E.ci.size();
        upos[i + 1] = (int32_t)ucol.size();
    }
}

void host_iluk(const HostCsr &A, int level, HostCsr &L, HostCsr &U) {
    HostCsr E;
    host_iluk_pattern(A, level, E);
    host_ilu0(E, L, U);
}

}  // namespace sait
