// Internal declarations of libsait (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "sait.h"

namespace sait {

// ---------------------------------------------------------------------------
// Error model: everything below the C ABI throws sait::Error; the extern "C"
// wrappers catch it, store the message thread-locally and return the status.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string &msg) : std::runtime_error(msg), status(st) {}
};

[[noreturn]] void fail(int status, const std::string &msg);

#define SAIT_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::sait::fail(e_ == hipErrorOutOfMemory ? SAIT_E_NOMEM : SAIT_E_DEVICE,      \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
    } while (0)

#define SAIT_LAUNCH_CHECK() SAIT_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Device memory owned through the handle's allocator.
// ---------------------------------------------------------------------------
struct Allocator {
    sait_allocator user{};
    bool has_user = false;
    void *alloc(size_t bytes);
    void release(void *p);
};

class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { *this = std::move(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            reset();
            p_ = o.p_;
            bytes_ = o.bytes_;
            a_ = o.a_;
            o.p_ = nullptr;
            o.bytes_ = 0;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void alloc(Allocator *a, size_t bytes);
    void reset();
    template <class T> T *as() const { return static_cast<T *>(p_); }
    size_t bytes() const { return bytes_; }
    bool empty() const { return p_ == nullptr; }

  private:
    void *p_ = nullptr;
    size_t bytes_ = 0;
    Allocator *a_ = nullptr;
};

// Host CSR (int32 pointers/indices, FP64 values).
struct HostCsr {
    int64_t n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Device CSR; `v` is FP64, `vs` the stored copy in the storage precision
// (points at `v` for SAIT_F64).
struct DevCsr {
    int64_t n = 0, nnz = 0;
    int precision = SAIT_F64;
    DevBuf rp, ci, v, vs;
    // Row blocks of the LDS-staged SpMV, one partition per chunk size (2040
    // and 4088 entries): block b covers rows [brow[b], brow[b+1]) -- at most
    // 256 rows and one chunk of entries, or one longer row alone.
    DevBuf brow[2];
    int64_t nblk[2] = {0, 0};
    // Sliced-ELL copy for the one-row-per-lane kernel: slice s holds rows
    // 64 s .. 64 s + 63 (one wavefront), padded to the slice's longest row
    // rounded up to a multiple of 4, in groups of 4 entries per row (256 per
    // group).  With g = sell_ptr[s] + (k / 4) * 256, the column of entry k of
    // row 64 s + l is at g + 4 l + k % 4; its value at the same place for
    // binary32 / bfloat16 storage, and at g + 128 ((k / 2) % 2) + 2 l + k % 2
    // for FP64 (two planes per group).  Padding holds column 0 and value 0
    // and is never used (row lengths come from rp).  Values are in the
    // storage precision.
    DevBuf sell_ptr, sell_ci, sell_v;
    int64_t nslices = 0, sell_nnz = 0;
    const void *stored() const { return precision == SAIT_F64 ? v.as<void>() : vs.as<void>(); }
};

// ---------------------------------------------------------------------------
// Host-side routines (ilu_host.cpp)
// ---------------------------------------------------------------------------
void validate_csr(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const char *what);
void host_ilu0(const HostCsr &A, HostCsr &L, HostCsr &U);
void host_ilut(const HostCsr &A, double tau, int fill, HostCsr &L, HostCsr &U);
void host_iluk(const HostCsr &A, int level, HostCsr &L, HostCsr &U);
// A on its level-p pattern: A's values, explicit zeros at the kept fill.
void host_iluk_pattern(const HostCsr &A, int level, HostCsr &E);

// ---------------------------------------------------------------------------
// SpGEMM construction of the SAIT factors (k_spgemm.hip)
// ---------------------------------------------------------------------------
struct SaitParams {
    int m = 3;
    double tau = 1e-2;
    int cap = 0;        // 0: no per-row cap
    int pattern_p = -1; // >= 0: SAIT_Pat(p, m)
    int precision = SAIT_F64;
    bool right = false; // passes M <- drop(M T~ + I) instead of drop(T~ M + I)
};

// Upload a host CSR.
void upload_csr(Allocator *a, const HostCsr &h, DevCsr &d, hipStream_t s);
// Download a device CSR (FP64 values).
void download_csr(const DevCsr &d, HostCsr &h, hipStream_t s);
// Fine-grained parallel ILU on the pattern of the device matrix E:
// `sweeps` synchronous fixed-point sweeps (k_parilu.hip); L unit lower with
// its diagonal stored, U upper, both on the device.  symmetric: the
// incomplete Cholesky form (structurally symmetric pattern, upper triangle
// of E read, l_ki = u_ik / u_ii).
void parilu_device(Allocator *a, const DevCsr &E, int sweeps, bool symmetric, DevCsr &L, DevCsr &U, hipStream_t s);
// Build M ~ T^-1 for a device-resident triangular T.
void build_sait_factor(Allocator *a, const DevCsr &T, const SaitParams &p, DevCsr &M, hipStream_t s);
// One unscaled pass M_next = drop(T~ M_prev + I), or drop(M_prev T~ + I)
// if right (test entry point).
void sait_single_pass(Allocator *a, const DevCsr &T, const DevCsr &Mprev, bool right, double tau, int cap,
                      DevCsr &Mnext, hipStream_t s);
// Device exclusive scan of int64 counts: out[0..n] (out[n] = total).
void scan_exclusive_i64(Allocator *a, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
// CSR transpose (structure and FP64 values); output rows sorted.
void transpose_csr(Allocator *a, const DevCsr &M, DevCsr &Mt, hipStream_t s);
// perm such that Mt.v[q] = M.v[perm[q]] for Mt = transpose_csr(M).
void transpose_perm(Allocator *a, const DevCsr &M, DevBuf &perm, hipStream_t s);
// dst[q] = src[perm[q]], q < nnz.
void gather_values(int64_t nnz, const int *perm, const double *src, double *dst, hipStream_t s);
// Re-derive the stored-precision copy `vs` of M from its FP64 values.
void cast_values(Allocator *a, DevCsr &M, int precision, hipStream_t s);

// ---------------------------------------------------------------------------
// SpMV / SpMM (k_spmv.hip)
// ---------------------------------------------------------------------------
enum class XKind { F64, F32 };   // element type of the gathered input vector
enum class YKind { F64, F32 };   // element type of the output vector

// y = M x for one CSR factor; lanes = lanes per row (1..64, power of two).
// `resid_b` != nullptr: y = b - M x (FP64 only).
void spmv(const DevCsr &M, const void *x, XKind xk, void *y, YKind yk, int nrhs, int64_t ldx, int64_t ldy,
          int lanes, hipStream_t s, const double *resid_b = nullptr);
int default_lanes(const DevCsr &M);
// Apply kernel shapes: > 0 lanes per row of the wavefront CSR kernel; < 0
// the sliced-ELL (needs prepare_sell) or LDS-staged (needs prepare_stream)
// kernels.
constexpr int kStream8 = -8, kStream = -16;  // LDS-staged CSR, 2040 / 4088-entry chunks
constexpr int kSell = -64, kSell1 = -65;     // sliced ELL, 2 / 1 groups of 4 entries per stage
bool valid_shape(int shape);
// Sliced-ELL copy of M's stored values (needs the storage cast done).
void prepare_sell(Allocator *a, DevCsr &M, hipStream_t s);
// Row blocks for the LDS-staged kernel (host pass over the row pointers).
void prepare_stream(Allocator *a, DevCsr &M, hipStream_t s);

// One Jacobi sweep ynew = (r - N yold) / d on the FP64 sliced-ELL matrix N.
void jacobi_sweep(const DevCsr &N, const double *d, const double *r, const double *yold, double *ynew, hipStream_t s);

// ---------------------------------------------------------------------------
// Comparison preconditioners (k_precond.hip)
// ---------------------------------------------------------------------------
// Jacobi sweeps on a triangular factor T: N = T without its diagonal
// (sliced ELL), d = diag(T).
struct JacobiFactor {
    DevCsr N;
    DevBuf d;
};
void build_jacobi(Allocator *a, const HostCsr &T, JacobiFactor &J, hipStream_t s);
// y = s Jacobi sweeps from zero for T y = r (tmp: n doubles of scratch).
void jacobi_apply(const JacobiFactor &J, int sweeps, const double *r, double *y, double *tmp, hipStream_t s);
// Level-scheduled exact solve with a triangular factor (rows grouped by
// dependency level; level_ptr on the host).
struct LevelFactor {
    DevCsr T;
    DevBuf rows;
    std::vector<int> level_ptr;
};
void build_levels(Allocator *a, const HostCsr &T, bool lower, LevelFactor &F, hipStream_t s);
void level_solve(const LevelFactor &F, const double *b, double *x, hipStream_t s);

// ---------------------------------------------------------------------------
// Krylov building blocks (k_krylov.hip)
// ---------------------------------------------------------------------------
struct GmresState;   // device-resident per-solve state (k_krylov.hip)
struct Krylov;       // host-side driver workspace

}  // namespace sait
