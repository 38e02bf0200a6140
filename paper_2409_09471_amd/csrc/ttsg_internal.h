// Internal declarations shared by the HIP translation units of libttsg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ttsg.h"

namespace ttsg {

// ---------------------------------------------------------------------------
// Errors: internal code throws ttsg::Error; the C ABI layer converts it to a
// negative return code and a thread-local message.
// ---------------------------------------------------------------------------
struct Error : public std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TTSG_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::ttsg::Error(TTSG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TTSG_CHECK(cond, code, msg)                                                      \
    do {                                                                                 \
        if (!(cond)) throw ::ttsg::Error((code), (msg));                                 \
    } while (0)

// ---------------------------------------------------------------------------
// Two-level strided index: x in [0, extent) is split as x0 = x % n0,
// x1 = x / n0 and addressed as x0 * s0 + x1 * s1.  n0 >= extent means the
// index is plain-strided (s1 unused).  Every operand of the contraction kernel
// describes its row, column, reduction and batch index this way, which lets
// one kernel walk the permuted core layouts of the TT sweeps without copies.
// ---------------------------------------------------------------------------
struct Idx2 {
    int32_t n0;
    int64_t s0;
    int64_t s1;
};

__host__ __device__ inline Idx2 idx1(int64_t s) { return Idx2{0x7fffffff, s, 0}; }
__host__ __device__ inline Idx2 idx2(int32_t n0, int64_t s0, int64_t s1) { return Idx2{n0, s0, s1}; }

__device__ __forceinline__ int64_t idx_off(const Idx2& ix, int32_t x) {
    if (x < ix.n0) return (int64_t)x * ix.s0;
    int32_t x1 = x / ix.n0;
    int32_t x0 = x - x1 * ix.n0;
    return (int64_t)x0 * ix.s0 + (int64_t)x1 * ix.s1;
}

// Largest element offset an index of `extent` values can reach.
inline int64_t idx_max(const Idx2& ix, int32_t extent) {
    if (extent <= 0) return 0;
    const int32_t x = extent - 1;
    if (extent <= ix.n0) return (int64_t)x * ix.s0;
    const int64_t inner = (int64_t)(ix.n0 - 1) * ix.s0;
    return inner + (int64_t)(x / ix.n0) * ix.s1;
}

// Host-side launch check (enabled by TTSG_CHECK_BOUNDS=1): the byte range
// [p, p + bytes) must lie inside the device allocation that contains p.
void check_range(const void* p, size_t bytes, const char* what);
bool bounds_checking();

// Launch measurement (stats.hip): when enabled, StatScope hands the launch a
// device slot in which its workgroups record the earliest start and latest end
// of the wall clock (so host gaps between launches are not counted), plus an
// auxiliary maximum (e.g. Jacobi sweeps).  Kernels take the slot pointer
// (nullptr when measurement is off) and call slot_begin / slot_end.
// A launch's workgroups spread their atomics over kSlotLanes sub-slots (by
// flat workgroup index, which also spreads them over the XCDs), so that a
// launch of thousands of workgroups does not serialize on one address.
constexpr int kSlotLanes = 8;
struct DevSlot {
    unsigned long long start_inv[kSlotLanes];   // max over workgroups of ~t_start
    unsigned long long end[kSlotLanes];         // max over workgroups of t_end
    unsigned long long aux;
    unsigned long long pad[7];
};
bool stats_on();
// Count one host-side event of class cls while measurement is on.
void stats_event(int cls);
struct StatScope {
    StatScope(int cls, double flops, double bytes, hipStream_t st);
    ~StatScope();
    DevSlot* slot() const { return slot_; }
    // Attach the launch shape (e.g. M, N, K, batch, splits) to the record; it is
    // written out by ttsg_stats_read when TTSG_SHAPE_LOG names a file.
    void shape(int a, int b, int c, int d, int e);
    DevSlot* slot_ = nullptr;
    int64_t rec_ = -1;
};

__device__ __forceinline__ int slot_lane() {
    return (int)((blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) & (kSlotLanes - 1));
}
__device__ __forceinline__ void slot_begin(DevSlot* s) {
    if (s != nullptr && threadIdx.x == 0) atomicMax(&s->start_inv[slot_lane()], ~(unsigned long long)wall_clock64());
}
// Call from all threads of the workgroup (contains a barrier when s != nullptr).
__device__ __forceinline__ void slot_end(DevSlot* s, unsigned long long aux = 0) {
    if (s == nullptr) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(&s->end[slot_lane()], (unsigned long long)wall_clock64());
        if (aux) atomicMax(&s->aux, aux);
    }
}

// C[b][m][n] = alpha * sum_k A[b][m][k] * B[b][k][n] + beta * C[b][m][n]
struct ContractDesc {
    int32_t M, N, K, batch;
    Idx2 am, ak, bk, bn, cm, cn;
    Idx2 ab, bb, cb;
    double alpha, beta;
    int32_t c_f64;   // F32/BF16 arithmetic writing a float64 C (strides in its elements)
    // Khatri-Rao step (kr_P != nullptr; float64/float32, operator rank kr_Rl of
    // 1..3): the A operand is not read but formed while it is staged,
    // A[m][k] = sum_al P[(j Rl + al) rl + a] SA[((j Rl + al) Rr + be) n + i]
    // with m = j Rr + be and k = a n + i (the A pointer and the am/ak/ab
    // strides are then unused).
    const void* kr_P;
    const void* kr_SA;
    int32_t kr_rl, kr_n, kr_Rl, kr_Rr;
    // Optional addend (c_add != nullptr, C's element type, c_f64 == 0):
    // C = alpha A B + beta C + X with X[b][m][n] at strides xb/xm/xn, added
    // last (the identity block of an operator step summed with a dense one).
    const void* c_add;
    Idx2 xb, xm, xn;
};

// Arithmetic of the contraction kernels.  F32 and BF16 share float32
// storage; BF16 rounds the operands to bfloat16 as they enter the matrix cores.
enum class Prec { F64 = 0, F32 = 1, BF16 = 2 };

class Arena;
// Launchers (contract.hip).  A/B are float64 for F64 and float32 otherwise
// (BF16 multiplies their bfloat16 roundings); C is float64 for F64 and float32
// otherwise.
// With an arena, reductions too long for the output tiles to fill the chip are
// split over several workgroups (partials in the arena, summed in fixed order).
void contract(Prec p, const ContractDesc& d, const void* A, const void* B, void* C, hipStream_t st,
              Arena* ar = nullptr);
// Tile autotuner of the contraction kernel (contract.hip).
int autotune_set(int on);
bool autotune_is_on();
int autotune_save(const char* path);
int autotune_load(const char* path);
int autotune_clear();

// Element-wise helpers (misc.hip).
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);   // y = a x + b y
void fill(int64_t n, double v, double* y, hipStream_t st);
// Pinned host staging for the small read-backs and uploads of the host-side
// rank decisions (a copy to or from pinned memory needs no bounce buffer:
// measured 14 us instead of 23 us per read-back and synchronization).  One
// buffer per host thread with two regions of kStageDoubles doubles: region 0
// for read-backs, region 1 for uploads, which must stay untouched until the
// stream that copies them has been synchronized.  nullptr when pinned memory
// cannot be had; callers then use pageable memory.
constexpr size_t kStageDoubles = 16384;
double* host_stage(int region);
// Copy `bytes` from device memory to the host through region 0 of the stage
// (or into `fallback` when the stage is unavailable or too small), then
// synchronize st.  Returns the host copy.
const void* read_back(const void* dev, size_t bytes, void* fallback, hipStream_t st);
void copy_f64(int64_t n, const double* x, double* y, hipStream_t st);
void convert_f64_f32(int64_t n, const double* x, float* y, hipStream_t st);
void convert_f32_f64(int64_t n, const float* x, double* y, hipStream_t st);
void convert_f64_bf16(int64_t n, const double* x, uint16_t* y, hipStream_t st);
void scale_f64(int64_t n, double a, double* y, hipStream_t st);
// y[i] = sum_t coef[t] * x_t[i] for up to 8 sources (coefficients in device memory).
void lin_comb_dev(int64_t n, int32_t nterms, const double* const* xs, const double* coef_dev,
                  const double* coef_sign, double* y, hipStream_t st);
// Sum of squares of x into out[0] (float64, device), via partial sums in part (>= 1024 doubles).
void sumsq(int64_t n, const double* x, double* part, double* out, hipStream_t st);
// Copy a row-major rows x cols block with source/destination leading dimensions.
void copy2d(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd,
            hipStream_t st);
// dst (cols x rows) = transpose(src (rows x cols)), both row-major with leading dims.
void transpose2d(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd,
                 hipStream_t st);

// Dense FP64 linear algebra (la.hip).  Matrices are column-major with leading
// dimension ld unless noted.
// Householder QR of `batch` m x c matrices (m >= 1, c >= 1), in place: on exit
// the upper triangle holds R (min(m,c) x c), below it the reflectors; tau
// receives min(m,c) coefficients per matrix.  One workgroup per matrix.
void qr_householder(int32_t batch, int32_t m, int32_t c, double* A, int32_t lda, int64_t strideA,
                    double* tau, int64_t strideTau, hipStream_t st);
// Form the explicit thin Q (m x k, k = min(m,c)) from the reflectors into Q.
void qr_form_q(int32_t batch, int32_t m, int32_t c, const double* A, int32_t lda, int64_t strideA,
               const double* tau, int64_t strideTau, double* Q, int32_t ldq, int64_t strideQ,
               hipStream_t st);
// One-sided Jacobi SVD of `batch` m x c matrices (m >= c): on exit A holds U*Sigma
// (column-major), V (c x c) the right singular vectors, sig the singular values
// (unsorted; the caller sorts).  One workgroup per matrix.
void svd_jacobi(int32_t batch, int32_t m, int32_t c, double* A, int32_t lda, int64_t strideA,
                double* V, int32_t ldv, int64_t strideV, double* sig, int64_t strideSig,
                hipStream_t st);

// The small host-side helper type for device buffers carved from a workspace.
class Arena {
  public:
    Arena() = default;
    void reset(char* base, size_t bytes) { base_ = base; cap_ = bytes; off_ = 0; }
    void measure() { base_ = nullptr; cap_ = (size_t)-1; off_ = 0; }
    template <typename T> T* get(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        size_t o = off_;
        off_ += bytes;
        if (base_ != nullptr && off_ > cap_) throw Error(TTSG_ERR_WS, "workspace exhausted");
        return base_ ? reinterpret_cast<T*>(base_ + o) : reinterpret_cast<T*>(o + 256);
    }
    size_t used() const { return off_; }
    size_t mark() const { return off_; }
    void release(size_t m) { off_ = m; }

  private:
    char* base_ = nullptr;
    size_t cap_ = 0;
    size_t off_ = 0;
};

// Scoped workspace: uses the caller's buffer when given and large enough,
// otherwise allocates with hipMallocAsync on the stream and frees on exit.
class Workspace {
  public:
    Workspace(void* ws, size_t ws_bytes, size_t need, hipStream_t st) : st_(st) {
        if (ws != nullptr) {
            TTSG_CHECK(ws_bytes >= need, TTSG_ERR_WS, "workspace too small");
            ptr_ = ws;
        } else if (need > 0) {
            TTSG_HIP(hipMallocAsync(&ptr_, need, st));
            owned_ = true;
        }
        arena.reset(static_cast<char*>(ptr_), need);
    }
    ~Workspace() {
        if (owned_) (void)hipFreeAsync(ptr_, st_);
    }
    Arena arena;

  private:
    void* ptr_ = nullptr;
    bool owned_ = false;
    hipStream_t st_;
};

}  // namespace ttsg
