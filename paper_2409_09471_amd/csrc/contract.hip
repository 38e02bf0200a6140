// Generic strided tensor contraction on CDNA4 matrix cores.
//
//   C[b][m][n] = alpha * sum_k A[b][m][k] * B[b][k][n] + beta * C[b][m][n]
//
// Every index (m, n, k, b) of every operand is addressed through a two-level
// stride (Idx2), so the permuted core layouts met in the TT sweeps -- merged
// (rank, mode) indices, operator ranks split from vector ranks -- are read in
// place.  A 256-thread workgroup computes a 64 x 64 tile of C: the four
// wavefronts each own a 32 x 32 block made of 2 x 2 MFMA 16x16 tiles; A and B
// are staged through LDS in k-slabs (16 for FP64/FP32, 32 for BF16), the next
// slab's global loads in flight while the matrix cores work on the current one.
//
// Matrix-core forms used (gfx950):
//   FP64: v_mfma_f64_16x16x4_f64      (A, B, C in float64)
//   FP32: v_mfma_f32_16x16x4_f32      (A, B, C in float32)
//   BF16: v_mfma_f32_16x16x32_bf16    (A, B stored as float32 and rounded to
//         bfloat16, nearest-even, while they are staged into LDS; C in float32)
// Operand layout of the 16x16xK forms: lane l supplies row (l % 16) of A and
// column (l % 16) of B for the k-group (l / 16) (one k for the 4-deep FP64/FP32
// forms, eight consecutive k for the 32-deep BF16 form); the accumulator of
// lane l holds column (l % 16), rows given by Traits<T>::acc_row.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>

#include "ttsg_internal.h"

namespace ttsg {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int BM64 = 64;   // tile edge that the split-K decision is based on
constexpr uint64_t kXcds = 8;   // accelerator complex dies of an MI355X, each with its own L2

// float32 -> bfloat16 bits, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct Bf16 {};  // tag: float32 operands, bfloat16 matrix-core inputs

template <typename T> struct Traits;
// in_t: operand type in memory; lds_t: type staged in LDS; out_t: C.
// Row of accumulator register r held by lane group g (= lane / 16):
// the f64 form interleaves (row g + 4 r), the f32/bf16 forms keep four
// consecutive rows per group (row 4 g + r).
template <> struct Traits<double> {
    using acc4 = d4_t;
    using in_t = double;
    using lds_t = double;
    using out_t = double;
    static constexpr int BK = 16;
    static __device__ __forceinline__ int acc_row(int g, int r) { return g + 4 * r; }
    static __device__ __forceinline__ lds_t stage(in_t v) { return v; }
};
template <> struct Traits<float> {
    using acc4 = f4_t;
    using in_t = float;
    using lds_t = float;
    using out_t = float;
    static constexpr int BK = 16;
    static __device__ __forceinline__ int acc_row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ lds_t stage(in_t v) { return v; }
};
template <> struct Traits<Bf16> {
    using acc4 = f4_t;
    using in_t = float;
    using lds_t = uint16_t;
    using out_t = float;
    static constexpr int BK = 32;
    static __device__ __forceinline__ int acc_row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ lds_t stage(in_t v) { return bf16_rne(v); }
};

// Global -> register -> LDS staging of one operand's k-slab.  The thread to
// element map follows whichever index has unit stride (k or the row), so
// consecutive lanes read consecutive addresses; each thread's row offsets are
// computed once per tile, so a slab costs one (k-fast) or PER (row-fast) index
// evaluations.  fetch() issues the global loads of the next slab before the
// matrix-core work on the current one, commit() writes them to LDS after it.
template <typename T, int ROWS>
struct SlabLoader {
    using in_t = typename Traits<T>::in_t;
    using lds_t = typename Traits<T>::lds_t;
    static constexpr int BK = Traits<T>::BK;
    static constexpr int PER = ROWS * BK / 256;
    const in_t* G;
    Idx2 kix;
    int kend;
    bool k_fast;
    bool k1;              // one-level k index (idx1: n0 at its sentinel): offsets advance linearly
    int fixed;            // kk (k-fast) or the row within the tile (row-fast)
    int64_t ro[PER];      // row offsets (k-fast: per element; row-fast: ro[0]); -1 = outside
    int64_t kthr;         // row-fast, one-level: this thread's first k offset past k0
    in_t buf[PER];

    __device__ __forceinline__ void init(const in_t* G_, const Idx2& rowix, const Idx2& kix_, int row0, int nrows,
                                         int kend_, bool kf) {
        G = G_;
        kix = kix_;
        kend = kend_;
        k_fast = kf;
        k1 = kix_.n0 == 0x7fffffff;
        const int tid = threadIdx.x;
        kthr = (int64_t)(tid / ROWS) * kix_.s0;
        if (kf) {
            fixed = tid % BK;
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int gr = row0 + tid / BK + (256 / BK) * t;
                ro[t] = gr < nrows ? idx_off(rowix, gr) : -1;
            }
        } else {
            fixed = tid % ROWS;
            const int gr = row0 + fixed;
            ro[0] = gr < nrows ? idx_off(rowix, gr) : -1;
#pragma unroll
            for (int t = 1; t < PER; ++t) ro[t] = ro[0];
        }
    }
    __device__ __forceinline__ void fetch(int k0) {
        const int tid = threadIdx.x;
        if (k_fast) {
            const int gk = k0 + fixed;
            const bool kin = gk < kend;
            const int64_t ko = kin ? (k1 ? (int64_t)gk * kix.s0 : idx_off(kix, gk)) : 0;
#pragma unroll
            for (int t = 0; t < PER; ++t) buf[t] = (kin && ro[t] >= 0) ? G[ro[t] + ko] : in_t(0);
        } else if (k1) {
            // one-level k index: element t sits (256 / ROWS) t k-steps past the first
            const in_t* g = G + ro[0] + (int64_t)k0 * kix.s0 + kthr;
            const int64_t step = (int64_t)(256 / ROWS) * kix.s0;
            const int gk0 = k0 + tid / ROWS;
#pragma unroll
            for (int t = 0; t < PER; ++t)
                buf[t] = (gk0 + (256 / ROWS) * t < kend && ro[0] >= 0) ? g[t * step] : in_t(0);
        } else {
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int gk = k0 + tid / ROWS + (256 / ROWS) * t;
                buf[t] = (gk < kend && ro[t] >= 0) ? G[ro[t] + idx_off(kix, gk)] : in_t(0);
            }
        }
    }
    __device__ __forceinline__ void commit(lds_t (*S)[ROWS + 1]) const {
        const int tid = threadIdx.x;
        if (k_fast) {
#pragma unroll
            for (int t = 0; t < PER; ++t) S[fixed][tid / BK + (256 / BK) * t] = Traits<T>::stage(buf[t]);
        } else {
#pragma unroll
            for (int t = 0; t < PER; ++t) S[tid / ROWS + (256 / ROWS) * t][fixed] = Traits<T>::stage(buf[t]);
        }
    }
};

// A operand of a Khatri-Rao step formed while it is staged: row m = (j, be),
// column k = (a, i), value sum_al P[j][al][a] SA[j][al][be][i], the RL terms
// added in order.  Each thread owns KG consecutive k of its rows (two for
// 32-row tiles, four for taller ones), so (for n a multiple of KG) the S A
// values come in 16-byte loads of two and the P value, the same for the whole
// group, in one: a half to a quarter of the load instructions of one k per
// thread, which is what the loader's time went on.  fetch() only issues the loads (they complete
// while the matrix cores work on the current slab); commit() forms the sums as
// it writes the LDS slab.  The s R r n intermediate is never stored.
template <typename T>
struct alignas(2 * sizeof(T)) Pair2 {
    T x, y;
};

template <typename T, int ROWS, int RL>
struct KrLoader {
    using in_t = typename Traits<T>::in_t;
    using lds_t = typename Traits<T>::lds_t;
    static constexpr int BK = Traits<T>::BK;
    static constexpr int KG = ROWS >= 64 ? 4 : 2;  // consecutive k per thread
    static constexpr int NG = BK / KG;             // k groups per slab
    static constexpr int RP = 256 / NG;            // rows per pass
    static constexpr int PER = ROWS / RP;          // passes (rows per thread)
    static_assert(ROWS % RP == 0, "tile rows");
    const in_t* P;
    const in_t* SA;
    int rl, n, Rr, kend;
    bool grp;                   // n % KG == 0: a thread's k share a, and the S A run is aligned loads
    int64_t pb[PER], sb[PER];   // per row: P offset of (j, 0, 0), SA offset of (j, 0, be, 0); pb < 0: outside
    in_t pv[PER][KG][RL], sv[PER][KG][RL];

    __device__ __forceinline__ void init(const ContractDesc& d, int row0, int kend_) {
        P = static_cast<const in_t*>(d.kr_P);
        SA = static_cast<const in_t*>(d.kr_SA);
        rl = d.kr_rl;
        n = d.kr_n;
        Rr = d.kr_Rr;
        kend = kend_;
        grp = n % KG == 0;
        const int tid = threadIdx.x;
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int gr = row0 + tid / NG + RP * t;
            if (gr < d.M) {
                const int64_t j = gr / Rr;
                const int be = gr - (int)(j * Rr);
                pb[t] = j * RL * rl;
                sb[t] = j * RL * n * Rr + (int64_t)be * n;
            } else {
                pb[t] = -1;
                sb[t] = 0;
            }
        }
    }
    // thread tid owns k = k0 + KG (tid % NG) + {0 .. KG-1} of rows tid / NG + RP t
    __device__ __forceinline__ void fetch(int k0) {
        const int gk = k0 + KG * (int)(threadIdx.x % NG);
        const int64_t nR = (int64_t)n * Rr;
        if (grp) {
            // gk and n multiples of KG: i + KG - 1 < n, one a for the group, the
            // S A run starts at an offset that is a multiple of KG (kend is too)
            const bool kin = gk < kend;
            const int a = kin ? gk / n : 0;
            const int i = kin ? gk - a * n : 0;
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const bool on = kin && pb[t] >= 0;
#pragma unroll
                for (int al = 0; al < RL; ++al) {
                    const in_t p = on ? P[pb[t] + a + (int64_t)al * rl] : in_t(0);
#pragma unroll
                    for (int h = 0; h < KG / 2; ++h) {
                        Pair2<in_t> q{in_t(0), in_t(0)};
                        if (on) q = *reinterpret_cast<const Pair2<in_t>*>(SA + sb[t] + i + 2 * h + al * nR);
                        pv[t][2 * h][al] = p;
                        pv[t][2 * h + 1][al] = p;
                        sv[t][2 * h][al] = q.x;
                        sv[t][2 * h + 1][al] = q.y;
                    }
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < KG; ++e) {
                const int g = gk + e;
                const bool kin = g < kend;
                const int a = kin ? g / n : 0;
                const int i = kin ? g - a * n : 0;
#pragma unroll
                for (int t = 0; t < PER; ++t) {
                    const bool on = kin && pb[t] >= 0;
#pragma unroll
                    for (int al = 0; al < RL; ++al) {
                        pv[t][e][al] = on ? P[pb[t] + a + (int64_t)al * rl] : in_t(0);
                        sv[t][e][al] = on ? SA[sb[t] + i + al * nR] : in_t(0);
                    }
                }
            }
        }
    }
    __device__ __forceinline__ void commit(lds_t (*S)[ROWS + 1]) const {
        const int tid = threadIdx.x;
        const int kg = tid % NG;
#pragma unroll
        for (int t = 0; t < PER; ++t)
#pragma unroll
            for (int e = 0; e < KG; ++e) {
                in_t acc = in_t(0);
#pragma unroll
                for (int al = 0; al < RL; ++al) acc += pv[t][e][al] * sv[t][e][al];
                S[KG * kg + e][tid / NG + RP * t] = Traits<T>::stage(acc);
            }
    }
};

__device__ __forceinline__ d4_t mfma(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// With splits > 1 every workgroup reduces one K-chunk of kchunk values and
// writes its unscaled partial tile to part[split][batch][M][N]; a second
// kernel sums the partials in a fixed order (deterministic) into C.
template <typename T, int WM, int WN, int KRL>
__global__ __launch_bounds__(256) void contract_kernel(ContractDesc d, const typename Traits<T>::in_t* __restrict__ A,
                                                       const typename Traits<T>::in_t* __restrict__ B,
                                                       typename Traits<T>::out_t* __restrict__ C,
                                                       int batch0, int splits, int kchunk,
                                                       typename Traits<T>::out_t* __restrict__ part,
                                                       DevSlot* slot) {
    using acc4 = typename Traits<T>::acc4;
    using in_t = typename Traits<T>::in_t;
    using lds_t = typename Traits<T>::lds_t;
    using out_t = typename Traits<T>::out_t;
    constexpr int BK = Traits<T>::BK;
    constexpr int TM = 32 * WM, TN = 32 * WN;   // tile: 2 x 2 wavefronts of WM x WN MFMA blocks
    __shared__ lds_t As[BK][TM + 1];
    __shared__ lds_t Bs[BK][TN + 1];

    slot_begin(slot);
    // XCD-aware tile order: workgroups are handed to the 8 XCDs round-robin in
    // launch order, so consecutive tiles (which share operand rows and
    // columns) would land on 8 different L2s.  Tile t of the launch is instead
    // given to the workgroup that makes each XCD process a contiguous run of
    // tiles (x fastest, then y, then batch/split).
    int tx, ty, tz;
    {
        const uint64_t gx = gridDim.x, gy = gridDim.y;
        const uint64_t total = gx * gy * gridDim.z;
        const uint64_t hw = blockIdx.x + gx * (blockIdx.y + gy * (uint64_t)blockIdx.z);
        const uint64_t q = total / kXcds, r = total % kXcds;
        const uint64_t xcd = hw % kXcds, pos = hw / kXcds;
        const uint64_t t = xcd * q + (xcd < r ? xcd : r) + pos;
        // The divisions run on the vector ALU, so the compiler cannot tell that
        // the tile is the same for every lane; saying so keeps the k-loop
        // uniform (a scalar trip count, no exec-masked loop around the MFMAs).
        tx = __builtin_amdgcn_readfirstlane((int)(t % gx));
        ty = __builtin_amdgcn_readfirstlane((int)((t / gx) % gy));
        tz = __builtin_amdgcn_readfirstlane((int)(t / (gx * gy)));
    }
    const int zz = batch0 + tz;
    const int bidx = __builtin_amdgcn_readfirstlane(zz / splits);
    const int split = zz - bidx * splits;
    const int kbeg = split * kchunk;
    const int kend = min(d.K, kbeg + kchunk);
    const int m0 = ty * TM;
    const int n0 = tx * TN;
    const in_t* Ab = KRL > 0 ? A : A + idx_off(d.ab, bidx);
    const in_t* Bb = B + idx_off(d.bb, bidx);
    out_t* Cb = C + idx_off(d.cb, bidx);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 16 * WM;
    const int wn = (wave & 1) * 16 * WN;
    const int lr = lane & 15;
    const int lg = lane >> 4;

    acc4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = acc4{0, 0, 0, 0};

    typename std::conditional<(KRL > 0), KrLoader<T, TM, (KRL > 0 ? KRL : 1)>, SlabLoader<T, TM>>::type la;
    SlabLoader<T, TN> lb;
    if constexpr (KRL > 0)
        la.init(d, m0, kend);
    else
        la.init(Ab, d.am, d.ak, m0, d.M, kend, d.ak.s0 == 1);
    lb.init(Bb, d.bn, d.bk, n0, d.N, kend, d.bk.s0 == 1);
    if (kbeg < kend) {
        la.fetch(kbeg);
        lb.fetch(kbeg);
    }

    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        la.commit(As);
        lb.commit(Bs);
        __syncthreads();
        if (k0 + BK < kend) {
            la.fetch(k0 + BK);
            lb.fetch(k0 + BK);
        }
        if constexpr (sizeof(lds_t) == 2) {
            // gfx950's 16x16x32 form: one instruction per 32-deep slab, lane l
            // supplying k = 8 (l / 16) + 0..7 of row / column l % 16
            static_assert(BK == 32, "the bf16 slab is one 16x16x32 step");
            s8_t a[WM], b[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int t = 0; t < 8; ++t) a[i][t] = (short)As[8 * lg + t][wm + 16 * i + lr];
#pragma unroll
            for (int j = 0; j < WN; ++j)
#pragma unroll
                for (int t = 0; t < 8; ++t) b[j][t] = (short)Bs[8 * lg + t][wn + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a[i]),
                                                                         __builtin_bit_cast(bf8_t, b[j]), acc[i][j],
                                                                         0, 0, 0);
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                lds_t a[WM], b[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) a[i] = As[kk + lg][wm + 16 * i + lr];
#pragma unroll
                for (int j = 0; j < WN; ++j) b[j] = Bs[kk + lg][wn + 16 * j + lr];
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
            }
        }
        __syncthreads();
    }

    const out_t alpha = (out_t)d.alpha;
    const out_t beta = (out_t)d.beta;
    // float32 arithmetic may write a float64 output (its strides count doubles)
    const bool wide = sizeof(out_t) == 4 && d.c_f64 != 0;
    double* Cw = reinterpret_cast<double*>(C) + idx_off(d.cb, bidx);
    const out_t* Xb = d.c_add != nullptr ? static_cast<const out_t*>(d.c_add) + idx_off(d.xb, bidx) : nullptr;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = m0 + wm + 16 * i + Traits<T>::acc_row(lg, r);
                int col = n0 + wn + 16 * j + lr;
                if (row < d.M && col < d.N) {
                    if (part != nullptr) {
                        part[(((int64_t)split * d.batch + bidx) * d.M + row) * d.N + col] = (out_t)acc[i][j][r];
                    } else if (wide) {
                        int64_t off = idx_off(d.cm, row) + idx_off(d.cn, col);
                        double v = d.alpha * (double)acc[i][j][r];
                        if (d.beta != 0.0) v += d.beta * Cw[off];
                        Cw[off] = v;
                    } else {
                        int64_t off = idx_off(d.cm, row) + idx_off(d.cn, col);
                        out_t v = alpha * (out_t)acc[i][j][r];
                        if (beta != out_t(0)) v += beta * Cb[off];
                        if (Xb != nullptr) v += Xb[idx_off(d.xm, row) + idx_off(d.xn, col)];
                        Cb[off] = v;
                    }
                }
            }
    slot_end(slot);
}

// Sum of the split-K partials.  Each output element belongs to a group of G
// lanes: lane g adds splits g, g + G, ... in order, then the group combines
// its lanes with a fixed xor tree -- the same order on every run.
template <typename O, int G>
__global__ __launch_bounds__(256) void reduce_splits(ContractDesc d, int splits, const O* __restrict__ part,
                                                     O* __restrict__ C) {
    const int64_t per = (int64_t)d.M * d.N;
    const int64_t total = per * d.batch;
    const O alpha = (O)d.alpha, beta = (O)d.beta;
    const int g = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / G);
    for (int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G; e < total; e += stride) {
        O acc = 0;
        for (int s = g; s < splits; s += G) acc += part[(int64_t)s * total + e];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
        if (g == 0) {
            // element -> (b, m, n): 32-bit divisions when the indices fit
            // (64-bit ones expand into long vector-ALU sequences)
            int b, m, n;
            if (total < ((int64_t)1 << 31)) {
                const unsigned e32 = (unsigned)e, pr = (unsigned)per;
                const unsigned bb = d.batch == 1 ? 0u : e32 / pr;
                const unsigned mn = e32 - bb * pr;
                const unsigned mm = mn / (unsigned)d.N;
                b = (int)bb;
                m = (int)mm;
                n = (int)(mn - mm * (unsigned)d.N);
            } else {
                b = (int)(e / per);
                const int64_t mn = e - (int64_t)b * per;
                m = (int)(mn / d.N);
                n = (int)(mn - (int64_t)m * d.N);
            }
            const int64_t off = idx_off(d.cb, b) + idx_off(d.cm, m) + idx_off(d.cn, n);
            if (sizeof(O) == 4 && d.c_f64 != 0) {
                double* Cw = reinterpret_cast<double*>(C);
                double v = d.alpha * (double)acc;
                if (d.beta != 0.0) v += d.beta * Cw[off];
                Cw[off] = v;
            } else {
                O v = alpha * acc;
                if (beta != O(0)) v += beta * C[off];
                if (d.c_add != nullptr)
                    v += static_cast<const O*>(d.c_add)[idx_off(d.xb, b) + idx_off(d.xm, m) + idx_off(d.xn, n)];
                C[off] = v;
            }
        }
    }
}

template <typename O>
void launch_reduce(const ContractDesc& d, int splits, const O* part, O* C, hipStream_t st) {
    const int64_t total = (int64_t)d.batch * d.M * d.N;
    const int G = splits <= 4 ? 4 : (splits <= 8 ? 8 : (splits <= 16 ? 16 : 32));
    const int64_t per_block = 256 / G;
    const int rb = (int)std::max<int64_t>(1, std::min<int64_t>((total + per_block - 1) / per_block, 16384));
    switch (G) {
        case 4: hipLaunchKernelGGL((reduce_splits<O, 4>), dim3(rb), dim3(256), 0, st, d, splits, part, C); break;
        case 8: hipLaunchKernelGGL((reduce_splits<O, 8>), dim3(rb), dim3(256), 0, st, d, splits, part, C); break;
        case 16: hipLaunchKernelGGL((reduce_splits<O, 16>), dim3(rb), dim3(256), 0, st, d, splits, part, C); break;
        default: hipLaunchKernelGGL((reduce_splits<O, 32>), dim3(rb), dim3(256), 0, st, d, splits, part, C); break;
    }
}

// ---------------------------------------------------------------------------
// Tile variants and the autotuner.  Variant v runs WM x WN MFMA blocks per
// wavefront: 0 = 64 x 64 tiles, 1 = 32 x 64, 2 = 64 x 32, 3 = 32 x 32,
// 4 = 128 x 64, 5 = 64 x 128, 6 = 128 x 128 (M x N).  The larger tiles halve
// or quarter the operand loads per flop (a 128 x 128 FP64 tile reuses each
// staged element 128 times), at the price of fewer workgroups.  The tuner
// times every variant the first time a shape class is met while tuning is on
// and keeps the fastest; the table can be saved and loaded.
// ---------------------------------------------------------------------------
constexpr int kVariants = 7;

template <typename T, int WM, int WN, int KRL>
void run_tiles(const ContractDesc& d, const typename Traits<T>::in_t* A, const typename Traits<T>::in_t* B,
               typename Traits<T>::out_t* C, int splits, int kchunk, hipStream_t st, Arena* ar, DevSlot* slot) {
    using out_t = typename Traits<T>::out_t;
    const int gx = (d.N + 32 * WN - 1) / (32 * WN);
    const int gy = (d.M + 32 * WM - 1) / (32 * WM);
    if (splits > 1) {
        const size_t mark = ar->mark();
        out_t* part = ar->get<out_t>((size_t)splits * d.batch * d.M * d.N);
        hipLaunchKernelGGL((contract_kernel<T, WM, WN, KRL>), dim3(gx, gy, d.batch * splits), dim3(256), 0, st, d,
                           A, B, C, 0, splits, kchunk, part, slot);
        launch_reduce<out_t>(d, splits, part, C, st);
        ar->release(mark);
    } else {
        for (int b0 = 0; b0 < d.batch; b0 += 65535) {
            const int nb = d.batch - b0 < 65535 ? d.batch - b0 : 65535;
            hipLaunchKernelGGL((contract_kernel<T, WM, WN, KRL>), dim3(gx, gy, nb), dim3(256), 0, st, d, A, B, C, b0,
                               1, d.K, static_cast<out_t*>(nullptr), slot);
        }
    }
    TTSG_HIP(hipGetLastError());
}

template <typename T, int KRL>
void run_shape(int v, const ContractDesc& d, const typename Traits<T>::in_t* A, const typename Traits<T>::in_t* B,
               typename Traits<T>::out_t* C, int splits, int kchunk, hipStream_t st, Arena* ar, DevSlot* slot) {
    switch (v) {
        case 1: run_tiles<T, 1, 2, KRL>(d, A, B, C, splits, kchunk, st, ar, slot); break;
        case 2: run_tiles<T, 2, 1, KRL>(d, A, B, C, splits, kchunk, st, ar, slot); break;
        case 3: run_tiles<T, 1, 1, KRL>(d, A, B, C, splits, kchunk, st, ar, slot); break;
        case 4: run_tiles<T, 4, 2, KRL>(d, A, B, C, splits, kchunk, st, ar, slot); break;
        case 5: run_tiles<T, 2, 4, KRL>(d, A, B, C, splits, kchunk, st, ar, slot); break;
        case 6:
            // 128 x 128 is FP64 only (the float32 accumulators of the 4 x 4 block spill)
            if constexpr (sizeof(typename Traits<T>::lds_t) == 8) {
                run_tiles<T, 4, 4, KRL>(d, A, B, C, splits, kchunk, st, ar, slot);
                break;
            }
            [[fallthrough]];
        default: run_tiles<T, 2, 2, KRL>(d, A, B, C, splits, kchunk, st, ar, slot); break;
    }
}

// Variants a precision has (the 128 x 128 tile is FP64 only).
template <typename T>
constexpr int variants_of() {
    return sizeof(typename Traits<T>::lds_t) == 8 ? 7 : 6;
}

template <typename T>
void run_variant(int v, const ContractDesc& d, const typename Traits<T>::in_t* A, const typename Traits<T>::in_t* B,
                 typename Traits<T>::out_t* C, int splits, int kchunk, hipStream_t st, Arena* ar, DevSlot* slot) {
    if (d.kr_P == nullptr) {
        run_shape<T, 0>(v, d, A, B, C, splits, kchunk, st, ar, slot);
        return;
    }
    if constexpr (sizeof(typename Traits<T>::lds_t) == 2) {
        TTSG_CHECK(false, TTSG_ERR_ARG, "contraction: the fused Khatri-Rao operand is float64/float32 only");
    } else {
        switch (d.kr_Rl) {
            case 1: run_shape<T, 1>(v, d, A, B, C, splits, kchunk, st, ar, slot); break;
            case 2: run_shape<T, 2>(v, d, A, B, C, splits, kchunk, st, ar, slot); break;
            default:
                TTSG_CHECK(d.kr_Rl == 3, TTSG_ERR_ARG, "contraction: fused Khatri-Rao operand rank must be 1..3");
                run_shape<T, 3>(v, d, A, B, C, splits, kchunk, st, ar, slot);
                break;
        }
    }
}

// Without a tuned entry: the smallest tile that covers a dimension of <= 32.
int default_variant(const ContractDesc& d) {
    const bool sm = d.M <= 32, sn = d.N <= 32;
    return sm && sn ? 3 : (sm ? 1 : (sn ? 2 : 0));
}

struct TuneKey {
    int cls, lm, ln, lk, lb, split, afast, bfast;
    bool operator<(const TuneKey& o) const {
        const int a[8] = {cls, lm, ln, lk, lb, split, afast, bfast};
        const int b[8] = {o.cls, o.lm, o.ln, o.lk, o.lb, o.split, o.afast, o.bfast};
        for (int i = 0; i < 8; ++i)
            if (a[i] != b[i]) return a[i] < b[i];
        return false;
    }
};

int ceil_log2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

TuneKey tune_key(int cls, const ContractDesc& d, int splits) {
    return TuneKey{cls, ceil_log2(d.M), ceil_log2(d.N), ceil_log2(d.K), ceil_log2(d.batch), splits > 1 ? 1 : 0,
                   d.ak.s0 == 1 ? 1 : 0, d.bk.s0 == 1 ? 1 : 0};
}

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_on = false;

int tuned_variant(const TuneKey& k) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(k);
    return it == g_tune.end() ? -1 : it->second;
}
bool autotune_on() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune_on;
}

// Time every variant (three launches each, HIP events on the stream) with the
// output redirected to a scratch buffer, record and return the fastest.
template <typename T>
int tune(const TuneKey& key, const ContractDesc& d, const void* A, const void* B, int splits, int kchunk,
         hipStream_t st, Arena* ar) {
    using in_t = typename Traits<T>::in_t;
    using out_t = typename Traits<T>::out_t;
    ContractDesc dc = d;
    dc.beta = 0.0;
    dc.c_f64 = 0;   // timed into a scratch of the arithmetic's type
    dc.c_add = nullptr;
    dc.cb = idx1((int64_t)d.M * d.N);
    dc.cm = idx1(d.N);
    dc.cn = idx1(1);
    out_t* scratch = nullptr;
    TTSG_HIP(hipMallocAsync(reinterpret_cast<void**>(&scratch), (size_t)d.batch * d.M * d.N * sizeof(out_t), st));
    constexpr int nvar = variants_of<T>();
    hipEvent_t ev[nvar + 1];
    for (auto& e : ev) TTSG_HIP(hipEventCreate(&e));
    TTSG_HIP(hipEventRecord(ev[0], st));
    for (int v = 0; v < nvar; ++v) {
        for (int rep = 0; rep < 3; ++rep)
            run_variant<T>(v, dc, static_cast<const in_t*>(A), static_cast<const in_t*>(B), scratch, splits, kchunk,
                           st, ar, nullptr);
        TTSG_HIP(hipEventRecord(ev[v + 1], st));
    }
    TTSG_HIP(hipEventSynchronize(ev[nvar]));
    int best = 0;
    float best_ms = 0.0f;
    for (int v = 0; v < nvar; ++v) {
        float ms = 0.0f;
        TTSG_HIP(hipEventElapsedTime(&ms, ev[v], ev[v + 1]));
        if (v == 0 || ms < best_ms) {
            best = v;
            best_ms = ms;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    TTSG_HIP(hipFreeAsync(scratch, st));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return best;
}

template <typename T>
void launch(const ContractDesc& d, const void* A, const void* B, void* C, hipStream_t st, Arena* ar) {
    if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
    TTSG_CHECK(d.c_f64 == 0 || sizeof(typename Traits<T>::out_t) == 4, TTSG_ERR_ARG,
               "contraction: a float64 output needs float32 arithmetic");
    TTSG_CHECK(d.c_add == nullptr || d.c_f64 == 0, TTSG_ERR_ARG, "contraction: an addend needs C in the arithmetic's type");
    using in_t = typename Traits<T>::in_t;
    if (bounds_checking()) {
        using out_t = typename Traits<T>::out_t;
        const int64_t ea = idx_max(d.ab, d.batch) + idx_max(d.am, d.M) + idx_max(d.ak, d.K) + 1;
        const int64_t eb = idx_max(d.bb, d.batch) + idx_max(d.bk, d.K) + idx_max(d.bn, d.N) + 1;
        const int64_t ec = idx_max(d.cb, d.batch) + idx_max(d.cm, d.M) + idx_max(d.cn, d.N) + 1;
        if (d.kr_P != nullptr) {
            const int64_t nj = (d.M + d.kr_Rr - 1) / d.kr_Rr;
            TTSG_CHECK((int64_t)d.K == (int64_t)d.kr_rl * d.kr_n && d.batch == 1, TTSG_ERR_ARG,
                       "contract: Khatri-Rao operand shape");
            check_range(d.kr_P, nj * d.kr_Rl * d.kr_rl * sizeof(in_t), "contract KR P");
            check_range(d.kr_SA, nj * d.kr_Rl * d.kr_n * d.kr_Rr * sizeof(in_t), "contract KR SA");
        } else {
            check_range(A, ea * sizeof(in_t), "contract A");
        }
        check_range(B, eb * sizeof(in_t), "contract B");
        check_range(C, ec * (d.c_f64 ? sizeof(double) : sizeof(out_t)), "contract C");
        if (d.c_add != nullptr) {
            const int64_t ex = idx_max(d.xb, d.batch) + idx_max(d.xm, d.M) + idx_max(d.xn, d.N) + 1;
            check_range(d.c_add, ex * sizeof(out_t), "contract addend");
        }
    }
    const int cls = sizeof(typename Traits<T>::lds_t) == 8
                        ? TTSG_ST_CONTRACT_F64
                        : (sizeof(typename Traits<T>::lds_t) == 4 ? TTSG_ST_CONTRACT_F32 : TTSG_ST_CONTRACT_BF16);
    double flops = 0.0, bytes = 0.0;
    if (stats_on()) {
        using out_t = typename Traits<T>::out_t;
        const double nb = (double)d.batch;
        flops = 2.0 * d.M * (double)d.N * d.K * nb;
        // the fused Khatri-Rao operand reads P and S A, not the M x K matrix
        const double ua = d.kr_P != nullptr
                              ? (double)(d.M / std::max(d.kr_Rr, 1)) * d.kr_Rl * ((double)d.kr_rl + (double)d.kr_n * d.kr_Rr)
                              : (double)d.M * d.K * (d.ab.s0 == 0 ? 1.0 : nb);
        const double ub = (double)d.K * d.N * (d.bb.s0 == 0 ? 1.0 : nb);
        const double uc = (double)d.M * d.N * nb * (d.beta != 0.0 ? 2.0 : 1.0);
        bytes = (ua + ub) * sizeof(in_t) + uc * (d.c_f64 ? sizeof(double) : sizeof(out_t));
    }
    StatScope scope(cls, flops, bytes, st);
    using out_t = typename Traits<T>::out_t;
    // split-K when the output tiles alone cannot fill the chip (at least four
    // k-slabs per split, at most 64 splits, about two workgroups per CU; four
    // per CU for reductions of 2048 or more, whose long k-loops otherwise run
    // with one workgroup per CU and expose the global-load latency of every
    // slab).  The decision uses 64 x 64 tiles whatever tile variant runs, so
    // every variant sums in the same order and gives bit-identical results.
    constexpr int BK = Traits<T>::BK;
    const int64_t gx64 = (d.N + BM64 - 1) / BM64, gy64 = (d.M + BM64 - 1) / BM64;
    TTSG_CHECK((d.M + 31) / 32 < 65536, TTSG_ERR_ARG, "contraction: M too large");
    const int64_t wgs = gx64 * gy64 * d.batch;
    const bool long_k = d.K >= 2048;
    const int64_t target = long_k ? 1024 : 512;
    int splits = 1, kchunk = d.K;
    if (ar != nullptr && wgs < target && d.K >= 8 * BK) {
        int want = (int)std::min<int64_t>((target + wgs - 1) / wgs, d.K / (4 * BK));
        want = std::min(want, 64);
        want = std::min<int64_t>(want, 65535 / std::max(d.batch, 1));
        // two to four splits of an already wide grid cost more in the extra
        // reduction than they save, unless the reduction is long
        if (want >= 5 || (long_k && want >= 2)) {
            kchunk = ((d.K + want - 1) / want + BK - 1) / BK * BK;
            splits = (d.K + kchunk - 1) / kchunk;
        }
    }
    scope.shape(d.M, d.N, d.K, d.batch, splits);
    const TuneKey key = tune_key(d.kr_P != nullptr ? cls + 16 : cls, d, splits);
    int variant = tuned_variant(key);
    if (variant < 0 && autotune_on()) variant = tune<T>(key, d, A, B, splits, kchunk, st, ar);
    if (variant < 0) variant = d.kr_P != nullptr ? 1 : default_variant(d);
    run_variant<T>(variant, d, static_cast<const in_t*>(A), static_cast<const in_t*>(B), static_cast<out_t*>(C),
                   splits, kchunk, st, ar, scope.slot());
}

}  // namespace

bool bounds_checking() {
    static const bool on = [] {
        const char* e = std::getenv("TTSG_CHECK_BOUNDS");
        return e != nullptr && e[0] == '1';
    }();
    return on;
}

void check_range(const void* p, size_t bytes, const char* what) {
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
    TTSG_CHECK(e == hipSuccess, TTSG_ERR_ARG, std::string(what) + ": pointer is not in a device allocation");
    const char* b0 = static_cast<const char*>(base);
    const char* q = static_cast<const char*>(p);
    TTSG_CHECK(q >= b0 && q + bytes <= b0 + size, TTSG_ERR_ARG,
               std::string(what) + ": access range exceeds its allocation");
}

void contract(Prec p, const ContractDesc& d, const void* A, const void* B, void* C, hipStream_t st, Arena* ar) {
    if (d.K <= 0) {
        // empty reduction: C = beta * C handled by callers never passing K = 0
        TTSG_CHECK(false, TTSG_ERR_ARG, "contraction with empty reduction");
    }
    switch (p) {
        case Prec::F64: launch<double>(d, A, B, C, st, ar); break;
        case Prec::F32: launch<float>(d, A, B, C, st, ar); break;
        case Prec::BF16: launch<Bf16>(d, A, B, C, st, ar); break;
    }
}

bool autotune_is_on() { return autotune_on(); }

int autotune_set(int on) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int old = g_tune_on ? 1 : 0;
    g_tune_on = on != 0;
    return old;
}

int autotune_save(const char* path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE* f = std::fopen(path, "w");
    if (f == nullptr) return -1;
    std::fprintf(f, "# ttsg contraction tile table: class log2M log2N log2K log2batch split afast bfast variant\n");
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d\n", k.cls, k.lm, k.ln, k.lk, k.lb, k.split, k.afast, k.bfast,
                     kv.second);
    }
    std::fclose(f);
    return (int)g_tune.size();
}

int autotune_load(const char* path) {
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return -1;
    std::map<TuneKey, int> t;
    char line[256];
    while (std::fgets(line, sizeof line, f) != nullptr) {
        if (line[0] == '#') continue;
        TuneKey k{};
        int v = 0;
        if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d", &k.cls, &k.lm, &k.ln, &k.lk, &k.lb, &k.split, &k.afast,
                        &k.bfast, &v) == 9 &&
            v >= 0 && v < kVariants)
            t[k] = v;
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : t) g_tune[kv.first] = kv.second;
    return (int)t.size();
}

int autotune_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int n = (int)g_tune.size();
    g_tune.clear();
    return n;
}

}  // namespace ttsg
