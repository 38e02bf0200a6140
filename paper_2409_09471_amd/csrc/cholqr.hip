// Cholesky QR in two passes (CholQR2) for the tall-skinny unfoldings of the
// TT-SVD: X = Q R through G = X^T X = R^T R and Q = X R^-1, repeated once on
// Q to restore orthogonality to working precision.  The Gram products and the
// multiplications by R^-1 are matrix-core contractions over the whole chip;
// only the c x c Cholesky factorization and the triangular inverse are
// sequential, inside one workgroup's LDS.
//
// CholQR2 is accurate while the column-equilibrated X is well conditioned.
// Each factorization raises a device flag when a pivot of the first pass falls
// below 1e-10 of its column's squared norm, when a pivot is not finite, or when
// the second-pass factor differs from the identity by more than 0.1 (the first
// Q was not nearly orthonormal); callers read the flag at their next
// synchronization and redo the factorization with Householder QR.
#include <cmath>
#include <mutex>

#include "tt_ops.h"

namespace ttsg {
namespace {

constexpr int CQ_T = 1024;
constexpr int CQ_RG = CQ_T / 64;   // row groups: thread (rg, l) owns column l, rows = rg mod CQ_RG
constexpr int CQ_MAX = 64;

// Cholesky of the c x c symmetric G (column-major) into upper R (G = R^T R),
// and R^-1; both written column-major with leading dimension c.
// Second pass (R1 != nullptr): also forms the CholQR2 factor R2 R1 into Rp
// (column-major) and, when RT != nullptr, its transpose.
//
// One elimination sweep gives both factors.  With G = L D L^T (L unit lower,
// D the pivots), step j takes the multipliers m_i = S[j][i] / S[j][j] of the
// current Schur complement S (upper triangle of A) and
//   - updates S[i][l] -= m_i S[j][l] for j < i <= l,
//   - applies the same row operation to W = L^-1 (strict lower triangle of A,
//     unit diagonal implied): W[i][l] -= m_i W[j][l] for i > j, l <= j.
// Row j is final once step j starts and no step writes it afterwards, so one
// barrier per step suffices.  Then R[j][l] = S_j[j][l] / sqrt(d_j) (row j of
// the upper triangle) and R^-1 = W^T D^-1/2, i.e. R^-1[a][b] = W[b][a] / sqrt(d_b).
__global__ __launch_bounds__(CQ_T) void k_chol_inv(int c, const double* __restrict__ G, double* __restrict__ R,
                                                    double* __restrict__ Ri, int* __restrict__ flag,
                                                    int second_pass, const double* __restrict__ R1,
                                                    double* __restrict__ Rp, double* __restrict__ RT,
                                                    DevSlot* slot) {
    __shared__ double A[CQ_MAX][CQ_MAX + 1];
    __shared__ double B[CQ_MAX][CQ_MAX + 1];   // second pass: R1, row-major
    __shared__ double d0[CQ_MAX], pd[CQ_MAX], rd[CQ_MAX];
    __shared__ int s_bad;
    slot_begin(slot);
    const int tid = threadIdx.x;
    for (int e = tid; e < c * c; e += CQ_T) {
        const int l = e / c, i = e - l * c;
        A[i][l] = i <= l ? G[i + (int64_t)l * c] : 0.0;
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int j = tid; j < c; j += CQ_T) d0[j] = A[j][j];
    __syncthreads();
    // thread (rg, l) owns column l and every CQ_RG-th row below the pivot:
    // Schur rows j < i <= l for l > j, rows of W below j for l <= j
    const int l = tid & 63, rg = tid >> 6;
    for (int j = 0; j < c; ++j) {
        double p = A[j][j];
        const double dj = d0[j];
        const bool ok = p > 1e-10 * dj && p <= 4.0 * dj && dj < INFINITY;
        if (!ok) p = (dj > 0.0 && dj < INFINITY) ? dj : 1.0;   // keep going; the flag discards the result
        if (tid == 0) {
            pd[j] = p;   // square roots after the sweep, off the barrier chain
            if (!ok) s_bad = 1;
        }
        if (l < c) {
            const double ip = 1.0 / p;
            const double x = l == j ? 1.0 : A[j][l];
            const int hi = l > j ? l : c - 1;
            for (int i = j + 1 + rg; i <= hi; i += CQ_RG) A[i][l] -= (A[j][i] * ip) * x;
        }
        __syncthreads();
    }
    for (int j = tid; j < c; j += CQ_T) rd[j] = sqrt(pd[j]);
    __syncthreads();
    for (int e = tid; e < c * c; e += CQ_T) {
        const int cl = e / c, j = e - cl * c;
        const double v = cl > j ? A[j][cl] / rd[j] : (cl == j ? rd[j] : 0.0);
        R[j + (int64_t)cl * c] = v;
        if (second_pass && fabs(v - (cl == j ? 1.0 : 0.0)) > 0.1) s_bad = 1;
        Ri[j + (int64_t)cl * c] = j <= cl ? (j == cl ? 1.0 : A[cl][j]) / rd[cl] : 0.0;
    }
    if (R1 != nullptr) {
        // R1 (upper, diagonal included) staged row-major: B[t][l] = R1[t][l]
        __syncthreads();
        for (int e = tid; e < c * c; e += CQ_T) {
            const int cl = e / c, t = e - cl * c;
            B[t][cl] = t <= cl ? R1[e] : 0.0;
        }
        __syncthreads();
        // (R2 R1)[i][l] = sum_{t=i..l} R2[i][t] R1[t][l], R2[i][t] = A[i][t] / rd[i]
        // (t > i); lanes run along l, so R1 is read along its rows and R2's
        // entries are shared by the lanes of one row i
        for (int e = tid; e < c * c; e += CQ_T) {
            const int i = e / c, cl = e - i * c;
            double v = 0.0;
            if (i <= cl) {
                // four independent partial sums: each group of eight LDS reads
                // is issued before any of them is waited for
                double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
                int t = i + 1;
                for (; t + 3 <= cl; t += 4) {
                    acc0 += A[i][t] * B[t][cl];
                    acc1 += A[i][t + 1] * B[t + 1][cl];
                    acc2 += A[i][t + 2] * B[t + 2][cl];
                    acc3 += A[i][t + 3] * B[t + 3][cl];
                }
                for (; t <= cl; ++t) acc0 += A[i][t] * B[t][cl];
                v = rd[i] * B[i][cl] + ((acc0 + acc1) + (acc2 + acc3)) / rd[i];
            }
            Rp[i + (int64_t)cl * c] = v;
            if (RT != nullptr) RT[cl + (int64_t)i * c] = v;
        }
    }
    __syncthreads();
    if (tid == 0 && s_bad) flag[0] = 1;
    slot_end(slot);
}

// The same elimination for 64 < c <= 128: the c x c working matrix lives in
// dynamic LDS (ld c | 1, 132 KB at c = 128), thread (rg, l) owns column
// l = tid % 128 and every 8th row.  The second pass's product R2 R1 is left to
// a matrix-core contraction (R1 does not fit beside the working matrix).
constexpr int CQ_BIG = 128;
constexpr int CQ_RG2 = CQ_T / CQ_BIG;

__global__ __launch_bounds__(CQ_T) void k_chol_inv_big(int c, const double* __restrict__ G, double* __restrict__ R,
                                                        double* __restrict__ Ri, int* __restrict__ flag,
                                                        int second_pass, DevSlot* slot) {
    extern __shared__ double lds[];
    __shared__ double d0[CQ_BIG], pd[CQ_BIG], rd[CQ_BIG];
    __shared__ int s_bad;
    slot_begin(slot);
    const int ld = c | 1;
    double* A = lds;   // A[i * ld + l]
    const int tid = threadIdx.x;
    for (int e = tid; e < c * c; e += CQ_T) {
        const int l = e / c, i = e - l * c;
        A[i * ld + l] = i <= l ? G[i + (int64_t)l * c] : 0.0;
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int j = tid; j < c; j += CQ_T) d0[j] = A[j * ld + j];
    __syncthreads();
    const int l = tid % CQ_BIG, rg = tid / CQ_BIG;
    for (int j = 0; j < c; ++j) {
        double p = A[j * ld + j];
        const double dj = d0[j];
        const bool ok = p > 1e-10 * dj && p <= 4.0 * dj && dj < INFINITY;
        if (!ok) p = (dj > 0.0 && dj < INFINITY) ? dj : 1.0;   // keep going; the flag discards the result
        if (tid == 0) {
            pd[j] = p;
            if (!ok) s_bad = 1;
        }
        if (l < c) {
            const double ip = 1.0 / p;
            const double x = l == j ? 1.0 : A[j * ld + l];
            const int hi = l > j ? l : c - 1;
            for (int i = j + 1 + rg; i <= hi; i += CQ_RG2) A[i * ld + l] -= (A[j * ld + i] * ip) * x;
        }
        __syncthreads();
    }
    for (int j = tid; j < c; j += CQ_T) rd[j] = sqrt(pd[j]);
    __syncthreads();
    for (int e = tid; e < c * c; e += CQ_T) {
        const int cl = e / c, j = e - cl * c;
        const double v = cl > j ? A[j * ld + cl] / rd[j] : (cl == j ? rd[j] : 0.0);
        R[j + (int64_t)cl * c] = v;
        if (second_pass && fabs(v - (cl == j ? 1.0 : 0.0)) > 0.1) s_bad = 1;
        Ri[j + (int64_t)cl * c] = j <= cl ? (j == cl ? 1.0 : A[cl * ld + j]) / rd[cl] : 0.0;
    }
    __syncthreads();
    if (tid == 0 && s_bad) flag[0] = 1;
    slot_end(slot);
}

std::mutex g_cq_mu;
size_t g_cq_lds = 0;

__global__ void k_zero_flags(int n, int* __restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = 0;
}

}  // namespace

void zero_flags(int n, int* f, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_flags, dim3((n + 255) / 256), dim3(256), 0, st, n, f);
    TTSG_HIP(hipGetLastError());
}

bool cholqr_fits(int m, int c) { return c >= 1 && c <= CQ_BIG && m >= c; }

void cholqr2(int m, int c, const double* X, int64_t xr, int64_t xc, double* Q, int64_t qr, int64_t qc, double* R,
             int* flag, Arena& ar, hipStream_t st, double* RT, double* rinv_fro2) {
    TTSG_CHECK(cholqr_fits(m, c), TTSG_ERR_ARG, "cholqr2: needs m >= c and c <= 128");
    const size_t mark = ar.mark();
    double* G = ar.get<double>((int64_t)c * c);
    double* R1 = ar.get<double>((int64_t)c * c);
    double* R1i = ar.get<double>((int64_t)c * c);
    double* R2 = ar.get<double>((int64_t)c * c);
    double* R2i = ar.get<double>((int64_t)c * c);
    double* Q1 = ar.get<double>((int64_t)m * c);
    auto gram = [&](const double* Y, int64_t yr, int64_t yc) {
        ContractDesc d = cdesc(c, c, m);
        d.am = idx1(yc);
        d.ak = idx1(yr);
        d.bk = idx1(yr);
        d.bn = idx1(yc);
        d.cm = idx1(1);
        d.cn = idx1(c);
        contract(Prec::F64, d, Y, Y, G, st, &ar);
    };
    auto times_inv = [&](const double* Y, int64_t yr, int64_t yc, const double* Ri, double* Z, int64_t zr,
                         int64_t zc) {
        ContractDesc d = cdesc(m, c, c);
        d.am = idx1(yr);
        d.ak = idx1(yc);
        d.bk = idx1(1);
        d.bn = idx1(c);
        d.cm = idx1(zr);
        d.cn = idx1(zc);
        contract(Prec::F64, d, Y, Ri, Z, st, &ar);
    };
    auto chol = [&](double* Rf, double* Rfi, int second, const double* Rprev, double* Rout, double* RTout) {
        if (c <= CQ_MAX) {
            StatScope sc(TTSG_ST_QR, (double)c * c * c / 3.0 + (double)c * c * c / 3.0, 0.0, st);
            hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(CQ_T), 0, st, c, G, Rf, Rfi, flag, second, Rprev, Rout,
                               RTout, sc.slot());
            TTSG_HIP(hipGetLastError());
            return;
        }
        const size_t lds = (size_t)(c | 1) * c * sizeof(double);
        {
            std::lock_guard<std::mutex> lk(g_cq_mu);
            if (lds > g_cq_lds) {
                TTSG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol_inv_big),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                g_cq_lds = lds;
            }
        }
        {
            StatScope sc(TTSG_ST_QR, (double)c * c * c / 3.0 + (double)c * c * c / 3.0, 0.0, st);
            hipLaunchKernelGGL(k_chol_inv_big, dim3(1), dim3(CQ_T), lds, st, c, G, Rf, Rfi, flag, second,
                               sc.slot());
            TTSG_HIP(hipGetLastError());
        }
        if (second) {
            // R = R2 R1 (column-major c x c) and, when asked, R^T
            ContractDesc d = cdesc(c, c, c);
            d.am = idx1(1);
            d.ak = idx1(c);
            d.bk = idx1(1);
            d.bn = idx1(c);
            d.cm = idx1(1);
            d.cn = idx1(c);
            contract(Prec::F64, d, Rf, Rprev, Rout, st, &ar);
            if (RTout != nullptr) {
                d.cm = idx1(c);
                d.cn = idx1(1);
                contract(Prec::F64, d, Rf, Rprev, RTout, st, &ar);
            }
        }
    };
    gram(X, xr, xc);
    chol(R1, R1i, 0, nullptr, nullptr, nullptr);
    times_inv(X, xr, xc, R1i, Q1, c, 1);
    gram(Q1, c, 1);
    chol(R2, R2i, 1, R1, R, RT);   // also R = R2 R1 (and R^T)
    times_inv(Q1, c, 1, R2i, Q, qr, qc);
    if (rinv_fro2 != nullptr) {
        // R^{-1} = R1^{-1} R2^{-1} (column-major c x c), then its squared Frobenius norm
        double* Ri = ar.get<double>((int64_t)c * c);
        double* part = ar.get<double>(1024);
        ContractDesc d = cdesc(c, c, c);
        d.am = idx1(1);
        d.ak = idx1(c);
        d.bk = idx1(1);
        d.bn = idx1(c);
        d.cm = idx1(1);
        d.cn = idx1(c);
        contract(Prec::F64, d, R1i, R2i, Ri, st, &ar);
        sumsq((int64_t)c * c, Ri, part, rinv_fro2, st);
    }
    ar.release(mark);
}

}  // namespace ttsg
