// Dense FP64 factorizations for the STTA recovery and the TT-SVD rounding.
//
// Each matrix is handled by one workgroup of 512 threads (8 wavefronts)
// working on column-major data in global memory (these matrices are at most a
// few MB and stay L2-resident).  Column operations are given to wavefronts,
// rows to lanes; reductions are wavefront shuffles.
//
//  * Householder QR (the unblocked right-looking algorithm; reflectors are
//    stored below the diagonal as in LAPACK's geqr2, with v_j = 1 implicit).
//  * Explicit thin Q from the stored reflectors (backward accumulation).
//  * One-sided Jacobi SVD (Hestenes): columns are rotated pairwise until every
//    pair is numerically orthogonal; the column pairs of a round come from the
//    circle method so that a round touches each column once and its pairs are
//    independent.  On exit the columns hold U*Sigma and V the rotations.
#include <algorithm>

#include "ttsg_internal.h"
#include "xlane.h"

namespace ttsg {
namespace {

constexpr int LA_THREADS = 512;


__global__ __launch_bounds__(LA_THREADS) void k_qr(int m, int c, double* __restrict__ A, int lda, int64_t sA,
                                                    double* __restrict__ tau, int64_t sT, DevSlot* slot) {
    slot_begin(slot);
    A += blockIdx.x * sA;
    tau += blockIdx.x * sT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int kmax = m < c ? m : c;
    __shared__ double s_tau, s_scale;
    for (int j = 0; j < kmax; ++j) {
        double* col = A + (int64_t)j * lda;
        if (wave == 0) {
            double s = 0.0;
            for (int i = j + 1 + lane; i < m; i += 64) s += col[i] * col[i];
            s = wave_sum64(s);
            if (lane == 0) {
                double alpha = col[j];
                if (s == 0.0) {
                    s_tau = 0.0;
                    s_scale = 0.0;
                    tau[j] = 0.0;
                } else {
                    double beta = -copysign(sqrt(alpha * alpha + s), alpha);
                    s_tau = (beta - alpha) / beta;
                    s_scale = 1.0 / (alpha - beta);
                    tau[j] = s_tau;
                    col[j] = beta;
                }
            }
        }
        __syncthreads();
        const double t = s_tau, sc = s_scale;
        if (t != 0.0) {
            for (int i = j + 1 + tid; i < m; i += blockDim.x) col[i] *= sc;
        }
        __syncthreads();
        if (t != 0.0) {
            for (int l = j + 1 + wave; l < c; l += nw) {
                double* cl = A + (int64_t)l * lda;
                double w = 0.0;
                for (int i = j + 1 + lane; i < m; i += 64) w += col[i] * cl[i];
                w = wave_sum64(w);
                w = t * (w + cl[j]);
                if (lane == 0) cl[j] -= w;
                for (int i = j + 1 + lane; i < m; i += 64) cl[i] -= w * col[i];
            }
        }
        __syncthreads();
    }
    slot_end(slot);
}

__global__ __launch_bounds__(LA_THREADS) void k_form_q(int m, int c, const double* __restrict__ A, int lda,
                                                        int64_t sA, const double* __restrict__ tau, int64_t sT,
                                                        double* __restrict__ Q, int ldq, int64_t sQ, DevSlot* slot) {
    slot_begin(slot);
    A += blockIdx.x * sA;
    tau += blockIdx.x * sT;
    Q += blockIdx.x * sQ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int k = m < c ? m : c;
    for (int l = 0; l < k; ++l)
        for (int i = tid; i < m; i += blockDim.x) Q[(int64_t)l * ldq + i] = (i == l) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {
        const double t = tau[j];
        if (t != 0.0) {
            const double* v = A + (int64_t)j * lda;
            for (int l = j + wave; l < k; l += nw) {
                double* ql = Q + (int64_t)l * ldq;
                double w = 0.0;
                for (int i = j + 1 + lane; i < m; i += 64) w += v[i] * ql[i];
                w = wave_sum64(w);
                w = t * (w + ql[j]);
                if (lane == 0) ql[j] -= w;
                for (int i = j + 1 + lane; i < m; i += 64) ql[i] -= w * v[i];
            }
        }
        __syncthreads();
    }
    slot_end(slot);
}

__device__ __forceinline__ void circle_pair(int r, int k, int cp, int& p, int& q) {
    if (k == 0) {
        p = cp - 1;
        q = r;
    } else {
        p = (r + k) % (cp - 1);
        q = (r - k + cp - 1) % (cp - 1);
    }
}

// One-sided Jacobi for matrices too large for LDS (they stay L2-resident).
// Same structure as the LDS kernel: a lane group of 32 lanes owns a column
// pair for a round, reduces the three dot products in registers and rotates
// the rows it owns; one barrier per round.
template <int G> __device__ __forceinline__ double gsum_g(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

__global__ __launch_bounds__(1024) void k_jacobi(int m, int c, double* __restrict__ A, int lda, int64_t sA,
                                                  double* __restrict__ V, int ldv, int64_t sV,
                                                  double* __restrict__ sig, int64_t sS, int maxsweeps,
                                                  double tol, DevSlot* slot) {
    slot_begin(slot);
    constexpr int G = 32;
    A += blockIdx.x * sA;
    V += blockIdx.x * sV;
    sig += blockIdx.x * sS;
    const int tid = threadIdx.x;
    const int grp = tid / G, lt = tid - grp * G, ngrp = blockDim.x / G;
    for (int l = 0; l < c; ++l)
        for (int i = tid; i < c; i += blockDim.x) V[(int64_t)l * ldv + i] = (i == l) ? 1.0 : 0.0;
    __shared__ int s_rot;
    __shared__ double s_fpart[1024 / G];
    if (tid == 0) s_rot = 0;
    double s_fro = 0.0;
    {
        // group partials summed in group order (the same bits every run)
        double f = 0.0;
        for (int l = grp; l < c; l += ngrp)
            for (int i = lt; i < m; i += G) f += A[(int64_t)l * lda + i] * A[(int64_t)l * lda + i];
        f = gsum_g<G>(f);
        if (lt == 0) s_fpart[grp] = f;
        __syncthreads();
        for (int g = 0; g < ngrp; ++g) s_fro += s_fpart[g];
    }
    // columns below 2 m eps ||A||_F carry only rounding noise (null space of a
    // rank-deficient matrix); their mutual dot products never look orthogonal,
    // so they are treated as converged
    const double nz = 2.0 * m * 2.220446049250313e-16;
    const double tiny = nz * nz * s_fro;
    const int cp = c + (c & 1);
    const int npair = cp / 2;
    int sweeps_done = 0;
    for (int sweep = 0; sweep < maxsweeps && cp > 1; ++sweep) {
        int rotated = 0;
        sweeps_done = sweep + 1;
        for (int r = 0; r < cp - 1; ++r) {
            for (int k = grp; k < npair; k += ngrp) {
                int p, q;
                if (k == 0) {
                    p = cp - 1;
                    q = r;
                } else {
                    p = (r + k) % (cp - 1);
                    q = (r - k + cp - 1) % (cp - 1);
                }
                if (p >= c || q >= c) continue;
                double* ap = A + (int64_t)p * lda;
                double* aq = A + (int64_t)q * lda;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lt; i < m; i += G) {
                    const double x = ap[i], y = aq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = gsum_g<G>(al);
                be = gsum_g<G>(be);
                ga = gsum_g<G>(ga);
                if (al <= tiny || be <= tiny || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t);
                const double sn = cs * t;
                for (int i = lt; i < m; i += G) {
                    const double x = ap[i], y = aq[i];
                    ap[i] = cs * x - sn * y;
                    aq[i] = sn * x + cs * y;
                }
                double* vp = V + (int64_t)p * ldv;
                double* vq = V + (int64_t)q * ldv;
                for (int i = lt; i < c; i += G) {
                    const double x = vp[i], y = vq[i];
                    vp[i] = cs * x - sn * y;
                    vq[i] = sn * x + cs * y;
                }
                rotated = 1;
            }
            __syncthreads();
        }
        if (rotated && lt == 0) s_rot = 1;
        __syncthreads();
        const int any = s_rot;
        __syncthreads();
        if (tid == 0) s_rot = 0;
        if (any == 0) break;
    }
    __syncthreads();
    for (int l = grp; l < c; l += ngrp) {
        const double* al = A + (int64_t)l * lda;
        double s2 = 0.0;
        for (int i = lt; i < m; i += G) s2 += al[i] * al[i];
        s2 = gsum_g<G>(s2);
        if (lt == 0) sig[l] = sqrt(s2);
    }
    slot_end(slot, (unsigned long long)sweeps_done);
}

}  // namespace

void qr_householder(int32_t batch, int32_t m, int32_t c, double* A, int32_t lda, int64_t strideA, double* tau,
                    int64_t strideTau, hipStream_t st) {
    if (batch <= 0 || m <= 0 || c <= 0) return;
    TTSG_CHECK(lda >= m, TTSG_ERR_ARG, "qr: lda < m");
    if (bounds_checking()) {
        check_range(A, ((int64_t)(batch - 1) * strideA + (int64_t)(c - 1) * lda + m) * 8, "qr A");
        check_range(tau, ((int64_t)(batch - 1) * strideTau + std::min(m, c)) * 8, "qr tau");
    }
    const double kq = std::min(m, c);
    StatScope scope(TTSG_ST_QR, batch * (2.0 * m * c * kq - 2.0 / 3.0 * kq * kq * kq),
                    batch * 16.0 * m * c, st);
    hipLaunchKernelGGL(k_qr, dim3(batch), dim3(LA_THREADS), 0, st, m, c, A, lda, strideA, tau, strideTau,
                       scope.slot());
    TTSG_HIP(hipGetLastError());
}

void qr_form_q(int32_t batch, int32_t m, int32_t c, const double* A, int32_t lda, int64_t strideA,
               const double* tau, int64_t strideTau, double* Q, int32_t ldq, int64_t strideQ, hipStream_t st) {
    if (batch <= 0 || m <= 0 || c <= 0) return;
    TTSG_CHECK(lda >= m && ldq >= m, TTSG_ERR_ARG, "form_q: leading dimension < m");
    if (bounds_checking()) {
        const int k = std::min(m, c);
        check_range(A, ((int64_t)(batch - 1) * strideA + (int64_t)(k - 1) * lda + m) * 8, "form_q A");
        check_range(Q, ((int64_t)(batch - 1) * strideQ + (int64_t)(k - 1) * ldq + m) * 8, "form_q Q");
    }
    const double kq = std::min(m, c);
    StatScope scope(TTSG_ST_QR, batch * (4.0 * m * kq * kq - 4.0 / 3.0 * kq * kq * kq),
                    batch * 16.0 * m * kq, st);
    hipLaunchKernelGGL(k_form_q, dim3(batch), dim3(LA_THREADS), 0, st, m, c, A, lda, strideA, tau, strideTau, Q,
                       ldq, strideQ, scope.slot());
    TTSG_HIP(hipGetLastError());
}

void svd_jacobi(int32_t batch, int32_t m, int32_t c, double* A, int32_t lda, int64_t strideA, double* V,
                int32_t ldv, int64_t strideV, double* sig, int64_t strideSig, hipStream_t st) {
    if (batch <= 0 || m <= 0 || c <= 0) return;
    TTSG_CHECK(m >= c, TTSG_ERR_ARG, "svd_jacobi needs m >= c");
    TTSG_CHECK(lda >= m && ldv >= c, TTSG_ERR_ARG, "svd_jacobi: leading dimension too small");
    if (bounds_checking()) {
        check_range(A, ((int64_t)(batch - 1) * strideA + (int64_t)(c - 1) * lda + m) * 8, "jacobi A");
        check_range(V, ((int64_t)(batch - 1) * strideV + (int64_t)(c - 1) * ldv + c) * 8, "jacobi V");
        check_range(sig, ((int64_t)(batch - 1) * strideSig + c) * 8, "jacobi sig");
    }
    // one sweep of c(c-1)/2 rotations, each three dot products and two
    // rotated column pairs (m and c long)
    StatScope scope(TTSG_ST_SVD, batch * 0.5 * c * (c - 1.0) * (12.0 * m + 6.0 * c), batch * 16.0 * m * c, st);
    hipLaunchKernelGGL(k_jacobi, dim3(batch), dim3(1024), 0, st, m, c, A, lda, strideA, V, ldv, strideV,
                       sig, strideSig, 30, 4.0 * m * 2.220446049250313e-16, scope.slot());
    TTSG_HIP(hipGetLastError());
}

}  // namespace ttsg
