// Exponential-sum right preconditioner (Sec. 4.1):
//   P^{-1} = sum_j alpha_j (x)_k exp(-beta_j M_k) ~ (M_1 (+) ... (+) M_d)^{-1}
//
// Coefficients come from an integral representation of 1/z (Sec. 4.1 takes
// them from such representations): with t = e^u,
//   1/z = int_0^inf exp(-t z) dt = int_R exp(u - e^u z) du,
// and the trapezoid rule with step h on [u_lo, u_hi] gives
//   beta_j = exp(u_j), alpha_j = h exp(u_j).
// For a relative accuracy tol of z E(z) on [zmin, zmax]: the lower cut costs at
// most e^{u_lo} zmax, the upper one exp(-e^{u_hi} zmin), each held to tol/4;
// the trapezoid error of this integrand decays like exp(-c/h) with c about 7,
// so h = 6.5 / log(2/tol).
//
// The mode factors exp(-beta_j M_k) are computed on the GPU by scaling and
// squaring: X = -beta_j M_k / 2^s with ||X||_1 <= 1/2, a degree-18 Taylor
// polynomial by Horner's rule (truncation below 1e-22 relative), then s
// squarings -- every step a batched FP64 matrix-core contraction over the
// zeta terms of one mode.
#include <algorithm>
#include <cmath>

#include "tt_ops.h"
#include "xlane.h"

namespace ttsg {

int expsum_coefficients(double zmin, double zmax, double tol, int max_terms, double* alpha, double* beta) {
    if (!(zmin > 0.0) || !(zmax >= zmin) || !(tol > 0.0 && tol < 1.0)) return -1;
    const double u_lo = std::log(tol / (4.0 * zmax));
    const double u_hi = std::log(std::log(4.0 / tol) / zmin);
    const double h = 6.5 / std::log(2.0 / tol);
    const int zeta = (int)std::ceil((u_hi - u_lo) / h) + 1;
    if (zeta > max_terms) return -zeta;
    for (int j = 0; j < zeta; ++j) {
        const double u = u_lo + h * j;
        beta[j] = std::exp(u);
        alpha[j] = h * std::exp(u);
    }
    return zeta;
}

namespace {

constexpr int TPB = 256;
constexpr int kTaylor = 18;

int nblk(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 65536)); }

// max_j sum_i |M[i][j]| (row-major n x n), one workgroup.
__global__ __launch_bounds__(TPB) void k_norm1(int n, const double* __restrict__ M, double* __restrict__ out) {
    __shared__ double red[TPB / 64];
    double best = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += fabs(M[(int64_t)i * n + j]);
        best = fmax(best, c);
    }
    for (int off = 32; off >= 1; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        *out = m;
    }
}

// out[b] = I for `batch` n x n matrices
__global__ void k_eye_batch(int64_t total, int n, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = e % ((int64_t)n * n);
        out[e] = (w / n == w % n) ? 1.0 : 0.0;
    }
}

// out[e] = c * M[e]
__global__ void k_scaled_copy(int64_t n, double c, const double* __restrict__ M, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = c * M[e];
}

// C[b] = alpha A[b] B[b] + beta C[b] for `batch` row-major n x n matrices
void batched_square_gemm(int n, int batch, double alpha, double beta, const double* A, const double* B, double* C,
                         hipStream_t st, Arena* ar) {
    ContractDesc dsc = cdesc(n, n, n, batch);
    const int64_t nn = (int64_t)n * n;
    dsc.ab = idx1(nn);
    dsc.am = idx1(n);
    dsc.ak = idx1(1);
    dsc.bb = idx1(nn);
    dsc.bk = idx1(n);
    dsc.bn = idx1(1);
    dsc.cb = idx1(nn);
    dsc.cm = idx1(n);
    dsc.cn = idx1(1);
    dsc.alpha = alpha;
    dsc.beta = beta;
    contract(Prec::F64, dsc, A, B, C, st, ar);
}

}  // namespace

void mode_exponentials(int zeta, const double* beta, int d, const int* n, const std::vector<const double*>& M,
                       const std::vector<double*>& out, Arena& ar, hipStream_t st) {
    TTSG_CHECK(zeta >= 1 && (int)M.size() == d && (int)out.size() == d, TTSG_ERR_ARG, "mode_exponentials: sizes");
    for (int j = 1; j < zeta; ++j)
        TTSG_CHECK(beta[j] >= beta[j - 1], TTSG_ERR_ARG, "preconditioner: beta must be ascending");
    for (int j = 0; j < zeta; ++j)
        TTSG_CHECK(beta[j] >= 0.0 && std::isfinite(beta[j]), TTSG_ERR_ARG, "preconditioner: beta must be finite, >= 0");
    const size_t mark = ar.mark();
    double* nrm = ar.get<double>(std::max(d, 1));
    for (int k = 0; k < d; ++k) {
        hipLaunchKernelGGL(k_norm1, dim3(1), dim3(TPB), 0, st, n[k], M[k], nrm + k);
        TTSG_HIP(hipGetLastError());
    }
    std::vector<double> hn(d, 0.0);
    const double* hp = static_cast<const double*>(read_back(nrm, d * sizeof(double), hn.data(), st));
    std::vector<double> norms(hp, hp + d);
    for (int k = 0; k < d; ++k) {
        TTSG_CHECK(std::isfinite(norms[k]), TTSG_ERR_NONFINITE, "preconditioner: mode matrix is not finite");
        const int nk = n[k];
        const int64_t nn = (int64_t)nk * nk;
        const size_t mk = ar.mark();
        double* X = ar.get<double>(zeta * nn);
        double* P = out[k];                 // result lands here: [zeta][n][n]
        double* Pn = ar.get<double>(zeta * nn);
        std::vector<int> sq(zeta, 0);
        for (int j = 0; j < zeta; ++j) {
            const double th = beta[j] * norms[k];
            sq[j] = th > 0.5 ? (int)std::ceil(std::log2(th / 0.5)) : 0;
            const double c = -beta[j] * std::ldexp(1.0, -sq[j]);
            hipLaunchKernelGGL(k_scaled_copy, dim3(nblk(nn)), dim3(TPB), 0, st, nn, c, M[k], X + j * nn);
        }
        TTSG_HIP(hipGetLastError());
        // Horner: P = I + X P / i for i = kTaylor .. 1, starting from P = I
        double* cur = Pn;
        double* nxt = P;
        hipLaunchKernelGGL(k_eye_batch, dim3(nblk(zeta * nn)), dim3(TPB), 0, st, (int64_t)zeta * nn, nk, cur);
        for (int i = kTaylor; i >= 1; --i) {
            hipLaunchKernelGGL(k_eye_batch, dim3(nblk(zeta * nn)), dim3(TPB), 0, st, (int64_t)zeta * nn, nk, nxt);
            TTSG_HIP(hipGetLastError());
            batched_square_gemm(nk, zeta, 1.0 / i, 1.0, X, cur, nxt, st, &ar);
            std::swap(cur, nxt);
        }
        // squarings: terms with larger beta need more (beta ascending, so a suffix)
        const int smax = *std::max_element(sq.begin(), sq.end());
        for (int t = 0; t < smax; ++t) {
            int j0 = 0;
            while (j0 < zeta && sq[j0] <= t) ++j0;
            const int cnt = zeta - j0;
            if (cnt <= 0) continue;
            batched_square_gemm(nk, cnt, 1.0, 0.0, cur + j0 * nn, cur + j0 * nn, nxt + j0 * nn, st, &ar);
            copy_f64(cnt * nn, nxt + j0 * nn, cur + j0 * nn, st);
        }
        if (cur != P) copy_f64(zeta * nn, cur, P, st);
        ar.release(mk);
    }
    ar.release(mark);
}

void mode_product_tt(int d, const int* n, const std::vector<int>& r, const std::vector<const double*>& x,
                     const std::vector<const double*>& E, double alpha, const std::vector<double*>& z, hipStream_t st,
                     Arena* ar) {
    // z_mu[a][i][b] = (alpha if mu == 0) sum_l E_mu[i][l] x_mu[a][l][b]:
    // one GEMM per mode with N = (a, b) walked as a two-level index
    for (int mu = 0; mu < d; ++mu) {
        const int nn = n[mu], rl = r[mu], rr = r[mu + 1];
        ContractDesc dsc = cdesc(nn, rl * rr, nn);
        dsc.am = idx1(nn);
        dsc.ak = idx1(1);
        dsc.bk = idx1(rr);
        dsc.bn = idx2(rr, 1, (int64_t)nn * rr);
        dsc.cm = idx1(rr);
        dsc.cn = idx2(rr, 1, (int64_t)nn * rr);
        dsc.alpha = mu == 0 ? alpha : 1.0;
        contract(Prec::F64, dsc, E[mu], x[mu], z[mu], st, ar);
    }
}

}  // namespace ttsg
