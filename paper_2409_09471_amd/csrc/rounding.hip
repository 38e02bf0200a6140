// Rounding pipeline in FP64: STTA recovery (Sec. 3.3) and TT-SVD (Sec. 2.2).
//
// Ranks are decided on the host from singular values read back once per
// bond (a few hundred doubles); the subsequent contractions then run at the
// exact new sizes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "tt_ops.h"

namespace ttsg {
namespace {

__global__ void k_extract_r(int k, int c, const double* __restrict__ A, int lda, double* __restrict__ R, int ldr) {
    int total = k * c;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        int l = e / k, i = e - l * k;
        R[(int64_t)l * ldr + i] = (i <= l) ? A[(int64_t)l * lda + i] : 0.0;
    }
}

// dst[:, t] = fac[t] * src[:, perm[t]]  (column-major, `rows` rows)
__global__ void k_gather_cols(int rows, int k, const double* __restrict__ src, int lds, double* __restrict__ dst,
                              int ldd, const int* __restrict__ perm, const double* __restrict__ fac) {
    int total = rows * k;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        int t = e / rows, i = e - t * rows;
        dst[(int64_t)t * ldd + i] = fac[t] * src[(int64_t)perm[t] * lds + i];
    }
}

// Several column gathers in one launch (blockIdx.y = job): column t, row i of
// dst = fac[t] * src[perm[t]][i], written to row rowperm[i] when rowperm is set.
struct GatherJob {
    int rows, k, lds, ldd;
    const double* src;
    double* dst;
    const int* perm;
    const double* fac;
    const int* rowperm;
};
struct GatherBatch {
    int count;
    GatherJob j[32];
};
__global__ void k_gather_batched(GatherBatch gb) {
    const GatherJob g = gb.j[blockIdx.y];
    const int total = g.rows * g.k;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int t = e / g.rows, i = e - t * g.rows;
        const int oi = g.rowperm != nullptr ? g.rowperm[i] : i;
        g.dst[(int64_t)t * g.ldd + oi] = g.fac[t] * g.src[(int64_t)g.perm[t] * g.lds + i];
    }
}

__global__ void k_eye(int c, double* __restrict__ I) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c * c; e += gridDim.x * blockDim.x)
        I[e] = (e / c == e % c) ? 1.0 : 0.0;
}

inline int nb(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

void extract_r(int k, int c, const double* A, int lda, double* R, int ldr, hipStream_t st) {
    hipLaunchKernelGGL(k_extract_r, dim3(nb((int64_t)k * c)), dim3(256), 0, st, k, c, A, lda, R, ldr);
    TTSG_HIP(hipGetLastError());
}

void eye(int c, double* I, hipStream_t st) {
    hipLaunchKernelGGL(k_eye, dim3(nb((int64_t)c * c)), dim3(256), 0, st, c, I);
    TTSG_HIP(hipGetLastError());
}

// SVD of a c x c column-major matrix in place (LDS kernel when it fits).
void svd_small(int c, double* A, double* V, double* sig, hipStream_t st, double tol = 0.0, double drop_abs2 = 0.0) {
    if (jacobi_lds_fits(c, c)) {
        svd_jacobi_batched({JacobiJob{c, c, c, A, V, sig, tol, drop_abs2, 0.0}}, st);
    } else {
        svd_jacobi(1, c, c, A, c, 0, V, c, 0, sig, 0, st);
    }
}

void gather_cols(int rows, int k, const double* src, int lds, double* dst, int ldd, const int* perm,
                 const double* fac, hipStream_t st) {
    if (rows <= 0 || k <= 0) return;
    hipLaunchKernelGGL(k_gather_cols, dim3(nb((int64_t)rows * k)), dim3(256), 0, st, rows, k, src, lds, dst, ldd,
                       perm, fac);
    TTSG_HIP(hipGetLastError());
}

// Row-major C (M x N) = A (row-major M x K) * B (column-major K x N, ld = ldb)
void gemm_rm_cm(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                hipStream_t st, Arena* ar = nullptr) {
    ContractDesc d = cdesc(M, N, K);
    d.am = idx1(lda);
    d.ak = idx1(1);
    d.bk = idx1(1);
    d.bn = idx1(ldb);
    d.cm = idx1(ldc);
    d.cn = idx1(1);
    contract(Prec::F64, d, A, B, C, st, ar);
}

// Row-major C (M x N) = A (row-major M x K) * B (row-major K x N)
void gemm_rm_rm(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                hipStream_t st, Arena* ar = nullptr) {
    ContractDesc d = cdesc(M, N, K);
    d.am = idx1(lda);
    d.ak = idx1(1);
    d.bk = idx1(ldb);
    d.bn = idx1(1);
    d.cm = idx1(ldc);
    d.cn = idx1(1);
    contract(Prec::F64, d, A, B, C, st, ar);
}

// Row-major C (M x N) = A (column-major M x K, ld lda) * B (column-major K x N, ld ldb)
void gemm_cm_cm(int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                hipStream_t st, Arena* ar = nullptr) {
    ContractDesc d = cdesc(M, N, K);
    d.am = idx1(1);
    d.ak = idx1(lda);
    d.bk = idx1(1);
    d.bn = idx1(ldb);
    d.cm = idx1(ldc);
    d.cn = idx1(1);
    contract(Prec::F64, d, A, B, C, st, ar);
}

// Bonds whose rank the cap (not the tolerance) decided, per host thread.
thread_local int t_cap_events = 0;

// Smallest k whose discarded tail is <= delta; at least 1; capped at maxrank.
int trunc_rank(const std::vector<double>& s_desc, double delta, int maxrank) {
    int m = (int)s_desc.size();
    std::vector<double> tail(m + 1, 0.0);
    for (int j = m - 1; j >= 0; --j) tail[j] = tail[j + 1] + s_desc[j] * s_desc[j];
    int k = m;
    for (int j = 0; j < m; ++j)
        if (std::sqrt(tail[j]) <= delta) {
            k = j;
            break;
        }
    k = std::max(k, 1);
    if (maxrank > 0 && k > maxrank) {
        k = maxrank;
        ++t_cap_events;
    }
    return k;
}

std::vector<int> argsort_desc(const std::vector<double>& s) {
    std::vector<int> p(s.size());
    std::iota(p.begin(), p.end(), 0);
    std::stable_sort(p.begin(), p.end(), [&](int a, int b) { return s[a] > s[b]; });
    return p;
}

double read_scalar(const double* dev, hipStream_t st) {
    double h = 0.0;
    return *static_cast<const double*>(read_back(dev, sizeof(double), &h, st));
}

// Upload perm (ints) and factors (doubles) into device buffers.
void upload_perm(const std::vector<int>& perm, const std::vector<double>& fac, int* perm_dev, double* fac_dev,
                 hipStream_t st) {
    TTSG_HIP(hipMemcpyAsync(perm_dev, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice, st));
    TTSG_HIP(hipMemcpyAsync(fac_dev, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice, st));
}

}  // namespace

size_t tt_svd_extra_bytes(int d, const int* n, const int* r) {
    size_t sum = 0, mx = 0, rmax = 1;
    for (int mu = 0; mu < d; ++mu) {
        const size_t e = (size_t)r[mu] * n[mu] * r[mu + 1];
        sum += e;
        mx = std::max(mx, e);
        rmax = std::max(rmax, (size_t)std::max(r[mu], r[mu + 1]));
    }
    // four core-sized buffers (A, Q, T, QV), the snapshot of every core, the
    // first CholQR2 pass's Q, the c x c factors (R, V, the Jacobi buffer and
    // CholQR2's five), + the host read-back block (squared norm, flags,
    // per-bond singular values)
    return (sum + 6 * mx + 12 * rmax * rmax + 4096) * sizeof(double) + (size_t)(d + 1) * 64 +
           (4 + (rmax + 2) * d) * sizeof(double) + 256;
}

double tt_svd_inplace(int d, const int* n, std::vector<int>& r, const std::vector<double*>& w,
                      const std::vector<int64_t>& cap_elems, double tol, int maxrank, Arena& ar, hipStream_t st,
                      double* norm_before) {
    const size_t mark = ar.mark();
    int64_t maxcore = 0, maxr = 1;
    for (int mu = 0; mu < d; ++mu) {
        maxcore = std::max<int64_t>(maxcore, (int64_t)r[mu] * n[mu] * r[mu + 1]);
        maxr = std::max<int64_t>(maxr, std::max(r[mu], r[mu + 1]));
    }
    double* A = ar.get<double>(maxcore);
    double* Q = ar.get<double>(maxcore);
    double* T = ar.get<double>(maxcore);
    double* Rm = ar.get<double>(maxr * maxr);
    double* V = ar.get<double>(maxr * maxr);
    double* QV = ar.get<double>(maxcore);
    double* Jb = ar.get<double>(maxr * maxr);   // 128-column Jacobi: R in, R V out
    double* tau = ar.get<double>(maxr);
    double* sig = ar.get<double>(maxr);
    double* part = ar.get<double>(1024);
    int* perm_dev = ar.get<int>(maxr);
    double* fac_dev = ar.get<double>(maxr);
    // Values the host reads back, packed so that each synchronization point
    // costs one copy: [squared norm, spare, right-to-left CholQR flag] and,
    // per left-to-right bond, [singular values (maxr), CholQR flag].
    const int64_t sbk = maxr + 2;
    double* rb = ar.get<double>(4 + sbk * d);
    fill(4 + sbk * d, 0.0, rb, st);   // clears every flag
    double* scal = rb;
    int* flags = reinterpret_cast<int*>(rb + 2);
    auto bond_blk = [&](int mu) { return rb + 4 + sbk * mu; };
    auto bond_flag = [&](int mu) { return reinterpret_cast<int*>(bond_blk(mu) + maxr); };
    std::vector<double> hb(4 + sbk);

    // 1) right-to-left QR orthogonalization.  Bonds whose unfolding fits
    // CholQR2 use it (matrix-core Gram products); if any of them reports an
    // untrustworthy factorization, the cores are restored from a snapshot and
    // the sweep is redone with Householder QR.
    std::vector<int> r_in = r;
    bool any_chol = false;
    for (int mu = d - 1; mu >= 1; --mu) any_chol = any_chol || cholqr_fits(n[mu] * r[mu + 1], r[mu]);
    std::vector<double*> snap(d, nullptr);
    if (any_chol)
        for (int mu = 0; mu < d; ++mu) {
            snap[mu] = ar.get<double>((int64_t)r[mu] * n[mu] * r[mu + 1]);
            copy_f64((int64_t)r[mu] * n[mu] * r[mu + 1], w[mu], snap[mu], st);
        }
    // The core that a bond factors is read from X: w[mu] for the first bond,
    // then T, where the previous bond left the core times its R factor (no
    // copy back into w per bond; the last such product is copied once).
    auto orthogonalize = [&](bool allow_chol) {
        const double* X = w[d - 1];
        for (int mu = d - 1; mu >= 1; --mu) {
            const int rl = r[mu], rr = r[mu + 1], m = n[mu] * rr, c = rl;
            const int k = std::min(m, c);
            if (allow_chol && cholqr_fits(m, c)) {
                // the row-major core is the column-major m x c matrix C^T; Q^T
                // is the new row-major core
                cholqr2(m, c, X, 1, m, w[mu], 1, m, Rm, flags, ar, st);
            } else if (tsqr_fits(m, c)) {
                const size_t mk = ar.mark();
                TsqrPlan plan;
                plan.factor(m, c, X, m, ar, st);
                double* I = ar.get<double>((int64_t)c * c);
                eye(c, I, st);
                copy_f64((int64_t)c * c, plan.R, Rm, st);          // R: c x c, ld c (k == c)
                plan.apply(c, I, c, w[mu], m, false, ar, st);      // Q^T as the new row-major core
                ar.release(mk);
            } else {
                copy_f64((int64_t)m * c, X, A, st);                // column-major m x c == row-major core
                qr_householder(1, m, c, A, m, 0, tau, 0, st);
                qr_form_q(1, m, c, A, m, 0, tau, 0, w[mu], m, 0, st);  // Q^T as the new row-major core
                extract_r(k, c, A, m, Rm, k, st);
            }
            const int rll = r[mu - 1], nl = n[mu - 1];
            // T (rll*nl x k) = W_{mu-1} (rll*nl x rl) * R^T
            // B[l][kk] = R[kk][l] = Rm[l*k + kk]: the column-major R read row-major
            gemm_rm_rm(rll * nl, k, rl, w[mu - 1], rl, Rm, k, T, k, st, &ar);
            X = T;
            r[mu] = k;
        }
        if (d >= 2) copy_f64((int64_t)r[0] * n[0] * r[1], T, w[0], st);
    };
    orthogonalize(true);
    // squared norm and flag in one read
    sumsq((int64_t)r[0] * n[0] * r[1], w[0], part, scal, st);
    const double* h3 = static_cast<const double*>(read_back(rb, 3 * sizeof(double), hb.data(), st));
    double nrm2 = h3[0];
    int hflag0 = 0;
    std::memcpy(&hflag0, &h3[2], sizeof(int));
    if (any_chol && hflag0 != 0) {
        stats_event(TTSG_ST_QR_REDO);
        r = r_in;
        for (int mu = 0; mu < d; ++mu) copy_f64((int64_t)r[mu] * n[mu] * r[mu + 1], snap[mu], w[mu], st);
        orthogonalize(false);
        sumsq((int64_t)r[0] * n[0] * r[1], w[0], part, scal, st);
        nrm2 = read_scalar(scal, st);
    }
    const double nrm = std::sqrt(nrm2);
    if (norm_before) *norm_before = nrm;
    if (nrm == 0.0 || d == 1) {
        ar.release(mark);
        return nrm;
    }
    const double delta = tol * nrm / std::sqrt((double)(d - 1));

    // 2) left-to-right truncated SVDs.  Host arrays handed to hipMemcpyAsync are
    // kept in `hold` until the stream is synchronized at the end.
    std::vector<double> hsig;
    std::vector<std::vector<int>> hold_i;
    std::vector<std::vector<double>> hold_d;
    // X: the unfolding of the current core (w[0], then T where the previous
    // bond left S V^T times the next core; T is scratch again once X is read)
    const double* X = w[0];
    for (int mu = 0; mu <= d - 2; ++mu) {
        const int rl = r[mu], rr = r[mu + 1], m = rl * n[mu], c = rr;
        const int r2 = r[mu + 2], n2 = n[mu + 1];
        int k;
        std::vector<int> perm;
        if (m >= c) {
            // QR of the unfolding: CholQR2 (Q row-major m x c in Q) when it fits,
            // TSQR or single-workgroup Householder otherwise or when CholQR2
            // flags the factorization
            bool chol = cholqr_fits(m, c);
            const bool tsqr = tsqr_fits(m, c);
            TsqrPlan plan;
            const size_t mk = ar.mark();
            auto householder = [&]() {
                transpose2d(m, c, X, c, A, m, st);               // column-major m x c
                if (tsqr) {
                    plan.factor(m, c, A, m, ar, st);
                    copy_f64((int64_t)c * c, plan.R, Rm, st);
                } else {
                    qr_householder(1, m, c, A, m, 0, tau, 0, st);
                    qr_form_q(1, m, c, A, m, 0, tau, 0, Q, m, 0, st);
                    extract_r(c, c, A, m, Rm, c, st);
                }
            };
            // 64 < c <= 128: one-sided Jacobi on R itself (the matrix fills the
            // LDS, so no rotation accumulator): R V = B = U_R S gives U_R = B / s,
            // and S V_R^T = U_R^T R is one small matrix-core product afterwards
            const bool big = c > 64 && jacobi_big_fits(c, c);
            auto small_svd = [&](bool have_rt) {
                if (big) {
                    // U_R = B / s is orthonormal only to the Jacobi tolerance, and the
                    // reconstruction Q U_k (U_k^T R) errs by about that much relative
                    // to ||R||: the tolerance follows the rounding tolerance
                    // (1e-3 of it, at most 1e-11, at least 4 c eps)
                    const double jt = std::max(4.0 * c * 2.220446049250313e-16, std::min(1e-11, 1e-3 * tol));
                    copy_f64((int64_t)c * c, Rm, Jb, st);
                    svd_jacobi_big({JacobiJob{c, c, c, Jb, nullptr, bond_blk(mu), jt, delta * delta / (16.0 * c),
                                              0.0}},
                                   false, st);
                    const double* hr =
                        static_cast<const double*>(read_back(bond_blk(mu), sbk * sizeof(double), hb.data(), st));
                    std::copy(hr, hr + sbk, hb.begin());
                    hsig.assign(hb.begin(), hb.begin() + c);
                    return;
                }
                // SVD of R through one-sided Jacobi on R^T (rows of a QR factor of a
                // graded unfolding converge in few sweeps): R^T V' = U' S gives
                // R = V' S U'^T, i.e. U_R = V' and S V_R^T = (U' S)^T.  Relative
                // orthogonality 1e-11 is far below every rounding tolerance used.
                // Columns of norm below delta / (4 sqrt(c)) hold at most delta^2 / 16
                // together, so the truncation drops all of them: they are not
                // rotated any more (the error of the truncation stays exactly the
                // norm of the dropped columns).
                if (!have_rt) transpose2d(c, c, Rm, c, QV, c, st);   // QV = R^T (column-major)
                svd_small(c, QV, V, bond_blk(mu), st, 1e-11, delta * delta / (16.0 * c));
                // singular values and the CholQR flag in one read
                const double* hr =
                    static_cast<const double*>(read_back(bond_blk(mu), sbk * sizeof(double), hb.data(), st));
                std::copy(hr, hr + sbk, hb.begin());
                hsig.assign(hb.begin(), hb.begin() + c);
            };
            // When 1 / ||R^{-1}||_F (a lower bound of the smallest singular
            // value) is above the truncation threshold and the cap does not
            // bind, no direction can be dropped (the tail of even one singular
            // value exceeds delta): the bond keeps Q and passes R on, the same
            // tensor without the SVD's gauge, and the Jacobi SVD (one workgroup,
            // 0.1 ms at 64 columns, about 1 ms at 128) is not run
            bool keep_all = false;
            if (chol && (maxrank <= 0 || c <= maxrank)) {
                cholqr2(m, c, X, c, 1, Q, c, 1, Rm, bond_flag(mu), ar, st, QV, bond_blk(mu) + maxr + 1);
                const double* hr =
                    static_cast<const double*>(read_back(bond_blk(mu), sbk * sizeof(double), hb.data(), st));
                std::copy(hr, hr + sbk, hb.begin());
                int hflag = 0;
                std::memcpy(&hflag, &hb[maxr], sizeof(int));
                const double f2 = hb[maxr + 1];
                if (hflag != 0) {
                    stats_event(TTSG_ST_QR_REDO);
                    chol = false;
                } else if (std::isfinite(f2) && f2 > 0.0 && 1.0 / std::sqrt(f2) > 2.0 * delta) {
                    keep_all = true;
                } else {
                    small_svd(true);
                }
            } else if (chol) {
                cholqr2(m, c, X, c, 1, Q, c, 1, Rm, bond_flag(mu), ar, st, QV);   // QV = R^T
                small_svd(true);
                int hflag = 0;
                std::memcpy(&hflag, &hb[maxr], sizeof(int));
                if (hflag != 0) {
                    stats_event(TTSG_ST_QR_REDO);
                    chol = false;
                }
            }
            if (keep_all) {
                // new core = Q (row-major m x c); S V^T read from QV = R^T
                copy_f64((int64_t)m * c, Q, w[mu], st);
                ar.release(mk);
                k = c;
            } else {
                if (!chol) {
                    householder();
                    small_svd(false);
                }
                perm = argsort_desc(hsig);
                std::vector<double> sd(c);
                for (int t = 0; t < c; ++t) sd[t] = hsig[perm[t]];
                k = trunc_rank(sd, delta, maxrank);
                k = std::min(k, c);
                // the LDS Jacobi returns its columns sorted by singular value, so
                // the kept vectors are the leading columns; otherwise gather them
                bool sorted = true;
                for (int t = 0; t < c; ++t) sorted = sorted && perm[t] == t;
                const double* Uk = V;
                if (big) {
                    // U_k = B[:, :k] / s (zero for a zero singular value)
                    std::vector<int> pk(k);
                    std::vector<double> inv(k);
                    for (int t = 0; t < k; ++t) {
                        pk[t] = t;
                        inv[t] = sd[t] > 0.0 ? 1.0 / sd[t] : 0.0;
                    }
                    hold_i.push_back(pk);
                    hold_d.push_back(inv);
                    upload_perm(hold_i.back(), hold_d.back(), perm_dev, fac_dev, st);
                    gather_cols(c, k, Jb, c, V, c, perm_dev, fac_dev, st);
                    // QV (column-major c x k) = R^T U_k, i.e. S V_R^T read row-major
                    ContractDesc dr = cdesc(c, k, c);
                    dr.am = idx1(c);
                    dr.ak = idx1(1);
                    dr.bk = idx1(1);
                    dr.bn = idx1(c);
                    dr.cm = idx1(1);
                    dr.cn = idx1(c);
                    contract(Prec::F64, dr, Rm, V, QV, st, &ar);
                } else if (!sorted) {
                    std::vector<int> pk(perm.begin(), perm.begin() + k);
                    hold_i.push_back(pk);
                    hold_d.push_back(std::vector<double>(k, 1.0));
                    upload_perm(hold_i.back(), hold_d.back(), perm_dev, fac_dev, st);
                    gather_cols(c, k, V, c, T, c, perm_dev, fac_dev, st);   // Uk (c x k, column-major) = V'[:, perm]
                    Uk = T;
                }
                // new core (row-major m x k) = Q (m x c) * Uk
                if (chol) {
                    ContractDesc dq = cdesc(m, k, c);
                    dq.am = idx1(c);
                    dq.ak = idx1(1);
                    dq.bk = idx1(1);
                    dq.bn = idx1(c);
                    dq.cm = idx1(k);
                    dq.cn = idx1(1);
                    contract(Prec::F64, dq, Q, Uk, w[mu], st, &ar);
                } else if (tsqr) {
                    plan.apply(k, Uk, c, w[mu], k, true, ar, st);
                } else {
                    gemm_cm_cm(m, k, c, Q, m, Uk, c, w[mu], k, st, &ar);
                }
                ar.release(mk);
                // S V_R^T (row-major k x c == column-major c x k) = (U' S)[:, perm]:
                // the leading k columns of QV when sorted
                if (!sorted && !big) {
                    gather_cols(c, k, QV, c, Rm, c, perm_dev, fac_dev, st);
                    copy_f64((int64_t)c * k, Rm, QV, st);
                }
            }
        } else {
            // wide unfolding: M^T (c x m) is the row-major core read column-major
            copy_f64((int64_t)m * c, X, A, st);
            qr_householder(1, c, m, A, c, 0, tau, 0, st);
            qr_form_q(1, c, m, A, c, 0, tau, 0, Q, c, 0, st);   // Q2: c x m
            extract_r(m, m, A, c, Rm, m, st);                    // R2: m x m (column-major)
            // R2^T column-major = transpose of R2
            transpose2d(m, m, Rm, m, T, m, st);                  // T = R2 row-major == R2^T column-major
            svd_small(m, T, V, sig, st);                         // R2^T = U2 S V2^T
            hsig.assign(m, 0.0);
            TTSG_HIP(hipMemcpyAsync(hsig.data(), sig, m * sizeof(double), hipMemcpyDeviceToHost, st));
            TTSG_HIP(hipStreamSynchronize(st));
            perm = argsort_desc(hsig);
            std::vector<double> sd(m);
            for (int t = 0; t < m; ++t) sd[t] = hsig[perm[t]];
            k = trunc_rank(sd, delta, maxrank);
            k = std::min(k, m);
            std::vector<int> pk(perm.begin(), perm.begin() + k);
            std::vector<double> inv(k), one(k, 1.0);
            for (int t = 0; t < k; ++t) inv[t] = hsig[pk[t]] > 0.0 ? 1.0 / hsig[pk[t]] : 0.0;
            hold_i.push_back(pk);
            hold_d.push_back(inv);
            upload_perm(hold_i.back(), hold_d.back(), perm_dev, fac_dev, st);
            // new core (row-major m x k): columns of U2 = (U2 S)[:, perm] / s, written row-major
            gather_cols(m, k, T, m, A, m, perm_dev, fac_dev, st);  // A: column-major m x k
            transpose2d(k, m, A, m, w[mu], k, st);                 // row-major m x k
            // (Q2 V2) column-major c x m, then SVt (row-major k x c) = S * (Q2 V2)[:, perm]^T
            gemm_cm_cm(c, m, m, Q, c, V, m, QV, m, st, &ar);            // row-major c x m == QV^T column-major
            // QV row-major c x m: column j of (Q2 V2) is strided by m -> transpose to column-major
            transpose2d(c, m, QV, m, A, c, st);                    // A column-major c x m
            std::vector<double> sv(k);
            for (int t = 0; t < k; ++t) sv[t] = hsig[pk[t]];
            hold_d.push_back(sv);
            TTSG_HIP(hipMemcpyAsync(fac_dev, hold_d.back().data(), k * sizeof(double), hipMemcpyHostToDevice, st));
            gather_cols(c, k, A, c, QV, c, perm_dev, fac_dev, st);
        }
        // W_{mu+1} (k x n2*r2) = SVt (row-major k x c == QV column-major c x k) * W_{mu+1} (c x n2*r2)
        {
            ContractDesc dd = cdesc(k, n2 * r2, c);
            dd.am = idx1(c);   // SVt[t][l] = QV[t*c + l]
            dd.ak = idx1(1);
            dd.bk = idx1((int64_t)n2 * r2);
            dd.bn = idx1(1);
            dd.cm = idx1((int64_t)n2 * r2);
            dd.cn = idx1(1);
            contract(Prec::F64, dd, QV, w[mu + 1], T, st, &ar);
            X = T;
        }
        r[mu + 1] = k;
        (void)cap_elems;
    }
    copy_f64((int64_t)r[d - 1] * n[d - 1] * r[d], T, w[d - 1], st);
    sumsq((int64_t)r[d - 1] * n[d - 1], w[d - 1], part, scal, st);
    const double nout = std::sqrt(read_scalar(scal, st));
    ar.release(mark);
    return nout;
}

void stta_recover(int d, const int* n, const std::vector<int>& rho, const std::vector<int>& rx,
                  const std::vector<const double*>& Psi, const std::vector<const double*>& Omega, double rcond,
                  const std::vector<double*>& out, std::vector<int>& r_out, Arena& ar, hipStream_t st) {
    const size_t mark = ar.mark();
    r_out.assign(d + 1, 1);
    if (d == 1) {
        copy_f64(n[0], Psi[0], out[0], st);
        return;
    }
    // SVD of every Omega_b (rho_b x rx_b, rho_b >= rx_b) as Omega = Q R followed
    // by one-sided Jacobi on R^T (graded matrices converge in a third of the
    // sweeps that Jacobi on Omega itself needs): R^T W = U_B S gives
    // Omega = (Q W) S U_B^T, so Omega^+ = U_B S^-1 (Q W)^T.
    std::vector<double*> Ab(d), Rt(d), Wb(d), Sb(d), Gb(d), Vk(d), Wk(d), Qb(d);
    std::vector<int*> permb(d, nullptr);
    std::vector<double*> facb(d, nullptr);
    // singular values of all bonds side by side: one read-back
    int64_t s_tot = 0;
    std::vector<int64_t> s_off(d, 0);
    for (int b = 1; b <= d - 1; ++b) {
        s_off[b] = s_tot;
        s_tot += rx[b];
    }
    double* Sall = ar.get<double>(std::max<int64_t>(s_tot, 1));
    // gather tables of all bonds (factors, then indices), one upload
    int64_t u_tot = 0;
    for (int b = 1; b <= d - 1; ++b) u_tot += rx[b] + (rx[b] + 1) / 2;
    double* Uall = ar.get<double>(std::max<int64_t>(u_tot, 1));
    std::vector<TsqrPlan> plans(d);
    std::vector<bool> use_tsqr(d, false), use_small(d, false), use_big(d, false);
    std::vector<int*> pivb(d, nullptr);
    std::vector<QrJob> qjobs;
    int64_t maxT = 1;
    for (int b = 1; b <= d - 1; ++b) {
        const int m = rho[b], c = rx[b];
        TTSG_CHECK(m >= c, TTSG_ERR_ARG, "STTA needs rho_b >= rx_b");
        Ab[b] = ar.get<double>((int64_t)m * c);
        Rt[b] = ar.get<double>((int64_t)c * c);
        Wb[b] = ar.get<double>((int64_t)c * c);
        Sb[b] = Sall + s_off[b];
        Gb[b] = ar.get<double>((int64_t)m * c);
        Vk[b] = ar.get<double>((int64_t)c * c);
        Wk[b] = ar.get<double>((int64_t)c * c);
        use_small[b] = qr_small_fits(m, c);
        use_tsqr[b] = !use_small[b] && tsqr_fits(m, c);
        // 64 < rx_b <= 128: one-sided Jacobi on Omega itself with the rotations
        // accumulated (Omega V = B = U S, so Omega^+ = (V S^-1) (B S^-1)^T)
        use_big[b] = !use_small[b] && !use_tsqr[b] && c > 64 && jacobi_big_fits(m, c);
        if (use_big[b]) {
            transpose2d(m, c, Omega[b - 1], c, Ab[b], m, st);    // column-major m x c
            continue;
        }
        if (use_small[b]) {
            // column-pivoted: R^T is then graded and the Jacobi SVD below
            // converges in fewer sweeps; Omega is read row-major as it is and
            // R^T written directly
            Qb[b] = ar.get<double>((int64_t)m * c);
            pivb[b] = ar.get<int>(c);
            QrJob qj{m, c, c, Omega[b - 1], Qb[b], Rt[b], pivb[b]};
            qj.a_rowmajor = true;
            qj.r_transposed = true;
            qjobs.push_back(qj);
            continue;
        }
        transpose2d(m, c, Omega[b - 1], c, Ab[b], m, st);        // column-major m x c
        if (use_tsqr[b]) {
            plans[b].factor(m, c, Ab[b], m, ar, st);
            transpose2d(c, c, plans[b].R, c, Rt[b], c, st);       // R (column-major) -> R^T
        } else {
            double* tau = ar.get<double>(c);
            double* Rm = ar.get<double>((int64_t)c * c);
            Qb[b] = ar.get<double>((int64_t)m * c);
            qr_householder(1, m, c, Ab[b], m, 0, tau, 0, st);
            qr_form_q(1, m, c, Ab[b], m, 0, tau, 0, Qb[b], m, 0, st);
            extract_r(c, c, Ab[b], m, Rm, c, st);
            transpose2d(c, c, Rm, c, Rt[b], c, st);
        }
    }
    // all small QRs of the bonds in one launch
    if (!qjobs.empty()) qr_small_batched(qjobs, st);
    {
        std::vector<JacobiJob> jobs, big_jobs;
        for (int b = 1; b <= d - 1; ++b) {
            // singular values below rcond * s_max are dropped, so rotations
            // that leave 1e-3 rcond of non-orthogonality change nothing kept
            const double jt = std::max(4.0 * rx[b] * 2.220446049250313e-16, 1e-3 * rcond);
            // singular values below rcond s_max are dropped: columns shorter
            // than rcond / 16 times the longest one are not rotated any more
            if (use_big[b])
                big_jobs.push_back(JacobiJob{rho[b], rx[b], rho[b], Ab[b], Wb[b], Sb[b], jt, 0.0,
                                             (rcond / 16.0) * (rcond / 16.0)});
            else if (jacobi_lds_fits(rx[b], rx[b]))
                jobs.push_back(JacobiJob{rx[b], rx[b], rx[b], Rt[b], Wb[b], Sb[b], jt, 0.0,
                                         (rcond / 16.0) * (rcond / 16.0)});
            else
                svd_jacobi(1, rx[b], rx[b], Rt[b], rx[b], 0, Wb[b], rx[b], 0, Sb[b], 0, st);
        }
        if (!jobs.empty()) svd_jacobi_batched(jobs, st);
        if (!big_jobs.empty()) svd_jacobi_big(big_jobs, true, st, &ar);
    }
    for (int mu = 0; mu < d; ++mu) maxT = std::max<int64_t>(maxT, (int64_t)rx[mu] * n[mu] * rx[mu + 1]);
    for (int b = 1; b <= d - 1; ++b) maxT = std::max<int64_t>(maxT, (int64_t)rho[b] * rx[b]);
    double* T = ar.get<double>(maxT);
    std::vector<std::vector<double>> hs(d);
    std::vector<double> hall(std::max<int64_t>(s_tot, 1));
    {
        const double* hr = static_cast<const double*>(read_back(Sall, s_tot * sizeof(double), hall.data(), st));
        if (hr != hall.data()) std::copy(hr, hr + s_tot, hall.begin());
    }
    std::vector<std::vector<int>> keep(d);
    std::vector<std::vector<double>> facs(d);
    // host image of the gather tables; alive until the final synchronization
    std::vector<double> hup(std::max<int64_t>(u_tot, 1), 0.0);
    int64_t u_off = 0;
    for (int b = 1; b <= d - 1; ++b) {
        hs[b].assign(hall.begin() + s_off[b], hall.begin() + s_off[b] + rx[b]);
        std::vector<int> p = argsort_desc(hs[b]);
        const double smax = hs[b][p[0]];
        int k = 0;
        while (k < (int)p.size() && hs[b][p[k]] > rcond * smax && hs[b][p[k]] > 0.0) ++k;
        k = std::max(k, 1);
        keep[b].assign(p.begin(), p.begin() + k);
        facs[b].resize(k);
        for (int t = 0; t < k; ++t) {
            double sv = hs[b][keep[b][t]];
            facs[b][t] = sv > 0.0 ? 1.0 / sv : 0.0;
        }
        r_out[b] = k;
        facb[b] = Uall + u_off;
        permb[b] = reinterpret_cast<int*>(Uall + u_off + k);
        std::memcpy(hup.data() + u_off, facs[b].data(), k * sizeof(double));
        std::memcpy(hup.data() + u_off + k, keep[b].data(), k * sizeof(int));
        u_off += k + (k + 1) / 2;
    }
    {
        // from pinned memory when it fits (kept untouched until the final synchronization below)
        double* up = (size_t)u_off <= kStageDoubles ? host_stage(1) : nullptr;
        if (up != nullptr) std::copy(hup.begin(), hup.begin() + u_off, up);
        TTSG_HIP(hipMemcpyAsync(Uall, up != nullptr ? up : hup.data(), u_off * sizeof(double), hipMemcpyHostToDevice,
                                st));
    }
    // the gathers of every bond, batched:
    //   V'_b (column-major rx x k) = U_B[:, keep] = (U_B S)[:, keep] / s; with
    //   Omega P = Q R the right factor is P U_B, rows of U_B scattered by P;
    //   W[:, keep] / s for G_b (row-major k x rho == column-major rho x k) = Q W[:, keep] / s
    {
        std::vector<GatherJob> gj;
        for (int b = 1; b <= d - 1; ++b) {
            const int k = r_out[b], c = rx[b];
            if (use_big[b]) {
                // V'_b = V[:, keep] / s and G_b = B[:, keep] / s (column-major rho x k)
                gj.push_back(GatherJob{c, k, c, c, Wb[b], Vk[b], permb[b], facb[b], nullptr});
                gj.push_back(GatherJob{rho[b], k, rho[b], rho[b], Ab[b], Gb[b], permb[b], facb[b], nullptr});
                continue;
            }
            gj.push_back(GatherJob{c, k, c, c, Rt[b], Vk[b], permb[b], facb[b], pivb[b]});
            gj.push_back(GatherJob{c, k, c, c, Wb[b], Wk[b], permb[b], facb[b], nullptr});
        }
        for (size_t j0 = 0; j0 < gj.size(); j0 += 32) {
            GatherBatch gb{};
            gb.count = (int)std::min<size_t>(32, gj.size() - j0);
            int64_t mx = 1;
            for (int t = 0; t < gb.count; ++t) {
                gb.j[t] = gj[j0 + t];
                mx = std::max<int64_t>(mx, (int64_t)gb.j[t].rows * gb.j[t].k);
            }
            hipLaunchKernelGGL(k_gather_batched, dim3(nb(mx), gb.count), dim3(256), 0, st, gb);
            TTSG_HIP(hipGetLastError());
        }
    }
    for (int b = 1; b <= d - 1; ++b) {
        const int k = r_out[b];
        const int m = rho[b], c = rx[b];
        if (use_big[b]) {
            // G_b was gathered directly
        } else if (use_small[b]) {
            // G_b (column-major m x k) = Q (column-major m x c) * W[:, keep] / s
            ContractDesc dg = cdesc(m, k, c);
            dg.am = idx1(1);
            dg.ak = idx1(m);
            dg.bk = idx1(1);
            dg.bn = idx1(c);
            dg.cm = idx1(1);
            dg.cn = idx1(m);
            contract(Prec::F64, dg, Qb[b], Wk[b], Gb[b], st, &ar);
        } else if (use_tsqr[b]) {
            plans[b].apply(k, Wk[b], c, Gb[b], m, false, ar, st);
        } else {
            gemm_cm_cm(m, k, c, Qb[b], m, Wk[b], c, T, k, st, &ar);   // row-major m x k
            transpose2d(m, k, T, k, Gb[b], m, st);                    // column-major m x k
        }
    }
    for (int mu = 0; mu < d; ++mu) {
        const int nn = n[mu];
        const int kl = r_out[mu], kr = r_out[mu + 1];
        const int qr = rx[mu + 1];
        const double* src = Psi[mu];
        double* mid = T;
        if (mu >= 1) {
            // T (kl x nn*qr) = G_mu (kl x rho_mu) * Psi_mu (rho_mu x nn*qr)
            gemm_rm_rm(kl, nn * qr, rho[mu], Gb[mu], rho[mu], Psi[mu], nn * qr, T, nn * qr, st, &ar);
            src = T;
        }
        if (mu <= d - 2) {
            // out (kl*nn x kr) = src (kl*nn x qr) * V'_{mu+1} (column-major qr x kr)
            gemm_rm_cm(kl * nn, kr, qr, src, qr, Vk[mu + 1], qr, out[mu], kr, st, &ar);
        } else {
            copy_f64((int64_t)kl * nn, src, out[mu], st);
        }
        (void)mid;
    }
    TTSG_HIP(hipStreamSynchronize(st));
    ar.release(mark);
}

double tt_norm_orth(int d, const int* n, std::vector<int>& r, const std::vector<double*>& w, Arena& ar,
                    hipStream_t st) {
    const size_t mark = ar.mark();
    int64_t maxcore = 1, maxr = 1;
    for (int mu = 0; mu < d; ++mu) {
        maxcore = std::max<int64_t>(maxcore, (int64_t)r[mu] * n[mu] * r[mu + 1]);
        maxr = std::max<int64_t>(maxr, std::max(r[mu], r[mu + 1]));
    }
    double* A = ar.get<double>(maxcore);
    double* T = ar.get<double>(maxcore);
    double* Rm = ar.get<double>(maxr * maxr);
    double* tau = ar.get<double>(maxr);
    double* part = ar.get<double>(1024);
    double* scal = ar.get<double>(2);
    for (int mu = 0; mu <= d - 2; ++mu) {
        const int m = r[mu] * n[mu], c = r[mu + 1];
        transpose2d(m, c, w[mu], c, A, m, st);
        qr_householder(1, m, c, A, m, 0, tau, 0, st);
        const int k = std::min(m, c);
        qr_form_q(1, m, c, A, m, 0, tau, 0, T, m, 0, st);
        transpose2d(k, m, T, m, w[mu], k, st);   // row-major m x k
        extract_r(k, c, A, m, Rm, k, st);
        // W_{mu+1} (k x n2 r2) = R (k x c, column-major ld k) * W_{mu+1}
        const int n2 = n[mu + 1], r2 = r[mu + 2];
        ContractDesc dd = cdesc(k, n2 * r2, c);
        dd.am = idx1(1);
        dd.ak = idx1(k);
        dd.bk = idx1((int64_t)n2 * r2);
        dd.bn = idx1(1);
        dd.cm = idx1((int64_t)n2 * r2);
        dd.cn = idx1(1);
        contract(Prec::F64, dd, Rm, w[mu + 1], T, st, &ar);
        copy_f64((int64_t)k * n2 * r2, T, w[mu + 1], st);
        r[mu + 1] = k;
    }
    sumsq((int64_t)r[d - 1] * n[d - 1], w[d - 1], part, scal, st);
    double nrm = std::sqrt(read_scalar(scal, st));
    ar.release(mark);
    return nrm;
}

int take_rank_cap_events() {
    const int v = t_cap_events;
    t_cap_events = 0;
    return v;
}

}  // namespace ttsg
