// TT-GMRES (Alg. 2) on one GPU: Arnoldi with full modified Gram-Schmidt in
// TT format, every new vector rounded by TT-SVD, with the inexact-Arnoldi
// relaxation of the rounding tolerance (Sec. 2.3), the Hessenberg least-squares
// problem (eq. argmin2) reduced by Givens rotations, and the solution formed by
// sequential rounded sums.  It is the deterministic baseline the sketched
// method is compared with (Sec. 5.2); every TT operation runs in the library's
// kernels (matrix-core contractions, LDS factorizations) and the Givens
// reduction in a one-thread kernel.
//
// Step k (x_0 = 0, r_0 = b, beta = ||b||, v_1 = b / beta):
//   eta_k  = tol / max(||r_{k-1}|| / ||b||, tol),  theta_k = min(eta_k tol, max_round)
//   w      = Round(A v_k, theta_k)
//   for i = 1..k:  h_{i,k} = <w, v_i>,  w = Round(w - h_{i,k} v_i, theta_k)
//   h_{k+1,k} = ||w||,  v_{k+1} = w / h_{k+1,k}
//   ||r_k|| = |last entry of Q^T beta e_1| after the Givens rotations
// Stop when ||r_k|| <= tol ||b|| or h_{k+1,k} = 0; then x = Round(x + y_i v_i,
// final_tol) term by term.
#include <algorithm>
#include <cmath>

#include "tt_ops.h"

namespace ttsg {
namespace {

// Column k of the Hessenberg matrix (h[0..k+1]) is reduced by the previous
// rotations and a new one; R (column-major, ld) keeps the triangular part, g the
// rotated right-hand side; res[0] = |g[k+1]|.
__global__ void k_gmres_givens(int k, int ld, const double* __restrict__ h, double* __restrict__ Rm,
                               double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                               double* __restrict__ res) {
    if (threadIdx.x != 0) return;
    double* col = Rm + (int64_t)k * ld;
    for (int i = 0; i <= k + 1; ++i) col[i] = h[i];
    for (int j = 0; j < k; ++j) {
        const double a = col[j], b = col[j + 1];
        col[j] = cs[j] * a + sn[j] * b;
        col[j + 1] = -sn[j] * a + cs[j] * b;
    }
    const double a = col[k], b = col[k + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0;
    const double s = r > 0.0 ? b / r : 0.0;
    cs[k] = c;
    sn[k] = s;
    col[k] = r;
    col[k + 1] = 0.0;
    g[k + 1] = -s * g[k];
    g[k] = c * g[k];
    res[0] = fabs(g[k + 1]);
}

// y = R^{-1} g (k x k upper triangle, column-major); zero pivots give y_i = 0.
__global__ void k_gmres_backsub(int k, int ld, const double* __restrict__ Rm, const double* __restrict__ g,
                                double* __restrict__ y) {
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double a = g[i];
        for (int j = i + 1; j < k; ++j) a -= Rm[(int64_t)j * ld + i] * y[j];
        const double rii = Rm[(int64_t)i * ld + i];
        y[i] = rii != 0.0 ? a / rii : 0.0;
    }
}

__global__ void k_gmres_init_g(int len, double beta, double* __restrict__ g) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) g[i] = i == 0 ? beta : 0.0;
}

class Gmres {
  public:
    Gmres(const GmresInputs& in, hipStream_t st) : in_(in), st_(st) {}

    size_t workspace_bytes() {
        Arena ar;
        ar.measure();
        carve(ar);
        return ar.used() + scratch_bytes() + (16u << 20);
    }

    int run(double* const* x_out, int32_t* x_r, ttsg_sgmres_info* info, void* ws, size_t ws_bytes);

  private:
    const GmresInputs& in_;
    hipStream_t st_;
    std::vector<int> cap_r_;            // rank capacity per bond
    std::vector<int64_t> cap_, wcap_;   // core capacities: basis/x, and sums/products
    std::vector<std::vector<double*>> V_;
    std::vector<std::vector<int>> Vr_;
    std::vector<double*> wa_, wb_, xa_, xb_;
    double *hcol_ = nullptr, *Rg_ = nullptr, *cs_ = nullptr, *sn_ = nullptr, *g_ = nullptr, *res_ = nullptr,
           *y_ = nullptr;
    int ld_ = 0;
    Arena scratch_;

    size_t scratch_bytes() const {
        int64_t mx = 1;
        for (int mu = 0; mu < in_.d; ++mu) mx = std::max(mx, wcap_[mu]);
        std::vector<int> wr(in_.d + 1);
        for (int k = 0; k <= in_.d; ++k) wr[k] = std::max(in_.R[k], 2) * cap_r_[k];
        return (size_t)(8 * mx) * 8 + tt_svd_extra_bytes(in_.d, in_.n, wr.data()) + ((size_t)80 << 20);
    }

    void carve(Arena& ar) {
        const int d = in_.d;
        const int* n = in_.n;
        const int m = in_.maxit;
        cap_r_.assign(d + 1, 1);
        double left = 1.0;
        for (int b = 1; b < d; ++b) {
            left *= n[b - 1];
            double right = 1.0;
            for (int k = b; k < d; ++k) right *= n[k];
            double c = std::min(left, right);
            if (in_.maxrank > 0) c = std::min(c, (double)in_.maxrank);
            cap_r_[b] = (int)c;
        }
        int Rm = 2;
        for (int k = 0; k <= d; ++k) Rm = std::max(Rm, in_.R[k]);
        cap_.assign(d, 0);
        wcap_.assign(d, 0);
        for (int mu = 0; mu < d; ++mu) {
            cap_[mu] = (int64_t)cap_r_[mu] * n[mu] * cap_r_[mu + 1];
            const int64_t lb = mu == 0 ? 1 : (int64_t)Rm * cap_r_[mu];
            const int64_t rb = mu == d - 1 ? 1 : (int64_t)Rm * cap_r_[mu + 1];
            wcap_[mu] = lb * n[mu] * rb + 64;
        }
        V_.assign(m + 1, std::vector<double*>(d));
        Vr_.assign(m + 1, std::vector<int>(d + 1, 1));
        for (int i = 0; i <= m; ++i)
            for (int mu = 0; mu < d; ++mu) V_[i][mu] = ar.get<double>(cap_[mu]);
        wa_.assign(d, nullptr);
        wb_.assign(d, nullptr);
        xa_.assign(d, nullptr);
        xb_.assign(d, nullptr);
        for (int mu = 0; mu < d; ++mu) {
            wa_[mu] = ar.get<double>(wcap_[mu]);
            wb_[mu] = ar.get<double>(wcap_[mu]);
            xa_[mu] = ar.get<double>(wcap_[mu]);
            xb_[mu] = ar.get<double>(wcap_[mu]);
        }
        ld_ = m + 2;
        hcol_ = ar.get<double>(ld_ + 2);
        Rg_ = ar.get<double>((int64_t)ld_ * ld_);
        cs_ = ar.get<double>(ld_);
        sn_ = ar.get<double>(ld_);
        g_ = ar.get<double>(ld_ + 1);
        res_ = ar.get<double>(8);
        y_ = ar.get<double>(ld_);
    }

    double read(const double* dev) {
        double h = 0.0;
        return *static_cast<const double*>(read_back(dev, sizeof(double), &h, st_));
    }
    std::vector<const double*> cv(const std::vector<double*>& v) const {
        return std::vector<const double*>(v.begin(), v.end());
    }
    void copy_tt(const std::vector<int>& r, const std::vector<double*>& src, const std::vector<double*>& dst) {
        for (int mu = 0; mu < in_.d; ++mu)
            copy_f64((int64_t)r[mu] * in_.n[mu] * r[mu + 1], src[mu], dst[mu], st_);
    }
    // TT-SVD of `w` (ranks r, capacities wcap_) at relative tol with the rank cap
    double round(std::vector<int>& r, const std::vector<double*>& w, double tol) {
        return tt_svd_inplace(in_.d, in_.n, r, w, wcap_, tol, in_.maxrank, scratch_, st_, nullptr);
    }
};

int Gmres::run(double* const* x_out, int32_t* x_r, ttsg_sgmres_info* info, void* ws, size_t ws_bytes) {
    const int d = in_.d;
    const int* n = in_.n;
    Arena meas;
    meas.measure();
    carve(meas);
    const size_t fixed = meas.used();
    const size_t scr = scratch_bytes();
    Workspace wsp(ws, ws_bytes, fixed + scr + 4096, st_);
    carve(wsp.arena);
    scratch_.reset(wsp.arena.get<char>(scr), scr);
    const std::vector<int> R1(d + 1, 1);

    // ||b|| by orthogonalization of a copy; v_1 = b / ||b|| (x_0 = 0)
    std::vector<int> r = in_.rb;
    for (int mu = 0; mu < d; ++mu) TTSG_CHECK(r[mu + 1] <= cap_r_[mu + 1] || mu == d - 1, TTSG_ERR_CAPACITY,
                                              "tt_gmres: rank of b above the rank capacity");
    for (int mu = 0; mu < d; ++mu) copy_f64((int64_t)r[mu] * n[mu] * r[mu + 1], in_.b[mu], wa_[mu], st_);
    const double nb = tt_norm_orth(d, n, r, wa_, scratch_, st_);
    TTSG_CHECK(std::isfinite(nb), TTSG_ERR_NONFINITE, "tt_gmres: right-hand side is not finite");
    int status = TTSG_NOT_CONVERGED, k = 0;
    double res_rel = 1.0, hk = 0.0;
    std::vector<int> xr(d + 1, 1);
    if (nb == 0.0) {
        for (int mu = 0; mu < d; ++mu) fill(n[mu], 0.0, x_out[mu], st_);
        for (int b = 0; b <= d; ++b) x_r[b] = 1;
        TTSG_HIP(hipStreamSynchronize(st_));
        if (info) {
            info->iterations = 0;
            info->status = TTSG_OK;
            info->true_residual = 0.0;
        }
        return TTSG_OK;
    }
    // tt_norm_orth left-orthogonalized the copy (same tensor): v_1 = copy / ||b||
    Vr_[0] = r;
    copy_tt(r, wa_, V_[0]);
    scale_f64((int64_t)r[d - 1] * n[d - 1] * r[d], 1.0 / nb, V_[0][d - 1], st_);
    hipLaunchKernelGGL(k_gmres_init_g, dim3(1), dim3(64), 0, st_, ld_ + 1, nb, g_);
    TTSG_HIP(hipGetLastError());
    int max_rank = 0;
    double last_res = nb;
    for (k = 0; k < in_.maxit; ++k) {
        const double eta = in_.tol / std::max(res_rel, in_.tol);
        const double rt = std::min(eta * in_.tol, in_.max_round);
        // w = Round(A v_k, rt)
        std::vector<int> wr(d + 1);
        for (int b = 0; b <= d; ++b) wr[b] = in_.R[b] * Vr_[k][b];
        for (int mu = 0; mu < d; ++mu)
            matvec_core(Vr_[k][mu], n[mu], Vr_[k][mu + 1], in_.R[mu], in_.R[mu + 1], in_.A[mu], V_[k][mu], false,
                        wa_[mu], st_);
        double wn = round(wr, wa_, rt);
        // modified Gram-Schmidt, rounding after every step
        for (int i = 0; i <= k; ++i) {
            std::vector<const void*> wv(wa_.begin(), wa_.end()), vi(V_[i].begin(), V_[i].end());
            inner_run(Prec::F64, d, n, R1, {}, wr, wv, Vr_[i], vi, hcol_ + i, scratch_, st_);
            const double h = read(hcol_ + i);
            std::vector<int> sr;
            tt_add_block(d, n, wr, wa_, Vr_[i], cv(V_[i]), -h, wb_, sr, st_);
            wn = round(sr, wb_, rt);
            std::swap(wa_, wb_);
            wr = sr;
        }
        // h_{k+1,k} = ||w||: the norm of the last rounding's output
        hk = wn;
        TTSG_CHECK(std::isfinite(hk), TTSG_ERR_NONFINITE, "tt_gmres: non-finite basis vector");
        fill(1, hk, hcol_ + k + 1, st_);
        hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(64), 0, st_, k, ld_, hcol_, Rg_, cs_, sn_, g_, res_);
        TTSG_HIP(hipGetLastError());
        last_res = read(res_);
        res_rel = last_res / nb;
        int mr = 0;
        for (int b = 0; b <= d; ++b) mr = std::max(mr, wr[b]);
        max_rank = std::max(max_rank, mr);
        if (info && info->sketched_history) info->sketched_history[k] = res_rel;
        if (info && info->rank_history) info->rank_history[k] = mr;
        if (last_res <= nb * in_.tol || hk == 0.0) {
            ++k;
            status = hk == 0.0 ? TTSG_BREAKDOWN : TTSG_OK;
            break;
        }
        // v_{k+1} = w / h_{k+1,k}
        Vr_[k + 1] = wr;
        copy_tt(wr, wa_, V_[k + 1]);
        scale_f64((int64_t)wr[d - 1] * n[d - 1] * wr[d], 1.0 / hk, V_[k + 1][d - 1], st_);
    }
    const int kk = std::min(k, in_.maxit);
    // y from the triangular factor; x = Round(x + y_i v_i, final_tol) term by term
    hipLaunchKernelGGL(k_gmres_backsub, dim3(1), dim3(64), 0, st_, kk, ld_, Rg_, g_, y_);
    TTSG_HIP(hipGetLastError());
    std::vector<double> hy(std::max(kk, 1));
    TTSG_HIP(hipMemcpyAsync(hy.data(), y_, kk * sizeof(double), hipMemcpyDeviceToHost, st_));
    TTSG_HIP(hipStreamSynchronize(st_));
    xr = Vr_[0];
    copy_tt(xr, V_[0], xa_);
    scale_f64((int64_t)xr[0] * n[0] * xr[1], hy[0], xa_[0], st_);
    for (int i = 1; i < kk; ++i) {
        std::vector<int> sr;
        tt_add_block(d, n, xr, xa_, Vr_[i], cv(V_[i]), hy[i], xb_, sr, st_);
        round(sr, xb_, in_.final_tol);
        std::swap(xa_, xb_);
        xr = sr;
    }
    for (int mu = 0; mu < d; ++mu) {
        TTSG_CHECK(xr[mu + 1] <= cap_r_[mu + 1] || mu == d - 1, TTSG_ERR_CAPACITY, "tt_gmres: solution rank");
        copy_f64((int64_t)xr[mu] * n[mu] * xr[mu + 1], xa_[mu], x_out[mu], st_);
    }
    for (int b = 0; b <= d; ++b) x_r[b] = xr[b];
    // true residual ||b - A x|| / ||b||: block TT, norm by orthogonalization
    double tr = 0.0;
    {
        std::vector<int> gr(d + 1);
        for (int b = 0; b <= d; ++b) gr[b] = in_.R[b] * xr[b];
        for (int mu = 0; mu < d; ++mu)
            matvec_core(xr[mu], n[mu], xr[mu + 1], in_.R[mu], in_.R[mu + 1], in_.A[mu], xa_[mu], false, wa_[mu],
                        st_);
        std::vector<double*> bw(d);
        for (int mu = 0; mu < d; ++mu) bw[mu] = const_cast<double*>(in_.b[mu]);
        const size_t mk = scratch_.mark();
        std::vector<double*> rc(d);
        for (int mu = 0; mu < d; ++mu)
            rc[mu] = scratch_.get<double>((int64_t)(in_.rb[mu] + gr[mu]) * n[mu] * (in_.rb[mu + 1] + gr[mu + 1]));
        std::vector<int> rr;
        tt_add_block(d, n, in_.rb, bw, gr, cv(wa_), -1.0, rc, rr, st_);
        tr = tt_norm_orth(d, n, rr, rc, scratch_, st_) / nb;
        scratch_.release(mk);
    }
    TTSG_HIP(hipStreamSynchronize(st_));
    if (info) {
        info->iterations = kk;
        info->cycles = 1;
        info->max_rank = max_rank;
        info->status = status;
        info->true_residual = tr;
        info->true_residual_is_bound = 0;
        info->sketched_residual = last_res / nb;
    }
    return status;
}

}  // namespace

int tt_gmres_solve(const GmresInputs& in, double* const* x, int32_t* x_r, ttsg_sgmres_info* info, void* ws,
                   size_t ws_bytes, hipStream_t st) {
    Gmres g(in, st);
    return g.run(x, x_r, info, ws, ws_bytes);
}

size_t tt_gmres_workspace(const GmresInputs& in) {
    Gmres g(in, nullptr);
    return g.workspace_bytes();
}

}  // namespace ttsg
