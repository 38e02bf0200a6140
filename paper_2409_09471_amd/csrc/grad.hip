// Gradient contraction of a Kronecker-sum solve: for A(theta) = sum_k theta_k L_k
// (L_k acting on mode k) and the adjoint state lambda, dLoss/dtheta_k =
// -<lambda, L_k x>.  The left environments E_k = <lambda_{<k}, x_{<k}> and right
// environments F_k = <lambda_{>=k}, x_{>=k}> are formed once; each mode then
// needs only the local contraction of (lambda_k, L_k x_k) between E_k and F_{k+1}.
#include <algorithm>

#include "tt_ops.h"

namespace ttsg {

void grad_kron_sum(int d, const int* n, const std::vector<const double*>& L, const std::vector<int>& rl,
                   const std::vector<const double*>& lam, const std::vector<int>& rx,
                   const std::vector<const double*>& x, double* out_dev, Arena& ar, hipStream_t st) {
    const size_t mark = ar.mark();
    int64_t env = 1, tmp = 1, core = 1;
    for (int k = 0; k <= d; ++k) env = std::max<int64_t>(env, (int64_t)rl[k] * rx[k]);
    for (int k = 0; k < d; ++k) {
        tmp = std::max<int64_t>(tmp, (int64_t)std::max(rl[k], rx[k]) * n[k] * std::max(rx[k + 1], rl[k + 1]));
        core = std::max<int64_t>(core, (int64_t)rx[k] * n[k] * rx[k + 1]);
    }
    std::vector<double*> E(d + 1), F(d + 1);
    for (int k = 0; k <= d; ++k) {
        E[k] = ar.get<double>((int64_t)rl[k] * rx[k]);
        F[k] = ar.get<double>((int64_t)rl[k] * rx[k]);
    }
    double* T1 = ar.get<double>(tmp);
    double* T2 = ar.get<double>(tmp);
    double* Y = ar.get<double>(core);
    double* En = ar.get<double>(env);
    fill(1, 1.0, E[0], st);
    fill(1, 1.0, F[d], st);
    for (int k = 0; k < d; ++k) {
        LeftDims s{rx[k], n[k], rx[k + 1], 1, 1, rl[k], rl[k + 1]};
        left_step(Prec::F64, s, E[k], x[k], nullptr, lam[k], T1, T2, E[k + 1], st, &ar);
    }
    for (int k = d - 1; k >= 1; --k) {
        LeftDims s{rx[k], n[k], rx[k + 1], 1, 1, rl[k], rl[k + 1]};
        right_step(Prec::F64, s, F[k + 1], x[k], nullptr, lam[k], T1, T2, F[k], st, &ar);
    }
    for (int k = 0; k < d; ++k) {
        // Y = L_k applied to mode k of x_k  (a rank-1 operator core 1 x n x n x 1)
        matvec_core(rx[k], n[k], rx[k + 1], 1, 1, L[k], x[k], false, Y, st);
        LeftDims s{rx[k], n[k], rx[k + 1], 1, 1, rl[k], rl[k + 1]};
        left_step(Prec::F64, s, E[k], Y, nullptr, lam[k], T1, T2, En, st, &ar);
        // g_k = -sum_{p,b} En[p][b] F_{k+1}[b][p]
        ContractDesc dd = cdesc(1, 1, rl[k + 1] * rx[k + 1]);
        dd.alpha = -1.0;
        dd.am = idx1(0);
        dd.ak = idx1(1);
        dd.bk = idx2(rx[k + 1], rl[k + 1], 1);
        dd.bn = idx1(0);
        dd.cm = idx1(0);
        dd.cn = idx1(0);
        contract(Prec::F64, dd, En, F[k + 1], out_dev + k, st, nullptr);
    }
    ar.release(mark);
}

}  // namespace ttsg
