// Enhanced sketched TT-GMRES (Alg. 4) on one GPU.
//
// Per Krylov step k (x_0 = 0 or the previous cycle's solution):
//   w_k   = S (A v_k)                          Khatri-Rao sketch, A v_k never formed
//   h_ik  = <A v_k, v_i>, i in the last q      left environment sweeps
//   sketch(A v_k) by STTA, minus sum_i h_ik sketch(v_i)      streaming combination
//   v~    = TT-SVD(STTA_recover(.), round_tol, maxrank)       FP64 rounding
//   v_k+1 = v~ / ||v~||, its STTA sketch stored for the final solution
//   W = [W, w_k]: incremental CGS2 QR of W in FP64; ||W y - S r0|| is the norm
//   of the part of S r0 outside range(W) (the same quantity the pseudo-inverse
//   solution of eq. pseudo_inv leaves as residual).
// After the cycle: y from the triangular factor, x = STTA_recover(sum y_i
// sketch(v_i)) rounded at final_tol, then the FP64 true residual decides
// whether another cycle (restart from r0 = b - A x) is needed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>

#include "tt_ops.h"
#include "xlane.h"

namespace ttsg {
namespace {

constexpr int LS_THREADS = 1024;


__device__ double block_sum(double v, double* red) {
    v = wave_sum64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Append column k (W + k*s) to the CGS2 QR of W.  Q: s x maxit (column-major),
// Rm: maxit x maxit (column-major), c: Q^T S r0 entries, z: S r0 minus its
// projection onto range(Q).  res[0] = ||z||, res[1] = R[k][k].
__global__ __launch_bounds__(LS_THREADS) void k_ls_append(int s, int k, int ld, const double* __restrict__ W,
                                                           double* __restrict__ Q, double* __restrict__ Rm,
                                                           double* __restrict__ c, double* __restrict__ z,
                                                           double* __restrict__ res) {
    __shared__ double red[LS_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const double* w = W + (int64_t)k * s;
    double* qk = Q + (int64_t)k * s;
    double* rk = Rm + (int64_t)k * ld;
    for (int j = tid; j < s; j += blockDim.x) qk[j] = w[j];
    for (int i = tid; i <= k; i += blockDim.x) rk[i] = 0.0;
    __syncthreads();
    double wn = 0.0;
    for (int j = tid; j < s; j += blockDim.x) wn += w[j] * w[j];
    wn = sqrt(block_sum(wn, red));
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = wave; i < k; i += nw) {
            const double* qi = Q + (int64_t)i * s;
            double a = 0.0;
            for (int j = lane; j < s; j += 64) a += qi[j] * qk[j];
            a = wave_sum64(a);
            if (lane == 0) {
                rk[i] += a;
                res[2 + i] = a;  // this pass's coefficients
            }
        }
        __syncthreads();
        for (int j = tid; j < s; j += blockDim.x) {
            double a = qk[j];
            for (int i = 0; i < k; ++i) a -= Q[(int64_t)i * s + j] * res[2 + i];
            qk[j] = a;
        }
        __syncthreads();
    }
    double nn = 0.0;
    for (int j = tid; j < s; j += blockDim.x) nn += qk[j] * qk[j];
    nn = sqrt(block_sum(nn, red));
    const bool dep = !(nn > 1e-13 * wn);
    const double inv = dep ? 0.0 : 1.0 / nn;
    for (int j = tid; j < s; j += blockDim.x) qk[j] *= inv;
    __syncthreads();
    double ck = 0.0;
    for (int j = tid; j < s; j += blockDim.x) ck += qk[j] * z[j];
    ck = block_sum(ck, red);
    for (int j = tid; j < s; j += blockDim.x) z[j] -= ck * qk[j];
    __syncthreads();
    double zz = 0.0;
    for (int j = tid; j < s; j += blockDim.x) zz += z[j] * z[j];
    zz = block_sum(zz, red);
    if (tid == 0) {
        rk[k] = dep ? 0.0 : nn;
        c[k] = ck;
        res[0] = sqrt(zz);
        res[1] = dep ? 0.0 : nn;
    }
}

// y = R^{-1} c by back substitution (one wavefront); columns with R[i][i] = 0
// (dependent sketch columns) get y_i = 0.
__global__ void k_ls_solve(int k, int ld, const double* __restrict__ Rm, const double* __restrict__ c,
                           double* __restrict__ y) {
    const int lane = threadIdx.x;
    for (int i = k - 1; i >= 0; --i) {
        double a = 0.0;
        for (int j = i + 1 + lane; j < k; j += 64) a += Rm[(int64_t)j * ld + i] * y[j];
        a = wave_sum64(a);
        if (lane == 0) {
            const double rii = Rm[(int64_t)i * ld + i];
            y[i] = rii != 0.0 ? (c[i] - a) / rii : 0.0;
        }
        __syncthreads();
    }
}

// out[e] = sum_i y[i] * base[i * stride + e]
__global__ void k_gemv_cols(int64_t len, int k, int64_t stride, const double* __restrict__ base,
                            const double* __restrict__ y, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int i = 0; i < k; ++i) a += y[i] * base[(int64_t)i * stride + e];
        out[e] = a;
    }
}

__global__ void k_nonfinite(int64_t n, const double* __restrict__ x, int* __restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) *flag = 1;
}

// out[t] = sum_j part[t * zeta + j] in order (the window coefficients h_{i,k}
// of a preconditioned step are sums over the zeta terms of A P^{-1} v_k).
__global__ void k_sum_terms(int nw, int zeta, const double* __restrict__ part, double* __restrict__ out) {
    const int t = threadIdx.x;
    if (t < nw) {
        double a = 0.0;
        for (int j = 0; j < zeta; ++j) a += part[t * zeta + j];
        out[t] = a;
    }
}

// Whitened least squares (Sec. 3.4).  T is the triangular factor of the QR of
// S V (column-major, leading dimension ld; T(r, i) = T[i * ld + r]); the
// sketched Arnoldi relation gives S A V_k = Q_{k+1} (T_{k+1} H_k), so y solves
// min || T_{k+1} H_k y - beta e_1 || (eq. sketched_argmin2 with z = T_k y).
// T_{k+1} H_k is upper Hessenberg: it is reduced by Givens rotations one column
// per iteration, as in GMRES, and |g[k+1]| is the residual of
// eq. sketched_residualnorm.
__global__ void k_whiten_init(int len, const double* __restrict__ zz, double* __restrict__ g) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) g[i] = (i == 0) ? sqrt(zz[0]) : 0.0;
}

// Column k (0-based) of H: h[t] for basis indices k - nw + 1 + t (t < nw),
// h_{k+1,k} = hk (has_next = 0 after a breakdown: no row k + 1).
__global__ void k_whiten_step(int k, int ld, int nw, const double* __restrict__ T, const double* __restrict__ h,
                              double hk, int has_next, double* __restrict__ Gr, double* __restrict__ cs,
                              double* __restrict__ sn, double* __restrict__ g, double* __restrict__ res) {
    if (threadIdx.x != 0) return;
    double* col = Gr + (int64_t)k * ld;
    const int lo = k - nw + 1;
    double extra = 0.0;
    for (int r = 0; r <= k + 1; ++r) {
        double a = 0.0;
        for (int t = 0; t < nw; ++t) {
            const int i = lo + t;
            if (r <= i) a += T[(int64_t)i * ld + r] * h[t];
        }
        if (has_next) a += T[(int64_t)(k + 1) * ld + r] * hk;
        if (r <= k) col[r] = a;
        else extra = a;
    }
    for (int j = 0; j < k; ++j) {
        const double a = col[j], b = col[j + 1];
        col[j] = cs[j] * a + sn[j] * b;
        col[j + 1] = -sn[j] * a + cs[j] * b;
    }
    const double a = col[k], b = extra;
    const double rr = hypot(a, b);
    const double c = rr > 0.0 ? a / rr : 1.0, sg = rr > 0.0 ? b / rr : 0.0;
    cs[k] = c;
    sn[k] = sg;
    col[k] = rr;
    const double gk = g[k];
    g[k] = c * gk;
    g[k + 1] = -sg * gk;
    res[0] = fabs(g[k + 1]);
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

// Block core of a sum of two TTs (Sec. 2.2 addition): for mode mu of d,
//   first core [A B], last core [A; B], middle cores diag(A, B).
__global__ void k_block_core(int rl1, int rr1, int rl2, int rr2, int n, int first, int last,
                             const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ out,
                             double bscale, double ascale) {
    const int rl = first ? 1 : rl1 + rl2;
    const int rr = last ? 1 : rr1 + rr2;
    const int64_t total = (int64_t)rl * n * rr;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int b = (int)(e % rr);
        int64_t t = e / rr;
        int i = (int)(t % n);
        int a = (int)(t / n);
        double v = 0.0;
        // source block A occupies rows [0, rl1) and columns [0, rr1)
        int aa = a, bb = b;
        bool inA = (first || aa < rl1) && (last || bb < rr1);
        if (first && last) {
            v = ascale * A[i] + bscale * B[i];
        } else if (inA) {
            v = (first ? ascale : 1.0) * A[((int64_t)aa * n + i) * rr1 + bb];
        } else {
            int a2 = first ? 0 : aa - rl1;
            int b2 = last ? 0 : bb - rr1;
            bool inB = (first || (aa >= rl1)) && (last || (bb >= rr1));
            if (inB) v = (first ? bscale : 1.0) * B[((int64_t)a2 * n + i) * rr2 + b2];
        }
        out[e] = v;
    }
}

}  // namespace

// Sum a + bscale * b of two TTs into block cores `out` (ranks ra + rb).
void tt_add_block(int d, const int* n, const std::vector<int>& ra, const std::vector<double*>& a,
                  const std::vector<int>& rb, const std::vector<const double*>& b, double bscale,
                  const std::vector<double*>& out, std::vector<int>& rout, hipStream_t st, double ascale) {
    rout.assign(d + 1, 1);
    for (int k = 1; k < d; ++k) rout[k] = ra[k] + rb[k];
    for (int mu = 0; mu < d; ++mu) {
        const int first = (mu == 0), last = (mu == d - 1);
        int64_t total = (int64_t)rout[mu] * n[mu] * rout[mu + 1];
        hipLaunchKernelGGL(k_block_core, dim3(grid_for(total)), dim3(256), 0, st, ra[mu], ra[mu + 1], rb[mu],
                           rb[mu + 1], n[mu], first, last, a[mu], b[mu], out[mu], bscale, ascale);
    }
    TTSG_HIP(hipGetLastError());
}

// Side streams (non-blocking, default priority) and events of one solve.
// Sets are created on first use per device and kept for the process; a solve
// takes one from the pool and returns it after draining its streams, so
// concurrent solves (the batched entry point's workers) each hold their own.
struct StreamSet {
    int dev = -1;
    hipStream_t k = nullptr, h = nullptr, r = nullptr;
    hipEvent_t ev[9] = {};
};

std::mutex g_set_mu;
std::vector<StreamSet> g_sets;

StreamSet acquire_stream_set() {
    int dev = 0;
    TTSG_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_set_mu);
        for (size_t i = 0; i < g_sets.size(); ++i)
            if (g_sets[i].dev == dev) {
                StreamSet s = g_sets[i];
                g_sets.erase(g_sets.begin() + (ptrdiff_t)i);
                return s;
            }
    }
    StreamSet s;
    s.dev = dev;
    TTSG_HIP(hipStreamCreateWithFlags(&s.k, hipStreamNonBlocking));
    TTSG_HIP(hipStreamCreateWithFlags(&s.h, hipStreamNonBlocking));
    TTSG_HIP(hipStreamCreateWithFlags(&s.r, hipStreamNonBlocking));
    for (hipEvent_t& e : s.ev) TTSG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return s;
}

void release_stream_set(const StreamSet& s) {
    std::lock_guard<std::mutex> lk(g_set_mu);
    g_sets.push_back(s);
}

class SgmresSolver {
  public:
    SgmresSolver(const SolverInputs& in, hipStream_t st) : in_(in), st_(st) {}

    // Size of every buffer, computed with the same code that carves them.
    size_t workspace_bytes() {
        Arena ar;
        ar.measure();
        carve(ar);
        return ar.used() + 4 * scratch_bytes() + (64u << 20);
    }

    int run(double* const* x_out, int32_t* x_r, ttsg_sgmres_info* info, void* ws, size_t ws_bytes);

  private:
    using clock = std::chrono::steady_clock;
    const SolverInputs& in_;
    hipStream_t st_;
    Prec p_ = Prec::F64;
    int maxit_ = 0, m_ = 0, q_ = 1;
    int64_t sk_len_ = 0;               // doubles in one vector's sketch (all Psi then all Omega)
    std::vector<int64_t> psi_off_, om_off_;
    std::vector<int64_t> cap_;         // elements of one TT core at the rx capacities
    // buffers
    std::vector<std::vector<double*>> slots_;   // q + 2 TT buffers at capacity rx
    std::vector<std::vector<int>> slot_r_;
    std::vector<double*> SA64_;                 // S_mu A_mu precomputed
    std::vector<double*> S1_;                   // S_mu (no operator)
    std::vector<void*> SAp_, Sp_, Dp_, Xp_, Yp_;  // operands in the working precision
    std::vector<std::vector<void*>> slot_lp_;   // low-precision copies of the slots
    double* sketches_ = nullptr;                // (m + 1) x sk_len
    double* skA_ = nullptr;                     // sketch of A v_k
    double* skC_ = nullptr;                     // combination
    double* W_ = nullptr;
    double* Q_ = nullptr;
    double* Rls_ = nullptr;
    double* cls_ = nullptr;
    double* z_ = nullptr;
    double* lsres_ = nullptr;
    double* hco_ = nullptr;                     // [1, h_1..h_q]
    bool vanilla_ = false;                      // Alg. 3 final sums: every basis vector of the cycle kept
    std::vector<std::vector<double*>> basis_;   // (m + 1) TT buffers at capacity rx (vanilla only)
    std::vector<std::vector<int>> basis_r_;
    std::vector<double*> vacc_;                 // running sum of the vanilla solution (capacity rx)
    std::vector<double*> xbest_;                // iterate with the smallest true residual so far
    std::vector<int> xbest_r_;
    double* y_ = nullptr;
    double* xw_ = nullptr;                      // one more TT at 2x capacity for sums
    std::vector<double*> xsum_;
    std::vector<double*> xcur_;
    std::vector<int> xcur_r_;
    double* scal_ = nullptr;
    int* flag_ = nullptr;
    // preconditioner (Alg. 5): mode factors [zeta][n][n] per mode, the TT of
    // one term alpha_j (x)_k E_jk v, its sketches and partial coefficients
    bool pre_ = false;
    std::vector<double*> Eblk_;
    std::vector<double*> zbuf_;
    std::vector<void*> zlp_;
    double* skT_ = nullptr;
    double* wtmp_ = nullptr;
    double* htmp_ = nullptr;
    // whitened least squares (Sec. 3.4): S V, its CGS2 QR and the Givens
    // factorization of T H
    bool white_ = false;
    int ldw_ = 0;
    double* SV_ = nullptr;
    double* Q2_ = nullptr;
    double* T2_ = nullptr;
    double* c2_ = nullptr;
    double* z2_ = nullptr;
    double* res2_ = nullptr;
    double* Gr_ = nullptr;
    double* cs_ = nullptr;
    double* sn_ = nullptr;
    double* g_ = nullptr;
    Arena scratch_;    // main stream
    Arena scratchK_;   // side stream K: Khatri-Rao column + least squares
    Arena scratchH_;   // side stream H: sketch of v_k + coefficients h
    Arena scratchR_;   // side stream R: right sweep and Omega of the sketch of A v_k

    size_t scratch_bytes() const;
    void carve(Arena& ar);
    void to_lp(int slot);
    std::vector<const void*> slot_ops(int slot) const;
    void sketch_vec(int slot, double* out);
    double tt_norm_copy(const std::vector<int>& r, const std::vector<const double*>& c);
    double true_residual(const std::vector<int>& rx, const std::vector<double*>& x, double nb);
};

size_t SgmresSolver::scratch_bytes() const {
    // generous bound for the sweep and rounding scratch: a few multiples of
    // the largest intermediate of the STTA/KR sweeps and of a doubled TT
    const int d = in_.d;
    int64_t big = 1;
    int Rm = 1;
    for (int k = 0; k <= d; ++k) Rm = std::max(Rm, in_.R[k]);
    for (int mu = 0; mu < d; ++mu) {
        const int64_t nn = in_.n[mu];
        const int64_t rl = in_.rx[mu], rr = in_.rx[mu + 1];
        const int64_t rhol = in_.rho[mu];
        big = std::max<int64_t>(big, rhol * Rm * nn * rr * Rm);
        big = std::max<int64_t>(big, rl * nn * Rm * std::max<int64_t>(rr, in_.rho[mu + 1]) * Rm);
        big = std::max<int64_t>(big, (int64_t)in_.s * Rm * rl * nn);
        big = std::max<int64_t>(big, (rl * Rm + in_.rb[mu] + rl) * nn * (rr * Rm + in_.rb[mu + 1] + rr));
    }
    // + the kept intermediates of the two-stream STTA sketch (every mode's T2
    // and left environment at the slot capacities)
    int64_t kept = 0;
    for (int mu = 0; mu < d; ++mu)
        kept += (int64_t)in_.rho[mu] * in_.n[mu] * Rm * in_.rx[mu + 1] + (int64_t)in_.rho[mu] * Rm * in_.rx[mu] + 64;
    return (size_t)(12 * big + 8 * (int64_t)in_.s * Rm * 512 + kept) * 8;
}

void SgmresSolver::carve(Arena& ar) {
    const int d = in_.d;
    const ttsg_sgmres_opts& o = in_.o;
    p_ = o.precision == TTSG_PREC_F64 ? Prec::F64 : (o.precision == TTSG_PREC_MIXED ? Prec::F32 : Prec::BF16);
    maxit_ = o.maxit;
    m_ = o.restart > 0 ? std::min(o.restart, o.maxit) : o.maxit;
    q_ = std::max(1, o.q);
    cap_.assign(d, 0);
    for (int mu = 0; mu < d; ++mu) cap_[mu] = (int64_t)in_.rx[mu] * in_.n[mu] * in_.rx[mu + 1];
    psi_off_.assign(d, 0);
    om_off_.assign(d, 0);
    sk_len_ = 0;
    for (int mu = 0; mu < d; ++mu) {
        psi_off_[mu] = sk_len_;
        sk_len_ += (int64_t)in_.rho[mu] * in_.n[mu] * in_.rx[mu + 1];
    }
    for (int b = 1; b < d; ++b) {
        om_off_[b] = sk_len_;
        sk_len_ += (int64_t)in_.rho[b] * in_.rx[b];
    }
    const int nslots = q_ + 2;
    slots_.assign(nslots, std::vector<double*>(d));
    slot_r_.assign(nslots, std::vector<int>(d + 1, 1));
    for (int sl = 0; sl < nslots; ++sl)
        for (int mu = 0; mu < d; ++mu) slots_[sl][mu] = ar.get<double>(cap_[mu]);
    const size_t es = elem_size(p_);
    slot_lp_.assign(nslots, std::vector<void*>(d, nullptr));
    if (p_ != Prec::F64)
        for (int sl = 0; sl < nslots; ++sl)
            for (int mu = 0; mu < d; ++mu) slot_lp_[sl][mu] = ar.get<char>(cap_[mu] * es);
    SA64_.assign(d, nullptr);
    S1_.assign(d, nullptr);
    SAp_.assign(d, nullptr);
    Sp_.assign(d, nullptr);
    Dp_.assign(d, nullptr);
    for (int mu = 0; mu < d; ++mu) {
        const int64_t nn = in_.n[mu];
        SA64_[mu] = ar.get<double>((int64_t)in_.s * in_.R[mu] * nn * in_.R[mu + 1]);
        if (p_ != Prec::F64) {
            SAp_[mu] = ar.get<char>((int64_t)in_.s * in_.R[mu] * nn * in_.R[mu + 1] * es);
            Sp_[mu] = ar.get<char>((int64_t)in_.s * nn * es);
            Dp_[mu] = ar.get<char>((int64_t)in_.R[mu] * nn * nn * in_.R[mu + 1] * es);
        }
    }
    Xp_.assign(d - 1, nullptr);
    Yp_.assign(d - 1, nullptr);
    if (p_ != Prec::F64) {
        for (int k = 0; k < d - 1; ++k) {
            Yp_[k] = ar.get<char>((int64_t)in_.rho[k] * in_.n[k] * in_.rho[k + 1] * es);
            Xp_[k] = ar.get<char>((int64_t)in_.rx[k + 1] * in_.n[k + 1] * in_.rx[k + 2] * es);
        }
    }
    sketches_ = ar.get<double>((int64_t)(m_ + 1) * sk_len_);
    skA_ = ar.get<double>(sk_len_);
    skC_ = ar.get<double>(sk_len_);
    W_ = ar.get<double>((int64_t)in_.s * (m_ + 1));
    Q_ = ar.get<double>((int64_t)in_.s * (m_ + 1));
    Rls_ = ar.get<double>((int64_t)(m_ + 1) * (m_ + 1));
    cls_ = ar.get<double>(m_ + 1);
    z_ = ar.get<double>(in_.s);
    lsres_ = ar.get<double>(std::max(m_ + 8, 1024));
    hco_ = ar.get<double>(16);
    y_ = ar.get<double>(m_ + 1);
    xsum_.assign(d, nullptr);
    xcur_.assign(d, nullptr);
    for (int mu = 0; mu < d; ++mu) {
        xsum_[mu] = ar.get<double>(4 * cap_[mu] + 64);
        xcur_[mu] = ar.get<double>(cap_[mu]);
    }
    scal_ = ar.get<double>(8);
    flag_ = ar.get<int>(8);
    xbest_.assign(d, nullptr);
    for (int mu = 0; mu < d; ++mu) xbest_[mu] = ar.get<double>(cap_[mu]);
    vanilla_ = in_.variant == TTSG_VARIANT_VANILLA;
    basis_.clear();
    basis_r_.clear();
    vacc_.assign(d, nullptr);
    if (vanilla_) {
        basis_.assign(m_ + 1, std::vector<double*>(d));
        basis_r_.assign(m_ + 1, std::vector<int>(d + 1, 1));
        for (int i = 0; i <= m_; ++i)
            for (int mu = 0; mu < d; ++mu) basis_[i][mu] = ar.get<double>(cap_[mu]);
        for (int mu = 0; mu < d; ++mu) vacc_[mu] = ar.get<double>(cap_[mu]);
    }
    pre_ = in_.zeta > 0;
    white_ = in_.ls_mode == TTSG_LS_WHITEN;
    Eblk_.assign(d, nullptr);
    zbuf_.assign(d, nullptr);
    zlp_.assign(d, nullptr);
    if (pre_) {
        for (int mu = 0; mu < d; ++mu) {
            Eblk_[mu] = ar.get<double>((int64_t)in_.zeta * in_.n[mu] * in_.n[mu]);
            zbuf_[mu] = ar.get<double>(cap_[mu]);
            if (p_ != Prec::F64) zlp_[mu] = ar.get<char>(cap_[mu] * es);
        }
        skT_ = ar.get<double>(sk_len_);
        wtmp_ = ar.get<double>(in_.s);
        htmp_ = ar.get<double>((int64_t)q_ * in_.zeta + 8);
    }
    if (white_) {
        ldw_ = m_ + 2;
        SV_ = ar.get<double>((int64_t)in_.s * ldw_);
        Q2_ = ar.get<double>((int64_t)in_.s * ldw_);
        T2_ = ar.get<double>((int64_t)ldw_ * ldw_);
        c2_ = ar.get<double>(ldw_);
        z2_ = ar.get<double>(in_.s);
        res2_ = ar.get<double>(ldw_ + 8);
        Gr_ = ar.get<double>((int64_t)ldw_ * ldw_);
        cs_ = ar.get<double>(ldw_);
        sn_ = ar.get<double>(ldw_);
        g_ = ar.get<double>(ldw_ + 1);
    }
}

}  // namespace ttsg

namespace ttsg {

void SgmresSolver::to_lp(int slot) {
    if (p_ == Prec::F64) return;
    for (int mu = 0; mu < in_.d; ++mu) {
        const std::vector<int>& r = slot_r_[slot];
        convert_f64_f32((int64_t)r[mu] * in_.n[mu] * r[mu + 1], slots_[slot][mu],
                        static_cast<float*>(slot_lp_[slot][mu]), st_);
    }
}

std::vector<const void*> SgmresSolver::slot_ops(int slot) const {
    std::vector<const void*> v(in_.d);
    for (int mu = 0; mu < in_.d; ++mu)
        v[mu] = p_ == Prec::F64 ? static_cast<const void*>(slots_[slot][mu]) : slot_lp_[slot][mu];
    return v;
}

double SgmresSolver::tt_norm_copy(const std::vector<int>& r, const std::vector<const double*>& c) {
    const size_t mark = scratch_.mark();
    std::vector<double*> w(in_.d);
    for (int mu = 0; mu < in_.d; ++mu) {
        const int64_t e = (int64_t)r[mu] * in_.n[mu] * r[mu + 1];
        w[mu] = scratch_.get<double>(e);
        copy_f64(e, c[mu], w[mu], st_);
    }
    std::vector<int> rr = r;
    double nrm = tt_norm_orth(in_.d, in_.n, rr, w, scratch_, st_);
    scratch_.release(mark);
    return nrm;
}

int sgmres_run_impl(SgmresSolver& s, double* const* x_out, int32_t* x_r, ttsg_sgmres_info* info, void* ws,
                    size_t ws_bytes) {
    return s.run(x_out, x_r, info, ws, ws_bytes);
}

int SgmresSolver::run(double* const* x_out, int32_t* x_r, ttsg_sgmres_info* info, void* ws, size_t ws_bytes) {
    const int d = in_.d;
    const int* n = in_.n;
    const ttsg_sgmres_opts& o = in_.o;
    const int s = in_.s;
    Arena meas;
    meas.measure();
    carve(meas);
    const size_t fixed = meas.used();
    const size_t scr = scratch_bytes();
    Workspace wsp(ws, ws_bytes, fixed + 4 * scr + 4 * 4096, st_);
    carve(wsp.arena);
    scratch_.reset(wsp.arena.get<char>(scr), scr);
    scratchK_.reset(wsp.arena.get<char>(scr), scr);
    scratchH_.reset(wsp.arena.get<char>(scr), scr);
    scratchR_.reset(wsp.arena.get<char>(scr), scr);

    // Within an iteration the Khatri-Rao column of A v_k (with the least-squares
    // update) and the sketch of v_k plus the coefficients h do not depend on the
    // STTA sketch of A v_k: they run on two side streams (default priority)
    // while the main stream sketches A v_k, each with its own scratch.
    // The STTA sketch of A v_k itself runs on two streams: its right sweep and
    // Omega sketches on side stream R, its left sweep and Psi sketches here.
    // With single_stream the three are the caller's stream itself: the events
    // then order nothing that program order does not already order.
    // The streams and events come from a per-process pool (created once per
    // device and reused by later solves) instead of being created and
    // destroyed by every solve.
    struct SideStreams {
        StreamSet set;
        hipStream_t k = nullptr, h = nullptr, r = nullptr;
        hipEvent_t v = nullptr, hd = nullptr;
        hipEvent_t zr = nullptr, kd = nullptr;   // a preconditioner term is in place / read by stream K
        hipEvent_t hz = nullptr;                 // ... / read by stream H
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        bool held = false;
        ~SideStreams() {
            if (!held) return;
            // every side stream drained before the set (and this solve's
            // workspace) can be used again
            (void)hipStreamSynchronize(k);
            (void)hipStreamSynchronize(h);
            (void)hipStreamSynchronize(r);
            release_stream_set(set);
        }
    } side;
    side.set = acquire_stream_set();
    side.held = true;
    if (in_.single_stream) {
        side.k = side.h = side.r = st_;
    } else {
        side.k = side.set.k;
        side.h = side.set.h;
        side.r = side.set.r;
    }
    side.v = side.set.ev[0];
    side.hd = side.set.ev[1];
    side.zr = side.set.ev[2];
    side.kd = side.set.ev[3];
    side.hz = side.set.ev[4];
    for (int i = 0; i < 4; ++i) side.ev[i] = side.set.ev[5 + i];
    TTSG_HIP(hipEventRecord(side.kd, side.k));
    TTSG_HIP(hipEventRecord(side.hz, side.h));
    SketchSide sk_side;
    sk_side.st = side.r;
    sk_side.ar = &scratchR_;
    sk_side.in = side.ev[0];
    sk_side.right = side.ev[1];
    sk_side.left = side.ev[2];
    sk_side.done = side.ev[3];

    const bool timing = info && info->phase_seconds;
    auto now = [&]() {
        if (timing) {
            TTSG_HIP(hipStreamSynchronize(st_));
            TTSG_HIP(hipStreamSynchronize(side.k));
            TTSG_HIP(hipStreamSynchronize(side.h));
            TTSG_HIP(hipStreamSynchronize(side.r));
        }
        return clock::now();
    };
    auto add_phase = [&](int ph, clock::time_point t0) {
        if (timing) info->phase_seconds[ph] += std::chrono::duration<double>(now() - t0).count();
    };
    if (timing)
        for (int i = 0; i < 8; ++i) info->phase_seconds[i] = 0.0;

    // ---- operands --------------------------------------------------------
    std::vector<int> R1(d + 1, 1);
    for (int mu = 0; mu < d; ++mu) {
        kr_precompute(Prec::F64, s, n[mu], in_.R[mu], in_.R[mu + 1], in_.S[mu], in_.A[mu], SA64_[mu], st_);
    }
    std::vector<const void*> Dv(d), SAv(d), Sv(d), Xv(d - 1), Yv(d - 1);
    for (int mu = 0; mu < d; ++mu) {
        const int64_t nn = n[mu];
        if (p_ == Prec::F64) {
            Dv[mu] = in_.A[mu];
            SAv[mu] = SA64_[mu];
            Sv[mu] = in_.S[mu];
        } else {
            convert_f64_f32((int64_t)in_.R[mu] * nn * nn * in_.R[mu + 1], in_.A[mu], (float*)Dp_[mu], st_);
            convert_f64_f32((int64_t)s * in_.R[mu] * nn * in_.R[mu + 1], SA64_[mu], (float*)SAp_[mu], st_);
            convert_f64_f32((int64_t)s * nn, in_.S[mu], (float*)Sp_[mu], st_);
            Dv[mu] = Dp_[mu];
            SAv[mu] = SAp_[mu];
            Sv[mu] = Sp_[mu];
        }
    }
    for (int k = 0; k < d - 1; ++k) {
        if (p_ == Prec::F64) {
            Yv[k] = in_.Y[k];
            Xv[k] = in_.X[k];
        } else {
            convert_f64_f32((int64_t)in_.rho[k] * n[k] * in_.rho[k + 1], in_.Y[k], (float*)Yp_[k], st_);
            convert_f64_f32((int64_t)in_.rx[k + 1] * n[k + 1] * in_.rx[k + 2], in_.X[k], (float*)Xp_[k], st_);
            Yv[k] = Yp_[k];
            Xv[k] = Xp_[k];
        }
    }
    // Preconditioner (Alg. 5): the factors E_jk = exp(-beta_j M_k), once per solve
    if (pre_) mode_exponentials(in_.zeta, in_.beta.data(), d, n, in_.M, Eblk_, scratch_, st_);
    auto Eterm = [&](int j) {
        std::vector<const double*> e(d);
        for (int mu = 0; mu < d; ++mu) e[mu] = Eblk_[mu] + (int64_t)j * n[mu] * n[mu];
        return e;
    };
    // Precision map: the Khatri-Rao column w_k, S r0, ||S b|| and the stored
    // STTA sketches of the basis vectors (which build the final solution) are
    // FP64; the STTA sketch of A v_k and the coefficients h (which only shape
    // the next basis vector) run in the working precision p_.
    SketchOperands so_op, so_plain;
    so_op.p = p_;
    so_plain.p = Prec::F64;
    so_op.n = so_plain.n = n;
    so_op.d = so_plain.d = d;
    so_op.rho = so_plain.rho = in_.rho;
    so_op.rx = so_plain.rx = in_.rx;
    so_op.Y = Yv;
    so_op.X = Xv;
    so_plain.Y.assign(in_.Y.begin(), in_.Y.end());
    so_plain.X.assign(in_.X.begin(), in_.X.end());
    so_op.R = in_.R;
    so_op.D = Dv;
    so_plain.R = R1;
    // zero and identity blocks of the operator cores (exact; the float32
    // copies keep them) are copied or skipped in the operator steps
    const std::vector<std::vector<uint8_t>> blocks =
        operator_blocks(d, n, in_.R, std::vector<const void*>(in_.A.begin(), in_.A.end()), st_, scratchR_);
    const std::vector<const uint8_t*> blk = block_ptrs(blocks);
    so_op.blk = blk;
    // FP64 sketches of A x for the restart residual
    SketchOperands so_op64 = so_plain;
    so_op64.R = in_.R;
    so_op64.D.assign(in_.A.begin(), in_.A.end());
    so_op64.blk = blk;

    auto sk_ptrs = [&](double* base, std::vector<double*>& psi, std::vector<double*>& om) {
        psi.assign(d, nullptr);
        om.assign(std::max(d - 1, 1), nullptr);
        for (int mu = 0; mu < d; ++mu) psi[mu] = base + psi_off_[mu];
        for (int b = 1; b < d; ++b) om[b - 1] = base + om_off_[b];
    };
    auto sketch_slot = [&](int slot, double* out, Arena& ar, hipStream_t stream) {
        std::vector<double*> psi, om;
        sk_ptrs(out, psi, om);
        std::vector<const void*> c64(slots_[slot].begin(), slots_[slot].end());
        stta_sketch(so_plain, slot_r_[slot], c64, psi.data(), om.data(), ar, stream);
    };
    auto read = [&](const double* dev) {
        double h = 0.0;
        return *static_cast<const double*>(read_back(dev, sizeof(double), &h, st_));
    };
    auto cvec = [](const std::vector<double*>& v) { return std::vector<const double*>(v.begin(), v.end()); };

    // ---- norms of b and S b ----------------------------------------------
    const double nb = tt_norm_copy(in_.rb, in_.b);
    TTSG_CHECK(std::isfinite(nb), TTSG_ERR_NONFINITE, "right-hand side is not finite");
    if (nb == 0.0) {
        for (int mu = 0; mu < d; ++mu) fill(n[mu], 0.0, x_out[mu], st_);
        for (int k = 0; k <= d; ++k) x_r[k] = 1;
        TTSG_HIP(hipStreamSynchronize(st_));
        if (info) {
            info->iterations = 0;
            info->cycles = 0;
            info->true_residual = 0.0;
            info->true_residual_is_bound = 0;
            info->status = TTSG_OK;
        }
        return TTSG_OK;
    }
    std::vector<const void*> bops(d);
    std::vector<void*> b_lp(d, nullptr);
    {
        const size_t mk = scratch_.mark();
        if (p_ != Prec::F64) {
            for (int mu = 0; mu < d; ++mu) {
                const int64_t e = (int64_t)in_.rb[mu] * n[mu] * in_.rb[mu + 1];
                b_lp[mu] = scratch_.get<float>(e);
                convert_f64_f32(e, in_.b[mu], (float*)b_lp[mu], st_);
                bops[mu] = b_lp[mu];
            }
        } else {
            for (int mu = 0; mu < d; ++mu) bops[mu] = in_.b[mu];
        }
        std::vector<const void*> b64(in_.b.begin(), in_.b.end()), S64(in_.S.begin(), in_.S.end());
        kr_sketch_run(Prec::F64, d, n, s, R1, S64, in_.rb, b64, z_, scratch_, st_);
        sumsq(s, z_, lsres_, scal_, st_);
        scratch_.release(mk);
    }
    const double Sb = std::sqrt(read(scal_));

    // ---- buffer for A x (true residual) -------------------------------------
    std::vector<double*> G(d);
    for (int mu = 0; mu < d; ++mu) {
        const int64_t gl = (int64_t)in_.R[mu] * in_.rx[mu], gr = (int64_t)in_.R[mu + 1] * in_.rx[mu + 1];
        G[mu] = scratch_.get<double>(gl * n[mu] * gr);
    }
    bool true_is_bound = false;
    auto true_res = [&](const std::vector<int>& xr, const std::vector<double*>& xc) -> double {
        // ||b - A x||^2 = ||b||^2 - 2 <A x, b> + ||A x||^2  (FP64 throughout)
        std::vector<int> gr(d + 1);
        for (int k = 0; k <= d; ++k) gr[k] = in_.R[k] * xr[k];
        for (int mu = 0; mu < d; ++mu)
            matvec_core(xr[mu], n[mu], xr[mu + 1], in_.R[mu], in_.R[mu + 1], in_.A[mu], xc[mu], false, G[mu], st_);
        std::vector<const void*> gv(G.begin(), G.end()), bv(in_.b.begin(), in_.b.end());
        inner_run(Prec::F64, d, n, R1, {}, gr, gv, in_.rb, bv, scal_ + 1, scratch_, st_);
        inner_run(Prec::F64, d, n, R1, {}, gr, gv, gr, gv, scal_ + 2, scratch_, st_);
        double hbuf[2];
        const double* hb = static_cast<const double*>(read_back(scal_ + 1, 2 * sizeof(double), hbuf, st_));
        const double r2 = nb * nb - 2.0 * hb[0] + hb[1];
        // The three terms cancel: below about 64 eps (||b||^2 + ||A x||^2) the
        // difference is rounding, not residual.  Then r = b - A x is formed as
        // a block TT and measured by orthogonalization, which does not cancel.
        const double noise2 = 64.0 * 2.220446049250313e-16 * (nb * nb + hb[1]);
        true_is_bound = false;
        if (r2 > noise2) return std::sqrt(r2) / nb;
        // Below the floor: when the floor itself is within tol the residual is
        // known to meet it; the floor is reported as an upper bound (forming
        // b - A x explicitly costs a QR sweep at ranks R r_x + r_b)
        const double floor_rel = std::sqrt(std::max(r2, 0.0) + noise2) / nb;
        if (floor_rel <= o.tol) {
            true_is_bound = true;
            return floor_rel;
        }
        const size_t mk = scratch_.mark();
        std::vector<double*> rc(d);
        for (int mu = 0; mu < d; ++mu)
            rc[mu] = scratch_.get<double>((int64_t)(in_.rb[mu] + gr[mu]) * n[mu] * (in_.rb[mu + 1] + gr[mu + 1]));
        std::vector<double*> bw(d);
        for (int mu = 0; mu < d; ++mu) bw[mu] = const_cast<double*>(in_.b[mu]);   // read only
        std::vector<const double*> gc(G.begin(), G.end());
        std::vector<int> rr;
        tt_add_block(d, n, in_.rb, bw, gr, gc, -1.0, rc, rr, st_);
        const double nr = tt_norm_orth(d, n, rr, rc, scratch_, st_);
        scratch_.release(mk);
        return nr / nb;
    };

    // One preconditioned step (Alg. 5): the Khatri-Rao column, the window
    // coefficients h_{i,k} and the STTA sketch of A P^{-1} v_k, each a sum over
    // the zeta terms alpha_j A ((x)_k E_jk v_k) in term order; the sketch of
    // v_k itself (kept for the final solution) runs on stream H meanwhile.
    // The combination with the window sketches follows as in Alg. 4.
    // Arithmetic of this step's sketch of A v_k and coefficients h.  In the
    // bfloat16 mode the float32 form runs until the sketched residual is below
    // tol / (4 u_bf16): the perturbation of A v_k that a Krylov step tolerates
    // grows like tol / (relative residual) (inexact Arnoldi, Sec. 2.3), and a
    // bfloat16 sketch perturbs the new direction by about its unit roundoff.
    Prec pk_cur = p_;
    auto precond_step = [&](int k, int vk, const std::vector<int>& window) {
        const int nw = (int)window.size();
        TTSG_HIP(hipStreamWaitEvent(side.h, side.v, 0));
        sketch_slot(vk, sketches_ + (int64_t)k * sk_len_, scratchH_, side.h);
        fill(1, 1.0, hco_, side.h);
        TTSG_HIP(hipEventRecord(side.hd, side.h));
        std::vector<const void*> z64(zbuf_.begin(), zbuf_.end());
        std::vector<const void*> zop(d);
        for (int mu = 0; mu < d; ++mu) zop[mu] = p_ == Prec::F64 ? static_cast<const void*>(zbuf_[mu]) : zlp_[mu];
        std::vector<double*> pa, oa, pt, ot;
        sk_ptrs(skA_, pa, oa);
        sk_ptrs(skT_, pt, ot);
        std::vector<const void*> SA64(SA64_.begin(), SA64_.end());
        double* wcol = W_ + (int64_t)k * s;
        for (int j = 0; j < in_.zeta; ++j) {
            // the term's mode products overwrite the previous term (of this or
            // the previous step), which streams K and H may still be reading
            if (!white_) TTSG_HIP(hipStreamWaitEvent(st_, side.kd, 0));
            TTSG_HIP(hipStreamWaitEvent(st_, side.hz, 0));
            mode_product_tt(d, n, slot_r_[vk], cvec(slots_[vk]), Eterm(j), in_.alpha[j], zbuf_, st_, &scratch_);
            if (p_ != Prec::F64)
                for (int mu = 0; mu < d; ++mu)
                    convert_f64_f32((int64_t)slot_r_[vk][mu] * n[mu] * slot_r_[vk][mu + 1], zbuf_[mu],
                                    static_cast<float*>(zlp_[mu]), st_);
            TTSG_HIP(hipEventRecord(side.zr, st_));
            if (!white_) {
                // (stream K) the term's Khatri-Rao column, summed into W's column
                // in term order, while this stream sketches the same term
                TTSG_HIP(hipStreamWaitEvent(side.k, side.zr, 0));
                kr_sketch_run(Prec::F64, d, n, s, in_.R, SA64, slot_r_[vk], z64, j == 0 ? wcol : wtmp_, scratchK_,
                              side.k);
                if (j > 0) axpby(s, 1.0, wtmp_, 1.0, wcol, side.k);
                TTSG_HIP(hipEventRecord(side.kd, side.k));
            }
            // (stream H) the term's coefficients against the window
            TTSG_HIP(hipStreamWaitEvent(side.h, side.zr, 0));
            for (int t = 0; t < nw; ++t)
                inner_run(pk_cur, d, n, in_.R, Dv, slot_r_[vk], zop, slot_r_[window[t]], slot_ops(window[t]),
                          htmp_ + t * in_.zeta + j, scratchH_, side.h, blk);
            TTSG_HIP(hipEventRecord(side.hz, side.h));
            stta_sketch(so_op, slot_r_[vk], zop, (j == 0 ? pa : pt).data(), (j == 0 ? oa : ot).data(), scratch_, st_,
                        &sk_side);
            if (j > 0) axpby(sk_len_, 1.0, skT_, 1.0, skA_, st_);
        }
        TTSG_HIP(hipStreamWaitEvent(st_, side.hz, 0));
        hipLaunchKernelGGL(k_sum_terms, dim3(1), dim3(64), 0, st_, nw, in_.zeta, htmp_, hco_ + 1);
        TTSG_HIP(hipGetLastError());
        if (!white_) {
            hipLaunchKernelGGL(k_ls_append, dim3(1), dim3(LS_THREADS), 0, side.k, s, k, m_ + 1, W_, Q_, Rls_, cls_,
                               z_, lsres_);
            TTSG_HIP(hipGetLastError());
        }
        TTSG_HIP(hipStreamWaitEvent(st_, side.hd, 0));
        std::vector<const double*> xs(1 + nw);
        std::vector<double> sg(1 + nw, -1.0);
        xs[0] = skA_;
        sg[0] = 1.0;
        for (int t = 0; t < nw; ++t) xs[1 + t] = sketches_ + (int64_t)(k - nw + 1 + t) * sk_len_;
        lin_comb_dev(sk_len_, 1 + nw, xs.data(), hco_, sg.data(), skC_, st_);
    };

    // ---- cycles ------------------------------------------------------------
    int total = 0, cycles = 0, status = TTSG_NOT_CONVERGED, max_rank = 0, cap_events = 0;
    bool have_x = false;
    if (!in_.x0_r.empty()) {
        // initial guess: the first cycle starts from r0 = b - A x0, like a restart
        for (int mu = 0; mu < d; ++mu)
            copy_f64((int64_t)in_.x0_r[mu] * n[mu] * in_.x0_r[mu + 1], in_.x0[mu], xcur_[mu], st_);
        xcur_r_ = in_.x0_r;
        have_x = true;
    }
    double last_sres = 1.0, last_true = 1.0, best_true = INFINITY;
    bool best_is_bound = false;
    const int max_cycles = o.max_cycles > 0 ? o.max_cycles : 50;
    const double final_tol = o.final_tol > 0.0 ? o.final_tol : o.round_tol;
    const double stop = o.stop_safety * o.tol * Sb;
    const int nslots = q_ + 2;
    std::vector<int> window;
    while (total < maxit_ && cycles < max_cycles) {
        ++cycles;
        auto t0 = now();
        // r0 into slot 0
        window.clear();
        const int s0 = 0;
        double beta;
        if (!have_x) {
            slot_r_[s0] = in_.rb;
            for (int mu = 0; mu < d; ++mu)
                copy_f64((int64_t)in_.rb[mu] * n[mu] * in_.rb[mu + 1], in_.b[mu], slots_[s0][mu], st_);
            beta = tt_norm_copy(slot_r_[s0], cvec(slots_[s0]));
        } else {
            // r0 = b - A x by the method's randomized rounding: FP64 STTA
            // sketches of b and of A x (operator fused, A x never formed) are
            // subtracted, recovered at the STTA ranks and recompressed by TT-SVD
            // at 1e-12 -- instead of a TT-SVD of the rank R r_x + r_b block sum.
            {
                std::vector<double*> pb, ob, pa, oa;
                sk_ptrs(skA_, pb, ob);
                sk_ptrs(skC_, pa, oa);
                std::vector<const void*> b64(in_.b.begin(), in_.b.end()), x64(xcur_.begin(), xcur_.end());
                stta_sketch(so_plain, in_.rb, b64, pb.data(), ob.data(), scratch_, st_);
                stta_sketch(so_op64, xcur_r_, x64, pa.data(), oa.data(), scratch_, st_);
                axpby(sk_len_, 1.0, skA_, -1.0, skC_, st_);      // skC = Psi(b) - Psi(A x)
                std::vector<const double*> cpsi(pa.begin(), pa.end()), com(oa.begin(), oa.end());
                // Psi(b) and Psi(A x) are O(||b||) while their difference is
                // O(res ||b||): the difference carries FP64 rounding of relative
                // size eps / res, and singular values of its Omega below that
                // are noise that the pseudo-inverse must not amplify
                const double rc = std::max(o.rcond, 64.0 * 2.220446049250313e-16 / std::max(last_true, 1e-300));
                std::vector<int> rr;
                stta_recover(d, n, in_.rho, in_.rx, cpsi, com, rc, slots_[s0], rr, scratch_, st_);
                int cap = 0;
                for (int k = 0; k <= d; ++k) cap = std::max(cap, in_.rx[k]);
                tt_svd_inplace(d, n, rr, slots_[s0], cap_, 1e-12, cap, scratch_, st_, nullptr);
                slot_r_[s0] = rr;
            }
            beta = tt_norm_copy(slot_r_[s0], cvec(slots_[s0]));
        }
        if (beta == 0.0) {
            status = TTSG_OK;
            break;
        }
        scale_f64((int64_t)slot_r_[s0][0] * n[0] * slot_r_[s0][1], 1.0 / beta, slots_[s0][0], st_);
        to_lp(s0);
        if (vanilla_) {
            basis_r_[0] = slot_r_[s0];
            for (int mu = 0; mu < d; ++mu)
                copy_f64((int64_t)slot_r_[s0][mu] * n[mu] * slot_r_[s0][mu + 1], slots_[s0][mu], basis_[0][mu], st_);
        }
        // S r0 = beta * S v1
        {
            std::vector<const void*> S64(in_.S.begin(), in_.S.end()), c64(slots_[s0].begin(), slots_[s0].end());
            kr_sketch_run(Prec::F64, d, n, s, R1, S64, slot_r_[s0], c64, z_, scratch_, st_);
        }
        if (white_) {
            // S v_1 opens the QR of S V; ||S r0|| = beta ||S v_1|| starts the rotated rhs
            copy_f64(s, z_, SV_, st_);
            fill(s, 0.0, z2_, st_);
            hipLaunchKernelGGL(k_ls_append, dim3(1), dim3(LS_THREADS), 0, st_, s, 0, ldw_, SV_, Q2_, T2_, c2_, z2_,
                               res2_);
            TTSG_HIP(hipGetLastError());
        }
        scale_f64(s, beta, z_, st_);
        if (white_) {
            sumsq(s, z_, lsres_, scal_ + 3, st_);
            hipLaunchKernelGGL(k_whiten_init, dim3(1), dim3(64), 0, st_, ldw_ + 1, scal_ + 3, g_);
            TTSG_HIP(hipGetLastError());
        }
        window.push_back(s0);
        add_phase(TTSG_PH_OTHER, t0);

        int kk = 0;  // columns of W in this cycle
        bool breakdown = false;
        std::vector<double> cyc_res;  // sketched residuals of this cycle
        for (int k = 0; k < m_ && total < maxit_; ++k) {
            const int vk = window.back();
            const int nw_k = (int)window.size();
            pk_cur = (p_ == Prec::BF16 && !(last_sres <= o.tol / (4.0 * 0.00390625))) ? Prec::F32 : p_;
            so_op.p = pk_cur;
            TTSG_HIP(hipEventRecord(side.v, st_));   // v_k (and S r0) are in place
            auto t1 = now();
            if (pre_) {
                precond_step(k, vk, window);
                add_phase(TTSG_PH_STTA, t1);
            } else {
            // 1) (stream K) w_k = S A v_k, then the least-squares update of W_k
            if (!white_) {
            TTSG_HIP(hipStreamWaitEvent(side.k, side.v, 0));
            {
                std::vector<const void*> SA64(SA64_.begin(), SA64_.end());
                std::vector<const void*> c64(slots_[vk].begin(), slots_[vk].end());
                kr_sketch_run(Prec::F64, d, n, s, in_.R, SA64, slot_r_[vk], c64, W_ + (int64_t)k * s, scratchK_,
                              side.k);
            }
            hipLaunchKernelGGL(k_ls_append, dim3(1), dim3(LS_THREADS), 0, side.k, s, k, m_ + 1, W_, Q_, Rls_, cls_,
                               z_, lsres_);
            TTSG_HIP(hipGetLastError());
            }
            add_phase(TTSG_PH_KR, t1);
            // 2) (stream H) the STTA sketch of v_k, kept for the final solution,
            // and h_{i,k} for the window
            t1 = now();
            TTSG_HIP(hipStreamWaitEvent(side.h, side.v, 0));
            sketch_slot(vk, sketches_ + (int64_t)k * sk_len_, scratchH_, side.h);
            fill(1, 1.0, hco_, side.h);
            const int nw = (int)window.size();
            for (int t = 0; t < nw; ++t) {
                const int vi = window[t];
                inner_run(pk_cur, d, n, in_.R, Dv, slot_r_[vk], slot_ops(vk), slot_r_[vi], slot_ops(vi), hco_ + 1 + t,
                          scratchH_, side.h, blk);
            }
            TTSG_HIP(hipEventRecord(side.hd, side.h));
            add_phase(TTSG_PH_INNER, t1);
            // 3) (main) STTA sketch of A v_k, combined with the window sketches
            // once stream H has delivered them and h
            t1 = now();
            {
                std::vector<double*> psi, om;
                sk_ptrs(skA_, psi, om);
                stta_sketch(so_op, slot_r_[vk], slot_ops(vk), psi.data(), om.data(), scratch_, st_, &sk_side);
                TTSG_HIP(hipStreamWaitEvent(st_, side.hd, 0));
                // window entry t holds basis index (k - nw + 1 + t) of this cycle
                std::vector<const double*> xs(1 + nw);
                std::vector<double> sg(1 + nw, -1.0);
                xs[0] = skA_;
                sg[0] = 1.0;
                for (int t = 0; t < nw; ++t) xs[1 + t] = sketches_ + (int64_t)(k - nw + 1 + t) * sk_len_;
                lin_comb_dev(sk_len_, 1 + nw, xs.data(), hco_, sg.data(), skC_, st_);
            }
            add_phase(TTSG_PH_STTA, t1);
            }
            // 4) recover + TT-SVD into a free slot
            t1 = now();
            int fs = -1;
            for (int sl = 0; sl < nslots; ++sl)
                if (std::find(window.begin(), window.end(), sl) == window.end()) {
                    fs = sl;
                    break;
                }
            {
                std::vector<double*> psi, om;
                sk_ptrs(skC_, psi, om);
                std::vector<const double*> cpsi(psi.begin(), psi.end()), com(om.begin(), om.end());
                // sketches of A v_k carry the working precision's rounding: singular
                // values of Omega below it are noise, not directions
                const double rc = pk_cur == Prec::F64 ? o.rcond
                                                      : std::max(o.rcond, pk_cur == Prec::F32 ? 1e-6 : 4e-3);
                stta_recover(d, n, in_.rho, in_.rx, cpsi, com, rc, slots_[fs], slot_r_[fs], scratch_, st_);
            }
            add_phase(TTSG_PH_RECOVER, t1);
            t1 = now();
            // bfloat16 sketches of A v_k err by about its unit roundoff (2^-8):
            // directions below that are noise and are not kept in the basis
            const double basis_tol = pk_cur == Prec::BF16 ? std::max(o.round_tol, 0.00390625) : o.round_tol;
            (void)take_rank_cap_events();
            const double h = tt_svd_inplace(d, n, slot_r_[fs], slots_[fs], cap_, basis_tol, o.maxrank, scratch_,
                                            st_, nullptr);
            cap_events += take_rank_cap_events();
            add_phase(TTSG_PH_TTSVD, t1);
            TTSG_CHECK(std::isfinite(h), TTSG_ERR_NONFINITE, "non-finite basis vector");
            // 5) least-squares residual (stream K finished long ago)
            t1 = now();
            double sres = 0.0;
            if (white_) {
                // S v_{k+1} extends the QR of S V; one Givens step of T H
                if (h > 0.0 && std::isfinite(h)) {
                    std::vector<const void*> S64(in_.S.begin(), in_.S.end()), c64(slots_[fs].begin(), slots_[fs].end());
                    kr_sketch_run(Prec::F64, d, n, s, R1, S64, slot_r_[fs], c64, SV_ + (int64_t)(k + 1) * s, scratch_,
                                  st_);
                    scale_f64(s, 1.0 / h, SV_ + (int64_t)(k + 1) * s, st_);
                    hipLaunchKernelGGL(k_ls_append, dim3(1), dim3(LS_THREADS), 0, st_, s, k + 1, ldw_, SV_, Q2_, T2_,
                                       c2_, z2_, res2_);
                    TTSG_HIP(hipGetLastError());
                }
                hipLaunchKernelGGL(k_whiten_step, dim3(1), dim3(64), 0, st_, k, ldw_, nw_k, T2_, hco_ + 1, h,
                                   h > 0.0 ? 1 : 0, Gr_, cs_, sn_, g_, lsres_);
                TTSG_HIP(hipGetLastError());
                sres = *static_cast<const double*>(read_back(lsres_, sizeof(double), &sres, st_));
            } else {
                sres = *static_cast<const double*>(read_back(lsres_, sizeof(double), &sres, side.k));
            }
            add_phase(TTSG_PH_LS, t1);
            TTSG_CHECK(std::isfinite(sres), TTSG_ERR_NONFINITE, "non-finite sketched residual");
            kk = k + 1;
            ++total;
            last_sres = sres / Sb;
            int mr = 0;
            for (int b = 0; b <= d; ++b) mr = std::max(mr, slot_r_[fs][b]);
            max_rank = std::max(max_rank, mr);
            if (info && info->sketched_history && total - 1 < o.maxit) info->sketched_history[total - 1] = last_sres;
            if (info && info->rank_history && total - 1 < o.maxit) info->rank_history[total - 1] = mr;
            // Lucky breakdown: v~ = A v_k - sum_i h_{i,k} v_i vanishes to rounding,
            // i.e. h_{k+1,k} <= 1e-12 ||A v_k|| with ||A v_k||^2 ~ h_{k+1,k}^2 +
            // sum_i h_{i,k}^2.  The coefficients are read back only when the
            // cycle stops anyway (the Krylov space is then invariant and the
            // least-squares residual is at rounding level too).
            if (h == 0.0 || sres <= stop) {
                double hb[16];  // hco_ holds 16 values; the ABI caps q at 7
                const int nwr = std::min(nw_k, 15);
                const double* hv =
                    static_cast<const double*>(read_back(hco_, (1 + nwr) * sizeof(double), hb, st_));
                double hn2 = h * h;
                for (int t = 1; t <= nwr; ++t) hn2 += hv[t] * hv[t];
                if (h <= 1e-12 * std::sqrt(hn2)) breakdown = true;
                break;
            }
            if (k + 1 >= m_ || total >= maxit_) break;
            // Low-precision sketches of A v_k put a floor under what one cycle can
            // reach (about the working precision's rounding relative to the
            // cycle's r0).  When the sketched residual has fallen by less than 20%
            // over the last kStall iterations the cycle ends; the next one restarts
            // from the FP64 residual b - A x (iterative refinement).
            cyc_res.push_back(sres);
            constexpr int kStall = 8;
            if (p_ != Prec::F64 && (int)cyc_res.size() > kStall &&
                sres > 0.8 * cyc_res[cyc_res.size() - 1 - kStall])
                break;
            // 6) v_{k+1} (its sketch is taken on stream H in the next iteration)
            t1 = now();
            scale_f64((int64_t)slot_r_[fs][0] * n[0] * slot_r_[fs][1], 1.0 / h, slots_[fs][0], st_);
            to_lp(fs);
            if (vanilla_) {
                basis_r_[k + 1] = slot_r_[fs];
                for (int mu = 0; mu < d; ++mu)
                    copy_f64((int64_t)slot_r_[fs][mu] * n[mu] * slot_r_[fs][mu + 1], slots_[fs][mu],
                             basis_[k + 1][mu], st_);
            }
            window.push_back(fs);
            if ((int)window.size() > q_) window.erase(window.begin());
            add_phase(TTSG_PH_STTA, t1);
        }
        // ---- solution of the cycle ----
        auto t2 = now();
        if (white_)
            hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(64), 0, st_, kk, ldw_, Gr_, g_, y_);
        else
            hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(64), 0, st_, kk, m_ + 1, Rls_, cls_, y_);
        TTSG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_gemv_cols, dim3(grid_for(sk_len_)), dim3(256), 0, st_, sk_len_, kk, sk_len_,
                           sketches_, y_, skC_);
        TTSG_HIP(hipGetLastError());
        std::vector<double*> corr = have_x ? xsum_ : xcur_;
        std::vector<int> cr;
        {
            std::vector<double*> psi, om;
            sk_ptrs(skC_, psi, om);
            std::vector<const double*> cpsi(psi.begin(), psi.end()), com(om.begin(), om.end());
            // recover into the free-slot buffers, then round
            int fs = -1;
            for (int sl = 0; sl < nslots; ++sl)
                if (std::find(window.begin(), window.end(), sl) == window.end()) {
                    fs = sl;
                    break;
                }
            int cap = 0;
            for (int k = 0; k <= d; ++k) cap = std::max(cap, in_.rx[k]);
            if (vanilla_) {
                // Alg. 3: x = Round(x + y_i v_i, final_tol) one basis vector at a time
                std::vector<double> hy(std::max(kk, 1));
                TTSG_HIP(hipMemcpyAsync(hy.data(), y_, kk * sizeof(double), hipMemcpyDeviceToHost, st_));
                TTSG_HIP(hipStreamSynchronize(st_));
                cr = basis_r_[0];
                for (int mu = 0; mu < d; ++mu)
                    copy_f64((int64_t)cr[mu] * n[mu] * cr[mu + 1], basis_[0][mu], vacc_[mu], st_);
                scale_f64((int64_t)cr[0] * n[0] * cr[1], hy[0], vacc_[0], st_);
                for (int i = 1; i < kk; ++i) {
                    std::vector<int> sr;
                    tt_add_block(d, n, cr, vacc_, basis_r_[i], cvec(basis_[i]), hy[i], xsum_, sr, st_);
                    tt_svd_inplace(d, n, sr, xsum_, cap_, final_tol, cap, scratch_, st_, nullptr);
                    for (int mu = 0; mu < d; ++mu)
                        copy_f64((int64_t)sr[mu] * n[mu] * sr[mu + 1], xsum_[mu], vacc_[mu], st_);
                    cr = sr;
                }
                for (int mu = 0; mu < d; ++mu)
                    copy_f64((int64_t)cr[mu] * n[mu] * cr[mu + 1], vacc_[mu], slots_[fs][mu], st_);
            } else {
                stta_recover(d, n, in_.rho, in_.rx, cpsi, com, o.rcond, slots_[fs], cr, scratch_, st_);
                tt_svd_inplace(d, n, cr, slots_[fs], cap_, final_tol, cap, scratch_, st_, nullptr);
            }
            if (pre_) {
                // x gains P^{-1} u: the STTA sketches of the zeta terms
                // alpha_j (x)_k E_jk u are summed, recovered and rounded
                std::vector<double*> pa, oa, pt, ot;
                sk_ptrs(skA_, pa, oa);
                sk_ptrs(skT_, pt, ot);
                std::vector<const void*> z64(zbuf_.begin(), zbuf_.end());
                for (int j = 0; j < in_.zeta; ++j) {
                    mode_product_tt(d, n, cr, cvec(slots_[fs]), Eterm(j), in_.alpha[j], zbuf_, st_, &scratch_);
                    stta_sketch(so_plain, cr, z64, (j == 0 ? pa : pt).data(), (j == 0 ? oa : ot).data(), scratch_,
                                st_, &sk_side);
                    if (j > 0) axpby(sk_len_, 1.0, skT_, 1.0, skA_, st_);
                }
                std::vector<const double*> ppsi(pa.begin(), pa.end()), pom(oa.begin(), oa.end());
                stta_recover(d, n, in_.rho, in_.rx, ppsi, pom, o.rcond, slots_[fs], cr, scratch_, st_);
                tt_svd_inplace(d, n, cr, slots_[fs], cap_, final_tol, cap, scratch_, st_, nullptr);
            }
            if (!have_x) {
                for (int mu = 0; mu < d; ++mu)
                    copy_f64((int64_t)cr[mu] * n[mu] * cr[mu + 1], slots_[fs][mu], xcur_[mu], st_);
                xcur_r_ = cr;
                have_x = true;
            } else {
                std::vector<int> sr;
                tt_add_block(d, n, xcur_r_, xcur_, cr, cvec(slots_[fs]), 1.0, xsum_, sr, st_);
                tt_svd_inplace(d, n, sr, xsum_, cap_, final_tol, cap, scratch_, st_, nullptr);
                for (int mu = 0; mu < d; ++mu)
                    copy_f64((int64_t)sr[mu] * n[mu] * sr[mu + 1], xsum_[mu], xcur_[mu], st_);
                xcur_r_ = sr;
            }
        }
        add_phase(TTSG_PH_FINAL, t2);
        t2 = now();
        last_true = true_res(xcur_r_, xcur_);
        add_phase(TTSG_PH_OTHER, t2);
        if (info && info->true_history && cycles - 1 < max_cycles) info->true_history[cycles - 1] = last_true;
        if (last_true <= o.tol) {
            status = breakdown ? TTSG_BREAKDOWN : (cap_events > 0 ? TTSG_RANK_CAPPED : TTSG_OK);
            break;
        }
        // A restart cycle that leaves a larger true residual than the best
        // iterate so far (its correction solved a residual that the rank caps
        // or the working precision could not represent) ends the solve with
        // that best iterate.
        if (cycles > 1 && !(last_true < best_true)) {
            for (int mu = 0; mu < d; ++mu)
                copy_f64((int64_t)xbest_r_[mu] * n[mu] * xbest_r_[mu + 1], xbest_[mu], xcur_[mu], st_);
            xcur_r_ = xbest_r_;
            last_true = best_true;
            true_is_bound = best_is_bound;
            break;
        }
        best_true = last_true;
        best_is_bound = true_is_bound;
        xbest_r_ = xcur_r_;
        for (int mu = 0; mu < d; ++mu)
            copy_f64((int64_t)xcur_r_[mu] * n[mu] * xcur_r_[mu + 1], xcur_[mu], xbest_[mu], st_);
        (void)corr;
    }
    // ---- output ----
    if (have_x) {
        for (int mu = 0; mu < d; ++mu)
            copy_f64((int64_t)xcur_r_[mu] * n[mu] * xcur_r_[mu + 1], xcur_[mu], x_out[mu], st_);
        for (int k = 0; k <= d; ++k) x_r[k] = xcur_r_[k];
    }
    TTSG_HIP(hipStreamSynchronize(st_));
    if (info) {
        info->iterations = total;
        info->cycles = cycles;
        info->max_rank = max_rank;
        info->status = status;
        info->true_residual = last_true;
        info->true_residual_is_bound = true_is_bound ? 1 : 0;
        info->sketched_residual = last_sres;
    }
    return status;
}

int sgmres_solve(const SolverInputs& in, double* const* x, int32_t* x_r, ttsg_sgmres_info* info, void* ws,
                 size_t ws_bytes, hipStream_t st) {
    SgmresSolver s(in, st);
    return s.run(x, x_r, info, ws, ws_bytes);
}

size_t sgmres_workspace(const SolverInputs& in) {
    SgmresSolver s(in, nullptr);
    return s.workspace_bytes();
}

}  // namespace ttsg
