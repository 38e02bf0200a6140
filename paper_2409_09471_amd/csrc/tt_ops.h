// Host-side building blocks of the TT sweeps (tt_ops.hip) and the rounding
// pipeline (rounding.hip).
#pragma once

#include "ttsg_internal.h"

namespace ttsg {

ContractDesc cdesc(int M, int N, int K, int batch = 1);

// Sizes of one environment step: vector core rl x n x rr, operator ranks
// Rl/Rr (1/1 when there is no operator), probe core pl x n x pr.
struct LeftDims {
    int rl, n, rr, Rl, Rr, pl, pr;
    // Kinds of the operator core's n x n blocks D[al][:, :][be] (Rl x Rr,
    // row-major; see operator_blocks), or nullptr: every block dense.
    const uint8_t* blk = nullptr;
};

// Kind of an n x n block of an operator core: exactly zero, exactly the
// identity, or anything else.  Kronecker-sum operators (Sec. 5.1) have mostly
// zero and identity blocks: the operator steps copy the identity blocks and
// skip the zero ones instead of multiplying by them.
enum : uint8_t { kBlkZero = 0, kBlkIdentity = 1, kBlkDense = 2 };
// Classify every block of the d float64 operator cores D[mu] (R[mu] x n x n x
// R[mu+1]); synchronizes st once.  Result: per core, R[mu] * R[mu+1] kinds.
// The device table (sum of R[mu] * R[mu+1] bytes) is carved from `ar` and
// released before returning.
std::vector<std::vector<uint8_t>> operator_blocks(int d, const int* n, const std::vector<int>& R,
                                                  const std::vector<const void*>& D, hipStream_t st, Arena& ar);
// Host pointers into operator_blocks' result (empty when it is empty).
std::vector<const uint8_t*> block_ptrs(const std::vector<std::vector<uint8_t>>& kinds);

void matvec_core(int rl, int n, int rr, int Rl, int Rr, const double* D, const double* C, bool transpose,
                 double* G, hipStream_t st);

// E (pl x Rl x rl) -> Eout (pr x Rr x rr).  T1 holds pl*Rl*n*rr and T2
// pl*n*Rr*rr elements; with D == nullptr T2 is not used (T1 plays its role).
// Z == nullptr stops after T1/T2 (what the core sketch Psi needs).
void left_step(Prec p, const LeftDims& s, const void* E, const void* C, const void* D, const void* Z, void* T1,
               void* T2, void* Eout, hipStream_t st, Arena* ar = nullptr);
// F (rr x Rr x pr) -> Fout (rl x Rl x pl).  U1: rl*n*Rr*pr, U2: rl*Rl*n*pr.
void right_step(Prec p, const LeftDims& s, const void* F, const void* C, const void* D, const void* Z, void* U1,
                void* U2, void* Fout, hipStream_t st, Arena* ar = nullptr);
// out_f64: float32 arithmetic (p != F64) writes a float64 Psi / Om.
void psi_step(Prec p, int pl, int n, int Rr, int rr, int qr, const void* T2, const void* F, void* Psi,
              hipStream_t st, Arena* ar = nullptr, bool out_f64 = false);
void omega_step(Prec p, int pl, int Rr, int rr, int qr, const void* E, const void* F, void* Om, hipStream_t st,
                Arena* ar = nullptr, bool out_f64 = false);

void kr_precompute(Prec p, int s, int n, int Rl, int Rr, const void* S, const void* D, void* SA, hipStream_t st);
// P (s x Rl x rl) -> Pout (s x Rr x rr); Xbuf holds s*Rr*rl*n elements.
void kr_step(Prec p, int s, int rl, int n, int rr, int Rl, int Rr, const void* P, const void* SA, const void* C,
             void* Xbuf, void* Pout, hipStream_t st, Arena* ar = nullptr);

// ---------------------------------------------------------------------------
// Views with host-known ranks.
// ---------------------------------------------------------------------------
struct TTView {
    int d = 0;
    const int* n = nullptr;
    std::vector<int> r;              // d + 1
    std::vector<const double*> c;    // d cores
};

struct TTOut {
    std::vector<int> r;              // d + 1
    std::vector<double*> c;          // d cores (capacity managed by the caller)
};

struct OpView {
    std::vector<int> R;              // d + 1
    std::vector<const double*> c;    // d cores, nullptr entries mean "identity"
    bool present = false;
};

// Element size of a precision's storage type.
inline size_t elem_size(Prec p) { return p == Prec::F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// STTA sketch (Sec. 3.3) of x or A x.  Y holds d-1 cores (modes 0..d-2),
// X holds d-1 cores (modes 1..d-1, entry k-1 for mode k).  Psi/Omega are
// float64 outputs.  Scratch comes from the arena (released on return).
// All operand pointers are of the element type of `p` except Psi/Omega.
// ---------------------------------------------------------------------------
struct SketchOperands {
    Prec p = Prec::F64;
    const int* n = nullptr;
    int d = 0;
    std::vector<int> rho, rx;                 // d + 1
    std::vector<const void*> Y, X;            // d - 1 each, element type of p
    std::vector<int> R;                       // d + 1 (all 1 without operator)
    std::vector<const void*> D;               // d, element type of p, or empty
    std::vector<const uint8_t*> blk;          // d block-kind tables of D (operator_blocks), or empty
};

// A second stream for stta_sketch: the right-environment sweep and the Omega
// sketches run on it while the calling stream runs the left sweep and the Psi
// sketches (the two sweeps are independent; Psi_mu and Omega_b need one
// environment of each).  The events belong to the caller (created once).
struct SketchSide {
    hipStream_t st = nullptr;
    Arena* ar = nullptr;   // scratch used only by st
    hipEvent_t in = nullptr, right = nullptr, left = nullptr, done = nullptr;
};
// x cores (element type of p), ranks r.  With side, every output is complete
// in stream order on st when the call returns (st waits for the side stream).
void stta_sketch(const SketchOperands& o, const std::vector<int>& r, const std::vector<const void*>& x,
                 double* const* Psi, double* const* Omega, Arena& ar, hipStream_t st,
                 const SketchSide* side = nullptr);

// Khatri-Rao sketch w = S x or S A x.  SA: d precomputed S_mu D_mu (or S_mu)
// of element type p; w: float64 output of length s.
void kr_sketch_run(Prec p, int d, const int* n, int s, const std::vector<int>& R,
                   const std::vector<const void*>& SA, const std::vector<int>& r,
                   const std::vector<const void*>& x, double* w, Arena& ar, hipStream_t st);

// Inner product <A x, z> (A optional) by a left sweep; result (float64) written
// to out_dev[0].
void inner_run(Prec p, int d, const int* n, const std::vector<int>& R, const std::vector<const void*>& D,
               const std::vector<int>& rx_, const std::vector<const void*>& x, const std::vector<int>& rz,
               const std::vector<const void*>& z, double* out_dev, Arena& ar, hipStream_t st,
               const std::vector<const uint8_t*>& blk = {});

// ---------------------------------------------------------------------------
// LDS-resident factorizations (la_lds.hip)
// ---------------------------------------------------------------------------
struct JacobiJob {
    int m, c, lda;        // column-major m x c (m >= c), leading dimension lda
    double* A;            // in: matrix; out: U * Sigma
    double* V;            // out: c x c right singular vectors (column-major, ld c)
    double* sig;          // out: c singular values (unsorted)
    double tol = 0.0;     // stop when every |a_p.a_q| <= tol ||a_p|| ||a_q|| (0: 4 m eps)
    // A column whose squared norm is at most max(drop_abs2, drop_rel2 *
    // (largest initial squared column norm)) takes part in no further rotation,
    // like the columns at rounding-noise level.  For callers that discard every
    // such column afterwards: with A V = B for the accumulated orthogonal V,
    // keeping any set of columns of B leaves an error of exactly the norm of
    // the dropped ones, whatever the angles between kept and dropped columns,
    // and the kept columns are still orthogonalized among themselves.
    double drop_abs2 = 0.0;
    double drop_rel2 = 0.0;
};
bool jacobi_lds_fits(int m, int c);
// One launch for up to 32 matrices (more are split into several launches).
void svd_jacobi_batched(const std::vector<JacobiJob>& jobs, hipStream_t st);
// One-sided Jacobi for 64 < c <= 128 (m <= 160): A (column-major, in place)
// becomes B = A V with columns sorted by norm, sig the sorted singular values;
// V (c x c, ld c, sorted like B) only when `accumulate` (else V is ignored).
bool jacobi_big_fits(int m, int c);
// With accumulate, V comes from a rotation log kept in `ar` (released on
// return; jacobi_big_log_bytes(c) per job of c columns, batches of 32 jobs).
void svd_jacobi_big(const std::vector<JacobiJob>& jobs, bool accumulate, hipStream_t st, Arena* ar = nullptr);
size_t jacobi_big_log_bytes(int c);

// Householder QR of several small column-major matrices in one launch (one
// workgroup each, the matrix and Q in LDS): Q (m x c, column-major, ld m) and
// R (c x c, column-major, ld c, zero below the diagonal).  With perm != nullptr
// the columns are pivoted (largest remaining norm first): A P = Q R, column l
// of A P being column perm[l] of A.
struct QrJob {
    int m, c, lda;
    const double* A;
    double* Q;
    double* R;
    int* perm = nullptr;
    bool a_rowmajor = false;   // A(i, j) at A[i * lda + j] instead of A[j * lda + i]
    bool r_transposed = false; // write R^T (column-major c x c) instead of R
};
bool qr_small_fits(int m, int c);
void qr_small_batched(const std::vector<QrJob>& jobs, hipStream_t st);

bool tsqr_fits(int m, int c);
// Tall-skinny QR of a column-major m x c matrix (m >= c, c <= 64) by a tree of
// LDS Householder leaves.  factor() leaves R (c x c, column-major, ld c, zero
// below the diagonal) in `R`; apply() writes Q * B (m x k) for a c x k matrix B.
struct TsqrPlan {
    struct Level {
        int rows, nleaves;
        double* refl;
        double* tau;
        double* stack;
    };
    int m = 0, c = 0;
    std::vector<Level> levels;
    double* R = nullptr;
    void factor(int m, int c, const double* A, int lda, Arena& ar, hipStream_t st);
    void apply(int k, const double* B, int ldb, double* Out, int ldo, bool out_rowmajor, Arena& ar,
               hipStream_t st) const;
};

// ---------------------------------------------------------------------------
// Rounding pipeline (rounding.hip), all FP64.
// ---------------------------------------------------------------------------
// TT-SVD rounding in place: cores `w` (capacity per core given by cap_elems)
// with ranks r; on return r holds the new ranks.  Returns ||T||_F.
// tol is relative, maxrank 0 = none.  Synchronizes the stream.
// Arena bytes that tt_svd_inplace needs beyond 6 cores of the largest size
// (core snapshot for the Householder redo and the CholQR2 scratch).
size_t tt_svd_extra_bytes(int d, const int* n, const int* r);
double tt_svd_inplace(int d, const int* n, std::vector<int>& r, const std::vector<double*>& w,
                      const std::vector<int64_t>& cap_elems, double tol, int maxrank, Arena& ar,
                      hipStream_t st, double* norm_before = nullptr);

// Number of bonds, since the last call on this host thread, whose TT-SVD rank
// was decided by the rank cap rather than the tolerance (then reset to 0).
int take_rank_cap_events();

// STTA recovery: cores of Omega^+ applied to Psi, compacted to the numerical
// ranks of the Omega_b (relative cutoff rcond).  out cores need capacity
// rx[mu] * n[mu] * rx[mu+1].  Writes the recovered ranks to r_out.
void stta_recover(int d, const int* n, const std::vector<int>& rho, const std::vector<int>& rx,
                  const std::vector<const double*>& Psi, const std::vector<const double*>& Omega, double rcond,
                  const std::vector<double*>& out, std::vector<int>& r_out, Arena& ar, hipStream_t st);

// Left orthogonalization sweep by Householder QR; returns ||T|| (reads one
// float64 back).  Cores are modified in place; ranks may shrink.
double tt_norm_orth(int d, const int* n, std::vector<int>& r, const std::vector<double*>& w, Arena& ar,
                    hipStream_t st);

// ---------------------------------------------------------------------------
// Exponential-sum preconditioner (precond.hip, Sec. 4.1)
// ---------------------------------------------------------------------------
// alpha_j, beta_j (j < zeta) with |z E(z) - 1| <= tol on [zmin, zmax]; returns
// zeta, -zeta when max_terms is too small, -1 for bad arguments.
int expsum_coefficients(double zmin, double zmax, double tol, int max_terms, double* alpha, double* beta);
// out[k] (zeta x n_k x n_k, row-major, term-major) = exp(-beta_j M_k) for every
// term j and mode k; beta ascending.  Synchronizes once (mode norms).
void mode_exponentials(int zeta, const double* beta, int d, const int* n, const std::vector<const double*>& M,
                       const std::vector<double*>& out, Arena& ar, hipStream_t st);
// z = alpha (x)_k E_k x: E_k applied to the mode index of core k (ranks kept),
// alpha folded into the first core.  E[k]: n_k x n_k row-major.
void mode_product_tt(int d, const int* n, const std::vector<int>& r, const std::vector<const double*>& x,
                     const std::vector<const double*>& E, double alpha, const std::vector<double*>& z, hipStream_t st,
                     Arena* ar = nullptr);

// ---------------------------------------------------------------------------
// Solver (solver.hip)
// ---------------------------------------------------------------------------
struct SolverInputs {
    int d;
    const int* n;
    std::vector<int> R;
    std::vector<const double*> A;
    std::vector<int> rb;
    std::vector<const double*> b;
    int s;
    std::vector<const double*> S;
    std::vector<int> rho, rx;
    std::vector<const double*> Y, X;
    ttsg_sgmres_opts o;
    // optional initial guess of x (x0_r empty: x0 = 0)
    std::vector<int> x0_r;
    std::vector<const double*> x0;
    // optional exponential-sum right preconditioner (zeta = 0: none)
    int zeta = 0;
    std::vector<double> alpha, beta;
    std::vector<const double*> M;     // d mode matrices n_k x n_k
    int ls_mode = TTSG_LS_PINV;
    int variant = TTSG_VARIANT_ENHANCED;
    bool single_stream = false;
};

// TT-GMRES (Alg. 2; gmres.hip): full modified Gram-Schmidt, TT-SVD rounding
// relaxed as eta_k tol, eta_k = tol / (relative residual of step k-1), capped at
// max_round; x_0 = 0; solution by sequential rounded sums at final_tol.
// maxrank > 0 caps every basis rank (and sizes the buffers); 0 = the full bond
// ranks.
struct GmresInputs {
    int d;
    const int* n;
    std::vector<int> R;
    std::vector<const double*> A;
    std::vector<int> rb;
    std::vector<const double*> b;
    int maxit = 1;
    int maxrank = 0;
    double tol = 1e-6, final_tol = 1e-6, max_round = 0.1;
};
int tt_gmres_solve(const GmresInputs& in, double* const* x, int32_t* x_r, ttsg_sgmres_info* info, void* ws,
                   size_t ws_bytes, hipStream_t st);
size_t tt_gmres_workspace(const GmresInputs& in);

int sgmres_solve(const SolverInputs& in, double* const* x, int32_t* x_r, ttsg_sgmres_info* info, void* ws,
                 size_t ws_bytes, hipStream_t st);
// Workspace bytes sgmres_solve needs for these sizes and options (reads no pointers).
size_t sgmres_workspace(const SolverInputs& in);

// a + bscale * b as block cores (ranks add); first/last cores concatenated.
void tt_add_block(int d, const int* n, const std::vector<int>& ra, const std::vector<double*>& a,
                  const std::vector<int>& rb, const std::vector<const double*>& b, double bscale,
                  const std::vector<double*>& out, std::vector<int>& rout, hipStream_t st,
                  double ascale = 1.0);

// CholQR2 of the m x c matrix X (element (i, j) at X[i*xr + j*xc]) into Q
// (same convention, strides qr/qc) and upper R (c x c, column-major).  Raises
// flag[0] = 1 on the device when the factorization is not trustworthy
// (cholqr.hip); requires cholqr_fits(m, c).
bool cholqr_fits(int m, int c);
// RT != nullptr also receives R^T (c x c, column-major).  rinv_fro2 !=
// nullptr receives ||R^{-1}||_F^2 (device scalar): sigma_min(R) >=
// 1 / ||R^{-1}||_F, so a caller can tell that no singular value is small.
void cholqr2(int m, int c, const double* X, int64_t xr, int64_t xc, double* Q, int64_t qr, int64_t qc, double* R,
             int* flag, Arena& ar, hipStream_t st, double* RT = nullptr, double* rinv_fro2 = nullptr);
void zero_flags(int n, int* f, hipStream_t st);

// -<lambda, L_k x> for every mode k (grad.hip); result in out_dev[0..d-1].
void grad_kron_sum(int d, const int* n, const std::vector<const double*>& L, const std::vector<int>& rl,
                   const std::vector<const double*>& lam, const std::vector<int>& rx,
                   const std::vector<const double*>& x, double* out_dev, Arena& ar, hipStream_t st);

}  // namespace ttsg
