/*
 * ttsg.h -- C ABI of the MI355X (gfx950) hot path of randomized sketched
 * TT-GMRES (Bucci, Palitta, Robol: "Randomized sketched TT-GMRES for linear
 * systems with tensor structure").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A TT tensor of order d with mode sizes n[0..d-1] and ranks r[0..d]
 *    (r[0] = r[d] = 1) is passed as an array of d DEVICE pointers; core k is a
 *    row-major float64 array of shape r[k] x n[k] x r[k+1] (eq. tt-format of
 *    Sec. 2.2, 0-based modes).  `n`, `r` and the pointer arrays live in HOST
 *    memory; the cores themselves in device memory.
 *  - A TT-matrix (operator) with ranks R[0..d] is an array of d DEVICE
 *    pointers; core k has shape R[k] x n[k] x n[k] x R[k+1], row index first
 *    (eq. operator tt-format of Sec. 2.2).  (A x)[i] = sum_j A[i, j] x[j].
 *  - Merged ranks of a matrix-vector product put the vector rank outer and the
 *    operator rank inner: index (a, alpha) -> a * R + alpha (Sec. 2.2).
 *  - Khatri-Rao sketch factors S_k (Sec. 3.1): d DEVICE pointers, each an
 *    s x n[k] row-major float64 array; row j of S is kron_k S_k[j, :].
 *  - STTA sketch tensors (Sec. 3.3): the left Gaussian TT-DRM Y has ranks
 *    rho[0..d] and cores for modes 0..d-2 (d-1 DEVICE pointers, core k is
 *    rho[k] x n[k] x rho[k+1]); the right DRM X has ranks rx[0..d] and cores for
 *    modes 1..d-1 (d-1 DEVICE pointers, entry k-1 holds the core of mode k,
 *    rx[k] x n[k] x rx[k+1]).  rho[0] = rho[d] = rx[0] = rx[d] = 1.
 *  - Every call is stream-ordered on `stream` (a hipStream_t; NULL = the
 *    default stream).  Calls that must return data-dependent ranks synchronize
 *    the stream before returning; the others do not.
 *  - The caller owns all buffers it passes.  Scratch memory is taken from the
 *    optional workspace (ws, ws_bytes); when ws is NULL the library allocates
 *    what it needs with hipMallocAsync on `stream` and releases it before
 *    returning.  Distinct workspaces make concurrent calls independent.
 *  - Return value: 0 on success, > 0 a warning (TTSG_NOT_CONVERGED, ...),
 *    < 0 an error (-TTSG_ERR_*).  No C++ exception crosses this boundary.
 *    ttsg_last_error() returns a static description of the last failure on
 *    the calling thread.
 */
#ifndef TTSG_H
#define TTSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* ttsg_stream_t; /* a hipStream_t */

enum {
    TTSG_OK = 0,
    TTSG_NOT_CONVERGED = 1, /* iteration budget spent before the true residual met tol */
    TTSG_BREAKDOWN = 2,     /* h_{k+1,k} = 0: the Krylov space is invariant, solution exact */
    TTSG_RANK_CAPPED = 3,   /* converged, but a basis rounding was limited by the rank cap
                               (maxrank of Sec. 4.2) rather than by its tolerance */
    TTSG_ERR_ARG = 1,       /* returned negated: bad sizes, ranks or pointers */
    TTSG_ERR_CAPACITY = 2,  /* an output capacity is smaller than required */
    TTSG_ERR_WS = 3,        /* workspace too small */
    TTSG_ERR_NONFINITE = 4, /* a NaN/Inf appeared in the inputs or the iteration */
    TTSG_ERR_HIP = 5,       /* a HIP runtime call failed (see ttsg_last_error) */
    TTSG_ERR_DTYPE = 6      /* unknown precision / arithmetic mode */
};

/* Least-squares form of the sketched problem (Sec. 3.4). */
enum {
    TTSG_LS_PINV = 0,   /* y = (S A V_k)^+ S r0 (eq. pseudo_inv): W_k = S A V_k is formed */
    TTSG_LS_WHITEN = 1  /* whitening: skinny QR of S V_{k+1} and the sketched Arnoldi
                           relation (eq. sketchedArnoldi); y from eq. sketched_argmin2,
                           the residual from eq. sketched_residualnorm.  W_k is not formed */
};

/* How a cycle's solution is formed from the basis (Alg. 3 vs Alg. 4). */
enum { TTSG_VARIANT_ENHANCED = 0, TTSG_VARIANT_VANILLA = 1 };

/* Arithmetic of the contraction kernels. */
typedef enum {
    TTSG_PREC_F64 = 0,   /* everything in float64 (FP64 MFMA) */
    TTSG_PREC_MIXED = 1, /* sketch/rounding contractions in float32 with float32
                            accumulation; least squares, QR/SVD, recovery and the
                            final solution in float64 */
    TTSG_PREC_BF16 = 2   /* as MIXED, but the STTA sketch of A v_k and the
                            orthogonalization coefficients use bfloat16 MFMA
                            inputs with float32 accumulation */
} ttsg_precision;

/* ------------------------------------------------------------------------- */
/* Library                                                                   */
/* ------------------------------------------------------------------------- */

/* Static, NUL-terminated description of the last error on this thread. */
const char* ttsg_last_error(void);

/* Version string of the library build. */
const char* ttsg_version(void);

/* ------------------------------------------------------------------------- */
/* TT matrix-vector product (Sec. 2.2):                                      */
/*   G_k[(a,al), i, (b,be)] = sum_j D_k[al, i, j, be] C_k[a, j, b]           */
/* ------------------------------------------------------------------------- */
/* y_cores[k] must hold (r[k]*R[k]) x n[k] x (r[k+1]*R[k+1]) float64 values.
 * transpose != 0 applies the transposed operator (row and column swapped).
 * Does not synchronize. */
int ttsg_matvec(int32_t d, const int32_t* n, const int32_t* R, const double* const* A,
                const int32_t* r, const double* const* x, int32_t transpose,
                double* const* y, ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Khatri-Rao sketch (Sec. 3.1): w = S x, or w = S (A x) when A != NULL       */
/* without forming A x.  (S x)_j = prod_k sum_i S_k[j, i] C_k[:, i, :].       */
/* ------------------------------------------------------------------------- */
/* w: DEVICE float64 array of length s.  R/A may be NULL (plain sketch).
 * precision: TTSG_PREC_F64, TTSG_PREC_MIXED (float32 contractions) or
 * TTSG_PREC_BF16 (bfloat16 matrix-core inputs, float32 accumulation).
 * Does not synchronize. */
int ttsg_kr_sketch(int32_t d, const int32_t* n, int32_t s, const double* const* S,
                   const int32_t* R, const double* const* A,
                   const int32_t* r, const double* const* x,
                   double* w, int32_t precision,
                   void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* STTA sketch (Sec. 3.3) of x, or of A x when A != NULL:                     */
/*   Psi_k   = (Y_{<=k-1}^T (x) I) T_{<=k} X_{>k}   shape rho[k] x n[k] x rx[k+1] */
/*   Omega_b = Y_{<=b}^T T_{<=b} X_{>b}             shape rho[b] x rx[b], b=1..d-1 */
/* ------------------------------------------------------------------------- */
/* Psi: d DEVICE pointers; Omega: d-1 DEVICE pointers (entry b-1 for bond b).
 * Does not synchronize. */
int ttsg_stta_sketch(int32_t d, const int32_t* n,
                     const int32_t* rho, const double* const* Y,
                     const int32_t* rx, const double* const* X,
                     const int32_t* R, const double* const* A,
                     const int32_t* r, const double* const* x,
                     double* const* Psi, double* const* Omega, int32_t precision,
                     void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * STTA sketch as ttsg_stta_sketch, with the same arguments, layouts, results
 * and stream ordering, but without a workspace argument.  Its scratch is a
 * static device buffer of 128 MiB inside the library (one per GPU, held until
 * the process ends); the call makes no hipMalloc/hipFree and no allocating
 * library call.  Shapes whose scratch exceeds the buffer return -TTSG_ERR_WS
 * before any work is queued (ttsg_stta_sketch_workspace_size gives the need;
 * e.g. d = 10, n = 64, ranks 64, rho 84, operator rank 3 needs about 101 MiB
 * in float64).  With the tile autotuner on it returns -TTSG_ERR_ARG (tuning
 * allocates).  Every call on one GPU shares that GPU's buffer: calls that
 * overlap on one GPU (different streams or host threads) race and must be
 * serialized by the caller.  The stream must belong to the current device.
 * Does not synchronize. */
int ttsg_stta_sketch_noalloc(int32_t d, const int32_t* n,
                             const int32_t* rho, const double* const* Y,
                             const int32_t* rx, const double* const* X,
                             const int32_t* R, const double* const* A,
                             const int32_t* r, const double* const* x,
                             double* const* Psi, double* const* Omega, int32_t precision,
                             ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Randomized rounding (Sec. 3.3, STTA_sketch + STTA_recover):                */
/* sketch x with (Y, X), recover C^_0 = Psi_0, C^_k = Omega_k^+ Psi_k (pseudo-  */
/* inverse by FP64 SVD with relative cutoff rcond), then TT-SVD of the small  */
/* recovered tensor at relative tolerance tol with every rank capped at       */
/* maxrank (0 = no cap) (Sec. 2.2 rounding; cap of Sec. 4.2).                  */
/* ------------------------------------------------------------------------- */
/* out: d DEVICE pointers, core k with capacity rx[k] x n[k] x rx[k+1];
 * out_r: HOST int32[d+1] receives the ranks of the result.
 * Synchronizes `stream` (the ranks are data dependent). */
int ttsg_round_rand(int32_t d, const int32_t* n,
                    const int32_t* r, const double* const* x,
                    const int32_t* rho, const double* const* Y,
                    const int32_t* rx, const double* const* X,
                    double tol, int32_t maxrank, double rcond,
                    double* const* out, int32_t* out_r, int32_t precision,
                    void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* Workspace bytes of ttsg_kr_sketch / ttsg_stta_sketch / ttsg_round_rand for
 * these shapes (R may be NULL: no operator).  A workspace of at least this
 * size, passed as (ws, ws_bytes), makes the call allocate no device memory.
 * Returns 0 and writes *bytes, or a negative error. */
int ttsg_kr_sketch_workspace_size(int32_t d, const int32_t* n, int32_t s, const int32_t* R, const int32_t* r,
                                  int32_t precision, size_t* bytes);
int ttsg_stta_sketch_workspace_size(int32_t d, const int32_t* n, const int32_t* rho, const int32_t* rx,
                                    const int32_t* R, const int32_t* r, int32_t precision, size_t* bytes);
int ttsg_round_rand_workspace_size(int32_t d, const int32_t* n, const int32_t* r, const int32_t* rho,
                                   const int32_t* rx, int32_t precision, size_t* bytes);

/* Deterministic TT-SVD rounding (Sec. 2.2) of x at relative tolerance tol,
 * ranks capped at maxrank (0 = none).  out cores have capacity r[k] x n[k] x
 * r[k+1] (rounding never increases ranks).  Synchronizes `stream`. */
int ttsg_round_svd(int32_t d, const int32_t* n, const int32_t* r, const double* const* x,
                   double tol, int32_t maxrank, double* const* out, int32_t* out_r,
                   void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Sketched TT-GMRES (Alg. 4, enhanced TT-sGMRES)                             */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t maxit;       /* total iteration budget over all cycles */
    int32_t restart;     /* cycle length m; 0 = maxit (restart of Sec. 3.4) */
    int32_t q;           /* incomplete orthogonalization window (paper's l) */
    int32_t maxrank;     /* rank cap of the basis vectors (0 = only rx caps) */
    int32_t precision;   /* ttsg_precision */
    int32_t max_cycles;  /* cap on restart cycles (0 = 50) */
    double tol;          /* target true relative residual ||b - A x|| / ||b|| */
    double round_tol;    /* basis rounding tolerance (eta * tol) */
    double final_tol;    /* rounding tolerance of the solution (0 = round_tol) */
    double stop_safety;  /* a cycle stops when ||W y - S r0|| <= stop_safety*tol*||S b|| */
    double rcond;        /* relative cutoff of the pseudo-inverses in STTA_recover */
} ttsg_sgmres_opts;

typedef struct {
    int32_t iterations;       /* total Krylov iterations */
    int32_t cycles;           /* restart cycles run */
    int32_t max_rank;         /* largest basis rank seen */
    int32_t status;           /* same as the return value */
    double true_residual;     /* FP64 ||b - A x|| / ||b|| of the returned x */
    double sketched_residual; /* last ||W y - S r0|| / ||S b|| */
    /* optional HOST arrays (may be NULL): per-iteration sketched residual and
       basis rank (length >= maxit), per-cycle true residual (>= max_cycles),
       and the seconds spent in each phase (length >= 8, see ttsg_phase). */
    double* sketched_history;
    int32_t* rank_history;
    double* true_history;
    double* phase_seconds;
    /* out: 1 when true_residual is the rounding floor of the FP64 identity
       ||b - A x||^2 = ||b||^2 - 2 <A x, b> + ||A x||^2 rather than a measured
       value.  The identity is evaluated first; below its floor
       sqrt(64 eps (||b||^2 + ||A x||^2)) / ||b|| the difference is rounding.  When
       that floor is already <= tol it is reported (an upper bound of the true
       residual at the identity's rounding level) and the solve ends; otherwise
       b - A x is formed as a block TT and its norm measured by
       orthogonalization (flag 0). */
    int32_t true_residual_is_bound;
} ttsg_sgmres_info;

/* Phases reported in info->phase_seconds (host wall clock with stream syncs
 * only when phase timing is requested). */
enum { TTSG_PH_KR = 0, TTSG_PH_INNER = 1, TTSG_PH_STTA = 2, TTSG_PH_RECOVER = 3,
       TTSG_PH_TTSVD = 4, TTSG_PH_LS = 5, TTSG_PH_FINAL = 6, TTSG_PH_OTHER = 7 };

/* Solve A x = b with x_0 = 0 (ttsg_sgmres_solve_ex adds an initial guess, a
 * right preconditioner and the whitened least squares).  The sketches S (s rows), Y and X are supplied
 * by the caller.  x: d DEVICE pointers with capacity rx[k] x n[k] x rx[k+1];
 * x_r: HOST int32[d+1] receives the solution ranks.  Returns TTSG_OK when the
 * FP64 true residual is <= tol, TTSG_NOT_CONVERGED when the budget ran out
 * (x is then the last iterate), or a negative error.  Synchronizes `stream`. */
int ttsg_sgmres_solve(int32_t d, const int32_t* n,
                      const int32_t* R, const double* const* A,
                      const int32_t* rb, const double* const* b,
                      int32_t s, const double* const* S,
                      const int32_t* rho, const double* const* Y,
                      const int32_t* rx, const double* const* X,
                      const ttsg_sgmres_opts* opts,
                      double* const* x, int32_t* x_r,
                      ttsg_sgmres_info* info,
                      void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* TT-sPGMRES (Alg. 5) and the other solve options                            */
/* ------------------------------------------------------------------------- */
/* Exponential-sum right preconditioner (Sec. 4.1):
 *   P^{-1} = sum_{j<zeta} alpha_j (x)_k exp(-beta_j M_k)  ~  (M_1 (+) .. (+) M_d)^{-1}.
 * With it the iteration runs on A P^{-1} (Alg. 5): A P^{-1} v_k is never formed;
 * its Khatri-Rao sketch, STTA sketch and inner products are sums over the zeta
 * terms alpha_j A ((x)_k exp(-beta_j M_k) v_k), each an operator-fused sweep
 * over v_k with its modes multiplied (ranks unchanged).  A cycle's recovered
 * correction u enters the solution as x += P^{-1} u, formed by the same STTA
 * streaming sum and rounded at final_tol.  The mode factors are computed once
 * per solve on the GPU (scaling and squaring, FP64 matrix cores). */
typedef struct {
    /* initial guess x0 (x0 == NULL: x0 = 0): d DEVICE pointers, HOST ranks
       x0_r[d+1], each rank <= rx; r0 = b - A x0 and the solution is x0 plus
       the corrections (for Alg. 5, x0 guesses x itself, not P x). */
    const int32_t* x0_r;
    const double* const* x0;
    /* preconditioner (zeta == 0: none).  alpha, beta: HOST arrays of zeta
       values, beta ascending and >= 0 (ttsg_expsum gives both); M: d DEVICE
       pointers to the n[k] x n[k] row-major mode matrices of the Kronecker
       sum.  Signs of alpha are free (e.g. alpha < 0 preconditions -M). */
    int32_t zeta;
    const double* alpha;
    const double* beta;
    const double* const* M;
    /* least-squares form: TTSG_LS_PINV (default) or TTSG_LS_WHITEN */
    int32_t ls_mode;
    /* final solution of a cycle: TTSG_VARIANT_ENHANCED (default; the STTA
       sketches of the basis combined once and recovered, Sec. 3.5) or
       TTSG_VARIANT_VANILLA (Alg. 3: every basis vector of the cycle is kept and
       x = Round(x + y_i v_i, final_tol) term by term) */
    int32_t variant;
    /* 0 (default): independent steps of an iteration (the Khatri-Rao column,
       the coefficients h, the two halves of the STTA sketch) run on three
       streams of the library's own beside the caller's, joined by events;
       1: every launch goes to the caller's stream, in program order (same
       results bit for bit; slower, but each launch has the GPU to itself,
       which is what per-launch timing and profiling want) */
    int32_t single_stream;
} ttsg_sgmres_ext;

/* ttsg_sgmres_solve with the options above (ext == NULL: plain Alg. 4).
 * Same arguments, ownership, synchronization and return values. */
int ttsg_sgmres_solve_ex(int32_t d, const int32_t* n,
                         const int32_t* R, const double* const* A,
                         const int32_t* rb, const double* const* b,
                         int32_t s, const double* const* S,
                         const int32_t* rho, const double* const* Y,
                         const int32_t* rx, const double* const* X,
                         const ttsg_sgmres_opts* opts, const ttsg_sgmres_ext* ext,
                         double* const* x, int32_t* x_r,
                         ttsg_sgmres_info* info,
                         void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* Bytes of workspace ttsg_sgmres_solve_ex needs for these shapes and options
 * (the pointers may be NULL: only sizes are read).  Passing a workspace of at
 * least this size makes the solve allocate no device memory.  Returns 0 and
 * writes *bytes, or a negative error. */
int ttsg_sgmres_workspace_size(int32_t d, const int32_t* n, const int32_t* R, const int32_t* rb, int32_t s,
                               const int32_t* rho, const int32_t* rx, const ttsg_sgmres_opts* opts,
                               const ttsg_sgmres_ext* ext, size_t* bytes);

/* Many independent systems (Alg. 4, or Alg. 5 with a preconditioner in `ext`,
 * on each), solved concurrently on one GPU.  Each entry carries exactly the
 * arguments of ttsg_sgmres_solve_ex (same meaning, layout and ownership);
 * `status` receives that system's return value.
 * Systems are taken longest-first by `concurrency` host workers (<= 0: 8),
 * each driving its own non-blocking stream of default priority, so the
 * kernels of different systems overlap on the GPU while each system's host
 * rank decisions proceed independently.  All worker streams first wait for
 * the work queued on `stream`.  Returns 0 when every system returned >= 0,
 * else the first negative code (ttsg_last_error names the system).  Returns
 * after every system has finished. */
typedef struct {
    int32_t d;
    const int32_t* n;
    const int32_t* R;
    const double* const* A;
    const int32_t* rb;
    const double* const* b;
    int32_t s;
    const double* const* S;
    const int32_t* rho;
    const double* const* Y;
    const int32_t* rx;
    const double* const* X;
    const ttsg_sgmres_opts* opts;
    double* const* x;
    int32_t* x_r;
    ttsg_sgmres_info* info;
    int32_t status;
    /* options of ttsg_sgmres_solve_ex (initial guess, preconditioner of Alg. 5,
       least-squares form, final-solution variant); NULL: plain Alg. 4 */
    const ttsg_sgmres_ext* ext;
} ttsg_system;

int ttsg_sgmres_solve_batched(int32_t count, ttsg_system* systems, int32_t concurrency,
                              ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* TT-GMRES (Alg. 2): the deterministic method the sketched one is compared   */
/* with (Sec. 5.2).                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t maxit;       /* Arnoldi steps (no restart) */
    int32_t maxrank;     /* cap of every basis and solution rank (0 = the full
                            bond ranks min(prod n_<b, prod n_>=b)); it also sizes
                            the workspace, which grows as (maxit+1) basis vectors */
    double tol;          /* stop when the Arnoldi residual <= tol ||b|| */
    double final_tol;    /* rounding tolerance of the sequential solution sums
                            (0 = tol) */
    double max_round;    /* cap of the relaxed rounding tolerance eta_k tol
                            (eta_k = tol / relative residual of step k-1); the
                            usual value is 0.1 */
} ttsg_gmres_opts;

/* Solve A x = b (x_0 = 0) by TT-GMRES: full modified Gram-Schmidt, TT-SVD
 * rounding of A v_k and after every Gram-Schmidt step at the relaxed
 * tolerance (Sec. 2.3), Givens reduction of the Hessenberg least-squares
 * problem (eq. argmin2), x = Round(x + y_i v_i, final_tol) term by term.
 * x: d DEVICE pointers with capacity c_k x n_k x c_{k+1}, c_b = the rank cap of
 * bond b; x_r: HOST int32[d+1].  info (may be NULL): iterations, status,
 * sketched_residual = the final Arnoldi residual / ||b||, true_residual = the
 * FP64 ||b - A x|| / ||b|| (block TT, orthogonalization norm),
 * sketched_history / rank_history per step when given (length >= maxit).
 * Returns TTSG_OK, TTSG_BREAKDOWN, TTSG_NOT_CONVERGED or a negative error.
 * Synchronizes `stream`. */
int ttsg_tt_gmres(int32_t d, const int32_t* n, const int32_t* R, const double* const* A,
                  const int32_t* rb, const double* const* b, const ttsg_gmres_opts* opts,
                  double* const* x, int32_t* x_r, ttsg_sgmres_info* info,
                  void* ws, size_t ws_bytes, ttsg_stream_t stream);
int ttsg_tt_gmres_workspace_size(int32_t d, const int32_t* n, const int32_t* R, const int32_t* rb,
                                 const ttsg_gmres_opts* opts, size_t* bytes);

/* Exponential-sum coefficients (Sec. 4.1) with |z E(z) - 1| <= tol for every
 * z in [zmin, zmax] (0 < zmin <= zmax, 0 < tol < 1), from the trapezoid rule
 * on 1/z = int_R exp(u - e^u z) du (beta_j = e^{u_j}, alpha_j = h e^{u_j}).
 * alpha, beta: HOST arrays of max_terms values.  Returns zeta (the number of
 * terms written), -TTSG_ERR_CAPACITY when max_terms is too small, or
 * -TTSG_ERR_ARG.  Pure host arithmetic; no GPU call. */
int ttsg_expsum(double zmin, double zmax, double tol, int32_t max_terms, double* alpha, double* beta);

/* P^{-1} x for the preconditioner above, rounded by the randomized streaming
 * sum of Sec. 3.3: the STTA sketches of the zeta TTs alpha_j (x)_k
 * exp(-beta_j M_k) x are summed, recovered (pseudo-inverse cutoff rcond) and
 * TT-SVD rounded at relative tol with ranks capped at maxrank (0 = rx only).
 * Shapes as ttsg_round_rand; out cores have capacity rx[k] x n[k] x rx[k+1];
 * out_r: HOST int32[d+1].  Synchronizes `stream`. */
int ttsg_precond_round(int32_t d, const int32_t* n, int32_t zeta, const double* alpha, const double* beta,
                       const double* const* M, const int32_t* r, const double* const* x,
                       const int32_t* rho, const double* const* Y, const int32_t* rx, const double* const* X,
                       double tol, int32_t maxrank, double rcond, double* const* out, int32_t* out_r,
                       void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* FP64 true residual ||b - A x|| / ||b|| through TT arithmetic on the GPU
 * (b - A x formed as a TT, its norm taken after QR orthogonalization).
 * Synchronizes `stream`; result in *res. */
int ttsg_true_residual(int32_t d, const int32_t* n,
                       const int32_t* R, const double* const* A,
                       const int32_t* rb, const double* const* b,
                       const int32_t* r, const double* const* x,
                       double* res, void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* <x, y> by a left-to-right environment sweep (Sec. 2.2).  Synchronizes. */
int ttsg_dot(int32_t d, const int32_t* n, const int32_t* rxr, const double* const* x,
             const int32_t* ryr, const double* const* y, double* out,
             void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Differentiation of a Kronecker-sum solve                                   */
/* ------------------------------------------------------------------------- */
/* For A(theta) = sum_k theta_k (I x .. x L_k x .. x I) and the adjoint state
 * lambda = A^-T dLoss/dx, dLoss/dtheta_k = -<lambda, L_k x>.  All d values come
 * from one left and one right environment sweep of <lambda, x> plus one local
 * contraction per mode: g_k = E_k . (lambda_k, L_k x_k) . F_{k+1}.
 * L: d DEVICE pointers to n[k] x n[k] row-major matrices (the unscaled L_k);
 * out: HOST double[d] receives -<lambda, L_k x>.  Synchronizes `stream`. */
int ttsg_grad_kron_sum(int32_t d, const int32_t* n, const double* const* L,
                       const int32_t* rl, const double* const* lam,
                       const int32_t* rx, const double* const* x,
                       double* out, void* ws, size_t ws_bytes, ttsg_stream_t stream);

/* z = alpha x + beta y as a TT with block cores (ranks add; Sec. 2.2).
 * z cores have shape (rx[k]+ry[k]) x n[k] x (rx[k+1]+ry[k+1]) for 0 < k < d-1,
 * 1 x n x (rx[1]+ry[1]) first and (rx[d-1]+ry[d-1]) x n x 1 last (d = 1: n).
 * Does not synchronize. */
int ttsg_tt_axpby(int32_t d, const int32_t* n, double alpha, const int32_t* rx, const double* const* x,
                  double beta, const int32_t* ry, const double* const* y, double* const* z,
                  ttsg_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Contraction tile autotuner.  Every contraction runs one of four tile      */
/* variants of the matrix-core kernel (64x64, 32x64, 64x32 or 32x32 entries  */
/* of C per workgroup); all of them sum in the same order, so the choice     */
/* never changes a result bit.  While tuning is on, the first contraction of */
/* each new shape class (precision; log2 of M, N, K and batch; split-K or    */
/* not; which operands have unit-stride reductions) times the four variants */
/* on that call's operands (output to a scratch buffer, one stream sync) and */
/* keeps the fastest.  Untuned classes use 32-wide tiles along dimensions    */
/* <= 32 and 64-wide ones otherwise.                                         */
/* ------------------------------------------------------------------------- */
/* on != 0 starts tuning new classes, 0 stops; returns the previous setting. */
int ttsg_autotune(int32_t on);
/* Write the table as text (one line per class); returns the entry count or  */
/* -TTSG_ERR_ARG when the file cannot be written.                            */
int ttsg_autotune_save(const char* path);
/* Merge a saved table; returns the entries read or -TTSG_ERR_ARG.           */
int ttsg_autotune_load(const char* path);
/* Forget every tuned class; returns how many there were.                    */
int ttsg_autotune_clear(void);

/* ------------------------------------------------------------------------- */
/* Measurement: per-kernel-class counters.  While enabled, every contraction */
/* and factorization launch records on the GPU the wall-clock time at which  */
/* its first workgroup started and its last one ended (one small device slot */
/* per launch); ttsg_stats_read synchronizes the device and returns, per     */
/* class, the launch count, the algorithmic flops (2*M*N*K*batch per         */
/* contraction; the textbook counts for QR; for a Jacobi launch one sweep's  */
/* rotations times the sweeps it ran, its slowest matrix's count), the operand */
/* bytes (A + B + C, an operand shared across a batch counted once) and the  */
/* summed kernel durations.  It is meant for benchmarking: each launch pays  */
/* two extra atomics per workgroup.                                           */
/* ------------------------------------------------------------------------- */
/* TTSG_ST_QR_REDO counts (in `launches` only) Cholesky-QR factorizations of */
/* the TT-SVD that were rejected as inaccurate and redone by Householder QR. */
enum { TTSG_ST_CONTRACT_F64 = 0, TTSG_ST_CONTRACT_F32 = 1, TTSG_ST_CONTRACT_BF16 = 2,
       TTSG_ST_QR = 3, TTSG_ST_SVD = 4, TTSG_ST_QR_REDO = 5, TTSG_ST_CLASSES = 8 };

typedef struct {
    int64_t launches[TTSG_ST_CLASSES];
    double flops[TTSG_ST_CLASSES];
    double bytes[TTSG_ST_CLASSES];
    double seconds[TTSG_ST_CLASSES];   /* sum of the launches' durations */
    double busy[TTSG_ST_CLASSES];      /* time during which at least one launch of the
                                          class ran (union of their intervals): below
                                          `seconds` when launches overlap on streams */
} ttsg_stats;

/* on != 0: clear the counters and start recording; on == 0: stop recording. */
int ttsg_stats_enable(int32_t on);
/* Synchronize the device, resolve the recorded slots into *out and clear.
 * When the environment variable TTSG_SHAPE_LOG names a file, one line per
 * measured launch is appended to it: class, M, N, K, batch, split count (0s
 * for non-contractions), seconds, flops, auxiliary maximum (Jacobi sweeps). */
int ttsg_stats_read(ttsg_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* TTSG_H */
