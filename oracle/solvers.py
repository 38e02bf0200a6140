"""Krylov solvers in TT format (Alg. 2, Alg. 3, Alg. 4 of the paper).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

`tt_gmres`         Alg. 2 (TT-GMRES): Arnoldi with full modified Gram-Schmidt,
                   TT-SVD rounding after A v_k and after every Gram-Schmidt
                   step at eta_k * tol with eta_k = tol / (relative residual of
                   the previous step), Hessenberg least squares (eq. argmin2),
                   final solution by sequential rounded sums.
`tt_sgmres`        Alg. 4 (enhanced TT-sGMRES), and with `variant="vanilla"`
                   the final sum of Alg. 3; `rounding="svd"` gives the
                   deterministic twin (explicit sums + TT-SVD in place of STTA);
                   `precond=(alpha, E)` gives TT-sPGMRES (Alg. 5) with an
                   exponential-sum right preconditioner (Sec. 4.1) and the
                   rank cap of Sec. 4.2; `ls="whiten"` computes y from the
                   sketched Arnoldi relation (Sec. 3.4) instead of eq. pseudo_inv.

Readings of the text used here (the paper is silent or inconsistent):
  * the combination of sketches inside the loop is
      Psi~ = Psi(A v_k) - sum_{i=max(1,k-q+1)}^{k} h_{i,k} Psi^(i)   (same for Omega),
    i.e. the sketch of A v_k minus the window terms (the printed combination
    repeats h_{1,k} and omits the sketch of A v_k itself);
  * h_{i,k} = <A v_k, v_i> with the Euclidean inner product, all taken from the
    unmodified A v_k (classical Gram-Schmidt, as the enhanced algorithm writes it);
  * STTA_Recover(., tol) recovers at the sketch ranks and then applies TT-SVD
    rounding at the given relative tolerance with the rank cap;
  * stopping: the sketched residual ||W_k y_k - S r0|| is compared with
    stop_safety * tol * ||S b||; after the final solution is formed the true
    residual ||b - A x|| / ||b|| decides, and if it is still above tol a new
    cycle starts from r0 = b - A x (restart, Sec. 3.4), reusing S, X and Y;
  * x_0 = 0 unless given; restart cycles of length `restart` (0 = maxit);
  * preconditioned (Alg. 5): x_0 is a guess of x itself (r0 = b - A x0) and each
    cycle's recovered correction u enters as x += P^{-1} u;
  * whitening (Sec. 3.4): the last row of the projected matrix is
    tau_{k+1} h_{k+1,k} / tau_k e_k^T, the value that makes
    S A V_k T_k^{-1} = Q_{k+1} [..] an identity when the Arnoldi relation holds
    (the printed [0, ..., 0, h_{k+1,k}] drops the factor tau_{k+1} / tau_k).

Parity status: iteration counts and ranks of the randomized method depend on the
sketch draw and on rounding order; they are compared as distributions/properties,
not exactly ("parity unpinned" for those two quantities).  The solution itself is
pinned by the closed forms (tests/test_oracle_solvers.py).
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import sketch as skm
from . import tt as ttm

Cores = List[np.ndarray]


def true_residual(A: Cores, b: Cores, x: Cores) -> float:
    """||b - A x|| / ||b|| formed as an explicit TT and measured by orthogonalization."""
    r = ttm.add(b, ttm.matvec(A, x), 1.0, -1.0)
    return ttm.norm(r) / ttm.norm(b)


def residual_tt(A: Cores, b: Cores, x: Optional[Cores], tol: float) -> Cores:
    if x is None:
        return ttm.copy(b)
    r = ttm.add(b, ttm.matvec(A, x), 1.0, -1.0)
    return ttm.round_svd(r, tol)


# ----------------------------------------------------------------------------
# Alg. 2: TT-GMRES
# ----------------------------------------------------------------------------

def tt_gmres(A: Cores, b: Cores, maxit: int, tol: float, x0: Optional[Cores] = None,
             final_tol: Optional[float] = None, max_round: float = 1e-1):
    final_tol = tol if final_tol is None else final_tol
    nb = ttm.norm(b)
    r0 = residual_tt(A, b, x0, 1e-14)
    beta = ttm.norm(r0)
    V = [ttm.scale(r0, 1.0 / beta)]
    H = np.zeros((maxit + 1, maxit))
    res_rel = beta / nb
    hist, rank_hist = [], []
    y = np.zeros(0)
    k = 0
    for k in range(1, maxit + 1):
        eta = tol / max(res_rel, tol)
        rt = min(eta * tol, max_round)
        w = ttm.round_svd(ttm.matvec(A, V[k - 1]), rt)
        for i in range(k):
            H[i, k - 1] = ttm.dot(w, V[i])
            w = ttm.round_svd(ttm.add(w, V[i], 1.0, -H[i, k - 1]), rt)
        H[k, k - 1] = ttm.norm(w)
        rhs = np.zeros(k + 1)
        rhs[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
        res = np.linalg.norm(H[:k + 1, :k] @ y - rhs)
        res_rel = res / nb
        hist.append(res_rel)
        rank_hist.append(max(ttm.ranks(w)))
        if res <= nb * tol or H[k, k - 1] == 0.0:
            break
        V.append(ttm.scale(w, 1.0 / H[k, k - 1]))
    x = ttm.copy(x0) if x0 is not None else None
    for i in range(len(y)):
        term = ttm.scale(V[i], y[i])
        x = term if x is None else ttm.round_svd(ttm.add(x, term), final_tol)
    return x, {"iterations": k, "residuals": hist, "max_ranks": rank_hist}


# ----------------------------------------------------------------------------
# Alg. 4 (enhanced TT-sGMRES); Alg. 3 final sum with variant="vanilla"
# ----------------------------------------------------------------------------

def _lin_comb_round(coeffs, vecs, tol, maxrank):
    return ttm.round_svd(ttm.lin_comb(coeffs, vecs), tol, maxrank)


def _whiten_solve(SV: np.ndarray, Hk: np.ndarray, beta_s: float):
    """y_k from eq. sketched_argmin2 and the residual of eq. sketched_residualnorm.

    SV = [S v_1, ..., S v_m] (s x m), Hk = the m x k Hessenberg matrix of the
    incomplete Arnoldi process (m = k + 1; m = k after a breakdown, when the
    Krylov space is invariant and S A V_k = S V_k H_k).  With the skinny QR Q T = S V (positive
    diagonal), S A V_k = Q_{k+1} (T_{k+1} H_k) when the Arnoldi relation holds, so
    y = argmin || T_{k+1} H_k y - beta e_1 ||, beta = ||S r0|| (S r0 = beta q_1).
    In the paper's notation T_{k+1} H_k T_k^{-1} = [H^ + h^ e_k^T; row], and
    solving for z = T_k y and back-substituting is the same problem."""
    m = Hk.shape[0]
    Q, T = np.linalg.qr(SV[:, :m])
    sg = np.sign(np.diag(T))
    sg[sg == 0] = 1.0
    T = sg[:, None] * T
    G = T @ Hk
    rhs = np.zeros(m)
    rhs[0] = beta_s
    y = np.linalg.lstsq(G, rhs, rcond=None)[0]
    return y, float(np.linalg.norm(G @ y - rhs))


def tt_sgmres(A: Cores, b: Cores, S: List[np.ndarray], X: Cores, Y: Cores, *,
              maxit: int, tol: float, q: int = 1, round_tol: float = 1e-7,
              maxrank: Optional[int] = None, stop_safety: float = 0.1,
              restart: int = 0, final_tol: Optional[float] = None,
              rounding: str = "stta", variant: str = "enhanced",
              rcond: float = 1e-12, x0: Optional[Cores] = None,
              track_true_residual: bool = False, max_cycles: int = 50,
              fixed_iterations: Optional[int] = None, keep_basis: bool = False,
              precond=None, ls: str = "pinv", final_rcond: Optional[float] = None,
              solution: bool = True):
    """Sketched TT-GMRES.  Returns (x, info).

    rounding: "stta" (Alg. 4: randomized streaming rounding through STTA) or
              "svd" (deterministic twin: explicit TT sums + TT-SVD rounding).
    variant:  "enhanced" (final solution from the combined sketches, Sec. 3.5) or
              "vanilla" (final solution by sequential rounded sums, Alg. 3).
    fixed_iterations: run exactly this many iterations in one cycle (no stopping
              test), for experiments that fix the iteration count.
    keep_basis: also return the last cycle's basis vectors, their STTA sketches,
              W_k and S r0 in info (for experiments that rebuild the solution of
              every iteration count, e.g. the vanilla/enhanced comparison of Sec. 5.2.1).
    precond:  (alpha, E) of an exponential-sum right preconditioner
              P^{-1} = sum_j alpha_j (x)_k E[j][k] (Sec. 4.1; oracle.precond): this
              is TT-sPGMRES (Alg. 5).  A v_k becomes A P^{-1} v_k, formed as the
              zeta terms alpha_j A ((x)_k E[j][k] v_k) whose sketches, inner
              products and Khatri-Rao columns are summed (all three are linear,
              Sec. 3.3), never as one TT; each cycle's correction u is mapped back
              as x += Round(P^{-1} u) (block sum of the zeta terms, TT-SVD at final_tol).
              x0 is an initial guess of x itself: r0 = b - A x0.
    ls:       "pinv" (y from the pseudo-inverse of W_k, eq. pseudo_inv) or
              "whiten" (Sec. 3.4: skinny QR of S V_{k+1}, y from the sketched
              Arnoldi relation, eq. sketched_argmin2, residual from
              eq. sketched_residualnorm; W_k is not formed).
    final_rcond: pseudo-inverse cutoff of the final solution's recovery
              (default rcond).
    solution: False stops after the first cycle's iterations, before the
              final solution is formed (x is then None): for comparisons of the
              iteration's own quantities at sizes where forming x is costly."""
    final_tol = round_tol if final_tol is None else final_tol
    final_rcond = rcond if final_rcond is None else final_rcond
    nb = ttm.norm(b)
    Sb = np.linalg.norm(skm.kr_sketch(S, b))
    cycle_len = restart if restart > 0 else maxit
    if fixed_iterations is not None:
        cycle_len = fixed_iterations
    x = ttm.copy(x0) if x0 is not None else None
    info = {"iterations": 0, "sketched_residuals": [], "max_ranks": [], "true_residuals": [],
            "cycles": 0, "h": [], "y": None}

    def op_terms(v):
        """TTs whose sum is A v (A P^{-1} v with a preconditioner), unrounded."""
        if precond is None:
            return [ttm.matvec(A, v)]
        from .precond import precond_terms
        alpha, E = precond
        return [ttm.matvec(A, t) for t in precond_terms(alpha, E, v)]

    total = 0
    while total < maxit and info["cycles"] < max_cycles:
        info["cycles"] += 1
        r0 = residual_tt(A, b, x, 1e-12)
        beta = ttm.norm(r0)
        if beta == 0.0:
            break
        Sr0 = skm.kr_sketch(S, r0)
        window: List[Cores] = [ttm.scale(r0, 1.0 / beta)]
        basis: List[Cores] = [window[0]]            # kept only for the vanilla/svd final sums
        sk = [skm.stta_sketch(window[0], X, Y)] if rounding == "stta" else None
        W = []
        SV = [skm.kr_sketch(S, window[0])] if ls == "whiten" else None
        H = np.zeros((cycle_len + 1, cycle_len))
        y = np.zeros(0)
        k = 0
        for k in range(1, cycle_len + 1):
            vk = window[-1]
            terms = op_terms(vk)                                # no truncation of A v_k
            if ls == "pinv":
                W.append(sum(skm.kr_sketch(S, t) for t in terms))
            lo = max(1, k - q + 1)
            idx = list(range(lo, k + 1))
            hs = [sum(ttm.dot(t, basis[i - 1] if rounding == "svd" or variant == "vanilla"
                              else window[len(window) - (k - i) - 1]) for t in terms) for i in idx]
            info["h"].append(hs)
            if rounding == "stta":
                tsk = [skm.stta_sketch(t, X, Y) for t in terms]
                comb = [(1.0, s_) for s_ in tsk] + [(-h, sk[i - 1]) for h, i in zip(hs, idx)]
                Psi, Om = skm.lin_comb_sketches([c for c, _ in comb], [s_ for _, s_ in comb])
                wt = ttm.round_svd(skm.stta_recover(Psi, Om, rcond), round_tol, maxrank)
            else:
                vecs = terms + [basis[i - 1] for i in idx]
                wt = _lin_comb_round([1.0] * len(terms) + [-h for h in hs], vecs, round_tol, maxrank)
            hk = ttm.norm(wt)
            for h, i in zip(hs, idx):
                H[i - 1, k - 1] = h
            H[k, k - 1] = hk
            if ls == "pinv":
                Wk = np.array(W).T
                y = np.linalg.lstsq(Wk, Sr0, rcond=None)[0]
                res = np.linalg.norm(Wk @ y - Sr0)
            else:
                if hk > 0.0:
                    SV.append(skm.kr_sketch(S, ttm.scale(wt, 1.0 / hk)))
                    y, res = _whiten_solve(np.array(SV).T, H[:k + 1, :k], np.linalg.norm(Sr0))
                else:
                    y, res = _whiten_solve(np.array(SV).T, H[:k, :k], np.linalg.norm(Sr0))
            info["sketched_residuals"].append(res / Sb)
            info["max_ranks"].append(max(ttm.ranks(wt)))
            total += 1
            if fixed_iterations is None and (res <= stop_safety * tol * Sb or hk == 0.0 or total >= maxit):
                break
            if hk == 0.0:
                break
            vnext = ttm.scale(wt, 1.0 / hk)
            window.append(vnext)
            if len(window) > q:
                window.pop(0)
            basis.append(vnext)
            if rounding == "stta":
                sk.append(skm.stta_sketch(vnext, X, Y))
        info["iterations"] = total
        info["y"] = y
        if not solution:
            break
        if keep_basis:
            info["basis"], info["sketches"] = basis, sk
            info["W"], info["Sr0"] = (np.array(W).T if W else None), Sr0
        # final solution of this cycle
        m = len(y)
        if variant == "vanilla":
            corr = None
            for i in range(m):
                term = ttm.scale(basis[i], y[i])
                corr = term if corr is None else ttm.round_svd(ttm.add(corr, term), final_tol)
        elif rounding == "stta":
            Psi, Om = skm.lin_comb_sketches(list(y), sk[:m])
            corr = ttm.round_svd(skm.stta_recover(Psi, Om, final_rcond), final_tol, maxrank)
        else:
            corr = _lin_comb_round(list(y), basis[:m], final_tol, None)
        if precond is not None:
            from .precond import apply_precond
            corr = apply_precond(precond[0], precond[1], corr, final_tol)
        x = corr if x is None else ttm.round_svd(ttm.add(x, corr), final_tol)
        tr = true_residual(A, b, x)
        info["true_residuals"].append(tr)
        if tr <= tol or fixed_iterations is not None:
            break
    info["true_residual"] = info["true_residuals"][-1] if info["true_residuals"] else None
    return x, info
