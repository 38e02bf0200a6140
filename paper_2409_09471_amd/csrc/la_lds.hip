// LDS-resident FP64 factorizations: batched one-sided Jacobi SVD and the
// leaf kernels of a tall-skinny QR (TSQR) tree.
//
// Jacobi: one workgroup (16 wavefronts) per matrix; the m x c matrix and the
// c x c rotation accumulator live in LDS, so every rotation reads and writes
// LDS instead of global memory.  Pairs of a round (circle method) go to
// different wavefronts; a pair's three dot products are wavefront reductions.
//
// TSQR: the rows of a tall m x c matrix are split into leaves of at most 256
// rows (and at least c); each leaf is factored by Householder QR in LDS; the c x c
// R factors are stacked and factored again until one leaf remains.  Q is never
// formed: tsqr_apply multiplies Q by a small c x k matrix from the root down,
// each leaf applying its reflectors (read once per column from global memory
// into LDS) to its slice.
#include <algorithm>

#include <mutex>

#include "tt_ops.h"
#include "xlane.h"

namespace ttsg {
namespace {

constexpr int JT = 512;    // threads of the Jacobi workgroup (32 lane groups of 16)
constexpr int QT = 1024;   // threads of the QR leaf workgroups
constexpr int LEAF = 256;  // maximum rows of a TSQR leaf


struct JacobiBatch {
    int count;
    int m[32], c[32], lda[32];
    double tol[32];
    double drop_abs2[32], drop_rel2[32];
    double* A[32];
    double* V[32];
    double* sig[32];
    // 128-column kernel with an accumulator: the rotation log (the tangent of
    // every rotation, 0 for none, per sweep, round and pair) and meta =
    // [active-column permutation (c), output rank of each column (c), active
    // columns, sweeps run], from which k_jacobi_apply_v forms V
    double* rot[32];
    int* meta[32];
};


// One-sided Jacobi with one lane group of JG lanes per column pair: the group
// forms the pair's three dot products over its strided rows, reduces them in
// registers, and rotates the same rows, so a round of the circle method costs
// a single barrier.  The pairs of every round come from a table built once.
constexpr int JG = 16;
constexpr int JROWS = 8;   // rows of a column held per lane: m <= JG * JROWS (kernel JR <= JROWS)

// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// each (the estimates carry about half the double mantissa; each step doubles
// the correct bits).  Shorter dependency chains than IEEE division and sqrt.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    r = r * fma(-h, r * r, 1.5);
    r = r * fma(-h, r * r, 1.5);
    return r;
}
template <int JR>
__global__ __launch_bounds__(JT) void k_jacobi_lds(JacobiBatch jb, int maxsweeps, DevSlot* slot) {
    extern __shared__ double lds[];
    slot_begin(slot);
    int sweeps_done = 0;
    __shared__ int s_rot;
    __shared__ unsigned long long s_moff;
    const int bi = blockIdx.x;
    const int m = jb.m[bi], c = jb.c[bi], lda = jb.lda[bi];
    const double tol = jb.tol[bi];
    double* Ag = jb.A[bi];
    double* Vg = jb.V[bi];
    const int ldm = m | 1;
    const int ldv = c | 1;
    double* A = lds;
    double* V = lds + (size_t)ldm * c;
    const int tid = threadIdx.x;
    for (int e = tid; e < m * c; e += blockDim.x) {
        int j = e / m, i = e - j * m;
        A[j * ldm + i] = Ag[(int64_t)j * lda + i];
    }
    for (int e = tid; e < c * c; e += blockDim.x) {
        int j = e / c, i = e - j * c;
        V[j * ldv + i] = (i == j) ? 1.0 : 0.0;
    }
    const int grp = tid / JG, lt = tid - grp * JG;
    const int ngrp = JT / JG;
    __shared__ double s_fpart[JT / 64];
    if (tid == 0) {
        s_rot = 0;
        s_moff = 0ull;
    }
    double s_fro = 0.0;
    {
        // squared Frobenius norm: columns below eps ||A||_F are rounding noise.
        // Wave partials are summed in wave order (the same bits every run).
        double f = 0.0;
        for (int e = tid; e < m * c; e += blockDim.x) {
            int j = e / m, i = e - j * m;
            f += A[j * ldm + i] * A[j * ldm + i];
        }
        f = wave_sum64(f);
        if ((tid & 63) == 0) s_fpart[tid >> 6] = f;
        __syncthreads();
        for (int w = 0; w < JT / 64; ++w) s_fro += s_fpart[w];
    }
    // columns below 2 m eps ||A||_F carry only rounding noise (null space of a
    // rank-deficient matrix); their mutual dot products never look orthogonal,
    // so they are treated as converged
    const double nz = 2.0 * m * 2.220446049250313e-16;
    const double tiny0 = nz * nz * s_fro;
    const double tol2 = tol * tol;
    // columns that the caller discards anyway take part in no rotation
    __shared__ double s_cn[64];
    __shared__ unsigned long long s_cmax;
    __shared__ int s_perm[64];
    __shared__ int s_cact;
    if (tid == 0) s_cmax = 0ull;
    __syncthreads();
    for (int l = grp; l < c; l += ngrp) {
        double s2 = 0.0;
        for (int i = lt; i < m; i += JG) s2 += A[l * ldm + i] * A[l * ldm + i];
        s2 = row_sum16(s2);
        if (lt == 0) {
            s_cn[l] = s2;
            // non-negative doubles order like their bit patterns
            atomicMax(&s_cmax, (unsigned long long)__double_as_longlong(s2));
        }
    }
    __syncthreads();
    double drop2 = jb.drop_abs2[bi];
    if (jb.drop_rel2[bi] > 0.0) drop2 = fmax(drop2, jb.drop_rel2[bi] * __longlong_as_double((long long)s_cmax));
    const double tiny = fmax(tiny0, drop2);
    // The columns that can rotate go first (in index order), the ones at or
    // below the threshold after them: the rounds then run over the active
    // columns only.  V starts as the permutation, so A V = B still holds.
    if (tid < 64) {
        const bool on = tid < c && s_cn[tid] > tiny;
        const unsigned long long act = __ballot(on);
        const unsigned long long below = (1ull << tid) - 1ull;
        const int nact = __popcll(act);
        if (tid < c) {
            const unsigned long long valid = c >= 64 ? ~0ull : ((1ull << c) - 1ull);
            const int pos = on ? __popcll(act & below) : nact + __popcll(~act & valid & below);
            s_perm[pos] = tid;
        }
        if (tid == 0) s_cact = nact;
    }
    __syncthreads();
    const int c_act = s_cact;
    if (c_act < c) {
        for (int e = tid; e < m * c; e += blockDim.x) {
            const int j = e / m, i = e - j * m;
            A[j * ldm + i] = Ag[(int64_t)s_perm[j] * lda + i];
        }
        for (int e = tid; e < c * c; e += blockDim.x) {
            const int j = e / c, i = e - j * c;
            V[j * ldv + i] = (i == s_perm[j]) ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    const int cp = c_act + (c_act & 1);
    const int npair = cp / 2;
    const int nround = cp - 1;
    for (int sweep = 0; sweep < maxsweeps && cp > 1; ++sweep) {
        int rotated = 0;
        double mo2 = 0.0;   // largest squared |cos| between a pair's columns met in this sweep
        sweeps_done = sweep + 1;
        // circle method, pair k = grp of round r (c <= 64: one pair per lane
        // group): k = 0 pairs the fixed column cp-1 with r; k > 0 pairs
        // (r + k, r - k) mod cp-1; both indices advance by one per round
        int p = grp == 0 ? cp - 1 : grp, q = grp == 0 ? 0 : cp - 1 - grp;
        for (int r = 0; r < nround; ++r) {
            if (grp < npair && p < c_act && q < c_act) {
                double* ap = A + p * ldm;
                double* aq = A + q * ldm;
                double* vp = V + p * ldv;
                double* vq = V + q * ldv;
                // the pair's rows stay in registers between the dot products
                // and the rotation (m <= JG * JR); the rotation accumulator's
                // columns are read with them so their latency overlaps
                double xp[JR], xq[JR], yp[4], yq[4];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int t = 0; t < JR; ++t) {
                    const int i = lt + t * JG;
                    xp[t] = 0.0;
                    xq[t] = 0.0;
                    if (i < m) {
                        xp[t] = ap[i];
                        xq[t] = aq[i];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = lt + u * JG;
                    const int ic = i < c ? i : 0;   // in-range index even where unused
                    yp[u] = i < c ? vp[ic] : 0.0;
                    yq[u] = i < c ? vq[ic] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < JR; ++t) {
                    al += xp[t] * xp[t];
                    be += xq[t] * xq[t];
                    ga += xp[t] * xq[t];
                }
                al = row_sum16(al);
                be = row_sum16(be);
                ga = row_sum16(ga);
                const double g2 = ga * ga, ab = al * be;
                if (al > tiny && be > tiny) {
                    mo2 = fmax(mo2, g2 * rcp_nr(ab));    // squared |cos| (off the rotation's path)
                    if (g2 > tol2 * ab) {
                        // rotation angle: with dd = be - al, t = tan(theta) =
                        // 2 ga sign(dd) / (|dd| + sqrt(dd^2 + 4 ga^2)) (the smaller root of
                        // t^2 + (dd / ga) t - 1 = 0); c = 1 / sqrt(1 + t^2), s = c t
                        const double dd = be - al;
                        const double qq = fma(dd, dd, 4.0 * g2);
                        double t = 2.0 * ga * rcp_nr(fabs(dd) + qq * rsq_nr(qq));
                        if (dd < 0.0) t = -t;
                        const double cs = rsq_nr(fma(t, t, 1.0));
                        const double sn = cs * t;
#pragma unroll
                        for (int u = 0; u < JR; ++u) {
                            const int i = lt + u * JG;
                            if (i < m) {
                                ap[i] = cs * xp[u] - sn * xq[u];
                                aq[i] = sn * xp[u] + cs * xq[u];
                            }
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int i = lt + u * JG;
                            if (i < c) {
                                vp[i] = cs * yp[u] - sn * yq[u];
                                vq[i] = sn * yp[u] + cs * yq[u];
                            }
                        }
                        rotated = 1;
                    }
                }
            }
            if (grp == 0) {
                q += 1;
            } else {
                p = p + 1 == cp - 1 ? 0 : p + 1;
                q = q + 1 == cp - 1 ? 0 : q + 1;
            }
            __syncthreads();
        }
        if (rotated && lt == 0) s_rot = 1;
        // non-negative doubles order like their bit patterns
        if (lt == 0 && mo2 > 0.0) atomicMax(&s_moff, (unsigned long long)__double_as_longlong(mo2));
        __syncthreads();
        const int any = s_rot;      // every thread reads the flags ...
        const double moff = __longlong_as_double((long long)s_moff);
        __syncthreads();            // ... before thread 0 clears them for the next sweep
        if (tid == 0) {
            s_rot = 0;
            s_moff = 0ull;
        }
        // Jacobi converges quadratically near the end: a sweep that started
        // with every |cos| below sqrt(tol) / 10 leaves them near tol, so the
        // confirming sweep without rotations is skipped (moff is squared)
        if (any == 0 || moff < 0.01 * tol) break;
    }
    __syncthreads();
    // singular values = column norms; the output is sorted in descending order
    // (ties by column index), so callers can take leading columns directly
    __shared__ double s_sig[64];
    __shared__ int s_rank[64];
    for (int l = grp; l < c; l += ngrp) {
        const double* al = A + l * ldm;
        double s2 = 0.0;
        for (int i = lt; i < m; i += JG) s2 += al[i] * al[i];
        s2 = row_sum16(s2);
        if (lt == 0) s_sig[l] = sqrt(s2);
    }
    __syncthreads();
    for (int l = tid; l < c; l += blockDim.x) {
        const double v = s_sig[l];
        int rk = 0;
        for (int t = 0; t < c; ++t) rk += (s_sig[t] > v || (s_sig[t] == v && t < l)) ? 1 : 0;
        s_rank[l] = rk;
        jb.sig[bi][rk] = v;
    }
    __syncthreads();
    for (int e = tid; e < m * c; e += blockDim.x) {
        int j = e / m, i = e - j * m;
        Ag[(int64_t)s_rank[j] * lda + i] = A[j * ldm + i];
    }
    for (int e = tid; e < c * c; e += blockDim.x) {
        int j = e / c, i = e - j * c;
        Vg[(int64_t)s_rank[j] * c + i] = V[j * ldv + i];
    }
    slot_end(slot, (unsigned long long)sweeps_done);
}

// One-sided Jacobi for 64 < c <= 128 columns and up to 16 JR rows: 64 lane
// groups of 16 (1024 threads), one column pair per group and round.  The m x c
// matrix fills the LDS (149 x 128 doubles = 149 KB at the largest shape used),
// so there is no room for the rotation accumulator.  When one is asked for
// (ACC), lane 0 of every group logs the tangent of its round's rotation (0 for
// none) and the accumulator is formed afterwards by k_jacobi_apply_v, which
// replays the log on the rows of V in parallel over many workgroups (the rows
// of V are independent).  Without ACC only the rotated matrix B = A V and the
// singular values are produced (callers that need a factor of V form it from
// B).  Norm reductions are fixed-order, so results do not depend on wavefront
// timing.
constexpr int JTB = 1024;
constexpr int JB_CMAX = 128;
constexpr int kJacobiBigSweeps = 30;   // sweep limit of the 128-column kernel

template <int JR, bool ACC>
__global__ __launch_bounds__(JTB) void k_jacobi_big(JacobiBatch jb, int maxsweeps, DevSlot* slot) {
    extern __shared__ double lds[];
    slot_begin(slot);
    int sweeps_done = 0;
    __shared__ int s_rot;
    __shared__ unsigned long long s_moff, s_cmax;
    __shared__ double s_part[JTB / 64];
    __shared__ double s_cn[JB_CMAX], s_sig[JB_CMAX];
    __shared__ int s_perm[JB_CMAX], s_rank[JB_CMAX];
    __shared__ int s_cact;
    __shared__ double s_fro;
    const int bi = blockIdx.x;
    const int m = jb.m[bi], c = jb.c[bi], lda = jb.lda[bi];
    const double tol = jb.tol[bi];
    double* Ag = jb.A[bi];
    double* Vg = jb.V[bi];
    const int ldm = m | 1;
    double* A = lds;
    const int tid = threadIdx.x;
    const int grp = tid / JG, lt = tid - grp * JG;
    for (int e = tid; e < m * c; e += JTB) {
        const int j = e / m, i = e - j * m;
        A[j * ldm + i] = Ag[(int64_t)j * lda + i];
    }
    if (tid == 0) {
        s_rot = 0;
        s_moff = 0ull;
        s_cmax = 0ull;
    }
    __syncthreads();
    // column norms (one lane group per column) and the Frobenius norm as their
    // sum in column order
    for (int l = grp; l < c; l += JTB / JG) {
        double s2 = 0.0;
        for (int i = lt; i < m; i += JG) s2 += A[l * ldm + i] * A[l * ldm + i];
        s2 = row_sum16(s2);
        if (lt == 0) {
            s_cn[l] = s2;
            atomicMax(&s_cmax, (unsigned long long)__double_as_longlong(s2));
        }
    }
    __syncthreads();
    if (tid == 0) {
        double f = 0.0;
        for (int l = 0; l < c; ++l) f += s_cn[l];
        s_fro = f;
    }
    __syncthreads();
    const double nz = 2.0 * m * 2.220446049250313e-16;
    const double tiny0 = nz * nz * s_fro;
    const double tol2 = tol * tol;
    double drop2 = jb.drop_abs2[bi];
    if (jb.drop_rel2[bi] > 0.0) drop2 = fmax(drop2, jb.drop_rel2[bi] * __longlong_as_double((long long)s_cmax));
    const double tiny = fmax(tiny0, drop2);
    // active columns first (index order), the rest after them
    if (tid == 0) {
        int pos = 0;
        for (int l = 0; l < c; ++l)
            if (s_cn[l] > tiny) s_perm[pos++] = l;
        s_cact = pos;
        for (int l = 0; l < c; ++l)
            if (!(s_cn[l] > tiny)) s_perm[pos++] = l;
    }
    __syncthreads();
    const int c_act = s_cact;
    if (c_act < c) {
        for (int e = tid; e < m * c; e += JTB) {
            const int j = e / m, i = e - j * m;
            A[j * ldm + i] = Ag[(int64_t)s_perm[j] * lda + i];
        }
    }
    double* rotg = ACC ? jb.rot[bi] : nullptr;
    if (ACC) {
        int* meta = jb.meta[bi];
        for (int l = tid; l < c; l += JTB) meta[l] = s_perm[l];
        if (tid == 0) meta[2 * c] = c_act;
    }
    (void)Vg;
    __syncthreads();
    const int cp = c_act + (c_act & 1);
    const int npair = cp / 2;
    const int nround = cp - 1;
    for (int sweep = 0; sweep < maxsweeps && cp > 1; ++sweep) {
        int rotated = 0;
        double mo2 = 0.0;
        sweeps_done = sweep + 1;
        int p = grp == 0 ? cp - 1 : grp, q = grp == 0 ? 0 : cp - 1 - grp;
        for (int r = 0; r < nround; ++r) {
            double tlog = 0.0;   // tangent of this group's rotation, 0 for none
            if (grp < npair && p < c_act && q < c_act) {
                double* ap = A + p * ldm;
                double* aq = A + q * ldm;
                double xp[JR], xq[JR];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int t = 0; t < JR; ++t) {
                    const int i = lt + t * JG;
                    xp[t] = 0.0;
                    xq[t] = 0.0;
                    if (i < m) {
                        xp[t] = ap[i];
                        xq[t] = aq[i];
                    }
                }
#pragma unroll
                for (int t = 0; t < JR; ++t) {
                    al += xp[t] * xp[t];
                    be += xq[t] * xq[t];
                    ga += xp[t] * xq[t];
                }
                al = row_sum16(al);
                be = row_sum16(be);
                ga = row_sum16(ga);
                const double g2 = ga * ga, ab = al * be;
                if (al > tiny && be > tiny) {
                    mo2 = fmax(mo2, g2 * rcp_nr(ab));
                    if (g2 > tol2 * ab) {
                        const double dd = be - al;
                        const double qq = fma(dd, dd, 4.0 * g2);
                        double t = 2.0 * ga * rcp_nr(fabs(dd) + qq * rsq_nr(qq));
                        if (dd < 0.0) t = -t;
                        const double cs = rsq_nr(fma(t, t, 1.0));
                        const double sn = cs * t;
#pragma unroll
                        for (int u = 0; u < JR; ++u) {
                            const int i = lt + u * JG;
                            if (i < m) {
                                ap[i] = cs * xp[u] - sn * xq[u];
                                aq[i] = sn * xp[u] + cs * xq[u];
                            }
                        }
                        tlog = t;
                        rotated = 1;
                    }
                }
            }
            if (ACC && grp < npair && lt == 0) rotg[((int64_t)sweep * nround + r) * npair + grp] = tlog;
            if (grp == 0) {
                q += 1;
            } else {
                p = p + 1 == cp - 1 ? 0 : p + 1;
                q = q + 1 == cp - 1 ? 0 : q + 1;
            }
            __syncthreads();
        }
        if (rotated && lt == 0) s_rot = 1;
        if (lt == 0 && mo2 > 0.0) atomicMax(&s_moff, (unsigned long long)__double_as_longlong(mo2));
        __syncthreads();
        const int any = s_rot;
        const double moff = __longlong_as_double((long long)s_moff);
        __syncthreads();
        if (tid == 0) {
            s_rot = 0;
            s_moff = 0ull;
        }
        if (any == 0 || moff < 0.01 * tol) break;
    }
    __syncthreads();
    // singular values = column norms, output sorted in descending order (ties
    // by column index)
    for (int l = grp; l < c; l += JTB / JG) {
        const double* al = A + l * ldm;
        double s2 = 0.0;
        for (int i = lt; i < m; i += JG) s2 += al[i] * al[i];
        s2 = row_sum16(s2);
        if (lt == 0) s_sig[l] = sqrt(s2);
    }
    __syncthreads();
    for (int l = tid; l < c; l += JTB) {
        const double v = s_sig[l];
        int rk = 0;
        for (int t = 0; t < c; ++t) rk += (s_sig[t] > v || (s_sig[t] == v && t < l)) ? 1 : 0;
        s_rank[l] = rk;
        jb.sig[bi][rk] = v;
    }
    __syncthreads();
    for (int e = tid; e < m * c; e += JTB) {
        const int j = e / m, i = e - j * m;
        Ag[(int64_t)s_rank[j] * lda + i] = A[j * ldm + i];
    }
    if (ACC) {
        int* meta = jb.meta[bi];
        for (int l = tid; l < c; l += JTB) meta[c + l] = s_rank[l];
        if (tid == 0) meta[2 * c + 1] = sweeps_done;
    }
    slot_end(slot, (unsigned long long)sweeps_done);
}

// The accumulator V of k_jacobi_big from its rotation log: V starts as the
// active-column permutation, every logged rotation of the circle method is
// applied to the columns (p, q) it rotated, in sweep and round order, and the
// columns are written in the output order.  Rows of V are independent, so a
// workgroup takes JAV_ROWS rows (one lane per row and pair: 16 x 64 = 1024
// lanes), with one barrier per round; the round's tangents are read one round
// ahead.  The pair of group g in round r is the one k_jacobi_big used:
// (cp - 1, r) for g = 0, ((g + r) mod (cp - 1), (cp - 1 - g + r) mod (cp - 1))
// otherwise, cp the active column count rounded up to even.
constexpr int JAV_ROWS = 16;
__global__ __launch_bounds__(JTB) void k_jacobi_apply_v(JacobiBatch jb) {
    __shared__ double v[JAV_ROWS][JB_CMAX + 1];
    const int bi = blockIdx.y;
    const int c = jb.c[bi];
    const int row0 = blockIdx.x * JAV_ROWS;
    if (row0 >= c) return;
    const int* meta = jb.meta[bi];
    const double* rot = jb.rot[bi];
    double* Vg = jb.V[bi];
    const int c_act = meta[2 * c], sweeps = meta[2 * c + 1];
    const int tid = threadIdx.x;
    const int rr = tid / 64, g = tid - (tid / 64) * 64;
    for (int e = tid; e < JAV_ROWS * c; e += JTB) {
        const int k = e / c, j = e - (e / c) * c;
        v[k][j] = (row0 + k == meta[j]) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int cp = c_act + (c_act & 1);
    const int npair = cp / 2, nround = cp - 1;
    const int64_t total = (int64_t)sweeps * nround;
    const bool mine = g < npair && cp > 1;
    double tn = (mine && total > 0) ? rot[g] : 0.0;
    for (int64_t e = 0; e < total; ++e) {
        const double t = tn;
        if (mine && e + 1 < total) tn = rot[(e + 1) * npair + g];
        const int r = (int)(e % nround);
        int p, q;
        if (g == 0) {
            p = cp - 1;
            q = r;
        } else {
            p = (g + r) % (cp - 1);
            q = (cp - 1 - g + r) % (cp - 1);
        }
        if (mine && t != 0.0) {
            const double cs = rsq_nr(fma(t, t, 1.0));
            const double sn = cs * t;
            const double yp = v[rr][p], yq = v[rr][q];
            v[rr][p] = cs * yp - sn * yq;
            v[rr][q] = sn * yp + cs * yq;
        }
        __syncthreads();
    }
    const int* rank = meta + c;
    for (int e = tid; e < JAV_ROWS * c; e += JTB) {
        const int k = e / c, j = e - (e / c) * c;
        if (row0 + k < c) Vg[(int64_t)rank[j] * c + row0 + k] = v[k][j];
    }
}

// Leaf i of a TSQR level: rows [r0, r1) of the column-major m x c matrix A.
__device__ __forceinline__ void leaf_rows(int m, int nleaves, int i, int& r0, int& r1) {
    r0 = (int)(((int64_t)i * m) / nleaves);
    r1 = (int)(((int64_t)(i + 1) * m) / nleaves);
}

// Householder QR of one leaf in LDS.  Step j: one wavefront forms the
// reflector of column j; then every trailing column is owned by a lane group
// of QG lanes that reduces v^T a_l in registers and updates its own rows.
constexpr int QG = 16;
static_assert(QG == 16, "lane groups are DPP rows");
__global__ __launch_bounds__(QT) void k_qr_leaf(int m, int c, const double* __restrict__ A, int lda,
                                                 int nleaves, double* __restrict__ refl, int ldr,
                                                 double* __restrict__ tau, double* __restrict__ Rs, int ldrs,
                                                 DevSlot* slot) {
    extern __shared__ double T[];
    slot_begin(slot);
    __shared__ double s_tau, s_scale;
    const int i = blockIdx.x;
    int r0, r1;
    leaf_rows(m, nleaves, i, r0, r1);
    const int rows = r1 - r0;
    const int ldt = rows | 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int grp = tid / QG, lt = tid - grp * QG, ngrp = QT / QG;
    for (int e = tid; e < rows * c; e += blockDim.x) {
        int j = e / rows, r = e - j * rows;
        T[j * ldt + r] = A[(int64_t)j * lda + r0 + r];
    }
    __syncthreads();
    const int kk = rows < c ? rows : c;
    for (int j = 0; j < kk; ++j) {
        double* col = T + j * ldt;
        if (wave == 0) {
            double sacc = 0.0;
            for (int r = j + 1 + lane; r < rows; r += 64) sacc += col[r] * col[r];
            sacc = wave_sum64(sacc);
            const double alpha = col[j];
            double tt = 0.0, sc = 0.0, beta = alpha;
            if (sacc != 0.0) {
                beta = -copysign(sqrt(alpha * alpha + sacc), alpha);
                tt = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
            for (int r = j + 1 + lane; r < rows; r += 64) col[r] *= sc == 0.0 ? 1.0 : sc;
            if (lane == 0) {
                col[j] = beta;
                s_tau = tt;
                s_scale = sc;
                tau[(int64_t)i * c + j] = tt;
            }
        }
        __syncthreads();
        const double t = s_tau;
        if (t != 0.0) {
            for (int l = j + 1 + grp; l < c; l += ngrp) {
                double* cl = T + l * ldt;
                double w = 0.0;
                for (int r = j + 1 + lt; r < rows; r += QG) w += col[r] * cl[r];
                w = row_sum16(w);
                w = t * (w + cl[j]);
                if (lt == 0) cl[j] -= w;
                for (int r = j + 1 + lt; r < rows; r += QG) cl[r] -= w * col[r];
            }
        }
        __syncthreads();
    }
    for (int j = kk; j < c; ++j)
        if (tid == 0) tau[(int64_t)i * c + j] = 0.0;
    for (int e = tid; e < rows * c; e += blockDim.x) {
        int j = e / rows, r = e - j * rows;
        refl[(int64_t)j * ldr + r0 + r] = T[j * ldt + r];
    }
    // R_i (c x c, zero below the diagonal and below row kk) at rows i*c of the stack
    for (int e = tid; e < c * c; e += blockDim.x) {
        int j = e / c, r = e - j * c;
        Rs[(int64_t)j * ldrs + (int64_t)i * c + r] = (r <= j && r < kk) ? T[j * ldt + r] : 0.0;
    }
    slot_end(slot);
}

// Out (rows of this level x k) = blockdiag(Q_i) [B_i; 0], B_i = rows i*c.. of Bin.
__global__ __launch_bounds__(QT) void k_qr_apply_leaf(int m, int c, int k, const double* __restrict__ refl, int ldr,
                                                       const double* __restrict__ tau, int nleaves,
                                                       const double* __restrict__ Bin, int ldb,
                                                       double* __restrict__ Out, int ldo, int out_rowmajor,
                                                       DevSlot* slot) {
    extern __shared__ double X[];
    slot_begin(slot);
    const int i = blockIdx.x;
    int r0, r1;
    leaf_rows(m, nleaves, i, r0, r1);
    const int rows = r1 - r0;
    const int ldx = rows | 1;
    double* v = X + (size_t)ldx * k;   // the current reflector
    const int tid = threadIdx.x;
    const int grp = tid / QG, lt = tid - grp * QG, ngrp = QT / QG;
    for (int e = tid; e < rows * k; e += blockDim.x) {
        int t = e / rows, r = e - t * rows;
        X[t * ldx + r] = (r < c) ? Bin[(int64_t)t * ldb + (int64_t)i * c + r] : 0.0;
    }
    const int kk = rows < c ? rows : c;
    for (int j = kk - 1; j >= 0; --j) {
        const double tj = tau[(int64_t)i * c + j];
        __syncthreads();
        if (tj == 0.0) continue;
        for (int r = j + 1 + tid; r < rows; r += blockDim.x) v[r] = refl[(int64_t)j * ldr + r0 + r];
        __syncthreads();
        for (int t = grp; t < k; t += ngrp) {
            double* xt = X + t * ldx;
            double w = 0.0;
            for (int r = j + 1 + lt; r < rows; r += QG) w += v[r] * xt[r];
            w = row_sum16(w);
            w = tj * (w + xt[j]);
            if (lt == 0) xt[j] -= w;
            for (int r = j + 1 + lt; r < rows; r += QG) xt[r] -= w * v[r];
        }
    }
    __syncthreads();
    for (int e = tid; e < rows * k; e += blockDim.x) {
        int t = e / rows, r = e - t * rows;
        if (out_rowmajor)
            Out[(int64_t)(r0 + r) * ldo + t] = X[t * ldx + r];
        else
            Out[(int64_t)t * ldo + r0 + r] = X[t * ldx + r];
    }
    slot_end(slot);
}

struct QrBatch {
    int count;
    int m[32], c[32], lda[32];
    const double* A[32];
    double* Q[32];
    double* R[32];
    int* perm[32];   // nullptr: no column pivoting
    int flags[32];   // bit 0: A row-major; bit 1: write R^T
};

// Householder QR of one small matrix per workgroup with the explicit Q:
// the factorization follows k_qr_leaf (one wavefront forms each reflector,
// lane groups of QG update the trailing columns), then the reflectors are
// applied in reverse order to the first c columns of the identity.
__global__ __launch_bounds__(QT) void k_qr_small(QrBatch jb, DevSlot* slot) {
    extern __shared__ double lds[];
    slot_begin(slot);
    __shared__ double s_tau[64];
    __shared__ double s_cn[64];    // squared norms of the columns' rows not yet factored
    __shared__ int s_perm[64];
    __shared__ int s_piv;
    const int bi = blockIdx.x;
    const int rows = jb.m[bi], c = jb.c[bi], lda = jb.lda[bi];
    const bool pivot = jb.perm[bi] != nullptr;
    const double* Ag = jb.A[bi];
    const int ldt = rows | 1;
    double* T = lds;
    double* X = lds + (size_t)ldt * c;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int grp = tid / QG, lt = tid - grp * QG, ngrp = QT / QG;
    const bool a_rm = (jb.flags[bi] & 1) != 0, r_tr = (jb.flags[bi] & 2) != 0;
    for (int e = tid; e < rows * c; e += blockDim.x) {
        if (a_rm) {
            const int r = e / c, j = e - r * c;   // consecutive threads read consecutive entries of a row
            T[j * ldt + r] = Ag[(int64_t)r * lda + j];
        } else {
            const int j = e / rows, r = e - j * rows;
            T[j * ldt + r] = Ag[(int64_t)j * lda + r];
        }
    }
    for (int e = tid; e < rows * c; e += blockDim.x) {
        const int j = e / rows, r = e - j * rows;
        X[j * ldt + r] = (r == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (pivot) {
        for (int l = grp; l < c; l += ngrp) {
            double s2 = 0.0;
            for (int r = lt; r < rows; r += QG) s2 += T[l * ldt + r] * T[l * ldt + r];
            s2 = row_sum16(s2);
            if (lt == 0) s_cn[l] = s2;
        }
        for (int l = tid; l < c; l += blockDim.x) s_perm[l] = l;
        __syncthreads();
    }
    const int kk = rows < c ? rows : c;
    for (int j = 0; j < kk; ++j) {
        double* col = T + j * ldt;
        if (pivot) {
            // column pivoting: bring the column with the largest remaining norm to j
            if (wave == 0) {
                const int idx = wave_argmax64((lane >= j && lane < c) ? s_cn[lane] : -1.0, lane);
                if (lane == 0) s_piv = idx;
            }
            __syncthreads();
            const int pj = s_piv;
            if (pj != j) {
                double* cp = T + pj * ldt;
                for (int r = tid; r < rows; r += blockDim.x) {
                    const double a = col[r];
                    col[r] = cp[r];
                    cp[r] = a;
                }
                if (tid == 0) {
                    const double a = s_cn[j];
                    s_cn[j] = s_cn[pj];
                    s_cn[pj] = a;
                    const int b = s_perm[j];
                    s_perm[j] = s_perm[pj];
                    s_perm[pj] = b;
                }
            }
            __syncthreads();
        }
        if (wave == 0) {
            double sacc = 0.0;
            for (int r = j + 1 + lane; r < rows; r += 64) sacc += col[r] * col[r];
            sacc = wave_sum64(sacc);
            const double alpha = col[j];
            double tt = 0.0, sc = 0.0, beta = alpha;
            if (sacc != 0.0) {
                beta = -copysign(sqrt(alpha * alpha + sacc), alpha);
                tt = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
            for (int r = j + 1 + lane; r < rows; r += 64) col[r] *= sc == 0.0 ? 1.0 : sc;
            if (lane == 0) {
                col[j] = beta;
                s_tau[j] = tt;
            }
        }
        __syncthreads();
        const double t = s_tau[j];
        for (int l = j + 1 + grp; l < c; l += ngrp) {
            double* cl = T + l * ldt;
            if (t != 0.0) {
                double w = 0.0;
                for (int r = j + 1 + lt; r < rows; r += QG) w += col[r] * cl[r];
                w = row_sum16(w);
                w = t * (w + cl[j]);
                if (lt == 0) cl[j] -= w;
                for (int r = j + 1 + lt; r < rows; r += QG) cl[r] -= w * col[r];
            }
            if (pivot) {
                // norm of the rows below j, recomputed (no downdating)
                double s2 = 0.0;
                for (int r = j + 1 + lt; r < rows; r += QG) s2 += cl[r] * cl[r];
                s2 = row_sum16(s2);
                if (lt == 0) s_cn[l] = s2;
            }
        }
        __syncthreads();
    }
    // Q = H_0 ... H_{kk-1} [I; 0]
    for (int j = kk - 1; j >= 0; --j) {
        const double tj = s_tau[j];
        if (tj != 0.0) {
            const double* v = T + j * ldt;
            for (int l = grp; l < c; l += ngrp) {
                double* xl = X + l * ldt;
                double w = 0.0;
                for (int r = j + 1 + lt; r < rows; r += QG) w += v[r] * xl[r];
                w = row_sum16(w);
                w = tj * (w + xl[j]);
                if (lt == 0) xl[j] -= w;
                for (int r = j + 1 + lt; r < rows; r += QG) xl[r] -= w * v[r];
            }
        }
        __syncthreads();
    }
    double* Qg = jb.Q[bi];
    double* Rg = jb.R[bi];
    for (int e = tid; e < rows * c; e += blockDim.x) {
        const int j = e / rows, r = e - j * rows;
        Qg[(int64_t)j * rows + r] = X[j * ldt + r];
    }
    for (int e = tid; e < c * c; e += blockDim.x) {
        const int j = e / c, r = e - j * c;
        Rg[r_tr ? (int64_t)r * c + j : (int64_t)j * c + r] = (r <= j && r < kk) ? T[j * ldt + r] : 0.0;
    }
    if (pivot)
        for (int l = tid; l < c; l += blockDim.x) jb.perm[bi][l] = s_perm[l];
    slot_end(slot);
}

// Dynamic LDS above the default limit must be requested per kernel; the
// request (dynamic bytes) plus the kernel's static LDS must fit in 160 KB.
std::mutex g_lds_mu;
void allow_lds(const void* fn, size_t bytes, size_t& granted) {
    std::lock_guard<std::mutex> lk(g_lds_mu);
    if (bytes <= granted) return;
    TTSG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    granted = bytes;
}
size_t g_lds_jacobi = 0, g_lds_jacobi4 = 0, g_lds_leaf = 0, g_lds_apply = 0, g_lds_small = 0;

int choose_leaves(int m, int c) {
    int nl = (m + LEAF - 1) / LEAF;
    nl = std::min(nl, std::max(1, m / std::max(c, 1)));
    return std::max(nl, 1);
}

}  // namespace

size_t jacobi_lds_bytes(int m, int c) { return ((size_t)(m | 1) * c + (size_t)(c | 1) * c) * 8; }

// dynamic LDS (matrix + rotations) plus ~26 KB of static scratch must fit in 160 KB
bool jacobi_lds_fits(int m, int c) {
    return m >= c && c <= 64 && m <= JG * JROWS && jacobi_lds_bytes(m, c) <= 128 * 1024;
}

void svd_jacobi_batched(const std::vector<JacobiJob>& jobs, hipStream_t st) {
    size_t i = 0;
    while (i < jobs.size()) {
        JacobiBatch jb{};
        size_t lds = 0;
        int cnt = 0, mmax = 0;
        double flops = 0.0;
        for (; i < jobs.size() && cnt < 32; ++i, ++cnt) {
            const JacobiJob& j = jobs[i];
            TTSG_CHECK(jacobi_lds_fits(j.m, j.c), TTSG_ERR_ARG, "jacobi job does not fit in LDS");
            jb.m[cnt] = j.m;
            jb.c[cnt] = j.c;
            jb.lda[cnt] = j.lda;
            jb.A[cnt] = j.A;
            jb.V[cnt] = j.V;
            jb.sig[cnt] = j.sig;
            // below m eps a computed dot product is rounding noise
            jb.tol[cnt] = j.tol > 0.0 ? j.tol : 4.0 * j.m * 2.220446049250313e-16;
            jb.drop_abs2[cnt] = j.drop_abs2;
            jb.drop_rel2[cnt] = j.drop_rel2;
            lds = std::max(lds, jacobi_lds_bytes(j.m, j.c));
            mmax = std::max(mmax, j.m);
            flops += 0.5 * j.c * (j.c - 1.0) * (12.0 * j.m + 6.0 * j.c);
            if (bounds_checking()) {
                check_range(j.A, ((int64_t)(j.c - 1) * j.lda + j.m) * 8, "jacobi_lds A");
                check_range(j.V, (int64_t)j.c * j.c * 8, "jacobi_lds V");
                check_range(j.sig, (int64_t)j.c * 8, "jacobi_lds sig");
            }
        }
        jb.count = cnt;
        int cmax = 0;
        for (int t = 0; t < cnt; ++t) cmax = std::max(cmax, jb.c[t]);
        StatScope scope(TTSG_ST_SVD, flops, 0.0, st);
        scope.shape(cnt, mmax, cmax, 0, 0);
        // four register rows per lane cover every matrix of up to 64 rows
        if (mmax <= 4 * JG) {
            allow_lds(reinterpret_cast<const void*>(&k_jacobi_lds<4>), lds, g_lds_jacobi4);
            hipLaunchKernelGGL(k_jacobi_lds<4>, dim3(cnt), dim3(JT), lds, st, jb, 30, scope.slot());
        } else {
            allow_lds(reinterpret_cast<const void*>(&k_jacobi_lds<JROWS>), lds, g_lds_jacobi);
            hipLaunchKernelGGL(k_jacobi_lds<JROWS>, dim3(cnt), dim3(JT), lds, st, jb, 30, scope.slot());
        }
        TTSG_HIP(hipGetLastError());
    }
}

size_t g_lds_big8 = 0, g_lds_big10 = 0, g_lds_big8v = 0, g_lds_big10v = 0;

size_t jacobi_big_lds_bytes(int m, int c) { return (size_t)(m | 1) * c * 8; }

// 64 < c <= 128 columns, m <= 160 rows, and the matrix within 152 KB of LDS
// (the kernel's static arrays take about 4 KB more)
bool jacobi_big_fits(int m, int c) {
    return m >= c && c <= JB_CMAX && m <= JG * 10 && jacobi_big_lds_bytes(m, c) <= 152 * 1024 + 1024;
}

size_t jacobi_big_log_bytes(int c) {
    // tangents of kJacobiBigSweeps sweeps of at most c rounds of (c + 1) / 2 pairs, and the meta block
    return ((size_t)kJacobiBigSweeps * c * ((c + 1) / 2) * sizeof(double) + 255) / 256 * 256 +
           ((size_t)(2 * c + 2) * sizeof(int) + 255) / 256 * 256;
}

void svd_jacobi_big(const std::vector<JacobiJob>& jobs, bool accumulate, hipStream_t st, Arena* ar) {
    TTSG_CHECK(!accumulate || ar != nullptr, TTSG_ERR_ARG, "jacobi: the accumulated form needs scratch");
    size_t i = 0;
    while (i < jobs.size()) {
        JacobiBatch jb{};
        size_t lds = 0;
        int cnt = 0, mmax = 0, cmax = 0;
        double flops = 0.0;
        const size_t mark = ar != nullptr ? ar->mark() : 0;
        for (; i < jobs.size() && cnt < 32; ++i, ++cnt) {
            const JacobiJob& j = jobs[i];
            TTSG_CHECK(jacobi_big_fits(j.m, j.c), TTSG_ERR_ARG, "jacobi job does not fit the 128-column kernel");
            TTSG_CHECK(!accumulate || j.V != nullptr, TTSG_ERR_ARG, "jacobi: accumulator requested without V");
            jb.m[cnt] = j.m;
            jb.c[cnt] = j.c;
            jb.lda[cnt] = j.lda;
            jb.A[cnt] = j.A;
            jb.V[cnt] = accumulate ? j.V : nullptr;
            jb.sig[cnt] = j.sig;
            jb.tol[cnt] = j.tol > 0.0 ? j.tol : 4.0 * j.m * 2.220446049250313e-16;
            jb.drop_abs2[cnt] = j.drop_abs2;
            jb.drop_rel2[cnt] = j.drop_rel2;
            if (accumulate) {
                jb.rot[cnt] = ar->get<double>((size_t)kJacobiBigSweeps * j.c * ((j.c + 1) / 2));
                jb.meta[cnt] = ar->get<int>(2 * j.c + 2);
            }
            lds = std::max(lds, jacobi_big_lds_bytes(j.m, j.c));
            mmax = std::max(mmax, j.m);
            cmax = std::max(cmax, j.c);
            flops += 0.5 * j.c * (j.c - 1.0) * ((accumulate ? 12.0 : 6.0) * j.m + (accumulate ? 6.0 * j.c : 0.0));
            if (bounds_checking()) {
                check_range(j.A, ((int64_t)(j.c - 1) * j.lda + j.m) * 8, "jacobi_big A");
                if (accumulate) check_range(j.V, (int64_t)j.c * j.c * 8, "jacobi_big V");
                check_range(j.sig, (int64_t)j.c * 8, "jacobi_big sig");
            }
        }
        jb.count = cnt;
        StatScope scope(TTSG_ST_SVD, flops, 0.0, st);
        scope.shape(cnt, mmax, cmax, 0, 0);
        const bool r8 = mmax <= 8 * JG;
        if (accumulate) {
            if (r8) {
                allow_lds(reinterpret_cast<const void*>(&k_jacobi_big<8, true>), lds, g_lds_big8v);
                hipLaunchKernelGGL((k_jacobi_big<8, true>), dim3(cnt), dim3(JTB), lds, st, jb, kJacobiBigSweeps,
                                   scope.slot());
            } else {
                allow_lds(reinterpret_cast<const void*>(&k_jacobi_big<10, true>), lds, g_lds_big10v);
                hipLaunchKernelGGL((k_jacobi_big<10, true>), dim3(cnt), dim3(JTB), lds, st, jb, kJacobiBigSweeps,
                                   scope.slot());
            }
        } else {
            if (r8) {
                allow_lds(reinterpret_cast<const void*>(&k_jacobi_big<8, false>), lds, g_lds_big8);
                hipLaunchKernelGGL((k_jacobi_big<8, false>), dim3(cnt), dim3(JTB), lds, st, jb, 30, scope.slot());
            } else {
                allow_lds(reinterpret_cast<const void*>(&k_jacobi_big<10, false>), lds, g_lds_big10);
                hipLaunchKernelGGL((k_jacobi_big<10, false>), dim3(cnt), dim3(JTB), lds, st, jb, 30, scope.slot());
            }
        }
        TTSG_HIP(hipGetLastError());
        if (accumulate) {
            hipLaunchKernelGGL(k_jacobi_apply_v, dim3((cmax + JAV_ROWS - 1) / JAV_ROWS, cnt), dim3(JTB), 0, st, jb);
            TTSG_HIP(hipGetLastError());
            ar->release(mark);
        }
    }
}

size_t qr_small_lds_bytes(int m, int c) { return 2 * (size_t)(m | 1) * c * 8; }
bool qr_small_fits(int m, int c) { return m >= c && c <= 64 && qr_small_lds_bytes(m, c) <= 140 * 1024; }

void qr_small_batched(const std::vector<QrJob>& jobs, hipStream_t st) {
    size_t i = 0;
    while (i < jobs.size()) {
        QrBatch jb{};
        size_t lds = 0;
        int cnt = 0;
        double flops = 0.0;
        for (; i < jobs.size() && cnt < 32; ++i, ++cnt) {
            const QrJob& j = jobs[i];
            TTSG_CHECK(qr_small_fits(j.m, j.c), TTSG_ERR_ARG, "qr job does not fit in LDS");
            jb.m[cnt] = j.m;
            jb.c[cnt] = j.c;
            jb.lda[cnt] = j.lda;
            jb.A[cnt] = j.A;
            jb.Q[cnt] = j.Q;
            jb.R[cnt] = j.R;
            jb.perm[cnt] = j.perm;
            jb.flags[cnt] = (j.a_rowmajor ? 1 : 0) | (j.r_transposed ? 2 : 0);
            lds = std::max(lds, qr_small_lds_bytes(j.m, j.c));
            flops += 4.0 * j.m * j.c * (double)j.c - 4.0 / 3.0 * j.c * (double)j.c * j.c;
            if (bounds_checking()) {
                check_range(j.A, (j.a_rowmajor ? (int64_t)(j.m - 1) * j.lda + j.c : (int64_t)(j.c - 1) * j.lda + j.m) * 8,
                            "qr_small A");
                check_range(j.Q, (int64_t)j.m * j.c * 8, "qr_small Q");
                check_range(j.R, (int64_t)j.c * j.c * 8, "qr_small R");
            }
        }
        jb.count = cnt;
        StatScope scope(TTSG_ST_QR, flops, 0.0, st);
        allow_lds(reinterpret_cast<const void*>(&k_qr_small), lds, g_lds_small);
        hipLaunchKernelGGL(k_qr_small, dim3(cnt), dim3(QT), lds, st, jb, scope.slot());
        TTSG_HIP(hipGetLastError());
    }
}

bool tsqr_fits(int m, int c) { return m >= c && c <= 64; }

void TsqrPlan::factor(int m_, int c_, const double* A, int lda, Arena& ar, hipStream_t st) {
    m = m_;
    c = c_;
    TTSG_CHECK(tsqr_fits(m, c), TTSG_ERR_ARG, "tsqr: needs m >= c and c <= 64");
    levels.clear();
    const double* in = A;
    int ld_in = lda;
    int rows = m;
    while (true) {
        Level L;
        L.rows = rows;
        L.nleaves = choose_leaves(rows, c);
        L.refl = ar.get<double>((int64_t)rows * c);
        L.tau = ar.get<double>((int64_t)L.nleaves * c);
        L.stack = ar.get<double>((int64_t)L.nleaves * c * c);
        const int ldstack = L.nleaves * c;
        const int maxrows = (rows + L.nleaves - 1) / L.nleaves;
        const size_t lds = (size_t)(maxrows | 1) * c * 8;
        TTSG_CHECK(lds <= 150 * 1024, TTSG_ERR_ARG, "tsqr leaf exceeds LDS");
        if (bounds_checking()) {
            check_range(in, ((int64_t)(c - 1) * ld_in + rows) * 8, "tsqr in");
            check_range(L.refl, (int64_t)rows * c * 8, "tsqr refl");
        }
        {
            const double kq = std::min(maxrows, c);
            StatScope scope(TTSG_ST_QR, L.nleaves * (2.0 * maxrows * c * kq - 2.0 / 3.0 * kq * kq * kq), 0.0, st);
            allow_lds(reinterpret_cast<const void*>(&k_qr_leaf), lds, g_lds_leaf);
            hipLaunchKernelGGL(k_qr_leaf, dim3(L.nleaves), dim3(QT), lds, st, rows, c, in, ld_in, L.nleaves, L.refl,
                               rows, L.tau, L.stack, ldstack, scope.slot());
            TTSG_HIP(hipGetLastError());
        }
        levels.push_back(L);
        if (L.nleaves == 1) break;
        in = L.stack;
        ld_in = ldstack;
        rows = ldstack;
    }
    R = levels.back().stack;   // c x c, column-major, ld c
}

void TsqrPlan::apply(int k, const double* B, int ldb, double* Out, int ldo, bool out_rowmajor, Arena& ar,
                     hipStream_t st) const {
    const size_t mark = ar.mark();
    const double* in = B;
    int ld_in = ldb;
    for (int li = (int)levels.size() - 1; li >= 0; --li) {
        const Level& L = levels[li];
        const bool last = (li == 0);
        double* out;
        int ld_out;
        if (last) {
            out = Out;
            ld_out = ldo;
        } else {
            out = ar.get<double>((int64_t)L.rows * k);
            ld_out = L.rows;
        }
        const int maxrows = (L.rows + L.nleaves - 1) / L.nleaves;
        const size_t lds = ((size_t)(maxrows | 1) * k + maxrows + 1) * 8;
        TTSG_CHECK(lds <= 150 * 1024, TTSG_ERR_ARG, "tsqr apply exceeds LDS");
        {
            StatScope scope(TTSG_ST_QR, L.nleaves * 4.0 * maxrows * c * (double)k, 0.0, st);
            allow_lds(reinterpret_cast<const void*>(&k_qr_apply_leaf), lds, g_lds_apply);
            hipLaunchKernelGGL(k_qr_apply_leaf, dim3(L.nleaves), dim3(QT), lds, st, L.rows, c, k, L.refl, L.rows,
                               L.tau, L.nleaves, in, ld_in, out, ld_out, (last && out_rowmajor) ? 1 : 0,
                               scope.slot());
            TTSG_HIP(hipGetLastError());
        }
        in = out;
        ld_in = ld_out;
    }
    ar.release(mark);
}

}  // namespace ttsg
