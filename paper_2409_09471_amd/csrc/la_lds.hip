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

#include "tt_ops.h"

namespace ttsg {
namespace {

constexpr int JT = 1024;   // threads of the Jacobi workgroup
constexpr int QT = 512;    // threads of the QR leaf workgroups
constexpr int LEAF = 256;  // maximum rows of a TSQR leaf

__device__ __forceinline__ double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct JacobiBatch {
    int count;
    int m[32], c[32], lda[32];
    double* A[32];
    double* V[32];
    double* sig[32];
};

__global__ __launch_bounds__(JT) void k_jacobi_lds(JacobiBatch jb, int maxsweeps, double tol) {
    extern __shared__ double lds[];
    const int bi = blockIdx.x;
    const int m = jb.m[bi], c = jb.c[bi], lda = jb.lda[bi];
    double* Ag = jb.A[bi];
    double* Vg = jb.V[bi];
    const int ldm = m | 1;          // odd leading dimensions spread the LDS banks
    const int ldv = c | 1;
    double* A = lds;
    double* V = lds + (size_t)ldm * c;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int e = tid; e < m * c; e += blockDim.x) {
        int j = e / m, i = e - j * m;
        A[j * ldm + i] = Ag[(int64_t)j * lda + i];
    }
    for (int e = tid; e < c * c; e += blockDim.x) {
        int j = e / c, i = e - j * c;
        V[j * ldv + i] = (i == j) ? 1.0 : 0.0;
    }
    __shared__ int s_rot;
    const int cp = c + (c & 1);
    __syncthreads();
    for (int sweep = 0; sweep < maxsweeps && cp > 1; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < cp - 1; ++r) {
            for (int pk = wave; pk < cp / 2; pk += nw) {
                int p, q;
                if (pk == 0) {
                    p = cp - 1;
                    q = r;
                } else {
                    p = (r + pk) % (cp - 1);
                    q = (r - pk + cp - 1) % (cp - 1);
                }
                if (p >= c || q >= c) continue;
                double* ap = A + p * ldm;
                double* aq = A + q * ldm;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lane; i < m; i += 64) {
                    double x = ap[i], y = aq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = wsum(al);
                be = wsum(be);
                ga = wsum(ga);
                if (al == 0.0 || be == 0.0) continue;
                if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
                double zeta = (be - al) / (2.0 * ga);
                double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int i = lane; i < m; i += 64) {
                    double x = ap[i], y = aq[i];
                    ap[i] = cs * x - sn * y;
                    aq[i] = sn * x + cs * y;
                }
                double* vp = V + p * ldv;
                double* vq = V + q * ldv;
                for (int i = lane; i < c; i += 64) {
                    double x = vp[i], y = vq[i];
                    vp[i] = cs * x - sn * y;
                    vq[i] = sn * x + cs * y;
                }
                if (lane == 0) s_rot = 1;
            }
            __syncthreads();
        }
        if (s_rot == 0) break;
        __syncthreads();
    }
    __syncthreads();
    for (int e = tid; e < m * c; e += blockDim.x) {
        int j = e / m, i = e - j * m;
        Ag[(int64_t)j * lda + i] = A[j * ldm + i];
    }
    for (int e = tid; e < c * c; e += blockDim.x) {
        int j = e / c, i = e - j * c;
        Vg[(int64_t)j * c + i] = V[j * ldv + i];
    }
    for (int l = wave; l < c; l += nw) {
        const double* al = A + l * ldm;
        double s = 0.0;
        for (int i = lane; i < m; i += 64) s += al[i] * al[i];
        s = wsum(s);
        if (lane == 0) jb.sig[bi][l] = sqrt(s);
    }
}

// Leaf i of a TSQR level: rows [r0, r1) of the column-major m x c matrix A.
__device__ __forceinline__ void leaf_rows(int m, int nleaves, int i, int& r0, int& r1) {
    r0 = (int)(((int64_t)i * m) / nleaves);
    r1 = (int)(((int64_t)(i + 1) * m) / nleaves);
}

__global__ __launch_bounds__(QT) void k_qr_leaf(int m, int c, const double* __restrict__ A, int lda,
                                                 int nleaves, double* __restrict__ refl, int ldr,
                                                 double* __restrict__ tau, double* __restrict__ Rs, int ldrs) {
    extern __shared__ double T[];
    const int i = blockIdx.x;
    int r0, r1;
    leaf_rows(m, nleaves, i, r0, r1);
    const int rows = r1 - r0;
    const int ldt = rows | 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int e = tid; e < rows * c; e += blockDim.x) {
        int j = e / rows, r = e - j * rows;
        T[j * ldt + r] = A[(int64_t)j * lda + r0 + r];
    }
    __shared__ double s_tau, s_scale;
    __syncthreads();
    const int kk = rows < c ? rows : c;
    for (int j = 0; j < kk; ++j) {
        double* col = T + j * ldt;
        if (wave == 0) {
            double s = 0.0;
            for (int r = j + 1 + lane; r < rows; r += 64) s += col[r] * col[r];
            s = wsum(s);
            if (lane == 0) {
                double alpha = col[j];
                if (s == 0.0) {
                    s_tau = 0.0;
                    s_scale = 0.0;
                } else {
                    double beta = -copysign(sqrt(alpha * alpha + s), alpha);
                    s_tau = (beta - alpha) / beta;
                    s_scale = 1.0 / (alpha - beta);
                    col[j] = beta;
                }
                tau[(int64_t)i * c + j] = s_tau;
            }
        }
        __syncthreads();
        const double t = s_tau, sc = s_scale;
        if (t != 0.0) {
            for (int r = j + 1 + tid; r < rows; r += blockDim.x) col[r] *= sc;
            __syncthreads();
            for (int l = j + 1 + wave; l < c; l += nw) {
                double* cl = T + l * ldt;
                double w = 0.0;
                for (int r = j + 1 + lane; r < rows; r += 64) w += col[r] * cl[r];
                w = wsum(w);
                w = t * (w + cl[j]);
                if (lane == 0) cl[j] -= w;
                for (int r = j + 1 + lane; r < rows; r += 64) cl[r] -= w * col[r];
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
}

// Out (rows of this level x k) = blockdiag(Q_i) [B_i; 0], B_i = rows i*c.. of Bin.
__global__ __launch_bounds__(QT) void k_qr_apply_leaf(int m, int c, int k, const double* __restrict__ refl, int ldr,
                                                       const double* __restrict__ tau, int nleaves,
                                                       const double* __restrict__ Bin, int ldb,
                                                       double* __restrict__ Out, int ldo, int out_rowmajor) {
    extern __shared__ double X[];
    const int i = blockIdx.x;
    int r0, r1;
    leaf_rows(m, nleaves, i, r0, r1);
    const int rows = r1 - r0;
    const int ldx = rows | 1;
    double* v = X + (size_t)ldx * k;   // the current reflector
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
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
        for (int t = wave; t < k; t += nw) {
            double* xt = X + t * ldx;
            double w = 0.0;
            for (int r = j + 1 + lane; r < rows; r += 64) w += v[r] * xt[r];
            w = wsum(w);
            w = tj * (w + xt[j]);
            if (lane == 0) xt[j] -= w;
            for (int r = j + 1 + lane; r < rows; r += 64) xt[r] -= w * v[r];
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
}

// Dynamic LDS above the default limit must be requested once per kernel.
void allow_lds(const void* fn, bool& done) {
    if (done) return;
    TTSG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
    done = true;
}
bool g_lds_jacobi = false, g_lds_leaf = false, g_lds_apply = false;

int choose_leaves(int m, int c) {
    int nl = (m + LEAF - 1) / LEAF;
    nl = std::min(nl, std::max(1, m / std::max(c, 1)));
    return std::max(nl, 1);
}

}  // namespace

size_t jacobi_lds_bytes(int m, int c) { return ((size_t)(m | 1) * c + (size_t)(c | 1) * c) * 8; }

bool jacobi_lds_fits(int m, int c) { return m >= c && jacobi_lds_bytes(m, c) <= 150 * 1024; }

void svd_jacobi_batched(const std::vector<JacobiJob>& jobs, hipStream_t st) {
    size_t i = 0;
    while (i < jobs.size()) {
        JacobiBatch jb{};
        size_t lds = 0;
        int cnt = 0;
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
            lds = std::max(lds, jacobi_lds_bytes(j.m, j.c));
            flops += 0.5 * j.c * (j.c - 1.0) * (12.0 * j.m + 6.0 * j.c);
            if (bounds_checking()) {
                check_range(j.A, ((int64_t)(j.c - 1) * j.lda + j.m) * 8, "jacobi_lds A");
                check_range(j.V, (int64_t)j.c * j.c * 8, "jacobi_lds V");
                check_range(j.sig, (int64_t)j.c * 8, "jacobi_lds sig");
            }
        }
        jb.count = cnt;
        StatScope scope(TTSG_ST_SVD, flops, 0.0, st);
        allow_lds(reinterpret_cast<const void*>(&k_jacobi_lds), g_lds_jacobi);
        hipLaunchKernelGGL(k_jacobi_lds, dim3(cnt), dim3(JT), lds, st, jb, 60, 1e-15);
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
            allow_lds(reinterpret_cast<const void*>(&k_qr_leaf), g_lds_leaf);
            hipLaunchKernelGGL(k_qr_leaf, dim3(L.nleaves), dim3(QT), lds, st, rows, c, in, ld_in, L.nleaves, L.refl,
                               rows, L.tau, L.stack, ldstack);
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
            allow_lds(reinterpret_cast<const void*>(&k_qr_apply_leaf), g_lds_apply);
            hipLaunchKernelGGL(k_qr_apply_leaf, dim3(L.nleaves), dim3(QT), lds, st, L.rows, c, k, L.refl, L.rows,
                               L.tau, L.nleaves, in, ld_in, out, ld_out, (last && out_rowmajor) ? 1 : 0);
            TTSG_HIP(hipGetLastError());
        }
        in = out;
        ld_in = ld_out;
    }
    ar.release(mark);
}

}  // namespace ttsg
