// TT operations of the sketched TT-GMRES hot path, expressed as sequences of
// strided contractions (contract.hip) and FP64 factorizations (la.hip).
//
// Layout conventions (row-major, 0-based modes):
//   core C_mu        [a][j][b]          r_l x n x r_r
//   operator D_mu    [al][i][j][be]     R_l x n x n x R_r
//   left env  E_mu   [p][al][a]         rho x R x r   (probe rank, op rank, vector rank)
//   right env F_mu   [b][be][q]         r x R x rx    (vector rank, op rank, probe rank)
//   Psi_mu           [p][i][q]          rho_mu x n x rx_{mu+1}
//   Omega_b          [p][q]             rho_b x rx_b
// The merged rank index of A v is (a, al) with the vector rank outer, so the
// environment orders above make every merged index a plain stride.
#include "tt_ops.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace ttsg {

ContractDesc cdesc(int M, int N, int K, int batch) {
    ContractDesc d{};
    d.M = M;
    d.N = N;
    d.K = K;
    d.batch = batch;
    d.alpha = 1.0;
    d.beta = 0.0;
    d.am = d.ak = d.bk = d.bn = d.cm = d.cn = idx1(0);
    d.ab = d.bb = d.cb = idx1(0);
    return d;
}

// ---------------------------------------------------------------------------
// Matrix-vector product (Sec. 2.2)
// ---------------------------------------------------------------------------
void matvec_core(int rl, int n, int rr, int Rl, int Rr, const double* D, const double* C, bool transpose,
                 double* G, hipStream_t st) {
    // G[(a,al)][i][(b,be)] = sum_j D[al][i][j][be] C[a][j][b], one product per (al, be)
    ContractDesc d = cdesc(n, rl * rr, n, Rl * Rr);
    d.ab = idx2(Rr, 1, (int64_t)n * n * Rr);
    d.am = transpose ? idx1(Rr) : idx1((int64_t)n * Rr);
    d.ak = transpose ? idx1((int64_t)n * Rr) : idx1(Rr);
    d.bb = idx1(0);
    d.bk = idx1(rr);
    d.bn = idx2(rr, 1, (int64_t)n * rr);
    const int64_t rowG = (int64_t)n * rr * Rr;
    d.cb = idx2(Rr, 1, rowG);
    d.cm = idx1((int64_t)rr * Rr);
    d.cn = idx2(rr, Rr, (int64_t)Rl * rowG);
    contract(Prec::F64, d, D, C, G, st);
}

// ---------------------------------------------------------------------------
// Operator block kinds
// ---------------------------------------------------------------------------
namespace {

// One workgroup per block (al, be) of a core D[al][i][j][be]: bit 0 = some
// entry is nonzero, bit 1 = the block differs from the identity.
__global__ __launch_bounds__(256) void k_block_kinds(int n, int Rr, const double* __restrict__ D,
                                                     uint8_t* __restrict__ out) {
    __shared__ int flags;
    if (threadIdx.x == 0) flags = 0;
    __syncthreads();
    const int al = blockIdx.x / Rr, be = blockIdx.x - (blockIdx.x / Rr) * Rr;
    const int64_t nn = (int64_t)n * n;
    int f = 0;
    for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        const double v = D[(((int64_t)al * n + i) * n + j) * Rr + be];
        if (v != 0.0) f |= 1;
        if (v != (i == j ? 1.0 : 0.0)) f |= 2;
    }
    if (f != 0) atomicOr(&flags, f);
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (flags & 1) == 0 ? kBlkZero : ((flags & 2) == 0 ? kBlkIdentity : kBlkDense);
}

// out[b][i][c] = in[b][i][c] (+ out[b][i][c] when acc), or 0, for b < B,
// i < I, c < Cn (c contiguous): a workgroup of 64 x 4 lanes covers 64
// consecutive c of 4 rows i of one b, so every index comes from the grid
// without a division.
constexpr int BLK_C = 64, BLK_I = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_block_copy(int I, int Cn, const T* __restrict__ in, int64_t sbi, int64_t sii,
                                                    T* __restrict__ out, int64_t sbo, int64_t sio, int acc) {
    const int c = blockIdx.x * BLK_C + (int)(threadIdx.x % BLK_C);
    const int i = blockIdx.y * BLK_I + (int)(threadIdx.x / BLK_C);
    const int64_t b = blockIdx.z;
    if (c >= Cn || i >= I) return;
    const T v = in[b * sbi + i * sii + c];
    T* o = out + b * sbo + i * sio + c;
    *o = acc ? *o + v : v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_block_zero(int I, int Cn, T* __restrict__ out, int64_t sbo, int64_t sio) {
    const int c = blockIdx.x * BLK_C + (int)(threadIdx.x % BLK_C);
    const int i = blockIdx.y * BLK_I + (int)(threadIdx.x / BLK_C);
    const int64_t b = blockIdx.z;
    if (c >= Cn || i >= I) return;
    out[b * sbo + i * sio + c] = T(0);
}

dim3 block_grid(int B, int I, int Cn) {
    TTSG_CHECK(B <= 65535 && (I + BLK_I - 1) / BLK_I <= 65535, TTSG_ERR_ARG, "block copy: extent too large");
    return dim3((unsigned)((Cn + BLK_C - 1) / BLK_C), (unsigned)((I + BLK_I - 1) / BLK_I), (unsigned)B);
}

void block_copy(Prec p, int B, int I, int Cn, const void* in, int64_t sbi, int64_t sii, void* out, int64_t sbo,
                int64_t sio, bool acc, hipStream_t st) {
    if (B <= 0 || I <= 0 || Cn <= 0) return;
    const dim3 g = block_grid(B, I, Cn);
    if (p == Prec::F64)
        hipLaunchKernelGGL(k_block_copy<double>, g, dim3(256), 0, st, I, Cn, static_cast<const double*>(in), sbi, sii,
                           static_cast<double*>(out), sbo, sio, acc ? 1 : 0);
    else
        hipLaunchKernelGGL(k_block_copy<float>, g, dim3(256), 0, st, I, Cn, static_cast<const float*>(in), sbi, sii,
                           static_cast<float*>(out), sbo, sio, acc ? 1 : 0);
    TTSG_HIP(hipGetLastError());
}

void block_zero(Prec p, int B, int I, int Cn, void* out, int64_t sbo, int64_t sio, hipStream_t st) {
    if (B <= 0 || I <= 0 || Cn <= 0) return;
    const dim3 g = block_grid(B, I, Cn);
    if (p == Prec::F64)
        hipLaunchKernelGGL(k_block_zero<double>, g, dim3(256), 0, st, I, Cn, static_cast<double*>(out), sbo, sio);
    else
        hipLaunchKernelGGL(k_block_zero<float>, g, dim3(256), 0, st, I, Cn, static_cast<float*>(out), sbo, sio);
    TTSG_HIP(hipGetLastError());
}

}  // namespace

std::vector<std::vector<uint8_t>> operator_blocks(int d, const int* n, const std::vector<int>& R,
                                                  const std::vector<const void*>& D, hipStream_t st, Arena& ar) {
    std::vector<std::vector<uint8_t>> out(d);
    if (D.empty()) return {};
    int64_t tot = 0;
    std::vector<int64_t> off(d + 1, 0);
    for (int mu = 0; mu < d; ++mu) off[mu + 1] = off[mu] + (int64_t)R[mu] * R[mu + 1];
    tot = off[d];
    const size_t mk = ar.mark();
    uint8_t* dev = ar.get<uint8_t>((size_t)std::max<int64_t>(tot, 1));
    for (int mu = 0; mu < d; ++mu) {
        hipLaunchKernelGGL(k_block_kinds, dim3(R[mu] * R[mu + 1]), dim3(256), 0, st, n[mu], R[mu + 1],
                           static_cast<const double*>(D[mu]), dev + off[mu]);
        TTSG_HIP(hipGetLastError());
    }
    std::vector<uint8_t> h((size_t)tot);
    TTSG_HIP(hipMemcpyAsync(h.data(), dev, (size_t)tot, hipMemcpyDeviceToHost, st));
    TTSG_HIP(hipStreamSynchronize(st));
    ar.release(mk);
    for (int mu = 0; mu < d; ++mu) out[mu].assign(h.begin() + off[mu], h.begin() + off[mu + 1]);
    return out;
}

std::vector<const uint8_t*> block_ptrs(const std::vector<std::vector<uint8_t>>& kinds) {
    std::vector<const uint8_t*> p;
    for (const auto& k : kinds) p.push_back(k.data());
    return p;
}

// ---------------------------------------------------------------------------
// Environment steps
// ---------------------------------------------------------------------------
static inline int64_t eoff(Prec p) { return p == Prec::F64 ? 8 : 4; }

void left_step(Prec p, const LeftDims& s, const void* E, const void* C, const void* D, const void* Z, void* T1,
               void* T2, void* Eout, hipStream_t st, Arena* ar) {
    const int rl = s.rl, n = s.n, rr = s.rr, Rl = s.Rl, Rr = s.Rr, pl = s.pl, pr = s.pr;
    // L1: T1[p'][al][j][b] = sum_a E[p'][al][a] C[a][j][b]
    {
        ContractDesc d = cdesc(pl * Rl, n * rr, rl);
        d.am = idx1(rl);
        d.ak = idx1(1);
        d.bk = idx1((int64_t)n * rr);
        d.bn = idx1(1);
        d.cm = idx1((int64_t)n * rr);
        d.cn = idx1(1);
        contract(p, d, E, C, T1, st, ar);
    }
    const void* T2in = T1;
    if (D != nullptr && s.blk != nullptr) {
        // L2 block by block: for each be, the dense blocks D[al][:, :][be] on
        // the matrix cores, the identity blocks as copies of T1[p'][al], in
        // ascending al; a column be with no nonzero block is zero
        const size_t es = elem_size(p);
        for (int be = 0; be < Rr; ++be) {
            bool first = true;
            // the sum runs over the nonzero blocks in ascending al; when its first
            // two are one identity and one dense block, the dense block's
            // contraction adds the identity's slice of T1 in its epilogue (the
            // same sum, one launch instead of two)
            int nz[8], nn = 0;
            for (int al = 0; al < Rl && nn < 8; ++al)
                if (s.blk[al * Rr + be] != kBlkZero) nz[nn++] = al;
            int skip = -1, add = -1;
            if (nn >= 2 && Rl <= 8) {
                const uint8_t k0 = s.blk[nz[0] * Rr + be], k1 = s.blk[nz[1] * Rr + be];
                if (k0 == kBlkIdentity && k1 == kBlkDense) skip = nz[0], add = nz[0];
                if (k0 == kBlkDense && k1 == kBlkIdentity) skip = nz[1], add = nz[1];
            }
            for (int al = 0; al < Rl; ++al) {
                const uint8_t kind = s.blk[al * Rr + be];
                if (kind == kBlkZero || al == skip) continue;
                void* Cb = static_cast<char*>(T2) + (size_t)be * rr * es;
                const void* Bb = static_cast<const char*>(T1) + (size_t)al * n * rr * es;
                if (kind == kBlkIdentity) {
                    block_copy(p, pl, n, rr, Bb, (int64_t)Rl * n * rr, rr, Cb, (int64_t)n * Rr * rr,
                               (int64_t)Rr * rr, !first, st);
                } else {
                    ContractDesc d = cdesc(n, rr, n, pl);
                    d.ab = idx1(0);
                    d.am = idx1((int64_t)n * Rr);
                    d.ak = idx1(Rr);
                    d.bb = idx1((int64_t)Rl * n * rr);
                    d.bk = idx1(rr);
                    d.bn = idx1(1);
                    d.cb = idx1((int64_t)n * Rr * rr);
                    d.cm = idx1((int64_t)Rr * rr);
                    d.cn = idx1(1);
                    d.beta = first ? 0.0 : 1.0;
                    if (first && add >= 0) {
                        d.c_add = static_cast<const char*>(T1) + (size_t)add * n * rr * es;
                        d.xb = idx1((int64_t)Rl * n * rr);
                        d.xm = idx1(rr);
                        d.xn = idx1(1);
                    }
                    contract(p, d, static_cast<const char*>(D) + ((size_t)al * n * n * Rr + be) * es, Bb, Cb, st, ar);
                }
                first = false;
            }
            if (first)
                block_zero(p, pl, n, rr, static_cast<char*>(T2) + (size_t)be * rr * es, (int64_t)n * Rr * rr,
                           (int64_t)Rr * rr, st);
        }
        T2in = T2;
    } else if (D != nullptr) {
        // L2: T2[p'][i][be][b] = sum_{(al,j)} D[al][i][j][be] T1[p'][al][j][b]
        ContractDesc d = cdesc(n * Rr, rr, Rl * n, pl);
        d.ab = idx1(0);
        d.am = idx2(Rr, 1, (int64_t)n * Rr);
        d.ak = idx2(n, Rr, (int64_t)n * n * Rr);
        d.bb = idx1((int64_t)Rl * n * rr);
        d.bk = idx1(rr);
        d.bn = idx1(1);
        d.cb = idx1((int64_t)n * Rr * rr);
        d.cm = idx1(rr);
        d.cn = idx1(1);
        contract(p, d, D, T1, T2, st, ar);
        T2in = T2;
    }
    if (Z != nullptr && Eout != nullptr) {
        // L3: E'[p][be][b] = sum_{(p',i)} Z[p'][i][p] T2[p'][i][be][b]
        ContractDesc d = cdesc(pr, Rr * rr, pl * n);
        d.am = idx1(1);
        d.ak = idx1(pr);
        d.bk = idx1((int64_t)Rr * rr);
        d.bn = idx1(1);
        d.cm = idx1((int64_t)Rr * rr);
        d.cn = idx1(1);
        contract(p, d, Z, T2in, Eout, st, ar);
    }
}

void right_step(Prec p, const LeftDims& s, const void* F, const void* C, const void* D, const void* Z, void* U1,
                void* U2, void* Fout, hipStream_t st, Arena* ar) {
    // here pl/pr are the probe ranks (rho_l x n x rho_r) of Z; F is r_r x R_r x pr
    const int rl = s.rl, n = s.n, rr = s.rr, Rl = s.Rl, Rr = s.Rr, pl = s.pl, pr = s.pr;
    // R1: U1[a][j][be][q] = sum_b C[a][j][b] F[b][be][q]
    {
        ContractDesc d = cdesc(rl * n, Rr * pr, rr);
        d.am = idx1(rr);
        d.ak = idx1(1);
        d.bk = idx1((int64_t)Rr * pr);
        d.bn = idx1(1);
        d.cm = idx1((int64_t)Rr * pr);
        d.cn = idx1(1);
        contract(p, d, C, F, U1, st, ar);
    }
    const void* U2in = U1;
    if (D != nullptr && s.blk != nullptr) {
        // R2 block by block: for each al, the dense blocks D[al][:, :][be] on
        // the matrix cores, the identity blocks as copies of U1[a][:, be], in
        // ascending be; a row al with no nonzero block is zero
        const size_t es = elem_size(p);
        for (int al = 0; al < Rl; ++al) {
            bool first = true;
            void* Cb = static_cast<char*>(U2) + (size_t)al * n * pr * es;
            // as in left_step: a leading (identity, dense) pair in ascending be
            // is one contraction whose epilogue adds the identity's slice of U1
            int nz[8], nn = 0;
            for (int be = 0; be < Rr && nn < 8; ++be)
                if (s.blk[al * Rr + be] != kBlkZero) nz[nn++] = be;
            int skip = -1, add = -1;
            if (nn >= 2 && Rr <= 8) {
                const uint8_t k0 = s.blk[al * Rr + nz[0]], k1 = s.blk[al * Rr + nz[1]];
                if (k0 == kBlkIdentity && k1 == kBlkDense) skip = nz[0], add = nz[0];
                if (k0 == kBlkDense && k1 == kBlkIdentity) skip = nz[1], add = nz[1];
            }
            for (int be = 0; be < Rr; ++be) {
                const uint8_t kind = s.blk[al * Rr + be];
                if (kind == kBlkZero || be == skip) continue;
                const void* Bb = static_cast<const char*>(U1) + (size_t)be * pr * es;
                if (kind == kBlkIdentity) {
                    block_copy(p, rl, n, pr, Bb, (int64_t)n * Rr * pr, (int64_t)Rr * pr, Cb, (int64_t)Rl * n * pr, pr,
                               !first, st);
                } else {
                    ContractDesc d = cdesc(n, pr, n, rl);
                    d.ab = idx1(0);
                    d.am = idx1((int64_t)n * Rr);
                    d.ak = idx1(Rr);
                    d.bb = idx1((int64_t)n * Rr * pr);
                    d.bk = idx1((int64_t)Rr * pr);
                    d.bn = idx1(1);
                    d.cb = idx1((int64_t)Rl * n * pr);
                    d.cm = idx1(pr);
                    d.cn = idx1(1);
                    d.beta = first ? 0.0 : 1.0;
                    if (first && add >= 0) {
                        d.c_add = static_cast<const char*>(U1) + (size_t)add * pr * es;
                        d.xb = idx1((int64_t)n * Rr * pr);
                        d.xm = idx1((int64_t)Rr * pr);
                        d.xn = idx1(1);
                    }
                    contract(p, d, static_cast<const char*>(D) + ((size_t)al * n * n * Rr + be) * es, Bb, Cb, st, ar);
                }
                first = false;
            }
            if (first) block_zero(p, rl, n, pr, Cb, (int64_t)Rl * n * pr, pr, st);
        }
        U2in = U2;
    } else if (D != nullptr) {
        // R2: U2[a][al][i][q] = sum_{(j,be)} D[al][i][j][be] U1[a][j][be][q]
        ContractDesc d = cdesc(Rl * n, pr, n * Rr, rl);
        d.ab = idx1(0);
        d.am = idx1((int64_t)n * Rr);
        d.ak = idx1(1);
        d.bb = idx1((int64_t)n * Rr * pr);
        d.bk = idx1(pr);
        d.bn = idx1(1);
        d.cb = idx1((int64_t)Rl * n * pr);
        d.cm = idx1(pr);
        d.cn = idx1(1);
        contract(p, d, D, U1, U2, st, ar);
        U2in = U2;
    }
    // R3: F'[a][al][p'] = sum_{(i,q)} U2[a][al][i][q] Z[p'][i][q]
    {
        ContractDesc d = cdesc(rl * Rl, pl, n * pr);
        d.am = idx1((int64_t)n * pr);
        d.ak = idx1(1);
        d.bk = idx1(1);
        d.bn = idx1((int64_t)n * pr);
        d.cm = idx1(pl);
        d.cn = idx1(1);
        contract(p, d, U2in, Z, Fout, st, ar);
    }
}

void psi_step(Prec p, int pl, int n, int Rr, int rr, int qr, const void* T2, const void* F, void* Psi,
              hipStream_t st, Arena* ar, bool out_f64) {
    // Psi[p'][i][q] = sum_{(be,b)} T2[p'][i][be][b] F[b][be][q]
    ContractDesc d = cdesc(pl * n, qr, Rr * rr);
    d.am = idx1((int64_t)Rr * rr);
    d.ak = idx1(1);
    d.bk = idx2(rr, (int64_t)Rr * qr, qr);
    d.bn = idx1(1);
    d.cm = idx1(qr);
    d.cn = idx1(1);
    d.c_f64 = out_f64 && p != Prec::F64 ? 1 : 0;
    contract(p, d, T2, F, Psi, st, ar);
}

void omega_step(Prec p, int pl, int Rr, int rr, int qr, const void* E, const void* F, void* Om, hipStream_t st,
                Arena* ar, bool out_f64) {
    // Om[p][q] = sum_{(be,b)} E[p][be][b] F[b][be][q]
    ContractDesc d = cdesc(pl, qr, Rr * rr);
    d.am = idx1((int64_t)Rr * rr);
    d.ak = idx1(1);
    d.bk = idx2(rr, (int64_t)Rr * qr, qr);
    d.bn = idx1(1);
    d.cm = idx1(qr);
    d.cn = idx1(1);
    d.c_f64 = out_f64 && p != Prec::F64 ? 1 : 0;
    contract(p, d, E, F, Om, st, ar);
}

// ---------------------------------------------------------------------------
// Khatri-Rao sketch steps.  P_mu[j][al][a] (s x R x r) is the row vector of
// sketch row j after mu cores; SA_mu[j][al][be][i'] = sum_i S_mu[j,i] D_mu[al,i,i',be]
// (or S_mu itself when there is no operator, R = 1).
// ---------------------------------------------------------------------------
void kr_precompute(Prec p, int s, int n, int Rl, int Rr, const void* S, const void* D, void* SA, hipStream_t st) {
    // SA[j][al][be][i'] = sum_i S[j][i] D[al][i][i'][be], batched over al; i'
    // runs fastest so that a Khatri-Rao step reads it along its reduction index
    ContractDesc d = cdesc(s, n * Rr, n, Rl);
    d.ab = idx1(0);
    d.am = idx1(n);
    d.ak = idx1(1);
    d.bb = idx1((int64_t)n * n * Rr);
    d.bk = idx1((int64_t)n * Rr);
    d.bn = idx1(1);
    d.cb = idx1((int64_t)Rr * n);
    d.cm = idx1((int64_t)Rl * n * Rr);
    d.cn = idx2(Rr, n, 1);
    contract(p, d, S, D, SA, st);
}

namespace {
// KR1 with a short operator-rank sum (Rl <= 4): one thread per output entry,
// the Rl products summed in order -- a streaming write of s Rr rl n values.
template <typename T>
__global__ void k_kr1(int64_t total, int rl, int n, int Rl, int Rr, const T* __restrict__ P,
                      const T* __restrict__ SA, T* __restrict__ X) {
    const int64_t per_j = (int64_t)Rr * rl * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / per_j;
        int64_t rem = e - j * per_j;
        const int be = (int)(rem / ((int64_t)rl * n));
        rem -= (int64_t)be * rl * n;
        const int a = (int)(rem / n);
        const int i = (int)(rem - (int64_t)a * n);
        const T* pj = P + j * Rl * rl + a;
        const T* sj = SA + (j * Rl) * n * Rr + (int64_t)be * n + i;
        T acc = 0;
        for (int al = 0; al < Rl; ++al) acc += pj[(int64_t)al * rl] * sj[(int64_t)al * n * Rr];
        X[e] = acc;
    }
}
}  // namespace

void kr_step(Prec p, int s, int rl, int n, int rr, int Rl, int Rr, const void* P, const void* SA, const void* C,
             void* Xbuf, void* Pout, hipStream_t st, Arena* ar) {
    // P'[(j,be)][b] = sum_{(a,i')} X[(j,be)][(a,i')] C[(a,i')][b] with
    // X[j][be][a][i'] = sum_al P[j][al][a] SA[j][al][be][i']: for operator ranks
    // up to 3, X is formed inside the contraction's operand staging and never
    // stored (the s R r n intermediate would be written and read back)
    if (Rl <= 3 && p != Prec::BF16) {
        ContractDesc d = cdesc(s * Rr, rr, rl * n);
        d.bk = idx1(rr);
        d.bn = idx1(1);
        d.cm = idx1(rr);
        d.cn = idx1(1);
        d.kr_P = P;
        d.kr_SA = SA;
        d.kr_rl = rl;
        d.kr_n = n;
        d.kr_Rl = Rl;
        d.kr_Rr = Rr;
        contract(p, d, P, C, Pout, st, ar);
        return;
    }
    // KR1: X[j][be][a][i'] = sum_al P[j][al][a] SA[j][al][be][i']
    if (Rl <= 4 && p != Prec::BF16) {
        const int64_t total = (int64_t)s * Rr * rl * n;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 1 << 16);
        if (p == Prec::F64)
            hipLaunchKernelGGL(k_kr1<double>, dim3(blocks), dim3(256), 0, st, total, rl, n, Rl, Rr,
                               static_cast<const double*>(P), static_cast<const double*>(SA),
                               static_cast<double*>(Xbuf));
        else
            hipLaunchKernelGGL(k_kr1<float>, dim3(blocks), dim3(256), 0, st, total, rl, n, Rl, Rr,
                               static_cast<const float*>(P), static_cast<const float*>(SA), static_cast<float*>(Xbuf));
        TTSG_HIP(hipGetLastError());
    } else {
        ContractDesc d = cdesc(rl, Rr * n, Rl, s);
        d.ab = idx1((int64_t)Rl * rl);
        d.am = idx1(1);
        d.ak = idx1(rl);
        d.bb = idx1((int64_t)Rl * n * Rr);
        d.bk = idx1((int64_t)n * Rr);
        d.bn = idx1(1);
        d.cb = idx1((int64_t)Rr * rl * n);
        d.cm = idx1(n);
        d.cn = idx2(n, 1, (int64_t)rl * n);
        contract(p, d, P, SA, Xbuf, st, ar);
    }
    // KR2: P'[(j,be)][b] = sum_{(a,i')} X[(j,be)][(a,i')] C[(a,i')][b]
    {
        ContractDesc d = cdesc(s * Rr, rr, rl * n);
        d.am = idx1((int64_t)rl * n);
        d.ak = idx1(1);
        d.bk = idx1(rr);
        d.bn = idx1(1);
        d.cm = idx1(rr);
        d.cn = idx1(1);
        contract(p, d, Xbuf, C, Pout, st, ar);
    }
}

}  // namespace ttsg

// ---------------------------------------------------------------------------
// Sweep drivers
// ---------------------------------------------------------------------------
namespace ttsg {

namespace {
// one float64 or float32 scalar 1 written into a tiny buffer
__global__ void k_set_one(void* p, int is_f64) {
    if (is_f64) *static_cast<double*>(p) = 1.0;
    else *static_cast<float*>(p) = 1.0f;
}
__global__ void k_to_f64(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}
__global__ void k_copy_scalar(const void* src, int is_f64, double* dst) {
    dst[0] = is_f64 ? *static_cast<const double*>(src) : (double)*static_cast<const float*>(src);
}
void set_one(Prec p, void* buf, hipStream_t st) {
    hipLaunchKernelGGL(k_set_one, dim3(1), dim3(1), 0, st, buf, p == Prec::F64 ? 1 : 0);
    TTSG_HIP(hipGetLastError());
}
void to_f64(Prec p, int64_t n, const void* src, double* dst, hipStream_t st) {
    if (n <= 0) return;
    if (p == Prec::F64) {
        copy_f64(n, static_cast<const double*>(src), dst, st);
        return;
    }
    int64_t b = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_to_f64, dim3((unsigned)std::max<int64_t>(b, 1)), dim3(256), 0, st, n,
                       static_cast<const float*>(src), dst);
    TTSG_HIP(hipGetLastError());
}
inline char* adv(const void* p, int64_t elems, Prec pr) {
    return (char*)p + elems * (int64_t)elem_size(pr);
}
}  // namespace

namespace {

const uint8_t* blk_of(const SketchOperands& o, int mu) {
    return !o.D.empty() && !o.blk.empty() ? o.blk[mu] : nullptr;
}

// Two-stream form of the STTA sketch: the side stream computes the right
// environments F_b (right-to-left) and then Omega_b = E_b F_b; the calling
// stream computes the left environments E_mu with their T2 intermediates
// (left-to-right, all kept) and then Psi_mu = T2_mu F_{mu+1}.
void stta_sketch_two_streams(const SketchOperands& o, const std::vector<int>& r, const std::vector<const void*>& x,
                             double* const* Psi, double* const* Omega, Arena& ar, hipStream_t st,
                             const SketchSide& sd) {
    const int d = o.d;
    const int* n = o.n;
    const Prec p = o.p;
    const size_t es = elem_size(p);
    const bool op = !o.D.empty();
    auto Rk = [&](int b) { return op ? o.R[b] : 1; };
    Arena& ar2 = *sd.ar;
    const size_t mark = ar.mark(), mark2 = ar2.mark();
    // side stream scratch: right-step intermediates
    int64_t u1 = 1, u2 = 1, t1 = 1;
    for (int mu = 0; mu < d; ++mu) {
        const int rl = r[mu], rr = r[mu + 1], nn = n[mu];
        u1 = std::max<int64_t>(u1, (int64_t)rl * nn * Rk(mu + 1) * o.rx[mu + 1]);
        u2 = std::max<int64_t>(u2, (int64_t)rl * Rk(mu) * nn * o.rx[mu + 1]);
        t1 = std::max<int64_t>(t1, (int64_t)o.rho[mu] * Rk(mu) * nn * rr);
    }
    void* U1 = ar2.get<char>(u1 * es);
    void* U2 = ar2.get<char>(u2 * es);
    // main stream scratch: T1, the kept T2 of every mode, all left
    // environments, the right environments (written by the side stream)
    void* T1 = ar.get<char>(t1 * es);
    std::vector<void*> T2(d, nullptr), E(d, nullptr), F(d + 1, nullptr);
    for (int mu = 0; mu < d; ++mu) {
        const int64_t t2 = (int64_t)o.rho[mu] * n[mu] * Rk(mu + 1) * r[mu + 1];
        T2[mu] = ar.get<char>((op ? t2 : (int64_t)o.rho[mu] * Rk(mu) * n[mu] * r[mu + 1]) * es);
        E[mu] = ar.get<char>(std::max<int64_t>((int64_t)o.rho[mu] * Rk(mu) * r[mu], 2) * es);
    }
    for (int b = 1; b <= d; ++b) F[b] = ar.get<char>((int64_t)r[b] * Rk(b) * o.rx[b] * es);

    // side: right sweep
    TTSG_HIP(hipEventRecord(sd.in, st));
    TTSG_HIP(hipStreamWaitEvent(sd.st, sd.in, 0));
    set_one(p, F[d], sd.st);
    for (int mu = d - 1; mu >= 1; --mu) {
        LeftDims s{r[mu], n[mu], r[mu + 1], Rk(mu), Rk(mu + 1), o.rx[mu], o.rx[mu + 1], blk_of(o, mu)};
        right_step(p, s, F[mu + 1], x[mu], op ? o.D[mu] : nullptr, o.X[mu - 1], U1, U2, F[mu], sd.st, &ar2);
    }
    TTSG_HIP(hipEventRecord(sd.right, sd.st));
    // main: left sweep, keeping T2 and E of every mode
    set_one(p, E[0], st);
    for (int mu = 0; mu < d; ++mu) {
        LeftDims s{r[mu], n[mu], r[mu + 1], Rk(mu), Rk(mu + 1), o.rho[mu], mu + 1 < d ? o.rho[mu + 1] : 1,
                   blk_of(o, mu)};
        // without an operator the first stage's output is the intermediate
        left_step(p, s, E[mu], x[mu], op ? o.D[mu] : nullptr, nullptr, op ? T1 : T2[mu], op ? T2[mu] : nullptr,
                  nullptr, st, &ar);
        if (mu + 1 < d) {
            ContractDesc dd = cdesc(o.rho[mu + 1], Rk(mu + 1) * r[mu + 1], o.rho[mu] * n[mu]);
            dd.am = idx1(1);
            dd.ak = idx1(o.rho[mu + 1]);
            dd.bk = idx1((int64_t)Rk(mu + 1) * r[mu + 1]);
            dd.bn = idx1(1);
            dd.cm = idx1((int64_t)Rk(mu + 1) * r[mu + 1]);
            dd.cn = idx1(1);
            contract(p, dd, o.Y[mu], T2[mu], E[mu + 1], st, &ar);
        }
    }
    TTSG_HIP(hipEventRecord(sd.left, st));
    // side: Omega_b = E_b F_b once the left sweep is done
    TTSG_HIP(hipStreamWaitEvent(sd.st, sd.left, 0));
    for (int b = 1; b <= d - 1; ++b)
        omega_step(p, o.rho[b], Rk(b), r[b], o.rx[b], E[b], F[b], Omega[b - 1], sd.st, &ar2, true);
    TTSG_HIP(hipEventRecord(sd.done, sd.st));
    // main: Psi_mu = T2_mu F_{mu+1} once the right sweep is done
    TTSG_HIP(hipStreamWaitEvent(st, sd.right, 0));
    for (int mu = 0; mu < d; ++mu)
        psi_step(p, o.rho[mu], n[mu], Rk(mu + 1), r[mu + 1], o.rx[mu + 1], T2[mu], F[mu + 1], Psi[mu], st, &ar, true);
    // everything (and the side stream's use of this scratch) ends before st goes on
    TTSG_HIP(hipStreamWaitEvent(st, sd.done, 0));
    ar2.release(mark2);
    ar.release(mark);
}

}  // namespace

void stta_sketch(const SketchOperands& o, const std::vector<int>& r, const std::vector<const void*>& x,
                 double* const* Psi, double* const* Omega, Arena& ar, hipStream_t st, const SketchSide* side) {
    if (side != nullptr && side->st != nullptr && o.d >= 2) {
        stta_sketch_two_streams(o, r, x, Psi, Omega, ar, st, *side);
        return;
    }
    const int d = o.d;
    const int* n = o.n;
    const Prec p = o.p;
    const size_t es = elem_size(p);
    const size_t mark = ar.mark();
    const bool op = !o.D.empty();
    auto Rk = [&](int b) { return op ? o.R[b] : 1; };
    // scratch sizes
    int64_t t1 = 1, t2 = 1, u1 = 1, u2 = 1, env = 1;
    for (int mu = 0; mu < d; ++mu) {
        const int rl = r[mu], rr = r[mu + 1], nn = n[mu];
        t1 = std::max<int64_t>(t1, (int64_t)o.rho[mu] * Rk(mu) * nn * rr);
        t2 = std::max<int64_t>(t2, (int64_t)o.rho[mu] * nn * Rk(mu + 1) * rr);
        u1 = std::max<int64_t>(u1, (int64_t)rl * nn * Rk(mu + 1) * o.rx[mu + 1]);
        u2 = std::max<int64_t>(u2, (int64_t)rl * Rk(mu) * nn * o.rx[mu + 1]);
        env = std::max<int64_t>(env, (int64_t)o.rho[mu + 1] * Rk(mu + 1) * rr);
    }
    void* T1 = ar.get<char>(t1 * es);
    void* T2 = ar.get<char>(t2 * es);
    void* U1 = ar.get<char>(u1 * es);
    void* U2 = ar.get<char>(u2 * es);
    void* Ea = ar.get<char>(env * es);
    void* Eb = ar.get<char>(env * es);
    void* one = ar.get<char>(16);
    // right environments F_b for b = d..1 (F_d = 1)
    std::vector<void*> F(d + 1, nullptr);
    for (int b = 1; b <= d; ++b) F[b] = ar.get<char>((int64_t)r[b] * Rk(b) * o.rx[b] * es);
    set_one(p, F[d], st);
    for (int mu = d - 1; mu >= 1; --mu) {
        LeftDims s{r[mu], n[mu], r[mu + 1], Rk(mu), Rk(mu + 1), o.rx[mu], o.rx[mu + 1], blk_of(o, mu)};
        right_step(p, s, F[mu + 1], x[mu], op ? o.D[mu] : nullptr, o.X[mu - 1], U1, U2, F[mu], st, &ar);
    }
    // left sweep with Psi and Omega
    set_one(p, Ea, st);
    void* E = Ea;
    void* En = Eb;
    for (int mu = 0; mu < d; ++mu) {
        LeftDims s{r[mu], n[mu], r[mu + 1], Rk(mu), Rk(mu + 1), o.rho[mu], mu + 1 < d ? o.rho[mu + 1] : 1,
                   blk_of(o, mu)};
        const bool last = (mu == d - 1);
        left_step(p, s, E, x[mu], op ? o.D[mu] : nullptr, nullptr, T1, T2, nullptr, st, &ar);
        const void* T2r = op ? T2 : T1;
        psi_step(p, o.rho[mu], n[mu], Rk(mu + 1), r[mu + 1], o.rx[mu + 1], T2r, F[mu + 1], Psi[mu], st, &ar, true);
        if (!last) {
            // E_{mu+1} = Y_mu contracted with T2
            ContractDesc dd = cdesc(o.rho[mu + 1], Rk(mu + 1) * r[mu + 1], o.rho[mu] * n[mu]);
            dd.am = idx1(1);
            dd.ak = idx1(o.rho[mu + 1]);
            dd.bk = idx1((int64_t)Rk(mu + 1) * r[mu + 1]);
            dd.bn = idx1(1);
            dd.cm = idx1((int64_t)Rk(mu + 1) * r[mu + 1]);
            dd.cn = idx1(1);
            contract(p, dd, o.Y[mu], T2r, En, st, &ar);
            const int b = mu + 1;
            omega_step(p, o.rho[b], Rk(b), r[b], o.rx[b], En, F[b], Omega[b - 1], st, &ar, true);
            std::swap(E, En);
        }
    }
    ar.release(mark);
    (void)adv;
}

void kr_sketch_run(Prec p, int d, const int* n, int s, const std::vector<int>& R,
                   const std::vector<const void*>& SA, const std::vector<int>& r,
                   const std::vector<const void*>& x, double* w, Arena& ar, hipStream_t st) {
    const size_t es = elem_size(p);
    const size_t mark = ar.mark();
    int64_t pmax = 1, xmax = 1;
    for (int mu = 0; mu < d; ++mu) {
        pmax = std::max<int64_t>(pmax, (int64_t)s * R[mu + 1] * r[mu + 1]);
        xmax = std::max<int64_t>(xmax, (int64_t)s * R[mu + 1] * r[mu] * n[mu]);
    }
    void* Pa = ar.get<char>(std::max<int64_t>(pmax, s) * es);
    void* Pb = ar.get<char>(std::max<int64_t>(pmax, s) * es);
    void* Xb = ar.get<char>(xmax * es);
    // P_0 = 1 for every sketch row
    if (p == Prec::F64) {
        fill(s, 1.0, static_cast<double*>(Pa), st);
    } else {
        // float ones: fill a double temp then convert
        double* tmpd = ar.get<double>(s);
        fill(s, 1.0, tmpd, st);
        convert_f64_f32(s, tmpd, static_cast<float*>(Pa), st);
    }
    void* P = Pa;
    void* Pn = Pb;
    for (int mu = 0; mu < d; ++mu) {
        kr_step(p, s, r[mu], n[mu], r[mu + 1], R[mu], R[mu + 1], P, SA[mu], x[mu], Xb, Pn, st, &ar);
        std::swap(P, Pn);
    }
    to_f64(p, s, P, w, st);
    ar.release(mark);
}

void inner_run(Prec p, int d, const int* n, const std::vector<int>& R, const std::vector<const void*>& D,
               const std::vector<int>& rx_, const std::vector<const void*>& x, const std::vector<int>& rz,
               const std::vector<const void*>& z, double* out_dev, Arena& ar, hipStream_t st,
               const std::vector<const uint8_t*>& blk) {
    const size_t es = elem_size(p);
    const size_t mark = ar.mark();
    const bool op = !D.empty();
    auto Rk = [&](int b) { return op ? R[b] : 1; };
    int64_t t1 = 1, t2 = 1, env = 1;
    for (int mu = 0; mu < d; ++mu) {
        t1 = std::max<int64_t>(t1, (int64_t)rz[mu] * Rk(mu) * n[mu] * rx_[mu + 1]);
        t2 = std::max<int64_t>(t2, (int64_t)rz[mu] * n[mu] * Rk(mu + 1) * rx_[mu + 1]);
        env = std::max<int64_t>(env, (int64_t)rz[mu + 1] * Rk(mu + 1) * rx_[mu + 1]);
    }
    void* T1 = ar.get<char>(t1 * es);
    void* T2 = ar.get<char>(t2 * es);
    void* Ea = ar.get<char>(env * es);
    void* Eb = ar.get<char>(env * es);
    set_one(p, Ea, st);
    void* E = Ea;
    void* En = Eb;
    for (int mu = 0; mu < d; ++mu) {
        LeftDims s{rx_[mu], n[mu], rx_[mu + 1], Rk(mu), Rk(mu + 1), rz[mu], rz[mu + 1],
                   op && !blk.empty() ? blk[mu] : nullptr};
        left_step(p, s, E, x[mu], op ? D[mu] : nullptr, z[mu], T1, T2, En, st, &ar);
        std::swap(E, En);
    }
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, st, E, p == Prec::F64 ? 1 : 0, out_dev);
    TTSG_HIP(hipGetLastError());
    ar.release(mark);
}

}  // namespace ttsg
