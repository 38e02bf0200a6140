// Element-wise and reduction kernels used between the contractions.
#include "ttsg_internal.h"
#include "xlane.h"

namespace ttsg {
namespace {

constexpr int TPB = 256;

inline int nblocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

__global__ void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}

__global__ void k_scale(int64_t n, double a, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] *= a;
}

__global__ void k_f64_f32(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

__global__ void k_f32_f64(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

// float64 -> bfloat16 with round-to-nearest-even on the float32 value.
__global__ void k_f64_bf16(int64_t n, const double* __restrict__ x, uint16_t* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float f = (float)x[i];
        uint32_t u = __float_as_uint(f);
        if ((u & 0x7f800000u) == 0x7f800000u) {
            y[i] = (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
        } else {
            uint32_t lsb = (u >> 16) & 1u;
            u += 0x7fffu + lsb;
            y[i] = (uint16_t)(u >> 16);
        }
    }
}

struct Ptrs8 {
    const double* p[8];
    double sign[8];
};

__global__ void k_lin_comb(int64_t n, int32_t nt, Ptrs8 xs, const double* __restrict__ coef, double* __restrict__ y) {
    double c[8];
    for (int t = 0; t < nt; ++t) c[t] = xs.sign[t] * (coef ? coef[t] : 1.0);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) acc += c[t] * xs.p[t][i];
        y[i] = acc;
    }
}


__global__ void k_sumsq_part(int64_t n, const double* __restrict__ x, double* __restrict__ part) {
    __shared__ double red[TPB / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += x[i] * x[i];
    acc = wave_sum64(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < TPB / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

__global__ void k_sum_final(int32_t np, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[TPB / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
    acc = wave_sum64(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < TPB / 64; ++w) s += red[w];
        out[0] = s;
    }
}

__global__ void k_copy2d(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                         double* __restrict__ dst, int64_t ldd) {
    int64_t total = rows * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e / cols, c = e - r * cols;
        dst[r * ldd + c] = src[r * lds + c];
    }
}

// dst[c][r] = src[r][c]; 32x32 tiles through LDS.
__global__ void k_transpose2d(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                              double* __restrict__ dst, int64_t ldd) {
    __shared__ double t[32][33];
    int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        int64_t r = r0 + k, c = c0 + tx;
        t[k][tx] = (r < rows && c < cols) ? src[r * lds + c] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        int64_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) dst[c * ldd + r] = t[tx][k];
    }
}

}  // namespace

void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(TPB), 0, st, n, a, x, b, y);
    TTSG_HIP(hipGetLastError());
}
namespace {
struct HostStage {
    double* p = nullptr;
    bool tried = false;
    ~HostStage() {
        if (p != nullptr) (void)hipHostFree(p);
    }
};
}  // namespace

double* host_stage(int region) {
    thread_local HostStage s;
    if (!s.tried) {
        s.tried = true;
        if (hipHostMalloc(reinterpret_cast<void**>(&s.p), 2 * kStageDoubles * sizeof(double), hipHostMallocDefault) !=
            hipSuccess) {
            s.p = nullptr;
            (void)hipGetLastError();
        }
    }
    return s.p != nullptr ? s.p + (region != 0 ? kStageDoubles : 0) : nullptr;
}

const void* read_back(const void* dev, size_t bytes, void* fallback, hipStream_t st) {
    double* stage = bytes <= kStageDoubles * sizeof(double) ? host_stage(0) : nullptr;
    void* dst = stage != nullptr ? static_cast<void*>(stage) : fallback;
    TTSG_HIP(hipMemcpyAsync(dst, dev, bytes, hipMemcpyDeviceToHost, st));
    TTSG_HIP(hipStreamSynchronize(st));
    return dst;
}

void fill(int64_t n, double v, double* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(TPB), 0, st, n, v, y);
    TTSG_HIP(hipGetLastError());
}
void copy_f64(int64_t n, const double* x, double* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(nblocks(n)), dim3(TPB), 0, st, n, x, y);
    TTSG_HIP(hipGetLastError());
}
void scale_f64(int64_t n, double a, double* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale, dim3(nblocks(n)), dim3(TPB), 0, st, n, a, y);
    TTSG_HIP(hipGetLastError());
}
void convert_f64_f32(int64_t n, const double* x, float* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f64_f32, dim3(nblocks(n)), dim3(TPB), 0, st, n, x, y);
    TTSG_HIP(hipGetLastError());
}
void convert_f32_f64(int64_t n, const float* x, double* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f32_f64, dim3(nblocks(n)), dim3(TPB), 0, st, n, x, y);
    TTSG_HIP(hipGetLastError());
}
void convert_f64_bf16(int64_t n, const double* x, uint16_t* y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_f64_bf16, dim3(nblocks(n)), dim3(TPB), 0, st, n, x, y);
    TTSG_HIP(hipGetLastError());
}
void lin_comb_dev(int64_t n, int32_t nterms, const double* const* xs, const double* coef_dev,
                  const double* coef_sign, double* y, hipStream_t st) {
    TTSG_CHECK(nterms >= 1 && nterms <= 8, TTSG_ERR_ARG, "lin_comb: 1..8 terms");
    if (n <= 0) return;
    Ptrs8 p{};
    for (int t = 0; t < nterms; ++t) {
        p.p[t] = xs[t];
        p.sign[t] = coef_sign ? coef_sign[t] : 1.0;
    }
    hipLaunchKernelGGL(k_lin_comb, dim3(nblocks(n)), dim3(TPB), 0, st, n, nterms, p, coef_dev, y);
    TTSG_HIP(hipGetLastError());
}
void sumsq(int64_t n, const double* x, double* part, double* out, hipStream_t st) {
    int nb = nblocks(n);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_sumsq_part, dim3(nb), dim3(TPB), 0, st, n, x, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, st, nb, part, out);
    TTSG_HIP(hipGetLastError());
}
void copy2d(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(k_copy2d, dim3(nblocks(rows * cols)), dim3(TPB), 0, st, rows, cols, src, lds, dst, ldd);
    TTSG_HIP(hipGetLastError());
}
void transpose2d(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd,
                 hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    TTSG_CHECK((rows + 31) / 32 < 65536, TTSG_ERR_ARG, "transpose: too many rows");
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(k_transpose2d, grid, dim3(256), 0, st, rows, cols, src, lds, dst, ldd);
    TTSG_HIP(hipGetLastError());
}

}  // namespace ttsg
