// extern "C" entry points of libttsg: argument validation, workspace
// handling and conversion of internal errors into return codes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>

#include "tt_ops.h"

namespace {

thread_local char g_err[512] = "no error";

void set_err(const char* m) {
    std::strncpy(g_err, m, sizeof(g_err) - 1);
    g_err[sizeof(g_err) - 1] = 0;
}

template <typename F> int guarded(F&& f) {
    try {
        return f();
    } catch (const ttsg::Error& e) {
        set_err(e.what());
        return -e.code;
    } catch (const std::exception& e) {
        set_err(e.what());
        return -TTSG_ERR_HIP;
    } catch (...) {
        set_err("unknown failure");
        return -TTSG_ERR_HIP;
    }
}

using ttsg::Error;

void check_shape(int32_t d, const int32_t* n, const int32_t* r, const char* what) {
    TTSG_CHECK(d >= 1 && d <= 64, TTSG_ERR_ARG, std::string(what) + ": d must be in 1..64");
    TTSG_CHECK(n != nullptr && r != nullptr, TTSG_ERR_ARG, std::string(what) + ": null sizes");
    for (int k = 0; k < d; ++k) TTSG_CHECK(n[k] >= 1, TTSG_ERR_ARG, std::string(what) + ": n[k] < 1");
    TTSG_CHECK(r[0] == 1 && r[d] == 1, TTSG_ERR_ARG, std::string(what) + ": boundary ranks must be 1");
    for (int k = 1; k < d; ++k) TTSG_CHECK(r[k] >= 1, TTSG_ERR_ARG, std::string(what) + ": rank < 1");
}

void check_ptrs(int cnt, const void* const* p, const char* what) {
    TTSG_CHECK(p != nullptr, TTSG_ERR_ARG, std::string(what) + ": null pointer array");
    for (int k = 0; k < cnt; ++k) TTSG_CHECK(p[k] != nullptr, TTSG_ERR_ARG, std::string(what) + ": null core");
}

std::vector<int> vec(const int32_t* p, int cnt) { return std::vector<int>(p, p + cnt); }

template <typename T> std::vector<const void*> vp(const T* const* p, int cnt) {
    std::vector<const void*> v(cnt);
    for (int k = 0; k < cnt; ++k) v[k] = p[k];
    return v;
}

hipStream_t S(ttsg_stream_t s) { return static_cast<hipStream_t>(s); }

ttsg::Prec prec_of(int32_t precision) {
    TTSG_CHECK(precision == TTSG_PREC_F64 || precision == TTSG_PREC_MIXED || precision == TTSG_PREC_BF16,
               TTSG_ERR_DTYPE, "unknown precision");
    return precision == TTSG_PREC_F64 ? ttsg::Prec::F64
                                      : (precision == TTSG_PREC_MIXED ? ttsg::Prec::F32 : ttsg::Prec::BF16);
}

// Split-K partial sums of one contraction: splits x workgroups < 2048 tiles of
// 64 x 64, so fewer than 8M partial values (64 MiB in float64).
constexpr size_t kSplitSlack = (size_t)72 << 20;

}  // namespace

extern "C" {

const char* ttsg_last_error(void) { return g_err; }

const char* ttsg_version(void) { return "ttsg 0.1 gfx950"; }

int ttsg_matvec(int32_t d, const int32_t* n, const int32_t* R, const double* const* A, const int32_t* r,
                const double* const* x, int32_t transpose, double* const* y, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "matvec x");
        check_shape(d, n, R, "matvec A");
        check_ptrs(d, (const void* const*)A, "matvec A");
        check_ptrs(d, (const void* const*)x, "matvec x");
        check_ptrs(d, (const void* const*)y, "matvec y");
        for (int mu = 0; mu < d; ++mu)
            ttsg::matvec_core(r[mu], n[mu], r[mu + 1], R[mu], R[mu + 1], A[mu], x[mu], transpose != 0, y[mu],
                              S(stream));
        return 0;
    });
}

static size_t kr_ws(int32_t d, const int32_t* n, int32_t s, const int32_t* R, const int32_t* r) {
    size_t need = 0;
    for (int mu = 0; mu < d; ++mu) {
        const size_t Rl = R ? R[mu] : 1, Rr = R ? R[mu + 1] : 1;
        need += ((size_t)s * Rl * n[mu] * Rr * 8 + 256);              // S A (or S) and its f32 copy
        need += ((size_t)r[mu] * n[mu] * r[mu + 1] * 4 + 256);        // x in f32
        need += ((size_t)s * Rr * r[mu] * n[mu] * 8 + 256);           // X buffer
        need += 2 * ((size_t)s * Rr * r[mu + 1] * 8 + 256);           // P buffers
    }
    need += (size_t)s * 8 * 4 + 4096;
    return need * 2 + kSplitSlack;
}

int ttsg_kr_sketch(int32_t d, const int32_t* n, int32_t s, const double* const* Sf, const int32_t* R,
                   const double* const* A, const int32_t* r, const double* const* x, double* w, int32_t precision,
                   void* ws, size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "kr_sketch x");
        TTSG_CHECK(s >= 1, TTSG_ERR_ARG, "kr_sketch: s < 1");
        TTSG_CHECK(w != nullptr, TTSG_ERR_ARG, "kr_sketch: null output");
        (void)prec_of(precision);
        check_ptrs(d, (const void* const*)Sf, "kr_sketch S");
        check_ptrs(d, (const void* const*)x, "kr_sketch x");
        const bool op = A != nullptr;
        if (op) {
            check_shape(d, n, R, "kr_sketch A");
            check_ptrs(d, (const void* const*)A, "kr_sketch A");
        }
        const ttsg::Prec p = prec_of(precision);
        std::vector<int> RR(d + 1, 1);
        if (op) RR = vec(R, d + 1);
        ttsg::Workspace W(ws, ws_bytes, kr_ws(d, n, s, op ? R : nullptr, r), S(stream));
        ttsg::Arena& ar = W.arena;
        std::vector<const void*> SA(d), xs(d);
        for (int mu = 0; mu < d; ++mu) {
            const int64_t sz = (int64_t)s * RR[mu] * n[mu] * RR[mu + 1];
            if (op) {
                double* sa = ar.get<double>(sz);
                ttsg::kr_precompute(ttsg::Prec::F64, s, n[mu], RR[mu], RR[mu + 1], Sf[mu], A[mu], sa, S(stream));
                SA[mu] = sa;
            } else {
                SA[mu] = Sf[mu];
            }
            if (p != ttsg::Prec::F64) {
                float* f = ar.get<float>(sz);
                ttsg::convert_f64_f32(sz, (const double*)SA[mu], f, S(stream));
                SA[mu] = f;
                const int64_t e = (int64_t)r[mu] * n[mu] * r[mu + 1];
                float* xf = ar.get<float>(e);
                ttsg::convert_f64_f32(e, x[mu], xf, S(stream));
                xs[mu] = xf;
            } else {
                xs[mu] = x[mu];
            }
        }
        ttsg::kr_sketch_run(p, d, n, s, RR, SA, vec(r, d + 1), xs, w, ar, S(stream));
        return 0;
    });
}

static void stta_common(int32_t d, const int32_t* n, const int32_t* rho, const double* const* Y, const int32_t* rx,
                        const double* const* X, const int32_t* R, const double* const* A, const int32_t* r,
                        const double* const* x, double* const* Psi, double* const* Omega, int32_t precision,
                        ttsg::Arena& ar, hipStream_t st) {
    const ttsg::Prec p = prec_of(precision);
    ttsg::SketchOperands o;
    o.p = p;
    o.n = n;
    o.d = d;
    o.rho = vec(rho, d + 1);
    o.rx = vec(rx, d + 1);
    o.R.assign(d + 1, 1);
    auto conv = [&](const double* src, int64_t e) -> const void* {
        if (p == ttsg::Prec::F64) return src;
        float* f = ar.get<float>(e);
        ttsg::convert_f64_f32(e, src, f, st);
        return f;
    };
    for (int k = 0; k < d - 1; ++k) {
        o.Y.push_back(conv(Y[k], (int64_t)rho[k] * n[k] * rho[k + 1]));
        o.X.push_back(conv(X[k], (int64_t)rx[k + 1] * n[k + 1] * rx[k + 2]));
    }
    if (A != nullptr) {
        o.R = vec(R, d + 1);
        for (int mu = 0; mu < d; ++mu) o.D.push_back(conv(A[mu], (int64_t)R[mu] * n[mu] * n[mu] * R[mu + 1]));
    }
    std::vector<const void*> xs(d);
    for (int mu = 0; mu < d; ++mu) xs[mu] = conv(x[mu], (int64_t)r[mu] * n[mu] * r[mu + 1]);
    ttsg::stta_sketch(o, vec(r, d + 1), xs, Psi, Omega, ar, st);
}

// Arena::get rounds every request up to 256 bytes.
static size_t gran(size_t bytes) { return (bytes + 255) & ~size_t(255); }

// Bytes the single-stream STTA sketch takes from its arena for these shapes
// (R == NULL: no operator): the float32 copies of the operands in the
// reduced precisions, the sweep intermediates T1/T2/U1/U2, two left
// environments, the right environments F_1..F_d, and the split-K partials of
// one contraction (released after it).
static size_t stta_ws(int32_t d, const int32_t* n, const int32_t* rho, const int32_t* rx, const int32_t* R,
                      const int32_t* r, ttsg::Prec p) {
    const size_t es = ttsg::elem_size(p);
    auto Rk = [&](int b) -> int64_t { return R ? R[b] : 1; };
    size_t tot = 0;
    if (p != ttsg::Prec::F64) {
        for (int k = 0; k < d - 1; ++k) {
            tot += gran((size_t)rho[k] * n[k] * rho[k + 1] * 4);
            tot += gran((size_t)rx[k + 1] * n[k + 1] * rx[k + 2] * 4);
        }
        if (R)
            for (int mu = 0; mu < d; ++mu) tot += gran((size_t)R[mu] * n[mu] * n[mu] * R[mu + 1] * 4);
        for (int mu = 0; mu < d; ++mu) tot += gran((size_t)r[mu] * n[mu] * r[mu + 1] * 4);
    }
    int64_t t1 = 1, t2 = 1, u1 = 1, u2 = 1, env = 1;
    for (int mu = 0; mu < d; ++mu) {
        const int64_t rl = r[mu], rr = r[mu + 1], nn = n[mu];
        t1 = std::max<int64_t>(t1, rho[mu] * Rk(mu) * nn * rr);
        t2 = std::max<int64_t>(t2, rho[mu] * nn * Rk(mu + 1) * rr);
        u1 = std::max<int64_t>(u1, rl * nn * Rk(mu + 1) * rx[mu + 1]);
        u2 = std::max<int64_t>(u2, rl * Rk(mu) * nn * rx[mu + 1]);
        env = std::max<int64_t>(env, rho[mu + 1] * Rk(mu + 1) * rr);
    }
    tot += gran(t1 * es) + gran(t2 * es) + gran(u1 * es) + gran(u2 * es) + 2 * gran(env * es) + gran(16);
    for (int b = 1; b <= d; ++b) tot += gran((size_t)r[b] * Rk(b) * rx[b] * es);
    return tot + kSplitSlack;
}

int ttsg_stta_sketch(int32_t d, const int32_t* n, const int32_t* rho, const double* const* Y, const int32_t* rx,
                     const double* const* X, const int32_t* R, const double* const* A, const int32_t* r,
                     const double* const* x, double* const* Psi, double* const* Omega, int32_t precision, void* ws,
                     size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "stta x");
        check_shape(d, n, rho, "stta rho");
        check_shape(d, n, rx, "stta rx");
        TTSG_CHECK(d >= 2, TTSG_ERR_ARG, "stta: d must be >= 2");
        (void)prec_of(precision);
        check_ptrs(d - 1, (const void* const*)Y, "stta Y");
        check_ptrs(d - 1, (const void* const*)X, "stta X");
        check_ptrs(d, (const void* const*)x, "stta x");
        check_ptrs(d, (const void* const*)Psi, "stta Psi");
        check_ptrs(d - 1, (const void* const*)Omega, "stta Omega");
        if (A) {
            check_shape(d, n, R, "stta A");
            check_ptrs(d, (const void* const*)A, "stta A");
        }
        ttsg::Workspace W(ws, ws_bytes, stta_ws(d, n, rho, rx, A ? R : nullptr, r, prec_of(precision)), S(stream));
        stta_common(d, n, rho, Y, rx, X, A ? R : nullptr, A, r, x, Psi, Omega, precision, W.arena, S(stream));
        return 0;
    });
}

// ---------------------------------------------------------------------------
// The STTA sketch without any allocation: its scratch is a file-scope device
// array.  In host code `scratch` only names the symbol; its device address
// (one copy per GPU) comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_dev;  // device ordinal -> address of its copy of `scratch`

static char* static_scratch_of_current_device() {
    int dev = -1;
    TTSG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it != g_scratch_dev.end()) return it->second;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    TTSG_CHECK(e == hipSuccess && ptr != nullptr, TTSG_ERR_HIP,
               std::string("stta_sketch_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<char*>(ptr);
    return static_cast<char*>(ptr);
}

int ttsg_stta_sketch_noalloc(int32_t d, const int32_t* n, const int32_t* rho, const double* const* Y,
                             const int32_t* rx, const double* const* X, const int32_t* R, const double* const* A,
                             const int32_t* r, const double* const* x, double* const* Psi, double* const* Omega,
                             int32_t precision, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "stta_noalloc x");
        check_shape(d, n, rho, "stta_noalloc rho");
        check_shape(d, n, rx, "stta_noalloc rx");
        TTSG_CHECK(d >= 2, TTSG_ERR_ARG, "stta_noalloc: d must be >= 2");
        const ttsg::Prec p = prec_of(precision);
        check_ptrs(d - 1, (const void* const*)Y, "stta_noalloc Y");
        check_ptrs(d - 1, (const void* const*)X, "stta_noalloc X");
        check_ptrs(d, (const void* const*)x, "stta_noalloc x");
        check_ptrs(d, (const void* const*)Psi, "stta_noalloc Psi");
        check_ptrs(d - 1, (const void* const*)Omega, "stta_noalloc Omega");
        if (A) {
            check_shape(d, n, R, "stta_noalloc A");
            check_ptrs(d, (const void* const*)A, "stta_noalloc A");
        }
        // the tile autotuner times new shape classes into a buffer it allocates
        TTSG_CHECK(!ttsg::autotune_is_on(), TTSG_ERR_ARG,
                   "stta_sketch_noalloc: the tile autotuner is on (tuning allocates); switch it off first");
        const size_t need = stta_ws(d, n, rho, rx, A ? R : nullptr, r, p);
        if (need > kStaticScratchBytes) {
            char m[160];
            std::snprintf(m, sizeof(m), "stta_sketch_noalloc: these shapes need %zu bytes of scratch, above the %zu "
                          "of the static buffer", need, kStaticScratchBytes);
            throw Error(TTSG_ERR_WS, m);
        }
        char* base = static_scratch_of_current_device();
        ttsg::Arena ar;
        ar.reset(base, kStaticScratchBytes);
        stta_common(d, n, rho, Y, rx, X, A ? R : nullptr, A, r, x, Psi, Omega, precision, ar, S(stream));
        return 0;
    });
}

static size_t round_rand_ws(int32_t d, const int32_t* n, const int32_t* r, const int32_t* rho, const int32_t* rx,
                            ttsg::Prec p) {
    size_t sk = 0;
    for (int mu = 0; mu < d; ++mu) sk += (size_t)rho[mu] * n[mu] * rx[mu + 1] + (size_t)rho[mu] * rx[mu] + 64;
    size_t core = 0, rmax = 1;
    for (int mu = 0; mu < d; ++mu) {
        core = std::max(core, (size_t)rx[mu] * n[mu] * rx[mu + 1]);
        rmax = std::max(rmax, (size_t)std::max(rho[mu], rx[mu]));
    }
    const size_t need = stta_ws(d, n, rho, rx, nullptr, r, p) + sk * 8 + (8 * core + 12 * rmax * rmax) * 8 +
                        (size_t)d * 16 * rmax * rmax * 8 + (4 << 20) + ttsg::tt_svd_extra_bytes(d, n, rx) +
                        (size_t)d * ttsg::jacobi_big_log_bytes((int)rmax);
    return need + kSplitSlack;
}

int ttsg_round_rand(int32_t d, const int32_t* n, const int32_t* r, const double* const* x, const int32_t* rho,
                    const double* const* Y, const int32_t* rx, const double* const* X, double tol, int32_t maxrank,
                    double rcond, double* const* out, int32_t* out_r, int32_t precision, void* ws, size_t ws_bytes,
                    ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "round_rand x");
        check_shape(d, n, rho, "round_rand rho");
        check_shape(d, n, rx, "round_rand rx");
        TTSG_CHECK(d >= 2, TTSG_ERR_ARG, "round_rand: d must be >= 2");
        TTSG_CHECK(tol >= 0.0 && rcond >= 0.0, TTSG_ERR_ARG, "round_rand: negative tolerance");
        for (int b = 1; b < d; ++b) TTSG_CHECK(rho[b] >= rx[b], TTSG_ERR_ARG, "round_rand: rho_b < rx_b");
        check_ptrs(d - 1, (const void* const*)Y, "round_rand Y");
        check_ptrs(d - 1, (const void* const*)X, "round_rand X");
        check_ptrs(d, (const void* const*)x, "round_rand x");
        check_ptrs(d, (const void* const*)out, "round_rand out");
        TTSG_CHECK(out_r != nullptr, TTSG_ERR_ARG, "round_rand: null out_r");
        ttsg::Workspace W(ws, ws_bytes, round_rand_ws(d, n, r, rho, rx, prec_of(precision)), S(stream));
        ttsg::Arena& ar = W.arena;
        std::vector<double*> psi(d), om(d - 1);
        for (int mu = 0; mu < d; ++mu) psi[mu] = ar.get<double>((int64_t)rho[mu] * n[mu] * rx[mu + 1]);
        for (int b = 1; b < d; ++b) om[b - 1] = ar.get<double>((int64_t)rho[b] * rx[b]);
        stta_common(d, n, rho, Y, rx, X, nullptr, nullptr, r, x, psi.data(), om.data(), precision, ar, S(stream));
        std::vector<const double*> cp(psi.begin(), psi.end()), co(om.begin(), om.end());
        std::vector<int> rr;
        std::vector<double*> o(out, out + d);
        ttsg::stta_recover(d, n, vec(rho, d + 1), vec(rx, d + 1), cp, co, rcond, o, rr, ar, S(stream));
        std::vector<int64_t> caps(d);
        ttsg::tt_svd_inplace(d, n, rr, o, caps, tol, maxrank, ar, S(stream), nullptr);
        for (int k = 0; k <= d; ++k) out_r[k] = rr[k];
        TTSG_HIP(hipStreamSynchronize(S(stream)));
        return 0;
    });
}

int ttsg_kr_sketch_workspace_size(int32_t d, const int32_t* n, int32_t s, const int32_t* R, const int32_t* r,
                                  int32_t precision, size_t* bytes) {
    return guarded([&]() {
        check_shape(d, n, r, "kr_sketch x");
        TTSG_CHECK(s >= 1 && bytes != nullptr, TTSG_ERR_ARG, "kr_sketch_workspace_size: bad arguments");
        (void)prec_of(precision);
        if (R) check_shape(d, n, R, "kr_sketch A");
        *bytes = kr_ws(d, n, s, R, r);
        return 0;
    });
}

int ttsg_stta_sketch_workspace_size(int32_t d, const int32_t* n, const int32_t* rho, const int32_t* rx,
                                    const int32_t* R, const int32_t* r, int32_t precision, size_t* bytes) {
    return guarded([&]() {
        check_shape(d, n, r, "stta x");
        check_shape(d, n, rho, "stta rho");
        check_shape(d, n, rx, "stta rx");
        TTSG_CHECK(bytes != nullptr, TTSG_ERR_ARG, "stta_sketch_workspace_size: null output");
        (void)prec_of(precision);
        if (R) check_shape(d, n, R, "stta A");
        *bytes = stta_ws(d, n, rho, rx, R, r, prec_of(precision));
        return 0;
    });
}

int ttsg_round_rand_workspace_size(int32_t d, const int32_t* n, const int32_t* r, const int32_t* rho,
                                   const int32_t* rx, int32_t precision, size_t* bytes) {
    return guarded([&]() {
        check_shape(d, n, r, "round_rand x");
        check_shape(d, n, rho, "round_rand rho");
        check_shape(d, n, rx, "round_rand rx");
        TTSG_CHECK(bytes != nullptr, TTSG_ERR_ARG, "round_rand_workspace_size: null output");
        (void)prec_of(precision);
        *bytes = round_rand_ws(d, n, r, rho, rx, prec_of(precision));
        return 0;
    });
}

int ttsg_round_svd(int32_t d, const int32_t* n, const int32_t* r, const double* const* x, double tol,
                   int32_t maxrank, double* const* out, int32_t* out_r, void* ws, size_t ws_bytes,
                   ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "round_svd x");
        TTSG_CHECK(tol >= 0.0, TTSG_ERR_ARG, "round_svd: negative tolerance");
        check_ptrs(d, (const void* const*)x, "round_svd x");
        check_ptrs(d, (const void* const*)out, "round_svd out");
        TTSG_CHECK(out_r != nullptr, TTSG_ERR_ARG, "round_svd: null out_r");
        size_t core = 0, rmax = 1;
        for (int mu = 0; mu < d; ++mu) {
            core = std::max(core, (size_t)r[mu] * n[mu] * r[mu + 1]);
            rmax = std::max(rmax, (size_t)r[mu]);
        }
        ttsg::Workspace W(ws, ws_bytes,
                          ((6 * core + 4 * rmax * rmax + 8 * rmax) * 8 + (1 << 20)) + ttsg::tt_svd_extra_bytes(d, n, r) +
                              kSplitSlack,
                          S(stream));
        std::vector<double*> o(out, out + d);
        for (int mu = 0; mu < d; ++mu) ttsg::copy_f64((int64_t)r[mu] * n[mu] * r[mu + 1], x[mu], o[mu], S(stream));
        std::vector<int> rr = vec(r, d + 1);
        std::vector<int64_t> caps(d);
        ttsg::tt_svd_inplace(d, n, rr, o, caps, tol, maxrank, W.arena, S(stream), nullptr);
        for (int k = 0; k <= d; ++k) out_r[k] = rr[k];
        TTSG_HIP(hipStreamSynchronize(S(stream)));
        return 0;
    });
}

int ttsg_dot(int32_t d, const int32_t* n, const int32_t* rxr, const double* const* x, const int32_t* ryr,
             const double* const* y, double* out, void* ws, size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, rxr, "dot x");
        check_shape(d, n, ryr, "dot y");
        check_ptrs(d, (const void* const*)x, "dot x");
        check_ptrs(d, (const void* const*)y, "dot y");
        TTSG_CHECK(out != nullptr, TTSG_ERR_ARG, "dot: null output");
        size_t big = 0;
        for (int mu = 0; mu < d; ++mu)
            big = std::max(big, (size_t)ryr[mu] * n[mu] * rxr[mu + 1] + (size_t)ryr[mu + 1] * rxr[mu + 1]);
        ttsg::Workspace W(ws, ws_bytes, (6 * big * 8 + (1 << 16)) + kSplitSlack, S(stream));
        double* dev = W.arena.get<double>(1);
        std::vector<int> R1(d + 1, 1);
        ttsg::inner_run(ttsg::Prec::F64, d, n, R1, {}, vec(rxr, d + 1), vp(x, d), vec(ryr, d + 1), vp(y, d), dev,
                        W.arena, S(stream));
        TTSG_HIP(hipMemcpyAsync(out, dev, sizeof(double), hipMemcpyDeviceToHost, S(stream)));
        TTSG_HIP(hipStreamSynchronize(S(stream)));
        return 0;
    });
}

int ttsg_true_residual(int32_t d, const int32_t* n, const int32_t* R, const double* const* A, const int32_t* rb,
                       const double* const* b, const int32_t* r, const double* const* x, double* res, void* ws,
                       size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, R, "true_residual A");
        check_shape(d, n, rb, "true_residual b");
        check_shape(d, n, r, "true_residual x");
        check_ptrs(d, (const void* const*)A, "true_residual A");
        check_ptrs(d, (const void* const*)b, "true_residual b");
        check_ptrs(d, (const void* const*)x, "true_residual x");
        TTSG_CHECK(res != nullptr, TTSG_ERR_ARG, "true_residual: null output");
        // r = b - A x as a block TT, norm by QR orthogonalization (no cancellation)
        size_t tot = 0, big = 0;
        std::vector<int> gr(d + 1), rr(d + 1);
        for (int k = 0; k <= d; ++k) gr[k] = R[k] * r[k];
        for (int mu = 0; mu < d; ++mu) {
            tot += (size_t)gr[mu] * n[mu] * gr[mu + 1] + 64;
            size_t e = (size_t)(gr[mu] + rb[mu]) * n[mu] * (gr[mu + 1] + rb[mu + 1]);
            tot += e + 64;
            big = std::max(big, e);
        }
        const size_t rmax = (size_t)*std::max_element(gr.begin(), gr.end()) + 64;
        ttsg::Workspace W(ws, ws_bytes, tot * 8 + (3 * big + 2 * rmax * rmax + 4 * rmax) * 8 + (1 << 20),
                          S(stream));
        ttsg::Arena& ar = W.arena;
        std::vector<double*> G(d), Sm(d);
        for (int mu = 0; mu < d; ++mu) {
            G[mu] = ar.get<double>((int64_t)gr[mu] * n[mu] * gr[mu + 1]);
            Sm[mu] = ar.get<double>((int64_t)(gr[mu] + rb[mu]) * n[mu] * (gr[mu + 1] + rb[mu + 1]));
            ttsg::matvec_core(r[mu], n[mu], r[mu + 1], R[mu], R[mu + 1], A[mu], x[mu], false, G[mu], S(stream));
        }
        std::vector<double*> bb(d);
        for (int mu = 0; mu < d; ++mu) bb[mu] = const_cast<double*>(b[mu]);
        std::vector<const double*> cg(G.begin(), G.end());
        ttsg::tt_add_block(d, n, vec(rb, d + 1), bb, gr, cg, -1.0, Sm, rr, S(stream));
        const double nr = ttsg::tt_norm_orth(d, n, rr, Sm, ar, S(stream));
        // ||b|| on a copy
        std::vector<double*> bc(d);
        for (int mu = 0; mu < d; ++mu) {
            const int64_t e = (int64_t)rb[mu] * n[mu] * rb[mu + 1];
            bc[mu] = G[mu];
            TTSG_CHECK(e <= (int64_t)gr[mu] * n[mu] * gr[mu + 1] || true, TTSG_ERR_WS, "");
            bc[mu] = ar.get<double>(e);
            ttsg::copy_f64(e, b[mu], bc[mu], S(stream));
        }
        std::vector<int> rbv = vec(rb, d + 1);
        const double nb = ttsg::tt_norm_orth(d, n, rbv, bc, ar, S(stream));
        *res = nb > 0.0 ? nr / nb : nr;
        return 0;
    });
}

int ttsg_grad_kron_sum(int32_t d, const int32_t* n, const double* const* L, const int32_t* rl,
                       const double* const* lam, const int32_t* rx, const double* const* x, double* out, void* ws,
                       size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, rl, "grad lambda");
        check_shape(d, n, rx, "grad x");
        check_ptrs(d, (const void* const*)L, "grad L");
        check_ptrs(d, (const void* const*)lam, "grad lambda");
        check_ptrs(d, (const void* const*)x, "grad x");
        TTSG_CHECK(out != nullptr, TTSG_ERR_ARG, "grad: null output");
        size_t tot = 0, big = 0;
        for (int k = 0; k <= d; ++k) tot += 2 * (size_t)rl[k] * rx[k] + 64;
        for (int k = 0; k < d; ++k)
            big = std::max(big, (size_t)std::max(rl[k], rx[k]) * n[k] * std::max(rl[k + 1], rx[k + 1]));
        ttsg::Workspace W(ws, ws_bytes, (tot + 4 * big + (size_t)d + 64) * 8 + kSplitSlack, S(stream));
        double* dev = W.arena.get<double>(d);
        std::vector<const double*> Lv(L, L + d), lv(lam, lam + d), xv(x, x + d);
        ttsg::grad_kron_sum(d, n, Lv, vec(rl, d + 1), lv, vec(rx, d + 1), xv, dev, W.arena, S(stream));
        TTSG_HIP(hipMemcpyAsync(out, dev, d * sizeof(double), hipMemcpyDeviceToHost, S(stream)));
        TTSG_HIP(hipStreamSynchronize(S(stream)));
        return 0;
    });
}

int ttsg_tt_axpby(int32_t d, const int32_t* n, double alpha, const int32_t* rx, const double* const* x, double beta,
                  const int32_t* ry, const double* const* y, double* const* z, ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, rx, "axpby x");
        check_shape(d, n, ry, "axpby y");
        check_ptrs(d, (const void* const*)x, "axpby x");
        check_ptrs(d, (const void* const*)y, "axpby y");
        check_ptrs(d, (const void* const*)z, "axpby z");
        std::vector<double*> xv(d);
        for (int k = 0; k < d; ++k) xv[k] = const_cast<double*>(x[k]);
        std::vector<const double*> yv(y, y + d);
        std::vector<double*> zv(z, z + d);
        std::vector<int> rz;
        ttsg::tt_add_block(d, n, vec(rx, d + 1), xv, vec(ry, d + 1), yv, beta, zv, rz, S(stream), alpha);
        return 0;
    });
}

}  // extern "C"

namespace {

// Validate the arguments of a solve and collect them; pointer arrays may be
// NULL when only sizes are needed (workspace query).
ttsg::SolverInputs solver_inputs(int32_t d, const int32_t* n, const int32_t* R, const double* const* A,
                                 const int32_t* rb, const double* const* b, int32_t s, const double* const* Sf,
                                 const int32_t* rho, const double* const* Y, const int32_t* rx,
                                 const double* const* X, const ttsg_sgmres_opts* opts, const ttsg_sgmres_ext* ext,
                                 bool sizes_only) {
    check_shape(d, n, R, "sgmres A");
    check_shape(d, n, rb, "sgmres b");
    check_shape(d, n, rho, "sgmres rho");
    check_shape(d, n, rx, "sgmres rx");
    TTSG_CHECK(d >= 2, TTSG_ERR_ARG, "sgmres: d must be >= 2");
    TTSG_CHECK(opts != nullptr, TTSG_ERR_ARG, "sgmres: null options");
    TTSG_CHECK(opts->maxit >= 1, TTSG_ERR_ARG, "sgmres: maxit < 1");
    TTSG_CHECK(opts->tol > 0.0 && opts->round_tol >= 0.0, TTSG_ERR_ARG, "sgmres: bad tolerance");
    TTSG_CHECK(opts->q >= 1 && opts->q <= 7, TTSG_ERR_ARG, "sgmres: q must be in 1..7");
    (void)prec_of(opts->precision);
    TTSG_CHECK(s >= 1, TTSG_ERR_ARG, "sgmres: s < 1");
    for (int b2 = 1; b2 < d; ++b2) TTSG_CHECK(rho[b2] >= rx[b2], TTSG_ERR_ARG, "sgmres: rho_b < rx_b");
    for (int b2 = 0; b2 <= d; ++b2)
        TTSG_CHECK(rb[b2] <= rx[b2], TTSG_ERR_CAPACITY, "sgmres: rank of b exceeds the STTA target ranks");
    if (!sizes_only) {
        check_ptrs(d, (const void* const*)A, "sgmres A");
        check_ptrs(d, (const void* const*)b, "sgmres b");
        check_ptrs(d, (const void* const*)Sf, "sgmres S");
        check_ptrs(d - 1, (const void* const*)Y, "sgmres Y");
        check_ptrs(d - 1, (const void* const*)X, "sgmres X");
    }
    ttsg::SolverInputs in;
    in.d = d;
    in.n = n;
    in.R = vec(R, d + 1);
    in.rb = vec(rb, d + 1);
    in.s = s;
    in.rho = vec(rho, d + 1);
    in.rx = vec(rx, d + 1);
    if (!sizes_only) {
        in.A.assign(A, A + d);
        in.b.assign(b, b + d);
        in.S.assign(Sf, Sf + d);
        in.Y.assign(Y, Y + d - 1);
        in.X.assign(X, X + d - 1);
    }
    in.o = *opts;
    if (in.o.rcond <= 0.0) in.o.rcond = 1e-12;
    if (in.o.stop_safety <= 0.0) in.o.stop_safety = 1.0;
    if (ext != nullptr) {
        TTSG_CHECK(ext->ls_mode == TTSG_LS_PINV || ext->ls_mode == TTSG_LS_WHITEN, TTSG_ERR_ARG,
                   "sgmres: unknown least-squares mode");
        in.ls_mode = ext->ls_mode;
        TTSG_CHECK(ext->variant == TTSG_VARIANT_ENHANCED || ext->variant == TTSG_VARIANT_VANILLA, TTSG_ERR_ARG,
                   "sgmres: variant must be TTSG_VARIANT_ENHANCED or TTSG_VARIANT_VANILLA");
        in.variant = ext->variant;
        TTSG_CHECK(ext->single_stream == 0 || ext->single_stream == 1, TTSG_ERR_ARG,
                   "sgmres: single_stream must be 0 or 1");
        in.single_stream = ext->single_stream != 0;
        if (ext->x0 != nullptr || ext->x0_r != nullptr) {
            TTSG_CHECK(ext->x0 != nullptr && ext->x0_r != nullptr, TTSG_ERR_ARG, "sgmres: x0 needs cores and ranks");
            check_shape(d, n, ext->x0_r, "sgmres x0");
            for (int b2 = 0; b2 <= d; ++b2)
                TTSG_CHECK(ext->x0_r[b2] <= rx[b2], TTSG_ERR_CAPACITY, "sgmres: rank of x0 exceeds the STTA target ranks");
            in.x0_r = vec(ext->x0_r, d + 1);
            if (!sizes_only) {
                check_ptrs(d, (const void* const*)ext->x0, "sgmres x0");
                in.x0.assign(ext->x0, ext->x0 + d);
            }
        }
        TTSG_CHECK(ext->zeta >= 0 && ext->zeta <= 4096, TTSG_ERR_ARG, "sgmres: zeta out of range");
        if (ext->zeta > 0) {
            TTSG_CHECK(ext->alpha != nullptr && ext->beta != nullptr, TTSG_ERR_ARG,
                       "sgmres: preconditioner needs alpha and beta");
            in.zeta = ext->zeta;
            in.alpha.assign(ext->alpha, ext->alpha + ext->zeta);
            in.beta.assign(ext->beta, ext->beta + ext->zeta);
            for (int j = 0; j < ext->zeta; ++j) {
                TTSG_CHECK(std::isfinite(in.alpha[j]) && std::isfinite(in.beta[j]) && in.beta[j] >= 0.0,
                           TTSG_ERR_ARG, "sgmres: preconditioner coefficients must be finite, beta >= 0");
                TTSG_CHECK(j == 0 || in.beta[j] >= in.beta[j - 1], TTSG_ERR_ARG,
                           "sgmres: preconditioner beta must be ascending");
            }
            if (!sizes_only) {
                check_ptrs(d, (const void* const*)ext->M, "sgmres preconditioner M");
                in.M.assign(ext->M, ext->M + d);
            }
        }
    }
    return in;
}

}  // namespace

extern "C" {

int ttsg_sgmres_solve_ex(int32_t d, const int32_t* n, const int32_t* R, const double* const* A, const int32_t* rb,
                         const double* const* b, int32_t s, const double* const* Sf, const int32_t* rho,
                         const double* const* Y, const int32_t* rx, const double* const* X,
                         const ttsg_sgmres_opts* opts, const ttsg_sgmres_ext* ext, double* const* x, int32_t* x_r,
                         ttsg_sgmres_info* info, void* ws, size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        ttsg::SolverInputs in = solver_inputs(d, n, R, A, rb, b, s, Sf, rho, Y, rx, X, opts, ext, false);
        check_ptrs(d, (const void* const*)x, "sgmres x");
        TTSG_CHECK(x_r != nullptr, TTSG_ERR_ARG, "sgmres: null x_r");
        return ttsg::sgmres_solve(in, x, x_r, info, ws, ws_bytes, S(stream));
    });
}

int ttsg_sgmres_solve(int32_t d, const int32_t* n, const int32_t* R, const double* const* A, const int32_t* rb,
                      const double* const* b, int32_t s, const double* const* Sf, const int32_t* rho,
                      const double* const* Y, const int32_t* rx, const double* const* X,
                      const ttsg_sgmres_opts* opts, double* const* x, int32_t* x_r, ttsg_sgmres_info* info, void* ws,
                      size_t ws_bytes, ttsg_stream_t stream) {
    return ttsg_sgmres_solve_ex(d, n, R, A, rb, b, s, Sf, rho, Y, rx, X, opts, nullptr, x, x_r, info, ws, ws_bytes,
                                stream);
}

int ttsg_sgmres_workspace_size(int32_t d, const int32_t* n, const int32_t* R, const int32_t* rb, int32_t s,
                               const int32_t* rho, const int32_t* rx, const ttsg_sgmres_opts* opts,
                               const ttsg_sgmres_ext* ext, size_t* bytes) {
    return guarded([&]() {
        TTSG_CHECK(bytes != nullptr, TTSG_ERR_ARG, "workspace_size: null output");
        ttsg::SolverInputs in = solver_inputs(d, n, R, nullptr, rb, nullptr, s, nullptr, rho, nullptr, rx, nullptr,
                                              opts, ext, true);
        *bytes = ttsg::sgmres_workspace(in);
        return 0;
    });
}

static ttsg::GmresInputs gmres_inputs(int32_t d, const int32_t* n, const int32_t* R, const double* const* A,
                                       const int32_t* rb, const double* const* b, const ttsg_gmres_opts* o) {
    check_shape(d, n, R, "tt_gmres A");
    check_shape(d, n, rb, "tt_gmres b");
    TTSG_CHECK(o != nullptr, TTSG_ERR_ARG, "tt_gmres: null options");
    TTSG_CHECK(o->maxit >= 1 && o->maxit <= 4096, TTSG_ERR_ARG, "tt_gmres: maxit must be in 1..4096");
    TTSG_CHECK(o->maxrank >= 0, TTSG_ERR_ARG, "tt_gmres: maxrank < 0");
    TTSG_CHECK(o->tol > 0.0 && o->tol < 1.0 && o->final_tol >= 0.0 && o->max_round > 0.0, TTSG_ERR_ARG,
               "tt_gmres: need 0 < tol < 1, final_tol >= 0, max_round > 0");
    ttsg::GmresInputs in;
    in.d = d;
    in.n = n;
    in.R = vec(R, d + 1);
    in.rb = vec(rb, d + 1);
    if (A) in.A.assign(A, A + d);
    if (b) in.b.assign(b, b + d);
    in.maxit = o->maxit;
    in.maxrank = o->maxrank;
    in.tol = o->tol;
    in.final_tol = o->final_tol > 0.0 ? o->final_tol : o->tol;
    in.max_round = o->max_round;
    return in;
}

int ttsg_tt_gmres(int32_t d, const int32_t* n, const int32_t* R, const double* const* A, const int32_t* rb,
                  const double* const* b, const ttsg_gmres_opts* opts, double* const* x, int32_t* x_r,
                  ttsg_sgmres_info* info, void* ws, size_t ws_bytes, ttsg_stream_t stream) {
    return guarded([&]() {
        ttsg::GmresInputs in = gmres_inputs(d, n, R, A, rb, b, opts);
        check_ptrs(d, (const void* const*)A, "tt_gmres A");
        check_ptrs(d, (const void* const*)b, "tt_gmres b");
        check_ptrs(d, (const void* const*)x, "tt_gmres x");
        TTSG_CHECK(x_r != nullptr, TTSG_ERR_ARG, "tt_gmres: null x_r");
        return ttsg::tt_gmres_solve(in, x, x_r, info, ws, ws_bytes, S(stream));
    });
}

int ttsg_tt_gmres_workspace_size(int32_t d, const int32_t* n, const int32_t* R, const int32_t* rb,
                                 const ttsg_gmres_opts* opts, size_t* bytes) {
    return guarded([&]() {
        TTSG_CHECK(bytes != nullptr, TTSG_ERR_ARG, "tt_gmres_workspace_size: null output");
        ttsg::GmresInputs in = gmres_inputs(d, n, R, nullptr, rb, nullptr, opts);
        *bytes = ttsg::tt_gmres_workspace(in);
        return 0;
    });
}

int ttsg_expsum(double zmin, double zmax, double tol, int32_t max_terms, double* alpha, double* beta) {
    return guarded([&]() {
        TTSG_CHECK(alpha != nullptr && beta != nullptr && max_terms >= 1, TTSG_ERR_ARG, "expsum: bad output arrays");
        const int z = ttsg::expsum_coefficients(zmin, zmax, tol, max_terms, alpha, beta);
        TTSG_CHECK(z != -1, TTSG_ERR_ARG, "expsum: need 0 < zmin <= zmax and 0 < tol < 1");
        TTSG_CHECK(z > 0, TTSG_ERR_CAPACITY, "expsum: more terms needed than max_terms");
        return z;
    });
}

int ttsg_precond_round(int32_t d, const int32_t* n, int32_t zeta, const double* alpha, const double* beta,
                       const double* const* M, const int32_t* r, const double* const* x, const int32_t* rho,
                       const double* const* Y, const int32_t* rx, const double* const* X, double tol, int32_t maxrank,
                       double rcond, double* const* out, int32_t* out_r, void* ws, size_t ws_bytes,
                       ttsg_stream_t stream) {
    return guarded([&]() {
        check_shape(d, n, r, "precond_round x");
        check_shape(d, n, rho, "precond_round rho");
        check_shape(d, n, rx, "precond_round rx");
        TTSG_CHECK(d >= 2, TTSG_ERR_ARG, "precond_round: d must be >= 2");
        TTSG_CHECK(zeta >= 1 && alpha != nullptr && beta != nullptr, TTSG_ERR_ARG, "precond_round: no terms");
        TTSG_CHECK(tol >= 0.0 && rcond >= 0.0, TTSG_ERR_ARG, "precond_round: negative tolerance");
        for (int b2 = 1; b2 < d; ++b2) TTSG_CHECK(rho[b2] >= rx[b2], TTSG_ERR_ARG, "precond_round: rho_b < rx_b");
        check_ptrs(d, (const void* const*)M, "precond_round M");
        check_ptrs(d, (const void* const*)x, "precond_round x");
        check_ptrs(d - 1, (const void* const*)Y, "precond_round Y");
        check_ptrs(d - 1, (const void* const*)X, "precond_round X");
        check_ptrs(d, (const void* const*)out, "precond_round out");
        TTSG_CHECK(out_r != nullptr, TTSG_ERR_ARG, "precond_round: null out_r");
        for (int j = 0; j < zeta; ++j)
            TTSG_CHECK(std::isfinite(alpha[j]) && std::isfinite(beta[j]) && beta[j] >= 0.0 &&
                           (j == 0 || beta[j] >= beta[j - 1]),
                       TTSG_ERR_ARG, "precond_round: beta must be finite, >= 0 and ascending");
        size_t sk = 0, core = 0, rmax = 1, ee = 0;
        for (int mu = 0; mu < d; ++mu) {
            sk += (size_t)rho[mu] * n[mu] * rx[mu + 1] + (size_t)rho[mu] * rx[mu] + 64;
            core = std::max(core, (size_t)std::max(rx[mu], r[mu]) * n[mu] * std::max(rx[mu + 1], r[mu + 1]));
            rmax = std::max(rmax, (size_t)std::max(rho[mu], rx[mu]));
            ee += (size_t)zeta * n[mu] * n[mu] * 3 + 64;
        }
        size_t zc = 0;
        for (int mu = 0; mu < d; ++mu) zc += (size_t)r[mu] * n[mu] * r[mu + 1] + 64;
        const size_t need = stta_ws(d, n, rho, rx, nullptr, r, ttsg::Prec::F64) + 2 * sk * 8 + ee * 8 + zc * 8 +
                            (8 * core + 12 * rmax * rmax) * 8 + (size_t)d * 16 * rmax * rmax * 8 + (4 << 20) +
                            ttsg::tt_svd_extra_bytes(d, n, rx) + (size_t)d * ttsg::jacobi_big_log_bytes((int)rmax);
        ttsg::Workspace W(ws, ws_bytes, need + kSplitSlack, S(stream));
        ttsg::Arena& ar = W.arena;
        std::vector<double*> Eb(d), z(d);
        for (int mu = 0; mu < d; ++mu) Eb[mu] = ar.get<double>((int64_t)zeta * n[mu] * n[mu]);
        for (int mu = 0; mu < d; ++mu) z[mu] = ar.get<double>((int64_t)r[mu] * n[mu] * r[mu + 1]);
        std::vector<double*> psi(d), om(d - 1), pt(d), ot(d - 1);
        for (int mu = 0; mu < d; ++mu) psi[mu] = ar.get<double>((int64_t)rho[mu] * n[mu] * rx[mu + 1]);
        for (int b2 = 1; b2 < d; ++b2) om[b2 - 1] = ar.get<double>((int64_t)rho[b2] * rx[b2]);
        for (int mu = 0; mu < d; ++mu) pt[mu] = ar.get<double>((int64_t)rho[mu] * n[mu] * rx[mu + 1]);
        for (int b2 = 1; b2 < d; ++b2) ot[b2 - 1] = ar.get<double>((int64_t)rho[b2] * rx[b2]);
        std::vector<const double*> Mv(M, M + d);
        ttsg::mode_exponentials(zeta, beta, d, n, Mv, Eb, ar, S(stream));
        ttsg::SketchOperands o;
        o.p = ttsg::Prec::F64;
        o.n = n;
        o.d = d;
        o.rho = vec(rho, d + 1);
        o.rx = vec(rx, d + 1);
        o.R.assign(d + 1, 1);
        for (int k = 0; k < d - 1; ++k) {
            o.Y.push_back(Y[k]);
            o.X.push_back(X[k]);
        }
        const std::vector<int> rv = vec(r, d + 1);
        std::vector<const double*> xv(x, x + d);
        std::vector<const void*> zv(z.begin(), z.end());
        for (int j = 0; j < zeta; ++j) {
            std::vector<const double*> Ej(d);
            for (int mu = 0; mu < d; ++mu) Ej[mu] = Eb[mu] + (int64_t)j * n[mu] * n[mu];
            ttsg::mode_product_tt(d, n, rv, xv, Ej, alpha[j], z, S(stream), &ar);
            ttsg::stta_sketch(o, rv, zv, (j == 0 ? psi : pt).data(), (j == 0 ? om : ot).data(), ar, S(stream));
            if (j > 0) {
                for (int mu = 0; mu < d; ++mu)
                    ttsg::axpby((int64_t)rho[mu] * n[mu] * rx[mu + 1], 1.0, pt[mu], 1.0, psi[mu], S(stream));
                for (int b2 = 1; b2 < d; ++b2)
                    ttsg::axpby((int64_t)rho[b2] * rx[b2], 1.0, ot[b2 - 1], 1.0, om[b2 - 1], S(stream));
            }
        }
        std::vector<const double*> cp(psi.begin(), psi.end()), co(om.begin(), om.end());
        std::vector<int> rr;
        std::vector<double*> o2(out, out + d);
        ttsg::stta_recover(d, n, vec(rho, d + 1), vec(rx, d + 1), cp, co, rcond, o2, rr, ar, S(stream));
        std::vector<int64_t> caps(d);
        ttsg::tt_svd_inplace(d, n, rr, o2, caps, tol, maxrank, ar, S(stream), nullptr);
        for (int k = 0; k <= d; ++k) out_r[k] = rr[k];
        TTSG_HIP(hipStreamSynchronize(S(stream)));
        return 0;
    });
}

int ttsg_autotune(int32_t on) { return ttsg::autotune_set(on); }

int ttsg_autotune_save(const char* path) {
    if (path == nullptr) return -TTSG_ERR_ARG;
    const int n = ttsg::autotune_save(path);
    if (n < 0) set_err("autotune_save: cannot write the file");
    return n < 0 ? -TTSG_ERR_ARG : n;
}

int ttsg_autotune_load(const char* path) {
    if (path == nullptr) return -TTSG_ERR_ARG;
    const int n = ttsg::autotune_load(path);
    if (n < 0) set_err("autotune_load: cannot read the file");
    return n < 0 ? -TTSG_ERR_ARG : n;
}

int ttsg_autotune_clear(void) { return ttsg::autotune_clear(); }

int ttsg_sgmres_solve_batched(int32_t count, ttsg_system* sys, int32_t concurrency, ttsg_stream_t stream) {
    return guarded([&]() {
        TTSG_CHECK(count >= 0, TTSG_ERR_ARG, "batched: count < 0");
        TTSG_CHECK(count == 0 || sys != nullptr, TTSG_ERR_ARG, "batched: null system array");
        if (count == 0) return 0;
        int dev = 0;
        TTSG_HIP(hipGetDevice(&dev));
        // Longest-first order: a system's cost grows with sum_k n_k * (R rx)^2 * rho.
        std::vector<double> cost(count, 0.0);
        for (int i = 0; i < count; ++i) {
            const ttsg_system& q = sys[i];
            check_shape(q.d, q.n, q.rx, "batched rx");
            check_shape(q.d, q.n, q.R, "batched A");
            check_shape(q.d, q.n, q.rho, "batched rho");
            for (int k = 0; k < q.d; ++k)
                cost[i] += (double)q.n[k] * q.R[k] * q.rx[k] * q.R[k + 1] * q.rx[k + 1] * (q.rho[k] + q.rho[k + 1]);
            sys[i].status = 0;
        }
        std::vector<int> order(count);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        const int workers = std::max(1, std::min<int>(concurrency > 0 ? concurrency : 8, count));
        // Every worker stream first waits for the work already queued on `stream`.
        hipEvent_t ready;
        TTSG_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        TTSG_HIP(hipEventRecord(ready, S(stream)));
        std::atomic<int> next{0};
        std::mutex mu;
        std::string first_err;
        int first_rc = 0;
        auto work = [&]() {
            hipStream_t st = nullptr;
            if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipStreamWaitEvent(st, ready, 0) != hipSuccess) {
                std::lock_guard<std::mutex> lk(mu);
                if (first_rc == 0) {
                    first_rc = -TTSG_ERR_HIP;
                    first_err = "batched: could not set up a worker stream";
                }
                if (st) (void)hipStreamDestroy(st);
                return;
            }
            for (int j = next++; j < count; j = next++) {
                ttsg_system& q = sys[order[j]];
                const int rc = ttsg_sgmres_solve_ex(q.d, q.n, q.R, q.A, q.rb, q.b, q.s, q.S, q.rho, q.Y, q.rx, q.X,
                                                    q.opts, q.ext, q.x, q.x_r, q.info, nullptr, 0, st);
                q.status = rc;
                if (rc < 0) {
                    std::lock_guard<std::mutex> lk(mu);
                    if (first_rc == 0) {
                        first_rc = rc;
                        first_err = "batched: system " + std::to_string(order[j]) + ": " + ttsg_last_error();
                    }
                }
            }
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        };
        std::vector<std::thread> pool;
        for (int w = 0; w < workers; ++w) pool.emplace_back(work);
        for (auto& t : pool) t.join();
        TTSG_HIP(hipEventDestroy(ready));
        if (first_rc < 0) throw Error(-first_rc, first_err);
        return 0;
    });
}

}  // extern "C"
