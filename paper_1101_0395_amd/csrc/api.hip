// C-ABI entry points of libcq: argument validation, workspace carving, kernel
// sequencing and the host side of the iteration loop.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "cq_internal.h"

namespace cq {

// kernels launched from the other translation units
cq_status launch_fill_zero(void* p, size_t bytes, hipStream_t s);
cq_status launch_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride,
                           uint32_t* keys, uint32_t* counts, int64_t capacity, void* ws,
                           const Layout& L, hipStream_t s);
cq_status launch_init(const uint32_t* keys, const uint32_t* counts, int64_t n, int K, int scheme,
                      uint64_t seed, double* centers, void* ws, const Layout& L, hipStream_t s);
cq_status launch_kmeans_begin(const double* centers, int K, void* ws, const Layout& L, hipStream_t s);
cq_status launch_kmeans_iters(const uint32_t* keys, const uint32_t* counts, int64_t n, int K,
                              double* centers, uint8_t* assign, int prune, int it0, int it1,
                              int max_iters, double tol, void* ws, const Layout& L, hipStream_t s);
cq_status launch_palette(const double* centers, int K, uint8_t* palette, hipStream_t s);
cq_status launch_identity_assign(uint8_t* assign, int64_t n, hipStream_t s);
cq_status launch_lut(const uint32_t* keys, const uint32_t* counts, int64_t n, const uint8_t* palette,
                     int K, void* ws, const Layout& L, hipStream_t s);
cq_status launch_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride,
                     const uint8_t* palette, int K, uint8_t* out_idx, uint8_t* out_rgb, void* ws,
                     const Layout& L, hipStream_t s);

static thread_local char g_error[512];

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

cq_status check_launch(const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s launch failed: %s", what, hipGetErrorString(e));
        return CQ_EDEVICE;
    }
    return CQ_OK;
}

static cq_status einval(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return CQ_EINVAL;
}

static cq_status check_image(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride)
{
    if (!img) return einval("img is null");
    if (H <= 0 || W <= 0) return einval("image size %d x %d must be positive", H, W);
    if (int64_t(H) * W > kMaxPixels) return einval("image has more than 2^28 pixels");
    if (row_stride < 3 * int64_t(W)) return einval("row stride %lld < 3 W", (long long)row_stride);
    return CQ_OK;
}

static cq_status check_ws(const void* ws, size_t ws_bytes, size_t need)
{
    if (!ws) {
        set_error("workspace is null");
        return CQ_EWORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) {
        set_error("workspace must be 256-byte aligned");
        return CQ_EWORKSPACE;
    }
    if (ws_bytes < need) {
        set_error("workspace has %zu bytes, %zu needed", ws_bytes, need);
        return CQ_EWORKSPACE;
    }
    return CQ_OK;
}

static cq_status check_k(int32_t K)
{
    if (K < 1 || K > kMaxK) return einval("K = %d outside [1, 256]", K);
    return CQ_OK;
}

#define CQ_TRY(expr)                     \
    do {                                 \
        cq_status st_ = (expr);          \
        if (st_ != CQ_OK) return st_;    \
    } while (0)

static cq_status sync_read(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    CQ_HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    CQ_HIP_TRY(hipStreamSynchronize(s));
    return CQ_OK;
}

// Host side of the iteration loop shared by cq_kmeans and cq_quantize.
// Iterations are enqueued in groups; the kernels of an iteration enqueued
// after the stop return immediately, so one readback per group suffices.
static cq_status run_kmeans(const uint32_t* keys, const uint32_t* counts, int64_t n, int K,
                            double* centers, int max_iters, double tol, int prune, uint8_t* assign,
                            uint8_t* palette, double* sse_trace, cq_stats* out, void* ws,
                            const Layout& L, hipStream_t s)
{
    cq_stats st;
    memset(&st, 0, sizeof st);
    st.prune = prune ? 1 : 0;
    st.n_unique = n;
    Meta* meta = at<Meta>(ws, L.meta);
    if (n <= K) {
        CQ_TRY(launch_init(keys, counts, n, K, CQ_INIT_USER, 0, centers, ws, L, s));
        CQ_TRY(launch_identity_assign(assign, n, s));
        st.k_used = int32_t(n);
        st.converged = 1;
    } else {
        st.k_used = K;
        CQ_TRY(launch_kmeans_begin(centers, K, ws, L, s));
        int it = 1;
        const int group = 8;
        while (it <= max_iters) {
            const int last = (it + group - 1 < max_iters) ? it + group - 1 : max_iters;
            CQ_TRY(launch_kmeans_iters(keys, counts, n, K, centers, assign, prune, it, last, max_iters,
                                       tol, ws, L, s));
            int32_t done = 0;
            CQ_TRY(sync_read(&done, &meta->done, sizeof done, s));
            if (done) break;
            it = last + 1;
        }
        Meta m;
        CQ_TRY(sync_read(&m, meta, sizeof m, s));
        if (m.bad_input) return einval("initial centres contain a non-finite value");
        st.iters = m.iters;
        st.converged = m.converged;
        st.ndc_total = int64_t(m.ndc);
        st.near_ties = int64_t(m.near_ties);
        st.sse_final = m.sse_last;
        st.mse_float = m.total_w ? m.sse_last / double(m.total_w) : 0.0;
        if (sse_trace && st.iters > 0) {
            CQ_TRY(sync_read(sse_trace, at<double>(ws, L.trace), sizeof(double) * size_t(st.iters), s));
        }
    }
    if (palette) CQ_TRY(launch_palette(centers, K, palette, s));
    if (out) *out = st;
    return CQ_OK;
}

}  // namespace cq

using namespace cq;

extern "C" {

size_t cq_workspace_bytes(int32_t H, int32_t W, int32_t K)
{
    if (H <= 0 || W <= 0 || K < 1 || K > kMaxK) return 0;
    const int64_t npix = int64_t(H) * W;
    if (npix > kMaxPixels) return 0;
    return make_layout(npix, true).total;
}

cq_status cq_workspace_prepare(void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    const Layout L = make_layout(0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.fixed_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the count table and the bitmap are adjacent: one fill covers both
    CQ_TRY(launch_fill_zero(at<char>(ws, L.tbl), L.lut - L.tbl, s));
    return CQ_OK;
}

cq_status cq_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                       uint32_t* keys, uint32_t* counts, int64_t capacity, int64_t* n_unique,
                       void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    if (!n_unique) return einval("n_unique is null");
    if (capacity < 0) return einval("capacity is negative");
    if (capacity > 0 && (!keys || !counts)) return einval("keys/counts are null");
    const Layout L = make_layout(0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.fixed_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    CQ_TRY(launch_histogram(img, H, W, row_stride_bytes, keys, counts, capacity, ws, L, s));
    int64_t n = 0;
    CQ_TRY(sync_read(&n, &at<Meta>(ws, L.meta)->n_unique, sizeof n, s));
    *n_unique = n;
    if (n > capacity) {
        set_error("%lld unique colours exceed capacity %lld", (long long)n, (long long)capacity);
        return CQ_ECAPACITY;
    }
    return CQ_OK;
}

cq_status cq_init(const uint32_t* keys, const uint32_t* counts, int64_t n_unique, int32_t K,
                  cq_init_t scheme, uint64_t seed, double* centers, int32_t* k_used, void* ws,
                  size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_k(K));
    if (!keys || !counts || !centers) return einval("keys/counts/centers is null");
    if (n_unique < 1 || n_unique > kMaxPixels) return einval("n_unique = %lld out of range", (long long)n_unique);
    if (int(scheme) < CQ_INIT_FORGY || int(scheme) > CQ_INIT_USER) return einval("unknown init scheme %d", int(scheme));
    const Layout L = make_layout(n_unique, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.total));
    hipStream_t s = static_cast<hipStream_t>(stream);
    CQ_TRY(launch_init(keys, counts, n_unique, K, int(scheme), seed, centers, ws, L, s));
    if (k_used) {
        CQ_HIP_TRY(hipStreamSynchronize(s));
        *k_used = int32_t(n_unique < K ? n_unique : K);
    }
    return CQ_OK;
}

cq_status cq_kmeans(const uint32_t* keys, const uint32_t* counts, int64_t n_unique, int32_t K,
                    double* centers, int32_t max_iters, double tol, int32_t prune, uint8_t* assign,
                    uint8_t* palette, double* sse_trace, cq_stats* stats, void* ws, size_t ws_bytes,
                    void* stream)
{
    clear_error();
    CQ_TRY(check_k(K));
    if (!keys || !counts || !centers || !assign) return einval("keys/counts/centers/assign is null");
    if (n_unique < 1 || n_unique > kMaxPixels) return einval("n_unique = %lld out of range", (long long)n_unique);
    if (max_iters < 1 || max_iters > kMaxIters) return einval("max_iters = %d outside [1, %d]", max_iters, kMaxIters);
    if (!(tol >= 0.0) || tol > 1e300) return einval("tol must be a finite value >= 0");
    const Layout L = make_layout(0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.fixed_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run_kmeans(keys, counts, n_unique, K, centers, max_iters, tol, prune ? 1 : 0, assign,
                      palette, sse_trace, stats, ws, L, s);
}

cq_status cq_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes,
                 const uint32_t* keys, const uint32_t* counts, int64_t n_unique,
                 const uint8_t* palette, int32_t K, uint8_t* out_idx, uint8_t* out_rgb,
                 uint64_t* sq_err_sum, void* ws, size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    CQ_TRY(check_k(K));
    if (!keys || !palette) return einval("keys/palette is null");
    if (n_unique < 1 || n_unique > int64_t(H) * W) return einval("n_unique = %lld out of range", (long long)n_unique);
    if (sq_err_sum && !counts) return einval("sq_err_sum needs counts");
    const Layout L = make_layout(0, false);
    CQ_TRY(check_ws(ws, ws_bytes, L.fixed_end));
    hipStream_t s = static_cast<hipStream_t>(stream);
    CQ_TRY(launch_lut(keys, sq_err_sum ? counts : nullptr, n_unique, palette, K, ws, L, s));
    CQ_TRY(launch_map(img, H, W, row_stride_bytes, palette, K, out_idx, out_rgb, ws, L, s));
    if (sq_err_sum) {
        uint64_t e = 0;
        CQ_TRY(sync_read(&e, &at<Meta>(ws, L.meta)->sq_err, sizeof e, s));
        *sq_err_sum = e;
    }
    return CQ_OK;
}

cq_status cq_quantize(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride_bytes, int32_t K,
                      cq_init_t scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                      uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, cq_stats* stats, void* ws,
                      size_t ws_bytes, void* stream)
{
    clear_error();
    CQ_TRY(check_image(img, H, W, row_stride_bytes));
    CQ_TRY(check_k(K));
    if (!palette) return einval("palette is null");
    if (int(scheme) < CQ_INIT_FORGY || int(scheme) > CQ_INIT_KMEANSPP)
        return einval("cq_quantize needs scheme FORGY, MAXMIN or KMEANSPP");
    if (max_iters < 1 || max_iters > kMaxIters) return einval("max_iters = %d outside [1, %d]", max_iters, kMaxIters);
    if (!(tol >= 0.0) || tol > 1e300) return einval("tol must be a finite value >= 0");
    const int64_t npix = int64_t(H) * W;
    const Layout L = make_layout(npix, true);
    CQ_TRY(check_ws(ws, ws_bytes, L.total));
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t* keys = at<uint32_t>(ws, L.keys);
    uint32_t* counts = at<uint32_t>(ws, L.counts);
    uint8_t* assign = at<uint8_t>(ws, L.assign);
    double* centers = at<double>(ws, L.centers);
    Meta* meta = at<Meta>(ws, L.meta);

    CQ_TRY(launch_histogram(img, H, W, row_stride_bytes, keys, counts, npix, ws, L, s));
    int64_t n = 0;
    CQ_TRY(sync_read(&n, &meta->n_unique, sizeof n, s));
    CQ_TRY(launch_init(keys, counts, n, K, int(scheme), seed, centers, ws, L, s));
    cq_stats st;
    CQ_TRY(run_kmeans(keys, counts, n, K, centers, max_iters, tol, prune ? 1 : 0, assign, palette,
                      nullptr, &st, ws, L, s));
    CQ_TRY(launch_lut(keys, counts, n, palette, st.k_used, ws, L, s));
    CQ_TRY(launch_map(img, H, W, row_stride_bytes, palette, st.k_used, out_idx, out_rgb, ws, L, s));
    uint64_t err = 0;
    CQ_TRY(sync_read(&err, &meta->sq_err, sizeof err, s));
    st.mse_img = double(err) / double(npix);
    if (stats) *stats = st;
    return CQ_OK;
}

const char* cq_last_error(void) { return g_error; }

}  // extern "C"
