// Dense and BLAS-1 pieces of ChFSI on gfx950: deterministic reductions, the
// Lanczos upper bound, Gram products, Cholesky-QR and Rayleigh-Ritz.
//
// Paper: ChFSI orthonormalises the filtered block and projects H onto it
// (the CheFSI paragraph; details of the PARSEC implementation are deferred to
// its ChFSI reference).  The Gram products X^T X and X^T (H X) and the
// N x M x M block updates X R^{-1} and X Q are plain GEMMs (rocBLAS on MFMA;
// the Gram in row slices whose partials are summed in FP64); the M x M
// Cholesky factorisation and symmetric eigensolve run in FP64 through
// rocSOLVER.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"
#include "kernels.hpp"

namespace chf {

// ---------------------------------------------------------------------------
// deterministic reductions: fixed grid, per-block tree, then one block sums
// the partials in order.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;

__device__ inline double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// out[blockIdx.x] = sum over this block's stride of x[i * incx] * y[i * incy]
template <class T>
__global__ void __launch_bounds__(256) dot_partial_kernel(int64_t n, const T* __restrict__ x, int64_t incx,
                                                          const T* __restrict__ y, int64_t incy, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        acc += double(x[i * incx]) * double(y[i * incy]);
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) sum_partials_kernel(int n, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = s;
}

template <class T>
void dot_device(chf_ctx* ctx, int64_t n, const T* x, int64_t incx, const T* y, int64_t incy, double* out_dev,
                hipStream_t s) {
    ctx->red.ensure(kRedBlocks * sizeof(double));
    const int nb = int(std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n + 255) / 256)));
    dot_partial_kernel<T><<<nb, 256, 0, s>>>(n, x, incx, y, incy, ctx->red.as<double>());
    LAUNCH_CHECK();
    sum_partials_kernel<<<1, 256, 0, s>>>(nb, ctx->red.as<double>(), out_dev);
    LAUNCH_CHECK();
}

template <class T>
double dot_host(chf_ctx* ctx, int64_t n, const T* x, int64_t incx, const T* y, int64_t incy, hipStream_t s) {
    double* d = reinterpret_cast<double*>(ctx->info.p);
    dot_device<T>(ctx, n, x, incx, y, incy, d, s);
    double h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return h;
}

// z[i] = a x[i] + b y[i] (strided)
__global__ void lincomb_kernel(int64_t n, double a, const double* __restrict__ x, int64_t incx, double b,
                               const double* __restrict__ y, int64_t incy, double* __restrict__ z, int64_t incz) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double yv = y ? y[i * incy] : 0.0;
    z[i * incz] = a * x[i * incx] + b * yv;
}

void lincomb(int64_t n, double a, const double* x, int64_t incx, double b, const double* y, int64_t incy, double* z,
             int64_t incz, hipStream_t s) {
    lincomb_kernel<<<unsigned((n + 255) / 256), 256, 0, s>>>(n, a, x, incx, b, y, incy, z, incz);
    LAUNCH_CHECK();
}

// Extreme eigenvalues of a symmetric tridiagonal matrix by Sturm-sequence
// bisection (count of eigenvalues below x = number of negative pivots of
// T - x I).
static int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (size_t i = 1; i < d.size(); ++i) {
        const double qq = (q == 0.0) ? 1e-300 : q;
        q = d[i] - x - e[i - 1] * e[i - 1] / qq;
        if (q < 0) ++cnt;
    }
    return cnt;
}

static double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int which /*0 min, 1 max*/) {
    double lo = d[0], hi = d[0];
    for (size_t i = 0; i < d.size(); ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < d.size() ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
    }
    const int target = which == 0 ? 1 : int(d.size());   // smallest x with count >= target
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (sturm_count(d, e, mid) >= target) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}


// ---------------------------------------------------------------------------
// Gram products S = A^T B
// ---------------------------------------------------------------------------
// S[i][j] (+)= sum over row slices of part[s][i][j], in FP64 and in slice
// order (accumulate: add to S, for the slice groups after the first); with a
// symmetric product only i <= j is summed and mirrored, so S is exactly
// symmetric.
template <class P>
__global__ void gram_slices_reduce_kernel(int m, int n, int n_slices, const P* __restrict__ part,
                                          double* __restrict__ S, int64_t lds, int symmetric, int accumulate) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(m) * n) return;
    const int i = int(idx / n), j = int(idx % n);
    if (symmetric && i > j) return;
    const int64_t stride = int64_t(m) * n;
    double acc = accumulate ? S[int64_t(i) * lds + j] : 0.0;
    for (int k = 0; k < n_slices; ++k) acc += double(part[k * stride + idx]);
    S[int64_t(i) * lds + j] = acc;
    if (symmetric && i < j) S[int64_t(j) * lds + i] = acc;
}

static rocblas_status gemm_sb(rocblas_handle h, rocblas_int M, rocblas_int N, rocblas_int K, const float* A,
                              rocblas_int lda, rocblas_stride sa, const float* B, rocblas_int ldb, rocblas_stride sb,
                              float* C, rocblas_int ldc, rocblas_stride sc, rocblas_int batch) {
    const float one = 1.f, zero = 0.f;
    return rocblas_sgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, M, N, K, &one, A, lda,
                                         sa, B, ldb, sb, &zero, C, ldc, sc, batch);
}
static rocblas_status gemm_sb(rocblas_handle h, rocblas_int M, rocblas_int N, rocblas_int K, const double* A,
                              rocblas_int lda, rocblas_stride sa, const double* B, rocblas_int ldb, rocblas_stride sb,
                              double* C, rocblas_int ldc, rocblas_stride sc, rocblas_int batch) {
    const double one = 1.0, zero = 0.0;
    return rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, M, N, K, &one, A, lda,
                                         sa, B, ldb, sb, &zero, C, ldc, sc, batch);
}

// Gram S = A^T B over n_rows rows.  X^T X is a plain GEMM, so the products of
// row slices run as strided-batched rocBLAS GEMMs (MFMA, accumulating in the
// block precision within a slice) into partials that are summed in FP64.
// Slices hold at most kGramSliceRows rows whatever the width, so an FP32
// sum never runs over more rows than that (the slice count grows with the
// grid instead); every GEMM operand spans fewer than kBlasMaxElems elements
// (the BLAS calls take 32-bit sizes and offsets); the slices run in groups
// of at most kGramMaxSlices whose partials fit kGramPartBytes, each group's
// sum added to S in slice order.
constexpr int64_t kGramSliceRows = 8192;
constexpr int64_t kGramMaxSlices = 256;
constexpr size_t kGramPartBytes = size_t(1) << 30;
constexpr int64_t kBlasMaxElems = (int64_t(1) << 31) - (int64_t(1) << 20);

struct GramSlices {
    int64_t rows;      // rows per slice
    int64_t full;      // slices of exactly `rows` rows
    int64_t tail;      // rows of the last, shorter slice (0: none)
    int64_t group;     // slices per batched GEMM (their partials at once)
    size_t part_bytes; // partials scratch
};

static GramSlices gram_slices(int64_t n_rows, int m, int n, size_t elem_bytes, int64_t ld) {
    const size_t per = size_t(m) * size_t(n) * elem_bytes;
    const int64_t ns = std::max<int64_t>(1, (n_rows + kGramSliceRows - 1) / kGramSliceRows);
    const int64_t max_group =
        std::max<int64_t>(1, std::min<int64_t>(kGramMaxSlices, int64_t(kGramPartBytes / std::max<size_t>(1, per))));
    GramSlices g;
    g.rows = std::max<int64_t>(1, (n_rows + ns - 1) / ns);     // <= kGramSliceRows, balanced
    g.rows = std::min<int64_t>(g.rows, std::max<int64_t>(1, kBlasMaxElems / std::max<int64_t>(1, ld)));
    g.full = n_rows / g.rows;
    g.tail = n_rows - g.full * g.rows;
    const int64_t total = g.full + (g.tail > 0 ? 1 : 0);
    g.group = std::max<int64_t>(1, std::min<int64_t>(total, max_group));
    g.part_bytes = size_t(std::max<int64_t>(1, g.group)) * per;
    return g;
}

template <class T>
void gram_product(chf_ctx* ctx, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n_rows, int m, int n,
                  double* S, int64_t lds, hipStream_t s) {
    const bool symmetric = (A == B) && (m == n) && (lda == ldb);
    const size_t per = size_t(m) * size_t(n) * sizeof(T);
    const GramSlices g = gram_slices(n_rows, m, n, sizeof(T), std::max(lda, ldb));
    const int64_t R = g.rows;
    const int64_t n_slices = g.full + (g.tail > 0 ? 1 : 0);
    CHF_REQUIRE(R <= INT32_MAX && lda <= INT32_MAX && ldb <= INT32_MAX, "gram: dimensions beyond 32-bit BLAS");
    ctx->scratch2.ensure(g.part_bytes);
    T* part = ctx->scratch2.as<T>();
    ROCBLAS_CHECK(rocblas_set_stream(ctx->blas, s));
    const int64_t tot = int64_t(m) * n;
    if (n_slices == 0) {
        HIP_CHECK(hipMemsetAsync(part, 0, per, s));
        gram_slices_reduce_kernel<T><<<unsigned((tot + 255) / 256), 256, 0, s>>>(m, n, 1, part, S, lds,
                                                                                symmetric ? 1 : 0, 0);
        LAUNCH_CHECK();
        return;
    }
    for (int64_t s0 = 0; s0 < n_slices; s0 += g.group) {
        const int64_t cnt = std::min<int64_t>(g.group, n_slices - s0);
        // full slices of this group, then (in the last group) the tail
        const int64_t nfull = std::max<int64_t>(0, std::min<int64_t>(cnt, g.full - s0));
        const T* A0 = A + s0 * R * lda;
        const T* B0 = B + s0 * R * ldb;
        // column-major view: part_k (n x m, ld n) = B_k (n x R, ld ldb) * A_k^T
        if (nfull > 0)
            ROCBLAS_CHECK(gemm_sb(ctx->blas, n, m, rocblas_int(R), B0, rocblas_int(ldb), R * ldb, A0,
                                  rocblas_int(lda), R * lda, part, n, int64_t(m) * n, rocblas_int(nfull)));
        if (nfull < cnt)
            ROCBLAS_CHECK(gemm_sb(ctx->blas, n, m, rocblas_int(g.tail), B0 + nfull * R * ldb, rocblas_int(ldb), 0,
                                  A0 + nfull * R * lda, rocblas_int(lda), 0, part + nfull * int64_t(m) * n, n, 0, 1));
        gram_slices_reduce_kernel<T><<<unsigned((tot + 255) / 256), 256, 0, s>>>(
            m, n, int(cnt), part, S, lds, symmetric ? 1 : 0, s0 > 0 ? 1 : 0);
        LAUNCH_CHECK();
    }
}

template void gram_product<float>(chf_ctx*, const float*, int64_t, const float*, int64_t, int64_t, int, int, double*,
                                  int64_t, hipStream_t);
template void gram_product<double>(chf_ctx*, const double*, int64_t, const double*, int64_t, int64_t, int, int,
                                   double*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// small element-wise helpers for the dense steps
// ---------------------------------------------------------------------------
template <class T>
__global__ void cast_matrix_kernel(int64_t n, const double* __restrict__ src, T* __restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = T(src[i]);
}

// column-major upper triangle kept, strictly lower part zeroed (M x M, ld M)
__global__ void keep_upper_kernel(int m, double* __restrict__ R) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(m) * m) return;
    const int col = int(idx / m), row = int(idx % m);
    if (row > col) R[idx] = 0.0;
}

__global__ void symmetrize_kernel(int m, double* __restrict__ S) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(m) * m) return;
    const int i = int(idx / m), j = int(idx % m);
    if (i < j) {
        const double v = 0.5 * (S[int64_t(i) * m + j] + S[int64_t(j) * m + i]);
        S[int64_t(i) * m + j] = v;
        S[int64_t(j) * m + i] = v;
    }
}

__global__ void add_diag_kernel(int m, double* __restrict__ S, double shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) S[int64_t(i) * m + i] += shift;
}

__global__ void trace_kernel(int m, const double* __restrict__ S, double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0;
    for (int i = threadIdx.x; i < m; i += 256) acc += S[int64_t(i) * m + i];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = r;
}

static void check_ctx_block(chf_ctx* ctx, int dtype, const void* X, int64_t ld, int nvec, const char* what) {
    if (!ctx) fail(CHF_EINVAL, "%s: null context", what);
    if (dtype != CHF_F32 && dtype != CHF_F64) fail(CHF_EINVAL, "%s: bad dtype", what);
    if (!X) fail(CHF_EINVAL, "%s: null block", what);
    if (nvec < 1 || ld < nvec) fail(CHF_EINVAL, "%s: need 1 <= nvec <= ld", what);
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev != ctx->device) fail(CHF_EINVAL, "%s: context belongs to device %d, current is %d", what, ctx->device, dev);
}

template <class F>
static int guard(F&& f) {
    try {
        f();
        return CHF_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return CHF_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return CHF_EHIP;
    }
}

// S (row-major M x M, FP64) lives at the start of ctx->scratch; the rest holds
// the cast factor for FP32 updates and rocSOLVER's info word.
static size_t mm_scratch_bytes(int m, size_t extra_bytes) {
    return size_t(m) * m * (sizeof(double) + sizeof(float)) + extra_bytes + 256;
}
static double* mm_scratch(chf_ctx* ctx, int m, size_t extra_bytes) {
    ctx->scratch.ensure(mm_scratch_bytes(m, extra_bytes));
    return ctx->scratch.as<double>();
}
// extra bytes after the M x M matrices: Cholesky-QR keeps the Gram diagonal,
// Rayleigh-Ritz the eigenvalues and the eigensolver's off-diagonal
static size_t cholqr_extra(int m) { return size_t(m) * sizeof(double); }
static size_t rr_extra(int m) { return size_t(m) * sizeof(double) * 2; }

__global__ void diag_copy_kernel(int m, const double* __restrict__ S, double* __restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) d[i] = S[int64_t(i) * m + i];
}

// out[0] = min_i R_ii^2 / d_i (the squared sine between column i and the span
// of the columns before it), out[1] = its index; one workgroup of 256
__global__ void __launch_bounds__(256) pivot_ratio_kernel(int m, const double* __restrict__ R,
                                                          const double* __restrict__ d, double* __restrict__ out) {
    __shared__ double v[256];
    __shared__ int at[256];
    double best = 2.0;
    int bi = 0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double r = R[int64_t(i) * m + i];
        const double q = d[i] > 0 ? r * r / d[i] : 1.0;
        if (q < best) best = q, bi = i;
    }
    v[threadIdx.x] = best;
    at[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w && (v[threadIdx.x + w] < v[threadIdx.x] ||
                                (v[threadIdx.x + w] == v[threadIdx.x] && at[threadIdx.x + w] < at[threadIdx.x]))) {
            v[threadIdx.x] = v[threadIdx.x + w];
            at[threadIdx.x] = at[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = double(at[0]);
    }
}

// A Cholesky pivot R_ii^2 below this fraction of column i's squared norm
// marks column i as numerically dependent on the ones before it (the
// factorisation "succeeds" on rounding noise): treated as a breakdown.  The
// fraction matches the precision of the Gram: an FP64 Gram resolves
// R_ii^2 / S_ii down to ~1e-16, an FP32 Gram (FP32 products within row
// slices) only to ~1e-6, and a first pass at that limit would leave the
// factor too inaccurate for the second pass to repair.
constexpr double kPivotRelF64 = 1e-13;
constexpr double kPivotRelF32 = 1e-5;

__global__ void cast_panel_kernel(int64_t rows, int m, const float* __restrict__ X, int64_t ldx,
                                  double* __restrict__ D) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= rows * m) return;
    const int64_t r = idx / m;
    const int c = int(idx - r * m);
    D[idx] = double(X[r * ldx + c]);
}

// S[i][j] = S[j][i] for i > j (row-major): mirror the upper triangle
__global__ void mirror_upper_kernel(int m, double* __restrict__ S) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(m) * m) return;
    const int i = int(idx / m), j = int(idx % m);
    if (i > j) S[idx] = S[int64_t(j) * m + i];
}

// S = X^T X of an FP32 block with FP64 products and sums: row panels of X are
// widened to FP64 (at most kGramPartBytes of scratch) and accumulated into S
// by FP64 GEMMs in panel order, then the upper triangle is mirrored.
static void gram_f32_in_f64(chf_ctx* ctx, const float* X, int64_t ldx, int64_t n_rows, int m, double* S,
                            hipStream_t s) {
    const int64_t P = std::max<int64_t>(1, std::min<int64_t>(n_rows, int64_t(kGramPartBytes / (size_t(m) * 8))));
    CHF_REQUIRE(P <= INT32_MAX, "gram: panel beyond 32-bit BLAS");
    ctx->scratch2.ensure(size_t(P) * size_t(m) * 8);
    double* D = ctx->scratch2.as<double>();
    ROCBLAS_CHECK(rocblas_set_stream(ctx->blas, s));
    const double one = 1.0, zero = 0.0;
    for (int64_t r0 = 0; r0 < n_rows; r0 += P) {
        const int64_t rows = std::min(P, n_rows - r0);
        cast_panel_kernel<<<unsigned((rows * m + 255) / 256), 256, 0, s>>>(rows, m, X + r0 * ldx, ldx, D);
        LAUNCH_CHECK();
        // column-major D is m x rows (ld m); S (col-major = row-major) += D D^T
        ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_transpose, m, m,
                                    rocblas_int(rows), &one, D, m, D, m, r0 == 0 ? &zero : &one, S, m));
    }
    mirror_upper_kernel<<<unsigned((int64_t(m) * m + 255) / 256), 256, 0, s>>>(m, S);
    LAUNCH_CHECK();
}

// One Cholesky-QR pass: S = X^T X (in the block precision, or in FP64 for an
// FP32 block when gram64), S = R^T R in FP64, X <- X R^{-1} in the block
// precision.  Returns 0, or the rocSOLVER info (> 0: leading minor not
// positive definite), or the 1-based index of a pivot below the threshold of
// the Gram's precision; X is unchanged unless 0 is returned.
template <class T>
static int cholqr_once(chf_ctx* ctx, T* X, int64_t ldx, int64_t n_rows, int m, double shift_rel, bool gram64,
                       hipStream_t s) {
    constexpr bool f64 = std::is_same<T, double>::value;
    double* S = mm_scratch(ctx, m, cholqr_extra(m));
    double* diag = reinterpret_cast<double*>(reinterpret_cast<char*>(S) + size_t(m) * m * (sizeof(double) + sizeof(float)) + 256);
    if (!f64 && gram64)
        gram_f32_in_f64(ctx, reinterpret_cast<const float*>(X), ldx, n_rows, m, S, s);
    else
        gram_product<T>(ctx, X, ldx, X, ldx, n_rows, m, m, S, m, s);
    if (shift_rel > 0) {
        double* tr = reinterpret_cast<double*>(ctx->info.p);
        trace_kernel<<<1, 256, 0, s>>>(m, S, tr);
        double htr = 0;
        HIP_CHECK(hipMemcpyAsync(&htr, tr, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        add_diag_kernel<<<(m + 255) / 256, 256, 0, s>>>(m, S, shift_rel * htr / m);
        LAUNCH_CHECK();
    }
    ROCBLAS_CHECK(rocblas_set_stream(ctx->blas, s));
    // row-major S equals its column-major view (symmetric); potrf(upper) gives
    // column-major U with S = U^T U, i.e. R = U.
    int* dinfo = reinterpret_cast<int*>(reinterpret_cast<char*>(S) + size_t(m) * m * sizeof(double) +
                                        size_t(m) * m * sizeof(float));
    diag_copy_kernel<<<(m + 255) / 256, 256, 0, s>>>(m, S, diag);
    LAUNCH_CHECK();
    ROCBLAS_CHECK(rocsolver_dpotrf(ctx->blas, rocblas_fill_upper, m, S, m, dinfo));
    double piv[2] = {1.0, 0.0};
    double* pr = reinterpret_cast<double*>(ctx->info.p) + 2;
    pivot_ratio_kernel<<<1, 256, 0, s>>>(m, S, diag, pr);
    LAUNCH_CHECK();
    HIP_CHECK(hipMemcpyAsync(piv, pr, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    int info = 0;
    HIP_CHECK(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (info != 0) return info;
    const double thr = (f64 || gram64) ? kPivotRelF64 : kPivotRelF32;
    if (shift_rel == 0 && !(piv[0] >= thr)) return int(piv[1]) + 1;
    keep_upper_kernel<<<unsigned((int64_t(m) * m + 255) / 256), 256, 0, s>>>(m, S);
    LAUNCH_CHECK();
    // X is row-major [n_rows][ldx] = column-major Xc [m][n_rows] (ld ldx).
    // X R^{-1}  <=>  Xc <- R^{-T} Xc : left-side solve with U^T.
    // (in row panels: each call's block spans fewer than kBlasMaxElems elements)
    const int64_t pt = std::max<int64_t>(1, std::min<int64_t>(n_rows, kBlasMaxElems / std::max<int64_t>(1, ldx)));
    float* R32 = reinterpret_cast<float*>(reinterpret_cast<char*>(S) + size_t(m) * m * sizeof(double));
    if (!f64) {
        cast_matrix_kernel<float><<<unsigned((int64_t(m) * m + 255) / 256), 256, 0, s>>>(int64_t(m) * m, S, R32);
        LAUNCH_CHECK();
    }
    for (int64_t r0 = 0; r0 < n_rows; r0 += pt) {
        const int64_t rows = std::min(pt, n_rows - r0);
        if (f64) {
            const double one = 1.0;
            ROCBLAS_CHECK(rocblas_dtrsm(ctx->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                                        rocblas_diagonal_non_unit, m, rocblas_int(rows), &one, S, m,
                                        reinterpret_cast<double*>(X + r0 * ldx), rocblas_int(ldx)));
        } else {
            const float one = 1.0f;
            ROCBLAS_CHECK(rocblas_strsm(ctx->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                                        rocblas_diagonal_non_unit, m, rocblas_int(rows), &one, R32, m,
                                        reinterpret_cast<float*>(X + r0 * ldx), rocblas_int(ldx)));
        }
    }
    return 0;
}

// Cholesky-QR (CheFSI paragraph: orthonormalisation of the filtered block).
// FP64 blocks: one pass.  FP32 blocks: two passes (CholQR2).  A filtered
// block has a condition number of the order of |T_m(t0)|, so one pass with
// FP32 arithmetic leaves an orthogonality error of about kappa^2 u_32; the
// second pass on the nearly orthonormal result brings it down to the
// rounding level.  The product of the two triangular factors is again upper
// triangular with a positive diagonal, so the result is the same Q as that
// of one exact pass.  Breakdown of the first pass: an FP32 block first
// retries with an FP64 Gram (gram_dtype CHF_F64 starts there), then any
// block takes a shifted pass; each retry is counted in *fallbacks.
template <class T>
void orthonormalize_t(chf_ctx* ctx, T* X, int64_t ldx, int64_t n_rows, int m, bool gram64, int* fallbacks,
                      hipStream_t s) {
    constexpr bool f64 = std::is_same<T, double>::value;
    int fb = 0;
    int info = cholqr_once<T>(ctx, X, ldx, n_rows, m, 0.0, gram64, s);
    if (info != 0 && !f64 && !gram64) {
        ++fb;
        gram64 = true;
        info = cholqr_once<T>(ctx, X, ldx, n_rows, m, 0.0, true, s);
    }
    bool shifted = false;
    if (info != 0) {
        // shifted Cholesky-QR: the shift makes the factorisation exist; the
        // plain pass after it restores orthonormality
        ++fb;
        shifted = true;
        const double shift = f64 ? 1e-14 : 1e-6;
        info = cholqr_once<T>(ctx, X, ldx, n_rows, m, shift, gram64, s);
        if (info == 0) info = cholqr_once<T>(ctx, X, ldx, n_rows, m, 0.0, gram64, s);
    }
    if (info == 0 && !f64 && !shifted) info = cholqr_once<T>(ctx, X, ldx, n_rows, m, 0.0, gram64, s);
    if (fallbacks) *fallbacks = fb;
    if (info != 0) fail(CHF_ENOTPD, "orthonormalize: Gram matrix not positive definite (minor %d)", info);
}

template <class T>
void rayleigh_ritz_t(chf_ham* H, chf_ctx* ctx, T* X, int64_t ldx, int m, double* eig_host, T* W, int64_t ldw,
                            hipStream_t s) {
    const int64_t n_rows = H->grid.n_rows;
    double* Hs = mm_scratch(ctx, m, rr_extra(m));
    double* evals = reinterpret_cast<double*>(reinterpret_cast<char*>(Hs) + size_t(m) * m * (sizeof(double) + sizeof(float)) + 256);
    double* E = evals + m;
    int* dinfo = reinterpret_cast<int*>(reinterpret_cast<char*>(Hs) + size_t(m) * m * (sizeof(double) + sizeof(float)));
    // Hs[:, c:c+nb] = X^T (H X[:, c:c+nb]), blockwise through W
    const int nb = int(std::min<int64_t>(m, ldw));
    for (int c = 0; c < m; c += nb) {
        const int w = std::min(nb, m - c);
        hx_step<T>(H, X + c, ldx, W, ldw, nullptr, 0, w, 1.0, 0.0, 0.0, s, 0);
        gram_product<T>(ctx, X, ldx, W, ldw, n_rows, m, w, Hs + c, m, s);
    }
    symmetrize_kernel<<<unsigned((int64_t(m) * m + 255) / 256), 256, 0, s>>>(m, Hs);
    LAUNCH_CHECK();
    ROCBLAS_CHECK(rocblas_set_stream(ctx->blas, s));
    ROCBLAS_CHECK(rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, m, Hs, m, evals, E, dinfo));
    int info = 0;
    HIP_CHECK(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(eig_host, evals, size_t(m) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (info != 0) fail(CHF_ENOTCONV, "rayleigh_ritz: eigensolver did not converge (info %d)", info);
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(eig_host[i])) fail(CHF_ENONFINITE, "rayleigh_ritz: non-finite Ritz value");
    // Hs now holds Q column-major (column j = eigenvector j).  X <- X Q in row
    // panels, in place: a panel of P rows of X (row-major, = column-major
    // Xc [m][P]) gives Qᵀ Xc, computed into the work block used as flat
    // storage of P x m values (P = n_rows ldw / m), then copied back.
    const int64_t P = std::max<int64_t>(
        1, std::min<int64_t>(std::min<int64_t>(n_rows, n_rows * ldw / m), kBlasMaxElems / std::max<int64_t>(ldx, m)));
    CHF_REQUIRE(P <= INT32_MAX, "rayleigh_ritz: panel beyond 32-bit BLAS");
    float* Q32 = reinterpret_cast<float*>(reinterpret_cast<char*>(Hs) + size_t(m) * m * sizeof(double));
    if (!std::is_same<T, double>::value) {
        cast_matrix_kernel<float><<<unsigned((int64_t(m) * m + 255) / 256), 256, 0, s>>>(int64_t(m) * m, Hs, Q32);
        LAUNCH_CHECK();
    }
    for (int64_t r0 = 0; r0 < n_rows; r0 += P) {
        const int64_t rows = std::min(P, n_rows - r0);
        if (std::is_same<T, double>::value) {
            const double one = 1.0, zero = 0.0;
            ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, m,
                                        rocblas_int(rows), m, &one, Hs, m,
                                        reinterpret_cast<const double*>(X + r0 * ldx), rocblas_int(ldx), &zero,
                                        reinterpret_cast<double*>(W), m));
        } else {
            const float one = 1.0f, zero = 0.0f;
            ROCBLAS_CHECK(rocblas_sgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, m,
                                        rocblas_int(rows), m, &one, Q32, m,
                                        reinterpret_cast<const float*>(X + r0 * ldx), rocblas_int(ldx), &zero,
                                        reinterpret_cast<float*>(W), m));
        }
        HIP_CHECK(hipMemcpy2DAsync(X + r0 * ldx, size_t(ldx) * sizeof(T), W, size_t(m) * sizeof(T),
                                   size_t(m) * sizeof(T), size_t(rows), hipMemcpyDeviceToDevice, s));
    }
}

// three vectors of n_rows as 2-column blocks
static size_t lanczos_vec_bytes(int64_t n_rows) { return size_t(n_rows) * 2 * 3 * sizeof(double); }

void lanczos_run(chf_ham* H, chf_ctx* ctx, const double* v0, int k, double* out3, hipStream_t s) {
    const int64_t n = H->grid.n_rows;
    // three vectors stored as 2-column blocks (second column zero) so the
    // tiled kernel's 16-byte rows apply
    ctx->vec.ensure(lanczos_vec_bytes(n));
    double* base = ctx->vec.as<double>();
    HIP_CHECK(hipMemsetAsync(base, 0, size_t(n) * 2 * 3 * sizeof(double), s));
    double* v = base;
    double* vp = base + 2 * n;
    double* f = base + 4 * n;
    const double nrm = std::sqrt(dot_host<double>(ctx, n, v0, 1, v0, 1, s));
    if (!(nrm > 0) || !std::isfinite(nrm)) fail(CHF_EINVAL, "lanczos_bound: zero or non-finite start vector");
    lincomb(n, 1.0 / nrm, v0, 1, 0.0, nullptr, 0, v, 2, s);
    std::vector<double> d, e;
    hx_step<double>(H, v, 2, f, 2, nullptr, 0, 2, 1.0, 0.0, 0.0, s, 0);
    double alpha = dot_host<double>(ctx, n, v, 2, f, 2, s);
    lincomb(n, 1.0, f, 2, -alpha, v, 2, f, 2, s);
    d.push_back(alpha);
    for (int j = 1; j < k; ++j) {
        const double beta = std::sqrt(dot_host<double>(ctx, n, f, 2, f, 2, s));
        if (!(beta > 0)) break;   // invariant subspace found
        std::swap(v, vp);
        lincomb(n, 1.0 / beta, f, 2, 0.0, nullptr, 0, v, 2, s);
        hx_step<double>(H, v, 2, f, 2, nullptr, 0, 2, 1.0, 0.0, 0.0, s, 0);
        lincomb(n, 1.0, f, 2, -beta, vp, 2, f, 2, s);
        alpha = dot_host<double>(ctx, n, v, 2, f, 2, s);
        lincomb(n, 1.0, f, 2, -alpha, v, 2, f, 2, s);
        d.push_back(alpha);
        e.push_back(beta);
    }
    const double fn = std::sqrt(dot_host<double>(ctx, n, f, 2, f, 2, s));
    const double tmax = tridiag_eig(d, e, 1), tmin = tridiag_eig(d, e, 0);
    out3[0] = tmax + fn;
    out3[1] = tmin;
    out3[2] = tmax;
    if (!std::isfinite(out3[0])) fail(CHF_ENONFINITE, "lanczos_bound: non-finite result");
}

}  // namespace chf

using namespace chf;

extern "C" {

int chf_ctx_create(int device, chf_ctx** out) {
    try {
        if (!out) fail(CHF_EINVAL, "chf_ctx_create: null out");
        *out = nullptr;
        int n = 0;
        HIP_CHECK(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) fail(CHF_EINVAL, "chf_ctx_create: device %d out of range (%d devices)", device, n);
        HIP_CHECK(hipSetDevice(device));
        auto* c = new chf_ctx;
        c->device = device;
        if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
            delete c;
            fail(CHF_EHIP, "rocblas_create_handle failed");
        }
        try {
            c->info.alloc(kInfoBytes);   // device scalars and the mixing coefficients
        } catch (...) {
            rocblas_destroy_handle(c->blas);
            delete c;
            throw;
        }
        *out = c;
        return CHF_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (...) {
        set_last_error("chf_ctx_create: unknown error");
        return CHF_EHIP;
    }
}

int chf_ctx_destroy(chf_ctx* ctx) {
    if (!ctx) return CHF_OK;
    (void)hipDeviceSynchronize();
    if (ctx->blas) rocblas_destroy_handle(ctx->blas);
    delete ctx;
    return CHF_OK;
}


int gram(chf_ctx* ctx, chf_dtype dtype, const void* A, int64_t lda, const void* B, int64_t ldb, int64_t n_rows, int m,
         int n, double* S, int64_t lds, void* stream) {
    return guard([&] {
        check_ctx_block(ctx, dtype, A, lda, m, "gram A");
        check_ctx_block(ctx, dtype, B, ldb, n, "gram B");
        if (!S || lds < n || n_rows < 1) fail(CHF_EINVAL, "gram: bad output or row count");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (dtype == CHF_F64)
            gram_product<double>(ctx, static_cast<const double*>(A), lda, static_cast<const double*>(B), ldb, n_rows, m, n,
                                 S, lds, s);
        else
            gram_product<float>(ctx, static_cast<const float*>(A), lda, static_cast<const float*>(B), ldb, n_rows, m, n,
                                S, lds, s);
    });
}

int orthonormalize(chf_ctx* ctx, chf_dtype dtype, void* X, int64_t ldx, int64_t n_rows, int nvec, chf_dtype gram_dtype,
                   int* fallbacks, void* stream) {
    return guard([&] {
        check_ctx_block(ctx, dtype, X, ldx, nvec, "orthonormalize");
        if (gram_dtype != CHF_F32 && gram_dtype != CHF_F64) fail(CHF_EINVAL, "orthonormalize: bad Gram dtype");
        if (dtype == CHF_F64 && gram_dtype != CHF_F64)
            fail(CHF_EINVAL, "orthonormalize: an FP64 block needs an FP64 Gram");
        if (n_rows < nvec) fail(CHF_EINVAL, "orthonormalize: n_rows < nvec");
        if (n_rows >= (int64_t(1) << 31) || ldx >= (int64_t(1) << 31)) fail(CHF_EINVAL, "orthonormalize: block too large");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (dtype == CHF_F64)
            orthonormalize_t<double>(ctx, static_cast<double*>(X), ldx, n_rows, nvec, true, fallbacks, s);
        else
            orthonormalize_t<float>(ctx, static_cast<float*>(X), ldx, n_rows, nvec, gram_dtype == CHF_F64, fallbacks, s);
    });
}

int rayleigh_ritz(chf_ham* H, chf_ctx* ctx, chf_dtype dtype, void* X, int64_t ldx, int nvec, double* eig_host,
                  void* work, int64_t ldw, void* stream) {
    return guard([&] {
        if (!H || !eig_host) fail(CHF_EINVAL, "rayleigh_ritz: null argument");
        check_ctx_block(ctx, dtype, X, ldx, nvec, "rayleigh_ritz X");
        check_ctx_block(ctx, dtype, work, ldw, std::min(nvec, int(ldw)), "rayleigh_ritz work");
        if (!(H->dtypes & (dtype == CHF_F64 ? 2 : 1))) fail(CHF_EINVAL, "rayleigh_ritz: handle not built for dtype");
        // an orthonormal block has at most as many columns as grid points
        // (this also keeps each row panel of the in-place rotation, m values
        // per row, within the work block's n_rows x ldw values)
        if (int64_t(nvec) > H->grid.n)
            fail(CHF_EINVAL, "rayleigh_ritz: nvec %d exceeds the %lld grid points", nvec, (long long)H->grid.n);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (dtype == CHF_F64)
            rayleigh_ritz_t<double>(H, ctx, static_cast<double*>(X), ldx, nvec, eig_host, static_cast<double*>(work), ldw, s);
        else
            rayleigh_ritz_t<float>(H, ctx, static_cast<float*>(X), ldx, nvec, eig_host, static_cast<float*>(work), ldw, s);
    });
}

// device scratch of one operation: on the Hamiltonian (KB coefficients) and on
// the context (M x M matrices, Gram partials, Lanczos vectors, reductions)
struct WsNeed {
    size_t kb = 0, scratch = 0, scratch2 = 0, vec = 0, red = 0;
};

static WsNeed ws_need(const chf_ham* H, int op, chf_dtype dtype, int nvec, int64_t ldw) {
    if (!H) fail(CHF_EINVAL, "chf_workspace_bytes: null Hamiltonian");
    if (dtype != CHF_F32 && dtype != CHF_F64) fail(CHF_EINVAL, "chf_workspace_bytes: bad dtype");
    if (nvec <= 0) fail(CHF_EINVAL, "chf_workspace_bytes: nvec must be positive");
    const size_t es = dtype == CHF_F64 ? 8 : 4;
    const int64_t n_rows = H->grid.n_rows;
    WsNeed w;
    switch (op) {
    case CHF_WS_FILTER:
        w.kb = kb_coef_bytes(H, nvec, es);
        break;
    case CHF_WS_ORTHONORMALIZE:
        w.scratch = mm_scratch_bytes(nvec, cholqr_extra(nvec));
        w.scratch2 = gram_slices(n_rows, nvec, nvec, es, nvec).part_bytes;
        break;
    case CHF_WS_RAYLEIGH_RITZ: {
        if (ldw <= 0) fail(CHF_EINVAL, "chf_workspace_bytes: Rayleigh-Ritz needs the work leading dimension");
        const int nb = int(std::min<int64_t>(nvec, ldw));
        w.kb = kb_coef_bytes(H, nb, es);
        w.scratch = mm_scratch_bytes(nvec, rr_extra(nvec));
        w.scratch2 = gram_slices(n_rows, nvec, nb, es, nvec).part_bytes;
        break;
    }
    case CHF_WS_LANCZOS:
        w.kb = kb_coef_bytes(H, 2, sizeof(double));
        w.vec = lanczos_vec_bytes(n_rows);
        w.red = kRedBlocks * sizeof(double);
        break;
    default:
        fail(CHF_EINVAL, "chf_workspace_bytes: unknown operation %d", op);
    }
    return w;
}

int chf_workspace_bytes(const chf_ham* H, int op, chf_dtype dtype, int nvec, int64_t ldw, int64_t* ham_bytes,
                        int64_t* ctx_bytes) {
    return guard([&] {
        const WsNeed w = ws_need(H, op, dtype, nvec, ldw);
        if (ham_bytes) *ham_bytes = int64_t(w.kb);
        if (ctx_bytes) *ctx_bytes = int64_t(w.scratch + w.scratch2 + w.vec + w.red);
    });
}

int chf_reserve(chf_ham* H, chf_ctx* ctx, int op, chf_dtype dtype, int nvec, int64_t ldw) {
    return guard([&] {
        CHF_REQUIRE(H, "chf_reserve: null Hamiltonian");
        const WsNeed w = ws_need(H, op, dtype, nvec, ldw);
        if ((w.scratch || w.scratch2 || w.vec || w.red) && !ctx) fail(CHF_EINVAL, "chf_reserve: operation needs a context");
        if (w.kb) H->kb_coef.ensure(w.kb);
        if (ctx) {
            ctx->scratch.ensure(w.scratch);
            ctx->scratch2.ensure(w.scratch2);
            ctx->vec.ensure(w.vec);
            ctx->red.ensure(w.red);
        }
    });
}

int64_t chf_device_allocations(void) { return g_device_allocations.load(std::memory_order_relaxed); }

int lanczos_bound(chf_ham* H, chf_ctx* ctx, const double* v0, int k, double* out3, void* stream) {
    return guard([&] {
        if (!H || !ctx || !v0 || !out3) fail(CHF_EINVAL, "lanczos_bound: null argument");
        if (k < 2 || k > 64) fail(CHF_EINVAL, "lanczos_bound: k must be in [2, 64]");
        if (!(H->dtypes & 2)) fail(CHF_EINVAL, "lanczos_bound: the handle was not built for FP64");
        lanczos_run(H, ctx, v0, k, out3, static_cast<hipStream_t>(stream));
    });
}

}  // extern "C"

namespace chf {
template void dot_device<double>(chf_ctx*, int64_t, const double*, int64_t, const double*, int64_t, double*, hipStream_t);
template void dot_device<float>(chf_ctx*, int64_t, const float*, int64_t, const float*, int64_t, double*, hipStream_t);
template double dot_host<double>(chf_ctx*, int64_t, const double*, int64_t, const double*, int64_t, hipStream_t);
template void orthonormalize_t<float>(chf_ctx*, float*, int64_t, int64_t, int, bool, int*, hipStream_t);
template void orthonormalize_t<double>(chf_ctx*, double*, int64_t, int64_t, int, bool, int*, hipStream_t);
template void rayleigh_ritz_t<float>(chf_ham*, chf_ctx*, float*, int64_t, int, double*, float*, int64_t, hipStream_t);
template void rayleigh_ritz_t<double>(chf_ham*, chf_ctx*, double*, int64_t, int, double*, double*, int64_t, hipStream_t);
}  // namespace chf
