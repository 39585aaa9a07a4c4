// Launchers shared between the library's translation units.
#pragma once
#include "internal.hpp"

namespace chf {

void launch_vloc(chf_ham* H, const double4* atoms, const double* width, int n_atoms, hipStream_t s);
void launch_cast_veff(chf_ham* H, const double* src, double* d64, float* d32, int* bad_dev, hipStream_t s);
template <class T>
void launch_kb_gather(chf_ham* H, const T* X, int64_t ldx, int nvec, T* C, hipStream_t s);
// Y = alpha (H X - shift X) - beta Z ; Z may be null or alias Y.  force_kernel:
// 0 = best available, 1 = generic neighbour-table kernel.  lap_only: H is
// replaced by -1/2 L (no V_eff, no projectors).
// C_ext: caller-provided KB-coefficient scratch for nvec vectors (no
// allocation, no kernel timing); NULL uses the handle's scratch.
template <class T>
void hx_step(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec, double alpha,
             double shift, double beta, hipStream_t s, int force_kernel, bool lap_only = false, T* C_ext = nullptr);

// Degree-m scaled Chebyshev filter in place over X and the work block W
// (column blocks of min(nvec, ldw) vectors)
template <class T>
void filter_run(chf_ham* H, T* X, int64_t ldx, T* W, int64_t ldw, int nvec, int m, double a, double b, double a0,
                hipStream_t s, int force_kernel, int64_t max_cols = INT64_MAX, T* C_ext = nullptr);
// the same filter with the KB coefficients in the library's fixed device
// scratch (no allocation); noalloc_scratch_init looks its address up for the
// current device (called by ham_build)
void noalloc_scratch_init(int device);
template <class T>
void filter_run_noalloc(chf_ham* H, T* X, int64_t ldx, T* W, int64_t ldw, int nvec, int m, double a, double b,
                        double a0, hipStream_t s);
// CHF_EINVAL unless the [n_rows][ld] spans of A and B are disjoint (capi.cpp)
void check_disjoint(const chf_ham* H, int dtype, const void* A, int64_t lda, const void* B, int64_t ldb,
                    const char* what);

// bytes of the KB coefficient scratch an H X launch on nvec vectors needs
size_t kb_coef_bytes(const chf_ham* H, int nvec, size_t elem_bytes);

void timer_enable(int on);
void timer_read(double* ms, int64_t* launches);

// dense.hip
template <class T>
void dot_device(chf_ctx* ctx, int64_t n, const T* x, int64_t incx, const T* y, int64_t incy, double* out_dev,
                hipStream_t s);
template <class T>
double dot_host(chf_ctx* ctx, int64_t n, const T* x, int64_t incx, const T* y, int64_t incy, hipStream_t s);
void lincomb(int64_t n, double a, const double* x, int64_t incx, double b, const double* y, int64_t incy, double* z,
             int64_t incz, hipStream_t s);
template <class T>
void orthonormalize_t(chf_ctx* ctx, T* X, int64_t ldx, int64_t n_rows, int m, bool gram64, int* fallbacks,
                      hipStream_t s);
template <class T>
void rayleigh_ritz_t(chf_ham* H, chf_ctx* ctx, T* X, int64_t ldx, int m, double* eig_host, T* W, int64_t ldw,
                     hipStream_t s);
void lanczos_run(chf_ham* H, chf_ctx* ctx, const double* v0, int k, double* out3, hipStream_t s);
template <class T>
void gram_product(chf_ctx* ctx, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n_rows, int m, int n,
                  double* S, int64_t lds, hipStream_t s);

}  // namespace chf
