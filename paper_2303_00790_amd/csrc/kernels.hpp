// Launchers shared between the library's translation units.
#pragma once
#include "internal.hpp"

namespace chf {

void launch_vloc(chf_ham* H, const double4* atoms, const double* width, int n_atoms, hipStream_t s);
void launch_cast_veff(chf_ham* H, const double* src, double* d64, float* d32, int* bad_dev, hipStream_t s);
template <class T>
void launch_kb_gather(chf_ham* H, const T* X, int64_t ldx, int nvec, T* C, hipStream_t s);
// Y = alpha (H X - shift X) - beta Z ; Z may be null or alias Y.  force_kernel:
// 0 = best available, 1 = generic neighbour-table kernel.
template <class T>
void hx_step(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec, double alpha,
             double shift, double beta, hipStream_t s, int force_kernel);

// dense.hip
template <class T>
void gram_product(chf_ctx* ctx, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n_rows, int m, int n,
                  double* S, int64_t lds, hipStream_t s);

}  // namespace chf
