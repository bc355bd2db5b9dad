// lre_project.hip -- step (iii) of LRE: the density matrix closest to mu.
//
// Sec. II, step (iii): mu from eq. (4) can have negative eigenvalues; the estimate is
// the physical state closest to it, computed with the fast algorithm the paper cites
// (Smolin, Gambetta and Smith 2012): eigendecompose mu, move the spectrum onto the
// probability simplex (negative eigenvalues removed, their mass shared equally over
// the eigenvalues kept), reassemble.  The eigendecomposition is rocSOLVER's
// divide-and-conquer Hermitian solver (zheevd) and the reassembly V diag(lambda) V^H a
// rocBLAS zgemm -- dense O(d^3) library work, bound by FP64 matrix throughput; the
// spectrum step and the column scaling are kernels of this file.
//
// Layout: mu and rho are row-major complex128 [d][d].  Read column-major, the row-major
// buffer of a Hermitian matrix is its conjugate; the projection commutes with complex
// conjugation, so running the column-major solver and product on the buffers as they
// are yields rho row-major.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "lre.h"
#include "lre_internal.hpp"
#include "lre_kernels.hpp"

namespace {

using lre_detail::DeviceGuard;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct ProjLayout {
  size_t a, b, w, e, lam, info, total;
};

ProjLayout proj_layout(int n) {
  const size_t d = (size_t)1 << n;
  ProjLayout L{};
  size_t off = 0;
  L.a = off; off += align256(16 * d * d);     // eigenvectors (the solver works in place)
  L.b = off; off += align256(16 * d * d);     // eigenvectors scaled by the new spectrum
  L.w = off; off += align256(8 * d);          // eigenvalues of mu, ascending
  L.e = off; off += align256(8 * d);          // solver scratch (off-diagonal)
  L.lam = off; off += align256(8 * d);        // projected spectrum
  L.info = off; off += align256(sizeof(rocblas_int));
  L.total = off;
  return L;
}

// Spectrum step on the ascending eigenvalues w[0..d): while the smallest eigenvalue
// still kept, plus the removed mass a shared over the k kept ones, is negative, drop
// it; raise the kept ones by a / k.  One thread (d <= 2^14); a solver failure (info !=
// 0) raises FLAG_EIG and leaves lambda = 0.
__global__ void spectrum_kernel(const double* __restrict__ w, double* __restrict__ lam,
                                const rocblas_int* __restrict__ info, int d, uint32_t* __restrict__ flags,
                                double* __restrict__ eig_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*info != 0) {
    atomicOr(flags, (uint32_t)lre::FLAG_EIG);
    for (int j = 0; j < d; ++j) lam[j] = 0.0;
    return;
  }
  double a = 0.0;
  int k = d, i = 0;
  while (i < d && w[i] + a / k < 0.0) {
    a += w[i];
    --k;
    ++i;
  }
  for (int j = 0; j < i; ++j) lam[j] = 0.0;
  for (int j = i; j < d; ++j) lam[j] = w[j] + a / k;
  if (eig_out)
    for (int j = 0; j < d; ++j) eig_out[j] = w[j];
}

// b[:, j] = a[:, j] * lam[j] (column-major d x d).
__global__ __launch_bounds__(256) void scale_columns_kernel(const double2* __restrict__ a,
                                                            const double* __restrict__ lam,
                                                            double2* __restrict__ b, int n) {
  const int64_t d = (int64_t)1 << n;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= d * d) return;
  const double s = lam[i >> n];
  const double2 v = a[i];
  b[i] = make_double2(v.x * s, v.y * s);
}

}  // namespace

namespace lre_detail {

void destroy_blas(void* handle) {
  if (handle) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(handle));
}

}  // namespace lre_detail

extern "C" {

size_t lre_project_workspace_bytes(int n) {
  if (n < 1 || n > LRE_MAX_QUBITS) return 0;
  return proj_layout(n).total;
}

lre_status lre_project(lre_ctx* ctx, int n, const void* mu, void* rho, double* eigvals, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (!ctx || !mu || !rho || !workspace || n < 1 || n > LRE_MAX_QUBITS) return LRE_E_ARG;
  if (((uintptr_t)mu & 15u) || ((uintptr_t)rho & 15u) || ((uintptr_t)workspace & 255u) ||
      ((uintptr_t)eigvals & 7u))
    return LRE_E_ARG;
  const ProjLayout L = proj_layout(n);
  if (workspace_bytes < L.total) return LRE_E_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return LRE_E_HIP;
    ctx->blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(ctx->blas);
  if (rocblas_set_stream(h, st) != rocblas_status_success) return LRE_E_HIP;

  const int d = 1 << n;
  char* ws = static_cast<char*>(workspace);
  auto* A = reinterpret_cast<rocblas_double_complex*>(ws + L.a);
  auto* B = reinterpret_cast<rocblas_double_complex*>(ws + L.b);
  auto* W = reinterpret_cast<double*>(ws + L.w);
  auto* E = reinterpret_cast<double*>(ws + L.e);
  auto* lam = reinterpret_cast<double*>(ws + L.lam);
  auto* info = reinterpret_cast<rocblas_int*>(ws + L.info);

  if (hipMemcpyAsync(A, mu, (size_t)16 * d * d, hipMemcpyDeviceToDevice, st) != hipSuccess) return LRE_E_HIP;
  if (rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, d, A, d, W, E, info) !=
      rocblas_status_success)
    return LRE_E_HIP;
  hipLaunchKernelGGL(spectrum_kernel, dim3(1), dim3(64), 0, st, W, lam, info, d, ctx->flags, eigvals);
  const int64_t elems = (int64_t)d * d;
  hipLaunchKernelGGL(scale_columns_kernel, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(A), lam, reinterpret_cast<double2*>(B), n);
  if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  if (rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_conjugate_transpose, d, d, d, &one, B, d, A,
                    d, &zero, static_cast<rocblas_double_complex*>(rho), d) != rocblas_status_success)
    return LRE_E_HIP;
  return LRE_OK;
}

}  // extern "C"
