// Marginal covariances of the tracking Hessian (Sec. 3.1, Eq. 1 and 2) in
// FP64 on gfx950: the producer of the per-pixel depth variances Sigma_D that
// weight the depth loss (Eq. 4).
//
//   H_T     = C - E P^{-1} E^T                 (Schur complement, c x c)
//   H_T     = L L^T,  Sigma_T = (L L^T)^{-1}   (Cholesky, then L^{-T} L^{-1})
//   Sigma_d = 1/P_j + e_j^T Sigma_T e_j / P_j^2   (diagonal of Eq. 2)
//   Sigma_D = Sigma_d / d_j^4                  (first order, D = 1/d)
//
// c (6 per keyframe, at most 60) is small and p (pixels) large: the Schur sum is split
// over pixel chunks with per-block partial matrices reduced in a fixed
// order; the factorisation runs in one workgroup in LDS; the quadratic forms
// run one thread per pixel with Sigma_T in LDS.
#include "kernels.h"

namespace nsl {

namespace {

constexpr int kCovThreads = 256;
constexpr int kPixChunk = 64;

// partial[blk] = sum over the block's pixels of e_j e_j^T / P_j
__global__ __launch_bounds__(kCovThreads) void schur_partial_kernel(const double* __restrict__ Et,
                                                                    const double* __restrict__ P, int c, int p,
                                                                    int per_block, double* __restrict__ partial) {
  extern __shared__ double sh[];
  double* e = sh;  // [kPixChunk][c]
  const int j0 = blockIdx.x * per_block, j1 = min(p, j0 + per_block);
  const int cc = c * c;
  double* out = partial + (size_t)blockIdx.x * cc;
  for (int base = 0; base < cc; base += kCovThreads * 12) {
    double a[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = 0.0;
    for (int jc = j0; jc < j1; jc += kPixChunk) {
      const int n = min(kPixChunk, j1 - jc);
      __syncthreads();
      for (int i = threadIdx.x; i < n * c; i += kCovThreads) {
        const int jj = i / c;
        e[i] = Et[(size_t)(jc + jj) * c + (i - jj * c)] / sqrt(P[jc + jj]);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const int idx = base + k * kCovThreads + threadIdx.x;
        if (idx < cc) {
          const int r = idx / c, s = idx - r * c;
          double v = 0.0;
          for (int jj = 0; jj < n; ++jj) v = fma(e[jj * c + r], e[jj * c + s], v);
          a[k] += v;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const int idx = base + k * kCovThreads + threadIdx.x;
      if (idx < cc) out[idx] = a[k];
    }
  }
}

// H = C - sum of partials (fixed order).
__global__ void schur_reduce_kernel(const double* __restrict__ C, const double* __restrict__ partial, int nblk,
                                    int cc, double* __restrict__ H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cc) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * cc + i];
  H[i] = C[i] - s;
}

// In place: H (c x c, symmetric positive definite) -> Sigma_T = H^{-1} via
// H = L L^T.  status = 1 (and NaN output) if a pivot is not positive.
__global__ __launch_bounds__(kCovThreads) void chol_inverse_kernel(double* __restrict__ H, int c,
                                                                   int* __restrict__ status) {
  extern __shared__ double sh[];
  double* A = sh;          // [c][c], becomes L (lower)
  double* X = sh + c * c;  // [c][c], becomes L^{-1}
  __shared__ int bad;
  const int cc = c * c, tid = threadIdx.x;
  for (int i = tid; i < cc; i += kCovThreads) A[i] = H[i];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < c; ++k) {
    if (tid == 0) {
      const double d = A[k * c + k];
      if (!(d > 0.0)) bad = 1;
      A[k * c + k] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double lkk = A[k * c + k];
    for (int i = k + 1 + tid; i < c; i += kCovThreads) A[i * c + k] /= lkk;
    __syncthreads();
    for (int idx = tid; idx < cc; idx += kCovThreads) {
      const int i = idx / c, j = idx - i * c;
      if (i > k && j > k && j <= i) A[i * c + j] -= A[i * c + k] * A[j * c + k];
    }
    __syncthreads();
  }
  // X = L^{-1}: column j solved by thread j (forward substitution)
  for (int j = tid; j < c; j += kCovThreads) {
    for (int i = 0; i < c; ++i) {
      double s = i == j ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= A[i * c + k] * X[k * c + j];
      X[i * c + j] = i < j ? 0.0 : s / A[i * c + i];
    }
  }
  __syncthreads();
  // Sigma_T = X^T X
  for (int idx = tid; idx < cc; idx += kCovThreads) {
    const int i = idx / c, j = idx - i * c;
    double s = 0.0;
    for (int k = max(i, j); k < c; ++k) s = fma(X[k * c + i], X[k * c + j], s);
    H[idx] = bad ? __longlong_as_double(0x7ff8000000000000ll) : s;
  }
  if (tid == 0) *status = bad;
}

// Per pixel: sigma_d = 1/P + e^T Sigma_T e / P^2, depth_var = sigma_d / d^4.
__global__ __launch_bounds__(kCovThreads) void marginal_kernel(const double* __restrict__ Et,
                                                               const double* __restrict__ P,
                                                               const double* __restrict__ inv_depth,
                                                               const double* __restrict__ S, int c, int p,
                                                               double* __restrict__ sigma_d,
                                                               float* __restrict__ depth_var) {
  extern __shared__ double sh[];
  for (int i = threadIdx.x; i < c * c; i += kCovThreads) sh[i] = S[i];
  __syncthreads();
  const int j = blockIdx.x * kCovThreads + threadIdx.x;
  if (j >= p) return;
  const double* e = Et + (size_t)j * c;
  double q = 0.0;
  for (int a = 0; a < c; ++a) {
    double v = 0.0;
    for (int b = 0; b < c; ++b) v = fma(sh[a * c + b], e[b], v);
    q = fma(e[a], v, q);
  }
  const double pi = 1.0 / P[j];
  const double sd = pi + pi * pi * q;
  if (sigma_d) sigma_d[j] = sd;
  if (depth_var) {
    const double d = inv_depth[j], d2 = d * d;
    depth_var[j] = (float)(sd / (d2 * d2));
  }
}

}  // namespace

size_t cov_partial_blocks(int p) { return (size_t)min(256, max(1, (p + 255) / 256)); }

hipError_t depth_covariance(int c, int p, const double* C, const double* Et, const double* P,
                            const double* inv_depth, double* sigma_T, double* sigma_d, float* depth_var,
                            int* status, double* partial, hipStream_t st) {
  const int nblk = (int)cov_partial_blocks(p);
  const int per_block = (p + nblk - 1) / nblk;
  const int cc = c * c;
  hipLaunchKernelGGL(schur_partial_kernel, dim3(nblk), dim3(kCovThreads), kPixChunk * c * sizeof(double), st, Et,
                     P, c, p, per_block, partial);
  hipLaunchKernelGGL(schur_reduce_kernel, dim3((cc + 255) / 256), dim3(256), 0, st, C, partial, nblk, cc, sigma_T);
  hipLaunchKernelGGL(chol_inverse_kernel, dim3(1), dim3(kCovThreads), 2 * cc * sizeof(double), st, sigma_T, c,
                     status);
  if (p > 0)
    hipLaunchKernelGGL(marginal_kernel, dim3((p + kCovThreads - 1) / kCovThreads), dim3(kCovThreads),
                       cc * sizeof(double), st, Et, P, inv_depth, sigma_T, c, p, sigma_d, depth_var);
  return hipGetLastError();
}

}  // namespace nsl
