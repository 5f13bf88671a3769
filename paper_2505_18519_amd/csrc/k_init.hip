// Initialisation from the trial and measurement with extra paths (App. B,
// Initialization and Measurement): the data movement around the per-path
// kernels.  All three are HBM-bound copies or a short per-walker reduction.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

// The determinant B_T(Y) phi_T as a walker: dst[w][s] = src[w * stride .. + MN)
// for both spins s, real into complex (row-major M x N, interleaved re/im).
__global__ void k_as_walker(int nw, int MN, size_t stride, const double* __restrict__ src,
                            double* __restrict__ dst) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nw * MN) return;
  const size_t w = idx / MN, i = idx % MN;
  const double v = src[w * stride + i];
  double* d = dst + (w * 2 * MN + i) * 2;
  d[0] = v;
  d[1] = 0.0;
  d[2 * (size_t)MN] = v;
  d[2 * (size_t)MN + 1] = 0.0;
}

// w[k] = Re sum_p S_p, S_p = e^{i Im l_p} over the paths with a finite Re l_p
__global__ void k_sign_sum(int nw, int P, const double* __restrict__ logov,
                           double* __restrict__ w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nw) return;
  double s = 0.0;
  for (int p = 0; p < P; ++p) {
    const double* l = logov + ((size_t)k * P + p) * 2;
    if (__builtin_isfinite(l[0])) s += cos(l[1]);
  }
  w[k] = s;
}

// Path q of walker w (of Pd) copies path q mod Ps (of Ps): one workgroup per
// destination path, threads over the MN doubles of its trial determinant.
__global__ void __launch_bounds__(256)
k_extend_paths(int Ps, int Pd, int K, int MN, const double* __restrict__ ys,
               const double* __restrict__ ps, const double* __restrict__ ls,
               double* __restrict__ yd, double* __restrict__ pd, double* __restrict__ ld) {
  const int q = blockIdx.x % Pd;
  const size_t w = blockIdx.x / Pd;
  const size_t s = w * Ps + q % Ps, d = w * Pd + q;
  for (int i = threadIdx.x; i < MN; i += blockDim.x) pd[d * MN + i] = ps[s * MN + i];
  for (int i = threadIdx.x; i < K; i += blockDim.x) yd[d * K + i] = ys[s * K + i];
  if (ls != nullptr && threadIdx.x < 2) ld[d * 2 + threadIdx.x] = ls[s * 2 + threadIdx.x];
}

}  // namespace

hipError_t launch_as_walker(const afqmc_ctx_s* c, int nw, const double* src, size_t stride,
                            double* dst) {
  const size_t total = (size_t)nw * c->M * c->N;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_as_walker, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                     nw, c->M * c->N, stride, src, dst);
  return hipGetLastError();
}

hipError_t launch_sign_sum(const afqmc_ctx_s* c, int nw, int P, const double* logov, double* w) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_sum, dim3((nw + 255) / 256), dim3(256), 0, c->stream, nw, P, logov, w);
  return hipGetLastError();
}

hipError_t launch_extend_paths(const afqmc_ctx_s* c, int nw, int Ps, int Pd, const double* ys,
                               const double* ps, const double* ls, double* yd, double* pd,
                               double* ld) {
  if (nw <= 0 || Pd <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_extend_paths, dim3((unsigned)((size_t)nw * Pd)), dim3(256), 0, c->stream,
                     Ps, Pd, c->K, c->tsz, ys, ps, ls, yd, pd, ld);
  return hipGetLastError();
}
