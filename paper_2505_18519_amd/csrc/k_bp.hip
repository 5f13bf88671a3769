// Back-propagated one-body density matrix (App. B, Measurement; Eqs.
// AFQMC_Metropolis_measure and AFQMC_Metropolis_measure2).  The projectors of
// the restored steps reuse the propagator's kernels (k_vbuild and k_taylor_g
// with one block per path, the walker's V shared by its paths); the overlap
// with the saved walker reuses the complex-trial overlap kernel.  Here: the
// field history, and the path-weighted density per walker and its weighted
// sum over walkers.
#include <algorithm>

#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

// hist_xi[w][slot][g] = xi[w][g], hist_xbar[w][slot][g] = xbar[w][g] (complex)
__global__ void k_bp_record(int nw, int h, int slot, int G, const double* __restrict__ xi,
                            const double* __restrict__ xbar, double* __restrict__ hxi,
                            double* __restrict__ hxb) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nw * G) return;
  const size_t w = idx / G, g = idx % G;
  const size_t d = (w * h + slot) * G + g;
  hxi[d] = xi[idx];
  hxb[2 * d] = xbar[2 * idx];
  hxb[2 * d + 1] = xbar[2 * idx + 1];
}

__global__ void k_real_to_complex(size_t n, const double* __restrict__ src, double* __restrict__ dst) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    dst[2 * q] = src[q];
    dst[2 * q + 1] = 0.0;
  }
}

// One 256-thread workgroup per walker.  Path weights a_p = exp(lt_p - Re l_p
// - max_p) (lt = log <Phi~_p|phi_mid>, l = log O_p at the measurement step;
// singular paths 0); R_k[i][j] = sum_p a_p sum_s sum_n Theta_p^s[i][n]
// Phi~_p[j][n] / sum_p a_p.  ok[k] = 1 when the walker has a live path and a
// finite R_k.
__global__ void __launch_bounds__(256)
k_bp_density(int nw, int P, int M, int N, const double* __restrict__ theta,
             const double* __restrict__ phit, const double* __restrict__ lt,
             const double* __restrict__ lend, double* __restrict__ rho, int* __restrict__ ok) {
  __shared__ double s_a[64][2];
  __shared__ double s_den[2];
  __shared__ int s_bad;
  const int k = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) {
    double mx = -__builtin_huge_val();
    for (int p = 0; p < P; ++p) {
      const double* a = lt + ((size_t)k * P + p) * 2;
      const double* b = lend + ((size_t)k * P + p) * 2;
      if (__builtin_isfinite(a[0]) && __builtin_isfinite(b[0])) mx = fmax(mx, a[0] - b[0]);
    }
    double dr = 0.0, di = 0.0;
    for (int p = 0; p < P; ++p) {
      const double* a = lt + ((size_t)k * P + p) * 2;
      const double* b = lend + ((size_t)k * P + p) * 2;
      double ar = 0.0, ai = 0.0;
      if (__builtin_isfinite(a[0]) && __builtin_isfinite(b[0])) {
        const double mag = exp(a[0] - b[0] - mx);
        double sn, cs;
        sincos(a[1], &sn, &cs);
        ar = mag * cs;
        ai = mag * sn;
      }
      s_a[p][0] = ar;
      s_a[p][1] = ai;
      dr += ar;
      di += ai;
    }
    s_den[0] = dr;
    s_den[1] = di;
    s_bad = 0;
  }
  __syncthreads();
  const double dr = s_den[0], di = s_den[1];
  const double dd = dr * dr + di * di;
  const size_t MN = (size_t)M * N;
  for (int e = tid; e < M * M; e += 256) {
    const int i = e / M, j = e % M;
    double ar = 0.0, ai = 0.0;
    for (int p = 0; p < P; ++p) {
      const double wr = s_a[p][0], wi = s_a[p][1];
      if (wr == 0.0 && wi == 0.0) continue;
      const double* X = phit + ((size_t)k * P + p) * MN * 2 + (size_t)j * N * 2;
      double sr = 0.0, si = 0.0;
      for (int sp = 0; sp < 2; ++sp) {
        const double* T = theta + (((size_t)k * P + p) * 2 + sp) * MN * 2 + (size_t)i * N * 2;
        for (int n = 0; n < N; ++n) {
          const double tr = T[2 * n], ti = T[2 * n + 1], xr = X[2 * n], xi = X[2 * n + 1];
          sr += tr * xr - ti * xi;
          si += tr * xi + ti * xr;
        }
      }
      ar += wr * sr - wi * si;
      ai += wr * si + wi * sr;
    }
    double* o = rho + ((size_t)k * M * M + e) * 2;
    if (dd > 0.0) {
      o[0] = (ar * dr + ai * di) / dd;
      o[1] = (ai * dr - ar * di) / dd;
    } else {
      o[0] = o[1] = 0.0;
    }
    if (!__builtin_isfinite(o[0])) s_bad = 1;  // benign race: any writer sets 1
  }
  __syncthreads();
  if (tid == 0) ok[k] = (dd > 0.0 && s_bad == 0) ? 1 : 0;
}

// error-free transformation a + b = s + e
__device__ __forceinline__ void two_sum_bp(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// out[e] = sum_k ok_k W_k Re R_k[e] for e < M^2, out[M^2] = sum_k ok_k W_k;
// thread e runs over the walkers in order (compensated)
__global__ void k_bp_reduce(int nw, int MM, const double* __restrict__ w,
                            const double* __restrict__ rho, const int* __restrict__ ok,
                            double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > MM) return;
  double s = 0.0, c = 0.0;
  for (int k = 0; k < nw; ++k) {
    if (!ok[k]) continue;
    const double v = (e == MM) ? w[k] : w[k] * rho[((size_t)k * MM + e) * 2];
    double t, err;
    two_sum_bp(s, v, t, err);
    s = t;
    c += err;
  }
  out[e] = s + c;
}

}  // namespace

hipError_t launch_bp_record(const afqmc_ctx_s* c, int nw, int h, int slot, const double* xi,
                            const double* xbar, double* hxi, double* hxb) {
  const size_t total = (size_t)nw * c->G;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bp_record, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                     nw, h, slot, c->G, xi, xbar, hxi, hxb);
  return hipGetLastError();
}

hipError_t launch_real_to_complex(const afqmc_ctx_s* c, size_t n, const double* src, double* dst) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_real_to_complex, dim3(blocks), dim3(256), 0, c->stream, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_bp_density(const afqmc_ctx_s* c, int nw, const double* theta, const double* phit,
                             const double* lt, const double* lend, double* rho, int* ok) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bp_density, dim3(nw), dim3(256), 0, c->stream, nw, c->P, c->M, c->N, theta,
                     phit, lt, lend, rho, ok);
  return hipGetLastError();
}

hipError_t launch_bp_reduce(const afqmc_ctx_s* c, int nw, const double* w, const double* rho,
                            const int* ok, double* out) {
  const int MM = c->M * c->M;
  hipLaunchKernelGGL(k_bp_reduce, dim3((MM + 1 + 255) / 256), dim3(256), 0, c->stream, nw, MM, w,
                     rho, ok, out);
  return hipGetLastError();
}
