// Set-up kernels (h1', e^{-tau h1/2}), counter-based random streams, the
// mixed-estimator sums and walker re-orthonormalisation.
#include <algorithm>
#include <vector>

#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

// h1' = h1 + 1/2 sum_g L_g L_g into slab G of the padded L array, the sum over g
// split into GS chunks of consecutive vectors (one grid row each) and the
// chunks' partial sums added in chunk order
__global__ void k_h1_part(int M, int G, int GS, const double* __restrict__ L,
                          double* __restrict__ part) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int i = e / M, j = e % M, q = blockIdx.y;
  const int g0 = (int)((long)G * q / GS), g1 = (int)((long)G * (q + 1) / GS);
  double acc = 0.0;
  for (int gm = g0; gm < g1; ++gm) {
    const double* Lg = L + (size_t)gm * M * M;
    double t = 0.0;
    for (int k = 0; k < M; ++k) t += Lg[i * M + k] * Lg[k * M + j];
    acc += t;
  }
  part[(size_t)q * M * M + e] = acc;
}

__global__ void k_h1_fin(int M, int MT, int G, int GS, const double* __restrict__ h1,
                         const double* __restrict__ part, double* __restrict__ Lpad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  double acc = 0.0;
  for (int q = 0; q < GS; ++q) acc += part[(size_t)q * M * M + e];
  const int i = e / M, j = e % M;
  Lpad[(size_t)G * MT * MT + i * MT + j] = h1[e] + 0.5 * acc;
}

// exp(X), X = -tau h1 / 2, by scaling and squaring of a 24-term Taylor series
// (|X / 2^s|_1 <= 1/4, s chosen on the host): one launch per term and per
// squaring, one thread per entry, each entry's sum over k in ascending k.
__global__ void k_expm_init(int M, double scale, const double* __restrict__ h1,
                            double* __restrict__ X, double* __restrict__ T,
                            double* __restrict__ E) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  X[e] = scale * h1[e];
  const double id = ((e / M) == (e % M)) ? 1.0 : 0.0;
  T[e] = id;
  E[e] = id;
}

// Tn = A B * f; with E given, E += Tn
__global__ void k_mm_f64(int M, const double* __restrict__ A, const double* __restrict__ B,
                         double f, double* __restrict__ Tn, double* __restrict__ E) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int r = e / M, cc = e % M;
  double acc = 0.0;
  for (int k = 0; k < M; ++k) acc += A[r * M + k] * B[k * M + cc];
  const double v = acc * f;
  Tn[e] = v;
  if (E != nullptr) E[e] += v;
}

__global__ void k_philox_normal(uint64_t seed, uint64_t step, const uint64_t* __restrict__ dstep,
                                uint64_t w3, int nw, int n, double* __restrict__ out) {
  const int nb = (n + 3) / 4;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nw * nb) return;
  if (dstep != nullptr) step = *dstep;
  const int w = (int)(idx / nb), b = (int)(idx % nb);
  ph4 blk = philox4x64_10((uint64_t)b, (uint64_t)w, step, w3, seed, 0);
  double z[4];
  normals4(blk, z);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * b + q < n) out[(size_t)w * n + 4 * b + q] = z[q];
}

__global__ void k_sample_prior(int nw, int P, int K, int hidden_kind, uint64_t seed, int sweep,
                               double* __restrict__ y) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nw * P * K) return;
  const int k = (int)(idx % K);
  const int p = (int)((idx / K) % P);
  const int w = (int)(idx / ((size_t)K * P));
  const uint64_t w3 = rng_word3(AFQMC_TAG_INIT, sweep, p);
  if (hidden_kind == AFQMC_HIDDEN_ISING)
    y[idx] = (stream_uniform(seed, w, 0, w3, k) < 0.5) ? -1.0 : 1.0;
  else
    y[idx] = stream_normal(seed, w, 0, w3, k);
}

// error-free transformation a + b = s + e
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// out[0] = sum W Re E_L, out[1] = sum W, compensated (sum + error term)
__global__ void __launch_bounds__(256)
k_estimator(int nw, const double* __restrict__ w, const double* __restrict__ eloc,
            double* __restrict__ out, const uint64_t* __restrict__ dstep, int cap) {
  __shared__ double s_v[4][256];
  const int tid = threadIdx.x;
  double n_s = 0.0, n_e = 0.0, d_s = 0.0, d_e = 0.0;
  for (int k = tid; k < nw; k += 256) {
    double s, e;
    const double el = eloc[2 * (size_t)k];
    const bool ok = __builtin_isfinite(el);  // a non-finite E_L drops out of both sums
    two_sum(n_s, ok ? w[k] * el : 0.0, s, e);
    n_s = s;
    n_e += e;
    two_sum(d_s, ok ? w[k] : 0.0, s, e);
    d_s = s;
    d_e += e;
  }
  s_v[0][tid] = n_s;
  s_v[1][tid] = n_e;
  s_v[2][tid] = d_s;
  s_v[3][tid] = d_e;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) {
      double s, e;
      two_sum(s_v[0][tid], s_v[0][tid + o], s, e);
      s_v[0][tid] = s;
      s_v[1][tid] += s_v[1][tid + o] + e;
      two_sum(s_v[2][tid], s_v[2][tid + o], s, e);
      s_v[2][tid] = s;
      s_v[3][tid] += s_v[3][tid + o] + e;
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* o = (dstep != nullptr) ? out + 2 * (size_t)(*dstep % (uint64_t)cap) : out;
    o[0] = s_v[0][0] + s_v[1][0];
    o[1] = s_v[2][0] + s_v[3][0];
  }
}

// Mixed estimator with a correction factor per walker (measurement with extra
// paths): R_k = sum_q S'_q / sum_p S_p from the new paths' log-overlaps (P)
// and the current ones (Pr); out[0] = sum W Re(R E_L), out[1] = sum W Re R,
// compensated as in k_estimator; R [nw] complex is written when non-null.
__global__ void __launch_bounds__(256)
k_estimator_corrected(int nw, int P, int Pr, const double* __restrict__ w,
                      const double* __restrict__ eloc, const double* __restrict__ logov,
                      const double* __restrict__ logov_ref, double* __restrict__ out,
                      double* __restrict__ R) {
  __shared__ double s_v[4][256];
  const int tid = threadIdx.x;
  double n_s = 0.0, n_e = 0.0, d_s = 0.0, d_e = 0.0;
  for (int k = tid; k < nw; k += 256) {
    cplx s2 = cmk(0.0, 0.0), s1 = cmk(0.0, 0.0);
    for (int q = 0; q < P; ++q) {
      const double* l = logov + ((size_t)k * P + q) * 2;
      if (__builtin_isfinite(l[0])) {
        double sn, cs;
        sincos(l[1], &sn, &cs);
        s2 = cadd(s2, cmk(cs, sn));
      }
    }
    for (int p = 0; p < Pr; ++p) {
      const double* l = logov_ref + ((size_t)k * Pr + p) * 2;
      if (__builtin_isfinite(l[0])) {
        double sn, cs;
        sincos(l[1], &sn, &cs);
        s1 = cadd(s1, cmk(cs, sn));
      }
    }
    const cplx r = (s1.re != 0.0 || s1.im != 0.0) ? cdiv(s2, s1) : cmk(0.0, 0.0);
    if (R != nullptr) cst(R + 2 * (size_t)k, r);
    const cplx re = cmul(r, cld(eloc + 2 * (size_t)k));
    const bool ok = __builtin_isfinite(re.re) && __builtin_isfinite(r.re);
    double s, e;
    two_sum(n_s, ok ? w[k] * re.re : 0.0, s, e);
    n_s = s;
    n_e += e;
    two_sum(d_s, ok ? w[k] * r.re : 0.0, s, e);
    d_s = s;
    d_e += e;
  }
  s_v[0][tid] = n_s;
  s_v[1][tid] = n_e;
  s_v[2][tid] = d_s;
  s_v[3][tid] = d_e;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) {
      double s, e;
      two_sum(s_v[0][tid], s_v[0][tid + o], s, e);
      s_v[0][tid] = s;
      s_v[1][tid] += s_v[1][tid + o] + e;
      two_sum(s_v[2][tid], s_v[2][tid + o], s, e);
      s_v[2][tid] = s;
      s_v[3][tid] += s_v[3][tid + o] + e;
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = s_v[0][0] + s_v[1][0];
    out[1] = s_v[2][0] + s_v[3][0];
  }
}

// Re-orthonormalisation by modified Gram-Schmidt applied twice, one 64-lane
// workgroup per walker (lane = orbital row; M <= 64, N <= 16).  R_jj is the
// norm of column j after both projection passes, hence real positive.
__global__ void __launch_bounds__(64)
k_qr(int nw, int P, int M, int N, double* __restrict__ phi, double* __restrict__ logov) {
  constexpr int NTQ = 16;
  const int w = blockIdx.x;
  const int m = threadIdx.x;
  double shift = 0.0;
  for (int sp = 0; sp < 2; ++sp) {
    double* base = phi + ((size_t)(w * 2 + sp) * M) * N * 2;
    cplx q[NTQ];
#pragma unroll
    for (int j = 0; j < NTQ; ++j)
      q[j] = (m < M && j < N) ? cmk(base[((size_t)m * N + j) * 2], base[((size_t)m * N + j) * 2 + 1])
                              : cmk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < NTQ; ++j) {
      if (j < N) {
        cplx v = q[j];
#pragma unroll
        for (int pass = 0; pass < 2; ++pass)
#pragma unroll
          for (int k = 0; k < j; ++k) {
            // h = q_k^H v
            double hr = q[k].re * v.re + q[k].im * v.im;
            double hi = q[k].re * v.im - q[k].im * v.re;
            hr = wave_sum(hr);
            hi = wave_sum(hi);
            v = cfms(v, cmk(hr, hi), q[k]);
          }
        const double nrm = sqrt(wave_sum(cabs2(v)));
        shift += log(nrm);
        q[j] = cscale(v, 1.0 / nrm);
      }
    }
    if (m < M)
#pragma unroll
      for (int j = 0; j < NTQ; ++j)
        if (j < N) {
          base[((size_t)m * N + j) * 2] = q[j].re;
          base[((size_t)m * N + j) * 2 + 1] = q[j].im;
        }
  }
  if (logov != nullptr)
    for (int p = m; p < P; p += 64) logov[((size_t)w * P + p) * 2] -= shift;
}

__global__ void k_to_float(size_t n, const double* __restrict__ src, float* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

__global__ void k_zero_int(int n, int* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_setup(afqmc_ctx_s* c) {
  const int M = c->M, MM = M * M;
  const int GS = std::max(1, std::min(c->G, 64));
  const dim3 eg((MM + 255) / 256);
  double* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, (size_t)std::max(GS, 5) * MM * sizeof(double));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_h1_part, dim3(eg.x, GS), dim3(256), 0, c->stream, M, c->G, GS, c->d_Lraw,
                     tmp);
  if ((e = hipGetLastError()) == hipSuccess) {
    hipLaunchKernelGGL(k_h1_fin, eg, dim3(256), 0, c->stream, M, c->MT, c->G, GS, c->d_h1, tmp,
                       c->d_Lpad);
    e = hipGetLastError();
  }
  // the squarings of exp(-tau h1 / 2): 1-norm of tau h1 / 2 halved until <= 1/4
  std::vector<double> h1((size_t)MM);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess)
    e = hipMemcpy(h1.data(), c->d_h1, (size_t)MM * sizeof(double), hipMemcpyDeviceToHost);
  int sq = 0;
  if (e == hipSuccess) {
    double nrm = 0.0;
    for (int j = 0; j < M; ++j) {
      double cs = 0.0;
      for (int i = 0; i < M; ++i) cs += fabs(h1[(size_t)i * M + j]);
      nrm = std::max(nrm, cs);
    }
    nrm *= 0.5 * c->dtau;
    while (nrm > 0.25 && sq < 64) {
      nrm *= 0.5;
      ++sq;
    }
  }
  double *X = tmp, *T = tmp + MM, *T2 = tmp + 2 * MM, *E = tmp + 3 * MM, *E2 = tmp + 4 * MM;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_expm_init, eg, dim3(256), 0, c->stream, M, -0.5 * c->dtau * ldexp(1.0, -sq),
                       c->d_h1, X, T, E);
    e = hipGetLastError();
  }
  for (int j = 1; j <= 24 && e == hipSuccess; ++j) {
    hipLaunchKernelGGL(k_mm_f64, eg, dim3(256), 0, c->stream, M, X, T, 1.0 / (double)j, T2, E);
    e = hipGetLastError();
    std::swap(T, T2);
  }
  for (int q = 0; q < sq && e == hipSuccess; ++q) {
    hipLaunchKernelGGL(k_mm_f64, eg, dim3(256), 0, c->stream, M, E, E, 1.0, E2,
                       (double*)nullptr);
    e = hipGetLastError();
    std::swap(E, E2);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d_Eh, E, (size_t)MM * sizeof(double), hipMemcpyDeviceToDevice,
                       c->stream);
  hipError_t e2 = hipStreamSynchronize(c->stream);
  const hipError_t e3 = hipFree(tmp);
  return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : e3);
}

hipError_t launch_philox_normal(const afqmc_ctx_s* c, uint64_t seed, uint64_t step, uint32_t tag,
                                int nw, int n, double* out) {
  const size_t total = (size_t)nw * ((n + 3) / 4);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_normal, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     c->stream, seed, step, c->dstep, ((uint64_t)tag << 48), nw, n, out);
  return hipGetLastError();
}

hipError_t launch_sample_prior(const afqmc_ctx_s* c, int nw, uint64_t seed, double* y, int sweep) {
  const size_t total = (size_t)nw * c->P * c->K;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample_prior, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     c->stream, nw, c->P, c->K, c->hidden_kind, seed, sweep, y);
  return hipGetLastError();
}

hipError_t launch_estimator_corrected(const afqmc_ctx_s* c, int nw, int Pr, const double* w,
                                      const double* eloc, const double* logov,
                                      const double* logov_ref, double* out, double* R) {
  hipLaunchKernelGGL(k_estimator_corrected, dim3(1), dim3(256), 0, c->stream, nw, c->P, Pr, w, eloc,
                     logov, logov_ref, out, R);
  return hipGetLastError();
}

hipError_t launch_estimator(const afqmc_ctx_s* c, int nw, const double* w, const double* eloc,
                            double* out) {
  hipLaunchKernelGGL(k_estimator, dim3(1), dim3(256), 0, c->stream, nw, w, eloc, out, c->dstep,
                     c->est_cap);
  return hipGetLastError();
}

hipError_t launch_qr(const afqmc_ctx_s* c, int nw, double* phi, double* logov) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qr, dim3(nw), dim3(64), 0, c->stream, nw, c->P, c->M, c->N, phi, logov);
  return hipGetLastError();
}

hipError_t launch_to_float(const afqmc_ctx_s* c, size_t n, const double* src, float* dst) {
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, src,
                     dst);
  return hipGetLastError();
}

namespace {

// complex64 walkers: exact widening to complex128, rounding to nearest back
__global__ void k_phi_widen(size_t n, const float2* __restrict__ src, double2* __restrict__ dst) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const float2 v = src[q];
    dst[q] = make_double2((double)v.x, (double)v.y);
  }
}
__global__ void k_phi_narrow(size_t n, const double2* __restrict__ src, float2* __restrict__ dst) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const double2 v = src[q];
    dst[q] = make_float2((float)v.x, (float)v.y);
  }
}

}  // namespace

hipError_t launch_phi_widen(const afqmc_ctx_s* c, size_t n, const float* src, double* dst) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_phi_widen, dim3(blocks), dim3(256), 0, c->stream, n,
                     reinterpret_cast<const float2*>(src), reinterpret_cast<double2*>(dst));
  return hipGetLastError();
}

hipError_t launch_phi_narrow(const afqmc_ctx_s* c, size_t n, const double* src, float* dst) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_phi_narrow, dim3(blocks), dim3(256), 0, c->stream, n,
                     reinterpret_cast<const double2*>(src), reinterpret_cast<float2*>(dst));
  return hipGetLastError();
}

hipError_t launch_zero_int(const afqmc_ctx_s* c, int n, int* p) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Re-orthonormalisation for larger systems (M <= 160, N <= 40): classical
// Gram-Schmidt applied twice (each column projected against all the previous
// ones at once, then again), one workgroup of QW wavefronts (64 QW >= M) per
// walker and spin, thread = orbital row, the columns in LDS.  The j inner
// products h = Q_{<j}^H v of column j are summed by lane k of each wavefront
// over that wavefront's 64 rows and the wavefronts' partial sums added through
// LDS: three barriers per pass instead of one workgroup reduction per inner
// product.  The rows in LDS are padded by one complex entry, so that the
// threads' reads along their own rows fall on different banks.
namespace {

template <int QW>
__global__ void __launch_bounds__(64 * QW)
k_qr_g(int nw, int P, int M, int N, double* __restrict__ phi, double* __restrict__ logshift) {
  constexpr int QRG_T = 64 * QW;
  extern __shared__ double sq[];           // [M][RS]: row m, N complex entries and a pad
  __shared__ double s_v[QRG_T][2];         // the column being orthogonalised
  __shared__ double s_hp[QW][64][2];       // per-wavefront partial inner products
  __shared__ double s_h[64][2];            // h = Q_{<j}^H v
  __shared__ double s_red[QW][2];
  const int w = blockIdx.x, sp = blockIdx.y;
  const int m = threadIdx.x, wave = m >> 6, lane = m & 63;
  const int RS = 2 * N + 2;  // LDS row stride (doubles)
  double* base = phi + ((size_t)(w * 2 + sp) * M) * N * 2;
  for (int q = threadIdx.x; q < M * N * 2; q += QRG_T) sq[(q / (2 * N)) * RS + q % (2 * N)] = base[q];
  __syncthreads();
  auto block_sum2 = [&](double& a, double& b) {
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      s_red[wave][0] = a;
      s_red[wave][1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int q = 0; q < QW; ++q) {
      a += s_red[q][0];
      b += s_red[q][1];
    }
    __syncthreads();
  };
  double shift = 0.0;
  double* row = sq + (size_t)m * RS;
  const bool own = m < M;
  const int r0 = 64 * wave, r1 = min(r0 + 64, M);  // this wavefront's rows
  for (int j = 0; j < N; ++j) {
    cplx v = own ? cmk(row[2 * j], row[2 * j + 1]) : cmk(0.0, 0.0);
    for (int pass = 0; pass < 2 && j > 0; ++pass) {
      s_v[m][0] = v.re;
      s_v[m][1] = v.im;
      __syncthreads();
      if (lane < j) {  // sum over this wavefront's rows of conj(q_mk) v_m, k = lane
        double hr[4] = {0.0, 0.0, 0.0, 0.0}, hi[4] = {0.0, 0.0, 0.0, 0.0};
        int mm = r0;
        for (; mm + 4 <= r1; mm += 4)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double* q = sq + (size_t)(mm + u) * RS + 2 * lane;
            const double vr = s_v[mm + u][0], vi = s_v[mm + u][1];
            hr[u] += q[0] * vr + q[1] * vi;
            hi[u] += q[0] * vi - q[1] * vr;
          }
        for (; mm < r1; ++mm) {
          const double* q = sq + (size_t)mm * RS + 2 * lane;
          const double vr = s_v[mm][0], vi = s_v[mm][1];
          hr[0] += q[0] * vr + q[1] * vi;
          hi[0] += q[0] * vi - q[1] * vr;
        }
        s_hp[wave][lane][0] = (hr[0] + hr[1]) + (hr[2] + hr[3]);
        s_hp[wave][lane][1] = (hi[0] + hi[1]) + (hi[2] + hi[3]);
      }
      __syncthreads();
      if (m < j) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < QW; ++q) {
          if (64 * q < M) {
            a += s_hp[q][m][0];
            b += s_hp[q][m][1];
          }
        }
        s_h[m][0] = a;
        s_h[m][1] = b;
      }
      __syncthreads();
      if (own)
        for (int k = 0; k < j; ++k)
          v = cfms(v, cmk(s_h[k][0], s_h[k][1]), cmk(row[2 * k], row[2 * k + 1]));
    }
    double n2 = cabs2(v), dummy = 0.0;
    block_sum2(n2, dummy);
    const double nrm = sqrt(n2);
    shift += log(nrm);
    if (own) {
      row[2 * j] = v.re / nrm;
      row[2 * j + 1] = v.im / nrm;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < M * N * 2; q += QRG_T) base[q] = sq[(q / (2 * N)) * RS + q % (2 * N)];
  if (m == 0) logshift[(size_t)w * 2 + sp] = shift;
}

__global__ void k_apply_shift(int nw, int P, const double* __restrict__ logshift,
                              double* __restrict__ logov) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw * P) return;
  const int w = i / P;
  logov[(size_t)i * 2] -= logshift[(size_t)w * 2] + logshift[(size_t)w * 2 + 1];
}

}  // namespace

namespace {

template <int QW>
hipError_t launch_qr_gw(const afqmc_ctx_s* c, int nw, double* phi, double* shift) {
  const size_t lds = (size_t)c->M * (2 * c->N + 2) * sizeof(double);
  auto kern = k_qr_g<QW>;
  hipError_t e =
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(nw, 2), dim3(64 * QW), lds, c->stream, nw, c->P, c->M, c->N, phi,
                     shift);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_qr_g(const afqmc_ctx_s* c, int nw, double* phi, double* logov, double* shift) {
  if (nw <= 0) return hipSuccess;
  if (c->M > 192) return hipErrorInvalidValue;
  hipError_t e = c->M <= 128 ? launch_qr_gw<2>(c, nw, phi, shift) : launch_qr_gw<3>(c, nw, phi, shift);
  if (e != hipSuccess) return e;
  if (logov != nullptr) {
    const int n = nw * c->P;
    hipLaunchKernelGGL(k_apply_shift, dim3((n + 255) / 256), dim3(256), 0, c->stream, nw, c->P,
                       shift, logov);
  }
  return hipGetLastError();
}
