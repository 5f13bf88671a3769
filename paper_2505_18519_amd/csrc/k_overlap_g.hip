// Overlap, log-determinant and Green's function for larger systems (N <= 32,
// M <= 128); same quantities and conventions as k_overlap (Sec. III.A, Eqs.
// ratio-update-phi and sign-path).  One workgroup of two wavefronts per path,
// wavefront s handling spin s:
//  1. A^s = Phi_T^T phi^s on the FP64 matrix cores (NTC x NTC tiles of 16);
//  2. LU with partial pivoting, one lane per row (N <= 32 lanes), pivot rows
//     found by a max reduction over the 64 lanes and broadcast by shuffles;
//  3. optionally Theta^s = phi^s (A^s)^{-1}, lanes over orbital rows m, and
//     the Green's function diagonal Re (G_up + G_dn)_mm.
// The two spins' log-determinants and diagonals are added through LDS.
// CT: complex trial determinants (multi-slice trials), A^s = Phi_T^T phi^s
// with both factors complex (no conjugation: the bilinear overlap of Eq.
// ratio-update-phi); the Green's-function diagonal is then not formed.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

template <int NTC, bool CT>
__global__ void __launch_bounds__(128)
k_overlap_g(int n_samples, int P, int M, int N, const double* __restrict__ phi,
            const double* __restrict__ phiT, double* __restrict__ logov, double* __restrict__ theta,
            double* __restrict__ gdiag) {
  constexpr int NT = 16 * NTC;
  __shared__ double s_lu[2][NT][NT + 1][2];
  __shared__ int s_perm[2][NT];
  __shared__ double s_res[2][3];
  __shared__ double s_gd[128];  // M <= 128

  const int s = blockIdx.x;
  const int sp = threadIdx.x >> 6;  // spin of this wavefront
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  if (s >= n_samples) return;  // whole block
  const int w = s / P;
  const double* pT = phiT + (size_t)s * M * N * (CT ? 2 : 1);
  const double* pw = phi + ((size_t)w * 2 + sp) * M * N * 2;

  // 1. A^sp tiles (it, jt): A[i][j] = sum_m Phi_T[m][i] phi[m][j]
  dx4 acc[NTC][NTC][2];
#pragma unroll
  for (int it = 0; it < NTC; ++it)
#pragma unroll
    for (int jt = 0; jt < NTC; ++jt) acc[it][jt][0] = acc[it][jt][1] = dx4_zero();
  for (int q = 0; q < (M + 3) / 4; ++q) {
    const int m = 4 * q + g;
    const bool okm = m < M;
    double a[NTC], ai[NTC], br[NTC], bi[NTC];
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int n = 16 * t + c;
      const bool ok = okm && n < N;
      if (CT) {
        a[t] = ok ? pT[((size_t)m * N + n) * 2] : 0.0;
        ai[t] = ok ? pT[((size_t)m * N + n) * 2 + 1] : 0.0;
      } else {
        a[t] = ok ? pT[m * N + n] : 0.0;
        ai[t] = 0.0;
      }
      br[t] = ok ? pw[((size_t)m * N + n) * 2] : 0.0;
      bi[t] = ok ? pw[((size_t)m * N + n) * 2 + 1] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < NTC; ++it)
#pragma unroll
      for (int jt = 0; jt < NTC; ++jt) {
        acc[it][jt][0] = mfma_f64(a[it], br[jt], acc[it][jt][0]);
        acc[it][jt][1] = mfma_f64(a[it], bi[jt], acc[it][jt][1]);
        if (CT) {
          acc[it][jt][0] = mfma_f64(-ai[it], bi[jt], acc[it][jt][0]);
          acc[it][jt][1] = mfma_f64(ai[it], br[jt], acc[it][jt][1]);
        }
      }
  }
#pragma unroll
  for (int it = 0; it < NTC; ++it)
#pragma unroll
    for (int jt = 0; jt < NTC; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        s_lu[sp][16 * it + g + 4 * r][16 * jt + c][0] = acc[it][jt][0][r];
        s_lu[sp][16 * it + g + 4 * r][16 * jt + c][1] = acc[it][jt][1][r];
      }
  __syncthreads();

  // 2. LU, lane i = row i (i < N)
  const int i = lane;
  cplx a[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j)
    a[j] = (i < NT) ? cmk(s_lu[sp][i][j][0], s_lu[sp][i][j][1]) : cmk(0.0, 0.0);
  __syncthreads();
  bool used = i >= N;
  int mystep = -1;
  int perm[NT];
  cplx pprod = cmk(1.0, 0.0);
  int pexp = 0;
  bool singular = false;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    perm[k] = 0;
    if (k < N) {
      double v = used ? -1.0 : cabs2(a[k]);
      if (!used && !(v >= 0.0)) v = 0.0;
      int idx = used ? 1000 : i;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double v2 = __shfl_xor(v, o, 64);
        const int i2 = __shfl_xor(idx, o, 64);
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      }
      const int prow = idx;
      perm[k] = prow;
      const int src = prow & 63;
      const cplx piv = cmk(__shfl(a[k].re, src, 64), __shfl(a[k].im, src, 64));
      if (!(v > 0.0)) singular = true;
      if (i == prow && !used) {
        used = true;
        mystep = k;
      }
      pprod = cmul(pprod, piv);
      const double mx = fmax(fabs(pprod.re), fabs(pprod.im));
      if (mx > 0.0 && isfinite(mx)) {
        const int ex = ilogb(mx);
        pprod = cscale(pprod, ldexp(1.0, -ex));
        pexp += ex;
      }
      cplx l = cmk(0.0, 0.0);
      if (!used && !singular) {
        l = cdiv(a[k], piv);
        a[k] = l;
      }
#pragma unroll
      for (int j = k + 1; j < NT; ++j) {
        const cplx pj = cmk(__shfl(a[j].re, src, 64), __shfl(a[j].im, src, 64));
        if (!used && !singular) a[j] = cfms(a[j], l, pj);
      }
    }
  }
  int inv = 0;
#pragma unroll
  for (int x = 0; x < NT; ++x)
#pragma unroll
    for (int y = x + 1; y < NT; ++y)
      if (y < N && perm[x] > perm[y]) ++inv;
  if (lane == 0) {
    s_res[sp][0] = 0.5 * log(cabs2(pprod)) + (double)pexp * M_LN2;
    s_res[sp][1] = atan2(pprod.im, pprod.re) + ((inv & 1) ? M_PI : 0.0);
    s_res[sp][2] = singular ? 1.0 : 0.0;
  }
  // LU rows in step order, permutation
  if (i < N && mystep >= 0) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      s_lu[sp][mystep][j][0] = a[j].re;
      s_lu[sp][mystep][j][1] = a[j].im;
    }
    s_perm[sp][mystep] = i;
  }
  __syncthreads();
  const bool sing_any = s_res[0][2] != 0.0 || s_res[1][2] != 0.0;
  if (threadIdx.x == 0) {
    double* o = logov + (size_t)s * 2;
    o[0] = sing_any ? neg_inf() : s_res[0][0] + s_res[1][0];
    o[1] = sing_any ? 0.0 : s_res[0][1] + s_res[1][1];
  }
  if (theta == nullptr && gdiag == nullptr) return;
  double* th = theta ? theta + ((size_t)s * 2 + sp) * M * N * 2 : nullptr;
  double* gd = gdiag ? gdiag + (size_t)s * M : nullptr;
  if (sing_any) {
    if (th)
      for (int q = lane; q < M * N * 2; q += 64) th[q] = 0.0;
    if (gd && sp == 0)
      for (int q = lane; q < M; q += 64) gd[q] = 0.0;
    return;
  }
  // 3. Theta rows (every lane reaches the barriers; lanes past M idle)
  for (int m0 = 0; m0 < M; m0 += 64) {
    const int m = m0 + lane;
    double gsum = 0.0;
    if (m < M) {
      cplx x[NT];
      const double* src = pw + (size_t)m * N * 2;
#pragma unroll
      for (int j = 0; j < NT; ++j) x[j] = (j < N) ? cmk(src[2 * j], src[2 * j + 1]) : cmk(0, 0);
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        if (j < N) {
          cplx acc2 = x[j];
#pragma unroll
          for (int k = 0; k < j; ++k)
            acc2 = cfms(acc2, x[k], cmk(s_lu[sp][k][j][0], s_lu[sp][k][j][1]));
          x[j] = cdiv(acc2, cmk(s_lu[sp][j][j][0], s_lu[sp][j][j][1]));
        }
      }
#pragma unroll
      for (int j = NT - 1; j >= 0; --j) {
        if (j < N) {
          cplx acc2 = x[j];
#pragma unroll
          for (int k = j + 1; k < NT; ++k)
            if (k < N) acc2 = cfms(acc2, x[k], cmk(s_lu[sp][k][j][0], s_lu[sp][k][j][1]));
          x[j] = acc2;
        }
      }
      double* dst = th ? th + (size_t)m * N * 2 : nullptr;
#pragma unroll
      for (int k = 0; k < NT; ++k)
        if (k < N) {
          const int col = min(max(s_perm[sp][k], 0), N - 1);
          if (dst) {
            dst[2 * col] = x[k].re;
            dst[2 * col + 1] = x[k].im;
          }
          if (!CT) gsum = fma(x[k].re, pT[m * N + col], gsum);
        }
      if (sp == 1) s_gd[m] = gsum;
    }
    if (gd == nullptr) continue;  // block-uniform
    __syncthreads();
    if (sp == 0 && m < M) gd[m] = gsum + s_gd[m];
    __syncthreads();
  }
}

template <int NTC>
hipError_t launch_g(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                    double* logov, double* theta, double* gdiag) {
  const int n = nw * c->P;
  if (c->ctrial) {
    if (gdiag != nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_overlap_g<NTC, true>), dim3(n), dim3(128), 0, c->stream, n, c->P, c->M,
                       c->N, phi, phiT, logov, theta, gdiag);
  } else {
    hipLaunchKernelGGL((k_overlap_g<NTC, false>), dim3(n), dim3(128), 0, c->stream, n, c->P, c->M,
                       c->N, phi, phiT, logov, theta, gdiag);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_overlap_g(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                            double* logov, double* theta, double* gdiag) {
  if (nw <= 0) return hipSuccess;
  switch ((c->N + 15) / 16) {
    case 1: return launch_g<1>(c, nw, phi, phiT, logov, theta, gdiag);
    case 2: return launch_g<2>(c, nw, phi, phiT, logov, theta, gdiag);
    default: return hipErrorInvalidValue;
  }
}
