// Overlap, log-determinant and Green's function for larger systems (N <= 40,
// M <= 160); same quantities and conventions as k_overlap (Sec. III.A, Eqs.
// ratio-update-phi and sign-path).  One workgroup of two wavefronts per path,
// wavefront s handling spin s:
//  1. A^s = Phi_T^T phi^s on the FP64 matrix cores (NTC x NTC tiles of 16),
//     operand loads clamped and bit-masked so that four k steps are in flight;
//  2. LU with partial pivoting, one lane per row (N <= 40 lanes): the pivot
//     (largest |a|^2, lowest row on ties) by DPP moves within each 16-lane
//     row and a comparison of the rows' results, the pivot row broadcast by
//     readlane (the pivot is uniform over the wavefront);
//  3. optionally Theta^s = phi^s (A^s)^{-1}: lanes j < N solve the unit rows
//     e_j X^s = e_j (A^s)^{-1} with the factors, X^s replaces the factors in
//     LDS, and Theta^s = phi^s X^s runs on the matrix cores (four real products
//     per tile), stored as whole 16-byte complex entries along each row; with
//     the Green's function diagonal Re (G_up + G_dn)_mm requested, lanes over
//     orbital rows m solve x (A^s)^{-1} for their rows of phi instead.
// The two spins' log-determinants and diagonals are added through LDS.  A
// zero pivot gives l = -inf + 0i, a non-finite overlap entry l = NaN + NaN i
// (Theta and the diagonal 0 in both cases).
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
  __shared__ double s_gd[160];  // M <= 160

  // workgroup b takes walker 8 (b / 8P) + b % 8 and its path (b / 8) % P: the
  // P paths of a walker, which read the same phi, run 8 launches apart on one
  // XCD (workgroups go round-robin over the 8) and share that XCD's L2
  const int s = (8 * ((int)blockIdx.x / (8 * P)) + ((int)blockIdx.x & 7)) * P +
                ((int)blockIdx.x >> 3) % P;
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
#pragma unroll 4
  for (int q = 0; q < (M + 3) / 4; ++q) {
    const int m = 4 * q + g;
    const bool okm = m < M;
    const int mc = min(m, M - 1);
    double a[NTC], ai[NTC], br[NTC], bi[NTC];
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
      const int n = 16 * t + c;
      const bool ok = okm && n < N;
      const size_t e = (size_t)mc * N + min(n, N - 1);
      if (CT) {
        const double2 v = *reinterpret_cast<const double2*>(pT + e * 2);
        a[t] = keep_if(v.x, ok);
        ai[t] = keep_if(v.y, ok);
      } else {
        a[t] = keep_if(pT[e], ok);
        ai[t] = 0.0;
      }
      const double2 x = *reinterpret_cast<const double2*>(pw + e * 2);
      br[t] = keep_if(x.x, ok);
      bi[t] = keep_if(x.y, ok);
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
  // a non-finite entry of either spin's overlap matrix makes l NaN (a
  // numerical event, not a singular path)
  bool nonfinite = false;
  if (!used) {
#pragma unroll
    for (int j = 0; j < NT; ++j)
      if (j < N) nonfinite |= !(isfinite(a[j].re) && isfinite(a[j].im));
  }
  nonfinite = __ballot(nonfinite) != 0;
  int mystep = -1;
  int perm[NT];
  cplx pprod = cmk(1.0, 0.0);
  int pexp = 0;
  bool singular = false;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    perm[k] = 0;
    if (k < N) {
      // NaN entries count as zero so that the order is total and every lane
      // agrees on the pivot
      double v = used ? -1.0 : cabs2(a[k]);
      if (!used && !(v >= 0.0)) v = 0.0;
      int idx = used ? 1000 : i;
      auto take = [&](double v2, int i2) {
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      };
      // within each 16-lane row: lane xor 1, xor 2, mirrored quad, mirrored half
      take(dpp_f64<0xB1>(v), dpp_i32<0xB1>(idx));
      take(dpp_f64<0x4E>(v), dpp_i32<0x4E>(idx));
      take(dpp_f64<0x141>(v), dpp_i32<0x141>(idx));
      take(dpp_f64<0x140>(v), dpp_i32<0x140>(idx));
      // rows 0 .. NTC-1 hold the N <= 16 NTC matrix rows; the lanes past 16 NTC
      // are all used
      const double v16 = readlane_f64(v, 16);
      const int i16 = __builtin_amdgcn_readlane(idx, 16);
      const double v32 = NTC > 2 ? readlane_f64(v, 32) : -1.0;
      const int i32 = NTC > 2 ? __builtin_amdgcn_readlane(idx, 32) : 1000;
      v = readlane_f64(v, 0);
      idx = __builtin_amdgcn_readlane(idx, 0);
      take(v16, i16);
      if (NTC > 2) take(v32, i32);
      const int prow = idx;  // uniform over the wavefront
      perm[k] = prow;
      const cplx piv = cmk(readlane_f64(a[k].re, prow), readlane_f64(a[k].im, prow));
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
        l = cmul(a[k], crecip(piv));  // the pivot's reciprocal: one real division
        a[k] = l;
      }
#pragma unroll
      for (int j = k + 1; j < NT; ++j) {
        const cplx pj = cmk(readlane_f64(a[j].re, prow), readlane_f64(a[j].im, prow));
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
    s_res[sp][2] = nonfinite ? 2.0 : singular ? 1.0 : 0.0;
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
  const bool nf_any = s_res[0][2] == 2.0 || s_res[1][2] == 2.0;
  if (threadIdx.x == 0) {
    double* o = logov + (size_t)s * 2;
    const double nan = __builtin_nan("");
    o[0] = nf_any ? nan : sing_any ? neg_inf() : s_res[0][0] + s_res[1][0];
    o[1] = nf_any ? nan : sing_any ? 0.0 : s_res[0][1] + s_res[1][1];
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
  if (gdiag == nullptr) {
    // 3. X = (A^sp)^{-1}: lane j < N solves e_j X = e_j A^{-1} with the factors
    //    (z U = e_j, v L = z, X[j][perm[k]] = v[k]); rows j >= N stay zero
    const int jr = lane;
    const bool solver = jr < N;
    cplx x[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) x[j] = cmk(j == jr ? 1.0 : 0.0, 0.0);
    if (solver) {
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
    }
    int pcol[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) pcol[k] = min(max(s_perm[sp][k], 0), NT - 1);
    // every lane of the wavefront has issued its factor reads: X replaces them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < NT) {
#pragma unroll
      for (int k = 0; k < NT; ++k) {  // unused columns first, then the solved row
        s_lu[sp][jr][k][0] = 0.0;
        s_lu[sp][jr][k][1] = 0.0;
      }
      if (solver) {
#pragma unroll
        for (int k = 0; k < NT; ++k)
          if (k < N) {
            s_lu[sp][jr][pcol[k]][0] = x[k].re;
            s_lu[sp][jr][pcol[k]][1] = x[k].im;
          }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // 4. Theta^sp = phi^sp X on the matrix cores: A[c][g] = phi[16t + c][4q + g],
    //    B[g][c] = X[4q + g][16ct + c]; the lane holds Theta[16t + g + 4r][16ct + c]
    double xr[NT / 4][NTC], xi[NT / 4][NTC];
#pragma unroll
    for (int q = 0; q < NT / 4; ++q)
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) {
        xr[q][ct] = s_lu[sp][4 * q + g][16 * ct + c][0];
        xi[q][ct] = s_lu[sp][4 * q + g][16 * ct + c][1];
      }
    for (int t = 0; t < (M + 15) / 16; ++t) {
      const int m = 16 * t + c;
      const int mc = min(m, M - 1);
      double2 v[NT / 4];
#pragma unroll
      for (int q = 0; q < NT / 4; ++q) {
        const int n = 4 * q + g;
        const double2 e =
            *reinterpret_cast<const double2*>(pw + ((size_t)mc * N + min(n, N - 1)) * 2);
        const bool ok = m < M && n < N;
        v[q] = make_double2(keep_if(e.x, ok), keep_if(e.y, ok));
      }
      dx4 tr[NTC], ti[NTC];
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) tr[ct] = ti[ct] = dx4_zero();
#pragma unroll
      for (int q = 0; q < NT / 4; ++q)
#pragma unroll
        for (int ct = 0; ct < NTC; ++ct) {
          tr[ct] = mfma_f64(v[q].x, xr[q][ct], tr[ct]);
          tr[ct] = mfma_f64(-v[q].y, xi[q][ct], tr[ct]);
          ti[ct] = mfma_f64(v[q].x, xi[q][ct], ti[ct]);
          ti[ct] = mfma_f64(v[q].y, xr[q][ct], ti[ct]);
        }
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mo = 16 * t + g + 4 * r, col = 16 * ct + c;
          if (mo < M && col < N)
            *reinterpret_cast<double2*>(th + ((size_t)mo * N + col) * 2) =
                make_double2(tr[ct][r], ti[ct][r]);
        }
    }
    return;
  }
  // 3. Theta rows with the diagonal (every lane reaches the barriers; lanes past M idle)
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
  const dim3 grid(8 * c->P * ((nw + 7) / 8));  // walkers padded to 8 (see the kernel)
  if (c->ctrial) {
    if (gdiag != nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_overlap_g<NTC, true>), grid, dim3(128), 0, c->stream, n, c->P, c->M,
                       c->N, phi, phiT, logov, theta, gdiag);
  } else {
    hipLaunchKernelGGL((k_overlap_g<NTC, false>), grid, dim3(128), 0, c->stream, n, c->P, c->M,
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
    case 3: return launch_g<3>(c, nw, phi, phiT, logov, theta, gdiag);
    default: return hipErrorInvalidValue;
  }
}
