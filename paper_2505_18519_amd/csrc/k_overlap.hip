// Overlap, log-determinant and Green's function of every (walker, path) pair
// (Sec. III.A, Eqs. ratio-update-phi and sign-path; Theta feeds Eq. local-obs).
//
// One wavefront per path handles both spins:
//  1. A^s = Phi_T^T phi^s (N x N complex) on the FP64 matrix cores, operands
//     read straight from HBM (real trial times the re / im parts of phi);
//  2. LU with partial pivoting, one lane per row (lanes 0-15 spin up, 16-31
//     spin down), pivot rows found by a 16-lane max reduction over DPP moves
//     (largest |a|^2, lowest row on ties) and broadcast by lane shuffles
//     instead of swapped;
//     det = parity(perm) prod u_kk, accumulated as a scaled complex product;
//  3. optionally Theta^s = phi^s (A^s)^{-1}: lanes (spin, j) solve the unit rows
//     e_j X^s = e_j (A^s)^{-1} with the factors (z U = e_j, v L = z,
//     X[j][perm[k]] = v[k]), X^s replaces the factors in LDS, and
//     Theta^s = phi^s X^s runs on the matrix cores (four real products per
//     spin), stored as whole 16-byte complex entries along each row;
//     with the Green's function diagonal Re (G_up + G_dn)_mm =
//     Re sum_s sum_n Theta^s_mn Phi_T,mn requested, one lane per orbital row m
//     solves x (A^s)^{-1} for its row of phi instead.
// A zero pivot marks the path singular: l = -inf + 0i and Theta = 0, diag = 0.
// A non-finite overlap entry gives l = NaN + NaN i (Theta and diag 0).
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

constexpr int OV_WAVES = 4;
constexpr int NT = 16;  // N <= 16

template <int MT>
__global__ void __launch_bounds__(OV_WAVES * 64) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_overlap(int n_samples, int P, int M, int N, const double* __restrict__ phi,
          const double* __restrict__ phiT, double* __restrict__ logov, double* __restrict__ theta,
          double* __restrict__ gdiag) {
  __shared__ double s_lu[OV_WAVES][2][NT][NT][2];  // LU rows in pivot order
  __shared__ int s_perm[OV_WAVES][2][NT];

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int s = blockIdx.x * OV_WAVES + wave;
  if (s >= n_samples) return;  // no block-level barriers below
  const int w = s / P;
  const double* pT = phiT + (size_t)s * M * N;
  const double* pw = phi + (size_t)w * 2 * M * N * 2;

  // 1. A^s via MFMA: tiles (re up, im up, re dn, im dn); lane holds A[g+4r][c]
  dx4 acc[4] = {dx4_zero(), dx4_zero(), dx4_zero(), dx4_zero()};
#pragma unroll 4
  for (int q = 0; q < MT / 4; ++q) {
    const int m = 4 * q + g;
    const bool okm = m < M, okc = c < N;
    const double a = (okm && okc) ? pT[m * N + c] : 0.0;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      double br = 0.0, bi = 0.0;
      if (okm && okc) {
        const double* src = pw + ((size_t)(sp * M + m) * N + c) * 2;
        br = src[0];
        bi = src[1];
      }
      acc[2 * sp] = mfma_f64(a, br, acc[2 * sp]);
      acc[2 * sp + 1] = mfma_f64(a, bi, acc[2 * sp + 1]);
    }
  }
  // stage A rows through LDS (reuse the LU buffer as the A buffer)
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      s_lu[wave][sp][g + 4 * r][c][0] = acc[2 * sp][r];
      s_lu[wave][sp][g + 4 * r][c][1] = acc[2 * sp + 1][r];
    }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  // 2. LU: lane = (sp, i) for lanes < 32
  const int sp = (lane >> 4) & 1;
  const int i = c;
  cplx a[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) a[j] = cmk(s_lu[wave][sp][i][j][0], s_lu[wave][sp][i][j][1]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  bool used = (i >= N) || (lane >= 32);
  // a non-finite entry of either spin's overlap matrix makes l NaN (a
  // numerical event, not a singular path)
  bool nonfinite = false;
  if (!used) {
#pragma unroll
    for (int k = 0; k < NT; ++k)
      if (k < N) nonfinite |= !(isfinite(a[k].re) && isfinite(a[k].im));
  }
  const bool nf_any = __ballot(nonfinite) != 0;
  int mystep = -1;
  int perm[NT];
  // det = prod of pivots, kept as a complex mantissa times 2^pexp so that it
  // neither overflows nor needs a logarithm per step
  cplx pprod = cmk(1.0, 0.0);
  int pexp = 0;
  bool singular = false;
  const int base = lane & ~15;  // first lane of my 16-lane group
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    if (k < N) {
      // pivot: max |a_ik|^2 over unused rows, lowest i on ties
      // NaN entries count as zero so that the reduction order is total and
      // every lane of the group agrees on the pivot
      double v = used ? -1.0 : cabs2(a[k]);
      if (!used && !(v >= 0.0)) v = 0.0;
      int idx = used ? 1000 : i;
      // across the 16-lane row with DPP moves (VALU latency, no LDS round trip):
      // partner lane xor 1, xor 2, then the mirrored quad, then the mirrored half
      auto take = [&](double v2, int i2) {
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      };
      take(dpp_f64<0xB1>(v), dpp_i32<0xB1>(idx));
      take(dpp_f64<0x4E>(v), dpp_i32<0x4E>(idx));
      take(dpp_f64<0x141>(v), dpp_i32<0x141>(idx));
      take(dpp_f64<0x140>(v), dpp_i32<0x140>(idx));
      const int prow = idx;  // uniform within the group
      perm[k] = prow;
      const int src = base + (prow & 15);
      const cplx piv = cmk(__shfl(a[k].re, src, 64), __shfl(a[k].im, src, 64));
      if (!(v > 0.0)) singular = true;
      if (i == prow && !used) {
        used = true;
        mystep = k;
      }
      pprod = cmul(pprod, piv);
      {
        const double mx = fmax(fabs(pprod.re), fabs(pprod.im));
        if (mx > 0.0 && isfinite(mx)) {
          const int ex = ilogb(mx);
          pprod = cscale(pprod, ldexp(1.0, -ex));
          pexp += ex;
        }
      }
      cplx l = cmk(0.0, 0.0);
      if (!used && !singular) {
        l = cmul(a[k], crecip(piv));  // the pivot's reciprocal: one real division
        a[k] = l;
      }
#pragma unroll
      for (int j = k + 1; j < NT; ++j) {
        const cplx pj = cmk(__shfl(a[j].re, src, 64), __shfl(a[j].im, src, 64));
        if (!used && !singular) a[j] = cfms(a[j], l, pj);
      }
    }
  }
  // parity of the step -> row permutation (uniform per group)
  int inv = 0;
#pragma unroll
  for (int x = 0; x < NT; ++x)
#pragma unroll
    for (int y = x + 1; y < NT; ++y)
      if (y < N && perm[x] > perm[y]) ++inv;
  double logabs = 0.5 * log(cabs2(pprod)) + (double)pexp * M_LN2;
  double argsum = atan2(pprod.im, pprod.re) + ((inv & 1) ? M_PI : 0.0);

  // both spins' results to lane 0 of the wave
  const double la_dn = __shfl(logabs, 16, 64), ar_dn = __shfl(argsum, 16, 64);
  const int sing_dn = __shfl((int)singular, 16, 64);
  const int sing_up = __shfl((int)singular, 0, 64);
  const bool sing_any = sing_up || sing_dn;
  if (lane == 0) {
    double* o = logov + (size_t)s * 2;
    if (nf_any) {
      o[0] = __builtin_nan("");
      o[1] = __builtin_nan("");
    } else if (sing_any) {
      o[0] = neg_inf();
      o[1] = 0.0;
    } else {
      o[0] = logabs + la_dn;
      o[1] = argsum + ar_dn;
    }
  }
  if (theta == nullptr && gdiag == nullptr) return;

  double* th = theta ? theta + (size_t)s * 2 * M * N * 2 : nullptr;
  double* gd = gdiag ? gdiag + (size_t)s * M : nullptr;
  if (sing_any || nf_any) {
    if (th)
      for (int q = lane; q < 2 * M * N * 2; q += 64) th[q] = 0.0;
    if (gd)
      for (int q = lane; q < M; q += 64) gd[q] = 0.0;
    return;
  }
  // LU rows in step order, and the permutation, to LDS
  if (lane < 32 && i < N && mystep >= 0) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      s_lu[wave][sp][mystep][j][0] = a[j].re;
      s_lu[wave][sp][mystep][j][1] = a[j].im;
    }
  }
  if (lane < 32 && i < N && mystep >= 0) s_perm[wave][sp][mystep] = i;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

  if (gdiag == nullptr) {
    // 3. X^s = (A^s)^{-1}: lane (spin, j) < 32 solves e_j X = e_j A^{-1} with the
    //    factors (z U = e_j, v L = z, X[j][perm[k]] = v[k]); rows j >= N stay zero
    const int jr = c, spn = (lane >> 4) & 1;
    const bool solver = lane < 32 && jr < N;
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
            acc2 = cfms(acc2, x[k], cmk(s_lu[wave][spn][k][j][0], s_lu[wave][spn][k][j][1]));
          x[j] = cdiv(acc2, cmk(s_lu[wave][spn][j][j][0], s_lu[wave][spn][j][j][1]));
        }
      }
#pragma unroll
      for (int j = NT - 1; j >= 0; --j) {
        if (j < N) {
          cplx acc2 = x[j];
#pragma unroll
          for (int k = j + 1; k < NT; ++k)
            if (k < N)
              acc2 = cfms(acc2, x[k], cmk(s_lu[wave][spn][k][j][0], s_lu[wave][spn][k][j][1]));
          x[j] = acc2;
        }
      }
    }
    int pcol[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) pcol[k] = min(max(s_perm[wave][spn][k], 0), NT - 1);
    // every lane of the wave has issued its factor reads: X replaces the factors in LDS
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < 32) {
#pragma unroll
      for (int k = 0; k < NT; ++k) {  // unused columns first, then the solved row
        s_lu[wave][spn][jr][k][0] = 0.0;
        s_lu[wave][spn][jr][k][1] = 0.0;
      }
      if (solver) {
#pragma unroll
        for (int k = 0; k < NT; ++k)
          if (k < N) {
            s_lu[wave][spn][jr][pcol[k]][0] = x[k].re;
            s_lu[wave][spn][jr][pcol[k]][1] = x[k].im;
          }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // 4. Theta^s = phi^s X^s on the matrix cores: A[c][g] = phi[16t + c][4q + g],
    //    B[g][c] = X[4q + g][c]; the lane holds Theta[16t + g + 4r][c]
#pragma unroll
    for (int spin = 0; spin < 2; ++spin) {
      double xr[4], xi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        xr[q] = s_lu[wave][spin][4 * q + g][c][0];
        xi[q] = s_lu[wave][spin][4 * q + g][c][1];
      }
#pragma unroll
      for (int t = 0; t < MT / 16; ++t) {
        dx4 tr = dx4_zero(), ti = dx4_zero();
        const int m = 16 * t + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int n = 4 * q + g;
          double2 v = make_double2(0.0, 0.0);
          if (m < M && n < N)
            v = *reinterpret_cast<const double2*>(pw + ((size_t)(spin * M + m) * N + n) * 2);
          tr = mfma_f64(v.x, xr[q], tr);
          tr = mfma_f64(-v.y, xi[q], tr);
          ti = mfma_f64(v.x, xi[q], ti);
          ti = mfma_f64(v.y, xr[q], ti);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mo = 16 * t + g + 4 * r;
          if (mo < M && c < N)
            *reinterpret_cast<double2*>(th + ((size_t)(spin * M + mo) * N + c) * 2) =
                make_double2(tr[r], ti[r]);
        }
      }
    }
    return;
  }

  // 3. Theta rows with the Green's function diagonal: lane = orbital row m
  for (int m0 = 0; m0 < M; m0 += 64) {
    double gsum = 0.0;
    for (int spin = 0; spin < 2; ++spin) {
      const int m = m0 + lane;
      if (m < M) {
        cplx x[NT];
        const double* src = pw + ((size_t)(spin * M + m) * N) * 2;
#pragma unroll
        for (int j = 0; j < NT; ++j) x[j] = (j < N) ? cmk(src[2 * j], src[2 * j + 1]) : cmk(0, 0);
        // z U = x  (forward in j)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          if (j < N) {
            cplx acc2 = x[j];
#pragma unroll
            for (int k = 0; k < j; ++k)
              acc2 = cfms(acc2, x[k], cmk(s_lu[wave][spin][k][j][0], s_lu[wave][spin][k][j][1]));
            x[j] = cdiv(acc2, cmk(s_lu[wave][spin][j][j][0], s_lu[wave][spin][j][j][1]));
          }
        }
        // v L = z  (backward in j, unit lower L_kj stored at row k, col j < k)
#pragma unroll
        for (int j = NT - 1; j >= 0; --j) {
          if (j < N) {
            cplx acc2 = x[j];
#pragma unroll
            for (int k = j + 1; k < NT; ++k)
              if (k < N)
                acc2 = cfms(acc2, x[k], cmk(s_lu[wave][spin][k][j][0], s_lu[wave][spin][k][j][1]));
            x[j] = acc2;
          }
        }
        double* dst = th ? th + ((size_t)(spin * M + m) * N) * 2 : nullptr;
#pragma unroll
        for (int k = 0; k < NT; ++k)
          if (k < N) {
            const int col = min(max(s_perm[wave][spin][k], 0), N - 1);
            if (dst) {
              dst[2 * col] = x[k].re;
              dst[2 * col + 1] = x[k].im;
            }
            gsum = fma(x[k].re, pT[m * N + col], gsum);
          }
      }
    }
    if (gd && m0 + lane < M) gd[m0 + lane] = gsum;
  }
}

template <int MT>
hipError_t launch_mt(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                     double* logov, double* theta, double* gdiag) {
  const int n = nw * c->P;
  dim3 grid((n + OV_WAVES - 1) / OV_WAVES), block(OV_WAVES * 64);
  hipLaunchKernelGGL(k_overlap<MT>, grid, block, 0, c->stream, n, c->P, c->M, c->N, phi, phiT,
                     logov, theta, gdiag);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_overlap(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                          double* logov, double* theta, double* gdiag) {
  if (nw <= 0) return hipSuccess;
  switch (c->MT) {
    case 16: return launch_mt<16>(c, nw, phi, phiT, logov, theta, gdiag);
    case 32: return launch_mt<32>(c, nw, phi, phiT, logov, theta, gdiag);
    case 48: return launch_mt<48>(c, nw, phi, phiT, logov, theta, gdiag);
    case 64: return launch_mt<64>(c, nw, phi, phiT, logov, theta, gdiag);
    default: return hipErrorInvalidValue;
  }
}
