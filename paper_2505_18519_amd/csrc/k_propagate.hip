// Walker propagation and hybrid phaseless weight (Sec. II.A, Eq. HS; Sec. II.B,
// Eqs. walker_prop, importance_function, importance_function_CP; Sec. III.A,
// Eq. ratio-update-phi for the overlap ratio; App. B step 1).
//
//   V = i sqrt(tau) sum_g (xi_g - xbar_g) L_g                      (k_vbuild)
//   phi' = e^{-tau h1/2} T_n(V) e^{-tau h1/2} phi, T_n = sum_{j<=n} V^j/j!
//                                                                  (k_taylor)
//   l'_p at the unchanged paths (overlap kernel), then per walker
//   num_r = sum_p exp(l'_p - Re l_p), r = num_r / sum_p S_p,
//   W <- W |exp(sum_g xi_g xbar_g - xbar_g^2 / 2) r| e^{tau E_T} max(0, cos arg r)
//                                                                  (k_weight)
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

// ---------------------------------------------------------------------------
// V build: with c = xi - xbar, R = sum_g Re(c_g) L_g and Q = sum_g Im(c_g) L_g,
// V = sqrt(tau) (-Q + i R).  A (walkers x G) by (G x M^2) product on the FP64
// matrix cores: each wavefront takes 16 walkers (both Re c and Im c as A
// operands) and 64 matrix entries; L is read once per 16 walkers.
__global__ void __launch_bounds__(256)
k_vbuild(int nw, int G, int MM, double sqrt_tau, const double* __restrict__ L,
         const double* __restrict__ xi, const double* __restrict__ xbar, double* __restrict__ vmat) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int w0 = (blockIdx.y * 4 + wave) * 16;
  const int e0 = blockIdx.x * 64;
  if (w0 >= nw) return;
  dx4 ar[4] = {dx4_zero(), dx4_zero(), dx4_zero(), dx4_zero()};
  dx4 ai[4] = {dx4_zero(), dx4_zero(), dx4_zero(), dx4_zero()};
  const int wa = w0 + c;
  for (int k0 = 0; k0 < G; k0 += 4) {
    const int k = k0 + g;
    double cr = 0.0, ci = 0.0;
    if (wa < nw && k < G) {
      cr = xi[(size_t)wa * G + k] - xbar[((size_t)wa * G + k) * 2];
      ci = -xbar[((size_t)wa * G + k) * 2 + 1];
    }
#pragma unroll
    for (int et = 0; et < 4; ++et) {
      const int e = e0 + 16 * et + c;
      const double b = (k < G && e < MM) ? L[(size_t)k * MM + e] : 0.0;
      ar[et] = mfma_f64(cr, b, ar[et]);
      ai[et] = mfma_f64(ci, b, ai[et]);
    }
  }
#pragma unroll
  for (int et = 0; et < 4; ++et)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int w = w0 + g + 4 * r, e = e0 + 16 * et + c;
      if (w < nw && e < MM) {
        double* o = vmat + ((size_t)w * MM + e) * 2;
        o[0] = -sqrt_tau * ai[et][r];
        o[1] = sqrt_tau * ar[et][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Taylor propagator.  One workgroup per walker, one wavefront per 16-row tile
// of the M x 2N complex block [phi_up phi_dn].  Each wavefront keeps its rows
// of V (and of e^{-tau h1/2}) in registers as FP64-MFMA A operands; the
// iterate Y is shared through a double-buffered LDS tile.  Horner form:
// Y = X; for j = n..1: Y = X + V Y / j.
template <int MT>
__global__ void __launch_bounds__(MT * 4)
k_taylor(int M, int N, int n_taylor, const double* __restrict__ vmat,
         const double* __restrict__ Eh, double* __restrict__ phi) {
  constexpr int NTILE = MT / 16;
  constexpr int NC = 32;  // 2 spins x 16 columns
  __shared__ double s_y[2][MT][NC][2];

  const int w = blockIdx.x;
  const int wave = threadIdx.x >> 6;  // my row tile
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const double* V = vmat + (size_t)w * M * M * 2;
  double* ph = phi + (size_t)w * 2 * M * N * 2;

  // A operands: rows 16 wave + c, columns 16t + 4r + g (V, E_h symmetric)
  double vr[NTILE][4], vi[NTILE][4], nvi[NTILE][4], eh[NTILE][4];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + 4 * r + g, col = 16 * wave + c;
      const bool ok = row < M && col < M;
      vr[t][r] = ok ? V[((size_t)row * M + col) * 2] : 0.0;
      vi[t][r] = ok ? V[((size_t)row * M + col) * 2 + 1] : 0.0;
      nvi[t][r] = -vi[t][r];
      eh[t][r] = ok ? Eh[row * M + col] : 0.0;
    }
  // phi -> LDS buffer 0 (columns: spin * 16 + n)
  for (int q = threadIdx.x; q < MT * NC; q += MT * 4) {
    const int m = q / NC, col = q % NC, sp = col >> 4, n = col & 15;
    double re = 0.0, im = 0.0;
    if (m < M && n < N) {
      const double* src = ph + ((size_t)(sp * M + m) * N + n) * 2;
      re = src[0];
      im = src[1];
    }
    s_y[0][m][col][0] = re;
    s_y[0][m][col][1] = im;
  }
  __syncthreads();

  // real-symmetric product with eh: out rows of this tile from buffer `src`
  auto apply_eh = [&](int src, dx4 (&o)[2][2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) o[ct][0] = o[ct][1] = dx4_zero();
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const double* yb = s_y[src][16 * t + 4 * r + g][16 * ct + c];
          o[ct][0] = mfma_f64(eh[t][r], yb[0], o[ct][0]);
          o[ct][1] = mfma_f64(eh[t][r], yb[1], o[ct][1]);
        }
  };
  auto store_rows = [&](int dst, const dx4 (&o)[2][2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        s_y[dst][16 * wave + 4 * r + g][16 * ct + c][0] = o[ct][0][r];
        s_y[dst][16 * wave + 4 * r + g][16 * ct + c][1] = o[ct][1][r];
      }
  };

  // X = E_h phi (kept in registers, rows of this tile) -> buffer 1
  dx4 x[2][2];
  apply_eh(0, x);
  store_rows(1, x);
  __syncthreads();
  int cur = 1;
  for (int j = n_taylor; j >= 1; --j) {
    dx4 acc[2][2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[ct][0] = acc[ct][1] = dx4_zero();
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const double* yb = s_y[cur][16 * t + 4 * r + g][16 * ct + c];
          const double yr = yb[0], yi = yb[1];
          acc[ct][0] = mfma_f64(vr[t][r], yr, acc[ct][0]);
          acc[ct][0] = mfma_f64(nvi[t][r], yi, acc[ct][0]);
          acc[ct][1] = mfma_f64(vr[t][r], yi, acc[ct][1]);
          acc[ct][1] = mfma_f64(vi[t][r], yr, acc[ct][1]);
        }
    const double invj = 1.0 / (double)j;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[ct][ri][r] = x[ct][ri][r] + acc[ct][ri][r] * invj;
    store_rows(cur ^ 1, acc);
    __syncthreads();
    cur ^= 1;
  }
  // phi' = E_h Y
  dx4 o[2][2];
  apply_eh(cur, o);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * wave + 4 * r + g;
      if (m < M && c < N) {
        double* d = ph + ((size_t)(ct * M + m) * N + c) * 2;
        d[0] = o[ct][0][r];
        d[1] = o[ct][1][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Hybrid weight with the phaseless cosine; one 64-lane workgroup per walker.
__global__ void __launch_bounds__(64)
k_weight(int nw, int P, int G, double dtau, double e_shift, int weight_mode,
         const double* __restrict__ xi, const double* __restrict__ xbar,
         const double* __restrict__ logov, const double* __restrict__ logov_new,
         double* __restrict__ w, double* __restrict__ ref) {
  const int wk = blockIdx.x;
  const int lane = threadIdx.x;
  // sum_g (xi_g xbar_g - xbar_g^2 / 2)
  double sr = 0.0, si = 0.0;
  for (int gm = lane; gm < G; gm += 64) {
    const double x = xi[(size_t)wk * G + gm];
    const double br = xbar[((size_t)wk * G + gm) * 2], bi = xbar[((size_t)wk * G + gm) * 2 + 1];
    sr += x * br - 0.5 * (br * br - bi * bi);
    si += x * bi - 0.5 * (2.0 * br * bi);
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  cplx num = cmk(0.0, 0.0), den = cmk(0.0, 0.0);
  for (int p = lane; p < P; p += 64) {
    const double* lo = logov + ((size_t)wk * P + p) * 2;
    const double* ln = logov_new + ((size_t)wk * P + p) * 2;
    if (!__builtin_isinf(lo[0])) {
      double s_, c_;
      sincos(lo[1], &s_, &c_);
      den = cadd(den, cmk(c_, s_));
      if (!__builtin_isinf(ln[0])) {
        const double mag = exp(ln[0] - lo[0]);
        sincos(ln[1], &s_, &c_);
        num = cadd(num, cmk(mag * c_, mag * s_));
      }
    }
  }
  num.re = wave_sum(num.re);
  num.im = wave_sum(num.im);
  den.re = wave_sum(den.re);
  den.im = wave_sum(den.im);
  if (lane != 0) return;
  const bool alive = (den.re != 0.0 || den.im != 0.0) && (num.re != 0.0 || num.im != 0.0);
  double wn = 0.0;
  if (alive) {
    const cplx r = cdiv(num, den);
    const double absr = sqrt(cabs2(r));
    const double mag = exp(sr + log(absr) + dtau * e_shift);
    if (weight_mode == AFQMC_WEIGHT_COMBINED)
      wn = w[wk] * mag;
    else
      wn = w[wk] * mag * fmax(0.0, cos(atan2(r.im, r.re)));
  }
  w[wk] = wn;
  const cplx rf = (weight_mode == AFQMC_WEIGHT_COMBINED) ? den : num;
  ref[(size_t)wk * 2] = rf.re;
  ref[(size_t)wk * 2 + 1] = rf.im;
}

template <int MT>
hipError_t launch_taylor_mt(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi) {
  hipLaunchKernelGGL(k_taylor<MT>, dim3(nw), dim3(MT * 4), 0, c->stream, c->M, c->N, c->n_taylor,
                     vmat, c->d_Eh, phi);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_vbuild(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         double* vmat) {
  if (nw <= 0) return hipSuccess;
  const int MM = c->M * c->M;
  dim3 grid((MM + 63) / 64, (nw + 63) / 64), block(256);
  hipLaunchKernelGGL(k_vbuild, grid, block, 0, c->stream, nw, c->G, MM, sqrt(c->dtau),
                     c->d_Lraw, xi, xbar, vmat);
  return hipGetLastError();
}

hipError_t launch_taylor(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi) {
  if (nw <= 0) return hipSuccess;
  switch (c->MT) {
    case 16: return launch_taylor_mt<16>(c, nw, vmat, phi);
    case 32: return launch_taylor_mt<32>(c, nw, vmat, phi);
    case 48: return launch_taylor_mt<48>(c, nw, vmat, phi);
    case 64: return launch_taylor_mt<64>(c, nw, vmat, phi);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_weight(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         const double* logov, const double* logov_new, double e_shift, double* w,
                         double* ref) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weight, dim3(nw), dim3(64), 0, c->stream, nw, c->P, c->G, c->dtau, e_shift,
                     c->weight_mode, xi, xbar, logov, logov_new, w, ref);
  return hipGetLastError();
}
