// Sampled trial determinants Phi_T(y) = exp(c sum_k y_k A_k) Phi_0 (Sec. II.C,
// Eq. trial_decomp; Sec. III.A, Eq. Metropolis_sampled_trial), one wavefront
// per path, FP64 matrix cores.
//
// U = c sum_k y_k A_k is assembled one 16-row tile at a time in LDS from the
// row-sorted entry list and then held in registers as MFMA A operands.  The
// Taylor series sum_j U^j Phi_0 / j! is run term by term: with the k index of
// the product taken in the order (16 t + 4 r + g) the accumulator of one term
// is, register for register, the B operand of the next, so the series needs
// no LDS traffic.  Terms are added until max|term| <= 2^-60 max|sum|; when the
// row-sum norm of U exceeds 8 the series is applied s = ceil(norm / 8) times
// to U / s.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

constexpr int TB_WAVES = 4;
constexpr int MAX_TERMS = 128;

template <int MT>
__global__ void __launch_bounds__(TB_WAVES * 64)
k_trial_build(int n_samples, int M, int N, int K, double coupling, const double* __restrict__ y,
              const double* __restrict__ phi0, const int* __restrict__ row_ptr,
              const int* __restrict__ ent_row, const int* __restrict__ ent_col,
              const int* __restrict__ ent_kptr,
              const int* __restrict__ con_k, const double* __restrict__ con_v,
              double* __restrict__ phiT) {
  constexpr int NTILE = MT / 16;  // row tiles
  __shared__ double s_tile[TB_WAVES][16 * MT];
  __shared__ double s_y[TB_WAVES][256];

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int s = blockIdx.x * TB_WAVES + wave;
  const bool active = s < n_samples;  // uniform per wave

  double* tile = s_tile[wave];
  double* ys = s_y[wave];
  if (active)
    for (int k = lane; k < K; k += 64) ys[k] = y[(size_t)s * K + k];

  // U in registers: ua[tp][t][r] = U[16 tp + c][16 t + 4 r + g]
  double ua[NTILE][NTILE][4];
  double rownorm = 0.0;
#pragma unroll
  for (int tp = 0; tp < NTILE; ++tp) {
    for (int q = lane; q < 16 * MT; q += 64) tile[q] = 0.0;
    __syncthreads();
    if (active) {
      const int r0 = 16 * tp, r1 = min(16 * tp + 16, M);
      for (int e = row_ptr[r0] + lane; e < row_ptr[r1]; e += 64) {
        const int i = ent_row[e];
        double u = 0.0;
        for (int q = ent_kptr[e]; q < ent_kptr[e + 1]; ++q) u += ys[con_k[q]] * con_v[q];
        tile[(i - r0) * MT + ent_col[e]] = coupling * u;
      }
    }
    __syncthreads();
    double rs = 0.0;
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ua[tp][t][r] = tile[c * MT + 16 * t + 4 * r + g];
        rs += fabs(ua[tp][t][r]);
      }
    rs += __shfl_xor(rs, 16, 64);
    rs += __shfl_xor(rs, 32, 64);
    rownorm = fmax(rownorm, rs);
    __syncthreads();
  }
  if (!active) return;
  rownorm = wave_max(rownorm);

  // a non-finite U gives a non-finite Phi_T after one stage; the stage count
  // is bounded so that every wavefront finishes
  int nstage = 1;
  if (rownorm > 8.0 && rownorm < 8.0 * 4096.0) nstage = (int)ceil(rownorm / 8.0);
  if (nstage > 1) {
    const double inv = 1.0 / nstage;
#pragma unroll
    for (int tp = 0; tp < NTILE; ++tp)
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) ua[tp][t][r] *= inv;
  }

  // X = Phi_0 in the accumulator layout: x[t][r] = X[16 t + 4 r + g][c]
  double x[NTILE][4];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int m = 16 * t + 4 * r + g;
      x[t][r] = (m < M && c < N) ? phi0[m * N + c] : 0.0;
    }

  for (int st = 0; st < nstage; ++st) {
    double sum[NTILE][4], term[NTILE][4];
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) sum[t][r] = term[t][r] = x[t][r];
    for (int j = 1; j <= MAX_TERMS; ++j) {
      dx4 acc[NTILE];
#pragma unroll
      for (int tp = 0; tp < NTILE; ++tp) acc[tp] = dx4_zero();
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int tp = 0; tp < NTILE; ++tp) acc[tp] = mfma_f64(ua[tp][t][r], term[t][r], acc[tp]);
      const double invj = 1.0 / (double)j;
      double tmax = 0.0, smax = 0.0;
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          term[t][r] = acc[t][r] * invj;
          sum[t][r] += term[t][r];
          tmax = fmax(tmax, fabs(term[t][r]));
          smax = fmax(smax, fabs(sum[t][r]));
        }
      tmax = wave_max(tmax);
      smax = wave_max(smax);
      if (tmax <= 0x1.0p-60 * smax) break;
    }
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) x[t][r] = sum[t][r];
  }

  double* out = phiT + (size_t)s * M * N;
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int m = 16 * t + 4 * r + g;
      if (m < M && c < N) out[m * N + c] = x[t][r];
    }
}

template <int MT>
hipError_t launch_mt(const afqmc_ctx_s* c, int n, const double* y, double* phiT) {
  dim3 grid((n + TB_WAVES - 1) / TB_WAVES), block(TB_WAVES * 64);
  hipLaunchKernelGGL(k_trial_build<MT>, grid, block, 0, c->stream, n, c->M, c->N, c->K,
                     c->coupling, y, c->d_phi0, c->d_row_ptr, c->d_ent_row, c->d_ent_col, c->d_ent_kptr,
                     c->d_con_k, c->d_con_v, phiT);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trial_build(const afqmc_ctx_s* c, int n_samples, const double* y, double* phiT) {
  if (n_samples <= 0) return hipSuccess;
  switch (c->MT) {
    case 16: return launch_mt<16>(c, n_samples, y, phiT);
    case 32: return launch_mt<32>(c, n_samples, y, phiT);
    case 48: return launch_mt<48>(c, n_samples, y, phiT);
    case 64: return launch_mt<64>(c, n_samples, y, phiT);
    default: return hipErrorInvalidValue;
  }
}
