// Sampled trial determinants Phi_T(y) = exp(c sum_k y_k A_k) Phi_0 (Sec. II.C,
// Eq. trial_decomp; Sec. III.A, Eq. Metropolis_sampled_trial), FP64 matrix cores.
//
// k_trial_diag: generators that are all diagonal (the Ising pair operators)
//   give a diagonal U, and exp(U) Phi_0 is a row scaling of Phi_0.
// U_s = c sum_k y_{s,k} A_k for every path s: one FP64 product (paths x K) by
//   (K x M^2) on the LDS-tiled kernel of the V build (launch_ubuild; split-BF16
//   products for BF16 contexts on the workgroup kernels).
// k_trial_taylor: one wavefront per path holds its U in registers as MFMA A
//   operands and runs the Taylor series sum_j U^j Phi_0 / j!.  With the k
//   index of the product visited as 16 t + 4 r + g, the accumulator of one
//   term is, register for register, the B operand of the next, so the series
//   needs no LDS traffic.  When the row-sum norm of U exceeds 16 the series
//   is applied s = ceil(norm / 16) times to U / s.  Every entry of term j + 1
//   is at most r / (j + 1) times the largest entry of term j (r = ||U / s||_inf),
//   so after term j the whole dropped tail is bounded by max|term_j| times
//   (r / (j + 1)) / (1 - r / (j + 2)) once j + 2 > r; the series stops (checked
//   every second term) when that bound is below 2^-56 max|sum|, a quarter of
//   an ulp of the largest entry.
// Mixed-precision contexts (any precision but FP64) run both Taylor kernels
// with FP32 products (v_mfma_f32_16x16x4f32: U and the terms rounded to FP32,
// FP32 accumulation within a product, the running sum kept in FP64) and stop
// when the tail bound is below 2^-26 max|sum|, a quarter of an FP32 ulp.
// BF16 contexts on the workgroup kernels run the series on split-BF16 products
// instead (k_trial_taylor_x3, below) and stop at 2^-20.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

constexpr int TB_WAVES = 4;
constexpr int MAX_TERMS = 128;

// Diagonal generators (the Ising pair operators): U is diagonal, so exp(U) Phi_0
// scales row i of Phi_0 by exp(c sum_k y_k A_k[i][i]); one thread per entry.
__global__ void k_trial_diag(int n_samples, int M, int N, int K, double coupling,
                             const double* __restrict__ y, const double* __restrict__ Adiag,
                             const double* __restrict__ phi0, double* __restrict__ phiT) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n_samples * M * N) return;
  const int n = (int)(idx % N), i = (int)((idx / N) % M);
  const size_t s = idx / ((size_t)M * N);
  double u = 0.0;
  for (int k = 0; k < K; ++k) u = fma(y[s * K + k], Adiag[(size_t)k * M + i], u);
  phiT[idx] = exp(coupling * u) * phi0[(size_t)i * N + n];
}

hipError_t launch_trial_diag(const afqmc_ctx_s* c, int n, const double* y, double* phiT) {
  const size_t total = (size_t)n * c->M * c->N;
  hipLaunchKernelGGL(k_trial_diag, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                     n, c->M, c->N, c->K, c->coupling, y, c->d_Adiag, c->d_phi0, phiT);
  return hipGetLastError();
}

// the dropped tail may be at most this fraction of max|sum|
template <typename T>
__device__ __forceinline__ constexpr double stop_ratio() {
  return sizeof(T) == 8 ? 0x1.0p-56 : 0x1.0p-26;
}

// Stop test after term j of exp(V) X with r = ||V||_inf: the tail
// sum_{i>j} V^i X / i! has entries at most tmax * q / (1 - r / (j + 2)),
// q = r / (j + 1), when j + 2 > r (no bound before that); tested with both
// sides multiplied by (j + 1)(j + 2) > 0, so without divisions.
template <typename T>
__device__ __forceinline__ bool series_done(double tmax, double smax, double r, int j) {
  const double nxt = (double)(j + 2);
  if (!(nxt > r)) return false;
  return tmax * r * nxt <= stop_ratio<T>() * smax * (nxt - r) * (double)(j + 1);
}

template <typename T, int MT>
__global__ void __launch_bounds__(TB_WAVES * 64, 2)
k_trial_taylor(int n_samples, int M, int N, const double* __restrict__ U,
               const double* __restrict__ phi0, double* __restrict__ phiT) {
  typedef MM<T> mm;
  typedef typename mm::acc_t acc_t;
  constexpr int NTILE = MT / 16;  // row tiles
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int s = blockIdx.x * TB_WAVES + wave;
  if (s >= n_samples) return;  // no block-level barriers in this kernel
  const double* Us = U + (size_t)s * M * M;

  // ua[tp][t][r] = U[16 tp + c][16 t + k(g, r)] = U[16 t + k(g, r)][16 tp + c],
  // k(g, r) = mm::row(g, r)
  T ua[NTILE][NTILE][4];
  double rownorm = 0.0;
#pragma unroll
  for (int tp = 0; tp < NTILE; ++tp) {
    double rs = 0.0;
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * t + mm::row(g, r), col = 16 * tp + c;
        const double u = (row < M && col < M) ? Us[(size_t)row * M + col] : 0.0;
        ua[tp][t][r] = (T)u;
        rs += fabs(u);
      }
    // row 16 tp + c of U: its entries are spread over the four lane groups
    rs += __shfl_xor(rs, 16, 64);
    rs += __shfl_xor(rs, 32, 64);
    rownorm = fmax(rownorm, rs);
  }
  rownorm = wave_max_full(rownorm);
  // a non-finite U gives a non-finite Phi_T after one stage; the stage count
  // is bounded so that every wavefront finishes
  int nstage = 1;
  if (rownorm > 16.0 && rownorm < 16.0 * 4096.0) nstage = (int)ceil(rownorm / 16.0);
  const double rn = rownorm / nstage;
  if (nstage > 1) {
    const T inv = (T)(1.0 / nstage);
#pragma unroll
    for (int tp = 0; tp < NTILE; ++tp)
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) ua[tp][t][r] *= inv;
  }

  // sum = Phi_0 in the accumulator layout: sum[t][r] = X[16 t + k(g, r)][c]
  double sum[NTILE][4];
  T term[NTILE][4];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * t + mm::row(g, r);
      sum[t][r] = (m < M && c < N) ? phi0[m * N + c] : 0.0;
    }

  for (int st = 0; st < nstage; ++st) {
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) term[t][r] = (T)sum[t][r];
    for (int j = 1; j <= MAX_TERMS; ++j) {
      acc_t acc[NTILE];
#pragma unroll
      for (int tp = 0; tp < NTILE; ++tp) acc[tp] = mm::zero();
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int tp = 0; tp < NTILE; ++tp) acc[tp] = mm::fma(ua[tp][t][r], term[t][r], acc[tp]);
      const T invj = (T)(1.0 / (double)j);
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          term[t][r] = acc[t][r] * invj;
          sum[t][r] += (double)term[t][r];
        }
      if (j & 1) continue;
      double tmax = 0.0, smax = 0.0;
#pragma unroll
      for (int t = 0; t < NTILE; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tmax = fmax(tmax, fabs((double)term[t][r]));
          smax = fmax(smax, fabs(sum[t][r]));
        }
      tmax = wave_max_full(tmax);
      smax = wave_max_full(smax);
      if (series_done<T>(tmax, smax, rn, j)) break;
    }
  }

  double* out = phiT + (size_t)s * M * N;
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * t + mm::row(g, r);
      if (m < M && c < N) out[m * N + c] = sum[t][r];
    }
}

template <int MT>
hipError_t launch_mt(const afqmc_ctx_s* c, int n, const double* U, double* phiT) {
  dim3 grid((n + TB_WAVES - 1) / TB_WAVES), block(TB_WAVES * 64);
  if (c->precision != AFQMC_PREC_FP64)
    hipLaunchKernelGGL((k_trial_taylor<float, MT>), grid, block, 0, c->stream, n, c->M, c->N, U,
                       c->d_phi0, phiT);
  else
    hipLaunchKernelGGL((k_trial_taylor<double, MT>), grid, block, 0, c->stream, n, c->M, c->N, U,
                       c->d_phi0, phiT);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_trial_build(const afqmc_ctx_s* c, int n_samples, const double* y, double* phiT,
                              double* ubuf) {
  if (n_samples <= 0) return hipSuccess;
  if (c->d_Adiag != nullptr) return launch_trial_diag(c, n_samples, y, phiT);
  {
    const hipError_t e = launch_ubuild(c, n_samples, y, ubuf, nullptr, 0);
    if (e != hipSuccess) return e;
  }
  switch (c->MT) {
    case 16: return launch_mt<16>(c, n_samples, ubuf, phiT);
    case 32: return launch_mt<32>(c, n_samples, ubuf, phiT);
    case 48: return launch_mt<48>(c, n_samples, ubuf, phiT);
    case 64: return launch_mt<64>(c, n_samples, ubuf, phiT);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Larger systems (M <= 160, N <= 40): one workgroup per path, one wavefront per
// 16-row tile of U (its rows held as MFMA A operands); the Taylor iterate is
// shared through a double-buffered LDS tile, one barrier per term.
namespace {

template <typename T, int KTMAX, int NTC>
__global__ void __launch_bounds__(64 * KTMAX)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1)))
k_trial_taylor_g(int n_samples, int M, int N, int MT, const double* __restrict__ U,
                 const double* __restrict__ phi0, double* __restrict__ phiT) {
  typedef MM<T> mm;
  typedef typename mm::acc_t acc_t;
  constexpr int NT = 16 * NTC;
  extern __shared__ double smem[];
  T* sT = reinterpret_cast<T*>(smem);                           // [2][MT][NT]
  double* sred = smem + (2 * MT * NT * sizeof(T) + 7) / 8;      // [KTMAX][2]
  const int KT = MT / 16;
  const int s = blockIdx.x;
  const int tp = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  if (s >= n_samples) return;
  const double* Us = U + (size_t)s * M * M;

  // ua[t][r] = U[16 tp + c][16 t + k(g, r)], k(g, r) = mm::row(g, r)
  T ua[KTMAX][4];
  double rs = 0.0;
#pragma unroll
  for (int t = 0; t < KTMAX; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + mm::row(g, r), col = 16 * tp + c;
      const double u = (t < KT && row < M && col < M) ? Us[(size_t)row * M + col] : 0.0;
      ua[t][r] = (T)u;
      rs += fabs(u);
    }
  rs += __shfl_xor(rs, 16, 64);
  rs += __shfl_xor(rs, 32, 64);
  rs = wave_max_full(rs);
  if (lane == 0) sred[tp * 2] = rs;
  // Phi_0 into buffer 0 and into the running sum (my rows)
  for (int q = threadIdx.x; q < MT * NT; q += blockDim.x) {
    const int m = q / NT, n = q % NT;
    sT[q] = (T)((m < M && n < N) ? phi0[m * N + n] : 0.0);
  }
  __syncthreads();
  double rownorm = 0.0;
  for (int w = 0; w < KT; ++w) rownorm = fmax(rownorm, sred[w * 2]);
  int nstage = 1;
  if (rownorm > 16.0 && rownorm < 16.0 * 4096.0) nstage = (int)ceil(rownorm / 16.0);
  const double rn = rownorm / nstage;
  if (nstage > 1) {
    const T inv = (T)(1.0 / nstage);
#pragma unroll
    for (int t = 0; t < KTMAX; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) ua[t][r] *= inv;
  }
  double sm[NTC][4];
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * tp + mm::row(g, r), n = 16 * ct + c;
      sm[ct][r] = (m < M && n < N) ? phi0[m * N + n] : 0.0;
    }
  __syncthreads();

  int cur = 0;
  for (int st = 0; st < nstage; ++st) {
    if (st > 0) {  // the stage starts from the previous stage's sum
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sT[cur * MT * NT + (16 * tp + mm::row(g, r)) * NT + 16 * ct + c] = (T)sm[ct][r];
      __syncthreads();
    }
    for (int j = 1; j <= MAX_TERMS; ++j) {
      const T* Tc = sT + cur * MT * NT;
      T* Tn = sT + (cur ^ 1) * MT * NT;
      acc_t acc[NTC];
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) acc[ct] = mm::zero();
#pragma unroll
      for (int t = 0; t < KTMAX; ++t)
        if (t < KT)
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int ct = 0; ct < NTC; ++ct)
              acc[ct] = mm::fma(ua[t][r], Tc[(16 * t + mm::row(g, r)) * NT + 16 * ct + c], acc[ct]);
      const T invj = (T)(1.0 / (double)j);
      // maxima only on the terms that test, in the series' own precision (an
      // FP32 series' terms and restarts are FP32 already)
      const bool check = (j & 1) == 0;
      T tmax = 0, smax = 0;
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T v = acc[ct][r] * invj;
          sm[ct][r] += (double)v;
          Tn[(16 * tp + mm::row(g, r)) * NT + 16 * ct + c] = v;
          if (check) {
            tmax = fmax(tmax, fabs(v));
            smax = fmax(smax, (T)fabs(sm[ct][r]));
          }
        }
      if (check) {
        if constexpr (sizeof(T) == 4) {
          tmax = wave_max_full_f32(tmax);
          smax = wave_max_full_f32(smax);
        } else {
          tmax = wave_max_full(tmax);
          smax = wave_max_full(smax);
        }
        if (lane == 0) {
          sred[tp * 2] = tmax;
          sred[tp * 2 + 1] = smax;
        }
      }
      __syncthreads();
      cur ^= 1;
      if (check) {
        double tm = 0.0, sx = 0.0;
        for (int w = 0; w < KT; ++w) {
          tm = fmax(tm, sred[w * 2]);
          sx = fmax(sx, sred[w * 2 + 1]);
        }
        if (series_done<T>(tm, sx, rn, j)) break;
      }
    }
  }
  double* out = phiT + (size_t)s * M * N;
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * tp + mm::row(g, r), n = 16 * ct + c;
      if (m < M && n < N) out[m * N + n] = sm[ct][r];
    }
}

template <typename T, int KTMAX, int NTC>
hipError_t launch_tgt(const afqmc_ctx_s* c, int n, const double* U, double* phiT) {
  const int NT = 16 * NTC;
  const size_t lds = ((2 * (size_t)c->MT * NT * sizeof(T) + 7) / 8 + 2 * KTMAX) * sizeof(double);
  auto kern = k_trial_taylor_g<T, KTMAX, NTC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n), dim3(64 * (c->MT / 16)), lds, c->stream, n, c->M, c->N, c->MT,
                     U, c->d_phi0, phiT);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BF16 contexts (real trials, M <= 128, N <= 32; the split-BF16 contexts keep
// FP32 products, whose contraction stays near FP32 accuracy): the same series
// with split-BF16 products on v_mfma_f32_16x16x32_bf16.  One workgroup
// per path, one wavefront per 16-row tile of U; wavefront tp keeps its rows of
// U / s as A operands (lane (g, c): row 16 tp + c, k = 32 t + 8 g + j, as BF16
// hi = bf16(u) and lo = bf16(u - hi)); the iterate X (MT x NT) sits in LDS
// transposed, X^T[n][m], as hi and lo planes whose rows are padded by 16
// bytes, so a B operand (8 consecutive m of column n) is one 16-byte read per
// part without bank conflicts.  Each product is hi hi + hi lo + lo hi with
// FP32 accumulation (the dropped lo lo is below 2^-16 relative); the term is
// rounded to hi and lo once as it leaves the accumulators, the running sum is
// kept in FP64, and the series stops when the tail bound is below 2^-20 of the
// largest sum entry (the products themselves carry about 2^-17).  One barrier
// per term.
template <int KTMAX, int NTC>
__global__ void __launch_bounds__(64 * KTMAX) __attribute__((amdgpu_waves_per_eu(6)))
k_trial_taylor_x3(int n_samples, int M, int N, int MT, const double* __restrict__ U,
                  const unsigned short* __restrict__ Us, const double* __restrict__ phi0,
                  double* __restrict__ phiT) {
  constexpr int NT = 16 * NTC;
  constexpr int KBM = (16 * KTMAX + 31) / 32;  // k blocks of 32 at most
  const int KB = (MT + 31) / 32;                // k blocks (the last may be padding)
  const int XS = 32 * KB + 8;                   // LDS row of X^T (bf16 entries)
  extern __shared__ double smem[];
  unsigned short* sX = reinterpret_cast<unsigned short*>(smem);  // [2 buffers][2 parts][NT][XS]
  double* sred = smem + (4 * NT * XS * 2 + 7) / 8;               // [KTMAX][2]
  const int s = blockIdx.x;
  const int tp = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  if (s >= n_samples) return;
  const double* Usd = U != nullptr ? U + (size_t)s * M * M : nullptr;
  auto xt = [&](int buf, int part, int n, int m) -> unsigned short* {
    return sX + ((size_t)(buf * 2 + part) * NT + n) * XS + m;
  };

  // rows of U: ua[t][j] = U[16 tp + c][32 t + 8 g + j], from FP64 U or from U
  // already split ([hi, lo][M][32 KB] BF16: one 16-byte load per part)
  float ua[KBM][8];
  double rs = 0.0;
  const int row = 16 * tp + c;
  if (Us != nullptr) {
    const unsigned short* uh = Us + (size_t)s * 2 * M * (32 * KB);
    const unsigned short* ul = uh + (size_t)M * (32 * KB);
#pragma unroll
    for (int t = 0; t < KBM; ++t) {
      const bool ok = t < KB && row < M;
      const size_t o = (size_t)min(row, M - 1) * (32 * KB) + 32 * min(t, KB - 1) + 8 * g;
      const uint4 h = *reinterpret_cast<const uint4*>(uh + o);
      const uint4 l = *reinterpret_cast<const uint4*>(ul + o);
      const unsigned hw[4] = {h.x, h.y, h.z, h.w}, lw[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ua[t][2 * q] = ok ? tbf_lo(hw[q]) + tbf_lo(lw[q]) : 0.f;
        ua[t][2 * q + 1] = ok ? tbf_hi(hw[q]) + tbf_hi(lw[q]) : 0.f;
        rs += fabs((double)ua[t][2 * q]) + fabs((double)ua[t][2 * q + 1]);
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < KBM; ++t)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int col = 32 * t + 8 * g + j;
        const double u = (t < KB && row < M && col < M) ? Usd[(size_t)row * M + col] : 0.0;
        ua[t][j] = (float)u;
        rs += fabs(u);
      }
  }
  rs += __shfl_xor(rs, 16, 64);
  rs += __shfl_xor(rs, 32, 64);
  rs = wave_max_full(rs);
  if (lane == 0) sred[tp * 2] = rs;
  // both buffers zero (the padding rows past MT and columns past N stay zero),
  // then Phi_0 into buffer 0
  for (int q = threadIdx.x; q < 4 * NT * XS; q += blockDim.x) sX[q] = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < MT * NT; q += blockDim.x) {
    const int m = q / NT, n = q % NT;
    const float x = (float)((m < M && n < N) ? phi0[m * N + n] : 0.0);
    const unsigned h = tpk_bf16(x, 0.f);
    *xt(0, 0, n, m) = (unsigned short)(h & 0xffffu);
    *xt(0, 1, n, m) = (unsigned short)(tpk_bf16(x - tbf_lo(h), 0.f) & 0xffffu);
  }
  double rownorm = 0.0;
  for (int w = 0; w < MT / 16; ++w) rownorm = fmax(rownorm, sred[w * 2]);
  int nstage = 1;
  if (rownorm > 16.0 && rownorm < 16.0 * 4096.0) nstage = (int)ceil(rownorm / 16.0);
  const double rn = rownorm / nstage;
  tsx8 ah[KBM], al[KBM];  // A operands: hi and lo of U / nstage
  {
    const float inv = (float)(1.0 / nstage);
#pragma unroll
    for (int t = 0; t < KBM; ++t) {
      unsigned hw[4], lw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float a = ua[t][2 * q] * inv, b = ua[t][2 * q + 1] * inv;
        hw[q] = tpk_bf16(a, b);
        lw[q] = tpk_bf16(a - tbf_lo(hw[q]), b - tbf_hi(hw[q]));
      }
      ah[t] = __builtin_bit_cast(tsx8, uint4{hw[0], hw[1], hw[2], hw[3]});
      al[t] = __builtin_bit_cast(tsx8, uint4{lw[0], lw[1], lw[2], lw[3]});
    }
  }
  // running sum (rows 16 tp + 4 g + r, column 16 ct + c), FP64
  double sm[NTC][4];
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * tp + 4 * g + r, n = 16 * ct + c;
      sm[ct][r] = (m < M && n < N) ? phi0[m * N + n] : 0.0;
    }
  // store four consecutive rows of one column (this lane's accumulator values) as hi and lo
  auto put = [&](int buf, int ct, const float (&v)[4]) {
    const unsigned h01 = tpk_bf16(v[0], v[1]), h23 = tpk_bf16(v[2], v[3]);
    const unsigned l01 = tpk_bf16(v[0] - tbf_lo(h01), v[1] - tbf_hi(h01));
    const unsigned l23 = tpk_bf16(v[2] - tbf_lo(h23), v[3] - tbf_hi(h23));
    const int n = 16 * ct + c, m = 16 * tp + 4 * g;
    *reinterpret_cast<uint2*>(xt(buf, 0, n, m)) = uint2{h01, h23};
    *reinterpret_cast<uint2*>(xt(buf, 1, n, m)) = uint2{l01, l23};
  };
  __syncthreads();

  int cur = 0;
  for (int st = 0; st < nstage; ++st) {
    if (st > 0) {  // the stage starts from the previous stage's sum
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) {
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (float)sm[ct][r];
        put(cur, ct, v);
      }
      __syncthreads();
    }
    for (int j = 1; j <= MAX_TERMS; ++j) {
      fx4 acc[NTC];
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) acc[ct] = fx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < KBM; ++t)
        if (t < KB)
#pragma unroll
          for (int ct = 0; ct < NTC; ++ct) {
            const int n = 16 * ct + c, m = 32 * t + 8 * g;
            const tsx8 bh = *reinterpret_cast<const tsx8*>(xt(cur, 0, n, m));
            const tsx8 bl = *reinterpret_cast<const tsx8*>(xt(cur, 1, n, m));
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(tbfx8, ah[t]),
                                                              __builtin_bit_cast(tbfx8, bh), acc[ct], 0, 0, 0);
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(tbfx8, ah[t]),
                                                              __builtin_bit_cast(tbfx8, bl), acc[ct], 0, 0, 0);
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(tbfx8, al[t]),
                                                              __builtin_bit_cast(tbfx8, bh), acc[ct], 0, 0, 0);
          }
      const float invj = (float)(1.0 / (double)j);
      // the stop test (every second term) takes the maxima in FP32: the term
      // entries are FP32 already and the test is at 2^-20
      const bool check = (j & 1) == 0;
      float tmax = 0.f, smax = 0.f;
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) {
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v[r] = acc[ct][r] * invj;
          sm[ct][r] += (double)v[r];
          if (check) {
            tmax = fmaxf(tmax, fabsf(v[r]));
            smax = fmaxf(smax, fabsf((float)sm[ct][r]));
          }
        }
        put(cur ^ 1, ct, v);
      }
      if (check) {
        tmax = wave_max_full_f32(tmax);
        smax = wave_max_full_f32(smax);
        if (lane == 0) {
          sred[tp * 2] = tmax;
          sred[tp * 2 + 1] = smax;
        }
      }
      __syncthreads();
      cur ^= 1;
      if (check) {
        double tm = 0.0, sx = 0.0;
        for (int w = 0; w < MT / 16; ++w) {
          tm = fmax(tm, sred[w * 2]);
          sx = fmax(sx, sred[w * 2 + 1]);
        }
        // tail bound tm rn / (j + 1) against 2^-20 sx (1 - rn / nxt), as in
        // series_done
        const double nxt = (double)(j + 2);
        if (nxt > rn && tm * rn * nxt <= 0x1.0p-20 * sx * (nxt - rn) * (double)(j + 1)) break;
      }
    }
  }
  double* out = phiT + (size_t)s * M * N;
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * tp + 4 * g + r, n = 16 * ct + c;
      if (m < M && n < N) out[m * N + n] = sm[ct][r];
    }
}

template <int KTMAX, int NTC>
hipError_t launch_tgx(const afqmc_ctx_s* c, int n, const double* U, const unsigned short* Us,
                      double* phiT) {
  const int NT = 16 * NTC, XS = 32 * ((c->MT + 31) / 32) + 8;
  const size_t lds = ((size_t)4 * NT * XS * 2 + 7) / 8 * 8 + (size_t)2 * KTMAX * sizeof(double);
  auto kern = k_trial_taylor_x3<KTMAX, NTC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n), dim3(64 * (c->MT / 16)), lds, c->stream, n, c->M, c->N, c->MT,
                     U, Us, c->d_phi0, phiT);
  return hipGetLastError();
}

template <int KTMAX, int NTC>
hipError_t launch_tg(const afqmc_ctx_s* c, int n, const double* U, double* phiT) {
  if constexpr (KTMAX <= 8 && NTC <= 2) {
    if (c->precision == AFQMC_PREC_BF16) return launch_tgx<KTMAX, NTC>(c, n, U, nullptr, phiT);
  }
  return c->precision != AFQMC_PREC_FP64 ? launch_tgt<float, KTMAX, NTC>(c, n, U, phiT)
                                         : launch_tgt<double, KTMAX, NTC>(c, n, U, phiT);
}

}  // namespace

// Multi-slice trials (Sec. II.C, Eqs. trial and trial-AF; Sec. III.B):
// Phi_T(Y) = F_m X_m ... F_1 X_1 F_0 Phi_0, X_l = T_n(i sqrt(s_l) sum_k y_{l,k} A_k),
// slice by slice with the walker propagator's kernels: V_l for every path
// (k_vbuild over the slice's block of y), then F_l T_n(V_l) [F_0] applied to
// the running determinant (the first slice reads Phi_0 for every path).
hipError_t launch_trial_slices(const afqmc_ctx_s* c, int n, const double* y, double* phiT,
                               double* vbuf) {
  if (n <= 0) return hipSuccess;
  const size_t MM = (size_t)c->M * c->M;
  for (int l = 0; l < c->n_slices; ++l) {
    hipError_t e = launch_vbuild_gen(c, n, c->kgen, c->K, sqrt(c->slice_s[l]), c->d_A,
                                     y + (size_t)l * c->kgen, vbuf);
    if (e != hipSuccess) return e;
    e = launch_taylor_g_gen(c, n, 1, c->trial_taylor, vbuf, c->d_F + (size_t)(l + 1) * MM,
                            l == 0 ? c->d_F : nullptr, l == 0 ? c->d_phi0c : phiT,
                            l == 0 ? 0 : 1, phiT);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_trial_build_g(const afqmc_ctx_s* c, int n_samples, const double* y, double* phiT,
                                double* ubuf, void* scratch, size_t scratch_bytes) {
  if (n_samples <= 0) return hipSuccess;
  if (c->ctrial) return launch_trial_slices(c, n_samples, y, phiT, ubuf);
  if (c->d_Adiag != nullptr) return launch_trial_diag(c, n_samples, y, phiT);
  const int KT = c->MT / 16, NTC = (c->N + 15) / 16;
  if (c->precision == AFQMC_PREC_BF16 && KT <= 8 && NTC <= 2 && scratch != nullptr &&
      ubuild_split_ok(c, n_samples, scratch_bytes)) {
    // U split once by its own build, in the U buffer (4 n M MP <= 8 n M^2 bytes)
    unsigned short* Us = reinterpret_cast<unsigned short*>(ubuf);
    const hipError_t e = launch_ubuild_split(c, n_samples, y, Us, scratch);
    if (e != hipSuccess) return e;
#define AFQMC_X(KM, NC) \
  if (KT <= KM && NTC == NC) return launch_tgx<KM, NC>(c, n_samples, nullptr, Us, phiT);
    AFQMC_X(4, 1) AFQMC_X(6, 1) AFQMC_X(8, 1)
    AFQMC_X(4, 2) AFQMC_X(6, 2) AFQMC_X(8, 2)
#undef AFQMC_X
  }
  {
    const hipError_t e = launch_ubuild(c, n_samples, y, ubuf, scratch, scratch_bytes);
    if (e != hipSuccess) return e;
  }
#define AFQMC_T(KM, NC) \
  if (KT <= KM && NTC == NC) return launch_tg<KM, NC>(c, n_samples, ubuf, phiT);
  AFQMC_T(4, 1) AFQMC_T(6, 1) AFQMC_T(8, 1) AFQMC_T(10, 1)
  AFQMC_T(4, 2) AFQMC_T(6, 2) AFQMC_T(8, 2) AFQMC_T(10, 2)
  AFQMC_T(4, 3) AFQMC_T(6, 3) AFQMC_T(8, 3) AFQMC_T(10, 3)
#undef AFQMC_T
  return hipErrorInvalidValue;
}
