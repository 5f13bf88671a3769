// Cholesky-vector contraction with reduced-precision matrix-core products and
// FP32 accumulation: FP32, split BF16 and BF16 (AFQMC_PREC_FP32 with a real
// trial, AFQMC_PREC_BF16X3, AFQMC_PREC_BF16).  Same quantities as k_contract
// (Sec. III.A, Eq. local-obs; Eq. shift1):
//   Y_g = Phi_T^T L_g,  f_g^s = Y_g Theta^s,  vb_g = sum_s tr f_g^s,
//   E_p = sum_s tr(Phi_T^T h1' Theta^s) + 1/2 sum_g [vb_g^2 - sum_s tr(f_g^s f_g^s)].
//
// Products: lane (g, c) supplies A[c][4g + j] and B[4g + j][c] (j = 0..3, four
// consecutive k values) and holds D[4g + r][c] -- one v_mfma_f32_16x16x16bf16_1k
// for BF16, four v_mfma_f32_16x16x4f32 (the j-th on k = 4g + j) for FP32.
// Split BF16: every operand x is carried as x_hi = bf16(x) and
// x_lo = bf16(x - x_hi), and a product a b as a_hi b_hi + a_hi b_lo + a_lo b_hi
// (three products; the dropped a_lo b_lo is below 2^-16 relative), which
// brings the contraction close to FP32 accuracy.  Plain BF16 takes a_hi b_hi.
//
// k_contract_sh: BCP paths per workgroup share each L slab through LDS.  Per
// path, 2 * NTC wavefronts (NTC = ceil(N/16)); wavefront w = (spin s = w % 2,
// column tile jt = w / 2) keeps Theta^s[:, jt] as B operands in registers for
// the whole loop over g, and Phi_T (all column tiles) as the stage-1 B
// operands.  Stage 1 (Y_g^T = L_g Phi_T) is split over the path's wavefronts by
// row tile, its A operands read from the shared slab.  Y_g^T is rounded to the
// operand form once, as stage 1 leaves it, and stored in LDS in the accumulator
// layout, which is stage 2's A-operand layout (rows 4g .. 4g+3 of a column in
// one lane); f is transposed through LDS for tr(f f); traces, vb_g^2 and the
// sums over g are FP64.

#include <type_traits>

#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

typedef short sx4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// hi / lo BF16 pair of a value: hi = bf16(x), lo = bf16(x - hi)
struct bsplit {
  sx4 hi, lo;
};
template <bool X3>
__device__ __forceinline__ bsplit split4(float a, float b, float c, float d) {
  bsplit s;
  const unsigned short h0 = f2bf(a), h1 = f2bf(b), h2 = f2bf(c), h3 = f2bf(d);
  s.hi = sx4{(short)h0, (short)h1, (short)h2, (short)h3};
  if (X3) {
    s.lo = sx4{(short)f2bf(a - bf2f(h0)), (short)f2bf(b - bf2f(h1)), (short)f2bf(c - bf2f(h2)),
               (short)f2bf(d - bf2f(h3))};
  } else {
    s.lo = sx4{0, 0, 0, 0};
  }
  return s;
}

template <bool X3>
__device__ __forceinline__ fx4 mma(const bsplit& a, const bsplit& b, fx4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, acc, 0, 0, 0);
  if (X3) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ fx4 fx4_zero() {
  fx4 z = {0.f, 0.f, 0.f, 0.f};
  return z;
}

// Operand forms of the contraction.  An operand is what one lane supplies to a
// 16 x 16 x 16 product: four consecutive k values (4g .. 4g+3) of one row or
// column, as NP parts of type V.  FP32 runs the product as four
// v_mfma_f32_16x16x4f32, the j-th taking k = 4g + j, so its lane layout is
// the BF16 one with float4 in place of four BF16 values.
enum { FM_BF16 = 0, FM_BF16X3 = 1, FM_FP32 = 2 };
template <int FM>
struct Form {
  static constexpr bool X3 = FM == FM_BF16X3;
  static constexpr bool F32 = FM == FM_FP32;
  static constexpr int NP = X3 ? 2 : 1;             // parts: hi (and lo)
  static constexpr int NB = FM == FM_BF16 ? 2 : 1;  // slab and Y^T buffers
  typedef typename std::conditional<F32, fx4, sx4>::type V;
  struct Op {
    V p[NP];
  };
  __device__ __forceinline__ static Op make(float a, float b, float c, float d) {
    Op o;
    if constexpr (F32) {
      o.p[0] = fx4{a, b, c, d};
    } else {
      const bsplit s = split4<X3>(a, b, c, d);
      o.p[0] = s.hi;
      if constexpr (X3) o.p[NP - 1] = s.lo;
    }
    return o;
  }
  __device__ __forceinline__ static fx4 mma(const Op& a, const Op& b, fx4 acc) {
    if constexpr (F32) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.p[0][j], b.p[0][j], acc, 0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.p[0], b.p[0], acc, 0, 0, 0);
      if constexpr (X3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.p[0], b.p[NP - 1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.p[NP - 1], b.p[0], acc, 0, 0, 0);
      }
    }
    return acc;
  }
};

// ---------------------------------------------------------------------------
// BCP paths per workgroup sharing each L slab: the slab of vector g + 1 goes
// from global memory straight into LDS (global_load_lds) during vector g,
// already in A-operand order ([row tile][k tile][lane][4]: one 8-byte LDS read
// per product, consecutive lanes on consecutive words), so every L byte crosses
// L2 once per workgroup instead of once per path.  f is staged for the
// transpose in FP32 (its products are FP32) and the diagonals flush every BFL
// vectors.
constexpr int BCP = 2;  // paths per workgroup
constexpr int BFL = 8;  // vectors per flush of the staged diagonals

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

template <int KT, int NTC, int FM>
__global__ void __launch_bounds__(128 * NTC * BCP)
k_contract_sh(int n_samples, int M, int N, int G, const void* __restrict__ Lop,
               const void* __restrict__ Lop_lo, const double* __restrict__ phiT,
               const double* __restrict__ theta,
               const double* __restrict__ logov, double* __restrict__ vb, double* __restrict__ ep) {
  constexpr int MT = 16 * KT;
  constexpr int NWV = 2 * NTC;                 // wavefronts per path
  constexpr int NWT = NWV * BCP;               // wavefronts per workgroup
  constexpr int NT = 16 * NTC;
  constexpr int S1MAX = (KT + NWV - 1) / NWV;  // stage-1 row tiles per wavefront
  typedef Form<FM> Fm;
  typedef typename Fm::V V;
  typedef typename Fm::Op Op;
  constexpr int SLAB = MT * MT;                // entries per slab
  constexpr int SV = SLAB / 4;                 // operands (V) per slab part
  constexpr int NU = SV * (int)sizeof(V) / 16; // 16-byte units per slab part
  constexpr int NCH = (NU + 63) / 64;          // 1 KB chunks per slab (the last may be partial)
  constexpr int YT = (MT / 4) * NT;            // operands of one Y^T tile part
  // plain BF16: slabs and Y^T tiles double-buffered (the next slab loads during
  // the whole vector); split BF16 (hi and lo of each) and FP32 (twice the
  // bytes): single buffers, the next slab loading from the barrier after stage 1
  // on, so that LDS still fits
  constexpr int NB = Fm::NB;                   // buffers
  constexpr int NP = Fm::NP;                   // parts (hi, lo)
  extern __shared__ double smem[];
  V* sL = reinterpret_cast<V*>(smem);                                      // [NB][NP][SV]
  V* sY = sL + NB * NP * SV;                                               // [BCP][NB][NP][YT]
  float* sF = reinterpret_cast<float*>(sY + BCP * NB * NP * YT);           // [BCP][2][NT][NT+1][2]
  double* sD = reinterpret_cast<double*>(sF + BCP * 2 * NT * (NT + 1) * 2);  // [BCP][BFL][NWV*16][2]
  double* sE = sD + BCP * BFL * NWV * 16 * 2;                              // [BCP][NWV][2]
  double* sT = sE + BCP * NWV * 2;                                         // [NWT][4]

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int pw = wave / NWV, wv = wave % NWV;  // path of the workgroup, wavefront of the path
  const int sp = wv & 1, jt = wv >> 1;
  const int s = blockIdx.x * BCP + pw;
  const bool valid = s < n_samples;            // every wavefront takes part in the barriers
  const int sc = valid ? s : n_samples - 1;
  const bool active = valid && !__builtin_isinf(logov[2 * sc]);

  auto copy_slab = [&](int slab, int buf) {
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      const char* src = reinterpret_cast<const char*>(part ? Lop_lo : Lop) +
                        (size_t)slab * SV * sizeof(V);
      char* dst = reinterpret_cast<char*>(sL + (buf * NP + part) * SV);
      for (int k = wave; k < NCH; k += NWT)
        if (k * 64 + lane < NU)  // lanes past a partial last chunk copy nothing
          __builtin_amdgcn_global_load_lds((gbl_ptr_t)(src + k * 1024 + lane * 16),
                                           (lds_ptr_t)(dst + k * 1024), 16, 0, 0);
    }
  };
  copy_slab(0, 0);

  // B operands (bit-masked unconditional loads)
  Op bT[NTC][KT], th[2][KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    float v[NTC][4], w[2][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = 16 * t + 4 * g + j;
      const bool okm = active && m < M;
      const int mc = min(m, M - 1);
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) {
        const int n = 16 * ct + c;
        const double x = phiT[((size_t)sc * M + mc) * N + min(n, N - 1)];
        v[ct][j] = (float)keep_if(x, okm && n < N);
      }
      const int n = 16 * jt + c;
      const double2 x2 = *reinterpret_cast<const double2*>(
          theta + ((((size_t)sc * 2 + sp) * M + mc) * N + min(n, N - 1)) * 2);
      w[0][j] = (float)keep_if(x2.x, okm && n < N);
      w[1][j] = (float)keep_if(x2.y, okm && n < N);
    }
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) bT[ct][t] = Fm::make(v[ct][0], v[ct][1], v[ct][2], v[ct][3]);
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) th[ri][t] = Fm::make(w[ri][0], w[ri][1], w[ri][2], w[ri][3]);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks of slab 0 are in LDS
  __syncthreads();

  V* Yp = sY + pw * NB * NP * YT;
  float* Fp = sF + (size_t)pw * 2 * NT * (NT + 1) * 2;
  double* Dp = sD + (size_t)pw * BFL * NWV * 16 * 2;
  double ex_re = 0.0, ex_im = 0.0, vb2_re = 0.0, vb2_im = 0.0, e1_re = 0.0, e1_im = 0.0;
  for (int gam = 0; gam <= G; ++gam) {
    const int b = NB == 2 ? (gam & 1) : 0;
    // stage 1: Y^T tiles (tp, ct) from the shared slab
    fx4 y1[S1MAX][NTC];
#pragma unroll
    for (int q = 0; q < S1MAX; ++q)
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) y1[q][ct] = fx4_zero();
    const V* Ls = sL + b * NP * SV;
#pragma unroll
    for (int q = 0; q < S1MAX; ++q) {
      const int tp = wv + NWV * q;
      if (active && tp < KT)
#pragma unroll
        for (int t = 0; t < KT; ++t) {
          Op a;
#pragma unroll
          for (int part = 0; part < NP; ++part) a.p[part] = Ls[part * SV + (tp * KT + t) * 64 + lane];
#pragma unroll
          for (int ct = 0; ct < NTC; ++ct) y1[q][ct] = Fm::mma(a, bT[ct][t], y1[q][ct]);
        }
    }
    // buffer b ^ 1 was last read in stage 1 of the previous vector, before its barriers
    if (NB == 2 && gam < G) copy_slab(gam + 1, b ^ 1);
    V* Yb = Yp + b * NP * YT;
#pragma unroll
    for (int q = 0; q < S1MAX; ++q) {
      const int tp = wv + NWV * q;
      if (tp < KT)
#pragma unroll
        for (int ct = 0; ct < NTC; ++ct) {
          const fx4 v = y1[q][ct];
          const Op yv = Fm::make(v[0], v[1], v[2], v[3]);
#pragma unroll
          for (int part = 0; part < NP; ++part) Yb[part * YT + (4 * tp + g) * NT + 16 * ct + c] = yv.p[part];
        }
    }
    __syncthreads();
    // single buffers: every stage-1 read of this slab is done, the next one can load
    if (NB == 1 && gam < G) copy_slab(gam + 1, 0);
    // stage 2: f^sp[it][jt], A[c][4g + j] = Y^T[16t + 4g + j][16it + c]
    fx4 f[NTC][2];
#pragma unroll
    for (int it = 0; it < NTC; ++it) f[it][0] = f[it][1] = fx4_zero();
    if (active) {
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int it = 0; it < NTC; ++it) {
          Op a;
#pragma unroll
          for (int part = 0; part < NP; ++part) a.p[part] = Yb[part * YT + (4 * t + g) * NT + 16 * it + c];
          f[it][0] = Fm::mma(a, th[0][t], f[it][0]);
          f[it][1] = Fm::mma(a, th[1][t], f[it][1]);
        }
    }
    // diagonal of f^sp in tile (jt, jt): element (4g + r, c) with 4g + r == c
    double d_re = 0.0, d_im = 0.0;
#pragma unroll
    for (int it = 0; it < NTC; ++it)
      if (it == jt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * g + r == c) {
            d_re = (double)f[it][0][r];
            d_im = (double)f[it][1][r];
          }
    if (gam == G) {  // h1': the path's one-body traces through LDS
      d_re = wave_sum(d_re);
      d_im = wave_sum(d_im);
      if (lane == 0) {
        sE[wave * 2] = d_re;
        sE[wave * 2 + 1] = d_im;
      }
      __syncthreads();
      if (wv == 0 && lane == 0) {
        for (int w = 0; w < NWV; ++w) {
          e1_re += sE[(pw * NWV + w) * 2];
          e1_im += sE[(pw * NWV + w) * 2 + 1];
        }
      }
      break;
    }
    // stage f^sp[:, jt] for the transpose, and the diagonal partials
    float* Fs = Fp + (size_t)sp * NT * (NT + 1) * 2;
#pragma unroll
    for (int it = 0; it < NTC; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * it + 4 * g + r, j = 16 * jt + c;
        Fs[(i * (NT + 1) + j) * 2] = f[it][0][r];
        Fs[(i * (NT + 1) + j) * 2 + 1] = f[it][1][r];
      }
    if (g == (c >> 2)) {
      double* d = Dp + ((size_t)(gam % BFL) * NWV * 16 + wv * 16 + c) * 2;
      d[0] = d_re;
      d[1] = d_im;
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks of the next slab landed
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NTC; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * it + 4 * g + r, j = 16 * jt + c;
        const double tr_ = Fs[(j * (NT + 1) + i) * 2], ti_ = Fs[(j * (NT + 1) + i) * 2 + 1];
        const double ar = (double)f[it][0][r], ai = (double)f[it][1][r];
        ex_re += ar * tr_ - ai * ti_;
        ex_im += ar * ti_ + ai * tr_;
      }
    // every BFL vectors: wavefront 0 of each path reduces its staged diagonals to vb_g
    if ((gam % BFL == BFL - 1 || gam == G - 1) && wv == 0 && valid) {
      const int cnt = gam % BFL + 1, g0 = gam - gam % BFL;
      const int gl = lane % BFL, part = (lane / BFL) & 1;
      double v = 0.0;
      if (lane < 2 * BFL && gl < cnt)
        for (int q = 0; q < NWV * 16; ++q) v += Dp[((size_t)gl * NWV * 16 + q) * 2 + part];
      const double vi = __shfl_down(v, BFL, 64);
      if (lane < BFL && gl < cnt) {
        vb2_re += v * v - vi * vi;
        vb2_im += 2.0 * v * vi;
        double* o = vb + ((size_t)s * G + g0 + gl) * 2;
        o[0] = v;
        o[1] = vi;
      }
    }
  }
  // totals per path: ex from every lane of its wavefronts, vb^2 from its wavefront 0
  ex_re = wave_sum(ex_re);
  ex_im = wave_sum(ex_im);
  vb2_re = wave_sum(vb2_re);
  vb2_im = wave_sum(vb2_im);
  if (lane == 0) {
    sT[wave * 4 + 0] = ex_re;
    sT[wave * 4 + 1] = ex_im;
    sT[wave * 4 + 2] = vb2_re;
    sT[wave * 4 + 3] = vb2_im;
  }
  __syncthreads();
  if (valid && wv == 0 && lane == 0) {
    double xr = 0.0, xi = 0.0;
    for (int w = 0; w < NWV; ++w) {
      xr += sT[(pw * NWV + w) * 4 + 0];
      xi += sT[(pw * NWV + w) * 4 + 1];
    }
    const double br = sT[pw * NWV * 4 + 2], bi = sT[pw * NWV * 4 + 3];
    double* o = ep + (size_t)s * 2;
    o[0] = active ? e1_re + 0.5 * br - 0.5 * xr : 0.0;
    o[1] = active ? e1_im + 0.5 * bi - 0.5 * xi : 0.0;
  }
  if (valid && !active && wv == 0)
    for (int q = lane; q < 2 * G; q += 64) vb[(size_t)s * G * 2 + q] = 0.0;
}

// the same for every form: buffers x parts x bytes per entry = 2 x 1 x 2 (BF16),
// 1 x 2 x 2 (split BF16) or 1 x 1 x 4 (FP32)
size_t lds_bytes_s(int KT, int NTC) {
  const int MT = 16 * KT, NT = 16 * NTC, NWV = 2 * NTC;
  size_t b = (size_t)4 * MT * MT;                     // slabs
  b += (size_t)BCP * (MT / 4) * NT * 16;              // Y^T tiles
  b += (size_t)BCP * 2 * NT * (NT + 1) * 2 * 4;       // f (FP32)
  b += (size_t)BCP * BFL * NWV * 16 * 2 * 8;          // staged diagonals
  b += (size_t)BCP * NWV * 2 * 8 + (size_t)BCP * NWV * 4 * 8;
  return b;
}

template <int KT, int NTC, int FM>
hipError_t launch_sh(const afqmc_ctx_s* c, int nw, const void* L, const void* L_lo,
                      const double* phiT, const double* theta, const double* logov, double* vb,
                      double* ep) {
  const int n = nw * c->P;
  const size_t lds = lds_bytes_s(KT, NTC);
  auto kern = k_contract_sh<KT, NTC, FM>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((n + BCP - 1) / BCP), dim3(128 * NTC * BCP), lds, c->stream, n,
                     c->M, c->N, c->G, L, L_lo, phiT, theta, logov, vb, ep);
  return hipGetLastError();
}

template <int FM>
hipError_t dispatch_s(const afqmc_ctx_s* c, int nw, const void* L, const void* L_lo,
                      const double* phiT, const double* theta, const double* logov, double* vb,
                      double* ep) {
  const int KT = c->MT / 16, NTC = (c->N + 15) / 16;
#define AFQMC_BS(KK, NC)    \
  if (KT == KK && NTC == NC) \
    return launch_sh<KK, NC, FM>(c, nw, L, L_lo, phiT, theta, logov, vb, ep);
  AFQMC_BS(1, 1) AFQMC_BS(2, 1) AFQMC_BS(3, 1) AFQMC_BS(4, 1)
  AFQMC_BS(5, 1) AFQMC_BS(6, 1) AFQMC_BS(7, 1) AFQMC_BS(8, 1)
  AFQMC_BS(2, 2) AFQMC_BS(3, 2) AFQMC_BS(4, 2)
  AFQMC_BS(5, 2) AFQMC_BS(6, 2) AFQMC_BS(7, 2) AFQMC_BS(8, 2)
#undef AFQMC_BS
  return hipErrorInvalidValue;
}

// L (double, row-major slabs) -> BF16 in A-operand order [slab][tp][t][g][c][j] =
// L[slab][16 tp + c][16 t + 4 g + j]; with lo given, also lo = bf16(L - hi) in that order
__global__ void k_to_bf16_op(size_t n, int MT, const double* __restrict__ src,
                             unsigned short* __restrict__ dst, unsigned short* __restrict__ lo) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int KT = MT / 16;
  const size_t slab = o / ((size_t)MT * MT);
  const int r = (int)(o % ((size_t)MT * MT));
  const int j = r & 3, cc = (r >> 2) & 15, gg = (r >> 6) & 3, t = (r >> 8) % KT, tp = (r >> 8) / KT;
  const float x = (float)src[slab * MT * MT + (size_t)(16 * tp + cc) * MT + 16 * t + 4 * gg + j];
  const unsigned short h = f2bf(x);
  dst[o] = h;
  if (lo != nullptr) lo[o] = f2bf(x - bf2f(h));
}

// the same order in FP32
__global__ void k_to_f32_op(size_t n, int MT, const double* __restrict__ src,
                            float* __restrict__ dst) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int KT = MT / 16;
  const size_t slab = o / ((size_t)MT * MT);
  const int r = (int)(o % ((size_t)MT * MT));
  const int j = r & 3, cc = (r >> 2) & 15, gg = (r >> 6) & 3, t = (r >> 8) % KT, tp = (r >> 8) / KT;
  dst[o] = (float)src[slab * MT * MT + (size_t)(16 * tp + cc) * MT + 16 * t + 4 * gg + j];
}

}  // namespace

hipError_t launch_contract_sh(const afqmc_ctx_s* c, int nw, const double* phiT,
                              const double* theta, const double* logov, double* vb, double* ep) {
  if (nw <= 0) return hipSuccess;
  if (c->ctrial) return hipErrorInvalidValue;  // real trial determinants only
  switch (c->precision) {
    case AFQMC_PREC_FP32:
      if (c->d_Lpad32 == nullptr) return hipErrorInvalidValue;
      return dispatch_s<FM_FP32>(c, nw, c->d_Lpad32, nullptr, phiT, theta, logov, vb, ep);
    case AFQMC_PREC_BF16X3:
      if (c->d_Lbf == nullptr || c->d_Lbf_lo == nullptr) return hipErrorInvalidValue;
      return dispatch_s<FM_BF16X3>(c, nw, c->d_Lbf, c->d_Lbf_lo, phiT, theta, logov, vb, ep);
    case AFQMC_PREC_BF16:
      if (c->d_Lbf == nullptr) return hipErrorInvalidValue;
      return dispatch_s<FM_BF16>(c, nw, c->d_Lbf, nullptr, phiT, theta, logov, vb, ep);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_to_bf16(const afqmc_ctx_s* c, size_t n, const double* src, unsigned short* hi,
                          unsigned short* lo) {
  if (n == 0) return hipSuccess;
  // the shared-slab kernels' A-operand order (lo only for the split form)
  hipLaunchKernelGGL(k_to_bf16_op, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n,
                     c->MT, src, hi, lo);
  return hipGetLastError();
}

hipError_t launch_to_f32_op(const afqmc_ctx_s* c, size_t n, const double* src, float* dst) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32_op, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n,
                     c->MT, src, dst);
  return hipGetLastError();
}
