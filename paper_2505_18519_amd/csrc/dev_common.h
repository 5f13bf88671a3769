// Device helpers shared by the gfx950 kernels of the AFQMC hot path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AFQMC_WAVE 64

// ---------------------------------------------------------------------------
// complex double, interleaved (re, im) in memory

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cmk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
// a / b with Smith's scaling
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return cplx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  } else {
    double r = b.re / b.im, d = b.im + b.re * r;
    return cplx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
  }
}
// 1 / b = conj(b) / |b|^2, b first scaled by a power of two so that |b|^2
// neither overflows nor underflows (one real division; b = 0 gives non-finite
// parts, which the callers never use)
__device__ __forceinline__ cplx crecip(cplx b) {
  const double m = fmax(fabs(b.re), fabs(b.im));
  const int e = (m > 0.0 && isfinite(m)) ? ilogb(m) : 0;
  const double r = ldexp(b.re, -e), i = ldexp(b.im, -e);
  const double d = 1.0 / (r * r + i * i);
  return cplx{ldexp(r * d, -e), ldexp(-i * d, -e)};
}
// a - b * c
__device__ __forceinline__ cplx cfms(cplx a, cplx b, cplx c) {
  return cplx{a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re};
}
// a + b * c
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx c) {
  return cplx{a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re};
}
__device__ __forceinline__ cplx cld(const double* p) { return cplx{p[0], p[1]}; }
__device__ __forceinline__ void cst(double* p, cplx v) {
  p[0] = v.re;
  p[1] = v.im;
}

// ---------------------------------------------------------------------------
// FP64 matrix core: D(16x16) += A(16x4) B(4x16).
// Lane l = 16 g + c (g = l / 16, c = l % 16) supplies A[c][g] and B[g][c] and
// holds D[g + 4 r][c] in element r of the accumulator (rows interleaved by 4).
// A product over m visited as k-steps (t, r) with m = 16 t + 4 r + g therefore
// takes the accumulator of tile t, element r, directly as its next operand.

typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma_f64(double a, double b, dx4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ dx4 dx4_zero() {
  dx4 z = {0.0, 0.0, 0.0, 0.0};
  return z;
}

// FP32 matrix core, v_mfma_f32_16x16x4f32: the same operand lanes as the FP64
// product (A[c][g], B[g][c]) but D[4 g + r][c] in element r.  MM<T> gives both
// forms one interface: a product over m visited as k-steps (t, r) with
// m = 16 t + MM<T>::row(g, r) takes the accumulator of tile t, element r,
// directly as its next operand, in either precision.
typedef float fx4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MM;
template <>
struct MM<double> {
  typedef dx4 acc_t;
  __device__ __forceinline__ static acc_t zero() { return dx4_zero(); }
  __device__ __forceinline__ static acc_t fma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int g, int r) { return g + 4 * r; }
};
template <>
struct MM<float> {
  typedef fx4 acc_t;
  __device__ __forceinline__ static acc_t zero() {
    fx4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
  }
  __device__ __forceinline__ static acc_t fma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int g, int r) { return 4 * g + r; }
};

// ---------------------------------------------------------------------------
// split bfloat16: x carried as hi = bf16(x) and lo = bf16(x - hi), a product as
// hi hi + hi lo + lo hi on v_mfma_f32_16x16x32_bf16.  That product's lane
// (g, c) supplies A[c][8 g + j] and B[8 g + j][c] (j < 8, one 16-byte operand
// each) and holds D[4 g + r][c] in element r, the FP32 layout above.
typedef short tsx8 __attribute__((ext_vector_type(8)));
typedef __bf16 tbfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 tbfx2 __attribute__((ext_vector_type(2)));
typedef float tfx2 __attribute__((ext_vector_type(2)));
// two floats -> two bfloat16 (round to nearest even), low and high halves of a word
__device__ __forceinline__ unsigned tpk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(tfx2{a, b}, tbfx2));
}
__device__ __forceinline__ float tbf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float tbf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ fx4 mfma_bf16x32(tsx8 a, tsx8 b, fx4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(tbfx8, a),
                                                 __builtin_bit_cast(tbfx8, b), acc, 0, 0, 0);
}
// eight values -> their split (hi, lo) operands
__device__ __forceinline__ void split8(const float (&v)[8], tsx8& hi, tsx8& lo) {
  unsigned hw[4], lw[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hw[q] = tpk_bf16(v[2 * q], v[2 * q + 1]);
    lw[q] = tpk_bf16(v[2 * q] - tbf_lo(hw[q]), v[2 * q + 1] - tbf_hi(hw[q]));
  }
  hi = __builtin_bit_cast(tsx8, uint4{hw[0], hw[1], hw[2], hw[3]});
  lo = __builtin_bit_cast(tsx8, uint4{lw[0], lw[1], lw[2], lw[3]});
}
// acc += a b in split form (three products)
__device__ __forceinline__ fx4 mfma_x3(tsx8 ah, tsx8 al, tsx8 bh, tsx8 bl, fx4 acc) {
  acc = mfma_bf16x32(ah, bh, acc);
  acc = mfma_bf16x32(ah, bl, acc);
  return mfma_bf16x32(al, bh, acc);
}

// ---------------------------------------------------------------------------
// wave-wide reductions (64 lanes)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, AFQMC_WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, AFQMC_WAVE));
  return v;
}

// x where ok, +0 elsewhere, as a bit mask: a load whose value feeds this stays
// unconditional (a select or branch would let the compiler move the load into a
// branch and wait for it there)
__device__ __forceinline__ double keep_if(double x, bool ok) {
  return __longlong_as_double(__double_as_longlong(x) & (ok ? ~0LL : 0LL));
}

// value of the lane that DPP control CTRL selects within this lane's 16-lane row
// (0xB1: lane xor 1, 0x4E: lane xor 2, 0x141: mirrored within 8, 0x140: mirrored within 16)
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i32<CTRL>((int)(b & 0xffffffffLL));
  const int hi = dpp_i32<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// wave_max for code where all 64 lanes are active: DPP moves within each 16-lane
// row, then the four row results by readlane; no LDS round trips.  fmax ignores
// NaN and is order-independent, so the result equals wave_max's.
__device__ __forceinline__ double wave_max_full(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
              fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// the same for a float
__device__ __forceinline__ float wave_max_full_f32(float v) {
  v = fmaxf(v, __int_as_float(dpp_i32<0xB1>(__float_as_int(v))));
  v = fmaxf(v, __int_as_float(dpp_i32<0x4E>(__float_as_int(v))));
  v = fmaxf(v, __int_as_float(dpp_i32<0x141>(__float_as_int(v))));
  v = fmaxf(v, __int_as_float(dpp_i32<0x140>(__float_as_int(v))));
  const int b = __float_as_int(v);
  return fmaxf(fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 0)),
                     __int_as_float(__builtin_amdgcn_readlane(b, 16))),
               fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 32)),
                     __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 256-bit counter, 128-bit key.

struct ph4 {
  uint64_t v[4];
};

__device__ __forceinline__ ph4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                             uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  ph4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

__device__ __forceinline__ uint64_t rng_word3(uint32_t tag, uint32_t sweep, uint32_t path) {
  return ((uint64_t)tag << 48) | ((uint64_t)sweep << 24) | (uint64_t)path;
}

__device__ __forceinline__ double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// The four normals of one block: Box-Muller on uniform pairs (words 0,1) and (2,3).
__device__ __forceinline__ void normals4(const ph4& b, double z[4]) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    double ua = u01(b.v[2 * j]), ub = u01(b.v[2 * j + 1]);
    double r = sqrt(-2.0 * log(1.0 - ua));
    double s, c;
    sincos(2.0 * M_PI * ub, &s, &c);
    z[2 * j] = r * c;
    z[2 * j + 1] = r * s;
  }
}

// normal i of stream (seed, walker, step, w3)
__device__ __forceinline__ double stream_normal(uint64_t seed, uint64_t walker, uint64_t step,
                                                uint64_t w3, uint32_t i) {
  ph4 b = philox4x64_10(i >> 2, walker, step, w3, seed, 0);
  const bool hi = (i >> 1) & 1;
  const double ua = u01(hi ? b.v[2] : b.v[0]), ub = u01(hi ? b.v[3] : b.v[1]);
  const double r = sqrt(-2.0 * log(1.0 - ua));
  double sn, cs;
  sincos(2.0 * M_PI * ub, &sn, &cs);
  return r * ((i & 1) ? sn : cs);
}

__device__ __forceinline__ double stream_uniform(uint64_t seed, uint64_t walker, uint64_t step,
                                                 uint64_t w3, uint32_t i) {
  ph4 b = philox4x64_10(i >> 2, walker, step, w3, seed, 0);
  const int j = i & 3;
  const uint64_t x = (j == 0) ? b.v[0] : (j == 1) ? b.v[1] : (j == 2) ? b.v[2] : b.v[3];
  return u01(x);
}

__device__ __forceinline__ double neg_inf() { return -__builtin_huge_val(); }
