// Cholesky-vector contraction with reduced-precision matrix-core products and
// FP32 accumulation: FP32, split BF16 and BF16 (AFQMC_PREC_FP32 with a real
// trial, AFQMC_PREC_BF16X3, AFQMC_PREC_BF16).  Same quantities as k_contract
// (Sec. III.A, Eq. local-obs; Eq. shift1):
//   Y_g = Phi_T^T L_g,  f_g^s = Y_g Theta^s,  vb_g = sum_s tr f_g^s,
//   E_p = sum_s tr(Phi_T^T h1' Theta^s) + 1/2 sum_g [vb_g^2 - sum_s tr(f_g^s f_g^s)].
//
// Products: lane (g, c) supplies KV consecutive k values of one row of A and
// one column of B and holds D[4g + r][c].  BF16 (and split BF16): one
// v_mfma_f32_16x16x32_bf16 per 32-wide k block, KV = 8 (k = 32 u + 8 g + j);
// FP32: four v_mfma_f32_16x16x4f32 per 16-wide k block, KV = 4 (k = 16 u +
// 4 g + j, the j-th product on the j-th value).  A and B take the same lane
// layout of k, so the product is the contraction over k whatever order the
// matrix core visits the block in.
// Split BF16: every operand x is carried as x_hi = bf16(x) and
// x_lo = bf16(x - x_hi), and a product a b as a_hi b_hi + a_hi b_lo + a_lo b_hi
// (three products; the dropped a_lo b_lo is below 2^-16 relative), which
// brings the contraction close to FP32 accuracy.  Plain BF16 takes a_hi b_hi.
//
// k_contract_sh: BCP paths per workgroup share each L slab through LDS (one
// path per workgroup: each wavefront loads its own slab operands).  Both
// spins' products f^s = Y Theta^s share the A operand Y, so their B operands
// are packed side by side: packed column q < 2N is column q mod N of spin
// q / N, and a path needs NCP = ceil(2N/16) 16-wide column tiles instead of
// 2 ceil(N/16) (at N = 24 three instead of four).  Per path, NCP wavefronts;
// wavefront w keeps packed column tile w of Theta as B operands in registers
// for the whole loop over g, and Phi_T (all column tiles) as the stage-1 B
// operands.  Stage 1 (Y_g^T = L_g Phi_T) is split over the path's wavefronts by
// row tile, its A operands read from the shared slab.  Y_g^T is rounded to the
// operand form once, as stage 1 leaves it, and stored in LDS in the accumulator
// layout, which is stage 2's A-operand layout (rows 4g .. 4g+3 of a column in
// one lane; in BF16 the two 4-row groups of one operand side by side, so that
// an operand is one 16-byte read); f is transposed through LDS for tr(f f), as
// separate real and imaginary planes whose rows start on 16-byte boundaries.
// Each lane's eight products of FP32 entries of f for tr(f f) are summed in
// FP32 per vector; the traces, the sums over lanes, vb_g^2 and the sums over g
// are FP64.

#include <type_traits>

#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

typedef short sx4 __attribute__((ext_vector_type(4)));
typedef short sx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bfx8 __attribute__((ext_vector_type(8)));

typedef __bf16 bfx2 __attribute__((ext_vector_type(2)));
typedef float fx2 __attribute__((ext_vector_type(2)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet): the host-side
// set-up conversion of the slabs
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// two floats -> two bfloat16 (round to nearest even, one v_cvt_pk_bf16_f32 on
// gfx950), as the low and high halves of a 32-bit word
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(fx2{a, b}, bfx2));
}
__device__ __forceinline__ float bf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ fx4 fx4_zero() {
  fx4 z = {0.f, 0.f, 0.f, 0.f};
  return z;
}

// Operand forms of the contraction.  An operand is what one lane supplies to
// one k block: KV consecutive k values of one row or column, as NP parts of
// type V (FP32: float4; BF16: eight BF16 values).  The Y^T tile is kept in
// LDS in 4-row groups of type V4 (the accumulator layout of stage 1), two of
// which make one BF16 operand.
enum { FM_BF16 = 0, FM_BF16X3 = 1, FM_FP32 = 2 };
template <int FM>
struct Form {
  static constexpr bool X3 = FM == FM_BF16X3;
  static constexpr bool F32 = FM == FM_FP32;
  static constexpr int NP = X3 ? 2 : 1;             // parts: hi (and lo)
  static constexpr int NB = FM == FM_BF16 ? 2 : 1;  // slab buffers (shared slabs)
  static constexpr int KV = F32 ? 4 : 8;            // k values per lane and block
  static constexpr int KB = 4 * KV;                 // k per block
  typedef typename std::conditional<F32, fx4, sx8>::type V;
  typedef typename std::conditional<F32, fx4, sx4>::type V4;
  struct Op {
    V p[NP];
  };
  struct Op4 {
    V4 p[NP];
  };
  // hi (and lo) parts of four values
  __device__ __forceinline__ static Op4 make4(float a, float b, float c, float d) {
    Op4 o;
    if constexpr (F32) {
      o.p[0] = fx4{a, b, c, d};
    } else {
      const unsigned h01 = pk_bf16(a, b), h23 = pk_bf16(c, d);
      o.p[0] = __builtin_bit_cast(sx4, (unsigned long long)h01 | ((unsigned long long)h23 << 32));
      if constexpr (X3) {
        const unsigned l01 = pk_bf16(a - bf_lo(h01), b - bf_hi(h01));
        const unsigned l23 = pk_bf16(c - bf_lo(h23), d - bf_hi(h23));
        o.p[NP - 1] =
            __builtin_bit_cast(sx4, (unsigned long long)l01 | ((unsigned long long)l23 << 32));
      }
    }
    return o;
  }
  __device__ __forceinline__ static Op make(const float (&x)[KV]) {
    Op o;
    if constexpr (F32) {
      o.p[0] = fx4{x[0], x[1], x[2], x[3]};
    } else {
      const Op4 a = make4(x[0], x[1], x[2], x[3]), b = make4(x[4], x[5], x[6], x[7]);
#pragma unroll
      for (int part = 0; part < NP; ++part) o.p[part] = join(a.p[part], b.p[part]);
    }
    return o;
  }
  __device__ __forceinline__ static sx8 join(sx4 a, sx4 b) {
    return sx8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  }
  __device__ __forceinline__ static fx4 mma(const Op& a, const Op& b, fx4 acc) {
    if constexpr (F32) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.p[0][j], b.p[0][j], acc, 0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bfx8, a.p[0]),
                                                    __builtin_bit_cast(bfx8, b.p[0]), acc, 0, 0, 0);
      if constexpr (X3) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bfx8, a.p[0]),
                                                      __builtin_bit_cast(bfx8, b.p[NP - 1]), acc, 0,
                                                      0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bfx8, a.p[NP - 1]),
                                                      __builtin_bit_cast(bfx8, b.p[0]), acc, 0, 0,
                                                      0);
      }
    }
    return acc;
  }
};

// ---------------------------------------------------------------------------
// BCP > 1 paths per workgroup sharing each L slab: the slab goes from global memory
// straight into LDS (global_load_lds), already in A-operand order
// ([row tile][k tile][lane][operand]: consecutive lanes on consecutive words),
// so every L byte crosses L2 once per workgroup instead of once per path.
// Double-buffered slabs load the slab of vector g + 1 during the whole of
// vector g; single buffers load it from the barrier after stage 1 on.  f is
// staged for the transpose in FP32 (its products are FP32); the diagonals are
// staged in FP32 and flush every BFL vectors, four lanes per sum.
constexpr int BFL = 8;  // vectors per flush of the staged diagonals

// Paths per workgroup.  Four when a path has three wavefronts (twelve
// wavefronts put three on every SIMD instead of two on some and one on
// others).  Plain BF16 with four wavefronts per path (N = 25 .. 32): one path,
// with no slab in LDS: each wavefront loads its own stage-1 A operands of
// vector g + 1 from global memory (L2) into registers during vector g, a whole
// vector ahead of their use, and two independent workgroups (about 30 KB of
// LDS each) share a CU, so that one's matrix-core phase overlaps the other's
// conversion, transpose and trace phase.  Two paths per workgroup would share
// the slab through LDS but run every phase of all eight wavefronts in step.
// Otherwise two.
constexpr int bcp_for(int fm, int ncp) { return ncp == 3 ? 4 : (fm == FM_BF16 && ncp == 4) ? 1 : 2; }

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

// FULL: N = 16 NTC (every column tile full, NCP = 2 NTC), so the packed
// columns are the two spins' tiles in order and no column or row is padding.
template <int KT, int NTC, int NCP, int FM, bool FULL, int BCP>
__global__ void __launch_bounds__(64 * NCP * BCP) __attribute__((amdgpu_waves_per_eu(2)))
k_contract_sh(int n_samples, int M, int N, int G, const void* __restrict__ Lop,
               const void* __restrict__ Lop_lo, const double* __restrict__ phiT,
               const double* __restrict__ theta,
               const double* __restrict__ logov, double* __restrict__ vb, double* __restrict__ ep) {
  constexpr int MT = 16 * KT;
  constexpr int NWV = NCP;                     // wavefronts per path
  constexpr int PW = 16 * NCP + 4;             // row length of the staged f (packed columns; 16-byte rows)
  constexpr int NWT = NWV * BCP;               // wavefronts per workgroup
  constexpr int NT = 16 * NTC;
  constexpr int S1MAX = (KT + NWV - 1) / NWV;  // stage-1 row tiles per wavefront
  typedef Form<FM> Fm;
  typedef typename Fm::V V;
  typedef typename Fm::V4 V4;
  typedef typename Fm::Op Op;
  constexpr int KV = Fm::KV, KB = Fm::KB;
  constexpr int KBN = (MT + KB - 1) / KB;      // k blocks (a BF16 block pads an odd KT)
  constexpr int MTP = KB * KBN;                // k extent, padded
  constexpr int SV = KT * KBN * 64;            // operands (V) per slab part
  constexpr int NU = SV * (int)sizeof(V) / 16; // 16-byte units per slab part
  constexpr int NCH = (NU + 63) / 64;          // 1 KB chunks per slab (the last may be partial)
  constexpr int YT = (MTP / 4) * NT;           // 4-row groups (V4) of one Y^T tile part
  // Slabs in LDS when several paths share them: plain BF16 double-buffered (the
  // next slab loads during the whole vector), split BF16 (hi and lo) and FP32
  // (twice the bytes) single, the next slab loading from the barrier after
  // stage 1 on.  One path per workgroup (DIRECT): no slab in LDS; each
  // wavefront loads its stage-1 A operands of vector g + 1 from global memory
  // into registers during vector g.  The Y^T tile is single: it is rewritten
  // only after the barrier that follows every stage-2 read of it.
  constexpr bool DIRECT = BCP == 1;
  constexpr int NB = DIRECT ? 0 : Fm::NB;      // slab buffers
  constexpr int NP = Fm::NP;                   // parts (hi, lo)
  extern __shared__ double smem[];
  V* sL = reinterpret_cast<V*>(smem);                                      // [NB][NP][SV]
  V4* sY = reinterpret_cast<V4*>(sL + NB * NP * SV);                       // [BCP][NP][YT]
  float* sF = reinterpret_cast<float*>(sY + BCP * NP * YT);           // [BCP][re, im][NT][PW]
  float* sD = sF + BCP * 2 * NT * PW;                                   // [BCP][BFL][re, im][NWV*16]
  double* sE = reinterpret_cast<double*>(sD + BCP * BFL * 2 * NWV * 16);  // [BCP][NWV][2]
  double* sT = sE + BCP * NWV * 2;                                         // [NWT][4]

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int pw = wave / NWV, wv = wave % NWV;  // path of the workgroup, wavefront of the path
  // this lane's packed column: spin sp, column n of f^sp (q >= 2N: padding)
  const int q = 16 * wv + c;
  const int NN = FULL ? 16 * NTC : N;
  const bool qok = FULL || q < 2 * N;
  const int sp = FULL ? (wv >= NTC ? 1 : 0) : (q >= N ? 1 : 0);
  const int n = FULL ? 16 * (wv - sp * NTC) + c : q - sp * N;
  const int s = blockIdx.x * BCP + pw;
  const bool valid = s < n_samples;            // every wavefront takes part in the barriers
  const int sc = valid ? s : n_samples - 1;
  const bool active = valid && !__builtin_isinf(logov[2 * sc]);

  // Y^T tile index of 4-row group grp, column col: BF16 keeps groups 2p and 2p + 1 of a
  // column side by side (one stage-2 operand is one 16-byte read)
  auto yidx = [&](int grp, int col) {
    if constexpr (Fm::F32)
      return grp * NT + col;
    else
      return ((grp >> 1) * NT + col) * 2 + (grp & 1);
  };
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
  Op an[DIRECT ? S1MAX : 1][DIRECT ? KBN : 1];  // direct form: the next vector's A operands
  auto load_ops = [&](int slab) {
    if constexpr (DIRECT) {
#pragma unroll
      for (int q = 0; q < S1MAX; ++q) {
        const int tp = wv + NWV * q;
        if (tp < KT)
#pragma unroll
          for (int t = 0; t < KBN; ++t)
#pragma unroll
            for (int part = 0; part < NP; ++part)
              an[q][t].p[part] = reinterpret_cast<const V*>(
                  part ? Lop_lo : Lop)[(size_t)slab * SV + (tp * KBN + t) * 64 + lane];
      }
    }
  };
  if constexpr (DIRECT)
    load_ops(0);
  else
    copy_slab(0, 0);
  if (MTP > MT) {  // the Y^T rows of a padded k block are never written: zero them once
    for (int q = threadIdx.x; q < BCP * NP * ((MTP - MT) / 4) * NT; q += blockDim.x) {
      const int per = ((MTP - MT) / 4) * NT;
      const int tile = q / per, e = q % per;
      V4 z;
#pragma unroll
      for (int i = 0; i < 4; ++i) z[i] = 0;
      sY[(size_t)tile * YT + (MT / 4) * NT + e] = z;
    }
  }

  // B operands (bit-masked unconditional loads): k = KB u + KV g + j
  Op bT[NTC][KBN], th[2][KBN];
#pragma unroll
  for (int t = 0; t < KBN; ++t) {
    float v[NTC][KV], w[2][KV];
#pragma unroll
    for (int j = 0; j < KV; ++j) {
      const int m = KB * t + KV * g + j;
      const bool okm = active && m < M;
      const int mc = min(m, M - 1);
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) {
        const int n = 16 * ct + c;
        const double x = phiT[((size_t)sc * M + mc) * N + min(n, N - 1)];
        v[ct][j] = (float)keep_if(x, okm && n < N);
      }
      const double2 x2 = *reinterpret_cast<const double2*>(
          theta + ((((size_t)sc * 2 + sp) * M + mc) * N + min(n, N - 1)) * 2);
      w[0][j] = (float)keep_if(x2.x, okm && qok);
      w[1][j] = (float)keep_if(x2.y, okm && qok);
    }
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) bT[ct][t] = Fm::make(v[ct]);
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) th[ri][t] = Fm::make(w[ri]);
  }
  if constexpr (!DIRECT) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks of slab 0 are in LDS
  __syncthreads();

  V4* Yb = sY + pw * NP * YT;  // the path's Y^T tile
  float* Fp = sF + (size_t)pw * 2 * NT * PW;
  float* Dp = sD + (size_t)pw * BFL * 2 * NWV * 16;
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
      if (tp < KT)  // an inactive path's operands are zero
#pragma unroll
        for (int t = 0; t < KBN; ++t) {
          Op a;
          if constexpr (DIRECT)
            a = an[q][t];
          else
#pragma unroll
            for (int part = 0; part < NP; ++part) a.p[part] = Ls[part * SV + (tp * KBN + t) * 64 + lane];
#pragma unroll
          for (int ct = 0; ct < NTC; ++ct) y1[q][ct] = Fm::mma(a, bT[ct][t], y1[q][ct]);
        }
    }
    if (DIRECT && gam < G) load_ops(gam + 1);
    // buffer b ^ 1 was last read in stage 1 of the previous vector, before its barriers
    if (NB == 2 && gam < G) copy_slab(gam + 1, b ^ 1);
#pragma unroll
    for (int q = 0; q < S1MAX; ++q) {
      const int tp = wv + NWV * q;
      if (tp < KT) {
        if constexpr (!Fm::F32 && NTC == 2) {
          // lanes of rows g and g ^ 1 (16 apart) trade tiles: row 2h keeps tile 0 and takes
          // its row 2h + 1 partner's tile 0 (the next 4-row group of the same column); row
          // 2h + 1 takes row 2h's tile 1; each lane then stores one whole BF16 operand, the
          // 4-row groups 4 tp + 2h and 4 tp + 2h + 1 of column 16 (g & 1) + c
          const fx4 v0 = y1[q][0], v1 = y1[q][1];
          const typename Fm::Op4 a = Fm::make4(v0[0], v0[1], v0[2], v0[3]);
          const typename Fm::Op4 b = Fm::make4(v1[0], v1[1], v1[2], v1[3]);
          V* Yv = reinterpret_cast<V*>(Yb);
#pragma unroll
          for (int part = 0; part < NP; ++part) {
            const uint2 x = __builtin_bit_cast(uint2, a.p[part]), y = __builtin_bit_cast(uint2, b.p[part]);
            const auto s0 = __builtin_amdgcn_permlane16_swap(x.x, y.x, false, false);
            const auto s1 = __builtin_amdgcn_permlane16_swap(x.y, y.y, false, false);
            const uint4 w = {s0[0], s1[0], s0[1], s1[1]};
            Yv[part * (YT / 2) + (2 * tp + (g >> 1)) * NT + 16 * (g & 1) + c] = __builtin_bit_cast(V, w);
          }
        } else {
#pragma unroll
          for (int ct = 0; ct < NTC; ++ct) {
            const fx4 v = y1[q][ct];
            const typename Fm::Op4 yv = Fm::make4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int part = 0; part < NP; ++part) Yb[part * YT + yidx(4 * tp + g, 16 * ct + c)] = yv.p[part];
          }
        }
      }
    }
    __syncthreads();
    // single buffers: every stage-1 read of this slab is done, the next one can load
    if (NB == 1 && gam < G) copy_slab(gam + 1, 0);
    // stage 2: packed f[it][wv], A[c][KV g + j] = Y^T[KB t + KV g + j][16it + c]: the
    // 4-row group (KB t + KV g) / 4, and for BF16 the next one too
    fx4 f[NTC][2];
#pragma unroll
    for (int it = 0; it < NTC; ++it) f[it][0] = f[it][1] = fx4_zero();
#pragma unroll
    for (int t = 0; t < KBN; ++t)
#pragma unroll
      for (int it = 0; it < NTC; ++it) {
        Op a;
        const int grp = (KB * t + KV * g) / 4;
#pragma unroll
        for (int part = 0; part < NP; ++part) {
          const V4* yg = Yb + part * YT + yidx(grp, 16 * it + c);
          if constexpr (Fm::F32)
            a.p[part] = yg[0];
          else
            a.p[part] = *reinterpret_cast<const V*>(yg);  // groups grp, grp + 1: one 16-byte read
        }
        f[it][0] = Fm::mma(a, th[0][t], f[it][0]);
        f[it][1] = Fm::mma(a, th[1][t], f[it][1]);
      }
    // diagonal of f^sp: the lane's element in row n of its packed column
    float d_re = 0.f, d_im = 0.f;
    if constexpr (FULL) {  // tile (it, it) of spin sp: element (4g + r, c) with 4g + r == c
      const int jd = __builtin_amdgcn_readfirstlane(wv - sp * NTC);  // the same on every lane
#pragma unroll
      for (int it = 0; it < NTC; ++it)
        if (it == jd)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (4 * g + r == c) {
              d_re = f[it][0][r];
              d_im = f[it][1][r];
            }
    } else {
#pragma unroll
      for (int it = 0; it < NTC; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (qok && 16 * it + 4 * g + r == n) {
            d_re = f[it][0][r];
            d_im = f[it][1][r];
          }
    }
    if (gam == G) {  // h1': the path's one-body traces through LDS
      const double t_re = wave_sum((double)d_re), t_im = wave_sum((double)d_im);
      if (lane == 0) {
        sE[wave * 2] = t_re;
        sE[wave * 2 + 1] = t_im;
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
    // stage the packed f[:, q] for the transpose, and the diagonal partials
#pragma unroll
    for (int it = 0; it < NTC; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * it + 4 * g + r;
        Fp[i * PW + q] = f[it][0][r];
        Fp[(NT + i) * PW + q] = f[it][1][r];
      }
    if (g == ((n & 15) >> 2)) {  // the lane group holding row n (0 for padding columns)
      float* d = Dp + (gam % BFL) * 2 * NWV * 16 + wv * 16 + c;
      d[0] = d_re;
      d[NWV * 16] = d_im;
    }
    if constexpr (!DIRECT) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks of the next slab landed
    __syncthreads();
    // this lane's share of tr(f f) for the vector: its eight FP32 products of
    // FP32 entries summed in FP32, the sum over lanes and vectors in FP64
    // f^sp_{i n} f^sp_{n i}: the partner sits in row n, packed column sp N + i
    float xr = 0.f, xi = 0.f;
#pragma unroll
    for (int it = 0; it < NTC; ++it) {
      float pr[4], pi[4];  // f^sp_{n i}, i = 16 it + 4 g + r
      if constexpr (FULL) {  // four consecutive packed columns: one 16-byte read per plane
        const int src = n * PW + sp * NN + 16 * it + 4 * g;
        const fx4 a = *reinterpret_cast<const fx4*>(Fp + src);
        const fx4 b = *reinterpret_cast<const fx4*>(Fp + NT * PW + src);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pr[r] = a[r];
          pi[r] = b[r];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * it + 4 * g + r;
          const bool ok = qok && i < N;
          const int src = ok ? n * PW + sp * NN + i : 0;
          pr[r] = ok ? Fp[src] : 0.f;
          pi[r] = ok ? Fp[NT * PW + src] : 0.f;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float ar = f[it][0][r], ai = f[it][1][r];
        xr = fmaf(ar, pr[r], xr);
        xr = fmaf(-ai, pi[r], xr);
        xi = fmaf(ar, pi[r], xi);
        xi = fmaf(ai, pr[r], xi);
      }
    }
    ex_re += (double)xr;
    ex_im += (double)xi;
    // every BFL vectors: wavefront 0 of each path reduces its staged diagonals to vb_g
    // four lanes per sum (vector gl, part re/im), NWV * 4 staged values each, summed in FP64
    if ((gam % BFL == BFL - 1 || gam == G - 1) && wv == 0 && valid) {
      static_assert(BFL * 2 * 4 == 64, "one lane quad per staged vector and part");
      constexpr int QN = NWV * 16, QL = QN / 4;
      const int cnt = gam % BFL + 1, g0 = gam - gam % BFL;
      const int gl = lane >> 3, part = (lane >> 2) & 1, qq = lane & 3;
      double v = 0.0;
      if (gl < cnt) {
        const fx4* src = reinterpret_cast<const fx4*>(Dp + (gl * 2 + part) * QN + qq * QL);
#pragma unroll
        for (int e = 0; e < QL / 4; ++e) {
          const fx4 x = src[e];
          v += ((double)x[0] + (double)x[1]) + ((double)x[2] + (double)x[3]);
        }
      }
      v += dpp_f64<0xB1>(v);  // quad sum
      v += dpp_f64<0x4E>(v);
      const double vi = __shfl_down(v, 4, 64);
      if ((lane & 7) == 0 && gl < cnt) {
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

// slabs: buffers x parts x bytes per entry = 2 x 1 x 2 (BF16 shared; 1 x 1 x 2
// for one path), 1 x 2 x 2 (split BF16) or 1 x 1 x 4 (FP32), over MT x MTP
// entries (MTP: k padded to whole blocks); Y^T tiles: parts x bytes per 4-row
// group = 1 x 8 (BF16), 2 x 8 (split BF16), 1 x 16 (FP32)
size_t lds_bytes_s(int KT, int NTC, int NCP, int FM, int BCP) {
  const int MT = 16 * KT, NT = 16 * NTC, NWV = NCP;
  const int KB = FM == FM_FP32 ? 16 : 32, MTP = (MT + KB - 1) / KB * KB;
  size_t b = BCP == 1 ? 0 : (size_t)4 * MT * MTP;  // slabs (none with one path per workgroup)
  b += (size_t)BCP * (MTP / 4) * NT * (FM == FM_FP32 ? 16 : FM == FM_BF16X3 ? 16 : 8);  // Y^T tiles
  b += (size_t)BCP * NT * (16 * NCP + 4) * 2 * 4;     // packed f (FP32)
  b += (size_t)BCP * BFL * NWV * 16 * 2 * 4;          // staged diagonals (FP32)
  b += (size_t)BCP * NWV * 2 * 8 + (size_t)BCP * NWV * 4 * 8;
  return b;
}

template <int KT, int NTC, int NCP, int FM, bool FULL, int BCP>
hipError_t launch_sh(const afqmc_ctx_s* c, int nw, const void* L, const void* L_lo,
                      const double* phiT, const double* theta, const double* logov, double* vb,
                      double* ep) {
  const int n = nw * c->P;
  const size_t lds = lds_bytes_s(KT, NTC, NCP, FM, BCP);
  auto kern = k_contract_sh<KT, NTC, NCP, FM, FULL, BCP>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((n + BCP - 1) / BCP), dim3(64 * NCP * BCP), lds, c->stream, n,
                     c->M, c->N, c->G, L, L_lo, phiT, theta, logov, vb, ep);
  return hipGetLastError();
}

template <int FM>
hipError_t dispatch_s(const afqmc_ctx_s* c, int nw, const void* L, const void* L_lo,
                      const double* phiT, const double* theta, const double* logov, double* vb,
                      double* ep) {
  const int KT = c->MT / 16, NTC = (c->N + 15) / 16, NCP = (2 * c->N + 15) / 16;
  const bool full = c->N == 16 * NTC;
#define AFQMC_BS(KK, NC, NP, FL)                           \
  if (KT == KK && NTC == NC && NCP == NP && full == FL) \
    return launch_sh<KK, NC, NP, FM, FL, bcp_for(FM, NP)>(c, nw, L, L_lo, phiT, theta, logov, vb, ep);
#define AFQMC_BS1(KK) AFQMC_BS(KK, 1, 1, false) AFQMC_BS(KK, 1, 2, false) AFQMC_BS(KK, 1, 2, true)
#define AFQMC_BS2(KK) AFQMC_BS(KK, 2, 3, false) AFQMC_BS(KK, 2, 4, false) AFQMC_BS(KK, 2, 4, true)
  AFQMC_BS1(1) AFQMC_BS1(2) AFQMC_BS1(3) AFQMC_BS1(4)
  AFQMC_BS1(5) AFQMC_BS1(6) AFQMC_BS1(7) AFQMC_BS1(8)
  AFQMC_BS2(2) AFQMC_BS2(3) AFQMC_BS2(4) AFQMC_BS2(5) AFQMC_BS2(6) AFQMC_BS2(7) AFQMC_BS2(8)
#undef AFQMC_BS2
#undef AFQMC_BS1
#undef AFQMC_BS
  return hipErrorInvalidValue;
}

// L (double, row-major slabs) -> BF16 in A-operand order [slab][tp][u][g][c][j] =
// L[slab][16 tp + c][32 u + 8 g + j] (0 for k = 32 u + 8 g + j >= MT, the padding of
// the last 32-wide block); with lo given, also lo = bf16(L - hi) in that order.
// n = slabs x MT x MTP.
__global__ void k_to_bf16_op(size_t n, int MT, const double* __restrict__ src,
                             unsigned short* __restrict__ dst, unsigned short* __restrict__ lo) {
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int KBN = (MT + 31) / 32, MTP = 32 * KBN;
  const size_t slab = o / ((size_t)MT * MTP);
  const int r = (int)(o % ((size_t)MT * MTP));
  const int j = r & 7, cc = (r >> 3) & 15, gg = (r >> 7) & 3, u = (r >> 9) % KBN, tp = (r >> 9) / KBN;
  const int k = 32 * u + 8 * gg + j;
  const float x = k < MT ? (float)src[slab * MT * MT + (size_t)(16 * tp + cc) * MT + k] : 0.f;
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
