// Cholesky-vector contraction for larger systems (M <= 128, N <= 32), in FP64
// or, for complex (multi-slice) trials, with FP32 matrix-core products (real
// trials with FP32 products run k_contract_sh).  Same
// quantities as k_contract (Sec. III.A, Eq. local-obs; Eq. shift1):
//   Y_g = Phi_T^T L_g,  f_g^s = Y_g Theta^s,  vb_g = sum_s tr f_g^s,
//   E_p = sum_s tr(Phi_T^T h1' Theta^s) + 1/2 sum_g [vb_g^2 - sum_s tr(f_g^s f_g^s)].
//
// Layout: one workgroup per path with 2 * NTC wavefronts (NTC = ceil(N/16)),
// compiled per exact number of 16-row tiles KT = M/16 rounded up.  Wavefront
// w = (spin s = w % 2, column tile jt = w / 2) keeps Theta^s[:, jt] in
// registers for the whole loop over g.  Stage 1 (Y_g^T = L_g Phi_T) is split
// over all wavefronts by row tile so every element of L_g is read once per
// path (straight from L2; L is shared by all paths) through one software
// pipeline over all (row tile, k tile) steps whose loads run up to three steps
// ahead and continue into the next vector across the barrier; its result goes
// through LDS.  Stage 2 gives each wavefront f^s[:, jt]; f is transposed through LDS
// for tr(f f).  In the FP32 form Phi_T, Theta and L enter the products as
// FP32 with FP32 accumulation over m; per-vector traces, vb_g^2 and the sums
// over g are carried in FP64.
//
// PR (real trials, FP64 products, 16 < N <= 24): stage 2 takes the vectors in
// pairs.  Y_g^T and Y_g+1^T share one LDS tile as columns [0, N) and [N, 2N),
// so f holds the rows of both vectors in 2N <= 48 = three row tiles instead of
// two tiles per vector (at N = 24 a third fewer stage-2 products); the
// transpose, the staged diagonals and the flushes follow the pair, and the
// h1' slab may close a pair or stand alone.
//
// CT (complex trial determinants of multi-slice trials): stage 1 runs on the
// real M x 2N matrix [Re Phi_T | Im Phi_T], giving Y_a = Re Phi_T^T L_g and
// Y_b = Im Phi_T^T L_g as extra column tiles that share every L operand; stage
// 2 forms Y_a Theta and Y_b Theta and combines f = Y_a Theta + i Y_b Theta.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {


template <typename T>
struct mm;
template <>
struct mm<double> {
  typedef dx4 acc_t;
  __device__ static acc_t zero() { return dx4_zero(); }
  __device__ static acc_t fma(double a, double b, acc_t c) { return mfma_f64(a, b, c); }
  // accumulator element r of lane group g holds row g + 4 r (FP64 16x16x4)
  __device__ static int row(int g, int r) { return g + 4 * r; }
};
template <>
struct mm<float> {
  typedef fx4 acc_t;
  __device__ static acc_t zero() {
    fx4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
  }
  __device__ static acc_t fma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane group g holds row 4 g + r (FP32 16x16x4)
  __device__ static int row(int g, int r) { return 4 * g + r; }
};

template <typename T, int KT, int NTC, bool CT, bool PR>
__global__ void __launch_bounds__(128 * NTC)
k_contract_g(int n_samples, int M, int N, int G, int MT, const T* __restrict__ Lpad,
             const double* __restrict__ phiT, const double* __restrict__ theta,
             const double* __restrict__ logov, double* __restrict__ vb, double* __restrict__ ep) {
  typedef mm<T> MM;
  typedef typename MM::acc_t acc_t;
  constexpr int KTMAX = KT;
  constexpr int NWV = 2 * NTC;             // wavefronts
  constexpr int NT = 16 * NTC;
  constexpr int NTC2 = CT ? 2 * NTC : NTC;     // stage-1 column tiles (re and im parts)
  constexpr int NT2 = 16 * NTC2;
  constexpr int S1MAX = (KT + NWV - 1) / NWV;  // stage-1 row tiles per wavefront
  constexpr int NS = S1MAX * KT;               // stage-1 (row tile, k tile) steps
  // L operand ring: loads run RING - 1 steps ahead; a depth that divides NS
  // leaves the next vector's first steps in slots 0 .. RING - 2 (no moves of
  // registers whose loads are still in flight)
  constexpr int RING = (NS % 4 == 0) ? 4 : (NS % 3 == 0) ? 3 : 2;
  // PR (pairs, real trials with 16 < N <= 24): vectors are taken two at a time in
  // stage 2; the rows of Y_g and Y_g+1 stack to 2N <= 48 = three row tiles
  // instead of two tiles each, and f holds both vectors' rows.
  static_assert(!PR || (!CT && NTC == 2), "pairs: real trials, 16 < N <= 24");
  constexpr int SYW = PR ? 48 : NT2;  // columns of sY
  constexpr int FR = PR ? 48 : NT;    // rows of f staged for the transpose
  constexpr int FT = PR ? 3 : NTC2;   // row tiles of f
  extern __shared__ double smem[];
  T* sY = reinterpret_cast<T*>(smem);                        // [MT][SYW]
  double* sF = smem + (MT * SYW * sizeof(T) + 7) / 8;         // [2][FR][NT+1][2]
  double* sD = sF + 2 * FR * (NT + 1) * 2;                    // [16][NWV*16][2]
  double* sE = sD + 16 * NWV * 16 * 2;                        // [NWV][2]

  const int s = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int sp = wave & 1, jt = wave >> 1;
  if (s >= n_samples) return;  // whole block exits together
  const bool active = !__builtin_isinf(logov[2 * s]);

  // Phi_T B operands for stage 1 (all column tiles), Theta^sp[:, jt] for stage 2.
  // FP32: loads clamped in range and unconditional (masked afterwards), so that they
  // are in flight together rather than one branch and conversion at a time
  // (measured: FP32 47.3 -> 46.9 ms at M = 128; the same form made FP64 slower,
  // 74.5 -> 82.4 ms, so FP64 keeps conditional loads, which it does not serialize)
  T bT[NTC2][KTMAX][4];
  T th[2][KTMAX][4];
#pragma unroll
  for (int t = 0; t < KTMAX; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * t + 4 * r + g;
      const bool okm = active && m < M;
      const int n = 16 * jt + c;
      if constexpr (sizeof(T) == 4) {
        const int mc = min(m, M - 1);
#pragma unroll
        for (int ct = 0; ct < NTC2; ++ct) {
          const int nb = 16 * (ct % NTC) + c, part = ct / NTC;
          const size_t e = ((size_t)s * M + mc) * N + min(nb, N - 1);
          const double x = CT ? phiT[2 * e + part] : phiT[e];
          bT[ct][t][r] = (T)keep_if(x, okm && nb < N);
        }
        const double2 x2 = *reinterpret_cast<const double2*>(
            theta + ((((size_t)s * 2 + sp) * M + mc) * N + min(n, N - 1)) * 2);
        th[0][t][r] = (T)keep_if(x2.x, okm && n < N);
        th[1][t][r] = (T)keep_if(x2.y, okm && n < N);
      } else {
#pragma unroll
        for (int ct = 0; ct < NTC2; ++ct) {
          const int nb = 16 * (ct % NTC) + c, part = ct / NTC;
          const size_t e = ((size_t)s * M + m) * N + nb;
          bT[ct][t][r] = (okm && nb < N) ? (T)(CT ? phiT[2 * e + part] : phiT[e]) : (T)0;
        }
        const double* src = theta + ((((size_t)s * 2 + sp) * M + m) * N + n) * 2;
        th[0][t][r] = (okm && n < N) ? (T)src[0] : (T)0;
        th[1][t][r] = (okm && n < N) ? (T)src[1] : (T)0;
      }
    }

  // stage-1 step k = (q = k / KT, t = k % KT) reads L_g rows 16 t + 4 r + g of
  // column tile tp(q) = wave + NWV q (row tiles past KT are skipped)
  auto lrow = [&](const T* Lg, int k, int r) -> T {
    const int q = k / KT, t = k % KT;
    const int tp = min(wave + NWV * q, KT - 1);  // clamped: in bounds for every wave
    return Lg[(size_t)(16 * t + 4 * r + g) * MT + 16 * tp + c];
  };
  T av[RING][4];
  const size_t slab = (size_t)MT * MT;
#pragma unroll
  for (int k = 0; k < RING - 1; ++k)
    if (k < NS)
#pragma unroll
      for (int r = 0; r < 4; ++r) av[k][r] = lrow(Lpad, k, r);

  double ex_re = 0.0, ex_im = 0.0, vb2_re = 0.0, vb2_im = 0.0, e1_re = 0.0, e1_im = 0.0;
  if (PR) {  // columns 2N .. 47 of sY are never written
    for (int q = threadIdx.x; q < MT * SYW; q += blockDim.x) sY[q] = (T)0;
  }
  for (int gam = 0; gam <= G; ++gam) {
    const int hv = PR ? (gam & 1) : 0;  // half of the pair this vector fills
    const T* Lg = Lpad + (size_t)gam * slab;
    const T* Ln = Lpad + (size_t)min(gam + 1, G) * slab;
    // stage 1: Y^T tiles (tp, ct), one software pipeline over all steps; the
    // first RING - 1 steps of the next vector are issued at the end
    acc_t y1[S1MAX][NTC2];
#pragma unroll
    for (int q = 0; q < S1MAX; ++q)
#pragma unroll
      for (int ct = 0; ct < NTC2; ++ct) y1[q][ct] = MM::zero();
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int q = k / KT, t = k % KT;
      const int kn = k + RING - 1;
      if (kn < NS) {
#pragma unroll
        for (int r = 0; r < 4; ++r) av[kn % RING][r] = lrow(Lg, kn, r);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) av[kn % RING][r] = lrow(Ln, kn - NS, r);
      }
      if (active && wave + NWV * q < KT)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int ct = 0; ct < NTC2; ++ct)
            y1[q][ct] = MM::fma(av[k % RING][r], bT[ct][t][r], y1[q][ct]);
    }
    // the ring now holds the next vector's first steps at slots NS % RING ...;
    // rotate them to slots 0 .. RING - 2 (only when RING does not divide NS)
    if (NS % RING != 0) {
      T tmp[RING][4];
#pragma unroll
      for (int k = 0; k < RING; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) tmp[k][r] = av[(k + NS) % RING][r];
#pragma unroll
      for (int k = 0; k < RING; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) av[k][r] = tmp[k][r];
    }
    // previous vector's (pair's) stage-2 and transpose reads are done; the
    // second vector of a pair writes the other half, which that barrier freed
    if (hv == 0) __syncthreads();
#pragma unroll
    for (int q = 0; q < S1MAX; ++q) {
      const int tp = wave + NWV * q;
      if (tp < KT)
#pragma unroll
        for (int ct = 0; ct < NTC2; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (PR) {
              if (16 * ct + c < N)
                sY[(16 * tp + MM::row(g, r)) * SYW + hv * N + 16 * ct + c] = y1[q][ct][r];
            } else {
              sY[(16 * tp + MM::row(g, r)) * NT2 + 16 * ct + c] = y1[q][ct][r];
            }
          }
    }
    if (PR && hv == 0 && gam < G) continue;  // stage 2 waits for the pair
    __syncthreads();
    // stage 2: f^sp[it][jt] = sum_m Y^T[m][it cols] Theta^sp[m][jt cols]
    acc_t f[FT][2];
#pragma unroll
    for (int it = 0; it < FT; ++it) f[it][0] = f[it][1] = MM::zero();
    if (active) {
#pragma unroll
      for (int t = 0; t < KTMAX; ++t) {
        if (t < KT) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = 16 * t + 4 * r + g;
#pragma unroll
            for (int it = 0; it < FT; ++it) {
              const T a = sY[m * SYW + 16 * it + c];
              f[it][0] = MM::fma(a, th[0][t][r], f[it][0]);
              f[it][1] = MM::fma(a, th[1][t][r], f[it][1]);
            }
          }
        }
      }
    }
    if (CT) {  // f = Y_a Theta + i Y_b Theta
#pragma unroll
      for (int it = 0; it < NTC; ++it) {
        const acc_t fr = f[it][0] - f[it + NTC * (CT ? 1 : 0)][1];
        const acc_t fi = f[it][1] + f[it + NTC * (CT ? 1 : 0)][0];
        f[it][0] = fr;
        f[it][1] = fi;
      }
    }
    if constexpr (PR) {
      // the group holds vectors g0v .. gam (gam = g0v + hv); the h1' slab G may be either
      const int g0v = gam - hv;
      const int j = 16 * jt + c;
      // stage f^sp[:, jt] (both halves) for the transpose
      double* Fs = sF + (size_t)sp * FR * (NT + 1) * 2;
#pragma unroll
      for (int it = 0; it < FT; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * it + MM::row(g, r);
          Fs[(i * (NT + 1) + j) * 2] = (double)f[it][0][r];
          Fs[(i * (NT + 1) + j) * 2 + 1] = (double)f[it][1][r];
        }
      // diagonal element (h N + j, j) of half h, held by one of the four lane groups
      double dr[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
      for (int it = 0; it < FT; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * it + MM::row(g, r);
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (j < N && i == h * N + j) {
              dr[h][0] = (double)f[it][0][r];
              dr[h][1] = (double)f[it][1][r];
            }
        }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h > hv) break;
        const int gv = g0v + h;
        if (gv < G) {  // staged for vb_gv: the sum over the lane groups to lane group 0
          double d0 = dr[h][0], d1 = dr[h][1];
          d0 += __shfl_xor(d0, 16, 64);
          d1 += __shfl_xor(d1, 16, 64);
          d0 += __shfl_xor(d0, 32, 64);
          d1 += __shfl_xor(d1, 32, 64);
          if (g == 0) {
            double* d = sD + ((size_t)(gv & 15) * NWV * 16 + wave * 16 + c) * 2;
            d[0] = d0;
            d[1] = d1;
          }
        } else {  // h1': this wavefront's part of the one-body trace
          const double e0 = wave_sum(dr[h][0]), e1 = wave_sum(dr[h][1]);
          if (lane == 0) {
            sE[wave * 2] = e0;
            sE[wave * 2 + 1] = e1;
          }
        }
      }
      __syncthreads();
      if (gam == G && threadIdx.x == 0) {
        for (int w = 0; w < NWV; ++w) {
          e1_re += sE[w * 2];
          e1_im += sE[w * 2 + 1];
        }
      }
      // exchange of the regular halves: sum_ij f_ij f_ji, f_ji at row h N + j, column i - h N
#pragma unroll
      for (int it = 0; it < FT; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * it + MM::row(g, r);
          const int h = i >= N ? 1 : 0, il = i - h * N;
          if (i < 2 * N && j < N && h <= hv && g0v + h < G) {
            const double* src = Fs + ((h * N + j) * (NT + 1) + il) * 2;
            const double tr_ = src[0], ti_ = src[1];
            const double ar = (double)f[it][0][r], ai = (double)f[it][1][r];
            ex_re += ar * tr_ - ai * ti_;
            ex_im += ar * ti_ + ai * tr_;
          }
        }
      // every 16 vectors: wavefront 0 reduces the staged diagonals to vb_g
      const int glast = min(gam, G - 1);  // last regular vector of the group
      if (g0v < G && ((glast & 15) == 15 || glast == G - 1) && wave == 0) {
        const int cnt = (glast & 15) + 1, gb = glast & ~15;
        const int gl = lane & 15, part = (lane >> 4) & 1;
        double v = 0.0;
        if (lane < 32 && gl < cnt)
          for (int q = 0; q < NWV * 16; ++q) v += sD[((size_t)gl * NWV * 16 + q) * 2 + part];
        const double vi = __shfl_down(v, 16, 64);
        if (lane < 16 && gl < cnt) {
          vb2_re += v * v - vi * vi;
          vb2_im += 2.0 * v * vi;
          double* o = vb + ((size_t)s * G + gb + gl) * 2;
          o[0] = v;
          o[1] = vi;
        }
      }
      if (gam == G) break;
    } else {
      // diagonal of f^sp in tile (jt, jt): element (row(g,r), c) with row == c
      double d_re = 0.0, d_im = 0.0;
#pragma unroll
      for (int it = 0; it < NTC; ++it)
        if (it == jt)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (MM::row(g, r) == c) {
              d_re = (double)f[it][0][r];
              d_im = (double)f[it][1][r];
            }
      if (gam == G) {
        d_re = wave_sum(d_re);
        d_im = wave_sum(d_im);
        // one-body term: both spins' traces, gathered through LDS below
        if (lane == 0) {
          sD[(wave * 16) * 2] = d_re;
          sD[(wave * 16) * 2 + 1] = d_im;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          for (int w = 0; w < NWV; ++w) {
            e1_re += sD[(w * 16) * 2];
            e1_im += sD[(w * 16) * 2 + 1];
          }
        }
        break;
      }
      // stage f^sp[:, jt] in LDS for the transpose, and the diagonal partials
      double* Fs = sF + (size_t)sp * NT * (NT + 1) * 2;
#pragma unroll
      for (int it = 0; it < NTC; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * it + MM::row(g, r), j = 16 * jt + c;
          Fs[(i * (NT + 1) + j) * 2] = (double)f[it][0][r];
          Fs[(i * (NT + 1) + j) * 2 + 1] = (double)f[it][1][r];
        }
      {
        double* d = sD + ((size_t)(gam & 15) * NWV * 16 + wave * 16 + c) * 2;
        if (MM::row(g, 0) == c || MM::row(g, 1) == c || MM::row(g, 2) == c || MM::row(g, 3) == c) {
          d[0] = d_re;
          d[1] = d_im;
        }
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < NTC; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * it + MM::row(g, r), j = 16 * jt + c;
          const double tr_ = Fs[(j * (NT + 1) + i) * 2], ti_ = Fs[(j * (NT + 1) + i) * 2 + 1];
          const double ar = (double)f[it][0][r], ai = (double)f[it][1][r];
          ex_re += ar * tr_ - ai * ti_;
          ex_im += ar * ti_ + ai * tr_;
        }
      // every 16 vectors: wavefront 0 reduces the staged diagonals to vb_g
      if (((gam & 15) == 15 || gam == G - 1) && wave == 0) {
        const int cnt = (gam & 15) + 1, g0 = gam & ~15;
        const int gl = lane & 15, part = (lane >> 4) & 1;
        double v = 0.0;
        if (lane < 32 && gl < cnt)
          for (int q = 0; q < NWV * 16; ++q) v += sD[((size_t)gl * NWV * 16 + q) * 2 + part];
        const double vi = __shfl_down(v, 16, 64);
        if (lane < 16 && gl < cnt) {
          vb2_re += v * v - vi * vi;
          vb2_im += 2.0 * v * vi;
          double* o = vb + ((size_t)s * G + g0 + gl) * 2;
          o[0] = v;
          o[1] = vi;
        }
      }
    }
  }
  // totals: ex from every lane of every wavefront, vb^2 from wavefront 0
  ex_re = wave_sum(ex_re);
  ex_im = wave_sum(ex_im);
  vb2_re = wave_sum(vb2_re);
  vb2_im = wave_sum(vb2_im);
  __syncthreads();
  if (lane == 0) {
    sD[wave * 4 + 0] = ex_re;
    sD[wave * 4 + 1] = ex_im;
    sD[wave * 4 + 2] = vb2_re;
    sD[wave * 4 + 3] = vb2_im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double xr = 0.0, xi = 0.0;
    for (int w = 0; w < NWV; ++w) {
      xr += sD[w * 4 + 0];
      xi += sD[w * 4 + 1];
    }
    const double br = sD[2], bi = sD[3];
    double* o = ep + (size_t)s * 2;
    o[0] = active ? e1_re + 0.5 * br - 0.5 * xr : 0.0;
    o[1] = active ? e1_im + 0.5 * bi - 0.5 * xi : 0.0;
  }
  if (!active)
    for (int q = threadIdx.x; q < 2 * G; q += blockDim.x) vb[(size_t)s * G * 2 + q] = 0.0;
}

// ---------------------------------------------------------------------------
// k_contract_gs: the FP64 contraction of real trials for shapes whose operands
// do not fit in registers (three column tiles, N > 32: a wavefront would need
// Phi_T for every column tile and its Theta^s[:, jt] at once, past the 256
// registers of two wavefronts per SIMD).  Same workgroup layout, LDS tiles and
// tail as k_contract_g, but no operand stays in registers across vectors: every
// stage-1 step loads its L rows and Phi_T entries, every stage-2 step its
// Theta entries, from global memory (L2: Phi_T and Theta are reused by every
// vector of the path, L by every path), one 16-wide k tile ahead of the
// products, and the first tile of the next vector (and of the next stage 2)
// ahead of the barriers.  Stage 1 visits the k tiles in the outer loop so that
// each Phi_T entry feeds the wavefront's row tiles together.
template <int KT, int NTC>
__global__ void __launch_bounds__(128 * NTC)
k_contract_gs(int n_samples, int M, int N, int G, int MT, const double* __restrict__ Lpad,
              const double* __restrict__ phiT, const double* __restrict__ theta,
              const double* __restrict__ logov, double* __restrict__ vb, double* __restrict__ ep) {
  constexpr int NWV = 2 * NTC;                 // wavefronts
  constexpr int NT = 16 * NTC;
  constexpr int S1MAX = (KT + NWV - 1) / NWV;  // stage-1 row tiles per wavefront
  extern __shared__ double smem[];
  double* sY = smem;                           // [MT][NT]
  double* sF = sY + MT * NT;                   // [2][NT][NT+1][2]
  double* sD = sF + 2 * NT * (NT + 1) * 2;     // [16][NWV*16][2]

  const int s = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int sp = wave & 1, jt = wave >> 1;
  if (s >= n_samples) return;  // whole block exits together
  const bool active = !__builtin_isinf(logov[2 * s]);
  const size_t slab = (size_t)MT * MT;

  // stage-1 operands of k tile t: L rows 16 t + 4 r + g of the wavefront's row
  // tiles (clamped in range; tiles past KT are never used) and Phi_T entries
  // (0 outside M x N or for an inactive path)
  struct S1 {
    double a[S1MAX][4];
    double b[NTC][4];
  };
  auto load1 = [&](const double* Lg, int t, S1& o) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * t + 4 * r + g;
#pragma unroll
      for (int q = 0; q < S1MAX; ++q) {
        const int tp = min(wave + NWV * q, KT - 1);
        o.a[q][r] = Lg[(size_t)m * MT + 16 * tp + c];
      }
      // clamped addresses and bit-masked values: unconditional loads, in flight together
      const bool okm = active && m < M;
      const int mc = min(m, M - 1);
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) {
        const int n = 16 * ct + c;
        o.b[ct][r] = keep_if(phiT[((size_t)s * M + mc) * N + min(n, N - 1)], okm && n < N);
      }
    }
  };
  // stage-2 operands of k tile t: Theta^sp[16 t + 4 r + g][16 jt + c]
  struct S2 {
    double re[4], im[4];
  };
  auto load2 = [&](int t, S2& o) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * t + 4 * r + g, n = 16 * jt + c;
      const bool ok = active && m < M && n < N;
      const double2 x = *reinterpret_cast<const double2*>(
          theta + ((((size_t)s * 2 + sp) * M + min(m, M - 1)) * N + min(n, N - 1)) * 2);
      o.re[r] = keep_if(x.x, ok);
      o.im[r] = keep_if(x.y, ok);
    }
  };

  S1 p1[2];
  S2 p2[2];
  load1(Lpad, 0, p1[0]);
  load2(0, p2[0]);
  double ex_re = 0.0, ex_im = 0.0, vb2_re = 0.0, vb2_im = 0.0, e1_re = 0.0, e1_im = 0.0;
  for (int gam = 0; gam <= G; ++gam) {
    const double* Lg = Lpad + (size_t)gam * slab;
    const double* Ln = Lpad + (size_t)min(gam + 1, G) * slab;
    // stage 1: Y^T tiles (tp, ct) of the wavefront's row tiles
    dx4 y1[S1MAX][NTC];
#pragma unroll
    for (int q = 0; q < S1MAX; ++q)
#pragma unroll
      for (int ct = 0; ct < NTC; ++ct) y1[q][ct] = dx4_zero();
    // products of tile t from `cur` while `nxt` receives tile t + 1 (or the
    // next vector's first); tiles in pairs through the two buffers
    auto step1 = [&](int t, S1& cur, S1& nxt) {
      if (t + 1 < KT) load1(Lg, t + 1, nxt);
      else load1(Ln, 0, nxt);
      if (active)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < S1MAX; ++q)
            if (wave + NWV * q < KT)
#pragma unroll
              for (int ct = 0; ct < NTC; ++ct)
                y1[q][ct] = mfma_f64(cur.a[q][r], cur.b[ct][r], y1[q][ct]);
    };
#pragma unroll 1
    for (int t = 0; t + 1 < KT; t += 2) {
      step1(t, p1[0], p1[1]);
      step1(t + 1, p1[1], p1[0]);
    }
    if (KT & 1) {  // the last tile; the next vector's first then moves to slot 0
      step1(KT - 1, p1[0], p1[1]);
      p1[0] = p1[1];
    }
    __syncthreads();  // the previous vector's stage-2 and transpose reads are done
#pragma unroll
    for (int q = 0; q < S1MAX; ++q) {
      const int tp = wave + NWV * q;
      if (tp < KT)
#pragma unroll
        for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) sY[(16 * tp + g + 4 * r) * NT + 16 * ct + c] = y1[q][ct][r];
    }
    __syncthreads();
    // stage 2: f^sp[it][jt] = sum_m Y^T[m][it cols] Theta^sp[m][jt cols]
    dx4 f[NTC][2];
#pragma unroll
    for (int it = 0; it < NTC; ++it) f[it][0] = f[it][1] = dx4_zero();
    auto step2 = [&](int t, S2& cur, S2& nxt) {
      load2(t + 1 < KT ? t + 1 : 0, nxt);  // or the next vector's first tile
      if (active)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = 16 * t + 4 * r + g;
#pragma unroll
          for (int it = 0; it < NTC; ++it) {
            const double a = sY[m * NT + 16 * it + c];
            f[it][0] = mfma_f64(a, cur.re[r], f[it][0]);
            f[it][1] = mfma_f64(a, cur.im[r], f[it][1]);
          }
        }
    };
#pragma unroll 1
    for (int t = 0; t + 1 < KT; t += 2) {
      step2(t, p2[0], p2[1]);
      step2(t + 1, p2[1], p2[0]);
    }
    if (KT & 1) {
      step2(KT - 1, p2[0], p2[1]);
      p2[0] = p2[1];
    }
    // diagonal of f^sp in tile (jt, jt): element (g + 4 r, c) with g + 4 r == c
    double d_re = 0.0, d_im = 0.0;
#pragma unroll
    for (int it = 0; it < NTC; ++it)
      if (it == jt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (g + 4 * r == c) {
            d_re = f[it][0][r];
            d_im = f[it][1][r];
          }
    if (gam == G) {
      d_re = wave_sum(d_re);
      d_im = wave_sum(d_im);
      // one-body term: both spins' traces, gathered through LDS below
      if (lane == 0) {
        sD[(wave * 16) * 2] = d_re;
        sD[(wave * 16) * 2 + 1] = d_im;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int w = 0; w < NWV; ++w) {
          e1_re += sD[(w * 16) * 2];
          e1_im += sD[(w * 16) * 2 + 1];
        }
      }
      break;
    }
    // stage f^sp[:, jt] in LDS for the transpose, and the diagonal partials
    double* Fs = sF + (size_t)sp * NT * (NT + 1) * 2;
#pragma unroll
    for (int it = 0; it < NTC; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * it + g + 4 * r, j = 16 * jt + c;
        Fs[(i * (NT + 1) + j) * 2] = f[it][0][r];
        Fs[(i * (NT + 1) + j) * 2 + 1] = f[it][1][r];
      }
    if ((c & 3) == g) {  // the lane group holding row c of the diagonal tile
      double* d = sD + ((size_t)(gam & 15) * NWV * 16 + wave * 16 + c) * 2;
      d[0] = d_re;
      d[1] = d_im;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NTC; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * it + g + 4 * r, j = 16 * jt + c;
        const double tr_ = Fs[(j * (NT + 1) + i) * 2], ti_ = Fs[(j * (NT + 1) + i) * 2 + 1];
        const double ar = f[it][0][r], ai = f[it][1][r];
        ex_re += ar * tr_ - ai * ti_;
        ex_im += ar * ti_ + ai * tr_;
      }
    // every 16 vectors: wavefront 0 reduces the staged diagonals to vb_g
    if (((gam & 15) == 15 || gam == G - 1) && wave == 0) {
      const int cnt = (gam & 15) + 1, g0 = gam & ~15;
      const int gl = lane & 15, part = (lane >> 4) & 1;
      double v = 0.0;
      if (lane < 32 && gl < cnt)
        for (int q = 0; q < NWV * 16; ++q) v += sD[((size_t)gl * NWV * 16 + q) * 2 + part];
      const double vi = __shfl_down(v, 16, 64);
      if (lane < 16 && gl < cnt) {
        vb2_re += v * v - vi * vi;
        vb2_im += 2.0 * v * vi;
        double* o = vb + ((size_t)s * G + g0 + gl) * 2;
        o[0] = v;
        o[1] = vi;
      }
    }
  }
  // totals: ex from every lane of every wavefront, vb^2 from wavefront 0
  ex_re = wave_sum(ex_re);
  ex_im = wave_sum(ex_im);
  vb2_re = wave_sum(vb2_re);
  vb2_im = wave_sum(vb2_im);
  __syncthreads();
  if (lane == 0) {
    sD[wave * 4 + 0] = ex_re;
    sD[wave * 4 + 1] = ex_im;
    sD[wave * 4 + 2] = vb2_re;
    sD[wave * 4 + 3] = vb2_im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double xr = 0.0, xi = 0.0;
    for (int w = 0; w < NWV; ++w) {
      xr += sD[w * 4 + 0];
      xi += sD[w * 4 + 1];
    }
    const double br = sD[2], bi = sD[3];
    double* o = ep + (size_t)s * 2;
    o[0] = active ? e1_re + 0.5 * br - 0.5 * xr : 0.0;
    o[1] = active ? e1_im + 0.5 * bi - 0.5 * xi : 0.0;
  }
  if (!active)
    for (int q = threadIdx.x; q < 2 * G; q += blockDim.x) vb[(size_t)s * G * 2 + q] = 0.0;
}

template <int KT, int NTC>
hipError_t launch_gs(const afqmc_ctx_s* c, int nw, const double* L, const double* phiT,
                     const double* theta, const double* logov, double* vb, double* ep) {
  const int n = nw * c->P;
  const int NT = 16 * NTC, NWV = 2 * NTC;
  const size_t lds = ((size_t)c->MT * NT + (size_t)2 * NT * (NT + 1) * 2 +
                      (size_t)16 * NWV * 16 * 2) * sizeof(double);
  auto kern = k_contract_gs<KT, NTC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n), dim3(128 * NTC), lds, c->stream, n, c->M, c->N, c->G, c->MT,
                     L, phiT, theta, logov, vb, ep);
  return hipGetLastError();
}

size_t lds_bytes(int MT, int NTC, size_t tsize, bool ct, bool pr) {
  const int NT = 16 * NTC, NWV = 2 * NTC;
  const int syw = pr ? 48 : NT * (ct ? 2 : 1), fr = pr ? 48 : NT;
  size_t b = ((size_t)MT * syw * tsize + 7) / 8 * 8;
  b += (size_t)2 * fr * (NT + 1) * 2 * 8;
  b += (size_t)16 * NWV * 16 * 2 * 8;
  b += (size_t)NWV * 2 * 8;
  return b;
}

template <typename T, int KT, int NTC, bool CT, bool PR = false>
hipError_t launch_g(const afqmc_ctx_s* c, int nw, const T* L, const double* phiT,
                    const double* theta, const double* logov, double* vb, double* ep) {
  const int n = nw * c->P;
  const size_t lds = lds_bytes(c->MT, NTC, sizeof(T), CT, PR);
  auto kern = k_contract_g<T, KT, NTC, CT, PR>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n), dim3(128 * NTC), lds, c->stream, n, c->M, c->N, c->G, c->MT,
                     L, phiT, theta, logov, vb, ep);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch(const afqmc_ctx_s* c, int nw, const T* L, const double* phiT,
                    const double* theta, const double* logov, double* vb, double* ep) {
  const int KT = c->MT / 16, NTC = (c->N + 15) / 16;
  if (c->ctrial) {  // complex trials: KT * NTC <= 8 (register budget of the doubled B operands)
#define AFQMC_GC(KK, NC)                                                                  \
  if (KT == KK && NTC == NC) return launch_g<T, KK, NC, true>(c, nw, L, phiT, theta, logov, vb, ep);
    AFQMC_GC(1, 1) AFQMC_GC(2, 1) AFQMC_GC(3, 1) AFQMC_GC(4, 1)
    AFQMC_GC(5, 1) AFQMC_GC(6, 1) AFQMC_GC(7, 1) AFQMC_GC(8, 1)
    AFQMC_GC(2, 2) AFQMC_GC(3, 2) AFQMC_GC(4, 2)
#undef AFQMC_GC
    return hipErrorInvalidValue;
  }
  if constexpr (sizeof(T) == 8) {  // real trials with FP32 products run k_contract_sh
    // operands streamed from L2: three column tiles always, fewer when asked for
    if (NTC == 3 || c->contract_variant == 1) {
#define AFQMC_GS(KK, NC) \
  if (KT == KK && NTC == NC) return launch_gs<KK, NC>(c, nw, L, phiT, theta, logov, vb, ep);
#define AFQMC_GSK(KK) AFQMC_GS(KK, 1) AFQMC_GS(KK, 2) AFQMC_GS(KK, 3)
      AFQMC_GSK(1) AFQMC_GSK(2) AFQMC_GSK(3) AFQMC_GSK(4) AFQMC_GSK(5)
      AFQMC_GSK(6) AFQMC_GSK(7) AFQMC_GSK(8) AFQMC_GSK(9) AFQMC_GSK(10)
#undef AFQMC_GSK
#undef AFQMC_GS
      return hipErrorInvalidValue;
    }
    // 16 < N <= 24: vectors in pairs (2N rows in three tiles; measured at M = 96,
    // N = 24: 86.9 -> 82.3 ms); the kernel spills at KT = 8, which keeps one vector
    // at a time
    if (NTC == 2 && c->N <= 24 && KT <= 7) {
#define AFQMC_GP(KK)                                                                       \
  if (KT == KK) return launch_g<T, KK, 2, false, true>(c, nw, L, phiT, theta, logov, vb, ep);
      AFQMC_GP(2) AFQMC_GP(3) AFQMC_GP(4) AFQMC_GP(5) AFQMC_GP(6) AFQMC_GP(7)
#undef AFQMC_GP
      return hipErrorInvalidValue;
    }
#define AFQMC_G(KK, NC)                                                            \
  if (KT == KK && NTC == NC) return launch_g<T, KK, NC, false>(c, nw, L, phiT, theta, logov, vb, ep);
    AFQMC_G(1, 1) AFQMC_G(2, 1) AFQMC_G(3, 1) AFQMC_G(4, 1)
    AFQMC_G(5, 1) AFQMC_G(6, 1) AFQMC_G(7, 1) AFQMC_G(8, 1)
    AFQMC_G(2, 2) AFQMC_G(3, 2) AFQMC_G(4, 2)
    AFQMC_G(5, 2) AFQMC_G(6, 2) AFQMC_G(7, 2) AFQMC_G(8, 2)
    AFQMC_G(9, 1) AFQMC_G(10, 1) AFQMC_G(9, 2) AFQMC_G(10, 2)
#undef AFQMC_G
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_contract_g(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                             const double* logov, double* vb, double* ep) {
  if (nw <= 0) return hipSuccess;
  if (c->precision == AFQMC_PREC_FP32)  // complex trials (real ones run k_contract_sh)
    return dispatch<float>(c, nw, c->d_Lpad32, phiT, theta, logov, vb, ep);
  return dispatch<double>(c, nw, c->d_Lpad, phiT, theta, logov, vb, ep);
}
