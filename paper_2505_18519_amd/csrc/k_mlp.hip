// Learned Metropolis proposal: the perceptron's forward pass, backward pass,
// weight gradients and Adam step on the matrix cores.  This is an extension
// beside the prior proposal of Sec. III.A (leapfrog step 2) and App. B; the
// acceptance that keeps the chains exact lives in k_metropolis.hip.
//
// Network: z = [Re diag G (M), y (K)] -> h1 = tanh(z W1 + b1) -> h2 =
// tanh(h1 W2 + b2) -> o = h2 W3 + b3, mu = y + o[0:K] (a displacement from
// the input state), lv = 4 tanh(o[K:2K] / 4), q(y' | z) = N(mu, diag exp(lv)).
// The proposal is N(mu, 2 exp(lv)): trained as the denoiser of the random-walk
// moves, mu - y is the drift s^2 grad log p of a Langevin step whose noise
// variance is 2 s^2.  H = 256 hidden units.  The forward pass stores o[0:K]
// and lv; the kernels that use mu add the input state in FP64.
//
// Data layout.
//  * One wavefront owns 16 samples (the columns of every 16x16 product) and
//    keeps a layer's activations in registers as the next product's operand:
//    lane (g, c) holds units 16t + 4g + j (j = 0..3) of sample c, which is
//    both what a product leaves in its accumulator (D[4g + r][c]) and what
//    the next product takes as its B operand for k tile t.  The weights
//    stream from L2 as the A operand: W^T rows for the forward pass, W rows
//    for the backward pass, four consecutive k values per lane.
//  * FP32 products: four v_mfma_f32_16x16x4f32, product r taking j = r from
//    every lane group.  BF16 products: one v_mfma_f32_16x16x16bf16_1k.
//    Accumulation is FP32 in both; tanh, biases and the loss terms are FP32 /
//    FP64 scalar code.
//  * Training stores the layer inputs and the back-propagated errors
//    feature-major (XT[feature][sample]), so that the weight gradients
//    C = X^T Y (a sum over samples) read four consecutive samples per lane.
//    The bias gradient is the extra row of C for a constant input 1.  Each
//    chunk of 512 samples writes its own partial C; the Adam kernel adds the
//    partials in a fixed order, so training is deterministic.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

constexpr int H = AFQMC_MLP_HIDDEN;
constexpr int HT = H / 16;
constexpr float LVMAX = 4.0f;

typedef short sx4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

// float -> bfloat16, round to nearest even on the upper half (quiet NaN kept)
__device__ __forceinline__ bf16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((unsigned)b << 16); }

template <class T>
struct MT;

template <>
struct MT<float> {
  typedef fx4 op;
  static __device__ __forceinline__ op load(const float* p) {
    return *reinterpret_cast<const fx4*>(p);
  }
  static __device__ __forceinline__ op make(float a, float b, float c, float d) {
    op v = {a, b, c, d};
    return v;
  }
  static __device__ __forceinline__ op zero() { return make(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ fx4 mma(const op& a, const op& b, fx4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
    return acc;
  }
  static __device__ __forceinline__ float conv(float v) { return v; }
  static __device__ __forceinline__ float tof(float v) { return v; }
};

template <>
struct MT<bf16_t> {
  typedef sx4 op;
  static __device__ __forceinline__ op load(const bf16_t* p) {
    return *reinterpret_cast<const sx4*>(p);
  }
  static __device__ __forceinline__ op make(float a, float b, float c, float d) {
    op v = {(short)f2bf(a), (short)f2bf(b), (short)f2bf(c), (short)f2bf(d)};
    return v;
  }
  static __device__ __forceinline__ op zero() {
    op v = {0, 0, 0, 0};
    return v;
  }
  static __device__ __forceinline__ fx4 mma(const op& a, const op& b, fx4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  static __device__ __forceinline__ bf16_t conv(float v) { return f2bf(v); }
  static __device__ __forceinline__ float tof(bf16_t v) { return bf2f(v); }
};

__device__ __forceinline__ fx4 fx4_zero() {
  fx4 z = {0.f, 0.f, 0.f, 0.f};
  return z;
}

// ---------------------------------------------------------------------------
// Forward pass.  out[s][0:K] = o[0:K] (mu - y), out[s][K:2K] = lv (FP32, row
// stride Op).
// TRAIN also stores zT [D][Sp], h1T [H][Sp], h2T [H][Sp] in the product type.

template <class T, bool TRAIN>
__global__ void __launch_bounds__(256)
k_mlp_fwd(int n, int Sp, int M, int K, int D, int Dp, int O, int Op,
          const double* __restrict__ gd, const double* __restrict__ y, const T* __restrict__ w1t,
          const T* __restrict__ w2t, const T* __restrict__ w3t, const float* __restrict__ b1,
          const float* __restrict__ b2, const float* __restrict__ b3, float* __restrict__ out,
          T* __restrict__ zT, T* __restrict__ h1T, T* __restrict__ h2T) {
  typedef MT<T> tr;
  typedef typename tr::op op;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int s0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (s0 >= Sp) return;  // no barriers below
  const int s = s0 + c;
  const bool oks = s < n;
  const int DQ = Dp >> 4;

  op xin[HT];
#pragma unroll
  for (int q = 0; q < HT; ++q) {
    xin[q] = tr::zero();
    if (q < DQ) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * q + 4 * g + j;
        double x = 0.0;
        if (oks && k < M) x = gd[(size_t)s * M + k];
        else if (oks && k < D) x = y[(size_t)s * K + (k - M)];
        v[j] = (float)x;
      }
      xin[q] = tr::make(v[0], v[1], v[2], v[3]);
      if (TRAIN) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 16 * q + 4 * g + j;
          if (k < D) zT[(size_t)k * Sp + s] = tr::conv(v[j]);
        }
      }
    }
  }
  // layer 1
  op hid[HT];
#pragma unroll
  for (int t = 0; t < HT; ++t) {
    fx4 acc = fx4_zero();
    const T* wr = w1t + (size_t)(16 * t + c) * Dp + 4 * g;
#pragma unroll
    for (int q = 0; q < HT; ++q)
      if (q < DQ) acc = tr::mma(tr::load(wr + 16 * q), xin[q], acc);
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * t + 4 * g + r;
      v[r] = tanhf(acc[r] + b1[j]);
    }
    hid[t] = tr::make(v[0], v[1], v[2], v[3]);
    if (TRAIN) {
#pragma unroll
      for (int r = 0; r < 4; ++r) h1T[(size_t)(16 * t + 4 * g + r) * Sp + s] = tr::conv(v[r]);
    }
  }
  // layer 2 (reuses xin for h2)
#pragma unroll
  for (int t = 0; t < HT; ++t) {
    fx4 acc = fx4_zero();
    const T* wr = w2t + (size_t)(16 * t + c) * H + 4 * g;
#pragma unroll
    for (int q = 0; q < HT; ++q) acc = tr::mma(tr::load(wr + 16 * q), hid[q], acc);
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * t + 4 * g + r;
      v[r] = tanhf(acc[r] + b2[j]);
    }
    xin[t] = tr::make(v[0], v[1], v[2], v[3]);
    if (TRAIN) {
#pragma unroll
      for (int r = 0; r < 4; ++r) h2T[(size_t)(16 * t + 4 * g + r) * Sp + s] = tr::conv(v[r]);
    }
  }
  // output layer
  const int OQ = Op >> 4;
#pragma unroll
  for (int t = 0; t < HT; ++t) {
    if (t >= OQ) break;
    fx4 acc = fx4_zero();
    const T* wr = w3t + (size_t)(16 * t + c) * H + 4 * g;
#pragma unroll
    for (int q = 0; q < HT; ++q) acc = tr::mma(tr::load(wr + 16 * q), xin[q], acc);
    fx4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = 16 * t + 4 * g + r;
      float v = 0.f;
      if (u < O) {
        v = acc[r] + b3[u];
        if (u >= K) v = LVMAX * tanhf(v / LVMAX);
      }
      o[r] = v;
    }
    *reinterpret_cast<fx4*>(out + (size_t)s * Op + 16 * t + 4 * g) = o;
  }
}

// ---------------------------------------------------------------------------
// Proposal y' = mu + sqrt(2 exp(lv)) eta (eta: stream PROPOSAL), mu = y + o,
// and log q(y' | z).  One 64-lane workgroup per path; lane = block of four
// hidden variables.

__global__ void __launch_bounds__(64)
k_mlp_propose(int P, int K, int Op, const float* __restrict__ out, const double* __restrict__ y,
              uint64_t seed, uint64_t step, const uint64_t* __restrict__ dstep, int sweep,
              double* __restrict__ ytry, double* __restrict__ lqf) {
  const int wp = blockIdx.x, lane = threadIdx.x;
  if (dstep != nullptr) step = *dstep;
  const int w = wp / P, p = wp % P;
  const double hl2pi = 0.5 * log(2.0 * M_PI);
  double lq = 0.0;
  for (int kb = lane; 4 * kb < K; kb += 64) {
    const ph4 b = philox4x64_10((uint64_t)kb, (uint64_t)w, step,
                                rng_word3(AFQMC_TAG_PROPOSAL, (uint32_t)sweep, (uint32_t)p), seed, 0);
    double z[4];
    normals4(b, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * kb + j;
      if (k < K) {
        const double mu = y[(size_t)wp * K + k] + (double)out[(size_t)wp * Op + k];
        const double lv = out[(size_t)wp * Op + K + k] + M_LN2;   // proposal variance
        const double yv = mu + exp(0.5 * lv) * z[j];
        ytry[(size_t)wp * K + k] = yv;
        const double d = yv - mu;
        lq += -0.5 * lv - 0.5 * d * d * exp(-lv) - hl2pi;
      }
    }
  }
  lq = wave_sum(lq);
  if (lane == 0) lqf[wp] = lq;
}

// lqx = log q(y | z') - log q(y' | z) - |y'|^2 / 2 + |y|^2 / 2 (log of the
// proposal and prior ratios in the Metropolis-Hastings acceptance); the
// reverse mean is y' + o(z')
__global__ void __launch_bounds__(64)
k_mlp_reverse(int K, int Op, const float* __restrict__ outR, const double* __restrict__ y,
              const double* __restrict__ ytry, const double* __restrict__ lqf,
              double* __restrict__ lqx) {
  const int wp = blockIdx.x, lane = threadIdx.x;
  const double hl2pi = 0.5 * log(2.0 * M_PI);
  double lq = 0.0, nn = 0.0, no = 0.0;
  for (int k = lane; k < K; k += 64) {
    const double yo = y[(size_t)wp * K + k], yn = ytry[(size_t)wp * K + k];
    const double mu = yn + (double)outR[(size_t)wp * Op + k];
    const double lv = outR[(size_t)wp * Op + K + k] + M_LN2;
    const double d = yo - mu;
    lq += -0.5 * lv - 0.5 * d * d * exp(-lv) - hl2pi;
    nn += yn * yn;
    no += yo * yo;
  }
  lq = wave_sum(lq);
  nn = wave_sum(nn);
  no = wave_sum(no);
  if (lane == 0) lqx[wp] = lq - lqf[wp] - 0.5 * nn + 0.5 * no;
}

// ---------------------------------------------------------------------------
// Backward pass for the loss sum_s mask_s (-log q(ytgt_s | z_s)) (the mean's
// 1/count is applied in the Adam kernel); yin = the y block of z_s, so that
// mu = yin + o; mask NULL = every row.  Writes dOT [Op][Sp], dh2T [H][Sp],
// dh1T [H][Sp] (errors at the pre-activations) and nlq[s] = -log q (masked).

template <class T>
__global__ void __launch_bounds__(256)
k_mlp_bwd(int n, int Sp, int K, int O, int Op, const float* __restrict__ out,
          const double* __restrict__ yin, const double* __restrict__ ytgt,
          const int* __restrict__ mask, const T* __restrict__ w2c,
          const T* __restrict__ w3c, const T* __restrict__ h1T, const T* __restrict__ h2T,
          T* __restrict__ dOT, T* __restrict__ dh2T, T* __restrict__ dh1T,
          double* __restrict__ nlq) {
  typedef MT<T> tr;
  typedef typename tr::op op;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const int s0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (s0 >= Sp) return;
  const int s = s0 + c;
  const bool on = s < n && (mask == nullptr || mask[s] != 0);
  const int OQ = Op >> 4;
  const double hl2pi = 0.5 * log(2.0 * M_PI);

  op dop[HT];
  double lsum = 0.0;
#pragma unroll
  for (int q = 0; q < HT; ++q) {
    dop[q] = tr::zero();
    if (q < OQ) {
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 16 * q + 4 * g + j;
        double gv = 0.0;
        if (on && u < O) {
          const int k = u < K ? u : u - K;
          const double mu = yin[(size_t)s * K + k] + (double)out[(size_t)s * Op + k];
          const double lv = out[(size_t)s * Op + K + k];
          const double d = ytgt[(size_t)s * K + k] - mu, e = exp(-lv);
          if (u < K) {
            gv = -d * e;
            lsum += 0.5 * lv + 0.5 * d * d * e + hl2pi;
          } else {
            const double th = lv / (double)LVMAX;
            gv = (0.5 - 0.5 * d * d * e) * (1.0 - th * th);
          }
        }
        v[j] = (float)gv;
        dOT[(size_t)u * Sp + s] = tr::conv(v[j]);
      }
      dop[q] = tr::make(v[0], v[1], v[2], v[3]);
    }
  }
  // errors at the second hidden layer
  op d2[HT];
#pragma unroll
  for (int t = 0; t < HT; ++t) {
    fx4 acc = fx4_zero();
    const T* wr = w3c + (size_t)(16 * t + c) * Op + 4 * g;
#pragma unroll
    for (int q = 0; q < HT; ++q)
      if (q < OQ) acc = tr::mma(tr::load(wr + 16 * q), dop[q], acc);
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const size_t at = (size_t)(16 * t + 4 * g + r) * Sp + s;
      const float h = tr::tof(h2T[at]);
      v[r] = acc[r] * (1.f - h * h);
      dh2T[at] = tr::conv(v[r]);
    }
    d2[t] = tr::make(v[0], v[1], v[2], v[3]);
  }
  // errors at the first hidden layer
#pragma unroll
  for (int t = 0; t < HT; ++t) {
    fx4 acc = fx4_zero();
    const T* wr = w2c + (size_t)(16 * t + c) * H + 4 * g;
#pragma unroll
    for (int q = 0; q < HT; ++q) acc = tr::mma(tr::load(wr + 16 * q), d2[q], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const size_t at = (size_t)(16 * t + 4 * g + r) * Sp + s;
      const float h = tr::tof(h1T[at]);
      dh1T[at] = tr::conv(acc[r] * (1.f - h * h));
    }
  }
  lsum += __shfl_xor(lsum, 16, 64);
  lsum += __shfl_xor(lsum, 32, 64);
  if (g == 0) nlq[s] = lsum;
}

// ---------------------------------------------------------------------------
// Weight gradients C_l = [X_l; 1]^T Y_l over one chunk of samples, for the
// three layers at once: (zT, dh1T), (h1T, dh2T), (h2T, dOT).  A wavefront
// computes a 32 x 32 block of one C_l; row `in` of C_l is the bias gradient.
// part[split][flat parameter index].

struct wg_layer {
  const void* X;
  const void* Y;
  int in, out, bc, nb;
  int64_t off;
};
struct wg_args {
  wg_layer l[3];
};

template <class T>
__global__ void __launch_bounds__(256)
k_mlp_wgrad(int Sp, wg_args a, float* __restrict__ part, int64_t np) {
  typedef MT<T> tr;
  typedef typename tr::op op;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  int li = 0;
  if (b >= a.l[0].nb) {
    b -= a.l[0].nb;
    li = 1;
    if (b >= a.l[1].nb) {
      b -= a.l[1].nb;
      li = 2;
      if (b >= a.l[2].nb) return;  // no barriers below
    }
  }
  const wg_layer L = (li == 0) ? a.l[0] : (li == 1) ? a.l[1] : a.l[2];
  const T* X = static_cast<const T*>(L.X);
  const T* Y = static_cast<const T*>(L.Y);
  const int i0 = 32 * (b / L.bc), j0 = 32 * (b % L.bc);
  const int sb = blockIdx.y * MLP_CHUNK, se = min(Sp, sb + MLP_CHUNK);

  const T* xr[2];
  const T* yr[2];
  int xsel[2];  // 0 load, 1 ones (bias row), 2 zeros
  bool yok[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = i0 + 16 * q + c, j = j0 + 16 * q + c;
    xsel[q] = (i < L.in) ? 0 : (i == L.in ? 1 : 2);
    xr[q] = X + (size_t)min(i, L.in - 1) * Sp + 4 * g;
    yok[q] = j < L.out;
    yr[q] = Y + (size_t)min(j, L.out - 1) * Sp + 4 * g;
  }
  const op ones = tr::make(1.f, 1.f, 1.f, 1.f), zero = tr::zero();
  fx4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = fx4_zero();
#pragma unroll 2
  for (int s = sb; s < se; s += 16) {
    op xa[2], yb[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const op lx = tr::load(xr[q] + s);
      xa[q] = xsel[q] == 0 ? lx : (xsel[q] == 1 ? ones : zero);
      const op ly = tr::load(yr[q] + s);
      yb[q] = yok[q] ? ly : zero;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = tr::mma(xa[p], yb[q], acc[p][q]);
  }
  float* dst = part + (size_t)blockIdx.y * np + L.off;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 16 * p + 4 * g + r, j = j0 + 16 * q + c;
        if (i <= L.in && j < L.out) dst[(size_t)i * L.out + j] = acc[p][q][r];
      }
}

// count of masked rows, mean loss, 1/count; Adam step counter += (count > 0)
__global__ void __launch_bounds__(256)
k_mlp_reduce(int n, const int* __restrict__ mask, const double* __restrict__ nlq,
             double* __restrict__ scal, int* __restrict__ tstep, double* __restrict__ loss) {
  __shared__ double s_c[256], s_l[256];
  const int tid = threadIdx.x;
  double cn = 0.0, ls = 0.0;
  for (int s = tid; s < n; s += 256)
    if (mask == nullptr || mask[s] != 0) {
      cn += 1.0;
      ls += nlq[s];
    }
  s_c[tid] = cn;
  s_l[tid] = ls;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) {
      s_c[tid] += s_c[tid + h];
      s_l[tid] += s_l[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double cnt = s_c[0];
    const double mean = cnt > 0.0 ? s_l[0] / cnt : 0.0;
    scal[0] = cnt;
    scal[1] = mean;
    scal[2] = cnt > 0.0 ? 1.0 / cnt : 0.0;
    if (cnt > 0.0) tstep[0] = tstep[0] + 1;
    if (loss != nullptr) loss[0] = mean;
  }
}

// ---------------------------------------------------------------------------
// Parameters: FP32 master copy, and the product-type copies W1^T, W2^T, W3^T
// (forward) and W2, W3 (backward).

struct mlp_geom {
  int D, Dp, O, Op;
  int64_t np, ob1, oW2, ob2, oW3, ob3;
};

template <class T>
__device__ __forceinline__ void write_copies(const mlp_geom& m, int64_t p, float w, T* w1t, T* w2t,
                                             T* w3t, T* w2c, T* w3c) {
  typedef MT<T> tr;
  if (p < m.ob1) {
    const int i = (int)(p / H), j = (int)(p % H);
    w1t[(size_t)j * m.Dp + i] = tr::conv(w);
  } else if (p >= m.oW2 && p < m.ob2) {
    const int64_t q = p - m.oW2;
    const int i = (int)(q / H), j = (int)(q % H);
    w2t[(size_t)j * H + i] = tr::conv(w);
    w2c[(size_t)i * H + j] = tr::conv(w);
  } else if (p >= m.oW3 && p < m.ob3) {
    const int64_t q = p - m.oW3;
    const int i = (int)(q / m.O), j = (int)(q % m.O);
    w3t[(size_t)j * H + i] = tr::conv(w);
    w3c[(size_t)i * m.Op + j] = tr::conv(w);
  }
}

template <class T>
__global__ void __launch_bounds__(256)
k_mlp_setparams(mlp_geom m, const double* __restrict__ src, float* __restrict__ master,
                float* __restrict__ m1, float* __restrict__ m2, T* w1t, T* w2t, T* w3t, T* w2c,
                T* w3c) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= m.np) return;
  const float w = (float)src[p];
  master[p] = w;
  m1[p] = 0.f;
  m2[p] = 0.f;
  write_copies<T>(m, p, w, w1t, w2t, w3t, w2c, w3c);
}

template <class T>
__global__ void __launch_bounds__(256)
k_mlp_adam(mlp_geom m, int nsplit, const float* __restrict__ part, const double* __restrict__ scal,
           const int* __restrict__ tstep, double lr, double beta1, double beta2, double eps,
           float* __restrict__ master, float* __restrict__ m1, float* __restrict__ m2, T* w1t,
           T* w2t, T* w3t, T* w2c, T* w3c, double* __restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= m.np) return;
  const double cnt = scal[0];
  double gs = 0.0;
  for (int k = 0; k < nsplit; ++k) gs += (double)part[(size_t)k * m.np + p];
  const double gr = cnt > 0.0 ? gs * scal[2] : 0.0;
  if (grad != nullptr) grad[p] = gr;
  if (!(cnt > 0.0)) return;
  const double t = (double)tstep[0];
  const double mo = beta1 * (double)m1[p] + (1.0 - beta1) * gr;
  const double vo = beta2 * (double)m2[p] + (1.0 - beta2) * gr * gr;
  const double mh = mo / (1.0 - pow(beta1, t)), vh = vo / (1.0 - pow(beta2, t));
  const float w = (float)((double)master[p] - lr * mh / (sqrt(vh) + eps));
  m1[p] = (float)mo;
  m2[p] = (float)vo;
  master[p] = w;
  write_copies<T>(m, p, w, w1t, w2t, w3t, w2c, w3c);
}

__global__ void k_mlp_outputs(int n, int K, int Op, const float* __restrict__ out,
                              const double* __restrict__ y, double* __restrict__ mu,
                              double* __restrict__ lv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * K) return;
  const size_t s = idx / K;
  const int k = (int)(idx % K);
  mu[idx] = y[idx] + (double)out[s * Op + k];
  lv[idx] = out[s * Op + K + k];
}

mlp_geom geom(const afqmc_ctx_s* c) {
  const auto& m = c->mlp;
  mlp_geom g;
  g.D = m.D;
  g.Dp = m.Dp;
  g.O = m.O;
  g.Op = m.Op;
  g.np = m.np;
  g.ob1 = m.ob1;
  g.oW2 = m.oW2;
  g.ob2 = m.ob2;
  g.oW3 = m.oW3;
  g.ob3 = m.ob3;
  return g;
}

unsigned blocks_of(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class T>
hipError_t forward_t(const afqmc_ctx_s* c, int n, int Sp, const double* gd, const double* y,
                     float* out, void* zT, void* h1T, void* h2T) {
  const auto& m = c->mlp;
  const dim3 grid(blocks_of(Sp / 16, 4)), block(256);
  const T* w1t = static_cast<const T*>(m.w1t);
  const T* w2t = static_cast<const T*>(m.w2t);
  const T* w3t = static_cast<const T*>(m.w3t);
  const float* b1 = m.master + m.ob1;
  const float* b2 = m.master + m.ob2;
  const float* b3 = m.master + m.ob3;
  if (zT != nullptr)
    hipLaunchKernelGGL((k_mlp_fwd<T, true>), grid, block, 0, c->stream, n, Sp, c->M, c->K, m.D,
                       m.Dp, m.O, m.Op, gd, y, w1t, w2t, w3t, b1, b2, b3, out,
                       static_cast<T*>(zT), static_cast<T*>(h1T), static_cast<T*>(h2T));
  else
    hipLaunchKernelGGL((k_mlp_fwd<T, false>), grid, block, 0, c->stream, n, Sp, c->M, c->K, m.D,
                       m.Dp, m.O, m.Op, gd, y, w1t, w2t, w3t, b1, b2, b3, out, nullptr, nullptr,
                       nullptr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mlp_setparams(const afqmc_ctx_s* c, const double* src) {
  const auto& m = c->mlp;
  const dim3 grid(blocks_of(m.np, 256)), block(256);
  if (m.prec == AFQMC_PREC_BF16)
    hipLaunchKernelGGL(k_mlp_setparams<bf16_t>, grid, block, 0, c->stream, geom(c), src, m.master,
                       m.mom1, m.mom2, static_cast<bf16_t*>(m.w1t), static_cast<bf16_t*>(m.w2t),
                       static_cast<bf16_t*>(m.w3t), static_cast<bf16_t*>(m.w2c),
                       static_cast<bf16_t*>(m.w3c));
  else
    hipLaunchKernelGGL(k_mlp_setparams<float>, grid, block, 0, c->stream, geom(c), src, m.master,
                       m.mom1, m.mom2, static_cast<float*>(m.w1t), static_cast<float*>(m.w2t),
                       static_cast<float*>(m.w3t), static_cast<float*>(m.w2c),
                       static_cast<float*>(m.w3c));
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const afqmc_ctx_s* c, int n, int Sp, const double* gd, const double* y,
                              float* out, void* zT, void* h1T, void* h2T) {
  if (Sp <= 0) return hipSuccess;
  return c->mlp.prec == AFQMC_PREC_BF16 ? forward_t<bf16_t>(c, n, Sp, gd, y, out, zT, h1T, h2T)
                                        : forward_t<float>(c, n, Sp, gd, y, out, zT, h1T, h2T);
}

hipError_t launch_mlp_propose(const afqmc_ctx_s* c, int nw, const float* out, const double* y,
                              uint64_t seed, uint64_t step, int sweep, double* ytry, double* lqf) {
  const int n = nw * c->P;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_propose, dim3(n), dim3(64), 0, c->stream, c->P, c->K, c->mlp.Op, out, y,
                     seed, step, c->dstep, sweep, ytry, lqf);
  return hipGetLastError();
}

hipError_t launch_mlp_reverse(const afqmc_ctx_s* c, int n, const float* outR, const double* y,
                              const double* ytry, const double* lqf, double* lqx) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_reverse, dim3(n), dim3(64), 0, c->stream, c->K, c->mlp.Op, outR, y,
                     ytry, lqf, lqx);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const afqmc_ctx_s* c, int n, int Sp, const float* out,
                               const double* yin, const double* ytgt, const int* mask,
                               const void* h1T, const void* h2T, void* dOT, void* dh2T, void* dh1T,
                               double* nlq) {
  if (Sp <= 0) return hipSuccess;
  const auto& m = c->mlp;
  const dim3 grid(blocks_of(Sp / 16, 4)), block(256);
  if (m.prec == AFQMC_PREC_BF16)
    hipLaunchKernelGGL(k_mlp_bwd<bf16_t>, grid, block, 0, c->stream, n, Sp, c->K, m.O, m.Op, out,
                       yin, ytgt, mask, static_cast<const bf16_t*>(m.w2c),
                       static_cast<const bf16_t*>(m.w3c), static_cast<const bf16_t*>(h1T),
                       static_cast<const bf16_t*>(h2T), static_cast<bf16_t*>(dOT),
                       static_cast<bf16_t*>(dh2T), static_cast<bf16_t*>(dh1T), nlq);
  else
    hipLaunchKernelGGL(k_mlp_bwd<float>, grid, block, 0, c->stream, n, Sp, c->K, m.O, m.Op, out,
                       yin, ytgt, mask, static_cast<const float*>(m.w2c),
                       static_cast<const float*>(m.w3c), static_cast<const float*>(h1T),
                       static_cast<const float*>(h2T), static_cast<float*>(dOT),
                       static_cast<float*>(dh2T), static_cast<float*>(dh1T), nlq);
  return hipGetLastError();
}

hipError_t launch_mlp_wgrad(const afqmc_ctx_s* c, int Sp, const void* zT, const void* h1T,
                            const void* h2T, const void* dOT, const void* dh2T, const void* dh1T,
                            float* part) {
  if (Sp <= 0) return hipSuccess;
  const auto& m = c->mlp;
  wg_args a;
  const void* X[3] = {zT, h1T, h2T};
  const void* Y[3] = {dh1T, dh2T, dOT};
  const int in[3] = {m.D, H, H}, outc[3] = {H, H, m.O};
  const int64_t off[3] = {0, m.oW2, m.oW3};
  int total = 0;
  for (int l = 0; l < 3; ++l) {
    const int rt = (in[l] + 1 + 15) / 16, ct = (outc[l] + 15) / 16;
    a.l[l].X = X[l];
    a.l[l].Y = Y[l];
    a.l[l].in = in[l];
    a.l[l].out = outc[l];
    a.l[l].bc = (ct + 1) / 2;
    a.l[l].nb = ((rt + 1) / 2) * a.l[l].bc;
    a.l[l].off = off[l];
    total += a.l[l].nb;
  }
  const int nsplit = (Sp + MLP_CHUNK - 1) / MLP_CHUNK;
  const dim3 grid(blocks_of(total, 4), nsplit), block(256);
  if (m.prec == AFQMC_PREC_BF16)
    hipLaunchKernelGGL(k_mlp_wgrad<bf16_t>, grid, block, 0, c->stream, Sp, a, part, m.np);
  else
    hipLaunchKernelGGL(k_mlp_wgrad<float>, grid, block, 0, c->stream, Sp, a, part, m.np);
  return hipGetLastError();
}

hipError_t launch_mlp_reduce(const afqmc_ctx_s* c, int n, const int* mask, const double* nlq,
                             double* loss) {
  hipLaunchKernelGGL(k_mlp_reduce, dim3(1), dim3(256), 0, c->stream, n, mask, nlq, c->mlp.scal,
                     c->mlp.tstep, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const afqmc_ctx_s* c, int Sp, const float* part, double* grad) {
  const auto& m = c->mlp;
  const int nsplit = (Sp + MLP_CHUNK - 1) / MLP_CHUNK;
  const dim3 grid(blocks_of(m.np, 256)), block(256);
  if (m.prec == AFQMC_PREC_BF16)
    hipLaunchKernelGGL(k_mlp_adam<bf16_t>, grid, block, 0, c->stream, geom(c), nsplit, part,
                       m.scal, m.tstep, m.lr, m.beta1, m.beta2, m.eps, m.master, m.mom1, m.mom2,
                       static_cast<bf16_t*>(m.w1t), static_cast<bf16_t*>(m.w2t),
                       static_cast<bf16_t*>(m.w3t), static_cast<bf16_t*>(m.w2c),
                       static_cast<bf16_t*>(m.w3c), grad);
  else
    hipLaunchKernelGGL(k_mlp_adam<float>, grid, block, 0, c->stream, geom(c), nsplit, part, m.scal,
                       m.tstep, m.lr, m.beta1, m.beta2, m.eps, m.master, m.mom1, m.mom2,
                       static_cast<float*>(m.w1t), static_cast<float*>(m.w2t),
                       static_cast<float*>(m.w3t), static_cast<float*>(m.w2c),
                       static_cast<float*>(m.w3c), grad);
  return hipGetLastError();
}

hipError_t launch_mlp_outputs(const afqmc_ctx_s* c, int n, const float* out, const double* y,
                              double* mu, double* lv) {
  const size_t total = (size_t)n * c->K;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_outputs, dim3(blocks_of((int64_t)total, 256)), dim3(256), 0, c->stream,
                     n, c->K, c->mlp.Op, out, y, mu, lv);
  return hipGetLastError();
}
