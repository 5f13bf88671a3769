// Walker propagation and hybrid phaseless weight (Sec. II.A, Eq. HS; Sec. II.B,
// Eqs. walker_prop, importance_function, importance_function_CP; Sec. III.A,
// Eq. ratio-update-phi for the overlap ratio; App. B step 1).
//
//   V = i sqrt(tau) sum_g (xi_g - xbar_g) L_g          (k_vbuild; k_vbuild_bx)
//   phi' = e^{-tau h1/2} T_n(V) e^{-tau h1/2} phi, T_n = sum_{j<=n} V^j/j!
//                                        (k_taylor, k_taylor_g; k_taylor_x3)
//   (the _bx and _x3 forms: split-BF16 products, for BF16 contexts on the
//   workgroup kernels)
//   l'_p at the unchanged paths (overlap kernel), then per walker
//   num_r = sum_p exp(l'_p - Re l_p), r = num_r / sum_p S_p,
//   W <- W |exp(sum_g xi_g xbar_g - xbar_g^2 / 2) r| e^{tau E_T} max(0, cos arg r)
//                                                                  (k_weight)
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

// ---------------------------------------------------------------------------
// V build: with c = xi - xbar, R = sum_g Re(c_g) L_g and Q = sum_g Im(c_g) L_g,
// V = sqrt(tau) (-Q + i R).  A (walkers x G) by (G x M^2) product on the matrix
// cores, tiled through LDS: a workgroup of four wavefronts takes VB_W = 64
// walkers by VB_E matrix entries (64 in FP64, 128 in FP32) and walks G in
// chunks of VB_KC vectors.  Each chunk's c (real and imaginary planes) and L
// entries are read from global memory once per workgroup, converted to T,
// and staged in double-buffered LDS while the previous chunk's products run;
// wavefront (wh, eh) holds 2 walker tiles by VB_E / 32 entry tiles of R and Q
// accumulators, so one staged c value feeds VB_E / 32 products and one L value
// four.  Row w of xi starts at w * xs and of xbar at w * xbs; xbar may be null
// (c = xi): the trial slices use this with the generators A_k and their block
// of y, the back-propagation with a walker's recorded fields.  XB = false (no
// xbar): Q = 0 and only the R products run.  With T = float (mixed-precision
// contexts with real trials) c and L are rounded to FP32 and the products run
// on v_mfma_f32_16x16x4f32 with FP32 accumulation over g.  RO (real output,
// with XB = false): the trial generators' U[s] = c sum_k y[s][k] A_k, stored
// as one real FP64 entry per (row, entry), scaled by sqrt_tau = c.
constexpr int VB_W = 64;   // walkers per workgroup
constexpr int VB_KC = 16;  // vectors per staged chunk
// LDS rows are padded by 16 values, so that the two k rows one 32-lane half of
// a wavefront reads (g = 0, 1) fall on different banks
template <typename T>
struct VbShape {
  static constexpr int ET = sizeof(T) == 4 ? 4 : 2;  // entry tiles per wavefront
  static constexpr int E = 32 * ET;                   // entries per workgroup
  static constexpr int SAW = VB_W + 16, SBE = E + 16; // padded LDS rows of c and L
};
template <typename T, bool XB>
size_t vb_lds_bytes() {
  typedef VbShape<T> S;
  return (size_t)2 * VB_KC * ((XB ? 2 : 1) * S::SAW + S::SBE) * sizeof(T);
}
template <typename T, bool XB, bool RO = false>
__global__ void __launch_bounds__(256)
k_vbuild(int nw, int G, int MM, int xs, int xbs, double sqrt_tau, const double* __restrict__ L,
         const double* __restrict__ xi, const double* __restrict__ xbar, double* __restrict__ vmat) {
  typedef ::MM<T> mm;  // (the parameter MM is the number of matrix entries)
  typedef typename mm::acc_t acc_t;
  constexpr int ET = VbShape<T>::ET, E = VbShape<T>::E, SAW = VbShape<T>::SAW, SBE = VbShape<T>::SBE;
  constexpr int NA = XB ? 2 : 1;                    // c planes (re, im)
  constexpr int CA = NA * VB_KC * SAW;              // staged c values per chunk
  constexpr int CH = CA + VB_KC * SBE;              // staged values per chunk
  extern __shared__ double smem[];
  T* sbuf = reinterpret_cast<T*>(smem);             // [2][ c: [NA][VB_KC][SAW], L: [VB_KC][SBE] ]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c = lane & 15;
  const int wh = wave >> 1, eh = wave & 1;          // walker half, entry half
  const int wb = blockIdx.y * VB_W, eb = blockIdx.x * E;
  // global -> register staging: thread (j, w) takes walker w's AV consecutive
  // vectors AV j .. AV j + AV - 1 of the chunk (consecutive lanes on consecutive
  // walkers, so the LDS stores are conflict-free), and BV L entries, e fastest
  constexpr int AV = VB_KC * VB_W / 256;            // (walker, k) pairs per thread
  constexpr int BV = VB_KC * E / 256;               // L entries per thread
  static_assert(VB_KC * VB_W % 256 == 0 && VB_KC * E % 256 == 0, "whole chunks per thread");
  const int wl = tid % VB_W, kj = AV * (tid / VB_W);
  T ra[NA][AV], rb[BV];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int k = k0 + kj + i, w = wb + wl;
      const bool ok = k < G && w < nw;
      const int kc = min(k, G - 1), wc = min(w, nw - 1);
      const double x = xi[(size_t)wc * xs + kc];
      if constexpr (XB) {
        const double br = xbar[((size_t)wc * xbs + kc) * 2], bi = xbar[((size_t)wc * xbs + kc) * 2 + 1];
        ra[0][i] = (T)keep_if(x - br, ok);
        ra[1][i] = (T)keep_if(-bi, ok);
      } else {
        ra[0][i] = (T)keep_if(x, ok);
      }
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int q = tid + 256 * i, k = k0 + q / E, e = eb + q % E;
      const bool ok = k < G && e < MM;
      rb[i] = (T)keep_if(L[(size_t)min(k, G - 1) * MM + min(e, MM - 1)], ok);
    }
  };
  auto sstore = [&](int buf) {
    T* sa = sbuf + buf * CH;
    T* sb = sa + CA;
#pragma unroll
    for (int i = 0; i < AV; ++i)
#pragma unroll
      for (int p = 0; p < NA; ++p) sa[(p * VB_KC + kj + i) * SAW + wl] = ra[p][i];
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int q = tid + 256 * i;
      sb[(q / E) * SBE + q % E] = rb[i];
    }
  };
  acc_t acc[NA][2][ET];
#pragma unroll
  for (int p = 0; p < NA; ++p)
#pragma unroll
    for (int wt = 0; wt < 2; ++wt)
#pragma unroll
      for (int et = 0; et < ET; ++et) acc[p][wt][et] = mm::zero();
  const int nch = (G + VB_KC - 1) / VB_KC;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) gload((ch + 1) * VB_KC);
    const T* sa = sbuf + (ch & 1) * CH;
    const T* sb = sa + CA;
#pragma unroll
    for (int ks = 0; ks < VB_KC / 4; ++ks) {
      const int k = 4 * ks + g;
      T a[NA][2], b[ET];
#pragma unroll
      for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int wt = 0; wt < 2; ++wt) a[p][wt] = sa[(p * VB_KC + k) * SAW + 32 * wh + 16 * wt + c];
#pragma unroll
      for (int et = 0; et < ET; ++et) b[et] = sb[k * SBE + (E / 2) * eh + 16 * et + c];
#pragma unroll
      for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int wt = 0; wt < 2; ++wt)
#pragma unroll
          for (int et = 0; et < ET; ++et) acc[p][wt][et] = mm::fma(a[p][wt], b[et], acc[p][wt][et]);
    }
    // the other buffer was last read in the previous chunk, before its barrier
    if (ch + 1 < nch) sstore((ch + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int wt = 0; wt < 2; ++wt)
#pragma unroll
    for (int et = 0; et < ET; ++et)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int w = wb + 32 * wh + 16 * wt + mm::row(g, r), e = eb + (E / 2) * eh + 16 * et + c;
        if (RO) {
          if (w < nw && e < MM) vmat[(size_t)w * MM + e] = sqrt_tau * (double)acc[0][wt][et][r];
        } else if (w < nw && e < MM) {
          const double re = -sqrt_tau * (XB ? (double)acc[NA - 1][wt][et][r] : 0.0);
          const double im = sqrt_tau * (double)acc[0][wt][et][r];
          *reinterpret_cast<double2*>(vmat + ((size_t)w * MM + e) * 2) = double2{re, im};
        }
      }
}

// ---------------------------------------------------------------------------
// Taylor propagator.  One workgroup per walker, one wavefront per 16-row tile
// of the M x 2N complex block [phi_up phi_dn].  Each wavefront keeps its rows
// of V (and of e^{-tau h1/2}) in registers as FP64-MFMA A operands; the
// iterate Y is shared through a double-buffered LDS tile.  Horner form:
// Y = X; for j = n..1: Y = X + V Y / j.
// T = float (mixed-precision contexts with real trials): V, E_h and the
// iterate rounded to FP32, v_mfma_f32_16x16x4f32 products.
template <typename T, int MT>
__global__ void __launch_bounds__(MT * 4)
k_taylor(int M, int N, int n_taylor, const double* __restrict__ vmat,
         const double* __restrict__ Eh, double* __restrict__ phi) {
  typedef MM<T> mm;
  typedef typename mm::acc_t acc_t;
  constexpr int NTILE = MT / 16;
  constexpr int NC = 32;  // 2 spins x 16 columns
  __shared__ T s_y[2][MT][NC][2];

  const int w = blockIdx.x;
  const int wave = threadIdx.x >> 6;  // my row tile
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const double* V = vmat + (size_t)w * M * M * 2;
  double* ph = phi + (size_t)w * 2 * M * N * 2;

  // A operands: rows 16 wave + c, columns 16t + k(g, r) (V, E_h symmetric)
  T vr[NTILE][4], vi[NTILE][4], nvi[NTILE][4], eh[NTILE][4];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + mm::row(g, r), col = 16 * wave + c;
      const bool ok = row < M && col < M;
      vr[t][r] = (T)(ok ? V[((size_t)row * M + col) * 2] : 0.0);
      vi[t][r] = (T)(ok ? V[((size_t)row * M + col) * 2 + 1] : 0.0);
      nvi[t][r] = -vi[t][r];
      eh[t][r] = (T)(ok ? Eh[row * M + col] : 0.0);
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
    s_y[0][m][col][0] = (T)re;
    s_y[0][m][col][1] = (T)im;
  }
  __syncthreads();

  // real-symmetric product with eh: out rows of this tile from buffer `src`
  auto apply_eh = [&](int src, acc_t (&o)[2][2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) o[ct][0] = o[ct][1] = mm::zero();
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const T* yb = s_y[src][16 * t + mm::row(g, r)][16 * ct + c];
          o[ct][0] = mm::fma(eh[t][r], yb[0], o[ct][0]);
          o[ct][1] = mm::fma(eh[t][r], yb[1], o[ct][1]);
        }
  };
  auto store_rows = [&](int dst, const acc_t (&o)[2][2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        s_y[dst][16 * wave + mm::row(g, r)][16 * ct + c][0] = o[ct][0][r];
        s_y[dst][16 * wave + mm::row(g, r)][16 * ct + c][1] = o[ct][1][r];
      }
  };

  // X = E_h phi (kept in registers, rows of this tile) -> buffer 1
  acc_t x[2][2];
  apply_eh(0, x);
  store_rows(1, x);
  __syncthreads();
  int cur = 1;
  for (int j = n_taylor; j >= 1; --j) {
    acc_t acc[2][2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) acc[ct][0] = acc[ct][1] = mm::zero();
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const T* yb = s_y[cur][16 * t + mm::row(g, r)][16 * ct + c];
          const T yr = yb[0], yi = yb[1];
          acc[ct][0] = mm::fma(vr[t][r], yr, acc[ct][0]);
          acc[ct][0] = mm::fma(nvi[t][r], yi, acc[ct][0]);
          acc[ct][1] = mm::fma(vr[t][r], yi, acc[ct][1]);
          acc[ct][1] = mm::fma(vi[t][r], yr, acc[ct][1]);
        }
    const T invj = (T)(1.0 / (double)j);
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
  acc_t o[2][2];
  apply_eh(cur, o);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * wave + mm::row(g, r);
      if (m < M && c < N) {
        double* d = ph + ((size_t)(ct * M + m) * N + c) * 2;
        d[0] = (double)o[ct][0][r];
        d[1] = (double)o[ct][1][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Phaseless weight, hybrid or local-energy formalism, with the cosine of the
// overlap ratio's argument; one 64-lane workgroup per walker.
__global__ void __launch_bounds__(64)
k_weight(int nw, int P, int G, double dtau, double e_shift, int weight_mode,
         const double* __restrict__ xi, const double* __restrict__ xbar,
         const double* __restrict__ logov, const double* __restrict__ logov_new,
         const double* __restrict__ eloc, double* __restrict__ w, double* __restrict__ ref,
         int* __restrict__ flags) {
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
    const double mag = (weight_mode == AFQMC_WEIGHT_LOCAL)
                           ? exp(-dtau * (eloc[2 * (size_t)wk] - e_shift))
                           : exp(sr + log(absr) + dtau * e_shift);
    if (weight_mode == AFQMC_WEIGHT_COMBINED)
      wn = w[wk] * mag;
    else
      wn = w[wk] * mag * fmax(0.0, cos(atan2(r.im, r.re)));
  }
  const bool finite = __builtin_isfinite(wn);
  w[wk] = finite ? wn : 0.0;  // a non-finite weight kills the walker, and is flagged
  if (!finite && flags != nullptr) flags[wk] |= AFQMC_NUMERIC_WEIGHT;
  const cplx rf = (weight_mode == AFQMC_WEIGHT_COMBINED) ? den : num;
  ref[(size_t)wk * 2] = rf.re;
  ref[(size_t)wk * 2 + 1] = rf.im;
}

// reduced-precision walker propagation: mixed-precision contexts with real trials
bool prop_f32(const afqmc_ctx_s* c) { return c->precision != AFQMC_PREC_FP64 && !c->ctrial; }

template <typename T, bool XB, bool RO = false>
hipError_t vb_launch(const afqmc_ctx_s* c, int n, int G, int MM, int xs, int xbs, double sqrt_s,
                     const double* L, const double* xi, const double* xbar, double* vmat) {
  const size_t lds = vb_lds_bytes<T, XB>();
  static_assert(!RO || !XB, "real output: no xbar");
  auto kern = k_vbuild<T, XB, RO>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((MM + VbShape<T>::E - 1) / VbShape<T>::E, (n + VB_W - 1) / VB_W);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, c->stream, n, G, MM, xs, xbs, sqrt_s, L, xi, xbar,
                     vmat);
  return hipGetLastError();
}

// The V and U builds of BF16 contexts on the workgroup kernels, on split-BF16
// products (v_mfma_f32_16x16x32_bf16, FP32 accumulation): their propagation
// and trial series split V and U again as they load them.  Both operands
// arrive split and k-contiguous, so the chunk staging is plain 16-byte copies:
// L (or the generators A_k) from a transposed split copy [2][M*M][GP] made at
// context creation, the coefficients from a per-call split [NA planes][2
// parts][rows][GP] (V: xi - Re xbar and -Im xbar; U: y).  Same workgroup tile
// as k_vbuild (64 walkers x 128 entries; wavefront (wh, eh) with 2 walker and
// 4 entry tiles); a chunk is one k block of 32 vectors, staged in LDS as rows
// of 40 entries (80 bytes), so that each operand (8 consecutive vectors of one
// walker or entry) is one 16-byte read.  NA = 1 (U) stores a real output.
// The output rows (M entries) sit MP apart (MP = M, or with SPLIT, for the
// split-BF16 trial series, M rounded up to 32: the entries past M are zero);
// SPLIT stores U itself split, [row][hi, lo][M][MP] BF16, or V as its real
// part and minus its imaginary part split, [walker][Re hi, Re lo, -Im hi,
// -Im lo][M][MP]: half the bytes of FP64 and in the A-operand form that the
// trial series and the propagation load.
constexpr int VX_KC = 32, VX_E = 128, VX_RS = VX_KC + 8;
template <int NA>
constexpr int vx_sb0() {  // start of the L planes in a buffer (16-bit units)
  return NA * 2 * VB_W * VX_RS;
}
template <int NA>
constexpr int vx_ch() {  // 16-bit units per buffer
  return vx_sb0<NA>() + 2 * VX_E * VX_RS;
}
template <int NA, bool SPLIT>
__global__ void __launch_bounds__(256)
k_vbuild_bx(int nw, int GP, int M, int MP, double sqrt_tau, const unsigned short* __restrict__ LT,
            const unsigned short* __restrict__ cf, void* __restrict__ out) {

  constexpr int VX_SB0 = vx_sb0<NA>(), VX_CH = vx_ch<NA>();
  const int MM = M * M, ET = M * MP;  // entries of L (or A_k) and of an output row
  extern __shared__ double smem[];
  unsigned short* sbuf = reinterpret_cast<unsigned short*>(smem);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c = lane & 15;
  const int wh = wave >> 1, eh = wave & 1;
  const int wb = blockIdx.y * VB_W, eb = blockIdx.x * VX_E;
  // staging: 512 NA 16-byte pieces of c and 1024 of L per chunk; piece q of c
  // is (plane-part q / 256, walker (q % 256) / 4, octet q % 4), piece q of L
  // is (part q / 512, entry (q % 512) / 4, octet q % 4)
  uint4 ra[2 * NA], rb[4];
  // this thread's L pieces: entry eb + (q % 512) / 4 of the output row, at
  // (row, col) of the M x M matrix; none past column M
  int lt_off[4];
  bool lt_ok[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i, e = eb + ((q & 511) >> 2);
    const int row = e / MP, col = e - row * MP;
    lt_ok[i] = e < ET && col < M;
    lt_off[i] = ((q >> 9) * MM + (lt_ok[i] ? row * M + col : 0)) * GP;
  }
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 2 * NA; ++i) {
      const int q = tid + 256 * i;
      const int pp = q >> 8, wl = (q & 255) >> 2, ko = q & 3, w = wb + wl;
      const uint4 v = *reinterpret_cast<const uint4*>(
          cf + ((size_t)pp * nw + min(w, nw - 1)) * GP + k0 + 8 * ko);
      ra[i] = w < nw ? v : uint4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i;
      const uint4 v = *reinterpret_cast<const uint4*>(LT + lt_off[i] + k0 + 8 * (q & 3));
      rb[i] = lt_ok[i] ? v : uint4{0u, 0u, 0u, 0u};
    }
  };
  auto sstore = [&](int buf) {
    unsigned short* sa = sbuf + buf * VX_CH;
    unsigned short* sb = sa + VX_SB0;
#pragma unroll
    for (int i = 0; i < 2 * NA; ++i) {
      const int q = tid + 256 * i;
      *reinterpret_cast<uint4*>(sa + ((q >> 8) * VB_W + ((q & 255) >> 2)) * VX_RS + 8 * (q & 3)) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i;
      *reinterpret_cast<uint4*>(sb + ((q >> 9) * VX_E + ((q & 511) >> 2)) * VX_RS + 8 * (q & 3)) = rb[i];
    }
  };
  fx4 acc[NA][2][4];
#pragma unroll
  for (int p = 0; p < NA; ++p)
#pragma unroll
    for (int wt = 0; wt < 2; ++wt)
#pragma unroll
      for (int et = 0; et < 4; ++et) acc[p][wt][et] = ::MM<float>::zero();
  const int nch = GP / VX_KC;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) gload((ch + 1) * VX_KC);
    const unsigned short* sa = sbuf + (ch & 1) * VX_CH;
    const unsigned short* sb = sa + VX_SB0;
    tsx8 ah[NA][2], al[NA][2];
#pragma unroll
    for (int p = 0; p < NA; ++p)
#pragma unroll
      for (int wt = 0; wt < 2; ++wt) {
        const int w = 32 * wh + 16 * wt + c;
        ah[p][wt] = *reinterpret_cast<const tsx8*>(sa + ((p * 2 + 0) * VB_W + w) * VX_RS + 8 * g);
        al[p][wt] = *reinterpret_cast<const tsx8*>(sa + ((p * 2 + 1) * VB_W + w) * VX_RS + 8 * g);
      }
#pragma unroll
    for (int et = 0; et < 4; ++et) {
      const int e = 64 * eh + 16 * et + c;
      const tsx8 bh = *reinterpret_cast<const tsx8*>(sb + e * VX_RS + 8 * g);
      const tsx8 bl = *reinterpret_cast<const tsx8*>(sb + (VX_E + e) * VX_RS + 8 * g);
#pragma unroll
      for (int p = 0; p < NA; ++p)
#pragma unroll
        for (int wt = 0; wt < 2; ++wt)
          acc[p][wt][et] = mfma_x3(ah[p][wt], al[p][wt], bh, bl, acc[p][wt][et]);
    }
    // the other buffer was last read in the previous chunk, before its barrier
    if (ch + 1 < nch) sstore((ch + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int wt = 0; wt < 2; ++wt)
#pragma unroll
    for (int et = 0; et < 4; ++et)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int w = wb + 32 * wh + 16 * wt + 4 * g + r, e = eb + 64 * eh + 16 * et + c;
        if (w >= nw || e >= ET) continue;
        if constexpr (SPLIT) {
          // U; or V_re = -sqrt(tau) Q and -V_im = -sqrt(tau) R
          unsigned short* us = static_cast<unsigned short*>(out) + (size_t)w * 2 * NA * ET + e;
#pragma unroll
          for (int p = 0; p < NA; ++p) {
            const double x = (double)acc[NA - 1 - p][wt][et][r];
            const float u = (float)(NA == 1 ? sqrt_tau * x : -sqrt_tau * x);
            const unsigned h = tpk_bf16(u, 0.f);
            us[(2 * p) * ET] = (unsigned short)(h & 0xffffu);
            us[(2 * p + 1) * ET] = (unsigned short)(tpk_bf16(u - tbf_lo(h), 0.f) & 0xffffu);
          }
        } else if constexpr (NA == 1) {
          static_cast<double*>(out)[(size_t)w * ET + e] = sqrt_tau * (double)acc[0][wt][et][r];
        } else {
          *reinterpret_cast<double2*>(static_cast<double*>(out) + ((size_t)w * ET + e) * 2) =
              double2{-sqrt_tau * (double)acc[1][wt][et][r], sqrt_tau * (double)acc[0][wt][et][r]};
        }
      }
}

// split coefficients: thread (w, o) takes row w's vectors 8 o .. 8 o + 7 (zero
// past G) into cf[plane][part][w][GP]; with xbar the planes xi - Re xbar and
// -Im xbar (the V build), without it the one plane xi (the U build's y)
template <bool XB>
__global__ void __launch_bounds__(256)
k_vcoef_split(int nw, int G, int GP, const double* __restrict__ xi, const double* __restrict__ xbar,
              unsigned short* __restrict__ cf) {
  const int no = GP / 8;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nw * no) return;
  const int w = q / no, o = q % no;
  float re[8], nim[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * o + j;
    const bool ok = k < G;
    const int kc = min(k, G - 1);
    const double x = xi[(size_t)w * G + kc];
    if constexpr (XB) {
      const double2 b = *reinterpret_cast<const double2*>(xbar + ((size_t)w * G + kc) * 2);
      re[j] = (float)keep_if(x - b.x, ok);
      nim[j] = (float)keep_if(-b.y, ok);
    } else {
      re[j] = (float)keep_if(x, ok);
    }
  }
  tsx8 h, l;
  const size_t row = (size_t)w * GP + 8 * o, plane = (size_t)nw * GP;
  split8(re, h, l);
  *reinterpret_cast<tsx8*>(cf + row) = h;
  *reinterpret_cast<tsx8*>(cf + plane + row) = l;
  if constexpr (XB) {
    split8(nim, h, l);
    *reinterpret_cast<tsx8*>(cf + 2 * plane + row) = h;
    *reinterpret_cast<tsx8*>(cf + 3 * plane + row) = l;
  }
}

// coefficient split and split-BF16 product of the V (NA = 2) or U (NA = 1)
// build; cf holds 4 NA n GP bytes; output rows MP apart (MP = M unless SPLIT)
template <int NA, bool SPLIT>
hipError_t vbx_run(const afqmc_ctx_s* c, int n, int G, int GP, int MP, double scale,
                   const unsigned short* LT, const double* x, const double* xbar,
                   unsigned short* cf, void* out) {
  const int ET = c->M * MP;
  const size_t nt = (size_t)n * (GP / 8);
  hipLaunchKernelGGL(k_vcoef_split<NA == 2>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                     c->stream, n, G, GP, x, xbar, cf);
  AFQMC_LAUNCH_CHECK();
  const size_t lds = (size_t)2 * vx_ch<NA>() * sizeof(unsigned short);
  hipError_t e = hipFuncSetAttribute((const void*)k_vbuild_bx<NA, SPLIT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((ET + VX_E - 1) / VX_E, (n + VB_W - 1) / VB_W);
  hipLaunchKernelGGL((k_vbuild_bx<NA, SPLIT>), grid, dim3(256), lds, c->stream, n, GP, c->M, MP,
                     scale, LT, cf, out);
  return hipGetLastError();
}

// L[g][e] -> LT[part][e][g] (split, transposed, zero for g >= G); thread (e, o)
// takes vectors 8 o .. 8 o + 7 of entry e
__global__ void __launch_bounds__(256)
k_lt_split(int G, int GP, int MM, const double* __restrict__ L, unsigned short* __restrict__ LT) {
  const int no = GP / 8;
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)MM * no) return;
  const int e = (int)(q / no), o = (int)(q % no);
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * o + j;
    v[j] = (float)keep_if(L[(size_t)min(k, G - 1) * MM + e], k < G);
  }
  tsx8 h, l;
  split8(v, h, l);
  *reinterpret_cast<tsx8*>(LT + (size_t)e * GP + 8 * o) = h;
  *reinterpret_cast<tsx8*>(LT + ((size_t)MM + e) * GP + 8 * o) = l;
}

template <int MT>
hipError_t launch_taylor_mt(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi) {
  if (prop_f32(c))
    hipLaunchKernelGGL((k_taylor<float, MT>), dim3(nw), dim3(MT * 4), 0, c->stream, c->M, c->N,
                       c->n_taylor, vmat, c->d_Eh, phi);
  else
    hipLaunchKernelGGL((k_taylor<double, MT>), dim3(nw), dim3(MT * 4), 0, c->stream, c->M, c->N,
                       c->n_taylor, vmat, c->d_Eh, phi);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lt_split(afqmc_ctx_s* c) {
  const int MM = c->M * c->M;
  auto one = [&](int G, const double* src, unsigned short** dst, int* GP) {
    *GP = (G + VX_KC - 1) / VX_KC * VX_KC;
    hipError_t e = hipMalloc(dst, (size_t)2 * MM * *GP * sizeof(unsigned short));
    if (e != hipSuccess) return e;
    const size_t n = (size_t)MM * (*GP / 8);
    hipLaunchKernelGGL(k_lt_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, G,
                       *GP, MM, src, *dst);
    return hipGetLastError();
  };
  hipError_t e = one(c->G, c->d_Lraw, &c->d_LTx, &c->GP);
  if (e == hipSuccess && c->d_Adiag == nullptr) e = one(c->K, c->d_A, &c->d_ATx, &c->KP);
  return e;
}

hipError_t launch_vbuild(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         double* vmat, void* scratch, size_t scratch_bytes) {
  if (nw <= 0) return hipSuccess;
  const int MM = c->M * c->M;
  if (c->d_LTx != nullptr && scratch != nullptr && scratch_bytes >= (size_t)8 * nw * c->GP)
    return vbx_run<2, false>(c, nw, c->G, c->GP, c->M, sqrt(c->dtau), c->d_LTx, xi, xbar,
                      static_cast<unsigned short*>(scratch), vmat);
  if (prop_f32(c))
    return vb_launch<float, true>(c, nw, c->G, MM, c->G, c->G, sqrt(c->dtau), c->d_Lraw, xi, xbar,
                                  vmat);
  return vb_launch<double, true>(c, nw, c->G, MM, c->G, c->G, sqrt(c->dtau), c->d_Lraw, xi, xbar,
                                 vmat);
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
                         const double* logov, const double* logov_new, const double* eloc,
                         double e_shift, double* w, double* ref, int* flags) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weight, dim3(nw), dim3(64), 0, c->stream, nw, c->P, c->G, c->dtau, e_shift,
                     c->weight_mode, xi, xbar, logov, logov_new, eloc, w, ref, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Taylor propagator for larger systems (M <= 160, N <= 40): one workgroup per
// (walker, spin), one wavefront per 16-row tile; V rows as MFMA A operands in
// registers (V_re and -V_im), the real one-body factors' operands read from L2
// at their uses, the iterate in one LDS tile with two barriers per Horner
// step, and X (the start of the Horner recursion) in a second LDS tile, or in
// registers (each wavefront its own rows) when two tiles exceed the LDS.  The
// imaginary part is accumulated as V_re Y_im - (-V_im) Y_re.
// Computes dst = El T_n(V) Er src per block (Er may be null: identity).  The
// walker step has El = Er = e^{-tau h1/2}, src = dst, two spins; a trial slice
// has one M x N block per path and src either the previous slice or, for the
// first slice, Phi_0 read by every path (src_ws = 0).
namespace {

template <typename T, int KTMAX, int NTC, bool XR>
__global__ void __launch_bounds__(64 * KTMAX)
k_taylor_g(int n, int M, int N, int MT, int n_taylor, int spins, const double* __restrict__ vmat,
           const double* __restrict__ El, const double* __restrict__ Er,
           const double* src, int src_ws, double* dst) {
  typedef MM<T> mm;
  typedef typename mm::acc_t acc_t;
  constexpr int NT = 16 * NTC;
  extern __shared__ double smem[];
  T* sY = reinterpret_cast<T*>(smem);  // [MT][NT][2] iterate
  T* sX = sY + MT * NT * 2;            // [MT][NT][2] X = Er src (unless XR)
  const int KT = MT / 16;
  // workgroup b takes V block 8 (b / 8S) + b % 8 and its block (b / 8) % S of
  // S = spins, so that the blocks that share V run 8 launches apart on one XCD
  // (workgroups go round-robin over the 8) and the later ones read V from its L2
  const int b = blockIdx.x;
  const int w = 8 * (b / (8 * spins)) + (b & 7), sp = (b >> 3) % spins;
  if (w >= n) return;  // whole workgroup, before any barrier
  const int tp = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const double* V = vmat + (size_t)w * M * M * 2;
  const double* in = src + ((size_t)w * src_ws + sp) * M * N * 2;
  double* ph = dst + ((size_t)w * spins + sp) * M * N * 2;

  T vr[KTMAX][4], nvi[KTMAX][4];
#pragma unroll
  for (int t = 0; t < KTMAX; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + mm::row(g, r), col = 16 * tp + c;
      const bool ok = t < KT && row < M && col < M;
      // clamped, unconditional loads masked afterwards: all in flight together
      const double2 v = *reinterpret_cast<const double2*>(
          V + ((size_t)min(row, M - 1) * M + min(col, M - 1)) * 2);
      vr[t][r] = (T)keep_if(v.x, ok);
      nvi[t][r] = (T)keep_if(-v.y, ok);
    }
  for (int q = threadIdx.x; q < MT * NT; q += blockDim.x) {
    const int m = q / NT, n = q % NT;
    const bool ok = m < M && n < N;
    const double2 v = *reinterpret_cast<const double2*>(
        in + ((size_t)min(m, M - 1) * N + min(n, N - 1)) * 2);
    sY[2 * q] = (T)keep_if(v.x, ok);
    sY[2 * q + 1] = (T)keep_if(v.y, ok);
  }
  __syncthreads();
  // o = E Y (rows of this tile)
  auto apply_eh = [&](const double* Eh, acc_t (&o)[NTC][2]) {
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) o[ct][0] = o[ct][1] = mm::zero();
#pragma unroll
    for (int t = 0; t < KTMAX; ++t)
      if (t < KT)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          {
            const int row = 16 * t + mm::row(g, r), col = 16 * tp + c;
            const T e =
                (T)keep_if(Eh[min(row, M - 1) * M + min(col, M - 1)], row < M && col < M);
#pragma unroll
            for (int ct = 0; ct < NTC; ++ct) {
              const T* yb = sY + ((16 * t + mm::row(g, r)) * NT + 16 * ct + c) * 2;
              o[ct][0] = mm::fma(e, yb[0], o[ct][0]);
              o[ct][1] = mm::fma(e, yb[1], o[ct][1]);
            }
          }
  };
  auto store = [&](T* dst, const acc_t (&o)[NTC][2]) {
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T* d = dst + ((16 * tp + mm::row(g, r)) * NT + 16 * ct + c) * 2;
        d[0] = o[ct][0][r];
        d[1] = o[ct][1][r];
      }
  };
  // X = Er src: a second LDS tile, or (XR, when two tiles do not fit in LDS)
  // registers, each wavefront holding its own rows in the accumulator layout
  acc_t x[NTC][2];
  if (Er != nullptr) {
    apply_eh(Er, x);
    __syncthreads();
    store(sY, x);
    if (!XR) store(sX, x);
    __syncthreads();
  } else if (XR) {
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T* d = sY + ((16 * tp + mm::row(g, r)) * NT + 16 * ct + c) * 2;
        x[ct][0][r] = d[0];
        x[ct][1][r] = d[1];
      }
  } else {
    for (int q = threadIdx.x; q < 2 * MT * NT; q += blockDim.x) sX[q] = sY[q];
    __syncthreads();
  }
  for (int j = n_taylor; j >= 1; --j) {
    acc_t are[NTC], aim1[NTC], aim2[NTC];
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) are[ct] = aim1[ct] = aim2[ct] = mm::zero();
#pragma unroll
    for (int t = 0; t < KTMAX; ++t)
      if (t < KT)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int ct = 0; ct < NTC; ++ct) {
            const T* yb = sY + ((16 * t + mm::row(g, r)) * NT + 16 * ct + c) * 2;
            const T yr = yb[0], yi = yb[1];
            are[ct] = mm::fma(vr[t][r], yr, are[ct]);
            are[ct] = mm::fma(nvi[t][r], yi, are[ct]);
            aim1[ct] = mm::fma(vr[t][r], yi, aim1[ct]);
            aim2[ct] = mm::fma(nvi[t][r], yr, aim2[ct]);
          }
    const T invj = (T)(1.0 / (double)j);
    acc_t y[NTC][2];
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T xr_, xi_;
        if (XR) {
          xr_ = x[ct][0][r];
          xi_ = x[ct][1][r];
        } else {
          const T* xv = sX + ((16 * tp + mm::row(g, r)) * NT + 16 * ct + c) * 2;
          xr_ = xv[0];
          xi_ = xv[1];
        }
        y[ct][0][r] = xr_ + are[ct][r] * invj;
        y[ct][1][r] = xi_ + (aim1[ct][r] - aim2[ct][r]) * invj;
      }
    __syncthreads();
    store(sY, y);
    __syncthreads();
  }
  acc_t o[NTC][2];
  apply_eh(El, o);
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * tp + mm::row(g, r), n = 16 * ct + c;
      if (m < M && n < N) {
        double* d = ph + ((size_t)m * N + n) * 2;
        d[0] = (double)o[ct][0][r];
        d[1] = (double)o[ct][1][r];
      }
    }
}

// ---------------------------------------------------------------------------
// The walker step e^{-tau h1/2} T_n(V) e^{-tau h1/2} phi for BF16 contexts on
// the workgroup kernels (real trials, M <= 128, N <= 32) with split-BF16
// products on v_mfma_f32_16x16x32_bf16 (FP32 accumulation within each product).
// One workgroup per (walker, spin), one wavefront per 16-row tile.  Wavefront
// tp keeps its rows of V_re and -V_im as split A operands (lane (g, c): row
// 16 tp + c, k = 32 t + 8 g + j); the operands of e^{-tau h1/2} are read from
// L2 and split at its two uses.  The iterate sits in LDS transposed, Y^T[part]
// [n][m] with the parts Re hi, Re lo, Im hi, Im lo and rows padded by 16 bytes
// (a B operand, 8 consecutive m of column n, is one 16-byte read), in two
// buffers so that each Horner step takes one barrier; X = e^{-tau h1/2} phi
// stays in registers in the accumulator layout.  The imaginary part is
// accumulated as V_re Y_im - (-V_im) Y_re.  Workgroup b takes walker
// 8 (b / 16) + b % 8 and spin (b / 8) % 2: the two spins of a walker are 8
// launches apart, on the same XCD (workgroups go round-robin over the 8), so
// the second finds V in that XCD's L2.
template <int KTMAX, int NTC>
__global__ void __launch_bounds__(64 * KTMAX) __attribute__((amdgpu_waves_per_eu(4)))
k_taylor_x3(int nw, int M, int N, int MT, int n_taylor, const double* __restrict__ vmat,
            const unsigned short* __restrict__ Vs, const double* __restrict__ Eh,
            double* __restrict__ phi) {
  constexpr int NT = 16 * NTC;
  constexpr int KBM = (16 * KTMAX + 31) / 32;  // k blocks of 32 at most
  const int KB = (MT + 31) / 32;                // k blocks (the last may be padding)
  const int XS = 32 * KB + 8;                   // LDS row of Y^T (bf16 entries)
  extern __shared__ double smem[];
  unsigned short* sY = reinterpret_cast<unsigned short*>(smem);  // [2 buffers][4 parts][NT][XS]
  const int w = 8 * (blockIdx.x >> 4) + (blockIdx.x & 7), sp = (blockIdx.x >> 3) & 1;
  if (w >= nw) return;  // whole workgroup, before any barrier
  const int tp = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int row = 16 * tp + c;
  const double* V = vmat != nullptr ? vmat + (size_t)w * M * M * 2 : nullptr;
  double* ph = phi + ((size_t)w * 2 + sp) * M * N * 2;
  auto yt = [&](int buf, int part, int n, int m) -> unsigned short* {
    return sY + ((size_t)(buf * 4 + part) * NT + n) * XS + m;
  };

  tsx8 vrh[KBM], vrl[KBM], vih[KBM], vil[KBM];  // V_re and -V_im, hi and lo
  if (Vs != nullptr) {  // V stored split: [Re hi, Re lo, -Im hi, -Im lo][M][32 KB]
    const size_t PL = (size_t)M * (32 * KB);
    const unsigned short* vb = Vs + (size_t)w * 4 * PL;
    const tsx8 z = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < KBM; ++t) {
      const bool ok = t < KB && row < M;
      const size_t o = (size_t)min(row, M - 1) * (32 * KB) + 32 * min(t, KB - 1) + 8 * g;
      const tsx8 a0 = *reinterpret_cast<const tsx8*>(vb + o);
      const tsx8 a1 = *reinterpret_cast<const tsx8*>(vb + PL + o);
      const tsx8 a2 = *reinterpret_cast<const tsx8*>(vb + 2 * PL + o);
      const tsx8 a3 = *reinterpret_cast<const tsx8*>(vb + 3 * PL + o);
      vrh[t] = ok ? a0 : z;
      vrl[t] = ok ? a1 : z;
      vih[t] = ok ? a2 : z;
      vil[t] = ok ? a3 : z;
    }
  } else {
#pragma unroll
    for (int t = 0; t < KBM; ++t) {
      float re[8], nim[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int col = 32 * t + 8 * g + j;
        const bool ok = t < KB && row < M && col < M;
        // clamped, unconditional loads masked afterwards: all in flight together
        const double2 v = *reinterpret_cast<const double2*>(
            V + ((size_t)min(row, M - 1) * M + min(col, M - 1)) * 2);
        re[j] = (float)keep_if(v.x, ok);
        nim[j] = (float)keep_if(-v.y, ok);
      }
      split8(re, vrh[t], vrl[t]);
      split8(nim, vih[t], vil[t]);
    }
  }
  // both buffers zero (rows past MT are read as padding and never written),
  // then phi into buffer 0
  for (int q = threadIdx.x; q < NT * XS; q += blockDim.x)
    reinterpret_cast<uint4*>(sY)[q] = uint4{0u, 0u, 0u, 0u};
  __syncthreads();
  for (int q = threadIdx.x; q < MT * NT; q += blockDim.x) {
    const int m = q / NT, n = q % NT;
    const bool ok = m < M && n < N;
    const double2 v = *reinterpret_cast<const double2*>(
        ph + ((size_t)min(m, M - 1) * N + min(n, N - 1)) * 2);
    const float re = (float)keep_if(v.x, ok), im = (float)keep_if(v.y, ok);
    const unsigned hr = tpk_bf16(re, 0.f), hi = tpk_bf16(im, 0.f);
    *yt(0, 0, n, m) = (unsigned short)(hr & 0xffffu);
    *yt(0, 1, n, m) = (unsigned short)(tpk_bf16(re - tbf_lo(hr), 0.f) & 0xffffu);
    *yt(0, 2, n, m) = (unsigned short)(hi & 0xffffu);
    *yt(0, 3, n, m) = (unsigned short)(tpk_bf16(im - tbf_lo(hi), 0.f) & 0xffffu);
  }
  __syncthreads();
  // o = e^{-tau h1/2} Y (this wavefront's rows) from buffer buf
  auto apply_e = [&](int buf, fx4 (&o)[NTC][2]) {
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) o[ct][0] = o[ct][1] = MM<float>::zero();
#pragma unroll
    for (int t = 0; t < KBM; ++t)
      if (t < KB) {
        float e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int col = 32 * t + 8 * g + j;
          e[j] = (float)keep_if(Eh[min(row, M - 1) * M + min(col, M - 1)], row < M && col < M);
        }
        tsx8 eh, el;
        split8(e, eh, el);
#pragma unroll
        for (int ct = 0; ct < NTC; ++ct) {
          const int n = 16 * ct + c, m = 32 * t + 8 * g;
          const tsx8 rh = *reinterpret_cast<const tsx8*>(yt(buf, 0, n, m));
          const tsx8 rl = *reinterpret_cast<const tsx8*>(yt(buf, 1, n, m));
          const tsx8 ih = *reinterpret_cast<const tsx8*>(yt(buf, 2, n, m));
          const tsx8 il = *reinterpret_cast<const tsx8*>(yt(buf, 3, n, m));
          o[ct][0] = mfma_x3(eh, el, rh, rl, o[ct][0]);
          o[ct][1] = mfma_x3(eh, el, ih, il, o[ct][1]);
        }
      }
  };
  // four consecutive rows of one column (this lane's accumulator values) as hi
  // and lo into parts (part, part + 1) of buffer buf
  auto put = [&](int buf, int part, int ct, const fx4& v) {
    const unsigned h01 = tpk_bf16(v[0], v[1]), h23 = tpk_bf16(v[2], v[3]);
    const unsigned l01 = tpk_bf16(v[0] - tbf_lo(h01), v[1] - tbf_hi(h01));
    const unsigned l23 = tpk_bf16(v[2] - tbf_lo(h23), v[3] - tbf_hi(h23));
    const int n = 16 * ct + c, m = 16 * tp + 4 * g;
    *reinterpret_cast<uint2*>(yt(buf, part, n, m)) = uint2{h01, h23};
    *reinterpret_cast<uint2*>(yt(buf, part + 1, n, m)) = uint2{l01, l23};
  };
  fx4 x[NTC][2];
  apply_e(0, x);
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct) {
    put(1, 0, ct, x[ct][0]);
    put(1, 2, ct, x[ct][1]);
  }
  __syncthreads();
  int cur = 1;
  // Horner: Y <- X + V Y / j for j = n .. 1; each step reads buffer cur and
  // writes the other, which every wavefront finished reading before the last
  // barrier
  for (int j = n_taylor; j >= 1; --j) {
    fx4 are[NTC], aim1[NTC], aim2[NTC];
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) are[ct] = aim1[ct] = aim2[ct] = MM<float>::zero();
#pragma unroll
    for (int t = 0; t < KBM; ++t)
      if (t < KB)
#pragma unroll
        for (int ct = 0; ct < NTC; ++ct) {
          const int n = 16 * ct + c, m = 32 * t + 8 * g;
          const tsx8 rh = *reinterpret_cast<const tsx8*>(yt(cur, 0, n, m));
          const tsx8 rl = *reinterpret_cast<const tsx8*>(yt(cur, 1, n, m));
          const tsx8 ih = *reinterpret_cast<const tsx8*>(yt(cur, 2, n, m));
          const tsx8 il = *reinterpret_cast<const tsx8*>(yt(cur, 3, n, m));
          are[ct] = mfma_x3(vrh[t], vrl[t], rh, rl, are[ct]);
          are[ct] = mfma_x3(vih[t], vil[t], ih, il, are[ct]);
          aim1[ct] = mfma_x3(vrh[t], vrl[t], ih, il, aim1[ct]);
          aim2[ct] = mfma_x3(vih[t], vil[t], rh, rl, aim2[ct]);
        }
    const float invj = (float)(1.0 / (double)j);
#pragma unroll
    for (int ct = 0; ct < NTC; ++ct) {
      fx4 yr, yi;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        yr[r] = x[ct][0][r] + are[ct][r] * invj;
        yi[r] = x[ct][1][r] + (aim1[ct][r] - aim2[ct][r]) * invj;
      }
      put(cur ^ 1, 0, ct, yr);
      put(cur ^ 1, 2, ct, yi);
    }
    __syncthreads();
    cur ^= 1;
  }
  fx4 o[NTC][2];
  apply_e(cur, o);
#pragma unroll
  for (int ct = 0; ct < NTC; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * tp + 4 * g + r, n = 16 * ct + c;
      if (m < M && n < N)
        *reinterpret_cast<double2*>(ph + ((size_t)m * N + n) * 2) =
            double2{(double)o[ct][0][r], (double)o[ct][1][r]};
    }
}

template <int KTMAX, int NTC>
hipError_t launch_taylor_x3(const afqmc_ctx_s* c, int nw, const double* vmat,
                            const unsigned short* Vs, double* phi) {
  const int NT = 16 * NTC, XS = 32 * ((c->MT + 31) / 32) + 8;
  const size_t lds = (size_t)8 * NT * XS * sizeof(unsigned short);
  auto kern = k_taylor_x3<KTMAX, NTC>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(16 * ((nw + 7) / 8)), dim3(64 * (c->MT / 16)), lds, c->stream, nw,
                     c->M, c->N, c->MT, c->n_taylor, vmat, Vs, c->d_Eh, phi);
  return hipGetLastError();
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, int KTMAX, int NTC>
hipError_t launch_taylor_g_kt(const afqmc_ctx_s* c, int n, int spins, int n_taylor,
                              const double* vmat, const double* El, const double* Er,
                              const double* src, int src_ws, double* dst) {
  const size_t tile = (size_t)c->MT * 16 * NTC * 2 * sizeof(T);
  const bool xr = 2 * tile > kMaxLds;
  const size_t lds = xr ? tile : 2 * tile;
  auto kern = xr ? k_taylor_g<T, KTMAX, NTC, true> : k_taylor_g<T, KTMAX, NTC, false>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid(8 * spins * ((n + 7) / 8));
  hipLaunchKernelGGL(kern, grid, dim3(64 * (c->MT / 16)), lds, c->stream, n, c->M, c->N, c->MT,
                     n_taylor, spins, vmat, El, Er, src, src_ws, dst);
  return hipGetLastError();
}

}  // namespace

namespace {

template <typename T>
hipError_t taylor_g_dispatch(const afqmc_ctx_s* c, int n, int spins, int n_taylor,
                             const double* vmat, const double* El, const double* Er,
                             const double* src, int src_ws, double* dst) {
  if (n <= 0) return hipSuccess;
  const int KT = c->MT / 16, NTC = (c->N + 15) / 16;
#define AFQMC_P(KM, NC)                                                                        \
  if (KT <= KM && NTC == NC)                                                                   \
    return launch_taylor_g_kt<T, KM, NC>(c, n, spins, n_taylor, vmat, El, Er, src, src_ws, dst);
  AFQMC_P(4, 1) AFQMC_P(6, 1) AFQMC_P(8, 1) AFQMC_P(10, 1)
  AFQMC_P(4, 2) AFQMC_P(6, 2) AFQMC_P(8, 2) AFQMC_P(10, 2)
  AFQMC_P(4, 3) AFQMC_P(6, 3) AFQMC_P(8, 3) AFQMC_P(10, 3)
#undef AFQMC_P
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_taylor_g_gen(const afqmc_ctx_s* c, int n, int spins, int n_taylor,
                               const double* vmat, const double* El, const double* Er,
                               const double* src, int src_ws, double* dst) {
  return taylor_g_dispatch<double>(c, n, spins, n_taylor, vmat, El, Er, src, src_ws, dst);
}

// the split-BF16 propagation from V stored split (launch_vbuild_split)
hipError_t launch_taylor_split(const afqmc_ctx_s* c, int nw, const unsigned short* Vs, double* phi) {
  if (nw <= 0) return hipSuccess;
  const int KT = c->MT / 16, NTC = (c->N + 15) / 16;
#define AFQMC_X(KM, NC) \
  if (KT <= KM && NTC == NC) return launch_taylor_x3<KM, NC>(c, nw, nullptr, Vs, phi);
  AFQMC_X(4, 1) AFQMC_X(6, 1) AFQMC_X(8, 1)
  AFQMC_X(4, 2) AFQMC_X(6, 2) AFQMC_X(8, 2)
#undef AFQMC_X
  return hipErrorInvalidValue;
}

hipError_t launch_taylor_g(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi) {
  if (nw <= 0) return hipSuccess;
  if (c->precision == AFQMC_PREC_BF16 && !c->ctrial) {
    // split-BF16 products (BF16 contexts take M <= 128, N <= 32)
    const int KT = c->MT / 16, NTC = (c->N + 15) / 16;
#define AFQMC_X(KM, NC) \
  if (KT <= KM && NTC == NC) return launch_taylor_x3<KM, NC>(c, nw, vmat, nullptr, phi);
    AFQMC_X(4, 1) AFQMC_X(6, 1) AFQMC_X(8, 1)
    AFQMC_X(4, 2) AFQMC_X(6, 2) AFQMC_X(8, 2)
#undef AFQMC_X
  }
  if (prop_f32(c))
    return taylor_g_dispatch<float>(c, nw, 2, c->n_taylor, vmat, c->d_Eh, c->d_Eh, phi, 2, phi);
  return taylor_g_dispatch<double>(c, nw, 2, c->n_taylor, vmat, c->d_Eh, c->d_Eh, phi, 2, phi);
}

// V split for the split-BF16 propagation of BF16 contexts: Vs [nw][Re hi, Re lo,
// -Im hi, -Im lo][M][MP] BF16, MP = M rounded up to 32 (zero past column M);
// scratch holds 8 nw GP bytes of split coefficients
bool vbuild_split_ok(const afqmc_ctx_s* c, int nw, size_t scratch_bytes) {
  return c->d_LTx != nullptr && c->precision == AFQMC_PREC_BF16 && !c->small && !c->ctrial &&
         c->MT / 16 <= 8 && (c->N + 15) / 16 <= 2 && scratch_bytes >= (size_t)8 * nw * c->GP;
}
hipError_t launch_vbuild_split(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                               unsigned short* Vs, void* scratch) {
  if (nw <= 0) return hipSuccess;
  return vbx_run<2, true>(c, nw, c->G, c->GP, (c->M + 31) / 32 * 32, sqrt(c->dtau), c->d_LTx, xi,
                          xbar, static_cast<unsigned short*>(scratch), Vs);
}

// U split for the split-BF16 trial series of BF16 contexts: Us [n][hi, lo][M][MP]
// BF16, MP = M rounded up to 32 (zero past column M), from split-BF16 products;
// scratch holds 4 n KP bytes of split coefficients
bool ubuild_split_ok(const afqmc_ctx_s* c, int n, size_t scratch_bytes) {
  return c->d_ATx != nullptr && scratch_bytes >= (size_t)4 * n * c->KP;
}
hipError_t launch_ubuild_split(const afqmc_ctx_s* c, int n, const double* y, unsigned short* Us,
                               void* scratch) {
  if (n <= 0) return hipSuccess;
  return vbx_run<1, true>(c, n, c->K, c->KP, (c->M + 31) / 32 * 32, c->coupling, c->d_ATx, y,
                          nullptr, static_cast<unsigned short*>(scratch), Us);
}

// U[s] = c sum_k y[s][k] A_k for n rows of y (the trial generators' product, Sec. II.C
// Eq. trial_decomp), stored as FP64.  FP64 products, except for BF16 contexts on the
// workgroup-per-path kernels, whose trial series rounds U to split BF16 (about 2^-17)
// as it loads it: split-BF16 products when scratch (4 n KP bytes) is given, else FP32.
hipError_t launch_ubuild(const afqmc_ctx_s* c, int n, const double* y, double* U, void* scratch,
                         size_t scratch_bytes) {
  if (n <= 0) return hipSuccess;
  const int MM = c->M * c->M;
  if (c->d_ATx != nullptr && scratch != nullptr && scratch_bytes >= (size_t)4 * n * c->KP)
    return vbx_run<1, false>(c, n, c->K, c->KP, c->M, c->coupling, c->d_ATx, y, nullptr,
                      static_cast<unsigned short*>(scratch), U);
  if (c->precision == AFQMC_PREC_BF16 && !c->small)
    return vb_launch<float, false, true>(c, n, c->K, MM, c->K, 0, c->coupling, c->d_A, y, nullptr,
                                         U);
  return vb_launch<double, false, true>(c, n, c->K, MM, c->K, 0, c->coupling, c->d_A, y, nullptr, U);
}

hipError_t launch_vbuild_gen(const afqmc_ctx_s* c, int n, int G, int xs, double sqrt_s,
                             const double* Lgen, const double* y, double* vmat,
                             const double* xbar, int xbs) {
  if (n <= 0) return hipSuccess;
  const int MM = c->M * c->M;
  if (xbar != nullptr)
    return vb_launch<double, true>(c, n, G, MM, xs, xbs, sqrt_s, Lgen, y, xbar, vmat);
  return vb_launch<double, false>(c, n, G, MM, xs, xbs, sqrt_s, Lgen, y, xbar, vmat);
}
