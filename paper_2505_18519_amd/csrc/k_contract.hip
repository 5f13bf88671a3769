// Cholesky-vector contraction: force bias and local energy of every path
// (Sec. III.A, Eq. local-obs; Eq. shift1; Wick's theorem for <1/2 sum L^2>).
//
// Per path p and vector g (both spins s):
//   Y_g = Phi_T^T L_g (N x M, real, shared by the spins)
//   f_g^s = Y_g Theta^s (N x N complex)
//   vb_g = sum_s tr f_g^s,   ex = sum_g sum_s tr(f_g^s f_g^s)
//   E_p = sum_s tr(Phi_T^T h1' Theta^s) + 1/2 sum_g vb_g^2 - 1/2 ex
// h1' rides along as slab g = n_chol of the padded L array, so the one-body
// term costs one more pass of the same loop.
//
// Layout on gfx950: one wavefront per path, CW wavefronts per workgroup.  The
// path's Phi_T and Theta live in registers as FP64-MFMA B operands for the
// whole loop over g.  L_g is double-buffered in LDS and shared by the CW
// wavefronts; each slab goes from global memory straight into LDS
// (global_load_lds, 16 bytes per lane), issued once the current slab's
// stage-1 reads are out, so no registers hold it in flight.  Stage 1
// (Y_g^T = L_g Phi_T) leaves Y_g in the accumulator layout, which is exactly
// the A-operand layout of stage 2 when the contraction index m is visited in
// the order m = 16 t + 4 r + g, so the two stages chain in registers; its A
// operands are read from LDS one step ahead.  tr(f f) needs f transposed: it
// goes through a per-wave LDS tile, and that tail of vector g - 1 is issued
// ahead of stage 1 of vector g, so its LDS traffic overlaps the matrix core.
// Nothing of size n_chol x N^2 touches HBM.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

constexpr int CW = 4;  // wavefronts (paths) per workgroup
constexpr int FL = 16;  // vectors per flush of the staged diagonals

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* gbl_ptr_t;

template <int MT>
__global__ void __launch_bounds__(CW * 64)
k_contract(int n_samples, int M, int N, int G, const double* __restrict__ Lpad,
           const double* __restrict__ phiT, const double* __restrict__ theta,
           const double* __restrict__ logov, double* __restrict__ vb, double* __restrict__ ep) {
  constexpr int NTILE = MT / 16;
  constexpr int SLAB = MT * MT;
  constexpr int NCH = SLAB / 128;  // 1 KB chunks of a slab: 64 lanes x 16 bytes
  constexpr int KS = 4 * NTILE;    // steps of the contraction index in stage 1
  __shared__ __attribute__((aligned(16))) double s_L[2][SLAB];
  __shared__ double s_f[CW][4][16][17];
  __shared__ double s_dg[CW][FL][2][17];  // diagonal partials; column 16 takes the other lanes

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4, c = lane & 15;
  const int s = blockIdx.x * CW + wave;
  bool active = s < n_samples;
  if (active) active = !__builtin_isinf(logov[2 * s]);  // singular paths contribute zero

  // slab copies go from global memory straight into LDS; wave w takes chunks w, w + CW, ...
  auto copy_slab = [&](int slab, int buf) {
    const double* src = Lpad + (size_t)slab * SLAB;
#pragma unroll
    for (int k = wave; k < NCH; k += CW)
      __builtin_amdgcn_global_load_lds((gbl_ptr_t)(src + k * 128 + lane * 2),
                                       (lds_ptr_t)(s_L[buf] + k * 128), 16, 0, 0);
  };
  copy_slab(0, 0);

  // B operands: bT[t][r] = Phi_T[16t+4r+g][c]; bth[sp][ri][t][r] = Theta^sp[16t+4r+g][c]
  double bT[NTILE][4];
  double bth[2][2][NTILE][4];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * t + 4 * r + g;
      const bool ok = active && m < M && c < N;
      bT[t][r] = ok ? phiT[((size_t)s * M + m) * N + c] : 0.0;
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        const double* src = theta + ((((size_t)s * 2 + sp) * M + m) * N + c) * 2;
        bth[sp][0][t][r] = ok ? src[0] : 0.0;
        bth[sp][1][t][r] = ok ? src[1] : 0.0;
      }
    }

  double vb2_re = 0.0, vb2_im = 0.0, ex_re = 0.0, ex_im = 0.0;
  double(*sf)[16][17] = s_f[wave];
  double(*sdg)[2][17] = s_dg[wave];
  // lanes holding a diagonal element f[c][c] (c = g + 4 r): r = c / 4 when c % 4 == g
  const int dcol = ((c & 3) == g) ? c : 16;

  // stage 1: y1[tp] = (L_g Phi_T)[16tp + 4r + g][c], A operands read one step ahead
  auto stage1 = [&](const double* Ls, dx4 (&y1)[NTILE]) {
#pragma unroll
    for (int tp = 0; tp < NTILE; ++tp) y1[tp] = dx4_zero();
    double ac[NTILE], an[NTILE];
#pragma unroll
    for (int tp = 0; tp < NTILE; ++tp) ac[tp] = Ls[g * MT + 16 * tp + c];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      if (k + 1 < KS) {
#pragma unroll
        for (int tp = 0; tp < NTILE; ++tp) an[tp] = Ls[(4 * (k + 1) + g) * MT + 16 * tp + c];
      }
      // A[c][g] = L[16tp+c][16t+4r+g] = L[16t+4r+g][16tp+c] (L symmetric), k = 4t + r
#pragma unroll
      for (int tp = 0; tp < NTILE; ++tp) y1[tp] = mfma_f64(ac[tp], bT[k >> 2][k & 3], y1[tp]);
      if (k + 1 < KS) {
#pragma unroll
        for (int tp = 0; tp < NTILE; ++tp) ac[tp] = an[tp];
      }
    }
  };
  // stage 2: f[sp][ri] = sum_m Y[c'][m] Theta^sp[m][c]  (rows g+4r, col c)
  auto stage2 = [&](const dx4 (&y1)[NTILE], dx4 (&f)[2][2]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) f[sp][0] = f[sp][1] = dx4_zero();
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int ri = 0; ri < 2; ++ri) f[sp][ri] = mfma_f64(y1[t][r], bth[sp][ri][t][r], f[sp][ri]);
  };
  // diagonal of f summed over the spins, in the lanes that hold one (0 elsewhere)
  auto diag = [&](const dx4 (&f)[2][2], double& d_re, double& d_im) {
    d_re = 0.0;
    d_im = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (c == g + 4 * r) {
        d_re = f[0][0][r] + f[1][0][r];
        d_im = f[0][1][r] + f[1][1][r];
      }
  };
  // tail of vector gv: stage its diagonal for vb_gv and add sum_ij f_ij f_ji to ex.  The
  // transpose goes through this wave's LDS tile.  LDS operations of one wavefront execute in
  // order, so the reads see the writes without a wait in between; the wave barrier only
  // keeps the compiler from moving the reads above the writes.
  auto tail = [&](const dx4 (&f)[2][2], int gv) {
    double d_re, d_im;
    diag(f, d_re, d_im);
    sdg[gv % FL][0][dcol] = d_re;
    sdg[gv % FL][1][dcol] = d_im;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int r = 0; r < 4; ++r) sf[2 * sp + ri][g + 4 * r][c] = f[sp][ri][r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double tr_ = sf[2 * sp][c][g + 4 * r];
        const double ti_ = sf[2 * sp + 1][c][g + 4 * r];
        const double ar = f[sp][0][r], ai = f[sp][1][r];
        ex_re += ar * tr_ - ai * ti_;
        ex_im += ar * ti_ + ai * tr_;
      }
  };
  // bulk reduction of FL staged vectors: lane l < 2 FL sums part l / FL of vector l % FL
  auto flush = [&](int g_first, int count) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int gl = lane % FL, part = (lane / FL) & 1;
    double v = 0.0;
    if (lane < 2 * FL && gl < count) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v += sdg[gl][part][q];
    }
    const double vi = __shfl_down(v, FL, 64);  // lanes < FL: imaginary part
    if (lane < FL && gl < count) {
      vb2_re += v * v - vi * vi;
      vb2_im += 2.0 * v * vi;
      double* o = vb + ((size_t)s * G + g_first + gl) * 2;
      o[0] = v;
      o[1] = vi;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };

  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks of slab 0 are in LDS
  __syncthreads();
  // vector 0: both stages; its tail runs during stage 1 of vector 1
  dx4 f[2][2];
  if (active) {
    dx4 y1[NTILE];
    stage1(s_L[0], y1);
    copy_slab(G > 0 ? 1 : 0, 1);
    stage2(y1, f);
  } else {
    copy_slab(G > 0 ? 1 : 0, 1);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();

  // slab gam is in buffer gam & 1; slab G is h1', whose diagonal gives the one-body term
  for (int gam = 1; gam <= G; ++gam) {
    const int b = gam & 1;
    const int nxt = gam < G ? gam + 1 : gam;  // the last copy repeats a slab no one reads
    if (active) {
      dx4 y1[NTILE];
      tail(f, gam - 1);
      stage1(s_L[b], y1);
      // buffer b ^ 1 was last read in the previous iteration, which the barrier closed
      copy_slab(nxt, b ^ 1);
      stage2(y1, f);
      if ((gam - 1) % FL == FL - 1 || gam == G) flush(gam - 1 - (gam - 1) % FL, (gam - 1) % FL + 1);
    } else {
      copy_slab(nxt, b ^ 1);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's chunks of the next slab landed
    __syncthreads();
  }

  if (s < n_samples) {
    double e1_re = 0.0, e1_im = 0.0;
    if (active) {
      double d_re, d_im;
      diag(f, d_re, d_im);
      e1_re = wave_sum(d_re);
      e1_im = wave_sum(d_im);
    }
    ex_re = wave_sum(ex_re);
    ex_im = wave_sum(ex_im);
    vb2_re = wave_sum(vb2_re);
    vb2_im = wave_sum(vb2_im);
    if (lane == 0) {
      double* o = ep + (size_t)s * 2;
      if (active) {
        o[0] = e1_re + 0.5 * vb2_re - 0.5 * ex_re;
        o[1] = e1_im + 0.5 * vb2_im - 0.5 * ex_im;
      } else {
        o[0] = 0.0;
        o[1] = 0.0;
      }
    }
    if (!active)
      for (int q = lane; q < 2 * G; q += 64) vb[(size_t)s * G * 2 + q] = 0.0;
  }
}

// Walker-level estimates over the P paths (Eq. local-obs, then Eq. shift1):
// S_p = exp(i Im l_p) (0 if singular), xbar_g = -i sqrt(tau) sum S vb / sum S,
// E_L = sum S E_p / sum S.  One workgroup of 64 threads per walker.  A
// non-finite E_L or force-bias component sets the walker's flag bits.  With
// ecap_half > 0 a finite Re E_L is clipped to [ecap_lo, ecap_hi] (Im E_L kept).
__global__ void __launch_bounds__(64)
k_combine(int nw, int P, int G, double sqrt_tau, double xbar_cap, double ecap_half,
          double ecap_lo, double ecap_hi, const double* __restrict__ vb,
          const double* __restrict__ ep, const double* __restrict__ logov,
          double* __restrict__ xbar, double* __restrict__ eloc, int* __restrict__ flags) {
  __shared__ double s_S[64][2];
  const int w = blockIdx.x;
  const int lane = threadIdx.x;
  for (int p = lane; p < P; p += 64) {
    const double lr = logov[((size_t)w * P + p) * 2], li = logov[((size_t)w * P + p) * 2 + 1];
    double sr = 0.0, si = 0.0;
    if (!__builtin_isinf(lr)) sincos(li, &si, &sr);
    s_S[p][0] = sr;
    s_S[p][1] = si;
  }
  __syncthreads();
  cplx den = cmk(0.0, 0.0);
  for (int p = 0; p < P; ++p) den = cadd(den, cmk(s_S[p][0], s_S[p][1]));
  const bool good = (den.re != 0.0 || den.im != 0.0);
  bool bad_xb = false;
  if (xbar != nullptr) {
    for (int gm = lane; gm < G; gm += 64) {
      cplx num = cmk(0.0, 0.0);
      for (int p = 0; p < P; ++p)
        num = cfma(num, cmk(s_S[p][0], s_S[p][1]), cld(vb + (((size_t)w * P + p) * G + gm) * 2));
      cplx v = good ? cdiv(num, den) : cmk(0.0, 0.0);
      // -i sqrt(tau) v, modulus optionally clipped to xbar_cap
      cplx xb = cmk(sqrt_tau * v.im, -sqrt_tau * v.re);
      if (xbar_cap > 0.0) {
        const double mag = sqrt(cabs2(xb));
        if (mag > xbar_cap) xb = cscale(xb, xbar_cap / mag);
      }
      cst(xbar + ((size_t)w * G + gm) * 2, xb);
      bad_xb |= !(__builtin_isfinite(xb.re) && __builtin_isfinite(xb.im));
    }
  }
  const bool any_bad_xb = __ballot(bad_xb) != 0;
  if (lane != 0) return;
  int bits = any_bad_xb ? AFQMC_NUMERIC_XBAR : 0;
  if (eloc != nullptr) {
    cplx num = cmk(0.0, 0.0);
    for (int p = 0; p < P; ++p)
      num = cfma(num, cmk(s_S[p][0], s_S[p][1]), cld(ep + ((size_t)w * P + p) * 2));
    cplx el = good ? cdiv(num, den) : cmk(0.0, 0.0);
    if (!(__builtin_isfinite(el.re) && __builtin_isfinite(el.im))) bits |= AFQMC_NUMERIC_ELOC;
    else if (ecap_half > 0.0) el.re = fmin(fmax(el.re, ecap_lo), ecap_hi);
    cst(eloc + (size_t)w * 2, el);
  }
  if (bits != 0 && flags != nullptr) flags[w] |= bits;
}

template <int MT>
hipError_t launch_mt(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                     const double* logov, double* vb, double* ep) {
  const int n = nw * c->P;
  dim3 grid((n + CW - 1) / CW), block(CW * 64);
  hipLaunchKernelGGL(k_contract<MT>, grid, block, 0, c->stream, n, c->M, c->N, c->G, c->d_Lpad,
                     phiT, theta, logov, vb, ep);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                           const double* logov, double* vb, double* ep) {
  if (nw <= 0) return hipSuccess;
  switch (c->MT) {
    case 32: return launch_mt<32>(c, nw, phiT, theta, logov, vb, ep);
    case 64: return launch_mt<64>(c, nw, phiT, theta, logov, vb, ep);
    case 16: return launch_mt<16>(c, nw, phiT, theta, logov, vb, ep);
    case 48: return launch_mt<48>(c, nw, phiT, theta, logov, vb, ep);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_combine(const afqmc_ctx_s* c, int nw, const double* vb, const double* ep,
                          const double* logov, double* xbar, double* eloc, int* flags) {
  if (nw <= 0) return hipSuccess;
  if (c->P > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_combine, dim3(nw), dim3(64), 0, c->stream, nw, c->P, c->G, sqrt(c->dtau),
                     c->xbar_cap, c->ecap_half, c->ecap_center - c->ecap_half,
                     c->ecap_center + c->ecap_half, vb, ep, logov, xbar, eloc, flags);
  return hipGetLastError();
}
