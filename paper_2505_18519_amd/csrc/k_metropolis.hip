// Metropolis update of the tethered paths at the moved walker and the hand-off
// projection (Sec. III.A, leapfrog step 2, Eqs. PDF-Y, AFQMC_Metro_correction,
// AFQMC_Metro_constraint_cos; App. B steps 2 and 3).
//
// One proposal round = k_proposal (y' for every path) -> trial build ->
// overlap (det only) at the moved walker -> k_accept.  The paths sample
// P(y; phi) ~ p_T(y) |O(y; phi)|: prior proposals (App. B) are accepted with
// |O(y')| / |O(y)|, the Gaussian random walk with |O(y')| N(y') / (|O(y)| N(y)),
// Ising single-spin flips with |O(y')| / |O(y)|, the learned proposal with
// |O(y')| N(y') q(y | z') / (|O(y)| N(y) q(y' | z)), whose log ratio of
// proposal and prior densities arrives precomputed (k_mlp_reverse).
// Accept iff u < alpha.
#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

// y' for every (walker, path): prior draw, random walk, or flip of y_k
__global__ void k_proposal(int nw, int P, int K, int hidden_kind, int proposal, double rw_step,
                           const double* __restrict__ y, double* __restrict__ ytry, uint64_t seed,
                           uint64_t step, const uint64_t* __restrict__ dstep, int sweep,
                           int flip_k) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)nw * P * K;
  if (idx >= total) return;
  if (dstep != nullptr) step = *dstep;
  const int k = (int)(idx % K);
  const size_t wp = idx / K;
  const int p = (int)(wp % P);
  const int w = (int)(wp / P);
  double v = y[idx];
  if (hidden_kind == AFQMC_HIDDEN_ISING) {
    if (k == flip_k) v = -v;
  } else {
    const double z =
        stream_normal(seed, w, step, rng_word3(AFQMC_TAG_PROPOSAL, sweep, p), (uint32_t)k);
    v = (proposal == AFQMC_PROPOSAL_RW) ? v + rw_step * z : z;
  }
  ytry[idx] = v;
}

// accept / reject per path; one workgroup of 256 threads per walker: the
// lanes of wavefront 0 decide, one per path, and every thread copies the
// accepted paths' rows over one flattened index
__global__ void __launch_bounds__(256)
k_accept(int nw, int P, int K, int MN, int hidden_kind, int proposal, double* __restrict__ y,
         double* __restrict__ phiT, double* __restrict__ logov, const double* __restrict__ ytry,
         const double* __restrict__ phiTtry, const double* __restrict__ ltry,
         int* __restrict__ nacc, uint64_t seed, uint64_t step, const uint64_t* __restrict__ dstep,
         int sweep, int flip_k, const double* __restrict__ lextra, int M,
         double* __restrict__ gd_cur, const double* __restrict__ gd_try, int* __restrict__ mask) {
  __shared__ int s_acc[64];
  __shared__ int s_list[64];  // the accepted paths of the chunk, in order
  __shared__ int s_nacc;
  if (dstep != nullptr) step = *dstep;
  const int w = blockIdx.x;
  const int tid = threadIdx.x, lane = tid;  // lanes of wavefront 0 decide, one per path
  int count = 0;
  for (int p0 = 0; p0 < P; p0 += 64) {
    const int p = p0 + lane;
    int acc = 0;
    if (tid < 64 && p < P) {
      const size_t wp = (size_t)w * P + p;
      const double lo = logov[wp * 2], ln = ltry[wp * 2];
      double la = ln - lo;
      if (proposal == AFQMC_PROPOSAL_RW && hidden_kind == AFQMC_HIDDEN_GAUSS) {
        double n_new = 0.0, n_old = 0.0;
        for (int k = 0; k < K; ++k) {
          const double a = ytry[wp * K + k], b = y[wp * K + k];
          n_new += a * a;
          n_old += b * b;
        }
        la += -0.5 * n_new + 0.5 * n_old;
      }
      if (lextra != nullptr) la += lextra[wp];
      const uint32_t ui = (hidden_kind == AFQMC_HIDDEN_ISING) ? (uint32_t)flip_k : 0u;
      const double u = stream_uniform(seed, w, step, rng_word3(AFQMC_TAG_ACCEPT, sweep, p), ui);
      if (__builtin_isnan(la)) la = neg_inf();
      acc = (la >= 0.0) || (u < exp(fmin(la, 0.0)));
      if (acc) {
        logov[wp * 2] = ln;
        logov[wp * 2 + 1] = ltry[wp * 2 + 1];
      }
      if (mask != nullptr) mask[wp] = acc;
    }
    if (tid < 64) s_acc[lane] = acc;
    __syncthreads();
    if (tid == 0) {  // compact list of the accepted paths
      const int np = min(64, P - p0);
      int n = 0;
      for (int q = 0; q < np; ++q)
        if (s_acc[q]) s_list[n++] = q;
      s_nacc = n;
    }
    __syncthreads();
    // copy the accepted paths' y and Phi_T (and Green's-function diagonals) with
    // every thread of the workgroup over one flattened index
    const int na = s_nacc;
    count += na;
    const size_t wp0 = (size_t)w * P + p0;
    for (size_t e = tid; e < (size_t)na * MN; e += blockDim.x) {
      const size_t wp = wp0 + s_list[e / MN];
      phiT[wp * MN + e % MN] = phiTtry[wp * MN + e % MN];
    }
    for (size_t e = tid; e < (size_t)na * K; e += blockDim.x) {
      const size_t wp = wp0 + s_list[e / K];
      y[wp * K + e % K] = ytry[wp * K + e % K];
    }
    if (gd_cur != nullptr)
      for (size_t e = tid; e < (size_t)na * M; e += blockDim.x) {
        const size_t wp = wp0 + s_list[e / M];
        gd_cur[wp * M + e % M] = gd_try[wp * M + e % M];
      }
    __syncthreads();
  }
  if (tid == 0 && nacc != nullptr) nacc[w] += count;
}

// W <- W max(0, cos(arg sum_p S'_p - arg ref)), or the half-plane rule; a
// non-finite sign sum, reference or weight sets W = 0 and the walker's flag
__global__ void __launch_bounds__(64)
k_handoff(int nw, int P, int weight_mode, const double* __restrict__ logov,
          const double* __restrict__ ref, double* __restrict__ w, int* __restrict__ flags) {
  const int wk = blockIdx.x;
  const int lane = threadIdx.x;
  double sr = 0.0, si = 0.0;
  for (int p = lane; p < P; p += 64) {
    const double* lo = logov + ((size_t)wk * P + p) * 2;
    if (!__builtin_isinf(lo[0])) {
      double s_, c_;
      sincos(lo[1], &s_, &c_);
      sr += c_;
      si += s_;
    }
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane != 0) return;
  const double rr = ref[(size_t)wk * 2], ri = ref[(size_t)wk * 2 + 1];
  const bool finite = __builtin_isfinite(sr) && __builtin_isfinite(si) &&
                      __builtin_isfinite(rr) && __builtin_isfinite(ri);
  const bool alive = finite && (sr != 0.0 || si != 0.0) && (rr != 0.0 || ri != 0.0);
  double fac = 0.0;
  if (alive) {
    const double dth = atan2(si, sr) - atan2(ri, rr);
    if (weight_mode == AFQMC_WEIGHT_HALFPLANE) {
      const double wrapped = atan2(sin(dth), cos(dth));
      fac = (fabs(wrapped) > 0.5 * M_PI) ? 0.0 : 1.0;
    } else {
      fac = fmax(0.0, cos(dth));
    }
  }
  const double wn = w[wk] * fac;
  const bool ok = finite && __builtin_isfinite(wn);
  w[wk] = ok ? wn : 0.0;
  if (!ok && flags != nullptr) flags[wk] |= AFQMC_NUMERIC_HANDOFF;
}

}  // namespace

hipError_t launch_proposal(const afqmc_ctx_s* c, int nw, const double* y, double* ytry,
                           uint64_t seed, uint64_t step, int sweep, int flip_k, int proposal) {
  const size_t total = (size_t)nw * c->P * c->K;
  if (total == 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_proposal, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, c->stream,
                     nw, c->P, c->K, c->hidden_kind, proposal, c->rw_step, y, ytry, seed, step,
                     c->dstep, sweep, flip_k);
  return hipGetLastError();
}

hipError_t launch_accept(const afqmc_ctx_s* c, int nw, double* y, double* phiT, double* logov,
                         const double* ytry, const double* phiTtry, const double* ltry, int* nacc,
                         uint64_t seed, uint64_t step, int sweep, int flip_k, int proposal,
                         const double* lextra, double* gd_cur, const double* gd_try, int* mask) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_accept, dim3(nw), dim3(256), 0, c->stream, nw, c->P, c->K, c->tsz,
                     c->hidden_kind, proposal, y, phiT, logov, ytry, phiTtry, ltry, nacc, seed,
                     step, c->dstep, sweep, flip_k, lextra, c->M, gd_cur, gd_try, mask);
  return hipGetLastError();
}

hipError_t launch_handoff(const afqmc_ctx_s* c, int nw, const double* logov, const double* ref,
                          double* w, int* flags) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_handoff, dim3(nw), dim3(64), 0, c->stream, nw, c->P, c->weight_mode, logov,
                     ref, w, flags);
  return hipGetLastError();
}
