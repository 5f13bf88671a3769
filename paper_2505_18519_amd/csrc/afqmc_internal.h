// Host-side context and kernel launchers of libafqmc (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/afqmc.h"

struct afqmc_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int M = 0, N = 0, G = 0, K = 0, P = 0, hidden_kind = 0;
  int MT = 0;  // M rounded up to a multiple of 16
  double coupling = 0, dtau = 0, rw_step = 0, xbar_cap = 0;
  int n_taylor = 10, weight_mode = 0, proposal = 0, precision = 0;

  // device copies owned by the context
  double* d_h1 = nullptr;    // [M][M]
  double* d_Lraw = nullptr;  // [G][M][M]
  double* d_Lpad = nullptr;  // [G+1][MT][MT], zero padded; slab G holds h1'
  double* d_Eh = nullptr;    // [M][M] = exp(-tau h1 / 2)
  double* d_phi0 = nullptr;  // [M][N]
  double* d_A = nullptr;      // [K][M][M] trial generators (dense)
  float* d_Lpad32 = nullptr;  // FP32 copy of d_Lpad (mixed-precision contraction)
  bool small = false;         // M <= 64 and N <= 16: register-resident kernels

  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
};

// Workspace carve-up for nw walkers (byte offsets, 256-aligned).
struct ws_layout {
  size_t vb, ep, vmat, ubuf, qrshift, ytry, phiTtry, ltry, acc, pc_C, pc_tot, pc_parent, pc_phi, pc_y, pc_phiT,
      pc_logov, total;
};
ws_layout afqmc_ws_layout(const afqmc_ctx_s* c, int nw);

#define AFQMC_LAUNCH_CHECK()                                   \
  do {                                                         \
    hipError_t e_ = hipGetLastError();                         \
    if (e_ != hipSuccess) return e_;                           \
  } while (0)

// kernel launchers (each returns the first HIP error it sees)
hipError_t launch_setup(afqmc_ctx_s* c);
hipError_t launch_trial_build(const afqmc_ctx_s* c, int n_samples, const double* y, double* phiT,
                              double* ubuf);
hipError_t launch_overlap(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                          double* logov, double* theta);
hipError_t launch_contract(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                           const double* logov, double* vb, double* ep);
hipError_t launch_combine(const afqmc_ctx_s* c, int nw, const double* vb, const double* ep,
                          const double* logov, double* xbar, double* eloc);
hipError_t launch_vbuild(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         double* vmat);
hipError_t launch_taylor(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi);
hipError_t launch_weight(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         const double* logov, const double* logov_new, double e_shift, double* w,
                         double* ref);
hipError_t launch_proposal(const afqmc_ctx_s* c, int nw, const double* y, double* ytry,
                           uint64_t seed, uint64_t step, int sweep, int flip_k);
hipError_t launch_accept(const afqmc_ctx_s* c, int nw, double* y, double* phiT, double* logov,
                         const double* ytry, const double* phiTtry, const double* ltry,
                         int* nacc, uint64_t seed, uint64_t step, int sweep, int flip_k);
hipError_t launch_handoff(const afqmc_ctx_s* c, int nw, const double* logov, const double* ref,
                          double* w);
hipError_t launch_qr(const afqmc_ctx_s* c, int nw, double* phi, double* logov);
hipError_t launch_estimator(const afqmc_ctx_s* c, int nw, const double* w, const double* eloc,
                            double* out);
hipError_t launch_philox_normal(const afqmc_ctx_s* c, uint64_t seed, uint64_t step, uint32_t tag,
                                int nw, int n, double* out);
hipError_t launch_sample_prior(const afqmc_ctx_s* c, int nw, uint64_t seed, double* y);
hipError_t launch_zero_int(const afqmc_ctx_s* c, int n, int* p);
hipError_t launch_trial_build_g(const afqmc_ctx_s* c, int n_samples, const double* y,
                                double* phiT, double* ubuf);
hipError_t launch_overlap_g(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                            double* logov, double* theta);
hipError_t launch_contract_g(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                             const double* logov, double* vb, double* ep);
hipError_t launch_taylor_g(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi);
hipError_t launch_qr_g(const afqmc_ctx_s* c, int nw, double* phi, double* logov, double* shift);
hipError_t launch_to_float(const afqmc_ctx_s* c, size_t n, const double* src, float* dst);
hipError_t launch_comb(const afqmc_ctx_s* c, int nw, double w_cap, double* w, double* C,
                       double* tot, int* parent, uint64_t seed, uint64_t step);
hipError_t launch_gather(const afqmc_ctx_s* c, int nw, size_t row, const int* parent,
                         const double* src, double* dst);
