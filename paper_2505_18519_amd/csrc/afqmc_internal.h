// Host-side context and kernel launchers of libafqmc (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/afqmc.h"

struct afqmc_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int M = 0, N = 0, G = 0, K = 0, P = 0, hidden_kind = 0;
  int MT = 0;  // M rounded up to a multiple of 16
  double coupling = 0, dtau = 0, rw_step = 0, xbar_cap = 0;
  // Re E_L clipped to [ecap_center - ecap_half, ecap_center + ecap_half] when ecap_half > 0
  double ecap_center = 0, ecap_half = 0;
  int n_taylor = 10, weight_mode = 0, proposal = 0, precision = 0;
  // FP64 contraction of real trials on the workgroup-per-path kernels: 0 keeps
  // Phi_T and Theta in registers (k_contract_g, N <= 32), 1 streams them from
  // L2 (k_contract_gs; always for 32 < N)
  int contract_variant = 0;

  // device copies owned by the context
  double* d_h1 = nullptr;    // [M][M]
  double* d_Lraw = nullptr;  // [G][M][M]
  double* d_Lpad = nullptr;  // [G+1][MT][MT], zero padded; slab G holds h1'
  double* d_Eh = nullptr;    // [M][M] = exp(-tau h1 / 2)
  double* d_phi0 = nullptr;  // [M][N]
  double* d_A = nullptr;      // [K][M][M] trial generators (dense)
  // every generator diagonal (the Ising pair operators): their diagonals, [K][M];
  // the trial build is then the row scaling exp(c sum_k y_k A_k[i][i]) of Phi_0
  double* d_Adiag = nullptr;
  float* d_Lpad32 = nullptr;  // FP32 copy of d_Lpad: A-operand order, row-major with ctrial
  unsigned short* d_Lbf = nullptr;     // BF16 copy of d_Lpad, A-operand order (BF16 contractions)
  unsigned short* d_Lbf_lo = nullptr;  // BF16 remainder d_Lpad - d_Lbf, same order (split BF16)
  // BF16 contexts on the workgroup kernels: L split into BF16 hi and lo and
  // transposed for the V build, [2][M*M][GP] (vectors contiguous, GP = G rounded
  // up to 32, zero padded)
  unsigned short* d_LTx = nullptr;
  int GP = 0;
  // the same for the trial generators A_k (U build), [2][M*M][KP], unless every
  // generator is diagonal
  unsigned short* d_ATx = nullptr;
  int KP = 0;
  bool small = false;         // M <= 64 and N <= 16: register-resident kernels
  bool c64 = false;           // walkers stored as complex64 (widened in the workspace)

  // trial family (AFQMC_TRIAL_*); multi-slice trials have complex Phi_T and
  // always run on the workgroup-per-path kernels
  int trial_kind = 0, n_slices = 0, kgen = 0, trial_taylor = 10;
  bool ctrial = false;
  int tsz = 0;                  // doubles per trial determinant: M N, or 2 M N if complex
  std::vector<double> slice_s;  // s_l of X_l = T_n(i sqrt(s_l) sum_k y_{l,k} A_k)
  double* d_F = nullptr;        // [m+1][M][M] one-body factors F_l
  double* d_phi0c = nullptr;    // [M][N] complex copy of Phi_0

  // Device-resident step counter (set by a batch whose step sequence is a
  // replayed graph): the kernels that take a step index read *dstep instead,
  // and the estimator writes its sums to out + 2 * (*dstep % est_cap).
  const uint64_t* dstep = nullptr;
  int est_cap = 1;

  void* ws = nullptr;
  size_t ws_bytes = 0;
  // device address of this GPU's fixed scratch array (afqmc_local_energy_static)
  void* d_scratch = nullptr;
  std::string err;
  // numerical-event flags: one int32 per walker at the start of the workspace;
  // the first flags_clear of them are known to be zero (host bookkeeping)
  int flags_clear = 0;
  bool numeric_check = false;  // per-step calls synchronise and report AFQMC_E_NUMERIC

  // learned proposal network (allocated by afqmc_mlp_init)
  struct mlp_state {
    bool ready = false, training = false;
    int prec = 0;             // AFQMC_PREC_FP32 or AFQMC_PREC_BF16
    int D = 0, Dp = 0;        // inputs M + K, rounded up to 16
    int O = 0, Op = 0;        // outputs 2K, rounded up to 16
    int64_t np = 0;           // parameters
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;  // flat offsets
    double lr = 1e-3, beta1 = 0.9, beta2 = 0.999, eps = 1e-8;
    float* master = nullptr;  // [np] FP32 parameters
    float* mom1 = nullptr;    // [np] Adam first moment
    float* mom2 = nullptr;    // [np] Adam second moment
    void* w1t = nullptr;      // [H][Dp]  W1^T in the product type
    void* w2t = nullptr;      // [H][H]   W2^T
    void* w3t = nullptr;      // [Op][H]  W3^T
    void* w2c = nullptr;      // [H][H]   W2
    void* w3c = nullptr;      // [H][Op]  W3
    int* tstep = nullptr;     // Adam step counter (device)
    double* scal = nullptr;   // [4] count, loss, 1/count (device)
  } mlp;
};

// Workspace carve-up for nw walkers (byte offsets, 256-aligned).
struct ws_layout {
  size_t flags;  // [nw] int32 numerical-event flags (AFQMC_NUMERIC_*), always at offset 0
  size_t vb, ep, vmat, ubuf, qrshift, ytry, phiTtry, ltry, acc, pc_C, pc_tot, pc_parent, pc_phi, pc_y, pc_phiT,
      pc_logov;
  // learned proposal (zero-sized unless proposal == LEARNED); Sp = paths rounded up to 16
  size_t gd_cur, gd_try, mlF, mlR, lqf, lqx, zT, h1T, h2T, dOT, dh2T, dh1T, nlq, part;
  // initialisation from the trial: the partner chain and both P = 1 chains'
  // determinants and log-overlaps (last, so that the same carve-up for P = 1
  // or without the network never reaches it)
  size_t in_yb, in_pa, in_pb, in_la, in_lb;
  size_t phi128;  // complex64 walkers: their FP64 copy [nw][2][M][N] complex (else 0 bytes)
  size_t total;
};
constexpr int MLP_CHUNK = 512;  // samples per split of the weight-gradient sums
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
                          double* logov, double* theta, double* gdiag);
hipError_t launch_contract(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                           const double* logov, double* vb, double* ep);
// flags (may be null): per-walker AFQMC_NUMERIC_* bits OR-ed in where a
// kernel finds a non-finite result
hipError_t launch_combine(const afqmc_ctx_s* c, int nw, const double* vb, const double* ep,
                          const double* logov, double* xbar, double* eloc, int* flags);
// scratch (may be null): device memory free for the call, used by BF16 contexts
// for their split coefficients when it holds scratch_bytes >= 8 nw GP
hipError_t launch_vbuild(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         double* vmat, void* scratch, size_t scratch_bytes);
// the split, transposed copy of L (d_LTx) of a BF16 context
hipError_t launch_lt_split(afqmc_ctx_s* c);
hipError_t launch_taylor(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi);
hipError_t launch_weight(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                         const double* logov, const double* logov_new, const double* eloc,
                         double e_shift, double* w, double* ref, int* flags);
// proposal: the kind of move (AFQMC_PROPOSAL_PRIOR or _RW; the learned
// proposal's random-walk moves pass _RW)
hipError_t launch_proposal(const afqmc_ctx_s* c, int nw, const double* y, double* ytry,
                           uint64_t seed, uint64_t step, int sweep, int flip_k, int proposal);
hipError_t launch_accept(const afqmc_ctx_s* c, int nw, double* y, double* phiT, double* logov,
                         const double* ytry, const double* phiTtry, const double* ltry,
                         int* nacc, uint64_t seed, uint64_t step, int sweep, int flip_k,
                         int proposal, const double* lextra = nullptr, double* gd_cur = nullptr,
                         const double* gd_try = nullptr, int* mask = nullptr);
hipError_t launch_handoff(const afqmc_ctx_s* c, int nw, const double* logov, const double* ref,
                          double* w, int* flags);
hipError_t launch_qr(const afqmc_ctx_s* c, int nw, double* phi, double* logov);
hipError_t launch_estimator(const afqmc_ctx_s* c, int nw, const double* w, const double* eloc,
                            double* out);
hipError_t launch_philox_normal(const afqmc_ctx_s* c, uint64_t seed, uint64_t step, uint32_t tag,
                                int nw, int n, double* out);
hipError_t launch_sample_prior(const afqmc_ctx_s* c, int nw, uint64_t seed, double* y,
                               int sweep = 0);
hipError_t launch_estimator_corrected(const afqmc_ctx_s* c, int nw, int Pr, const double* w,
                                      const double* eloc, const double* logov,
                                      const double* logov_ref, double* out, double* R);
// initialisation from the trial and measurement with extra paths (k_init.hip)
hipError_t launch_as_walker(const afqmc_ctx_s* c, int nw, const double* src, size_t stride,
                            double* dst);
hipError_t launch_sign_sum(const afqmc_ctx_s* c, int nw, int P, const double* logov, double* w);
hipError_t launch_extend_paths(const afqmc_ctx_s* c, int nw, int Ps, int Pd, const double* ys,
                               const double* ps, const double* ls, double* yd, double* pd,
                               double* ld);
hipError_t launch_zero_int(const afqmc_ctx_s* c, int n, int* p);
// complex64 <-> complex128 walker copies, n complex entries
hipError_t launch_phi_widen(const afqmc_ctx_s* c, size_t n, const float* src, double* dst);
hipError_t launch_phi_narrow(const afqmc_ctx_s* c, size_t n, const double* src, float* dst);
// scratch (may be null): device memory free for the call, passed to launch_ubuild
hipError_t launch_trial_build_g(const afqmc_ctx_s* c, int n_samples, const double* y,
                                double* phiT, double* ubuf, void* scratch = nullptr,
                                size_t scratch_bytes = 0);
hipError_t launch_overlap_g(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                            double* logov, double* theta, double* gdiag);
hipError_t launch_contract_g(const afqmc_ctx_s* c, int nw, const double* phiT, const double* theta,
                             const double* logov, double* vb, double* ep);
hipError_t launch_taylor_g(const afqmc_ctx_s* c, int nw, const double* vmat, double* phi);
// dst = El T_n(V) Er src for n blocks of `spins` M x N complex matrices (Er may be
// null); src block (w, sp) at (w * src_ws + sp) M N
hipError_t launch_taylor_g_gen(const afqmc_ctx_s* c, int n, int spins, int n_taylor,
                               const double* vmat, const double* El, const double* Er,
                               const double* src, int src_ws, double* dst);
// vmat[w] = i sqrt_s sum_k (y[w * xs + k] - xbar[w * xbs + k]) Lgen_k  (k < G;
// xbar complex, may be null)
// scratch (may be null): device memory free for the call (split coefficients of
// BF16 contexts, 4 n KP bytes)
hipError_t launch_ubuild(const afqmc_ctx_s* c, int n, const double* y, double* U, void* scratch,
                         size_t scratch_bytes);
// U split into BF16 hi and lo for the split-BF16 trial series, Us [n][2][M][MP]
// with MP = M rounded up to 32, when ubuild_split_ok (the split generator copy
// exists and scratch holds 4 n KP bytes)
bool ubuild_split_ok(const afqmc_ctx_s* c, int n, size_t scratch_bytes);
// V split for the split-BF16 propagation, Vs [nw][4][M][MP], and that
// propagation, when vbuild_split_ok (a BF16 context on the workgroup kernels
// and scratch of 8 nw GP bytes)
bool vbuild_split_ok(const afqmc_ctx_s* c, int nw, size_t scratch_bytes);
hipError_t launch_vbuild_split(const afqmc_ctx_s* c, int nw, const double* xi, const double* xbar,
                               unsigned short* Vs, void* scratch);
hipError_t launch_taylor_split(const afqmc_ctx_s* c, int nw, const unsigned short* Vs, double* phi);
hipError_t launch_ubuild_split(const afqmc_ctx_s* c, int n, const double* y, unsigned short* Us,
                               void* scratch);
hipError_t launch_vbuild_gen(const afqmc_ctx_s* c, int n, int G, int xs, double sqrt_s,
                             const double* Lgen, const double* y, double* vmat,
                             const double* xbar = nullptr, int xbs = 0);
// back-propagation (k_bp.hip)
hipError_t launch_bp_record(const afqmc_ctx_s* c, int nw, int h, int slot, const double* xi,
                            const double* xbar, double* hxi, double* hxb);
hipError_t launch_real_to_complex(const afqmc_ctx_s* c, size_t n, const double* src, double* dst);
hipError_t launch_bp_density(const afqmc_ctx_s* c, int nw, const double* theta, const double* phit,
                             const double* lt, const double* lend, double* rho, int* ok);
hipError_t launch_bp_reduce(const afqmc_ctx_s* c, int nw, const double* w, const double* rho,
                            const int* ok, double* out);
// multi-slice trial determinants Phi_T(Y) for n paths; vbuf holds n complex M x M
hipError_t launch_trial_slices(const afqmc_ctx_s* c, int n, const double* y, double* phiT,
                               double* vbuf);
hipError_t launch_qr_g(const afqmc_ctx_s* c, int nw, double* phi, double* logov, double* shift);
hipError_t launch_to_float(const afqmc_ctx_s* c, size_t n, const double* src, float* dst);
// FP32 (real trial), split-BF16 and BF16 contractions, two paths per workgroup
hipError_t launch_contract_sh(const afqmc_ctx_s* c, int nw, const double* phiT,
                              const double* theta, const double* logov, double* vb, double* ep);
hipError_t launch_to_bf16(const afqmc_ctx_s* c, size_t n, const double* src, unsigned short* hi,
                          unsigned short* lo);
hipError_t launch_to_f32_op(const afqmc_ctx_s* c, size_t n, const double* src, float* dst);
hipError_t launch_comb(const afqmc_ctx_s* c, int nw, double w_cap, int normalize, double* w,
                       double* C, double* tot, int* parent, uint64_t seed, uint64_t step);
hipError_t launch_gather(const afqmc_ctx_s* c, int nw, size_t row, const int* parent,
                         const double* src, double* dst);
hipError_t launch_copy(const afqmc_ctx_s* c, size_t n, const double* src, double* dst);
// the comb's walker arrays (row of row[p] doubles per walker), gathered by parent
// into their scratch copies tmp[p] and written back, in two launches
struct GatherParts {
  static constexpr int NPART = 4;
  double* state[NPART];
  double* tmp[NPART];
  size_t row[NPART];
  int nchunk[NPART];  // set by the launcher
};
hipError_t launch_gather_parts(const afqmc_ctx_s* c, int nw, const int* parent, GatherParts set);

// learned proposal network (k_mlp.hip); n = feature rows, Sp = n rounded up to 16
hipError_t launch_mlp_setparams(const afqmc_ctx_s* c, const double* src);
hipError_t launch_mlp_forward(const afqmc_ctx_s* c, int n, int Sp, const double* gd, const double* y,
                              float* out, void* zT, void* h1T, void* h2T);
hipError_t launch_mlp_propose(const afqmc_ctx_s* c, int nw, const float* out, const double* y,
                              uint64_t seed, uint64_t step, int sweep, double* ytry, double* lqf);
hipError_t launch_mlp_reverse(const afqmc_ctx_s* c, int n, const float* outR, const double* y,
                              const double* ytry, const double* lqf, double* lqx);
// yin: the y block of the forward pass's input; mask NULL = every row
hipError_t launch_mlp_backward(const afqmc_ctx_s* c, int n, int Sp, const float* out,
                               const double* yin, const double* ytgt, const int* mask,
                               const void* h1T, const void* h2T, void* dOT, void* dh2T, void* dh1T,
                               double* nlq);
hipError_t launch_mlp_wgrad(const afqmc_ctx_s* c, int Sp, const void* zT, const void* h1T,
                            const void* h2T, const void* dOT, const void* dh2T, const void* dh1T,
                            float* part);
hipError_t launch_mlp_reduce(const afqmc_ctx_s* c, int n, const int* mask, const double* nlq,
                             double* loss);
hipError_t launch_mlp_adam(const afqmc_ctx_s* c, int Sp, const float* part, double* grad);
hipError_t launch_mlp_outputs(const afqmc_ctx_s* c, int n, const float* out, const double* y,
                              double* mu, double* lv);
