/*
 * afqmc.h -- C ABI of the MI355X (gfx950) hot path of phaseless AFQMC with a
 * stochastically sampled correlated trial wave function
 * Psi_T = int dy p_T(y) det Phi_T(y), each walker tethered to P Metropolis
 * paths over the hidden variables y (Sec. III.A and App. B of the paper).
 *
 * Conventions shared by every call
 * --------------------------------
 * Hamiltonian (Sec. II.A, Eqs. H and H_MC):  H = sum_s h1 + 1/2 sum_g L_g^2
 * with real symmetric h1 [M][M] and L_g [M][M]; restricted closed-shell
 * walkers with N electrons of each spin.
 * Trial (Sec. II.C, Eq. trial_decomp, m = 1):  Phi_T(y) = exp(c sum_k y_k A_k) Phi_0
 * with real symmetric generators A_k and hidden variables y_k either Ising
 * (+-1, uniform prior) or Gaussian (N(0,1) prior).
 * Propagator (Eqs. HS, walker_prop):  B(x) = e^{-tau h1/2} exp(V) e^{-tau h1/2},
 * V = i sqrt(tau) sum_g (x_g - xbar_g) L_g, exp(V) applied as the Taylor
 * series of fixed order n_taylor.
 *
 * All array arguments of the per-step calls are DEVICE pointers to
 * contiguous row-major arrays; "complex" means interleaved (re, im) doubles:
 *   phi    [nw][2][M][N]    complex  walker determinants (spin up, spin down)
 *   w      [nw]             double   walker weights
 *   y      [nw][P][K]       double   hidden variables of the P paths
 *   phiT   [nw][P][M][N]    double   sampled trial determinants Phi_T(y_p)
 *   logov  [nw][P]          complex  l_p = sum_s log det(Phi_T(y_p)^T phi^s)
 *                                    (-inf + 0i marks a singular overlap)
 *   theta  [nw][P][2][M][N] complex  Theta^s = phi^s (Phi_T^T phi^s)^{-1}
 * The caller owns every state array and the workspace; the library owns the
 * device copy of the system made by afqmc_create.  Calls are asynchronous on
 * the context's stream; they validate arguments on the host and never abort.
 * Non-finite results are data, flagged per walker (see "Numerical events").
 * Walker k's random numbers depend only on (seed, step, k), so any nw-prefix
 * of a batch reproduces the same walkers.
 */
#ifndef AFQMC_H
#define AFQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afqmc_ctx_s* afqmc_ctx;

typedef enum {
  AFQMC_OK = 0,
  AFQMC_E_INVALID = 1,      /* null pointer, bad enum or parameter value           */
  AFQMC_E_SHAPE = 2,        /* sizes outside what the kernels support             */
  AFQMC_E_DEVICE = 3,       /* a HIP runtime call failed                           */
  AFQMC_E_NOMEM = 4,        /* device allocation in afqmc_create failed            */
  AFQMC_E_NUMERIC = 5,      /* a kernel produced a non-finite E_L, force bias or weight
                               (afqmc_numeric_flags; per-step calls with the check on) */
  AFQMC_E_UNSUPPORTED = 6,  /* valid request this build does not implement         */
  AFQMC_E_WORKSPACE = 7     /* no workspace set, or smaller than afqmc_workspace_size */
} afqmc_status;

enum { AFQMC_HIDDEN_ISING = 0, AFQMC_HIDDEN_GAUSS = 1 };

/* Weight projections (Sec. III.A after Eq. AFQMC_Metro_constraint_cos; App. B):
 * SEPARATE: |I| max(0, cos dtheta) at the walker move, then max(0, cos dtheta_T)
 *           at the hand-off (the pseudo-code of App. B);
 * COMBINED: |I| at the move and one max(0, cos(dtheta + dtheta_T)) at the hand-off;
 * HALFPLANE: cosine at the move, W = 0 if |dtheta_T| > pi/2 at the hand-off;
 * LOCAL: the local-energy formalism (Sec. III.A, after Eq. importance_function_CP):
 *           |I| = exp(-tau (Re E_L - E_T)) with the walker's E_L of Eq.
 *           local-obs before the move, times max(0, cos dtheta); hand-off as
 *           SEPARATE.                                                          */
enum { AFQMC_WEIGHT_SEPARATE = 0, AFQMC_WEIGHT_COMBINED = 1, AFQMC_WEIGHT_HALFPLANE = 2,
       AFQMC_WEIGHT_LOCAL = 3 };

/* Metropolis proposals for the paths (Sec. III.A, leapfrog step 2):
 * PRIOR: independent draw from p_T (App. B); for Ising y one sweep flips
 *        y_0 .. y_{K-1} in turn.  RW: Gaussian random walk y' = y + rw_step * eta.
 * LEARNED (an extension, Gaussian y only): a block move of all K variables from
 *        the proposal network below (afqmc_mlp_*). */
enum { AFQMC_PROPOSAL_PRIOR = 0, AFQMC_PROPOSAL_RW = 1, AFQMC_PROPOSAL_LEARNED = 2 };

/* Precision of the Cholesky contraction (force bias and local energy):
 * FP64 throughout; FP32: Phi_T, Theta and L enter the FP32 matrix-core
 * products with FP32 accumulation over the orbital index; BF16: the same
 * products with bfloat16 operands (one product per pair, about 3 significant
 * digits); BF16X3 (split bfloat16): each operand x carried as hi = bf16(x) and
 * lo = bf16(x - hi), each product as hi*hi + hi*lo + lo*hi (close to FP32
 * accuracy).  In every form the traces, vb_g^2, the sums over g and every
 * other step of the path stay FP64.  Contexts other than FP64 also build the
 * trial series and propagate the walkers with FP32 products; BF16 contexts
 * on the workgroup-per-path kernels (M > 64 or N > 16) build U, the trial
 * series, V and the walker propagation on split-bfloat16 products instead
 * (Phi_T within about 2e-5, phi' about 1e-5 of FP64); their contexts keep
 * split, transposed copies of L and the generators (4 G M^2 + 4 K M^2 bytes).
 * BF16 and BF16X3 need the real trial family (AFQMC_E_UNSUPPORTED otherwise).  The proposal network's own
 * precision is set separately (afqmc_mlp_init: FP32 or BF16). */
enum {
  AFQMC_PREC_FP64 = 0,
  AFQMC_PREC_FP32 = 1,
  AFQMC_PREC_BF16 = 2,
  AFQMC_PREC_BF16X3 = 3
};

/* Trial families (Sec. II.C, Eqs. trial, trial-AF and trial_decomp):
 * JASTROW: Phi_T(y) = exp(c sum_k y_k A_k) Phi_0, real;
 * SLICES:  Phi_T(Y) = F_m X_m ... F_1 X_1 F_0 Phi_0 with Y = (y_1 .. y_m),
 *          X_l = T_n(i sqrt(s_l) sum_k y_{l,k} A_k) (n = trial_taylor, the
 *          Taylor map of the propagator) and real one-body factors F_l: the
 *          imaginary-time-evolved trial e^{-m tau_T H} Phi_0 of Sec. III.B and
 *          the VAFQMC form of Eq. VAFQMC.  Complex: every phiT argument of a
 *          SLICES context is interleaved complex [..][M][N][2], the overlaps
 *          stay the bilinear det(Phi_T^T phi).  SLICES needs Gaussian hidden
 *          variables, a non-learned proposal and (ceil(M/16)) (ceil(N/16)) <= 8,
 *          and uses the workgroup-per-path kernels at every size. */
enum { AFQMC_TRIAL_JASTROW = 0, AFQMC_TRIAL_SLICES = 1 };

typedef struct {
  int32_t M;            /* one-particle basis size                         */
  int32_t N;            /* electrons per spin (n_up = n_dn)                */
  int32_t n_chol;       /* number of vectors L_g                           */
  int32_t K;            /* hidden variables per path                       */
  int32_t P;            /* paths tethered to each walker                   */
  int32_t hidden_kind;  /* AFQMC_HIDDEN_*                                   */
  double coupling;      /* c in Phi_T(y) = exp(c sum_k y_k A_k) Phi_0        */
  const double* h1;     /* HOST [M][M], symmetric                           */
  const double* L;      /* HOST [n_chol][M][M], each symmetric              */
  const double* phi0;   /* HOST [M][N]                                      */
  const double* A;      /* HOST [K][M][M] each symmetric ([K/m] for SLICES)  */
  double dtau;          /* time step tau                                    */
  int32_t n_taylor;     /* Taylor order of exp(V) in the propagator (>= 1)  */
  int32_t weight_mode;  /* AFQMC_WEIGHT_*                                    */
  int32_t proposal;     /* AFQMC_PROPOSAL_*                                  */
  double rw_step;       /* random-walk proposal step                        */
  int32_t precision;    /* AFQMC_PREC_*                                      */
  double xbar_cap;      /* > 0: clip |xbar_g| to xbar_cap, phase kept (a common
                           AFQMC stabilisation the paper does not use); 0: off */
  int32_t trial_kind;   /* AFQMC_TRIAL_* (0: JASTROW)                        */
  int32_t n_slices;     /* SLICES: m >= 1; K = m * (generators in A)         */
  const double* slice_s;  /* SLICES: HOST [m], s_l >= 0                      */
  const double* slice_F;  /* SLICES: HOST [m+1][M][M], F_0 .. F_m             */
  int32_t trial_taylor; /* SLICES: Taylor order n of X_l (>= 1)              */
  int32_t walker_c64;   /* 1: every phi argument (walkers) is complex64, [nw][2][M][N]
                           interleaved FLOAT pairs: the calls widen it to FP64 in
                           the workspace and round the moved or re-orthonormalised
                           walkers back to complex64.  Needs a reduced-precision
                           contraction (precision != FP64) and the real trial
                           family; not with afqmc_init_metropolis, the
                           back-propagation calls or batches. 0: complex128. */
} afqmc_system;

/* Copies the system to device `device`, derives h1' = h1 + 1/2 sum_g L_g^2 and
 * e^{-tau h1/2} there, and binds the context to `stream` (a hipStream_t, NULL
 * for the default stream).  Host arrays may be freed on return.
 * Supported sizes: 1 <= N <= M <= 160, N <= 40, n_chol >= 1, K >= 1,
 * 1 <= P <= 64; other sizes return AFQMC_E_SHAPE.  Past M = 128 or N = 32
 * only the FP64 contraction and the prior and random-walk proposals are
 * built (AFQMC_E_UNSUPPORTED otherwise).  The learned proposal needs
 * Gaussian hidden variables and K <= 128.  Real-trial systems with
 * M <= 64 and N <= 16 use register-resident kernels, larger ones (and every
 * multi-slice trial) workgroup-per-path kernels.  Multi-slice trials need
 * ceil(M/16) ceil(N/16) <= 8 (AFQMC_E_UNSUPPORTED otherwise), Gaussian hidden
 * variables and a non-learned proposal.  Invalid arguments (missing arrays,
 * non-finite dtau or coupling, an unknown mode) return AFQMC_E_INVALID.
 * Synchronises `stream`. */
afqmc_status afqmc_create(const afqmc_system* sys, int device, void* stream, afqmc_ctx* out);
afqmc_status afqmc_destroy(afqmc_ctx ctx);
/* Text of the last error on this context (static storage owned by ctx). */
const char* afqmc_last_error(afqmc_ctx ctx);
afqmc_status afqmc_set_stream(afqmc_ctx ctx, void* stream);

/* Device scratch the per-step calls need for up to nw walkers.  The caller
 * allocates it (>= 256-byte aligned) and hands it over; calls that overlap on
 * one context must not share a workspace.  No per-step call allocates.      */
afqmc_status afqmc_workspace_size(afqmc_ctx ctx, int32_t nw, size_t* bytes);
afqmc_status afqmc_set_workspace(afqmc_ctx ctx, void* dptr, size_t bytes);

/* ---- Numerical events --------------------------------------------------------
 * A walker whose local energy, force bias or weight comes out non-finite (for
 * instance from a NaN or Inf in its inputs, or an overlap too ill-conditioned
 * for FP64) is kept as data: its E_L leaves the estimator sums and its weight
 * is set to 0, so one such walker never turns a population estimate into NaN.
 * The kernels that write E_L, the force bias and W also OR these bits into a
 * per-walker int32 flag word, flags[k], held in the first 4 nw bytes of the
 * workspace:
 *   AFQMC_NUMERIC_ELOC     E_L non-finite             (afqmc_local_energy)
 *   AFQMC_NUMERIC_XBAR     a force-bias component     (afqmc_local_energy,
 *                          non-finite                  afqmc_force_bias)
 *   AFQMC_NUMERIC_WEIGHT   the move's weight update   (afqmc_propagate)
 *                          non-finite (W set to 0)
 *   AFQMC_NUMERIC_HANDOFF  the hand-off's sign sum,   (afqmc_metropolis_x)
 *                          reference or weight non-finite (W set to 0)
 * Flags accumulate until afqmc_numeric_flags reads and clears them, or until
 * afqmc_set_workspace installs a new workspace (whose flags start clear).  A
 * call made with no workspace set (afqmc_local_energy or afqmc_force_bias
 * with every per-path output given) records no flags. */
enum { AFQMC_NUMERIC_ELOC = 1, AFQMC_NUMERIC_XBAR = 2, AFQMC_NUMERIC_WEIGHT = 4,
       AFQMC_NUMERIC_HANDOFF = 8 };

/* Synchronises the context's stream, copies the flag words of walkers
 * 0 .. nw-1 to flags (HOST int32 [nw], may be NULL), stores the number of
 * flagged walkers in *n_flagged (may be NULL), and clears those words.
 * Returns AFQMC_E_NUMERIC if any of them was set (the text of
 * afqmc_last_error names the count and the first walker), AFQMC_OK if none
 * was, AFQMC_E_WORKSPACE without a workspace for nw walkers. */
afqmc_status afqmc_numeric_flags(afqmc_ctx ctx, int32_t nw, int32_t* flags, int32_t* n_flagged);

/* on = 1: afqmc_local_energy, afqmc_force_bias, afqmc_propagate and
 * afqmc_metropolis_x clear the flags of their nw walkers first, synchronise
 * the stream after their kernels, and return AFQMC_E_NUMERIC if one of those
 * walkers was flagged (their outputs are written as always; the flags stay
 * for afqmc_numeric_flags).  on = 0 (the default): those calls stay
 * asynchronous and never report numerical events themselves. */
afqmc_status afqmc_set_numeric_check(afqmc_ctx ctx, int32_t on);

/* Local-energy cap (a stabilisation the paper does not state; the usual
 * phaseless-AFQMC practice of clipping E_L at E_T +- sqrt(2 / tau)): with
 * half_width > 0, every walker's E_L that afqmc_local_energy (and its
 * static variant) writes has its real part clipped to
 * [center - half_width, center + half_width] before it reaches the caller,
 * the estimator or the local-energy weight; the imaginary part, the per-path
 * E_p and non-finite values (which set AFQMC_NUMERIC_ELOC) are not changed.
 * half_width = 0 (the default) turns it off.  The setting belongs to the
 * context and holds for every later call until changed; centre and width
 * must be finite and width >= 0 (AFQMC_E_INVALID otherwise, setting
 * unchanged). */
afqmc_status afqmc_set_eloc_cap(afqmc_ctx ctx, double center, double half_width);

/* Tile strategy of the FP64 Cholesky contraction (Sec. III.A, Eq. local-obs)
 * for real trials on the workgroup-per-path kernels (M > 64 or N > 16):
 * variant 0 (default) keeps Phi_T and Theta in registers across the vectors
 * (N <= 32), variant 1 streams them from L2 one k tile ahead of the products;
 * N > 32 always streams.  Same results to rounding.  Other contexts ignore it.
 * AFQMC_E_INVALID for a variant other than 0 or 1. */
afqmc_status afqmc_set_contraction_variant(afqmc_ctx ctx, int32_t variant);

/* Initial paths y ~ p_T (stream INIT of the counter layout below). */
afqmc_status afqmc_sample_prior(afqmc_ctx ctx, int32_t nw, uint64_t seed, double* y);

/* Phi_T(y_p) = exp(c sum_k y_k A_k) Phi_0 for every path (Sec. II.C, Eq.
 * trial_decomp; Sec. III.A, Eq. Metropolis_sampled_trial), or the multi-slice
 * product of a SLICES context (complex phiT).  y -> phiT. */
afqmc_status afqmc_trial_build(afqmc_ctx ctx, int32_t nw, const double* y, double* phiT);

/* l_p = sum_s log det(Phi_T(y_p)^T phi^s) with partial-pivoting LU (the
 * overlaps O_p of Eqs. ratio-update-phi and sign-path, kept as logarithms).
 * phi, phiT -> logov.  A zero pivot gives l_p = -inf + 0i. */
afqmc_status afqmc_overlap(afqmc_ctx ctx, int32_t nw, const void* phi, const double* phiT,
                           void* logov);

/* As afqmc_overlap, plus Theta^s = phi^s (Phi_T^T phi^s)^{-1}, so that the
 * one-body Green's function of path p is G^s = Theta^s Phi_T^T (Sec. III.A,
 * Eq. local-obs needs it for every path).  Theta = 0 for a singular path. */
afqmc_status afqmc_green(afqmc_ctx ctx, int32_t nw, const void* phi, const double* phiT,
                         void* logov, void* theta);

/* Force bias (Eq. shift1 with Eq. local-obs over the P paths):
 *   vb_pg = sum_s tr(Phi_T^T L_g Theta^s),  S_p = exp(i Im l_p) (Eq. sign-path),
 *   xbar_g = -i sqrt(tau) sum_p S_p vb_pg / sum_p S_p.
 * phiT, theta, logov -> xbar [nw][n_chol] complex; vb_sample [nw][P][n_chol]
 * complex if non-NULL.  Singular paths (l = -inf) are left out of the sums. */
afqmc_status afqmc_force_bias(afqmc_ctx ctx, int32_t nw, const double* phiT, const void* theta,
                              const void* logov, void* xbar, void* vb_sample);

/* Local energy (Eq. local-obs of H, the mixed estimator's E_L of Eq.
 * mixed_estimator): per path, with f_g^s = Phi_T^T L_g Theta^s,
 *   E_p = sum_s tr(Phi_T^T h1' Theta^s) + 1/2 sum_g [(sum_s tr f_g^s)^2 - sum_s tr(f_g^s f_g^s)],
 *   E_L = sum_p S_p E_p / sum_p S_p.
 * phiT, theta, logov -> eloc [nw] complex; e_sample [nw][P] complex and xbar
 * [nw][n_chol] complex (the force bias of the same contraction) if non-NULL. */
afqmc_status afqmc_local_energy(afqmc_ctx ctx, int32_t nw, const double* phiT, const void* theta,
                                const void* logov, void* eloc, void* e_sample, void* xbar);

/* For callers that cannot allocate device memory -- code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc: the local
 * energy of afqmc_local_energy (same arguments, same kernels, same results),
 * with its per-path scratch -- vb [nw][P][n_chol] complex and, when e_sample
 * is NULL, E_p [nw][P] complex -- in a fixed device array of
 * AFQMC_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the workspace.  It needs no workspace,
 * allocates nothing and records no numerical-event flags (those live in the
 * workspace).  Returns AFQMC_E_SHAPE if its scratch, 16 nw P n_chol bytes plus
 * 16 nw P without e_sample (each rounded up to 256), exceeds that size.  Every
 * call on one GPU shares that GPU's array and leaves its contents behind (no
 * entry needs to start at zero: the call writes each one it reads), so calls
 * that overlap on one GPU -- two streams, two contexts, two threads -- race
 * and must be ordered by the caller. */
#define AFQMC_STATIC_SCRATCH_BYTES (64u << 20)
afqmc_status afqmc_local_energy_static(afqmc_ctx ctx, int32_t nw, const double* phiT,
                                       const void* theta, const void* logov, void* eloc,
                                       void* e_sample, void* xbar);

/* One walker move with the phaseless weight (Eqs. walker_prop,
 * importance_function, importance_function_CP; Eq. ratio-update-phi for the
 * overlap ratio; App. B step 1):
 *   phi <- e^{-tau h1/2} T_n(V) e^{-tau h1/2} phi,  V = i sqrt(tau) sum_g (xi_g - xbar_g) L_g
 *   l'_p = l_p(phi') at the unchanged paths        -> logov_new [nw][P]
 *   num_r = sum_p exp(l'_p - Re l_p),  r = num_r / sum_p S_p
 *   hybrid: W <- W |exp(sum_g (xi_g xbar_g - xbar_g^2/2)) r| e^{tau e_shift} [max(0, cos arg r)]
 *   LOCAL:  W <- W exp(-tau (Re E_L - e_shift)) max(0, cos arg r)
 * xi [nw][n_chol] double, xbar [nw][n_chol] complex, logov = l at (phi, paths),
 * eloc [nw] complex (the pre-move E_L; needed by LOCAL, else may be NULL).
 * ref [nw] complex receives the hand-off phase reference: num_r, or sum_p S_p
 * in COMBINED mode.  W = 0 when every path is singular. */
afqmc_status afqmc_propagate(afqmc_ctx ctx, int32_t nw, void* phi, const double* xi,
                             const void* xbar, const double* phiT, const void* logov,
                             const void* eloc, double e_shift, double* w, void* ref,
                             void* logov_new);

/* Metropolis update of the paths at the moved walker, then the hand-off
 * projection (Sec. III.A leapfrog step 2, Eqs. PDF-Y, AFQMC_Metro_correction,
 * AFQMC_Metro_constraint_cos; App. B steps 2-3).  For each path and each of
 * n_sweep sweeps a proposal y' is drawn (stream PROPOSAL), Phi_T(y') and
 * l(y'; phi) are formed, and y' is accepted iff u < alpha (stream ACCEPT),
 * alpha = |O(y')|/|O(y)| for prior proposals, times N(y')/N(y) for the
 * random walk, times N(y')q(y|z',y')/(N(y)q(y'|z,y)) for the learned proposal
 * (z, z' the network features at y and y', see afqmc_mlp_init).  With the
 * learned proposal and rw_step > 0 each sweep is a random-walk move y~ = y +
 * rw_step eta (stream sweep index 2s) followed by a network move (2s + 1), a
 * cycle of two exact kernels; with training on, one Adam step on the mean
 * over all paths of -log q(y | z(y~)) (denoising score matching on the
 * random-walk pairs) precedes each random-walk accept test.  n_accept counts
 * both kinds of move.  Accepted paths update y, phiT and logov in place.
 * Then
 *   dtheta_T = arg sum_p S'_p - arg ref,  W <- W max(0, cos dtheta_T)
 * (HALFPLANE: W <- 0 if |dtheta_T| > pi/2).  n_accept [nw] int32 counts
 * accepted moves per walker (may be NULL).  With w = NULL the paths move and
 * no hand-off is applied (ref may then be NULL too): the form the
 * initialisation and the measurement chains use. */
afqmc_status afqmc_metropolis_x(afqmc_ctx ctx, int32_t nw, const void* phi, double* y,
                                double* phiT, void* logov, const void* ref, double* w,
                                uint64_t seed, uint64_t step, int32_t n_sweep, int32_t* n_accept);

/* Re-orthonormalise every walker determinant: phi^s = Q R with real positive
 * diag(R), phi^s <- Q; logov (may be NULL) shifts by -sum_s sum_i log R_ii so
 * that it stays the log-overlap of the new phi.  Overlap ratios, the force
 * bias and E_L are unchanged (Eq. WF-imp is invariant under phi -> phi R). */
afqmc_status afqmc_reorthogonalize(afqmc_ctx ctx, int32_t nw, void* phi, void* logov);

/* Comb population control (branching of the random walk; Sec. II.B speaks of
 * a branching random walk without fixing the scheme).  With w_cap > 0 each
 * weight is first clipped to w_cap times the mean weight.  With C_k the
 * inclusive prefix sums of W and u the uniform of stream (seed, walker 0,
 * step, tag COMB), new walker j is a copy of old walker
 *   parent[j] = min{k : C_k > (j + u) sum(W) / nw}
 * (phi, y, phiT and logov are gathered in place) and every weight becomes
 * sum(W) / nw, or 1 with normalize = 1 (a common factor of all weights, which
 * cancels in Eq. mixed_estimator and keeps long runs inside the FP64 range).
 * parent [nw] int32 receives the parents if non-NULL.  A population whose
 * weights sum to zero is left unchanged. */
afqmc_status afqmc_population_control(afqmc_ctx ctx, int32_t nw, void* phi, double* w, double* y,
                                      double* phiT, void* logov, uint64_t seed, uint64_t step,
                                      double w_cap, int32_t normalize, int32_t* parent);

/* Mixed-estimator sums (Eq. mixed_estimator): out[0] = sum_k W_k Re E_L,k,
 * out[1] = sum_k W_k, compensated FP64 summation; out is a DEVICE double[2].
 * A walker whose Re E_L is not finite (numerically singular overlaps) is left
 * out of both sums; afqmc_propagate sets a non-finite new weight to 0. */
afqmc_status afqmc_estimator(afqmc_ctx ctx, int32_t nw, const double* w, const void* eloc,
                             double* out);

/* ---- Back-propagated measurement (App. B, Measurement; Eqs.
 * AFQMC_Metropolis_measure and AFQMC_Metropolis_measure2) ------------------
 *
 * The operator is inserted h steps back along each walker's path: between the
 * walker phi_mid saved h steps before the measurement and the measurement
 * step's sampled trial propagated back through the h restored projectors
 * B_i = e^{-tau h1/2} T_n(V_i) e^{-tau h1/2}, V_i = i sqrt(tau) sum_g
 * (xi_g - xbar_g) L_g with the fields the walker's line of descent drew.  The
 * caller keeps the field history [nw][h][G] (afqmc_bp_record after each
 * afqmc_propagate) and phi_mid, and moves both with the walkers at every comb
 * (afqmc_gather_rows with the comb's parent array). */

/* hist_xi[w][slot][.] = xi[w][.] (double), hist_xbar[w][slot][.] = xbar[w][.]
 * (complex); 0 <= slot < h. */
afqmc_status afqmc_bp_record(afqmc_ctx ctx, int32_t nw, int32_t h, int32_t slot, const double* xi,
                             const void* xbar, double* hist_xi, void* hist_xbar);

/* One-body density matrix with the last h projectors restored: per walker k
 * and path p (phiT, logov at the measurement step, complex or real trial),
 *   Phi~_p = B_1 ... B_h Phi_T(Y_p)          (slot h-1 applied first)
 *   R_p = sum_s phi_mid^s (Phi~_p^T phi_mid^s)^{-1} Phi~_p^T,
 *         R_p[i][j] = <Phi~_p| c+_j c_i |phi_mid> / <Phi~_p|phi_mid>
 *   a_p = <Phi~_p|phi_mid> / |O_p(phi_end)|  (the sampled trial's path weights)
 *   R_k = sum_p a_p R_p / sum_p a_p          -> rho [nw][M][M] complex
 *   out[i M + j] = sum_k W_k Re R_k[i][j],  out[M M] = sum_k W_k
 * over walkers with a live path and finite R_k (compensated FP64 sums).
 * Scratch owned by the caller: phit_bp [nw][P][M][N] complex, theta_bp
 * [nw][P][2][M][N] complex, logov_bp [nw][P] complex.  h = 0 gives the
 * path-weighted mixed estimate.  Uses the workspace; out is DEVICE double[M M + 1]. */
afqmc_status afqmc_bp_density(afqmc_ctx ctx, int32_t nw, int32_t h, const void* phi_mid,
                              const double* hist_xi, const void* hist_xbar, const double* phiT,
                              const void* logov, const double* w, void* phit_bp, void* theta_bp,
                              void* logov_bp, void* rho, double* out);

/* Device copy of n doubles, and dst[j] = src[parent[j]] for nw rows of `row`
 * doubles (rows whose parent is outside [0, nw) are left as they are): the
 * data movement that keeps per-walker buffers in step with the walkers. */
afqmc_status afqmc_copy(afqmc_ctx ctx, int64_t n, const void* src, void* dst);
afqmc_status afqmc_gather_rows(afqmc_ctx ctx, int32_t nw, const int32_t* parent, int64_t row,
                               const void* src, void* dst);

/* ---- Initialisation from the trial and measurement with extra paths ------- */

/* Step indices of the Metropolis streams reserved for these chains: the
 * initialisation uses AFQMC_INIT_STEP + j; measurement chains are meant to use
 * AFQMC_MEASURE_STEP + (step index), apart from the propagation's steps. */
#define AFQMC_INIT_STEP 0x8000000000000000ull
#define AFQMC_MEASURE_STEP 0x4000000000000000ull

/* Walkers sampled from the trial (App. B, Initialization; Eq. Metropolis and
 * Eq. Metropolis_chain): pairs (Y_k, Y') from
 *   pi(Y, Y') ~ p_T(Y) p_T(Y') |<phi_T|B_T(Y') B_T(Y)|phi_T>|
 * by n_pair rounds of the two conditional Metropolis updates (each is the
 * path density of Eq. PDF-Y with the other member's determinant as walker):
 * the partner Y' at step AFQMC_INIT_STEP + 2j, then Y_k at + 2j + 1, both
 * with the context's proposal (a learned proposal is replaced by the random
 * walk of step rw_step, 0.5 if rw_step is 0).  Y_k and Y' start from the
 * prior (stream INIT, sweeps 1 and 2).  Outputs:
 *   yw   [nw][K]          the walker fields Y_k
 *   phi  [nw][2][M][N]    phi^0_k = B_T(Y_k) phi_T = Phi_T(Y_k) for both spins
 *   y, phiT, logov        P paths per walker, each a copy of the partner Y'
 *                         moved n_burn sweeps at phi^0_k (step
 *                         AFQMC_INIT_STEP + 2 n_pair); every walker-path pair
 *                         then has the law pi
 *   w    [nw]             W^0_k = Re sum_p S_p (the pair phases summed over
 *                         the paths; = P for this trial family, whose overlaps
 *                         are squares of real determinants)
 * The mixed estimator of this population is the Metropolis estimate of the
 * trial's variational energy (App. B, Eq. AFQMC_Metropolis_initial).  Uses the
 * workspace (for nw walkers); all buffers are device memory owned by the
 * caller and must not overlap. */
afqmc_status afqmc_init_metropolis(afqmc_ctx ctx, int32_t nw, uint64_t seed, int32_t n_pair,
                                   int32_t n_burn, double* yw, void* phi, double* y, double* phiT,
                                   void* logov, double* w);

/* Paths of a measurement trial (Sec. III.A, end of the composite-walker part;
 * App. B, Measurement): the context's P paths of each walker start from the
 * walker's p_src current ones, path q copying path q mod p_src:
 *   y_src [nw][p_src][K], phiT_src [nw][p_src][M][N], logov_src [nw][p_src]
 *   -> y [nw][P][K], phiT [nw][P][M][N], logov [nw][P] (complex).
 * Source and destination must not overlap.  Moving them afterwards with
 * afqmc_metropolis_x (w = NULL) gives the new paths Y'. */
afqmc_status afqmc_extend_paths(afqmc_ctx ctx, int32_t nw, int32_t p_src, const double* y_src,
                                const double* phiT_src, const void* logov_src, double* y,
                                double* phiT, void* logov);

/* Mixed estimator with the measurement trial's correction factor (Sec. III.A,
 * end of the composite-walker part; App. B, Measurement):
 *   R_k = sum_q S'_q / sum_p S_p   (new paths: logov [nw][P] of this context;
 *                                   current: logov_ref [nw][p_ref])
 *   out[0] = sum_k W_k Re(R_k E'_L,k),  out[1] = sum_k W_k Re R_k
 * with E'_L (eloc [nw] complex) from the new paths; R_k = 0 when the current
 * sign sum is 0.  Compensated FP64 sums; out is a DEVICE double[2]; R [nw]
 * complex receives R_k (may be NULL). */
afqmc_status afqmc_estimator_corrected(afqmc_ctx ctx, int32_t nw, const double* w,
                                       const void* eloc, const void* logov, int32_t p_ref,
                                       const void* logov_ref, double* out, void* R);

/* Counter-based normals: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 * counter (i / 4, walker, step, tag << 48 | sweep << 24 | path).  Fills
 * out [nw][n] with normal i of walker k's stream (tag, sweep 0, path 0), from
 * Box-Muller pairs of the uniforms (word >> 11) * 2^-53 of words (2j, 2j+1).
 * tag 1 (FIELD) gives the auxiliary fields xi of step `step`. */
afqmc_status afqmc_philox_normal(afqmc_ctx ctx, uint64_t seed, uint64_t step, uint32_t tag,
                                 int32_t nw, int32_t n, double* out);

/* ---- Learned Metropolis proposal (an extension; the paper leaves the proposal
 * of Sec. III.A leapfrog step 2 open and draws from the prior in App. B) -----
 *
 * A perceptron with two hidden layers of AFQMC_MLP_HIDDEN units proposes all K
 * Gaussian hidden variables of a path at once from the features
 *   z = [Re diag(G_up + G_dn) (M values), y (K values)]   (D = M + K inputs),
 *   h1 = tanh(z W1 + b1), h2 = tanh(h1 W2 + b2), o = h2 W3 + b3,
 *   mu = y + o[0:K], lv = 4 tanh(o[K:2K] / 4),  y' = mu + sqrt(2 exp(lv)) eta,
 * eta from stream PROPOSAL; a zero output layer (W3 = b3 = 0) is the random
 * walk of step sqrt(2).  The acceptance uses the exact Metropolis-Hastings ratio with
 * the reverse density at the proposal's own features, so the paths keep
 * sampling P(y; phi) of Eq. PDF-Y whatever the weights are.  Training (Adam)
 * makes mu(y~) the denoiser E[y | y~] and exp(lv) the variance Var[y | y~]
 * of the chains' random-walk moves y~ = y + s eta (see afqmc_metropolis_x):
 * mu - y is then the drift s^2 grad log p of a Langevin step whose noise
 * variance is 2 s^2, the proposal above.
 * Parameters are one flat array in the order W1 [D][H], b1 [H], W2 [H][H],
 * b2 [H], W3 [H][2K], b3 [2K] (row-major, H = AFQMC_MLP_HIDDEN).  The context
 * keeps FP32 master weights and Adam moments; the products run on the matrix
 * cores in FP32 (AFQMC_PREC_FP32) or BF16 (AFQMC_PREC_BF16, weights and
 * activations rounded to bfloat16) with FP32 accumulation.  The afqmc_mlp_*
 * calls need a context created with proposal = AFQMC_PROPOSAL_LEARNED. */
#define AFQMC_MLP_HIDDEN 256

/* Number of network parameters, D*H + H + H*H + H + 2K*H + 2K (0 on error). */
int64_t afqmc_mlp_num_params(afqmc_ctx ctx);

/* Loads the parameters (HOST double [n_params], rounded to FP32), resets Adam
 * (moments 0, step 0) and sets the matrix-core precision and the Adam
 * hyper-parameters (lr > 0, 0 <= beta1, beta2 < 1, eps > 0).  Training starts
 * off.  Allocates the network's device state on the first call; synchronises
 * the stream. */
afqmc_status afqmc_mlp_init(afqmc_ctx ctx, int32_t precision, const double* params, double lr,
                            double beta1, double beta2, double eps);

/* Copies the FP32 master parameters to HOST double [n_params]; synchronises. */
afqmc_status afqmc_mlp_get_params(afqmc_ctx ctx, double* params);

/* Whether afqmc_metropolis_x trains the network in each sweep (0 / 1);
 * training needs rw_step > 0 (AFQMC_E_INVALID otherwise). */
afqmc_status afqmc_mlp_set_training(afqmc_ctx ctx, int32_t enabled);

/* Network outputs for n feature rows given as gdiag [n][M] and y [n][K]
 * (DEVICE double): mu [n][K] (= y + o) and lv [n][K] (DEVICE double).  Needs
 * the workspace of ceil(n / P) walkers. */
afqmc_status afqmc_mlp_forward(afqmc_ctx ctx, int32_t n, const double* gdiag, const double* y,
                               double* mu, double* lv);

/* One training step on n rows: loss = mean over rows with mask[i] != 0 of
 * -log q(ytarget_i | z_i), z_i = [gdiag_i, y_i], its gradient, then one Adam
 * step (none if no row is masked in).  gdiag [n][M], y [n][K], ytarget [n][K]
 * DEVICE double; mask [n] DEVICE int32.  loss: DEVICE double[1] or NULL;
 * grad: DEVICE double [n_params] (the gradient before the step) or NULL.
 * Needs the workspace of ceil(n / P) walkers. */
afqmc_status afqmc_mlp_train_step(afqmc_ctx ctx, int32_t n, const double* gdiag, const double* y,
                                  const double* ytarget, const int32_t* mask, double* loss,
                                  double* grad);

/* The network's first input block for every path: as afqmc_overlap, plus
 * gdiag [nw][P][M] = Re diag(G_up + G_dn) with G^s = Theta^s Phi_T^T (the
 * diagonal of the one-body Green's function of Eq. local-obs); 0 for a
 * singular path. */
afqmc_status afqmc_green_diag(afqmc_ctx ctx, int32_t nw, const void* phi, const double* phiT,
                              void* logov, double* gdiag);

/* ---- Uneven batching (an extension: many independent systems per launch) --
 *
 * A batch advances n_systems independent systems (each an afqmc_system with
 * its own sizes, within afqmc_create's limits, prior or random-walk
 * proposals) together.  Each system's walkers start at phi = Phi_0, W = 1,
 * y ~ p_T (stream INIT, key seed + i), and every step is the App. B step of
 * the per-system calls: green -> local energy (with x-bar) -> estimator ->
 * fields (stream FIELD) -> propagate (E_T = 0) -> Metropolis -> QR every
 * n_qr steps -> comb every n_pc steps with weights reset to 1.  A cycle of
 * afqmc_batch_cycle() steps of all systems is captured once as one hipGraph
 * in which each system's kernels run on one of up to max_branches parallel
 * branches (systems assigned by longest processing time); each system's step
 * index lives in device memory, so replays advance the random streams.  With
 * autotune = 1 the batch times, per system, the kernel families that apply
 * (register-resident for M <= 64 and N <= 16, workgroup-per-path for any
 * size) and, for the whole cycle, 1, 2 and 4 branches, and keeps the fastest;
 * those timing steps advance the systems (they are part of the warm-up).
 * The batch owns all state (one device arena) and its workspaces. */
typedef struct afqmc_batch_s* afqmc_batch;

typedef struct {
  uint64_t seed;         /* Philox key of system i: seed + i                         */
  int32_t n_sweep;       /* Metropolis sweeps per step                               */
  int32_t n_qr;          /* re-orthonormalise every n_qr steps (0: never)            */
  int32_t n_pc;          /* comb every n_pc >= 1 steps                                */
  double w_cap;          /* comb weight cap relative to the mean (0: none)            */
  int32_t max_branches;  /* 1..4 parallel branches in the step graph                  */
  int32_t autotune;      /* 0 / 1                                                     */
  int32_t history;       /* estimator sums kept per system: a ring of `history` steps */
} afqmc_batch_options;

/* systems, walkers: HOST arrays [n_systems].  Creates contexts, state and the
 * step graph on `device`; orders itself after `stream` and synchronises it.
 * Errors: AFQMC_E_INVALID (bad options), the afqmc_create codes of a system. */
afqmc_status afqmc_batch_create(const afqmc_system* systems, const int32_t* walkers,
                                int32_t n_systems, const afqmc_batch_options* opt, int device,
                                void* stream, afqmc_batch* out);
/* Steps per replay of the step graph (a multiple of n_qr and n_pc, even). */
int32_t afqmc_batch_cycle(afqmc_batch b);
/* Launches the step graph n_cycles times after the work already on the
 * creation stream; that stream waits for the cycles.  Asynchronous. */
afqmc_status afqmc_batch_run(afqmc_batch b, int32_t n_cycles);
/* Synchronises and copies, for every system i, the estimator sums of
 * Eq. mixed_estimator (sum W Re E_L, sum W) of step t to
 * out[(i * history + t % history) * 2 + {0, 1}] (HOST double), and the steps
 * done to steps[i] (HOST uint64). */
afqmc_status afqmc_batch_estimates(afqmc_batch b, double* out, uint64_t* steps);
/* The tuner's choices (HOST arrays [n_systems], each may be NULL): kernel
 * family (0 register-resident, 1 workgroup-per-path, 2 workgroup-per-path
 * with the FP64 contraction's operands streamed, afqmc_set_contraction_variant),
 * branch, the measured time of one step of the system alone (ms), and the
 * number of branches. */
afqmc_status afqmc_batch_plan(afqmc_batch b, int32_t* family, int32_t* branch, double* step_ms,
                              int32_t* n_branches);
const char* afqmc_batch_last_error(afqmc_batch b);
afqmc_status afqmc_batch_destroy(afqmc_batch b);

/* Counter tags of the streams above. */
enum { AFQMC_TAG_FIELD = 1, AFQMC_TAG_PROPOSAL = 2, AFQMC_TAG_ACCEPT = 3, AFQMC_TAG_COMB = 4,
       AFQMC_TAG_INIT = 5 };

#ifdef __cplusplus
}
#endif
#endif /* AFQMC_H */
