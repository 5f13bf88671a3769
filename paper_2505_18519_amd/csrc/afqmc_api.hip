// C ABI entry points of libafqmc: argument checks, context set-up and the
// kernel sequences of each call.  Every numerical step runs in the gfx950
// kernels of the k_*.hip files; the host only validates, lays out and launches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "afqmc_internal.h"

// Fixed per-GPU scratch of the entry point that allocates nothing
// (afqmc_local_energy_static).  In host code this name is only a stand-in for
// the symbol: every host use goes through the device address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) unsigned char scratch[AFQMC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The address of `device`'s scratch array, looked up once per device with that
// device current (afqmc_create calls this after hipSetDevice(device)).
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

afqmc_status fail(afqmc_ctx_s* c, afqmc_status st, const std::string& msg) {
  if (c != nullptr) c->err = msg;
  return st;
}

afqmc_status hip_fail(afqmc_ctx_s* c, hipError_t e, const char* where) {
  return fail(c, AFQMC_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <class T>
hipError_t dev_copy(T** dst, const T* src, size_t n) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

void free_ctx(afqmc_ctx_s* c) {
  auto& m = c->mlp;
  void* ptrs[] = {c->d_h1,  c->d_Lraw, c->d_Lpad,  c->d_Eh,   c->d_phi0, c->d_A,   c->d_Lpad32,
                  c->d_Lbf, c->d_Lbf_lo, c->d_F,    c->d_phi0c, m.master,  m.mom1,   m.mom2,
                  m.w1t,    m.w2t,     m.w3t,       m.w2c,      m.w3c,     m.tstep,  m.scal,
                  c->d_Adiag, c->d_LTx, c->d_ATx};
  for (void* p : ptrs)
    if (p != nullptr) (void)hipFree(p);
}

int round16(int x) { return (x + 15) & ~15; }

#define CHECK_CTX(c)                                        \
  do {                                                      \
    if ((c) == nullptr) return AFQMC_E_INVALID;             \
    hipError_t se_ = hipSetDevice((c)->device);             \
    if (se_ != hipSuccess) return hip_fail((c), se_, "hipSetDevice"); \
  } while (0)

#define CHECK_NW(c, nw)                                                      \
  do {                                                                       \
    if ((nw) < 0) return fail((c), AFQMC_E_INVALID, "nw must be >= 0");      \
  } while (0)

#define REQUIRE(c, p, name)                                                  \
  do {                                                                       \
    if ((p) == nullptr) return fail((c), AFQMC_E_INVALID, name " is NULL");  \
  } while (0)

#define HIPCALL(c, expr, where)                                              \
  do {                                                                       \
    hipError_t he_ = (expr);                                                 \
    if (he_ != hipSuccess) return hip_fail((c), he_, where);                 \
  } while (0)

afqmc_status need_ws(afqmc_ctx_s* c, int nw, ws_layout* L) {
  *L = afqmc_ws_layout(c, nw);
  if (c->ws == nullptr) return fail(c, AFQMC_E_WORKSPACE, "no workspace set (afqmc_set_workspace)");
  if (c->ws_bytes < L->total)
    return fail(c, AFQMC_E_WORKSPACE,
                "workspace too small: " + std::to_string(c->ws_bytes) + " < " +
                    std::to_string(L->total) + " bytes for nw=" + std::to_string(nw));
  return AFQMC_OK;
}

template <class T>
T* ws_ptr(afqmc_ctx_s* c, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(c->ws) + off);
}

// Walkers of a complex64 context: their FP64 copy in the workspace (widened
// exactly), on which every kernel runs; after a move or re-orthonormalisation
// the copy is rounded back into the caller's complex64 array.  complex128
// contexts use the caller's array directly.
afqmc_status phi_in(afqmc_ctx_s* c, int nw, const void* phi, double** out) {
  if (!c->c64) {
    *out = const_cast<double*>(static_cast<const double*>(phi));
    return AFQMC_OK;
  }
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  double* d = ws_ptr<double>(c, L.phi128);
  HIPCALL(c, launch_phi_widen(c, (size_t)nw * 2 * c->M * c->N, static_cast<const float*>(phi), d),
          "widen walkers");
  *out = d;
  return AFQMC_OK;
}

afqmc_status phi_out(afqmc_ctx_s* c, int nw, const double* w128, void* phi) {
  if (!c->c64) return AFQMC_OK;
  HIPCALL(c, launch_phi_narrow(c, (size_t)nw * 2 * c->M * c->N, w128, static_cast<float*>(phi)),
          "round walkers");
  return AFQMC_OK;
}

#define PHI_IN(c, nw, phi, out)                     \
  do {                                              \
    afqmc_status pst_ = phi_in((c), (nw), (phi), (out)); \
    if (pst_ != AFQMC_OK) return pst_;              \
  } while (0)

// The numerical-event flag words of walkers [0, nw) (the workspace's first
// 4 nw bytes), null if no workspace that large is set.  Words not yet known
// to be clear are cleared first, on the stream, by a fill kernel; with the
// numeric check on, all nw are cleared so that the call reports only its own.
int* flag_words(afqmc_ctx_s* c, int nw, hipError_t* e) {
  *e = hipSuccess;
  if (c->ws == nullptr || c->ws_bytes < align256((size_t)nw * 4)) return nullptr;
  int* f = static_cast<int*>(c->ws);
  const int from = c->numeric_check ? 0 : c->flags_clear;
  if (nw > from) {
    *e = launch_zero_int(c, nw - from, f + from);
    if (*e != hipSuccess) return nullptr;
  }
  c->flags_clear = std::max(c->flags_clear, nw);
  return f;
}

// Copies the flag words of walkers [0, nw) to host (synchronising the
// stream) and counts the flagged ones.
hipError_t read_flags(afqmc_ctx_s* c, int nw, std::vector<int32_t>* out, int* n_bad, int* first) {
  out->assign((size_t)nw, 0);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && nw > 0)
    e = hipMemcpy(out->data(), c->ws, (size_t)nw * 4, hipMemcpyDeviceToHost);
  *n_bad = 0;
  *first = -1;
  for (int k = 0; k < nw && e == hipSuccess; ++k)
    if ((*out)[k] != 0) {
      if (*first < 0) *first = k;
      ++*n_bad;
    }
  return e;
}

afqmc_status numeric_report(afqmc_ctx_s* c, int n_bad, int first, int bits) {
  return fail(c, AFQMC_E_NUMERIC,
              std::to_string(n_bad) + " walker(s) with a non-finite result; first: walker " +
                  std::to_string(first) + ", flag bits " + std::to_string(bits));
}

// With the numeric check on, the end of a per-step call: synchronise and
// report the walkers this call flagged.
afqmc_status numeric_check_end(afqmc_ctx_s* c, int nw, const int* f) {
  if (!c->numeric_check || f == nullptr) return AFQMC_OK;
  std::vector<int32_t> h;
  int n_bad = 0, first = -1;
  hipError_t e = read_flags(c, nw, &h, &n_bad, &first);
  if (e != hipSuccess) return hip_fail(c, e, "numeric check");
  return n_bad ? numeric_report(c, n_bad, first, h[first]) : AFQMC_OK;
}

// ub: the workspace's U buffer; the V buffer (idle outside the move) is the U
// build's scratch
hipError_t do_trial_build(afqmc_ctx_s* c, const ws_layout& L, const afqmc_ctx_s* cb, int n,
                          const double* y, double* phiT) {
  double* ub = ws_ptr<double>(c, L.ubuf);
  return cb->small ? launch_trial_build(cb, n, y, phiT, ub)
                   : launch_trial_build_g(cb, n, y, phiT, ub, ws_ptr<void>(c, L.vmat),
                                          L.ubuf - L.vmat);
}
hipError_t do_overlap(const afqmc_ctx_s* c, int nw, const double* phi, const double* phiT,
                      double* logov, double* theta, double* gdiag = nullptr) {
  return c->small ? launch_overlap(c, nw, phi, phiT, logov, theta, gdiag)
                  : launch_overlap_g(c, nw, phi, phiT, logov, theta, gdiag);
}

// backward pass, weight gradients, loss reduction and Adam step on the rows
// whose mask is set; out holds the forward outputs, zT/h1T/h2T its activations
afqmc_status mlp_train(afqmc_ctx_s* c, const ws_layout& L, int n, const float* out,
                       const double* yin, const double* ytgt, const int* mask, const void* zT,
                       double* loss, double* grad);

}  // namespace

ws_layout afqmc_ws_layout(const afqmc_ctx_s* c, int nw) {
  ws_layout L;
  const size_t S = (size_t)nw * c->P;
  size_t off = 0;
  L.flags = off;
  off += align256((size_t)nw * 4);
  L.vb = off;
  off += align256(S * c->G * 16);
  L.ep = off;
  off += align256(S * 16);
  L.vmat = off;
  off += align256((size_t)nw * c->M * c->M * 16);
  L.ubuf = off;  // trial generator sums U (real) or slice matrices V (complex)
  off += align256(S * c->M * c->M * (c->ctrial ? 16 : 8));
  L.qrshift = off;
  off += align256((size_t)nw * 2 * 8);
  L.ytry = off;
  off += align256(S * c->K * 8);
  L.phiTtry = off;
  off += align256(S * c->tsz * 8);
  L.ltry = off;
  off += align256(S * 16);
  L.acc = off;
  off += align256((size_t)nw * 4);
  L.pc_C = off;
  off += align256((size_t)nw * 8);
  L.pc_tot = off;
  off += 256;
  L.pc_parent = off;
  off += align256((size_t)nw * 4);
  L.pc_phi = off;
  off += align256((size_t)nw * 2 * c->M * c->N * 16);
  L.pc_y = off;
  off += align256(S * c->K * 8);
  L.pc_phiT = off;
  off += align256(S * c->tsz * 8);
  L.pc_logov = off;
  off += align256(S * 16);
  // learned proposal: sizes for 4-byte product elements (BF16 uses half)
  const bool ml = c->proposal == AFQMC_PROPOSAL_LEARNED;
  const size_t Sp = ml ? (size_t)round16((int)S) : 0;
  const size_t D = (size_t)c->M + c->K, Op = (size_t)round16(2 * c->K), H = AFQMC_MLP_HIDDEN;
  const size_t np = D * H + H + H * H + H + H * 2 * c->K + 2 * c->K;
  const size_t nsplit = (Sp + MLP_CHUNK - 1) / MLP_CHUNK;
  const size_t sizes[] = {ml ? S * c->M * 8 : 0, ml ? S * c->M * 8 : 0, Sp * Op * 4, Sp * Op * 4,
                          ml ? S * 8 : 0,       ml ? S * 8 : 0,       D * Sp * 4,  H * Sp * 4,
                          H * Sp * 4,           Op * Sp * 4,          H * Sp * 4,  H * Sp * 4,
                          Sp * 8,               nsplit * np * 4};
  size_t* dst[] = {&L.gd_cur, &L.gd_try, &L.mlF,  &L.mlR,  &L.lqf, &L.lqx, &L.zT,
                   &L.h1T,    &L.h2T,    &L.dOT,  &L.dh2T, &L.dh1T, &L.nlq, &L.part};
  for (int i = 0; i < 14; ++i) {
    *dst[i] = off;
    off += align256(sizes[i]);
  }
  const size_t MN = (size_t)c->M * c->N;
  const size_t isz[] = {(size_t)nw * c->K * 8, (size_t)nw * MN * 8, (size_t)nw * MN * 8,
                        (size_t)nw * 16, (size_t)nw * 16};
  size_t* idst[] = {&L.in_yb, &L.in_pa, &L.in_pb, &L.in_la, &L.in_lb};
  for (int i = 0; i < 5; ++i) {
    *idst[i] = off;
    off += align256(isz[i]);
  }
  L.phi128 = off;
  off += c->c64 ? align256((size_t)nw * 2 * MN * 16) : 0;
  L.total = off;
  return L;
}

namespace {

afqmc_status mlp_train(afqmc_ctx_s* c, const ws_layout& L, int n, const float* out,
                       const double* yin, const double* ytgt, const int* mask, const void* zT,
                       double* loss, double* grad) {
  const int Sp = round16(n);
  void* h1T = ws_ptr<void>(c, L.h1T);
  void* h2T = ws_ptr<void>(c, L.h2T);
  void* dOT = ws_ptr<void>(c, L.dOT);
  void* dh2T = ws_ptr<void>(c, L.dh2T);
  void* dh1T = ws_ptr<void>(c, L.dh1T);
  double* nlq = ws_ptr<double>(c, L.nlq);
  float* part = ws_ptr<float>(c, L.part);
  HIPCALL(c,
          launch_mlp_backward(c, n, Sp, out, yin, ytgt, mask, h1T, h2T, dOT, dh2T, dh1T, nlq),
          "mlp backward");
  HIPCALL(c, launch_mlp_wgrad(c, Sp, zT, h1T, h2T, dOT, dh2T, dh1T, part), "mlp weight gradients");
  HIPCALL(c, launch_mlp_reduce(c, n, mask, nlq, loss), "mlp loss");
  HIPCALL(c, launch_mlp_adam(c, Sp, part, grad), "mlp adam");
  return AFQMC_OK;
}

afqmc_status mlp_check(afqmc_ctx_s* c, int n, ws_layout* L) {
  if (c->proposal != AFQMC_PROPOSAL_LEARNED)
    return fail(c, AFQMC_E_INVALID, "network calls need proposal = AFQMC_PROPOSAL_LEARNED");
  if (!c->mlp.ready) return fail(c, AFQMC_E_INVALID, "network not initialised (afqmc_mlp_init)");
  return need_ws(c, (n + c->P - 1) / c->P, L);
}

}  // namespace

extern "C" {

afqmc_status afqmc_create(const afqmc_system* sys, int device, void* stream, afqmc_ctx* out) {
  if (sys == nullptr || out == nullptr) return AFQMC_E_INVALID;
  *out = nullptr;
  if (sys->h1 == nullptr || sys->L == nullptr || sys->phi0 == nullptr || sys->A == nullptr)
    return AFQMC_E_INVALID;
  const int M = sys->M, N = sys->N, G = sys->n_chol, K = sys->K, P = sys->P;
  if (M < 1 || N < 1 || N > M || M > 160 || N > 40 || G < 1 || K < 1 || P < 1 || P > 64)
    return AFQMC_E_SHAPE;
  // past M = 128 or N = 32 only the FP64 contraction and the non-learned
  // proposals are built
  const bool big = M > 128 || N > 32;
  if (big && (sys->precision != AFQMC_PREC_FP64 || sys->proposal == AFQMC_PROPOSAL_LEARNED))
    return AFQMC_E_UNSUPPORTED;
  if (sys->hidden_kind != AFQMC_HIDDEN_ISING && sys->hidden_kind != AFQMC_HIDDEN_GAUSS)
    return AFQMC_E_INVALID;
  if (sys->weight_mode < 0 || sys->weight_mode > 3) return AFQMC_E_INVALID;
  if (sys->proposal < 0 || sys->proposal > 2) return AFQMC_E_INVALID;
  if (sys->proposal == AFQMC_PROPOSAL_LEARNED &&
      (sys->hidden_kind != AFQMC_HIDDEN_GAUSS || K > 128))
    return AFQMC_E_UNSUPPORTED;
  if (sys->precision < AFQMC_PREC_FP64 || sys->precision > AFQMC_PREC_BF16X3)
    return AFQMC_E_INVALID;
  if (sys->n_taylor < 1 || !(sys->dtau > 0.0) || !isfinite(sys->coupling)) return AFQMC_E_INVALID;
  if (!(sys->xbar_cap >= 0.0)) return AFQMC_E_INVALID;
  if (sys->walker_c64 != 0 && sys->walker_c64 != 1) return AFQMC_E_INVALID;
  if (sys->walker_c64 == 1 &&
      (sys->precision == AFQMC_PREC_FP64 || sys->trial_kind != AFQMC_TRIAL_JASTROW))
    return AFQMC_E_UNSUPPORTED;
  const bool slices = sys->trial_kind == AFQMC_TRIAL_SLICES;
  if (sys->trial_kind != AFQMC_TRIAL_JASTROW && !slices) return AFQMC_E_INVALID;
  if (slices) {
    const int m = sys->n_slices;
    if (m < 1 || K % m != 0 || sys->slice_s == nullptr || sys->slice_F == nullptr ||
        sys->trial_taylor < 1 || sys->hidden_kind != AFQMC_HIDDEN_GAUSS)
      return AFQMC_E_INVALID;
    for (int l = 0; l < m; ++l)
      if (!(sys->slice_s[l] >= 0.0) || !isfinite(sys->slice_s[l])) return AFQMC_E_INVALID;
    if (sys->proposal == AFQMC_PROPOSAL_LEARNED) return AFQMC_E_UNSUPPORTED;
    // the BF16 contraction takes real trial determinants only
    if (sys->precision == AFQMC_PREC_BF16 || sys->precision == AFQMC_PREC_BF16X3)
      return AFQMC_E_UNSUPPORTED;
    // complex stage-1 operands of the contraction: (M/16) ceil(N/16) <= 8
    if (((M + 15) / 16) * ((N + 15) / 16) > 8) return AFQMC_E_UNSUPPORTED;
  }

  afqmc_ctx_s* c = new (std::nothrow) afqmc_ctx_s();
  if (c == nullptr) return AFQMC_E_NOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->M = M;
  c->N = N;
  c->G = G;
  c->K = K;
  c->P = P;
  c->MT = ((M + 15) / 16) * 16;
  c->small = (M <= 64 && N <= 16) && !slices;
  c->trial_kind = sys->trial_kind;
  c->ctrial = slices;
  c->tsz = M * N * (slices ? 2 : 1);
  if (slices) {
    c->n_slices = sys->n_slices;
    c->kgen = K / sys->n_slices;
    c->trial_taylor = sys->trial_taylor;
    c->slice_s.assign(sys->slice_s, sys->slice_s + sys->n_slices);
  }
  c->hidden_kind = sys->hidden_kind;
  c->coupling = sys->coupling;
  c->dtau = sys->dtau;
  c->rw_step = sys->rw_step;
  c->n_taylor = sys->n_taylor;
  c->weight_mode = sys->weight_mode;
  c->proposal = sys->proposal;
  c->precision = sys->precision;
  c->xbar_cap = sys->xbar_cap;
  c->c64 = sys->walker_c64 == 1;

  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = scratch_address(device, &c->d_scratch);
  if (e != hipSuccess) {
    delete c;
    return AFQMC_E_DEVICE;
  }
  // padded L slabs (slab G is filled with h1' on the device)
  const int MT = c->MT;
  std::vector<double> Lpad((size_t)(G + 1) * MT * MT, 0.0);
  for (int gm = 0; gm < G; ++gm)
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j)
        Lpad[((size_t)gm * MT + i) * MT + j] = sys->L[((size_t)gm * M + i) * M + j];
  if ((e = dev_copy(&c->d_h1, sys->h1, (size_t)M * M)) != hipSuccess ||
      (e = dev_copy(&c->d_Lraw, sys->L, (size_t)G * M * M)) != hipSuccess ||
      (e = dev_copy(&c->d_Lpad, Lpad.data(), Lpad.size())) != hipSuccess ||
      (e = dev_copy(&c->d_phi0, sys->phi0, (size_t)M * N)) != hipSuccess ||
      (e = dev_copy(&c->d_A, sys->A, (size_t)(slices ? c->kgen : K) * M * M)) != hipSuccess ||
      (e = hipMalloc(&c->d_Eh, (size_t)M * M * sizeof(double))) != hipSuccess) {
    free_ctx(c);
    delete c;
    return e == hipErrorOutOfMemory ? AFQMC_E_NOMEM : AFQMC_E_DEVICE;
  }
  if (slices) {  // one-body factors and Phi_0 as the complex input of the first slice
    std::vector<double> p0c((size_t)M * N * 2, 0.0);
    for (size_t q = 0; q < (size_t)M * N; ++q) p0c[2 * q] = sys->phi0[q];
    if ((e = dev_copy(&c->d_F, sys->slice_F, (size_t)(sys->n_slices + 1) * M * M)) != hipSuccess ||
        (e = dev_copy(&c->d_phi0c, p0c.data(), p0c.size())) != hipSuccess) {
      free_ctx(c);
      delete c;
      return e == hipErrorOutOfMemory ? AFQMC_E_NOMEM : AFQMC_E_DEVICE;
    }
  }
  if (!slices) {  // diagonal generators: keep only their diagonals for the row-scaling build
    bool diag = K > 0;
    for (int k = 0; k < K && diag; ++k)
      for (int i = 0; i < M && diag; ++i)
        for (int j = 0; j < M; ++j)
          if (i != j && sys->A[((size_t)k * M + i) * M + j] != 0.0) {
            diag = false;
            break;
          }
    if (diag) {
      std::vector<double> d((size_t)K * M);
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < M; ++i) d[(size_t)k * M + i] = sys->A[((size_t)k * M + i) * M + i];
      if ((e = dev_copy(&c->d_Adiag, d.data(), d.size())) != hipSuccess) {
        free_ctx(c);
        delete c;
        return e == hipErrorOutOfMemory ? AFQMC_E_NOMEM : AFQMC_E_DEVICE;
      }
    }
  }
  if ((e = launch_setup(c)) == hipSuccess && c->precision == AFQMC_PREC_FP32) {
    const size_t n = Lpad.size();
    if ((e = hipMalloc(&c->d_Lpad32, n * sizeof(float))) == hipSuccess &&
        (e = c->ctrial ? launch_to_float(c, n, c->d_Lpad, c->d_Lpad32)
                       : launch_to_f32_op(c, n, c->d_Lpad, c->d_Lpad32)) == hipSuccess)
      e = hipStreamSynchronize(c->stream);
  }
  if (e == hipSuccess &&
      (c->precision == AFQMC_PREC_BF16 || c->precision == AFQMC_PREC_BF16X3)) {
    // slabs of MT rows by the k extent padded to whole 32-wide blocks
    const size_t n = (size_t)(G + 1) * MT * ((MT + 31) / 32 * 32);
    const bool x3 = c->precision == AFQMC_PREC_BF16X3;
    if ((e = hipMalloc(&c->d_Lbf, n * sizeof(unsigned short))) == hipSuccess &&
        (!x3 || (e = hipMalloc(&c->d_Lbf_lo, n * sizeof(unsigned short))) == hipSuccess) &&
        (e = launch_to_bf16(c, n, c->d_Lpad, c->d_Lbf, c->d_Lbf_lo)) == hipSuccess &&
        (x3 || c->small || (e = launch_lt_split(c)) == hipSuccess))
      e = hipStreamSynchronize(c->stream);
  }
  if (e != hipSuccess) {
    free_ctx(c);
    delete c;
    return AFQMC_E_DEVICE;
  }
  *out = c;
  return AFQMC_OK;
}

afqmc_status afqmc_destroy(afqmc_ctx c) {
  if (c == nullptr) return AFQMC_E_INVALID;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  delete c;
  return AFQMC_OK;
}

const char* afqmc_last_error(afqmc_ctx c) {
  if (c == nullptr) return "null context";
  return c->err.c_str();
}

afqmc_status afqmc_set_stream(afqmc_ctx c, void* stream) {
  if (c == nullptr) return AFQMC_E_INVALID;
  c->stream = static_cast<hipStream_t>(stream);
  return AFQMC_OK;
}

afqmc_status afqmc_workspace_size(afqmc_ctx c, int32_t nw, size_t* bytes) {
  if (c == nullptr) return AFQMC_E_INVALID;
  REQUIRE(c, bytes, "bytes");
  CHECK_NW(c, nw);
  *bytes = afqmc_ws_layout(c, nw).total;
  return AFQMC_OK;
}

afqmc_status afqmc_set_workspace(afqmc_ctx c, void* dptr, size_t bytes) {
  if (c == nullptr) return AFQMC_E_INVALID;
  if (dptr != nullptr && (reinterpret_cast<uintptr_t>(dptr) & 255) != 0)
    return fail(c, AFQMC_E_INVALID, "workspace must be 256-byte aligned");
  c->ws = dptr;
  c->ws_bytes = dptr ? bytes : 0;
  c->flags_clear = 0;  // a new workspace's flag words are cleared at first use
  return AFQMC_OK;
}

afqmc_status afqmc_numeric_flags(afqmc_ctx c, int32_t nw, int32_t* flags, int32_t* n_flagged) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (n_flagged != nullptr) *n_flagged = 0;
  if (c->ws == nullptr || c->ws_bytes < align256((size_t)nw * 4))
    return fail(c, AFQMC_E_WORKSPACE, "no workspace for the flags of nw walkers");
  if (nw == 0) return AFQMC_OK;
  hipError_t e;
  if (nw > c->flags_clear) {  // words not written since the workspace was set
    HIPCALL(c, launch_zero_int(c, nw - c->flags_clear, static_cast<int*>(c->ws) + c->flags_clear),
            "numeric flags");
    c->flags_clear = nw;
  }
  std::vector<int32_t> h;
  int n_bad = 0, first = -1;
  e = read_flags(c, nw, &h, &n_bad, &first);
  if (e != hipSuccess) return hip_fail(c, e, "numeric flags");
  if (flags != nullptr) memcpy(flags, h.data(), (size_t)nw * 4);
  if (n_flagged != nullptr) *n_flagged = n_bad;
  if (n_bad == 0) return AFQMC_OK;
  HIPCALL(c, launch_zero_int(c, nw, static_cast<int*>(c->ws)), "numeric flags");
  HIPCALL(c, hipStreamSynchronize(c->stream), "numeric flags");
  return numeric_report(c, n_bad, first, h[first]);
}

afqmc_status afqmc_set_numeric_check(afqmc_ctx c, int32_t on) {
  if (c == nullptr) return AFQMC_E_INVALID;
  if (on != 0 && on != 1) return fail(c, AFQMC_E_INVALID, "on must be 0 or 1");
  c->numeric_check = on == 1;
  return AFQMC_OK;
}

afqmc_status afqmc_set_eloc_cap(afqmc_ctx c, double center, double half_width) {
  if (c == nullptr) return AFQMC_E_INVALID;
  if (!(half_width >= 0.0) || !__builtin_isfinite(half_width) || !__builtin_isfinite(center))
    return fail(c, AFQMC_E_INVALID, "the local-energy cap needs a finite centre and a finite width >= 0");
  c->ecap_center = center;
  c->ecap_half = half_width;
  return AFQMC_OK;
}

afqmc_status afqmc_set_contraction_variant(afqmc_ctx c, int32_t variant) {
  if (c == nullptr) return AFQMC_E_INVALID;
  if (variant != 0 && variant != 1) return fail(c, AFQMC_E_INVALID, "variant must be 0 or 1");
  c->contract_variant = variant;
  return AFQMC_OK;
}

afqmc_status afqmc_sample_prior(afqmc_ctx c, int32_t nw, uint64_t seed, double* y) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, y, "y");
  HIPCALL(c, launch_sample_prior(c, nw, seed, y), "sample_prior");
  return AFQMC_OK;
}

afqmc_status afqmc_trial_build(afqmc_ctx c, int32_t nw, const double* y, double* phiT) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, y, "y");
  REQUIRE(c, phiT, "phiT");
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  HIPCALL(c, do_trial_build(c, L, c, nw * c->P, y, phiT), "trial_build");
  return AFQMC_OK;
}

afqmc_status afqmc_overlap(afqmc_ctx c, int32_t nw, const void* phi, const double* phiT,
                           void* logov) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  double* ph;
  PHI_IN(c, nw, phi, &ph);
  HIPCALL(c, do_overlap(c, nw, ph, phiT, static_cast<double*>(logov), nullptr), "overlap");
  return AFQMC_OK;
}

afqmc_status afqmc_green(afqmc_ctx c, int32_t nw, const void* phi, const double* phiT, void* logov,
                         void* theta) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, theta, "theta");
  double* ph;
  PHI_IN(c, nw, phi, &ph);
  HIPCALL(c,
          do_overlap(c, nw, ph, phiT, static_cast<double*>(logov), static_cast<double*>(theta)),
          "green");
  return AFQMC_OK;
}

// The contraction kernel of the context's family and precision into per-path
// vb and ep, then the walker-level combination.
static hipError_t contraction_kernels(afqmc_ctx c, int32_t nw, const double* phiT,
                                      const void* theta, const void* logov, void* xbar, double* vb,
                                      void* eloc, double* ep, int* flags) {
  const double* th = static_cast<const double*>(theta);
  const double* lo = static_cast<const double*>(logov);
  hipError_t e;
  if (c->small && c->precision == AFQMC_PREC_FP64)
    e = launch_contract(c, nw, phiT, th, lo, vb, ep);
  else if (c->precision != AFQMC_PREC_FP64 && !c->ctrial)
    e = launch_contract_sh(c, nw, phiT, th, lo, vb, ep);
  else
    e = launch_contract_g(c, nw, phiT, th, lo, vb, ep);
  if (e != hipSuccess) return e;
  return launch_combine(c, nw, vb, ep, lo, static_cast<double*>(xbar),
                        static_cast<double*>(eloc), flags);
}

static afqmc_status contraction(afqmc_ctx c, int32_t nw, const double* phiT, const void* theta,
                                const void* logov, void* xbar, void* vb_sample, void* eloc,
                                void* e_sample) {
  ws_layout L;
  const bool need = (vb_sample == nullptr) || (e_sample == nullptr);
  if (need) {
    afqmc_status st = need_ws(c, nw, &L);
    if (st != AFQMC_OK) return st;
  }
  double* vb = vb_sample ? static_cast<double*>(vb_sample) : ws_ptr<double>(c, L.vb);
  double* ep = e_sample ? static_cast<double*>(e_sample) : ws_ptr<double>(c, L.ep);
  hipError_t fe;
  int* flags = flag_words(c, nw, &fe);
  HIPCALL(c, fe, "flags");
  HIPCALL(c, contraction_kernels(c, nw, phiT, theta, logov, xbar, vb, eloc, ep, flags),
          "contraction");
  return numeric_check_end(c, nw, flags);
}

afqmc_status afqmc_force_bias(afqmc_ctx c, int32_t nw, const double* phiT, const void* theta,
                              const void* logov, void* xbar, void* vb_sample) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, theta, "theta");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, xbar, "xbar");
  return contraction(c, nw, phiT, theta, logov, xbar, vb_sample, nullptr, nullptr);
}

afqmc_status afqmc_local_energy(afqmc_ctx c, int32_t nw, const double* phiT, const void* theta,
                                const void* logov, void* eloc, void* e_sample, void* xbar) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, theta, "theta");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, eloc, "eloc");
  return contraction(c, nw, phiT, theta, logov, xbar, nullptr, eloc, e_sample);
}

afqmc_status afqmc_local_energy_static(afqmc_ctx c, int32_t nw, const double* phiT,
                                       const void* theta, const void* logov, void* eloc,
                                       void* e_sample, void* xbar) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, theta, "theta");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, eloc, "eloc");
  if (c->d_scratch == nullptr) return fail(c, AFQMC_E_DEVICE, "no scratch address for this device");
  // vb [nw][P][G] complex, then (unless the caller takes E_p) ep [nw][P] complex
  const size_t S = (size_t)nw * c->P;
  const size_t vb_bytes = align256(S * c->G * 16);
  const size_t need = vb_bytes + (e_sample ? 0 : align256(S * 16));
  if (need > (size_t)AFQMC_STATIC_SCRATCH_BYTES)
    return fail(c, AFQMC_E_SHAPE,
                "afqmc_local_energy_static needs " + std::to_string(need) +
                    " bytes of scratch for nw=" + std::to_string(nw) + ", more than the fixed " +
                    std::to_string((size_t)AFQMC_STATIC_SCRATCH_BYTES));
  unsigned char* base = static_cast<unsigned char*>(c->d_scratch);
  double* vb = reinterpret_cast<double*>(base);
  double* ep = e_sample ? static_cast<double*>(e_sample) : reinterpret_cast<double*>(base + vb_bytes);
  HIPCALL(c, contraction_kernels(c, nw, phiT, theta, logov, xbar, vb, eloc, ep, nullptr),
          "static contraction");
  return AFQMC_OK;
}

afqmc_status afqmc_propagate(afqmc_ctx c, int32_t nw, void* phi, const double* xi, const void* xbar,
                             const double* phiT, const void* logov, const void* eloc,
                             double e_shift, double* w, void* ref, void* logov_new) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  REQUIRE(c, xi, "xi");
  REQUIRE(c, xbar, "xbar");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, w, "w");
  REQUIRE(c, ref, "ref");
  REQUIRE(c, logov_new, "logov_new");
  if (!isfinite(e_shift)) return fail(c, AFQMC_E_INVALID, "e_shift must be finite");
  if (c->weight_mode == AFQMC_WEIGHT_LOCAL && eloc == nullptr)
    return fail(c, AFQMC_E_INVALID, "the local-energy formalism needs eloc");
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  double* vmat = ws_ptr<double>(c, L.vmat);
  double* ph;
  PHI_IN(c, nw, phi, &ph);
  // the trial build's U buffer is free during the move
  void* scr = ws_ptr<void>(c, L.ubuf);
  const size_t scr_bytes = L.qrshift - L.ubuf;
  if (vbuild_split_ok(c, nw, scr_bytes)) {  // V stored split (8 nw M MP <= 16 nw M^2 bytes)
    unsigned short* Vs = ws_ptr<unsigned short>(c, L.vmat);
    HIPCALL(c, launch_vbuild_split(c, nw, xi, static_cast<const double*>(xbar), Vs, scr), "vbuild");
    HIPCALL(c, launch_taylor_split(c, nw, Vs, ph), "taylor");
  } else {
    HIPCALL(c, launch_vbuild(c, nw, xi, static_cast<const double*>(xbar), vmat, scr, scr_bytes),
            "vbuild");
    HIPCALL(c, c->small ? launch_taylor(c, nw, vmat, ph) : launch_taylor_g(c, nw, vmat, ph),
            "taylor");
  }
  st = phi_out(c, nw, ph, phi);
  if (st != AFQMC_OK) return st;
  if (c->c64) PHI_IN(c, nw, phi, &ph);  // the ratio is that of the stored (rounded) walkers
  HIPCALL(c, do_overlap(c, nw, ph, phiT, static_cast<double*>(logov_new), nullptr), "ratio overlap");
  hipError_t fe;
  int* flags = flag_words(c, nw, &fe);
  HIPCALL(c, fe, "flags");
  HIPCALL(c,
          launch_weight(c, nw, xi, static_cast<const double*>(xbar),
                        static_cast<const double*>(logov), static_cast<double*>(logov_new),
                        static_cast<const double*>(eloc), e_shift, w, static_cast<double*>(ref),
                        flags),
          "weight");
  return numeric_check_end(c, nw, flags);
}

afqmc_status afqmc_metropolis_x(afqmc_ctx c, int32_t nw, const void* phi, double* y, double* phiT,
                                void* logov, const void* ref, double* w, uint64_t seed,
                                uint64_t step, int32_t n_sweep, int32_t* n_accept) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  REQUIRE(c, y, "y");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  if (w != nullptr) REQUIRE(c, ref, "ref");
  if (n_sweep < 0) return fail(c, AFQMC_E_INVALID, "n_sweep must be >= 0");
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  double* ytry = ws_ptr<double>(c, L.ytry);
  double* phiTtry = ws_ptr<double>(c, L.phiTtry);
  double* ltry = ws_ptr<double>(c, L.ltry);
  int* nacc = n_accept ? n_accept : ws_ptr<int>(c, L.acc);
  double* ph;
  PHI_IN(c, nw, phi, &ph);
  double* lo = static_cast<double*>(logov);
  HIPCALL(c, launch_zero_int(c, nw, nacc), "zero");
  if (c->proposal == AFQMC_PROPOSAL_LEARNED) {
    if (!c->mlp.ready) return fail(c, AFQMC_E_INVALID, "learned proposal needs afqmc_mlp_init");
    const int n = nw * c->P, Sp = round16(n);
    double* gdc = ws_ptr<double>(c, L.gd_cur);
    double* gdt = ws_ptr<double>(c, L.gd_try);
    float* mlF = ws_ptr<float>(c, L.mlF);
    float* mlR = ws_ptr<float>(c, L.mlR);
    double* lqf = ws_ptr<double>(c, L.lqf);
    double* lqx = ws_ptr<double>(c, L.lqx);
    const bool tr = c->mlp.training;
    void* zT = ws_ptr<void>(c, L.zT);
    void* h1T = ws_ptr<void>(c, L.h1T);
    void* h2T = ws_ptr<void>(c, L.h2T);
    const bool hybrid = c->rw_step > 0.0;
    if (n_sweep > 0)
      HIPCALL(c, do_overlap(c, nw, ph, phiT, ltry, nullptr, gdc), "green diagonal");
    for (int s = 0; s < n_sweep; ++s) {
      int sl = s;
      if (hybrid) {  // random-walk move first (stream sweep index 2s), diagonals kept current
        HIPCALL(c, launch_proposal(c, nw, y, ytry, seed, step, 2 * s, -1, AFQMC_PROPOSAL_RW),
                "rw proposal");
        HIPCALL(c, do_trial_build(c, L, c, n, ytry, phiTtry),
                "rw trial build");
        HIPCALL(c, do_overlap(c, nw, ph, phiTtry, ltry, nullptr, gdt), "rw overlap");
        if (tr) {  // denoising score matching: q(y | z(y~)) on this move's pairs
          HIPCALL(c, launch_mlp_forward(c, n, Sp, gdt, ytry, mlF, zT, h1T, h2T),
                  "mlp training forward");
          afqmc_status st2 = mlp_train(c, L, n, mlF, ytry, y, nullptr, zT, nullptr, nullptr);
          if (st2 != AFQMC_OK) return st2;
        }
        HIPCALL(c,
                launch_accept(c, nw, y, phiT, lo, ytry, phiTtry, ltry, nacc, seed, step, 2 * s, -1,
                              AFQMC_PROPOSAL_RW, nullptr, gdc, gdt, nullptr),
                "rw accept");
        sl = 2 * s + 1;
      }
      HIPCALL(c, launch_mlp_forward(c, n, Sp, gdc, y, mlF, nullptr, nullptr, nullptr),
              "mlp forward");
      HIPCALL(c, launch_mlp_propose(c, nw, mlF, y, seed, step, sl, ytry, lqf), "mlp propose");
      HIPCALL(c, do_trial_build(c, L, c, n, ytry, phiTtry),
              "proposal trial build");
      HIPCALL(c, do_overlap(c, nw, ph, phiTtry, ltry, nullptr, gdt), "proposal overlap");
      HIPCALL(c, launch_mlp_forward(c, n, Sp, gdt, ytry, mlR, nullptr, nullptr, nullptr),
              "mlp reverse forward");
      HIPCALL(c, launch_mlp_reverse(c, n, mlR, y, ytry, lqf, lqx), "mlp reverse");
      HIPCALL(c,
              launch_accept(c, nw, y, phiT, lo, ytry, phiTtry, ltry, nacc, seed, step, sl, -1,
                            AFQMC_PROPOSAL_LEARNED, lqx, gdc, gdt, nullptr),
              "accept");
    }
    if (w == nullptr) return AFQMC_OK;
    hipError_t fe;
    int* flags = flag_words(c, nw, &fe);
    HIPCALL(c, fe, "flags");
    HIPCALL(c, launch_handoff(c, nw, lo, static_cast<const double*>(ref), w, flags), "handoff");
    return numeric_check_end(c, nw, flags);
  }
  const int nflip = (c->hidden_kind == AFQMC_HIDDEN_ISING) ? c->K : 1;
  for (int s = 0; s < n_sweep; ++s) {
    for (int f = 0; f < nflip; ++f) {
      const int flip_k = (c->hidden_kind == AFQMC_HIDDEN_ISING) ? f : -1;
      HIPCALL(c, launch_proposal(c, nw, y, ytry, seed, step, s, flip_k, c->proposal), "proposal");
      HIPCALL(c, do_trial_build(c, L, c, nw * c->P, ytry, phiTtry),
              "proposal trial build");
      HIPCALL(c, do_overlap(c, nw, ph, phiTtry, ltry, nullptr), "proposal overlap");
      HIPCALL(c,
              launch_accept(c, nw, y, phiT, lo, ytry, phiTtry, ltry, nacc, seed, step, s, flip_k,
                            c->proposal),
              "accept");
    }
  }
  if (w == nullptr) return AFQMC_OK;
  hipError_t fe;
  int* flags = flag_words(c, nw, &fe);
  HIPCALL(c, fe, "flags");
  HIPCALL(c, launch_handoff(c, nw, lo, static_cast<const double*>(ref), w, flags), "handoff");
  return numeric_check_end(c, nw, flags);
}

// Pair chain of the initialisation from the trial: two P = 1 chains whose
// walker is the other member's determinant; the walker field lives in yw, the
// partner and both determinants and log-overlaps in the workspace, the
// complex walker built from either determinant in phi.
afqmc_status afqmc_init_metropolis(afqmc_ctx c, int32_t nw, uint64_t seed, int32_t n_pair,
                                   int32_t n_burn, double* yw, void* phi, double* y, double* phiT,
                                   void* logov, double* w) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (c->ctrial)
    return fail(c, AFQMC_E_UNSUPPORTED,
                "initialisation from the trial needs the real symmetric trial family");
  if (c->c64)
    return fail(c, AFQMC_E_UNSUPPORTED, "initialisation from the trial needs complex128 walkers");
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, yw, "yw");
  REQUIRE(c, phi, "phi");
  REQUIRE(c, y, "y");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, w, "w");
  if (n_pair < 0 || n_burn < 0) return fail(c, AFQMC_E_INVALID, "n_pair and n_burn must be >= 0");
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  afqmc_ctx_s cp = *c;  // the chains' proposal: a learned one is replaced by the random walk
  if (cp.proposal == AFQMC_PROPOSAL_LEARNED) {
    cp.proposal = AFQMC_PROPOSAL_RW;
    if (!(cp.rw_step > 0.0)) cp.rw_step = 0.5;
  }
  afqmc_ctx_s c1 = cp;
  c1.P = 1;
  double* yb = ws_ptr<double>(c, L.in_yb);
  double* pa = ws_ptr<double>(c, L.in_pa);
  double* pb = ws_ptr<double>(c, L.in_pb);
  double* la = ws_ptr<double>(c, L.in_la);
  double* lb = ws_ptr<double>(c, L.in_lb);
  double* ph = static_cast<double*>(phi);
  const size_t MN = (size_t)c->M * c->N;
  auto sub = [&](afqmc_status s2, const afqmc_ctx_s& from) {
    if (s2 != AFQMC_OK) c->err = from.err;
    return s2;
  };
  HIPCALL(c, launch_sample_prior(&c1, nw, seed, yw, 1), "walker fields");
  HIPCALL(c, launch_sample_prior(&c1, nw, seed, yb, 2), "partner fields");
  HIPCALL(c, do_trial_build(c, L, &c1, nw, yw, pa), "walker trial build");
  HIPCALL(c, do_trial_build(c, L, &c1, nw, yb, pb), "partner trial build");
  for (int j = 0; j < n_pair; ++j) {
    HIPCALL(c, launch_as_walker(c, nw, pa, MN, ph), "walker from field");
    HIPCALL(c, do_overlap(&c1, nw, ph, pb, lb, nullptr), "partner overlap");
    st = sub(afqmc_metropolis_x(&c1, nw, ph, yb, pb, lb, nullptr, nullptr, seed,
                                AFQMC_INIT_STEP + 2 * (uint64_t)j, 1, nullptr), c1);
    if (st != AFQMC_OK) return st;
    HIPCALL(c, launch_as_walker(c, nw, pb, MN, ph), "walker from partner");
    HIPCALL(c, do_overlap(&c1, nw, ph, pa, la, nullptr), "walker-field overlap");
    st = sub(afqmc_metropolis_x(&c1, nw, ph, yw, pa, la, nullptr, nullptr, seed,
                                AFQMC_INIT_STEP + 2 * (uint64_t)j + 1, 1, nullptr), c1);
    if (st != AFQMC_OK) return st;
  }
  HIPCALL(c, launch_as_walker(c, nw, pa, MN, ph), "initial walkers");
  HIPCALL(c, launch_extend_paths(c, nw, 1, c->P, yb, pb, nullptr, y, phiT, nullptr), "paths");
  HIPCALL(c, do_overlap(c, nw, ph, phiT, static_cast<double*>(logov), nullptr), "overlap");
  st = sub(afqmc_metropolis_x(&cp, nw, ph, y, phiT, logov, nullptr, nullptr, seed,
                              AFQMC_INIT_STEP + 2 * (uint64_t)n_pair, n_burn, nullptr), cp);
  if (st != AFQMC_OK) return st;
  HIPCALL(c, launch_sign_sum(c, nw, c->P, static_cast<const double*>(logov), w), "weights");
  return AFQMC_OK;
}

afqmc_status afqmc_copy(afqmc_ctx c, int64_t n, const void* src, void* dst) {
  CHECK_CTX(c);
  if (n < 0) return fail(c, AFQMC_E_INVALID, "n must be >= 0");
  if (n == 0) return AFQMC_OK;
  REQUIRE(c, src, "src");
  REQUIRE(c, dst, "dst");
  HIPCALL(c, launch_copy(c, (size_t)n, static_cast<const double*>(src), static_cast<double*>(dst)),
          "copy");
  return AFQMC_OK;
}

afqmc_status afqmc_gather_rows(afqmc_ctx c, int32_t nw, const int32_t* parent, int64_t row,
                               const void* src, void* dst) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (row < 0) return fail(c, AFQMC_E_INVALID, "row must be >= 0");
  if (nw == 0 || row == 0) return AFQMC_OK;
  REQUIRE(c, parent, "parent");
  REQUIRE(c, src, "src");
  REQUIRE(c, dst, "dst");
  HIPCALL(c,
          launch_gather(c, nw, (size_t)row, parent, static_cast<const double*>(src),
                        static_cast<double*>(dst)),
          "gather_rows");
  return AFQMC_OK;
}

afqmc_status afqmc_bp_record(afqmc_ctx c, int32_t nw, int32_t h, int32_t slot, const double* xi,
                             const void* xbar, double* hist_xi, void* hist_xbar) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (h < 1 || slot < 0 || slot >= h) return fail(c, AFQMC_E_INVALID, "need 0 <= slot < h");
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, xi, "xi");
  REQUIRE(c, xbar, "xbar");
  REQUIRE(c, hist_xi, "hist_xi");
  REQUIRE(c, hist_xbar, "hist_xbar");
  HIPCALL(c,
          launch_bp_record(c, nw, h, slot, xi, static_cast<const double*>(xbar), hist_xi,
                           static_cast<double*>(hist_xbar)),
          "bp_record");
  return AFQMC_OK;
}

// Back-propagation: the measurement step's path bras through the recorded
// projectors (most recent first), their overlap with the saved walker on the
// complex-trial overlap kernel, then the path-weighted density per walker and
// its weighted sum.
afqmc_status afqmc_bp_density(afqmc_ctx c, int32_t nw, int32_t h, const void* phi_mid,
                              const double* hist_xi, const void* hist_xbar, const double* phiT,
                              const void* logov, const double* w, void* phit_bp, void* theta_bp,
                              void* logov_bp, void* rho, double* out) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (c->c64)
    return fail(c, AFQMC_E_UNSUPPORTED, "back-propagation needs complex128 walkers");
  if (h < 0) return fail(c, AFQMC_E_INVALID, "h must be >= 0");
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi_mid, "phi_mid");
  if (h > 0) {
    REQUIRE(c, hist_xi, "hist_xi");
    REQUIRE(c, hist_xbar, "hist_xbar");
  }
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, w, "w");
  REQUIRE(c, phit_bp, "phit_bp");
  REQUIRE(c, theta_bp, "theta_bp");
  REQUIRE(c, logov_bp, "logov_bp");
  REQUIRE(c, rho, "rho");
  REQUIRE(c, out, "out");
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  const size_t n = (size_t)nw * c->P * c->M * c->N;
  double* X = static_cast<double*>(phit_bp);
  if (c->ctrial)
    HIPCALL(c, launch_copy(c, 2 * n, phiT, X), "bp bra copy");
  else
    HIPCALL(c, launch_real_to_complex(c, n, phiT, X), "bp bra copy");
  double* vmat = ws_ptr<double>(c, L.vmat);
  const int G = c->G;
  const double* hxb = static_cast<const double*>(hist_xbar);
  for (int i = h - 1; i >= 0; --i) {
    HIPCALL(c,
            launch_vbuild_gen(c, nw, G, h * G, sqrt(c->dtau), c->d_Lraw, hist_xi + (size_t)i * G,
                              vmat, hxb + (size_t)2 * i * G, h * G),
            "bp V build");
    HIPCALL(c, launch_taylor_g_gen(c, nw, c->P, c->n_taylor, vmat, c->d_Eh, c->d_Eh, X, c->P, X),
            "bp projector");
  }
  afqmc_ctx_s cc = *c;  // the back-propagated bras are complex
  cc.ctrial = true;
  HIPCALL(c,
          launch_overlap_g(&cc, nw, static_cast<const double*>(phi_mid), X,
                           static_cast<double*>(logov_bp), static_cast<double*>(theta_bp), nullptr),
          "bp overlap");
  int* okw = ws_ptr<int>(c, L.acc);
  HIPCALL(c,
          launch_bp_density(c, nw, static_cast<const double*>(theta_bp), X,
                            static_cast<const double*>(logov_bp), static_cast<const double*>(logov),
                            static_cast<double*>(rho), okw),
          "bp density");
  HIPCALL(c, launch_bp_reduce(c, nw, w, static_cast<const double*>(rho), okw, out), "bp reduce");
  return AFQMC_OK;
}

afqmc_status afqmc_extend_paths(afqmc_ctx c, int32_t nw, int32_t p_src, const double* y_src,
                                const double* phiT_src, const void* logov_src, double* y,
                                double* phiT, void* logov) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  if (p_src < 1) return fail(c, AFQMC_E_INVALID, "p_src must be >= 1");
  REQUIRE(c, y_src, "y_src");
  REQUIRE(c, phiT_src, "phiT_src");
  REQUIRE(c, logov_src, "logov_src");
  REQUIRE(c, y, "y");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  HIPCALL(c,
          launch_extend_paths(c, nw, p_src, c->P, y_src, phiT_src,
                              static_cast<const double*>(logov_src), y, phiT,
                              static_cast<double*>(logov)),
          "extend_paths");
  return AFQMC_OK;
}

afqmc_status afqmc_estimator_corrected(afqmc_ctx c, int32_t nw, const double* w, const void* eloc,
                                       const void* logov, int32_t p_ref, const void* logov_ref,
                                       double* out, void* R) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (p_ref < 1) return fail(c, AFQMC_E_INVALID, "p_ref must be >= 1");
  REQUIRE(c, w, "w");
  REQUIRE(c, eloc, "eloc");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, logov_ref, "logov_ref");
  REQUIRE(c, out, "out");
  HIPCALL(c,
          launch_estimator_corrected(c, nw, p_ref, w, static_cast<const double*>(eloc),
                                     static_cast<const double*>(logov),
                                     static_cast<const double*>(logov_ref), out,
                                     static_cast<double*>(R)),
          "estimator_corrected");
  return AFQMC_OK;
}

afqmc_status afqmc_reorthogonalize(afqmc_ctx c, int32_t nw, void* phi, void* logov) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  double* ph;
  PHI_IN(c, nw, phi, &ph);
  if (c->small) {
    HIPCALL(c, launch_qr(c, nw, ph, static_cast<double*>(logov)), "qr");
  } else {
    ws_layout L;
    afqmc_status st = need_ws(c, nw, &L);
    if (st != AFQMC_OK) return st;
    HIPCALL(c, launch_qr_g(c, nw, ph, static_cast<double*>(logov), ws_ptr<double>(c, L.qrshift)),
            "qr");
  }
  return phi_out(c, nw, ph, phi);
}

afqmc_status afqmc_population_control(afqmc_ctx c, int32_t nw, void* phi, double* w, double* y,
                                      double* phiT, void* logov, uint64_t seed, uint64_t step,
                                      double w_cap, int32_t normalize, int32_t* parent) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  REQUIRE(c, w, "w");
  REQUIRE(c, y, "y");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  if (!(w_cap >= 0.0)) return fail(c, AFQMC_E_INVALID, "w_cap must be >= 0");
  if (normalize != 0 && normalize != 1) return fail(c, AFQMC_E_INVALID, "normalize must be 0 or 1");
  ws_layout L;
  afqmc_status st = need_ws(c, nw, &L);
  if (st != AFQMC_OK) return st;
  int* par = parent ? parent : ws_ptr<int>(c, L.pc_parent);
  HIPCALL(c,
          launch_comb(c, nw, w_cap, normalize, w, ws_ptr<double>(c, L.pc_C),
                      ws_ptr<double>(c, L.pc_tot), par, seed, step),
          "comb");
  const size_t S = (size_t)c->P;
  struct {
    double* state;
    size_t off, row;
  // a walker's row: 2 M N complex entries, 16 bytes each, or 8 if complex64
  } parts[4] = {{static_cast<double*>(phi), L.pc_phi, (size_t)2 * c->M * c->N * (c->c64 ? 1 : 2)},
                {y, L.pc_y, S * c->K},
                {phiT, L.pc_phiT, S * c->tsz},
                {static_cast<double*>(logov), L.pc_logov, S * 2}};
  GatherParts set{};
  for (int p = 0; p < GatherParts::NPART; ++p) {
    set.state[p] = parts[p].state;
    set.tmp[p] = ws_ptr<double>(c, parts[p].off);
    set.row[p] = parts[p].row;
  }
  HIPCALL(c, launch_gather_parts(c, nw, par, set), "gather");
  return AFQMC_OK;
}

afqmc_status afqmc_estimator(afqmc_ctx c, int32_t nw, const double* w, const void* eloc,
                             double* out) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  REQUIRE(c, w, "w");
  REQUIRE(c, eloc, "eloc");
  REQUIRE(c, out, "out");
  HIPCALL(c, launch_estimator(c, nw, w, static_cast<const double*>(eloc), out), "estimator");
  return AFQMC_OK;
}

afqmc_status afqmc_philox_normal(afqmc_ctx c, uint64_t seed, uint64_t step, uint32_t tag, int32_t nw,
                                 int32_t n, double* out) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (n < 0) return fail(c, AFQMC_E_INVALID, "n must be >= 0");
  if (tag > 0xFFFF) return fail(c, AFQMC_E_INVALID, "tag must fit in 16 bits");
  if (nw == 0 || n == 0) return AFQMC_OK;
  REQUIRE(c, out, "out");
  HIPCALL(c, launch_philox_normal(c, seed, step, tag, nw, n, out), "philox_normal");
  return AFQMC_OK;
}

int64_t afqmc_mlp_num_params(afqmc_ctx c) {
  if (c == nullptr || c->proposal != AFQMC_PROPOSAL_LEARNED) return 0;
  const int64_t D = (int64_t)c->M + c->K, H = AFQMC_MLP_HIDDEN, O = 2 * (int64_t)c->K;
  return D * H + H + H * H + H + H * O + O;
}

afqmc_status afqmc_mlp_init(afqmc_ctx c, int32_t precision, const double* params, double lr,
                            double beta1, double beta2, double eps) {
  CHECK_CTX(c);
  if (c->proposal != AFQMC_PROPOSAL_LEARNED)
    return fail(c, AFQMC_E_INVALID, "network calls need proposal = AFQMC_PROPOSAL_LEARNED");
  REQUIRE(c, params, "params");
  if (precision != AFQMC_PREC_FP32 && precision != AFQMC_PREC_BF16)
    return fail(c, AFQMC_E_UNSUPPORTED, "network precision must be FP32 or BF16");
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return fail(c, AFQMC_E_INVALID, "Adam hyper-parameters out of range");
  auto& m = c->mlp;
  const int H = AFQMC_MLP_HIDDEN;
  m.D = c->M + c->K;
  m.Dp = round16(m.D);
  m.O = 2 * c->K;
  m.Op = round16(m.O);
  m.np = afqmc_mlp_num_params(c);
  m.ob1 = (int64_t)m.D * H;
  m.oW2 = m.ob1 + H;
  m.ob2 = m.oW2 + (int64_t)H * H;
  m.oW3 = m.ob2 + H;
  m.ob3 = m.oW3 + (int64_t)H * m.O;
  const size_t sz[] = {(size_t)H * m.Dp * 4, (size_t)H * H * 4, (size_t)m.Op * H * 4,
                       (size_t)H * H * 4, (size_t)H * m.Op * 4};
  void** cp[] = {&m.w1t, &m.w2t, &m.w3t, &m.w2c, &m.w3c};
  if (m.master == nullptr) {
    HIPCALL(c, hipMalloc(&m.master, m.np * sizeof(float)), "mlp alloc");
    HIPCALL(c, hipMalloc(&m.mom1, m.np * sizeof(float)), "mlp alloc");
    HIPCALL(c, hipMalloc(&m.mom2, m.np * sizeof(float)), "mlp alloc");
    for (int i = 0; i < 5; ++i) HIPCALL(c, hipMalloc(cp[i], sz[i]), "mlp alloc");
    HIPCALL(c, hipMalloc(&m.tstep, 256), "mlp alloc");
    HIPCALL(c, hipMalloc(&m.scal, 256), "mlp alloc");
  }
  m.prec = precision;
  m.lr = lr;
  m.beta1 = beta1;
  m.beta2 = beta2;
  m.eps = eps;
  m.training = false;
  double* src = nullptr;
  HIPCALL(c, hipMalloc(&src, m.np * sizeof(double)), "mlp alloc");
  hipError_t e = hipMemcpy(src, params, m.np * sizeof(double), hipMemcpyHostToDevice);
  for (int i = 0; i < 5 && e == hipSuccess; ++i) e = hipMemsetAsync(*cp[i], 0, sz[i], c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m.tstep, 0, 256, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m.scal, 0, 256, c->stream);
  if (e == hipSuccess) e = launch_mlp_setparams(c, src);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(src);
  if (e != hipSuccess) return hip_fail(c, e, "mlp init");
  m.ready = true;
  return AFQMC_OK;
}

afqmc_status afqmc_mlp_get_params(afqmc_ctx c, double* params) {
  CHECK_CTX(c);
  REQUIRE(c, params, "params");
  if (!c->mlp.ready) return fail(c, AFQMC_E_INVALID, "network not initialised (afqmc_mlp_init)");
  std::vector<float> h((size_t)c->mlp.np);
  HIPCALL(c, hipStreamSynchronize(c->stream), "sync");
  HIPCALL(c, hipMemcpy(h.data(), c->mlp.master, h.size() * sizeof(float), hipMemcpyDeviceToHost),
          "mlp params");
  for (size_t i = 0; i < h.size(); ++i) params[i] = h[i];
  return AFQMC_OK;
}

afqmc_status afqmc_mlp_set_training(afqmc_ctx c, int32_t enabled) {
  if (c == nullptr) return AFQMC_E_INVALID;
  if (!c->mlp.ready) return fail(c, AFQMC_E_INVALID, "network not initialised (afqmc_mlp_init)");
  if (enabled != 0 && enabled != 1) return fail(c, AFQMC_E_INVALID, "enabled must be 0 or 1");
  if (enabled && !(c->rw_step > 0.0))
    return fail(c, AFQMC_E_INVALID, "training uses the random-walk moves: needs rw_step > 0");
  c->mlp.training = enabled != 0;
  return AFQMC_OK;
}

afqmc_status afqmc_mlp_forward(afqmc_ctx c, int32_t n, const double* gdiag, const double* y,
                               double* mu, double* lv) {
  CHECK_CTX(c);
  if (n < 0) return fail(c, AFQMC_E_INVALID, "n must be >= 0");
  if (n == 0) return AFQMC_OK;
  REQUIRE(c, gdiag, "gdiag");
  REQUIRE(c, y, "y");
  REQUIRE(c, mu, "mu");
  REQUIRE(c, lv, "lv");
  ws_layout L;
  afqmc_status st = mlp_check(c, n, &L);
  if (st != AFQMC_OK) return st;
  float* out = ws_ptr<float>(c, L.mlF);
  HIPCALL(c, launch_mlp_forward(c, n, round16(n), gdiag, y, out, nullptr, nullptr, nullptr),
          "mlp forward");
  HIPCALL(c, launch_mlp_outputs(c, n, out, y, mu, lv), "mlp outputs");
  return AFQMC_OK;
}

afqmc_status afqmc_mlp_train_step(afqmc_ctx c, int32_t n, const double* gdiag, const double* y,
                                  const double* ytarget, const int32_t* mask, double* loss,
                                  double* grad) {
  CHECK_CTX(c);
  if (n < 0) return fail(c, AFQMC_E_INVALID, "n must be >= 0");
  if (n == 0) return AFQMC_OK;
  REQUIRE(c, gdiag, "gdiag");
  REQUIRE(c, y, "y");
  REQUIRE(c, ytarget, "ytarget");
  REQUIRE(c, mask, "mask");
  ws_layout L;
  afqmc_status st = mlp_check(c, n, &L);
  if (st != AFQMC_OK) return st;
  float* out = ws_ptr<float>(c, L.mlF);
  void* zT = ws_ptr<void>(c, L.zT);
  HIPCALL(c,
          launch_mlp_forward(c, n, round16(n), gdiag, y, out, zT, ws_ptr<void>(c, L.h1T),
                             ws_ptr<void>(c, L.h2T)),
          "mlp forward");
  return mlp_train(c, L, n, out, y, ytarget, mask, zT, loss, grad);
}

afqmc_status afqmc_green_diag(afqmc_ctx c, int32_t nw, const void* phi, const double* phiT,
                              void* logov, double* gdiag) {
  CHECK_CTX(c);
  CHECK_NW(c, nw);
  if (c->ctrial)
    return fail(c, AFQMC_E_UNSUPPORTED, "the Green's-function diagonal needs a real trial");
  if (nw == 0) return AFQMC_OK;
  REQUIRE(c, phi, "phi");
  REQUIRE(c, phiT, "phiT");
  REQUIRE(c, logov, "logov");
  REQUIRE(c, gdiag, "gdiag");
  double* ph;
  PHI_IN(c, nw, phi, &ph);
  HIPCALL(c, do_overlap(c, nw, ph, phiT, static_cast<double*>(logov), nullptr, gdiag),
          "green diagonal");
  return AFQMC_OK;
}

}  // extern "C"
