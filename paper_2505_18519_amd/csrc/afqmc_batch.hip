// Uneven batching: many independent systems of different size advanced
// together, each step of every system being the App. B step of the per-system
// calls (green -> local energy -> estimator -> fields -> propagate ->
// Metropolis -> QR -> comb).
//
// MI355X design.  One persistent kernel across systems would run every
// system at the register footprint and tile padding of the largest (N = 6
// padded to the 32 columns of an M = 128 system wastes 28x in the N x N
// stage), so each system keeps its own size-specialised kernels and the batch
// overlaps them instead:
//  * the walker state of all systems lives in one packed device arena, the
//    per-system workspaces in another;
//  * a cycle of n steps (the QR period, made even so that the log-overlap
//    double buffer returns to its start) of every system is captured once as
//    one hipGraph and replayed: one host launch per cycle;
//  * inside the graph each system's kernel chain runs on one of S parallel
//    branches (fork/join through events), so small systems fill the compute
//    units while large ones run; systems are assigned to branches by the
//    longest-processing-time rule on their measured step time;
//  * every system has its own step counter in device memory, which the
//    random-number, comb and estimator kernels read, so the replayed graph
//    advances the streams without host updates;
//  * the autotuner times, per system, the kernel families that apply to its
//    (M, N) (register-resident wavefront-per-path kernels for M <= 64,
//    N <= 16; workgroup-per-path kernels for any size, with the FP64
//    contraction's operands in registers or streamed from L2 for N <= 32) and,
//    for the batch, S in {1, 2, 4}, and keeps the fastest.
#include <algorithm>
#include <chrono>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "afqmc_internal.h"

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ void k_batch_init(int nw, int M, int N, const double* __restrict__ phi0,
                             double* __restrict__ phi, double* __restrict__ w) {
  const size_t total = (size_t)nw * 2 * M * N;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    const size_t mn = q % ((size_t)M * N);
    phi[2 * q] = phi0[mn];
    phi[2 * q + 1] = 0.0;
    if (q < (size_t)nw) w[q] = 1.0;
  }
}

__global__ void k_step_incr(uint64_t* s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) s[0] = s[0] + 1;
}

struct sys_state {
  afqmc_ctx c = nullptr;
  int nw = 0, M = 0, N = 0, G = 0, K = 0, P = 0;
  uint64_t seed = 0;
  double *phi = nullptr, *w = nullptr, *y = nullptr, *phiT = nullptr, *logov = nullptr,
         *logov_new = nullptr, *theta = nullptr, *xbar = nullptr, *eloc = nullptr, *xi = nullptr,
         *ref = nullptr, *est = nullptr;
  int* nacc = nullptr;
  uint64_t* dstep = nullptr;
  // 0 register-resident kernels, 1 workgroup-per-path kernels, 2 the same with the
  // FP64 contraction's operands streamed (contract_variant 1)
  int family = 1;
  int branch = 0;
  double ms = 0.0;  // measured time of one step alone
  bool can_small = false;
  bool can_stream = false;  // FP64 real trial with N <= 32 (past that it always streams)
};

}  // namespace

struct afqmc_batch_s {
  int device = 0;
  hipStream_t user = nullptr;    // the caller's stream
  hipStream_t stream = nullptr;  // the batch's own stream: set-up, capture and replays
  afqmc_batch_options opt{};
  int cycle = 0;
  std::vector<sys_state> s;
  void* arena = nullptr;
  void* ws = nullptr;
  uint64_t* steps = nullptr;
  hipStream_t br[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_in = nullptr, ev_out = nullptr;  // ordering with the caller's stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_branches = 1;
  std::string err;
};

namespace {

afqmc_status bfail(afqmc_batch_s* b, afqmc_status st, const std::string& m) {
  b->err = m;
  return st;
}

#define BCALL(b, expr, what)                                                               \
  do {                                                                                     \
    afqmc_status st_ = (expr);                                                             \
    if (st_ != AFQMC_OK) return bfail((b), st_, std::string(what) + ": " + afqmc_last_error(sys.c)); \
  } while (0)

#define BHIP(b, expr, what)                                                                \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return bfail((b), AFQMC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

// one App. B step of one system on stream st (eager or under capture)
afqmc_status one_step(afqmc_batch_s* b, sys_state& sys, hipStream_t st, bool qr, bool pc) {
  afqmc_ctx c = sys.c;
  c->stream = st;
  const int nw = sys.nw;
  BCALL(b, afqmc_green(c, nw, sys.phi, sys.phiT, sys.logov, sys.theta), "green");
  BCALL(b, afqmc_local_energy(c, nw, sys.phiT, sys.theta, sys.logov, sys.eloc, nullptr, sys.xbar),
        "local energy");
  BCALL(b, afqmc_estimator(c, nw, sys.w, sys.eloc, sys.est), "estimator");
  BCALL(b, afqmc_philox_normal(c, sys.seed, 0, AFQMC_TAG_FIELD, nw, sys.G, sys.xi), "fields");
  BCALL(b,
        afqmc_propagate(c, nw, sys.phi, sys.xi, sys.xbar, sys.phiT, sys.logov, sys.eloc, 0.0,
                        sys.w, sys.ref, sys.logov_new),
        "propagate");
  BCALL(b,
        afqmc_metropolis_x(c, nw, sys.phi, sys.y, sys.phiT, sys.logov_new, sys.ref, sys.w, sys.seed,
                           0, b->opt.n_sweep, sys.nacc),
        "metropolis");
  std::swap(sys.logov, sys.logov_new);
  if (qr) BCALL(b, afqmc_reorthogonalize(c, nw, sys.phi, sys.logov), "qr");
  if (pc)
    BCALL(b,
          afqmc_population_control(c, nw, sys.phi, sys.w, sys.y, sys.phiT, sys.logov, sys.seed, 0,
                                   b->opt.w_cap, 1, nullptr),
          "population control");
  hipLaunchKernelGGL(k_step_incr, dim3(1), dim3(64), 0, st, sys.dstep);
  BHIP(b, hipGetLastError(), "step counter");
  return AFQMC_OK;
}

// step k of the cycle (0-based): QR after the last step of the cycle's QR
// period, comb every n_pc steps
bool qr_at(const afqmc_batch_s* b, int k) {
  return b->opt.n_qr > 0 && (k + 1) % b->opt.n_qr == 0;
}
bool pc_at(const afqmc_batch_s* b, int k) { return (k + 1) % b->opt.n_pc == 0; }

void destroy_graph(afqmc_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// longest-processing-time assignment of systems to S branches
void assign_branches(afqmc_batch_s* b, int S) {
  std::vector<int> order(b->s.size());
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return b->s[x].ms > b->s[y].ms; });
  std::vector<double> load(S, 0.0);
  for (int i : order) {
    const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->s[i].branch = j;
    load[j] += b->s[i].ms;
  }
  b->n_branches = S;
}

afqmc_status capture(afqmc_batch_s* b) {
  destroy_graph(b);
  const int S = b->n_branches;
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  auto abort_capture = [&](afqmc_status st) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    for (auto& sys : b->s) sys.c->stream = b->stream;
    return st;
  };
  if (S > 1) {
    if (hipEventRecord(b->ev_fork, b->stream) != hipSuccess)
      return abort_capture(bfail(b, AFQMC_E_DEVICE, "fork event"));
    for (int j = 0; j < S; ++j)
      if (hipStreamWaitEvent(b->br[j], b->ev_fork, 0) != hipSuccess)
        return abort_capture(bfail(b, AFQMC_E_DEVICE, "fork wait"));
  }
  for (int k = 0; k < b->cycle; ++k)
    for (auto& sys : b->s) {
      hipStream_t st = (S > 1) ? b->br[sys.branch] : b->stream;
      afqmc_status r = one_step(b, sys, st, qr_at(b, k), pc_at(b, k));
      if (r != AFQMC_OK) return abort_capture(r);
    }
  if (S > 1)
    for (int j = 0; j < S; ++j) {
      if (hipEventRecord(b->ev_join[j], b->br[j]) != hipSuccess ||
          hipStreamWaitEvent(b->stream, b->ev_join[j], 0) != hipSuccess)
        return abort_capture(bfail(b, AFQMC_E_DEVICE, "join"));
    }
  for (auto& sys : b->s) sys.c->stream = b->stream;
  BHIP(b, hipStreamEndCapture(b->stream, &b->graph), "end capture");
  BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate");
  return AFQMC_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t z) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, z);
  return ms;
}

afqmc_status tune(afqmc_batch_s* b) {
  hipEvent_t t0, t1;
  BHIP(b, hipEventCreate(&t0), "event");
  BHIP(b, hipEventCreate(&t1), "event");
  struct guard {
    hipEvent_t a, z;
    ~guard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(z);
    }
  } g{t0, t1};
  // 1. kernel family per system, from one eager step of each candidate (after
  //    a first untimed step that settles clocks and caches)
  for (auto& sys : b->s) {
    const int fams[3] = {0, 1, 2};
    double best = 1e300;
    int best_f = 1;
    for (int f : fams) {
      if (f == 0 && !sys.can_small) continue;
      if (f == 2 && !sys.can_stream) continue;
      sys.c->small = (f == 0);
      sys.c->contract_variant = (f == 2) ? 1 : 0;
      for (int rep = 0; rep < 2; ++rep) {
        BHIP(b, hipEventRecord(t0, b->stream), "event");
        afqmc_status r = one_step(b, sys, b->stream, false, true);
        if (r != AFQMC_OK) return r;
        BHIP(b, hipEventRecord(t1, b->stream), "event");
        BHIP(b, hipEventSynchronize(t1), "sync");
      }
      const double ms = elapsed_ms(t0, t1);
      if (ms < best) {
        best = ms;
        best_f = f;
      }
    }
    sys.family = best_f;
    sys.c->small = (best_f == 0);
    sys.c->contract_variant = (best_f == 2) ? 1 : 0;
    sys.ms = best;
  }
  // 2. number of parallel branches, from a replay of the whole captured cycle
  double best = 1e300;
  int best_S = 1;
  const int cand[3] = {1, 2, 4};
  for (int S : cand) {
    if (S > b->opt.max_branches || S > (int)b->s.size()) continue;
    assign_branches(b, S);
    afqmc_status r = capture(b);
    if (r != AFQMC_OK) return r;
    BHIP(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
    BHIP(b, hipEventRecord(t0, b->stream), "event");
    BHIP(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
    BHIP(b, hipEventRecord(t1, b->stream), "event");
    BHIP(b, hipEventSynchronize(t1), "sync");
    const double ms = elapsed_ms(t0, t1);
    if (ms < best) {
      best = ms;
      best_S = S;
    }
  }
  assign_branches(b, best_S);
  return capture(b);
}

void free_batch(afqmc_batch_s* b) {
  destroy_graph(b);
  for (auto& sys : b->s)
    if (sys.c) (void)afqmc_destroy(sys.c);
  if (b->arena) (void)hipFree(b->arena);
  if (b->ws) (void)hipFree(b->ws);
  if (b->steps) (void)hipFree(b->steps);
  for (auto& st : b->br)
    if (st) (void)hipStreamDestroy(st);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  for (auto& e : b->ev_join)
    if (e) (void)hipEventDestroy(e);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->stream) (void)hipStreamDestroy(b->stream);
}

afqmc_status build(afqmc_batch_s* b, const afqmc_system* systems, const int32_t* walkers, int n) {
  BHIP(b, hipSetDevice(b->device), "device");
  BHIP(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "stream");
  BHIP(b, hipStreamSynchronize(b->user), "sync");
  b->s.resize(n);
  // contexts, sizes
  size_t arena = 0, wsb = 0;
  const int H = b->opt.history;
  for (int i = 0; i < n; ++i) {
    sys_state& sys = b->s[i];
    afqmc_system sd = systems[i];
    if (sd.proposal == AFQMC_PROPOSAL_LEARNED)
      return bfail(b, AFQMC_E_UNSUPPORTED, "the batch runs prior / random-walk proposals");
    afqmc_status st = afqmc_create(&sd, b->device, b->stream, &sys.c);
    if (st != AFQMC_OK) return bfail(b, st, "system " + std::to_string(i) + ": afqmc_create failed");
    sys.nw = walkers[i];
    sys.M = sd.M;
    sys.N = sd.N;
    sys.G = sd.n_chol;
    sys.K = sd.K;
    sys.P = sd.P;
    sys.seed = b->opt.seed + (uint64_t)i;
    sys.can_small = sys.c->small;
    sys.can_stream = sd.precision == AFQMC_PREC_FP64 && !sys.c->ctrial && sd.N <= 32;
    sys.family = sys.c->small ? 0 : 1;
    const size_t nw = sys.nw, M = sys.M, N = sys.N, P = sys.P, K = sys.K, G = sys.G;
    const size_t tsz = (size_t)sys.c->tsz;  // doubles per trial determinant (complex: 2 M N)
    arena += al256(nw * 2 * M * N * 16) + al256(nw * 8) + al256(nw * P * K * 8) +
             al256(nw * P * tsz * 8) + 2 * al256(nw * P * 16) + al256(nw * P * 2 * M * N * 16) +
             al256(nw * G * 16) + al256(nw * 16) + al256(nw * G * 8) + al256(nw * 16) +
             al256(nw * 4) + al256((size_t)H * 16);
    size_t wsz = 0;
    if (afqmc_workspace_size(sys.c, sys.nw, &wsz) != AFQMC_OK)
      return bfail(b, AFQMC_E_INVALID, "workspace size");
    wsb += al256(wsz);
  }
  BHIP(b, hipMalloc(&b->arena, std::max<size_t>(arena, 256)), "state arena");
  BHIP(b, hipMalloc(&b->ws, std::max<size_t>(wsb, 256)), "workspace arena");
  BHIP(b, hipMalloc(&b->steps, std::max<size_t>(n, 1) * sizeof(uint64_t)), "step counters");
  BHIP(b, hipMemsetAsync(b->steps, 0, n * sizeof(uint64_t), b->stream), "step counters");
  char* p = static_cast<char*>(b->arena);
  char* q = static_cast<char*>(b->ws);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += al256(bytes);
    return r;
  };
  for (int i = 0; i < n; ++i) {
    sys_state& sys = b->s[i];
    const size_t nw = sys.nw, M = sys.M, N = sys.N, P = sys.P, K = sys.K, G = sys.G;
    sys.phi = (double*)take(nw * 2 * M * N * 16);
    sys.w = (double*)take(nw * 8);
    sys.y = (double*)take(nw * P * K * 8);
    sys.phiT = (double*)take(nw * P * (size_t)sys.c->tsz * 8);
    sys.logov = (double*)take(nw * P * 16);
    sys.logov_new = (double*)take(nw * P * 16);
    sys.theta = (double*)take(nw * P * 2 * M * N * 16);
    sys.xbar = (double*)take(nw * G * 16);
    sys.eloc = (double*)take(nw * 16);
    sys.xi = (double*)take(nw * G * 8);
    sys.ref = (double*)take(nw * 16);
    sys.nacc = (int*)take(nw * 4);
    sys.est = (double*)take((size_t)H * 16);
    sys.dstep = b->steps + i;
    size_t wsz = 0;
    (void)afqmc_workspace_size(sys.c, sys.nw, &wsz);
    if (afqmc_set_workspace(sys.c, q, wsz) != AFQMC_OK)
      return bfail(b, AFQMC_E_INVALID, "set workspace");
    q += al256(wsz);
    sys.c->dstep = sys.dstep;
    sys.c->est_cap = H;
    sys.c->stream = b->stream;
    // initial state: phi = Phi_0 for both spins, W = 1, y ~ p_T, Phi_T(y), l
    hipLaunchKernelGGL(k_batch_init, dim3(1024), dim3(256), 0, b->stream, sys.nw, sys.M, sys.N,
                       sys.c->d_phi0, sys.phi, sys.w);
    BHIP(b, hipGetLastError(), "init");
    BCALL(b, afqmc_sample_prior(sys.c, sys.nw, sys.seed, sys.y), "prior");
    BCALL(b, afqmc_trial_build(sys.c, sys.nw, sys.y, sys.phiT), "trial build");
    BCALL(b, afqmc_overlap(sys.c, sys.nw, sys.phi, sys.phiT, sys.logov), "overlap");
  }
  for (auto& st : b->br) BHIP(b, hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
  BHIP(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "event");
  for (auto& e : b->ev_join) BHIP(b, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  BHIP(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "event");
  BHIP(b, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "event");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  if (b->opt.autotune) {
    afqmc_status r = tune(b);
    if (r != AFQMC_OK) return r;
  } else {
    for (auto& sys : b->s) sys.ms = (double)sys.nw * sys.P * sys.G * sys.M * sys.M * sys.N;
    assign_branches(b, std::min<int>(b->opt.max_branches, (int)b->s.size()));
    afqmc_status r = capture(b);
    if (r != AFQMC_OK) return r;
  }
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  return AFQMC_OK;
}

}  // namespace

extern "C" {

afqmc_status afqmc_batch_create(const afqmc_system* systems, const int32_t* walkers,
                                int32_t n_systems, const afqmc_batch_options* opt, int device,
                                void* stream, afqmc_batch* out) {
  if (systems == nullptr || walkers == nullptr || opt == nullptr || out == nullptr)
    return AFQMC_E_INVALID;
  *out = nullptr;
  if (n_systems < 1) return AFQMC_E_INVALID;
  for (int i = 0; i < n_systems; ++i) {
    if (walkers[i] < 1) return AFQMC_E_INVALID;
    if (systems[i].walker_c64 != 0) return AFQMC_E_UNSUPPORTED;  // the arena holds complex128
  }
  if (opt->n_sweep < 0 || opt->n_qr < 0 || opt->n_pc < 1 || !(opt->w_cap >= 0.0) ||
      opt->max_branches < 1 || opt->max_branches > 4 || opt->history < 1 ||
      (opt->autotune != 0 && opt->autotune != 1))
    return AFQMC_E_INVALID;
  afqmc_batch_s* b = new (std::nothrow) afqmc_batch_s();
  if (b == nullptr) return AFQMC_E_NOMEM;
  b->device = device;
  b->user = static_cast<hipStream_t>(stream);
  b->opt = *opt;
  // cycle: a multiple of the QR and comb periods, even (log-overlap buffers)
  int cyc = std::max(1, opt->n_qr);
  while (cyc % opt->n_pc != 0) cyc += std::max(1, opt->n_qr);
  if (cyc % 2) cyc *= 2;
  b->cycle = cyc;
  afqmc_status st = build(b, systems, walkers, n_systems);
  if (st != AFQMC_OK) {
    free_batch(b);
    delete b;
    return st;
  }
  *out = b;
  return AFQMC_OK;
}

int32_t afqmc_batch_cycle(afqmc_batch b) { return b ? b->cycle : 0; }

afqmc_status afqmc_batch_run(afqmc_batch b, int32_t n_cycles) {
  if (b == nullptr || n_cycles < 0) return AFQMC_E_INVALID;
  BHIP(b, hipSetDevice(b->device), "device");
  // ordered after the caller's stream, and the caller's stream after the cycles
  BHIP(b, hipEventRecord(b->ev_in, b->user), "event");
  BHIP(b, hipStreamWaitEvent(b->stream, b->ev_in, 0), "wait");
  for (int i = 0; i < n_cycles; ++i) BHIP(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
  BHIP(b, hipEventRecord(b->ev_out, b->stream), "event");
  BHIP(b, hipStreamWaitEvent(b->user, b->ev_out, 0), "wait");
  return AFQMC_OK;
}

afqmc_status afqmc_batch_estimates(afqmc_batch b, double* out, uint64_t* steps) {
  if (b == nullptr || out == nullptr || steps == nullptr) return AFQMC_E_INVALID;
  BHIP(b, hipSetDevice(b->device), "device");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  const size_t H = (size_t)b->opt.history;
  for (size_t i = 0; i < b->s.size(); ++i)
    BHIP(b, hipMemcpy(out + i * H * 2, b->s[i].est, H * 16, hipMemcpyDeviceToHost), "estimates");
  BHIP(b, hipMemcpy(steps, b->steps, b->s.size() * sizeof(uint64_t), hipMemcpyDeviceToHost),
       "steps");
  return AFQMC_OK;
}

afqmc_status afqmc_batch_plan(afqmc_batch b, int32_t* family, int32_t* branch, double* step_ms,
                              int32_t* n_branches) {
  if (b == nullptr) return AFQMC_E_INVALID;
  for (size_t i = 0; i < b->s.size(); ++i) {
    if (family) family[i] = b->s[i].family;
    if (branch) branch[i] = b->s[i].branch;
    if (step_ms) step_ms[i] = b->s[i].ms;
  }
  if (n_branches) *n_branches = b->n_branches;
  return AFQMC_OK;
}

const char* afqmc_batch_last_error(afqmc_batch b) { return b ? b->err.c_str() : "null batch"; }

afqmc_status afqmc_batch_destroy(afqmc_batch b) {
  if (b == nullptr) return AFQMC_E_INVALID;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  delete b;
  return AFQMC_OK;
}

}  // extern "C"
