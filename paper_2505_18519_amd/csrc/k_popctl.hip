// Comb population control: optional weight cap, inclusive prefix sums of W,
// comb teeth (j + u) sum(W) / nw, parent of each new walker, gather.
#include <algorithm>

#include "afqmc_internal.h"
#include "dev_common.h"

namespace {

constexpr int PC_THREADS = 1024;

// One block: W <- min(W, cap * mean W) (cap > 0), C = inclusive prefix sums of
// W (written to C), tot[0] = sum W.  Each thread scans a contiguous chunk.
__global__ void __launch_bounds__(PC_THREADS)
k_comb_scan(int nw, double w_cap, const double* __restrict__ w, double* __restrict__ C,
            double* __restrict__ tot) {
  __shared__ double s_part[PC_THREADS];
  __shared__ double s_mean;
  const int tid = threadIdx.x;
  const int chunk = (nw + PC_THREADS - 1) / PC_THREADS;
  const int b = tid * chunk, e = min(b + chunk, nw);
  double acc = 0.0;
  for (int k = b; k < e; ++k) acc += w[k];
  s_part[tid] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < PC_THREADS; ++q) s += s_part[q];
    s_mean = s / (double)nw;
  }
  __syncthreads();
  const double cap = (w_cap > 0.0) ? w_cap * s_mean : __builtin_huge_val();
  acc = 0.0;
  for (int k = b; k < e; ++k) acc += fmin(w[k], cap);
  s_part[tid] = acc;
  __syncthreads();
  // exclusive offsets of the chunks (Hillis-Steele on the 1024 partial sums)
  for (int o = 1; o < PC_THREADS; o <<= 1) {
    const double v = (tid >= o) ? s_part[tid - o] : 0.0;
    __syncthreads();
    s_part[tid] += v;
    __syncthreads();
  }
  double run = (tid > 0) ? s_part[tid - 1] : 0.0;
  for (int k = b; k < e; ++k) {
    run += fmin(w[k], cap);
    C[k] = run;
  }
  if (tid == PC_THREADS - 1) tot[0] = s_part[PC_THREADS - 1];
}

// parent[j] = min{k : C_k > (j + u) tot / nw}; new weight tot / nw (1 if normalize)
__global__ void k_comb_parent(int nw, int normalize, uint64_t seed, uint64_t step,
                              const uint64_t* __restrict__ dstep, const double* __restrict__ C,
                              const double* __restrict__ tot, int* __restrict__ parent,
                              double* __restrict__ w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nw) return;
  const double T = tot[0];
  if (!(T > 0.0)) {  // dead (or non-finite) population: unchanged
    parent[j] = j;
    return;
  }
  if (dstep != nullptr) step = *dstep;
  const double u = stream_uniform(seed, 0, step, rng_word3(AFQMC_TAG_COMB, 0, 0), 0);
  const double t = ((double)j + u) * (T / (double)nw);
  int lo = 0, hi = nw - 1;  // first k with C[k] > t, clamped to nw - 1
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  parent[j] = lo;
  w[j] = normalize ? 1.0 : T / (double)nw;
}

__global__ void k_copy_f64(size_t n, const double* __restrict__ src, double* __restrict__ dst) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = src[q];
}

// dst[j] = src[parent[j]] for rows of `row` doubles; block b copies chunk
// b % nchunk of walker b / nchunk
__global__ void k_gather_rows(int nw, size_t row, int nchunk, const int* __restrict__ parent,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const int j = blockIdx.x / nchunk;
  const int ch = blockIdx.x % nchunk;
  if (j >= nw) return;
  const int pj = parent[j];
  if (pj < 0 || pj >= nw) return;  // a parent out of range copies nothing
  const size_t base_d = (size_t)j * row, base_s = (size_t)pj * row;
  for (size_t q = (size_t)ch * blockDim.x + threadIdx.x; q < row; q += (size_t)nchunk * blockDim.x)
    dst[base_d + q] = src[base_s + q];
}

// The comb's four walker arrays in two launches: part p = blockIdx.y gathers
// rows of set.row[p] doubles into its scratch copy (as k_gather_rows), then
// k_copy_parts writes the scratch copies back over the arrays.
__global__ void k_gather_parts(int nw, GatherParts set, const int* __restrict__ parent) {
  const int p = blockIdx.y;
  const int nchunk = set.nchunk[p];
  const int j = blockIdx.x / nchunk, ch = blockIdx.x % nchunk;
  if (j >= nw) return;  // the grid is sized for the widest part
  const int pj = parent[j];
  if (pj < 0 || pj >= nw) return;  // a parent out of range copies nothing
  const size_t row = set.row[p];
  const double* src = set.state[p] + (size_t)pj * row;
  double* dst = set.tmp[p] + (size_t)j * row;
  for (size_t q = (size_t)ch * blockDim.x + threadIdx.x; q < row; q += (size_t)nchunk * blockDim.x)
    dst[q] = src[q];
}

__global__ void k_copy_parts(int nw, GatherParts set) {
  const int p = blockIdx.y;
  const size_t n = (size_t)nw * set.row[p];
  const double* src = set.tmp[p];
  double* dst = set.state[p];
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = src[q];
}

}  // namespace

hipError_t launch_gather_parts(const afqmc_ctx_s* c, int nw, const int* parent, GatherParts set) {
  if (nw <= 0) return hipSuccess;
  int wide = 1;
  size_t most = 0;
  for (int p = 0; p < GatherParts::NPART; ++p) {
    set.nchunk[p] = (int)std::max<size_t>(1, std::min<size_t>((set.row[p] + 255) / 256, 64));
    wide = std::max(wide, set.nchunk[p]);
    most = std::max(most, (size_t)nw * set.row[p]);
  }
  hipLaunchKernelGGL(k_gather_parts, dim3((unsigned)(wide * nw), GatherParts::NPART), dim3(256), 0,
                     c->stream, nw, set, parent);
  AFQMC_LAUNCH_CHECK();
  const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>((most + 255) / 256, 1024));
  hipLaunchKernelGGL(k_copy_parts, dim3(blocks, GatherParts::NPART), dim3(256), 0, c->stream, nw, set);
  return hipGetLastError();
}

hipError_t launch_comb(const afqmc_ctx_s* c, int nw, double w_cap, int normalize, double* w,
                       double* C, double* tot, int* parent, uint64_t seed, uint64_t step) {
  hipLaunchKernelGGL(k_comb_scan, dim3(1), dim3(PC_THREADS), 0, c->stream, nw, w_cap, w, C, tot);
  AFQMC_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_comb_parent, dim3((nw + 255) / 256), dim3(256), 0, c->stream, nw,
                     normalize, seed, step, c->dstep, C, tot, parent, w);
  return hipGetLastError();
}

hipError_t launch_gather(const afqmc_ctx_s* c, int nw, size_t row, const int* parent,
                         const double* src, double* dst) {
  if (nw <= 0 || row == 0) return hipSuccess;
  const int nchunk = (int)std::min<size_t>((row + 255) / 256, 64);
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)(nchunk * nw)), dim3(256), 0, c->stream, nw, row,
                     nchunk, parent, src, dst);
  return hipGetLastError();
}

hipError_t launch_copy(const afqmc_ctx_s* c, size_t n, const double* src, double* dst) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy_f64, dim3(blocks), dim3(256), 0, c->stream, n, src, dst);
  return hipGetLastError();
}
