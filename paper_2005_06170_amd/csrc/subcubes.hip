// Split of a catalog into n_div^3 equal sub-cubes of the periodic box (the
// sub-samples of Sec. 2.4.1, whose spectra Secs. 3.3 and 4.1 average and
// compare): a histogram pass, a scan, and a permute that writes each
// sub-cube's particles contiguously with positions relative to the cube.
//
// Rule, in FP64 without fused operations: u = x (n_div / L), g = floor(u),
// cube index m = g - n_div floor(g / n_div) clamped to [0, n_div - 1],
// position x' = x - g (L / n_div) rounded to float32; sub-cube number
// (m_x n_div + m_y) n_div + m_z.
#include <hip/hip_runtime.h>

#include "common.h"

namespace mps {
namespace {

constexpr int kSplitThreads = 256;
constexpr int kSplitPer = 16;  // particles per thread and block pass
constexpr int kSplitChunk = kSplitThreads * kSplitPer;

__device__ __forceinline__ int cube_axis(float x, const SplitParams& sp, double* g_out, bool* ok) {
#pragma clang fp contract(off)
  double u = static_cast<double>(x) * sp.scale;
  const bool fin = isfinite(u);
  if (!fin) u = 0.0;
  const double g = floor(u);
  const double nd = static_cast<double>(sp.n_div);
  double m = g - nd * floor(g / nd);
  m = fmin(fmax(m, 0.0), nd - 1.0);
  *g_out = g;
  *ok = fin;
  return static_cast<int>(m);
}

__device__ __forceinline__ int cube_of(const float* __restrict__ pos, int64_t i, const SplitParams& sp,
                                       double (&g)[3], bool* ok) {
  bool a, b, c;
  const int mx = cube_axis(pos[3 * i], sp, &g[0], &a);
  const int my = cube_axis(pos[3 * i + 1], sp, &g[1], &b);
  const int mz = cube_axis(pos[3 * i + 2], sp, &g[2], &c);
  *ok = a && b && c;
  return (mx * sp.n_div + my) * sp.n_div + mz;
}

__global__ __launch_bounds__(kSplitThreads) void split_reset_kernel(uint32_t* count, int n_cubes) {
  for (int i = threadIdx.x; i <= n_cubes; i += kSplitThreads) count[i] = 0;  // counts, flag
}

// Per-block histogram in LDS; non-zero bins go to the global counts.
// count[n_cubes] is set to 1 if a position is not finite.
__global__ __launch_bounds__(kSplitThreads) void split_count_kernel(const float* __restrict__ pos, int64_t n,
                                                                    SplitParams sp, uint32_t* __restrict__ count) {
  __shared__ uint32_t hist[kMaxCubes];
  __shared__ int bad;
  for (int i = threadIdx.x; i < sp.n_cubes; i += kSplitThreads) hist[i] = 0;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kSplitChunk;
  const int64_t c1 = c0 + kSplitChunk < n ? c0 + kSplitChunk : n;
  bool any_bad = false;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kSplitThreads) {
    double g[3];
    bool ok;
    const int s = cube_of(pos, i, sp, g, &ok);
    any_bad |= !ok;
    atomicAdd(&hist[s], 1u);
  }
  if (any_bad) bad = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < sp.n_cubes; i += kSplitThreads)
    if (hist[i]) atomicAdd(&count[i], hist[i]);
  if (threadIdx.x == 0 && bad) atomicOr(&count[sp.n_cubes], 1u);
}

// Exclusive scan of the counts (one workgroup; n_cubes <= kMaxCubes):
// offset[s] and the permute cursors.
__global__ __launch_bounds__(kMaxCubes) void split_scan_kernel(const uint32_t* __restrict__ count, int n_cubes,
                                                               uint32_t* __restrict__ offset,
                                                               uint32_t* __restrict__ cursor) {
  __shared__ uint32_t buf[kMaxCubes];
  const int t = threadIdx.x;
  const uint32_t v = t < n_cubes ? count[t] : 0u;
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < kMaxCubes; off <<= 1) {
    const uint32_t o = t >= off ? buf[t - off] : 0u;
    __syncthreads();
    buf[t] += o;
    __syncthreads();
  }
  if (t < n_cubes) {
    offset[t] = buf[t] - v;
    cursor[t] = buf[t] - v;
  }
  if (t == n_cubes - 1) offset[n_cubes] = buf[t];
}

// Each block recounts its chunk in LDS, reserves one range per sub-cube and
// writes its particles there (positions relative to the cube).
template <bool kHasW>
__global__ __launch_bounds__(kSplitThreads) void split_permute_kernel(
    const float* __restrict__ pos, const float* __restrict__ vel, const float* __restrict__ wgt, int64_t n,
    SplitParams sp, uint32_t* __restrict__ cursor, float* __restrict__ out_pos, float* __restrict__ out_vel,
    float* __restrict__ out_w) {
#pragma clang fp contract(off)
  __shared__ uint32_t hist[kMaxCubes];
  __shared__ uint32_t base[kMaxCubes];
  for (int i = threadIdx.x; i < sp.n_cubes; i += kSplitThreads) hist[i] = 0;
  __syncthreads();
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kSplitChunk;
  const int64_t c1 = c0 + kSplitChunk < n ? c0 + kSplitChunk : n;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kSplitThreads) {
    double g[3];
    bool ok;
    atomicAdd(&hist[cube_of(pos, i, sp, g, &ok)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < sp.n_cubes; i += kSplitThreads) {
    const uint32_t h = hist[i];
    base[i] = h ? atomicAdd(&cursor[i], h) : 0u;
    hist[i] = 0;
  }
  __syncthreads();
  for (int64_t i = c0 + threadIdx.x; i < c1; i += kSplitThreads) {
    double g[3];
    bool ok;
    const int s = cube_of(pos, i, sp, g, &ok);
    const int64_t d = static_cast<int64_t>(base[s]) + atomicAdd(&hist[s], 1u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = static_cast<double>(pos[3 * i + a]);
      out_pos[3 * d + a] = static_cast<float>(x - g[a] * sp.sub_box);
      out_vel[3 * d + a] = vel[3 * i + a];
    }
    if (kHasW) out_w[d] = wgt[i];
  }
}

unsigned split_blocks(int64_t n) { return static_cast<unsigned>((n + kSplitChunk - 1) / kSplitChunk); }

}  // namespace

hipError_t launch_split_count(const mps_catalog* c, const SplitParams& sp, uint32_t* count, hipStream_t s) {
  split_reset_kernel<<<1, kSplitThreads, 0, s>>>(count, sp.n_cubes);
  split_count_kernel<<<split_blocks(c->n_particles), kSplitThreads, 0, s>>>(c->pos, c->n_particles, sp, count);
  return hipGetLastError();
}

hipError_t launch_split_permute(const mps_catalog* c, const SplitParams& sp, const uint32_t* count,
                                uint32_t* offset, uint32_t* cursor, float* out_pos, float* out_vel, float* out_w,
                                hipStream_t s) {
  split_scan_kernel<<<1, kMaxCubes, 0, s>>>(count, sp.n_cubes, offset, cursor);
  const unsigned nb = split_blocks(c->n_particles);
  if (c->weight)
    split_permute_kernel<true><<<nb, kSplitThreads, 0, s>>>(c->pos, c->vel, c->weight, c->n_particles, sp, cursor,
                                                            out_pos, out_vel, out_w);
  else
    split_permute_kernel<false><<<nb, kSplitThreads, 0, s>>>(c->pos, c->vel, nullptr, c->n_particles, sp, cursor,
                                                             out_pos, out_vel, nullptr);
  return hipGetLastError();
}

}  // namespace mps
