// Particle-side stages of the estimator on gfx950:
//   moments + tile histogram -> derive -> tile scan -> permute -> BL3 scatter.
//
// The moments are the FP64 sums that the shot-noise and bulk-flow terms need
// (Eqs. rawppnoise, thetanoise; v_b of Sec. 3.1).  The scatter assigns
// rho, rho v_x, rho v_y, rho v_z to the periodic grid with the truncated
// cubic Battle-Lemarie kernel (Eq. rawFFTed with the BL3 window,
// Sec. 2.4.1): particles are counting-sorted by T^3 tile, one workgroup
// accumulates a tile plus its 5-cell halo in LDS with ds_add, then flushes
// the block to HBM with global atomic adds.
#include <hip/hip_runtime.h>

#include "common.h"

namespace mps {
namespace {

constexpr int kCountThreads = 256;

// Grid coordinate of one float32 coordinate: u = x * (N / L) in FP64, cell
// floor(u) mod N, fraction f = u - floor(u).  The same expression, without
// fused operations, decides the tile in the sort and the taps in the
// scatter.
__device__ __forceinline__ int locate(float x, double scale, int n, double* frac, bool* ok) {
#pragma clang fp contract(off)
  double u = static_cast<double>(x) * scale;
  const bool fin = isfinite(u);
  if (!fin) u = 0.0;
  const double uf = floor(u);
  *frac = u - uf;
  const double m = uf - static_cast<double>(n) * floor(uf / static_cast<double>(n));
  int c = static_cast<int>(m);
  c = c < 0 ? 0 : (c >= n ? n - 1 : c);
  *ok = fin;
  return c;
}

// Lanes of a wave that carry equal keys in consecutive positions add their
// run length to counters[key] with one atomic; each lane gets
// old_value + (its rank within the run).  Invalid lanes take no part.
__device__ __forceinline__ uint32_t wave_run_atomic(uint32_t key, bool valid, uint32_t* counters) {
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(key, 1);
  const bool head = valid && (lane == 0 || key != prev);
  const unsigned long long heads = __ballot(head);
  const unsigned long long vmask = __ballot(valid);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long mine = heads & upto;
  const int start = mine ? 63 - __clzll(static_cast<long long>(mine)) : lane;
  const unsigned long long after = (heads | ~vmask) & ~upto;
  const int end = after ? __ffsll(static_cast<long long>(after)) - 1 : 64;
  uint32_t base = 0;
  if (head) base = atomicAdd(&counters[key], static_cast<uint32_t>(end - lane));
  base = __shfl(base, start);
  return base + static_cast<uint32_t>(lane - start);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

struct KeyParams {
  double scale;  // N / L
  int n;         // grid size
  int tshift;    // log2(tile)
  int nt;        // tiles per axis
};

__device__ __forceinline__ uint32_t tile_key(float x, float y, float z, const KeyParams& kp, bool* ok) {
  double f;
  bool a, b, c;
  const int cx = locate(x, kp.scale, kp.n, &f, &a);
  const int cy = locate(y, kp.scale, kp.n, &f, &b);
  const int cz = locate(z, kp.scale, kp.n, &f, &c);
  *ok = a && b && c;
  return static_cast<uint32_t>(((cx >> kp.tshift) * kp.nt + (cy >> kp.tshift)) * kp.nt + (cz >> kp.tshift));
}

// Moments (FP64) and tile histogram in one pass over the catalog.
template <bool kHasW>
__global__ __launch_bounds__(kCountThreads) void count_kernel(
    const float* __restrict__ pos, const float* __restrict__ vel, const float* __restrict__ wgt,
    int64_t np, KeyParams kp, uint32_t* __restrict__ tile_count, double* __restrict__ partials,
    ResultHeader* hdr) {
  double acc[kMomentSums];
#pragma unroll
  for (int q = 0; q < kMomentSums; ++q) acc[q] = 0.0;
  bool bad = false;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCountThreads;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCountThreads; base < np; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < np;
    uint32_t key = 0xffffffffu;
    if (valid) {
      const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
      bool ok;
      key = tile_key(x, y, z, kp, &ok);
      bad |= !ok;
      const double w = kHasW ? static_cast<double>(wgt[i]) : 1.0;
      const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
      const double w2 = w * w;
      acc[0] += w;
      acc[1] += w2;
      acc[2] += w * vx;
      acc[3] += w * vy;
      acc[4] += w * vz;
      acc[5] += w2 * vx;
      acc[6] += w2 * vy;
      acc[7] += w2 * vz;
      acc[8] += w2 * vx * vx;
      acc[9] += w2 * vy * vy;
      acc[10] += w2 * vz * vz;
      acc[11] += w2 * vx * vy;
      acc[12] += w2 * vx * vz;
      acc[13] += w2 * vy * vz;
    }
    wave_run_atomic(key, valid, tile_count);
  }
  __shared__ double red[kCountThreads / 64][kMomentSums];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < kMomentSums; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kMomentSums) {
    double s = 0.0;
    for (int w = 0; w < kCountThreads / 64; ++w) s += red[w][threadIdx.x];
    partials[blockIdx.x * kMomentSums + threadIdx.x] = s;
  }
  if (bad) atomicOr(&hdr->flags, 1u);
}

// Fixed-order sum of the per-block moment partials, then the derived shot
// and bulk-flow scalars.
__global__ __launch_bounds__(64) void derive_kernel(const double* __restrict__ partials, int nblocks,
                                                    ResultHeader* hdr, int bulk) {
  __shared__ double sums[kMomentSums];
  if (threadIdx.x < kMomentSums) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partials[b * kMomentSums + threadIdx.x];
    sums[threadIdx.x] = s;
    hdr->sums[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  Derived d;
  d.W = sums[0];
  d.W2 = sums[1];
  const double iw = 1.0 / d.W;
  for (int a = 0; a < 3; ++a) d.vb[a] = sums[2 + a] * iw;
  const double iw2 = iw * iw;
  d.s_dd = d.W2 * iw2;
  // sum w^2 v_a v_b, ordered xx yy zz xy xz yz
  double m2[6] = {sums[8], sums[9], sums[10], sums[11], sums[12], sums[13]};
  if (bulk) {
    // sum w^2 (v - v_b)_a (v - v_b)_b = M_ab - s_a vb_b - vb_a s_b + W2 vb_a vb_b
    const double* s = sums + 5;
    const double* vb = d.vb;
    const int ia[6] = {0, 1, 2, 0, 0, 1};
    const int ib[6] = {0, 1, 2, 1, 2, 2};
    for (int q = 0; q < 6; ++q)
      m2[q] = m2[q] - s[ia[q]] * vb[ib[q]] - vb[ia[q]] * s[ib[q]] + d.W2 * vb[ia[q]] * vb[ib[q]];
  }
  for (int q = 0; q < 6; ++q) d.S[q] = m2[q] * iw2;
  d.s_pp = d.S[0] + d.S[1] + d.S[2];
  d.inv_W = iw;
  d.sigma_v2 = (m2[0] + m2[1] + m2[2]) / d.W2;
  d.bulk = bulk;
  hdr->d = d;
}

// Exclusive scan of the tile counts (one workgroup); also resets the cursor.
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t* __restrict__ count, int64_t n_tiles,
                                                    uint32_t* __restrict__ offset, uint32_t* __restrict__ cursor) {
  __shared__ uint32_t part[1024];
  const int64_t per = (n_tiles + 1023) / 1024;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < n_tiles ? lo + per : n_tiles;
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += count[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int64_t i = lo; i < hi; ++i) {
    offset[i] = run;
    cursor[i] = run;
    run += count[i];
  }
  if (threadIdx.x == 1023) offset[n_tiles] = part[1023];
}

// Counting-sort scatter of the particle records into tile order.  Record:
// (x, y, z, w), (v_x, v_y, v_z, 0).
template <bool kHasW>
__global__ __launch_bounds__(kCountThreads) void permute_kernel(
    const float* __restrict__ pos, const float* __restrict__ vel, const float* __restrict__ wgt,
    int64_t np, KeyParams kp, uint32_t* __restrict__ cursor, float4* __restrict__ sorted) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCountThreads;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCountThreads; base < np; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < np;
    uint32_t key = 0xffffffffu;
    float x = 0.f, y = 0.f, z = 0.f;
    if (valid) {
      x = pos[3 * i];
      y = pos[3 * i + 1];
      z = pos[3 * i + 2];
      bool ok;
      key = tile_key(x, y, z, kp, &ok);
    }
    const uint32_t slot = wave_run_atomic(key, valid, cursor);
    if (valid) {
      const float w = kHasW ? wgt[i] : 1.0f;
      sorted[2 * static_cast<int64_t>(slot)] = make_float4(x, y, z, w);
      sorted[2 * static_cast<int64_t>(slot) + 1] = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void clear_kernel(T* __restrict__ g, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) g[i] = T(0);
}

__device__ __forceinline__ double tap_weight(const TapPoly& tp, int j, double f) {
  return ((tp.c[j][3] * f + tp.c[j][2]) * f + tp.c[j][1]) * f + tp.c[j][0];
}

// One workgroup per occupied tile.  LDS holds the four fields over the tile
// plus a halo of 2 cells below and 3 above along each axis (taps -2..3).
template <typename T, int TS, int NT>
__global__ __launch_bounds__(NT) void scatter_kernel(
    const float4* __restrict__ sorted, const uint32_t* __restrict__ offset, T* __restrict__ grid,
    KeyParams kp, int64_t n_tiles, int64_t xcd_chunk, TapPoly tp, Derived* dsrc, int bulk) {
  constexpr int E = TS + 5;
  constexpr int VOL = E * E * E;
  __shared__ T acc[kNumFields * VOL];
  const int64_t b = blockIdx.x;
  // consecutive tiles (spatial neighbours, which share halo cache lines) go
  // to one XCD: workgroups are dealt to the 8 XCDs round robin
  const int64_t tile = xcd_chunk > 0 ? (b & 7) * xcd_chunk + (b >> 3) : b;
  if (tile >= n_tiles) return;
  const uint32_t p0 = offset[tile], p1 = offset[tile + 1];
  if (p0 == p1) return;
  for (int i = threadIdx.x; i < kNumFields * VOL; i += NT) acc[i] = T(0);
  // bulk-flow removal in the grid itself (the assign diagnostic): v - v_b
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  if (bulk) {
    vb0 = dsrc->vb[0];
    vb1 = dsrc->vb[1];
    vb2 = dsrc->vb[2];
  }
  __syncthreads();
  const int nt = kp.nt;
  const int tz = static_cast<int>(tile % nt);
  const int ty = static_cast<int>((tile / nt) % nt);
  const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
  const int ox = tx * TS, oy = ty * TS, oz = tz * TS;
  for (uint32_t p = p0 + threadIdx.x; p < p1; p += NT) {
    const float4 a = sorted[2 * static_cast<int64_t>(p)];
    const float4 v = sorted[2 * static_cast<int64_t>(p) + 1];
    double fx, fy, fz;
    bool ok;
    int cx = locate(a.x, kp.scale, kp.n, &fx, &ok) - ox;
    int cy = locate(a.y, kp.scale, kp.n, &fy, &ok) - oy;
    int cz = locate(a.z, kp.scale, kp.n, &fz, &ok) - oz;
    cx = min(max(cx, 0), TS - 1);
    cy = min(max(cy, 0), TS - 1);
    cz = min(max(cz, 0), TS - 1);
    T wx[kTaps], wy[kTaps], wz[kTaps];
#pragma unroll
    for (int j = 0; j < kTaps; ++j) {
      wx[j] = static_cast<T>(tap_weight(tp, j, fx));
      wy[j] = static_cast<T>(tap_weight(tp, j, fy));
      wz[j] = static_cast<T>(tap_weight(tp, j, fz));
    }
    T q[kNumFields];
    if (bulk) {
      const double w = a.w;
      q[0] = static_cast<T>(w);
      q[1] = static_cast<T>(w * (static_cast<double>(v.x) - vb0));
      q[2] = static_cast<T>(w * (static_cast<double>(v.y) - vb1));
      q[3] = static_cast<T>(w * (static_cast<double>(v.z) - vb2));
    } else {
      q[0] = static_cast<T>(a.w);
      q[1] = static_cast<T>(a.w) * static_cast<T>(v.x);
      q[2] = static_cast<T>(a.w) * static_cast<T>(v.y);
      q[3] = static_cast<T>(a.w) * static_cast<T>(v.z);
    }
    T qz[kNumFields][kTaps];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f)
#pragma unroll
      for (int j = 0; j < kTaps; ++j) qz[f][j] = q[f] * wz[j];
    const int base = (cx * E + cy) * E + cz;
#pragma unroll
    for (int jx = 0; jx < kTaps; ++jx) {
#pragma unroll
      for (int jy = 0; jy < kTaps; ++jy) {
        const T wxy = wx[jx] * wy[jy];
        T* row = acc + base + (jx * E + jy) * E;
#pragma unroll
        for (int f = 0; f < kNumFields; ++f)
#pragma unroll
          for (int jz = 0; jz < kTaps; ++jz) atomicAdd(row + f * VOL + jz, wxy * qz[f][jz]);
      }
    }
  }
  __syncthreads();
  const int n = kp.n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  for (int i = threadIdx.x; i < VOL; i += NT) {
    const int ez = i % E, ey = (i / E) % E, ex = i / (E * E);
    const int gx = (ox + ex - 2) & (n - 1);
    const int gy = (oy + ey - 2) & (n - 1);
    const int gz = (oz + ez - 2) & (n - 1);
    const int64_t gi = (static_cast<int64_t>(gx) * n + gy) * n + gz;
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) {
      const T val = acc[f * VOL + i];
      if (val != T(0)) atomicAdd(grid + f * n3 + gi, val);
    }
  }
}

KeyParams key_params(const Plan* p, const mps_catalog* c) {
  KeyParams kp;
  kp.scale = static_cast<double>(p->n) / c->box;
  kp.n = p->n;
  int ts = 0;
  while ((1 << ts) < p->tile) ++ts;
  kp.tshift = ts;
  kp.nt = p->n / p->tile;
  return kp;
}

int count_blocks(int64_t np) {
  int64_t b = (np + kCountThreads - 1) / kCountThreads;
  return static_cast<int>(b < kMomentBlocks ? (b < 1 ? 1 : b) : kMomentBlocks);
}

}  // namespace

hipError_t launch_count(Plan* p, const mps_catalog* c, hipStream_t s) {
  const KeyParams kp = key_params(p, c);
  // zero-fill kernels rather than memset nodes, so that the sequence can be
  // captured in a HIP graph
  clear_kernel<uint32_t><<<static_cast<unsigned>((p->n_tiles + 255) / 256 < 4096 ? (p->n_tiles + 255) / 256 : 4096),
                           256, 0, s>>>(p->tile_count, p->n_tiles);
  clear_kernel<uint32_t><<<1, 256, 0, s>>>(reinterpret_cast<uint32_t*>(p->d_header),
                                           static_cast<int64_t>(sizeof(ResultHeader) / sizeof(uint32_t)));
  const int nb = kMomentBlocks;  // fixed grid: the moment sums keep one order
  if (c->weight)
    count_kernel<true><<<nb, kCountThreads, 0, s>>>(c->pos, c->vel, c->weight, c->n_particles, kp,
                                                   p->tile_count, p->moment_partials, p->d_header);
  else
    count_kernel<false><<<nb, kCountThreads, 0, s>>>(c->pos, c->vel, nullptr, c->n_particles, kp,
                                                    p->tile_count, p->moment_partials, p->d_header);
  return hipGetLastError();
}

hipError_t launch_derive(Plan* p, const mps_catalog* c, hipStream_t s) {
  derive_kernel<<<1, 64, 0, s>>>(p->moment_partials, kMomentBlocks, p->d_header,
                                 (c->flags & MPS_BULKFLOW_SUBTRACT) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_scan(Plan* p, hipStream_t s) {
  scan_kernel<<<1, 1024, 0, s>>>(p->tile_count, p->n_tiles, p->tile_offset, p->tile_cursor);
  return hipGetLastError();
}

hipError_t launch_permute(Plan* p, const mps_catalog* c, hipStream_t s) {
  const KeyParams kp = key_params(p, c);
  const int nb = count_blocks(c->n_particles);
  if (c->weight)
    permute_kernel<true><<<nb, kCountThreads, 0, s>>>(c->pos, c->vel, c->weight, c->n_particles, kp,
                                                     p->tile_cursor, p->sorted);
  else
    permute_kernel<false><<<nb, kCountThreads, 0, s>>>(c->pos, c->vel, nullptr, c->n_particles, kp,
                                                      p->tile_cursor, p->sorted);
  return hipGetLastError();
}

hipError_t launch_clear_grid(Plan* p, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(kNumFields) * p->n * p->n * p->n;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (p->prec == MPS_F32)
    clear_kernel<float><<<static_cast<int>(blocks), 256, 0, s>>>(static_cast<float*>(p->grid), n);
  else
    clear_kernel<double><<<static_cast<int>(blocks), 256, 0, s>>>(static_cast<double*>(p->grid), n);
  return hipGetLastError();
}

// bulk: 1 = deposit w (v - v_b) (only the assign diagnostic asks for it; the
// estimator removes the bulk flow in Fourier space, p' = p - v_b delta).
hipError_t launch_scatter_impl(Plan* p, const mps_catalog* c, hipStream_t s, int bulk) {
  const KeyParams kp = key_params(p, c);
  const int64_t xcd_chunk = (p->n_tiles % 8 == 0) ? p->n_tiles / 8 : 0;
  Derived* dsrc = &p->d_header->d;
  const unsigned grid = static_cast<unsigned>(p->n_tiles);
  if (p->prec == MPS_F32) {
    if (p->tile == 16)
      scatter_kernel<float, 16, 1024><<<grid, 1024, 0, s>>>(p->sorted, p->tile_offset,
                                                              static_cast<float*>(p->grid), kp, p->n_tiles,
                                                              xcd_chunk, p->taps, dsrc, bulk);
    else
      scatter_kernel<float, 8, 512><<<grid, 512, 0, s>>>(p->sorted, p->tile_offset,
                                                          static_cast<float*>(p->grid), kp, p->n_tiles,
                                                          xcd_chunk, p->taps, dsrc, bulk);
  } else {
    scatter_kernel<double, 8, 512><<<grid, 512, 0, s>>>(p->sorted, p->tile_offset,
                                                         static_cast<double*>(p->grid), kp, p->n_tiles,
                                                         xcd_chunk, p->taps, dsrc, bulk);
  }
  return hipGetLastError();
}

hipError_t launch_scatter(Plan* p, const mps_catalog* c, hipStream_t s) {
  return launch_scatter_impl(p, c, s, 0);
}

}  // namespace mps
