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

#include <type_traits>

#include "common.h"

namespace mps {
namespace {

constexpr int kCountThreads = 256;
// The FP32 scatter forms (see ScatterForm): the owner-computes kernel's
// threads per workgroup, and the largest mean numbers of particles per 16^3
// tile for which the owner-computes and the halo forms are taken.
constexpr int kGatherThreads = 512;
constexpr int64_t kGatherMaxMean = MPS_SCATTER_GATHER_MAX_MEAN;
constexpr int64_t kHaloMaxMean = MPS_SCATTER_HALO_MAX_MEAN;
constexpr int64_t kGather64MaxMean = MPS_SCATTER_GATHER64_MAX_MEAN;

// Grid coordinate of one float32 coordinate: u = x * (N / L) + shift in FP64
// (shift = 1/2 for the odd-order B-splines, whose taps are centred on the
// nearest node; 0 otherwise), cell floor(u) mod N, fraction f = u - floor(u).
// The same expression, without fused operations, decides the tile in the
// sort and the taps in the scatter.
__device__ __forceinline__ int locate(float x, double scale, double shift, int n, double* frac, bool* ok) {
#pragma clang fp contract(off)
  double u = static_cast<double>(x) * scale;
  u = u + shift;
  const bool fin = isfinite(u);
  if (!fin) u = 0.0;
  const double uf = floor(u);
  *frac = u - uf;
  // n is a power of two: uf * (1 / n) is exactly uf / n
  const double m = uf - static_cast<double>(n) * floor(uf * (1.0 / static_cast<double>(n)));
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

// wave_run_atomic split in two, so that several claims can be in flight:
// the run heads' atomics, then each lane's slot from its head's result.
struct WaveRun {
  uint32_t base;  // the head's atomic result (valid in head lanes)
  int start;      // lane of this lane's run head
};

__device__ __forceinline__ WaveRun wave_run_claim(uint32_t key, bool valid, uint32_t* counters) {
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(key, 1);
  const bool head = valid && (lane == 0 || key != prev);
  const unsigned long long heads = __ballot(head);
  const unsigned long long vmask = __ballot(valid);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long mine = heads & upto;
  WaveRun r;
  r.start = mine ? 63 - __clzll(static_cast<long long>(mine)) : lane;
  const unsigned long long after = (heads | ~vmask) & ~upto;
  const int end = after ? __ffsll(static_cast<long long>(after)) - 1 : 64;
  r.base = 0;
  if (head) r.base = atomicAdd(&counters[key], static_cast<uint32_t>(end - lane));
  return r;
}

__device__ __forceinline__ uint32_t wave_run_slot(const WaveRun& r) {
  const int lane = threadIdx.x & 63;
  return __shfl(r.base, r.start) + static_cast<uint32_t>(lane - r.start);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}


__device__ __forceinline__ uint32_t tile_key(float x, float y, float z, const KeyParams& kp, bool* ok) {
  double f;
  bool a, b, c;
  const int cx = locate(x, kp.scale, kp.shift, kp.n, &f, &a);
  const int cy = locate(y, kp.scale, kp.shift, kp.n, &f, &b);
  const int cz = locate(z, kp.scale, kp.shift, kp.n, &f, &c);
  *ok = a && b && c;
  return static_cast<uint32_t>(((cx >> kp.tshift) * kp.nt + (cy >> kp.tshift)) * kp.nt + (cz >> kp.tshift));
}

// Moments (FP64) and tile histogram in one pass over the catalog.  Each
// thread takes kUnroll consecutive particles per step and issues all their
// loads first.
constexpr int kUnroll = 4;

// Tile histograms: with at most kLdsTiles tiles each workgroup counts in
// LDS and adds its non-zero counts to the global histogram once at the end,
// so that catalogs in random order over few tiles do not serialise on a few
// global counters; larger grids count with wave-aggregated global atomics.
// Up to kLdsTilesRandom tiles (a 512^3 grid of 16^3 tiles) a catalog in
// random order still takes the LDS histograms (128 KB, one workgroup per
// CU), since one global atomic per particle would bound the sort; a catalog
// in spatial order, whose waves hold long runs of one tile, keeps the
// global form, which runs at full occupancy.  order_probe_kernel decides on
// the device, and the count and permute launch both forms, of which one
// returns at once.
constexpr int kLdsTiles = 16384;
constexpr int kLdsTilesRandom = 32768;
constexpr int kProbeChunks = 64;  // chunks of kCountThreads consecutive particles sampled

// A catalog is in random order when at most a quarter of its sampled
// neighbouring pairs fall in one tile.
__device__ __forceinline__ bool random_order(const ResultHeader* hdr) {
  return 4ull * hdr->order_same <= static_cast<unsigned long long>(hdr->order_pairs);
}

// Catalog records of particles i0 .. i0+kUnroll-1 (one lane's group): with
// 16-byte aligned arrays and a whole group, three 16-byte loads per array
// (12 floats = 4 particles' xyz) instead of twelve 4-byte ones.  Missing
// particles read as (0, 0, 0), velocity 0, weight 1.
template <bool kHasW>
__device__ __forceinline__ void load_group(const float* __restrict__ pos, const float* __restrict__ vel,
                                           const float* __restrict__ wgt, int64_t np, int64_t i0, bool vec,
                                           float4 (&a)[kUnroll], float4 (&v)[kUnroll]) {
  static_assert(kUnroll == 4, "one group is four particles");
  if (vec && i0 + kUnroll <= np) {
    const float4* p4 = reinterpret_cast<const float4*>(pos + 3 * i0);
    const float4* v4 = reinterpret_cast<const float4*>(vel + 3 * i0);
    const float4 p0 = p4[0], p1 = p4[1], p2 = p4[2];
    const float4 q0 = v4[0], q1 = v4[1], q2 = v4[2];
    float4 w = make_float4(1.f, 1.f, 1.f, 1.f);
    if (kHasW) w = *reinterpret_cast<const float4*>(wgt + i0);
    a[0] = make_float4(p0.x, p0.y, p0.z, w.x);
    a[1] = make_float4(p0.w, p1.x, p1.y, w.y);
    a[2] = make_float4(p1.z, p1.w, p2.x, w.z);
    a[3] = make_float4(p2.y, p2.z, p2.w, w.w);
    v[0] = make_float4(q0.x, q0.y, q0.z, 0.f);
    v[1] = make_float4(q0.w, q1.x, q1.y, 0.f);
    v[2] = make_float4(q1.z, q1.w, q2.x, 0.f);
    v[3] = make_float4(q2.y, q2.z, q2.w, 0.f);
    return;
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int64_t i = i0 + u;
    a[u] = make_float4(0.f, 0.f, 0.f, 1.f);
    v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < np) {
      a[u] = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], kHasW ? wgt[i] : 1.f);
      v[u] = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
    }
  }
}

// The sort's order probe: kProbeChunks chunks of kCountThreads consecutive
// particles spread over the catalog; counts the neighbouring pairs of a
// chunk and those whose two particles share a tile.
__global__ __launch_bounds__(kCountThreads) void order_probe_kernel(const float* __restrict__ pos, int64_t np,
                                                                   KeyParams kp, ResultHeader* hdr) {
  __shared__ uint32_t keys[kCountThreads];
  const int64_t span = np > kCountThreads ? np - kCountThreads : 0;
  const int64_t start = span * blockIdx.x / kProbeChunks;
  const int64_t i = start + threadIdx.x;
  bool ok;
  keys[threadIdx.x] = i < np ? tile_key(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], kp, &ok) : 0xffffffffu;
  __syncthreads();
  const bool pair = threadIdx.x > 0 && i < np;
  const bool same = pair && keys[threadIdx.x] == keys[threadIdx.x - 1];
  const unsigned long long sm = __ballot(same), pm = __ballot(pair);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&hdr->order_same, static_cast<uint32_t>(__popcll(sm)));
    atomicAdd(&hdr->order_pairs, static_cast<uint32_t>(__popcll(pm)));
  }
}

// order_mode: -1 runs always; 0 only for a catalog in spatial order, 1 only
// for one in random order (random_order()).  key_shift: the histogram counts
// tile >> key_shift (the two-level sort's buckets; n_tiles is then the
// number of buckets).
template <bool kHasW, bool kLds>
__global__ __launch_bounds__(kCountThreads) void count_kernel(
    const float* __restrict__ pos, const float* __restrict__ vel, const float* __restrict__ wgt,
    int64_t np, KeyParams kp, int64_t n_tiles, uint32_t* __restrict__ tile_count,
    double* __restrict__ partials, ResultHeader* hdr, bool vec, int order_mode, int key_shift) {
  extern __shared__ uint32_t hist[];  // n_tiles counters when kLds
  if (order_mode >= 0 && random_order(hdr) != (order_mode == 1)) return;  // uniform
  if (kLds) {
    for (int64_t i = threadIdx.x; i < n_tiles; i += kCountThreads) hist[i] = 0u;
    __syncthreads();
  }
  uint32_t* counts = kLds ? hist : tile_count;
  double acc[kMomentSums];
#pragma unroll
  for (int q = 0; q < kMomentSums; ++q) acc[q] = 0.0;
  double mx[kMomentMax] = {0.0, 0.0, 0.0, 0.0};
  bool bad = false;
  // each lane takes a group of kUnroll consecutive particles per step; for a
  // given u the wave's lanes hold particles 4 apart, still in input order
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCountThreads * kUnroll;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kCountThreads * kUnroll; base < np; base += stride) {
    const int64_t i0 = base + static_cast<int64_t>(threadIdx.x) * kUnroll;
    float4 a[kUnroll], v[kUnroll];
    load_group<kHasW>(pos, vel, wgt, np, i0, vec, a, v);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool valid = i0 + u < np;
      uint32_t key = 0xffffffffu;
      if (valid) {
        bool ok;
        key = tile_key(a[u].x, a[u].y, a[u].z, kp, &ok);
        bad |= !ok;
        const double w = a[u].w;
        const double dvx = v[u].x, dvy = v[u].y, dvz = v[u].z;
        const double w2 = w * w;
        acc[0] += w;
        acc[1] += w2;
        acc[2] += w * dvx;
        acc[3] += w * dvy;
        acc[4] += w * dvz;
        acc[5] += w2 * dvx;
        acc[6] += w2 * dvy;
        acc[7] += w2 * dvz;
        acc[8] += w2 * dvx * dvx;
        acc[9] += w2 * dvy * dvy;
        acc[10] += w2 * dvz * dvz;
        acc[11] += w2 * dvx * dvy;
        acc[12] += w2 * dvx * dvz;
        acc[13] += w2 * dvy * dvz;
        mx[0] = fmax(mx[0], fabs(w));
        mx[1] = fmax(mx[1], fabs(w * dvx));
        mx[2] = fmax(mx[2], fabs(w * dvy));
        mx[3] = fmax(mx[3], fabs(w * dvz));
      }
      wave_run_atomic(valid ? key >> key_shift : key, valid, counts);
    }
  }
  if (kLds) {
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n_tiles; i += kCountThreads)
      if (hist[i]) atomicAdd(tile_count + i, hist[i]);
  }
  __shared__ double red[kCountThreads / 64][kMomentSums + kMomentMax];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < kMomentSums; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = s;
  }
#pragma unroll
  for (int q = 0; q < kMomentMax; ++q) {
    double m = mx[q];
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) red[wave][kMomentSums + q] = m;
  }
  __syncthreads();
  if (threadIdx.x < kMomentSums) {
    double s = 0.0;
    for (int w = 0; w < kCountThreads / 64; ++w) s += red[w][threadIdx.x];
    partials[blockIdx.x * kMomentSums + threadIdx.x] = s;
  } else if (threadIdx.x < kMomentSums + kMomentMax) {
    const int q = threadIdx.x - kMomentSums;
    double m = 0.0;
    for (int w = 0; w < kCountThreads / 64; ++w) m = fmax(m, red[w][threadIdx.x]);
    partials[kMomentBlocks * kMomentSums + blockIdx.x * kMomentMax + q] = m;
  }
  if (bad) atomicOr(&hdr->flags, 1u);
}

// Fixed-order sum of the per-block moment partials, then the derived shot
// and bulk-flow scalars.  One workgroup of kMomentBlocks threads: thread b
// holds block b's partials (zero beyond the nb blocks the count ran) and a
// fixed reduction tree combines them.
__device__ __forceinline__ void derive_block(const double* __restrict__ partials, int nb, ResultHeader* hdr,
                                             int bulk) {
  constexpr int kW = kMomentBlocks / 64;
  __shared__ double red[kW][kMomentSums + kMomentMax];
  __shared__ double sums[kMomentSums];
  __shared__ double maxes[kMomentMax];
  const int b = threadIdx.x, wave = b >> 6, lane = b & 63;
#pragma unroll
  for (int q = 0; q < kMomentSums; ++q) {
    const double v = wave_sum(b < nb ? partials[b * kMomentSums + q] : 0.0);
    if (lane == 0) red[wave][q] = v;
  }
#pragma unroll
  for (int q = 0; q < kMomentMax; ++q) {
    double m = b < nb ? partials[kMomentBlocks * kMomentSums + b * kMomentMax + q] : 0.0;
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) red[wave][kMomentSums + q] = m;
  }
  __syncthreads();
  if (b < kMomentSums) {
    double v = 0.0;
    for (int w = 0; w < kW; ++w) v += red[w][b];
    sums[b] = v;
    hdr->sums[b] = v;
  } else if (b < kMomentSums + kMomentMax) {
    double m = 0.0;
    for (int w = 0; w < kW; ++w) m = fmax(m, red[w][b]);
    maxes[b - kMomentSums] = m;
  }
  __syncthreads();
  if (b != 0) return;
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
  // sum w^2 (v - v_b) = sum w^2 v - v_b W2
  for (int a = 0; a < 3; ++a) {
    d.sp[a] = (sums[5 + a] - d.vb[a] * d.W2) * iw2;
    d.s[a] = bulk ? d.sp[a] : sums[5 + a] * iw2;
  }
  d.s_pp = d.S[0] + d.S[1] + d.S[2];
  d.inv_W = iw;
  d.sigma_v2 = (m2[0] + m2[1] + m2[2]) / d.W2;
  for (int q = 0; q < kMomentMax; ++q) d.qmax[q] = maxes[q];
  d.bulk = bulk;
  hdr->d = d;
}

__global__ __launch_bounds__(kMomentBlocks) void derive_kernel(const double* __restrict__ partials, int nb,
                                                               ResultHeader* hdr, int bulk) {
  derive_block(partials, nb, hdr, bulk);
}

// Exclusive scan of the tile counts (one workgroup); also resets the cursor.
__device__ __forceinline__ void scan_block(const uint32_t* __restrict__ count, int64_t n_tiles,
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

__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t* __restrict__ count, int64_t n_tiles,
                                                    uint32_t* __restrict__ offset, uint32_t* __restrict__ cursor,
                                                    const ResultHeader* __restrict__ hdr, int order_mode) {
  if (order_mode >= 0 && random_order(hdr) != (order_mode == 1)) return;  // uniform
  scan_block(count, n_tiles, offset, cursor);
}

// The two one-workgroup stages after the count in one launch (the one-level
// sort): the moments' derivation, then the scan of the tile counts.  They
// read and write disjoint data.
static_assert(kMomentBlocks == 1024, "derive and scan share the workgroup");
__global__ __launch_bounds__(1024) void derive_scan_kernel(const double* __restrict__ partials, int nb,
                                                           ResultHeader* hdr, int bulk,
                                                           const uint32_t* __restrict__ count, int64_t n_tiles,
                                                           uint32_t* __restrict__ offset,
                                                           uint32_t* __restrict__ cursor) {
  derive_block(partials, nb, hdr, bulk);
  scan_block(count, n_tiles, offset, cursor);
}

// Zeroes, in one launch, the grid (nc reals, stored as clear_kernel does)
// and two word ranges (the tile counters and the result header).
template <typename T>
__global__ __launch_bounds__(256) void clear3_kernel(uint32_t* __restrict__ a, int64_t na, uint32_t* __restrict__ b,
                                                     int64_t nb, T* __restrict__ c, int64_t nc) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  for (int64_t i = t0; i < nc; i += stride) c[i] = T(0);
  for (int64_t i = t0; i < na; i += stride) a[i] = 0u;
  for (int64_t i = t0; i < nb; i += stride) b[i] = 0u;
}

// Sorted particle records.  A catalog with weights stores (x, y, z, w) and
// (v_x, v_y, v_z, 0) as two float4 (32 bytes); a catalog without stores
// (x, y, z, v_x, v_y, v_z) in 24 bytes as three float2 and reads back w = 1,
// a quarter less traffic for the permute's writes and the scatter's reads.
template <bool kW>
__device__ __forceinline__ float4 rec_pos(const float4* __restrict__ s, int64_t p) {
  if constexpr (kW) {
    return s[2 * p];
  } else {
    const float2* r = reinterpret_cast<const float2*>(s) + 3 * p;
    const float2 a = r[0], b = r[1];
    return make_float4(a.x, a.y, b.x, 1.f);
  }
}

template <bool kW>
__device__ __forceinline__ float4 rec_vel(const float4* __restrict__ s, int64_t p) {
  if constexpr (kW) {
    return s[2 * p + 1];
  } else {
    const float2* r = reinterpret_cast<const float2*>(s) + 3 * p;
    const float2 b = r[1], c = r[2];
    return make_float4(b.y, c.x, c.y, 0.f);
  }
}

template <bool kW>
__device__ __forceinline__ void rec_store(float4* __restrict__ s, int64_t p, const float4& a, const float4& v) {
  if constexpr (kW) {
    s[2 * p] = a;
    s[2 * p + 1] = v;
  } else {
    float2* r = reinterpret_cast<float2*>(s) + 3 * p;
    r[0] = make_float2(a.x, a.y);
    r[1] = make_float2(a.z, v.x);
    r[2] = make_float2(v.y, v.z);
  }
}

// Counting-sort scatter of the particle records into tile order (record
// layout above).  With at most kLdsTiles tiles a
// workgroup first counts its own particles per tile in LDS, reserves one
// contiguous range per tile with a single global atomic, and then hands out
// slots from LDS; otherwise every wave claims slots with global atomics.
template <bool kHasW, bool kLds>
__global__ __launch_bounds__(kCountThreads) void permute_kernel(
    const float* __restrict__ pos, const float* __restrict__ vel, const float* __restrict__ wgt,
    int64_t np, KeyParams kp, int64_t n_tiles, uint32_t* __restrict__ cursor, float4* __restrict__ sorted,
    bool vec, const ResultHeader* __restrict__ hdr, int order_mode) {
  extern __shared__ uint32_t hist[];  // n_tiles counters when kLds
  if (order_mode >= 0 && random_order(hdr) != (order_mode == 1)) return;  // uniform
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kCountThreads * kUnroll;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kCountThreads * kUnroll;
  if (kLds) {
    for (int64_t i = threadIdx.x; i < n_tiles; i += kCountThreads) hist[i] = 0u;
    __syncthreads();
    for (int64_t base = first; base < np; base += stride) {
      const int64_t i0 = base + static_cast<int64_t>(threadIdx.x) * kUnroll;
      float4 a[kUnroll], v[kUnroll];
      load_group<false>(pos, vel, nullptr, np, i0, vec, a, v);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const bool valid = i0 + u < np;
        uint32_t key = 0xffffffffu;
        if (valid) {
          bool ok;
          key = tile_key(a[u].x, a[u].y, a[u].z, kp, &ok);
        }
        wave_run_atomic(key, valid, hist);
      }
    }
    __syncthreads();
    // reserve this workgroup's ranges; hist[t] becomes the next free slot
    for (int64_t t = threadIdx.x; t < n_tiles; t += kCountThreads)
      if (hist[t]) hist[t] = atomicAdd(cursor + t, hist[t]);
    __syncthreads();
  }
  uint32_t* slots = kLds ? hist : cursor;
  // one particle per lane per slab here (not the count's groups of four):
  // consecutive lanes then write consecutive slots of a tile, so a wave's
  // records go out in a few long runs
  for (int64_t base = first; base < np; base += stride) {
    float4 a[kUnroll], v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * kCountThreads + threadIdx.x;
      a[u] = make_float4(0.f, 0.f, 0.f, 1.f);
      v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i < np) {
        a[u] = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], kHasW ? wgt[i] : 1.f);
        v[u] = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
      }
    }
    // all slots are claimed before any record is written, so the returning
    // atomics of the kUnroll slabs overlap
    WaveRun run[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * kCountThreads + threadIdx.x;
      const bool valid = i < np;
      uint32_t key = 0xffffffffu;
      if (valid) {
        bool ok;
        key = tile_key(a[u].x, a[u].y, a[u].z, kp, &ok);
      }
      run[u] = wave_run_claim(key, valid, slots);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + u * kCountThreads + threadIdx.x;
      const uint32_t slot = wave_run_slot(run[u]);
      if (i < np) {
        rec_store<kHasW>(sorted, static_cast<int64_t>(slot), a[u], v[u]);
      }
    }
  }
}

// Two-level counting sort of a catalog in random order on grids whose tile
// histogram does not fit in LDS, where one global atomic per particle would
// bound the count (1024^3, 5e8 particles: 18.5 ms against 2.2 with bucket
// histograms).  The tiles form kSortBuckets or fewer buckets of
// consecutive tiles; the count histograms buckets, pass A moves the records
// bucket by bucket to a temporary array (the grid's memory, unused until
// the scatter), and pass B, one workgroup per bucket, counts its tiles,
// writes their offsets and moves the records to their tiles.  Both passes
// sort chunks of kSortChunk particles in LDS first, so that the records of
// one bucket (tile) leave a chunk as one contiguous run.
constexpr int kSortThreads = 512;
constexpr int kSortChunk = 8192;
constexpr int kSortBuckets = 1024;  // also the largest number of tiles per bucket
static_assert(kSortChunk <= 65536, "local indices are 16-bit");

// Exclusive prefix sums of a[0..n) in LDS (n <= 2 kSortThreads), in place;
// returns the total to every thread.  Ends with a barrier.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t* a, int n, uint32_t* wsum) {
  constexpr int kWaves = kSortThreads / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t v0 = 2 * t < n ? a[2 * t] : 0u, v1 = 2 * t + 1 < n ? a[2 * t + 1] : 0u;
  uint32_t incl = v0 + v1;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < kWaves; ++w) {
    before += w < wave ? wsum[w] : 0u;
    total += wsum[w];
  }
  const uint32_t excl = before + incl - (v0 + v1);
  if (2 * t < n) a[2 * t] = excl;
  if (2 * t + 1 < n) a[2 * t + 1] = excl + v0;
  __syncthreads();
  return total;
}

// A catalog particle's record fields (w = 1 without weights).
template <bool kHasW>
__device__ __forceinline__ void catalog_record(const float* __restrict__ pos, const float* __restrict__ vel,
                                               const float* __restrict__ wgt, int64_t i, float4* a, float4* v) {
  *a = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], kHasW ? wgt[i] : 1.f);
  *v = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
}

// Pass A: the catalog's particles to `temp`, grouped by bucket (tile >>
// shift); bucket_cur[b] starts at bucket b's first slot.
template <bool kHasW>
__global__ __launch_bounds__(kSortThreads) void sort_pass_a_kernel(
    const float* __restrict__ pos, const float* __restrict__ vel, const float* __restrict__ wgt, int64_t np,
    KeyParams kp, int shift, int n_buckets, uint32_t* __restrict__ bucket_cur, float4* __restrict__ temp,
    const ResultHeader* __restrict__ hdr) {
  constexpr int NT = kSortThreads, K = kSortChunk, PER = K / NT;
  __shared__ uint32_t lstart[kSortBuckets];
  __shared__ uint32_t gbase[kSortBuckets];
  __shared__ unsigned short bkey[K], rank[K], perm[K];
  __shared__ uint32_t wsum[NT / 64];
  if (!random_order(hdr)) return;  // uniform: the one-level sort runs instead
  const int t = threadIdx.x;
  for (int64_t c0 = static_cast<int64_t>(blockIdx.x) * K; c0 < np; c0 += static_cast<int64_t>(gridDim.x) * K) {
    const int m = static_cast<int>(np - c0 < K ? np - c0 : K);
    for (int b = t; b < n_buckets; b += NT) lstart[b] = 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int li = t + r * NT;
      if (li < m) {
        const int64_t i = c0 + li;
        bool ok;
        const uint32_t b = tile_key(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], kp, &ok) >> shift;
        bkey[li] = static_cast<unsigned short>(b);
        rank[li] = static_cast<unsigned short>(atomicAdd(&lstart[b], 1u));
      }
    }
    __syncthreads();
    // one global reservation per bucket present in the chunk
    for (int b = t; b < n_buckets; b += NT)
      if (lstart[b]) gbase[b] = atomicAdd(bucket_cur + b, lstart[b]);
    (void)block_exclusive_scan(lstart, n_buckets, wsum);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int li = t + r * NT;
      if (li < m) perm[lstart[bkey[li]] + rank[li]] = static_cast<unsigned short>(li);
    }
    __syncthreads();
    // consecutive threads store consecutive slots of a bucket's run
    for (int j = t; j < m; j += NT) {
      const int li = perm[j];
      const uint32_t b = bkey[li];
      float4 a, v;
      catalog_record<kHasW>(pos, vel, wgt, c0 + li, &a, &v);
      rec_store<kHasW>(temp, static_cast<int64_t>(gbase[b]) + (j - static_cast<int>(lstart[b])), a, v);
    }
    __syncthreads();
  }
}

// Pass B: workgroup b sorts bucket b (temp[bucket_start[b] ..
// bucket_start[b + 1])) by tile into `sorted` and writes its tiles' offsets
// (the last bucket also offset[n_tiles]).
template <bool kHasW>
__global__ __launch_bounds__(kSortThreads) void sort_pass_b_kernel(
    const float4* __restrict__ temp, const uint32_t* __restrict__ bucket_start, KeyParams kp, int shift,
    int n_buckets, int64_t n_tiles, uint32_t* __restrict__ tile_offset, float4* __restrict__ sorted,
    const ResultHeader* __restrict__ hdr) {
  constexpr int NT = kSortThreads, K = kSortChunk, PER = K / NT;
  __shared__ uint32_t tcur[kSortBuckets];    // next free slot of each tile of the bucket
  __shared__ uint32_t lstart[kSortBuckets];  // chunk counts, then starts
  __shared__ uint32_t gbase[kSortBuckets];
  __shared__ unsigned short tkey[K], rank[K], perm[K];
  __shared__ uint32_t wsum[NT / 64];
  if (!random_order(hdr)) return;  // uniform
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  const int tiles = 1 << shift;
  const uint32_t tile0 = static_cast<uint32_t>(b) << shift;
  const uint32_t start = bucket_start[b], end = bucket_start[b + 1];
  auto local_tile = [&](int64_t rec) -> uint32_t {
    const float4 a = rec_pos<kHasW>(temp, rec);
    bool ok;
    return tile_key(a.x, a.y, a.z, kp, &ok) - tile0;
  };
  // the bucket's tile counts and offsets
  for (int k = t; k < tiles; k += NT) tcur[k] = 0u;
  __syncthreads();
  for (uint32_t i = start + t; i < end; i += NT) atomicAdd(&tcur[local_tile(i)], 1u);
  __syncthreads();
  (void)block_exclusive_scan(tcur, tiles, wsum);
  for (int k = t; k < tiles; k += NT) {
    tcur[k] += start;
    tile_offset[tile0 + k] = tcur[k];
  }
  if (b == n_buckets - 1 && t == 0) tile_offset[n_tiles] = end;
  __syncthreads();
  for (uint32_t c0 = start; c0 < end; c0 += K) {
    const int m = static_cast<int>(end - c0 < static_cast<uint32_t>(K) ? end - c0 : K);
    for (int k = t; k < tiles; k += NT) lstart[k] = 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int li = t + r * NT;
      if (li < m) {
        const uint32_t lt = local_tile(c0 + li);
        tkey[li] = static_cast<unsigned short>(lt);
        rank[li] = static_cast<unsigned short>(atomicAdd(&lstart[lt], 1u));
      }
    }
    __syncthreads();
    for (int k = t; k < tiles; k += NT) {  // this workgroup owns the bucket: no global atomics
      gbase[k] = tcur[k];
      tcur[k] += lstart[k];
    }
    (void)block_exclusive_scan(lstart, tiles, wsum);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int li = t + r * NT;
      if (li < m) perm[lstart[tkey[li]] + rank[li]] = static_cast<unsigned short>(li);
    }
    __syncthreads();
    for (int j = t; j < m; j += NT) {
      const int li = perm[j];
      const uint32_t lt = tkey[li];
      const int64_t src = static_cast<int64_t>(c0) + li;
      rec_store<kHasW>(sorted, static_cast<int64_t>(gbase[lt]) + (j - static_cast<int>(lstart[lt])),
                       rec_pos<kHasW>(temp, src), rec_vel<kHasW>(temp, src));
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void clear_kernel(T* __restrict__ g, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) g[i] = T(0);
}

// w_j(f): one polynomial of degree DEG, or (DEG == kDegSplit2) the
// quadratic-spline BL3 reading's two quadratics, c[j][0..2] for f < 1/2 and
// c[j][3..5] for f >= 1/2.
template <int DEG>
__device__ __forceinline__ double tap_weight(const TapPoly& tp, int j, double f) {
  if constexpr (DEG == kDegSplit2) {
    const bool upper = f >= 0.5;
    const double c0 = upper ? tp.c[j][3] : tp.c[j][0];
    const double c1 = upper ? tp.c[j][4] : tp.c[j][1];
    const double c2 = upper ? tp.c[j][5] : tp.c[j][2];
    return (c2 * f + c1) * f + c0;
  } else {
    double v = tp.c[j][DEG];
#pragma unroll
    for (int q = DEG - 1; q >= 0; --q) v = v * f + tp.c[j][q];
    return v;
  }
}

template <typename T>
struct DepositQ {
  T q[kNumFields];
};

// Charges (w, w v_x, w v_y, w v_z) of one particle record; bulk = 1 deposits
// w (v - v_b) instead (the assign diagnostic's bulk-flow grids).
template <typename T>
__device__ __forceinline__ DepositQ<T> charges(const float4& a, const float4& v, int bulk, double vb0,
                                               double vb1, double vb2) {
  DepositQ<T> d;
  if (bulk) {
    const double w = a.w;
    d.q[0] = static_cast<T>(w);
    d.q[1] = static_cast<T>(w * (static_cast<double>(v.x) - vb0));
    d.q[2] = static_cast<T>(w * (static_cast<double>(v.y) - vb1));
    d.q[3] = static_cast<T>(w * (static_cast<double>(v.z) - vb2));
  } else {
    d.q[0] = static_cast<T>(a.w);
    d.q[1] = static_cast<T>(a.w) * static_cast<T>(v.x);
    d.q[2] = static_cast<T>(a.w) * static_cast<T>(v.y);
    d.q[3] = static_cast<T>(a.w) * static_cast<T>(v.z);
  }
  return d;
}

// Kernels with NTAP taps per axis whose weights are polynomials of degree
// DEG in the fraction: the truncated BL3 function (6 taps, j = -2..3, cubic)
// or the B-spline of order NTAP (taps j = -(NTAP-1)/2 .. NTAP/2, degree
// NTAP - 1; for odd orders relative to the nearest node).  The LDS block is
// the tile plus a halo of kHaloLo cells below and NTAP - 1 - kHaloLo above.
template <int NTAP>
constexpr int kHaloLo = (NTAP - 1) / 2;

// Tap weights and the particle's cell relative to the tile origin.
template <typename T, int TS, int NTAP, int DEG>
__device__ __forceinline__ unsigned particle_taps(const float4& a, const KeyParams& kp, int ox, int oy, int oz,
                                                  const TapPoly& tp, T* wx, T* wy, T* wz) {
  constexpr int E = TS + NTAP - 1;
  double fx, fy, fz;
  bool ok;
  int cx = locate(a.x, kp.scale, kp.shift, kp.n, &fx, &ok) - ox;
  int cy = locate(a.y, kp.scale, kp.shift, kp.n, &fy, &ok) - oy;
  int cz = locate(a.z, kp.scale, kp.shift, kp.n, &fz, &ok) - oz;
  // the sort placed the particle in this tile with the same locate(); the
  // clamp only keeps LDS indices in range
  cx = min(max(cx, 0), TS - 1);
  cy = min(max(cy, 0), TS - 1);
  cz = min(max(cz, 0), TS - 1);
#pragma unroll
  for (int j = 0; j < NTAP; ++j) {
    wx[j] = static_cast<T>(tap_weight<DEG>(tp, j, fx));
    wy[j] = static_cast<T>(tap_weight<DEG>(tp, j, fy));
    wz[j] = static_cast<T>(tap_weight<DEG>(tp, j, fz));
  }
  return static_cast<unsigned>((cx * E + cy) * E + cz);
}

__device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t xcd_chunk) {
  // consecutive tiles (spatial neighbours, which share halo cache lines) go
  // to one XCD: workgroups are dealt to the 8 XCDs round robin
  return xcd_chunk > 0 ? (b & 7) * xcd_chunk + (b >> 3) : b;
}

// Nearest integer of an FP32 value with |x| < 2^31 in one instruction:
// v_cvt_rpi_i32_f32 returns floor(x + 0.5).
__device__ __forceinline__ int round_to_int(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Two int32 deposits (lo, hi) as the int64 hi 2^32 + lo, added with one
// 64-bit LDS atomic.  The 64-bit sum is hi_sum 2^32 + lo_sum modulo 2^64:
// as long as the final lo_sum fits int32, its low word is lo_sum and the high
// word, corrected for lo_sum's sign, is hi_sum modulo 2^32.

// The pair (round(wlo wz), round(whi wz)) packed as above in five VALU
// operations: lo < 0 exactly when x = wlo wz < -1/2, and the indicator
// clamp(-2^40 (x + 1/2)) to [0, 1] is exactly 0 or 1 for every FP32 x (the
// FP32 values below -1/2 lie at least 2^-25 below it), so the sign correction
// folds into the high product as round(whi wz - [lo < 0]).  That rounds the
// exact product once; it may differ from rounding the FP32 product by one
// unit, or by one FP32 spacing where that exceeds a unit, and the 64-bit sum
// remains exact.
__device__ __forceinline__ unsigned long long deposit_pair(float wlo, float whi, float wz) {
  const float x = wlo * wz;
  const int lo = round_to_int(x);
  const float neg = __builtin_amdgcn_fmed3f(fmaf(x, -0x1p40f, -0x1p39f), 0.f, 1.f);
  const int hi = round_to_int(fmaf(whi, wz, -neg));
  return (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo);
}

__device__ __forceinline__ void unpack_pair(unsigned long long s, int* lo, int* hi) {
  *lo = static_cast<int>(static_cast<unsigned>(s));
  *hi = static_cast<int>(static_cast<unsigned>(s >> 32) + (*lo < 0 ? 1u : 0u));
}

// Two particles' deposits into one cell, packed as deposit_pair: the low and
// high words round wlo_a wz_a + wlo_b wz_b and whi_a wz_a + whi_b wz_b (each
// an FP32 fused sum) once; the sign indicator is that of the low word.
__device__ __forceinline__ unsigned long long deposit_pair2(float alo, float ahi, float wa, float blo, float bhi,
                                                            float wb) {
  const float x = fmaf(blo, wb, alo * wa);
  const int lo = round_to_int(x);
  const float neg = __builtin_amdgcn_fmed3f(fmaf(x, -0x1p40f, -0x1p39f), 0.f, 1.f);
  const int hi = round_to_int(fmaf(ahi, wa, fmaf(bhi, wb, -neg)));
  return (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo);
}

// Cell (x, y, z fastest) of a 16^3 tile holding a tap origin of its 21^3
// block (6 taps: the origin is 2 cells below the particle's cell).
__device__ __forceinline__ unsigned origin_cell(unsigned base) {
  constexpr unsigned E = 21;
  const unsigned cx = base / (E * E), cy = (base / E) % E, cz = base % E;
  return (cx * 16u + cy) * 16u + cz;
}

// cell | rank << 12: the rank is the particle's place among its cell's
// particles, from 16-bit counters packed two per word.
__device__ __forceinline__ unsigned cell_rank(unsigned base, unsigned* ccnt) {
  const unsigned cell = origin_cell(base);
  const unsigned sh = (cell & 1u) << 4;
  const unsigned rank = (atomicAdd(ccnt + (cell >> 1), 1u << sh) >> sh) & 0xffffu;
  return cell | rank << 12;
}

// LDS word index of a particle's tap origin (cell relative to the tile
// origin, halo offset included) without the tap weights.
template <int TS, int NTAP>
__device__ __forceinline__ unsigned tap_origin(const float4& a, const KeyParams& kp, int ox, int oy, int oz) {
  constexpr int E = TS + NTAP - 1;
  double f;
  bool ok;
  int cx = locate(a.x, kp.scale, kp.shift, kp.n, &f, &ok) - ox;
  int cy = locate(a.y, kp.scale, kp.shift, kp.n, &f, &ok) - oy;
  int cz = locate(a.z, kp.scale, kp.shift, kp.n, &f, &ok) - oz;
  cx = min(max(cx, 0), TS - 1);
  cy = min(max(cy, 0), TS - 1);
  cz = min(max(cz, 0), TS - 1);
  return static_cast<unsigned>((cx * E + cy) * E + cz);
}

// Lane assignment that spreads a wave over the LDS banks.  A super-chunk of
// up to kPer * NT particles is counting-sorted by the bank pair of its tap
// origin (64-bit element index mod 32: the 8-byte accumulators of both
// kernels span two 4-byte banks); with W = ceil(m/64) wave slots, lane l of
// slot s takes bank-sorted position l' W + s with l' = 2 (l mod 32) + l / 32,
// so that each half-wave draws one lane from each of 32 consecutive bank
// segments: one access per bank pair, two lanes on one address only when
// two particles share a cell.
template <int NT, int kPer>
struct BankSort {
  int cnt[64];
  unsigned short idx[NT * kPer];
};

// Threads first count their particles per bank pair (bs.cnt, taking slots
// with LDS atomics); this turns the counts into bucket starts, after which
// each particle's local index goes to bs.idx[start + slot].
template <int NT, int kPer>
__device__ __forceinline__ void bank_scan(BankSort<NT, kPer>& bs) {
  const int t = threadIdx.x;
  if (t < 64) {  // exclusive scan of 64 counters in one wave
    const int v = bs.cnt[t];
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off);
      if (t >= off) incl += o;
    }
    bs.cnt[t] = incl - v;
  }
}

// Index of block cell (ex, ey, ez) among the halo cells of a 16^3 tile's
// 21^3 block (2 cells below and 3 above the tile along each axis): the 5
// halo x planes, then within the tile's x range the 5 halo y rows, then
// within the tile's x and y range the 5 halo z cells.
__device__ __forceinline__ int halo_index(int ex, int ey, int ez) {
  constexpr int E = 21, H = 2, TS = 16, B = E - TS;
  auto band = [](int e) { return e < H ? e : e - TS; };
  if (ex < H || ex >= H + TS) return (band(ex) * E + ey) * E + ez;
  if (ey < H || ey >= H + TS) return B * E * E + ((ex - H) * B + band(ey)) * E + ez;
  return B * E * E + TS * B * E + ((ex - H) * TS + ey - H) * B + band(ez);
}

// The paired deposits' cell sort and job list of one dense tile of cnt
// particles (cnt <= kPairCap), shared by the FP32 and FP64 atomic scatters:
// on entry the 16-bit cell counts are in ccnt (the particles' cell | rank
// keys in key0 for t + r NT < m0, in words[2 E^3 + i] beyond) and the
// accumulator block, seen as words, is zero; on return the bank-sorted job
// list (a | b << 16 for a pair, a for a single; pairs first) is in pjob and
// the block is zero again.  Returns the number of pair jobs.  The bank
// counters bs.cnt are cleared here (they size the jobs' slots in pjob).
template <int NT, int kPer, int E>
__device__ __forceinline__ int pair_jobs(unsigned* words, unsigned* ccnt, unsigned* wsum, BankSort<NT, kPer>& bs,
                                         const unsigned (&key0)[kPer], int m0, uint32_t cnt,
                                         uint32_t* __restrict__ pjob) {
  constexpr int VOL = E * E * E;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  if (t < 64) bs.cnt[t] = 0;  // first read after the barriers below
  // exclusive scan of the 4096 cell counts (2 CW per thread) into cell starts
  {
    constexpr int CW = 2048 / NT;  // count words per thread
    static_assert(CW * NT == 2048, "the threads cover the 4096 counts");
    unsigned cw[CW];
    unsigned sum = 0;
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      cw[c] = ccnt[CW * t + c];
      sum += (cw[c] & 0xffffu) + (cw[c] >> 16);
    }
    unsigned incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    unsigned e = incl - sum;
    for (int w = 0; w < wave; ++w) e += wsum[w];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const unsigned lo = e, hi = e + (cw[c] & 0xffffu);
      e = hi + (cw[c] >> 16);
      ccnt[CW * t + c] = lo | hi << 16;
    }
  }
  __syncthreads();
  // The accumulators are zero here and the sort runs in them (words of
  // the u32 view; cnt <= 2 VOL): the cell-sorted entries (local index |
  // cell << 16) at 0.., the cell keys of particles kSuper.. and then
  // the job keys at 2 VOL..; both ranges are cleared again before the
  // deposits.
  unsigned* const fsorted = words;
  auto place = [&](unsigned key, unsigned i) {
    const unsigned cell = key & 4095u;
    fsorted[((ccnt[cell >> 1] >> ((cell & 1u) << 4)) & 0xffffu) + (key >> 12)] = i | cell << 16;
  };
#pragma unroll
  for (int r = 0; r < kPer; ++r)
    if (t + r * NT < m0) place(key0[r], static_cast<unsigned>(t + r * NT));
  for (uint32_t i = static_cast<uint32_t>(m0) + t; i < cnt; i += NT) place(words[2 * VOL + i], i);
  __syncthreads();
  // Jobs: along each run of sorted positions whose neighbours are linked
  // (cells equal or z-neighbours), positions pair greedily from the run's
  // start; the others are single jobs.  Each thread walks a contiguous
  // segment of positions, marking the link of i and i + 1 in bit 28 of
  // position i's entry and finding the segment's last run start; a block
  // max-scan gives each segment the run it begins in; a second walk writes
  // each job's bucket ((pair ? 0 : 32) + bank pair of the first particle's
  // tap origin) at its first position, ~0 at a pair's second; the slots
  // are claimed in a strided pass.
  constexpr unsigned kLink = 1u << 28;
  unsigned* const jkey = words + 2 * VOL;  // the job keys, by first position
  auto bank_of = [&](unsigned cell) {
    return (((cell >> 8) * E + ((cell >> 4) & 15u)) * E + (cell & 15u)) & 31u;
  };
  auto linkable = [&](unsigned e0, unsigned e1) {
    const unsigned c0 = (e0 >> 16) & 4095u, c1 = (e1 >> 16) & 4095u;
    return c1 == c0 || (c1 == c0 + 1u && (c0 & 15u) != 15u);
  };
  const int per = (static_cast<int>(cnt) + NT - 1) / NT;
  const int s0 = min(t * per, static_cast<int>(cnt)), s1 = min(s0 + per, static_cast<int>(cnt));
  // the segment's links (bit 28) and its last run start; whether s0 - 1
  // links to s0 is kept for the second walk
  const bool link_in = s0 > 0 && s0 < s1 && linkable(fsorted[s0 - 1], fsorted[s0]);
  int last = -1;
  {
    bool prev = link_in;
    for (int i = s0; i < s1; ++i) {
      if (!prev) last = i;
      const unsigned e0 = fsorted[i];
      prev = i + 1 < static_cast<int>(cnt) && linkable(e0, fsorted[i + 1]);
      if (prev) fsorted[i] = e0 | kLink;  // the cell bits that others read are unchanged
    }
  }
  {
    int incl = last;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off);
      if (lane >= off) incl = max(incl, o);
    }
    if (lane == 63) wsum[wave] = static_cast<unsigned>(incl + 1);
    int before = __shfl_up(incl, 1);
    if (lane == 0) before = -1;
    __syncthreads();
    for (int w = 0; w < wave; ++w) before = max(before, static_cast<int>(wsum[w]) - 1);
    int rs = before;  // run start entering the segment (position 0 starts one)
    bool prev = link_in;
    for (int i = s0; i < s1; ++i) {
      const unsigned e = fsorted[i];
      if (!prev) rs = i;
      prev = (e & kLink) != 0u;
      if (((i - rs) & 1) != 0) {
        jkey[i] = ~0u;  // second of the pair that starts at i - 1
      } else {
        jkey[i] = (prev ? 0u : 32u) + bank_of((e >> 16) & 4095u);
      }
    }
  }
  __syncthreads();
  for (int i = t; i < static_cast<int>(cnt); i += NT) {
    const unsigned b = jkey[i];
    if (b != ~0u) jkey[i] = b | static_cast<unsigned>(atomicAdd(&bs.cnt[b], 1)) << 6;
  }
  __syncthreads();
  bank_scan<NT, kPer>(bs);
  __syncthreads();
  // bank-sorted jobs in the workgroup's scratch: a | b << 16 for a pair,
  // a for a single
  for (int i = t; i < static_cast<int>(cnt); i += NT) {
    const unsigned k0 = jkey[i];
    if (k0 == ~0u) continue;
    const unsigned i0 = fsorted[i] & 0xffffu;
    const bool pr = (k0 & 63u) < 32u;
    pjob[bs.cnt[k0 & 63u] + (k0 >> 6)] = pr ? (i0 | (fsorted[i + 1] & 0xffffu) << 16) : i0;
  }
  const int n_pair = bs.cnt[32];
  __syncthreads();
  for (uint32_t i = t; i < cnt; i += NT) {
    words[i] = 0u;
    words[2 * VOL + i] = 0u;
  }
  __syncthreads();
  return n_pair;
}

// Work queues of the persistent scatter: 8 (one per XCD, each over a
// contiguous range of tiles, so that halo lines shared by neighbouring tiles
// stay in one L2) or 1.  A block takes tiles from its own queue, then from
// the others.  Block 0..G-1 runs on XCD (b mod 8): workgroups are dealt to the
// XCDs round robin.
struct TileQueues {
  uint32_t* counter;  // nq counters, zeroed before the launch
  int nq;
  int64_t per_queue;
};

template <int NT>
__device__ __forceinline__ int64_t next_tile(const TileQueues& tq, int64_t n_tiles, long long* s_tile) {
  if (threadIdx.x == 0) {
    long long got = -1;
    const int mine = static_cast<int>(blockIdx.x % tq.nq);
    for (int k = 0; k < tq.nq && got < 0; ++k) {
      const int q = (mine + k) % tq.nq;
      const uint32_t i = atomicAdd(tq.counter + q, 1u);
      const int64_t tl = q * tq.per_queue + static_cast<int64_t>(i);
      if (static_cast<int64_t>(i) < tq.per_queue && tl < n_tiles) got = tl;
    }
    *s_tile = got;
  }
  __syncthreads();
  const int64_t v = *s_tile;
  __syncthreads();
  // uniform: keep the tile index and everything derived from it in SGPRs
  const uint64_t u = static_cast<uint64_t>(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// Tiles of several catalogs in one persistent launch: the work items are the
// catalogs' tiles one catalog after another, item i of catalog c being tile
// i - starts[c] (starts: n_cats + 1 prefix sums of the tile counts).  Thread 0
// claims an item from the queues and finds its catalog; the workgroup
// receives (c << 32) | tile, or -1 when every queue is empty.
template <int NT, bool kMulti>
__device__ __forceinline__ int64_t next_item(const TileQueues& tq, int64_t n_items, const int64_t* starts,
                                             int n_cats, long long* s_tile) {
  if (threadIdx.x == 0) {
    long long got = -1;
    const int mine = static_cast<int>(blockIdx.x % tq.nq);
    for (int k = 0; k < tq.nq && got < 0; ++k) {
      const int q = (mine + k) % tq.nq;
      const uint32_t i = atomicAdd(tq.counter + q, 1u);
      const int64_t tl = q * tq.per_queue + static_cast<int64_t>(i);
      if (static_cast<int64_t>(i) < tq.per_queue && tl < n_items) got = tl;
    }
    if (kMulti && got >= 0) {
      int lo = 0, hi = n_cats;  // starts[lo] <= got < starts[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (starts[mid] <= got) lo = mid; else hi = mid;
      }
      got = (static_cast<long long>(lo) << 32) | static_cast<long long>(got - starts[lo]);
    }
    *s_tile = got;
  }
  __syncthreads();
  const int64_t v = *s_tile;
  __syncthreads();
  const uint64_t u = static_cast<uint64_t>(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// FP32 grids.  A persistent grid of one workgroup per CU walks the occupied
// T^3 tiles.  LDS holds the four fields over the tile plus a halo (2 cells
// below and 3 above along each axis for taps -2..3; 1 and 2 for the cubic
// B-spline's -1..2) as 32-bit fixed point, two fields per 64-bit word: gfx950's LDS adds 64-bit integers at ~9.4
// lanes/clk/CU and 32-bit ones at ~14, but FP32 at ~0.3.
//
// Sums of fixed-point deposits are exact modulo 2^32 in any order, so only
// the final value of each cell has to fit int32.  Per tile and field the
// scale comes from a bound on that value: every cell c of the tile gets
// C(c) = sum of |q| over the tile's particles in c (upper-rounded integer
// adds); then A(g) = sum_j C(g - j) k_j, convolved along x, y and z with
// k_j >= |w_j(f)| for all f, bounds sum_p |q_p phi(g - x_p)| at every cell g
// of the tile and halo.  The scale maps max_g A(g) to just under 2^31, less
// the worst-case sum of the per-deposit rounding errors (half a unit per
// particle).  A single pass over LDS gives both the bound and the zeroed
// accumulator.
//
// kMulti: one launch over the tiles of several catalogs (ScatterCat array
// `cats`, item prefix sums `starts`), so that catalogs with few tiles share
// the GPU; otherwise the one catalog `one`.
//
// Paired deposits (atomic form, 16^3 tiles, truncated BL3, one catalog,
// scratch in pw): a dense tile's particles are counting-sorted by cell in
// LDS (pair_jobs), and along each run of sorted particles whose cells are
// equal or z-neighbours of one (x, y) column they pair greedily.  A pair
// deposits both particles over the 7 z cells they span with 7 atomics per
// (x, y) tap and field pair instead of 12, and fewer VALU operations than
// the two alone (the two products are summed in FP32, then rounded and
// packed once).  Jobs are bank-sorted like particles, pairs and singles in
// wave slots of their own, which the waves claim one at a time; the job
// list is the only thing in the workgroup's global scratch.  Which
// particles pair follows the order of the counters' LDS atomics, so the
// FP32 roundings (not the accuracy) of a grid vary from run to run.
template <int TS, int NT, int NTAP, int DEG, bool kW, bool kMulti, bool kHalo = false>
__global__ __launch_bounds__(NT) void scatter_fixed_kernel(
    ScatterCat one, const ScatterCat* __restrict__ cats, const int64_t* __restrict__ starts, int n_cats,
    int64_t n_items, TileQueues tq, TapPoly tp, TapBound kb, PairWork pw) {
  static_assert(!kHalo || (TS == 16 && NTAP == 6), "the halo layout is that of 16^3 tiles with taps -2..3");
  constexpr int H = kHaloLo<NTAP>;
  constexpr int E = TS + NTAP - 1;
  constexpr int VOL = E * E * E;
  constexpr int kPer = 6;
  constexpr int kSuper = kPer * NT;
  constexpr int kWaves = NT / 64;
  constexpr int kCellOff = (H * E + H) * E + H;  // tap origin -> the particle's own cell
  constexpr int kBoundFields = 2;                 // rho, and the momentum fields together
  __shared__ __align__(16) int acc[kNumFields * VOL];
  __shared__ BankSort<NT, kPer> bs;
  // paired deposits: the 16-bit cell counts, then cell starts, of a tile
  // (two per word) in the bank sort's index array, which they do not use
  constexpr bool kPairOK = TS == 16 && NT == 1024 && NTAP == 6 && DEG == 3 && !kMulti && !kHalo;
  constexpr int kCellWords = TS * TS * TS / 2;
  static_assert(!kPairOK || kCellWords * 4 <= NT * kPer * 2, "cell counts alias the bank-sort index array");
  static_assert(!kPairOK || kCellWords == 2 * NT, "two count words per thread");
  static_assert(!kPairOK || kPairCap <= 2 * VOL, "the paired sort's arrays fit the accumulator block");
  unsigned* ccnt = reinterpret_cast<unsigned*>(bs.idx);
  __shared__ unsigned wsum[kWaves];
  __shared__ int s_slot;  // paired deposits: the next wave slot to claim
  __shared__ float red[kWaves][kNumFields];
  __shared__ float scale_s[kNumFields], inv_s[kNumFields];
  __shared__ long long s_tile;
  // sparse tiles: tap-origin bounding box (min x, y, z, max x, y, z)
  __shared__ int bb[6];
  constexpr uint32_t kSparse = 128;  // at most this many particles: one per thread
  // the current catalog's parameters (uniform; reloaded when it changes)
  const float4* sorted = nullptr;
  const uint32_t* offset = nullptr;
  float* grid = nullptr;
  float* halo = nullptr;
  KeyParams kp = one.kp;
  int bulk = 0;
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  double qmax[kNumFields] = {0.0, 0.0, 0.0, 0.0};
  int nt = 0, n = 0;
  int64_t n3 = 0;
  int cur_cat = -1;
  auto set_cat = [&](const ScatterCat& c) {
    sorted = c.sorted;
    offset = c.offset;
    grid = c.grid;
    halo = c.halo;
    kp = c.kp;
    bulk = c.bulk;
    const Derived* dsrc = c.dsrc;
    vb0 = vb1 = vb2 = 0.0;
    if (bulk) {
      vb0 = dsrc->vb[0];
      vb1 = dsrc->vb[1];
      vb2 = dsrc->vb[2];
    }
    // catalog-wide bound of |q| per field for the charges deposited here
    qmax[0] = dsrc->qmax[0];
    qmax[1] = dsrc->qmax[1] + (bulk ? dsrc->qmax[0] * fabs(vb0) : 0.0);
    qmax[2] = dsrc->qmax[2] + (bulk ? dsrc->qmax[0] * fabs(vb1) : 0.0);
    qmax[3] = dsrc->qmax[3] + (bulk ? dsrc->qmax[0] * fabs(vb2) : 0.0);
    nt = kp.nt;
    n = kp.n;
    n3 = static_cast<int64_t>(n) * n * n;
  };
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  unsigned* cnt_u = reinterpret_cast<unsigned*>(acc);
  unsigned long long* acc2 = reinterpret_cast<unsigned long long*>(acc);

  // largest tap-weight bound, cubed: bounds |wx wy wz| of every deposit
  float kmax = 0.f;
  double ksum = 0.0;
#pragma unroll
  for (int j = 0; j < NTAP; ++j) {
    kmax = fmaxf(kmax, kb.k[j]);
    ksum += static_cast<double>(kb.k[j]);
  }
  const float kmax3 = kmax * kmax * kmax;
  // a cell receives from the 6^3 cells around it: A(g) <= max_c C(c) (sum_j k_j)^3
  const double ksum3 = ksum * ksum * ksum * 1.00001;
  if (t < 6) bb[t] = t < 3 ? E : -1;
  int64_t item = next_item<NT, kMulti>(tq, n_items, starts, n_cats, &s_tile);
  for (int i = t; i < kNumFields * VOL; i += NT) acc[i] = 0;
  if (t < 64) bs.cnt[t] = 0;
  if constexpr (kPairOK)
    for (int i = t; i < kCellWords; i += NT) ccnt[i] = 0u;
  __syncthreads();

  while (item >= 0) {
    const int c_item = static_cast<int>(item >> 32);
    const int64_t tile = item & 0xffffffffll;
    if (c_item != cur_cat) {
      set_cat(kMulti ? cats[c_item] : one);
      cur_cat = c_item;
    }
    const uint32_t p0 = offset[tile], p1 = offset[tile + 1];
    const uint32_t cnt = p1 - p0;
    const int tz = static_cast<int>(tile % nt);
    const int ty = static_cast<int>((tile / nt) % nt);
    const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
    const int ox = tx * TS, oy = ty * TS, oz = tz * TS;
    if (cnt == 0) {  // nothing to deposit (uniform across the workgroup)
      if constexpr (kHalo) {  // the tile's own cells start at zero (no clear in this form)
        for (int i = t; i < TS * TS * TS; i += NT) {
          const int64_t gi = (static_cast<int64_t>(ox + i / (TS * TS)) * n + oy + (i / TS) % TS) * n + oz + i % TS;
#pragma unroll
          for (int f = 0; f < kNumFields; ++f) grid[f * n3 + gi] = 0.f;
        }
      }
      item = next_item<NT, kMulti>(tq, n_items, starts, n_cats, &s_tile);
      continue;
    }
    // integer scale of the cell sums C: n_tile * qmax maps just under 2^32,
    // and upper rounding adds at most one unit per particle
    float csc[kNumFields];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f)
      csc[f] = (qmax[f] > 0.0 && cnt > 0)
                   ? static_cast<float>((4294967295.0 - cnt) * (1.0 - 1e-6) / (static_cast<double>(cnt) * qmax[f]))
                   : 0.f;
    // Two bound fields: rho's scaled charges, and for the three momentum
    // fields the largest of their scaled charges (each field's own scale
    // then divides that bound); u32 cannot overflow, since every scaled
    // charge is at most (2^32 - 1 - cnt) / cnt.
    auto add_cell_sums = [&](const float4& a, const float4& v, unsigned cell) {
      const DepositQ<float> d = charges<float>(a, v, bulk, vb0, vb1, vb2);
      const unsigned u0 = static_cast<unsigned>(ceilf(fabsf(d.q[0]) * csc[0]));
      unsigned u1 = 0;
#pragma unroll
      for (int f = 1; f < kNumFields; ++f) u1 = max(u1, static_cast<unsigned>(ceilf(fabsf(d.q[f]) * csc[f])));
      if (u0) atomicAdd(cnt_u + cell, u0);
      if (u1) atomicAdd(cnt_u + VOL + cell, u1);
    };
    // first super-chunk: bank keys (the counters were zeroed before the
    // previous flush) and cell sums; then the cell sums of the rest
    const int m0 = static_cast<int>(min(static_cast<uint32_t>(kSuper), cnt));
    // A sparse tile skips the per-cell bound: every cell holds at most
    // sum_p |q_p| K^3, and only the tap-origin bounding box is flushed.
    const bool sparse = cnt <= kSparse;  // uniform across the workgroup
    const bool paired = kPairOK && !sparse && pw.base != nullptr && cnt <= static_cast<uint32_t>(kPairCap) &&
                        static_cast<int>(blockIdx.x) < pw.blocks;
    uint32_t* const pjobs = paired ? pw.base + static_cast<int64_t>(blockIdx.x) * kPairCap : nullptr;
    // paired: the cell keys of particles kSuper.. go to the accumulator
    // words of fields 2, 3 (2 VOL + i), zero and unused until the deposits
    unsigned* const words = reinterpret_cast<unsigned*>(acc);
    float qsum[kNumFields] = {0.f, 0.f, 0.f, 0.f};
    unsigned key0[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      key0[r] = 0;
      if (t + r * NT < m0) {
        const int64_t p = static_cast<int64_t>(p0) + t + r * NT;
        const float4 a = rec_pos<kW>(sorted, p);
        const unsigned base = tap_origin<TS, NTAP>(a, kp, ox, oy, oz);
        if (paired) {
          key0[r] = cell_rank(base, ccnt);
        } else {
          const unsigned b = base & 31u;
          key0[r] = b | (static_cast<unsigned>(atomicAdd(&bs.cnt[b], 1)) << 6);
        }
        if (sparse) {
          const DepositQ<float> d = charges<float>(a, rec_vel<kW>(sorted, p), bulk, vb0, vb1, vb2);
#pragma unroll
          for (int f = 0; f < kNumFields; ++f) qsum[f] += fabsf(d.q[f]);
          const int cx = static_cast<int>(base) / (E * E), cy = (static_cast<int>(base) / E) % E,
                    cz = static_cast<int>(base) % E;
          atomicMin(&bb[0], cx);
          atomicMin(&bb[1], cy);
          atomicMin(&bb[2], cz);
          atomicMax(&bb[3], cx);
          atomicMax(&bb[4], cy);
          atomicMax(&bb[5], cz);
        } else {
          add_cell_sums(a, rec_vel<kW>(sorted, p), base + kCellOff);
        }
      }
    }
    if (sparse) {
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) {
        float v = qsum[f];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][f] = v;
      }
    } else {
    for (uint32_t p = p0 + static_cast<uint32_t>(m0) + t; p < p1; p += NT) {
      const float4 a = rec_pos<kW>(sorted, static_cast<int64_t>(p));
      const unsigned base = tap_origin<TS, NTAP>(a, kp, ox, oy, oz);
      const float4 v = rec_vel<kW>(sorted, static_cast<int64_t>(p));
      add_cell_sums(a, v, base + kCellOff);
      if (paired) words[2 * VOL + (p - p0)] = cell_rank(base, ccnt);
    }
    __syncthreads();
    // the largest cell sum of each bound field (only the tile's own cells
    // hold sums), clearing the sums for the deposits
    float amax[kBoundFields] = {0.f, 0.f};
    for (int rr = t; rr < kBoundFields * TS * TS * TS; rr += NT) {
      const int f = rr / (TS * TS * TS);
      const int c = rr % (TS * TS * TS);
      int* cell = acc + f * VOL + ((H + c / (TS * TS)) * E + H + (c / TS) % TS) * E + H + c % TS;
      const float v = static_cast<float>(static_cast<unsigned>(*cell));
      *cell = 0;
#pragma unroll
      for (int ff = 0; ff < kBoundFields; ++ff)
        if (ff == f) amax[ff] = fmaxf(amax[ff], v);
    }
#pragma unroll
    for (int f = 0; f < kBoundFields; ++f) {
      float m = amax[f];
      for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
      if (lane == 0) red[wave][f] = m;
    }
    }  // dense tile
    // The tile's fixed-point scale of each field (one thread per field).
    auto set_scale = [&]() {
      float mx = 0.f;
      const int bf = t < kBoundFields ? t : kBoundFields - 1;  // dense: the field's bound field
      for (int w = 0; w < kWaves; ++w) mx = sparse ? mx + red[w][t] : fmaxf(mx, red[w][bf]);
      // A in charge units (with a margin for the FP32 convolution, or the
      // sum bound of a sparse tile); room for the rounding errors of up to
      // cnt deposits per cell
      const double bound = sparse ? static_cast<double>(mx) * static_cast<double>(kmax3) * 1.0001
                                  : static_cast<double>(mx) * ksum3 / static_cast<double>(csc[t]);
      const double room = 0.99 * 2147483648.0 - 0.5 * static_cast<double>(cnt) - 64.0;
      const double scl = (mx > 0.f && (sparse || csc[t] > 0.f)) ? fmin(room / bound, 1e30) : 0.0;
      scale_s[t] = static_cast<float>(scl);
      inv_s[t] = scl > 0.0 ? static_cast<float>(1.0 / static_cast<double>(static_cast<float>(scl))) : 0.f;
    };
    // Paired path, one particle (record p):
    auto deposit_one = [&](uint32_t p, const float (&sc)[kNumFields]) {
      const float4 a = rec_pos<kW>(sorted, static_cast<int64_t>(p));
      const float4 v = rec_vel<kW>(sorted, static_cast<int64_t>(p));
      float wx[NTAP], wy[NTAP], wz[NTAP];
      const unsigned base = particle_taps<float, TS, NTAP, DEG>(a, kp, ox, oy, oz, tp, wx, wy, wz);
      const DepositQ<float> d = charges<float>(a, v, bulk, vb0, vb1, vb2);
      float qs[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) qs[f] = d.q[f] * sc[f];
#pragma unroll
      for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
        for (int jy = 0; jy < NTAP; ++jy) {
          const float wxy = wx[jx] * wy[jy];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const float wlo = wxy * qs[2 * k], whi = wxy * qs[2 * k + 1];
            unsigned long long* row = acc2 + k * VOL + base + (jx * E + jy) * E;
#pragma unroll
            for (int jz = 0; jz < NTAP; ++jz) atomicAdd(row + jz, deposit_pair(wlo, whi, wz[jz]));
          }
        }
      }
    };
    // Two particles (records pa, pb; pb's cell is pa's or the one above it
    // along z) over the NTAP + 1 z cells from pa's tap origin.
    auto deposit_two = [&](uint32_t pa, uint32_t pb, const float (&sc)[kNumFields]) {
      const float4 a0 = rec_pos<kW>(sorted, static_cast<int64_t>(pa));
      const float4 v0 = rec_vel<kW>(sorted, static_cast<int64_t>(pa));
      const float4 a1 = rec_pos<kW>(sorted, static_cast<int64_t>(pb));
      const float4 v1 = rec_vel<kW>(sorted, static_cast<int64_t>(pb));
      float wx0[NTAP], wy0[NTAP], wz0[NTAP], wx1[NTAP], wy1[NTAP], wz1[NTAP];
      const unsigned base = particle_taps<float, TS, NTAP, DEG>(a0, kp, ox, oy, oz, tp, wx0, wy0, wz0);
      const unsigned base1 = particle_taps<float, TS, NTAP, DEG>(a1, kp, ox, oy, oz, tp, wx1, wy1, wz1);
      const bool up = base1 != base;
      float wzb[NTAP + 1];  // the second particle's z weights on the pair's cells
      wzb[0] = up ? 0.f : wz1[0];
#pragma unroll
      for (int j = 1; j < NTAP; ++j) wzb[j] = up ? wz1[j - 1] : wz1[j];
      wzb[NTAP] = up ? wz1[NTAP - 1] : 0.f;
      const DepositQ<float> d0 = charges<float>(a0, v0, bulk, vb0, vb1, vb2);
      const DepositQ<float> d1 = charges<float>(a1, v1, bulk, vb0, vb1, vb2);
      float qa[kNumFields], qb[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) {
        qa[f] = d0.q[f] * sc[f];
        qb[f] = d1.q[f] * sc[f];
      }
#pragma unroll
      for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
        for (int jy = 0; jy < NTAP; ++jy) {
          const float wxa = wx0[jx] * wy0[jy], wxb = wx1[jx] * wy1[jy];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const float alo = wxa * qa[2 * k], ahi = wxa * qa[2 * k + 1];
            const float blo = wxb * qb[2 * k], bhi = wxb * qb[2 * k + 1];
            unsigned long long* row = acc2 + k * VOL + base + (jx * E + jy) * E;
#pragma unroll
            for (int jz = 0; jz < NTAP; ++jz)
              atomicAdd(row + jz, deposit_pair2(alo, ahi, wz0[jz], blo, bhi, wzb[jz]));
            if (up) atomicAdd(row + NTAP, deposit_pair(blo, bhi, wzb[NTAP]));
          }
        }
      }
    };
    // One super-chunk: scan the bank counters, place local indices in bank
    // order, deposit.  key[r] = bank | slot << 6 of local particle t + r NT.
    auto deposit_chunk = [&](uint32_t c0, int m, const unsigned (&key)[kPer], bool first) {
      __syncthreads();
      if (first && t < kNumFields) set_scale();
      bank_scan<NT, kPer>(bs);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const int i = t + r * NT;
        if (i < m) bs.idx[bs.cnt[key[r] & 63u] + (key[r] >> 6)] = static_cast<unsigned short>(i);
      }
      float sc[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) sc[f] = scale_s[f];
      __syncthreads();
      const int slots = (m + 63) >> 6;
      // each half-wave takes one lane from each of the 32 bank pairs
      const int lr = ((lane & 31) << 1) | (lane >> 5);
      for (int sl = wave; sl < slots; sl += kWaves) {
        const int q = lr * slots + sl;
        if (q >= m) continue;
        // deposit_one's body, written out: as a call here it costs the other
        // 6-tap kernels registers
        const uint32_t p = c0 + bs.idx[q];
        const float4 a = rec_pos<kW>(sorted, static_cast<int64_t>(p));
        const float4 v = rec_vel<kW>(sorted, static_cast<int64_t>(p));
        float wx[NTAP], wy[NTAP], wz[NTAP];
        const unsigned base = particle_taps<float, TS, NTAP, DEG>(a, kp, ox, oy, oz, tp, wx, wy, wz);
        const DepositQ<float> d = charges<float>(a, v, bulk, vb0, vb1, vb2);
        float qs[kNumFields];
#pragma unroll
        for (int f = 0; f < kNumFields; ++f) qs[f] = d.q[f] * sc[f];
        unsigned long long* accp[2] = {acc2 + base, acc2 + VOL + base};
#pragma unroll
        for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
          for (int jy = 0; jy < NTAP; ++jy) {
            const float wxy = wx[jx] * wy[jy];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const float wlo = wxy * qs[2 * k], whi = wxy * qs[2 * k + 1];
#pragma unroll
              for (int jz = 0; jz < NTAP; ++jz)
                atomicAdd(accp[k] + (jx * E + jy) * E + jz, deposit_pair(wlo, whi, wz[jz]));
            }
          }
        }
      }
      __syncthreads();
    };
    if (paired) {
      __syncthreads();  // cell counts and bound maxima complete
      if (t < kNumFields) set_scale();
      const int n_pair = pair_jobs<NT, kPer, E>(words, ccnt, wsum, bs, key0, m0, cnt, pjobs);
      uint32_t* const pjob = pjobs;
      float sc[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) sc[f] = scale_s[f];
      if (t == 0) s_slot = kWaves;
      __syncthreads();
      // wave slots: the pair jobs, then the single jobs
      const int n_single = static_cast<int>(cnt) - 2 * n_pair;
      const int wp = (n_pair + 63) >> 6, ws = (n_single + 63) >> 6;
      const int lr = ((lane & 31) << 1) | (lane >> 5);
      // each wave claims its next slot when it is done with one, so that
      // the waves leave the loop together however the LDS unit serves them
      for (int sl = wave; sl < wp + ws;) {
        if (sl < wp) {
          const int q = lr * wp + sl;
          if (q < n_pair) {
            const unsigned jd = pjob[q];
            deposit_two(p0 + (jd & 0xffffu), p0 + (jd >> 16), sc);
          }
        } else {
          const int q = lr * ws + (sl - wp);
          if (q < n_single) deposit_one(p0 + pjob[n_pair + q], sc);
        }
        int next = 0;
        if (lane == 0) next = atomicAdd(&s_slot, 1);
        sl = __shfl(next, 0);
      }
      __syncthreads();
    } else {
    deposit_chunk(p0, m0, key0, true);
    for (uint32_t c0 = p0 + kSuper; c0 < p1; c0 += kSuper) {
      const int m = static_cast<int>(min(static_cast<uint32_t>(kSuper), p1 - c0));
      if (t < 64) bs.cnt[t] = 0;
      __syncthreads();
      unsigned key[kPer];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        key[r] = 0;
        if (t + r * NT < m) {
          const unsigned b =
              tap_origin<TS, NTAP>(rec_pos<kW>(sorted, static_cast<int64_t>(c0 + t + r * NT)), kp, ox, oy, oz) & 31u;
          key[r] = b | (static_cast<unsigned>(atomicAdd(&bs.cnt[b], 1)) << 6);
        }
      }
      deposit_chunk(c0, m, key, false);
    }
    }  // unpaired
    // take the next tile, then flush this one (clearing it)
    item = next_item<NT, kMulti>(tq, n_items, starts, n_cats, &s_tile);
    if (t < 64) bs.cnt[t] = 0;
    if constexpr (kPairOK)  // the deposits no longer read the bank-sort index array
      for (int i = t; i < kCellWords; i += NT) ccnt[i] = 0u;
    float inv[kNumFields];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) inv[f] = inv_s[f];
    // atomic form: a dense tile's whole block, a sparse tile's tap-origin box
    // grown by the taps; halo form: the whole block (every halo cell is read
    // by the fix-up)
    int fx0 = 0, fy0 = 0, fz0 = 0, fdx = E, fdy = E, fdz = E;
    if (sparse) {
      if constexpr (!kHalo) {
        fx0 = bb[0];
        fy0 = bb[1];
        fz0 = bb[2];
        fdx = bb[3] + NTAP - fx0;
        fdy = bb[4] + NTAP - fy0;
        fdz = bb[5] + NTAP - fz0;
      }
      __syncthreads();  // every thread has read the box
      if (t < 6) bb[t] = t < 3 ? E : -1;  // visible to the next tile after the final barrier
    }
    const int fvol = fdx * fdy * fdz;
    float* hbase = kHalo ? halo + tile * (static_cast<int64_t>(kNumFields) * kHaloCells) : nullptr;
    const bool whole = fdx == E && fdy == E && fdz == E;  // uniform: constant divisors
    for (int j = t; j < fvol; j += NT) {
      int ex, ey, ez;
      if (whole) {
        ez = j % E;
        ey = (j / E) % E;
        ex = j / (E * E);
      } else {
        ez = fz0 + j % fdz;
        ey = fy0 + (j / fdz) % fdy;
        ex = fx0 + j / (fdy * fdz);
      }
      const int i = (ex * E + ey) * E + ez;
      const int gx = (ox + ex - H) & (n - 1);
      const int gy = (oy + ey - H) & (n - 1);
      const int gz = (oz + ez - H) & (n - 1);
      const int64_t gi = (static_cast<int64_t>(gx) * n + gy) * n + gz;
      const bool core = ex >= H && ex < H + TS && ey >= H && ey < H + TS && ez >= H && ez < H + TS;
      const int hc = kHalo && !core ? halo_index(ex, ey, ez) : 0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const unsigned long long sum = acc2[k * VOL + i];
        acc2[k * VOL + i] = 0ull;
        int lo, hi;
        unpack_pair(sum, &lo, &hi);
        const float vlo = static_cast<float>(lo) * inv[2 * k], vhi = static_cast<float>(hi) * inv[2 * k + 1];
        if constexpr (kHalo) {
          if (core) {
            grid[(2 * k) * n3 + gi] = vlo;
            grid[(2 * k + 1) * n3 + gi] = vhi;
          } else {
            hbase[(2 * k) * kHaloCells + hc] = vlo;
            hbase[(2 * k + 1) * kHaloCells + hc] = vhi;
          }
        } else {
          if (lo != 0) atomicAdd(grid + (2 * k) * n3 + gi, vlo);
          if (hi != 0) atomicAdd(grid + (2 * k + 1) * n3 + gi, vhi);
        }
      }
    }
    __syncthreads();
  }
}

// FP32 grids of sparse catalogs, owner-computes ("gather") form.  A tile
// computes the final values of its own T^3 cells (T = 16) and writes them
// with plain stores: no halo, no global atomics and no grid clear.  Its
// sources are the particles whose taps reach it, those in cells
// [o - 3, o + T + 1] per axis for the truncated BL3 taps j = -2..3 (the
// source region, 21 cells), drawn from the tile and its 26 periodic
// neighbours (at least 4 tiles per axis, so that the neighbours are
// distinct and a cell's periodic offset from the tile is unambiguous).  Two
// passes over these candidates:
//   1. per-cell sums of the scaled |q| over the source region, whose largest
//      value (from the atomics' returns) times (sum_j k_j)^3 bounds every
//      cell of the tile, as in the atomic form; the in-region candidates go
//      to an LDS list;
//   2. the deposits of the taps that land in the tile, in 32-bit fixed point,
//      two fields per 64-bit LDS word: the listed records dealt to all
//      lanes, or, when more than the list holds are in the region, each
//      wave's in-region candidates found again and queued in a ring of 128
//      LDS slots, deposited 64 at a time, so that the many neighbour
//      candidates outside the region do not leave lanes idle through the
//      deposit loop.
// The candidates' records are read from 27 tiles (twice when the list
// overflows): this pays while tiles hold few particles and the atomic
// form's halo flush dominates.
template <int NT, bool kW, bool kMulti>
__global__ __launch_bounds__(NT) void scatter_gather_kernel(
    ScatterCat one, const ScatterCat* __restrict__ cats, const int64_t* __restrict__ starts, int n_cats,
    int64_t n_items, TileQueues tq, TapPoly tp, TapBound kb) {
  constexpr int TS = 16, NTAP = 6, DEG = 3;
  constexpr int H = kHaloLo<NTAP>;   // taps reach H cells below a particle's cell
  constexpr int HI = NTAP - 1 - H;   // and HI cells above it
  constexpr int R = TS + NTAP - 1;   // source region per axis: cells [-HI, TS + H)
  constexpr int RV = R * R * R;
  constexpr int CV = TS * TS * TS;
  constexpr int kWaves = NT / 64;
  constexpr int kRing = 128;
  constexpr int kList = 1152;
  static_assert(2 * CV * 2 <= 2 * RV, "the deposit pairs alias the cell sums");
  static_assert(kWaves * kRing * 4 <= kList * 6, "the ring aliases the list");
  __shared__ __align__(16) unsigned blk[2 * RV];  // cell sums, then 2 x CV 64-bit pairs
  // the in-region candidates' records and cells (pass 1 to pass 2), or,
  // when they overflow the list, each wave's queue of candidates (pass 2)
  __shared__ __align__(16) unsigned char lbuf[kList * 6];
  __shared__ int list_n;
  uint32_t* list_rec = reinterpret_cast<uint32_t*>(lbuf);
  unsigned short* list_cell = reinterpret_cast<unsigned short*>(lbuf + 4 * kList);
  int (*ring)[kRing] = reinterpret_cast<int (*)[kRing]>(lbuf);
  __shared__ int nb_first[28];                    // prefix sums of the 27 candidate ranges
  __shared__ uint32_t nb_start[27];
  __shared__ unsigned red[kWaves][2];
  __shared__ float scale_s[kNumFields], inv_s[kNumFields];
  __shared__ long long s_tile;
  unsigned long long* acc2 = reinterpret_cast<unsigned long long*>(blk);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;

  const float4* sorted = nullptr;
  const uint32_t* offset = nullptr;
  float* grid = nullptr;
  KeyParams kp = one.kp;
  int bulk = 0;
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  double qmax[kNumFields] = {0.0, 0.0, 0.0, 0.0};
  int nt = 0, n = 0;
  int64_t n3 = 0;
  int cur_cat = -1;
  auto set_cat = [&](const ScatterCat& c) {
    sorted = c.sorted;
    offset = c.offset;
    grid = c.grid;
    kp = c.kp;
    bulk = c.bulk;
    const Derived* dsrc = c.dsrc;
    vb0 = vb1 = vb2 = 0.0;
    if (bulk) {
      vb0 = dsrc->vb[0];
      vb1 = dsrc->vb[1];
      vb2 = dsrc->vb[2];
    }
    qmax[0] = dsrc->qmax[0];
    qmax[1] = dsrc->qmax[1] + (bulk ? dsrc->qmax[0] * fabs(vb0) : 0.0);
    qmax[2] = dsrc->qmax[2] + (bulk ? dsrc->qmax[0] * fabs(vb1) : 0.0);
    qmax[3] = dsrc->qmax[3] + (bulk ? dsrc->qmax[0] * fabs(vb2) : 0.0);
    nt = kp.nt;
    n = kp.n;
    n3 = static_cast<int64_t>(n) * n * n;
  };
  double ksum = 0.0;
#pragma unroll
  for (int j = 0; j < NTAP; ++j) ksum += static_cast<double>(kb.k[j]);
  const double ksum3 = ksum * ksum * ksum * 1.00001;

  // A record's position, its cell rc relative to this tile's origin and its
  // fractions fr; true when the cell lies in the source region.  The cells
  // of the 27-tile neighbourhood lie within [-16, 32) of the origin, so on
  // grids of N >= 64 the periodic offset taken in [-N/2, N/2) is the true one.
  int ox = 0, oy = 0, oz = 0;
  auto record_cell = [&](uint32_t rec, float4* a, int* rc, double* fr) -> bool {
    *a = rec_pos<kW>(sorted, static_cast<int64_t>(rec));
    const int o[3] = {ox, oy, oz};
    const float xs[3] = {a->x, a->y, a->z};
    bool in = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      bool ok;
      const int c = locate(xs[ax], kp.scale, kp.shift, kp.n, &fr[ax], &ok);
      rc[ax] = ((c - o[ax] + n / 2) & (n - 1)) - n / 2;
      in = in && rc[ax] >= -HI && rc[ax] < TS + H;
    }
    return in;
  };
  // Candidate i (0 <= i < total) of the neighbourhood's 27 record ranges.
  auto candidate = [&](int i, float4* a, uint32_t* rec, int* rc, double* fr) -> bool {
    int lo = 0, hi = 27;  // nb_first[lo] <= i < nb_first[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nb_first[mid] <= i) lo = mid; else hi = mid;
    }
    *rec = nb_start[lo] + static_cast<uint32_t>(i - nb_first[lo]);
    return record_cell(*rec, a, rc, fr);
  };

  for (int i = t; i < 2 * RV; i += NT) blk[i] = 0u;
  int64_t item = next_item<NT, kMulti>(tq, n_items, starts, n_cats, &s_tile);
  while (item >= 0) {
    const int c_item = static_cast<int>(item >> 32);
    const int64_t tile = item & 0xffffffffll;
    if (c_item != cur_cat) {
      set_cat(kMulti ? cats[c_item] : one);
      cur_cat = c_item;
    }
    const int tz = static_cast<int>(tile % nt);
    const int ty = static_cast<int>((tile / nt) % nt);
    const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
    ox = tx * TS;
    oy = ty * TS;
    oz = tz * TS;
    if (t < 27) {
      const int dx = t / 9 - 1, dy = (t / 3) % 3 - 1, dz = t % 3 - 1;
      const int64_t tn = (static_cast<int64_t>((tx + dx + nt) % nt) * nt + (ty + dy + nt) % nt) * nt +
                         (tz + dz + nt) % nt;
      nb_start[t] = offset[tn];
      nb_first[t + 1] = static_cast<int>(offset[tn + 1] - offset[tn]);
    }
    __syncthreads();
    if (t == 0) {
      nb_first[0] = 0;
      for (int r = 0; r < 27; ++r) nb_first[r + 1] += nb_first[r];
      list_n = 0;
    }
    __syncthreads();
    const int total = nb_first[27];
    if (total > 0) {  // uniform; otherwise the tile is written with zeros
      // integer scale of the cell sums: the candidates bound the count, and
      // upper rounding adds at most one unit per candidate
      float csc[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f)
        csc[f] = qmax[f] > 0.0
                     ? static_cast<float>((4294967295.0 - total) * (1.0 - 1e-6) / (static_cast<double>(total) * qmax[f]))
                     : 0.f;
      // pass 1: cell sums over the source region (rho; the largest of the
      // momentum fields' scaled charges), their maxima from the atomics'
      // returns, and a list of the in-region candidates (up to kList)
      unsigned m0 = 0, m1 = 0;
      for (int b = wave * 64; b < total; b += NT) {  // uniform within the wave
        const int i = b + lane;
        float4 a;
        uint32_t rec;
        int rc[3];
        double fr[3];
        const bool in = i < total && candidate(i, &a, &rec, rc, fr);
        const unsigned long long mask = __ballot(in);
        int base = 0;
        if (lane == 0 && mask) base = atomicAdd(&list_n, __popcll(mask));
        base = __shfl(base, 0);
        if (in) {
          const int cell = ((rc[0] + HI) * R + rc[1] + HI) * R + rc[2] + HI;
          const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
          if (slot < kList) {
            list_rec[slot] = rec;
            list_cell[slot] = static_cast<unsigned short>(cell);
          }
          const DepositQ<float> q = charges<float>(a, rec_vel<kW>(sorted, static_cast<int64_t>(rec)), bulk, vb0, vb1, vb2);
          const unsigned u0 = static_cast<unsigned>(ceilf(fabsf(q.q[0]) * csc[0]));
          unsigned u1 = 0;
#pragma unroll
          for (int f = 1; f < kNumFields; ++f) u1 = max(u1, static_cast<unsigned>(ceilf(fabsf(q.q[f]) * csc[f])));
          if (u0) m0 = max(m0, atomicAdd(&blk[cell], u0) + u0);
          if (u1) m1 = max(m1, atomicAdd(&blk[RV + cell], u1) + u1);
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        m0 = max(m0, static_cast<unsigned>(__shfl_xor(static_cast<int>(m0), off)));
        m1 = max(m1, static_cast<unsigned>(__shfl_xor(static_cast<int>(m1), off)));
      }
      if (lane == 0) {
        red[wave][0] = m0;
        red[wave][1] = m1;
      }
      __syncthreads();
      const int listed = list_n;
      const bool fits = listed <= kList;  // uniform
      if (t < kNumFields) {
        unsigned mx = 0;
        const int bf = t == 0 ? 0 : 1;
        for (int w = 0; w < kWaves; ++w) mx = max(mx, red[w][bf]);
        // bound in charge units; room for the rounding errors of up to
        // `total` deposits per cell
        const double bound = static_cast<double>(mx) * ksum3 / static_cast<double>(csc[t]);
        const double room = 0.99 * 2147483648.0 - 0.5 * static_cast<double>(total) - 64.0;
        const double scl = (mx > 0 && csc[t] > 0.f) ? fmin(room / bound, 1e30) : 0.0;
        scale_s[t] = static_cast<float>(scl);
        inv_s[t] = scl > 0.0 ? static_cast<float>(1.0 / static_cast<double>(static_cast<float>(scl))) : 0.f;
      }
      // clear the cell sums for the deposits: the listed cells, or all
      if (fits) {
        for (int j = t; j < listed; j += NT) {
          blk[list_cell[j]] = 0u;
          blk[RV + list_cell[j]] = 0u;
        }
      } else {
        for (int i = t; i < 2 * RV; i += NT) blk[i] = 0u;
      }
      __syncthreads();
      float sc[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) sc[f] = scale_s[f];
      // pass 2: one in-region particle's deposits of the taps that land in
      // the tile
      auto deposit_one = [&](const float4& a, uint32_t rec, const int* rc, const double* fr) {
        float wx[NTAP], wy[NTAP], wz[NTAP];
#pragma unroll
        for (int j = 0; j < NTAP; ++j) {
          wx[j] = static_cast<float>(tap_weight<DEG>(tp, j, fr[0]));
          wy[j] = static_cast<float>(tap_weight<DEG>(tp, j, fr[1]));
          wz[j] = static_cast<float>(tap_weight<DEG>(tp, j, fr[2]));
        }
        const DepositQ<float> q = charges<float>(a, rec_vel<kW>(sorted, static_cast<int64_t>(rec)), bulk, vb0, vb1, vb2);
        float qs[kNumFields];
#pragma unroll
        for (int f = 0; f < kNumFields; ++f) qs[f] = q.q[f] * sc[f];
        // tap j lands on cell rc + j - H
#pragma unroll
        for (int jx = 0; jx < NTAP; ++jx) {
          const int gx = rc[0] + jx - H;
          if (gx < 0 || gx >= TS) continue;
#pragma unroll
          for (int jy = 0; jy < NTAP; ++jy) {
            const int gy = rc[1] + jy - H;
            if (gy < 0 || gy >= TS) continue;
            const float wxy = wx[jx] * wy[jy];
            const int row = (gx * TS + gy) * TS;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const float wlo = wxy * qs[2 * k], whi = wxy * qs[2 * k + 1];
#pragma unroll
              for (int jz = 0; jz < NTAP; ++jz) {
                const int gz = rc[2] + jz - H;
                if (gz >= 0 && gz < TS) atomicAdd(acc2 + k * CV + row + gz, deposit_pair(wlo, whi, wz[jz]));
              }
            }
          }
        }
      };
      if (fits) {  // the listed records, dealt to all lanes
        for (int j = t; j < listed; j += NT) {
          const uint32_t rec = list_rec[j];
          float4 a;
          int rc[3];
          double fr[3];
          (void)record_cell(rec, &a, rc, fr);
          deposit_one(a, rec, rc, fr);
        }
      } else {
        // more in-region candidates than the list holds: each wave evaluates
        // the candidates again and queues its in-region ones in a ring of
        // kRing LDS slots, depositing 64 at a time (lanes beyond `m` idle)
        auto deposit = [&](int head, int m) {
          if (lane >= m) return;
          float4 a;
          uint32_t rec;
          int rc[3];
          double fr[3];
          (void)candidate(ring[wave][(head + lane) & (kRing - 1)], &a, &rec, rc, fr);
          deposit_one(a, rec, rc, fr);
        };
        int head = 0, queued = 0;  // uniform within the wave
        for (int b = wave * 64; b < total; b += NT) {
          const int i = b + lane;
          float4 a;
          uint32_t rec;
          int rc[3];
          double fr[3];
          const bool in = i < total && candidate(i, &a, &rec, rc, fr);
          const unsigned long long mask = __ballot(in);
          if (in) {
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            ring[wave][(head + queued + rank) & (kRing - 1)] = i;
          }
          queued += __popcll(mask);
          __builtin_amdgcn_wave_barrier();
          if (queued >= 64) {
            deposit(head, 64);
            head = (head + 64) & (kRing - 1);
            queued -= 64;
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (queued > 0) deposit(head, queued);
      }
      __syncthreads();
    }
    // write the tile's cells with plain stores, clearing the block
    float inv[kNumFields];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) inv[f] = total > 0 ? inv_s[f] : 0.f;
    for (int i = t; i < CV; i += NT) {
      const int ez = i % TS, ey = (i / TS) % TS, ex = i / (TS * TS);
      const int64_t gi = (static_cast<int64_t>(ox + ex) * n + oy + ey) * n + oz + ez;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const unsigned long long sum = acc2[k * CV + i];
        acc2[k * CV + i] = 0ull;
        int lo, hi;
        unpack_pair(sum, &lo, &hi);
        grid[(2 * k) * n3 + gi] = static_cast<float>(lo) * inv[2 * k];
        grid[(2 * k + 1) * n3 + gi] = static_cast<float>(hi) * inv[2 * k + 1];
      }
    }
    item = next_item<NT, kMulti>(tq, n_items, starts, n_cats, &s_tile);
  }
}

// The halo form's fix-up.  A cell receives the halo cells of the
// neighbouring tiles' blocks that cover it when it lies within 3 cells of
// its tile's low face or 2 of its high face along some axis (the band: 2765
// of a tile's 4096 cells); the fix-up adds them to the value the cell's own
// tile stored, in a fixed order (neighbour offsets ascending), skipping
// neighbours without particles.  One workgroup per tile.
template <bool kMulti>
__global__ __launch_bounds__(256) void halo_fixup_kernel(ScatterCat one, const ScatterCat* __restrict__ cats,
                                                         const int64_t* __restrict__ starts, int n_cats) {
  constexpr int TS = 16, H = 2, B = 5, IN = TS - B;
  constexpr int kBand = TS * TS * TS - IN * IN * IN;
  __shared__ int nb_full[27];
  const int t = threadIdx.x;
  int64_t tile = blockIdx.x;
  int c = 0;
  if constexpr (kMulti) {
    int lo = 0, hi = n_cats;  // starts[lo] <= item < starts[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (starts[mid] <= tile) lo = mid; else hi = mid;
    }
    c = lo;
    tile -= starts[c];
  }
  const ScatterCat& cat = kMulti ? cats[c] : one;
  const uint32_t* offset = cat.offset;
  float* grid = cat.grid;
  const float* halo = cat.halo;
  const int nt = cat.kp.nt, n = cat.kp.n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const int tz = static_cast<int>(tile % nt);
  const int ty = static_cast<int>((tile / nt) % nt);
  const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
  auto neighbour = [&](int dx, int dy, int dz) -> int64_t {
    return (static_cast<int64_t>((tx + dx + nt) % nt) * nt + (ty + dy + nt) % nt) * nt + (tz + dz + nt) % nt;
  };
  bool full = false;
  if (t < 27 && t != 13) {
    const int64_t tn = neighbour(t / 9 - 1, (t / 3) % 3 - 1, t % 3 - 1);
    full = offset[tn + 1] > offset[tn];
  }
  if (t < 27) nb_full[t] = full ? 1 : 0;
  if (!__syncthreads_or(full)) return;  // uniform: no neighbour halo reaches this tile
  auto band_cell = [](int i) { return i < 3 ? i : i + IN; };  // 0..4 -> 0, 1, 2, 14, 15
  for (int b = t; b < kBand; b += 256) {
    int l[3];
    if (b < B * TS * TS) {
      l[0] = band_cell(b / (TS * TS));
      l[1] = (b / TS) % TS;
      l[2] = b % TS;
    } else if (b < B * TS * TS + IN * B * TS) {
      const int r = b - B * TS * TS;
      l[0] = 3 + r / (B * TS);
      l[1] = band_cell((r / TS) % B);
      l[2] = r % TS;
    } else {
      const int r = b - B * TS * TS - IN * B * TS;
      l[0] = 3 + r / (IN * B);
      l[1] = 3 + (r / B) % IN;
      l[2] = band_cell(r % B);
    }
    int dlo[3], dhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dlo[a] = l[a] < 3 ? -1 : 0;
      dhi[a] = l[a] >= TS - 2 ? 1 : 0;
    }
    const int64_t gi = (static_cast<int64_t>(tx * TS + l[0]) * n + ty * TS + l[1]) * n + tz * TS + l[2];
    float v[kNumFields];
    bool touched = false;
    for (int dx = dlo[0]; dx <= dhi[0]; ++dx)
      for (int dy = dlo[1]; dy <= dhi[1]; ++dy)
        for (int dz = dlo[2]; dz <= dhi[2]; ++dz) {
          if ((dx | dy | dz) == 0 || !nb_full[(dx + 1) * 9 + (dy + 1) * 3 + dz + 1]) continue;
          if (!touched) {
#pragma unroll
            for (int f = 0; f < kNumFields; ++f) v[f] = grid[f * n3 + gi];
            touched = true;
          }
          const float* hb = halo + neighbour(dx, dy, dz) * (static_cast<int64_t>(kNumFields) * kHaloCells) +
                            halo_index(l[0] - TS * dx + H, l[1] - TS * dy + H, l[2] - TS * dz + H);
#pragma unroll
          for (int f = 0; f < kNumFields; ++f) v[f] += hb[f * kHaloCells];
        }
    if (touched) {
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) grid[f * n3 + gi] = v[f];
    }
  }
}

// FP64 grids: LDS accumulation with ds_add_f64 (~7 lanes/clk/CU on gfx950),
// same tiles and bank-sorted lane order as the FP32 kernel (a double spans
// two banks, so the key is the element index mod 32).
template <int TS, int NT, int NTAP, int DEG, bool kW>
__global__ __launch_bounds__(NT) void scatter_f64_kernel(
    const float4* __restrict__ sorted, const uint32_t* __restrict__ offset, double* __restrict__ grid,
    KeyParams kp, int64_t n_tiles, int64_t xcd_chunk, TapPoly tp, const Derived* dsrc, int bulk) {
  constexpr int H = kHaloLo<NTAP>;
  constexpr int E = TS + NTAP - 1;
  constexpr int VOL = E * E * E;
  constexpr int kPer = 4;
  constexpr int kSuper = kPer * NT;
  constexpr int kWaves = NT / 64;
  __shared__ double acc[kNumFields * VOL];
  __shared__ BankSort<NT, kPer> bs;
  const int64_t tile = tile_of_block(blockIdx.x, xcd_chunk);
  if (tile >= n_tiles) return;
  const uint32_t p0 = offset[tile], p1 = offset[tile + 1];
  if (p0 == p1) return;
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  for (int i = t; i < kNumFields * VOL; i += NT) acc[i] = 0.0;
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  if (bulk) {
    vb0 = dsrc->vb[0];
    vb1 = dsrc->vb[1];
    vb2 = dsrc->vb[2];
  }
  const int nt = kp.nt;
  const int tz = static_cast<int>(tile % nt);
  const int ty = static_cast<int>((tile / nt) % nt);
  const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
  const int ox = tx * TS, oy = ty * TS, oz = tz * TS;
  for (uint32_t c0 = p0; c0 < p1; c0 += kSuper) {
    const int m = static_cast<int>(min(static_cast<uint32_t>(kSuper), p1 - c0));
    if (t < 64) bs.cnt[t] = 0;
    __syncthreads();
    unsigned bank[kPer], slot[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int i = t + r * NT;
      if (i < m) {
        bank[r] = tap_origin<TS, NTAP>(rec_pos<kW>(sorted, static_cast<int64_t>(c0 + i)), kp, ox, oy, oz) & 31u;
        slot[r] = static_cast<unsigned>(atomicAdd(&bs.cnt[bank[r]], 1));
      }
    }
    __syncthreads();
    bank_scan<NT, kPer>(bs);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int i = t + r * NT;
      if (i < m) bs.idx[bs.cnt[bank[r]] + slot[r]] = static_cast<unsigned short>(i);
    }
    __syncthreads();
    const int slots = (m + 63) >> 6;
    const int lr = ((lane & 31) << 1) | (lane >> 5);
    for (int sl = wave; sl < slots; sl += kWaves) {
      const int q = lr * slots + sl;
      if (q >= m) continue;
      const uint32_t p = c0 + bs.idx[q];
      const float4 a = rec_pos<kW>(sorted, static_cast<int64_t>(p));
      const float4 v = rec_vel<kW>(sorted, static_cast<int64_t>(p));
      double wx[NTAP], wy[NTAP], wz[NTAP];
      const unsigned base = particle_taps<double, TS, NTAP, DEG>(a, kp, ox, oy, oz, tp, wx, wy, wz);
      const DepositQ<double> d = charges<double>(a, v, bulk, vb0, vb1, vb2);
      double qz[kNumFields][NTAP];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f)
#pragma unroll
        for (int j = 0; j < NTAP; ++j) qz[f][j] = d.q[f] * wz[j];
      double* accf[kNumFields] = {acc + base, acc + VOL + base, acc + 2 * VOL + base, acc + 3 * VOL + base};
#pragma unroll
      for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
        for (int jy = 0; jy < NTAP; ++jy) {
          const double wxy = wx[jx] * wy[jy];
#pragma unroll
          for (int f = 0; f < kNumFields; ++f)
#pragma unroll
            for (int jz = 0; jz < NTAP; ++jz) atomicAdd(accf[f] + (jx * E + jy) * E + jz, wxy * qz[f][jz]);
        }
      }
    }
    __syncthreads();
  }
  const int n = kp.n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  for (int i = t; i < VOL; i += NT) {
    const int ez = i % E, ey = (i / E) % E, ex = i / (E * E);
    const int gx = (ox + ex - H) & (n - 1);
    const int gy = (oy + ey - H) & (n - 1);
    const int gz = (oz + ez - H) & (n - 1);
    const int64_t gi = (static_cast<int64_t>(gx) * n + gy) * n + gz;
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) {
      const double val = acc[f * VOL + i];
      if (val != 0.0) atomicAdd(grid + f * n3 + gi, val);
    }
  }
}

KeyParams key_params(const Plan* p, const mps_catalog* c) {
  KeyParams kp;
  kp.scale = static_cast<double>(p->n) / c->box;
  kp.shift = kernel_shift(kernel_id(c->flags));
  kp.n = p->n;
  int ts = 0;
  while ((1 << ts) < p->tile) ++ts;
  kp.tshift = ts;
  kp.nt = p->n / p->tile;
  return kp;
}

// 16-byte aligned catalog arrays: the particle loads can be vectorised
bool vec_aligned(const mps_catalog* c) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(c->pos) | reinterpret_cast<uintptr_t>(c->vel) |
                      reinterpret_cast<uintptr_t>(c->weight);
  return (a & 15u) == 0;
}

int count_blocks(int64_t np) {
  int64_t b = (np + kCountThreads * kUnroll - 1) / (kCountThreads * kUnroll);
  return static_cast<int>(b < kMomentBlocks ? (b < 1 ? 1 : b) : kMomentBlocks);
}

// The two-level sort (for a catalog in random order, decided on the device):
// grids of more than kLdsTilesRandom tiles, whose tile histogram does not
// fit in LDS, when their memory holds the temporary records.  (On 512^3 the
// one-level LDS form is faster: with 6e7 particles count + permute take
// 3.0 ms against 3.4.)  *shift: tiles per bucket = 2^shift, about the
// square root of the tile count (buckets and tiles per bucket both at most
// kSortBuckets).
bool sort_two_level(const Plan* p, const mps_catalog* c, int* shift) {
  if (p->n_tiles <= kLdsTilesRandom) return false;
  int l = 0;
  while ((static_cast<int64_t>(1) << l) < p->n_tiles) ++l;
  *shift = l / 2;
  if ((p->n_tiles >> *shift) > kSortBuckets || (1 << *shift) > kSortBuckets) return false;
  const size_t rec = c->weight ? 2 * sizeof(float4) : 6 * sizeof(float);
  const size_t grid = static_cast<size_t>(kNumFields) * p->n * p->n * p->n * p->real_size;
  return rec * static_cast<size_t>(c->n_particles) <= grid;
}

}  // namespace

namespace {

// The count's kernels, the tile counters and the header already zero.
hipError_t launch_count_kernels(Plan* p, const mps_catalog* c, hipStream_t s) {
  const KeyParams kp = key_params(p, c);
  // the grid depends only on the particle count, so the moment sums of a
  // catalog are added in one order whatever else runs
  const int nb = count_blocks(c->n_particles);
  auto go = [&](auto has_w, auto use_lds, int mode) {
    constexpr bool kW = decltype(has_w)::value, kL = decltype(use_lds)::value;
    const size_t dyn = kL ? sizeof(uint32_t) * static_cast<size_t>(p->n_tiles) : 0;
    if (dyn > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&count_kernel<kW, kL>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn));
    count_kernel<kW, kL><<<nb, kCountThreads, dyn, s>>>(c->pos, c->vel, c->weight, c->n_particles, kp, p->n_tiles,
                                                        p->tile_count, p->moment_partials, p->d_header,
                                                        vec_aligned(c), mode, 0);
  };
  int shift = 0;
  const bool two = sort_two_level(p, c, &shift);
  auto both = [&](auto has_w) {
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (p->n_tiles <= kLdsTiles) {
      go(has_w, T_{}, -1);
    } else if (two) {  // random order: bucket histograms in LDS
      order_probe_kernel<<<kProbeChunks, kCountThreads, 0, s>>>(c->pos, c->n_particles, kp, p->d_header);
      go(has_w, F_{}, 0);
      constexpr bool kW = decltype(has_w)::value;
      const int64_t nbk = p->n_tiles >> shift;
      count_kernel<kW, true><<<nb, kCountThreads, sizeof(uint32_t) * nbk, s>>>(
          c->pos, c->vel, c->weight, c->n_particles, kp, nbk, p->tile_count, p->moment_partials, p->d_header,
          vec_aligned(c), 1, shift);
    } else if (p->n_tiles <= kLdsTilesRandom) {
      order_probe_kernel<<<kProbeChunks, kCountThreads, 0, s>>>(c->pos, c->n_particles, kp, p->d_header);
      go(has_w, F_{}, 0);
      go(has_w, T_{}, 1);
    } else {
      go(has_w, F_{}, -1);
    }
  };
  if (c->weight) both(std::true_type{});
  else both(std::false_type{});
  return hipGetLastError();
}

}  // namespace

hipError_t launch_count(Plan* p, const mps_catalog* c, hipStream_t s) {
  // zero-fill kernels rather than memset nodes, so that the sequence can be
  // captured in a HIP graph
  clear_kernel<uint32_t><<<static_cast<unsigned>((p->n_tiles + 255) / 256 < 4096 ? (p->n_tiles + 255) / 256 : 4096),
                           256, 0, s>>>(p->tile_count, p->n_tiles);
  clear_kernel<uint32_t><<<1, 256, 0, s>>>(reinterpret_cast<uint32_t*>(p->d_header),
                                           static_cast<int64_t>(sizeof(ResultHeader) / sizeof(uint32_t)));
  return launch_count_kernels(p, c, s);
}

hipError_t launch_sort_fused(Plan* p, const mps_catalog* c, hipStream_t s, bool clear_grid, bool* grid_cleared) {
  int shift = 0;
  const bool two = sort_two_level(p, c, &shift);
  // the two-level sort keeps temporary records in the grid
  *grid_cleared = clear_grid && !two;
  const int64_t hdr_words = static_cast<int64_t>(sizeof(ResultHeader) / sizeof(uint32_t));
  const int64_t grid_n = *grid_cleared ? static_cast<int64_t>(kNumFields) * p->n * p->n * p->n : 0;
  int64_t blocks = ((grid_n > p->n_tiles ? grid_n : p->n_tiles) + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  uint32_t* hdr = reinterpret_cast<uint32_t*>(p->d_header);
  if (p->prec == MPS_F32)
    clear3_kernel<float><<<static_cast<unsigned>(blocks), 256, 0, s>>>(p->tile_count, p->n_tiles, hdr, hdr_words,
                                                                       static_cast<float*>(p->grid), grid_n);
  else
    clear3_kernel<double><<<static_cast<unsigned>(blocks), 256, 0, s>>>(p->tile_count, p->n_tiles, hdr, hdr_words,
                                                                        static_cast<double*>(p->grid), grid_n);
  hipError_t e = launch_count_kernels(p, c, s);
  if (e != hipSuccess) return e;
  if (two) {
    if ((e = launch_derive(p, c, s)) != hipSuccess) return e;
    if ((e = launch_scan(p, c, s)) != hipSuccess) return e;
  } else {
    derive_scan_kernel<<<1, 1024, 0, s>>>(p->moment_partials, count_blocks(c->n_particles), p->d_header,
                                          (c->flags & MPS_BULKFLOW_SUBTRACT) ? 1 : 0, p->tile_count, p->n_tiles,
                                          p->tile_offset, p->tile_cursor);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return launch_permute(p, c, s);
}

hipError_t launch_derive(Plan* p, const mps_catalog* c, hipStream_t s) {
  derive_kernel<<<1, kMomentBlocks, 0, s>>>(p->moment_partials, count_blocks(c->n_particles), p->d_header,
                                            (c->flags & MPS_BULKFLOW_SUBTRACT) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_scan(Plan* p, const mps_catalog* c, hipStream_t s) {
  int shift = 0;
  if (sort_two_level(p, c, &shift)) {
    // spatial order: the tiles; random order: the buckets (starts in
    // tile_cursor[0 .. B], pass A's cursors in tile_count[B .. 2B))
    const int64_t nbk = p->n_tiles >> shift;
    scan_kernel<<<1, 1024, 0, s>>>(p->tile_count, p->n_tiles, p->tile_offset, p->tile_cursor, p->d_header, 0);
    scan_kernel<<<1, 1024, 0, s>>>(p->tile_count, nbk, p->tile_cursor, p->tile_count + nbk, p->d_header, 1);
  } else {
    scan_kernel<<<1, 1024, 0, s>>>(p->tile_count, p->n_tiles, p->tile_offset, p->tile_cursor, p->d_header, -1);
  }
  return hipGetLastError();
}

hipError_t launch_permute(Plan* p, const mps_catalog* c, hipStream_t s) {
  const KeyParams kp = key_params(p, c);
  const int nb = count_blocks(c->n_particles);
  auto go = [&](auto has_w, auto use_lds, int mode) {
    constexpr bool kW = decltype(has_w)::value, kL = decltype(use_lds)::value;
    const size_t dyn = kL ? sizeof(uint32_t) * static_cast<size_t>(p->n_tiles) : 0;
    if (dyn > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&permute_kernel<kW, kL>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn));
    permute_kernel<kW, kL><<<nb, kCountThreads, dyn, s>>>(c->pos, c->vel, c->weight, c->n_particles, kp,
                                                          p->n_tiles, p->tile_cursor, p->sorted, vec_aligned(c),
                                                          p->d_header, mode);
  };
  int shift = 0;
  const bool two = sort_two_level(p, c, &shift);
  auto both = [&](auto has_w) {
    using T_ = std::true_type;
    using F_ = std::false_type;
    constexpr bool kW = decltype(has_w)::value;
    if (p->n_tiles <= kLdsTiles) {
      go(has_w, T_{}, -1);
    } else if (two) {  // the order probe ran with the count; temporary records in the grid
      go(has_w, F_{}, 0);
      const int nbk = static_cast<int>(p->n_tiles >> shift);
      float4* temp = static_cast<float4*>(p->grid);
      const int64_t chunks = (c->n_particles + kSortChunk - 1) / kSortChunk;
      const int64_t cap = 2 * static_cast<int64_t>(p->num_cus);
      sort_pass_a_kernel<kW><<<static_cast<unsigned>(chunks < cap ? (chunks < 1 ? 1 : chunks) : cap), kSortThreads, 0,
                               s>>>(c->pos, c->vel, c->weight, c->n_particles, kp, shift, nbk, p->tile_count + nbk,
                                    temp, p->d_header);
      sort_pass_b_kernel<kW><<<static_cast<unsigned>(nbk), kSortThreads, 0, s>>>(
          temp, p->tile_cursor, kp, shift, nbk, p->n_tiles, p->tile_offset, p->sorted, p->d_header);
    } else if (p->n_tiles <= kLdsTilesRandom) {  // the order probe ran with the count
      go(has_w, F_{}, 0);
      go(has_w, T_{}, 1);
    } else {
      go(has_w, F_{}, -1);
    }
  };
  if (c->weight) both(std::true_type{});
  else both(std::false_type{});
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

// The integer nearest to x (|x| < 2^51) as 64-bit two's complement: adding
// 1.5 * 2^52 rounds x to an integer held in the low mantissa bits.
__device__ __forceinline__ unsigned long long fixed64(double x) {
  constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
  return static_cast<unsigned long long>(__double_as_longlong(x + kMagic) - __double_as_longlong(kMagic));
}

// FP64 grids on 16^3 tiles.  Four FP64 fields of a 21^3 block would need
// 296 KB of LDS, so the block holds two at a time (148 KB, one workgroup per
// CU) and each tile is deposited and flushed twice: (rho, rho v_x), then
// (rho v_y, rho v_z).  Against 8^3 tiles (one 13^3 block per tile, 4.3x the
// tile's cells) the flush's global FP64 atomics fall to 2.3x the tile's
// cells.  Persistent over the same tile queues as the FP32 kernel; lanes in
// the same bank-sorted order.
//
// The LDS sums are 64-bit fixed point, added with ds_add_u64 (9.4 lanes/clk
// per CU against 7.2 for ds_add_f64) and exact whatever the order.  Field f
// of a tile is scaled so that one deposit, at most max|q_f| K^3 (K the
// largest tap bound), maps to at most 2^50 and a cell's sum, at most
// cnt_tile times that, to at most 2^62; a deposit x becomes the integer
// nearest to it as the bits of x + 1.5 * 2^52 minus those of 1.5 * 2^52.
// For tiles of up to 4096 particles the unit is 2^-50 of the largest
// possible deposit, the resolution of the FP64 products themselves.
//
// Dense tiles (truncated BL3, scratch in pw) take the FP32 atomic form's
// paired deposits (see scatter_fixed_kernel): one cell sort and job list per
// tile serve both passes.  The FP64 pair sum rounds at 2^-53 of the pair,
// below the fixed-point unit of the largest deposit, so which particles pair
// moves a cell's integer sum by at most a unit here and there.
template <int TS, int NT, int NTAP, int DEG, bool kW>
__global__ __launch_bounds__(NT) void scatter_f64_pair_kernel(
    const float4* __restrict__ sorted, const uint32_t* __restrict__ offset, double* __restrict__ grid,
    KeyParams kp, int64_t n_tiles, TileQueues tq, TapPoly tp, TapBound kb, const Derived* dsrc, int bulk,
    PairWork pw) {
  constexpr int H = kHaloLo<NTAP>;
  constexpr int E = TS + NTAP - 1;
  constexpr int VOL = E * E * E;
  constexpr int kPer = NT == 512 ? 8 : 6;
  constexpr int kSuper = kPer * NT;
  constexpr int kWaves = NT / 64;
  __shared__ unsigned long long acc[2 * VOL];
  __shared__ BankSort<NT, kPer> bs;
  __shared__ long long s_tile;
  // 512 threads (256 registers per lane) for the paired path's two
  // particles' FP64 weights
  constexpr bool kPairOK = TS == 16 && NT == 512 && NTAP == 6 && DEG == 3;
  constexpr int kCellWords = TS * TS * TS / 2;
  static_assert(!kPairOK || kCellWords * 4 <= NT * kPer * 2, "cell counts alias the bank-sort index array");
  static_assert(!kPairOK || kPairCap <= 2 * VOL, "the paired sort's arrays fit the accumulator block");
  unsigned* ccnt = reinterpret_cast<unsigned*>(bs.idx);
  unsigned* const words = reinterpret_cast<unsigned*>(acc);
  __shared__ unsigned wsum[kWaves];
  __shared__ int s_slot;  // paired deposits: the next wave slot to claim
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  if (bulk) {
    vb0 = dsrc->vb[0];
    vb1 = dsrc->vb[1];
    vb2 = dsrc->vb[2];
  }
  double kmax = 0.0;
#pragma unroll
  for (int j = 0; j < NTAP; ++j) kmax = fmax(kmax, static_cast<double>(kb.k[j]));
  const double kmax3 = kmax * kmax * kmax;
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int nt = kp.nt;
  const int n = kp.n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  for (int i = t; i < 2 * VOL; i += NT) acc[i] = 0ull;
  if constexpr (kPairOK)
    for (int i = t; i < kCellWords; i += NT) ccnt[i] = 0u;
  int64_t tile = next_tile<NT>(tq, n_tiles, &s_tile);
  while (tile >= 0) {
    const uint32_t p0 = offset[tile], p1 = offset[tile + 1];
    if (p0 == p1) {  // nothing to deposit or flush (uniform across the workgroup)
      tile = next_tile<NT>(tq, n_tiles, &s_tile);
      continue;
    }
    const int tz = static_cast<int>(tile % nt);
    const int ty = static_cast<int>((tile / nt) % nt);
    const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
    const int ox = tx * TS, oy = ty * TS, oz = tz * TS;
    const uint32_t cnt = p1 - p0;
    const bool paired = kPairOK && cnt > 128u && pw.base != nullptr && cnt <= static_cast<uint32_t>(kPairCap) &&
                        static_cast<int>(blockIdx.x) < pw.blocks;
    uint32_t* const pjob = paired ? pw.base + static_cast<int64_t>(blockIdx.x) * kPairCap : nullptr;
    int n_pair = 0;
    if (paired) {  // cell keys (registers, then the accumulator words of the second pair), sort, jobs
      const int m0 = static_cast<int>(min(static_cast<uint32_t>(kSuper), cnt));
      unsigned key0[kPer];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        key0[r] = 0u;
        if (t + r * NT < m0)
          key0[r] = cell_rank(tap_origin<TS, NTAP>(rec_pos<kW>(sorted, static_cast<int64_t>(p0 + t + r * NT)), kp,
                                                   ox, oy, oz),
                              ccnt);
      }
      for (uint32_t i = static_cast<uint32_t>(m0) + t; i < cnt; i += NT)
        words[2 * VOL + i] = cell_rank(tap_origin<TS, NTAP>(rec_pos<kW>(sorted, static_cast<int64_t>(p0 + i)), kp,
                                                            ox, oy, oz),
                                       ccnt);
      __syncthreads();
      n_pair = pair_jobs<NT, kPer, E>(words, ccnt, wsum, bs, key0, m0, cnt, pjob);
    }
    for (int pass = 0; pass < 2; ++pass) {
      // fixed-point scales of this pass's two fields (uniform): one deposit
      // at most 2^50 (the rounding below needs |x| < 2^51), a cell's sum of
      // the tile's deposits at most 2^62
      double scl[2], inv[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        // catalog-wide bound of |q| for the field's charges (with the bulk
        // term when the assign diagnostic deposits v - v_b)
        const int f = 2 * pass + k;
        const double vbf = f == 1 ? vb0 : (f == 2 ? vb1 : vb2);
        const double qmax = dsrc->qmax[f] + (bulk && f > 0 ? dsrc->qmax[0] * fabs(vbf) : 0.0);
        const double dep = qmax * kmax3 * 1.0001;
        const double cell = static_cast<double>(p1 - p0) * dep;
        scl[k] = dep > 0.0 ? fmin(0x1p50 / dep, 0x1p62 / cell) : 0.0;
        inv[k] = dep > 0.0 ? 1.0 / scl[k] : 0.0;
      }
      // paired: the job list's wave slots, pairs then singles
      if (paired) {
        const int n_single = static_cast<int>(cnt) - 2 * n_pair;
        const int wp = (n_pair + 63) >> 6, ws = (n_single + 63) >> 6;
        const int lr = ((lane & 31) << 1) | (lane >> 5);
        if (t == 0) s_slot = kWaves;
        __syncthreads();
        // each wave claims its next slot when it is done with one
        for (int sl = wave; sl < wp + ws;) {
          const bool two = sl < wp;
          const int q = two ? lr * wp + sl : lr * ws + (sl - wp);
          if (q < (two ? n_pair : n_single)) {
            const unsigned jd = pjob[two ? q : n_pair + q];
            const uint32_t pa = p0 + (jd & 0xffffu);
            const float4 a0 = rec_pos<kW>(sorted, static_cast<int64_t>(pa));
            const float4 v0 = rec_vel<kW>(sorted, static_cast<int64_t>(pa));
            double wx0[NTAP], wy0[NTAP], wz0[NTAP];
            const unsigned base = particle_taps<double, TS, NTAP, DEG>(a0, kp, ox, oy, oz, tp, wx0, wy0, wz0);
            const DepositQ<double> d0 = charges<double>(a0, v0, bulk, vb0, vb1, vb2);
            const double qa0 = (pass ? d0.q[2] : d0.q[0]) * scl[0];
            const double qa1 = (pass ? d0.q[3] : d0.q[1]) * scl[1];
            unsigned long long* accf[2] = {acc + base, acc + VOL + base};
            if (two) {
              const uint32_t pb = p0 + (jd >> 16);
              const float4 a1 = rec_pos<kW>(sorted, static_cast<int64_t>(pb));
              const float4 v1 = rec_vel<kW>(sorted, static_cast<int64_t>(pb));
              double wx1[NTAP], wy1[NTAP], wz1[NTAP];
              const unsigned base1 = particle_taps<double, TS, NTAP, DEG>(a1, kp, ox, oy, oz, tp, wx1, wy1, wz1);
              const bool up = base1 != base;  // else one cell
              double wzb[NTAP + 1];  // the second particle's z weights on the pair's cells
              wzb[0] = up ? 0.0 : wz1[0];
#pragma unroll
              for (int j = 1; j < NTAP; ++j) wzb[j] = up ? wz1[j - 1] : wz1[j];
              wzb[NTAP] = up ? wz1[NTAP - 1] : 0.0;
              const DepositQ<double> d1 = charges<double>(a1, v1, bulk, vb0, vb1, vb2);
              const double qb0 = (pass ? d1.q[2] : d1.q[0]) * scl[0];
              const double qb1 = (pass ? d1.q[3] : d1.q[1]) * scl[1];
#pragma unroll
              for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
                for (int jy = 0; jy < NTAP; ++jy) {
                  const double wa = wx0[jx] * wy0[jy], wb = wx1[jx] * wy1[jy];
#pragma unroll
                  for (int k = 0; k < 2; ++k) {
                    const double ta = wa * (k ? qa1 : qa0), tb = wb * (k ? qb1 : qb0);
                    unsigned long long* row = accf[k] + (jx * E + jy) * E;
#pragma unroll
                    for (int jz = 0; jz < NTAP; ++jz) atomicAdd(row + jz, fixed64(fma(tb, wzb[jz], ta * wz0[jz])));
                    if (up) atomicAdd(row + NTAP, fixed64(tb * wzb[NTAP]));
                  }
                }
              }
            } else {
#pragma unroll
              for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
                for (int jy = 0; jy < NTAP; ++jy) {
                  const double wa = wx0[jx] * wy0[jy];
#pragma unroll
                  for (int k = 0; k < 2; ++k) {
                    const double ta = wa * (k ? qa1 : qa0);
#pragma unroll
                    for (int jz = 0; jz < NTAP; ++jz)
                      atomicAdd(accf[k] + (jx * E + jy) * E + jz, fixed64(ta * wz0[jz]));
                  }
                }
              }
            }
          }
          int next = 0;
          if (lane == 0) next = atomicAdd(&s_slot, 1);
          sl = __shfl(next, 0);
        }
        __syncthreads();
      } else {
      // a tile of one super-chunk keeps its bank order for the second pass
      const bool resort = pass == 0 || p1 - p0 > static_cast<uint32_t>(kSuper);
      for (uint32_t c0 = p0; c0 < p1; c0 += kSuper) {
        const int m = static_cast<int>(min(static_cast<uint32_t>(kSuper), p1 - c0));
        if (resort) {
          if (t < 64) bs.cnt[t] = 0;
          __syncthreads();
          unsigned bank[kPer], slot[kPer];
#pragma unroll
          for (int r = 0; r < kPer; ++r) {
            const int i = t + r * NT;
            if (i < m) {
              bank[r] = tap_origin<TS, NTAP>(rec_pos<kW>(sorted, static_cast<int64_t>(c0 + i)), kp, ox, oy, oz) & 31u;
              slot[r] = static_cast<unsigned>(atomicAdd(&bs.cnt[bank[r]], 1));
            }
          }
          __syncthreads();
          bank_scan<NT, kPer>(bs);
          __syncthreads();
#pragma unroll
          for (int r = 0; r < kPer; ++r) {
            const int i = t + r * NT;
            if (i < m) bs.idx[bs.cnt[bank[r]] + slot[r]] = static_cast<unsigned short>(i);
          }
          __syncthreads();
        }
        const int slots = (m + 63) >> 6;
        const int lr = ((lane & 31) << 1) | (lane >> 5);
        for (int sl = wave; sl < slots; sl += kWaves) {
          const int q = lr * slots + sl;
          if (q >= m) continue;
          const uint32_t p = c0 + bs.idx[q];
          const float4 a = rec_pos<kW>(sorted, static_cast<int64_t>(p));
          const float4 v = rec_vel<kW>(sorted, static_cast<int64_t>(p));
          double wx[NTAP], wy[NTAP], wz[NTAP];
          const unsigned base = particle_taps<double, TS, NTAP, DEG>(a, kp, ox, oy, oz, tp, wx, wy, wz);
          const DepositQ<double> d = charges<double>(a, v, bulk, vb0, vb1, vb2);
          const double q0 = (pass ? d.q[2] : d.q[0]) * scl[0];
          const double q1 = (pass ? d.q[3] : d.q[1]) * scl[1];
          double qz[2][NTAP];
#pragma unroll
          for (int j = 0; j < NTAP; ++j) {
            qz[0][j] = q0 * wz[j];
            qz[1][j] = q1 * wz[j];
          }
          unsigned long long* accf[2] = {acc + base, acc + VOL + base};
#pragma unroll
          for (int jx = 0; jx < NTAP; ++jx) {
#pragma unroll
            for (int jy = 0; jy < NTAP; ++jy) {
              const double wxy = wx[jx] * wy[jy];
#pragma unroll
              for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int jz = 0; jz < NTAP; ++jz) atomicAdd(accf[k] + (jx * E + jy) * E + jz, fixed64(wxy * qz[k][jz]));
            }
          }
        }
        __syncthreads();
      }
      }  // unpaired
      // flush this pass's two fields, clearing the block for the next
      for (int i = t; i < VOL; i += NT) {
        const int ez = i % E, ey = (i / E) % E, ex = i / (E * E);
        const int gx = (ox + ex - H) & (n - 1);
        const int gy = (oy + ey - H) & (n - 1);
        const int gz = (oz + ez - H) & (n - 1);
        const int64_t gi = (static_cast<int64_t>(gx) * n + gy) * n + gz;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const long long v = static_cast<long long>(acc[k * VOL + i]);
          acc[k * VOL + i] = 0ull;
          if (v != 0) atomicAdd(grid + (2 * pass + k) * n3 + gi, static_cast<double>(v) * inv[k]);
        }
      }
      __syncthreads();
    }
    if constexpr (kPairOK)  // the unpaired path's bank sort wrote over the counts
      for (int i = t; i < kCellWords; i += NT) ccnt[i] = 0u;
    tile = next_tile<NT>(tq, n_tiles, &s_tile);
  }
}

// FP64 grids of sparse catalogs, owner-computes form: the FP32 form's
// candidate search and in-region list (see scatter_gather_kernel), with the
// FP64 path's 64-bit fixed point (one field per ds_add_u64, all four fields
// of the tile's 16^3 cells in LDS: 128 KB, one workgroup per CU).  The
// scale of a field maps the largest possible deposit, max|q| K^3, to 2^50
// and caps a cell's sum over the n_in in-region particles below 2^62, as the
// atomic FP64 form does for a tile's particles; no per-cell bound is needed.
template <int NT, bool kW>
__global__ __launch_bounds__(NT) void scatter_gather64_kernel(
    const float4* __restrict__ sorted, const uint32_t* __restrict__ offset, double* __restrict__ grid, KeyParams kp,
    int64_t n_tiles, TileQueues tq, TapPoly tp, TapBound kb, const Derived* dsrc, int bulk) {
  constexpr int TS = 16, NTAP = 6, DEG = 3;
  constexpr int H = kHaloLo<NTAP>;
  constexpr int HI = NTAP - 1 - H;
  constexpr int CV = TS * TS * TS;
  constexpr int kWaves = NT / 64;
  constexpr int kRing = 128;
  constexpr int kList = kWaves * kRing;  // the ring aliases the list
  __shared__ unsigned long long acc[kNumFields * CV];
  __shared__ uint32_t lbuf[kList];
  __shared__ int list_n;
  __shared__ int nb_first[28];
  __shared__ uint32_t nb_start[27];
  __shared__ long long s_tile;
  uint32_t* list_rec = lbuf;
  int (*ring)[kRing] = reinterpret_cast<int (*)[kRing]>(lbuf);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  if (bulk) {
    vb0 = dsrc->vb[0];
    vb1 = dsrc->vb[1];
    vb2 = dsrc->vb[2];
  }
  double kmax = 0.0;
#pragma unroll
  for (int j = 0; j < NTAP; ++j) kmax = fmax(kmax, static_cast<double>(kb.k[j]));
  const double kmax3 = kmax * kmax * kmax;
  double dep[kNumFields];  // the largest possible deposit per field
#pragma unroll
  for (int f = 0; f < kNumFields; ++f) {
    const double vbf = f == 1 ? vb0 : (f == 2 ? vb1 : vb2);
    dep[f] = (dsrc->qmax[f] + (bulk && f > 0 ? dsrc->qmax[0] * fabs(vbf) : 0.0)) * kmax3 * 1.0001;
  }
  const int nt = kp.nt, n = kp.n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  int ox = 0, oy = 0, oz = 0;
  // a record's position, cell relative to the tile origin (the periodic
  // offset in [-N/2, N/2), unambiguous for N >= 64) and fractions; true in
  // the source region
  auto record_cell = [&](uint32_t rec, float4* a, int* rc, double* fr) -> bool {
    *a = rec_pos<kW>(sorted, static_cast<int64_t>(rec));
    const int o[3] = {ox, oy, oz};
    const float xs[3] = {a->x, a->y, a->z};
    bool in = true;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      bool ok;
      const int c = locate(xs[ax], kp.scale, kp.shift, kp.n, &fr[ax], &ok);
      rc[ax] = ((c - o[ax] + n / 2) & (n - 1)) - n / 2;
      in = in && rc[ax] >= -HI && rc[ax] < TS + H;
    }
    return in;
  };
  auto candidate = [&](int i, float4* a, uint32_t* rec, int* rc, double* fr) -> bool {
    int lo = 0, hi = 27;  // nb_first[lo] <= i < nb_first[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nb_first[mid] <= i) lo = mid; else hi = mid;
    }
    *rec = nb_start[lo] + static_cast<uint32_t>(i - nb_first[lo]);
    return record_cell(*rec, a, rc, fr);
  };

  for (int i = t; i < kNumFields * CV; i += NT) acc[i] = 0ull;
  int64_t tile = next_tile<NT>(tq, n_tiles, &s_tile);
  while (tile >= 0) {
    const int tz = static_cast<int>(tile % nt);
    const int ty = static_cast<int>((tile / nt) % nt);
    const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
    ox = tx * TS;
    oy = ty * TS;
    oz = tz * TS;
    if (t < 27) {
      const int dx = t / 9 - 1, dy = (t / 3) % 3 - 1, dz = t % 3 - 1;
      const int64_t tn = (static_cast<int64_t>((tx + dx + nt) % nt) * nt + (ty + dy + nt) % nt) * nt +
                         (tz + dz + nt) % nt;
      nb_start[t] = offset[tn];
      nb_first[t + 1] = static_cast<int>(offset[tn + 1] - offset[tn]);
    }
    __syncthreads();
    if (t == 0) {
      nb_first[0] = 0;
      for (int r = 0; r < 27; ++r) nb_first[r + 1] += nb_first[r];
      list_n = 0;
    }
    __syncthreads();
    const int total = nb_first[27];
    double inv[kNumFields] = {0.0, 0.0, 0.0, 0.0};
    if (total > 0) {  // uniform; otherwise the tile is written with zeros
      // pass 1: the in-region candidates (up to kList listed)
      for (int b = wave * 64; b < total; b += NT) {  // uniform within the wave
        const int i = b + lane;
        float4 a;
        uint32_t rec;
        int rc[3];
        double fr[3];
        const bool in = i < total && candidate(i, &a, &rec, rc, fr);
        const unsigned long long mask = __ballot(in);
        int base = 0;
        if (lane == 0 && mask) base = atomicAdd(&list_n, __popcll(mask));
        base = __shfl(base, 0);
        if (in) {
          const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
          if (slot < kList) list_rec[slot] = rec;
        }
      }
      __syncthreads();
      const int n_in = list_n;
      const bool fits = n_in <= kList;  // uniform
      double scl[kNumFields];
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) {
        scl[f] = dep[f] > 0.0 ? fmin(0x1p50 / dep[f], 0x1p62 / (static_cast<double>(n_in) * dep[f])) : 0.0;
        inv[f] = dep[f] > 0.0 ? 1.0 / scl[f] : 0.0;
      }
      // pass 2: one in-region particle's deposits of the taps that land in
      // the tile
      auto deposit_one = [&](const float4& a, uint32_t rec, const int* rc, const double* fr) {
        double wx[NTAP], wy[NTAP], wz[NTAP];
#pragma unroll
        for (int j = 0; j < NTAP; ++j) {
          wx[j] = tap_weight<DEG>(tp, j, fr[0]);
          wy[j] = tap_weight<DEG>(tp, j, fr[1]);
          wz[j] = tap_weight<DEG>(tp, j, fr[2]);
        }
        const DepositQ<double> d = charges<double>(a, rec_vel<kW>(sorted, static_cast<int64_t>(rec)), bulk, vb0, vb1, vb2);
        double qs[kNumFields];
#pragma unroll
        for (int f = 0; f < kNumFields; ++f) qs[f] = d.q[f] * scl[f];
#pragma unroll
        for (int jx = 0; jx < NTAP; ++jx) {
          const int gx = rc[0] + jx - H;
          if (gx < 0 || gx >= TS) continue;
#pragma unroll
          for (int jy = 0; jy < NTAP; ++jy) {
            const int gy = rc[1] + jy - H;
            if (gy < 0 || gy >= TS) continue;
            const double wxy = wx[jx] * wy[jy];
            const int row = (gx * TS + gy) * TS;
#pragma unroll
            for (int jz = 0; jz < NTAP; ++jz) {
              const int gz = rc[2] + jz - H;
              if (gz < 0 || gz >= TS) continue;
              const double w = wxy * wz[jz];
#pragma unroll
              for (int f = 0; f < kNumFields; ++f) atomicAdd(acc + f * CV + row + gz, fixed64(w * qs[f]));
            }
          }
        }
      };
      if (fits) {
        for (int j = t; j < n_in; j += NT) {
          const uint32_t rec = list_rec[j];
          float4 a;
          int rc[3];
          double fr[3];
          (void)record_cell(rec, &a, rc, fr);
          deposit_one(a, rec, rc, fr);
        }
      } else {  // the list overflowed and is not read: the ring takes its place
        auto deposit = [&](int head, int m) {
          if (lane >= m) return;
          float4 a;
          uint32_t rec;
          int rc[3];
          double fr[3];
          (void)candidate(ring[wave][(head + lane) & (kRing - 1)], &a, &rec, rc, fr);
          deposit_one(a, rec, rc, fr);
        };
        int head = 0, queued = 0;  // uniform within the wave
        for (int b = wave * 64; b < total; b += NT) {
          const int i = b + lane;
          float4 a;
          uint32_t rec;
          int rc[3];
          double fr[3];
          const bool in = i < total && candidate(i, &a, &rec, rc, fr);
          const unsigned long long mask = __ballot(in);
          if (in) {
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            ring[wave][(head + queued + rank) & (kRing - 1)] = i;
          }
          queued += __popcll(mask);
          __builtin_amdgcn_wave_barrier();
          if (queued >= 64) {
            deposit(head, 64);
            head = (head + 64) & (kRing - 1);
            queued -= 64;
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (queued > 0) deposit(head, queued);
      }
      __syncthreads();
    }
    // store the tile's cells, clearing the block
    for (int i = t; i < CV; i += NT) {
      const int64_t gi = (static_cast<int64_t>(ox + i / (TS * TS)) * n + oy + (i / TS) % TS) * n + oz + i % TS;
#pragma unroll
      for (int f = 0; f < kNumFields; ++f) {
        const long long v = static_cast<long long>(acc[f * CV + i]);
        acc[f * CV + i] = 0ull;
        grid[f * n3 + gi] = static_cast<double>(v) * inv[f];
      }
    }
    tile = next_tile<NT>(tq, n_tiles, &s_tile);
  }
}

template <int NTAP, int DEG, bool kW>
hipError_t launch_scatter_taps(Plan* p, const mps_catalog* c, hipStream_t s, int bulk, const TapPoly& tp,
                               const TapBound& tb) {
  const KeyParams kp = key_params(p, c);
  const int64_t xcd_chunk = (p->n_tiles % 8 == 0) ? p->n_tiles / 8 : 0;
  const Derived* dsrc = &p->d_header->d;
  if (p->prec == MPS_F32) {
    TileQueues tq;
    tq.counter = p->tile_queue;
    tq.nq = xcd_chunk > 0 ? 8 : 1;
    tq.per_queue = xcd_chunk > 0 ? xcd_chunk : p->n_tiles;
    clear_kernel<uint32_t><<<1, 64, 0, s>>>(p->tile_queue, 8);
    const ScatterCat one{p->sorted, p->tile_offset, static_cast<float*>(p->grid), kp, dsrc, bulk};
    if (p->tile == 16) {
      // one workgroup per CU (the LDS holds one), never more than the tiles
      const int64_t blocks = p->n_tiles < p->num_cus ? p->n_tiles : p->num_cus;
      scatter_fixed_kernel<16, 1024, NTAP, DEG, kW, false><<<static_cast<unsigned>(blocks), 1024, 0, s>>>(
          one, nullptr, nullptr, 1, p->n_tiles, tq, tp, tb, PairWork{p->pair_scratch, p->pair_blocks});
    } else {
      const int64_t cap = 4 * static_cast<int64_t>(p->num_cus);
      const int64_t blocks = p->n_tiles < cap ? p->n_tiles : cap;
      scatter_fixed_kernel<8, 512, NTAP, DEG, kW, false><<<static_cast<unsigned>(blocks), 512, 0, s>>>(
          one, nullptr, nullptr, 1, p->n_tiles, tq, tp, tb, PairWork{nullptr, 0});
    }
  } else if (p->tile == 16) {
    TileQueues tq;
    tq.counter = p->tile_queue;
    tq.nq = xcd_chunk > 0 ? 8 : 1;
    tq.per_queue = xcd_chunk > 0 ? xcd_chunk : p->n_tiles;
    clear_kernel<uint32_t><<<1, 64, 0, s>>>(p->tile_queue, 8);
    const int64_t blocks = p->n_tiles < p->num_cus ? p->n_tiles : p->num_cus;
    if constexpr (NTAP == 6 && DEG == 3)  // paired deposits: 512 threads
      scatter_f64_pair_kernel<16, 512, NTAP, DEG, kW><<<static_cast<unsigned>(blocks), 512, 0, s>>>(
          p->sorted, p->tile_offset, static_cast<double*>(p->grid), kp, p->n_tiles, tq, tp, tb, dsrc, bulk,
          PairWork{p->pair_scratch, p->pair_blocks});
    else
      scatter_f64_pair_kernel<16, 1024, NTAP, DEG, kW><<<static_cast<unsigned>(blocks), 1024, 0, s>>>(
          p->sorted, p->tile_offset, static_cast<double*>(p->grid), kp, p->n_tiles, tq, tp, tb, dsrc, bulk,
          PairWork{nullptr, 0});
  } else {
    scatter_f64_kernel<8, 512, NTAP, DEG, kW><<<static_cast<unsigned>(p->n_tiles), 512, 0, s>>>(
        p->sorted, p->tile_offset, static_cast<double*>(p->grid), kp, p->n_tiles, xcd_chunk, tp, dsrc, bulk);
  }
  return hipGetLastError();
}

template <bool kW>
hipError_t launch_scatter_kernel(Plan* p, const mps_catalog* c, hipStream_t s, int bulk, int k, const TapPoly& tp,
                                 const TapBound& tb) {
  switch (k) {
    case 1: return launch_scatter_taps<1, 0, kW>(p, c, s, bulk, tp, tb);
    case 2: return launch_scatter_taps<2, 1, kW>(p, c, s, bulk, tp, tb);
    case 3: return launch_scatter_taps<3, 2, kW>(p, c, s, bulk, tp, tb);
    case 4: return launch_scatter_taps<4, 3, kW>(p, c, s, bulk, tp, tb);
    case 5: return launch_scatter_taps<5, 4, kW>(p, c, s, bulk, tp, tb);
    case 6: return launch_scatter_taps<6, 5, kW>(p, c, s, bulk, tp, tb);
    case kKernelBl3Quadratic: return launch_scatter_taps<6, kDegSplit2, kW>(p, c, s, bulk, tp, tb);
    default: return launch_scatter_taps<6, 3, kW>(p, c, s, bulk, tp, tb);
  }
}

// bulk: 1 = deposit w (v - v_b) (only the assign diagnostic asks for it; the
// estimator removes the bulk flow in Fourier space, p' = p - v_b delta).
hipError_t launch_scatter_impl(Plan* p, const mps_catalog* c, hipStream_t s, int bulk) {
  const int k = kernel_id(c->flags);
  const TapPoly& tp = p->taps[k];
  const TapBound& tb = p->tap_bound[k];
  const int form = scatter_form(p, c);
  if (form == kFormGather && p->prec == MPS_F64) {
    // persistent, one workgroup per CU (the LDS holds one), over every tile
    TileQueues tq;
    const int64_t xcd_chunk = (p->n_tiles % 8 == 0) ? p->n_tiles / 8 : 0;
    tq.counter = p->tile_queue;
    tq.nq = xcd_chunk > 0 ? 8 : 1;
    tq.per_queue = xcd_chunk > 0 ? xcd_chunk : p->n_tiles;
    clear_kernel<uint32_t><<<1, 64, 0, s>>>(p->tile_queue, 8);
    const KeyParams kp = key_params(p, c);
    const unsigned blocks = static_cast<unsigned>(p->n_tiles < p->num_cus ? p->n_tiles : p->num_cus);
    double* g = static_cast<double*>(p->grid);
    if (c->weight)
      scatter_gather64_kernel<1024, true><<<blocks, 1024, 0, s>>>(p->sorted, p->tile_offset, g, kp, p->n_tiles, tq,
                                                                   tp, tb, &p->d_header->d, bulk);
    else
      scatter_gather64_kernel<1024, false><<<blocks, 1024, 0, s>>>(p->sorted, p->tile_offset, g, kp, p->n_tiles, tq,
                                                                    tp, tb, &p->d_header->d, bulk);
    return hipGetLastError();
  }
  if (form != kFormAtomic) {
    TileQueues tq;
    const int64_t xcd_chunk = (p->n_tiles % 8 == 0) ? p->n_tiles / 8 : 0;
    tq.counter = p->tile_queue;
    tq.nq = xcd_chunk > 0 ? 8 : 1;
    tq.per_queue = xcd_chunk > 0 ? xcd_chunk : p->n_tiles;
    clear_kernel<uint32_t><<<1, 64, 0, s>>>(p->tile_queue, 8);
    ScatterCat one = scatter_cat(p, c);
    one.bulk = bulk;
    if (form == kFormGather) {
      // persistent, two workgroups per CU (the LDS holds two), over every
      // tile: each writes its own cells, zeros included
      const int64_t cap = 2 * static_cast<int64_t>(p->num_cus);
      const unsigned blocks = static_cast<unsigned>(p->n_tiles < cap ? p->n_tiles : cap);
      if (c->weight)
        scatter_gather_kernel<kGatherThreads, true, false><<<blocks, kGatherThreads, 0, s>>>(
            one, nullptr, nullptr, 1, p->n_tiles, tq, tp, tb);
      else
        scatter_gather_kernel<kGatherThreads, false, false><<<blocks, kGatherThreads, 0, s>>>(
            one, nullptr, nullptr, 1, p->n_tiles, tq, tp, tb);
    } else {
      const unsigned blocks = static_cast<unsigned>(p->n_tiles < p->num_cus ? p->n_tiles : p->num_cus);
      if (c->weight)
        scatter_fixed_kernel<16, 1024, 6, 3, true, false, true><<<blocks, 1024, 0, s>>>(
            one, nullptr, nullptr, 1, p->n_tiles, tq, tp, tb, PairWork{p->pair_scratch, p->pair_blocks});
      else
        scatter_fixed_kernel<16, 1024, 6, 3, false, false, true><<<blocks, 1024, 0, s>>>(
            one, nullptr, nullptr, 1, p->n_tiles, tq, tp, tb, PairWork{p->pair_scratch, p->pair_blocks});
      halo_fixup_kernel<false><<<static_cast<unsigned>(p->n_tiles), 256, 0, s>>>(one, nullptr, nullptr, 1);
    }
    return hipGetLastError();
  }
  // the record layout the permute wrote for this catalog
  return c->weight ? launch_scatter_kernel<true>(p, c, s, bulk, k, tp, tb)
                   : launch_scatter_kernel<false>(p, c, s, bulk, k, tp, tb);
}

hipError_t launch_scatter(Plan* p, const mps_catalog* c, hipStream_t s) {
  return launch_scatter_impl(p, c, s, 0);
}

ScatterCat scatter_cat(Plan* p, const mps_catalog* c) {
  return ScatterCat{p->sorted, p->tile_offset, static_cast<float*>(p->grid), key_params(p, c), &p->d_header->d, 0,
                    p->halo};
}

size_t pair_scratch_bytes(int64_t n_tiles, int num_cus) {
  int64_t b = n_tiles < num_cus ? n_tiles : num_cus;
  if (b > kPairBlocks) b = kPairBlocks;
  return static_cast<size_t>(b) * kPairCap * sizeof(uint32_t);
}

int scatter_form_for(int n_grid, mps_precision prec, int64_t np) {
  // on fewer than 8^3 tiles the atomic form's few workgroups are the fastest
  if (n_grid < MPS_SCATTER_MIN_GRID || np >= (static_cast<int64_t>(1) << 31)) return kFormAtomic;
  const int64_t nt = n_grid / 16;
  const int64_t tiles = nt * nt * nt;
  if (prec == MPS_F64) return np <= kGather64MaxMean * tiles ? kFormGather : kFormAtomic;
  if (np <= kGatherMaxMean * tiles) return kFormGather;
  if (np <= kHaloMaxMean * tiles) return kFormHalo;
  return kFormAtomic;
}

size_t halo_bytes(int n_grid, mps_precision prec) {
  if (prec != MPS_F32 || n_grid < MPS_SCATTER_MIN_GRID) return 0;
  const size_t nt = static_cast<size_t>(n_grid / 16);
  return nt * nt * nt * kNumFields * kHaloCells * sizeof(float);
}

int scatter_form(const Plan* p, const mps_catalog* c) {
  if (kernel_id(c->flags) != 0) return kFormAtomic;
  const int f = scatter_form_for(p->n, p->prec, c->n_particles);
  return f == kFormHalo && !p->halo ? kFormAtomic : f;
}

int scatter_group(const Plan* p, const mps_catalog* c) {
  if (p->prec != MPS_F32 || p->tile != 16 || kernel_id(c->flags) != 0) return -1;
  return 2 * scatter_form(p, c) + (c->weight ? 1 : 0);
}

hipError_t launch_scatter_multi(const ScatterCat* d_cats, const int64_t* d_starts, int n_cats, int64_t n_items,
                                int group, const TapPoly& tp, const TapBound& tb, uint32_t* d_queue, int num_cus,
                                hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  TileQueues tq;
  tq.counter = d_queue;
  tq.nq = 8;
  tq.per_queue = (n_items + 7) / 8;
  clear_kernel<uint32_t><<<1, 64, 0, s>>>(d_queue, 8);
  const ScatterCat none{};
  const bool has_w = (group & 1) != 0;
  const int form = group >> 1;
  if (form == kFormGather) {
    const int64_t cap = 2 * static_cast<int64_t>(num_cus);
    const unsigned blocks = static_cast<unsigned>(n_items < cap ? n_items : cap);
    if (has_w)
      scatter_gather_kernel<kGatherThreads, true, true><<<blocks, kGatherThreads, 0, s>>>(
          none, d_cats, d_starts, n_cats, n_items, tq, tp, tb);
    else
      scatter_gather_kernel<kGatherThreads, false, true><<<blocks, kGatherThreads, 0, s>>>(
          none, d_cats, d_starts, n_cats, n_items, tq, tp, tb);
    return hipGetLastError();
  }
  const unsigned blocks = static_cast<unsigned>(n_items < num_cus ? n_items : num_cus);
  if (form == kFormHalo) {
    if (has_w)
      scatter_fixed_kernel<16, 1024, 6, 3, true, true, true><<<blocks, 1024, 0, s>>>(
          none, d_cats, d_starts, n_cats, n_items, tq, tp, tb, PairWork{nullptr, 0});
    else
      scatter_fixed_kernel<16, 1024, 6, 3, false, true, true><<<blocks, 1024, 0, s>>>(
          none, d_cats, d_starts, n_cats, n_items, tq, tp, tb, PairWork{nullptr, 0});
    halo_fixup_kernel<true><<<static_cast<unsigned>(n_items), 256, 0, s>>>(none, d_cats, d_starts, n_cats);
    return hipGetLastError();
  }
  if (has_w)
    scatter_fixed_kernel<16, 1024, 6, 3, true, true><<<blocks, 1024, 0, s>>>(
        none, d_cats, d_starts, n_cats, n_items, tq, tp, tb, PairWork{nullptr, 0});
  else
    scatter_fixed_kernel<16, 1024, 6, 3, false, true><<<blocks, 1024, 0, s>>>(
        none, d_cats, d_starts, n_cats, n_items, tq, tp, tb, PairWork{nullptr, 0});
  return hipGetLastError();
}

}  // namespace mps
