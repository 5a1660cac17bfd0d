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

// Largest |phi_t(x) phi_t(y) phi_t(z)| over the truncated kernel: phi(0)^3
// = 1.0890^3 = 1.2916, rounded up.
constexpr double kPhiMax = 1.3;

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

// Tap weights and the particle's cell relative to the tile origin.
template <typename T, int TS>
__device__ __forceinline__ unsigned particle_taps(const float4& a, const KeyParams& kp, int ox, int oy, int oz,
                                                  const TapPoly& tp, T* wx, T* wy, T* wz) {
  constexpr int E = TS + 5;
  double fx, fy, fz;
  bool ok;
  int cx = locate(a.x, kp.scale, kp.n, &fx, &ok) - ox;
  int cy = locate(a.y, kp.scale, kp.n, &fy, &ok) - oy;
  int cz = locate(a.z, kp.scale, kp.n, &fz, &ok) - oz;
  // the sort placed the particle in this tile with the same locate(); the
  // clamp only keeps LDS indices in range
  cx = min(max(cx, 0), TS - 1);
  cy = min(max(cy, 0), TS - 1);
  cz = min(max(cz, 0), TS - 1);
#pragma unroll
  for (int j = 0; j < kTaps; ++j) {
    wx[j] = static_cast<T>(tap_weight(tp, j, fx));
    wy[j] = static_cast<T>(tap_weight(tp, j, fy));
    wz[j] = static_cast<T>(tap_weight(tp, j, fz));
  }
  return static_cast<unsigned>((cx * E + cy) * E + cz);
}

__device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t xcd_chunk) {
  // consecutive tiles (spatial neighbours, which share halo cache lines) go
  // to one XCD: workgroups are dealt to the 8 XCDs round robin
  return xcd_chunk > 0 ? (b & 7) * xcd_chunk + (b >> 3) : b;
}

// Rounds wxy * qs to the nearest integer in two instructions: for
// |x| < 2^22, x + 1.5 * 2^23 is an integer-valued float whose bit pattern
// minus that of 1.5 * 2^23 is round(x).
constexpr float kMagic = 12582912.0f;      // 1.5 * 2^23
constexpr int kMagicBits = 0x4B400000;

// Lane assignment that spreads a wave over the LDS banks.  Each chunk of NT
// particles is counting-sorted by (LDS word index mod 64) of its tap origin;
// lane l of wave w then takes bank-sorted position l * W + w, W = the number
// of waves the chunk fills, so the 64 lanes of a wave come from 64
// consecutive bank segments: about one lane per bank (two on a 32-bank LDS)
// and never two lanes on one address.
template <int NT>
struct BankSort {
  int cnt[64];
  unsigned short idx[NT];
};

template <int NT>
__device__ __forceinline__ int bank_sorted_index(BankSort<NT>& bs, bool valid, unsigned bank, int m) {
  const int t = threadIdx.x;
  if (t < 64) bs.cnt[t] = 0;
  __syncthreads();
  int slot = 0;
  if (valid) slot = atomicAdd(&bs.cnt[bank], 1);
  __syncthreads();
  if (t < 64) {  // exclusive scan of 64 counters in one wave
    int v = bs.cnt[t];
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off);
      if (t >= off) incl += o;
    }
    bs.cnt[t] = incl - v;
  }
  __syncthreads();
  if (valid) bs.idx[bs.cnt[bank] + slot] = static_cast<unsigned short>(t);
  __syncthreads();
  // a partial chunk (m < NT) occupies only ceil(m / 64) full waves
  const int waves = (m + 63) >> 6;
  const int w = t >> 6;
  const int q = (t & 63) * waves + w;
  return (w < waves && q < m) ? bs.idx[q] : -1;
}

// FP32 grids.  One workgroup per occupied tile.  LDS holds the four fields
// over the tile plus a halo of 2 cells below and 3 above along each axis
// (taps -2..3) as 32-bit fixed point: gfx950's LDS adds integers at ~14
// lanes/clk/CU but FP32 at ~0.3.  Each field's scale is chosen per tile so
// that no cell total can leave int32 (|cell| <= kPhiMax sum_tile |q|; the
// final value is exact modulo 2^32 whatever the order of the adds) and no
// single deposit reaches 2^22 (the rounding above).
template <int TS, int NT>
__global__ __launch_bounds__(NT) void scatter_fixed_kernel(
    const float4* __restrict__ sorted, const uint32_t* __restrict__ offset, float* __restrict__ grid,
    KeyParams kp, int64_t n_tiles, int64_t xcd_chunk, TapPoly tp, const Derived* dsrc, int bulk) {
  constexpr int E = TS + 5;
  constexpr int VOL = E * E * E;
  __shared__ int acc[kNumFields * VOL];
  __shared__ BankSort<NT> bs;
  __shared__ double red[NT / 64][2 * kNumFields];
  __shared__ float scale_s[kNumFields], inv_s[kNumFields];
  const int64_t tile = tile_of_block(blockIdx.x, xcd_chunk);
  if (tile >= n_tiles) return;
  const uint32_t p0 = offset[tile], p1 = offset[tile + 1];
  if (p0 == p1) return;
  double vb0 = 0.0, vb1 = 0.0, vb2 = 0.0;
  if (bulk) {
    vb0 = dsrc->vb[0];
    vb1 = dsrc->vb[1];
    vb2 = dsrc->vb[2];
  }
  // pass 1: per-field sum and max of |q| over the tile's particles (FP64)
  double sq[kNumFields] = {0.0, 0.0, 0.0, 0.0}, mq[kNumFields] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t p = p0 + threadIdx.x; p < p1; p += NT) {
    const DepositQ<double> d =
        charges<double>(sorted[2 * static_cast<int64_t>(p)], sorted[2 * static_cast<int64_t>(p) + 1], bulk,
                        vb0, vb1, vb2);
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) {
      sq[f] += fabs(d.q[f]);
      mq[f] = fmax(mq[f], fabs(d.q[f]));
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int f = 0; f < kNumFields; ++f) {
    double t = wave_sum(sq[f]);
    double m = mq[f];
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) {
      red[wave][f] = t;
      red[wave][kNumFields + f] = m;
    }
  }
  for (int i = threadIdx.x; i < kNumFields * VOL; i += NT) acc[i] = 0;
  __syncthreads();
  if (threadIdx.x < kNumFields) {
    double b = 0.0, m = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      b += red[w][threadIdx.x];
      m = fmax(m, red[w][kNumFields + threadIdx.x]);
    }
    const double by_sum = b > 0.0 ? 0.98 * 2147483648.0 / (kPhiMax * 1.0001 * b) : 0.0;
    const double by_max = m > 0.0 ? 0.99 * 4194304.0 / (kPhiMax * m) : 0.0;
    const double sc = fmin(by_sum, by_max);
    scale_s[threadIdx.x] = static_cast<float>(sc);
    inv_s[threadIdx.x] = sc > 0.0 ? static_cast<float>(1.0 / static_cast<double>(static_cast<float>(sc))) : 0.f;
  }
  __syncthreads();
  float sc[kNumFields];
#pragma unroll
  for (int f = 0; f < kNumFields; ++f) sc[f] = scale_s[f];
  const int nt = kp.nt;
  const int tz = static_cast<int>(tile % nt);
  const int ty = static_cast<int>((tile / nt) % nt);
  const int tx = static_cast<int>(tile / (static_cast<int64_t>(nt) * nt));
  const int ox = tx * TS, oy = ty * TS, oz = tz * TS;
  // pass 2: deposit, chunk by chunk in bank-sorted lane order
  for (uint32_t c0 = p0; c0 < p1; c0 += NT) {
    const int m = static_cast<int>(min(static_cast<uint32_t>(NT), p1 - c0));
    const bool mine = static_cast<int>(threadIdx.x) < m;
    unsigned bank = 0;
    if (mine) {
      float wx[kTaps], wy[kTaps], wz[kTaps];
      bank = particle_taps<float, TS>(sorted[2 * static_cast<int64_t>(c0 + threadIdx.x)], kp, ox, oy, oz, tp, wx,
                                      wy, wz) & 63u;
    }
    const int j = bank_sorted_index<NT>(bs, mine, bank, m);
    if (j < 0) continue;
    const uint32_t p = c0 + static_cast<uint32_t>(j);
    const float4 a = sorted[2 * static_cast<int64_t>(p)];
    const float4 v = sorted[2 * static_cast<int64_t>(p) + 1];
    float wx[kTaps], wy[kTaps], wz[kTaps];
    const unsigned base = particle_taps<float, TS>(a, kp, ox, oy, oz, tp, wx, wy, wz);
    const DepositQ<float> d = charges<float>(a, v, bulk, vb0, vb1, vb2);
    float qs[kNumFields][kTaps];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f)
#pragma unroll
      for (int jj = 0; jj < kTaps; ++jj) qs[f][jj] = d.q[f] * sc[f] * wz[jj];
    int* accf[kNumFields] = {acc + base, acc + VOL + base, acc + 2 * VOL + base, acc + 3 * VOL + base};
#pragma unroll
    for (int jx = 0; jx < kTaps; ++jx) {
#pragma unroll
      for (int jy = 0; jy < kTaps; ++jy) {
        const float wxy = wx[jx] * wy[jy];
#pragma unroll
        for (int f = 0; f < kNumFields; ++f)
#pragma unroll
          for (int jz = 0; jz < kTaps; ++jz)
            atomicAdd(accf[f] + (jx * E + jy) * E + jz,
                      __float_as_int(fmaf(wxy, qs[f][jz], kMagic)) - kMagicBits);
      }
    }
  }
  __syncthreads();
  const int n = kp.n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  float inv[kNumFields];
#pragma unroll
  for (int f = 0; f < kNumFields; ++f) inv[f] = inv_s[f];
  for (int i = threadIdx.x; i < VOL; i += NT) {
    const int ez = i % E, ey = (i / E) % E, ex = i / (E * E);
    const int gx = (ox + ex - 2) & (n - 1);
    const int gy = (oy + ey - 2) & (n - 1);
    const int gz = (oz + ez - 2) & (n - 1);
    const int64_t gi = (static_cast<int64_t>(gx) * n + gy) * n + gz;
#pragma unroll
    for (int f = 0; f < kNumFields; ++f) {
      const int val = acc[f * VOL + i];
      if (val != 0) atomicAdd(grid + f * n3 + gi, static_cast<float>(val) * inv[f]);
    }
  }
}

// FP64 grids: LDS accumulation with ds_add_f64 (~7 lanes/clk/CU on gfx950).
template <int TS, int NT>
__global__ __launch_bounds__(NT) void scatter_f64_kernel(
    const float4* __restrict__ sorted, const uint32_t* __restrict__ offset, double* __restrict__ grid,
    KeyParams kp, int64_t n_tiles, int64_t xcd_chunk, TapPoly tp, const Derived* dsrc, int bulk) {
  constexpr int E = TS + 5;
  constexpr int VOL = E * E * E;
  __shared__ double acc[kNumFields * VOL];
  __shared__ BankSort<NT> bs;
  const int64_t tile = tile_of_block(blockIdx.x, xcd_chunk);
  if (tile >= n_tiles) return;
  const uint32_t p0 = offset[tile], p1 = offset[tile + 1];
  if (p0 == p1) return;
  for (int i = threadIdx.x; i < kNumFields * VOL; i += NT) acc[i] = 0.0;
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
  // bank-sorted lane order (see the FP32 kernel); one double spans two banks,
  // so the bank key is the word index of the double mod 64 halved
  for (uint32_t c0 = p0; c0 < p1; c0 += NT) {
    const int m = static_cast<int>(min(static_cast<uint32_t>(NT), p1 - c0));
    const bool mine = static_cast<int>(threadIdx.x) < m;
    unsigned bank = 0;
    if (mine) {
      double wx[kTaps], wy[kTaps], wz[kTaps];
      bank = particle_taps<double, TS>(sorted[2 * static_cast<int64_t>(c0 + threadIdx.x)], kp, ox, oy, oz, tp, wx,
                                       wy, wz) & 31u;
    }
    const int j = bank_sorted_index<NT>(bs, mine, bank, m);
    if (j < 0) continue;
    const uint32_t p = c0 + static_cast<uint32_t>(j);
    const float4 a = sorted[2 * static_cast<int64_t>(p)];
    const float4 v = sorted[2 * static_cast<int64_t>(p) + 1];
    double wx[kTaps], wy[kTaps], wz[kTaps];
    const unsigned base = particle_taps<double, TS>(a, kp, ox, oy, oz, tp, wx, wy, wz);
    const DepositQ<double> d = charges<double>(a, v, bulk, vb0, vb1, vb2);
    double qz[kNumFields][kTaps];
#pragma unroll
    for (int f = 0; f < kNumFields; ++f)
#pragma unroll
      for (int j = 0; j < kTaps; ++j) qz[f][j] = d.q[f] * wz[j];
    double* accf[kNumFields] = {acc + base, acc + VOL + base, acc + 2 * VOL + base, acc + 3 * VOL + base};
#pragma unroll
    for (int jx = 0; jx < kTaps; ++jx) {
#pragma unroll
      for (int jy = 0; jy < kTaps; ++jy) {
        const double wxy = wx[jx] * wy[jy];
#pragma unroll
        for (int f = 0; f < kNumFields; ++f)
#pragma unroll
          for (int jz = 0; jz < kTaps; ++jz) atomicAdd(accf[f] + (jx * E + jy) * E + jz, wxy * qz[f][jz]);
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
      const double val = acc[f * VOL + i];
      if (val != 0.0) atomicAdd(grid + f * n3 + gi, val);
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
  const Derived* dsrc = &p->d_header->d;
  const unsigned grid = static_cast<unsigned>(p->n_tiles);
  if (p->prec == MPS_F32) {
    if (p->tile == 16)
      scatter_fixed_kernel<16, 1024><<<grid, 1024, 0, s>>>(p->sorted, p->tile_offset, static_cast<float*>(p->grid),
                                                            kp, p->n_tiles, xcd_chunk, p->taps, dsrc, bulk);
    else
      scatter_fixed_kernel<8, 512><<<grid, 512, 0, s>>>(p->sorted, p->tile_offset, static_cast<float*>(p->grid), kp,
                                                         p->n_tiles, xcd_chunk, p->taps, dsrc, bulk);
  } else {
    scatter_f64_kernel<8, 512><<<grid, 512, 0, s>>>(p->sorted, p->tile_offset, static_cast<double*>(p->grid), kp,
                                                     p->n_tiles, xcd_chunk, p->taps, dsrc, bulk);
  }
  return hipGetLastError();
}

hipError_t launch_scatter(Plan* p, const mps_catalog* c, hipStream_t s) {
  return launch_scatter_impl(p, c, s, 0);
}

}  // namespace mps
