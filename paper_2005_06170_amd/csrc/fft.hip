// Fourier-side stages on gfx950: three pencil passes of a 3D real-to-complex
// FFT kept in LDS (Stockham autosort, radix 8/4/2), the last of which is fused
// with the per-mode estimator and |k|-shell binning, then a fixed-order
// finalize.
//
// Layout.  Field f's real grid is [x][y][z], z fastest (4 fields stacked).
// The z pass turns each row of N reals into N/2 complex values in place
// (bins 0..N/2-1; the kz = N/2 plane is dropped: every mode on it has
// |k| >= k_N and is never binned).  The y and x passes work on columns of the
// resulting [x][y][kz] complex array.  The FFT sign is e^{-2 pi i n.g / N}.
//
// Per mode (the estimator of Eqs. rawPp, rawPtheta, rawPx with the BL3 window,
// bulk-flow removal of Sec. 3.1 in Fourier space, p' = p - v_b delta):
//   delta = F_0 / W, p = F_{1..3} / W,
//   P_dd = (|delta|^2 - S_dd C) / W_t^2,  P_pp = (|p|^2 - tr S C) / W_t^2,
//   P_tt = (|k.p|^2 - k^T S k C) / (Haf^2 W_t^2),
//   P_dt = Re(delta conj(-i k.p / Haf)) / W_t^2,
// with W_t^2 and C products of per-axis tables of the truncated kernel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"

namespace mps {
namespace {

template <typename T>
struct cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.im, -a.re}; }  // * (-i)

template <typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
  const cpx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T>
__device__ __forceinline__ void dft4(cpx<T>& a, cpx<T>& b, cpx<T>& c, cpx<T>& d) {
  const cpx<T> s02 = a + c, d02 = a - c, s13 = b + d, d13 = mul_mi(b - d);
  a = s02 + s13;
  b = d02 + d13;
  c = s02 - s13;
  d = d02 - d13;
}

template <typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const T h = static_cast<T>(0.70710678118654752440);
  // o_k *= e^{-2 pi i k / 8}
  o1 = {h * (o1.re + o1.im), h * (o1.im - o1.re)};
  o2 = mul_mi(o2);
  o3 = {h * (o3.im - o3.re), -h * (o3.re + o3.im)};
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + o1;
  v[5] = e1 - o1;
  v[2] = e2 + o2;
  v[6] = e2 - o2;
  v[3] = e3 + o3;
  v[7] = e3 - o3;
}

template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T>* v) {
  if constexpr (R == 8) dft8(v);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
  else dft2(v);
}

// One radix-R Stockham pass over COUNT transforms of length L held in LDS
// (element j of transform t at buf[t * tstride + j]).  tw[m * TWS] is
// e^{-2 pi i m / L}.  Butterflies are dealt transform-fastest over NT threads.
template <typename T, int L, int R, int NS, int COUNT, int NT, int TWS>
__device__ __forceinline__ void stockham_pass(cpx<T>* buf, int tstride, const cpx<T>* tw) {
  constexpr int NB = COUNT * (L / R);
  constexpr int PER = (NB + NT - 1) / NT;
  cpx<T> v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      const int t = b % COUNT, j = b / COUNT;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = buf[t * tstride + j + r * (L / R)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      const int t = b % COUNT, j = b / COUNT;
      const int kk = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[k][r] = cmul(v[k][r], tw[(kk * r * (L / (NS * R))) * TWS]);
      }
      dft<T, R>(v[k]);
      const int idx = (j / NS) * NS * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[t * tstride + idx + r * NS] = v[k][r];
    }
  }
  __syncthreads();
}

template <typename T, int L, int NS, int COUNT, int NT, int TWS>
__device__ __forceinline__ void fft_passes(cpx<T>* buf, int tstride, const cpx<T>* tw) {
  if constexpr (NS < L) {
    constexpr int REM = L / NS;
    constexpr int R = REM >= 8 ? 8 : REM;
    stockham_pass<T, L, R, NS, COUNT, NT, TWS>(buf, tstride, tw);
    fft_passes<T, L, NS * R, COUNT, NT, TWS>(buf, tstride, tw);
  }
}

template <typename T, int N, int NT>
__device__ __forceinline__ void load_twiddles(cpx<T>* tw, const cpx<T>* __restrict__ gtw) {
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = gtw[i];
}

// 16-byte vectors of complex values: two FP32 or one FP64.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 2;
  __device__ static cpx<float> get(const float4& v, int e) { return e == 0 ? cpx<float>{v.x, v.y} : cpx<float>{v.z, v.w}; }
  __device__ static float4 make(const cpx<float>* c) { return make_float4(c[0].re, c[0].im, c[1].re, c[1].im); }
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 1;
  __device__ static cpx<double> get(const double2& v, int) { return {v.x, v.y}; }
  __device__ static double2 make(const cpx<double>* c) { return make_double2(c[0].re, c[0].im); }
};

// Global -> LDS staging of ROWS rows of COLS consecutive complex values (row r
// starts at src(r), 16-byte aligned): each thread issues GROUP 16-byte loads
// before writing any of them to LDS element put(r, c), so that many loads
// are in flight per wave.
template <typename T, int ROWS, int COLS, int NT, int MAXG = 16, typename Src, typename Put>
__device__ __forceinline__ void gather_rows(Src src, Put put) {
  using V = Vec16<T>;
  static_assert(COLS % V::n == 0, "rows must hold whole 16-byte vectors");
  constexpr int CV = COLS / V::n;
  constexpr int TOTAL = ROWS * CV;
  constexpr int ITER = (TOTAL + NT - 1) / NT;
  constexpr int GROUP = ITER < MAXG ? ITER : MAXG;
  constexpr bool kExact = TOTAL % NT == 0 && ITER % GROUP == 0;
  for (int k0 = 0; k0 < ITER; k0 += GROUP) {
    typename V::type v[GROUP];
#pragma unroll
    for (int k = 0; k < GROUP; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      if (kExact || (k0 + k < ITER && i < TOTAL))
        v[k] = *reinterpret_cast<const typename V::type*>(src(i / CV) + (i % CV) * V::n);
    }
#pragma unroll
    for (int k = 0; k < GROUP; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      if (kExact || (k0 + k < ITER && i < TOTAL)) {
        const int r = i / CV, c = (i % CV) * V::n;
#pragma unroll
        for (int e = 0; e < V::n; ++e) put(r, c + e, V::get(v[k], e));
      }
    }
  }
}

// LDS -> global: value(r, c) for ROWS rows of COLS consecutive complex values
// stored from dst(r), GROUP vectors gathered per thread before the stores.
template <typename T, int ROWS, int COLS, int NT, typename Dst, typename Get>
__device__ __forceinline__ void scatter_rows(Dst dst, Get value) {
  using V = Vec16<T>;
  static_assert(COLS % V::n == 0, "rows must hold whole 16-byte vectors");
  constexpr int CV = COLS / V::n;
  constexpr int TOTAL = ROWS * CV;
  constexpr int ITER = (TOTAL + NT - 1) / NT;
  constexpr int GROUP = ITER < 8 ? ITER : 8;
  constexpr bool kExact = TOTAL % NT == 0 && ITER % GROUP == 0;
  for (int k0 = 0; k0 < ITER; k0 += GROUP) {
    typename V::type v[GROUP];
#pragma unroll
    for (int k = 0; k < GROUP; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      if (kExact || (k0 + k < ITER && i < TOTAL)) {
        const int r = i / CV, c = (i % CV) * V::n;
        cpx<T> e[V::n];
#pragma unroll
        for (int q = 0; q < V::n; ++q) e[q] = value(r, c + q);
        v[k] = V::make(e);
      }
    }
#pragma unroll
    for (int k = 0; k < GROUP; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      if (kExact || (k0 + k < ITER && i < TOTAL))
        *reinterpret_cast<typename V::type*>(dst(i / CV) + (i % CV) * V::n) = v[k];
    }
  }
}

// ---------------------------------------------------------------- z pass
// P rows of N reals per workgroup: complex FFT of length N/2 on the packed
// even/odd samples, then the real-to-complex split.
template <typename T, int N, int P, int NT>
__global__ __launch_bounds__(NT) void fft_z_kernel(T* __restrict__ grid, const cpx<T>* __restrict__ gtw) {
  constexpr int M = N / 2;
  constexpr int TS = M + 1;
  __shared__ cpx<T> buf[P * TS];
  __shared__ cpx<T> tw[N];
  load_twiddles<T, N, NT>(tw, gtw);
  cpx<T>* rows = reinterpret_cast<cpx<T>*>(grid) + static_cast<int64_t>(blockIdx.x) * P * M;
  gather_rows<T, P, M, NT>([&](int q) { return rows + q * M; },
                           [&](int q, int j, cpx<T> v) { buf[q * TS + j] = v; });
  __syncthreads();
  fft_passes<T, M, 1, P, NT, 2>(buf, TS, tw);
  const T half = static_cast<T>(0.5);
  scatter_rows<T, P, M, NT>([&](int q) { return rows + q * M; }, [&](int q, int k) {
    const cpx<T> a = buf[q * TS + k];
    const cpx<T> z2 = buf[q * TS + (M - k) % M];
    const cpx<T> b = {z2.re, -z2.im};
    const cpx<T> s = a + b, d = a - b;
    const cpx<T> t = cmul(tw[k], mul_mi(d));
    return cpx<T>{half * (s.re + t.re), half * (s.im + t.im)};
  });
}

// ------------------------------------------------------------- y, x passes
// B columns (consecutive kz) of N complex values spaced by `stride` complex.
// Workgroup index -> (field f, outer index o, column block kb); the column
// block is fastest.  For the y pass outer = x and stride = N/2; for the x
// pass outer = y and stride = N * N/2.
template <typename T, int N, int B, int NT>
__global__ __launch_bounds__(NT) void fft_cols_kernel(T* __restrict__ grid, const cpx<T>* __restrict__ gtw,
                                                      int64_t stride, int64_t outer_stride) {
  constexpr int M = N / 2;
  constexpr int TS = N + 1;
  constexpr int KB = M / B;
  __shared__ cpx<T> buf[B * TS];
  __shared__ cpx<T> tw[N];
  load_twiddles<T, N, NT>(tw, gtw);
  const int64_t blk = blockIdx.x;
  const int kb = static_cast<int>(blk % KB);
  const int64_t fo = blk / KB;                 // f * N + o
  const int64_t f = fo / N, o = fo % N;
  cpx<T>* base = reinterpret_cast<cpx<T>*>(grid) + f * static_cast<int64_t>(N) * N * M + o * outer_stride +
                 kb * B;
  gather_rows<T, N, B, NT>([&](int r) { return base + r * stride; },
                           [&](int r, int c, cpx<T> v) { buf[c * TS + r] = v; });
  __syncthreads();
  fft_passes<T, N, 1, B, NT, 1>(buf, TS, tw);
  scatter_rows<T, N, B, NT>([&](int r) { return base + r * stride; },
                            [&](int r, int c) { return buf[c * TS + r]; });
}

// ------------------------------------------------- x pass fused with bins
struct BinParams {
  double kf;        // 2 pi / L
  double haf;
  double inv_haf;   // 1 / Haf
  double inv_haf2;  // 1 / Haf^2
  int n_bins;
  int no_shot;
  int no_deconv;
  int bulk;
};

// Adds one run of unweighted per-mode sums to the workgroup's LDS bins, with
// the half-space weight w (1 on the kz = 0 plane, else 2) and k = kf |n|.
__device__ __forceinline__ void flush_bin(double* lbins, int bin, const double* acc, double w, double kf) {
#pragma unroll
  for (int q = 0; q < kNumQ; ++q) atomicAdd(lbins + bin * kNumQ + q, (q == QKsum ? w * kf : w) * acc[q]);
}

// Persistent: workgroup g handles items g, g + G, ... where an item is one
// y row and a block of B consecutive kz columns, for all four fields.  Items
// whose every mode lies outside |n| < N/2 are skipped.  LDS bin sums of the
// workgroup are written to partials[g] at the end (no global atomics, fixed
// summation order in the finalize).
template <typename T, int N, int B, int NT>
__global__ __launch_bounds__(NT) void fft_x_bin_kernel(const T* __restrict__ grid, const cpx<T>* __restrict__ gtw,
                                                       const ResultHeader* __restrict__ hdr,
                                                       const double* __restrict__ iwin2_tab,
                                                       const double* __restrict__ alias_tab,
                                                       const int32_t* __restrict__ lut, BinParams bp,
                                                       double* __restrict__ partials) {
  constexpr int M = N / 2;
  constexpr int TS = N + 1;
  constexpr int KB = M / B;
  constexpr int COUNT = kNumFields * B;
  constexpr int MODES = B * N;
  constexpr int RUN = MODES >= NT ? MODES / NT : 1;
  constexpr int64_t H2 = static_cast<int64_t>(M) * M;
  __shared__ cpx<T> buf[COUNT * TS];
  __shared__ cpx<T> tw[N];
  __shared__ double lbins[kMaxBins * kNumQ];
  // per-axis window and alias tables in LDS when they fit beside the pencils
  constexpr size_t kBase = sizeof(cpx<T>) * (COUNT * TS + N) + sizeof(double) * kMaxBins * kNumQ;
  constexpr bool kTabLds = kBase + 2 * sizeof(double) * (M + 1) <= 163840;
  __shared__ double s_tab[kTabLds ? 2 * (M + 1) : 1];
  const double* s_iwin2 = kTabLds ? s_tab : iwin2_tab;
  const double* s_alias = kTabLds ? s_tab + M + 1 : alias_tab;
  load_twiddles<T, N, NT>(tw, gtw);
  for (int i = threadIdx.x; i < kMaxBins * kNumQ; i += NT) lbins[i] = 0.0;
  if constexpr (kTabLds) {
    for (int i = threadIdx.x; i <= M; i += NT) {
      s_tab[i] = iwin2_tab[i];
      s_tab[M + 1 + i] = alias_tab[i];
    }
  }

  const Derived d = hdr->d;
  const int64_t field_stride = static_cast<int64_t>(N) * N * M;
  const int64_t xstride = static_cast<int64_t>(N) * M;
  const cpx<T>* g = reinterpret_cast<const cpx<T>*>(grid);
  const int n_items = N * KB;
  // Items 2j and 2j+1 (kz blocks 2i, 2i+1 of one y row) read the two halves
  // of the same 128-byte lines; with a grid of 16m workgroups they go to
  // workgroups g and g + 8, which sit on the same XCD (workgroups are dealt
  // to the 8 XCDs round robin), so the second read hits that XCD's L2.
  const int G = gridDim.x, wg = blockIdx.x;
  const bool paired = KB % 2 == 0 && G % 16 == 0;
  const int lane_id = paired ? (wg % 8) + 8 * (wg / 16) : wg;
  const int half = paired ? (wg / 8) % 2 : 0;
  const int per_it = paired ? G / 2 : G;
  for (int it = 0;; ++it) {
    const int item = paired ? 2 * (it * per_it + lane_id) + half : it * per_it + lane_id;
    if (item >= n_items) break;
    const int y = item / KB, kb = item % KB;
    const int ny = y < M ? y : y - N;
    const int kz0 = kb * B;
    if (static_cast<int64_t>(ny) * ny + static_cast<int64_t>(kz0) * kz0 >= H2) continue;
    __syncthreads();  // previous item's LDS reads are done
    const cpx<T>* col0 = g + static_cast<int64_t>(y) * M + kz0;
    gather_rows<T, kNumFields * N, B, NT, 8>(
        [&](int fr) { return col0 + (fr / N) * field_stride + (fr % N) * xstride; },
        [&](int fr, int c, cpx<T> v) { buf[((fr / N) * B + c) * TS + fr % N] = v; });
    __syncthreads();
    fft_passes<T, N, 1, COUNT, NT, 1>(buf, TS, tw);

    // per-mode estimator; each thread walks RUN consecutive kx of one column,
    // with the column's y and z factors hoisted; sums are unweighted until a
    // bin is flushed (the half-space weight is constant along the column)
    int cur = -1;
    double acc[kNumQ];
#pragma unroll
    for (int q = 0; q < kNumQ; ++q) acc[q] = 0.0;
    const int m0 = threadIdx.x * RUN;
    double wgt = 0.0;
    if (m0 < MODES) {
      const int c = m0 / N;
      const int nz = kz0 + c;
      wgt = nz == 0 ? 1.0 : 2.0;
      const int ay = ny < 0 ? -ny : ny;
      const double col_iw = bp.no_deconv ? 1.0 : s_iwin2[ay] * s_iwin2[nz];
      const double col_cal = s_alias[ay] * s_alias[nz];
      const double ky_ = bp.kf * ny, kz_ = bp.kf * nz;
      const double ksk0 = d.S[1] * ky_ * ky_ + d.S[2] * kz_ * kz_ + 2.0 * d.S[5] * ky_ * kz_;
      const double ksk1 = 2.0 * (d.S[3] * ky_ + d.S[4] * kz_);
      const int64_t n2yz = static_cast<int64_t>(ny) * ny + static_cast<int64_t>(nz) * nz;
      const cpx<T>* col = buf + c * TS;
      for (int r = 0; r < RUN; ++r) {
        const int kx = (m0 % N) + r;
        const int nx = kx < M ? kx : kx - N;
        const int64_t n2 = static_cast<int64_t>(nx) * nx + n2yz;
        if (n2 == 0 || n2 >= H2) continue;
        const int bin = lut[n2];
        if (bin < 0) continue;
        const int ax = nx < 0 ? -nx : nx;
        const double iw2 = bp.no_deconv ? 1.0 : col_iw * s_iwin2[ax];
        const double cal = col_cal * s_alias[ax];
        const cpx<T> F0 = col[kx];
        const cpx<T> F1 = col[B * TS + kx];
        const cpx<T> F2 = col[2 * B * TS + kx];
        const cpx<T> F3 = col[3 * B * TS + kx];
        const double dr = static_cast<double>(F0.re) * d.inv_W, di = static_cast<double>(F0.im) * d.inv_W;
        double pxr = static_cast<double>(F1.re) * d.inv_W, pxi = static_cast<double>(F1.im) * d.inv_W;
        double pyr = static_cast<double>(F2.re) * d.inv_W, pyi = static_cast<double>(F2.im) * d.inv_W;
        double pzr = static_cast<double>(F3.re) * d.inv_W, pzi = static_cast<double>(F3.im) * d.inv_W;
        if (bp.bulk) {
          pxr -= d.vb[0] * dr;
          pxi -= d.vb[0] * di;
          pyr -= d.vb[1] * dr;
          pyi -= d.vb[1] * di;
          pzr -= d.vb[2] * dr;
          pzi -= d.vb[2] * di;
        }
        const double kx_ = bp.kf * nx;
        const double kpr = kx_ * pxr + ky_ * pyr + kz_ * pzr;
        const double kpi = kx_ * pxi + ky_ * pyi + kz_ * pzi;
        const double raw_dd = (dr * dr + di * di) * iw2;
        const double raw_pp = (pxr * pxr + pxi * pxi + pyr * pyr + pyi * pyi + pzr * pzr + pzi * pzi) * iw2;
        const double raw_tt = (kpr * kpr + kpi * kpi) * iw2 * bp.inv_haf2;
        const double raw_dt = (dr * kpi - di * kpr) * iw2 * bp.inv_haf;
        const double ksk = (d.S[0] * kx_ + ksk1) * kx_ + ksk0;
        const double ciw = cal * iw2;
        const double sdd = d.s_dd * ciw;
        const double spp = d.s_pp * ciw;
        const double stt = ksk * ciw * bp.inv_haf2;
        if (bin != cur) {
          if (cur >= 0) flush_bin(lbins, cur, acc, wgt, bp.kf);
#pragma unroll
          for (int q = 0; q < kNumQ; ++q) acc[q] = 0.0;
          cur = bin;
        }
        acc[QCount] += 1.0;
        acc[QKsum] += sqrt(static_cast<double>(n2));
        acc[QPdd] += bp.no_shot ? raw_dd : raw_dd - sdd;
        acc[QPpp] += bp.no_shot ? raw_pp : raw_pp - spp;
        acc[QPtt] += bp.no_shot ? raw_tt : raw_tt - stt;
        acc[QPdt] += raw_dt;
        acc[QSdd] += sdd;
        acc[QSpp] += spp;
        acc[QStt] += stt;
      }
    }
    if (cur >= 0) flush_bin(lbins, cur, acc, wgt, bp.kf);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < bp.n_bins * kNumQ; i += NT)
    partials[static_cast<int64_t>(blockIdx.x) * kMaxBins * kNumQ + i] = lbins[i];
}

// ------------------------------------------- anisotropic (k, mu_b) binning
struct MuParams {
  double kf, inv_haf, inv_haf2;
  double axis[3];   // unit axis from the host, if axis_given
  int axis_given;
  int n_bins, n_mu, no_shot, no_deconv, bulk;
};

// Running sums of one (k, mu) cell, flushed to the workgroup's LDS cells
// when the cell changes.
struct MuRun {
  int cell = -1;
  double q[kNumQMu];
  __device__ void reset(int c) {
    cell = c;
#pragma unroll
    for (int i = 0; i < kNumQMu; ++i) q[i] = 0.0;
  }
  __device__ void flush(double* lbins) const {
    if (cell < 0) return;
#pragma unroll
    for (int i = 0; i < kNumQMu; ++i) atomicAdd(lbins + cell * kNumQMu + i, q[i]);
  }
};

// mu = (n.a) / |n| with each operation rounded separately, and its bin
// min(floor((mu + 1) n_mu / 2), n_mu - 1) clamped at 0.
__device__ __forceinline__ int mu_cell(double mu, int n_mu) {
  const double t = __dmul_rn(__dadd_rn(mu, 1.0), 0.5 * n_mu);
  int m = static_cast<int>(floor(t));
  m = m < 0 ? 0 : m;
  return m > n_mu - 1 ? n_mu - 1 : m;
}

// Every stored mode (kx, ky, kz < N/2) of the fully transformed grid, with
// kz > 0 modes also standing for -n (real fields: F(-n) = conj F(n), so the
// auto spectra and real parts repeat and the imaginary parts change sign).
// Each thread walks RUN consecutive kz of one (kx, ky) row.  Per mode, in
// the paper's Fourier convention (fields e^{+ik.r}, the complex conjugates
// of the stored e^{-ik.r} transforms):
//   Re P_dt = (dr kpi - di kpr) / (Haf W^2),  Im P_dt = -(dr kpr + di kpi) /
//   (Haf W^2) less its shot term -(k.s) C / (Haf W^2) (Eq. rawPx),
//   P_dpb = (dr pbr + di pbi, dr pbi - di pbr) / W^2 with pb = a.(p - v_b
//   delta), the real part less (a.s') C / W^2 (Eq. bfpp),
// and P_dd, P_pp, P_tt as in the isotropic pass.
template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void mu_bin_kernel(const T* __restrict__ grid, const ResultHeader* __restrict__ hdr,
                                                    const double* __restrict__ iwin2_tab,
                                                    const double* __restrict__ alias_tab,
                                                    const int32_t* __restrict__ lut, MuParams mp,
                                                    double* __restrict__ partials) {
  constexpr int M = N / 2;
  constexpr int RUN = M >= 8 ? 8 : M;
  constexpr int CH = M / RUN;
  constexpr int64_t H2 = static_cast<int64_t>(M) * M;
  __shared__ double lbins[kMaxMuCells * kNumQMu];
  __shared__ double s_iwin2[M + 1], s_alias[M + 1];
  for (int i = threadIdx.x; i < kMaxMuCells * kNumQMu; i += NT) lbins[i] = 0.0;
  for (int i = threadIdx.x; i <= M; i += NT) {
    s_iwin2[i] = mp.no_deconv ? 1.0 : iwin2_tab[i];
    s_alias[i] = alias_tab[i];
  }
  __syncthreads();
  const Derived d = hdr->d;
  double a0, a1, a2;
  if (mp.axis_given) {
    a0 = mp.axis[0];
    a1 = mp.axis[1];
    a2 = mp.axis[2];
  } else {
    const double nrm =
        __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(d.vb[0], d.vb[0]), __dmul_rn(d.vb[1], d.vb[1])),
                             __dmul_rn(d.vb[2], d.vb[2])));
    a0 = nrm > 0.0 ? __ddiv_rn(d.vb[0], nrm) : 0.0;
    a1 = nrm > 0.0 ? __ddiv_rn(d.vb[1], nrm) : 0.0;
    a2 = nrm > 0.0 ? __ddiv_rn(d.vb[2], nrm) : 0.0;
  }
  const double sa = (d.sp[0] * a0 + d.sp[1] * a1) + d.sp[2] * a2;   // a.s'
  const int64_t fstride = static_cast<int64_t>(N) * N * M;
  const cpx<T>* g = reinterpret_cast<const cpx<T>*>(grid);
  const int64_t items = static_cast<int64_t>(N) * N * CH;
  for (int64_t it = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x; it < items;
       it += static_cast<int64_t>(gridDim.x) * NT) {
    const int ch = static_cast<int>(it % CH);
    const int64_t row = it / CH;
    const int ky = static_cast<int>(row % N), kx = static_cast<int>(row / N);
    const int nx = kx < M ? kx : kx - N, ny = ky < M ? ky : ky - N;
    const int nz0 = ch * RUN;
    const int64_t n2xy = static_cast<int64_t>(nx) * nx + static_cast<int64_t>(ny) * ny;
    if (n2xy + static_cast<int64_t>(nz0) * nz0 >= H2) continue;
    const int ax = nx < 0 ? -nx : nx, ay = ny < 0 ? -ny : ny;
    const double col_iw = s_iwin2[ax] * s_iwin2[ay];
    const double col_cal = s_alias[ax] * s_alias[ay];
    const double kx_ = mp.kf * nx, ky_ = mp.kf * ny;
    const cpx<T>* base = g + row * M;
    MuRun ra, rb;
    // the run's bin lookups go out together (one L2 round trip, not RUN)
    int kbs[RUN];
#pragma unroll
    for (int r = 0; r < RUN; ++r) {
      const int nz = nz0 + r;
      const int64_t n2 = n2xy + static_cast<int64_t>(nz) * nz;
      kbs[r] = (n2 == 0 || n2 >= H2) ? -1 : lut[n2];
    }
    for (int r = 0; r < RUN; ++r) {
      const int nz = nz0 + r;
      const int64_t n2 = n2xy + static_cast<int64_t>(nz) * nz;
      const int kb = kbs[r];
      if (kb < 0) continue;
      const double iw2 = col_iw * s_iwin2[nz];
      const double cal = col_cal * s_alias[nz];
      const cpx<T> F0 = base[nz], F1 = base[fstride + nz], F2 = base[2 * fstride + nz],
                   F3 = base[3 * fstride + nz];
      const double dr = static_cast<double>(F0.re) * d.inv_W, di = static_cast<double>(F0.im) * d.inv_W;
      const double qxr = static_cast<double>(F1.re) * d.inv_W, qxi = static_cast<double>(F1.im) * d.inv_W;
      const double qyr = static_cast<double>(F2.re) * d.inv_W, qyi = static_cast<double>(F2.im) * d.inv_W;
      const double qzr = static_cast<double>(F3.re) * d.inv_W, qzi = static_cast<double>(F3.im) * d.inv_W;
      // p' = p - v_b delta (exact by linearity of the assignment)
      const double bxr = qxr - d.vb[0] * dr, bxi = qxi - d.vb[0] * di;
      const double byr = qyr - d.vb[1] * dr, byi = qyi - d.vb[1] * di;
      const double bzr = qzr - d.vb[2] * dr, bzi = qzi - d.vb[2] * di;
      const double pxr = mp.bulk ? bxr : qxr, pxi = mp.bulk ? bxi : qxi;
      const double pyr = mp.bulk ? byr : qyr, pyi = mp.bulk ? byi : qyi;
      const double pzr = mp.bulk ? bzr : qzr, pzi = mp.bulk ? bzi : qzi;
      const double kz_ = mp.kf * nz;
      const double kpr = kx_ * pxr + ky_ * pyr + kz_ * pzr;
      const double kpi = kx_ * pxi + ky_ * pyi + kz_ * pzi;
      const double pbr = a0 * bxr + a1 * byr + a2 * bzr;
      const double pbi = a0 * bxi + a1 * byi + a2 * bzi;
      const double ciw = cal * iw2;
      const double raw_dd = (dr * dr + di * di) * iw2;
      const double raw_pp = (pxr * pxr + pxi * pxi + pyr * pyr + pyi * pyi + pzr * pzr + pzi * pzi) * iw2;
      const double raw_tt = (kpr * kpr + kpi * kpi) * iw2 * mp.inv_haf2;
      const double dt_re = (dr * kpi - di * kpr) * iw2 * mp.inv_haf;
      const double dt_im = -(dr * kpr + di * kpi) * iw2 * mp.inv_haf;
      const double dpb_re = (dr * pbr + di * pbi) * iw2;
      const double dpb_im = (dr * pbi - di * pbr) * iw2;
      const double ksk = d.S[0] * kx_ * kx_ + d.S[1] * ky_ * ky_ + d.S[2] * kz_ * kz_ +
                         2.0 * (d.S[3] * kx_ * ky_ + d.S[4] * kx_ * kz_ + d.S[5] * ky_ * kz_);
      const double sdd = d.s_dd * ciw, spp = d.s_pp * ciw, stt = ksk * ciw * mp.inv_haf2;
      const double sdt = -(kx_ * d.s[0] + ky_ * d.s[1] + kz_ * d.s[2]) * ciw * mp.inv_haf;
      const double sdpb = sa * ciw;
      const double pdd = mp.no_shot ? raw_dd : raw_dd - sdd;
      const double ppp = mp.no_shot ? raw_pp : raw_pp - spp;
      const double ptt = mp.no_shot ? raw_tt : raw_tt - stt;
      const double pim = mp.no_shot ? dt_im : dt_im - sdt;
      const double pbre = mp.no_shot ? dpb_re : dpb_re - sdpb;
      const double kmag = mp.kf * sqrt(static_cast<double>(n2));
      const double mu = __ddiv_rn(__dadd_rn(__dadd_rn(__dmul_rn(static_cast<double>(nx), a0),
                                                      __dmul_rn(static_cast<double>(ny), a1)),
                                            __dmul_rn(static_cast<double>(nz), a2)),
                                  __dsqrt_rn(static_cast<double>(n2)));
      // this mode and, for kz > 0, its mirror -n
      for (int side = 0; side < (nz > 0 ? 2 : 1); ++side) {
        const double sg = side ? -1.0 : 1.0;
        const double mus = side ? -mu : mu;
        const int cell = kb * mp.n_mu + mu_cell(mus, mp.n_mu);
        MuRun& run = side ? rb : ra;
        if (cell != run.cell) {
          run.flush(lbins);
          run.reset(cell);
        }
        run.q[MCount] += 1.0;
        run.q[MKsum] += kmag;
        run.q[MMusum] += mus;
        run.q[MPdd] += pdd;
        run.q[MPpp] += ppp;
        run.q[MPtt] += ptt;
        run.q[MPdtRe] += dt_re;
        run.q[MPdtIm] += sg * pim;
        run.q[MPdpbRe] += pbre;
        run.q[MPdpbIm] += sg * dpb_im;
        run.q[MSdd] += sdd;
        run.q[MSpp] += spp;
        run.q[MStt] += stt;
        run.q[MSdtIm] += sg * sdt;
        run.q[MSdpb] += sdpb;
      }
    }
    ra.flush(lbins);
    rb.flush(lbins);
  }
  __syncthreads();
  const int ncell = mp.n_bins * mp.n_mu;
  for (int i = threadIdx.x; i < ncell * kNumQMu; i += NT)
    partials[static_cast<int64_t>(blockIdx.x) * kMaxMuCells * kNumQMu + i] = lbins[i];
}

// Sum of one quantity over the per-workgroup partials (stride `stride`
// doubles apart) by one wave, in a fixed order: lane l adds partials
// l, l + 64, ... in turn, then the lanes combine in a fixed butterfly.  The
// result (valid in every lane) does not depend on timing.
__device__ __forceinline__ double wave_fixed_sum(const double* __restrict__ p, int nblocks, int64_t stride) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += p[static_cast<int64_t>(b) * stride];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

// Fixed-order sum of the (k, mu) partials, then means (times V); empty cells
// NaN.  One workgroup per cell, one wave per quantity.
__global__ __launch_bounds__(64 * kNumQMu) void finalize_mu_kernel(const double* __restrict__ partials,
                                                                  int nblocks, double volume,
                                                                  double* __restrict__ out) {
  const int c = blockIdx.x, q = threadIdx.x >> 6;
  __shared__ double sums[kNumQMu];
  const double s = wave_fixed_sum(partials + static_cast<int64_t>(c) * kNumQMu + q, nblocks,
                                  static_cast<int64_t>(kMaxMuCells) * kNumQMu);
  if ((threadIdx.x & 63) == 0) sums[q] = s;
  __syncthreads();
  if (threadIdx.x >= kNumQMu) return;
  const int k = threadIdx.x;
  const double cnt = sums[MCount];
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  const double inv = cnt > 0 ? 1.0 / cnt : 0.0;
  double v;
  if (k == MCount) v = cnt;
  else if (k == MKsum || k == MMusum) v = cnt > 0 ? sums[k] * inv : nan;
  else v = cnt > 0 ? volume * sums[k] * inv : nan;
  out[static_cast<int64_t>(c) * kNumQMu + k] = v;
}

// Fixed-order reduction of the workgroup partials and the final per-bin
// means (times V = L^3); empty bins are NaN.  One workgroup per bin, one
// wave per accumulated quantity.
__global__ __launch_bounds__(64 * kNumQ) void finalize_kernel(const double* __restrict__ partials, int nblocks,
                                                             double volume, double* __restrict__ out) {
  const int b = blockIdx.x, q = threadIdx.x >> 6;
  __shared__ double sums[kNumQ];
  const double s = wave_fixed_sum(partials + static_cast<int64_t>(b) * kNumQ + q, nblocks,
                                  static_cast<int64_t>(kMaxBins) * kNumQ);
  if ((threadIdx.x & 63) == 0) sums[q] = s;
  __syncthreads();
  if (threadIdx.x >= kNumQ) return;
  const int k = threadIdx.x;
  const double cnt = sums[QCount];
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  const double inv = cnt > 0 ? 1.0 / cnt : 0.0;
  double v;
  if (k == QCount) v = cnt;
  else if (k == QKsum) v = cnt > 0 ? sums[k] * inv : nan;
  else v = cnt > 0 ? volume * sums[k] * inv : nan;
  out[b * kNumQ + k] = v;
}

template <typename T>
struct FftDims {
  // 128-byte row segments on grids up to 1024^3 (at 1024^3 one workgroup
  // per CU: 131 KB of LDS, against 64-byte segments at two per CU, FP64
  // 28.1 -> 18.6 ms)
  static constexpr int ColsY(int n) {
    const int b = (std::is_same<T, float>::value ? 16 : 8) * 512 / (n > 1024 ? n / 2 : 512);
    return b < n / 2 ? b : n / 2;
  }
  static constexpr int ColsX(int n) {
    const int b = (std::is_same<T, float>::value ? 8 : 4) * 512 / (n > 512 ? n : 512);
    return b < n / 2 ? b : n / 2;
  }
  static constexpr int RowsZ(int n) {
    const int m = n / 2;
    const int p = (std::is_same<T, float>::value ? 4096 : 2048) / m;
    const int rows = 4 * n * n;
    return p < rows ? (p < 1 ? 1 : p) : rows;
  }
};

template <typename T, int N>
hipError_t run_z(Plan* p, void* grid, hipStream_t s) {
  constexpr int P = FftDims<T>::RowsZ(N);
  const int64_t rows = static_cast<int64_t>(kNumFields) * N * N;
  fft_z_kernel<T, N, P, 256><<<static_cast<unsigned>(rows / P), 256, 0, s>>>(
      static_cast<T*>(grid), static_cast<const cpx<T>*>(p->d_twiddle));
  return hipGetLastError();
}

template <typename T, int N>
hipError_t run_cols(Plan* p, void* grid, hipStream_t s, bool x_axis) {
  constexpr int B = FftDims<T>::ColsY(N);
  constexpr int M = N / 2;
  const int64_t blocks = static_cast<int64_t>(kNumFields) * N * (M / B);
  const int64_t stride = x_axis ? static_cast<int64_t>(N) * M : M;
  const int64_t outer = x_axis ? M : static_cast<int64_t>(N) * M;
  fft_cols_kernel<T, N, B, 256><<<static_cast<unsigned>(blocks), 256, 0, s>>>(
      static_cast<T*>(grid), static_cast<const cpx<T>*>(p->d_twiddle), stride, outer);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t run_x_bin(Plan* p, const mps_catalog* c, hipStream_t s) {
  constexpr int B = FftDims<T>::ColsX(N);
  BinParams bp;
  bp.kf = 2.0 * M_PI / c->box;
  bp.haf = c->haf;
  bp.inv_haf = 1.0 / c->haf;
  bp.inv_haf2 = bp.inv_haf * bp.inv_haf;
  bp.n_bins = c->n_bins;
  bp.no_shot = (c->flags & MPS_NO_SHOTNOISE) ? 1 : 0;
  bp.no_deconv = (c->flags & MPS_NO_DECONVOLVE) ? 1 : 0;
  bp.bulk = (c->flags & MPS_BULKFLOW_SUBTRACT) ? 1 : 0;
  const int kid = kernel_id(c->flags);
  fft_x_bin_kernel<T, N, B, 512><<<static_cast<unsigned>(p->bin_blocks), 512, 0, s>>>(
      static_cast<const T*>(p->grid), static_cast<const cpx<T>*>(p->d_twiddle), p->d_header, p->d_iwin2[kid],
      p->d_alias[kid], p->d_lut, bp, p->d_bin_partials);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t run_mu_bin(Plan* p, const mps_catalog* c, int n_mu, const double* axis, hipStream_t s) {
  MuParams mp;
  mp.kf = 2.0 * M_PI / c->box;
  mp.inv_haf = 1.0 / c->haf;
  mp.inv_haf2 = mp.inv_haf * mp.inv_haf;
  mp.axis_given = axis ? 1 : 0;
  for (int a = 0; a < 3; ++a) mp.axis[a] = axis ? axis[a] : 0.0;
  mp.n_bins = c->n_bins;
  mp.n_mu = n_mu;
  mp.no_shot = (c->flags & MPS_NO_SHOTNOISE) ? 1 : 0;
  mp.no_deconv = (c->flags & MPS_NO_DECONVOLVE) ? 1 : 0;
  mp.bulk = (c->flags & MPS_BULKFLOW_SUBTRACT) ? 1 : 0;
  const int kid = kernel_id(c->flags);
  mu_bin_kernel<T, N, 512><<<static_cast<unsigned>(p->num_cus), 512, 0, s>>>(
      static_cast<const T*>(p->grid), p->d_header, p->d_iwin2[kid], p->d_alias[kid], p->d_lut, mp,
      p->d_mu_partials);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_mu(Plan* p, const mps_catalog* c, int n_mu, const double* axis, hipStream_t s) {
  switch (p->n) {
    case 8: return run_mu_bin<T, 8>(p, c, n_mu, axis, s);
    case 16: return run_mu_bin<T, 16>(p, c, n_mu, axis, s);
    case 32: return run_mu_bin<T, 32>(p, c, n_mu, axis, s);
    case 64: return run_mu_bin<T, 64>(p, c, n_mu, axis, s);
    case 128: return run_mu_bin<T, 128>(p, c, n_mu, axis, s);
    case 256: return run_mu_bin<T, 256>(p, c, n_mu, axis, s);
    case 512: return run_mu_bin<T, 512>(p, c, n_mu, axis, s);
    case 1024: return run_mu_bin<T, 1024>(p, c, n_mu, axis, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_z(Plan* p, void* g, hipStream_t s) {
  switch (p->n) {
    case 8: return run_z<T, 8>(p, g, s);
    case 16: return run_z<T, 16>(p, g, s);
    case 32: return run_z<T, 32>(p, g, s);
    case 64: return run_z<T, 64>(p, g, s);
    case 128: return run_z<T, 128>(p, g, s);
    case 256: return run_z<T, 256>(p, g, s);
    case 512: return run_z<T, 512>(p, g, s);
    case 1024: return run_z<T, 1024>(p, g, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_cols(Plan* p, void* g, hipStream_t s, bool x_axis) {
  switch (p->n) {
    case 8: return run_cols<T, 8>(p, g, s, x_axis);
    case 16: return run_cols<T, 16>(p, g, s, x_axis);
    case 32: return run_cols<T, 32>(p, g, s, x_axis);
    case 64: return run_cols<T, 64>(p, g, s, x_axis);
    case 128: return run_cols<T, 128>(p, g, s, x_axis);
    case 256: return run_cols<T, 256>(p, g, s, x_axis);
    case 512: return run_cols<T, 512>(p, g, s, x_axis);
    case 1024: return run_cols<T, 1024>(p, g, s, x_axis);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_x_bin(Plan* p, const mps_catalog* c, hipStream_t s) {
  switch (p->n) {
    case 8: return run_x_bin<T, 8>(p, c, s);
    case 16: return run_x_bin<T, 16>(p, c, s);
    case 32: return run_x_bin<T, 32>(p, c, s);
    case 64: return run_x_bin<T, 64>(p, c, s);
    case 128: return run_x_bin<T, 128>(p, c, s);
    case 256: return run_x_bin<T, 256>(p, c, s);
    case 512: return run_x_bin<T, 512>(p, c, s);
    case 1024: return run_x_bin<T, 1024>(p, c, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_fft_z(Plan* p, void* grid, hipStream_t s) {
  return p->prec == MPS_F32 ? dispatch_z<float>(p, grid, s) : dispatch_z<double>(p, grid, s);
}

hipError_t launch_fft_y(Plan* p, void* grid, hipStream_t s) {
  return p->prec == MPS_F32 ? dispatch_cols<float>(p, grid, s, false) : dispatch_cols<double>(p, grid, s, false);
}

hipError_t launch_fft_x_store(Plan* p, void* grid, hipStream_t s) {
  return p->prec == MPS_F32 ? dispatch_cols<float>(p, grid, s, true) : dispatch_cols<double>(p, grid, s, true);
}

hipError_t launch_fft_x_bin(Plan* p, const mps_catalog* c, hipStream_t s) {
  return p->prec == MPS_F32 ? dispatch_x_bin<float>(p, c, s) : dispatch_x_bin<double>(p, c, s);
}

hipError_t launch_mu_bin(Plan* p, const mps_catalog* c, int n_mu, const double* axis, hipStream_t s) {
  return p->prec == MPS_F32 ? dispatch_mu<float>(p, c, n_mu, axis, s) : dispatch_mu<double>(p, c, n_mu, axis, s);
}

hipError_t launch_finalize_mu(Plan* p, const mps_catalog* c, int n_mu, hipStream_t s) {
  const int ncell = c->n_bins * n_mu;
  const double vol = c->box * c->box * c->box;
  finalize_mu_kernel<<<ncell, 64 * kNumQMu, 0, s>>>(p->d_mu_partials, p->num_cus, vol, p->d_mu_bins);
  return hipGetLastError();
}

hipError_t launch_finalize(Plan* p, const mps_catalog* c, hipStream_t s) {
  const double vol = c->box * c->box * c->box;
  finalize_kernel<<<c->n_bins, 64 * kNumQ, 0, s>>>(p->d_bin_partials, p->bin_blocks, vol, p->d_bins);
  return hipGetLastError();
}

}  // namespace mps
