// One-loop standard perturbation theory predictions of the momentum
// spectra (the one-loop section and its appendices: Eqs. Ppd, PpdD4,
// pdivpD4, the P13 / P22 formulas, Eq. intBktree with I1-I3, Eq. Pcov),
// evaluated on the GPU in FP64.
//
// Every quantity is an integral over a tabulated linear spectrum P0
// (log-log linear between nodes, zero outside the table):
//   P_xy,13 = c_xy P0(k) k^3/(4 pi^2) int dr P0(kr) K_xy(r)
//   P_xy,22 = k^3/(98 4 pi^2) int dr P0(kr) int dx P0(k sqrt(y)) N_x N_y / y^2
//   I1, I2, I3, P_cov^I, P_cov^II as printed, y = 1 + r^2 - 2 r x.
// The logarithm of each K_xy is multiplied by 3/r^3 (read so: with the
// printed 3/r^2 the kernels diverge as r -> 0).
//
// Quadrature.  Outer variable q = k r, in ln q, on panels between
// breakpoints built on the host: the table nodes (kinks of P0(q)), the q
// where a kink of P0(|k - q|) enters or leaves the x range (|k +- q| = node),
// r = 1 and points graded geometrically towards it (the (r-1)^3 ln|r-1|
// term of K_xy), and decades below the table for I2, which has no P0(kr)
// factor.  Inner variable p = k sqrt(y) = |k - q| in ln p, on panels
// between the table nodes, with dx = p dp / (k q).  Gauss-Legendre with
// kGl nodes per panel throughout.  One wave per outer node: lanes share its
// inner nodes and the wave reduces; per-block partial sums are reduced in a
// fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace mps {
namespace {

constexpr int kGl = 8;
constexpr int kSptThreads = 256;
constexpr int kSptSums = 11;  // 7 double integrals, 3 P13 integrals, I3's integral
enum SptSum { SP22 = 0, SP22dt, SP22tt, SI1, SPcov1, SPcov2, SI2, SP13, SP13dt, SP13tt, SI3 };

// Gauss-Legendre nodes and weights on [-1, 1], 8 points
__constant__ double c_gl_x[kGl] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                                    -0.1834346424956498, 0.1834346424956498,  0.5255324099163290,
                                    0.7966664774136267,  0.9602898564975363};
__constant__ double c_gl_w[kGl] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                                    0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                                    0.2223810344533745, 0.1012285362903763};

// K_xy(r) of the three P13 integrals.  Between 0.2 and 5 the closed form
// (its cancellations cost at most ~1e-13 there); outside, its expansions in
// r^2 and in 1/r^2 (coefficients of r^0, r^2, ..., r^16 and of r^0,
// r^-2, ..., r^-16, exact rationals of the closed form's series).
struct K13 {
  double a0, a1, a2, a3, A, B;
  double small[9], large[9];
};

__constant__ K13 c_k13[3] = {
    {12, -158, 100, -42, 7, 2,
     {-168.0, 928.0 / 5, -4512.0 / 35, 416.0 / 21, 2656.0 / 1155, 3232.0 / 5005, 544.0 / 2145, 4384.0 / 36465,
      2976.0 / 46189},
     {-488.0 / 5, 96.0 / 5, -160.0 / 21, -1376.0 / 1155, -1952.0 / 5005, -2528.0 / 15015, -3104.0 / 36465,
      -2208.0 / 46189, -32.0 / 1105}},
    {24, -202, 56, -30, 5, 4,
     {-168.0, 416.0 / 5, -2976.0 / 35, 224.0 / 15, 2144.0 / 1155, 544.0 / 1001, 3296.0 / 15015, 352.0 / 3315,
      13344.0 / 230945},
     {-200.0, 2208.0 / 35, -1312.0 / 105, -1888.0 / 1155, -32.0 / 65, -608.0 / 3003, -3616.0 / 36465,
      -12576.0 / 230945, -4768.0 / 146965}},
    {12, -82, 4, -6, 1, 2,
     {-56.0, -32.0 / 5, -96.0 / 7, 352.0 / 105, 544.0 / 1155, 736.0 / 5005, 928.0 / 15015, 224.0 / 7293,
      3936.0 / 230945},
     {-504.0 / 5, 1248.0 / 35, -608.0 / 105, -160.0 / 231, -992.0 / 5005, -1184.0 / 15015, -1376.0 / 36465,
      -4704.0 / 230945, -352.0 / 29393}},
};

__device__ double kernel13(int kind, double r) {
  const K13& c = c_k13[kind];
  if (r < 0.2 || r > 5.0) {
    const double t = r < 0.2 ? r * r : 1.0 / (r * r);
    const double* s = r < 0.2 ? c.small : c.large;
    double v = s[8];
    for (int j = 7; j >= 0; --j) v = v * t + s[j];
    return v;
  }
  const double r2 = r * r;
  const double d = r2 - 1.0;
  if (d == 0.0) return c.a0 + c.a1 + c.a2 + c.a3;  // the log term vanishes at r = 1
  const double lg = log(fabs((1.0 + r) / (1.0 - r)));
  return c.a0 / r2 + c.a1 + c.a2 * r2 + c.a3 * r2 * r2 + 3.0 / (r2 * r) * d * d * d * (c.A * r2 + c.B) * lg;
}

struct SptArgs {
  const double* k;      // n_k
  const double* bp;     // n_k x stride breakpoints (ascending q)
  const int* nbp;       // n_k
  int stride;
  const double* lk;     // ln k_i
  const double* lp;     // ln P_i
  const double* slope;  // (lp[i+1] - lp[i]) / (lk[i+1] - lk[i])
  int n_tab;
  double* partials;     // n_k x blocks_per_k x kSptSums
  int blocks_per_k;
};

// index i of the table interval [lk[i], lk[i+1]] holding s (clamped)
__device__ __forceinline__ int interval(const double* lk, int n, double s) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (lk[mid] <= s) lo = mid; else hi = mid;
  }
  return lo;
}

// first index with lk[i] > s (n if none)
__device__ __forceinline__ int first_above(const double* lk, int n, double s) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (lk[mid] > s) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__global__ __launch_bounds__(kSptThreads) void spt_kernel(SptArgs a) {
  extern __shared__ double tab[];  // lk, lp, slope
  double* lk = tab;
  double* lp = tab + a.n_tab;
  double* sl = tab + 2 * a.n_tab;
  for (int i = threadIdx.x; i < a.n_tab; i += kSptThreads) {
    lk[i] = a.lk[i];
    lp[i] = a.lp[i];
    sl[i] = a.slope[i];
  }
  __shared__ double red[kSptThreads / 64][kSptSums];
  __syncthreads();
  const int kid = blockIdx.y;
  const double k = a.k[kid];
  const double* bp = a.bp + static_cast<int64_t>(kid) * a.stride;
  const int n_outer = (a.nbp[kid] - 1) * kGl;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n_waves = a.blocks_per_k * (kSptThreads / 64);
  const double q0 = exp(lk[0]), q1 = exp(lk[a.n_tab - 1]);
  double acc[kSptSums];
  for (int j = 0; j < kSptSums; ++j) acc[j] = 0.0;

  for (int o = blockIdx.x * (kSptThreads / 64) + wave; o < n_outer; o += n_waves) {
    const int pan = o / kGl, g = o % kGl;
    const double sa = log(bp[pan]), sb = log(bp[pan + 1]);
    const double half = 0.5 * (sb - sa);
    const double sq = 0.5 * (sa + sb) + half * c_gl_x[g];
    const double q = exp(sq);
    const double dr = half * c_gl_w[g] * q / k;  // dr = dq / k = q ds / k
    const double r = q / k;
    double p0q = 0.0;
    if (q >= q0 && q <= q1) {
      const int i = interval(lk, a.n_tab, sq);
      p0q = exp(lp[i] + sl[i] * (sq - lk[i]));
    }
    // inner range of p = |k - q| over x in [-1, 1], within the table
    const double plo = fmax(fabs(k - q), q0), phi = fmin(k + q, q1);
    double s7[7] = {0, 0, 0, 0, 0, 0, 0};
    if (plo < phi) {
      const double slo = log(plo), shi = log(phi);
      // >= 1 as plo >= k_0 (clamped against rounding of ln k_0)
      const int i_first = max(1, min(first_above(lk, a.n_tab, slo), a.n_tab - 1));
      int i_last = first_above(lk, a.n_tab, shi) - 1;      // last node <= shi
      if (i_last >= 0 && lk[i_last] >= shi) --i_last;      // strictly below
      const int n_pan = (i_last >= i_first ? i_last - i_first + 1 : 0) + 1;
      const double inv_kq = 1.0 / (k * q);
      for (int m = lane; m < n_pan * kGl; m += 64) {
        const int j = m / kGl, h = m % kGl;
        const double ea = j == 0 ? slo : lk[i_first + j - 1];
        const double eb = j == n_pan - 1 ? shi : lk[i_first + j];
        const int it = i_first - 1 + j;  // table interval of this panel
        const double hh = 0.5 * (eb - ea);
        const double s = 0.5 * (ea + eb) + hh * c_gl_x[h];
        const double p = exp(s);
        const double w = hh * c_gl_w[h] * p * p * inv_kq * exp(lp[it] + sl[it] * (s - lk[it]));
        const double x = (k * k + q * q - p * p) * 0.5 * inv_kq;
        const double y = (p / k) * (p / k);
        const double nd = 3.0 * r + 7.0 * x - 10.0 * r * x * x;
        const double nt = 7.0 * x - r - 6.0 * r * x * x;
        const double iy = 1.0 / y;
        const double iy2 = iy * iy;
        s7[SP22] += w * nd * nd * iy2;
        s7[SP22dt] += w * nd * nt * iy2;
        s7[SP22tt] += w * nt * nt * iy2;
        s7[SI1] += w * x * (r - 7.0 * x + 6.0 * r * x * x) * iy;
        s7[SPcov1] += w;
        s7[SPcov2] += w * r * (x - r) * iy;
        s7[SI2] += w * r * r * r * x * (7.0 * r * x - 1.0 - 6.0 * x * x) * iy;
      }
      for (int j = 0; j < 7; ++j)
        for (int off = 32; off > 0; off >>= 1) s7[j] += __shfl_xor(s7[j], off);
    }
    if (lane == 0) {
      for (int j = 0; j < 6; ++j) acc[j] += dr * p0q * s7[j];
      acc[SI2] += dr * s7[SI2];
      if (p0q > 0.0) {
        acc[SP13] += dr * p0q * kernel13(0, r);
        acc[SP13dt] += dr * p0q * kernel13(1, r);
        acc[SP13tt] += dr * p0q * kernel13(2, r);
        acc[SI3] += dr * p0q * (r * r + 1.0);
      }
    }
  }
  if (lane == 0)
    for (int j = 0; j < kSptSums; ++j) red[wave][j] = acc[j];
  __syncthreads();
  if (threadIdx.x < kSptSums) {
    double v = 0.0;
    for (int w = 0; w < kSptThreads / 64; ++w) v += red[w][threadIdx.x];
    a.partials[(static_cast<int64_t>(kid) * a.blocks_per_k + blockIdx.x) * kSptSums + threadIdx.x] = v;
  }
}

constexpr int kSptOut = MPS_SPT_NUM_OUT;

// One thread per k: fixed-order sum of the partials, prefactors, and the
// combined one-loop spectra.
__global__ void spt_finish_kernel(const double* __restrict__ partials, int blocks_per_k, const double* kv, int n_k,
                                  const double* lk, const double* lp, const double* slope, int n_tab, double d_z,
                                  double haf, double* out) {
  const int kid = blockIdx.x * blockDim.x + threadIdx.x;
  if (kid >= n_k) return;
  double s[kSptSums];
  for (int j = 0; j < kSptSums; ++j) s[j] = 0.0;
  for (int b = 0; b < blocks_per_k; ++b)
    for (int j = 0; j < kSptSums; ++j) s[j] += partials[(static_cast<int64_t>(kid) * blocks_per_k + b) * kSptSums + j];
  const double k = kv[kid];
  const double sk = log(k);
  double p0 = 0.0;
  if (sk >= lk[0] && sk <= lk[n_tab - 1]) {
    const int i = interval(lk, n_tab, sk);
    p0 = exp(lp[i] + slope[i] * (sk - lk[i]));
  }
  const double f3 = k * k * k / (4.0 * M_PI * M_PI), f1 = k / (4.0 * M_PI * M_PI);
  double* o = out + static_cast<int64_t>(kid) * kSptOut;
  const double p13 = p0 * f3 / 504.0 * s[SP13], p13dt = p0 * f3 / 504.0 * s[SP13dt];
  const double p13tt = p0 * f3 / 168.0 * s[SP13tt];
  const double p22 = f3 / 98.0 * s[SP22], p22dt = f3 / 98.0 * s[SP22dt], p22tt = f3 / 98.0 * s[SP22tt];
  const double i1 = -f1 / 7.0 * s[SI1], i2 = f1 / 7.0 * p0 * s[SI2], i3 = -2.0 / 3.0 * f1 * p0 * s[SI3];
  const double c1 = f3 * s[SPcov1], c2 = f3 * s[SPcov2];
  const double d2 = d_z * d_z, d4 = d2 * d2;
  o[0] = p13;
  o[1] = p22;
  o[2] = p13dt;
  o[3] = p22dt;
  o[4] = p13tt;
  o[5] = p22tt;
  o[6] = i1;
  o[7] = i2;
  o[8] = i3;
  o[9] = c1;
  o[10] = c2;
  o[11] = d2 * p0;
  o[12] = d2 * p0 + d4 * (2.0 * p13 + p22);
  o[13] = d2 * p0 + d4 * (6.0 * p13 + 4.0 * p22);
  o[14] = d2 * p0 + d4 * (4.0 * p13 + 2.0 * p22);
  const double ptt1 = 2.0 * p13tt + p22tt;
  o[15] = (haf / k) * (haf / k) * (d2 * p0 + d4 * (ptt1 + c1 + c2 + 2.0 * k * k * (i1 + i2 + i3)));
}

// Breakpoints of the outer integral at one k (ascending, unique).
void breakpoints(double k, const std::vector<double>& tk, std::vector<double>* out) {
  const double k0 = tk.front(), k1 = tk.back();
  const double lo = std::min(k0, 1e-6 * k), hi = k + k1;
  std::vector<double>& v = *out;
  v.clear();
  v.push_back(lo);
  v.push_back(hi);
  for (double t : tk) {
    v.push_back(t);
    v.push_back(std::fabs(k - t));
    v.push_back(k + t);
  }
  v.push_back(k);
  for (int j = 0; j <= 26; ++j) {  // graded towards r = 1
    const double e = 0.5 * std::ldexp(1.0, -j);
    v.push_back(k * (1.0 - e));
    v.push_back(k * (1.0 + e));
  }
  for (double d = lo * 3.1622776601683795; d < k0; d *= 3.1622776601683795) v.push_back(d);  // half decades
  std::sort(v.begin(), v.end());
  std::vector<double> u;
  for (double x : v)
    if (x >= lo && x <= hi && (u.empty() || x > u.back())) u.push_back(x);
  v.swap(u);
}

}  // namespace
}  // namespace mps

using namespace mps;

extern "C" int mps_spt_one_loop(const double* k, int n_k, const double* table_k, const double* table_p,
                                int n_table, double d_z, double haf, mps_spt_result* out, hipStream_t stream) {
  if (!k || !table_k || !table_p || !out) return MPS_E_ARG;
  if (n_k < 1 || n_k > MPS_SPT_MAX_K || n_table < 2 || n_table > MPS_SPT_MAX_TABLE) return MPS_E_ARG;
  if (!std::isfinite(d_z) || !(haf > 0.0) || !std::isfinite(haf)) return MPS_E_ARG;
  std::vector<double> tk(table_k, table_k + n_table), lk(n_table), lp(n_table), sl(n_table, 0.0);
  for (int i = 0; i < n_table; ++i) {
    if (!(table_k[i] > 0.0) || !std::isfinite(table_k[i]) || !(table_p[i] > 0.0) || !std::isfinite(table_p[i]))
      return MPS_E_ARG;
    if (i > 0 && !(table_k[i] > table_k[i - 1])) return MPS_E_ARG;
    lk[i] = std::log(table_k[i]);
    lp[i] = std::log(table_p[i]);
  }
  for (int i = 0; i + 1 < n_table; ++i) sl[i] = (lp[i + 1] - lp[i]) / (lk[i + 1] - lk[i]);
  std::vector<std::vector<double>> bps(n_k);
  int stride = 0;
  for (int i = 0; i < n_k; ++i) {
    if (!(k[i] > 0.0) || !std::isfinite(k[i])) return MPS_E_ARG;
    breakpoints(k[i], tk, &bps[i]);
    stride = std::max(stride, static_cast<int>(bps[i].size()));
  }
  std::vector<double> bp(static_cast<size_t>(n_k) * stride, 0.0);
  std::vector<int> nbp(n_k);
  for (int i = 0; i < n_k; ++i) {
    std::copy(bps[i].begin(), bps[i].end(), bp.begin() + static_cast<size_t>(i) * stride);
    nbp[i] = static_cast<int>(bps[i].size());
  }
  int bpk = 2048 / n_k;
  bpk = bpk < 1 ? 1 : (bpk > 64 ? 64 : bpk);

  double *d_k = nullptr, *d_bp = nullptr, *d_tab = nullptr, *d_part = nullptr, *d_out = nullptr;
  int* d_nbp = nullptr;
  const size_t out_n = static_cast<size_t>(n_k) * kSptOut;
  std::vector<double> h_out(out_n);
  int st = MPS_OK;
  bool ok = hipMalloc(&d_k, sizeof(double) * n_k) == hipSuccess;
  ok = ok && hipMalloc(&d_bp, sizeof(double) * bp.size()) == hipSuccess;
  ok = ok && hipMalloc(&d_nbp, sizeof(int) * n_k) == hipSuccess;
  ok = ok && hipMalloc(&d_tab, sizeof(double) * 3 * n_table) == hipSuccess;
  ok = ok && hipMalloc(&d_part, sizeof(double) * n_k * bpk * kSptSums) == hipSuccess;
  ok = ok && hipMalloc(&d_out, sizeof(double) * out_n) == hipSuccess;
  if (!ok) st = MPS_E_NOMEM;
  if (st == MPS_OK) {
    bool up = hipMemcpyAsync(d_k, k, sizeof(double) * n_k, hipMemcpyHostToDevice, stream) == hipSuccess;
    up = up && hipMemcpyAsync(d_bp, bp.data(), sizeof(double) * bp.size(), hipMemcpyHostToDevice, stream) == hipSuccess;
    up = up && hipMemcpyAsync(d_nbp, nbp.data(), sizeof(int) * n_k, hipMemcpyHostToDevice, stream) == hipSuccess;
    up = up && hipMemcpyAsync(d_tab, lk.data(), sizeof(double) * n_table, hipMemcpyHostToDevice, stream) == hipSuccess;
    up = up && hipMemcpyAsync(d_tab + n_table, lp.data(), sizeof(double) * n_table, hipMemcpyHostToDevice, stream) ==
                   hipSuccess;
    up = up && hipMemcpyAsync(d_tab + 2 * n_table, sl.data(), sizeof(double) * n_table, hipMemcpyHostToDevice,
                              stream) == hipSuccess;
    SptArgs a;
    a.k = d_k;
    a.bp = d_bp;
    a.nbp = d_nbp;
    a.stride = stride;
    a.lk = d_tab;
    a.lp = d_tab + n_table;
    a.slope = d_tab + 2 * n_table;
    a.n_tab = n_table;
    a.partials = d_part;
    a.blocks_per_k = bpk;
    if (up) {
      spt_kernel<<<dim3(bpk, n_k), kSptThreads, sizeof(double) * 3 * n_table, stream>>>(a);
      spt_finish_kernel<<<(n_k + 127) / 128, 128, 0, stream>>>(d_part, bpk, d_k, n_k, a.lk, a.lp, a.slope, n_table,
                                                               d_z, haf, d_out);
      up = hipGetLastError() == hipSuccess;
    }
    up = up && hipMemcpyAsync(h_out.data(), d_out, sizeof(double) * out_n, hipMemcpyDeviceToHost, stream) ==
                   hipSuccess;
    up = up && hipStreamSynchronize(stream) == hipSuccess;
    if (!up) st = MPS_E_HIP;
  }
  for (void* ptr : {static_cast<void*>(d_k), static_cast<void*>(d_bp), static_cast<void*>(d_nbp),
                    static_cast<void*>(d_tab), static_cast<void*>(d_part), static_cast<void*>(d_out)})
    if (ptr) (void)hipFree(ptr);
  if (st != MPS_OK) return st;
  double* const dst[kSptOut] = {out->p13,  out->p22, out->p13_dt, out->p22_dt, out->p13_tt, out->p22_tt,
                                out->i1,   out->i2,  out->i3,     out->pcov1,  out->pcov2,  out->p_lin,
                                out->p_dd, out->p_theta_p, out->p_dtheta_p, out->p_mom};
  for (int j = 0; j < kSptOut; ++j)
    if (dst[j])
      for (int i = 0; i < n_k; ++i) dst[j][i] = h_out[static_cast<size_t>(i) * kSptOut + j];
  return MPS_OK;
}
