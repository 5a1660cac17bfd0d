// C ABI of the estimator: plan management, argument validation, stage
// scheduling on the caller's stream and result unpacking.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.h"

namespace mps {

hipError_t launch_scatter_impl(Plan* p, const mps_catalog* c, hipStream_t s, int bulk);

namespace {

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <typename T>
hipError_t dalloc(T** ptr, size_t bytes) {
  *ptr = nullptr;
  return hipMalloc(reinterpret_cast<void**>(ptr), bytes < 1 ? 1 : bytes);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

size_t real_bytes(mps_precision prec) { return prec == MPS_F64 ? 8 : 4; }


int num_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}


void release(Plan* p) {
  if (!p) return;
  dfree(p->grid);
  dfree(p->sorted);
  dfree(p->tile_count);
  dfree(p->tile_offset);
  dfree(p->tile_cursor);
  dfree(p->tile_queue);
  dfree(p->halo);
  dfree(p->pair_scratch);
  dfree(p->moment_partials);
  dfree(p->d_header);
  for (int k = 0; k < kNumKernels; ++k) {
    dfree(p->d_iwin2[k]);
    dfree(p->d_alias[k]);
  }
  dfree(p->d_twiddle);
  dfree(p->d_lut);
  dfree(p->d_bin_partials);
  dfree(p->d_bins);
  dfree(p->d_mu_partials);
  dfree(p->d_mu_bins);
  dfree(p->host_stage);
  dfree(p->split_pos);
  dfree(p->split_vel);
  dfree(p->split_w);
  dfree(p->split_count);
  dfree(p->split_offset);
  dfree(p->split_cursor);
  if (p->h_split) (void)hipHostFree(p->h_split);
  if (p->h_stage_sub) (void)hipHostFree(p->h_stage_sub);
  if (p->h_stage_mu) (void)hipHostFree(p->h_stage_mu);
  if (p->h_stage) (void)hipHostFree(p->h_stage);
  for (int i = 0; i < Plan::kSubLanes; ++i) {
    if (i > 0 && p->sub_plan[i - 1]) release(p->sub_plan[i - 1]);
    if (p->sub_stream[i]) (void)hipStreamDestroy(p->sub_stream[i]);
    if (p->sub_done[i]) (void)hipEventDestroy(p->sub_done[i]);
  }
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

}  // namespace

int validate_catalog(const Plan* p, const mps_catalog* c) {
  if (!c || !c->pos || !c->vel) return MPS_E_ARG;
  if (c->n_particles < 1 || c->n_particles > 0x7fffffffll) return MPS_E_ARG;
  if (!(c->box > 0.0) || !std::isfinite(c->box)) return MPS_E_ARG;
  if (!(c->haf > 0.0) || !std::isfinite(c->haf)) return MPS_E_ARG;
  if (c->n_bins < 1 || c->n_bins > kMaxBins) return MPS_E_ARG;
  if (c->flags & ~(15u | (7u << MPS_KERNEL_ORDER_SHIFT) | MPS_CATALOG_HOST)) return MPS_E_ARG;
  const uint32_t order = (c->flags >> MPS_KERNEL_ORDER_SHIFT) & 7u;
  if (order != 0 && (c->flags & MPS_KERNEL_BL3_EXACT)) return MPS_E_ARG;
  (void)p;
  return MPS_OK;
}

int ensure_bins(Plan* p, const mps_catalog* c) {
  std::vector<double> key;
  if (c->k_edges) key.assign(c->k_edges, c->k_edges + c->n_bins + 1);
  if (p->lut_box == c->box && p->lut_nbins == c->n_bins && p->lut_edges == key) return MPS_OK;
  std::vector<int32_t> lut;
  std::vector<double> edges;
  if (!bin_lut(p->n, c->box, c->n_bins, c->k_edges, &lut, &edges)) return MPS_E_ARG;
  if (hipMemcpy(p->d_lut, lut.data(), lut.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
    return MPS_E_HIP;
  p->lut_box = c->box;
  p->lut_nbins = c->n_bins;
  p->lut_edges = key;
  p->edges_used = edges;
  return MPS_OK;
}

int ensure_particles(Plan* p, int64_t np) {
  if (np <= p->sorted_cap) return MPS_OK;
  dfree(p->sorted);
  p->sorted = nullptr;
  p->sorted_cap = 0;
  if (dalloc(&p->sorted, static_cast<size_t>(np) * 2 * sizeof(float4)) != hipSuccess) return MPS_E_NOMEM;
  p->sorted_cap = np;
  return MPS_OK;
}

int ensure_halo(Plan* p) {
  if (p->halo) return MPS_OK;
  const size_t b = halo_bytes(p->n, p->prec);
  if (b == 0) return MPS_OK;
  return dalloc(&p->halo, b) == hipSuccess ? MPS_OK : MPS_E_NOMEM;
}

// Whether the scatter of np particles can take paired deposits: 16^3 tiles
// in the atomic form (FP32 or FP64 grids).
bool pairs_reachable(int n, mps_precision prec, int64_t np) {
  return tile_for(n, prec) == 16 && scatter_form_for(n, prec, np) == kFormAtomic;
}

int ensure_pair_scratch(Plan* p) {
  if (p->pair_scratch) return MPS_OK;
  const size_t b = pair_scratch_bytes(p->n_tiles, p->num_cus);
  if (dalloc(&p->pair_scratch, b) != hipSuccess) return MPS_E_NOMEM;
  p->pair_blocks = static_cast<int>(b / (kPairCap * sizeof(uint32_t)));
  return MPS_OK;
}

int ensure_scatter_space(Plan* p, const mps_catalog* c) {
  int st = ensure_particles(p, c->n_particles);
  if (st != MPS_OK) return st;
  if (kernel_id(c->flags) == 0 && pairs_reachable(p->n, p->prec, c->n_particles) &&
      (st = ensure_pair_scratch(p)) != MPS_OK)
    return st;
  if (kernel_id(c->flags) == 0 && scatter_form_for(p->n, p->prec, c->n_particles) == kFormHalo) return ensure_halo(p);
  return MPS_OK;
}

int ensure_host_stage(Plan* p, int64_t np) {
  if (np <= p->host_cap) return MPS_OK;
  dfree(p->host_stage);
  p->host_stage = nullptr;
  p->host_cap = 0;
  if (dalloc(&p->host_stage, kHostStageBytes * static_cast<size_t>(np)) != hipSuccess) return MPS_E_NOMEM;
  p->host_cap = np;
  return MPS_OK;
}

#define MPS_TRY(expr)                               \
  do {                                              \
    if ((expr) != hipSuccess) return MPS_E_HIP;     \
  } while (0)

void mark(Plan* p, int i, hipStream_t s) {
  if (p->timing) (void)hipEventRecord(p->ev[i], s);
}

// Stages before the scatter: moments, tile sort and the grid clear.  A
// host-resident catalog is first copied to the plan's staging buffer; *used
// receives the catalog the later particle stages read.
int enqueue_prescatter(Plan* p, const mps_catalog* c0, hipStream_t s, mps_catalog* used) {
  *used = *c0;
  if (c0->flags & MPS_CATALOG_HOST) {
    const int st = ensure_host_stage(p, c0->n_particles);
    if (st != MPS_OK) return st;
    const size_t n = static_cast<size_t>(c0->n_particles);
    used->flags &= ~MPS_CATALOG_HOST;
    used->pos = p->host_stage;
    used->vel = p->host_stage + 3 * n;
    used->weight = c0->weight ? p->host_stage + 6 * n : nullptr;
    MPS_TRY(hipMemcpyAsync(p->host_stage, c0->pos, sizeof(float) * 3 * n, hipMemcpyHostToDevice, s));
    MPS_TRY(hipMemcpyAsync(p->host_stage + 3 * n, c0->vel, sizeof(float) * 3 * n, hipMemcpyHostToDevice, s));
    if (c0->weight)
      MPS_TRY(hipMemcpyAsync(p->host_stage + 6 * n, c0->weight, sizeof(float) * n, hipMemcpyHostToDevice, s));
  }
  // only the atomic scatter adds into the grid; the other forms store every cell
  const bool clear_grid = scatter_form(p, used) == kFormAtomic;
  if (!p->timing) {  // a short chain of dependent launches: what small catalogs wait on
    bool cleared = false;
    MPS_TRY(launch_sort_fused(p, used, s, clear_grid, &cleared));
    if (clear_grid && !cleared) MPS_TRY(launch_clear_grid(p, s));
    return MPS_OK;
  }
  mark(p, 0, s);
  MPS_TRY(launch_count(p, used, s));
  MPS_TRY(launch_derive(p, used, s));
  mark(p, 1, s);
  MPS_TRY(launch_scan(p, used, s));
  mark(p, 2, s);
  MPS_TRY(launch_permute(p, used, s));
  mark(p, 3, s);
  if (clear_grid) MPS_TRY(launch_clear_grid(p, s));
  mark(p, 4, s);
  return MPS_OK;
}

// Stages up to (and including) the scatter; `bulk_grid` deposits v - v_b.
int enqueue_particles(Plan* p, const mps_catalog* c0, hipStream_t s, int bulk_grid) {
  mps_catalog c;
  const int st = enqueue_prescatter(p, c0, s, &c);
  if (st != MPS_OK) return st;
  MPS_TRY(launch_scatter_impl(p, &c, s, bulk_grid));
  mark(p, 5, s);
  return MPS_OK;
}

// The stages after the scatter and the copy of the results to `stage`.
int enqueue_postscatter(Plan* p, const mps_catalog* c, hipStream_t s, void* stage) {
  if (!stage) stage = p->h_stage;
  MPS_TRY(launch_fft_z(p, p->grid, s));
  mark(p, 6, s);
  MPS_TRY(launch_fft_y(p, p->grid, s));
  mark(p, 7, s);
  MPS_TRY(launch_fft_x_bin(p, c, s));
  mark(p, 8, s);
  MPS_TRY(launch_finalize(p, c, s));
  mark(p, 9, s);
  const size_t bytes = sizeof(ResultHeader) + sizeof(double) * kNumQ * c->n_bins;
  MPS_TRY(hipMemcpyAsync(stage, p->d_header, sizeof(ResultHeader), hipMemcpyDeviceToHost, s));
  MPS_TRY(hipMemcpyAsync(static_cast<char*>(stage) + sizeof(ResultHeader), p->d_bins,
                         bytes - sizeof(ResultHeader), hipMemcpyDeviceToHost, s));
  return MPS_OK;
}

int enqueue_estimate(Plan* p, const mps_catalog* c, hipStream_t s, void* stage) {
  const int st = enqueue_particles(p, c, s, 0);
  if (st != MPS_OK) return st;
  return enqueue_postscatter(p, c, s, stage);
}

// ------------------------------------------------------------ batches
int BatchWorkspace::ensure(int n) {
  for (hipEvent_t& e : done)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MPS_E_HIP;
  if (n <= cap) return MPS_OK;
  if (d_cats) (void)hipFree(d_cats);
  if (d_starts) (void)hipFree(d_starts);
  if (h_cats) (void)hipHostFree(h_cats);
  if (h_starts) (void)hipHostFree(h_starts);
  d_cats = nullptr;
  d_starts = nullptr;
  h_cats = nullptr;
  h_starts = nullptr;
  cap = 0;
  const int c = n < 64 ? 64 : n;
  bool ok = hipMalloc(reinterpret_cast<void**>(&d_cats), sizeof(ScatterCat) * c) == hipSuccess;
  ok = ok && hipMalloc(reinterpret_cast<void**>(&d_starts), sizeof(int64_t) * (c + kScatterGroups)) == hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h_cats), sizeof(ScatterCat) * c, hipHostMallocDefault) ==
                 hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&h_starts), sizeof(int64_t) * (c + kScatterGroups),
                           hipHostMallocDefault) ==
                 hipSuccess;
  if (!d_queue)
    ok = ok && hipMalloc(reinterpret_cast<void**>(&d_queue), sizeof(uint32_t) * 8 * kScatterGroups) == hipSuccess;
  if (!ok) return MPS_E_NOMEM;
  cap = c;
  return MPS_OK;
}

// Several catalogs, each with its own plan, on n_lanes streams:
//   1. per catalog, round robin on the lanes: moments, sort, clear;
//   2. once every lane has got there: on lanes[0] the own scatter launches
//      of the catalogs no multi-catalog group takes (FP64 grids, the other
//      kernels), then one persistent multi-catalog scatter launch per group
//      (scatter_group: form and record layout), the groups round robin on
//      the lanes so that they overlap each other and the later stages;
//   3. per catalog, round robin, after its group's scatter: FFTs,
//      estimator, finalize, copy back to stages[i] (the plan's own staging
//      buffer when NULL).
// lanes[1..] must be ordered after earlier work by the caller.
int enqueue_batch(Plan* const* plans, const mps_catalog* cats, int n, hipStream_t* lanes, int n_lanes,
                  hipEvent_t* events, BatchWorkspace* ws, void* const* stages) {
  std::vector<mps_catalog> used(n);
  int st = MPS_OK;
  for (int i = 0; i < n && st == MPS_OK; ++i) st = enqueue_prescatter(plans[i], &cats[i], lanes[i % n_lanes], &used[i]);
  if (st != MPS_OK) return st;
  if ((st = ws->ensure(n)) != MPS_OK) return st;
  for (int l = 1; l < n_lanes; ++l) {
    MPS_TRY(hipEventRecord(events[l], lanes[l]));
    MPS_TRY(hipStreamWaitEvent(lanes[0], events[l], 0));
  }
  constexpr int kGroups = kScatterGroups;
  std::vector<int> group(n);
  std::vector<int> multi[kGroups];
  for (int i = 0; i < n; ++i) {
    group[i] = scatter_group(plans[i], &used[i]);
    if (group[i] >= 0) multi[group[i]].push_back(i);
    else MPS_TRY(launch_scatter_impl(plans[i], &used[i], lanes[0], 0));
  }
  MPS_TRY(hipEventRecord(ws->done[kGroups], lanes[0]));
  int nm = 0;
  for (int g = 0; g < kGroups; ++g) nm += static_cast<int>(multi[g].size());
  if (nm > 0) {
    // descriptors of group g at [k_g, k_g + m_g), its prefix sums at [k_g + g, k_g + g + m_g]
    int k = 0;
    for (int g = 0; g < kGroups; ++g) {
      int64_t* starts = ws->h_starts + k + g;
      starts[0] = 0;
      for (size_t j = 0; j < multi[g].size(); ++j) {
        Plan* p = plans[multi[g][j]];
        ws->h_cats[k + j] = scatter_cat(p, &used[multi[g][j]]);
        starts[j + 1] = starts[j] + p->n_tiles;
      }
      k += static_cast<int>(multi[g].size());
    }
    MPS_TRY(hipMemcpyAsync(ws->d_cats, ws->h_cats, sizeof(ScatterCat) * nm, hipMemcpyHostToDevice, lanes[0]));
    MPS_TRY(hipMemcpyAsync(ws->d_starts, ws->h_starts, sizeof(int64_t) * (nm + kGroups), hipMemcpyHostToDevice,
                           lanes[0]));
    MPS_TRY(hipEventRecord(events[0], lanes[0]));  // descriptors in place, every catalog sorted
    k = 0;
    int launched = 0;
    for (int g = 0; g < kGroups; ++g) {
      const int m = static_cast<int>(multi[g].size());
      if (m > 0) {
        hipStream_t lane = lanes[launched++ % n_lanes];
        if (lane != lanes[0]) MPS_TRY(hipStreamWaitEvent(lane, events[0], 0));
        Plan* p0 = plans[multi[g][0]];
        MPS_TRY(launch_scatter_multi(ws->d_cats + k, ws->d_starts + k + g, m, ws->h_starts[k + g + m], g,
                                     p0->taps[0], p0->tap_bound[0], ws->d_queue + 8 * g, p0->num_cus, lane));
        MPS_TRY(hipEventRecord(ws->done[g], lane));
      }
      k += m;
    }
  }
  for (int i = 0; i < n && st == MPS_OK; ++i) {
    hipStream_t lane = lanes[i % n_lanes];
    MPS_TRY(hipStreamWaitEvent(lane, ws->done[group[i] >= 0 ? group[i] : kGroups], 0));
    st = enqueue_postscatter(plans[i], &cats[i], lane, stages ? stages[i] : nullptr);
  }
  return st;
}

namespace {

// a / |a| with |a| = sqrt(a0 a0 + a1 a1 + a2 a2), each operation rounded
// separately (no fused multiply-adds), as the mu bins are documented; false
// for a zero or non-finite vector.
bool unit_axis(const double* a, double* out) {
#pragma clang fp contract(off)
  const double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
  for (int i = 0; i < 3; ++i) out[i] = a[i] / nrm;
  return true;
}

int check_header(const ResultHeader* h) {
  if (h->flags & 1u) return MPS_E_NONFINITE;
  for (int q = 0; q < kMomentSums; ++q)
    if (!std::isfinite(h->sums[q])) return MPS_E_NONFINITE;
  if (h->sums[0] == 0.0) return MPS_E_ZEROWEIGHT;
  return MPS_OK;
}

}  // namespace

int unpack(Plan* p, const mps_catalog* c, mps_result* out, const void* stage) {
  if (!stage) stage = p->h_stage;
  const ResultHeader* h = static_cast<const ResultHeader*>(stage);
  const int st = check_header(h);
  if (st != MPS_OK) return st;
  const double* bins = reinterpret_cast<const double*>(static_cast<const char*>(stage) + sizeof(ResultHeader));
  for (int b = 0; b < c->n_bins; ++b) {
    const double* s = bins + b * kNumQ;
    if (out->n_modes) out->n_modes[b] = static_cast<int64_t>(std::llround(s[QCount]));
    if (out->k_mean) out->k_mean[b] = s[QKsum];
    if (out->p_dd) out->p_dd[b] = s[QPdd];
    if (out->p_pp) out->p_pp[b] = s[QPpp];
    if (out->p_tt) out->p_tt[b] = s[QPtt];
    if (out->p_dt) out->p_dt[b] = s[QPdt];
    if (out->sn_dd) out->sn_dd[b] = s[QSdd];
    if (out->sn_pp) out->sn_pp[b] = s[QSpp];
    if (out->sn_tt) out->sn_tt[b] = s[QStt];
  }
  for (int a = 0; a < 3; ++a) out->v_bulk[a] = h->d.vb[a];
  out->sigma_v2 = h->d.sigma_v2;
  out->n_eff = h->d.W * h->d.W / h->d.W2;
  if (p->timing)
    for (int i = 0; i < kNumStages; ++i) {
      float ms = 0.f;
      p->stage_ms[i] = hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]) == hipSuccess ? ms : -1.0;
    }
  return MPS_OK;
}

namespace {

// Streams, events and multi-scatter workspace of mps_estimate_batch, one set
// per device, created on first use and kept for the process.  Batch calls on
// one device take turns.
struct BatchLanes {
  static constexpr int kLanes = 4;
  std::mutex mu;
  bool made = false;
  hipStream_t lanes[kLanes] = {};
  hipEvent_t ev[kLanes] = {};
  hipEvent_t join[kLanes] = {};
  hipEvent_t start = nullptr;
  BatchWorkspace ws;
  int ready() {
    if (made) return MPS_OK;
    for (int j = 0; j < kLanes; ++j) {
      if (!lanes[j] && hipStreamCreateWithFlags(&lanes[j], hipStreamNonBlocking) != hipSuccess) return MPS_E_HIP;
      if (!ev[j] && hipEventCreateWithFlags(&ev[j], hipEventDisableTiming) != hipSuccess) return MPS_E_HIP;
      if (!join[j] && hipEventCreateWithFlags(&join[j], hipEventDisableTiming) != hipSuccess) return MPS_E_HIP;
    }
    if (!start && hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess) return MPS_E_HIP;
    made = true;
    return MPS_OK;
  }
};

constexpr int kMaxDevices = 16;

BatchLanes& batch_lanes(int dev) {
  static BatchLanes* lanes = new BatchLanes[kMaxDevices];  // kept until the process ends
  return lanes[dev];
}

}  // namespace
}  // namespace mps

using namespace mps;

extern "C" {

int mps_plan_create(mps_plan** out, int n_grid, mps_precision prec) {
  if (!out) return MPS_E_ARG;
  *out = nullptr;
  if (!is_pow2(n_grid) || n_grid < 8 || n_grid > 1024) return MPS_E_ARG;
  if (prec != MPS_F32 && prec != MPS_F64) return MPS_E_ARG;
  Plan* p = new (std::nothrow) Plan();
  if (!p) return MPS_E_NOMEM;
  p->n = n_grid;
  p->prec = prec;
  p->real_size = real_bytes(prec);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return MPS_E_HIP;
  }
  p->tile = tile_for(n_grid, prec);
  const int64_t nt = n_grid / p->tile;
  p->n_tiles = nt * nt * nt;
  const int64_t n3 = static_cast<int64_t>(n_grid) * n_grid * n_grid;
  const int half = n_grid / 2;
  const int items = x_bin_items(n_grid, prec);
  const int cus = num_cus();
  p->num_cus = cus;
  p->bin_blocks = items < cus ? items : cus;
  bool ok = true;
  ok = ok && dalloc(&p->grid, static_cast<size_t>(kNumFields) * n3 * p->real_size) == hipSuccess;
  ok = ok && dalloc(&p->tile_count, sizeof(uint32_t) * p->n_tiles) == hipSuccess;
  ok = ok && dalloc(&p->tile_offset, sizeof(uint32_t) * (p->n_tiles + 1)) == hipSuccess;
  ok = ok && dalloc(&p->tile_cursor, sizeof(uint32_t) * p->n_tiles) == hipSuccess;
  ok = ok && dalloc(&p->tile_queue, sizeof(uint32_t) * 8) == hipSuccess;
  ok = ok && dalloc(&p->moment_partials, sizeof(double) * kMomentBlocks * (kMomentSums + kMomentMax)) == hipSuccess;
  ok = ok && dalloc(&p->d_header, sizeof(ResultHeader)) == hipSuccess;
  for (int k = 0; k < kNumKernels; ++k) {
    ok = ok && dalloc(&p->d_iwin2[k], sizeof(double) * (half + 1)) == hipSuccess;
    ok = ok && dalloc(&p->d_alias[k], sizeof(double) * (half + 1)) == hipSuccess;
  }
  ok = ok && dalloc(&p->d_twiddle, 2 * p->real_size * n_grid) == hipSuccess;
  ok = ok && dalloc(&p->d_lut, sizeof(int32_t) * half * half) == hipSuccess;
  ok = ok && dalloc(&p->d_bin_partials, sizeof(double) * p->bin_blocks * kMaxBins * kNumQ) == hipSuccess;
  ok = ok && dalloc(&p->d_bins, sizeof(double) * kMaxBins * kNumQ) == hipSuccess;
  p->stage_bytes = sizeof(ResultHeader) + sizeof(double) * kMaxBins * kNumQ;
  ok = ok && hipHostMalloc(&p->h_stage, p->stage_bytes, hipHostMallocDefault) == hipSuccess;
  for (auto& e : p->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  if (!ok) {
    release(p);
    return MPS_E_NOMEM;
  }
  const std::vector<double> tw = twiddles(n_grid);
  bool up = true;
  for (int k = 0; k < kNumKernels; ++k) {
    std::vector<double> iwin2, alias;
    if (k == 0) {
      p->taps[k] = bl3_tap_polynomials();
      bl3_axis_tables(n_grid, &iwin2, &alias);
      // the x pass multiplies by W_t^-2 per axis
      for (double& w : iwin2) w = 1.0 / w;
      p->tap_bound[k] = tap_bounds(p->taps[k], kernel_taps(k));
    } else if (k == kKernelBl3Quadratic) {
      p->taps[k] = bl3q_tap_polynomials();
      bl3q_axis_tables(n_grid, &iwin2, &alias);
      for (double& w : iwin2) w = 1.0 / w;
      p->tap_bound[k] = bl3q_tap_bounds(p->taps[k]);
    } else {
      p->taps[k] = bspline_tap_polynomials(k);
      bspline_axis_tables(n_grid, k, &iwin2, &alias);
      p->tap_bound[k] = tap_bounds(p->taps[k], kernel_taps(k));
    }
    up = up && hipMemcpy(p->d_iwin2[k], iwin2.data(), sizeof(double) * (half + 1), hipMemcpyHostToDevice) ==
                   hipSuccess;
    up = up && hipMemcpy(p->d_alias[k], alias.data(), sizeof(double) * (half + 1), hipMemcpyHostToDevice) ==
                   hipSuccess;
  }
  if (prec == MPS_F32) {
    std::vector<float> twf(tw.begin(), tw.end());
    up = up && hipMemcpy(p->d_twiddle, twf.data(), sizeof(float) * twf.size(), hipMemcpyHostToDevice) == hipSuccess;
  } else {
    up = up && hipMemcpy(p->d_twiddle, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!up) {
    release(p);
    return MPS_E_HIP;
  }
  *out = reinterpret_cast<mps_plan*>(p);
  return MPS_OK;
}

int mps_plan_destroy(mps_plan* plan) {
  if (!plan) return MPS_E_ARG;
  release(reinterpret_cast<Plan*>(plan));
  return MPS_OK;
}

int mps_plan_reserve(mps_plan* plan, int64_t max_particles) {
  if (!plan || max_particles < 1 || max_particles > 0x7fffffffll) return MPS_E_ARG;
  Plan* p = reinterpret_cast<Plan*>(plan);
  int st = ensure_particles(p, max_particles);
  if (st != MPS_OK) return st;
  // the paired deposits' scratch, if such a catalog can take the atomic
  // scatter
  if (pairs_reachable(p->n, p->prec, max_particles) && (st = ensure_pair_scratch(p)) != MPS_OK) return st;
  // the halo buffer too, if a catalog of at most max_particles can take the
  // halo scatter (the catalogs just above the owner-computes range)
  const int64_t nt = p->n / 16;
  const int64_t above = static_cast<int64_t>(MPS_SCATTER_GATHER_MAX_MEAN) * nt * nt * nt + 1;
  if (max_particles >= above && scatter_form_for(p->n, p->prec, above) == kFormHalo) return ensure_halo(p);
  return MPS_OK;
}

size_t mps_footprint(int n_grid, mps_precision prec, int64_t n_particles) {
  if (!is_pow2(n_grid) || n_grid < 8 || n_grid > 1024) return 0;
  const size_t rs = real_bytes(prec);
  const int64_t n3 = static_cast<int64_t>(n_grid) * n_grid * n_grid;
  const int64_t nt = n_grid / tile_for(n_grid, prec);
  const int64_t tiles = nt * nt * nt;
  const int half = n_grid / 2;
  size_t b = static_cast<size_t>(kNumFields) * n3 * rs;              // grids
  b += static_cast<size_t>(n_particles) * 2 * sizeof(float4);        // sorted records
  b += sizeof(uint32_t) * (3 * tiles + 1);                           // tile tables
  b += sizeof(int32_t) * half * half;                                // bin LUT
  b += sizeof(double) * (static_cast<size_t>(256) + 1) * kMaxBins * kNumQ;
  b += sizeof(double) * (kMomentBlocks * (kMomentSums + kMomentMax) + 2 * kNumKernels * (half + 1)) +
       2 * rs * n_grid + sizeof(ResultHeader);
  if (scatter_form_for(n_grid, prec, n_particles) == kFormHalo) b += halo_bytes(n_grid, prec);
  if (pairs_reachable(n_grid, prec, n_particles)) b += pair_scratch_bytes(tiles, kPairBlocks);
  return b;
}

int mps_estimate(mps_plan* plan, const mps_catalog* cat, mps_result* out, hipStream_t stream) {
  if (!plan || !out) return MPS_E_ARG;
  Plan* p = reinterpret_cast<Plan*>(plan);
  int st = validate_catalog(p, cat);
  if (st != MPS_OK) return st;
  if (hipSetDevice(p->device) != hipSuccess) return MPS_E_HIP;
  if ((st = ensure_bins(p, cat)) != MPS_OK) return st;
  if ((st = ensure_scatter_space(p, cat)) != MPS_OK) return st;
  if ((st = enqueue_estimate(p, cat, stream)) != MPS_OK) return st;
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;
  return unpack(p, cat, out);
}

int mps_estimate_mu(mps_plan* plan, const mps_catalog* cat, int n_mu, const double* axis, mps_result_mu* out,
                    hipStream_t stream) {
  if (!plan || !out) return MPS_E_ARG;
  Plan* p = reinterpret_cast<Plan*>(plan);
  int st = validate_catalog(p, cat);
  if (st != MPS_OK) return st;
  if (n_mu < 1 || n_mu > MPS_MAX_MU_BINS || cat->n_bins * n_mu > kMaxMuCells) return MPS_E_ARG;
  double ahat[3] = {0.0, 0.0, 0.0};
  if (axis && !unit_axis(axis, ahat)) return MPS_E_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return MPS_E_HIP;
  if (!p->d_mu_partials) {
    const size_t cells = static_cast<size_t>(kMaxMuCells) * kNumQMu;
    bool ok = dalloc(&p->d_mu_partials, sizeof(double) * cells * p->num_cus) == hipSuccess;
    ok = ok && dalloc(&p->d_mu_bins, sizeof(double) * cells) == hipSuccess;
    ok = ok && hipHostMalloc(&p->h_stage_mu, sizeof(ResultHeader) + sizeof(double) * cells,
                             hipHostMallocDefault) == hipSuccess;
    if (!ok) {
      dfree(p->d_mu_partials);
      dfree(p->d_mu_bins);
      if (p->h_stage_mu) (void)hipHostFree(p->h_stage_mu);
      p->d_mu_partials = nullptr;
      p->d_mu_bins = nullptr;
      p->h_stage_mu = nullptr;
      return MPS_E_NOMEM;
    }
  }
  if ((st = ensure_bins(p, cat)) != MPS_OK) return st;
  if ((st = ensure_scatter_space(p, cat)) != MPS_OK) return st;
  if ((st = enqueue_particles(p, cat, stream, 0)) != MPS_OK) return st;
  MPS_TRY(launch_fft_z(p, p->grid, stream));
  mark(p, 6, stream);
  MPS_TRY(launch_fft_y(p, p->grid, stream));
  mark(p, 7, stream);
  MPS_TRY(launch_fft_x_store(p, p->grid, stream));
  MPS_TRY(launch_mu_bin(p, cat, n_mu, axis ? ahat : nullptr, stream));
  mark(p, 8, stream);
  MPS_TRY(launch_finalize_mu(p, cat, n_mu, stream));
  mark(p, 9, stream);
  const int ncell = cat->n_bins * n_mu;
  MPS_TRY(hipMemcpyAsync(p->h_stage_mu, p->d_header, sizeof(ResultHeader), hipMemcpyDeviceToHost, stream));
  MPS_TRY(hipMemcpyAsync(static_cast<char*>(p->h_stage_mu) + sizeof(ResultHeader), p->d_mu_bins,
                         sizeof(double) * kNumQMu * ncell, hipMemcpyDeviceToHost, stream));
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;

  const ResultHeader* h = static_cast<const ResultHeader*>(p->h_stage_mu);
  if ((st = check_header(h)) != MPS_OK) return st;
  if (!axis && !unit_axis(h->d.vb, ahat)) return MPS_E_ARG;  // no bulk flow to define mu_b
  const double* cells = reinterpret_cast<const double*>(static_cast<const char*>(p->h_stage_mu) + sizeof(ResultHeader));
  for (int i = 0; i < ncell; ++i) {
    const double* q = cells + static_cast<size_t>(i) * kNumQMu;
    if (out->n_modes) out->n_modes[i] = static_cast<int64_t>(std::llround(q[MCount]));
    double* dst[] = {out->k_mean, out->mu_mean, out->p_dd, out->p_pp, out->p_tt, out->p_dt_re, out->p_dt_im,
                     out->p_dpb_re, out->p_dpb_im, out->sn_dd, out->sn_pp, out->sn_tt, out->sn_dt_im, out->sn_dpb};
    const int src[] = {MKsum, MMusum, MPdd, MPpp, MPtt, MPdtRe, MPdtIm, MPdpbRe, MPdpbIm, MSdd, MSpp, MStt,
                       MSdtIm, MSdpb};
    for (int k = 0; k < 14; ++k)
      if (dst[k]) dst[k][i] = q[src[k]];
  }
  for (int a = 0; a < 3; ++a) {
    out->axis[a] = ahat[a];
    out->v_bulk[a] = h->d.vb[a];
  }
  out->sigma_v2 = h->d.sigma_v2;
  out->n_eff = h->d.W * h->d.W / h->d.W2;
  if (p->timing)
    for (int i = 0; i < kNumStages; ++i) {
      float ms = 0.f;
      p->stage_ms[i] = hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]) == hipSuccess ? ms : -1.0;
    }
  return MPS_OK;
}

int mps_estimate_batch(mps_plan* const* plans, const mps_catalog* cats, mps_result* outs, int n,
                       hipStream_t stream) {
  if (!plans || !cats || !outs || n < 0) return MPS_E_ARG;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return MPS_E_ARG;
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return MPS_E_ARG;
    const int st = validate_catalog(reinterpret_cast<Plan*>(plans[i]), &cats[i]);
    if (st != MPS_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    Plan* p = reinterpret_cast<Plan*>(plans[i]);
    int st;
    if ((st = ensure_bins(p, &cats[i])) != MPS_OK) return st;
    if ((st = ensure_scatter_space(p, &cats[i])) != MPS_OK) return st;
  }
  // the catalogs' stages go to the device's batch lanes (created once), each
  // started after the caller's earlier work on `stream`; `stream` then waits
  // for all of them
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MPS_E_HIP;
  BatchLanes& bl = batch_lanes(dev);
  std::lock_guard<std::mutex> guard(bl.mu);
  int st = bl.ready();
  if (st != MPS_OK) return st;
  std::vector<Plan*> ps(n);
  for (int i = 0; i < n; ++i) ps[i] = reinterpret_cast<Plan*>(plans[i]);
  if (hipEventRecord(bl.start, stream) != hipSuccess) return MPS_E_HIP;
  for (int j = 0; j < BatchLanes::kLanes; ++j)
    if (hipStreamWaitEvent(bl.lanes[j], bl.start, 0) != hipSuccess) return MPS_E_HIP;
  st = n > 0 ? enqueue_batch(ps.data(), cats, n, bl.lanes, BatchLanes::kLanes, bl.ev, &bl.ws, nullptr) : MPS_OK;
  for (int j = 0; j < BatchLanes::kLanes; ++j) {  // join even after a failure, so nothing is left running
    if (hipEventRecord(bl.join[j], bl.lanes[j]) == hipSuccess) (void)hipStreamWaitEvent(stream, bl.join[j], 0);
  }
  const bool synced = hipStreamSynchronize(stream) == hipSuccess;
  if (st != MPS_OK) return st;
  if (!synced) return MPS_E_HIP;
  int first = MPS_OK;
  for (int i = 0; i < n; ++i) {
    const int s2 = unpack(ps[i], &cats[i], &outs[i]);
    if (s2 != MPS_OK && first == MPS_OK) first = s2;
  }
  return first;
}

}  // extern "C"

namespace mps {
namespace {

int ensure_split(Plan* p, int64_t np) {
  if (!p->split_count) {
    bool ok = dalloc(&p->split_count, sizeof(uint32_t) * (kMaxCubes + 1)) == hipSuccess;
    ok = ok && dalloc(&p->split_offset, sizeof(uint32_t) * (kMaxCubes + 1)) == hipSuccess;
    ok = ok && dalloc(&p->split_cursor, sizeof(uint32_t) * kMaxCubes) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&p->h_split), sizeof(uint32_t) * (kMaxCubes + 1),
                             hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(&p->h_stage_sub, p->stage_bytes * kMaxCubes, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
      dfree(p->split_count);
      dfree(p->split_offset);
      dfree(p->split_cursor);
      if (p->h_split) (void)hipHostFree(p->h_split);
      if (p->h_stage_sub) (void)hipHostFree(p->h_stage_sub);
      p->split_count = p->split_offset = p->split_cursor = p->h_split = nullptr;
      p->h_stage_sub = nullptr;
      return MPS_E_NOMEM;
    }
  }
  if (np <= p->split_cap) return MPS_OK;
  dfree(p->split_pos);
  dfree(p->split_vel);
  dfree(p->split_w);
  p->split_pos = p->split_vel = p->split_w = nullptr;
  p->split_cap = 0;
  const size_t n = static_cast<size_t>(np);
  bool ok = dalloc(&p->split_pos, sizeof(float) * 3 * n) == hipSuccess;
  ok = ok && dalloc(&p->split_vel, sizeof(float) * 3 * n) == hipSuccess;
  ok = ok && dalloc(&p->split_w, sizeof(float) * n) == hipSuccess;
  if (!ok) {
    dfree(p->split_pos);
    dfree(p->split_vel);
    dfree(p->split_w);
    p->split_pos = p->split_vel = p->split_w = nullptr;
    return MPS_E_NOMEM;
  }
  p->split_cap = np;
  return MPS_OK;
}

// Helper plans and streams for running sub-sample estimates concurrently.
int ensure_sub_lanes(Plan* p) {
  // created in order and kept: resumes where an earlier failure stopped
  for (int i = 0; i < Plan::kSubLanes; ++i) {
    if (i > 0 && !p->sub_plan[i - 1]) {
      mps_plan* h = nullptr;
      const int st = mps_plan_create(&h, p->n, p->prec);
      if (st != MPS_OK) return st;
      p->sub_plan[i - 1] = reinterpret_cast<Plan*>(h);
    }
    if (!p->sub_stream[i] && hipStreamCreateWithFlags(&p->sub_stream[i], hipStreamNonBlocking) != hipSuccess) {
      p->sub_stream[i] = nullptr;
      return MPS_E_HIP;
    }
    if (!p->sub_done[i] && hipEventCreateWithFlags(&p->sub_done[i], hipEventDisableTiming) != hipSuccess) {
      p->sub_done[i] = nullptr;
      return MPS_E_HIP;
    }
  }
  return MPS_OK;
}

// Mean and sample standard deviation (divisor m - 1) of one value over the
// m staged sub-cube results; v(i) is the value of the i-th.
template <typename F>
void spread(int m, F v, double* mean, double* sdev) {
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += v(i);
  const double mu = m > 0 ? s / m : NAN;
  double q = 0.0;
  for (int i = 0; i < m; ++i) {
    const double d = v(i) - mu;
    q += d * d;
  }
  if (mean) *mean = mu;
  if (sdev) *sdev = m > 1 ? std::sqrt(q / (m - 1)) : NAN;
}

void subcube_stats(const std::vector<const char*>& ok_stages, int n_bins, mps_result* mean, mps_result* sdev) {
  const int m = static_cast<int>(ok_stages.size());
  auto bins = [&](int i) {
    return reinterpret_cast<const double*>(ok_stages[i] + sizeof(ResultHeader));
  };
  auto head = [&](int i) { return reinterpret_cast<const ResultHeader*>(ok_stages[i]); };
  struct Field {
    int q;
    double* mps_result::*member;
  };
  const Field fields[] = {{QKsum, &mps_result::k_mean}, {QPdd, &mps_result::p_dd}, {QPpp, &mps_result::p_pp},
                          {QPtt, &mps_result::p_tt},    {QPdt, &mps_result::p_dt}, {QSdd, &mps_result::sn_dd},
                          {QSpp, &mps_result::sn_pp},   {QStt, &mps_result::sn_tt}};
  for (const Field& f : fields) {
    double* om = mean ? mean->*(f.member) : nullptr;
    double* os = sdev ? sdev->*(f.member) : nullptr;
    for (int b = 0; b < n_bins; ++b)
      spread(m, [&](int i) { return bins(i)[b * kNumQ + f.q]; }, om ? om + b : nullptr, os ? os + b : nullptr);
  }
  for (mps_result* r : {mean, sdev})
    if (r && r->n_modes)
      for (int b = 0; b < n_bins; ++b)
        r->n_modes[b] = m > 0 ? static_cast<int64_t>(std::llround(bins(0)[b * kNumQ + QCount])) : 0;
  double dm = 0.0, ds = 0.0;
  for (int a = 0; a < 3; ++a) {
    spread(m, [&](int i) { return head(i)->d.vb[a]; }, &dm, &ds);
    if (mean) mean->v_bulk[a] = dm;
    if (sdev) sdev->v_bulk[a] = ds;
  }
  spread(m, [&](int i) { return head(i)->d.sigma_v2; }, &dm, &ds);
  if (mean) mean->sigma_v2 = dm;
  if (sdev) sdev->sigma_v2 = ds;
  spread(m, [&](int i) { return head(i)->d.W * head(i)->d.W / head(i)->d.W2; }, &dm, &ds);
  if (mean) mean->n_eff = dm;
  if (sdev) sdev->n_eff = ds;
}

}  // namespace
}  // namespace mps

extern "C" {

int mps_estimate_subcubes(mps_plan* plan, const mps_catalog* cat, int n_div, mps_result* outs, int* status,
                          mps_result* mean, mps_result* sdev, hipStream_t stream) {
  if (!plan || !outs || !status) return MPS_E_ARG;
  Plan* p = reinterpret_cast<Plan*>(plan);
  int st = validate_catalog(p, cat);
  if (st != MPS_OK) return st;
  if (n_div < 1 || n_div > MPS_MAX_DIV) return MPS_E_ARG;
  const int n_cubes = n_div * n_div * n_div;
  mps_catalog sub = *cat;
  sub.box = cat->box / n_div;
  sub.flags &= ~MPS_CATALOG_HOST;  // the sub-catalogs live in plan workspace
  if (!(sub.box > 0.0)) return MPS_E_ARG;
  if (hipSetDevice(p->device) != hipSuccess) return MPS_E_HIP;
  if ((st = ensure_bins(p, &sub)) != MPS_OK) return st;
  if ((st = ensure_split(p, cat->n_particles)) != MPS_OK) return st;
  mps_catalog staged = *cat;
  if (cat->flags & MPS_CATALOG_HOST) {  // the split reads a device copy
    if ((st = ensure_host_stage(p, cat->n_particles)) != MPS_OK) return st;
    const size_t n = static_cast<size_t>(cat->n_particles);
    staged.flags &= ~MPS_CATALOG_HOST;
    staged.pos = p->host_stage;
    staged.vel = p->host_stage + 3 * n;
    staged.weight = cat->weight ? p->host_stage + 6 * n : nullptr;
    MPS_TRY(hipMemcpyAsync(p->host_stage, cat->pos, sizeof(float) * 3 * n, hipMemcpyHostToDevice, stream));
    MPS_TRY(hipMemcpyAsync(p->host_stage + 3 * n, cat->vel, sizeof(float) * 3 * n, hipMemcpyHostToDevice, stream));
    if (cat->weight)
      MPS_TRY(hipMemcpyAsync(p->host_stage + 6 * n, cat->weight, sizeof(float) * n, hipMemcpyHostToDevice, stream));
    cat = &staged;
  }

  SplitParams sp;
  sp.scale = static_cast<double>(n_div) / cat->box;
  sp.sub_box = sub.box;
  sp.n_div = n_div;
  sp.n_cubes = n_cubes;
  MPS_TRY(launch_split_count(cat, sp, p->split_count, stream));
  MPS_TRY(hipMemcpyAsync(p->h_split, p->split_count, sizeof(uint32_t) * (n_cubes + 1), hipMemcpyDeviceToHost,
                         stream));
  MPS_TRY(launch_split_permute(cat, sp, p->split_count, p->split_offset, p->split_cursor, p->split_pos,
                               p->split_vel, cat->weight ? p->split_w : nullptr, stream));
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;
  if (p->h_split[n_cubes]) return MPS_E_NONFINITE;
  std::vector<uint32_t> count(p->h_split, p->h_split + n_cubes);
  int64_t largest = 0;
  for (uint32_t c : count) largest = c > largest ? c : largest;
  if ((st = ensure_particles(p, largest)) != MPS_OK) return st;

  // the split is complete (synchronised above); the cubes' estimates run
  // round robin on kSubLanes plans, each with its own stream, so that the
  // small grids' kernels overlap
  if ((st = ensure_sub_lanes(p)) != MPS_OK) return st;
  Plan* lane[Plan::kSubLanes];
  bool halo = false;  // a sub-catalog takes the halo scatter
  bool pairs = false;  // or paired deposits
  for (uint32_t c : count) {
    halo = halo || (c > 0 && kernel_id(sub.flags) == 0 && scatter_form_for(p->n, p->prec, c) == kFormHalo);
    pairs = pairs || (c > 0 && kernel_id(sub.flags) == 0 && pairs_reachable(p->n, p->prec, c));
  }
  for (int i = 0; i < Plan::kSubLanes; ++i) {
    lane[i] = i == 0 ? p : p->sub_plan[i - 1];
    if ((st = ensure_bins(lane[i], &sub)) != MPS_OK) return st;
    if ((st = ensure_particles(lane[i], largest)) != MPS_OK) return st;
    if (halo && (st = ensure_halo(lane[i])) != MPS_OK) return st;
    if (pairs && (st = ensure_pair_scratch(lane[i])) != MPS_OK) return st;
  }
  std::vector<mps_catalog> cats(n_cubes, sub);
  int64_t off = 0;
  char* stage = static_cast<char*>(p->h_stage_sub);
  for (int s = 0; s < n_cubes; ++s) {
    cats[s].n_particles = count[s];
    cats[s].pos = p->split_pos + 3 * off;
    cats[s].vel = p->split_vel + 3 * off;
    cats[s].weight = cat->weight ? p->split_w + off : nullptr;
    off += count[s];
    status[s] = MPS_E_ZEROWEIGHT;
    if (count[s] == 0) continue;
    const int l = s % Plan::kSubLanes;
    if ((st = enqueue_estimate(lane[l], &cats[s], p->sub_stream[l], stage + p->stage_bytes * s)) != MPS_OK)
      return st;
  }
  for (int i = 0; i < Plan::kSubLanes; ++i) {
    MPS_TRY(hipEventRecord(p->sub_done[i], p->sub_stream[i]));
    MPS_TRY(hipStreamWaitEvent(stream, p->sub_done[i], 0));
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;
  std::vector<const char*> ok_stages;
  for (int s = 0; s < n_cubes; ++s) {
    if (count[s] == 0) continue;
    const char* slot = stage + p->stage_bytes * s;
    status[s] = unpack(lane[s % Plan::kSubLanes], &cats[s], &outs[s], slot);
    if (status[s] == MPS_OK) ok_stages.push_back(slot);
  }
  if (mean || sdev) subcube_stats(ok_stages, sub.n_bins, mean, sdev);
  return MPS_OK;
}

int mps_assign(mps_plan* plan, const mps_catalog* cat, void* grids, hipStream_t stream) {
  if (!plan || !grids) return MPS_E_ARG;
  Plan* p = reinterpret_cast<Plan*>(plan);
  int st = validate_catalog(p, cat);
  if (st != MPS_OK) return st;
  if (hipSetDevice(p->device) != hipSuccess) return MPS_E_HIP;
  if ((st = ensure_scatter_space(p, cat)) != MPS_OK) return st;
  const bool was = p->timing;
  p->timing = false;
  st = enqueue_particles(p, cat, stream, (cat->flags & MPS_BULKFLOW_SUBTRACT) ? 1 : 0);
  p->timing = was;
  if (st != MPS_OK) return st;
  const size_t bytes = static_cast<size_t>(kNumFields) * p->n * p->n * p->n * p->real_size;
  if (hipMemcpyAsync(grids, p->grid, bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess) return MPS_E_HIP;
  if (hipMemcpyAsync(p->h_stage, p->d_header, sizeof(ResultHeader), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return MPS_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;
  return check_header(static_cast<const ResultHeader*>(p->h_stage));
}

int mps_fft(mps_plan* plan, void* grids, hipStream_t stream) {
  if (!plan || !grids) return MPS_E_ARG;
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (hipSetDevice(p->device) != hipSuccess) return MPS_E_HIP;
  if (launch_fft_z(p, grids, stream) != hipSuccess) return MPS_E_HIP;
  if (launch_fft_y(p, grids, stream) != hipSuccess) return MPS_E_HIP;
  if (launch_fft_x_store(p, grids, stream) != hipSuccess) return MPS_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;
  return MPS_OK;
}

int mps_plan_set_timing(mps_plan* plan, int enable) {
  if (!plan) return MPS_E_ARG;
  reinterpret_cast<Plan*>(plan)->timing = enable != 0;
  return MPS_OK;
}

int mps_plan_stage_times(const mps_plan* plan, double* ms, int n) {
  if (!plan || !ms || n < 0) return MPS_E_ARG;
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  for (int i = 0; i < n && i < kNumStages; ++i) ms[i] = p->stage_ms[i];
  return MPS_OK;
}

const char* mps_strerror(int status) {
  switch (status) {
    case MPS_OK: return "ok";
    case MPS_E_ARG: return "invalid argument";
    case MPS_E_NONFINITE: return "non-finite position, velocity or weight";
    case MPS_E_ZEROWEIGHT: return "sum of weights is zero";
    case MPS_E_NOMEM: return "out of device or pinned memory";
    case MPS_E_HIP: return "HIP runtime error";
    case MPS_E_TIMEOUT: return "timed out";
    case MPS_E_BUSY: return "server queue full";
    case MPS_E_TOOBIG: return "request exceeds the server's memory budget or the static workspace";
  }
  return "unknown status";
}

}  // extern "C"
