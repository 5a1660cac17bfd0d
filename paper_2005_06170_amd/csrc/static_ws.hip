// mps_estimate_static: the estimate of mps_estimate without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  Every buffer a plan
// would own lives in one file-scope device array, `scratch`, of fixed size;
// the kernels are those of mps_estimate.
//
// Each GPU holds its own copy of `scratch` (until the process ends).  Its
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current; host code only ever passes that address on.  Calls on
// one GPU share the array: the host side is serialised by a lock, but calls
// whose work overlaps on the device (different streams) race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"

namespace mps {
namespace {

constexpr int kStaticMaxGrid = MPS_STATIC_MAX_GRID;
constexpr int64_t kStaticMaxParticles = MPS_STATIC_MAX_PARTICLES;
constexpr int kStaticMaxDevices = 16;
constexpr int kStaticCus = 256;  // bound on the x pass's workgroups
static_assert(kStaticMaxGrid < MPS_SCATTER_MIN_GRID, "the workspace holds no halo buffer");

constexpr size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Byte offsets of the plan's buffers in `scratch`, sized for the largest
// grid (FP64) and catalog the entry point accepts.  Grids this small take
// the atomic scatter (which needs no halo buffer).
struct Layout {
  static constexpr int64_t kN3 = static_cast<int64_t>(kStaticMaxGrid) * kStaticMaxGrid * kStaticMaxGrid;
  static constexpr int kHalf = kStaticMaxGrid / 2;
  static constexpr int64_t kTiles = kN3 / (8 * 8 * 8);  // the smallest tile is 8^3
  static constexpr size_t grid = 0;
  static constexpr size_t sorted = align256(grid + kNumFields * kN3 * sizeof(double));
  static constexpr size_t tile_count = align256(sorted + kStaticMaxParticles * 2 * sizeof(float4));
  static constexpr size_t tile_offset = align256(tile_count + kTiles * sizeof(uint32_t));
  static constexpr size_t tile_cursor = align256(tile_offset + (kTiles + 1) * sizeof(uint32_t));
  static constexpr size_t tile_queue = align256(tile_cursor + kTiles * sizeof(uint32_t));
  static constexpr size_t moments = align256(tile_queue + 8 * sizeof(uint32_t));
  static constexpr size_t header = align256(moments + kMomentBlocks * (kMomentSums + kMomentMax) * sizeof(double));
  static constexpr size_t iwin2 = align256(header + sizeof(ResultHeader));
  static constexpr size_t alias = align256(iwin2 + (kHalf + 1) * sizeof(double));
  static constexpr size_t twiddle = align256(alias + (kHalf + 1) * sizeof(double));
  static constexpr size_t lut = align256(twiddle + 2 * kStaticMaxGrid * sizeof(double));
  static constexpr size_t bin_partials = align256(lut + kHalf * kHalf * sizeof(int32_t));
  static constexpr size_t bins = align256(bin_partials + static_cast<size_t>(kStaticCus) * kMaxBins * kNumQ * sizeof(double));
  static constexpr size_t total = align256(bins + kMaxBins * kNumQ * sizeof(double));
};

}  // namespace
}  // namespace mps

// The workspace.  In host code this name stands for the host-side shadow of
// the symbol, not a device address: only the address hipGetSymbolAddress
// returns (DeviceState::base) is passed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[mps::Layout::total];

namespace mps {
namespace {

// Host tables of one (grid size, precision, kernel), cached on the host.
struct Tables {
  int n = 0;
  mps_precision prec = MPS_F32;
  int kernel = -1;
  TapPoly taps{};
  TapBound bound{};
  std::vector<double> iwin2, alias;
  std::vector<double> tw64;
  std::vector<float> tw32;
};

struct DeviceState {
  bool ready = false;
  unsigned char* base = nullptr;   // device address of `scratch` on this device
  std::mutex mu;
  Plan plan;                       // host view; every pointer is into `base`
  Tables tables;
  // what the device copy of the tables currently holds
  int dev_n = 0, dev_kernel = -1;
  mps_precision dev_prec = MPS_F32;
  // result staging (pageable host memory: the copy back is synchronous)
  alignas(16) unsigned char stage[sizeof(ResultHeader) + sizeof(double) * kMaxBins * kNumQ];
};

DeviceState g_state[kStaticMaxDevices];
std::mutex g_init;

// Once per device, with that device current: the device address of scratch.
int device_state(int dev, DeviceState** out) {
  if (dev < 0 || dev >= kStaticMaxDevices) return MPS_E_ARG;
  std::lock_guard<std::mutex> g(g_init);
  DeviceState& st = g_state[dev];
  if (!st.ready) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MPS_E_HIP;
    st.base = static_cast<unsigned char*>(ptr);
    st.ready = true;
  }
  *out = &st;
  return MPS_OK;
}

void build_tables(Tables* t, int n, mps_precision prec, int k) {
  t->n = n;
  t->prec = prec;
  t->kernel = k;
  if (k == 0) {
    t->taps = bl3_tap_polynomials();
    bl3_axis_tables(n, &t->iwin2, &t->alias);
    for (double& w : t->iwin2) w = 1.0 / w;
    t->bound = tap_bounds(t->taps, kernel_taps(k));
  } else if (k == kKernelBl3Quadratic) {
    t->taps = bl3q_tap_polynomials();
    bl3q_axis_tables(n, &t->iwin2, &t->alias);
    for (double& w : t->iwin2) w = 1.0 / w;
    t->bound = bl3q_tap_bounds(t->taps);
  } else {
    t->taps = bspline_tap_polynomials(k);
    bspline_axis_tables(n, k, &t->iwin2, &t->alias);
    t->bound = tap_bounds(t->taps, kernel_taps(k));
  }
  t->tw64 = twiddles(n);
  t->tw32.assign(t->tw64.begin(), t->tw64.end());
}

// Point the host plan view at the workspace for an N^3 grid.
void lay_out(DeviceState* st, int dev, int n, mps_precision prec) {
  Plan& p = st->plan;
  unsigned char* b = st->base;
  p.n = n;
  p.prec = prec;
  p.device = dev;
  p.tile = tile_for(n, prec);
  const int64_t nt = n / p.tile;
  p.n_tiles = nt * nt * nt;
  p.real_size = prec == MPS_F64 ? 8 : 4;
  p.grid = b + Layout::grid;
  p.sorted = reinterpret_cast<float4*>(b + Layout::sorted);
  p.sorted_cap = kStaticMaxParticles;
  p.tile_count = reinterpret_cast<uint32_t*>(b + Layout::tile_count);
  p.tile_offset = reinterpret_cast<uint32_t*>(b + Layout::tile_offset);
  p.tile_cursor = reinterpret_cast<uint32_t*>(b + Layout::tile_cursor);
  p.tile_queue = reinterpret_cast<uint32_t*>(b + Layout::tile_queue);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  p.num_cus = cus < kStaticCus ? cus : kStaticCus;
  const int items = x_bin_items(n, prec);
  p.bin_blocks = items < p.num_cus ? items : p.num_cus;
  p.moment_partials = reinterpret_cast<double*>(b + Layout::moments);
  p.d_header = reinterpret_cast<ResultHeader*>(b + Layout::header);
  for (int k = 0; k < kNumKernels; ++k) {  // only the catalog's kernel is filled
    p.d_iwin2[k] = reinterpret_cast<double*>(b + Layout::iwin2);
    p.d_alias[k] = reinterpret_cast<double*>(b + Layout::alias);
  }
  p.d_twiddle = b + Layout::twiddle;
  p.d_lut = reinterpret_cast<int32_t*>(b + Layout::lut);
  p.d_bin_partials = reinterpret_cast<double*>(b + Layout::bin_partials);
  p.d_bins = reinterpret_cast<double*>(b + Layout::bins);
  p.h_stage = st->stage;
  p.stage_bytes = sizeof(st->stage);
  p.timing = false;
}

}  // namespace
}  // namespace mps

using namespace mps;

extern "C" {

int mps_estimate_static(const mps_catalog* cat, int n_grid, mps_precision prec, mps_result* out,
                        hipStream_t stream) {
  if (!cat || !out) return MPS_E_ARG;
  if (n_grid < 8 || (n_grid & (n_grid - 1)) || (prec != MPS_F32 && prec != MPS_F64)) return MPS_E_ARG;
  int st = validate_catalog(nullptr, cat);
  if (st != MPS_OK) return st;
  if (cat->flags & MPS_CATALOG_HOST) return MPS_E_ARG;  // no staging buffer here
  if (n_grid > kStaticMaxGrid || cat->n_particles > kStaticMaxParticles) return MPS_E_TOOBIG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MPS_E_HIP;
  DeviceState* ds = nullptr;
  if ((st = device_state(dev, &ds)) != MPS_OK) return st;
  std::lock_guard<std::mutex> g(ds->mu);
  const int k = kernel_id(cat->flags);
  if (ds->tables.n != n_grid || ds->tables.prec != prec || ds->tables.kernel != k)
    build_tables(&ds->tables, n_grid, prec, k);
  if (ds->plan.n != n_grid || ds->plan.prec != prec || ds->plan.device != dev) {
    lay_out(ds, dev, n_grid, prec);
    ds->plan.lut_box = -1.0;  // the bin table must be rebuilt for this layout
  }
  Plan* p = &ds->plan;
  p->taps[k] = ds->tables.taps;
  p->tap_bound[k] = ds->tables.bound;
  if (ds->dev_n != n_grid || ds->dev_prec != prec || ds->dev_kernel != k) {
    const size_t tb = sizeof(double) * (n_grid / 2 + 1);
    if (hipMemcpyAsync(p->d_iwin2[k], ds->tables.iwin2.data(), tb, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(p->d_alias[k], ds->tables.alias.data(), tb, hipMemcpyHostToDevice, stream) != hipSuccess)
      return MPS_E_HIP;
    const hipError_t e =
        prec == MPS_F32
            ? hipMemcpyAsync(p->d_twiddle, ds->tables.tw32.data(), sizeof(float) * ds->tables.tw32.size(),
                             hipMemcpyHostToDevice, stream)
            : hipMemcpyAsync(p->d_twiddle, ds->tables.tw64.data(), sizeof(double) * ds->tables.tw64.size(),
                             hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return MPS_E_HIP;
    ds->dev_n = n_grid;
    ds->dev_prec = prec;
    ds->dev_kernel = k;
  }
  if ((st = ensure_bins(p, cat)) != MPS_OK) return st;
  if ((st = enqueue_estimate(p, cat, stream)) != MPS_OK) return st;
  if (hipStreamSynchronize(stream) != hipSuccess) return MPS_E_HIP;
  return unpack(p, cat, out);
}

}  // extern "C"
