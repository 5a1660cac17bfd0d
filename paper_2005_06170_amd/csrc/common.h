// Internal declarations of the MI355X momentum-power-spectrum library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mps.h"

namespace mps {

constexpr int kNumFields = 4;     // rho, rho v_x, rho v_y, rho v_z
constexpr int kTaps = 6;          // BL3 taps j = -2..3
constexpr int kTapLo = -2;
constexpr int kNumQ = 9;          // per-bin accumulators (see BinQ)
constexpr int kMaxBins = MPS_MAX_BINS;
constexpr int kMomentSums = 14;   // W, W2, sum w v (3), sum w^2 v (3), sum w^2 v v^T (6)
constexpr int kMomentMax = 4;     // max |w|, max |w v_a| (a = x, y, z)
constexpr int kNumStages = 9;

// Per-bin accumulators, in order.
enum BinQ { QCount = 0, QKsum, QPdd, QPpp, QPtt, QPdt, QSdd, QSpp, QStt };

// Per-(k, mu) cell accumulators of the anisotropic estimate, in order.
enum MuQ {
  MCount = 0, MKsum, MMusum, MPdd, MPpp, MPtt, MPdtRe, MPdtIm, MPdpbRe, MPdpbIm,
  MSdd, MSpp, MStt, MSdtIm, MSdpb, kNumQMu
};
constexpr int kMaxMuCells = MPS_MAX_MU_CELLS;
constexpr int kMaxCubes = MPS_MAX_SUBCUBES;  // n_div^3 for n_div <= MPS_MAX_DIV

// Split of a catalog into n_div^3 sub-cubes (subcubes.hip).
struct SplitParams {
  double scale;    // n_div / L
  double sub_box;  // L / n_div
  int n_div;
  int n_cubes;     // n_div^3
};

// Polynomial weights of up to six taps: w_j(f) = sum_p coef[j][p] f^p with
// f = u - floor(u) in [0, 1) (u shifted by half a cell for the odd-order
// B-splines), degree <= 5.  FP64.
constexpr int kPolyCoef = 6;
struct TapPoly {
  double c[kTaps][kPolyCoef];
};

// Assignment kernels: 0 the truncated BL3 function (6 taps, cubic pieces);
// p = 1..6 the centred B-spline of order p (p taps, degree p - 1; order 4
// also serves the untruncated BL3 function, whose deconvolved spectra are
// those of the cubic B-spline); 7 the quadratic-spline reading of BL3 (6
// taps, two quadratic pieces per tap split at f = 1/2, see kDegSplit2).
constexpr int kNumKernels = 8;
constexpr int kKernelBl3Quadratic = 7;
inline int kernel_id(uint32_t flags) {
  if (flags & MPS_KERNEL_BL3_EXACT) return 4;
  return static_cast<int>((flags >> MPS_KERNEL_ORDER_SHIFT) & 7u);
}
inline int kernel_taps(int id) { return (id == 0 || id == kKernelBl3Quadratic) ? kTaps : id; }
// half a cell for odd B-spline orders: taps are centred on the nearest node
inline double kernel_shift(int id) { return (id != kKernelBl3Quadratic && (id & 1)) ? 0.5 : 0.0; }

// Tap polynomials of the quadratic-spline BL3 reading: c[j][0..2] is the
// weight for f < 1/2 and c[j][3..5] for f >= 1/2, both as quadratics in f.
constexpr int kDegSplit2 = -2;

// Upper bounds of |w_j(f)| over f in [0, 1) for the six taps.
struct TapBound {
  float k[kTaps];
};

// Scalars derived on the device from the moment sums (FP64).
struct Derived {
  double W, W2;
  double vb[3];          // bulk flow
  double s_dd;           // W2 / W^2
  double S[6];           // shot tensor of the velocities used: xx yy zz xy xz yz
  double s_pp;           // trace S
  double inv_W;          // 1 / W
  double sigma_v2;       // trace(sum w^2 v v^T) / W2 of the velocities used
  double qmax[kNumFields];  // max |w|, max |w v_a| over the catalog
  double s[3];           // sum w^2 v / W^2 of the velocities used
  double sp[3];          // sum w^2 (v - v_b) / W^2
  int bulk;              // 1 if p is replaced by p - v_b delta
};

// Sort parameters of a catalog on a plan's grid (see particles.hip locate()).
struct KeyParams {
  double scale;  // N / L
  double shift;  // added to u = x N / L
  int n;         // grid size
  int tshift;    // log2(tile)
  int nt;        // tiles per axis
};

// One catalog's part of a (possibly multi-catalog) FP32 scatter launch.
struct ScatterCat {
  const float4* sorted;    // tile-sorted records
  const uint32_t* offset;  // n_tiles + 1 record offsets
  float* grid;             // four N^3 FP32 grids (zeroed for the atomic form)
  KeyParams kp;
  const Derived* dsrc;     // moments and bounds of the catalog
  int bulk;                // 1: deposit w (v - v_b)
  float* halo;             // halo form: kHaloCells x 4 fields per tile
};

// The scatter's forms (16^3 tiles, truncated BL3; FP64 grids only the atomic
// and owner-computes forms).  Each tile
// accumulates its particles' deposits over the tile and a halo (2 cells
// below, 3 above per axis) in LDS, then
//   kFormAtomic: adds the whole block to the (cleared) grid with FP32 atomics;
//   kFormHalo:   stores its own cells in the grid and its halo cells in a
//                per-tile halo buffer, and a fix-up pass adds each cell's
//                neighbour halos in a fixed order (no atomics, no clear);
//   kFormGather: (owner-computes) gathers the particles of its 27-tile
//                neighbourhood whose taps reach it and stores its own cells.
// The gather pays for its candidate reads at all but low densities, the
// halo form for its halo traffic once the tiles are dense enough that the
// atomic form's deposits, not its flush, dominate.
enum ScatterForm { kFormAtomic = 0, kFormGather = 1, kFormHalo = 2 };
constexpr int kHaloCells = 21 * 21 * 21 - 16 * 16 * 16;  // halo cells of a 16^3 tile's block

// Paired deposits of the FP32 atomic form (16^3 tiles, truncated BL3, one
// catalog per launch): a dense tile's particles are sorted by cell, and two
// particles in one cell or in z-neighbouring cells of one (x, y) column
// deposit together over 7 z cells instead of 2 x 6.  Each workgroup keeps
// its tile's job list in its own slice of global scratch, kPairCap words;
// tiles of more than kPairCap particles (the sort runs in the accumulator
// block, 2 x 21^3 words per pair of fields), and workgroups beyond
// `blocks`, deposit unpaired.
constexpr int kPairCap = 16384;
constexpr int kPairBlocks = 256;  // most workgroups a plan's scratch covers
struct PairWork {
  uint32_t* base;  // blocks x kPairCap words, or null (unpaired only)
  int blocks;
};
size_t pair_scratch_bytes(int64_t n_tiles, int num_cus);

// Layout of the device result block copied back to the host.
struct ResultHeader {
  double sums[kMomentSums];
  Derived d;
  uint32_t flags;        // bit 0: non-finite position seen
  uint32_t order_same;   // sampled neighbouring particles in one tile (the sort's order probe)
  uint32_t order_pairs;  // sampled neighbouring pairs
  uint32_t pad;
};

struct Plan;

// ----------------------------------------------------------------- tables
// Host-side FP64 construction of the truncated cubic Battle-Lemarie kernel.
TapPoly bl3_tap_polynomials();
// Bounds of |w_j| on [0, 1] for the first n_taps taps, with a small margin.
TapBound tap_bounds(const TapPoly& tp, int n_taps);
// Tap polynomials of the centred B-spline of order p = 1..6.
TapPoly bspline_tap_polynomials(int order);
// Quadratic-spline BL3 reading: tap polynomials in the split layout
// (kDegSplit2), bounds of |w_j| over both pieces, and per-axis tables
// W_t(2 pi n / N)^2 and C_t(2 pi n / N), n = 0..N/2.
TapPoly bl3q_tap_polynomials();
TapBound bl3q_tap_bounds(const TapPoly& tp);
void bl3q_axis_tables(int n_grid, std::vector<double>* win2, std::vector<double>* alias);
// 1 / sinc^(2p)(w/2) and the alias sum sum_m beta_{2p-1}(m) cos(m w) for
// w = 2 pi n / N, n = 0..N/2.
void bspline_axis_tables(int n_grid, int order, std::vector<double>* inv_win2, std::vector<double>* alias);
// W_t(2 pi n / N)^2 and C_t(2 pi n / N) for n = 0..N/2.
void bl3_axis_tables(int n_grid, std::vector<double>* win2, std::vector<double>* alias);
// e^{-2 pi i m / N}, m = 0..N-1, interleaved (re, im).
std::vector<double> twiddles(int n_grid);
// n^2 -> bin (or -1) for n^2 in [0, (N/2)^2).  Returns false for bad edges.
bool bin_lut(int n_grid, double box, int n_bins, const double* k_edges,
             std::vector<int32_t>* lut, std::vector<double>* edges_out);

// ----------------------------------------------------------------- plan
struct Plan {
  int n = 0;
  mps_precision prec = MPS_F32;
  int device = 0;
  int tile = 16;
  int64_t n_tiles = 0;
  size_t real_size = 4;

  void* grid = nullptr;              // 4 N^3 reals
  float4* sorted = nullptr;          // 2 float4 per particle
  int64_t sorted_cap = 0;
  uint32_t* tile_count = nullptr;    // n_tiles
  uint32_t* tile_offset = nullptr;   // n_tiles + 1
  uint32_t* tile_cursor = nullptr;   // n_tiles
  uint32_t* tile_queue = nullptr;    // 8 work-queue counters of the scatter
  float* halo = nullptr;             // halo form: n_tiles x 4 x kHaloCells (allocated on first use)
  uint32_t* pair_scratch = nullptr;  // paired deposits (FP32, 16^3 tiles; allocated on first use)
  int pair_blocks = 0;
  int num_cus = 256;
  double* moment_partials = nullptr; // kMomentBlocks x (kMomentSums + kMomentMax)
  ResultHeader* d_header = nullptr;
  double* d_iwin2[kNumKernels] = {};  // per kernel, N/2 + 1: 1 / W(2 pi n / N)^2
  double* d_alias[kNumKernels] = {};  // per kernel, N/2 + 1: sum_J W^2(w + 2 pi J)
  void* d_twiddle = nullptr;         // N complex of the plan's precision
  int32_t* d_lut = nullptr;          // (N/2)^2
  double* d_bin_partials = nullptr;  // bin_blocks x kMaxBins x kNumQ
  double* d_bins = nullptr;          // kMaxBins x kNumQ (final sums)
  int bin_blocks = 0;

  // anisotropic estimate (allocated on first use)
  double* d_mu_partials = nullptr;   // bin_blocks x kMaxMuCells x kNumQMu
  double* d_mu_bins = nullptr;       // kMaxMuCells x kNumQMu
  void* h_stage_mu = nullptr;        // pinned: header + kMaxMuCells x kNumQMu

  // device copy of a host-resident catalog (MPS_CATALOG_HOST)
  float* host_stage = nullptr;       // host_cap x 7: pos, vel, weight
  int64_t host_cap = 0;

  // sub-cube split (allocated on first use)
  float* split_pos = nullptr;        // split_cap x 3
  float* split_vel = nullptr;        // split_cap x 3
  float* split_w = nullptr;          // split_cap
  int64_t split_cap = 0;
  uint32_t* split_count = nullptr;   // kMaxCubes counts + 1 flag
  uint32_t* split_offset = nullptr;  // kMaxCubes + 1
  uint32_t* split_cursor = nullptr;  // kMaxCubes
  uint32_t* h_split = nullptr;       // pinned copy of split_count
  void* h_stage_sub = nullptr;       // pinned: kMaxCubes result slots of stage_bytes
  // concurrent sub-sample estimates: helper plans of the same shape, each
  // on its own stream (created on first use)
  static constexpr int kSubLanes = 4;
  Plan* sub_plan[kSubLanes - 1] = {};
  hipStream_t sub_stream[kSubLanes] = {};
  hipEvent_t sub_done[kSubLanes] = {};

  // host staging (pinned): header + bins
  void* h_stage = nullptr;
  size_t stage_bytes = 0;

  // bin-table cache key
  double lut_box = -1.0;
  int lut_nbins = -1;
  std::vector<double> lut_edges;     // edges the LUT was built for (empty: default)
  std::vector<double> edges_used;    // n_bins + 1 edges actually used

  TapPoly taps[kNumKernels];         // per kernel (see kernel_id)
  TapBound tap_bound[kNumKernels];

  // stage timing
  bool timing = false;
  hipEvent_t ev[kNumStages + 1] = {};
  double stage_ms[kNumStages] = {};
};

constexpr int kMomentBlocks = 1024;

// Sort/scatter tile edge for an N^3 grid.
inline int tile_for(int n, mps_precision) { return n >= 16 ? 16 : 8; }
// Work items of the fused x pass (ky rows times kz blocks of the pencils).
inline int x_bin_items(int n, mps_precision prec) {
  int b = (prec == MPS_F32 ? 8 : 4) * 512 / (n > 512 ? n : 512);
  if (b > n / 2) b = n / 2;
  return n * ((n / 2) / b);
}

// Estimate steps shared by the C ABI and the server (api.cpp).
int validate_catalog(const Plan* p, const mps_catalog* c);
int ensure_bins(Plan* p, const mps_catalog* c);
int ensure_particles(Plan* p, int64_t np);
int ensure_host_stage(Plan* p, int64_t np);
constexpr size_t kHostStageBytes = 7 * sizeof(float);  // per particle
// Bytes of the device copy a host-resident catalog of np particles needs.
inline size_t host_stage_bytes(const mps_catalog* c) {
  return (c->flags & MPS_CATALOG_HOST) ? kHostStageBytes * static_cast<size_t>(c->n_particles) : 0;
}
// Async, including the copy of the results to `stage` (the plan's own
// staging buffer when NULL).
int enqueue_estimate(Plan* p, const mps_catalog* c, hipStream_t s, void* stage = nullptr);

// Groups of the multi-catalog scatter launches (see scatter_group).
constexpr int kScatterGroups = 6;
// Device and pinned buffers of the multi-catalog scatter launches: catalog
// descriptors (cap of them), tile prefix sums (cap + kScatterGroups: one
// array per group), queue counters (8 per group), and one event per group
// (and one for the catalogs scattered on their own) that the catalogs'
// later stages wait for.  Grown on demand, kept by their owner.
struct BatchWorkspace {
  ScatterCat* d_cats = nullptr;
  int64_t* d_starts = nullptr;
  uint32_t* d_queue = nullptr;
  hipEvent_t done[kScatterGroups + 1] = {};
  ScatterCat* h_cats = nullptr;
  int64_t* h_starts = nullptr;
  int cap = 0;
  int ensure(int n);
};
// Estimates of n catalogs (plans[i] for cats[i]) on n_lanes streams with the
// multi-catalog scatter (events: n_lanes events for the joins); results go to
// stages[i] (or each plan's own staging buffer).  Async.
int enqueue_batch(Plan* const* plans, const mps_catalog* cats, int n, hipStream_t* lanes, int n_lanes,
                  hipEvent_t* events, BatchWorkspace* ws, void* const* stages);
// After the stream synced; reads `stage` (the plan's own when NULL).
int unpack(Plan* p, const mps_catalog* c, mps_result* out, const void* stage = nullptr);

// Launchers (particles.hip).  All enqueue on `stream`.
hipError_t launch_count(Plan* p, const mps_catalog* c, hipStream_t s);
hipError_t launch_derive(Plan* p, const mps_catalog* c, hipStream_t s);
hipError_t launch_scan(Plan* p, const mps_catalog* c, hipStream_t s);
hipError_t launch_permute(Plan* p, const mps_catalog* c, hipStream_t s);
hipError_t launch_clear_grid(Plan* p, hipStream_t s);
// The count, derive, scan and permute with fewer dependent launches (no
// stage marks between them): one clear of the tile counters, the header and,
// when clear_grid and the sort keeps no records in the grid, the grid
// (*grid_cleared then true); the count; the derivation and the scan in one
// launch for the one-level sort; the permute.
hipError_t launch_sort_fused(Plan* p, const mps_catalog* c, hipStream_t s, bool clear_grid, bool* grid_cleared);
hipError_t launch_scatter(Plan* p, const mps_catalog* c, hipStream_t s);
// The catalog's scatter form (ScatterForm; FP64 grids take kFormGather or
// kFormAtomic, the kernels other than the truncated BL3 kFormAtomic).
int scatter_form(const Plan* p, const mps_catalog* c);
// The form a truncated-BL3 catalog of np particles takes on an N^3 grid of
// this precision, and the halo buffer's bytes.
int scatter_form_for(int n_grid, mps_precision prec, int64_t np);
size_t halo_bytes(int n_grid, mps_precision prec);
// Allocate what the catalog's scatter needs: sorted records and, for the
// halo form, the halo buffer (api.cpp).
int ensure_scatter_space(Plan* p, const mps_catalog* c);
int ensure_halo(Plan* p);
int ensure_pair_scratch(Plan* p);
// Whether a catalog of np particles on this grid can take paired deposits
// (its plan then needs the job scratch).
bool pairs_reachable(int n, mps_precision prec, int64_t np);
// The multi-catalog scatter: one launch over the tiles of several catalogs
// of one group (d_cats, d_starts: device arrays of n_cats descriptors and
// n_cats + 1 tile prefix sums; d_queue: 8 counters), followed for the halo
// form by its fix-up.  scatter_group: the catalog's group, 2 x form +
// (records carry weights ? 1 : 0), or -1 when it takes a launch of its own.
ScatterCat scatter_cat(Plan* p, const mps_catalog* c);
int scatter_group(const Plan* p, const mps_catalog* c);
hipError_t launch_scatter_multi(const ScatterCat* d_cats, const int64_t* d_starts, int n_cats, int64_t n_items,
                                int group, const TapPoly& tp, const TapBound& tb, uint32_t* d_queue, int num_cus,
                                hipStream_t s);

// Launchers (fft.hip).
hipError_t launch_fft_z(Plan* p, void* grid, hipStream_t s);
hipError_t launch_fft_y(Plan* p, void* grid, hipStream_t s);
hipError_t launch_fft_x_store(Plan* p, void* grid, hipStream_t s);
hipError_t launch_fft_x_bin(Plan* p, const mps_catalog* c, hipStream_t s);
hipError_t launch_finalize(Plan* p, const mps_catalog* c, hipStream_t s);
// (k, mu) binning of the stored transform; axis is a host unit vector or
// NULL for the bulk-flow direction (computed on the device).
hipError_t launch_mu_bin(Plan* p, const mps_catalog* c, int n_mu, const double* axis, hipStream_t s);
hipError_t launch_finalize_mu(Plan* p, const mps_catalog* c, int n_mu, hipStream_t s);

// Launchers (subcubes.hip).  count: n_cubes counts, then a non-finite flag.
hipError_t launch_split_count(const mps_catalog* c, const SplitParams& sp, uint32_t* count, hipStream_t s);
hipError_t launch_split_permute(const mps_catalog* c, const SplitParams& sp, const uint32_t* count,
                                uint32_t* offset, uint32_t* cursor, float* out_pos, float* out_vel, float* out_w,
                                hipStream_t s);

}  // namespace mps
