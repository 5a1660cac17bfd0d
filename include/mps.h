/*
 * mps.h -- momentum power spectra of a periodic particle catalog on one
 * AMD Instinct MI355X (gfx950), C ABI.
 *
 * The library implements the FFT estimator of J. Pan, "Estimating power
 * spectrum of discrete cosmic momentum field with fast Fourier transform":
 *
 *   - the momentum field p = (1 + delta) v (Eq. 1) and its Fourier estimator
 *     p_hat(k) = (1/N) sum_j v_j e^{i k.r_j} (Eq. 4), generalised to weights
 *     w_j (N -> W = sum w, shot terms use sum w^2);
 *   - assignment of rho, rho v_x, rho v_y, rho v_z to a periodic N^3 grid
 *     with the third-order (cubic) orthogonalised Battle-Lemarie scaling
 *     function (Sec. 2.4.1), truncated to six taps per axis (d in (-3, 3]);
 *   - 3D real-to-complex FFTs of the four fields;
 *   - deconvolution by the window W_t(k)^2 of the truncated kernel and
 *     subtraction of the shot noise scaled by its alias sum
 *     sum_J W_t^2(k + 2 k_N J) (Eqs. rawPp, rawPtheta, rawPx);
 *   - the divergence theta_p = i k.p / (Haf) (Sec. 2.2), with the
 *     directional shot noise k^T S k / Haf^2 (Eq. thetanoise);
 *   - optional bulk-flow removal v' = v - v_b, v_b = sum w v / W (Sec. 3.1);
 *   - averages in |k| shells of P_pp = <|p|^2> (Eq. 3), P_theta-theta,
 *     Re P_delta-theta (its shot noise is purely imaginary, Eq. rawPx) and the
 *     density spectrum P_dd.
 *
 * Conventions (where the paper is silent):
 *   - grid node g sits at g L / N; a particle's grid coordinate is
 *     u = (double)x * ((double)N / L), its cell floor(u) mod N, and it
 *     deposits phi(j - f) on nodes cell + j, j = -2..3, f = u - floor(u);
 *   - spectra are multiplied by V = L^3 (units (Mpc/h)^3 (km/s)^2 for P_pp,
 *     (Mpc/h)^3 otherwise when L is in Mpc/h and velocities in km/s);
 *   - bins are half-open shells [k_b, k_{b+1}); the DC mode and every mode
 *     with |k| >= k_N = pi N / L are excluded.  Without explicit edges the
 *     bins are n_bins linear bins on [0, k_N) and a mode with integer vector
 *     n joins bin b iff (b N/2)^2 <= n_bins^2 |n|^2 < ((b+1) N/2)^2, decided
 *     in exact integer arithmetic.  With edges, bin b holds modes with
 *     t_b <= |n|^2 < t_{b+1}, t_b = (k_b / k_f)^2, k_f = 2 pi / L, in FP64;
 *   - empty bins report n_modes = 0 and NaN values.
 *
 * All functions return an int status: MPS_OK (0) or a negative MPS_E_* code.
 * No exception crosses the ABI.  Device pointers are HIP device (or managed)
 * pointers on the plan's device; host pointers are ordinary host memory.
 */
#ifndef MPS_H_
#define MPS_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPS_OK 0
#define MPS_E_ARG (-1)        /* invalid argument (null pointer, size, bins) */
#define MPS_E_NONFINITE (-2)  /* a position, velocity or weight is NaN/Inf */
#define MPS_E_ZEROWEIGHT (-3) /* sum of weights is zero */
#define MPS_E_NOMEM (-4)      /* device or pinned allocation failed */
#define MPS_E_HIP (-5)        /* a HIP runtime call failed */
#define MPS_E_TIMEOUT (-6)    /* mps_wait timed out */
#define MPS_E_BUSY (-7)       /* the server queue is full */
#define MPS_E_TOOBIG (-8)     /* request can never fit the server's budget,
                                 or exceeds the static workspace */

#define MPS_MAX_BINS 128

typedef enum { MPS_F32 = 1, MPS_F64 = 2 } mps_precision;

enum {
  MPS_BULKFLOW_SUBTRACT = 1u << 0, /* use v - v_b (Sec. 3.1) */
  MPS_NO_SHOTNOISE = 1u << 1,      /* report raw (deconvolved) spectra */
  MPS_NO_DECONVOLVE = 1u << 2,     /* do not divide by W_t(k)^2 */
  /* Assign with the untruncated BL3 function phi = sum_n c_n beta3(x - n)
   * (Sec. 2.4.1) instead of its six-tap truncation.  Since c_n is a periodic
   * filter with transform A(w)^(-1/2), the deconvolved spectra equal those of
   * the cubic B-spline assignment (4 taps) deconvolved by sinc^4(w/2) per
   * axis, with the alias sum A(w) in the shot terms; that is what is
   * computed.  mps_assign then returns the cubic B-spline grids. */
  MPS_KERNEL_BL3_EXACT = 1u << 3
};

/* Assignment with the centred B-spline of order p (degree p - 1) instead of
 * BL3: the comparison kernels of Sec. 2.4.1 (a fifth-order B-spline) and
 * Sec. 2.4.3 (nearest grid point).  p = 1 NGP, 2 CIC, 3 TSC, 4 PCS, 5 PQS,
 * 6 the quintic.  Node g receives beta_{p-1}(g - u) (u the particle's grid
 * coordinate; the box beta_0 is 1 on (-1/2, 1/2], so with p = 1 a particle
 * joins node floor(u + 1/2), the sum rounded in FP64).  The spectra are
 * deconvolved by the window sinc^p(w/2) per axis, and the shot terms scale
 * with the alias sum sum_m beta_{2p-1}(m) cos(m w).  Put
 * MPS_KERNEL_BSPLINE(p) in the flags; it cannot be combined with
 * MPS_KERNEL_BL3_EXACT (which equals MPS_KERNEL_BSPLINE(4) in its
 * spectra). */
#define MPS_KERNEL_ORDER_SHIFT 4
#define MPS_KERNEL_BSPLINE(p) ((uint32_t)(p) << MPS_KERNEL_ORDER_SHIFT)

/* The other reading of the "third-order" Battle-Lemarie function of
 * Sec. 2.4.1, order counted as the number of polynomial coefficients: the
 * quadratic-spline member, phi_hat(w) = sinc^3(w/2) / sqrt(A2(w)) with
 * A2(w) = (66 + 52 cos w + 2 cos 2w) / 120, phi = sum_n c_n beta2(x - n)
 * (knots at the half-integers).  Same six taps and support d in (-3, 3] as
 * the default cubic reading; each tap weight is two quadratics in the
 * fraction, split at f = 1/2.  Deconvolved by the truncated function's own
 * window, shot terms scaled by its own alias sum.  Cannot be combined with
 * MPS_KERNEL_BL3_EXACT. */
#define MPS_KERNEL_BL3_QUADRATIC (7u << MPS_KERNEL_ORDER_SHIFT)

/* The catalog's pos, vel and weight are host pointers: the plan copies them
 * to device workspace (28 bytes per particle, kept for reuse) on the call's
 * stream before the first kernel.  Page-locked (pinned) host memory lets the
 * copy run asynchronously and overlap other streams' work; pageable memory
 * works but copies synchronously.  Accepted by every estimate entry point
 * and by mps_submit. */
#define MPS_CATALOG_HOST (1u << 7)

/* One catalog.  The caller owns every buffer; they must stay valid until the
 * call that uses them returns (or, for mps_submit, until mps_wait reports the
 * ticket done).  The library never frees or retains them. */
typedef struct {
  int64_t n_particles;   /* 1 .. 2^31 - 1 */
  const float* pos;      /* device, n x 3 interleaved (x, y, z); any finite
                            value, wrapped periodically into [0, L) */
  const float* vel;      /* device, n x 3 interleaved */
  const float* weight;   /* device, n; NULL means unit weights */
  double box;            /* L > 0 */
  double haf;            /* H a f > 0, velocity units per length unit */
  int n_bins;            /* 1 .. MPS_MAX_BINS */
  const double* k_edges; /* host, n_bins + 1 strictly ascending values in
                            [0, k_N], or NULL for linear bins on [0, k_N) */
  uint32_t flags;        /* MPS_BULKFLOW_SUBTRACT | MPS_NO_SHOTNOISE | ... */
} mps_catalog;

/* Results.  Array members are caller-allocated host arrays of length n_bins;
 * any of them may be NULL to skip that output.  The scalar members are
 * written by the library. */
typedef struct {
  double* k_mean;   /* mode-averaged |k| per bin */
  double* p_pp;     /* momentum auto spectrum, shot noise subtracted */
  double* p_tt;     /* momentum-divergence auto spectrum */
  double* p_dt;     /* Re of the density x divergence cross spectrum */
  double* p_dd;     /* density spectrum */
  double* sn_pp;    /* bin-averaged shot terms that were (or would be) */
  double* sn_tt;    /*   subtracted, after deconvolution */
  double* sn_dd;
  int64_t* n_modes; /* modes in the bin (full sphere, both k and -k) */
  double v_bulk[3]; /* v_b = sum w v / W */
  double sigma_v2;  /* sum w^2 |v|^2 / sum w^2 of the velocities used */
  double n_eff;     /* W^2 / sum w^2 (= N for unit weights) */
} mps_result;

/* Results of mps_estimate_mu: the spectra of Sec. 3 binned in (k, mu_b),
 * mu_b the cosine between k and a unit axis a (by default the bulk flow
 * direction v_b / |v_b|).  Array members are caller-allocated host arrays of
 * n_bins * n_mu values, element [b * n_mu + m] for k bin b and mu bin m
 * (mu bins uniform on [-1, 1]); any may be NULL.  Complex cross spectra are
 * given in the paper's Fourier convention (fields sum_j w_j ... e^{+ik.r_j},
 * Eq. 4): P_dt = delta theta^* (Eq. rawPx) and P_dpb = delta conj(a.p')
 * with p' the momentum of v - v_b (Eq. bfpp). */
typedef struct {
  double* k_mean;    /* mode-averaged |k| */
  double* mu_mean;   /* mode-averaged mu_b */
  double* p_pp;      /* as in mps_result */
  double* p_tt;
  double* p_dd;
  double* p_dt_re;   /* Re P_delta-theta (no shot term) */
  double* p_dt_im;   /* Im P_delta-theta, shot term subtracted */
  double* p_dpb_re;  /* Re P_{delta p'_b}, shot term subtracted */
  double* p_dpb_im;  /* Im P_{delta p'_b} (no shot term) */
  double* sn_pp;     /* bin-averaged shot terms, after deconvolution */
  double* sn_tt;
  double* sn_dd;
  double* sn_dt_im;  /* -(k.s) C / (Haf W^2), s = sum w^2 v / W^2 (v used) */
  double* sn_dpb;    /* (a.s') C / W^2, s' = sum w^2 (v - v_b) / W^2 */
  int64_t* n_modes;  /* modes in the cell (k and -k counted separately) */
  double axis[3];    /* the unit axis used */
  double v_bulk[3];
  double sigma_v2;
  double n_eff;
} mps_result_mu;

#define MPS_MAX_MU_BINS 64
#define MPS_MAX_MU_CELLS 512   /* n_bins * n_mu */
#define MPS_MAX_DIV 8          /* sub-cubes per axis in mps_estimate_subcubes */
#define MPS_MAX_SUBCUBES 512   /* MPS_MAX_DIV^3 */
/* MPS_F32 with the truncated BL3 kernel on grids of N >= MPS_SCATTER_MIN_GRID:
 * the scatter's form follows the mean number of particles per 16^3 tile,
 * m = n_particles / (N/16)^3 (see mps_plan_create): m <=
 * MPS_SCATTER_GATHER_MAX_MEAN, the owner-computes scatter; else m <=
 * MPS_SCATTER_HALO_MAX_MEAN, the halo scatter (its halo buffer, 5165 x 16
 * bytes per tile, is allocated on first use and counted by mps_footprint);
 * else, and on smaller grids, the atomic scatter, whose dense tiles deposit
 * pairs of particles in one cell or z-neighbouring cells together (its job
 * scratch, 64 KB per workgroup for up to 256 workgroups, is likewise
 * allocated on first use and counted by mps_footprint). */
#define MPS_SCATTER_MIN_GRID 128
#define MPS_SCATTER_GATHER_MAX_MEAN 384
#define MPS_SCATTER_HALO_MAX_MEAN 2048
/* MPS_F64 with the truncated BL3 kernel on grids of N >= MPS_SCATTER_MIN_GRID:
 * m <= MPS_SCATTER_GATHER64_MAX_MEAN, the owner-computes scatter (64-bit
 * fixed point, as the atomic FP64 scatter); else the atomic scatter, with
 * the paired deposits and job scratch of the FP32 atomic scatter. */
#define MPS_SCATTER_GATHER64_MAX_MEAN 384

typedef struct mps_plan mps_plan;
typedef struct mps_server mps_server;

/* Create a plan for N^3 grids (N a power of two in [8, 1024]) on the current
 * HIP device.  The plan owns the four grids, FFT twiddles, the BL3 tables
 * and the bin tables; particle workspace grows on demand (or see
 * mps_plan_reserve).  A plan is not thread-safe.
 *
 * prec is the grid and FFT precision.  MPS_F32: the assignment sums in
 * 32-bit fixed point scaled per tile from a bound on every cell, so the
 * grid carries FP32-level resolution.  Each 16^3 tile deposits its
 * particles over itself and a halo (2 cells below, 3 above per axis) and
 * adds the block to the grid with FP32 atomics (the atomic scatter), or
 * stores its own cells and its halo in a halo buffer, a fix-up pass adding
 * the neighbours' halos to each cell in a fixed order (the halo scatter,
 * deterministic), or gathers the particles whose taps reach it and stores
 * its own cells (the owner-computes scatter, deterministic); see
 * MPS_SCATTER_GATHER_MAX_MEAN.  MPS_F64: the assignment sums in
 * 64-bit fixed point with a unit of 2^-50 of the largest possible deposit
 * (coarser only for tiles of more than 4096 particles), FP64-level.  The
 * moments, tables, per-mode estimator and shell sums are FP64 in both. */
int mps_plan_create(mps_plan** out, int n_grid, mps_precision prec);
int mps_plan_destroy(mps_plan* plan);

/* Pre-allocate workspace for catalogs of up to max_particles particles so
 * that later calls allocate nothing: the sorted records and, for MPS_F32
 * plans on which such a catalog can take the halo or the atomic scatter,
 * the halo buffer or the paired deposits' job scratch (see
 * MPS_SCATTER_GATHER_MAX_MEAN). */
int mps_plan_reserve(mps_plan* plan, int64_t max_particles);

/* Device bytes a plan of this shape holds when used for n_particles. */
size_t mps_footprint(int n_grid, mps_precision prec, int64_t n_particles);

/* Estimate the binned spectra of one catalog.  All work is enqueued on
 * `stream`; the call returns after the few-KB result copy has completed. */
int mps_estimate(mps_plan* plan, const mps_catalog* cat, mps_result* out,
                 hipStream_t stream);

/* Estimate n catalogs, each with its own plan (plans may differ in N and
 * precision; a plan may not appear twice).  The catalogs' stages are
 * enqueued round robin on four internal streams that start after the
 * earlier work on `stream`, so that small catalogs' kernels overlap on the
 * device; `stream` waits for all of them and the call returns after every
 * result is copied. */
int mps_estimate_batch(mps_plan* const* plans, const mps_catalog* cats,
                       mps_result* outs, int n, hipStream_t stream);

/* Anisotropic spectra (Sec. 3: the bulk-flow terms of Eqs. thetanoise,
 * rawPx, bfpp and bfpdpx resolved by mu_b).  n_mu in [1, MPS_MAX_MU_BINS]
 * with n_bins * n_mu <= MPS_MAX_MU_CELLS.  axis: host pointer to 3 doubles
 * (need not be unit; must be non-zero), or NULL to use v_b, in which case a
 * catalog with v_b = 0 exactly returns MPS_E_ARG.  mu is computed in FP64 as
 * (n.a)/|n| with a = axis/|axis| and every operation separately rounded, and
 * mode n goes to mu bin min(floor((mu + 1) n_mu / 2), n_mu - 1).  The flags
 * act as in mps_estimate (MPS_BULKFLOW_SUBTRACT: p' replaces p in P_pp,
 * P_tt and P_dt).  Same stream semantics as mps_estimate; the x transform is
 * stored and binned by a separate pass, so the call costs one extra pass
 * over the grid. */
int mps_estimate_mu(mps_plan* plan, const mps_catalog* cat, int n_mu,
                    const double* axis, mps_result_mu* out, hipStream_t stream);

/* Spectra of sub-samples (Sec. 2.4.1: the periodic box cut evenly into
 * n_div^3 non-overlapping cubes of side L / n_div; Secs. 3.3 and 4.1 average
 * them and take their scatter as error bars).
 *
 * The catalog `cat` (box L) is split on the device: per axis
 * u = x (n_div / L) in FP64, g = floor(u), cube index
 * m = g - n_div floor(g / n_div) clamped to [0, n_div - 1], and the particle's
 * position within its cube x' = x - g (L / n_div) rounded to float32 (FP64,
 * no fused operations).  Sub-cube s = (m_x n_div + m_y) n_div + m_z is then
 * estimated exactly as mps_estimate estimates a catalog of those particles
 * (velocities and weights unchanged) in a periodic box of side L / n_div on
 * the plan's N^3 grid: k_edges, if given, apply to every sub-cube, the
 * default bins are linear on [0, k_N) of the sub-box, and
 * MPS_BULKFLOW_SUBTRACT removes each sub-cube's own bulk flow.
 *
 * n_div: 1 .. MPS_MAX_DIV.  outs: host array of n_div^3 results (array
 * members caller-allocated as for mps_estimate, or NULL); status: host array
 * of n_div^3 ints, MPS_OK or the sub-cube's error (MPS_E_ZEROWEIGHT for a
 * cube without particles, whose outs arrays are left untouched).  mean, sdev:
 * NULL or results that receive, per bin, the mean and the sample standard
 * deviation (divisor m - 1; NaN for m < 2) over the m sub-cubes with status
 * MPS_OK, likewise for v_bulk, sigma_v2 and n_eff; their n_modes is the mode
 * count of one sub-cube (the same for all).  Returns MPS_E_NONFINITE if any
 * position is not finite, MPS_E_ARG, MPS_E_NOMEM or MPS_E_HIP for the whole
 * call, else MPS_OK.  The sub-catalogs live in plan workspace (28 bytes per
 * particle with weights, 24 without).  The split runs on `stream` after its
 * earlier work; the cubes' estimates then run round robin on this plan and
 * three helper plans of the same shape (created on first use and owned by
 * this plan), each on its own stream, and the call returns after all
 * results are copied. */
int mps_estimate_subcubes(mps_plan* plan, const mps_catalog* cat, int n_div,
                          mps_result* outs, int* status, mps_result* mean,
                          mps_result* sdev, hipStream_t stream);

/* One-loop standard perturbation theory predictions (the one-loop section
 * and its appendices: Eqs. Ppd, PpdD4, pdivpD4, the P13 and P22 formulas,
 * Eq. intBktree, Eq. Pcov), FP64 on the device.
 *
 * Inputs (host): k[n_k] > 0, the wavenumbers to predict at; a table of the
 * z = 0 linear spectrum P0, table_k[n_table] strictly ascending > 0 and
 * table_p[n_table] > 0, interpolated linearly in (ln k, ln P) and zero
 * outside [table_k[0], table_k[n_table - 1]]; d_z = D(z)/D(0); haf = H a f.
 * n_k in [1, MPS_SPT_MAX_K], n_table in [2, MPS_SPT_MAX_TABLE].
 *
 * Outputs (host arrays of n_k, each may be NULL), with K_xy the P13 kernels
 * (their logarithm read with the factor 3/r^3), y = 1 + r^2 - 2 r x:
 *   p13, p13_dt, p13_tt: c P0(k) k^3/(4 pi^2) int dr P0(kr) K_xy(r),
 *     c = 1/504, 1/504, 1/168;
 *   p22, p22_dt, p22_tt: k^3/(98 4 pi^2) int dr P0(kr) int dx P0(k sqrt(y))
 *     N_x N_y / y^2, N_delta = 3r + 7x - 10 r x^2, N_theta = 7x - r - 6 r x^2;
 *   i1, i2, i3: the three terms of the tree-level bispectrum integral
 *     B_dtt,0 = i1 + i2 + i3 (Eq. intBktree);
 *   pcov1, pcov2: P_cov^I and P_cov^II (Eq. Pcov);
 *   p_lin = D^2 P0; p_dd = D^2 P0 + D^4 (2 p13 + p22);
 *   p_theta_p = D^2 P0 + D^4 (6 p13 + 4 p22) and
 *   p_dtheta_p = D^2 P0 + D^4 (4 p13 + 2 p22) (Eq. pdivpD4);
 *   p_mom = (Haf/k)^2 [D^2 P0 + D^4 (2 p13_tt + p22_tt + pcov1 + pcov2
 *     + 2 k^2 (i1 + i2 + i3))] (Eq. PpdD4).
 * The integrals use fixed Gauss-Legendre panels between the points where
 * the integrands are not smooth.  MPS_E_ARG for bad sizes, non-positive or
 * non-finite k, table values or haf, or a table that is not ascending;
 * MPS_E_NOMEM, MPS_E_HIP.  Work is enqueued on `stream`; the call returns
 * after the results are copied. */
#define MPS_SPT_MAX_K 65536
#define MPS_SPT_MAX_TABLE 2048
#define MPS_SPT_NUM_OUT 16
typedef struct {
  double *p13, *p22, *p13_dt, *p22_dt, *p13_tt, *p22_tt;
  double *i1, *i2, *i3;
  double *pcov1, *pcov2;
  double *p_lin, *p_dd, *p_theta_p, *p_dtheta_p, *p_mom;
} mps_spt_result;

int mps_spt_one_loop(const double* k, int n_k, const double* table_k,
                     const double* table_p, int n_table, double d_z,
                     double haf, mps_spt_result* out, hipStream_t stream);

/* Diagnostics of the hot path's first stages, using the same kernels as
 * mps_estimate.  mps_assign writes the four assigned real grids
 * (rho, rho v_x, rho v_y, rho v_z; layout [field][x][y][z], z fastest, the
 * plan's precision) to `grids`, a device buffer of 4 N^3 reals.  With
 * MPS_BULKFLOW_SUBTRACT the momentum grids are those of v - v_b.
 * mps_fft transforms such grids in place: on return `grids` holds, per field,
 * the complex array F[x][y][kz] for kz in [0, N/2) (e^{-2 pi i n.g / N}; the
 * kz = N/2 plane, never binned, is dropped), interleaved (re, im). */
int mps_assign(mps_plan* plan, const mps_catalog* cat, void* grids,
               hipStream_t stream);
int mps_fft(mps_plan* plan, void* grids, hipStream_t stream);

/* Per-stage device time of the last mps_estimate on this plan when stage
 * timing is on (mps_plan_set_timing).  ms[0..n) receives, in order:
 * moments+count, scan, permute, clear, scatter, fft_z, fft_y, fft_x+bin,
 * finalize.  With timing off the first stages run as fewer launches (the
 * clears together before the count, the moments' derivation and the scan
 * in one), which only their boundaries tell apart; results agree as those
 * of two untimed runs do. */
int mps_plan_set_timing(mps_plan* plan, int enable);
int mps_plan_stage_times(const mps_plan* plan, double* ms, int n);

/* Serving: continuous batching of catalogs of uneven sizes.
 * hbm_budget_bytes bounds the device memory the server's plans and
 * workspaces may hold; max_inflight bounds requests on the device at once;
 * small_particles is the particle count below which requests of one grid
 * size are batched together.  mps_submit copies the catalog descriptor (not
 * the buffers) and returns a ticket; mps_wait blocks until the ticket is done
 * (then its mps_result is filled and its status returned) or timeout_s
 * elapses (MPS_E_TIMEOUT).  The server is thread-safe.
 *
 * Ordering: `stream` is the stream on which the catalog's device buffers are
 * produced (NULL: the null stream).  mps_submit records an event on it, and
 * the request's kernels start only after everything enqueued on `stream`
 * before the call has completed, so a catalog written by a kernel still in
 * flight is never read early.  Host-resident catalogs (MPS_CATALOG_HOST)
 * must be complete when mps_submit is called.
 *
 * Admission: a request runs once a worker is free and a plan of its grid
 * size and precision with room for its particles fits the budget (idle
 * plans are evicted least-recently-used; plans are created, grown and
 * destroyed outside the server's lock).  Later requests may overtake a
 * waiting one, at most 8 times; after that nothing behind it is admitted
 * until it fits. */
int mps_server_create(mps_server** out, size_t hbm_budget_bytes,
                      int max_inflight, int64_t small_particles);
int mps_submit(mps_server* srv, const mps_catalog* cat, int n_grid,
               mps_precision prec, mps_result* out, hipStream_t stream,
               uint64_t* ticket);
int mps_wait(mps_server* srv, uint64_t ticket, double timeout_s);
int mps_server_destroy(mps_server* srv);

/* The estimate of mps_estimate with no device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  No plan: every buffer a plan would own
 * lives in a fixed workspace, a file-scope device array of the library
 * (about 43 MB, held on each GPU the call runs on until the process ends).
 * Limits: n_grid a power of two in [8, MPS_STATIC_MAX_GRID] and at most
 * MPS_STATIC_MAX_PARTICLES particles, else MPS_E_TOOBIG; device-resident
 * catalogs only (MPS_CATALOG_HOST gives MPS_E_ARG); every other argument,
 * flag and error as mps_estimate.  Enqueues on `stream` and returns after the
 * results are copied back.  All calls on one GPU share the workspace, which
 * keeps the last call's contents (every stage clears what it accumulates
 * into): the host side is serialised, but calls whose work overlaps on the
 * device, on different streams, race.  Host-side tables are rebuilt only
 * when the grid size, precision, kernel or bins change. */
#define MPS_STATIC_MAX_GRID 64
#define MPS_STATIC_MAX_PARTICLES (1 << 20)
int mps_estimate_static(const mps_catalog* cat, int n_grid, mps_precision prec,
                        mps_result* out, hipStream_t stream);

const char* mps_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MPS_H_ */
