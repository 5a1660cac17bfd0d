"""Python face of libmps.so.  Only argument marshalling happens here: every
step of the estimator runs in the library's HIP kernels.  torch tensors supply
device memory and the stream."""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_OUT_KEYS = ("k_mean", "p_pp", "p_tt", "p_dt", "p_dd", "sn_pp", "sn_tt", "sn_dd")


def _prec(precision) -> int:
    if precision in ("f32", "float32", torch.float32, L.MPS_F32):
        return L.MPS_F32
    if precision in ("f64", "float64", torch.float64, L.MPS_F64):
        return L.MPS_F64
    raise ValueError(f"unknown precision {precision!r}")


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _device_f32(t, name, cols, host_ok=False):
    if not isinstance(t, torch.Tensor) or not (t.is_cuda or (host_ok and t.device.type == "cpu")):
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor"
                        + (" or a CPU tensor (pinned memory recommended)" if host_ok else ""))
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if cols and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{name} must have shape (n, {cols})")
    return t


def _flags(bulk_flow, no_shotnoise, no_deconvolve, kernel="bl3") -> int:
    if kernel not in L.KERNELS:
        raise ValueError(f"kernel must be one of {sorted(L.KERNELS)}")
    return ((L.BULKFLOW_SUBTRACT if bulk_flow else 0) | (L.NO_SHOTNOISE if no_shotnoise else 0)
            | (L.NO_DECONVOLVE if no_deconvolve else 0) | L.KERNELS[kernel])


def make_catalog(pos, vel, weight=None, *, box, haf=1.0, n_bins=32, k_edges=None, flags=0):
    """Build an mps_catalog; returns (struct, objects that must stay alive).
    CPU tensors (all three on the host) are passed as a host-resident catalog
    (MPS_CATALOG_HOST): the library copies them to the device."""
    host = isinstance(pos, torch.Tensor) and pos.device.type == "cpu"
    _device_f32(pos, "pos", 3, host_ok=True)
    _device_f32(vel, "vel", 3, host_ok=True)
    for t, name in ((vel, "vel"), (weight, "weight")):
        if t is not None and (t.device.type == "cpu") != host:
            raise ValueError(f"pos and {name} must both be on the host or both on the device")
    if host:
        flags |= L.CATALOG_HOST
    if vel.shape[0] != pos.shape[0]:
        raise ValueError("pos and vel differ in length")
    keep = [pos, vel]
    cat = L.Catalog()
    cat.n_particles = pos.shape[0]
    cat.pos = pos.data_ptr()
    cat.vel = vel.data_ptr()
    cat.weight = None
    if weight is not None:
        _device_f32(weight, "weight", 0, host_ok=True)
        if weight.dim() != 1 or weight.shape[0] != pos.shape[0]:
            raise ValueError("weight must have shape (n,)")
        cat.weight = weight.data_ptr()
        keep.append(weight)
    cat.box = float(box)
    cat.haf = float(haf)
    if k_edges is not None:
        edges = np.ascontiguousarray(k_edges, dtype=np.float64)
        n_bins = len(edges) - 1
        keep.append(edges)
        cat.k_edges = edges.ctypes.data_as(C.POINTER(C.c_double))
    else:
        cat.k_edges = None
    cat.n_bins = int(n_bins)
    cat.flags = int(flags)
    return cat, keep


def make_result(n_bins):
    arrays = {k: np.full(n_bins, np.nan) for k in _OUT_KEYS}
    arrays["n_modes"] = np.zeros(n_bins, np.int64)
    res = L.Result()
    for k in _OUT_KEYS:
        setattr(res, k, arrays[k].ctypes.data_as(C.POINTER(C.c_double)))
    res.n_modes = arrays["n_modes"].ctypes.data_as(C.POINTER(C.c_int64))
    return res, arrays


def unpack_result(res, arrays, box, n_grid, k_edges, n_bins):
    out = dict(arrays)
    out["v_bulk"] = np.array(res.v_bulk[:])
    out["sigma_v2"] = float(res.sigma_v2)
    out["n_eff"] = float(res.n_eff)
    if k_edges is None:
        k_nyq = (2.0 * np.pi / box) * (n_grid // 2)
        out["k_edges"] = k_nyq * np.arange(n_bins + 1) / n_bins
    else:
        out["k_edges"] = np.asarray(k_edges, dtype=np.float64)
    return out


class Plan:
    """Device grids, FFT twiddles and BL3/bin tables for N^3 grids."""

    def __init__(self, n_grid: int, precision="f32"):
        self.n_grid = int(n_grid)
        self.prec = _prec(precision)
        self.real_dtype = torch.float32 if self.prec == L.MPS_F32 else torch.float64
        h = C.c_void_p()
        L.check(L.lib().mps_plan_create(C.byref(h), self.n_grid, self.prec), "mps_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            L.lib().mps_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_particles: int):
        L.check(L.lib().mps_plan_reserve(self._h, int(max_particles)), "mps_plan_reserve")

    def estimate(self, pos, vel, weight=None, *, box, haf, n_bins=32, k_edges=None,
                 bulk_flow=False, no_shotnoise=False, no_deconvolve=False, kernel="bl3",
                 stream=None):
        """Binned P_pp, P_tt, Re P_dt, P_dd (x V) of one catalog; dict of arrays.
        kernel: "bl3" (six-tap truncated BL3), "bl3q" (its quadratic-spline
        reading, same six taps), "bl3_exact" (untruncated, by a
        cubic B-spline scatter and spectral correction), or a centred B-spline
        of order p: "ngp", "cic", "tsc", "pcs", "pqs", "bspline6" (also
        "bspline1" .. "bspline6")."""
        cat, keep = make_catalog(pos, vel, weight, box=box, haf=haf, n_bins=n_bins,
                                 k_edges=k_edges,
                                 flags=_flags(bulk_flow, no_shotnoise, no_deconvolve, kernel))
        res, arrays = make_result(cat.n_bins)
        L.check(L.lib().mps_estimate(self._h, C.byref(cat), C.byref(res), _stream(stream)),
                "mps_estimate")
        del keep
        return unpack_result(res, arrays, box, self.n_grid, k_edges, cat.n_bins)

    def estimate_mu(self, pos, vel, weight=None, *, box, haf, n_mu, axis=None, n_bins=32,
                    k_edges=None, bulk_flow=False, no_shotnoise=False, no_deconvolve=False,
                    kernel="bl3", stream=None):
        """(k, mu_b)-binned spectra (Sec. 3); arrays of shape (n_bins, n_mu).

        mu_b is the cosine to `axis` (3 numbers) or, by default, to the bulk
        flow.  Complex cross spectra follow the paper's Fourier convention.
        """
        cat, keep = make_catalog(pos, vel, weight, box=box, haf=haf, n_bins=n_bins,
                                 k_edges=k_edges,
                                 flags=_flags(bulk_flow, no_shotnoise, no_deconvolve, kernel))
        nb = cat.n_bins
        ncell = nb * int(n_mu)
        arrays = {k: np.full(ncell, np.nan) for k in L.MU_KEYS}
        arrays["n_modes"] = np.zeros(ncell, np.int64)
        res = L.ResultMu()
        for k in L.MU_KEYS:
            setattr(res, k, arrays[k].ctypes.data_as(C.POINTER(C.c_double)))
        res.n_modes = arrays["n_modes"].ctypes.data_as(C.POINTER(C.c_int64))
        ax = None
        if axis is not None:
            ax = np.ascontiguousarray(axis, dtype=np.float64)
            if ax.shape != (3,):
                raise ValueError("axis must have 3 components")
            keep.append(ax)
        L.check(L.lib().mps_estimate_mu(
            self._h, C.byref(cat), int(n_mu),
            ax.ctypes.data_as(C.POINTER(C.c_double)) if ax is not None else None,
            C.byref(res), _stream(stream)), "mps_estimate_mu")
        del keep
        out = {k: v.reshape(nb, int(n_mu)) for k, v in arrays.items()}
        out["axis"] = np.array(res.axis[:])
        out["v_bulk"] = np.array(res.v_bulk[:])
        out["sigma_v2"] = float(res.sigma_v2)
        out["n_eff"] = float(res.n_eff)
        return out

    def estimate_subcubes(self, pos, vel, weight=None, *, box, haf, n_div=4, n_bins=32,
                          k_edges=None, bulk_flow=False, no_shotnoise=False, no_deconvolve=False,
                          kernel="bl3", stream=None):
        """Spectra of the n_div^3 sub-samples of a periodic catalog of side
        `box` (Sec. 2.4.1), each a periodic catalog of side box / n_div on
        this plan's grid, plus their per-bin mean and sample standard
        deviation.  Returns {"sub": list of per-cube dicts (None for an empty
        cube), "status": int array, "mean": dict, "sdev": dict, "sub_box"}."""
        n_div = int(n_div)
        if not 1 <= n_div <= L.MAX_DIV:
            raise ValueError(f"n_div must be in [1, {L.MAX_DIV}]")
        cat, keep = make_catalog(pos, vel, weight, box=box, haf=haf, n_bins=n_bins,
                                 k_edges=k_edges,
                                 flags=_flags(bulk_flow, no_shotnoise, no_deconvolve, kernel))
        nc = n_div ** 3
        nb = cat.n_bins
        outs = (L.Result * nc)()
        arrays = []
        for s in range(nc):
            res, arr = make_result(nb)
            outs[s] = res
            arrays.append(arr)
        status = np.zeros(nc, dtype=np.int32)
        mean, mean_arr = make_result(nb)
        sdev, sdev_arr = make_result(nb)
        L.check(L.lib().mps_estimate_subcubes(
            self._h, C.byref(cat), n_div, outs, status.ctypes.data_as(C.POINTER(C.c_int)),
            C.byref(mean), C.byref(sdev), _stream(stream)), "mps_estimate_subcubes")
        del keep
        sub_box = float(box) / n_div
        subs = [unpack_result(outs[s], arrays[s], sub_box, self.n_grid, k_edges, nb)
                if status[s] == L.MPS_OK else None for s in range(nc)]
        return {"sub": subs, "status": status, "sub_box": sub_box,
                "mean": unpack_result(mean, mean_arr, sub_box, self.n_grid, k_edges, nb),
                "sdev": unpack_result(sdev, sdev_arr, sub_box, self.n_grid, k_edges, nb)}

    def assign(self, pos, vel, weight=None, *, box, bulk_flow=False, kernel="bl3", stream=None):
        """The four assigned real grids, torch tensor (4, N, N, N) [field, x, y, z]
        (for kernel="bl3_exact", the cubic B-spline grids)."""
        n = self.n_grid
        dev = torch.device("cuda") if pos.device.type == "cpu" else pos.device
        out = torch.empty((4, n, n, n), dtype=self.real_dtype, device=dev)
        cat, keep = make_catalog(pos, vel, weight, box=box, haf=1.0, n_bins=1,
                                 flags=_flags(bulk_flow, False, False, kernel))
        L.check(L.lib().mps_assign(self._h, C.byref(cat), C.c_void_p(out.data_ptr()),
                                   _stream(stream)), "mps_assign")
        del keep
        return out

    def fft(self, grids: torch.Tensor, stream=None):
        """In-place 3D R2C FFT of (4, N, N, N) real grids; returns the complex
        view (4, N, N, N/2) [field, kx, ky, kz] (the kz = N/2 plane dropped)."""
        n = self.n_grid
        if grids.dtype != self.real_dtype or not grids.is_cuda or not grids.is_contiguous():
            raise TypeError("grids must be a contiguous CUDA tensor of the plan's precision")
        if grids.numel() != 4 * n ** 3:
            raise ValueError("grids must hold 4 N^3 reals")
        L.check(L.lib().mps_fft(self._h, C.c_void_p(grids.data_ptr()), _stream(stream)), "mps_fft")
        return torch.view_as_complex(grids.view(4, n, n, n // 2, 2))

    def set_timing(self, enable: bool = True):
        L.check(L.lib().mps_plan_set_timing(self._h, 1 if enable else 0), "mps_plan_set_timing")

    def stage_times(self):
        ms = (C.c_double * L.NUM_STAGES)()
        L.check(L.lib().mps_plan_stage_times(self._h, ms, L.NUM_STAGES), "mps_plan_stage_times")
        return dict(zip(L.STAGES, list(ms)))


def spt_one_loop(k, table_k, table_p, *, d_z=1.0, haf=50.0, stream=None):
    """One-loop SPT predictions at wavenumbers k from a tabulated z = 0 linear
    spectrum (log-log interpolated, zero outside the table); dict of arrays
    (keys as mps_spt_result: p13, p22, ..., p_mom)."""
    kk = np.ascontiguousarray(k, dtype=np.float64).ravel()
    tk = np.ascontiguousarray(table_k, dtype=np.float64).ravel()
    tp = np.ascontiguousarray(table_p, dtype=np.float64).ravel()
    if tk.shape != tp.shape:
        raise ValueError("table_k and table_p differ in length")
    out = {key: np.full(kk.shape[0], np.nan) for key in L.SPT_KEYS}
    res = L.SptResult()
    for key in L.SPT_KEYS:
        setattr(res, key, out[key].ctypes.data_as(C.POINTER(C.c_double)))
    dp = C.POINTER(C.c_double)
    L.check(L.lib().mps_spt_one_loop(kk.ctypes.data_as(dp), kk.shape[0], tk.ctypes.data_as(dp),
                                     tp.ctypes.data_as(dp), tk.shape[0], float(d_z), float(haf),
                                     C.byref(res), _stream(stream)), "mps_spt_one_loop")
    return out


def footprint(n_grid: int, precision, n_particles: int) -> int:
    return int(L.lib().mps_footprint(int(n_grid), _prec(precision), int(n_particles)))


def estimate(pos, vel, weight=None, *, box, n_grid, haf, precision="f32", **kw):
    """One-shot estimate with a temporary plan."""
    plan = Plan(n_grid, precision)
    try:
        return plan.estimate(pos, vel, weight, box=box, haf=haf, **kw)
    finally:
        plan.close()


def estimate_batch(plans: Sequence[Plan], catalogs: Sequence[dict], stream=None):
    """Estimate catalogs[i] (dict of estimate() keyword arguments plus pos, vel,
    weight) with plans[i], all stages enqueued together."""
    n = len(plans)
    if len(catalogs) != n:
        raise ValueError("one plan per catalog")
    cats = (L.Catalog * n)()
    ress = (L.Result * n)()
    keep, arrays, meta = [], [], []
    for i, (p, c) in enumerate(zip(plans, catalogs)):
        flags = _flags(c.get("bulk_flow", False), c.get("no_shotnoise", False),
                       c.get("no_deconvolve", False))
        cat, k = make_catalog(c["pos"], c["vel"], c.get("weight"), box=c["box"], haf=c["haf"],
                              n_bins=c.get("n_bins", 32), k_edges=c.get("k_edges"), flags=flags)
        res, arr = make_result(cat.n_bins)
        cats[i] = cat
        ress[i] = res
        keep.append(k)
        arrays.append(arr)
        meta.append((c["box"], p.n_grid, c.get("k_edges"), cat.n_bins))
    handles = (C.c_void_p * n)(*[p.handle.value for p in plans])
    L.check(L.lib().mps_estimate_batch(handles, cats, ress, n, _stream(stream)), "mps_estimate_batch")
    return [unpack_result(ress[i], arrays[i], *meta[i]) for i in range(n)]


class Server:
    """Continuous-batching request server (mps_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 8,
                 small_particles: int = 4_000_000):
        h = C.c_void_p()
        L.check(L.lib().mps_server_create(C.byref(h), int(hbm_budget_bytes), int(max_inflight),
                                          int(small_particles)), "mps_server_create")
        self._h = h
        self._pending = {}

    def submit(self, pos, vel, weight=None, *, box, haf, n_grid, precision="f32", n_bins=32,
               k_edges=None, bulk_flow=False, no_shotnoise=False, no_deconvolve=False,
               stream=None) -> int:
        """Queue one catalog.  Its kernels start after the work already
        enqueued on `stream` (default: torch's current stream), the stream
        that produced the catalog."""
        cat, keep = make_catalog(pos, vel, weight, box=box, haf=haf, n_bins=n_bins,
                                 k_edges=k_edges,
                                 flags=_flags(bulk_flow, no_shotnoise, no_deconvolve))
        res, arrays = make_result(cat.n_bins)
        ticket = C.c_uint64()
        L.check(L.lib().mps_submit(self._h, C.byref(cat), int(n_grid), _prec(precision),
                                   C.byref(res), _stream(stream), C.byref(ticket)), "mps_submit")
        self._pending[ticket.value] = (res, arrays, keep, cat, box, n_grid, k_edges)
        return ticket.value

    def wait(self, ticket: int, timeout_s: float = 60.0):
        st = L.lib().mps_wait(self._h, C.c_uint64(ticket), float(timeout_s))
        if st == -6:
            raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")
        res, arrays, keep, cat, box, n_grid, k_edges = self._pending.pop(ticket)
        L.check(st, "mps_wait")
        return unpack_result(res, arrays, box, n_grid, k_edges, cat.n_bins)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            L.lib().mps_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
