#!/usr/bin/env python3
"""Write the oracle's reference spectra of the two large synthetic workloads
to tests/golden/ (calls only oracle/ and synth/; CPU, FP64).

* zeldovich256_rms3.json: a 256^3 Zel'dovich lattice (rms displacement
  3 Mpc/h, L = 1000 Mpc/h, Haf = 50) on a 256^3 grid, the bulk-flow study of
  Sec. 3.1: the catalog as generated (its bulk flow is ~0) and with the
  artificial 51.5 km/s bulk flow of the Fig. 3 experiment added along
  (1, 2, 2)/3, each with bulk-flow removal off and on.
* zeldovich512_rms8.json: the benchmark workload, a 512^3 Zel'dovich lattice
  (rms 8 Mpc/h) on a 512^3 grid (the precision study: FP32 and FP64 grids
  against these values).

Every file records its catalog's fingerprint (SHA-256 of the float32
positions then velocities, the FP64 velocity moments and mean position) so
that a consumer can check it regenerated the same catalog.

Usage: python tests/golden/make_reference_spectra.py [256] [512]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import large  # noqa: E402
from synth import catalogs  # noqa: E402

BOX, HAF = 1000.0, 50.0
WORKERS = min(6, os.cpu_count() or 1)   # processes for the assignment's chunks


def fingerprint(pos, vel):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pos, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(vel, dtype=np.float32).tobytes())
    m = oracle.moments(vel, np.ones(pos.shape[0]))
    return {"sha256": h.hexdigest(), "n_particles": int(pos.shape[0]),
            "W": m["W"], "sum_v": m["sv"].tolist(), "sum_vv": m["s2vv"].ravel().tolist(),
            "mean_pos": np.mean(pos.astype(np.float64), axis=0).tolist()}


def spectra_json(r):
    nan = lambda a: [None if not np.isfinite(x) else float(x) for x in a]
    return {"k_edges": r.k_edges.tolist(), "n_modes": r.n_modes.tolist(), "k_mean": nan(r.k_mean),
            "p_pp": nan(r.p_pp), "p_tt": nan(r.p_tt), "p_dt": nan(r.p_dt), "p_dd": nan(r.p_dd),
            "sn_pp": nan(r.sn_pp), "sn_tt": nan(r.sn_tt), "sn_dd": nan(r.sn_dd),
            "v_bulk": r.v_bulk.tolist(), "sigma_v2": r.sigma_v2, "n_eff": r.n_eff}


def run(n_lat, rms, variants, out_name, where):
    t0 = time.perf_counter()
    pos, vel = catalogs.zeldovich(n_lat, BOX, rms, haf=HAF, seed=catalogs.seed_for(2 if n_lat == 256 else 3))
    doc = {"where": where,
           "catalog": {"generator": "synth.catalogs.zeldovich", "n_lattice": n_lat, "box": BOX, "rms_disp": rms,
                       "haf": HAF, "seed": catalogs.seed_for(2 if n_lat == 256 else 3)},
           "estimate": {"n_grid": n_lat, "n_bins": 32, "kernel": "bl3", "haf": HAF},
           "variants": {}}
    for name, added, flags in variants:
        v = vel if added is None else (vel.astype(np.float64) + catalogs.bulk_vector(added)).astype(np.float32)
        print(f"{out_name} {name}: estimating", flush=True)
        t1 = time.perf_counter()
        r = large.estimate_large(pos, v, box=BOX, n_grid=n_lat, haf=HAF, n_bins=32, flags=flags,
                                 workers=WORKERS)
        print(f"  {time.perf_counter() - t1:.0f} s", flush=True)
        doc["variants"][name] = {"added_bulk_flow_km_s": added, "bulk_flow_subtract": bool(flags & 1),
                                 "fingerprint": fingerprint(pos, v), "spectra": spectra_json(r)}
    with open(os.path.join(HERE, out_name), "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {out_name} in {time.perf_counter() - t0:.0f} s", flush=True)


def main():
    which = sys.argv[1:] or ["256", "512"]
    if "256" in which:
        run(256, 3.0, [("as_generated", None, 0), ("as_generated_bulk_removed", None, 1),
                       ("vb51.5", 51.5, 0), ("vb51.5_bulk_removed", 51.5, 1)],
            "zeldovich256_rms3.json",
            "Sec. 3.1 (bulk flow and its removal, p' = p - (1 + delta) v_b) with the artificial 51.5 km/s "
            "bulk flow of the Fig. 3 experiment; oracle reference spectra of a synthetic catalog")
    if "512" in which:
        run(512, 8.0, [("as_generated", None, 0)], "zeldovich512_rms8.json",
            "the precision study of the FP32 and FP64 grids on the benchmark workload; oracle reference "
            "spectra of a synthetic catalog")


if __name__ == "__main__":
    main()
