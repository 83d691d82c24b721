"""Comparison of GPU fields against the oracle (test infrastructure).

Error measure: err_d(p) = |f_gpu - f_oracle| / S_d with S_d the range of the
input values of attribute d.  Nodes are compared where both sides are
determined and agree on the accepted degree; the "pass set" further requires
the oracle's smallest equilibrated pivot d_min >= 1e-3.
"""
from __future__ import annotations

import numpy as np


def compare(gpu_fields, gpu_deg, or_fields, or_deg, or_dmin, values, dmin_pass=1e-3):
    """Flattened per-node comparison.  gpu_fields/or_fields: (D, P)."""
    vals = np.asarray(values, dtype=np.float64)
    S = vals.max(axis=0) - vals.min(axis=0)
    S = np.where(S > 0, S, 1.0)
    gf = np.asarray(gpu_fields, dtype=np.float64)
    of = np.asarray(or_fields, dtype=np.float64)
    gd = np.asarray(gpu_deg).ravel()
    od = np.asarray(or_deg).ravel()
    dm = np.asarray(or_dmin).ravel()
    both = (gd == od) & (od != 255)
    passset = both & (dm >= dmin_pass)
    err = np.abs(gf - of) / S[:, None]
    out = {
        "nodes": int(od.size),
        "degree_mismatch": int(np.sum(gd != od)),
        "nan_mismatch": int(np.sum((gd == 255) != (od == 255))),
        "same_degree": int(both.sum()),
        "pass_set": int(passset.sum()),
        "max_err_pass": float(err[:, passset].max()) if passset.any() else 0.0,
        "rms_err_pass": float(np.sqrt(np.mean(err[:, passset] ** 2))) if passset.any() else 0.0,
        "max_err_same_degree": float(err[:, both].max()) if both.any() else 0.0,
        "per_field_max_pass": (err[:, passset].max(axis=1).tolist() if passset.any()
                               else [0.0] * gf.shape[0]),
    }
    # same-degree nodes by the oracle's smallest equilibrated pivot
    bins = {}
    for name, lo, hi in (("dmin>=1e-2", 1e-2, np.inf), ("1e-3<=dmin<1e-2", 1e-3, 1e-2),
                         ("1e-5<=dmin<1e-3", 1e-5, 1e-3), ("dmin<1e-5", -np.inf, 1e-5)):
        sel = both & (dm >= lo) & (dm < hi)
        bins[name] = {"nodes": int(sel.sum()),
                      "max": float(err[:, sel].max()) if sel.any() else 0.0,
                      "rms": float(np.sqrt(np.mean(err[:, sel] ** 2))) if sel.any() else 0.0}
    out["bins"] = bins
    # the conditioning-scaled error err * d_min^2 over same-degree nodes with
    # 1e-3 <= d_min < 1e-2 (where the amplified float32 sums dominate every
    # other error source), and the largest oracle d_min among degree
    # mismatches
    sel = both & (dm >= 1e-3) & (dm < 1e-2)
    out["max_err_dmin2"] = float((err[:, sel] * dm[sel] ** 2).max()) if sel.any() else 0.0
    mis = (gd != od) & (od != 255) & (gd != 255)
    out["mismatch_dmin_max"] = float(dm[mis].max()) if mis.any() else 0.0
    # NaN exactly where undetermined
    und = gd == 255
    out["nan_ok"] = bool(np.all(np.isnan(gf[:, und])) and np.all(np.isfinite(gf[:, ~und])))
    return out
