"""Error metrics for comparing forces with the FP64 oracle.

(i)   max_i |dF_i| / |F_i|            raw per-atom relative error
(ii)  max_i |dF_i| / sum_j |f_ij|     normalised by the magnitude of the terms summed
(iii) |dF|_2 / |F|_2                  RMS relative error over all atoms
"""
import numpy as np


def force_errors(f_test, f_ref, abs_sum):
    f_test = np.asarray(f_test, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    d = np.linalg.norm(f_test - f_ref, axis=1)
    fr = np.linalg.norm(f_ref, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        raw = np.where(fr > 0, d / fr, np.where(d > 0, np.inf, 0.0))
        norm = np.where(abs_sum > 0, d / abs_sum, np.where(d > 0, np.inf, 0.0))
    rms = float(np.linalg.norm(f_test - f_ref) / max(np.linalg.norm(f_ref), 1e-300))
    return dict(max_raw=float(raw.max(initial=0.0)), max_norm=float(norm.max(initial=0.0)),
                rms=rms, n_raw_over_1e5=int((raw > 1e-5).sum()))
