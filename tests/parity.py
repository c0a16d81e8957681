"""Comparison helpers for GPU-vs-oracle parity tests.

Error metric per Gaussian g (all (L+1)^2 x C coefficients):
    e_g = ||c_gpu - c_ref||_F / max(||c_ref||_F, tau),  tau = 1e-3 * median ||c_ref||
Gate: e_g <= TOL_F32 for every observed Gaussian whose decisions are not in
doubt.  Pixel decisions (footprint edge, alpha floor, transmittance stop)
that fall within rounding of their threshold may legitimately go either way
in the FP32 kernel and the FP64 oracle; then several results are correct.
The oracle bounds, per Gaussian, the coefficient change such decisions could
cause (`flip`, first order); a Gaussian is excluded from the element-wise
gate ("flagged") when that bound exceeds FLIP_SHARE of the tolerance.
Contribution counts: each near-threshold decision changes the count by at
most one, so |count_gpu - count_oracle| <= events.
"""
import numpy as np

TOL_F32 = 1e-4
FLIP_SHARE = 0.5


def to_device_targets(y):
    import torch
    if y.dtype == np.uint16:
        return torch.from_numpy(y.view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()


def rel_errors(c_gpu, ref):
    N = c_gpu.shape[0]
    nrm = np.linalg.norm(ref["coeffs"].reshape(N, -1), axis=1)
    obs = (ref["status"] & 1) == 0
    tau = 1e-3 * np.median(nrm[obs]) if obs.any() else 1.0
    e = np.linalg.norm((c_gpu.astype(np.float64) - ref["coeffs"]).reshape(N, -1), axis=1) / np.maximum(nrm, tau)
    return e, obs


def flagged(ref, tol=TOL_F32):
    N = ref["coeffs"].shape[0]
    nrm = np.linalg.norm(ref["coeffs"].reshape(N, -1), axis=1)
    obs = (ref["status"] & 1) == 0
    tau = 1e-3 * np.median(nrm[obs]) if obs.any() else 1.0
    return ref["flip"] > FLIP_SHARE * tol * np.maximum(nrm, tau)


def summary(e, sel):
    if not sel.any():
        return "none compared"
    v = e[sel]
    return "n=%d p50=%.2e p99=%.2e max=%.2e" % (v.size, np.median(v), np.percentile(v, 99), v.max())


def check_colorize(c_gpu, st_gpu, ref, want=None, tol=TOL_F32, count_gpu=None, label=""):
    e, obs = rel_errors(c_gpu, ref)
    fl = flagged(ref)
    sel = obs & ~fl
    if want is not None:
        sel &= want.astype(bool)
    msg = f"{label}: compared {summary(e, sel)}; flagged {int((obs & fl).sum())} ({summary(e, obs & fl)})"
    assert sel.sum() > 0, msg
    assert e[sel].max() <= tol, msg
    # unobserved Gaussians are reported as such with zero coefficients
    un_ref = (ref["status"] & 1) == 1
    un_gpu = (st_gpu & 1) == 1
    chk = ~fl if want is None else (~fl & want.astype(bool))
    assert np.array_equal(un_ref[chk], un_gpu[chk]), msg + " (unobserved sets differ)"
    assert np.all(c_gpu[un_gpu] == 0), msg
    if count_gpu is not None:
        assert abs(int(count_gpu) - ref["count"]) <= max(ref["events"], 0), \
            msg + f" (count gpu {count_gpu} oracle {ref['count']} events {ref['events']})"
    return msg
