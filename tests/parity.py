"""Comparison helpers for GPU-vs-oracle parity tests.

Error metric per Gaussian g (all (L+1)^2 x C coefficients):
    e_g = ||c_gpu - c_ref||_F / max(||c_ref||_F, tau),  tau = 1e-3 * median ||c_ref||

Pixel decisions (footprint edge, alpha floor, transmittance stop) that fall
within the binary32 evaluation error of their threshold may legitimately go
either way in the FP32 kernel and the FP64 oracle; then several results are
correct.  The oracle records every such decision and bounds, per Gaussian,
the coefficient change they can cause (`flip`, pinned in
tests/test_oracle_events.py).  The gate therefore holds for EVERY observed
Gaussian:
    e_g <= tol + flip_g / max(||c_ref||_F, tau)
Gaussians whose bound exceeds half the tolerance are reported as flagged.

Integer results are compared exactly where no decision is in doubt: a
Gaussian's contribution count equals the oracle's when the oracle recorded no
near-threshold decision on its own acceptance (ndec_g = 0) and differs by at
most ndec_g otherwise; the unobserved sets agree wherever ndec_g = 0.
"""
import numpy as np

TOL_F32 = 1e-4
FLAG_SHARE = 0.5


def to_device_targets(y):
    import torch
    if y.dtype == np.uint16:
        return torch.from_numpy(y.view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()


def norms(ref):
    N = ref["coeffs"].shape[0]
    nrm = np.linalg.norm(ref["coeffs"].reshape(N, -1), axis=1)
    obs = (ref["status"] & 1) == 0
    tau = 1e-3 * np.median(nrm[obs]) if obs.any() else 1.0
    return np.maximum(nrm, tau), obs


def rel_errors(c_gpu, ref):
    N = c_gpu.shape[0]
    scale, obs = norms(ref)
    e = np.linalg.norm((c_gpu.astype(np.float64) - ref["coeffs"]).reshape(N, -1), axis=1) / scale
    return e, obs


def bound(ref):
    """Per Gaussian, the part of the gate the near-threshold decisions allow
    (flip / max(||c||, tau)); infinite where the decisions leave it open."""
    scale, _ = norms(ref)
    return ref["flip"] / scale


def flagged(ref, tol=TOL_F32):
    return bound(ref) > FLAG_SHARE * tol


def summary(e, sel):
    if not sel.any():
        return "none"
    v = e[sel]
    return "n=%d p50=%.2e p99=%.2e max=%.2e" % (v.size, np.median(v), np.percentile(v, 99), v.max())


def check_colorize(c_gpu, st_gpu, ref, want=None, tol=TOL_F32, count_gpu=None, cnt_gpu=None,
                   label="", max_flagged=None):
    """Gate one GPU colorize result against the oracle's (see module doc).
    count_gpu: total accepted contributions; cnt_gpu: per-Gaussian counts
    (only meaningful for calls on the whole scene, want=None).
    max_flagged: if given, the largest allowed fraction of flagged Gaussians."""
    e, obs = rel_errors(c_gpu, ref)
    b = bound(ref)
    fl = b > FLAG_SHARE * tol
    sel = obs.copy()
    if want is not None:
        sel &= want.astype(bool)
    nfl = int((sel & fl).sum())
    over = e - tol
    # how much of its bound a flagged Gaussian used
    used = np.where(sel & fl & (over > 0) & np.isfinite(b), over / np.where(b > 0, b, 1), 0.0)
    msg = (f"{label}: {summary(e, sel & ~fl)}; flagged {nfl} ({100.0 * nfl / max(1, int(sel.sum())):.2f}%: "
           f"{summary(e, sel & fl)}, bound used at most {used.max() if used.size else 0:.2f}, "
           f"open {int((sel & ~np.isfinite(b)).sum())})")
    assert sel.sum() > 0, msg
    worst = np.flatnonzero(sel & ~(e <= tol + b))
    assert worst.size == 0, msg + f" | outside the gate: g={worst[:5]} e={e[worst[:5]]} bound={b[worst[:5]]}"
    if max_flagged is not None:
        assert nfl <= max_flagged * sel.sum(), msg + " (too many flagged)"
    sure = ref["ndec"] == 0
    if want is not None:
        sure = sure & want.astype(bool)
    # unobserved Gaussians are reported as such, with zero coefficients
    un_ref = (ref["status"] & 1) == 1
    un_gpu = (st_gpu & 1) == 1
    assert np.array_equal(un_ref[sure], un_gpu[sure]), msg + " (unobserved sets differ)"
    assert np.all(c_gpu[un_gpu] == 0), msg
    if cnt_gpu is not None:
        assert want is None, "per-Gaussian counts are compared on whole-scene calls"
        d = np.abs(np.asarray(cnt_gpu, np.int64) - ref["cnt"])
        bad = np.flatnonzero(d > ref["ndec"])
        assert bad.size == 0, msg + f" (counts differ beyond the decisions: g={bad[:5]} d={d[bad[:5]]})"
        msg += f"; counts exact on {int(sure.sum())}, differ on {int((d > 0).sum())}"
    if count_gpu is not None:
        assert abs(int(count_gpu) - ref["count"]) <= max(ref["events"], 0), \
            msg + f" (count gpu {count_gpu} oracle {ref['count']} decisions {ref['events']})"
    return msg


def check_render(img_gpu, img_ref, pix_bound, tol_abs=1e-5, label=""):
    """Every pixel within tol_abs (+ the oracle's bound where a near-threshold
    decision may change it), element by element."""
    err = np.abs(np.asarray(img_gpu, np.float64) - img_ref).max(axis=1)
    over = np.flatnonzero(~(err <= tol_abs + pix_bound))
    msg = (f"{label}: max err {err.max():.2e} (median {np.median(err):.1e}); pixels with a bound "
           f"{int((pix_bound > 0).sum())}, max err among them {err[pix_bound > 0].max() if (pix_bound > 0).any() else 0:.2e}")
    assert over.size == 0, msg + f" | outside: rows {over[:5]} err {err[over[:5]]} bound {pix_bound[over[:5]]}"
    return msg


# Binary32 per-view sums.  The GPU forms each view's sums V_gj = sum_p w and
# S_gj = sum_p w y_p in binary32 (binary32 pixel weights, each pixel's band
# sum, the wave's reduction, then one addition per tile in any order) and
# folds them in FP64.  If every V_gj carries a relative error of at most eps,
# then every term V_gj (phi phi^T + Lambda) of M = A + w Lambda is scaled by a
# factor in [1 - eps, 1 + eps], so the perturbed matrix satisfies
#   (1 - eps) M <= M~ <= (1 + eps) M          (Loewner order),
# and each S_gj[c] moves by at most eps V_gj Y_c (Y_c = max |y_c|).  With
# X = [sqrt(V_gj) phi_gj] (X X^T = A <= M), |M^{-1/2} dB[:, c]| <=
# eps Y_c sqrt(w_g).  Hence, in the norm |x|_M = sqrt(x^T M x) (summed over
# channels),
#   |c~ - c|_M <= eps (|c|_M + sqrt(w_g) |Y|) / (1 - eps),
# and |x| <= |x|_M / sqrt(lambda_min(M)):  the error grows with sqrt(kappa),
# not with kappa.
#   eps = werr_g (the oracle's bound on the binary32 weights, margin model)
#       + SUM_DEPTH * 2^-24 (the summation: 4 band terms, 6 reduction levels
#         and up to 64 tile additions of one Gaussian in one view).
SUM_DEPTH = 74


def fp32_sum_bound(ref, Y, sum_depth=SUM_DEPTH):
    """Per Gaussian, the bound above divided by max(|c_ref|, tau) (the e_g
    scale); zero for unobserved Gaussians."""
    A = ref["A"]
    c = ref["coeffs"]
    scale, obs = norms(ref)
    N = c.shape[0]
    out = np.zeros(N)
    Yn = float(np.linalg.norm(np.asarray(Y, np.float64)))
    for g in np.flatnonzero(obs):
        eps = ref["werr"][g] + sum_depth * 2.0 ** -24
        lmin = np.linalg.eigvalsh(A[g])[0]
        if not lmin > 0:
            out[g] = np.inf
            continue
        cM = np.sqrt(max(0.0, float(np.einsum("mc,mn,nc->", c[g], A[g], c[g]))))
        out[g] = eps * (cM + np.sqrt(ref["w"][g]) * Yn) / ((1 - eps) * np.sqrt(lmin)) / scale[g]
    return out
