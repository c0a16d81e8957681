"""Incremental finite differences of the re-render loss, in FP64 on the oracle
(test infrastructure).

    L(y1, o) = mean over every (view, pixel, channel) of
               (render(colorize(y1, o), o) - y2)^2

A full evaluation of L at the differentiation workload's size takes minutes,
so each entry's central difference is formed from what the perturbation
changes:

- target entry (row p, channel c): only the Gaussians seen at p change, by
  dc_g = (A_g + w_g Lambda)^{-1} w_gp phi_g e_c h; L is quadratic in y1, so
  the central difference is 2 <resid, render(dc)> / (n h) exactly (the
  squared terms cancel), over the rows those Gaussians cover;
- opacity entry g (t_min = 0, where every decision is smooth in o_g): the
  pixel weights change only at g's own pixels, where the walk is redone
  exactly for o_g +- h; the Gaussians seen there respond through their
  normal equations, dc = (A + w Lambda)^{-1} (dB - dA c) from those weight
  changes; the loss change is exact at g's pixels given dc, and elsewhere it
  is <G_out, dc> with G_out the render adjoint of the base point restricted
  to the other rows.  The terms left out are second order in h with the same
  sign for +h and -h, so they cancel in the central difference up to
  O(h^2).

Everything here is computed with oracle functions and numpy in FP64."""
from dataclasses import dataclass

import numpy as np

import oracle


def loss_and_parts(sc, y1, y2, opts, threads=None):
    """The base point: coefficients, normal equations, render, residual, the
    render adjoint of the loss and the oracle's adjoint gradients."""
    r = oracle.colorize(sc, y1, opts=opts, threads=threads)
    c = r["coeffs"]
    img = oracle.render(sc, c, opts=opts, threads=threads)
    y2d = oracle.decode_targets(y2).astype(np.float64)
    resid = img - y2d
    n = resid.size
    ibar = 2.0 * resid / n
    gc, go_r = oracle.render_backward(sc, c, ibar, opts=opts, threads=threads)
    gy, go_c = oracle.colorize_backward(sc, y1, c, gc, opts=opts, threads=threads)
    return Base(sc=sc, opts=opts, y1=oracle.decode_targets(y1).astype(np.float64), y2=y2d, c=c,
                A=r["A"], B=r["B"], w=r["w"], img=img, resid=resid, n=n, gc=gc,
                grad_y=gy, grad_o=go_r + go_c, loss=float((resid ** 2).mean()))


@dataclass
class Base:
    sc: object
    opts: object
    y1: np.ndarray
    y2: np.ndarray
    c: np.ndarray
    A: np.ndarray
    B: np.ndarray
    w: np.ndarray
    img: np.ndarray
    resid: np.ndarray
    n: int
    gc: np.ndarray
    grad_y: np.ndarray
    grad_o: np.ndarray
    loss: float


def _centres(sc):
    return np.stack([-c.R.astype(np.float64).T @ c.t.astype(np.float64) for c in sc.cams])


def _phi(sc, views, gs):
    """SH basis of the direction camera -> Gaussian for (view, Gaussian) pairs."""
    d = sc.means[gs].astype(np.float64) - _centres(sc)[views]
    return oracle.sh_basis(sc.sh_deg, d)


def fd_target(base: Base, row: int, ch: int, h: float = 1e-3, threads=None) -> float:
    sc = base.sc
    idx, w = oracle.contributions_rows(sc, np.array([row]), base.opts, threads)
    if idx.shape[0] == 0:
        return 0.0
    ph = _phi(sc, idx[:, 0], idx[:, 2])
    dc = np.zeros_like(base.c)
    for (j, r, g), wg, p in zip(idx, w, ph):
        rhs = np.zeros((sc.n_b, sc.C))
        rhs[:, ch] = wg * p * h
        dc[g] += np.linalg.solve(base.A[g], rhs)
    want = np.zeros(sc.N, np.uint8)
    want[np.unique(idx[:, 2])] = 1
    rows = oracle.wanted_rows(sc, want, base.opts)
    dimg = oracle.render_rows(sc, dc, rows, base.opts, threads)
    return float(2.0 * np.sum(base.resid[rows] * dimg) / (base.n * h))


def _walk(sc, rows, opts, threads):
    idx, w = oracle.contributions_rows(sc, rows, opts, threads)
    return idx, w


def _scatter_outer(n_g, gi, a, b, chunk=100_000):
    """out[g] = sum over entries e with gi[e] = g of outer(a[e], b[e]), as
    sparse (group x entry) products over chunks of entries."""
    import scipy.sparse as sp
    p, q = a.shape[1], b.shape[1]
    out = np.zeros((n_g, p * q))
    for s in range(0, gi.size, chunk):
        e = slice(s, s + chunk)
        k = gi[e].size
        S = sp.csr_matrix((np.ones(k), (gi[e], np.arange(k))), shape=(n_g, k))
        out += S @ (a[e][:, :, None] * b[e][:, None, :]).reshape(k, p * q)
    return out.reshape(n_g, p, q)


def _projections(base: Base):
    """Per view: visibility, centre and footprint half-widths of every
    Gaussian (sigma_cut times the projected standard deviations), cached."""
    if getattr(base, "_proj", None) is None:
        sc = base.sc
        cut = float(np.float32(base.opts.sigma_cut))
        base._proj = []
        for j in range(len(sc.cams)):
            P = oracle.project(sc, j, base.opts)
            base._proj.append((P[:, 0] > 0, P[:, 2], P[:, 3], cut * np.sqrt(np.maximum(P[:, 7], 0)),
                               cut * np.sqrt(np.maximum(P[:, 9], 0))))
    return base._proj


def _subscene(base: Base, rows):
    """The Gaussians whose footprint box reaches a pixel of `rows` in some
    view, as a scene of their own (ascending original indices, so depth ties
    keep their order), and those indices.  A pixel's walk over the sub-scene
    equals its walk over the whole scene."""
    import copy
    sc = base.sc
    keep = np.zeros(sc.N, bool)
    offs = sc.pixel_offsets()
    for j, cam in enumerate(sc.cams):
        off = int(offs[j])
        sel = rows[(rows >= off) & (rows < off + cam.width * cam.height)] - off
        if sel.size == 0:
            continue
        px, py = sel % cam.width + 0.5, sel // cam.width + 0.5
        vis, u, v, rx, ry = _projections(base)[j]
        cand = vis & (u + rx >= px.min()) & (u - rx <= px.max()) & (v + ry >= py.min()) & (v - ry <= py.max())
        keep |= cand
    ids = np.flatnonzero(keep)
    sub = copy.copy(sc)
    sub.means, sub.scales = sc.means[ids], sc.scales[ids]
    sub.quats, sub.opacities = sc.quats[ids], sc.opacities[ids].copy()
    return sub, ids


def fd_opacity(base: Base, g: int, h: float = 1e-3, threads=None) -> float:
    """Central difference of L in o_g (t_min = 0 options expected: then no
    decision depends on o_g and both walks list the same contributions)."""
    full = base.sc
    want = np.zeros(full.N, np.uint8)
    want[g] = 1
    rows = oracle.wanted_rows(full, want, base.opts)  # every pixel g may touch
    sc, ids = _subscene(base, rows)
    gs = int(np.searchsorted(ids, g))
    idx0, w0 = _walk(sc, rows, base.opts, threads)
    idx0[:, 2] = ids[idx0[:, 2]]  # back to the scene's Gaussian indices
    ph = _phi(full, idx0[:, 0], idx0[:, 2])
    ring, gi = np.unique(idx0[:, 2], return_inverse=True)
    pos = np.searchsorted(rows, idx0[:, 1])
    lam = oracle.expand_lambda(full.lam, full.sh_deg)
    # the base render at these rows from the walk, and the render adjoint's
    # share of these rows
    ibar = 2.0 * base.resid[rows] / base.n
    g_in = _scatter_outer(ring.size, gi, w0[:, None] * ph, ibar[pos])
    col0 = np.einsum("em,emc->ec", ph, base.c[idx0[:, 2]])  # each entry's colour
    deltas = []
    o_save = sc.opacities[gs]
    o_pm = [np.float32(float(o_save) + h), np.float32(float(o_save) - h)]  # binary32, as stored
    for o_new in o_pm:
        sc.opacities[gs] = o_new
        try:
            idx1, w1 = _walk(sc, rows, base.opts, threads)
        finally:
            sc.opacities[gs] = o_save
        idx1[:, 2] = ids[idx1[:, 2]]
        assert np.array_equal(idx0, idx1), "a decision moved with the opacity"
        dw = w1 - w0
        # the solve's response to first order: dc = A^{-1} (dB - dA c) with
        # dB - dA c = sum_e dw_e (phi_e (y_e - phi_e^T c)^T - Lambda c); its
        # second-order part has the same sign for +h and -h and cancels in
        # the central difference
        r = _scatter_outer(ring.size, gi, dw[:, None] * ph, base.y1[idx0[:, 1]] - col0)
        dw_g = np.zeros(ring.size)
        np.add.at(dw_g, gi, dw)
        r -= dw_g[:, None, None] * lam[None, :, None] * base.c[ring]
        dcr = np.linalg.solve(base.A[ring], r)
        c1r = base.c[ring] + dcr
        # the render's change at these rows, formed directly (no difference
        # of two large sums): d = sum_e (w1 col1 - w0 col0)
        d = np.zeros((rows.size, full.C))
        np.add.at(d, pos, w1[:, None] * np.einsum("em,emc->ec", ph, c1r[gi]) - w0[:, None] * col0)
        inside = float(np.sum(d * (d + 2.0 * base.resid[rows]))) / base.n
        outside = float(np.sum((base.gc[ring] - g_in) * dcr))
        deltas.append(inside + outside)
    # the actual step between the two binary32 opacities, not 2 h
    return (deltas[0] - deltas[1]) / (float(o_pm[0]) - float(o_pm[1]))
