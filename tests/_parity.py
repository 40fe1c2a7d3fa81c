"""Helpers shared by the GPU parity tests: oracle-state conversion and the
error metrics.  Test infrastructure only."""
from __future__ import annotations

import numpy as np


def oracle_state_to_gpu(ostate: dict, init_idx, k: int, W: int, b_max: int) -> dict:
    """Ring-slot image (include/mbkk.h, mbkk_state) of the oracle's centers.

    The oracle keeps every center as a list of terms (tag 0: initial point,
    tag l >= 1: the points of batch B_l assigned to it).  Batch l lives in
    ring slot (l-1) mod W, its points grouped by center in center order and in
    batch order within a center, with per-(center, slot) coefficients."""
    coef = np.zeros((k, W + 1))
    slot_b = np.zeros(W, np.int32)
    slot_idx = np.zeros((W, b_max), np.int32)
    slot_off = np.zeros((W, k + 1), np.int32)
    init = np.asarray(init_idx, np.int32).copy()
    per_tag: dict = {}
    pos = 0
    for c, tag, w, npts in zip(ostate["term_center"], ostate["term_tag"], ostate["term_coef"],
                               ostate["term_npts"]):
        pts = ostate["points"][pos: pos + npts]
        pos += npts
        if tag == 0:
            assert npts == 1, "initial terms are single points"
            init[c] = pts[0]
            coef[c, 0] = w
        else:
            per_tag.setdefault(int(tag), []).append((int(c), pts, float(w)))
    for tag, lst in per_tag.items():
        r = (tag - 1) % W
        lst.sort(key=lambda e: e[0])
        counts = np.zeros(k, np.int64)
        allpts = []
        for c, pts, w in lst:
            counts[c] = len(pts)
            allpts.extend(pts.tolist())
            coef[c, 1 + r] = w
        slot_b[r] = len(allpts)
        slot_idx[r, : len(allpts)] = allpts
        slot_off[r, 1:] = np.cumsum(counts)
    return dict(iteration=ostate["iteration"], init_idx=init, slot_b=slot_b, slot_idx=slot_idx,
                slot_off=slot_off, coef=coef, cum=np.asarray(ostate["cum"], np.float64).copy())


def dist_rel_err(D_gpu: np.ndarray, D_ref: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """Error of a distance computed by the expansion K(x,x) - 2P + N, relative
    to the size of its terms: |D_gpu - D| / max(|D|, K(x,x) + N_j).

    The expansion cancels when x lies near a center, so any finite-precision
    evaluation has an absolute error of a few ulps of its largest term (P, N
    and K(x,x) are all O(K(x,x) + N_j) by Cauchy-Schwarz); dividing by D
    itself would demand accuracy below one ulp of those terms near D = 0."""
    den = np.maximum(np.abs(D_ref), scale)
    return np.abs(D_gpu - D_ref) / den


def dist_rel_err_floor(D_gpu: np.ndarray, D_ref: np.ndarray, scale: np.ndarray,
                       floor: float = 1e-3) -> np.ndarray:
    """Plain relative error with a floor (reported, not gated)."""
    den = np.maximum(np.abs(D_ref), floor * scale)
    return np.abs(D_gpu - D_ref) / den


def agreement(lab_gpu, lab_ref, margin_ref, min_margin):
    lab_gpu = np.asarray(lab_gpu)
    lab_ref = np.asarray(lab_ref)
    sel = np.asarray(margin_ref) >= min_margin
    return dict(all=float((lab_gpu == lab_ref).mean()),
                on_margin=bool((lab_gpu[sel] == lab_ref[sel]).all()),
                n_margin=int(sel.sum()), mismatches=np.nonzero(lab_gpu != lab_ref)[0])


def oracle_from_gpu_state(orc, st, k, window):
    """Loads a truncated-form state image (mbkk_get_state) into the oracle as
    explicit centers: every live term of every center, one entry per point."""
    coef, off, sidx = st["coef"], st["slot_off"], st["slot_idx"]
    cen, pts, wts = [], [], []
    j0 = np.flatnonzero(coef[:, 0] != 0.0)
    cen.append(j0)
    pts.append(st["init_idx"][j0])
    wts.append(coef[j0, 0])
    for r in range(window):
        cnt = np.diff(off[r])
        cj = np.repeat(np.arange(k), cnt)
        keep = coef[cj, 1 + r] != 0.0
        cen.append(cj[keep])
        pts.append(sidx[r, : off[r][-1]][keep])
        wts.append(coef[cj[keep], 1 + r])
    orc.set_centers(np.concatenate(cen), np.concatenate(pts), np.concatenate(wts))
    return int(sum(len(p) for p in pts))
