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


def state_image_to_oracle(st: dict, k: int, W: int) -> dict:
    """The oracle's term list (Oracle.set_state) of a truncated-form state
    image (mbkk_get_state): the initial term of every center whose coefficient
    is not 0 (tag 0), then, oldest first, the part of each live batch
    l = max(1, i-W) .. i-1 (ring slot (l-1) mod W) assigned to it (tag l).
    For states of the window rule (tau = 0)."""
    i = int(st["iteration"])
    coef, off, sidx = st["coef"], st["slot_off"], st["slot_idx"]
    tc, tt, tw, tn, pts = [], [], [], [], []
    for j in range(k):
        if coef[j, 0] != 0.0:
            tc.append(j), tt.append(0), tw.append(coef[j, 0]), tn.append(1)
            pts.append(np.array([st["init_idx"][j]], np.int32))
        for l in range(max(1, i - W), i):
            r = (l - 1) % W
            seg = sidx[r, off[r][j]: off[r][j + 1]]
            if seg.size and coef[j, 1 + r] != 0.0:
                tc.append(j), tt.append(l), tw.append(coef[j, 1 + r]), tn.append(seg.size)
                pts.append(seg.astype(np.int32))
    return dict(iteration=i, term_center=np.array(tc, np.int32), term_tag=np.array(tt, np.int64),
                term_coef=np.array(tw, np.float64), term_npts=np.array(tn, np.int32),
                points=np.concatenate(pts) if pts else np.zeros(0, np.int32),
                cum=np.asarray(st["cum"], np.float64))
