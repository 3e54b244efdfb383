"""Self-consistency model of the library's monopole acceptance.

NOT AN ORACLE.  This restates, in FP64 numpy, the acceptance decisions the
library's list builder takes: 64-particle target blocks cut at 2 r_cut
extent, source nodes of every level of the hierarchy over the leaves
(single leaves, groups of 8 consecutive leaves, and up), and the same FP64
operation sequence for the geometric and relative tests.  It is used only to check that the library takes the
decisions it is designed to take (the (target, monopole) pair counts match
exactly); the accuracy of the monopole forces is checked against the exact
pair sum and the octree dual tree traversal of oracle/tree.py instead.

The model, in the library's order:

* particles in Peano-Hilbert order with the octree leaves (maximal nodes
  with at most leaf_max particles);
* target blocks: runs of at most 64 consecutive particles, cut where their
  integer box would grow wider than 2 r_cut;
* source nodes: the hierarchy over the leaves in which a node of level h
  groups 8 consecutive nodes of level h - 1, each with its integer bounding
  box, mass and centre of mass;
* per target block A and periodic image s, walk the source hierarchy from
  the root: a node whose box lies at r_cut or more from A's box is skipped;
  a node of any level is taken as a monopole when every enabled test
  holds: (A + B) / R <= theta (A, B the longest box sides, R the distance of
  the box centres) and G M B^2 / r^4 <= alpha |a| (M the node mass, r the gap
  between the two boxes, |a| the smallest reference acceleration among A's
  targets); other nodes are opened; leaves reached this way are summed
  particle by particle;
* a monopole acts on every target of A as a particle of the node's mass at
  its centre of mass: the same softened, split, cut pair force.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc

from oracle import hilbert_keys, sort_order, leaves, leaf_boxes, quantise


def _split(x):
    return erfc(x) + 2.0 * x / np.sqrt(np.pi) * np.exp(-x * x)


def _blocks(q, n, emax):
    """Target nodes: (start, count, lo[3], hi[3]) in key order."""
    out = []
    for k0 in range(0, n, 64):
        k1 = min(k0 + 64, n)
        qs = q[:, k0:k1].astype(np.int64)
        lo, hi = qs.min(1), qs.max(1) + 1
        if np.all(hi - lo <= emax):
            out.append((k0, k1 - k0, lo, hi))
            continue
        start = k0
        blo, bhi = qs[:, 0].copy(), qs[:, 0] + 1
        for kk in range(k0 + 1, k1):
            qq = qs[:, kk - k0]
            ulo, uhi = np.minimum(blo, qq), np.maximum(bhi, qq + 1)
            if np.any(uhi - ulo > emax):
                out.append((start, kk - start, blo, bhi))
                start, blo, bhi = kk, qq.copy(), qq + 1
            else:
                blo, bhi = ulo, uhi
        out.append((start, k1 - start, blo, bhi))
    return out


def _gap2(alo, ahi, blo, bhi, s, W):
    sh = np.asarray(s, dtype=np.int64) * W
    g = np.maximum(np.maximum(blo + sh - ahi, alo - bhi - sh), 0)
    return int((g * g).sum())


def _accept(alo, ahi, blo, bhi, s, W, theta, rel=None):
    """The enabled acceptance tests, each squared so that it is a fixed
    sequence of FP64 operations on integers and the given masses: the
    geometric one as (2 (A + B))^2 <= theta^2 (2 R)^2 in half cells, the
    relative one as (G M (B cell)^2)^2 <= alpha^2 |a|^2 (r cell)^8.
    rel = (G, M, cell, alpha, |a|^2) or None."""
    A = int((ahi - alo).max())
    B = int((bhi - blo).max())
    if theta > 0:
        D = (blo + bhi + 2 * np.asarray(s, dtype=np.int64) * W) - (alo + ahi)
        R2x4 = int((D * D).sum())
        lhs = float(2 * (A + B)) ** 2
        if not lhs <= (theta * theta) * float(R2x4):
            return False
    if rel is not None:
        G, M, cell, alpha, a2 = rel
        bc = float(B) * cell
        lhs = ((G * M) * bc) * bc
        g2 = (float(_gap2(alo, ahi, blo, bhi, s, W)) * cell) * cell
        if not lhs * lhs <= ((alpha * alpha) * a2) * ((g2 * g2) * (g2 * g2)):
            return False
    return True


def _seq_sum(v):
    """Sum in index order (the order of the node moments' definition)."""
    return np.cumsum(v, axis=0)[-1]


def monopole_accel(pos, mass, params, theta, min_level=0, alpha=0.0, acc_ref=None):
    """Accelerations [3][n] (input order) with monopole acceptance, and the
    number of (target, monopole) and (target, source particle) pairs taken.
    theta: the geometric test (0: off); alpha > 0 adds the relative test
    against acc_ref [3][n] (input order)."""
    p = params
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    n = pos.shape[1]
    L, bits = p.L, p.key_bits
    W = 1 << bits
    T = int(np.ceil((p.rcut * W / L) ** 2))
    emax = int(np.floor(2.0 * p.rcut * W / L))
    keys = hilbert_keys(pos, L, bits)
    order = sort_order(keys)
    sk = keys[order]
    wpos = np.mod(pos, L)[:, order]
    m_s = mass[order]
    q = quantise(pos[:, order], L, bits)
    lv = leaves(sk, bits, p.leaf_max)
    llo, lhi = leaf_boxes(q, lv)
    lbeg, lcnt = lv["begin"], lv["count"]
    nleaf = lbeg.size
    # the source hierarchy
    cnt = [nleaf]
    while cnt[-1] > 1:
        cnt.append((cnt[-1] + 7) // 8)
    boxes_lo, boxes_hi, nmass, ncom = [llo.T.copy()], [lhi.T.copy()], [], []
    lm = np.array([_seq_sum(m_s[b:b + c]) for b, c in zip(lbeg, lcnt)])
    lx = np.array([(m_s[b:b + c] * wpos[:, b:b + c]).sum(1) for b, c in zip(lbeg, lcnt)]).reshape(-1, 3)
    nmass.append(lm)
    ncom.append(lx)                      # sum of m x for now
    for h in range(1, len(cnt)):
        lo = np.empty((cnt[h], 3), dtype=np.int64)
        hi = np.empty((cnt[h], 3), dtype=np.int64)
        mm = np.empty(cnt[h])
        mx = np.empty((cnt[h], 3))
        for i in range(cnt[h]):
            a, b = 8 * i, min(8 * i + 8, cnt[h - 1])
            lo[i] = boxes_lo[h - 1][a:b].min(0)
            hi[i] = boxes_hi[h - 1][a:b].max(0)
            mm[i] = _seq_sum(nmass[h - 1][a:b])
            mx[i] = ncom[h - 1][a:b].sum(0)
        boxes_lo.append(lo)
        boxes_hi.append(hi)
        nmass.append(mm)
        ncom.append(mx)
    com = [mx / np.where(mm > 0, mm, 1.0)[:, None] for mm, mx in zip(nmass, ncom)]
    top = len(cnt) - 1
    shifts = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    acc_s = np.zeros((3, n))
    n_mono = 0
    n_pp = 0
    ell2 = p.eps * p.eps
    if alpha > 0:
        ar = np.asarray(acc_ref, dtype=np.float64)[:, order]
        amag2 = (ar[0] * ar[0] + ar[1] * ar[1]) + ar[2] * ar[2]
    cell = L / float(W)
    for start, count, alo, ahi in _blocks(q, n, emax):
        mono, ppl = [], []
        a2 = float(amag2[start:start + count].min()) if alpha > 0 else 0.0

        def visit(h, i, s):
            rel = (p.G, float(nmass[h][i]), cell, alpha, a2) if alpha > 0 else None
            if h >= min_level and (theta > 0 or alpha > 0) and \
                    _accept(alo, ahi, boxes_lo[h][i], boxes_hi[h][i], s, W, theta, rel):
                mono.append((h, i, s))
                return
            if h == 0:
                ppl.append((i, s))
                return
            for c in range(8 * i, min(8 * i + 8, cnt[h - 1])):
                if _gap2(alo, ahi, boxes_lo[h - 1][c], boxes_hi[h - 1][c], s, W) < T:
                    visit(h - 1, c, s)

        for s in shifts:
            if _gap2(alo, ahi, boxes_lo[top][0], boxes_hi[top][0], s, W) < T:
                visit(top, 0, s)
        xi = wpos[:, start:start + count]                        # [3, t]
        src, sm = [], []
        for leaf, s in ppl:
            b, c = lbeg[leaf], lcnt[leaf]
            src.append(wpos[:, b:b + c] + L * np.array(s, dtype=np.float64)[:, None])
            sm.append(m_s[b:b + c])
        for h, i, s in mono:
            src.append(com[h][i][:, None] + L * np.array(s, dtype=np.float64)[:, None])
            sm.append(np.array([nmass[h][i]]))
        if not src:
            continue
        xs = np.concatenate(src, axis=1)                         # [3, S]
        ms = np.concatenate(sm)
        d = xs[:, None, :] - xi[:, :, None]                      # [3, t, S]
        s2 = (d * d).sum(0)
        keep = (s2 < p.rcut * p.rcut) & (s2 > 0)
        se2 = s2 + ell2
        se = np.sqrt(np.where(keep, se2, 1.0))
        f = np.where(keep, p.G * ms[None, :] * _split(se / (2 * p.rs)) / (se2 * se), 0.0)
        acc_s[:, start:start + count] = (f[None] * d).sum(2)
        n_mono += count * len(mono)
        n_pp += int(keep[:, :-len(mono) or None].sum()) if mono else int(keep.sum())
    acc = np.zeros((3, n))
    acc[:, order] = acc_s
    return {"acc": acc, "n_mono_pairs": n_mono, "n_pp_pairs": n_pp}
