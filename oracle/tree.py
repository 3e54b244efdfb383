"""FP64 CPU oracle: the short-range force by the dual tree traversal of
sec. 3.3, with monopole (1-to-N) acceptance.

TEST INFRASTRUCTURE ONLY: only the tests may import this module.  It shares
no code with the HIP library and never imports it.  It builds its own tree
from the oracle's keys, sort order and cells (oracle/__init__.py); the
library's blocks, node groups and operation order appear nowhere here.

Tree (sec. 3.2): the oct-tree over the particles sorted along the
Peano-Hilbert curve.  The node of level l that holds particle k is the set of
particles whose keys share the top 3 l bits with k's key: a contiguous run
of the sorted particles, occupying the aligned cube of side L / 2^l (in grid
cells: side 2^(b - l), lower corner = any of its cells with the low b - l
bits cleared).  A node is a leaf (sec. 3.3, "a package of a given number of
particles") when it holds at most leaf_max particles or lies at the finest
level; otherwise its children are its non-empty octants.  Every node carries
its mass M (the sum of its particles' masses) and its centre of mass.

Traversal (sec. 3.3), with the policy the paper takes on MIC: the target node
is kept and the other node is opened.  Each target leaf A is walked against
the source tree from the root, once per periodic image sigma of the sources
(shift sigma L, sigma in {-1, 0, 1}^3):

* a source node B whose shifted cube lies at r_cut or more from A's cube is
  skipped: the short-range force vanishes there (sec. 3.1);
* B is accepted when every enabled test holds:
    - geometric (theta > 0): the two opening angles of sec. 3.3,
        theta1 = (B + A) / R,   theta2 = B / (R - A),
      are both at most theta (A, B the cube sides, R the distance between
      the cube centres; theta2 counts as infinite when R <= A);
    - relative (alpha > 0): Gadget-2's criterion that sec. 3.1 follows,
        G M / s^2 (l / s)^2 <= alpha |a|,
      holds for every target particle of A, with s the particle's distance
      to B's centre of mass, l the side of B's cube and |a| the particle's
      reference acceleration;
  a node whose cube holds targets of A (A itself or one of its ancestors,
  unshifted) is never accepted.  Then every target of A gains the force of
  one particle of mass M at B's centre of mass (the 1-to-N case);
* otherwise a leaf B is summed particle by particle with A (the N-to-M case,
  the PP kernel of sec. 3.3), and any other B is opened.

With both tests off nothing is accepted and the walk reaches every pair: the
result is the plain short-range sum.  Every interaction, particle or
monopole, uses the short-range pair force of the rest of the oracle:
    a_i += G m_j d g(s_eps / 2 r_s) / s_eps^3,  d = x_j + sigma L - x_i,
kept when the unsoftened distance s satisfies 0 < s < r_cut, with
s_eps^2 = s^2 + eps^2 and g the factor of Eq. equ:split.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erfc

from . import hilbert_keys, sort_order, quantise

SHIFTS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]


def split_factor(x):
    """g(x) = erfc(x) + (2 x / sqrt(pi)) exp(-x^2), x = s / (2 r_s): Eq. equ:split."""
    return erfc(x) + 2.0 * x / np.sqrt(np.pi) * np.exp(-x * x)


@dataclasses.dataclass
class Node:
    level: int
    begin: int          # particles [begin, end) in key order
    end: int
    lo: tuple           # lower cube corner, grid cells
    side: int           # cube side, grid cells
    flo: tuple          # lower cube corner, lengths
    width: float        # cube side, length
    centre: tuple       # cube centre, lengths
    mass: float
    com: np.ndarray     # centre of mass [3]
    children: list
    leaf: bool


class Tree:
    """The oct-tree of sec. 3.2 over one periodic box (key order)."""

    def __init__(self, pos, mass, params):
        p = params
        self.params = p
        self.L = float(p.L)
        self.bits = int(p.key_bits)
        self.cell = self.L / float(1 << self.bits)
        pos = np.asarray(pos, dtype=np.float64)
        self.n = pos.shape[1]
        keys = hilbert_keys(pos, self.L, self.bits)
        self.order = sort_order(keys)
        self.keys = keys[self.order]
        self.q = quantise(pos, self.L, self.bits)[:, self.order].astype(np.int64)
        self.x = (pos - self.L * np.floor(pos / self.L))[:, self.order]
        self.m = np.asarray(mass, dtype=np.float64)[self.order]
        self.nodes: list[Node] = []
        self.root = self._make(0, 0, self.n) if self.n > 0 else None

    def _make(self, level, b0, e0):
        b = self.bits
        idx = len(self.nodes)
        self.nodes.append(None)
        side = 1 << (b - level)
        lo = tuple(int((self.q[k, b0] >> (b - level)) << (b - level)) for k in range(3))
        msum = float(self.m[b0:e0].sum())
        com = (self.m[b0:e0] * self.x[:, b0:e0]).sum(axis=1) / msum if msum > 0 else \
            self.x[:, b0:e0].mean(axis=1)
        leaf = (e0 - b0) <= self.params.leaf_max or level == b
        children = []
        if not leaf:
            digit = (self.keys[b0:e0] >> np.uint64(3 * (b - level - 1))) & np.uint64(7)
            cuts = b0 + np.searchsorted(digit, np.arange(9, dtype=np.uint64))
            for d in range(8):
                if cuts[d + 1] > cuts[d]:
                    children.append(self._make(level + 1, int(cuts[d]), int(cuts[d + 1])))
        flo = tuple(c * self.cell for c in lo)
        width = side * self.cell
        centre = tuple(c + 0.5 * width for c in flo)
        self.nodes[idx] = Node(level, b0, e0, lo, side, flo, width, centre, msum, com, children, leaf)
        return idx

    def leaves(self):
        return [i for i, nd in enumerate(self.nodes) if nd.leaf]

    def contains(self, outer, inner):
        """Node `outer` is `inner` or one of its ancestors."""
        o, i = self.nodes[outer], self.nodes[inner]
        return o.level <= i.level and o.begin <= i.begin and i.end <= o.end

    def cube_gap2(self, a, b, s):
        """Squared distance between node a's cube and node b's cube shifted by s L."""
        A, B = self.nodes[a], self.nodes[b]
        d2 = 0.0
        for k in range(3):
            blo = B.flo[k] + s[k] * self.L
            g = max(0.0, blo - (A.flo[k] + A.width), A.flo[k] - (blo + B.width))
            d2 += g * g
        return d2


def opening_angles(tree, a, b, s):
    """(theta1, theta2) of sec. 3.3 for target node a and source node b shifted by s L."""
    A, B = tree.nodes[a], tree.nodes[b]
    L = tree.L
    dx = B.centre[0] + s[0] * L - A.centre[0]
    dy = B.centre[1] + s[1] * L - A.centre[1]
    dz = B.centre[2] + s[2] * L - A.centre[2]
    R = math.sqrt(dx * dx + dy * dy + dz * dz)
    th1 = (B.width + A.width) / R if R > 0 else math.inf
    th2 = B.width / (R - A.width) if R > A.width else math.inf
    return th1, th2


def _pair_force(xt, xs, ms, p):
    """Short-range accelerations [3, t] on targets xt [3, t] from sources xs
    [3, S] of masses ms [S] (already shifted to their image)."""
    d = xs[:, None, :] - xt[:, :, None]
    s2 = (d * d).sum(axis=0)
    keep = (s2 < p.rcut * p.rcut) & (s2 > 0)
    se2 = np.where(keep, s2 + p.eps * p.eps, 1.0)
    se = np.sqrt(se2)
    f = np.where(keep, p.G * ms[None, :] * split_factor(se / (2.0 * p.rs)) / (se2 * se), 0.0)
    return (f[None] * d).sum(axis=2), int(keep.sum())


def dtt_accel(pos, mass, params, theta=0.0, alpha=0.0, acc_ref=None, tree=None):
    """Short-range accelerations [3][n] (input order) by the dual tree
    traversal with monopole acceptance.

    theta: geometric test (0: off); alpha > 0 with acc_ref [3][n] (input
    order): the relative test.  Returns a dict with 'acc', 'n_mono_pairs'
    (target particles x accepted monopoles), 'n_pp_pairs' (particle pairs
    within the cut summed directly), 'accepted' (the list of (target leaf,
    source node, shift) taken as monopoles) and 'tree'."""
    p = params
    if tree is None:
        tree = Tree(pos, mass, p)
    n = tree.n
    acc_sorted = np.zeros((3, n))
    out = {"acc": np.zeros((3, n)), "n_mono_pairs": 0, "n_pp_pairs": 0, "accepted": [], "tree": tree}
    if n == 0:
        return out
    amag = None
    if alpha > 0:
        ar = np.asarray(acc_ref, dtype=np.float64)[:, tree.order]
        amag = np.sqrt((ar * ar).sum(axis=0))
    rc2 = p.rcut * p.rcut
    L = tree.L

    def accept(a, b, s, xt):
        if theta <= 0 and alpha <= 0:
            return False
        if s == (0, 0, 0) and tree.contains(b, a):
            return False
        if theta > 0:
            th1, th2 = opening_angles(tree, a, b, s)
            if not (th1 <= theta and th2 <= theta):
                return False
        if alpha > 0:
            B = tree.nodes[b]
            A = tree.nodes[a]
            c = B.com + L * np.asarray(s, dtype=np.float64)
            sd = np.sqrt(((xt - c[:, None]) ** 2).sum(axis=0))
            if np.any(sd <= 0):
                return False
            lhs = p.G * B.mass / sd ** 2 * (B.width / sd) ** 2
            if not np.all(lhs <= alpha * amag[A.begin:A.end]):
                return False
        return True

    for a in tree.leaves():
        A = tree.nodes[a]
        xt = tree.x[:, A.begin:A.end]
        pp_x, pp_m, mono_x, mono_m = [], [], [], []
        for s in SHIFTS:
            sh = L * np.asarray(s, dtype=np.float64)
            stack = [tree.root]
            while stack:
                b = stack.pop()
                if tree.cube_gap2(a, b, s) >= rc2:
                    continue
                B = tree.nodes[b]
                if accept(a, b, s, xt):
                    out["accepted"].append((a, b, s))
                    mono_x.append((B.com + sh)[:, None])
                    mono_m.append(np.array([B.mass]))
                elif B.leaf:
                    pp_x.append(tree.x[:, B.begin:B.end] + sh[:, None])
                    pp_m.append(tree.m[B.begin:B.end])
                else:
                    stack.extend(B.children)
        if pp_x:
            f, kept = _pair_force(xt, np.concatenate(pp_x, axis=1), np.concatenate(pp_m), p)
            acc_sorted[:, A.begin:A.end] += f
            out["n_pp_pairs"] += kept
        if mono_x:
            f, _ = _pair_force(xt, np.concatenate(mono_x, axis=1), np.concatenate(mono_m), p)
            acc_sorted[:, A.begin:A.end] += f
            out["n_mono_pairs"] += len(mono_x) * (A.end - A.begin)
    out["acc"][:, tree.order] = acc_sorted
    return out
