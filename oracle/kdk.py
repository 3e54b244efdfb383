"""FP64 CPU oracle for the adaptive Kick-Drift-Kick time integration.

TEST INFRASTRUCTURE ONLY: only the tests may import this module.  It shares
no code with the HIP library and never imports it.

Sec. 3.4 (adaptive KDK stepping), restated for a non-expanding box (scale
factor a = 1, so the drift and kick integrals of dt / a^2 and dt / a are
both the step length):
  * Kick  K(t1; t2): v <- v + acc (t2 - t1);
  * Drift D(t1; t2): x <- x + v (t2 - t1), wrapped into the periodic box;
  * KDK: half kick, full drift, force evaluation, half kick.
Step lengths are powers of two below the top step dt (sec. 3.4): particle
i takes dt / 2^k_i with the smallest k_i >= 0 for which the step meets the
Gadget-2 criterion dt_i <= sqrt(2 eta eps / |a_i|) (the paper prints the
criterion with its square root misplaced), capped at max_level.  Levels are
set from the accelerations at the start of a top step and kept for it.
Within the top step there are 2^K substeps of dt / 2^K, K the deepest level:
at a substep, every particle whose own step starts there gets its opening
half kick, all particles drift, the forces are evaluated, and every particle
whose step ends there gets its closing half kick.
"""
from __future__ import annotations

import numpy as np


def step_levels(acc: np.ndarray, eta: float, eps: float, dt: float, max_level: int) -> np.ndarray:
    """Smallest k in [0, max_level] with dt / 2^k <= sqrt(2 eta eps / |a|)."""
    amag = np.linalg.norm(np.asarray(acc, dtype=np.float64), axis=0)
    lev = np.zeros(amag.shape, dtype=np.int64)
    for i, a in enumerate(amag):
        if a == 0.0:
            continue
        t = np.sqrt(2.0 * eta * eps / a)
        k = 0
        while k < max_level and dt / 2.0 ** k > t:
            k += 1
        lev[i] = k
    return lev


def kdk_top_step(pos, vel, acc, force, dt, levels, L):
    """One top step of the block KDK scheme.  force(pos) -> acc [3][n];
    acc holds the accelerations at pos on entry.  Returns pos, vel, acc at
    the end of the step and the number of force evaluations."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    acc = np.array(acc, dtype=np.float64)
    K = int(levels.max()) if levels.size else 0
    nsub = 2 ** K
    h = dt / nsub
    span = 2 ** (K - levels)                  # substeps per particle step
    evals = 0
    for s in range(nsub):
        opening = (s % span) == 0
        vel[:, opening] += acc[:, opening] * (0.5 * dt / 2.0 ** levels[opening])
        pos = np.mod(pos + vel * h, L)
        acc = np.asarray(force(pos), dtype=np.float64)
        evals += 1
        closing = ((s + 1) % span) == 0
        vel[:, closing] += acc[:, closing] * (0.5 * dt / 2.0 ** levels[closing])
    return pos, vel, acc, evals


def dkd_step(pos, vel, force, dt, L):
    """Drift-Kick-Drift with one shared step (for the robustness comparison
    of sec. 3.4)."""
    pos = np.mod(np.asarray(pos, dtype=np.float64) + np.asarray(vel) * 0.5 * dt, L)
    vel = np.asarray(vel, dtype=np.float64) + np.asarray(force(pos)) * dt
    pos = np.mod(pos + vel * 0.5 * dt, L)
    return pos, vel
