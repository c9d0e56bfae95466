"""Systematic resampling of a walker ensemble at a fixed walker count --
test infrastructure, written independently of the device implementation.

The paper's CPU code spawned walkers whenever a transition probability
exceeded a random number (Sec. II.B), so the walker count grew; its GPU code
keeps the count fixed and lets the weights grow instead.  This is the
fixed-budget middle ground: between propagation calls the ensemble is
resampled in proportion to |w|, keeping T walkers, and each copy carries a
weight that keeps every walker's expected contribution unchanged.

Steps, in exact integer arithmetic wherever a decision is taken:

1. w_max = max |w_i| over walkers with finite w and phase (0 if none).
2. k_i = ceil(|w_i| / w_max * 2^32) for those walkers with w_i != 0, else 0
   (the ratio is one binary64 division, the scaling by 2^32 is exact).
3. Prefix sums P_i = k_0 + ... + k_{i-1}, total K = P_T.
4. One offset U (32 bits): word 0 of Philox4x32-10 with key (seed lo, seed
   hi) and counter (traj_offset lo, traj_offset hi, step lo, 3).
5. Output walker j (0 <= j < T) copies source i(j), the walker whose interval
   [P_i, P_i + k_i) contains the comb point X_j = floor((j 2^32 + U) K /
   (T 2^32)).
6. The copy's weight is w_i * (K / (T k_i)), with K, T and k_i converted to
   binary64 and the product T k_i formed in binary64.  The expected number
   of copies of i is T k_i / K up to the comb's integer grid (within 2^-32
   over the 2^32 offsets), so the expected weight is w_i to that accuracy.

If K = 0 (no walker has a nonzero finite weight) the ensemble is copied
unchanged.  The state (q, p, U, phase, a, b, flags) of walker i is copied as
is; the copy continues as walker j, with the random stream of global id
traj_offset + j.
"""
from __future__ import annotations

import bisect
import itertools
import math

import numpy as np

from . import core as oc

TWO32 = 1 << 32


def offset_word(seed: int, traj_offset: int, step: int) -> int:
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    counter = [traj_offset & 0xFFFFFFFF, (traj_offset >> 32) & 0xFFFFFFFF, step & 0xFFFFFFFF, 3]
    return int(oc.philox(counter, key)[0])


def quantized(w, phase):
    """Steps 1-2: (k list of Python ints, w_max)."""
    finite = [math.isfinite(x) and math.isfinite(f) for x, f in zip(w, phase)]
    w_max = max((abs(x) for x, ok in zip(w, finite) if ok), default=0.0)
    k = []
    for x, ok in zip(w, finite):
        if ok and x != 0.0:
            k.append(math.ceil(abs(x) / w_max * TWO32))
        else:
            k.append(0)
    return k, w_max


def indices(k, U: int):
    """Steps 3 and 5: the source of every output walker (Python ints)."""
    T = len(k)
    P = [0]
    for x in k:
        P.append(P[-1] + x)
    K = P[-1]
    if K == 0:
        return list(range(T)), K
    src = []
    i = 0
    for j in range(T):
        X = ((j * TWO32 + U) * K) // (T * TWO32)
        while not (P[i] <= X < P[i + 1]):  # outputs visit sources in order
            i += 1
        src.append(i)
    return src, K


def prefix(k):
    """Step 3 alone: [P_0 = 0, P_1, ..., P_T = K] (Python ints)."""
    return [0] + list(itertools.accumulate(k))


def source(P, U: int, j: int) -> int:
    """Step 5 for one output walker j: the i with P_i <= X_j < P_{i+1}
    (requires K = P[-1] > 0)."""
    T, K = len(P) - 1, P[-1]
    X = ((j * TWO32 + U) * K) // (T * TWO32)
    return bisect.bisect_right(P, X) - 1


def resample(st: "oc.State", seed: int) -> "oc.State":
    """A new State with the resampled walkers (st is not changed)."""
    T = st.n_traj
    k, _ = quantized(st.w.tolist(), st.phase.tolist())
    U = offset_word(seed, st.traj_offset, st.step)
    src, K = indices(k, U)
    out = st.copy()
    if K == 0:
        return out
    idx = np.array(src, dtype=np.int64)
    for name in ("q", "p", "U", "phase", "a", "b", "flags"):
        setattr(out, name, getattr(st, name)[idx].copy())
    scale = np.array([float(K) / (float(T) * float(k[i])) for i in src])
    out.w = st.w[idx] * scale
    return out
