"""Count sketch SA = Phi D A (Def. 2.3 and the worked example after it).

TEST INFRASTRUCTURE ONLY (see the package docstring): the oracle's own hash,
sign and sketch, written from the definition.

Definition 2.3: D is diagonal with independent equiprobable +-1 entries, Phi is
s x m binary with Phi[h(i), i] = 1, h(i) uniform on [0, s).  S = Phi D has one
nonzero per column, so row j of SA is the signed sum of the rows i of A with
h(i) = j, and S never needs to be formed (Sec. 2.2).

The paper fixes no generator.  The reading used on both sides of the parity
check is a counter-based SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014):

    x_h(i)  = mix64(seed + (i+1) * GAMMA)            (mod 2^64)
    x_s(i)  = mix64((seed ^ SIGN_SALT) + (i+1) * GAMMA)
    h(i)    = ((x_h >> 32) * s) >> 32                (multiply-shift range map)
    sign(i) = +1 if the top bit of x_s is 0 else -1

The summation order inside a bucket is not specified by the paper; the reading
is ascending original row index, starting from +0.0, with plain (unfused) adds.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX_M1 = np.uint64(0xBF58476D1CE4E5B9)
MIX_M2 = np.uint64(0x94D049BB133111EB)
SIGN_SALT = 0x5555555555555555
MASK64 = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * MIX_M1
        z = (z ^ (z >> np.uint64(27))) * MIX_M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    """The first `count` outputs of a SplitMix64 generator whose state starts at `seed`."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = np.uint64(seed & MASK64) + k * GAMMA
    return mix64(states)


def hash_sign(m: int, s: int, seed: int):
    """h: int32[m] in [0, s) and sign: int8[m] in {+1, -1} (Def. 2.3)."""
    if s <= 0 or s >= (1 << 31):
        raise ValueError("s must be in [1, 2^31)")
    xh = splitmix64_stream(seed, m)
    xs = splitmix64_stream(seed ^ SIGN_SALT, m)
    with np.errstate(over="ignore"):
        h = ((xh >> np.uint64(32)) * np.uint64(s)) >> np.uint64(32)
    sign = np.where((xs >> np.uint64(63)) == 0, 1, -1).astype(np.int8)
    return h.astype(np.int32), sign


def bucket_rows(h: np.ndarray, s: int):
    """Rows grouped by bucket, ascending row index inside each bucket.
    Returns (bucket_ptr int64[s+1], perm int32[m])."""
    perm = np.argsort(h, kind="stable").astype(np.int32)
    counts = np.bincount(h, minlength=s).astype(np.int64)
    ptr = np.zeros(s + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, perm


def _row_entries(row_ptr, rows):
    """Flat indices into col/val of all entries of `rows` and the owning row of each."""
    starts = row_ptr[rows]
    lens = row_ptr[rows + 1] - starts
    owner = np.repeat(np.arange(len(rows)), lens)
    offs = np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens)
    return starts[owner] + offs, owner


def sketch_dense(row_ptr, col, val, h, sign, s: int, n: int, b=None):
    """Dense SA (s x n, float64) and optionally Sb (for b of shape [m] or [k, m]).

    Rows enter their bucket in ascending row order: round r adds the r-th row of
    every bucket, so each element of SA receives at most one add per round and
    the additions happen in exactly the order of the reading above."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    m = len(row_ptr) - 1
    ptr, perm = bucket_rows(h, s)
    rank = np.arange(m) - np.repeat(ptr[:-1], np.diff(ptr))
    SA = np.zeros((s, n), dtype=np.float64)
    bb = None if b is None else np.atleast_2d(np.asarray(b, dtype=np.float64))
    Sb = None if b is None else np.zeros((bb.shape[0], s), dtype=np.float64)
    sgn = sign.astype(np.float64)
    for r in range(int(rank.max()) + 1 if m else 0):
        rows = perm[rank == r].astype(np.int64)
        idx, owner = _row_entries(row_ptr, rows)
        tgt = h[rows][owner]
        SA[tgt, col[idx]] += sgn[rows][owner] * val[idx]
        if Sb is not None:
            Sb[:, h[rows]] += sgn[rows][None, :] * bb[:, rows]
    if Sb is not None and np.ndim(b) == 1:
        Sb = Sb[0]
    return SA, Sb


def explicit_S(h: np.ndarray, sign: np.ndarray, s: int) -> np.ndarray:
    """The s x m matrix S = Phi D itself (only for tiny cases)."""
    m = h.shape[0]
    S = np.zeros((s, m))
    S[h, np.arange(m)] = sign
    return S


def sketch_rows(row_ptr, col, val, h, sign, n: int, buckets):
    """Rows `buckets` of SA only (same ascending-row summation), for spot checks
    of large sketches."""
    out = np.zeros((len(buckets), n))
    for k, j in enumerate(buckets):
        for i in np.nonzero(h == j)[0]:  # ascending row order
            lo, hi = row_ptr[i], row_ptr[i + 1]
            out[k, col[lo:hi]] += float(sign[i]) * val[lo:hi]
    return out
