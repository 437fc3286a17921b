"""Probe vectors for Hutchinson's estimator (Section 2.1, eq. def:mcEstimate).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Rademacher probes are drawn from a counter-based generator so that any entry
z_i^(p) can be regenerated independently.  The generator is SplitMix64
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), implemented here from its published definition:

    state_{k+1} = state_k + GAMMA                (mod 2^64)
    output_k    = MIX(state_{k+1})
    MIX(x): x ^= x>>30; x *= 0xBF58476D1CE4E5B9; x ^= x>>27;
            x *= 0x94D049BB133111EB; x ^= x>>31

so the k-th output (k = 0, 1, ...) of a stream started at s is
MIX(s + (k+1)*GAMMA).  Probe p of seed ``seed``:

    key_p       = output_p of the stream started at ``seed``
    word_{p,c}  = output_c of the stream started at key_p
    z_i^(p)     = +1 if bit (i mod 64) of word_{p, floor(i/64)} is 0, else -1
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB


def mix64(x: int) -> int:
    """SplitMix64 output function on a Python int (exact mod 2^64)."""
    x &= MASK
    x = ((x ^ (x >> 30)) * MUL1) & MASK
    x = ((x ^ (x >> 27)) * MUL2) & MASK
    return x ^ (x >> 31)


def splitmix_output(state: int, k: int) -> int:
    """k-th output (0-based) of SplitMix64 started at ``state``."""
    return mix64((state + (k + 1) * GAMMA) & MASK)


def _mix64_vec(x: np.ndarray) -> np.ndarray:
    # numpy uint64 arithmetic wraps modulo 2^64, which is exactly what the
    # definition asks for.
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        x = (x ^ (x >> np.uint64(30))) * np.uint64(MUL1)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(MUL2)
    return x ^ (x >> np.uint64(31))


def rademacher(d: int, probe_ids, seed: int) -> np.ndarray:
    """Rademacher probes as float64 array [len(probe_ids), d] of +-1."""
    probe_ids = np.asarray(probe_ids, dtype=np.uint64).reshape(-1)
    nwords = (d + 63) // 64
    with np.errstate(over="ignore"):
        keys = _mix64_vec(np.uint64(seed & MASK)
                          + (probe_ids + np.uint64(1)) * np.uint64(GAMMA))
        c = np.arange(nwords, dtype=np.uint64)
        words = _mix64_vec(keys[:, None]
                           + (c[None, :] + np.uint64(1)) * np.uint64(GAMMA))
    i = np.arange(d, dtype=np.uint64)
    bits = (words[:, (i >> np.uint64(6)).astype(np.int64)]
            >> (i & np.uint64(63))) & np.uint64(1)
    return 1.0 - 2.0 * bits.astype(np.float64)


def rademacher_slow(d: int, p: int, seed: int) -> np.ndarray:
    """Same probe as ``rademacher`` computed with Python integers, one entry at
    a time (used to cross-check the vectorised form on small d)."""
    key = splitmix_output(seed, p)
    z = np.empty(d)
    for i in range(d):
        w = splitmix_output(key, i // 64)
        z[i] = -1.0 if (w >> (i % 64)) & 1 else 1.0
    return z


def unit_probes(d: int) -> np.ndarray:
    """All basis vectors e_i as probes: sum_i e_i^T M e_i = tr M."""
    return np.eye(d)
