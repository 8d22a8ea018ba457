"""Counter-based random streams for block selection and importance sampling.

TEST INFRASTRUCTURE (oracle). The paper only says blocks are chosen at random
(Algorithm 1, block-selection step) and that sub-detectors are importance
sampled (Algorithm 2); it fixes no generator. The reading used here makes every
draw a pure function of (seed, stream, counters) so that any implementation can
reproduce it bit for bit:

* mix(z): the SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
* hash(seed, stream, k1, k2, ...): h = mix(seed + golden * (1 + stream)), then
  h = mix(h xor k) for each key k, all modulo 2^64.
* bounded(h, n) = floor(h * n / 2^64).
* choose m of n without replacement: partial Fisher-Yates over [0..n) where step
  t swaps position t with t + bounded(hash(seed, stream, k, t), n - t); the first
  m entries, sorted ascending, are the selection.

Pinned by the published SplitMix64 output sequence (tests) and frequency tests.
"""
from __future__ import annotations

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

STREAM_PARTITION = 1
STREAM_ROWS = 2
STREAM_BLOCKS = 3
STREAM_IM = 4


def mix(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_sequence(state: int, n: int):
    """The plain SplitMix64 generator: state += golden; output mix(state)."""
    out = []
    for _ in range(n):
        state = (state + GOLDEN) & MASK
        out.append(mix(state))
    return out


def hash_keys(seed: int, stream: int, *keys: int) -> int:
    h = mix((seed + GOLDEN * (1 + stream)) & MASK)
    for k in keys:
        h = mix(h ^ (k & MASK))
    return h


def bounded(h: int, n: int) -> int:
    return (h * n) >> 64


def choose(seed: int, stream: int, k: int, n: int, m: int):
    """m distinct indices of [0, n) for iteration k, ascending."""
    if not 0 < m <= n:
        raise ValueError("need 0 < m <= n")
    a = list(range(n))
    for t in range(m):
        jj = t + bounded(hash_keys(seed, stream, k, t), n - t)
        a[t], a[jj] = a[jj], a[t]
    return sorted(a[:m])


def permutation(seed: int, stream: int, n: int):
    """A full Fisher-Yates permutation of [0, n) keyed only by position."""
    a = list(range(n))
    for t in range(n - 1):
        jj = t + bounded(hash_keys(seed, stream, t), n - t)
        a[t], a[jj] = a[jj], a[t]
    return a
