"""Counter-based SplitMix64 random numbers for seeded synthetic inputs.

SplitMix64 is the generator of Steele, Lea and Flood, "Fast splittable
pseudorandom number generators" (OOPSLA 2014): an additive Weyl step by the
golden-ratio constant followed by a 64-bit finalizer.  Here it is used as a
*counter* generator: every random number is the finalizer applied to a key
that is a chain of finalizer calls over (seed, stream, index...).  The same
(seed, stream, index) therefore always yields the same number, independent of
how the caller chunks the work.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output function applied elementwise to uint64 input (in place on a copy)."""
    z = np.array(x, dtype=np.uint64, copy=True)
    t = np.empty_like(z)
    with np.errstate(over="ignore"):
        z += _GAMMA
        np.right_shift(z, np.uint64(30), out=t)
        z ^= t
        z *= _M1
        np.right_shift(z, np.uint64(27), out=t)
        z ^= t
        z *= _M2
        np.right_shift(z, np.uint64(31), out=t)
        z ^= t
    return z[()] if z.ndim == 0 else z


def key(*fields):
    """Chain the finalizer over integer fields (scalars or broadcastable arrays)."""
    k = np.zeros((), dtype=np.uint64)
    for f in fields:
        k = splitmix64(k ^ np.asarray(f, dtype=np.uint64))
    return k


def uniform01(k):
    """Top 53 bits of the finalizer of key k, as a double in [0, 1)."""
    return (splitmix64(k) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm1(k):
    """Double in [-1, 1) from key k."""
    return 2.0 * uniform01(k) - 1.0


# stream identifiers (distinct constants so different uses never collide)
STREAM_NOISE = 1
STREAM_PHASE = 2
STREAM_BUMP = 3
STREAM_SYSTEM = 4
STREAM_GLOBAL_PHASE = 5
STREAM_IMBALANCE = 6
