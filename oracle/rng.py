"""SplitMix64 counter-based generator (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written from its published
definition.

Test infrastructure (see ``oracle/__init__``).

The smoother's eigenvalue estimate starts from a random vector.  So that the
oracle and the device library start from the same vector whatever their dof
numbering, each entry is drawn from the counter
    c = 3 * (canonical node key) + component
as  x = c + seed * 0xD1B54A32D192ED03 (mod 2^64), z = mix(x + 0x9E3779B97F4A7C15),
    value = 2 * (z >> 11) * 2^-53 - 1   in [-1, 1).
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_SEEDMUL = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output for state x (array of uint64): one step of the
    generator (state += golden gamma, then the variant-13 finaliser)."""
    with np.errstate(over='ignore'):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(seed, counters):
    """Values in [-1, 1) for the given counters (array-like of non-negative ints)."""
    with np.errstate(over='ignore'):
        c = np.asarray(counters, dtype=np.uint64)
        x = c + np.uint64(seed) * _SEEDMUL
    z = splitmix64(x)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def dof_vector(mesh, seed):
    """Start vector over the velocity dofs of a level mesh (3 node + comp)."""
    c = (3 * mesh.keys[:, None].astype(np.int64) + np.arange(3)[None, :]).ravel()
    return uniform_pm1(seed, c)
