"""Oracle: seeded N(0,1) draws from their published definitions.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state += 0x9e3779b97f4a7c15, then
z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9, z = (z ^ (z >> 27)) * 0x94d049bb133111eb,
output z ^ (z >> 31); output i of a stream seeded with s therefore mixes
s + (i + 1) * 0x9e3779b97f4a7c15.  Box & Muller (1958): from uniforms u1, u2,
r = sqrt(-2 ln(1 - u1)), z0 = r cos(2 pi u2), z1 = r sin(2 pi u2), with
u = (output >> 11) * 2^-53.  Element e of a draw takes z0 (e even) or z1 (e odd)
of pair e // 2.  Used for seeded start vectors (Algorithm 1 takes any starting
vector; the workload's reading is an iid N(0, 1) field).

Parity status: pinned by the generator's published first outputs for seed 0
(tests/golden/splitmix64_seed0.txt) and by the moments of a large draw.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, count, start=0):
    """Outputs start .. start+count-1 of the splitmix64 stream seeded with ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start, start + count, dtype=np.uint64) + np.uint64(1)
        z = np.uint64(seed) + i * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def normal(count, seed):
    """``count`` N(0,1) draws (element e from pair e // 2)."""
    npair = (count + 1) // 2
    o = splitmix64(seed, 2 * npair)
    u1 = (o[0::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (o[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(1.0 - u1))
    th = 2.0 * np.pi * u2
    out = np.empty(2 * npair)
    out[0::2] = r * np.cos(th)
    out[1::2] = r * np.sin(th)
    return out[:count]
