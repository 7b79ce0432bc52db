"""SplitMix64 counter generator (oracle; test infrastructure only).

Published definition (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014): the n-th output of the stream with seed
s is mix(s + n * 0x9E3779B97F4A7C15) with the variant-13 finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)
all modulo 2^64.  Output n of sub-stream ``stream`` is taken at counter
n + 1 + stream * 2^40, and mapped to [-1, 1) as (z >> 11) * 2^-52 - 1.
The Lanczos start vector of each (level, block) is drawn this way, so
that both implementations draw the same vector without sharing code.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
C1 = np.uint64(0xBF58476D1CE4E5B9)
C2 = np.uint64(0x94D049BB133111EB)


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * C1
        z = (z ^ (z >> np.uint64(27))) * C2
    return z ^ (z >> np.uint64(31))


def uniform_pm1(seed: int, stream: int, n: int) -> np.ndarray:
    ctr = np.arange(n, dtype=np.uint64) + np.uint64(1) + (np.uint64(stream) << np.uint64(40))
    with np.errstate(over="ignore"):
        z = mix64(np.uint64(seed) + ctr * GAMMA)
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
