"""Counter-based random iterates for served requests, host side.

TEST INFRASTRUCTURE (see the package docstring).  Written independently of
the library's device generator from the published definitions:
  - SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
    pseudorandom number generators", OOPSLA 2014): z = x ^ (x >> 30),
    z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB,
    z ^= z >> 31, applied to x = seed + (j + 1) * 0x9E3779B97F4A7C15 (mod 2^64)
    for stream element j;
  - a double in [0, 1) from the top 53 bits;
  - Box-Muller normals sqrt(-2 ln(1 - u1)) cos(2 pi u2).
The request iterate layout: x = [theta ~ U(-0.2, 0.2); v ~ U(0.95, 1.05);
Pg ~ U(pmin, pmax); Qg ~ U(qmin, qmax)] from elements 0..n-1, and lambda_r
from elements n + 2r, n + 2r + 1.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, j: np.ndarray) -> np.ndarray:
    """Raw 64-bit output for stream elements j: output j + 1 of SplitMix64
    started at state `seed`."""
    with np.errstate(over="ignore"):
        x = np.uint64(seed) + (np.asarray(j).astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (x ^ (x >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniforms(seed: int, j: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of splitmix64(seed, j)."""
    return (splitmix64(seed, j) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def request_iterate(seed: int, nb: int, ng: int, m: int, bounds):
    pmin, pmax, qmin, qmax = bounds
    n = 2 * nb + 2 * ng
    u = uniforms(seed, np.arange(n))
    x = np.empty(n)
    x[:nb] = -0.2 + 0.4 * u[:nb]
    x[nb:2 * nb] = 0.95 + 0.1 * u[nb:2 * nb]
    x[2 * nb:2 * nb + ng] = pmin + (pmax - pmin) * u[2 * nb:2 * nb + ng]
    x[2 * nb + ng:] = qmin + (qmax - qmin) * u[2 * nb + ng:]
    r = np.arange(m)
    u1 = uniforms(seed, n + 2 * r)
    u2 = uniforms(seed, n + 2 * r + 1)
    lam = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)
    return x, lam
