"""Counter-based Gaussian stream for the Davidson restart (Sec. II-C: the
routine uses randomization when reorthogonalization fails).

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finaliser of Vigna's splitmix64.c): the
n-th output (n = 0, 1, ...) of the stream seeded with key is
mix(key + (n + 1) * 0x9E3779B97F4A7C15 mod 2^64).

Uniforms u = (x >> 11) * 2^-53.  Element e of a restart vector takes outputs 2e
and 2e + 1 and the Box-Muller cosine branch
  z = sqrt(-2 ln(1 - u1)) cos(2 pi u2).
The stream key of restart (seed, iteration, attempt) is
  seed + 0x632BE59BD9B4E019 * (1 + 65536 * iteration + attempt)  (mod 2^64).
"""
import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z):
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64_stream(key, n):
    return [mix64((key + (i + 1) * GOLDEN) & M64) for i in range(n)]


def restart_key(seed, iteration, attempt):
    return (int(seed) + 0x632BE59BD9B4E019 * (1 + 65536 * int(iteration) + int(attempt))) & M64


def _mix64_vec(z):
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def gaussian_at(key, idx):
    """Gaussian values for element indices ``idx`` (int array) of stream ``key``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s1 = np.uint64(key) + (np.uint64(2) * idx + np.uint64(1)) * np.uint64(GOLDEN)
        s2 = np.uint64(key) + (np.uint64(2) * idx + np.uint64(2)) * np.uint64(GOLDEN)
    u1 = (_mix64_vec(s1) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (_mix64_vec(s2) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * np.pi * u2)
