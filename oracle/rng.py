"""Counter-based noise for the stochastic estimators.

The paper only asks that the noise components be isotropic (Sec. 1, eq.
random_props): E|z_i|^2 = 1 and E[z_i z_j] = 0 for i != j; it names Rademacher
vectors (z uniform in {-1, +1}) and Z4 vectors (Sec. 2).  We use

* Rademacher: z = +-1 (real);
* Z2xZ2:      z = (+-1 +- i) / sqrt(2), i.e. exp(i pi/4) times a Z4 variable,
              which has the same Hutchinson variance as Z4.

Random words come from SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used as a counter
generator so that any element of any vector can be drawn in any order:

    base    = mix64(seed + GOLDEN)        (first SplitMix64 output from state seed)
    key     = base XOR (purpose << 56) XOR (level << 48) XOR index
    state0  = mix64(key)
    word_i  = mix64(state0 + (i + 1) * GOLDEN)          (mod 2^64)

(Hashing the seed first keeps runs with neighbouring seeds independent; a
plain ``seed XOR index`` would give seed s, index i+1 the stream of seed s+1,
index i.)

where ``mix64`` is SplitMix64's output function and ``i`` is the *logical*
element index of the vector on its level.  Bit 63 of ``word_i`` gives the sign
of the real part, bit 62 the sign of the imaginary part.

Parity: pinned by tests against the published SplitMix64 output stream for
seed 1234567 and by the isotropy moments.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)

PURPOSE_SETUP = 1    # multigrid test vectors
PURPOSE_SKETCH = 2   # Hutch++ block power iteration start vectors S_l
PURPOSE_SAMPLE = 3   # stochastic samples zeta_s
PURPOSE_DEFLATE = 5  # start block of the deflation subspace iteration
PURPOSE_PILOT = 6    # pilot samples of the adaptive choice of d_l (discarded)

RADEMACHER = "rademacher"
Z2Z2 = "z2z2"


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    """The first ``count`` outputs of SplitMix64 started from state ``seed``."""
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed) + i * GOLDEN)


def stream_key(seed: int, purpose: int, level: int, index: int) -> int:
    if not (0 <= index < (1 << 48)) or not (0 <= level < 256) or not (0 <= purpose < 256):
        raise ValueError("noise key field out of range")
    base = int(splitmix64_stream(seed & 0xFFFFFFFFFFFFFFFF, 1)[0])
    return (base ^ (purpose << 56) ^ (level << 48) ^ index) & 0xFFFFFFFFFFFFFFFF


def words(seed: int, purpose: int, level: int, index: int, n: int) -> np.ndarray:
    state0 = mix64(np.uint64(stream_key(seed, purpose, level, index)))
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(state0 + i * GOLDEN)


def noise_vector(kind: str, seed: int, purpose: int, level: int, index: int, n: int) -> np.ndarray:
    """One isotropic noise vector of length n (complex128)."""
    w = words(seed, purpose, level, index, n)
    re_neg = (w >> np.uint64(63)) & np.uint64(1)
    if kind == RADEMACHER:
        return np.where(re_neg == 1, -1.0, 1.0).astype(np.complex128)
    if kind == Z2Z2:
        im_neg = (w >> np.uint64(62)) & np.uint64(1)
        h = np.sqrt(0.5)
        re = np.where(re_neg == 1, -h, h)
        im = np.where(im_neg == 1, -h, h)
        return re + 1j * im
    raise ValueError(f"unknown noise kind {kind!r}")


def noise_block(kind: str, seed: int, purpose: int, level: int, index0: int, count: int,
                n: int) -> np.ndarray:
    """Columns index0 .. index0+count-1 as an (n, count) matrix."""
    out = np.empty((n, count), dtype=np.complex128)
    for j in range(count):
        out[:, j] = noise_vector(kind, seed, purpose, level, index0 + j, n)
    return out
