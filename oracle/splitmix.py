"""Oracle: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), from its published definition.

The library draws U, V, D_r and D_c from a counter-based SplitMix64: the
random choices of step 2 of the "Block Wiedemann Rank Algorithm" (Section 2.5)
are the only ones the method makes.  The paper does not say how to draw them;
the reading used here:

    gamma      = 0x9E3779B97F4A7C15
    mix(z)     = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
                 z *= 0x94D049BB133111EB; z ^= z >> 31          (mod 2^64)
    output(state, i) = mix(state + (i + 1) * gamma)     (i-th output, i >= 0)
    key(seed, t)     = output(seed, t)
    element(seed, t, i) = output(key(seed, t), i)

Streams t: 0 = V (n*s, row-major), 1 = U (n*s), 2 = D_r (m), 3 = D_c (n).
Residues: U, V take h mod p; diagonals take 1 + h mod (p - 1).

Pinned by the known first outputs of SplitMix64 seeded with 0.
"""
MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
STREAM_V, STREAM_U, STREAM_DROW, STREAM_DCOL = 0, 1, 2, 3


def mix(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def output(state: int, i: int) -> int:
    return mix(state + (i + 1) * GAMMA)


def element(seed: int, stream: int, i: int) -> int:
    return output(output(seed, stream), i)


def block(seed: int, stream: int, count: int, p: int, diag: bool = False):
    """``count`` residues of one stream: h mod p, or 1 + h mod (p - 1) for diagonals."""
    key = output(seed, stream)
    if diag:
        return [1 + output(key, i) % (p - 1) for i in range(count)]
    return [output(key, i) % p for i in range(count)]
