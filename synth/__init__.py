"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module only draws numbers: a SplitMix64 stream (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) in counter
form, reduced into [0, m) for a list of moduli. It holds none of the
KeySwitch arithmetic; the moduli are passed in by the caller.

Draw number ``i`` (0-based) of the stream with seed ``s`` is
``mix(s + (i + 1) * 0x9E3779B97F4A7C15)`` with SplitMix64's finaliser ``mix``.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the named inputs: ciphertext item b uses D_SEED_BASE + b.
SEED_S, SEED_S2, SEED_A, SEED_E = 1, 2, 3, 4
D_SEED_BASE = 1000


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of the stream with the given seed (uint64)."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = idx * GAMMA + np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform_residues(seed: int, moduli, n: int, start: int = 0) -> np.ndarray:
    """[len(moduli)][n] uint64; entry (i, x) is draw start + i*n + x reduced mod moduli[i]."""
    moduli = [int(m) for m in moduli]
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, m in enumerate(moduli):
        out[i] = splitmix64(seed, start + i * n, n) % np.uint64(m)
    return out


def ciphertext_batch(q_moduli, n: int, batch: int, seed_base: int = D_SEED_BASE) -> np.ndarray:
    """[batch][ell][n] uniform residues; item b uses seed seed_base + b."""
    return np.stack([uniform_residues(seed_base + b, q_moduli, n) for b in range(batch)])


def uniform_key(pq_moduli, n: int, ndig: int, seed: int = SEED_A) -> np.ndarray:
    """[ndig][2][len(pq_moduli)][n] uniform residues, a stand-in evaluation key.

    A real evaluation key is uniform modulo each prime too (its a-part is
    uniform and its b-part is masked by a), so this has the key's size and
    value distribution without a secret."""
    nl = len(pq_moduli)
    out = np.empty((ndig, 2, nl, n), dtype=np.uint64)
    for j in range(ndig):
        for c in range(2):
            out[j, c] = uniform_residues(seed, pq_moduli, n, start=(j * 2 + c) * nl * n)
    return out
