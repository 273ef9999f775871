"""Seeded random draws (numpy PCG64 via default_rng).  No scheme arithmetic.

Conventions (both sides receive exactly these arrays):
  * secret s: ternary, uniform over {-1, 0, 1} (the paper's X_key, read as
    uniform ternary), int64 [N].
  * errors: zero-centred rounded Gaussian with sigma = 3.2 (Sec. 6.4), cut at
    |e| <= 19 (6 sigma), int64.
  * uniform masks: per modulus, uniform over [0, q), uint64 [limbs, N],
    in coefficient form.
  * encryption randomness v: ternary; e0, e1: errors.
"""

import numpy as np

SIGMA = 3.2
ERR_BOUND = 19

__all__ = [
    "rng", "ternary", "gaussian", "uniform_mod", "slots_uniform", "slots_unit",
    "plaintext_coeffs", "KeyDraws", "key_draws", "EncDraws", "enc_draws",
    "switch_key_draws", "SIGMA", "ERR_BOUND", "bow_documents", "bow_weights",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def ternary(g: np.random.Generator, n: int) -> np.ndarray:
    return g.integers(-1, 2, size=n, dtype=np.int64)


def gaussian(g: np.random.Generator, n: int, sigma: float = SIGMA, bound: int = ERR_BOUND) -> np.ndarray:
    x = np.rint(g.normal(0.0, sigma, size=n))
    return np.clip(x, -bound, bound).astype(np.int64)


def uniform_mod(g: np.random.Generator, moduli, n: int) -> np.ndarray:
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[i] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def slots_uniform(g: np.random.Generator, n_slots: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Complex slots with real and imaginary parts uniform in [lo, hi]."""
    return g.uniform(lo, hi, n_slots) + 1j * g.uniform(lo, hi, n_slots)


def slots_unit(g: np.random.Generator, n_slots: int) -> np.ndarray:
    """Unit-modulus complex slots e^{i theta}, theta uniform in [0, 2 pi)."""
    return np.exp(1j * g.uniform(0.0, 2.0 * np.pi, n_slots))


def plaintext_coeffs(g: np.random.Generator, n: int, bound: int) -> np.ndarray:
    """Integer plaintext polynomial with coefficients uniform in [-bound, bound].

    The bit-exact parity tests drive both sides with integer plaintexts drawn
    here, so that no encoder (a floating-point step) sits between the shared
    input and the compared residues."""
    return g.integers(-bound, bound + 1, size=n, dtype=np.int64)


class KeyDraws:
    """Randomness of KEYGEN: s, the public-key mask/error, and per switching key
    (relinearisation or rotation) the per-digit masks and errors."""

    def __init__(self, s, pk_a, pk_e):
        self.s = s
        self.pk_a = pk_a
        self.pk_e = pk_e


def key_draws(seed: int, n: int, q_moduli) -> KeyDraws:
    g = rng(seed)
    s = ternary(g, n)
    pk_a = uniform_mod(g, q_moduli, n)
    pk_e = gaussian(g, n)
    return KeyDraws(s, pk_a, pk_e)


def switch_key_draws(seed: int, key_id: int, n: int, all_moduli, dnum: int):
    """(a [dnum, L+K, N] uniform, e [dnum, N] errors) for one switching key.
    key_id separates the streams of different keys drawn from one seed."""
    g = np.random.default_rng([seed, 0x5157, key_id])
    a = np.stack([uniform_mod(g, all_moduli, n) for _ in range(dnum)])
    e = np.stack([gaussian(g, n) for _ in range(dnum)])
    return a, e


class EncDraws:
    def __init__(self, v, e0, e1):
        self.v = v
        self.e0 = e0
        self.e1 = e1


def enc_draws(seed: int, n: int) -> EncDraws:
    g = rng(seed)
    return EncDraws(ternary(g, n), gaussian(g, n), gaussian(g, n))


def bow_documents(seed: int, n_docs: int, vocab: int, w_min: int = 50, w_max: int = 500):
    """Bag-of-words count vectors: per document a length w ~ U{w_min..w_max},
    w tokens drawn as Zipf ranks r in 1..vocab with P(r) proportional to 1/r
    (inverse-CDF sampling), mapped to word indices through a fixed seeded
    permutation of the vocabulary.  Returns (counts [n_docs, vocab] int64,
    w [n_docs] int64)."""
    g = rng(seed)
    perm = np.random.default_rng([seed, 7]).permutation(vocab)
    cdf = np.cumsum(1.0 / np.arange(1, vocab + 1))
    cdf /= cdf[-1]
    counts = np.zeros((n_docs, vocab), dtype=np.int64)
    lengths = g.integers(w_min, w_max + 1, size=n_docs)
    for d in range(n_docs):
        ranks = np.searchsorted(cdf, g.random(int(lengths[d])), side="right")
        np.add.at(counts[d], perm[np.minimum(ranks, vocab - 1)], 1)
    return counts, lengths.astype(np.int64)


def bow_weights(seed: int, vocab: int, dim: int, classes: int, sigma: float = 0.1):
    """Embedding H [vocab, dim] and classifier O [dim, classes], entries
    N(0, sigma^2) in fp64."""
    g = rng(seed)
    return g.normal(0.0, sigma, (vocab, dim)), g.normal(0.0, sigma, (dim, classes))
