"""Encrypted bag-of-words inference of PrivFT (Sec. 4.1, Alg. 1 steps 2-3)
as a sequence of libpft calls; every step runs in the HIP kernels.

Server side, per batch of documents (client input: the count vector v split
over n_in ciphertexts at the top level, and the word count w in plaintext):
  h = RESCALE(PtMatVec(H^T, v))      stage 1, v H
  h = RESCALE(h * (1/w))             the average
  s = RESCALE(PtMatVec(O^T, h))      stage 2, h O  (h is periodic with period n)
Three levels in total; the client decrypts s and reads class j at slot j.
"""

import numpy as np


class BowModel:
    """Plaintext weights H (vocab x dim) and O (dim x classes) as device
    plaintext matrices for a given top level."""

    def __init__(self, ctx, H, O, level, n_in=None):
        t = ctx.params.n // 2
        vocab, dim = H.shape
        classes = O.shape[1]
        self.n_in = n_in or -(-vocab // t)
        padded = np.zeros((self.n_in * t, dim))
        padded[:vocab] = H
        self.dim, self.classes, self.level, self.t = dim, classes, level, t
        self.stage1 = ctx.ptmat(padded.T, dim, t, self.n_in, level)
        O_pad = np.zeros((dim, classes if classes & (classes - 1) == 0 else 1 << classes.bit_length()))
        O_pad[:, :classes] = O
        self.c_pad = O_pad.shape[1]
        self.stage2 = ctx.ptmat(O_pad.T, self.c_pad, dim, 1, level - 2)

    @staticmethod
    def _steps(m):
        # the order pft_ptmatvec rotates in: baby steps, giant steps, then
        # the rotate-and-sum over the n_i / n_o blocks
        b, G = m.b, m.G
        out = list(range(1, b)) + [g * b for g in range(1, G)]
        s = m.n_o
        while s < m.n_i:
            out.append(s)
            s *= 2
        return out

    def rotation_steps(self):
        return sorted(set(self._steps(self.stage1) + self._steps(self.stage2)))

    def rotation_order(self):
        """The rotation steps of one inference in the order they run."""
        return self._steps(self.stage1) + self._steps(self.stage2)


def encrypted_inference(ctx, model, inputs, words):
    """inputs: per document a list of model.n_in ciphertexts; words: per
    document the word count w.  Returns one score ciphertext per document."""
    h = ctx.rescale_batch(ctx.ptmatvec(model.stage1, inputs))
    h = ctx.rescale_batch(ctx.mul_const_batch(h, [1.0 / float(w) for w in words]))
    return ctx.rescale_batch(ctx.ptmatvec(model.stage2, [[x] for x in h]))


def split_counts(counts, n_in, t):
    """Count vector (vocab,) -> n_in slot vectors of length t (zero padded)."""
    v = np.zeros(n_in * t)
    v[:len(counts)] = counts
    return [v[c * t:(c + 1) * t] for c in range(n_in)]
