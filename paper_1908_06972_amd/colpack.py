"""The paper's own column-packed encrypted inference (Sec. 4.1, the matrix
packing of the prediction task; Alg. 1 steps 2-3) as a sequence of libpft
calls; every step runs in the HIP kernels.

H (m x n) is packed vertically: plaintext H_{c,j} holds rows c t .. c t + t-1
of column j (t = N/2 slots, n_in = ceil(m/t) input ciphertexts).  O (n x c)
is packed horizontally: plaintext O_j holds row j in slots 0 .. c-1.
  h_j = RESCALE(TotalSum(sum_c v_c H_{c,j}))     n TotalSums, n log2(t) rotations
  h_j = RESCALE(h_j (1/w))
  s   = RESCALE(sum_j h_j O_j)                   slot k of s = (h O)_k
Three levels.  The diagonal form of the same products is inference.py.
"""

import numpy as np


def column_slots(H, t):
    """[n][n_in][t]: slot vector of plaintext H_{c,j} at [j][c], zero padded."""
    m, n = H.shape
    n_in = -(-m // t)
    padded = np.zeros((n_in * t, n))
    padded[:m] = H
    return np.ascontiguousarray(padded.T.reshape(n, n_in, t))


def row_slots(O, t):
    """[1][n][t]: slot vector of plaintext O_j at [0][j]."""
    n, c = O.shape
    out = np.zeros((1, n, t))
    out[0, :, :c] = O
    return out


class ColPackModel:
    """Device plaintexts of both stages for inputs at `level`."""

    def __init__(self, ctx, H, O, level):
        t = ctx.params.n // 2
        self.t = t
        self.n_in = -(-H.shape[0] // t)
        self.dim, self.classes = H.shape[1], O.shape[1]
        self.stage1 = ctx.ptdot(column_slots(H, t), level)
        self.stage2 = ctx.ptdot(row_slots(O, t), level - 2)

    def rotation_steps(self):
        return [1 << i for i in range(self.t.bit_length() - 1)]


def encrypted_inference(ctx, model, inputs, words):
    """inputs: per document a list of model.n_in ciphertexts; words: per
    document the word count.  Returns one score ciphertext per document."""
    n = model.dim
    hs = ctx.ptdot_apply(model.stage1, inputs, n_sum=model.t)
    flat = ctx.rescale_batch([h for doc in hs for h in doc])
    flat = ctx.rescale_batch(ctx.mul_const_batch(flat, [1.0 / float(w) for w in words for _ in range(n)]))
    per_doc = [flat[d * n:(d + 1) * n] for d in range(len(inputs))]
    s = ctx.ptdot_apply(model.stage2, per_doc, n_sum=1)
    return ctx.rescale_batch([x[0] for x in s])
