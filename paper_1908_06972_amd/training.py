"""The predict step of PrivFT training with encrypted weights (Sec. 4.2) and
its degree-2 softmax approximation, as a sequence of libpft calls; every
step runs in the HIP kernels.

Per batch of documents (client input: the count vector v split over n_in
ciphertexts at level l, the word count w; model: the pre-rotated diagonals
of H^T and O^T, encrypted by the model owner at scale q_{l-1} and
q_{l-3}, levels l and l-2):
  h = RESCALE(CtMatVec(E_H, v))        stage 1, v H with HMUL
  h = RESCALE(h * (1/w))               the average (HMULPLAIN by a constant)
  s = RESCALE(CtMatVec(E_O, h))        stage 2, h O with HMUL
  y = (s + 2)^2 / 8 - 1/4              = s^2/8 + s/2 + 1/4, the softmax
                                         approximation: two more levels
Five levels in all; slot j of y holds the approximated softmax input of
class j.
"""

from .inference import split_counts  # noqa: F401  (same client-side input layout)


def bsgs_plan(n_o, n_in=1):
    """(b, G), the plan rule of pft_ptmatvec / pft_ctmatvec: the power of two
    b minimising n_in (b - 1) + (n_o / b - 1) rotations, larger b on ties;
    G = n_o / b."""
    best = None
    bb = 1
    while bb <= n_o:
        cost = n_in * (bb - 1) + n_o // bb - 1
        if best is None or cost <= best[0]:
            best = (cost, bb)
        bb *= 2
    return best[1], n_o // best[1]


def rotation_steps(n_o, n_i, n_in=1):
    """Rotation keys a product with n_o outputs over period n_i and n_in
    input ciphertexts needs."""
    b, G = bsgs_plan(n_o, n_in)
    steps = list(range(1, b)) + [g * b for g in range(1, G)]
    s = n_o
    while s < n_i:
        steps.append(s)
        s *= 2
    return steps


def encrypt_diagonals(ctx, M, n_o, n_i, n_in, level, draws):
    """Client side: encode the pre-rotated diagonals of M at scale q_{level-1}
    and encrypt each at `level`; draws() yields the encryption randomness
    (v, e0, e1) of one ciphertext.  Flat list in [n_in][G][b] order."""
    p = ctx.params
    qs = float(p.q[level - 1])
    plains = p.diagonals_encode(M, n_o, n_i, n_in, qs)
    out = []
    for m in plains.reshape(-1, p.n):
        v, e0, e1 = draws()
        out.append(ctx.encrypt(m, level, qs, v, e0, e1))
    return out


def softmax_approx(ctx, cts):
    """X^2/8 + X/2 + 1/4 on a batch of ciphertexts, evaluated as
    (X + 2)^2 / 8 - 1/4 so that only equal scales are added."""
    n = len(cts)
    a = ctx.add_const_batch(cts, [2.0] * n)
    b = ctx.rescale_batch(ctx.mul_relin_batch(a, a))
    c = ctx.rescale_batch(ctx.mul_const_batch(b, [0.125] * n))
    return ctx.add_const_batch(c, [-0.25] * n)


class EncryptedBowModel:
    """Encrypted diagonals of H^T (dim x vocab) and O^T (classes x dim):
    flat lists in [n_in][G][b] order, as pft_ctmatvec takes them."""

    def __init__(self, stage1, stage2, dim, classes, n_in, t):
        self.stage1, self.stage2 = stage1, stage2
        self.dim, self.classes, self.n_in, self.t = dim, classes, n_in, t


def predict_encrypted(ctx, model, inputs, words):
    """inputs: per document a list of model.n_in ciphertexts; words: per
    document the word count.  Returns one ciphertext per document."""
    m = model
    h = ctx.rescale_batch(ctx.ctmatvec(m.stage1, m.dim, m.t, m.n_in, inputs))
    h = ctx.rescale_batch(ctx.mul_const_batch(h, [1.0 / float(w) for w in words]))
    s = ctx.rescale_batch(ctx.ctmatvec(m.stage2, m.classes, m.dim, 1, [[x] for x in h]))
    return softmax_approx(ctx, s)
