"""Oracle of the encrypted-weight forward pass of PrivFT training and of its
degree-2 softmax approximation -- TEST INFRASTRUCTURE ONLY (imported by
tests/ and nothing else).

What is computed (Sec. 4.2, the predict step of minibatch training): the
same two vector-matrix products as inference (Sec. 4.1, Alg. 1 steps 2-3),
but with the weight matrices encrypted, so every diagonal product is a
ciphertext-ciphertext HMUL instead of HMULPLAIN; then the softmax is replaced
by the polynomial X^2/8 + X/2 + 1/4 (Sec. 4.2, one HMUL).

Encrypted matrix x encrypted vector (diagonal method, baby-step/giant-step;
the same plan and pre-rotation as the plaintext-matrix oracle in
ptmatvec.py, with the pre-rotated diagonals E^c_{g,r} encrypted):

  u = sum_g rot( Relin( sum_c sum_r E^c_{g,r} (x) rot(v_c, r) ), g b )
  y = u + rot(u, n_o) + ... (steps n_o 2^s while n_o 2^s < n_i)

where (x) is the HMUL tensor (d0, d1, d2) and the tensors of one giant step
are added before a single relinearisation (relinearisation is linear in d2
up to its own rounding, so this is one key switch per giant step instead of
one per diagonal).  Slot k of y holds (M v)_{k mod n_o}.

Softmax approximation: X^2/8 + X/2 + 1/4 = (X + 2)^2 / 8 - 1/4 (an identity
of polynomials), evaluated as
  a = X + 2                    (HADDPLAIN of a constant at X's scale)
  b = RESCALE(HMUL+relin(a, a))
  c = RESCALE(b * (1/8))       (constant at scale q_{level-1}, as for 1/w)
  y = c - 1/4                  (HADDPLAIN of a constant at c's scale)
which adds ciphertexts of equal scale only; two levels.

A constant plaintext at scale S is the integer polynomial round(value * S) at
X^0 (product in double precision, rounded half away from zero): every slot of
its encoding equals value at scale S.
"""

import numpy as np

from . import ckks as C
from .ptmatvec import bsgs_plan


def constant_at_scale(params, value, scale):
    """round(value * scale) at X^0 as an integer polynomial (half away from
    zero, product in double precision)."""
    x = float(value) * float(scale)
    m = int(np.floor(x + 0.5)) if x >= 0 else -int(np.floor(-x + 0.5))
    if abs(m) >= 1 << 62:
        raise ValueError("constant exceeds 2^62 at this scale")
    out = np.zeros(params.n, dtype=np.int64)
    out[0] = m
    return out


def hadd_const(params, x, value):
    """HADDPLAIN of the constant `value` encoded at x's own scale (Sec. 3.4)."""
    return C.hadd_plain(params, x, constant_at_scale(params, value, x.scale))


def _tensor_sum(params, pairs):
    """sum over (e, v) of the HMUL tensors e (x) v, residue-wise mod q."""
    level = pairs[0][0].level
    mods = params.q[:level]
    acc = None
    for e, v in pairs:
        t = C.tensor(params, e, v)
        acc = t if acc is None else tuple(C.add(a, b, mods) for a, b in zip(acc, t))
    return acc


def relin_tensor(params, d, rlk, scale):
    """Relinearise a tensor (d0, d1, d2) at `scale`: (d0 + ks0, d1 + ks1)."""
    d0, d1, d2 = d
    level = d0.shape[0]
    mods = params.q[:level]
    k0, k1 = C.key_switch(params, d2, rlk, level)
    return C.Ciphertext(C.add(d0, k0, mods), C.add(d1, k1, mods), scale)


def ctmatvec(params, inputs, diags, n_o, n_i, rlk, rot_keys):
    """Encrypted-weight BSGS matrix-vector product.  inputs[c]: ciphertexts
    of the vector parts; diags[c][g][r]: ciphertexts of the pre-rotated
    diagonals, all at the inputs' level and of equal scale.  No rescale:
    the result has scale diag scale x input scale."""
    b, G = bsgs_plan(n_o, len(inputs))
    baby = [[v if r == 0 else C.rotate(params, v, r, rot_keys[r]) for r in range(b)] for v in inputs]
    scale = diags[0][0][0].scale * inputs[0].scale
    total = None
    for g in range(G):
        pairs = [(diags[c][g][r], baby[c][r]) for c in range(len(inputs)) for r in range(b)]
        acc = relin_tensor(params, _tensor_sum(params, pairs), rlk, scale)
        if g:
            acc = C.rotate(params, acc, g * b, rot_keys[g * b])
        total = acc if total is None else C.hadd(params, total, acc)
    s = n_o
    while s < n_i:
        total = C.hadd(params, total, C.rotate(params, total, s, rot_keys[s]))
        s *= 2
    return total


def softmax_approx(params, x, rlk):
    """(X + 2)^2 / 8 - 1/4 = X^2/8 + X/2 + 1/4 (Sec. 4.2), two levels."""
    a = hadd_const(params, x, 2.0)
    b = C.rescale(params, C.hmul_relin(params, a, a, rlk))
    qs = float(params.q[b.level - 1])
    c = C.rescale(params, C.hmul_plain(params, b, constant_at_scale(params, 0.125, qs), qs))
    return hadd_const(params, c, -0.25)


def softmax_approx_plain(x):
    """The approximation polynomial in fp64."""
    x = np.asarray(x, dtype=np.float64)
    return x * x / 8.0 + x / 2.0 + 0.25


def predict_encrypted(params, inputs, H_diags, O_diags, n_dim, n_cls, w, rlk, rot_keys):
    """The predict step with encrypted weights (Sec. 4.2): h = v H (stage 1),
    h * (1/w), s = h O (stage 2, diagonals at two levels below the input),
    then the softmax approximation; one RESCALE after each product.  Five
    levels in all."""
    t = params.n // 2
    h = C.rescale(params, ctmatvec(params, inputs, H_diags, n_dim, t, rlk, rot_keys))
    qs = float(params.q[h.level - 1])
    h = C.rescale(params, C.hmul_plain(params, h, constant_at_scale(params, 1.0 / w, qs), qs))
    s = C.rescale(params, ctmatvec(params, [h], O_diags, n_cls, n_dim, rlk, rot_keys))
    return softmax_approx(params, s, rlk)
