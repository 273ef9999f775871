"""Oracle of the plaintext-matrix x ciphertext-vector product (PtMatVec) and
of the encrypted bag-of-words inference built on it -- TEST INFRASTRUCTURE
ONLY (imported by tests/, smoke and the benchmark's CPU baseline).

What is computed (Sec. 4.1): the server evaluates h = (1/w) v H and
s = h O (Alg. 1, steps 2 and 3) on the encrypted count vector v with the
plaintext embedding matrix H (m x n) and classifier O (n x c), using only
HMULPLAIN, HADD and ROTATE; the client decrypts s and applies softmax/argmax.

The matrix-vector product uses the diagonal method in baby-step/giant-step
form.  For a matrix M with n_o rows acting on a vector laid out in slots with
period n_i (n_o divides n_i, n_i divides t = number of slots), split over
n_in input ciphertexts:

  D^c_i[k]  = M[k mod n_o, c n_i + (k + i) mod n_i]          (i < n_o)
  u         = sum_c sum_i D^c_i * rot(v_c, i)
  y         = u + rot(u, n_o) + rot(., 2 n_o) ...             (log2(n_i/n_o) steps)

so slot k of y holds (M v)_{k mod n_o}.  With i = g b + r (b baby steps,
G = n_o / b giant steps) and pre-rotated diagonals
P^c_{g,r} = rot(D^c_{g b + r}, -g b):

  u = sum_g rot( sum_c sum_r P^c_{g,r} * rot(v_c, r), g b ).

Plan rule (shared convention, stated here and in the library header): b
minimises the rotations of one product, n_in (b - 1) + (G - 1) with
G = n_o / b, the larger b on ties (b = 2^ceil(log2(n_o)/2) for one input
ciphertext).  Rotation steps used: 1..b-1, g b for 1 <= g < G, and
n_o 2^s for s < log2(n_i/n_o).
"""

import math

import numpy as np

from . import ckks as C


def bsgs_plan(n_o: int, n_in: int = 1):
    """(b, G) for n_o diagonals over n_in input ciphertexts, both powers of
    two, b * G = n_o: the b that minimises the rotations of one product,
    n_in (b - 1) + (G - 1), the larger b on ties (for n_in = 1,
    b = 2^ceil(log2(n_o)/2))."""
    if n_o < 1 or n_o & (n_o - 1):
        raise ValueError("n_o must be a power of two")
    cands = [1 << k for k in range(int(math.log2(n_o)) + 1)]
    b = min(cands, key=lambda bb: (n_in * (bb - 1) + n_o // bb - 1, -bb))
    return b, n_o // b


def rotation_steps(n_o: int, n_i: int, n_in: int = 1):
    b, G = bsgs_plan(n_o, n_in)
    steps = list(range(1, b)) + [g * b for g in range(1, G)]
    s = n_o
    while s < n_i:
        steps.append(s)
        s *= 2
    return steps


def diagonal(M, n_o, n_i, c, i, t):
    """D^c_i as a length-t real vector (periodic with period n_i)."""
    k = np.arange(t)
    return M[k % n_o, c * n_i + (k + i) % n_i]


def prerotated_diagonals(M, n_o, n_i, n_in, t):
    """P[c][g][r] = rot(D^c_{g b + r}, -g b) as length-t real vectors, where
    rot(x, s)[k] = x[(k + s) mod t] (left rotation by s)."""
    b, G = bsgs_plan(n_o, n_in)
    out = []
    for c in range(n_in):
        per_c = []
        for g in range(G):
            per_g = []
            for r in range(b):
                d = diagonal(M, n_o, n_i, c, g * b + r, t)
                per_g.append(np.roll(d, g * b))  # rot(d, -g b)[k] = d[k - g b]
            per_c.append(per_g)
        out.append(per_c)
    return out


def slot_bsgs(P, vs, n_o, n_i):
    """The BSGS evaluation on plain slot vectors (numpy), the same sequence
    of rotations, products and sums as the encrypted evaluation."""
    b, G = bsgs_plan(n_o, len(vs))
    rot = lambda x, s: np.roll(x, -s)  # noqa: E731  (left rotation by s)
    baby = [[v if r == 0 else rot(v, r) for r in range(b)] for v in vs]
    total = None
    for g in range(G):
        acc = sum(P[c][g][r] * baby[c][r] for c in range(len(vs)) for r in range(b))
        if g:
            acc = rot(acc, g * b)
        total = acc if total is None else total + acc
    s = n_o
    while s < n_i:
        total = total + rot(total, s)
        s *= 2
    return total


def ptmatvec(params, inputs, plains, n_o, n_i, rot_keys, pt_scale):
    """Encrypted BSGS PtMatVec: inputs[c] ciphertexts, plains[c][g][r]
    integer plaintext polynomials (pre-rotated diagonals encoded at pt_scale),
    rot_keys {step: SwitchKey}.  No rescale."""
    b, G = bsgs_plan(n_o, len(inputs))
    baby = [[v if r == 0 else C.rotate(params, v, r, rot_keys[r]) for r in range(b)] for v in inputs]
    total = None
    for g in range(G):
        acc = None
        for c in range(len(inputs)):
            for r in range(b):
                term = C.hmul_plain(params, baby[c][r], plains[c][g][r], pt_scale)
                acc = term if acc is None else C.hadd(params, acc, term)
        if g:
            acc = C.rotate(params, acc, g * b, rot_keys[g * b])
        total = acc if total is None else C.hadd(params, total, acc)
    s = n_o
    while s < n_i:
        total = C.hadd(params, total, C.rotate(params, total, s, rot_keys[s]))
        s *= 2
    return total


def constant_plain(params, value, level):
    """Integer constant polynomial round(value * q_{level-1}), the product
    taken in double precision and rounded half away from zero (every slot
    equals value at scale q_{level-1}), and that scale."""
    qs = float(params.q[level - 1])
    x = value * qs
    m = int(np.floor(x + 0.5)) if x >= 0 else -int(np.floor(-x + 0.5))  # round half away from zero
    return np.array([m] + [0] * (params.n - 1), dtype=np.int64), qs


def inference_plain(v, H, O, w):
    """Alg. 1 steps 2-3 in fp64: h = (1/w) v H, s = h O."""
    h = (v @ H) / w
    return h @ O
