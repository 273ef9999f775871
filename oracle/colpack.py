"""Oracle of the paper's own column-packed encrypted inference -- TEST
INFRASTRUCTURE ONLY (imported by tests/ and nothing else).

What is computed (Sec. 4.1, the matrix packing of the prediction task and
its figure; Alg. 1 steps 2-3): the client's count vector v (length m) is
split over n_in = ceil(m/t) ciphertexts of t = N/2 slots.  The server holds
the hidden matrix H (m x n) packed vertically -- plaintext H_{c,j} holds
rows c t .. c t + t - 1 of column j -- and the output matrix O (n x c)
packed horizontally -- plaintext O_j holds row j of O in slots 0 .. c-1:

  h_j = TotalSum( sum_c v_c * H_{c,j} )     one TotalSum per column (Alg. 2),
                                             so h_j sits in every slot
  h_j = RESCALE(h_j);  h_j = RESCALE(h_j * (1/w))
  s   = RESCALE( sum_j h_j * O_j )           slot k of s = (h O)_k

Three levels; n HMULPLAIN-sums and n TotalSums (n log2 t rotations) for
stage 1, n HMULPLAIN for stage 2.  Plaintexts are integer polynomials at
scale q_{level-1} of the level they are used at (the diagonal form of the
same products is in ptmatvec.py).
"""

import numpy as np

from . import ckks as C


def column_slots(H, t):
    """Slot vectors of the vertically packed H: [n][n_in][t], zero padded."""
    m, n = H.shape
    n_in = -(-m // t)
    out = np.zeros((n, n_in, t))
    for j in range(n):
        col = np.zeros(n_in * t)
        col[:m] = H[:, j]
        out[j] = col.reshape(n_in, t)
    return out


def row_slots(O, t):
    """Slot vectors of the horizontally packed O: [n][t], row j in slots 0..c-1."""
    n, c = O.shape
    out = np.zeros((n, t))
    out[:, :c] = O
    return out


def dot_plain(params, inputs, plains, pt_scale):
    """sum_j HMULPLAIN(inputs[j], plains[j]) (HADD of the products)."""
    acc = None
    for x, p in zip(inputs, plains):
        term = C.hmul_plain(params, x, p, pt_scale)
        acc = term if acc is None else C.hadd(params, acc, term)
    return acc


def stage1(params, inputs, plains, pt_scale, rot_keys):
    """h_j = TotalSum(sum_c v_c H_{c,j}) for every column j; plains[j][c]."""
    t = params.n // 2
    return [C.total_sum(params, dot_plain(params, inputs, pj, pt_scale), t, rot_keys) for pj in plains]


def stage2(params, hs, plains, pt_scale):
    """s = sum_j h_j O_j; plains[j]."""
    return dot_plain(params, hs, plains, pt_scale)


def inference(params, inputs, plains_h, scale_h, plains_o, scale_o, w, rot_keys, const_plain):
    """The whole server side; const_plain(params, value, level) gives the
    integer constant polynomial for 1/w and its scale."""
    hs = [C.rescale(params, h) for h in stage1(params, inputs, plains_h, scale_h, rot_keys)]
    m, ms = const_plain(params, 1.0 / w, hs[0].level)
    hs = [C.rescale(params, C.hmul_plain(params, h, m, ms)) for h in hs]
    return C.rescale(params, stage2(params, hs, plains_o, scale_o))
