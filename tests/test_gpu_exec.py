"""The op-list executor on the GPU: a mixed-level batch (the batched-primitives
configuration: N = 2^14, L = 8, 64 ciphertext pairs at levels 3..8, HMult+relin,
rescale, 16 rotation steps, additions and NTT/INTT) run by pft_exec_batch
equals the same list issued op by op, bit for bit, eagerly and replayed from
one HIP graph."""

import numpy as np
import pytest

import synth as S

pytestmark = pytest.mark.gpu

STEPS = (1, 2, 3, 5, 7, 11, 13, 17, 100, 257, 1000, 2047, 4096, 5000, 8000, -1)


def _setup(torch):
    import paper_1908_06972_amd.ckks as L
    cfg = S.CONFIGS["C2"]
    lp = L.Params.from_config(cfg)
    side = torch.cuda.Stream()
    ctx = L.Context(lp, stream=side)
    n = lp.n
    kd = S.key_draws(7, n, lp.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    a, e = S.switch_key_draws(7, 0, n, lp.key_moduli(), lp.dnum)
    ctx.gen_relin_key(a, e)
    for st in STEPS:
        a, e = S.switch_key_draws(7, 1000 + (st % (n // 2)), n, lp.key_moduli(), lp.dnum)
        ctx.gen_rotation_key(st, a, e)
    return L, lp, ctx, side


def _inputs(ctx, lp, n_pairs):
    n = lp.n
    cts = []
    for i in range(n_pairs):
        lvl = 3 + i % 6
        for k in range(2):
            d = S.enc_draws(900 + 2 * i + k, n)
            cts.append(ctx.encrypt(S.plaintext_coeffs(S.rng(1900 + 2 * i + k), n, 2 ** 30), lvl, lp.scale,
                                   d.v, d.e0, d.e1))
    return cts


def _op_list(ctx, inputs):
    """Per pair i: m = a*b, r = rescale(m), t = rotate(r, step_i), s = t + r;
    every 4th pair also round-trips a copy of a through NTT/INTT."""
    cts = list(inputs)
    ops = []
    n_pairs = len(inputs) // 2
    for i in range(n_pairs):
        a, b = 2 * i, 2 * i + 1
        lvl = inputs[a].level
        m, r, t, s = len(cts), len(cts) + 1, len(cts) + 2, len(cts) + 3
        cts += [ctx.empty_ct(lvl), ctx.empty_ct(lvl - 1), ctx.empty_ct(lvl - 1), ctx.empty_ct(lvl - 1)]
        ops += [("mul_relin", a, b, m, 0, 0), ("rescale", m, 0, r, 0, 0),
                ("rotate", r, 0, t, STEPS[i % len(STEPS)], 0), ("add", t, r, s, 0, 0)]
        if i % 4 == 0:
            x = len(cts)
            cts.append(ctx.empty_ct(lvl))
            cts[x].data.copy_(inputs[a].data)
            cts[x].level, cts[x].scale = inputs[a].level, inputs[a].scale
            ops += [("ntt", x, 0, 0, 0, 0), ("intt", x, 0, 0, 0, 0)]
    return cts, ops


def _per_op(ctx, cts, ops):
    for kind, a, b, out, step, mode in ops:
        if kind == "mul_relin":
            ctx.mul_relin(cts[a], cts[b], out=cts[out])
        elif kind == "rescale":
            ctx.rescale(cts[a], mode, out=cts[out])
        elif kind == "rotate":
            ctx.rotate(cts[a], step, out=cts[out])
        elif kind == "add":
            ctx.add(cts[a], cts[b], out=cts[out])
        elif kind == "ntt":
            ctx.ntt_forward(cts[a].data, cts[a].level)
        elif kind == "intt":
            ctx.ntt_inverse(cts[a].data, cts[a].level)


def _same(x, y):
    assert len(x) == len(y)
    for i, (p, q) in enumerate(zip(x, y)):
        assert p.level == q.level and p.scale == q.scale, i
        assert bool((p.data[:, :p.level] == q.data[:, :q.level]).all()), i


def test_exec_batch_equals_per_op(torch_cuda):
    torch = torch_cuda
    L, lp, ctx, side = _setup(torch)
    inputs = _inputs(ctx, lp, 64)
    ref, ops = _op_list(ctx, inputs)
    _per_op(ctx, ref, ops)
    got, ops2 = _op_list(ctx, inputs)
    assert ops2 == ops
    ctx.exec_batch(got, ops)
    ctx.synchronize()
    _same(got, ref)
    # the NTT -> INTT copies came back unchanged
    for kind, a, *_ in ops:
        if kind == "intt":
            assert bool((got[a].data == ref[a].data).all())

    # the same list captured once and replayed: every replay equals the eager result
    rep, _ = _op_list(ctx, inputs)
    ctx.exec_batch(rep, ops)            # sizes the side-stream workspaces outside the capture
    ctx.synchronize()
    for c in rep[len(inputs):]:
        with torch.cuda.stream(side):
            c.data.zero_()
    graph = ctx.capture(lambda: ctx.exec_batch(rep, ops))
    for k in range(3):
        with torch.cuda.stream(side):
            for c in rep[len(inputs):]:
                c.data.fill_(k)
        # the NTT/INTT copies are transformed in place: restore them first
        for kind, a, *_ in ops:
            if kind == "ntt":
                with torch.cuda.stream(side):
                    rep[a].data.copy_(ref[a].data)
        graph.launch()
        ctx.synchronize()
        _same(rep, ref)
    graph.close()
    ctx.close()


def test_exec_batch_errors(torch_cuda):
    import paper_1908_06972_amd.native as N
    torch = torch_cuda
    L, lp, ctx, side = _setup(torch)
    inputs = _inputs(ctx, lp, 2)    # levels 3 and 4
    out = ctx.empty_ct(4)
    cts = inputs + [out]
    with pytest.raises(N.PftError) as e:
        ctx.exec_batch(cts, [("mul_relin", 0, 2, 4, 0, 0)])   # levels 3 and 4
    assert e.value.code == N.PFT_ELEVEL
    with pytest.raises(N.PftError) as e:
        ctx.exec_batch(cts, [("rotate", 0, 0, 0, 1, 0)])      # output aliases input
    assert e.value.code == N.PFT_EINVAL
    with pytest.raises(N.PftError) as e:
        ctx.exec_batch(cts, [("add", 0, 1, 9, 0, 0)])          # index out of range
    assert e.value.code == N.PFT_EINVAL
    ctx.close()
