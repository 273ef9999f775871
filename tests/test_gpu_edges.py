"""Edge cases of the batched entry points on the GPU: batches longer than
one launch holds (64 ciphertexts per launch), empty batches, and the
rotation by a multiple of N/2 slots (the identity, R20)."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C

pytestmark = pytest.mark.gpu

SMALL = dict(log_n=12, n_q=3, q0_bits=60, q_bits=40, n_p=1, p_bits=60, dnum=3, scale=2 ** 40)
N_ITEMS = 70  # more than the 64 ciphertexts of one batched launch


@pytest.fixture(scope="module")
def world(torch_cuda):
    import paper_1908_06972_amd.ckks as L
    op = C.Params(**SMALL)
    lp = L.Params(*SMALL.values())
    C.set_mul_mode(1)
    ctx = L.Context(lp)
    n = op.n
    kd = S.key_draws(29, n, op.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    a, e = S.switch_key_draws(29, 0, n, op.key_moduli(), op.dnum)
    ctx.gen_relin_key(a, e)
    ra, re = S.switch_key_draws(29, 5003, n, op.key_moduli(), op.dnum)
    ctx.gen_rotation_key(3, ra, re)
    pk = C.public_key(op, kd.s, kd.pk_a, kd.pk_e)
    keys = {"rlk": C.relin_key(op, kd.s, a, e), 3: C.rotation_key(op, kd.s, 3, ra, re)}
    pairs = []
    for i in range(N_ITEMS):
        m = S.plaintext_coeffs(S.rng(2900 + i), n, 2 ** 30)
        d = S.enc_draws(2950 + i, n)
        pairs.append((ctx.encrypt(m, op.L, op.scale, d.v, d.e0, d.e1),
                      C.encrypt(op, pk, m, op.L, d.v, d.e0, d.e1, op.scale)))
    return op, ctx, keys, pairs


def _same(ctx, g, o):
    host = ctx.export(g)
    return np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)


def test_batches_longer_than_one_launch(world):
    op, ctx, keys, pairs = world
    g = [p[0] for p in pairs]
    muls = ctx.mul_relin_batch(g, g[::-1])
    rss = ctx.rescale_batch(muls)
    rots = ctx.rotate_batch(rss, 3)
    for i in (0, 63, 64, N_ITEMS - 1):  # both sides of the launch boundary
        o = C.rotate(op, C.rescale(op, C.hmul_relin(op, pairs[i][1], pairs[N_ITEMS - 1 - i][1], keys["rlk"])), 3,
                     keys[3])
        assert _same(ctx, rots[i], o), i
    # every item equals its own single-ciphertext computation
    for i in range(N_ITEMS):
        single = ctx.rotate(ctx.rescale(ctx.mul_relin(g[i], g[N_ITEMS - 1 - i])), 3)
        assert bool((single.data == rots[i].data).all()), i


def test_empty_batches(world):
    op, ctx, keys, pairs = world
    assert ctx.mul_relin_batch([], []) == []
    assert ctx.rescale_batch([]) == []
    assert ctx.rotate_batch([], 3) == []
    ctx.synchronize()


def test_rotation_by_a_multiple_of_half_n_is_the_identity(world):
    op, ctx, keys, pairs = world
    g, o = pairs[5]
    half = op.n // 2
    for step in (0, half, -half, 3 * half):
        r = ctx.rotate(g, step)  # no key for these steps is needed
        assert r.level == g.level and r.scale == g.scale
        assert bool((r.data == g.data).all()), step
        assert _same(ctx, r, o)
    outs = ctx.rotate_batch([p[0] for p in pairs[:3]], half)
    for (gi, _), r in zip(pairs[:3], outs):
        assert bool((r.data == gi.data).all())
