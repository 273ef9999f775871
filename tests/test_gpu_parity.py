"""Bit-exact parity of the HIP path (through the C ABI) with the oracle.

Every ciphertext the library produces is exported in coefficient form and
compared residue by residue with the oracle's result on the same seeded
draws.  Levels are chosen so that the last key-switching digit is both full
and ragged (level not a multiple of alpha)."""

import numpy as np
import pytest

import synth as S
from oracle import _ring
from oracle import ckks as C
from tests.gpu_env import World

pytestmark = pytest.mark.gpu


# ---------------------------------------------------------------------------
# the transform (row a1/a2): forward/inverse NTT against the oracle definition
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_ntt_forward_inverse(torch_cuda, log_n):
    import paper_1908_06972_amd.ckks as L
    lp = L.Params(log_n, 5, 60, 50, 1, 60, 2, 2 ** 40)
    op = C.Params(log_n, 5, 60, 50, 1, 60, 2, 2 ** 40)
    assert lp.q == op.q
    ctx = L.Context(lp)
    n, n_polys, n_limbs = 1 << log_n, 3, 5
    g = np.random.default_rng(log_n)
    host = np.stack([np.stack([g.integers(0, q, n, dtype=np.uint64) for q in op.q]) for _ in range(n_polys)])
    dev = L.to_device_u64(host, ctx.device)
    ctx.ntt_forward(dev, n_limbs)
    fwd = L.to_host_u64(dev)
    for p in range(n_polys):
        for i, q in enumerate(op.q):
            want = np.empty(n, dtype=np.uint64)
            _ring.lib().or_ntt_fast(_ring.ptr(np.ascontiguousarray(host[p, i])), _ring.ptr(want), n, q,
                                    op.psi[q])
            assert np.array_equal(fwd[p, i], want), (p, i)
    ctx.ntt_inverse(dev, n_limbs)
    assert np.array_equal(L.to_host_u64(dev), host)


def _oracle_ntt(op, host):
    n = host.shape[-1]
    out = np.empty_like(host)
    for p in range(host.shape[0]):
        for i in range(host.shape[1]):
            q = op.q[i]
            _ring.lib().or_ntt_fast(_ring.ptr(np.ascontiguousarray(host[p, i])), _ring.ptr(out[p, i]), n, q,
                                    op.psi[q])
    return out


@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_ntt_every_schedule(torch_cuda, log_n):
    """Every candidate pass schedule (integer limbs: the 60-bit q0; fp64
    limbs: the 50- and 40-bit primes) gives the oracle's transform and
    round-trips, on random rows plus all-(q-1) and spike rows."""
    import paper_1908_06972_amd.ckks as L
    lp = L.Params(log_n, 4, 60, 50, 1, 40, 2, 2 ** 40)
    op = C.Params(log_n, 4, 60, 50, 1, 40, 2, 2 ** 40)
    assert lp.q == op.q
    ctx = L.Context(lp)
    n = 1 << log_n
    g = np.random.default_rng(100 + log_n)
    host = np.stack([np.stack([g.integers(0, q, n, dtype=np.uint64) for q in op.q]) for _ in range(3)])
    for i, q in enumerate(op.q):
        host[1, i] = q - 1
        host[2, i] = 0
        host[2, i, (7 * i + 1) % n] = q - 1
    want = _oracle_ntt(op, host)
    cands = ctx.ntt_candidates()
    assert len(cands) >= 4 and all(sum(c[0]) == log_n for c in cands)
    for sched in cands:
        ctx.ntt_set_schedule(False, sched)
        ctx.ntt_set_schedule(True, sched)
        assert ctx.ntt_get_schedule(False, 12) == sched
        dev = L.to_device_u64(host, ctx.device)
        ctx.ntt_forward(dev, len(op.q))
        assert np.array_equal(L.to_host_u64(dev), want), sched
        ctx.ntt_inverse(dev, len(op.q))
        assert np.array_equal(L.to_host_u64(dev), host), sched


def test_ntt_autotune_picks_a_candidate(torch_cuda):
    import paper_1908_06972_amd.ckks as L
    import paper_1908_06972_amd.native as N
    lp = L.Params(14, 4, 60, 50, 1, 60, 2, 2 ** 40)
    ctx = L.Context(lp)
    cands = ctx.ntt_candidates()
    for inv in (False, True):
        for limbs in (1, 40, 5000):
            assert ctx.ntt_get_schedule(inv, limbs) in cands
    ctx.ntt_autotune(False)
    assert ctx.ntt_get_schedule(False, 40) == cands[0]
    with pytest.raises(N.PftError):
        ctx.ntt_set_schedule(False, ((7, 6, 1), 0))
    with pytest.raises(N.PftError):
        ctx.ntt_set_schedule(False, ((8, 8), 0))
    with pytest.raises(N.PftError):
        ctx.ntt_set_schedule(False, ((7, 7), 4))
    ctx.ntt_set_schedule(True, cands[-1])
    assert ctx.ntt_get_schedule(True, 7) == cands[-1]
    ctx.ntt_set_schedule(True, None)


@pytest.mark.parametrize("bits", [(60, 60, 60), (60, 50, 60), (40, 40, 50)])
def test_ntt_extreme_values(torch_cuda, bits):
    """All-zero, all q-1 and a single spike: exercises the lazy ranges of the
    integer butterflies (60-bit primes) and the fp64 bounds (<= 50 bits)."""
    import paper_1908_06972_amd.ckks as L
    lp = L.Params(16, 2, bits[0], bits[1], 1, bits[2], 1, 2 ** 40)
    op = C.Params(16, 2, bits[0], bits[1], 1, bits[2], 1, 2 ** 40)
    ctx = L.Context(lp)
    n = 1 << 16
    host = np.zeros((3, 2, n), dtype=np.uint64)
    for i, q in enumerate(op.q):
        host[1, i] = q - 1
        host[2, i, 12345] = q - 1
    dev = L.to_device_u64(host, ctx.device)
    ctx.ntt_forward(dev, 2)
    fwd = L.to_host_u64(dev)
    for p in range(3):
        for i, q in enumerate(op.q):
            want = np.empty(n, dtype=np.uint64)
            _ring.lib().or_ntt_fast(_ring.ptr(np.ascontiguousarray(host[p, i])), _ring.ptr(want), n, q, op.psi[q])
            assert np.array_equal(fwd[p, i], want)
    ctx.ntt_inverse(dev, 2)
    assert np.array_equal(L.to_host_u64(dev), host)


# ---------------------------------------------------------------------------
# worlds per configuration
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1(torch_cuda):
    return World(S.CONFIGS["C1"], seed=1, rot_steps=(1, 2, -1, 5))


@pytest.fixture(scope="module")
def c2(torch_cuda):
    return World(S.CONFIGS["C2"], seed=2, rot_steps=(1, 3))


@pytest.fixture(scope="module")
def c3(torch_cuda):
    return World(S.CONFIGS["C3"], seed=3, rot_steps=(1,))


def _world(request, name):
    return request.getfixturevalue(name)


@pytest.mark.parametrize("name,levels", [("c1", (2, 1)), ("c2", (8, 5, 3, 1)), ("c3", (24, 23))])
def test_encrypt_decrypt_parity(request, name, levels):
    w = _world(request, name)
    m = w.random_plain(11)
    for lvl in levels:
        g, o = w.encrypt_pair(m, lvl, 100 + lvl)
        w.assert_same(g, o)
        assert np.array_equal(w.ctx.decrypt(g), C.decrypt(w.op, w.kd.s, o))


@pytest.mark.parametrize("name,levels", [("c1", (2, 1)), ("c2", (8, 7, 4, 3)), ("c3", (24, 19))])
def test_mul_relin_parity(request, name, levels):
    w = _world(request, name)
    for lvl in levels:
        ga, oa = w.encrypt_pair(w.random_plain(21), lvl, 200 + lvl)
        gb, ob = w.encrypt_pair(w.random_plain(22), lvl, 300 + lvl)
        w.assert_same(w.ctx.mul_relin(ga, gb), C.hmul_relin(w.op, oa, ob, w.rlk))


@pytest.mark.parametrize("name,levels", [("c1", (2, 1)), ("c2", (8, 5, 2)), ("c3", (24, 17, 6))])
def test_bconv_modes_parity(request, name, levels):
    """Key switching with the base conversions on the matrix cores (int8
    digits; fused with the adjacent transform passes and the key inner
    product fused with the row pass of ModUp's rows, two digits per row pass
    (the default) or one; fused passes only; separate) and on the VALU
    (128-bit MACs): all equal the oracle, at full, ragged-last-digit and low
    levels."""
    w = _world(request, name)
    for lvl in levels:
        ga, oa = w.encrypt_pair(w.random_plain(23), lvl, 700 + lvl)
        gb, ob = w.encrypt_pair(w.random_plain(24), lvl, 800 + lvl)
        want = C.hmul_relin(w.op, oa, ob, w.rlk)
        st = sorted(w.rot)[0]
        want_rot = C.rotate(w.op, oa, st, w.rot[st])
        for mfma, fused, inner, pairs in ((True, True, True, True), (True, True, True, False),
                                          (True, True, False, False), (True, False, False, False),
                                          (False, False, False, False)):
            w.ctx.bconv_mode(mfma, fused=fused, inner=inner, pairs=pairs)
            w.assert_same(w.ctx.mul_relin(ga, gb), want)
            w.assert_same(w.ctx.rotate(ga, st), want_rot)
    w.ctx.bconv_mode(True)


@pytest.mark.parametrize("name,levels", [("c1", (2,)), ("c2", (8, 3, 2)), ("c3", (24, 13))])
@pytest.mark.parametrize("mode", [0, 1])
def test_rescale_parity(request, name, levels, mode):
    w = _world(request, name)
    for lvl in levels:
        g, o = w.encrypt_pair(w.random_plain(31), lvl, 400 + lvl)
        w.assert_same(w.ctx.rescale(g, mode=mode), C.rescale(w.op, o, mode="round" if mode == 0 else "floor"))


@pytest.mark.parametrize("name,steps,levels", [("c1", (1, -1, 5), (2, 1)), ("c2", (1, 3), (8, 5)),
                                               ("c3", (1,), (24,))])
def test_rotate_parity(request, name, steps, levels):
    w = _world(request, name)
    for lvl in levels:
        g, o = w.encrypt_pair(w.random_plain(41), lvl, 500 + lvl)
        for st in steps:
            w.assert_same(w.ctx.rotate(g, st), C.rotate(w.op, o, st, w.rot[st]))


def test_rotate_pow2_parity(c1):
    """Rotation from power-of-two keys (low and high Hamming weight steps, a
    negative step): bit-exact against the oracle's same decomposition."""
    w = c1
    for k in range(11):
        if (1 << k) not in w.rot:
            w.add_rotation(1 << k)
    keys = {1 << k: w.rot[1 << k] for k in range(11)}
    for lvl in (2, 1):
        g, o = w.encrypt_pair(w.random_plain(42), lvl, 520 + lvl)
        for st in (1, 11, -3, 2047):
            w.assert_same(w.ctx.rotate_pow2(g, st), C.rotate_pow2(w.op, o, st, keys))
        out = w.ctx.rotate_pow2_batch([g, g], 6)
        want = C.rotate_pow2(w.op, o, 6, keys)
        for x in out:
            w.assert_same(x, want)


def test_total_sum_parity(c1):
    w = c1
    g, o = w.encrypt_pair(w.random_plain(51), 2, 600)
    keys = {s: w.rot[s] for s in (1, 2)}
    w.assert_same(w.ctx.total_sum(g, 4), C.total_sum(w.op, o, 4, keys))


def test_batched_ops_mixed_levels(c2):
    """Batched HMult+relin, rescale, rotate and TotalSum over ciphertexts of
    mixed levels (3..8) equal the oracle element by element."""
    w = c2
    lv = [8, 3, 6, 8, 5, 4, 7, 3]
    a = [w.encrypt_pair(w.random_plain(1100 + i), l, 1200 + i) for i, l in enumerate(lv)]
    b = [w.encrypt_pair(w.random_plain(1300 + i), l, 1400 + i) for i, l in enumerate(lv)]
    prod = w.ctx.mul_relin_batch([x[0] for x in a], [x[0] for x in b])
    oprod = [C.hmul_relin(w.op, x[1], y[1], w.rlk) for x, y in zip(a, b)]
    for g, o in zip(prod, oprod):
        w.assert_same(g, o)
    rs = w.ctx.rescale_batch(prod)
    ors = [C.rescale(w.op, o) for o in oprod]
    for g, o in zip(rs, ors):
        w.assert_same(g, o)
    rot = w.ctx.rotate_batch(rs, 3)
    for g, o in zip(rot, ors):
        w.assert_same(g, C.rotate(w.op, o, 3, w.rot[3]))
    ts = w.ctx.total_sum_batch(rs[:3], 2)
    for g, o in zip(ts, ors[:3]):
        w.assert_same(g, C.total_sum(w.op, o, 2, {1: w.rot[1]}))


def test_plain_ops_parity(c2):
    w = c2
    lvl = 6
    g, o = w.encrypt_pair(w.random_plain(61), lvl, 700)
    g2, o2 = w.encrypt_pair(w.random_plain(62), lvl, 701)
    m = w.random_plain(63, bound=2 ** 30)
    pt = w.ctx.plaintext(m, lvl, 2.0 ** 30)
    w.assert_same(w.ctx.add(g, g2), C.hadd(w.op, o, o2))
    w.assert_same(w.ctx.mul_plain(g, pt), C.hmul_plain(w.op, o, m, 2.0 ** 30))
    pt_s = w.ctx.plaintext(m, lvl, w.op.scale)
    w.assert_same(w.ctx.add_plain(g, pt_s), C.hadd_plain(w.op, o, m))
    w.assert_same(w.ctx.mod_drop(g, 3), C.mod_drop(w.op, o, 3))


def test_import_export_roundtrip(c2):
    w = c2
    g = np.random.default_rng(5)
    host = np.stack([np.stack([g.integers(0, q, w.n, dtype=np.uint64) for q in w.op.q[:4]]) for _ in range(2)])
    ct = w.ctx.import_(host, 4, 1.0)
    assert np.array_equal(w.ctx.export(ct), host)


def test_batch_equals_singles(c2):
    w = c2
    cts = [w.encrypt_pair(w.random_plain(70 + i), lvl, 800 + i) for i, lvl in enumerate((8, 6, 5))]
    others = [w.encrypt_pair(w.random_plain(80 + i), lvl, 900 + i) for i, lvl in enumerate((8, 6, 5))]
    batch = w.ctx.mul_relin_batch([c[0] for c in cts], [c[0] for c in others])
    for (ga, oa), (gb, ob), gbat in zip(cts, others, batch):
        w.assert_same(gbat, C.hmul_relin(w.op, oa, ob, w.rlk))


def test_chain_parity_c2(c2):
    """encrypt -> HMult+relin -> rescale -> rotate -> HMult+relin -> rescale."""
    w = c2
    ga, oa = w.encrypt_pair(w.random_plain(91), 8, 1001)
    gb, ob = w.encrypt_pair(w.random_plain(92), 8, 1002)
    g = w.ctx.rescale(w.ctx.mul_relin(ga, gb))
    o = C.rescale(w.op, C.hmul_relin(w.op, oa, ob, w.rlk))
    g = w.ctx.rotate(g, 3)
    o = C.rotate(w.op, o, 3, w.rot[3])
    g2, o2 = w.encrypt_pair(w.random_plain(93), 7, 1003)
    g = w.ctx.rescale(w.ctx.mul_relin(g, g2))
    o = C.rescale(w.op, C.hmul_relin(w.op, o, o2, w.rlk))
    w.assert_same(g, o)


def test_slots_c1(c1):
    """Decoded slots of encrypt -> HMult+relin -> rescale -> decrypt, each side
    encoding z1, z2 with its own encoder: both track z1*z2 within the noise
    bound, so they agree with each other within twice that bound."""
    from tests import noise
    w = c1
    n = w.n
    z1 = S.slots_uniform(S.rng(101), n // 2)
    z2 = S.slots_uniform(S.rng(102), n // 2)
    d1, d2 = S.enc_draws(1001, n), S.enc_draws(1002, n)
    g1 = w.ctx.encrypt(w.lp.encode(z1), 2, w.op.scale, d1.v, d1.e0, d1.e1)
    g2 = w.ctx.encrypt(w.lp.encode(z2), 2, w.op.scale, d2.v, d2.e0, d2.e1)
    gp = w.ctx.rescale(w.ctx.mul_relin(g1, g2))
    lib_slots = w.lp.decode(w.ctx.decrypt(gp), gp.scale)
    o1 = C.encrypt(w.op, w.pk, C.encode(z1, n, w.op.scale), 2, d1.v, d1.e0, d1.e1, w.op.scale)
    o2 = C.encrypt(w.op, w.pk, C.encode(z2, n, w.op.scale), 2, d2.v, d2.e0, d2.e1, w.op.scale)
    op_ = C.rescale(w.op, C.hmul_relin(w.op, o1, o2, w.rlk))
    ora_slots = C.decode(C.decrypt(w.op, w.kd.s, op_), w.op.q[:1], n, op_.scale, n // 2)
    h = 2 * n / 3
    fresh = noise.fresh(n, h, h, w.op.scale) + n / w.op.scale
    bound = 2 * np.sqrt(2) * fresh + noise.rescale_round(n, h, gp.scale) + 1e-6
    assert np.max(np.abs(lib_slots - z1 * z2)) <= bound
    assert np.max(np.abs(ora_slots - z1 * z2)) <= bound
    assert np.max(np.abs(lib_slots - ora_slots)) <= 2 * bound


def test_slots_c3_within_2_20(c3):
    """At the large ring (scale 2^50) the decoded product agrees with the
    oracle's decoded product within 2^-20."""
    w = c3
    n = w.n
    z1 = S.slots_unit(S.rng(303), n // 2)
    z2 = S.slots_unit(S.rng(304), n // 2)
    d1, d2 = S.enc_draws(3001, n), S.enc_draws(3002, n)
    g1 = w.ctx.encrypt(w.lp.encode(z1), 24, w.op.scale, d1.v, d1.e0, d1.e1)
    g2 = w.ctx.encrypt(w.lp.encode(z2), 24, w.op.scale, d2.v, d2.e0, d2.e1)
    gp = w.ctx.rescale(w.ctx.mul_relin(g1, g2))
    lib_slots = w.lp.decode(w.ctx.decrypt(gp), gp.scale)
    o1 = C.encrypt(w.op, w.pk, C.encode(z1, n, w.op.scale), 24, d1.v, d1.e0, d1.e1, w.op.scale)
    o2 = C.encrypt(w.op, w.pk, C.encode(z2, n, w.op.scale), 24, d2.v, d2.e0, d2.e1, w.op.scale)
    op_ = C.rescale(w.op, C.hmul_relin(w.op, o1, o2, w.rlk))
    ora_slots = C.decode(C.decrypt(w.op, w.kd.s, op_), w.op.q[:23], n, op_.scale, n // 2)
    assert np.max(np.abs(lib_slots - ora_slots)) <= 2.0 ** -20
    assert np.max(np.abs(lib_slots - z1 * z2)) <= 2.0 ** -20


def test_errors(c1):
    import paper_1908_06972_amd.native as N
    w = c1
    g, _ = w.encrypt_pair(w.random_plain(1), 2, 1)
    h, _ = w.encrypt_pair(w.random_plain(2), 1, 2)
    with pytest.raises(N.PftError) as e:
        w.ctx.rotate(g, 7)
    assert e.value.code == N.PFT_ENOKEY
    with pytest.raises(N.PftError) as e:
        w.ctx.add(g, h)
    assert e.value.code == N.PFT_ELEVEL
    with pytest.raises(N.PftError) as e:
        w.ctx.rescale(h)
    assert e.value.code == N.PFT_ELEVEL
    with pytest.raises(N.PftError) as e:
        w.ctx.mul_relin(g, g, out=g)
    assert e.value.code == N.PFT_EINVAL


def test_graph_replay_matches_eager(torch_cuda):
    """HMult+relin -> rescale -> rotate captured in a HIP graph: every replay,
    with other work on the stream in between, equals the eager result."""
    import paper_1908_06972_amd.ckks as L
    torch = torch_cuda
    cfg = S.CONFIGS["C2"]
    lp = L.Params.from_config(cfg)
    side = torch.cuda.Stream()
    ctx = L.Context(lp, stream=side)
    n = lp.n
    kd = S.key_draws(2, n, lp.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    a, e = S.switch_key_draws(2, 0, n, lp.key_moduli(), lp.dnum)
    ctx.gen_relin_key(a, e)
    a, e = S.switch_key_draws(2, 1003, n, lp.key_moduli(), lp.dnum)
    ctx.gen_rotation_key(3, a, e)
    d1, d2 = S.enc_draws(61, n), S.enc_draws(62, n)
    ga = ctx.encrypt(S.plaintext_coeffs(S.rng(63), n, 2 ** 40), 8, lp.scale, d1.v, d1.e0, d1.e1)
    gb = ctx.encrypt(S.plaintext_coeffs(S.rng(64), n, 2 ** 40), 8, lp.scale, d2.v, d2.e0, d2.e1)
    eager = ctx.export(ctx.rotate(ctx.rescale(ctx.mul_relin(ga, gb)), 3))
    m_out, r_out, rot_out = ctx.empty_ct(8), ctx.empty_ct(7), ctx.empty_ct(7)

    def chain():
        ctx.mul_relin(ga, gb, out=m_out)
        ctx.rescale(m_out, out=r_out)
        ctx.rotate(r_out, 3, out=rot_out)

    graph = ctx.capture(chain)
    for rep in range(3):
        with torch.cuda.stream(side):
            rot_out.data.zero_()
            m_out.data.fill_(rep)
        ctx.rescale(ctx.mul_relin(gb, ga))  # unrelated eager work on the same stream
        graph.launch()
        ctx.synchronize()
        assert np.array_equal(ctx.export(rot_out), eager), rep
    graph.close()
    ctx.close()


@pytest.mark.parametrize("flags", [0, 1])
def test_fused_first_pass_c3(c3, flags):
    """At the large ring with the forward schedule pinned to (4, 12): the
    base conversions and RESCALE's expansion apply the first transform pass
    themselves; relinearisation, rotation and RESCALE equal the oracle at a
    full and a ragged-last-digit level."""
    w = c3
    sched = [c for c in w.ctx.ntt_candidates() if tuple(c[0]) == (4, 12) and c[1] == flags][0]
    w.ctx.ntt_set_schedule(False, sched)
    try:
        for lvl in (24, 19):
            ga, oa = w.encrypt_pair(w.random_plain(41), lvl, 900 + lvl)
            gb, ob = w.encrypt_pair(w.random_plain(42), lvl, 950 + lvl)
            w.assert_same(w.ctx.mul_relin(ga, gb), C.hmul_relin(w.op, oa, ob, w.rlk))
            w.assert_same(w.ctx.rotate(ga, 1), C.rotate(w.op, oa, 1, w.rot[1]))
            w.assert_same(w.ctx.rescale(ga), C.rescale(w.op, oa))
    finally:
        w.ctx.ntt_set_schedule(False, None)


def test_tuning_table_restricted_classes(torch_cuda):
    """Tuning entries of the first-radix-4 classes (32 + class): accepted with
    a schedule starting with radix 4 and exported back, refused otherwise."""
    import paper_1908_06972_amd.ckks as L
    import paper_1908_06972_amd.native as N
    lp = L.Params(16, 4, 60, 50, 1, 60, 2, 2 ** 40)
    ctx = L.Context(lp)
    ok = [(True, 40, ((4, 12), 3)), (False, 9, ((4, 12), 0))]
    ctx.ntt_tuning_import(ok)
    got = ctx.ntt_tuning_export()
    for entry in ok:
        assert entry in got
    for bad in [(True, 40, ((8, 8), 0)), (True, 43, ((4, 12), 0)), (True, 11, ((4, 12), 0))]:
        with pytest.raises(N.PftError):
            ctx.ntt_tuning_import([bad])
