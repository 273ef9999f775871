"""The boundary's memory budget and allocator, the explicit prime chain, the
default rescale mode and the PtMatVec plan export, on the GPU.

Budget: a context refuses, with PFT_ENOMEM, every allocation that would take
its own device memory past the budget (at creation, key generation and
workspace growth) and works again once the budget allows it, with the same
residues.  Allocator: a context whose memory comes from torch's caching
allocator gives the same residues and hands every byte back when destroyed.
Plan export: the op list and integer diagonals of a plaintext matrix,
replayed by the oracle, give pft_ptmatvec's result bit for bit (Sec. 4.1)."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import ptmatvec as PM
from oracle import sampler as SP

pytestmark = pytest.mark.gpu

SMALL = dict(log_n=12, n_q=4, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=2, scale=2 ** 40)


def _params():
    import paper_1908_06972_amd.ckks as L
    return L.Params(*SMALL.values())


def _pair(ctx, op, seed, level):
    m = S.plaintext_coeffs(S.rng(seed), op.n, 2 ** 30)
    return ctx.encrypt_seeded(m, level, op.scale, 600 + seed)


def test_budget_refuses_and_recovers():
    import torch
    import paper_1908_06972_amd.ckks as L
    from paper_1908_06972_amd.native import PFT_ENOMEM, PftError
    assert torch.cuda.is_available()
    lp, op = _params(), C.Params(**SMALL)
    ref = L.Context(lp)
    tables = ref.memory()["tables_keys"]
    ref.keygen(21, [1])
    with pytest.raises(PftError) as e:
        L.Context(lp, budget_bytes=tables // 2)
    assert e.value.code == PFT_ENOMEM
    ctx = L.Context(lp, budget_bytes=tables + (1 << 20))
    assert ctx.memory()["budget"] == tables + (1 << 20)
    with pytest.raises(PftError) as e:
        ctx.keygen(21, [1])  # the keys do not fit
    assert e.value.code == PFT_ENOMEM
    ctx.set_budget(0)
    ctx.keygen(21, [1])
    a, b = _pair(ctx, op, 1, op.L), _pair(ctx, op, 2, op.L)
    ra, rb = _pair(ref, op, 1, op.L), _pair(ref, op, 2, op.L)
    used = ctx.memory()
    ctx.set_budget(used["tables_keys"] + used["scratch"] + 4096)  # no room for a larger workspace
    with pytest.raises(PftError) as e:
        ctx.mul_relin(a, b)
    assert e.value.code == PFT_ENOMEM
    with pytest.raises(PftError) as e:
        ctx.set_budget(used["tables_keys"] // 2)  # below what the context holds: refused, unchanged
    assert e.value.code == PFT_ENOMEM
    ctx.set_budget(0)
    assert np.array_equal(ctx.export(ctx.mul_relin(a, b)), ref.export(ref.mul_relin(ra, rb)))
    assert np.array_equal(ctx.export(ctx.rotate(a, 1)), ref.export(ref.rotate(ra, 1)))


def test_torch_allocator_gives_same_residues_and_returns_memory():
    import gc

    import torch
    import paper_1908_06972_amd.ckks as L
    assert torch.cuda.is_available()
    lp, op = _params(), C.Params(**SMALL)
    ref = L.Context(lp)
    ref.keygen(22, [3])
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = L.Context(lp, torch_memory=True)
    ctx.keygen(22, [3])
    mem = ctx.memory()
    assert torch.cuda.memory_allocated() - base >= mem["tables_keys"]
    a, b = _pair(ctx, op, 3, op.L), _pair(ctx, op, 4, op.L)
    ra, rb = _pair(ref, op, 3, op.L), _pair(ref, op, 4, op.L)
    assert np.array_equal(ctx.export(ctx.mul_relin(a, b)), ref.export(ref.mul_relin(ra, rb)))
    assert np.array_equal(ctx.export(ctx.rotate(a, 3)), ref.export(ref.rotate(ra, 3)))
    assert len(ctx._alloc.live) > 0
    alloc = ctx._alloc
    gc.collect()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated()
    ctx.close()
    torch.cuda.synchronize()
    assert not alloc.live  # every buffer went back to torch
    assert held - torch.cuda.memory_allocated() >= mem["tables_keys"]


def test_default_rescale_mode_follows_the_parameters():
    """RESCALE with PFT_RESCALE_DEFAULT uses the parameter set's mode: floor
    (Alg. 3 as printed) for a chain created with rescale_mode 1, from the
    explicit primes of the rounding chain."""
    import torch
    import paper_1908_06972_amd.ckks as L
    from paper_1908_06972_amd.native import PFT_RESCALE_DEFAULT
    assert torch.cuda.is_available()
    base = _params()
    lp = L.Params.from_primes(12, base.q, base.p, 2, 2 ** 40, rescale_mode=1)
    op = C.Params(**SMALL)
    assert lp.q == op.q and lp.p == op.p
    ctx = L.Context(lp)
    ctx.keygen(23, [])
    s = SP.secret(23, op.n)
    pk = C.public_key(op, s, *SP.public_key_draws(23, op.q, op.n))
    m = S.plaintext_coeffs(S.rng(5), op.n, 2 ** 30)
    g = ctx.encrypt_seeded(m, op.L, op.scale, 605)
    o = C.encrypt(op, pk, m, op.L, *SP.encryption_draws(605, op.n), op.scale)
    for mode, want in ((PFT_RESCALE_DEFAULT, "floor"), (0, "round"), (1, "floor")):
        host = ctx.export(ctx.rescale(g, mode=mode))
        w = C.rescale(op, o, mode=want)
        assert np.array_equal(host[0], w.c0) and np.array_equal(host[1], w.c1), mode


@pytest.mark.parametrize("n_o,n_i,n_in", [(16, 2048, 2), (4, 16, 1)])
def test_ptmat_plan_export_replays_with_the_oracle(n_o, n_i, n_in):
    import torch
    import paper_1908_06972_amd.ckks as L
    assert torch.cuda.is_available()
    lp, op = _params(), C.Params(**SMALL)
    C.set_mul_mode(1)
    n = op.n
    steps = sorted(set(PM.rotation_steps(n_o, n_i, n_in)))
    ctx = L.Context(lp)
    ctx.keygen(24, steps)
    s = SP.secret(24, n)
    pk = C.public_key(op, s, *SP.public_key_draws(24, op.q, n))
    mods = op.key_moduli()
    keys = {st: C.rotation_key(op, s, st, *SP.switch_key_draws(24, SP.rotation_key_id(st, n), mods, op.dnum, n))
            for st in steps}
    b, G = PM.bsgs_plan(n_o, n_in)
    g = S.rng(70 + n_o)
    plains = np.stack([np.stack([np.stack([S.plaintext_coeffs(g, n, 2 ** 20) for _ in range(b)])
                                 for _ in range(G)]) for _ in range(n_in)])
    level = 3
    pt_scale = float(op.q[level - 1])
    mat = ctx.ptmat_from_coeffs(plains, n_o, n_i, n_in, level, pt_scale)
    ops, coeffs = mat.plan_export()
    assert np.array_equal(coeffs, plains)
    ms = [S.plaintext_coeffs(S.rng(80 + c), n, 2 ** 36) for c in range(n_in)]
    gin = [ctx.encrypt_seeded(m, level, op.scale, 700 + c) for c, m in enumerate(ms)]
    oin = [C.encrypt(op, pk, m, level, *SP.encryption_draws(700 + c, n), op.scale) for c, m in enumerate(ms)]
    got = ctx.ptmatvec(mat, [gin])[0]
    diags = [coeffs[c][gg][r] for c in range(n_in) for gg in range(G) for r in range(b)]
    regs = dict(enumerate(oin))
    for kind, a, bb, out, step in ops:
        if kind == "rotate":
            regs[out] = C.rotate(op, regs[a], step, keys[step])
        elif kind == "mul_plain":
            regs[out] = C.hmul_plain(op, regs[a], diags[bb], pt_scale)
        else:
            regs[out] = C.hadd(op, regs[a], regs[bb])
    want = regs[ops[-1][3]]
    host = ctx.export(got)
    assert np.array_equal(host[0], want.c0) and np.array_equal(host[1], want.c1)
