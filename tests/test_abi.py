"""The C ABI without a GPU: the library loads, exports every symbol that
include/pft.h declares, and its host-side logic (prime chain, roots, encode,
decode) agrees with the oracle.  No device call is made here."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from paper_1908_06972_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pft_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("pft_params_create", "pft_ctx_create", "pft_set_secret", "pft_gen_public_key",
                 "pft_gen_relin_key", "pft_gen_rotation_key", "pft_encrypt", "pft_decrypt",
                 "pft_mul_relin", "pft_rescale", "pft_rotate", "pft_total_sum", "pft_ntt_forward"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = N.load()
    for name in _declared():
        assert hasattr(lib, name), name
    bound = {s[0] for s in N.SIGNATURES}
    assert set(_declared()) == bound


@pytest.mark.parametrize("name", sorted(S.CONFIGS))
def test_library_prime_chain_matches_oracle(name):
    from paper_1908_06972_amd.ckks import Params
    cfg = S.CONFIGS[name]
    lp = Params.from_config(cfg)
    op = C.Params.from_config(cfg)
    assert lp.q == op.q and lp.p == op.p and lp.alpha == op.alpha


def test_params_rejects_bad_specs():
    from paper_1908_06972_amd.ckks import Params
    with pytest.raises(N.PftError) as e:
        Params(11, 2, 40, 40, 1, 50, 2, 2 ** 30)       # log_n below the supported range
    assert e.value.code == N.PFT_EPARAM
    with pytest.raises(N.PftError):
        Params(12, 4, 40, 40, 1, 50, 5, 2 ** 30)       # dnum > L
    with pytest.raises(N.PftError):
        Params(12, 4, 30, 40, 1, 50, 2, 2 ** 30)       # q0 smaller than the chain
    with pytest.raises(N.PftError):
        Params(12, 2, 61, 40, 1, 50, 1, 2 ** 30)       # primes above 60 bits


@pytest.mark.parametrize("log_n", [12, 14])
def test_library_encode_within_one_of_oracle(log_n):
    from paper_1908_06972_amd.ckks import Params
    P = Params(log_n, 3, 60, 40, 1, 60, 1, 2 ** 40)
    g = S.rng(log_n)
    z = S.slots_uniform(g, P.n // 2)
    lib_m = P.encode(z)
    ora_m = C.encode(z, P.n, P.scale)
    assert np.max(np.abs(lib_m - ora_m)) <= 1
    sparse = P.encode(z[:5])
    assert np.max(np.abs(sparse - C.encode(z[:5], P.n, P.scale))) <= 1


@pytest.mark.parametrize("n_o,n_i,n_in", [(16, 2048, 2), (4, 16, 1), (8, 64, 3)])
def test_library_diagonals_within_one_of_oracle(n_o, n_i, n_in):
    """pft_diagonals_encode: the pre-rotated diagonals of the BSGS plan,
    encoded, against the oracle's diagonals and encoder (Sec. 4.1/4.2)."""
    from oracle import ptmatvec as PM
    from paper_1908_06972_amd.ckks import Params
    P = Params(12, 3, 60, 40, 1, 60, 1, 2 ** 40)
    g = np.random.default_rng(n_o + n_i)
    M = g.normal(0, 0.1, size=(n_o, n_in * n_i))
    scale = 2.0 ** 38
    lib = P.diagonals_encode(M, n_o, n_i, n_in, scale)
    D = PM.prerotated_diagonals(M, n_o, n_i, n_in, P.n // 2)
    b, G = PM.bsgs_plan(n_o, n_in)
    assert lib.shape == (n_in, G, b, P.n)
    for c in range(n_in):
        for gg in range(G):
            for r in range(b):
                assert np.max(np.abs(lib[c, gg, r] - C.encode(D[c][gg][r], P.n, scale))) <= 1


def test_library_decode_matches_oracle():
    from paper_1908_06972_amd.ckks import Params
    P = Params(12, 3, 60, 40, 1, 60, 1, 2 ** 40)
    op = C.Params(12, 3, 60, 40, 1, 60, 1, 2 ** 40)
    g = S.rng(3)
    m = S.plaintext_coeffs(g, P.n, 2 ** 45)
    res = C.rns_from_int(m, op.q)
    a = P.decode(res, 2.0 ** 40)
    b = C.decode(res, op.q, op.n, 2.0 ** 40, op.n // 2)
    assert np.max(np.abs(a - b)) <= 2.0 ** -20
    # single limb, negative values
    a1 = P.decode(res[:1], 2.0 ** 40)
    b1 = C.decode(res[:1], op.q[:1], op.n, 2.0 ** 40, op.n // 2)
    assert np.max(np.abs(a1 - b1)) <= 2.0 ** -20


def test_ntt_candidate_schedules():
    """Schedules cover log2 N exactly, default first, at most two passes, only
    the last window may exceed radix 8 (column passes need >= 16 sub-problems
    per workgroup), each radix split comes staged and direct, with 16 and 8
    residues per thread, and every size has the (4, log2 N - 4) split."""
    from paper_1908_06972_amd.ckks import Params
    lib = N.load()
    for log_n in range(12, 17):
        p = Params(log_n, 2, 40, 40, 1, 50, 1, 2 ** 30)
        n = lib.pft_ntt_candidates(p.handle, None, 0)
        assert n >= 4
        buf = (ctypes.c_uint32 * (4 * n))()
        assert lib.pft_ntt_candidates(p.handle, buf, n) == n
        scheds = [(tuple(r for r in buf[4 * i:4 * i + 3] if r), buf[4 * i + 3]) for i in range(n)]
        assert len(set(scheds)) == n
        for radices, flags in scheds:
            assert sum(radices) == log_n and 1 <= len(radices) <= 2
            assert all(r <= 8 for r in radices[:-1])
            assert flags in (0, 1, 2, 3)
        # every size offers the split the fused conversions need: a radix-16
        # column pass, then one row pass, in all four variants
        for flags in (0, 1, 2, 3):
            assert ((4, log_n - 4), flags) in scheds, (log_n, flags)
            assert all((radices, f) in scheds for f in (0, 1, 2, 3))
        assert scheds[0] == ({12: (12,), 13: (7, 6), 14: (7, 7), 15: (8, 7), 16: (8, 8)}[log_n], 0)


def _plan(ops, levels):
    n = len(ops)
    O = (N.OpDesc * max(n, 1))()
    for i, (kind, a, b, out, step, mode) in enumerate(ops):
        O[i] = N.OpDesc(kind, a, b, out, step, mode)
    L = (ctypes.c_uint32 * max(len(levels), 1))(*levels)
    w = (ctypes.c_uint32 * max(n, 1))()
    g = (ctypes.c_uint32 * max(n, 1))()
    nw = N.load().pft_exec_plan(O, n, L, len(levels), w, g)
    return nw, list(w)[:n], list(g)[:n]


def test_exec_plan_waves_and_groups():
    """Independent ops share wave 0; equal (kind, level, step) share a group;
    read-after-write, write-after-read and write-after-write each start a later
    wave; rescale lowers the simulated level of its output."""
    MUL, RS, ROT, ADD, NTT = N.PFT_OP_MUL_RELIN, N.PFT_OP_RESCALE, N.PFT_OP_ROTATE, N.PFT_OP_ADD, N.PFT_OP_NTT
    levels = [5, 5, 4, 4, 5, 5, 4, 4, 0, 0, 0, 0]
    ops = [(MUL, 0, 1, 8, 0, 0),      # wave 0, level 5
           (MUL, 2, 3, 9, 0, 0),      # wave 0, level 4 -> other group
           (MUL, 4, 5, 10, 0, 0),     # wave 0, same group as op 0
           (RS, 8, 0, 11, 0, 0),      # reads 8 (written by op 0) -> wave 1
           (ROT, 11, 0, 0, 3, 0),     # writes 0, read by op 0 (WAR) and reads 11 (RAW) -> wave 2
           (NTT, 6, 0, 0, 0, 0),      # independent, in place -> wave 0
           (ADD, 6, 7, 9, 0, 0)]      # reads 6 (written by op 5), writes 9 (written by op 1) -> wave 1
    nw, w, g = _plan(ops, levels)
    assert nw == 3
    assert w == [0, 0, 0, 1, 2, 0, 1]
    assert g[0] == g[2] != g[1]
    assert len({g[0], g[1], g[5]}) == 3
    assert g[3] != g[6]


def test_exec_plan_rejects_bad_lists():
    MUL, RS, ROT = N.PFT_OP_MUL_RELIN, N.PFT_OP_RESCALE, N.PFT_OP_ROTATE
    assert _plan([(MUL, 0, 1, 2, 0, 0)], [3, 4, 0])[0] == N.PFT_ELEVEL
    assert _plan([(ROT, 0, 0, 0, 1, 0)], [3])[0] == N.PFT_EINVAL
    assert _plan([(RS, 0, 0, 1, 0, 0)], [1, 0])[0] == N.PFT_ELEVEL
    assert _plan([(99, 0, 0, 0, 0, 0)], [3])[0] == N.PFT_EINVAL
    assert _plan([(MUL, 0, 1, 5, 0, 0)], [3, 3])[0] == N.PFT_EINVAL
    # a rescale chain: the simulated level drops, so the second rescale of a
    # level-2 input fails
    assert _plan([(RS, 0, 0, 1, 0, 0), (RS, 1, 0, 2, 0, 0)], [2, 0, 0])[0] == N.PFT_ELEVEL


def test_library_gaussian_table_equals_oracle():
    """pft_gaussian_cdt (120-bit fixed point in the library) against the
    oracle's 60-digit decimal table: every threshold identical."""
    from oracle import sampler as SP
    lib = N.load()
    t = np.zeros(64, dtype=np.uint64)
    cnt = ctypes.c_uint32(0)
    N.check(lib.pft_gaussian_cdt(N.u64p(t), 64, ctypes.byref(cnt)))
    assert cnt.value == 2 * SP.BOUND
    assert t[:cnt.value].tolist() == SP.gaussian_cdt()
    with pytest.raises(N.PftError):
        N.check(lib.pft_gaussian_cdt(N.u64p(t), 37, ctypes.byref(cnt)))


def test_shipped_tuning_table_is_valid():
    """Every entry of the large-ring tuning table bench.py imports is a
    candidate schedule at N = 2^16 (pft_ntt_candidates, host only), classes
    are 0..10 or 32 + 0..10, and the first-radix-4 classes start with 4."""
    import json
    from paper_1908_06972_amd.ckks import Params
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1908_06972_amd",
                        "tuning", "large_ring_n16_l24.json")
    table = json.load(open(path))
    lib = N.load()
    p = Params(16, 24, 60, 50, 6, 60, 4, 2 ** 50)
    n = lib.pft_ntt_candidates(p.handle, None, 0)
    buf = (ctypes.c_uint32 * (4 * n))()
    assert lib.pft_ntt_candidates(p.handle, buf, n) == n
    cands = {(tuple(r for r in buf[4 * i:4 * i + 3] if r), buf[4 * i + 3]) for i in range(n)}
    assert table
    for inv, cls, radices, flags in table:
        assert isinstance(inv, bool) and (0 <= cls <= 10 or 32 <= cls <= 42)
        assert (tuple(radices), flags) in cands
        if cls >= 32:
            assert radices[0] == 4 and len(radices) >= 2


def test_explicit_prime_chain_and_rejections():
    """pft_params_create_primes takes the caller's chain and refuses every
    modulus that is not prime, not 1 mod 2N, outside (2^20, 2^60), repeated,
    or out of descending order; rescale_mode is carried and bounded."""
    from paper_1908_06972_amd.ckks import Params
    ref = Params(12, 4, 60, 40, 2, 60, 2, 2 ** 40)
    P = Params.from_primes(12, ref.q, ref.p, 2, 2 ** 40, rescale_mode=1)
    assert P.q == ref.q and P.p == ref.p and P.alpha == ref.alpha and P.rescale_mode == 1
    two_n = 2 * 4096
    q, p = list(ref.q), list(ref.p)
    comp = next(q[2] - k * two_n for k in range(1, 1000) if not C.is_prime(q[2] - k * two_n))
    assert q[3] < comp < q[2] and comp % two_n == 1
    bad = {
        "composite": ([q[0], q[1], comp, q[3]], p),
        "not 1 mod 2N": ([q[0], q[1], q[2] + 2, q[3]], p),
        "too large": ([(1 << 60) + 1, q[1], q[2], q[3]], p),
        "too small": (q[:3] + [two_n + 1], p),
        "repeated": (q, [p[0], p[0]]),
        "special equals a q": (q, [p[0], q[1]]),
        "not descending": ([q[1], q[0], q[2], q[3]], p),
    }
    reason = {"composite": "not prime", "not 1 mod 2N": "not 1 mod 2N", "too large": "not in", "too small": "not in",
              "repeated": "twice", "special equals a q": "twice", "not descending": "descending"}
    for what, (qq, pp) in bad.items():
        with pytest.raises(N.PftError) as e:
            Params.from_primes(12, qq, pp, 2, 2 ** 40)
        assert e.value.code == N.PFT_EPARAM and reason[what] in str(e.value), (what, str(e.value))
    with pytest.raises(N.PftError) as e:
        Params.from_primes(12, q, p, 2, 2 ** 40, rescale_mode=2)
    assert e.value.code == N.PFT_EPARAM
    with pytest.raises(N.PftError) as e:
        Params(12, 4, 60, 40, 2, 60, 2, 2 ** 40, rescale_mode=3)
    assert e.value.code == N.PFT_EPARAM


def _replay_plan(ops, inputs, diags, t):
    """The exported PtMatVec op list on plain slot vectors: rotation is a
    left rotation of the t slots, mul_plain a slot-wise product with the
    diagonal, add a sum."""
    regs = {c: v.copy() for c, v in enumerate(inputs)}
    for kind, a, b, out, step in ops:
        if kind == "rotate":
            regs[out] = np.roll(regs[a], -step)
        elif kind == "mul_plain":
            regs[out] = regs[a] * diags[b]
        else:
            regs[out] = regs[a] + regs[b]
    return regs[ops[-1][3]]


@pytest.mark.parametrize("n_o,n_i,n_in", [(16, 64, 2), (4, 16, 1), (8, 8, 3), (32, 256, 1), (2, 32, 5)])
def test_ptmat_plan_replays_to_the_matrix_product(n_o, n_i, n_in):
    """pft_ptmat_plan's op list, replayed on slot vectors with the pre-rotated
    diagonals of the header's convention, leaves (M v)_{k mod n_o} in slot k."""
    from oracle import ptmatvec as PM
    from paper_1908_06972_amd.ckks import ptmat_plan
    t = 256
    g = np.random.default_rng(n_o * 1000 + n_i + n_in)
    M = g.normal(size=(n_o, n_in * n_i))
    v = g.normal(size=n_in * n_i)
    inputs = [np.tile(v[c * n_i:(c + 1) * n_i], t // n_i) for c in range(n_in)]
    P = PM.prerotated_diagonals(M, n_o, n_i, n_in, t)
    b, G = PM.bsgs_plan(n_o, n_in)
    diags = [P[c][gg][r] for c in range(n_in) for gg in range(G) for r in range(b)]
    ops = ptmat_plan(n_o, n_i, n_in)
    y = _replay_plan(ops, inputs, diags, t)
    assert np.allclose(y, (M @ v)[np.arange(t) % n_o])
    rot = [o for o in ops if o[0] == "rotate"]
    assert len(rot) == n_in * (b - 1) + (G - 1) + int(np.log2(n_i // n_o))


def test_ptmat_plan_rejections_and_short_buffer():
    lib = N.load()
    cnt = ctypes.c_uint32()
    for args in ((3, 16, 1), (32, 16, 1), (4, 16, 0), (4, 12, 1)):
        assert lib.pft_ptmat_plan(*args, None, 0, ctypes.byref(cnt)) == N.PFT_EINVAL
    assert lib.pft_ptmat_plan(16, 64, 2, None, 0, ctypes.byref(cnt)) == N.PFT_OK
    full = cnt.value
    buf = (N.OpDesc * 3)()
    assert lib.pft_ptmat_plan(16, 64, 2, buf, 3, ctypes.byref(cnt)) == N.PFT_OK
    assert cnt.value == full and buf[0].kind == N.PFT_OP_ROTATE
