"""Planted mistakes in the oracle (on the CPU only): each mutant must make at
least one pin fail, which shows that the pins can see that kind of error."""

import numpy as np
import pytest

from oracle import ckks as C
from tests import test_oracle_ring as TR
from tests import test_oracle_scheme as TS


def _tiny():
    P = C.Params(**TS.TINY)
    import synth as S
    return P, S.key_draws(3, P.n, P.q)


def _expect_fail(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_mutant_rescale_without_rounding_offset(monkeypatch):
    real = C.rescale
    monkeypatch.setattr(C, "rescale", lambda P, x, mode="round": real(P, x, mode="floor"))
    _expect_fail(TR.test_rescale_matches_bigint_division, "round")


def test_mutant_automorphism_without_sign(monkeypatch):
    def bad(a, kappa, mods, n):
        out = np.empty_like(a)
        for j in range(n):
            out[:, (j * kappa) % (2 * n) % n] = a[:, j]
        return out
    monkeypatch.setattr(C, "automorphism", bad)
    _expect_fail(TR.test_automorphism_is_substitution, 3)


def test_mutant_tensor_dropped_cross_term(monkeypatch):
    def bad(params, x, y):
        mods = params.q[:x.level]
        return (C.ring_mul(params, x.c0, y.c0, mods), C.ring_mul(params, x.c0, y.c1, mods),
                C.ring_mul(params, x.c1, y.c1, mods))
    monkeypatch.setattr(C, "tensor", bad)
    _expect_fail(TS.test_tensor_exact, _tiny())


def test_mutant_gadget_on_wrong_digit(monkeypatch):
    real = C.switch_key

    def bad(params, s, s_prime, a, e):
        k = real(params, s, s_prime, a, e)
        k.b = k.b[::-1]
        k.a = k.a[::-1]
        return k
    monkeypatch.setattr(C, "switch_key", bad)
    _expect_fail(TS.test_switch_key_gadget_exact, _tiny(), "relin")


def test_mutant_moddown_missing_inverse(monkeypatch):
    def bad(params, acc, level):
        qs = params.q[:level]
        conv = C.base_convert(acc[level:], params.p, qs, params.n)
        return C.sub(acc[:level], conv, qs)
    monkeypatch.setattr(C, "mod_down", bad)
    _expect_fail(TS.test_key_switch_error_bound, _tiny(), 3)


def test_mutant_encode_wrong_generator(monkeypatch):
    def bad(n, n_slots):
        e = np.empty(n_slots, dtype=np.int64)
        x = 1
        for j in range(n_slots):
            e[j] = x
            x = x * 3 % (2 * n)
        return e
    monkeypatch.setattr(C, "slot_exponents", bad)
    _expect_fail(TS.test_c1_rotate, TS.c1_env(), 3)


def test_mutant_decrypt_sign(monkeypatch):
    def bad(params, s, ct):
        mods = params.q[:ct.level]
        return C.sub(ct.c0, C.ring_mul(params, ct.c1, C.rns_from_int(s, mods), mods), mods)
    monkeypatch.setattr(C, "decrypt", bad)
    _expect_fail(TS.test_encrypt_decrypt_exact, _tiny())


def test_mutant_ctmatvec_unrotated_giant_step(monkeypatch):
    """A giant-step partial sum added without its rotation by g b."""
    from oracle import training as T
    from tests import test_oracle_training as TT
    real_rotate = C.rotate
    C.set_mul_mode(1)
    fx = TT.make_train()

    def bad_ctmatvec(params, inputs, diags, n_o, n_i, rlk, rot_keys):
        b, G = T.bsgs_plan(n_o)
        baby = [[v if r == 0 else real_rotate(params, v, r, rot_keys[r]) for r in range(b)] for v in inputs]
        scale = diags[0][0][0].scale * inputs[0].scale
        total = None
        for g in range(G):
            pairs = [(diags[c][g][r], baby[c][r]) for c in range(len(inputs)) for r in range(b)]
            acc = T.relin_tensor(params, T._tensor_sum(params, pairs), rlk, scale)
            total = acc if total is None else C.hadd(params, total, acc)
        s = n_o
        while s < n_i:
            total = C.hadd(params, total, real_rotate(params, total, s, rot_keys[s]))
            s *= 2
        return total
    monkeypatch.setattr(T, "ctmatvec", bad_ctmatvec)
    _expect_fail(TT.test_encrypted_ctmatvec, fx)


def test_mutant_softmax_wrong_shift(monkeypatch):
    """(X + 1)^2 / 8 in place of (X + 2)^2 / 8 - 1/4."""
    from oracle import training as T
    from tests import test_oracle_training as TT
    C.set_mul_mode(1)
    fx = TT.make_train()
    real = T.hadd_const
    monkeypatch.setattr(T, "hadd_const", lambda P, x, v: real(P, x, 1.0 if v == 2.0 else v))
    _expect_fail(TT.test_encrypted_softmax_approx, fx)


def test_mutant_colpack_half_totalsum(monkeypatch):
    """TotalSum over half of the slots in the column-packed stage 1."""
    from tests import test_oracle_colpack as TC
    C.set_mul_mode(1)
    fx = TC.make_small()
    real = C.total_sum
    monkeypatch.setattr(C, "total_sum", lambda P, x, n_slots, keys: real(P, x, n_slots // 2, keys))
    _expect_fail(TC.test_stage1_replicates_column_dot, fx)


# ---- the seeded sampler (oracle/sampler.py)

def _philox_pins():
    from tests import test_oracle_sampler as TSm
    for key in TSm.KEYS:
        for ctr in TSm.CTRS:
            TSm.test_philox_matches_numpy(key, ctr)


def test_mutant_philox_wrong_weyl_constant(monkeypatch):
    from oracle import sampler as SP
    monkeypatch.setattr(SP, "W1", SP.W1 ^ 1)
    _expect_fail(_philox_pins)


def test_mutant_philox_no_key_bump(monkeypatch):
    from oracle import sampler as SP
    monkeypatch.setattr(SP, "W0", 0)
    monkeypatch.setattr(SP, "W1", 0)
    _expect_fail(_philox_pins)


def test_mutant_philox_swapped_round_outputs(monkeypatch):
    from oracle import sampler as SP
    real = SP.mulhilo
    monkeypatch.setattr(SP, "mulhilo", lambda a, b: tuple(reversed(real(a, b))))
    _expect_fail(_philox_pins)


def test_mutant_gaussian_variance_sigma_not_2sigma(monkeypatch):
    from decimal import Decimal, localcontext

    from oracle import sampler as SP
    from tests import test_oracle_sampler as TSm

    def bad(sigma=SP.SIGMA, bound=SP.BOUND):
        with localcontext() as ctx:
            ctx.prec = 60
            var = Decimal(sigma) * Decimal(sigma)  # exp(-x^2 / sigma^2): the factor 2 dropped
            rho = [(Decimal(-x * x) / var).exp() for x in range(-bound, bound + 1)]
            total, acc, out = sum(rho), Decimal(0), []
            for r in rho[:-1]:
                acc += r
                out.append(int((acc * (1 << 64)) // total))
        return out
    monkeypatch.setattr(SP, "gaussian_cdt", bad)
    _expect_fail(TSm.test_cdt_variance_is_sigma_squared, "3.2", 19)


def test_mutant_uniform_off_by_one(monkeypatch):
    from oracle import sampler as SP
    from tests import test_oracle_sampler as TSm
    real = SP.uniform
    monkeypatch.setattr(SP, "uniform", lambda w0, w1, q: real(w0, w1, q) + np.uint64(1))
    _expect_fail(TSm.test_uniform_is_its_definition_and_in_range)


def test_mutant_ternary_unbalanced(monkeypatch):
    from oracle import sampler as SP
    from tests import test_oracle_sampler as TSm
    monkeypatch.setattr(SP, "ternary", lambda w0: (w0 % np.uint64(4)).astype(np.int64) - 1)
    _expect_fail(TSm.test_gaussian_and_ternary_draws)
