"""Big-integer helpers for pinning the oracle.  They use Python integers and
sympy only, and share nothing with the oracle's own code paths."""

from sympy.ntheory.modular import crt as sympy_crt


def negacyclic_int(a, b, n):
    """Product of two integer polynomials in Z[X]/(X^N+1), exact."""
    full = [0] * (2 * n)
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            full[i + j] += ai * bj
    return [full[k] - full[k + n] for k in range(n)]


def add_int(a, b):
    return [x + y for x, y in zip(a, b)]


def mod_list(a, q):
    return [x % q for x in a]


def crt_value(residues, moduli):
    """The integer in [0, prod(moduli)) with the given residues (sympy)."""
    return int(sympy_crt([int(m) for m in moduli], [int(r) for r in residues])[0])


def bitrev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def evaluate(a, x, q):
    """a(x) mod q by Horner's rule."""
    acc = 0
    for c in reversed(list(a)):
        acc = (acc * x + int(c)) % q
    return acc
