"""Abelian charges and fermion parity (Sec. II.A, II.B).

Charges are tuples: ``(q,)`` for Z2 (q in {0, 1}) and U(1); ``(n_up, n_dn)``
for U(1)xU(1). Sums are taken modulo 2 for Z2 (finite Abelian group, Sec.
II.A) and over the integers for U(1). Parity: a Z2 charge is its own parity;
an odd U(1) charge has odd parity (Sec. II.B); for U(1)xU(1) the parity is
that of the total particle number ``n_up + n_dn``.
"""

Z2 = "Z2"
U1 = "U1"
U1U1 = "U1xU1"


def nq(sym):
    return 2 if sym == U1U1 else 1


def canon(sym, q):
    q = tuple(int(x) for x in q)
    if sym == Z2:
        return (q[0] % 2,)
    return q


def zero(sym):
    return (0,) * nq(sym)


def add(sym, a, b):
    return canon(sym, tuple(x + y for x, y in zip(a, b)))


def neg(sym, a):
    return canon(sym, tuple(-x for x in a))


def signed(sym, dual, q):
    """sigma(dual) * q with sigma('+') = +1, sigma('-') = -1 (dual 1 = '-')."""
    return neg(sym, q) if dual else canon(sym, q)


def parity(sym, q):
    return int(sum(q)) % 2
