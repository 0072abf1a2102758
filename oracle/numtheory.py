"""Number theory for the oracle, in Python integers (test infrastructure only).

Section 1 of the paper fixes the fields of interest: F_p with p = k 2^l + 1 where
p fits in a 32- or 64-bit word and l is large.  Section 5.1 needs a primitive n-th
root of unity w (w^n = 1, w^j != 1 for 0 < j < n).  Section 2 defines the
precomputed constants: Barrett's pre-inverse q = floor(2^(s+t)/p) (section 2.2,
Table 3), the fixed-multiplicand constant psi = floor(2^n y / p) (Function 8) and
Montgomery's rho, chi with rho 2^m - chi p = 1 (section 2.3).
"""
from __future__ import annotations

# Deterministic Miller-Rabin: the first twelve primes as bases are enough for every
# n < 3.3e24 (Sorenson and Webster), which covers all 64-bit integers.
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for q in _MR_BASES:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x == 1 or x == n - 1:
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def two_adic(p: int) -> tuple[int, int]:
    """(k, l) with p - 1 = k 2^l and k odd."""
    k, l = p - 1, 0
    while k % 2 == 0 and k:
        k //= 2
        l += 1
    return k, l


def prime_factors(m: int) -> list[int]:
    """Distinct prime factors by trial division (m = p - 1 is 2^l times a small k)."""
    out = []
    d = 2
    while d * d <= m:
        if m % d == 0:
            out.append(d)
            while m % d == 0:
                m //= d
        d += 1 if d == 2 else 2
    if m > 1:
        out.append(m)
    return out


def is_generator(g: int, p: int) -> bool:
    """g generates F_p^* iff g^((p-1)/q) != 1 for every prime q | p - 1."""
    if g % p == 0:
        return False
    return all(pow(g, (p - 1) // q, p) != 1 for q in prime_factors(p - 1))


def smallest_generator(p: int) -> int:
    g = 2
    while not is_generator(g, p):
        g += 1
    return g


def root_of_unity(p: int, n: int, g: int | None = None) -> int:
    """w_n = g^((p-1)/n), a primitive n-th root of unity when g generates F_p^*."""
    if (p - 1) % n:
        raise ValueError("n does not divide p - 1")
    if g is None:
        g = smallest_generator(p)
    return pow(g, (p - 1) // n, p)


def has_exact_order(w: int, n: int, p: int) -> bool:
    """w^n = 1 and w^(n/q) != 1 for each prime q | n."""
    if pow(w, n, p) != 1:
        return False
    return all(pow(w, n // q, p) != 1 for q in prime_factors(n)) if n > 1 else True


def largest_prime_below(bound_log2: int, l: int) -> int:
    """Largest prime p < 2^bound_log2 with p = 1 mod 2^l (p = k 2^l + 1, k searched
    downward) -- the rule that fixes the ~62-bit prime of the serving mix."""
    k = ((1 << bound_log2) - 2) >> l
    while k > 0:
        p = (k << l) + 1
        if p < (1 << bound_log2) and is_prime(p):
            return p
        k -= 1
    raise ValueError("no prime found")


def barrett_params(p: int, n: int) -> dict:
    """Section 2.2 / Table 3: r with 2^(r-1) < p <= 2^r, and (alpha, s, t, h) for the
    tightest column the bit-size allows; q = floor(2^(s+t)/p)."""
    r = (p - 1).bit_length()
    if r <= n - 2:
        alpha, s, t, h = 1 << (n - 2), max(r - 2, 0), n + 1, 1
    elif r <= n - 1:
        alpha, s, t, h = 1 << (n - 1), r - 1, n, 2
    else:
        alpha, s, t, h = 1 << n, r - 1, n, 3
    return dict(r=r, alpha=alpha, s=s, t=t, h=h, q=(1 << (s + t)) // p)


def shoup_constant(y: int, p: int, n: int) -> int:
    """Function 8's psi = floor(2^n y / p)."""
    return (y << n) // p


def montgomery_constants(p: int, m: int) -> tuple[int, int]:
    """Section 2.3: (rho, chi) with 0 < chi < 2^m, 0 < rho < p, rho 2^m - chi p = 1,
    by the extended Euclidean algorithm."""
    # Solve rho * 2^m = 1 (mod p): rho = (2^m)^-1 mod p, then chi = (rho 2^m - 1)/p.
    old_r, r = (1 << m) % p, p
    old_s, s = 1, 0
    while r:
        qt = old_r // r
        old_r, r = r, old_r - qt * r
        old_s, s = s, old_s - qt * s
    if old_r != 1:
        raise ValueError("2^m not invertible mod p")
    rho = old_s % p
    chi = (rho * (1 << m) - 1) // p
    return rho, chi
