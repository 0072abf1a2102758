"""The truncated Fourier transform and the paper's Algorithm 1, in Python integers.

Test infrastructure only; small sizes (pure-Python loops).

Section 5.1 defines, for n = 2^k and w a primitive n-th root of unity,
  FFT_w(a)_i = sum_j w^(ij) a_j = A(w^i),
the bitwise mirror [i]_k, and the truncated transform of an l-tuple
  TFT_w(a) = (A(w^[0]_k), ..., A(w^[l-1]_k)).
Algorithm 1 reduces one TFT of size l over K to a TFT of size lambda = ceil(l / n1)
over K^n1 (vectors of n1 consecutive coefficients), a twiddle step, a full TFT of
size n1 over K^lambda, and a reordering; Proposition 15 states that its output is
A(w^[i]_k) for the first lambda * n1 indices i.
"""
from __future__ import annotations


def mirror(i: int, k: int) -> int:
    """[i]_k: reverse the k low bits of i."""
    r = 0
    for b in range(k):
        r |= ((i >> b) & 1) << (k - 1 - b)
    return r


def eval_poly(a, x: int, p: int) -> int:
    """A(x) for A(X) = sum_j a_j X^j."""
    r = 0
    for c in reversed(list(a)):
        r = (r * x + int(c)) % p
    return r


def tft_definition(a, l: int, n: int, w: int, p: int) -> list[int]:
    """TFT_w(a) of section 5.1: (A(w^[0]_k), ..., A(w^[l-1]_k)), k = log2 n."""
    k = n.bit_length() - 1
    return [eval_poly(a, pow(w, mirror(i, k), p), p) for i in range(l)]


def _tft_vectors(vecs, size: int, order_log2: int, w: int, p: int):
    """TFT of a size-`size` tuple of vectors w.r.t. w of order 2^order_log2, applied
    component-wise: out[i] = sum_j vecs[j] * w^(j [i]_order_log2), i < size."""
    width = len(vecs[0]) if vecs else 0
    out = []
    for i in range(size):
        x = pow(w, mirror(i, order_log2), p)
        acc = [0] * width
        xp = 1
        for j in range(len(vecs)):
            for c in range(width):
                acc[c] = (acc[c] + vecs[j][c] * xp) % p
            xp = xp * x % p
        out.append(acc)
    return out


def algorithm1(a, l: int, n: int, n1: int, w: int, p: int) -> list[int]:
    """Algorithm 1 of section 5.1, step by step.

    a: the l input coefficients (a_i = 0 for i >= l); n = 2^k; n1 = 2^k1 <= l divides n.
    Returns the lambda * n1 values of step 4, which Proposition 15 identifies with
    A(w^[i]_k) for i < lambda * n1.
    """
    k = n.bit_length() - 1
    k1 = n1.bit_length() - 1
    n2 = n // n1
    k2 = n2.bit_length() - 1
    lam = -(-l // n1)
    coeffs = [int(x) for x in a] + [0] * (n - l)
    # Step 1: b_j2 = (a_{j2 n1}, ..., a_{(j2+1) n1 - 1}); TFT of size lambda over K^n1
    # with respect to w^n1 (order n2): bhat[i] stands for b^_{[i]_k2}.
    b = [coeffs[j2 * n1:(j2 + 1) * n1] for j2 in range(lam)]
    bhat = _tft_vectors(b, lam, k2, pow(w, n1, p), p)
    # Step 2: c_j1 = (b^_{[j2],j1} w^(j1 [j2]_k2))_{j2 < lambda}, vectors of K^lambda.
    c = [[bhat[j2][j1] * pow(w, j1 * mirror(j2, k2), p) % p for j2 in range(lam)] for j1 in range(n1)]
    # Step 3: full TFT of size n1 over K^lambda with respect to w^n2 (order n1).
    chat = _tft_vectors(c, n1, k1, pow(w, n2, p), p)
    # Step 4: (c^_{[0],0}, ..., c^_{[n1-1],0}, c^_{[0],1}, ..., c^_{[n1-1],lambda-1}).
    return [chat[j1][j2] for j2 in range(lam) for j1 in range(n1)]


def itft_definition(values, l: int, n: int, w: int, p: int) -> list[int]:
    """The inverse truncated transform by definition: the unique l-tuple
    (a_0, ..., a_{l-1}) whose TFT_w of section 5.1 is `values`, i.e. the solution of
    sum_j a_j x_i^j = values_i, x_i = w^[i]_k (i < l), a Vandermonde system over F_p
    with distinct points, solved by Gauss-Jordan elimination.  O(l^3): small l only."""
    k = n.bit_length() - 1
    xs = [pow(w, mirror(i, k), p) for i in range(l)]
    m = [[pow(x, j, p) for j in range(l)] + [int(values[i]) % p] for i, x in enumerate(xs)]
    for col in range(l):
        piv = next(r for r in range(col, l) if m[r][col] % p)
        m[col], m[piv] = m[piv], m[col]
        inv = pow(m[col][col], p - 2, p)
        m[col] = [v * inv % p for v in m[col]]
        for r in range(l):
            if r != col and m[r][col]:
                f = m[r][col]
                m[r] = [(vr - f * vc) % p for vr, vc in zip(m[r], m[col])]
    return [m[i][l] for i in range(l)]
