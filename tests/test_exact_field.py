"""CPU checks of the number facts the exact transform relies on (Z_p with
p = 2^64 - 2^32 + 1): p is prime, p - 1 has the factor 2^32 (roots of unity of
every order 2^k, k <= 32), 7^((p-1)/2^32) has order exactly 2^32, the two
congruences the reduction uses, and that every convolution coefficient of the
admitted operands is its own residue and fits the carry scan's 48-bit input."""
P = 2 ** 64 - 2 ** 32 + 1


def is_prime(n):
    """Deterministic Miller-Rabin for n < 3.3 * 10^24 (bases 2..41)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for q in small:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_modulus_is_prime_with_power_of_two_roots():
    assert is_prime(P)
    assert not is_prime(P + 2) and is_prime(97) and not is_prime(91)
    assert P - 1 == 2 ** 32 * (2 ** 32 - 1)


def test_root_of_order_2_to_the_32():
    w = pow(7, (P - 1) >> 32, P)
    assert pow(w, 2 ** 32, P) == 1
    assert pow(w, 2 ** 31, P) == P - 1  # so the order is exactly 2^32
    for k in (1, 9, 18, 27):
        wk = pow(w, 2 ** (32 - k), P)
        assert pow(wk, 2 ** (k - 1), P) == P - 1


def test_reduction_congruences():
    assert 2 ** 64 % P == 2 ** 32 - 1
    assert 2 ** 96 % P == P - 1


def test_coefficients_are_their_own_residues():
    # operands of at most 2^26 bytes each (na + nb - 1 <= 2^27)
    worst = 2 ** 26 * 255 ** 2
    assert worst < 2 ** 48 < P
