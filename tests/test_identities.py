"""Arithmetic identities the kernels rely on, checked on the CPU.

First in closed form: the canonical First recurrence first[Lmax] = 0,
first[l] = ceil((first[l+1] + cnt[l+1]) / 2) equals
ceil(S_l / 2^(Lmax - l)) with S_l = sum over k > l of cnt[k] 2^(Lmax - k)
(ceil(ceil(x / 2) / 2^j) = ceil(x / 2^(j+1)) for integers).  The codebook's
small-book path computes First this way with one wave suffix sum."""
import random


def first_recurrence(cnt, lmax):
    f = [0] * (lmax + 2)
    for l in range(lmax - 1, 0, -1):
        f[l] = (f[l + 1] + cnt[l + 1] + 1) // 2
    return f[1:lmax + 1]


def first_closed_form(cnt, lmax):
    out = []
    for l in range(1, lmax + 1):
        s = sum(cnt[k] << (lmax - k) for k in range(l + 1, lmax + 1))
        out.append((s + (1 << (lmax - l)) - 1) >> (lmax - l))
    return out


def test_first_closed_form_matches_recurrence():
    rng = random.Random(11)
    for _ in range(5000):
        lmax = rng.randint(1, 46)
        cnt = [0] + [rng.choice([0, 1, 2, rng.randint(0, 300)]) for _ in range(lmax)] + [0]
        assert first_closed_form(cnt, lmax) == first_recurrence(cnt, lmax)


def test_first_closed_form_fits_53_bits_for_small_books():
    """At most 256 codes of length <= 46 (sums of counts < 2^32): S < 2^53."""
    lmax = 46
    cnt = [0] * (lmax + 2)
    cnt[2] = 256
    s = max(sum(cnt[k] << (lmax - k) for k in range(l + 1, lmax + 1)) for l in range(1, lmax + 1))
    assert s < 1 << 53
