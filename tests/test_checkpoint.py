"""tn_result_combine, the host-side (+) of results over disjoint slice
ranges (checkpoint and resume of sliced contractions, Sec. 4.2), on results
built by hand: the combination rules of each algebra, the exact count's CRT
recomputed from added residues (and its check prime catching a value beyond
the CRT range), and the refusals."""
import math

import pytest

import paper_2501_00227_amd as tn


def _is_prime(n):
    if n < 2:
        return False
    f = 2
    while f * f <= n:
        if n % f == 0:
            return False
        f += 1
    return True


def _primes_below_2_30(k):
    out, n = [], (1 << 30) - 1
    while len(out) < k:
        if _is_prime(n):
            out.append(n)
        n -= 2
    return out


def _res(semiring, **kw):
    r = tn.tn_result()
    r.semiring = tn.SEMIRING[semiring] if isinstance(semiring, str) else semiring
    for k, v in kw.items():
        setattr(r, k, v)
    return r


def test_counting_tropical_and_tropical_rules():
    ct = tn.SEMIRING["counting_tropical"]
    a = _res(ct, size_i32=5, size_f32=5.0, count_mod_2_64=3)
    assert (tn.result_combine(a, _res(ct, size_i32=5, size_f32=5.0, count_mod_2_64=4)).count_mod_2_64) == 7
    r = tn.result_combine(a, _res(ct, size_i32=6, size_f32=6.0, count_mod_2_64=1))
    assert (r.size_i32, r.count_mod_2_64) == (6, 1)
    r = tn.result_combine(_res(ct, size_i32=9, size_f32=9.0, count_mod_2_64=2), a)
    assert (r.size_i32, r.count_mod_2_64) == (9, 2)
    wrap = tn.result_combine(_res(ct, size_i32=1, count_mod_2_64=2 ** 64 - 1), _res(ct, size_i32=1, count_mod_2_64=5))
    assert wrap.count_mod_2_64 == 4  # counts mod 2^64
    none = _res(ct, size_i32=-(1 << 31), size_is_neg_inf=1)
    r = tn.result_combine(none, a)
    assert (r.size_i32, r.count_mod_2_64, r.size_is_neg_inf) == (5, 3, 0)
    assert tn.result_combine(none, none).size_is_neg_inf == 1
    t32 = tn.SEMIRING["tropical_i32"]
    assert tn.result_combine(_res(t32, size_i32=4), _res(t32, size_i32=7)).size_i32 == 7
    tf = tn.SEMIRING["tropical_f32"]
    assert tn.result_combine(_res(tf, size_f32=2.5), _res(tf, size_f32=1.25)).size_f32 == 2.5
    assert tn.result_combine(_res(tf, size_f32=-math.inf, size_is_neg_inf=1), _res(tf, size_f32=0.5)).size_f32 == 0.5


def _count_result(x, primes):
    r = _res("count_exact", nresidues=len(primes))
    for k, p in enumerate(primes):
        r.primes[k] = p
        r.residues[k] = x % p
    return r


def test_exact_count_residues_added_and_recombined():
    primes = _primes_below_2_30(4)  # three for the value, the last checks it
    x, y = 2 ** 70 + 12345, 3 ** 40 + 7
    r = tn.result_combine(_count_result(x, primes), _count_result(y, primes))
    got = sum(int(r.count_limbs[k]) << (32 * k) for k in range(r.count_nlimbs))
    assert got == x + y and r.count_mod_2_64 == (x + y) % 2 ** 64
    assert [r.residues[k] for k in range(4)] == [(x + y) % p for p in primes]
    # a sum beyond the product of the three value primes: the check prime disagrees
    big = primes[0] * primes[1] * primes[2] - 1
    with pytest.raises(tn.TnError) as ei:
        tn.result_combine(_count_result(big, primes), _count_result(big, primes))
    assert ei.value.code == tn.TN_EOVERFLOW
    other = _count_result(x, _primes_below_2_30(5)[1:])
    with pytest.raises(tn.TnError):
        tn.result_combine(_count_result(x, primes), other)


def test_partition_function_sum():
    z = tn.SEMIRING["partition_f32"]
    a = _res(z, z_mant=1.5, z_exp2=10, z_range_log2=3.0)
    b = _res(z, z_mant=1.25, z_exp2=8, z_range_log2=7.5)
    r = tn.result_combine(a, b)
    assert (r.z_mant, r.z_exp2, r.z_range_log2) == (1.8125, 10, 7.5)  # 1536 + 320 = 1856
    assert r.z == 1856.0 and abs(r.log_z - math.log(1856.0)) < 1e-12
    far = _res(z, z_mant=1.0, z_exp2=5000)
    r = tn.result_combine(far, b)
    assert (r.z_mant, r.z_exp2, r.z) == (1.0, 5000, math.inf)
    assert abs(r.log_z - 5000 * math.log(2.0)) < 1e-9
    zero = _res(z, z_mant=0.0, z_exp2=0)
    r = tn.result_combine(zero, b)
    assert (r.z_mant, r.z_exp2) == (1.25, 8)


def test_refusals():
    with pytest.raises(tn.TnError):
        tn.result_combine(_res("tropical_i32", size_i32=1), _res("counting_tropical", size_i32=1))
    with pytest.raises(tn.TnError):
        tn.result_combine(_res(6), _res(6))  # an internal algebra: no combination
