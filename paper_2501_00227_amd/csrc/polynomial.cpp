// Independence polynomial by the finite-field method (Sec. 6.2; the
// GraphPolynomial property of the Sec. 5 table): the counting network is
// contracted with vertex tensors [1, t] for t = 0 .. alpha in arithmetic mod
// several primes (every evaluation is one mod-p pass of the persistent
// batched executor, many passes per launch), the values are interpolated mod
// each prime, and the coefficients recombined by CRT with one more prime as a
// check.  alpha (the largest independent-set size, the polynomial's degree)
// and the total count (which bounds every coefficient) come from one tropical
// and one exact-count contraction first.
#include <algorithm>
#include <cstring>

#include "batch_host.h"

namespace tn {

namespace {

uint32_t pw(uint64_t b, uint64_t e, uint32_t p) {
    uint64_t r = 1 % p;
    b %= p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return (uint32_t)r;
}

bool prime32(uint32_t p) {
    if (p < 2) return false;
    for (uint64_t d = 2; d * d <= p; d++)
        if (p % d == 0) return false;
    return true;
}

// little-endian 32-bit limbs
struct Big {
    std::vector<uint32_t> d;
    void mul_add(uint32_t m, uint32_t a) {  // *this = *this * m + a
        uint64_t carry = a;
        for (auto& x : d) {
            uint64_t t = (uint64_t)x * m + carry;
            x = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) d.push_back((uint32_t)carry);
    }
    uint32_t mod(uint32_t p) const {
        uint64_t r = 0;
        for (size_t k = d.size(); k-- > 0;) r = ((r << 32) | d[k]) % p;
        return (uint32_t)r;
    }
    void add(const Big& o) {
        uint64_t carry = 0;
        if (d.size() < o.d.size()) d.resize(o.d.size(), 0u);
        for (size_t k = 0; k < d.size(); k++) {
            uint64_t t = (uint64_t)d[k] + (k < o.d.size() ? o.d[k] : 0u) + carry;
            d[k] = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) d.push_back((uint32_t)carry);
    }
    void trim() {
        while (!d.empty() && d.back() == 0) d.pop_back();
    }
    int bits() const {
        for (size_t k = d.size(); k-- > 0;)
            if (d[k]) return (int)(32 * k) + 32 - __builtin_clz(d[k]);
        return 0;
    }
};

// Newton interpolation mod p through (t, y[t]), t = 0 .. D; returns the
// monomial coefficients c[0 .. D].
std::vector<uint32_t> interpolate(const std::vector<uint32_t>& y, uint32_t p) {
    const int D = (int)y.size() - 1;
    std::vector<uint64_t> a(y.begin(), y.end());
    for (int j = 1; j <= D; j++) {
        const uint64_t inv = pw(j, p - 2, p);  // points are 0..D: x_i - x_{i-j} = j
        for (int i = D; i >= j; i--) a[i] = (a[i] + p - a[i - 1]) % p * inv % p;
    }
    // sum_j a_j prod_{m<j} (x - m), by Horner from the top
    std::vector<uint64_t> c(D + 1, 0);
    c[0] = a[D];
    int deg = 0;
    for (int j = D - 1; j >= 0; j--) {
        // c <- c * (x - j) + a_j
        c[deg + 1] = c[deg];
        for (int k = deg; k >= 1; k--) c[k] = (c[k - 1] + (uint64_t)(p - j % p) * c[k]) % p;
        c[0] = ((uint64_t)(p - j % p) * c[0] + a[j]) % p;
        deg++;
    }
    return std::vector<uint32_t>(c.begin(), c.end());
}

}  // namespace

tn_status solve_polynomial(tn_ctx* ctx, const Net& net, const Plan& plan, int limbs, uint32_t* coeffs, int* degree) {
    if (limbs < 1 || !coeffs) return fail(TN_EINVAL, "coeffs and limbs >= 1 are required");
    if (net.kind != 0) return fail(TN_EINVAL, "the independence polynomial needs an independent-set network");
    for (float w : net.w)
        if (w != 1.0f) return fail(TN_EINVAL, "the independence polynomial needs unit weights");
    if (!plan.sliced.empty()) return fail(TN_EINVAL, "the independence polynomial needs an unsliced plan");
    if (net.nv > 512) return fail(TN_ETOOBIG, "the independence polynomial is limited to 512 vertices");
    std::memset(coeffs, 0, sizeof(uint32_t) * (size_t)limbs * (size_t)(net.nv + 1));
    // 1. degree (largest independent set) and total count
    std::vector<BatchItem> items(2);
    for (auto& it : items) {
        it.net = &net;
        it.plan = &plan;
        it.opts = tn_solve_opts{};
    }
    items[0].opts.semiring = TN_TROPICAL_I32;
    items[1].opts.semiring = TN_COUNT_EXACT;
    std::vector<tn_result> first;
    tn_status st = solve_batch_sync(ctx, items, first);
    if (st != TN_OK) return st;
    const int D = first[0].size_is_neg_inf ? 0 : first[0].size_i32;
    Big total;
    total.d.assign(first[1].count_limbs, first[1].count_limbs + first[1].count_nlimbs);
    total.trim();
    // 2. primes: their product (without the check prime) exceeds the total
    // count, hence every coefficient
    std::vector<uint32_t> primes;
    int need = total.bits() + 1, have = 0;
    for (uint32_t p = (1u << 30) - 1; (have < need || primes.size() < 2) && p > (1u << 29); p -= 2)
        if (prime32(p)) {
            primes.push_back(p);
            have += 29;
        }
    for (uint32_t p = primes.back() - 2; p > (1u << 29); p -= 2)
        if (prime32(p)) {  // the check prime
            primes.push_back(p);
            break;
        }
    const int R = (int)primes.size();
    // 3. evaluations P(t) mod p for t = 0 .. D, at most 256 passes per launch
    std::vector<PassSpec> all;
    for (int r = 0; r < R; r++)
        for (int t = 0; t <= D; t++) {
            PassSpec ps;
            ps.dsr = DSR_MODP;
            ps.prime = primes[r];
            ps.xval = (uint32_t)t;
            all.push_back(ps);
        }
    std::vector<uint32_t> vals(all.size());
    for (size_t b = 0; b < all.size(); b += 256) {
        std::vector<PassSpec> chunk(all.begin() + b, all.begin() + std::min(all.size(), b + 256));
        std::vector<std::array<unsigned char, kAccSlotBytes>> accs;
        st = run_passes_sync(ctx, net, plan, chunk, accs);
        if (st != TN_OK) return st;
        for (size_t k = 0; k < chunk.size(); k++) {
            uint32_t xm;
            std::memcpy(&xm, accs[k].data(), 4);
            const uint32_t p = chunk[k].prime;
            vals[b + k] = (uint32_t)((uint64_t)xm * pw((1ull << 32) % p, p - 2, p) % p);  // out of Montgomery form
        }
    }
    // 4. interpolate mod each prime, CRT (Garner) over all but the last prime
    std::vector<std::vector<uint32_t>> res(R);
    for (int r = 0; r < R; r++)
        res[r] = interpolate(std::vector<uint32_t>(vals.begin() + (size_t)r * (D + 1),
                                                   vals.begin() + (size_t)(r + 1) * (D + 1)),
                             primes[r]);
    Big sum;
    int deg = 0;
    for (int k = 0; k <= D; k++) {
        Big x, M;
        x.d = {res[0][k]};
        M.d = {primes[0]};
        for (int r = 1; r < R - 1; r++) {
            const uint32_t p = primes[r];
            const uint32_t t = (uint32_t)((uint64_t)((res[r][k] + (uint64_t)p - x.mod(p)) % p) *
                                          pw(M.mod(p), p - 2, p) % p);
            Big add = M;
            add.mul_add(t, 0);
            x.add(add);
            M.mul_add(p, 0);
        }
        x.trim();
        if (x.mod(primes[R - 1]) != res[R - 1][k])
            return fail(TN_EOVERFLOW, "independence polynomial: the check prime disagrees");
        if ((int)x.d.size() > limbs) return fail(TN_EOVERFLOW, "a coefficient needs more limbs than given");
        for (size_t l = 0; l < x.d.size(); l++) coeffs[(size_t)k * limbs + l] = x.d[l];
        if (!x.d.empty()) deg = k;
        sum.add(x);
    }
    sum.trim();
    if (sum.d != total.d) return fail(TN_EDEVICE, "independence polynomial: coefficients do not sum to the count");
    if (degree) *degree = deg;
    return TN_OK;
}

}  // namespace tn
