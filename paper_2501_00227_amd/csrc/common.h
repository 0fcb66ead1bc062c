// Shared host-side definitions of the tensor-network library: status plumbing,
// index bitsets, the random stream used by the planner, and small helpers.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <string>
#include <vector>

#include "../../include/tn.h"

namespace tn {

// ---------------------------------------------------------------- errors --
// Every ABI call returns a tn_status; the text of the last failure on this
// thread is kept for tn_last_error().
void set_error(const std::string& msg);
tn_status fail(tn_status st, const std::string& msg);

// ----------------------------------------------------------------- random --
// SplitMix64 seeding a xoshiro256** stream (Blackman & Vigna 2018).
struct Rng {
    uint64_t s[4];
    explicit Rng(uint64_t seed = 0) { reseed(seed); }
    void reseed(uint64_t seed) {
        uint64_t z = seed;
        for (int i = 0; i < 4; i++) {
            z += 0x9E3779B97F4A7C15ull;
            uint64_t x = z;
            x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
            x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
            s[i] = x ^ (x >> 31);
        }
    }
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t next() {
        uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], 45);
        return r;
    }
    double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
    uint32_t below(uint32_t n) { return (uint32_t)(((next() >> 32) * (uint64_t)n) >> 32); }
};

// ------------------------------------------------------------------- bits --
// A set of vertex indices as a fixed-width bitset; W 64-bit words.
template <int W>
struct Bits {
    uint64_t w[W];
    Bits() { std::memset(w, 0, sizeof w); }
    static Bits one(int i) {
        Bits b;
        b.set(i);
        return b;
    }
    void set(int i) { w[i >> 6] |= 1ull << (i & 63); }
    void clear(int i) { w[i >> 6] &= ~(1ull << (i & 63)); }
    bool has(int i) const { return (w[i >> 6] >> (i & 63)) & 1; }
    int count() const {
        int c = 0;
        for (int k = 0; k < W; k++) c += __builtin_popcountll(w[k]);
        return c;
    }
    bool empty() const {
        uint64_t o = 0;
        for (int k = 0; k < W; k++) o |= w[k];
        return o == 0;
    }
    Bits operator|(const Bits& o) const {
        Bits r;
        for (int k = 0; k < W; k++) r.w[k] = w[k] | o.w[k];
        return r;
    }
    Bits operator&(const Bits& o) const {
        Bits r;
        for (int k = 0; k < W; k++) r.w[k] = w[k] & o.w[k];
        return r;
    }
    Bits operator-(const Bits& o) const {
        Bits r;
        for (int k = 0; k < W; k++) r.w[k] = w[k] & ~o.w[k];
        return r;
    }
    bool operator==(const Bits& o) const { return std::memcmp(w, o.w, sizeof w) == 0; }
    bool operator!=(const Bits& o) const { return !(*this == o); }
    bool intersects(const Bits& o) const {
        for (int k = 0; k < W; k++)
            if (w[k] & o.w[k]) return true;
        return false;
    }
    template <class F>
    void for_each(F f) const {
        for (int k = 0; k < W; k++) {
            uint64_t x = w[k];
            while (x) {
                int b = __builtin_ctzll(x);
                f(k * 64 + b);
                x &= x - 1;
            }
        }
    }
    std::vector<int> list() const {
        std::vector<int> v;
        for_each([&](int i) { v.push_back(i); });
        return v;
    }
};

// log2(2^a + 2^b) without overflow, for complexity sums kept in log2 form.
inline double log2_add(double a, double b) {
    if (a < b) std::swap(a, b);
    if (b == -1.0 / 0.0) return a;
    return a + std::log2(1.0 + std::exp2(b - a));
}

}  // namespace tn
