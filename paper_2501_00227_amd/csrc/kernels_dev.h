// Device-side building blocks shared by the stream kernels (kernels.hip) and
// the persistent batched kernel (batch_kernels.hip): the element algebras of
// the Sec. 5 property table, leaf initialisation (Sec. 3.2 tensors), one tile
// of the bit permute, one tile of the batched semiring GEMM, the split-K
// reduction of one output and the slice accumulator.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace tn {

typedef int64_t i64;
typedef unsigned long long u64;

struct CTv {  // counting-tropical value: (size, count)
    int n;
    u64 c;
};

// ----------------------------------------------------------- algebras ----
// Each algebra provides zero (additive identity), one (multiplicative
// identity), add, mul, global loads/stores over its planes, and prescale
// (applied to GEMM inputs: the partition function's per-tensor exponent).
template <int D>
struct Alg;

template <>
struct Alg<DSR_TROP_I32> {  // max-plus, -inf = INT_MIN, saturating add
    using V = int;
    __device__ static V zero(const AlgebraParams&) { return INT_MIN; }
    __device__ static V one(const AlgebraParams&) { return 0; }
    __device__ static V add(V a, V b, const AlgebraParams&) { return max(a, b); }
    __device__ static V mul(V a, V b, const AlgebraParams&) { return __builtin_elementwise_add_sat(a, b); }
    __device__ static V weight(float w, const AlgebraParams&) { return (int)w; }
    __device__ static V load(const Planes& p, i64 i) { return ((const int*)p.p0)[i]; }
    __device__ static void store(const Planes& p, i64 i, V v) { ((int*)p.p0)[i] = v; }
    __device__ static V prescale(V v, float) { return v; }
};

template <>
struct Alg<DSR_TROP_F32> {  // max-plus over float32, -inf = -INFINITY
    using V = float;
    __device__ static V zero(const AlgebraParams&) { return -INFINITY; }
    __device__ static V one(const AlgebraParams&) { return 0.0f; }
    __device__ static V add(V a, V b, const AlgebraParams&) { return fmaxf(a, b); }
    __device__ static V mul(V a, V b, const AlgebraParams&) { return a + b; }
    __device__ static V weight(float w, const AlgebraParams&) { return w; }
    __device__ static V load(const Planes& p, i64 i) { return ((const float*)p.p0)[i]; }
    __device__ static void store(const Planes& p, i64 i, V v) { ((float*)p.p0)[i] = v; }
    __device__ static V prescale(V v, float) { return v; }
};

template <>
struct Alg<DSR_CTROP> {  // (size, count): larger size wins, equal sizes add counts
    using V = CTv;
    __device__ static V zero(const AlgebraParams&) { return CTv{INT_MIN, 0ull}; }
    __device__ static V one(const AlgebraParams&) { return CTv{0, 1ull}; }
    __device__ static V add(V a, V b, const AlgebraParams&) {
        int n = max(a.n, b.n);
        u64 c = (a.n == n ? a.c : 0ull) + (b.n == n ? b.c : 0ull);
        return CTv{n, c};
    }
    __device__ static V mul(V a, V b, const AlgebraParams&) {
        return CTv{__builtin_elementwise_add_sat(a.n, b.n), a.c * b.c};
    }
    __device__ static V weight(float w, const AlgebraParams&) { return CTv{(int)w, 1ull}; }
    __device__ static V load(const Planes& p, i64 i) { return CTv{((const int*)p.p0)[i], ((const u64*)p.p1)[i]}; }
    __device__ static void store(const Planes& p, i64 i, V v) {
        ((int*)p.p0)[i] = v.n;
        ((u64*)p.p1)[i] = v.c;
    }
    __device__ static V prescale(V v, float) { return v; }
};

// Truncated polynomial (CountingMax(k), k <= 4, of the Sec. 5 table): the
// four highest-order terms c[0] x^m + c[1] x^(m-1) + c[2] x^(m-2) +
// c[3] x^(m-3) of a polynomial in x whose exponents are integer set weights
// (or -H), counts modulo 2^64.  (+) aligns the two by their top exponent and
// keeps the higher four orders; (x) adds top exponents and multiplies the
// coefficient lists, truncated.  Zero: m = INT_MIN, no counts (as the
// counting tropical algebra, exponents at or below -2^30 mean no term).
struct TP4 {
    int m;
    u64 c[4];
};

template <>
struct Alg<DSR_TPOLY> {
    using V = TP4;
    __device__ static V zero(const AlgebraParams&) { return TP4{INT_MIN, {0ull, 0ull, 0ull, 0ull}}; }
    __device__ static V one(const AlgebraParams&) { return TP4{0, {1ull, 0ull, 0ull, 0ull}}; }
    __device__ static V add(const V& a, const V& b, const AlgebraParams&) {
        const bool sw = b.m > a.m;
        const V& hi = sw ? b : a;
        const V& lo = sw ? a : b;
        // orders below the top: lo's term c[t] lands at hi's c[t + s]
        const long long s = (long long)hi.m - (long long)lo.m;
        V r;
        r.m = hi.m;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            u64 x = 0ull;
#pragma unroll
            for (int t = 0; t <= d; t++) x = s == d - t ? lo.c[t] : x;
            r.c[d] = hi.c[d] + x;
        }
        return r;
    }
    __device__ static V mul(const V& a, const V& b, const AlgebraParams&) {
        V r;
        r.m = __builtin_elementwise_add_sat(a.m, b.m);
#pragma unroll
        for (int d = 0; d < 4; d++) {
            u64 x = 0ull;
#pragma unroll
            for (int t = 0; t <= d; t++) x += a.c[t] * b.c[d - t];
            r.c[d] = x;
        }
        return r;
    }
    __device__ static V weight(float w, const AlgebraParams&) { return TP4{(int)w, {1ull, 0ull, 0ull, 0ull}}; }
    __device__ static V load(const Planes& p, i64 i) {
        const uint4* s = (const uint4*)((const unsigned char*)p.p1 + 32 * i);
        const uint4 x = s[0], y = s[1];
        V r;
        r.m = ((const int*)p.p0)[i];
        r.c[0] = (u64)x.x | ((u64)x.y << 32);
        r.c[1] = (u64)x.z | ((u64)x.w << 32);
        r.c[2] = (u64)y.x | ((u64)y.y << 32);
        r.c[3] = (u64)y.z | ((u64)y.w << 32);
        return r;
    }
    __device__ static void store(const Planes& p, i64 i, const V& v) {
        ((int*)p.p0)[i] = v.m;
        uint4* d = (uint4*)((unsigned char*)p.p1 + 32 * i);
        d[0] = make_uint4((unsigned int)v.c[0], (unsigned int)(v.c[0] >> 32), (unsigned int)v.c[1],
                          (unsigned int)(v.c[1] >> 32));
        d[1] = make_uint4((unsigned int)v.c[2], (unsigned int)(v.c[2] >> 32), (unsigned int)v.c[3],
                          (unsigned int)(v.c[3] >> 32));
    }
    __device__ static V prescale(const V& v, float) { return v; }
};

template <>
struct Alg<DSR_MODP> {  // counting modulo p < 2^30, Montgomery form with R = 2^32
    using V = unsigned int;
    __device__ static V zero(const AlgebraParams&) { return 0u; }
    __device__ static V one(const AlgebraParams& ap) { return ap.r1; }
    __device__ static V add(V a, V b, const AlgebraParams& ap) {
        V s = a + b;
        return s >= ap.p ? s - ap.p : s;
    }
    __device__ static V mul(V a, V b, const AlgebraParams& ap) {
        u64 t = (u64)a * b;                          // < p^2 < 2^62
        unsigned int m = (unsigned int)t * ap.pinv;  // t + m p == 0 mod 2^32
        u64 u = (t + (u64)m * ap.p) >> 32;           // < 2p
        return (V)(u >= ap.p ? u - ap.p : u);
    }
    __device__ static V weight(float, const AlgebraParams& ap) { return ap.xv; }
    __device__ static V load(const Planes& p, i64 i) { return ((const unsigned int*)p.p0)[i]; }
    __device__ static void store(const Planes& p, i64 i, V v) { ((unsigned int*)p.p0)[i] = v; }
    __device__ static V prescale(V v, float) { return v; }
};

template <>
struct Alg<DSR_Z_F32> {  // real (+, x) over float32
    using V = float;
    __device__ static V zero(const AlgebraParams&) { return 0.0f; }
    __device__ static V one(const AlgebraParams&) { return 1.0f; }
    __device__ static V add(V a, V b, const AlgebraParams&) { return a + b; }
    __device__ static V mul(V a, V b, const AlgebraParams&) { return a * b; }
    __device__ static V load(const Planes& p, i64 i) { return ((const float*)p.p0)[i]; }
    __device__ static void store(const Planes& p, i64 i, V v) { ((float*)p.p0)[i] = v; }
    __device__ static V prescale(V v, float s) { return v * s; }
};

__device__ inline float round_bf16(float x) {  // round to nearest even on the top 16 bits
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

template <>
struct Alg<DSR_Z_BF16> : Alg<DSR_Z_F32> {
    __device__ static V prescale(V v, float s) { return round_bf16(v * s); }
};

// The eight largest values with multiplicity (SizeMax(k), k <= 8, of the
// Sec. 5 table: max-plus over sorted lists).  v[0] >= v[1] >= ... >= v[7],
// missing values -inf.  (+) keeps the eight largest of the union of two
// lists, (x) the eight largest pairwise sums.
struct Top8 {
    float v[8];
};

// the eight largest of two sorted lists: max(a[t], b[7 - t]) keeps them as
// a bitonic sequence, which three compare-exchange stages sort
__device__ inline Top8 top8_merge(const Top8& a, const Top8& b) {
    Top8 r;
#pragma unroll
    for (int t = 0; t < 8; t++) r.v[t] = fmaxf(a.v[t], b.v[7 - t]);
#pragma unroll
    for (int d = 4; d >= 1; d >>= 1)
#pragma unroll
        for (int t = 0; t < 8; t++)
            if ((t & d) == 0) {
                const float hi = fmaxf(r.v[t], r.v[t + d]), lo = fminf(r.v[t], r.v[t + d]);
                r.v[t] = hi;
                r.v[t + d] = lo;
            }
    return r;
}

// x joins the sorted list r, keeping the eight largest, when at least F
// entries of r are known to be >= x: entry t > F becomes the median of
// r[t], r[t-1] and x (x clamped into [r[t], r[t-1]]), entry F max(r[F], x).
// Lists hold no NaN (entries are finite or -inf), so the median is exact.
template <int F>
__device__ inline void top8_insert(Top8& r, float x) {
#pragma unroll
    for (int t = 7; t > F; t--) r.v[t] = __builtin_amdgcn_fmed3f(r.v[t], r.v[t - 1], x);
    r.v[F] = fmaxf(r.v[F], x);
}

template <>
struct Alg<DSR_TOPK> {
    using V = Top8;
    __device__ static V zero(const AlgebraParams&) {
        V r;
#pragma unroll
        for (int t = 0; t < 8; t++) r.v[t] = -INFINITY;
        return r;
    }
    __device__ static V one(const AlgebraParams& ap) {
        V r = zero(ap);
        r.v[0] = 0.0f;
        return r;
    }
    __device__ static V add(const V& a, const V& b, const AlgebraParams&) { return top8_merge(a, b); }
    // The candidates a[i] + b[j] with (i+1)(j+1) <= 8 (twenty; no other pair
    // can be among the eight largest).  Start from column j = 0 (sorted), then
    // insert the rest in an order where every pair (i', j') <= (i, j) is
    // already in: then (i+1)(j+1) - 1 entries are known to be >= a[i] + b[j],
    // and its insertion touches only the list's tail.
    __device__ static V mul(const V& a, const V& b, const AlgebraParams&) {
        V r;
#pragma unroll
        for (int i = 0; i < 8; i++) r.v[i] = a.v[i] + b.v[0];
        top8_insert<1>(r, a.v[0] + b.v[1]);
        top8_insert<2>(r, a.v[0] + b.v[2]);
        top8_insert<3>(r, a.v[0] + b.v[3]);
        top8_insert<4>(r, a.v[0] + b.v[4]);
        top8_insert<5>(r, a.v[0] + b.v[5]);
        top8_insert<6>(r, a.v[0] + b.v[6]);
        top8_insert<7>(r, a.v[0] + b.v[7]);
        top8_insert<3>(r, a.v[1] + b.v[1]);
        top8_insert<5>(r, a.v[2] + b.v[1]);
        top8_insert<5>(r, a.v[1] + b.v[2]);
        top8_insert<7>(r, a.v[3] + b.v[1]);
        top8_insert<7>(r, a.v[1] + b.v[3]);
        return r;
    }
    __device__ static V weight(float w, const AlgebraParams& ap) {
        V r = zero(ap);
        r.v[0] = w;
        return r;
    }
    __device__ static V load(const Planes& p, i64 i) {
        const uint4* s = (const uint4*)((const unsigned char*)p.p0 + 32 * i);
        const uint4 x = s[0], y = s[1];
        V r;
        r.v[0] = __uint_as_float(x.x);
        r.v[1] = __uint_as_float(x.y);
        r.v[2] = __uint_as_float(x.z);
        r.v[3] = __uint_as_float(x.w);
        r.v[4] = __uint_as_float(y.x);
        r.v[5] = __uint_as_float(y.y);
        r.v[6] = __uint_as_float(y.z);
        r.v[7] = __uint_as_float(y.w);
        return r;
    }
    __device__ static void store(const Planes& p, i64 i, const V& v) {
        uint4* d = (uint4*)((unsigned char*)p.p0 + 32 * i);
        d[0] = make_uint4(__float_as_uint(v.v[0]), __float_as_uint(v.v[1]), __float_as_uint(v.v[2]),
                          __float_as_uint(v.v[3]));
        d[1] = make_uint4(__float_as_uint(v.v[4]), __float_as_uint(v.v[5]), __float_as_uint(v.v[6]),
                          __float_as_uint(v.v[7]));
    }
    __device__ static V prescale(const V& v, float) { return v; }
};

// acc + a0 b0 + a1 b1 + a2 b2 + a3 b3 (Montgomery form), one reduction:
// the sum of four products is below 4 p^2 < p 2^32 for p < 2^30, so the
// reduced value is below 2p.
__device__ inline unsigned int modp_mac4(unsigned int acc, const unsigned int* a, const unsigned int* b,
                                         const AlgebraParams& ap) {
    const u64 t = (u64)a[0] * b[0] + (u64)a[1] * b[1] + (u64)a[2] * b[2] + (u64)a[3] * b[3];
    const unsigned int m = (unsigned int)t * ap.pinv;
    unsigned int u = (unsigned int)((t + (u64)m * ap.p) >> 32);
    u = min(u, u - ap.p);
    const unsigned int s2 = acc + u;
    return min(s2, s2 - ap.p);
}

// acc + a0 b0 + a1 b1 (mod p) in Montgomery form with one reduction for the two
// products: t = a0 b0 + a1 b1 < 2 p^2 < p 2^32 (p < 2^30), so REDC(t) < 2p and
// REDC(t) = a0 b0 R^-1 + a1 b1 R^-1 (mod p).  min(x, x - p) reduces x < 2p.
__device__ inline unsigned int modp_mac2(unsigned int acc, unsigned int a0, unsigned int b0, unsigned int a1,
                                         unsigned int b1, const AlgebraParams& ap) {
    const u64 t = (u64)a0 * b0 + (u64)a1 * b1;
    const unsigned int m = (unsigned int)t * ap.pinv;
    unsigned int u = (unsigned int)((t + (u64)m * ap.p) >> 32);
    u = min(u, u - ap.p);
    const unsigned int s2 = acc + u;
    return min(s2, s2 - ap.p);
}

template <int D>
constexpr bool is_z() {
    return D == DSR_Z_F32 || D == DSR_Z_BF16;
}

// bytes per entry of plane 0 / plane 1 of an algebra (0: no such plane)
template <int D>
__host__ __device__ constexpr int plane_bytes_dev(int plane) {
    return D == DSR_CTROP   ? (plane == 0 ? 4 : 8)
           : D == DSR_TOPK  ? (plane == 0 ? 32 : 0)
           : D == DSR_TPOLY ? (plane == 0 ? 4 : 32)
                            : (plane == 0 ? 4 : 0);
}

// Partition-function bookkeeping is read and written with device-scope
// atomics only, so it is coherent between workgroups on any chiplet.
__device__ inline unsigned int meta_maxbits(const TensorMeta* m, int i) {
    return __hip_atomic_load(&m[i].maxbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline long long meta_exp(const TensorMeta* m, int i) {
    return __hip_atomic_load(&m[i].exp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void meta_set(TensorMeta* m, int i, long long e, unsigned int bits) {
    __hip_atomic_store(&m[i].exp, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&m[i].maxbits, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&m[i].minnz_inv, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&m[i].operand_range, 0.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned int meta_minnz_inv(const TensorMeta* m, int i) {
    return __hip_atomic_load(&m[i].minnz_inv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// log2(max / smallest nonzero) from a tensor's record (0 when empty)
__device__ inline float bits_range(unsigned mx, unsigned mn_inv) {
    return (mx != 0u && mn_inv != 0u) ? log2f(__uint_as_float(mx)) - log2f(__uint_as_float(~mn_inv)) : 0.0f;
}
__device__ inline float meta_range(const TensorMeta* m, int i) {
    return bits_range(meta_maxbits(m, i), meta_minnz_inv(m, i));
}
__device__ inline void meta_set_exp(TensorMeta* m, int i, long long e) {
    __hip_atomic_store(&m[i].exp, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void meta_max(TensorMeta* m, int i, unsigned int bits) {
    __hip_atomic_fetch_max(&m[i].maxbits, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the smallest nonzero entry, as the complement of its bits under an atomic
// maximum (positive floats order as their bits)
__device__ inline void meta_min_nonzero(TensorMeta* m, int i, float v) {
    if (v > 0.0f && v < INFINITY)
        __hip_atomic_fetch_max(&m[i].minnz_inv, ~__float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The dynamic range of the stored partition-function entries: the largest
// and the smallest nonzero value seen by a thread.
__device__ inline void z_track(float v, float& lmax, float& lmin) {
    lmax = fmaxf(lmax, v);
    if (v > 0.0f) lmin = fminf(lmin, v);
}
// A workgroup barrier that orders LDS only: __syncthreads() would also wait
// for the workgroup's global stores to complete, a round trip on the tail of
// a launch that no LDS exchange needs.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// The extremes of a tensor's stored entries, added to its record.  Atomics
// on one record serialise where its line lives: a large launch first reduces
// over the workgroup (one atomic pair per workgroup); a small one, whose
// cost is the latency of its tail, lets each wave add its own pair.  Every
// thread of the workgroup calls (the branch is uniform over the launch);
// every launch that calls has 256-thread workgroups (reading blockDim would
// cost a vector load, whose wait also waits for the tile's stores).
constexpr unsigned kZWaveAtomicGrid = 64;
constexpr int kZWaves = 4;
__device__ inline void z_meta_block(TensorMeta* m, int i, float lmax, float lmin) {
    __shared__ float2 ext[kZWaves];
    for (int off = 32; off > 0; off >>= 1) {
        lmax = fmaxf(lmax, __shfl_xor(lmax, off));
        lmin = fminf(lmin, __shfl_xor(lmin, off));
    }
    if (gridDim.x > kZWaveAtomicGrid) {
        if ((threadIdx.x & 63) == 0) ext[threadIdx.x >> 6] = make_float2(lmax, lmin);
        lds_barrier();
        // wave 0: lane w takes wave w's pair
        const float2 e = (int)threadIdx.x < kZWaves ? ext[threadIdx.x] : make_float2(0.0f, INFINITY);
        lds_barrier();  // ext is free for the workgroup's next call
        if (threadIdx.x >= 64) return;
        lmax = e.x;
        lmin = e.y;
        for (int off = kZWaves / 2; off > 0; off >>= 1) {
            lmax = fmaxf(lmax, __shfl_xor(lmax, off));
            lmin = fminf(lmin, __shfl_xor(lmin, off));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        if (lmax > 0.0f) meta_max(m, i, __float_as_uint(lmax));
        meta_min_nonzero(m, i, lmin);
    }
}

// exponent m with 2^m <= max < 2^(m+1) of a non-negative float given by its bits
__device__ inline int max_exponent(unsigned int bits) {
    if (bits == 0u) return 0;
    int e = (int)((bits >> 23) & 0xffu);
    return e == 0 ? -126 : e - 127;
}

// --------------------------------------------------------------- leaves --
// A leaf is the product of its factors: the edge tensor B(n_u, n_v) =
// [[1,1],[1,0]] and the vertex tensors W(n) = [1, x^w] folded into it
// (Sec. 3.2), summed over its indices that occur nowhere else, with sliced
// indices fixed to this slice's values.  A fixed vertex (conditioning, the
// fixed vertices of the Sec. 5 network object) multiplies every leaf it
// occurs in by the indicator of its value; the indicator is idempotent, so
// applying it in several leaves changes nothing.
__device__ inline int leaf_fixed(int v, const float* w, const AlgebraParams& ap) {
    return (ap.fix_off >= 0 && v >= 0) ? (int)w[ap.fix_off + v] : -1;
}

__device__ inline int leaf_var_value(int var, const LeafDev& d, int e, const int* spos, u64 sid) {
    if (var == d.var0) return e & 1;
    if (var == d.var1) return (e >> 1) & 1;
    int sp = spos[var];
    if (sp >= 0) return (int)((sid >> sp) & 1ull);
    return -1;  // summed at the leaf
}

template <int D>
__device__ void leaf_one(const LeafDev& d, int leaf_id, const float* w, const int* spos, u64 sid, Planes arena,
                         const AlgebraParams& ap, TensorMeta* meta) {
    using A = Alg<D>;
    using V = typename A::V;
    int nent = 1 << d.rank;
    const int xu = leaf_fixed(d.u, w, ap), xv = leaf_fixed(d.v, w, ap);
    for (int e = 0; e < nent; e++) {
        int fu = leaf_var_value(d.u, d, e, spos, sid);
        int fv = d.v >= 0 ? leaf_var_value(d.v, d, e, spos, sid) : 0;
        V acc = A::zero(ap);
        for (int a = 0; a < 4; a++) {
            int nu = a & 1, nv = (a >> 1) & 1;
            if (fu >= 0 && nu != fu) continue;
            if (fv >= 0 && nv != fv) continue;
            if (d.v < 0 && nv) continue;
            if ((xu >= 0 && nu != xu) || (xv >= 0 && nv != xv)) continue;
            V prod = A::one(ap);
            if (d.flags & 8) {  // spin glass: x^(-J s_u s_v), x^(-h s), s = 2n - 1
                if (d.flags & 1) prod = A::weight(nu == nv ? -w[d.jidx] : w[d.jidx], ap);
                if (d.flags & 2) prod = A::mul(prod, A::weight(nu ? -w[d.u] : w[d.u], ap), ap);
                if (d.flags & 4) prod = A::mul(prod, A::weight(nv ? -w[d.v] : w[d.v], ap), ap);
            } else {  // independent set: B = [[1, 1], [1, 0]], W = [1, x^w]
                if ((d.flags & 1) && nu && nv) prod = A::zero(ap);
                if ((d.flags & 2) && nu) prod = A::mul(prod, A::weight(w ? w[d.u] : 1.0f, ap), ap);
                if ((d.flags & 4) && nv) prod = A::mul(prod, A::weight(w ? w[d.v] : 1.0f, ap), ap);
            }
            acc = A::add(acc, prod, ap);
        }
        A::store(arena, d.off + e, acc);
    }
}

// Partition function: leaf values in double, stored as float scaled by a
// power of two so the largest entry lies in [1, 2).
__device__ inline void leaf_one_z(const LeafDev& d, int leaf_id, const float* w, const int* spos, u64 sid,
                                  Planes arena, const AlgebraParams& ap, TensorMeta* meta) {
    int nent = 1 << d.rank;
    double val[4] = {0, 0, 0, 0};
    double mx = 0.0;
    const int xu = leaf_fixed(d.u, w, ap), xv = leaf_fixed(d.v, w, ap);
    for (int e = 0; e < nent; e++) {
        int fu = leaf_var_value(d.u, d, e, spos, sid);
        int fv = d.v >= 0 ? leaf_var_value(d.v, d, e, spos, sid) : 0;
        double acc = 0.0;
        for (int a = 0; a < 4; a++) {
            int nu = a & 1, nv = (a >> 1) & 1;
            if (fu >= 0 && nu != fu) continue;
            if (fv >= 0 && nv != fv) continue;
            if (d.v < 0 && nv) continue;
            if ((xu >= 0 && nu != xu) || (xv >= 0 && nv != xv)) continue;
            double prod = 1.0;
            if (d.flags & 8) {  // spin glass: e^(-beta J s_u s_v), e^(-beta h s)
                double ex = 0.0;
                if (d.flags & 1) ex += nu == nv ? -(double)w[d.jidx] : (double)w[d.jidx];
                if (d.flags & 2) ex += nu ? -(double)w[d.u] : (double)w[d.u];
                if (d.flags & 4) ex += nv ? -(double)w[d.v] : (double)w[d.v];
                prod = exp(ap.beta * ex);
            } else {
                if ((d.flags & 1) && nu && nv) prod = 0.0;
                if ((d.flags & 2) && nu) prod *= exp(ap.beta * (double)(w ? w[d.u] : 1.0f));
                if ((d.flags & 4) && nv) prod *= exp(ap.beta * (double)(w ? w[d.v] : 1.0f));
            }
            acc += prod;
        }
        val[e] = acc;
        mx = fmax(mx, acc);
    }
    int ex = mx > 0.0 ? ilogb(mx) : 0;
    float fmx = 0.0f, fmn = INFINITY;
    for (int e = 0; e < nent; e++) {
        float f = (float)ldexp(val[e], -ex);
        z_track(f, fmx, fmn);
        ((float*)arena.p0)[d.off + e] = f;
    }
    meta_set(meta, leaf_id, ex, __float_as_uint(fmx));
    meta_min_nonzero(meta, leaf_id, fmn);
}

template <int D>
__device__ inline void leaf_dispatch(const LeafDev& d, int leaf_id, const float* w, const int* spos, u64 sid,
                                     Planes arena, const AlgebraParams& ap, TensorMeta* meta) {
    if constexpr (is_z<D>())
        leaf_one_z(d, leaf_id, w, spos, sid, arena, ap, meta);
    else
        leaf_one<D>(d, leaf_id, w, spos, sid, arena, ap, meta);
}

// -------------------------------------------------------------- permute --
// out[pi(x)] = in[x], pi a permutation of the bits of x.  A workgroup moves a
// tile of 2^u entries through LDS: read in input order (contiguous runs of
// the input's low bits), write in output order (contiguous runs of the
// output's low bits).  Tables (see build_perm_params): in_lo/in_hi give the
// input offset of tile entry e from its low 6 / high bits, out_lo/out_hi the
// output offset of write slot f, e_lo/e_hi map f to e, and tin/tout place
// the tile index bits.
//
// The tile's low entry bits are the input's lowest bits and its low slot bits
// the output's lowest bits, so once u >= 4 every 16-byte group of entries is
// 16 contiguous input bytes and every group of slots 16 contiguous output
// bytes: both global passes move whole 16-byte vectors.  In LDS, entry e sits
// at perm_lds_pos(e): the 16-byte group index within a 256-byte row is XORed
// with a fold of the row number, so the gathers of the write pass spread over
// the banks instead of stacking up on one.
struct PermLds {
    i64 in_lo[64], in_hi[64], out_lo[64], out_hi[64];
    int e_lo[64], e_hi[64];
    signed char tin[48], tout[48];
};
constexpr int kPermTile = 4096;  // entries; must equal 1 << the tile bits the host plans with

// Entry x (six bits) of the lookup tables: the input offset of read-order
// bits t (in_lo) and t + 6 (in_hi) set in x, likewise the output offset of
// write-order bits (out_lo, out_hi) and the read-order index feeding them
// (e_lo, e_hi).  Tile bits beyond tile_bits contribute nothing.
__host__ __device__ inline void perm_table_entry(const PermParams& pp, int x, long long& il, long long& ih,
                                                 long long& ol, long long& oh, int& el, int& eh) {
    const int nu = pp.tile_bits;
    il = ih = ol = oh = 0;
    el = eh = 0;
    for (int t = 0; t < 6; t++) {
        if (!((x >> t) & 1)) continue;
        if (t < nu) {
            il |= 1ll << pp.u[t];
            ol |= 1ll << pp.vo[t];
            el |= 1 << pp.ef[t];
        }
        if (t + 6 < nu) {
            ih |= 1ll << pp.u[t + 6];
            oh |= 1ll << pp.vo[t + 6];
            eh |= 1 << pp.ef[t + 6];
        }
    }
}

__device__ inline void perm_load_tables(PermLds* s, const PermTables* pp) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        s->in_lo[tid] = pp->in_lo[tid];
        s->in_hi[tid] = pp->in_hi[tid];
        s->out_lo[tid] = pp->out_lo[tid];
        s->out_hi[tid] = pp->out_hi[tid];
        s->e_lo[tid] = pp->e_lo[tid];
        s->e_hi[tid] = pp->e_hi[tid];
    }
    if (tid < 48) {
        s->tin[tid] = pp->tin[tid];
        s->tout[tid] = pp->tout[tid];
    }
}

template <typename T>
__device__ inline int perm_lds_pos(int e) {
    constexpr int LG = sizeof(T) == 4 ? 2 : 1;  // log2 entries per 16 bytes
    constexpr int R = LG + 4;                   // log2 entries per 256-byte row
    const int row = e >> R;
    return e ^ (((row ^ (row >> 4) ^ (row >> 8)) & 15) << LG);
}

// One tile; tables must already be in LDS (and a barrier passed).  Ends with
// a barrier so the tile buffer can be reused.
template <typename T>
__device__ inline void permute_tile(const T* __restrict__ in, T* __restrict__ out, const PermLds* s, T* tile, int u,
                                    int nt, i64 t) {
    constexpr int G = 16 / sizeof(T);  // entries per 16-byte vector
    const int tid = threadIdx.x;
    const int n = 1 << u;
    i64 bin = 0, bout = 0;
    for (int k = 0; k < nt; k++) {
        i64 bit = (t >> k) & 1;
        bin |= bit << s->tin[k];
        bout |= bit << s->tout[k];
    }
    if (u >= 4) {
        for (int e = tid * G; e < n; e += 256 * G) {
            const uint4 v = *(const uint4*)(in + bin + s->in_lo[e & 63] + s->in_hi[e >> 6]);
            *(uint4*)(tile + perm_lds_pos<T>(e)) = v;
        }
        __syncthreads();
        for (int f = tid * G; f < n; f += 256 * G) {
            T v[G];
#pragma unroll
            for (int c = 0; c < G; c++) {
                const int e = s->e_lo[(f + c) & 63] | s->e_hi[(f + c) >> 6];
                v[c] = tile[perm_lds_pos<T>(e)];
            }
            *(uint4*)(out + bout + s->out_lo[f & 63] + s->out_hi[f >> 6]) = *(const uint4*)v;
        }
    } else {
        for (int e = tid; e < n; e += blockDim.x) tile[e] = in[bin + s->in_lo[e & 63] + s->in_hi[e >> 6]];
        __syncthreads();
        for (int f = tid; f < n; f += blockDim.x) {
            const int e = s->e_lo[f & 63] | s->e_hi[f >> 6];
            out[bout + s->out_lo[f & 63] + s->out_hi[f >> 6]] = tile[e];
        }
    }
    __syncthreads();
}

// ----------------------------------------------------------------- GEMM --
// C[b][i][j] = (+)_k A[b][i][k] (*) B[b][k][j], all extents powers of two.
// A is [b][i][k] (k fastest) or, with a_t, [b][k][i]; B is [b][k][j] or, with
// b_t, [b][j][k]; C is [b][i][j].  A workgroup owns a tile of 2^tb batches x
// 2^ti rows x 2^tj columns and walks K in steps of 2^tk: both operand tiles
// are staged in LDS as [batch][k][row] and [batch][k][col], read from global
// memory in memory order (contiguous runs), and each thread accumulates an
// RM x RN register tile with rows y + r*TMt, columns x + c*TNt.  With
// lsplit > 0 the K range is split over workgroups and partial results go to
// `P` ([split][b][i][j]) for the split reduction.
struct GemmArgs {
    Planes A, B, C, P;
    int lb, li, lj, lk, a_t, b_t, tb, ti, tj, tk, lsplit;
    AlgebraParams ap;
    TensorMeta* meta;
    int ma, mb, mc;
};

template <int D>
__device__ inline float input_scale(const GemmArgs& g, int m) {
    if constexpr (is_z<D>()) {
        return ldexpf(1.0f, -max_exponent(meta_maxbits(g.meta, m)));
    } else {
        return 1.0f;
    }
}

__host__ __device__ inline int pad_dim(int t) { return t + (t >= 32 ? 1 : 0); }

// Position of one workgroup tile: split index, first batch / row / column,
// first k of its K range and the length of that range.
struct TilePos {
    int split;
    i64 b0, i0, j0, kbeg;
    int Kc;
};

__device__ inline TilePos tile_pos(const GemmArgs& g, u64 tile) {
    TilePos p;
    p.split = (int)(tile & ((1u << g.lsplit) - 1));
    tile >>= g.lsplit;
    const int ntn = g.lj - g.tj, ntm = g.li - g.ti;
    const i64 jt = (i64)(tile & ((1ull << ntn) - 1));
    tile >>= ntn;
    const i64 it = (i64)(tile & ((1ull << ntm) - 1));
    tile >>= ntm;
    p.b0 = (i64)tile << g.tb;
    p.i0 = it << g.ti;
    p.j0 = jt << g.tj;
    const int lkc = g.lk - g.lsplit;
    p.kbeg = (i64)p.split << lkc;
    p.Kc = 1 << lkc;
    return p;
}

// Stage the A tile as As[batch][k][row] and the B tile as Bs[batch][k][col]
// for k in [k0, k0 + TK), reading global memory in its own order.
template <int D>
__device__ inline unsigned gemm_stage(const GemmArgs& g, const TilePos& p, i64 k0, typename Alg<D>::V* As,
                                      typename Alg<D>::V* Bs, float sA, float sB) {
    // returns, for counting tropical, the OR of the staged counts' high words
    using A = Alg<D>;
    unsigned hi = 0;
    const int TB = 1 << g.tb, TM = 1 << g.ti, TN = 1 << g.tj, TK = 1 << g.tk;
    const int TMp = pad_dim(TM), TNp = pad_dim(TN);
    const int tid = threadIdx.x;
    const int na = TB * TM * TK, nb = TB * TK * TN;
    for (int idx = tid; idx < na; idx += 256) {
        int bb, i, k;
        i64 addr;
        if (!g.a_t) {  // memory order (b, i, k)
            k = idx & (TK - 1);
            i = (idx >> g.tk) & (TM - 1);
            bb = idx >> (g.tk + g.ti);
            addr = ((((p.b0 + bb) << g.li) | (p.i0 + i)) << g.lk) | (k0 + k);
        } else {  // memory order (b, k, i)
            i = idx & (TM - 1);
            k = (idx >> g.ti) & (TK - 1);
            bb = idx >> (g.tk + g.ti);
            addr = ((((p.b0 + bb) << g.lk) | (k0 + k)) << g.li) | (p.i0 + i);
        }
        const typename A::V v = A::load(g.A, addr);
        if constexpr (D == DSR_CTROP) hi |= (unsigned)(v.c >> 32);
        As[(bb * TK + k) * TMp + i] = A::prescale(v, sA);
    }
    for (int idx = tid; idx < nb; idx += 256) {
        int bb, j, k;
        i64 addr;
        if (!g.b_t) {  // memory order (b, k, j)
            j = idx & (TN - 1);
            k = (idx >> g.tj) & (TK - 1);
            bb = idx >> (g.tk + g.tj);
            addr = ((((p.b0 + bb) << g.lk) | (k0 + k)) << g.lj) | (p.j0 + j);
        } else {  // memory order (b, j, k)
            k = idx & (TK - 1);
            j = (idx >> g.tk) & (TN - 1);
            bb = idx >> (g.tk + g.tj);
            addr = ((((p.b0 + bb) << g.lj) | (p.j0 + j)) << g.lk) | (k0 + k);
        }
        const typename A::V v = A::load(g.B, addr);
        if constexpr (D == DSR_CTROP) hi |= (unsigned)(v.c >> 32);
        Bs[(bb * TK + k) * TNp + j] = A::prescale(v, sB);
    }
    return hi;
}

// Partition function.  The first tile reads its operands' records when it
// starts (sharing the round trip of the input scales), derives C's exponent
// and the operands' ranges added once its own operand loads have landed
// (before it stores: a wait there is free, after the stores it would wait for
// them too), and writes both at its end; every tile adds the extremes of
// what it stored (split partials leave them to the split reduction).
struct ZOperands {
    long long ea, eb;
    unsigned xa, xb, na, nb;
};
struct ZDerived {
    long long exp;
    float range;
};
template <int D>
__device__ inline ZOperands z_prologue(const GemmArgs& g, u64 tile) {
    ZOperands z{};
    if constexpr (is_z<D>()) {
        if (tile == 0) {
            z.ea = meta_exp(g.meta, g.ma);
            z.eb = meta_exp(g.meta, g.mb);
            z.xa = meta_maxbits(g.meta, g.ma);
            z.xb = meta_maxbits(g.meta, g.mb);
            z.na = meta_minnz_inv(g.meta, g.ma);
            z.nb = meta_minnz_inv(g.meta, g.mb);
        }
    }
    return z;
}
template <int D>
__device__ inline ZDerived z_derive(u64 tile, const ZOperands& z) {
    ZDerived d{0, 0.0f};
    if constexpr (is_z<D>()) {
        if (tile == 0) {
            d.exp = z.ea + max_exponent(z.xa) + z.eb + max_exponent(z.xb);
            d.range = bits_range(z.xa, z.na) + bits_range(z.xb, z.nb);
        }
    }
    return d;
}
template <int D>
__device__ inline void z_epilogue(const GemmArgs& g, u64 tile, const ZDerived& z, float lmax, float lmin) {
    if constexpr (is_z<D>()) {
        if (tile == 0 && threadIdx.x == 0) {
            meta_set_exp(g.meta, g.mc, z.exp);
            __hip_atomic_store(&g.meta[g.mc].operand_range, z.range, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!g.lsplit) z_meta_block(g.meta, g.mc, lmax, lmin);
    }
}

template <int D, int RM, int RN>
__device__ void gemm_tile(const GemmArgs& g, u64 tile, unsigned char* smem) {
    using A = Alg<D>;
    using V = typename A::V;
    const int TB = 1 << g.tb, TM = 1 << g.ti, TN = 1 << g.tj, TK = 1 << g.tk;
    const int TMp = pad_dim(TM), TNp = pad_dim(TN);
    V* As = (V*)smem;
    V* Bs = As + (size_t)TB * TK * TMp;
    const TilePos p = tile_pos(g, tile);

    const int TNt = TN / RN, TMt = TM / RM;
    const int active = TB * TMt * TNt;
    const int tid = threadIdx.x;
    const int x = tid % TNt, y = (tid / TNt) % TMt, z = tid / (TNt * TMt);

    const float sA = input_scale<D>(g, g.ma), sB = input_scale<D>(g, g.mb);
    const ZOperands zo = z_prologue<D>(g, tile);

    V acc[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; r++)
#pragma unroll
        for (int c = 0; c < RN; c++) acc[r][c] = A::zero(g.ap);

    // counting tropical: per K step (two alternating slots, each cleared one
    // step ahead) whether a staged count reaches 2^32; if none does, count
    // products take one 32 x 32 -> 64 multiply
    __shared__ int s_wide[2];
    if constexpr (D == DSR_CTROP) {
        if (tid == 0) s_wide[0] = s_wide[1] = 0;
        __syncthreads();
    }
    int step = 0;
    for (int kk = 0; kk < p.Kc; kk += TK, step ^= 1) {
        if constexpr (D == DSR_CTROP)
            if (tid == 0) s_wide[step ^ 1] = 0;
        const unsigned hi = gemm_stage<D>(g, p, p.kbeg + kk, As, Bs, sA, sB);
        if constexpr (D == DSR_CTROP)
            if (__any(hi != 0) && (tid & 63) == 0) s_wide[step] = 1;
        __syncthreads();
        if (tid < active) {
            const V* ap_ = As + (size_t)z * TK * TMp + y;
            const V* bp_ = Bs + (size_t)z * TK * TNp + x;
            int k = 0;
            if constexpr (D == DSR_CTROP) {
                if (s_wide[step] == 0) {
                    for (; k < TK; k++) {
                        int an[RM], bn[RN];
                        unsigned ac[RM], bc[RN];
#pragma unroll
                        for (int r = 0; r < RM; r++) {
                            const V v = ap_[k * TMp + r * TMt];
                            an[r] = v.n;
                            ac[r] = (unsigned)v.c;
                        }
#pragma unroll
                        for (int c = 0; c < RN; c++) {
                            const V v = bp_[k * TNp + c * TNt];
                            bn[c] = v.n;
                            bc[c] = (unsigned)v.c;
                        }
#pragma unroll
                        for (int r = 0; r < RM; r++)
#pragma unroll
                            for (int c = 0; c < RN; c++) {
                                const int sz = __builtin_elementwise_add_sat(an[r], bn[c]);
                                const u64 prod = (u64)ac[r] * bc[c];
                                const int n = max(acc[r][c].n, sz);
                                acc[r][c].c = (acc[r][c].n == n ? acc[r][c].c : 0ull) + (sz == n ? prod : 0ull);
                                acc[r][c].n = n;
                            }
                    }
                }
            }
            if constexpr (D == DSR_MODP) {  // four k steps per Montgomery reduction, then two
                for (; k + 3 < TK; k += 4) {
                    V av[4][RM], bv[4][RN];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
#pragma unroll
                        for (int r = 0; r < RM; r++) av[u][r] = ap_[(k + u) * TMp + r * TMt];
#pragma unroll
                        for (int c = 0; c < RN; c++) bv[u][c] = bp_[(k + u) * TNp + c * TNt];
                    }
#pragma unroll
                    for (int r = 0; r < RM; r++)
#pragma unroll
                        for (int c = 0; c < RN; c++) {
                            const V a4[4] = {av[0][r], av[1][r], av[2][r], av[3][r]};
                            const V b4[4] = {bv[0][c], bv[1][c], bv[2][c], bv[3][c]};
                            acc[r][c] = modp_mac4(acc[r][c], a4, b4, g.ap);
                        }
                }
                for (; k + 1 < TK; k += 2) {
                    V av0[RM], bv0[RN], av1[RM], bv1[RN];
#pragma unroll
                    for (int r = 0; r < RM; r++) {
                        av0[r] = ap_[k * TMp + r * TMt];
                        av1[r] = ap_[(k + 1) * TMp + r * TMt];
                    }
#pragma unroll
                    for (int c = 0; c < RN; c++) {
                        bv0[c] = bp_[k * TNp + c * TNt];
                        bv1[c] = bp_[(k + 1) * TNp + c * TNt];
                    }
#pragma unroll
                    for (int r = 0; r < RM; r++)
#pragma unroll
                        for (int c = 0; c < RN; c++) acc[r][c] = modp_mac2(acc[r][c], av0[r], bv0[c], av1[r], bv1[c], g.ap);
                }
            }
            for (; k < TK; k++) {
                V av[RM], bv[RN];
#pragma unroll
                for (int r = 0; r < RM; r++) av[r] = ap_[k * TMp + r * TMt];
#pragma unroll
                for (int c = 0; c < RN; c++) bv[c] = bp_[k * TNp + c * TNt];
#pragma unroll
                for (int r = 0; r < RM; r++)
#pragma unroll
                    for (int c = 0; c < RN; c++) acc[r][c] = A::add(acc[r][c], A::mul(av[r], bv[c], g.ap), g.ap);
            }
        }
        __syncthreads();
    }

    float lmax = 0.0f, lmin = INFINITY;
    const ZDerived zd = z_derive<D>(tile, zo);
    if (tid < active) {
        const i64 nout = (i64)1 << (g.lb + g.li + g.lj);
        const Planes dst = g.lsplit ? g.P : g.C;
        const i64 base = g.lsplit ? (i64)p.split * nout : 0;
#pragma unroll
        for (int r = 0; r < RM; r++)
#pragma unroll
            for (int c = 0; c < RN; c++) {
                i64 o = ((((p.b0 + z) << g.li) | (p.i0 + y + r * TMt)) << g.lj) | (p.j0 + x + c * TNt);
                A::store(dst, base + o, acc[r][c]);
                if constexpr (is_z<D>()) z_track(acc[r][c], lmax, lmin);
            }
    }
    z_epilogue<D>(g, tile, zd, lmax, lmin);
}

// Register-tiled GEMM of the 4-byte VALU algebras (max-plus int32/f32, counts
// mod p) for nodes with large M and N (128 x 128 tile) or one large and one
// small side (256 x 64, 256 x 32 and the mirrored 64 x 256, 32 x 256).  Each
// of the 256 threads owns RMT x RNT outputs: rows in groups of four
// (ty*4 + r, and TM/2 + ty*4 + r when RMT = 8), columns likewise, so every LDS
// operand read is one 16-byte load; two k steps per iteration fold into one
// three-input max.
template <int D>
constexpr bool big_tile_ok() {
    return D == DSR_TROP_I32 || D == DSR_TROP_F32 || D == DSR_MODP;
}

template <typename V>
__device__ inline void lds_load4(const V* p, V* out) {
    const uint4 u = *(const uint4*)p;
    out[0] = __builtin_bit_cast(V, u.x);
    out[1] = __builtin_bit_cast(V, u.y);
    out[2] = __builtin_bit_cast(V, u.z);
    out[3] = __builtin_bit_cast(V, u.w);
}

template <typename V>
__device__ inline void global_store4(V* p, const V* v) {
    uint4 u;
    u.x = __builtin_bit_cast(unsigned int, v[0]);
    u.y = __builtin_bit_cast(unsigned int, v[1]);
    u.z = __builtin_bit_cast(unsigned int, v[2]);
    u.w = __builtin_bit_cast(unsigned int, v[3]);
    *(uint4*)p = u;
}

// Four consecutive entries i..i+3 (i a multiple of 4) of an algebra's planes
// by 16-byte stores.
template <int D>
__device__ inline void store4(const Planes& p, i64 i, const typename Alg<D>::V* v) {
    using V = typename Alg<D>::V;
    if constexpr (D == DSR_CTROP) {
        const int n[4] = {v[0].n, v[1].n, v[2].n, v[3].n};
        global_store4((int*)p.p0 + i, n);
        uint4 c0, c1;
        c0.x = (unsigned)v[0].c, c0.y = (unsigned)(v[0].c >> 32), c0.z = (unsigned)v[1].c, c0.w = (unsigned)(v[1].c >> 32);
        c1.x = (unsigned)v[2].c, c1.y = (unsigned)(v[2].c >> 32), c1.z = (unsigned)v[3].c, c1.w = (unsigned)(v[3].c >> 32);
        *(uint4*)((u64*)p.p1 + i) = c0;
        *(uint4*)((u64*)p.p1 + i + 2) = c1;
    } else if constexpr (sizeof(V) == 4) {
        global_store4((V*)p.p0 + i, v);
    } else {
#pragma unroll
        for (int u = 0; u < 4; u++) Alg<D>::store(p, i + u, v[u]);
    }
}

template <int D>
__device__ inline typename Alg<D>::V big_mac2(typename Alg<D>::V acc, typename Alg<D>::V a0, typename Alg<D>::V b0,
                                              typename Alg<D>::V a1, typename Alg<D>::V b1, const AlgebraParams& ap) {
    using A = Alg<D>;
    if constexpr (D == DSR_MODP)
        return modp_mac2(acc, a0, b0, a1, b1, ap);
    else
        return A::add(acc, A::add(A::mul(a0, b0, ap), A::mul(a1, b1, ap), ap), ap);
}

template <int LTM, int LTN>
struct BigTile {
    static constexpr int TM = 1 << LTM, TN = 1 << LTN;
    // outputs per thread: 8 x 8, or 8 x 4 / 4 x 8 on the 32- and 64-wide sides
    static constexpr int RMT = (LTM == 6 && LTN == 7) ? 4 : (TM >= 64 ? 8 : 4);
    static constexpr int RNT = (LTM == 7 && LTN == 6) ? 4 : (TN >= 64 ? 8 : 4);
    static constexpr int CT = TN / RNT;                                   // column threads
    static constexpr int TMP = TM + 4, TNP = TN + 4;                      // padded LDS rows, 16-byte aligned
    static_assert((TM / RMT) * CT == 256, "256 threads per tile");
};

// the tile shapes of the family, (log2 TM, log2 TN)
__host__ __device__ constexpr bool big_tile_shape(int ti, int tj) {
    return (ti == 7 && (tj == 6 || tj == 7)) || (ti == 6 && tj == 7) || (ti == 8 && (tj == 5 || tj == 6)) ||
           (tj == 8 && (ti == 5 || ti == 6));
}

template <int D, int LTM, int LTN>
__device__ void gemm_tile_big(const GemmArgs& g, u64 tile, unsigned char* smem) {
    static_assert(big_tile_ok<D>(), "4-byte VALU algebras only");
    using A = Alg<D>;
    using V = typename A::V;
    using T = BigTile<LTM, LTN>;
    constexpr int RMT = T::RMT, RNT = T::RNT, TM = T::TM, TN = T::TN, TMP = T::TMP, TNP = T::TNP;
    const int TK = 1 << g.tk;
    V* As = (V*)smem;  // [TK][TMP]
    V* Bs = As + (size_t)TK * TMP;  // [TK][TNP]
    const TilePos p = tile_pos(g, tile);
    const int tid = threadIdx.x, tx = tid % T::CT, ty = tid / T::CT;
    V acc[RMT][RNT];
#pragma unroll
    for (int r = 0; r < RMT; r++)
#pragma unroll
        for (int c = 0; c < RNT; c++) acc[r][c] = A::zero(g.ap);
    const int na = TM * TK, nb = TN * TK;
    for (int kk = 0; kk < p.Kc; kk += TK) {
        const i64 k0 = p.kbeg + kk;
        for (int idx = tid; idx < na; idx += 256) {
            int i, k;
            i64 addr;
            if (!g.a_t) {  // memory order (b, i, k)
                k = idx & (TK - 1);
                i = idx >> g.tk;
                addr = (((p.b0 << g.li) | (p.i0 + i)) << g.lk) | (k0 + k);
            } else {  // (b, k, i)
                i = idx & (TM - 1);
                k = idx >> LTM;
                addr = (((p.b0 << g.lk) | (k0 + k)) << g.li) | (p.i0 + i);
            }
            As[k * TMP + i] = A::load(g.A, addr);
        }
        for (int idx = tid; idx < nb; idx += 256) {
            int j, k;
            i64 addr;
            if (!g.b_t) {  // (b, k, j)
                j = idx & (TN - 1);
                k = idx >> LTN;
                addr = (((p.b0 << g.lk) | (k0 + k)) << g.lj) | (p.j0 + j);
            } else {  // (b, j, k)
                k = idx & (TK - 1);
                j = idx >> g.tk;
                addr = (((p.b0 << g.lj) | (p.j0 + j)) << g.lk) | (k0 + k);
            }
            Bs[k * TNP + j] = A::load(g.B, addr);
        }
        __syncthreads();
        int k0s = 0;
        if constexpr (D == DSR_MODP) {  // four k steps per Montgomery reduction
            for (; k0s + 3 < TK; k0s += 4) {
                V a[4][RMT];
#pragma unroll
                for (int u = 0; u < 4; u++)
#pragma unroll
                    for (int h = 0; h < RMT / 4; h++) lds_load4(As + (k0s + u) * TMP + h * (TM / 2) + ty * 4, a[u] + 4 * h);
#pragma unroll
                for (int h = 0; h < RNT / 4; h++) {  // four columns at a time keeps the operands in registers
                    V b[4][4];
#pragma unroll
                    for (int u = 0; u < 4; u++) lds_load4(Bs + (k0s + u) * TNP + h * (TN / 2) + tx * 4, b[u]);
#pragma unroll
                    for (int r = 0; r < RMT; r++)
#pragma unroll
                        for (int c = 0; c < 4; c++) {
                            const V a4[4] = {a[0][r], a[1][r], a[2][r], a[3][r]};
                            const V b4[4] = {b[0][c], b[1][c], b[2][c], b[3][c]};
                            acc[r][4 * h + c] = modp_mac4(acc[r][4 * h + c], a4, b4, g.ap);
                        }
                }
            }
        }
        // two k per step
        auto load2 = [&](int k, V* a0, V* a1, V* b0, V* b1) {
#pragma unroll
            for (int h = 0; h < RMT / 4; h++) {
                lds_load4(As + k * TMP + h * (TM / 2) + ty * 4, a0 + 4 * h);
                lds_load4(As + (k + 1) * TMP + h * (TM / 2) + ty * 4, a1 + 4 * h);
            }
#pragma unroll
            for (int h = 0; h < RNT / 4; h++) {
                lds_load4(Bs + k * TNP + h * (TN / 2) + tx * 4, b0 + 4 * h);
                lds_load4(Bs + (k + 1) * TNP + h * (TN / 2) + tx * 4, b1 + 4 * h);
            }
        };
        for (int k = k0s; k < TK; k += 2) {  // TK >= 2
            V a0[RMT], b0[RNT], a1[RMT], b1[RNT];
            load2(k, a0, a1, b0, b1);
#pragma unroll
            for (int r = 0; r < RMT; r++)
#pragma unroll
                for (int c = 0; c < RNT; c++) acc[r][c] = big_mac2<D>(acc[r][c], a0[r], b0[c], a1[r], b1[c], g.ap);
        }
        __syncthreads();
    }
    const i64 nout = (i64)1 << (g.lb + g.li + g.lj);
    V* dst = (V*)(g.lsplit ? g.P.p0 : g.C.p0) + (g.lsplit ? (i64)p.split * nout : 0);
#pragma unroll
    for (int r = 0; r < RMT; r++) {
        const int row = (r / 4) * (TM / 2) + ty * 4 + (r & 3);
        const i64 base = ((p.b0 << g.li) | (p.i0 + row)) << g.lj;
#pragma unroll
        for (int h = 0; h < RNT / 4; h++) global_store4(dst + base + p.j0 + h * (TN / 2) + tx * 4, &acc[r][4 * h]);
    }
}

// Launch the family member for (ti, tj); false if (ti, tj) is not one.
template <int D>
__device__ inline bool gemm_tile_big_any(const GemmArgs& g, u64 tile, unsigned char* smem) {
    if (g.ti == 7 && g.tj == 7) gemm_tile_big<D, 7, 7>(g, tile, smem);
    else if (g.ti == 7 && g.tj == 6) gemm_tile_big<D, 7, 6>(g, tile, smem);
    else if (g.ti == 6 && g.tj == 7) gemm_tile_big<D, 6, 7>(g, tile, smem);
    else if (g.ti == 8 && g.tj == 6) gemm_tile_big<D, 8, 6>(g, tile, smem);
    else if (g.ti == 8 && g.tj == 5) gemm_tile_big<D, 8, 5>(g, tile, smem);
    else if (g.ti == 6 && g.tj == 8) gemm_tile_big<D, 6, 8>(g, tile, smem);
    else if (g.ti == 5 && g.tj == 8) gemm_tile_big<D, 5, 8>(g, tile, smem);
    else return false;
    return true;
}

// Counting tropical, register-tiled: (size, count) planes staged separately
// in LDS (counts first for 8-byte alignment), each thread owning 8 x 4 (or
// 4 x 8) outputs in groups of four rows / columns as above.  Tiles 128 x 64,
// 64 x 128, 256 x 32, 32 x 256.
//
// Each K step runs in two passes.  The first takes, for every output, the
// largest size a + b over the step's k (plain max-plus: two adds and one
// three-input max per two k); outputs whose size grows drop the counts they
// had.  The second adds the count products of exactly the terms whose size
// equals the output's size, through a select on the B count and one
// 64-bit multiply-add.  When no staged count of the step (A or B) reaches
// 2^32 (the usual case: counts of optimal configurations are small) the
// product's cross terms vanish and the second pass takes a 32 x 32 -> 64
// multiply-add per term only; when none reaches 2^floor((32 - tk) / 2) the
// step's products and their sum fit 32 bits, and it takes a 24-bit
// multiply-add into a 32-bit partial per output.  The staging loop ORs the
// words and the tile's waves agree on the path through flags in LDS.  Sizes are staged
// clamped at -2^30, so sums of two
// never overflow int32 (-inf = INT32_MIN outside); an output whose size stays
// below -2^29 is -inf (count 0) when stored.  Real sizes satisfy |s| <= 2^28.
__host__ __device__ constexpr bool ct_tile_shape(int ti, int tj) {
    return (ti == 7 && tj == 6) || (ti == 6 && tj == 7) || (ti == 8 && tj == 5) || (ti == 5 && tj == 8);
}

constexpr int kCtNegInf = -(1 << 30);        // staged -inf
constexpr int kCtNegInfBelow = -(1 << 29);   // results below this are -inf

// acc += a * (bhi : blo) mod 2^64, with one 32 x 32 -> 64 multiply-add for
// the low words and two 32-bit multiplies for the cross terms
__device__ inline u64 mad_u64_mod(u64 acc, unsigned alo, unsigned ahi, unsigned blo, unsigned bhi) {
    const u64 t = (u64)alo * blo + acc;
    const unsigned hi = (unsigned)(t >> 32) + alo * bhi + ahi * blo;  // cross terms touch the high word only
    return ((u64)hi << 32) | (unsigned)t;
}

// Operand tiles of a K step read ahead into LDS (the 128 x 64 and 64 x 128
// tiles, 4 <= TK <= 16): the next step's sizes and counts travel from global
// memory into a raw staging area while the current step computes, by
// global-to-LDS loads that hold no registers; the planes are then filled
// from LDS.  raw holds, in global-memory order, the A sizes, A counts,
// B sizes and B counts of one step, 16 bytes per load.
constexpr int kCtRawSlots = 3 * (128 + 64) * 16 / 4;
// s_waitcnt vmcnt(0): this thread's vector memory operations, global-to-LDS
// loads included, have completed
__device__ inline void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// One 16-byte global-to-LDS load: the wave's 64 lanes fill 64 consecutive
// 16-byte slots from LDS address lds_base (wave-uniform).  Written in asm so
// that the compiler does not make every LDS read of the other buffers wait
// for it (it cannot tell them apart).  It has no register result (the data
// goes to LDS; its address registers are read when it issues), and the
// caller waits for it (vm_wait_all) and synchronises before reading the
// slots.
__device__ inline void global_to_lds16(const void* src, unsigned lds_base) {
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(lds_base) : "memory", "m0");
}

template <int LTM, int LTN, bool AHEAD = false>
__device__ void gemm_tile_ct_big(const GemmArgs& g, u64 tile, unsigned char* smem) {
    constexpr int TM = 1 << LTM, TN = 1 << LTN;
    constexpr int RMT = LTM >= LTN ? 8 : 4, RNT = LTM >= LTN ? 4 : 8;
    constexpr int CTH = TN / RNT, TMP = TM + 4, TNP = TN + 4;
    static_assert((TM / RMT) * CTH == 256, "256 threads per tile");
    const int TK = 1 << g.tk;
    // counts as separate low- and high-word planes, so that the usual
    // (32-bit) path reads low words only, four per 16-byte LDS load
    unsigned* Acl = (unsigned*)smem;               // [TK][TMP]
    unsigned* Ach = Acl + (size_t)TK * TMP;        // [TK][TMP]
    unsigned* Bcl = Ach + (size_t)TK * TMP;        // [TK][TNP]
    unsigned* Bch = Bcl + (size_t)TK * TNP;        // [TK][TNP]
    int* An = (int*)(Bch + (size_t)TK * TNP);      // [TK][TMP]
    int* Bn = An + (size_t)TK * TMP;               // [TK][TNP]
    const TilePos p = tile_pos(g, tile);
    const int tid = threadIdx.x, tx = tid % CTH, ty = tid / CTH;
    int accn[RMT][RNT];
    u64 accc[RMT][RNT];
#pragma unroll
    for (int r = 0; r < RMT; r++)
#pragma unroll
        for (int c = 0; c < RNT; c++) {
            accn[r][c] = INT_MIN;
            accc[r][c] = 0ull;
        }
    const int na = TM * TK, nb = TN * TK;
    // per K step (two alternating slots): s_wide is set when a staged count
    // has a nonzero high word, s_big when one reaches small_lim; a slot is
    // cleared one step ahead, after the barrier that ends the last step
    // reading it.  Below small_lim the step's products and their sum over
    // the step fit 32 bits: TK (small_lim - 1)^2 < 2^32.
    __shared__ int s_wide[2], s_big[2];
    const unsigned small_lim = 1u << ((32 - g.tk) / 2);
    // element idx of a staged operand (the staging order is global-memory
    // order) and its address in the operand's planes
    auto a_pos = [&](int idx, i64 k0, int& i, int& k) -> i64 {
        if (!g.a_t) {
            k = idx & (TK - 1);
            i = idx >> g.tk;
            return (((p.b0 << g.li) | (p.i0 + i)) << g.lk) | (k0 + k);
        }
        i = idx & (TM - 1);
        k = idx >> LTM;
        return (((p.b0 << g.lk) | (k0 + k)) << g.li) | (p.i0 + i);
    };
    auto b_pos = [&](int idx, i64 k0, int& j, int& k) -> i64 {
        if (!g.b_t) {
            j = idx & (TN - 1);
            k = idx >> LTN;
            return (((p.b0 << g.lk) | (k0 + k)) << g.lj) | (p.j0 + j);
        }
        k = idx & (TK - 1);
        j = idx >> g.tk;
        return (((p.b0 << g.lj) | (p.j0 + j)) << g.lk) | (k0 + k);
    };
    [[maybe_unused]] const int nraw = 3 * (na + nb) / 4;  // 16-byte loads per step
    [[maybe_unused]] unsigned char* raw = nullptr;
    [[maybe_unused]] unsigned raw_base = 0;  // its LDS address
    if constexpr (AHEAD) {
        __shared__ __align__(16) unsigned char raw_lds[kCtRawSlots * 16];
        raw = raw_lds;
        raw_base = (unsigned)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)raw_lds;
    }
    // one step's operands into raw: load q of this thread fills 16-byte slot
    // q * 256 + tid (a wave's 64 lanes fill 64 consecutive slots, as the
    // global-to-LDS load writes them); 4 sizes or 2 counts per slot, each
    // run contiguous in global memory (TK >= 4, rows of 2^tk or more)
    [[maybe_unused]] auto read_ahead = [&](i64 k0) {
        // the wave's first slot of each load is uniform (an SGPR), and so is
        // the region it falls in: nraw and the region bounds are multiples of 64
        const int lane = tid & 63;
        for (int s0 = __builtin_amdgcn_readfirstlane(tid & ~63); s0 < nraw; s0 += 256) {
            const int slot = s0 + lane;
            int r0, r1;
            const void* src;
            if (s0 < na / 4) {
                src = (const int*)g.A.p0 + a_pos(4 * slot, k0, r0, r1);
            } else if (s0 < 3 * na / 4) {
                src = (const u64*)g.A.p1 + a_pos(2 * (slot - na / 4), k0, r0, r1);
            } else if (s0 < 3 * na / 4 + nb / 4) {
                src = (const int*)g.B.p0 + b_pos(4 * (slot - 3 * na / 4), k0, r0, r1);
            } else {
                src = (const u64*)g.B.p1 + b_pos(2 * (slot - 3 * na / 4 - nb / 4), k0, r0, r1);
            }
            global_to_lds16(src, raw_base + s0 * 16);
        }
    };
    // the barrier that ends a step; with read-ahead it first waits for this
    // thread's loads of the next step (its own wait, not the barrier's: the
    // compiler does not see them)
    auto end_step = [&]() {
        if constexpr (AHEAD) vm_wait_all();
        __syncthreads();
    };
    if (tid == 0) s_wide[0] = s_wide[1] = s_big[0] = s_big[1] = 0;
    if constexpr (AHEAD) {
        read_ahead(p.kbeg);
        vm_wait_all();
    }
    __syncthreads();
    int step = 0;
    for (int kk = 0; kk < p.Kc; kk += TK, step ^= 1) {
        const i64 k0 = p.kbeg + kk;
        if (tid == 0) s_wide[step ^ 1] = s_big[step ^ 1] = 0;
        unsigned hi_or = 0, lo_or = 0;
        if constexpr (AHEAD) {
            // four consecutive entries of raw per thread (one 16-byte read of
            // sizes, two of counts); along the planes' fast index they are one
            // 16-byte write per plane, across it four 4-byte writes
            auto put4 = [&](int* n, unsigned* cl, unsigned* ch, int base, int stride, const unsigned char* rs,
                            const unsigned char* rc, int g4) {
                int sz[4];
                unsigned cw[8];
                lds_load4((const int*)rs + 4 * g4, sz);
                lds_load4((const unsigned*)rc + 8 * g4, cw);
                lds_load4((const unsigned*)rc + 8 * g4 + 4, cw + 4);
                unsigned lo[4], hi[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    sz[u] = max(sz[u], kCtNegInf);
                    lo[u] = cw[2 * u];
                    hi[u] = cw[2 * u + 1];
                    lo_or |= lo[u];
                    hi_or |= hi[u];
                }
                if (stride == 1) {
                    global_store4(n + base, sz);  // (a plain 16-byte store, here into LDS)
                    global_store4(cl + base, lo);
                    global_store4(ch + base, hi);
                } else {
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        n[base + u * stride] = sz[u];
                        cl[base + u * stride] = lo[u];
                        ch[base + u * stride] = hi[u];
                    }
                }
            };
            for (int g4 = tid; g4 < na / 4; g4 += 256) {
                int i, k;
                a_pos(4 * g4, k0, i, k);  // the first of the four: along k (A) or i (A transposed)
                put4(An, Acl, Ach, k * TMP + i, g.a_t ? 1 : TMP, raw, raw + na * 4, g4);
            }
            for (int g4 = tid; g4 < nb / 4; g4 += 256) {
                int j, k;
                b_pos(4 * g4, k0, j, k);  // along j (B) or k (B transposed)
                put4(Bn, Bcl, Bch, k * TNP + j, g.b_t ? TNP : 1, raw + na * 12, raw + na * 12 + nb * 4, g4);
            }
        } else {
            for (int idx = tid; idx < na; idx += 256) {
                int i, k;
                const i64 addr = a_pos(idx, k0, i, k);
                An[k * TMP + i] = max(((const int*)g.A.p0)[addr], kCtNegInf);
                const u64 c = ((const u64*)g.A.p1)[addr];
                hi_or |= (unsigned)(c >> 32);
                lo_or |= (unsigned)c;
                Acl[k * TMP + i] = (unsigned)c;
                Ach[k * TMP + i] = (unsigned)(c >> 32);
            }
            for (int idx = tid; idx < nb; idx += 256) {
                int j, k;
                const i64 addr = b_pos(idx, k0, j, k);
                Bn[k * TNP + j] = max(((const int*)g.B.p0)[addr], kCtNegInf);
                const u64 c = ((const u64*)g.B.p1)[addr];
                hi_or |= (unsigned)(c >> 32);
                lo_or |= (unsigned)c;
                Bcl[k * TNP + j] = (unsigned)c;
                Bch[k * TNP + j] = (unsigned)(c >> 32);
            }
        }
        const bool any_hi = __any(hi_or != 0), any_big = __any(lo_or >= small_lim);
        if ((tid & 63) == 0) {
            if (any_hi) s_wide[step] = 1;
            if (any_big) s_big[step] = 1;
        }
        __syncthreads();
        const bool wide = s_wide[step] != 0, small = !wide && s_big[step] == 0;
        // raw is free (every wave has staged from it): the next step's loads
        // run during this one, and the barrier ending this step waits for them
        if constexpr (AHEAD) {
            if (kk + TK < p.Kc) read_ahead(k0 + TK);
        }
        // pass 1: the step's largest size per output
        int m[RMT][RNT];
#pragma unroll
        for (int r = 0; r < RMT; r++)
#pragma unroll
            for (int c = 0; c < RNT; c++) m[r][c] = accn[r][c];
        auto load_sizes = [&](int k, int* an, int* bn) {
#pragma unroll
            for (int h = 0; h < RMT / 4; h++) lds_load4(An + k * TMP + h * (TM / 2) + ty * 4, an + 4 * h);
#pragma unroll
            for (int h = 0; h < RNT / 4; h++) lds_load4(Bn + k * TNP + h * (TN / 2) + tx * 4, bn + 4 * h);
        };
        int k = 0;
        for (; k + 1 < TK; k += 2) {
            int a0[RMT], a1[RMT], b0[RNT], b1[RNT];
            load_sizes(k, a0, b0);
            load_sizes(k + 1, a1, b1);
#pragma unroll
            for (int r = 0; r < RMT; r++)
#pragma unroll
                for (int c = 0; c < RNT; c++) m[r][c] = max(m[r][c], max(a0[r] + b0[c], a1[r] + b1[c]));
        }
        if (k < TK) {
            int a0[RMT], b0[RNT];
            load_sizes(k, a0, b0);
#pragma unroll
            for (int r = 0; r < RMT; r++)
#pragma unroll
                for (int c = 0; c < RNT; c++) m[r][c] = max(m[r][c], a0[r] + b0[c]);
        }
        // outputs whose size grew drop the counts of the smaller size
#pragma unroll
        for (int r = 0; r < RMT; r++)
#pragma unroll
            for (int c = 0; c < RNT; c++) {
                accc[r][c] = m[r][c] > accn[r][c] ? 0ull : accc[r][c];
                accn[r][c] = m[r][c];
            }
        // pass 2: count products of the terms at the output's size
        if (small) {  // 24-bit multiply-adds into a 32-bit partial per output
            unsigned part[RMT][RNT];
#pragma unroll
            for (int r = 0; r < RMT; r++)
#pragma unroll
                for (int c = 0; c < RNT; c++) part[r][c] = 0u;
            for (k = 0; k < TK; k++) {
                int an[RMT], bn[RNT];
                unsigned ac[RMT], bc[RNT];
                load_sizes(k, an, bn);
#pragma unroll
                for (int h = 0; h < RMT / 4; h++) lds_load4(Acl + k * TMP + h * (TM / 2) + ty * 4, ac + 4 * h);
#pragma unroll
                for (int h = 0; h < RNT / 4; h++) lds_load4(Bcl + k * TNP + h * (TN / 2) + tx * 4, bc + 4 * h);
#pragma unroll
                for (int r = 0; r < RMT; r++)
#pragma unroll
                    for (int c = 0; c < RNT; c++) {
                        const unsigned b = an[r] + bn[c] == accn[r][c] ? bc[c] : 0u;
                        part[r][c] = __umul24(ac[r], b) + part[r][c];
                    }
            }
#pragma unroll
            for (int r = 0; r < RMT; r++)
#pragma unroll
                for (int c = 0; c < RNT; c++) accc[r][c] += part[r][c];
            end_step();
            continue;
        }
        if (!wide) {  // every count of the step below 2^32: low words only
            for (k = 0; k < TK; k++) {
                int an[RMT], bn[RNT];
                unsigned ac[RMT], bc[RNT];
                load_sizes(k, an, bn);
#pragma unroll
                for (int h = 0; h < RMT / 4; h++) lds_load4(Acl + k * TMP + h * (TM / 2) + ty * 4, ac + 4 * h);
#pragma unroll
                for (int h = 0; h < RNT / 4; h++) lds_load4(Bcl + k * TNP + h * (TN / 2) + tx * 4, bc + 4 * h);
#pragma unroll
                for (int r = 0; r < RMT; r++)
#pragma unroll
                    for (int c = 0; c < RNT; c++) {
                        const unsigned b = an[r] + bn[c] == accn[r][c] ? bc[c] : 0u;
                        accc[r][c] += (u64)ac[r] * b;
                    }
            }
            end_step();
            continue;
        }
        for (k = 0; k < TK; k++) {
            int an[RMT], bn[RNT];
            unsigned al[RMT], ah[RMT], bl[RNT], bh[RNT];
            load_sizes(k, an, bn);
#pragma unroll
            for (int h = 0; h < RMT / 4; h++) {
                lds_load4(Acl + k * TMP + h * (TM / 2) + ty * 4, al + 4 * h);
                lds_load4(Ach + k * TMP + h * (TM / 2) + ty * 4, ah + 4 * h);
            }
#pragma unroll
            for (int h = 0; h < RNT / 4; h++) {
                lds_load4(Bcl + k * TNP + h * (TN / 2) + tx * 4, bl + 4 * h);
                lds_load4(Bch + k * TNP + h * (TN / 2) + tx * 4, bh + 4 * h);
            }
#pragma unroll
            for (int r = 0; r < RMT; r++)
#pragma unroll
                for (int c = 0; c < RNT; c++) {
                    const bool eq = an[r] + bn[c] == accn[r][c];
                    accc[r][c] = mad_u64_mod(accc[r][c], al[r], ah[r], eq ? bl[c] : 0u, eq ? bh[c] : 0u);
                }
        }
        end_step();
    }
    const i64 nout = (i64)1 << (g.lb + g.li + g.lj);
    const Planes dst = g.lsplit ? g.P : g.C;
    const i64 sbase = g.lsplit ? (i64)p.split * nout : 0;
    int* dn = (int*)dst.p0 + sbase;
    u64* dc = (u64*)dst.p1 + sbase;
#pragma unroll
    for (int r = 0; r < RMT; r++)
#pragma unroll
        for (int c = 0; c < RNT; c++)
            if (accn[r][c] < kCtNegInfBelow) {
                accn[r][c] = INT_MIN;
                accc[r][c] = 0ull;
            }
#pragma unroll
    for (int r = 0; r < RMT; r++) {
        const int row = (r / 4) * (TM / 2) + ty * 4 + (r & 3);
        const i64 base = ((p.b0 << g.li) | (p.i0 + row)) << g.lj;
#pragma unroll
        for (int h = 0; h < RNT / 4; h++) {
            const i64 o = base + p.j0 + h * (TN / 2) + tx * 4;
            global_store4(dn + o, &accn[r][4 * h]);
            uint4 u0, u1;
            u0.x = (unsigned)accc[r][4 * h + 0];
            u0.y = (unsigned)(accc[r][4 * h + 0] >> 32);
            u0.z = (unsigned)accc[r][4 * h + 1];
            u0.w = (unsigned)(accc[r][4 * h + 1] >> 32);
            u1.x = (unsigned)accc[r][4 * h + 2];
            u1.y = (unsigned)(accc[r][4 * h + 2] >> 32);
            u1.z = (unsigned)accc[r][4 * h + 3];
            u1.w = (unsigned)(accc[r][4 * h + 3] >> 32);
            *(uint4*)(dc + o) = u0;
            *(uint4*)(dc + o + 2) = u1;
        }
    }
}

template <int D>
__device__ inline bool gemm_tile_ct_big_any(const GemmArgs& g, u64 tile, unsigned char* smem) {
    if (g.ti == 7 && g.tj == 6) gemm_tile_ct_big<7, 6>(g, tile, smem);
    else if (g.ti == 6 && g.tj == 7) gemm_tile_ct_big<6, 7>(g, tile, smem);
    else if (g.ti == 8 && g.tj == 5) gemm_tile_ct_big<8, 5>(g, tile, smem);
    else if (g.ti == 5 && g.tj == 8) gemm_tile_ct_big<5, 8>(g, tile, smem);
    else return false;
    return true;
}

// Partition function on the matrix cores: a 64 x 64 tile (tb = 0), four
// waves in a 2 x 2 grid, each accumulating a 32 x 32 block with
// v_mfma_f32_32x32x2f32 (float32 inputs) or v_mfma_f32_32x32x16_bf16
// (bfloat16 inputs, the staged values are already rounded), float32
// accumulation.  Lane l holds A[l%32][k + l/32] (x2f32; for x16_bf16 eight
// consecutive k starting at 8*(l/32)), B likewise by column, and result
// register r is row 8*(r/4) + 4*(l/32) + r%4, column l%32.
typedef float tn_v16f __attribute__((ext_vector_type(16)));
typedef short tn_v8s __attribute__((ext_vector_type(8)));

template <int D>
__device__ void gemm_tile_mfma(const GemmArgs& g, u64 tile, unsigned char* smem) {
    static_assert(is_z<D>(), "matrix cores serve the real algebra only");
    const int TK = 1 << g.tk;
    const int TMp = pad_dim(64), TNp = pad_dim(64);
    float* As = (float*)smem;
    float* Bs = As + (size_t)TK * TMp;
    const TilePos p = tile_pos(g, tile);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int half = lane >> 5, l32 = lane & 31;
    const float sA = input_scale<D>(g, g.ma), sB = input_scale<D>(g, g.mb);
    const ZOperands zo = z_prologue<D>(g, tile);
    tn_v16f acc;
#pragma unroll
    for (int r = 0; r < 16; r++) acc[r] = 0.0f;
    for (int kk = 0; kk < p.Kc; kk += TK) {
        gemm_stage<D>(g, p, p.kbeg + kk, As, Bs, sA, sB);
        __syncthreads();
        const float* ap_ = As + wr * 32 + l32;
        const float* bp_ = Bs + wc * 32 + l32;
        if constexpr (D == DSR_Z_BF16) {
            for (int k = 0; k < TK; k += 16) {
                tn_v8s a, b;
#pragma unroll
                for (int t = 0; t < 8; t++) {
                    a[t] = (short)(__float_as_uint(ap_[(k + 8 * half + t) * TMp]) >> 16);
                    b[t] = (short)(__float_as_uint(bp_[(k + 8 * half + t) * TNp]) >> 16);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
        } else {
            for (int k = 0; k < TK; k += 2) {
                float a = ap_[(k + half) * TMp], b = bp_[(k + half) * TNp];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const i64 nout = (i64)1 << (g.lb + g.li + g.lj);
    float* dst = (float*)(g.lsplit ? g.P.p0 : g.C.p0) + (g.lsplit ? (i64)p.split * nout : 0);
    float lmax = 0.0f, lmin = INFINITY;
    const ZDerived zd = z_derive<D>(tile, zo);
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int row = 8 * (r >> 2) + 4 * half + (r & 3);
        const i64 o = (((p.b0 << g.li) | (p.i0 + wr * 32 + row)) << g.lj) | (p.j0 + wc * 32 + l32);
        dst[o] = acc[r];
        z_track(acc[r], lmax, lmin);
    }
    z_epilogue<D>(g, tile, zd, lmax, lmin);
}

// Partition function on the matrix cores, large tiles: a 128 x 128 output
// tile, four waves in a 2 x 2 grid, each wave 64 x 64 as 2 x 2 blocks of
// 32 x 32 (so every A fragment serves two B fragments and back).  Operand
// tiles sit in LDS with k contiguous per row (A as [i][k], B as [j][k], rows
// padded by 16 bytes), written once per K step from 16-byte global loads that
// were issued before the previous step's MFMAs (two LDS buffers, one barrier
// per step).  The sum over k may take any order as long as A and B agree: in
// float32 (TK = 16, v_mfma_f32_32x32x2f32) lane half h feeds k = h*8 + s to
// step s, so a lane reads its eight k of a step block with two 16-byte LDS
// loads; in bfloat16 (TK = 32, v_mfma_f32_32x32x16_bf16, values rounded and
// packed to 16 bits when staged) lane half h feeds k = h*16 + 8*s .. +7 to
// step s, one 16-byte load per step.
template <int D>
struct Mfma128 {
    static constexpr bool kBf16 = D == DSR_Z_BF16;
    static constexpr int TK = kBf16 ? 32 : 16;            // k per LDS step
    static constexpr int EB = kBf16 ? 2 : 4;              // bytes per staged value
    static constexpr int ROW = TK * EB + 16;               // padded row bytes
    static constexpr int OPB = 128 * ROW;                  // one operand tile
    static constexpr int BUF = 2 * OPB;                    // A and B
    static constexpr int LDS = 2 * BUF;                    // two buffers
    static constexpr int NV = 128 * TK / 4 / 256;          // float4 loads per thread per operand
};

__device__ inline unsigned int bf16_bits(float x) { return __float_as_uint(x) >> 16; }

template <int D>
__device__ void gemm_tile_mfma128(const GemmArgs& g, u64 tile, unsigned char* smem) {
    static_assert(is_z<D>(), "matrix cores serve the real algebra only");
    using M = Mfma128<D>;
    using A = Alg<D>;
    constexpr int TK = M::TK, NV = M::NV;
    const TilePos p = tile_pos(g, tile);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1, half = lane >> 5, l32 = lane & 31;
    const float sA = input_scale<D>(g, g.ma), sB = input_scale<D>(g, g.mb);
    const ZOperands zo = z_prologue<D>(g, tile);
    // global -> register prefetch of one K step: NV float4 per operand per
    // thread; element e = tid + 256 v of the 128 x TK tile, 4 values each
    float4 ra[NV], rb[NV];
    auto fetch = [&](i64 k0) {
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int e = tid + 256 * v;
            i64 addr;
            if (!g.a_t) {  // (b, i, k): 4 consecutive k of row i
                const int i = e / (TK / 4), k = 4 * (e % (TK / 4));
                addr = (((p.b0 << g.li) | (p.i0 + i)) << g.lk) | (k0 + k);
            } else {  // (b, k, i): 4 consecutive rows at one k
                const int k = e / 32, i = 4 * (e % 32);
                addr = (((p.b0 << g.lk) | (k0 + k)) << g.li) | (p.i0 + i);
            }
            ra[v] = *(const float4*)((const float*)g.A.p0 + addr);
            if (!g.b_t) {  // (b, k, j): 4 consecutive columns at one k
                const int k = e / 32, j = 4 * (e % 32);
                addr = (((p.b0 << g.lk) | (k0 + k)) << g.lj) | (p.j0 + j);
            } else {  // (b, j, k): 4 consecutive k of column j
                const int j = e / (TK / 4), k = 4 * (e % (TK / 4));
                addr = (((p.b0 << g.lj) | (p.j0 + j)) << g.lk) | (k0 + k);
            }
            rb[v] = *(const float4*)((const float*)g.B.p0 + addr);
        }
    };
    // registers -> LDS buffer `buf` ([row][k], k contiguous), scaled (and
    // rounded to bfloat16 and packed)
    auto put = [&](int buf) {
        unsigned char* As = smem + buf * M::BUF;
        unsigned char* Bs = As + M::OPB;
        auto put4 = [&](unsigned char* base, bool along_k, int e, float4 x, float s) {
            const float v[4] = {A::prescale(x.x, s), A::prescale(x.y, s), A::prescale(x.z, s), A::prescale(x.w, s)};
            if (along_k) {
                const int r = e / (TK / 4), k = 4 * (e % (TK / 4));
                unsigned char* q = base + r * M::ROW + k * M::EB;
                if constexpr (M::kBf16) {
                    uint2 u;
                    u.x = bf16_bits(v[0]) | (bf16_bits(v[1]) << 16);
                    u.y = bf16_bits(v[2]) | (bf16_bits(v[3]) << 16);
                    *(uint2*)q = u;
                } else {
                    *(float4*)q = make_float4(v[0], v[1], v[2], v[3]);
                }
            } else {
                const int k = e / 32, r = 4 * (e % 32);
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    unsigned char* q = base + (r + t) * M::ROW + k * M::EB;
                    if constexpr (M::kBf16)
                        *(unsigned short*)q = (unsigned short)bf16_bits(v[t]);
                    else
                        *(float*)q = v[t];
                }
            }
        };
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int e = tid + 256 * v;
            put4(As, !g.a_t, e, ra[v], sA);
            put4(Bs, g.b_t != 0, e, rb[v], sB);
        }
    };
    tn_v16f acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[bi][bj][r] = 0.0f;
    const int nsteps = p.Kc / TK;
    fetch(p.kbeg);
    put(0);
    __syncthreads();
    for (int st = 0; st < nsteps; st++) {
        const int buf = st & 1;
        if (st + 1 < nsteps) fetch(p.kbeg + (i64)(st + 1) * TK);  // in flight during the MFMAs below
        const unsigned char* As = smem + buf * M::BUF;
        const unsigned char* Bs = As + M::OPB;
        if constexpr (M::kBf16) {
#pragma unroll
            for (int s = 0; s < 2; s++) {
                tn_v8s a[2], b[2];
#pragma unroll
                for (int x = 0; x < 2; x++) {
                    a[x] = *(const tn_v8s*)(As + (wr * 64 + x * 32 + l32) * M::ROW + (half * 16 + 8 * s) * 2);
                    b[x] = *(const tn_v8s*)(Bs + (wc * 64 + x * 32 + l32) * M::ROW + (half * 16 + 8 * s) * 2);
                }
#pragma unroll
                for (int bi = 0; bi < 2; bi++)
#pragma unroll
                    for (int bj = 0; bj < 2; bj++)
                        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
            }
        } else {
            float4 a[2][2], b[2][2];  // [block][two float4 = eight k]
#pragma unroll
            for (int x = 0; x < 2; x++)
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    a[x][q] = *(const float4*)(As + (wr * 64 + x * 32 + l32) * M::ROW + (half * 8 + 4 * q) * 4);
                    b[x][q] = *(const float4*)(Bs + (wc * 64 + x * 32 + l32) * M::ROW + (half * 8 + 4 * q) * 4);
                }
#pragma unroll
            for (int s = 0; s < 8; s++) {
#pragma unroll
                for (int bi = 0; bi < 2; bi++)
#pragma unroll
                    for (int bj = 0; bj < 2; bj++) {
                        const float4& av = a[bi][s >> 2];
                        const float4& bv = b[bj][s >> 2];
                        const float ax = (s & 3) == 0 ? av.x : (s & 3) == 1 ? av.y : (s & 3) == 2 ? av.z : av.w;
                        const float bx = (s & 3) == 0 ? bv.x : (s & 3) == 1 ? bv.y : (s & 3) == 2 ? bv.z : bv.w;
                        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(ax, bx, acc[bi][bj], 0, 0, 0);
                    }
            }
        }
        if (st + 1 < nsteps) put(buf ^ 1);  // the other buffer: last read before the previous barrier
        __syncthreads();
    }
    const i64 nout = (i64)1 << (g.lb + g.li + g.lj);
    float* dst = (float*)(g.lsplit ? g.P.p0 : g.C.p0) + (g.lsplit ? (i64)p.split * nout : 0);
    float lmax = 0.0f, lmin = INFINITY;
    const ZDerived zd = z_derive<D>(tile, zo);
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < 2; bj++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int row = wr * 64 + bi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                const int col = wc * 64 + bj * 32 + l32;
                const i64 o = (((p.b0 << g.li) | (p.i0 + row)) << g.lj) | (p.j0 + col);
                dst[o] = acc[bi][bj][r];
                z_track(acc[bi][bj][r], lmax, lmin);
            }
    z_epilogue<D>(g, tile, zd, lmax, lmin);
}

// ----------------------------------------------------- thin / dot GEMM --
// Thin node (GEMM_THIN): a tile is 2^ti (>= 1024) consecutive rows of one
// batch; B (K x N <= 32 entries) is staged in LDS.  Each thread takes four
// rows per step (tid + 256 q) and issues all their loads (K <= 4 entries of
// at most 4 bytes, or K <= 2 of 8) before computing, so a wave keeps
// 4 x 64 row loads in flight; neighbouring lanes touch neighbouring rows, so
// loads and stores are contiguous across a wave in either operand order.
template <int D>
__device__ void gemm_tile_thin(const GemmArgs& g, u64 tile, unsigned char* smem) {
    using A = Alg<D>;
    using V = typename A::V;
    constexpr int RQ = 4, KMAX = 4;
    V* Bs = (V*)smem;  // [k][j]
    const TilePos p = tile_pos(g, tile);
    const int K = 1 << g.lk, N = 1 << g.lj;
    const float sA = input_scale<D>(g, g.ma), sB = input_scale<D>(g, g.mb);
    const ZOperands zo = z_prologue<D>(g, tile);
    for (int q = threadIdx.x; q < K * N; q += 256) {
        const int k = q >> g.lj, j = q & (N - 1);
        const i64 addr = g.b_t ? (((p.b0 << g.lj) | j) << g.lk) | k : (((p.b0 << g.lk) | k) << g.lj) | j;
        Bs[q] = A::prescale(A::load(g.B, addr), sB);
    }
    __syncthreads();
    float lmax = 0.0f, lmin = INFINITY;
    const ZDerived zd = z_derive<D>(tile, zo);
    const int rows = 1 << g.ti;
    if constexpr (D != DSR_TOPK && D != DSR_TPOLY) {
        if (g.lj >= 2) {
            // N >= 4: N / 4 lanes per row, four consecutive outputs each, so
            // that a wave's stores cover one contiguous run of rows (16-byte
            // stores per lane; the lanes of a row read the same A entries)
            const int llpr = g.lj - 2, rpp = 256 >> llpr;  // rows per pass
            const int rl = threadIdx.x >> llpr, j0 = (threadIdx.x & ((1 << llpr) - 1)) * 4;
            for (int r0 = 0; r0 < rows; r0 += rpp * RQ) {
                V av[RQ][KMAX];
#pragma unroll
                for (int q = 0; q < RQ; q++) {
                    const i64 i = p.i0 + r0 + q * rpp + rl;
#pragma unroll
                    for (int k = 0; k < KMAX; k++)
                        if (k < K) {
                            const i64 addr =
                                g.a_t ? (((p.b0 << g.lk) | k) << g.li) | i : (((p.b0 << g.li) | i) << g.lk) | k;
                            av[q][k] = A::prescale(A::load(g.A, addr), sA);
                        }
                }
#pragma unroll
                for (int q = 0; q < RQ; q++) {
                    V acc[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        acc[u] = A::zero(g.ap);
#pragma unroll
                        for (int k = 0; k < KMAX; k++)
                            if (k < K) acc[u] = A::add(acc[u], A::mul(av[q][k], Bs[(k << g.lj) | (j0 + u)], g.ap), g.ap);
                        if constexpr (is_z<D>()) z_track(acc[u], lmax, lmin);
                    }
                    store4<D>(g.C, (((p.b0 << g.li) | (p.i0 + r0 + q * rpp + rl)) << g.lj) | j0, acc);
                }
            }
            z_epilogue<D>(g, tile, zd, lmax, lmin);
            return;
        }
    }
    for (int r0 = 0; r0 < rows; r0 += 256 * RQ) {
        V av[RQ][KMAX];
#pragma unroll
        for (int q = 0; q < RQ; q++) {
            const i64 i = p.i0 + r0 + q * 256 + threadIdx.x;
#pragma unroll
            for (int k = 0; k < KMAX; k++)
                if (k < K) {
                    const i64 addr = g.a_t ? (((p.b0 << g.lk) | k) << g.li) | i : (((p.b0 << g.li) | i) << g.lk) | k;
                    av[q][k] = A::load(g.A, addr);
                }
        }
#pragma unroll
        for (int q = 0; q < RQ; q++) {
            const i64 obase = ((p.b0 << g.li) | (p.i0 + r0 + q * 256 + threadIdx.x)) << g.lj;
            for (int j = 0; j < N; j++) {
                V acc = A::zero(g.ap);
#pragma unroll
                for (int k = 0; k < KMAX; k++)
                    if (k < K) acc = A::add(acc, A::mul(A::prescale(av[q][k], sA), Bs[(k << g.lj) | j], g.ap), g.ap);
                A::store(g.C, obase | j, acc);
                if constexpr (is_z<D>()) z_track(acc, lmax, lmin);
            }
        }
    }
    z_epilogue<D>(g, tile, zd, lmax, lmin);
}

// One output per batch (GEMM_DOT): a tile is one (batch, K-split) pair; the
// workgroup's threads stride over the K range (A and B are both contiguous in
// k when M = N = 1), then reduce through LDS.
template <int D>
__device__ void gemm_tile_dot(const GemmArgs& g, u64 tile, unsigned char* smem) {
    using A = Alg<D>;
    using V = typename A::V;
    V* red = (V*)smem;
    const TilePos p = tile_pos(g, tile);
    const float sA = input_scale<D>(g, g.ma), sB = input_scale<D>(g, g.mb);
    const ZOperands zo = z_prologue<D>(g, tile);
    V acc = A::zero(g.ap);
    const i64 base = p.b0 << g.lk;
    for (i64 k = p.kbeg + threadIdx.x; k < p.kbeg + p.Kc; k += 256)
        acc = A::add(acc, A::mul(A::prescale(A::load(g.A, base | k), sA), A::prescale(A::load(g.B, base | k), sB), g.ap),
                     g.ap);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = A::add(red[threadIdx.x], red[threadIdx.x + w], g.ap);
        __syncthreads();
    }
    float lmax = 0.0f, lmin = INFINITY;
    const ZDerived zd = z_derive<D>(tile, zo);
    if (threadIdx.x == 0) {
        const i64 nout = (i64)1 << g.lb;
        if (g.lsplit)
            A::store(g.P, (i64)p.split * nout + p.b0, red[0]);
        else
            A::store(g.C, p.b0, red[0]);
        if constexpr (is_z<D>()) z_track(red[0], lmax, lmin);
    }
    z_epilogue<D>(g, tile, zd, lmax, lmin);
    __syncthreads();
}

// --------------------------------------------------------- split reduce --
// C[o] = (+)_s part[s][o] for one output o, by the whole workgroup.
// (+) of the S partials of output o, folded in split order; the loads are
// issued eight at a time so their latencies overlap.
template <int D>
__device__ inline typename Alg<D>::V split_sum(Planes part, i64 nout, i64 o, int S, const AlgebraParams& ap) {
    using A = Alg<D>;
    using V = typename A::V;
    V acc = A::zero(ap);
    int s = 0;
    for (; s + 8 <= S; s += 8) {
        V v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = A::load(part, (i64)(s + u) * nout + o);
#pragma unroll
        for (int u = 0; u < 8; u++) acc = A::add(acc, v[u], ap);
    }
    for (; s < S; s++) acc = A::add(acc, A::load(part, (i64)s * nout + o), ap);
    return acc;
}

template <int D>
__device__ void split_reduce_one(Planes part, Planes C, i64 nout, int lsplit, const AlgebraParams& ap,
                                 TensorMeta* meta, int mc, i64 o, typename Alg<D>::V* red) {
    using A = Alg<D>;
    using V = typename A::V;
    const int S = 1 << lsplit;
    V acc = A::zero(ap);
    for (int s = threadIdx.x; s < S; s += blockDim.x) acc = A::add(acc, A::load(part, (i64)s * nout + o), ap);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = A::add(red[threadIdx.x], red[threadIdx.x + w], ap);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        A::store(C, o, red[0]);
        if constexpr (is_z<D>()) {
            if (red[0] > 0.0f) meta_max(meta, mc, __float_as_uint(red[0]));
            meta_min_nonzero(meta, mc, red[0]);
        }
    }
    __syncthreads();
}

// The partition function's dynamic range: over the n tensors of a
// contraction, the largest log2(max / smallest nonzero) of the stored
// float32 entries, or of the two operands of a product added together (the
// span a product of their entries needs; past the float32 exponent range the
// smallest products underflow), by one workgroup (every thread calls); written as a float
// at byte kZRangeOffset of the pass's accumulator slot, or raised to it when
// first is 0 (later slices).
__device__ inline void z_range_block(const TensorMeta* m, int n, void* acc, int first, float* red) {
    float best = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        best = fmaxf(best, fmaxf(meta_range(m, i),
                                 __hip_atomic_load(&m[i].operand_range, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    red[threadIdx.x] = best;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float* slot = (float*)((char*)acc + kZRangeOffset);
        *slot = first ? red[0] : fmaxf(*slot, red[0]);
    }
    __syncthreads();
}

// ---------------------------------------------------------- accumulate ---
// Slice accumulation (Sec. 4.2): the per-slice roots are combined with the
// algebra's addition.  The partition function keeps {mantissa, exponent}.
struct ZAcc {
    double m;
    i64 e;
};

__device__ inline void zacc_add(ZAcc& a, double v, i64 e) {
    if (v == 0.0) return;
    int e2;
    double fr = frexp(v, &e2);  // v = fr * 2^e2, fr in [0.5, 1)
    double m = 2.0 * fr;
    i64 E = e + e2 - 1;
    if (a.m == 0.0) {
        a.m = m;
        a.e = E;
        return;
    }
    if (E > a.e) {
        double t = a.m;
        i64 te = a.e;
        a.m = m;
        a.e = E;
        m = t;
        E = te;
    }
    i64 d = E - a.e;  // <= 0
    if (d > -1100) a.m += ldexp(m, (int)d);
    if (a.m >= 2.0) {
        a.m *= 0.5;
        a.e += 1;
    }
}

template <int D>
__device__ void accumulate_one(Planes root, int mroot, TensorMeta* meta, void* acc, int first,
                               const AlgebraParams& ap) {
    using A = Alg<D>;
    if constexpr (is_z<D>()) {
        ZAcc* z = (ZAcc*)acc;
        if (first) {
            z->m = 0.0;
            z->e = 0;
        }
        zacc_add(*z, (double)((const float*)root.p0)[0], meta_exp(meta, mroot));
    } else if constexpr (D == DSR_CTROP) {
        CTv v = A::load(root, 0);
        int* n = (int*)acc;
        u64* c = (u64*)((char*)acc + 8);
        CTv a = first ? A::zero(ap) : CTv{*n, *c};
        a = A::add(a, v, ap);
        *n = a.n;
        *c = a.c;
    } else if constexpr (D == DSR_TPOLY) {  // slot: int32 top exponent, then four counts from byte 8
        TP4 v = A::load(root, 0);
        int* m = (int*)acc;
        u64* c = (u64*)((char*)acc + 8);
        TP4 a = A::zero(ap);
        if (!first) a = TP4{*m, {c[0], c[1], c[2], c[3]}};
        a = A::add(a, v, ap);
        *m = a.m;
        for (int d = 0; d < 4; d++) c[d] = a.c[d];
    } else {
        using V = typename A::V;
        V v = A::load(root, 0);
        V* a = (V*)acc;
        *a = first ? v : A::add(*a, v, ap);
    }
}

template <int D>
__device__ void set_one(void* acc, const AlgebraParams& ap) {
    using A = Alg<D>;
    if constexpr (is_z<D>()) {
        ZAcc* z = (ZAcc*)acc;
        z->m = 1.0;
        z->e = 0;
    } else if constexpr (D == DSR_CTROP) {
        *(int*)acc = 0;
        *(u64*)((char*)acc + 8) = 1ull;
    } else if constexpr (D == DSR_TPOLY) {
        *(int*)acc = 0;
        u64* c = (u64*)((char*)acc + 8);
        c[0] = 1ull;
        c[1] = c[2] = c[3] = 0ull;
    } else {
        *(typename A::V*)acc = A::one(ap);
    }
}

}  // namespace tn
