// gfx950 kernels of the tensor-network executor.
//
// Every index has dimension 2, so a rank-r tensor has 2^r entries and the
// value of index t is bit t of the entry's linear offset.  One binary
// contraction (Sec. 4.1 maps it onto a matrix product) becomes
//   permute  -- move the operand's bits into [batch | rows | cols] order,
//   GEMM     -- C[b][i][j] = (+)_k A[b][i][k] (*) B[b][k][j]  over a semiring
// with the algebras of the Sec. 5 property table.
//
// Kernels: leaf initialisation (edge tensor [[1,1],[1,0]] and vertex tensor
// [1, x^w], Sec. 3.2), LDS-staged bit permute, LDS-tiled batched semiring GEMM
// on the vector ALUs (max-plus has no matrix-core form), split-K reduce, and
// slice accumulation (Sec. 4.2 slicing).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>

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

template <>
struct Alg<DSR_U64> {  // counting in Z / 2^64
    using V = u64;
    __device__ static V zero(const AlgebraParams&) { return 0ull; }
    __device__ static V one(const AlgebraParams&) { return 1ull; }
    __device__ static V add(V a, V b, const AlgebraParams&) { return a + b; }
    __device__ static V mul(V a, V b, const AlgebraParams&) { return a * b; }
    __device__ static V weight(float, const AlgebraParams&) { return 1ull; }
    __device__ static V load(const Planes& p, i64 i) { return ((const u64*)p.p0)[i]; }
    __device__ static void store(const Planes& p, i64 i, V v) { ((u64*)p.p0)[i] = v; }
    __device__ static V prescale(V v, float) { return v; }
};

template <>
struct Alg<DSR_MODP> {  // counting modulo p < 2^31, Montgomery form with R = 2^32
    using V = unsigned int;
    __device__ static V zero(const AlgebraParams&) { return 0u; }
    __device__ static V one(const AlgebraParams& ap) { return ap.r1; }
    __device__ static V add(V a, V b, const AlgebraParams& ap) {
        V s = a + b;
        return s >= ap.p ? s - ap.p : s;
    }
    __device__ static V mul(V a, V b, const AlgebraParams& ap) {
        u64 t = (u64)a * b;                       // < p^2 < 2^62
        unsigned int m = (unsigned int)t * ap.pinv;  // t + m p == 0 mod 2^32
        u64 u = (t + (u64)m * ap.p) >> 32;        // < 2p
        return (V)(u >= ap.p ? u - ap.p : u);
    }
    __device__ static V weight(float, const AlgebraParams& ap) { return ap.r1; }
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

int plane_bytes(int dsr, int plane) {
    switch (dsr) {
    case DSR_CTROP: return plane == 0 ? 4 : 8;
    case DSR_U64: return plane == 0 ? 8 : 0;
    default: return plane == 0 ? 4 : 0;
    }
}

static int lds_elem_bytes(int dsr) {
    switch (dsr) {
    case DSR_CTROP: return 16;
    case DSR_U64: return 8;
    default: return 4;
    }
}

// exponent m with 2^m <= max < 2^(m+1) of a non-negative float given by its bits
__device__ inline int max_exponent(unsigned int bits) {
    if (bits == 0u) return 0;
    int e = (int)((bits >> 23) & 0xffu);
    return e == 0 ? -126 : e - 127;
}

// ------------------------------------------------------------ meta init --
__global__ void meta_init_kernel(TensorMeta* meta, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        meta[i].exp = 0;
        meta[i].maxbits = 0u;
        meta[i].pad = 0u;
    }
}

hipError_t launch_meta_init(TensorMeta* meta, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    meta_init_kernel<<<(n + 255) / 256, 256, 0, s>>>(meta, n);
    return hipGetLastError();
}

// --------------------------------------------------------------- leaves --
// One thread per leaf.  A leaf is the product of its factors: the edge
// tensor B(n_u, n_v) = [[1,1],[1,0]] and the vertex tensors W(n) = [1, x^w]
// folded into it (Sec. 3.2), summed over its indices that occur nowhere
// else, with sliced indices fixed to this slice's values.
__device__ inline int leaf_var_value(int var, const LeafDev& d, int e, const int* spos, u64 sid) {
    if (var == d.var0) return e & 1;
    if (var == d.var1) return (e >> 1) & 1;
    int sp = spos[var];
    if (sp >= 0) return (int)((sid >> sp) & 1ull);
    return -1;  // summed at the leaf
}

template <int D>
__global__ void leaf_kernel(const LeafDev* leaves, int nleaf, const float* w, const int* spos, u64 sid,
                            Planes arena, AlgebraParams ap, TensorMeta* meta) {
    using A = Alg<D>;
    using V = typename A::V;
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nleaf) return;
    LeafDev d = leaves[l];
    int nent = 1 << d.rank;
    for (int e = 0; e < nent; e++) {
        int fu = leaf_var_value(d.u, d, e, spos, sid);
        int fv = d.v >= 0 ? leaf_var_value(d.v, d, e, spos, sid) : 0;
        V acc = A::zero(ap);
        for (int a = 0; a < 4; a++) {
            int nu = a & 1, nv = (a >> 1) & 1;
            if (fu >= 0 && nu != fu) continue;
            if (fv >= 0 && nv != fv) continue;
            if (d.v < 0 && nv) continue;
            V prod = A::one(ap);
            if ((d.flags & 1) && nu && nv) prod = A::zero(ap);
            if ((d.flags & 2) && nu) prod = A::mul(prod, A::weight(w ? w[d.u] : 1.0f, ap), ap);
            if ((d.flags & 4) && nv) prod = A::mul(prod, A::weight(w ? w[d.v] : 1.0f, ap), ap);
            acc = A::add(acc, prod, ap);
        }
        A::store(arena, d.off + e, acc);
    }
}

// Partition function: leaf values in double, stored as float scaled by a
// power of two so the largest entry lies in [1, 2).
template <int D>
__global__ void leaf_kernel_z(const LeafDev* leaves, int nleaf, const float* w, const int* spos, u64 sid,
                              Planes arena, AlgebraParams ap, TensorMeta* meta) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nleaf) return;
    LeafDev d = leaves[l];
    int nent = 1 << d.rank;
    double val[4] = {0, 0, 0, 0};
    double mx = 0.0;
    for (int e = 0; e < nent; e++) {
        int fu = leaf_var_value(d.u, d, e, spos, sid);
        int fv = d.v >= 0 ? leaf_var_value(d.v, d, e, spos, sid) : 0;
        double acc = 0.0;
        for (int a = 0; a < 4; a++) {
            int nu = a & 1, nv = (a >> 1) & 1;
            if (fu >= 0 && nu != fu) continue;
            if (fv >= 0 && nv != fv) continue;
            if (d.v < 0 && nv) continue;
            double prod = 1.0;
            if ((d.flags & 1) && nu && nv) prod = 0.0;
            if ((d.flags & 2) && nu) prod *= exp(ap.beta * (double)(w ? w[d.u] : 1.0f));
            if ((d.flags & 4) && nv) prod *= exp(ap.beta * (double)(w ? w[d.v] : 1.0f));
            acc += prod;
        }
        val[e] = acc;
        mx = fmax(mx, acc);
    }
    int ex = mx > 0.0 ? ilogb(mx) : 0;
    float fmx = 0.0f;
    for (int e = 0; e < nent; e++) {
        float f = (float)ldexp(val[e], -ex);
        fmx = fmaxf(fmx, f);
        ((float*)arena.p0)[d.off + e] = f;
    }
    meta[l].exp = ex;
    meta[l].maxbits = __float_as_uint(fmx);
}

hipError_t launch_leaves(int dsr, const LeafDev* leaves, int nleaf, const float* w, const int* spos, u64 sid,
                         Planes arena, const AlgebraParams& ap, TensorMeta* meta, hipStream_t s) {
    if (nleaf <= 0) return hipSuccess;
    dim3 grid((nleaf + 127) / 128), block(128);
    switch (dsr) {
    case DSR_TROP_I32: leaf_kernel<DSR_TROP_I32><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); break;
    case DSR_TROP_F32: leaf_kernel<DSR_TROP_F32><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); break;
    case DSR_CTROP: leaf_kernel<DSR_CTROP><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); break;
    case DSR_U64: leaf_kernel<DSR_U64><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); break;
    case DSR_MODP: leaf_kernel<DSR_MODP><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); break;
    case DSR_Z_F32:
    case DSR_Z_BF16: leaf_kernel_z<DSR_Z_F32><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- permute --
// out[pi(x)] = in[x], pi a permutation of the bits of x.  A workgroup moves a
// tile of 2^u entries: the tile bits U are the input's lowest bits and the
// input bits feeding the output's lowest bits, interleaved, so both the read
// and the write side are contiguous runs.  The tile goes through LDS:
//   read  e = 0..2^u-1 in input order  (in_lo/in_hi: offset of e's bits)
//   write f = 0..2^u-1 in output order (out_lo/out_hi; e_lo/e_hi map f->e)
// The remaining rank-u bits enumerate tiles (tin/tout: their positions).
void build_perm_params(int rank, const int* src, PermParams& pp) {
    std::memset(&pp, 0, sizeof pp);
    int r = rank;
    int u = r < 11 ? r : 11;
    int inv[64];
    for (int q = 0; q < r; q++) inv[src[q]] = q;
    bool inU[64] = {false};
    int nU = 0;
    for (int k = 0; k < r && nU < u; k++) {
        if (!inU[k]) {
            inU[k] = true;
            nU++;
        }
        if (nU < u && !inU[src[k]]) {
            inU[src[k]] = true;
            nU++;
        }
    }
    int U[64], nu = 0, Vo[64], nvo = 0;
    for (int b = 0; b < r; b++)
        if (inU[b]) U[nu++] = b;  // e bit t <-> input bit U[t]
    for (int q = 0; q < r; q++)
        if (inU[src[q]]) Vo[nvo++] = q;  // f bit t <-> output bit Vo[t]
    int posU[64];
    for (int t = 0; t < nu; t++) posU[U[t]] = t;
    for (int x = 0; x < 64; x++) {
        long long il = 0, ih = 0, ol = 0, oh = 0;
        int el = 0, eh = 0;
        for (int t = 0; t < 6; t++) {
            if (!((x >> t) & 1)) continue;
            if (t < nu) il |= 1ll << U[t];
            if (t + 6 < nu) ih |= 1ll << U[t + 6];
            if (t < nvo) {
                ol |= 1ll << Vo[t];
                el |= 1 << posU[src[Vo[t]]];
            }
            if (t + 6 < nvo) {
                oh |= 1ll << Vo[t + 6];
                eh |= 1 << posU[src[Vo[t + 6]]];
            }
        }
        pp.in_lo[x] = il;
        pp.in_hi[x] = ih;
        pp.out_lo[x] = ol;
        pp.out_hi[x] = oh;
        pp.e_lo[x] = el;
        pp.e_hi[x] = eh;
    }
    int nt = 0;
    for (int b = 0; b < r; b++)
        if (!inU[b]) {
            pp.tin[nt] = (signed char)b;
            pp.tout[nt] = (signed char)inv[b];
            nt++;
        }
    pp.rank = r;
    pp.tile_bits = u;
    pp.ntile_bits = nt;
}

template <typename T>
__global__ __launch_bounds__(256) void permute_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                      const PermParams* __restrict__ pp, i64 ntiles) {
    __shared__ i64 s_in_lo[64], s_in_hi[64], s_out_lo[64], s_out_hi[64];
    __shared__ int s_e_lo[64], s_e_hi[64];
    __shared__ signed char s_tin[48], s_tout[48];
    __shared__ T tile[2048 + 64];
    const int tid = threadIdx.x;
    if (tid < 64) {
        s_in_lo[tid] = pp->in_lo[tid];
        s_in_hi[tid] = pp->in_hi[tid];
        s_out_lo[tid] = pp->out_lo[tid];
        s_out_hi[tid] = pp->out_hi[tid];
        s_e_lo[tid] = pp->e_lo[tid];
        s_e_hi[tid] = pp->e_hi[tid];
    }
    if (tid < 48) {
        s_tin[tid] = pp->tin[tid];
        s_tout[tid] = pp->tout[tid];
    }
    const int u = pp->tile_bits, nt = pp->ntile_bits;
    const int n = 1 << u;
    __syncthreads();
    for (i64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
        i64 bin = 0, bout = 0;
        for (int k = 0; k < nt; k++) {
            i64 bit = (t >> k) & 1;
            bin |= bit << s_tin[k];
            bout |= bit << s_tout[k];
        }
        for (int e = tid; e < n; e += 256) tile[e + (e >> 5)] = in[bin + s_in_lo[e & 63] + s_in_hi[e >> 6]];
        __syncthreads();
        for (int f = tid; f < n; f += 256) {
            int e = s_e_lo[f & 63] | s_e_hi[f >> 6];
            out[bout + s_out_lo[f & 63] + s_out_hi[f >> 6]] = tile[e + (e >> 5)];
        }
        __syncthreads();
    }
}

hipError_t launch_permute(int elem_bytes, const void* in, void* out, const PermParams* pp_dev, int rank,
                          int tile_bits, hipStream_t s) {
    i64 ntiles = (i64)1 << (rank - tile_bits);
    int grid = (int)(ntiles < 4096 ? ntiles : 4096);
    if (elem_bytes == 4)
        permute_kernel<unsigned int><<<grid, 256, 0, s>>>((const unsigned int*)in, (unsigned int*)out, pp_dev, ntiles);
    else if (elem_bytes == 8)
        permute_kernel<u64><<<grid, 256, 0, s>>>((const u64*)in, (u64*)out, pp_dev, ntiles);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
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
// `part` ([split][b][i][j]) for launch_split_reduce.
struct GemmArgs {
    Planes A, B, C, P;
    int lb, li, lj, lk, a_t, b_t, tb, ti, tj, tk, lsplit;
    AlgebraParams ap;
    TensorMeta* meta;
    int ma, mb, mc;
};

template <int D>
__device__ inline float input_scale(const GemmArgs& g, int m) {
    if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) {
        return ldexpf(1.0f, -max_exponent(g.meta[m].maxbits));
    } else {
        return 1.0f;
    }
}

template <int D, int RM, int RN>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    using A = Alg<D>;
    using V = typename A::V;
    extern __shared__ __align__(16) unsigned char smem[];
    const int TB = 1 << g.tb, TM = 1 << g.ti, TN = 1 << g.tj, TK = 1 << g.tk;
    const int TMp = TM + (TM >= 32 ? 1 : 0), TNp = TN + (TN >= 32 ? 1 : 0);
    V* As = (V*)smem;
    V* Bs = As + (size_t)TB * TK * TMp;

    u64 tile = blockIdx.x;
    const int split = (int)(tile & ((1u << g.lsplit) - 1));
    tile >>= g.lsplit;
    const int ntn = g.lj - g.tj, ntm = g.li - g.ti;
    const i64 jt = (i64)(tile & ((1ull << ntn) - 1));
    tile >>= ntn;
    const i64 it = (i64)(tile & ((1ull << ntm) - 1));
    tile >>= ntm;
    const i64 b0 = (i64)tile << g.tb, i0 = it << g.ti, j0 = jt << g.tj;
    const int lkc = g.lk - g.lsplit;
    const i64 kbeg = (i64)split << lkc;
    const int Kc = 1 << lkc;

    const int TNt = TN / RN, TMt = TM / RM;
    const int active = TB * TMt * TNt;
    const int tid = threadIdx.x;
    const int x = tid % TNt, y = (tid / TNt) % TMt, z = tid / (TNt * TMt);

    const float sA = input_scale<D>(g, g.ma), sB = input_scale<D>(g, g.mb);

    V acc[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; r++)
#pragma unroll
        for (int c = 0; c < RN; c++) acc[r][c] = A::zero(g.ap);

    const int na = TB * TM * TK, nb = TB * TK * TN;
    for (int kk = 0; kk < Kc; kk += TK) {
        const i64 k0 = kbeg + kk;
        for (int idx = tid; idx < na; idx += 256) {
            int bb, i, k;
            i64 addr;
            if (!g.a_t) {  // memory order (b, i, k)
                k = idx & (TK - 1);
                i = (idx >> g.tk) & (TM - 1);
                bb = idx >> (g.tk + g.ti);
                addr = ((((b0 + bb) << g.li) | (i0 + i)) << g.lk) | (k0 + k);
            } else {  // memory order (b, k, i)
                i = idx & (TM - 1);
                k = (idx >> g.ti) & (TK - 1);
                bb = idx >> (g.tk + g.ti);
                addr = ((((b0 + bb) << g.lk) | (k0 + k)) << g.li) | (i0 + i);
            }
            As[(bb * TK + k) * TMp + i] = A::prescale(A::load(g.A, addr), sA);
        }
        for (int idx = tid; idx < nb; idx += 256) {
            int bb, j, k;
            i64 addr;
            if (!g.b_t) {  // memory order (b, k, j)
                j = idx & (TN - 1);
                k = (idx >> g.tj) & (TK - 1);
                bb = idx >> (g.tk + g.tj);
                addr = ((((b0 + bb) << g.lk) | (k0 + k)) << g.lj) | (j0 + j);
            } else {  // memory order (b, j, k)
                k = idx & (TK - 1);
                j = (idx >> g.tk) & (TN - 1);
                bb = idx >> (g.tk + g.tj);
                addr = ((((b0 + bb) << g.lj) | (j0 + j)) << g.lk) | (k0 + k);
            }
            Bs[(bb * TK + k) * TNp + j] = A::prescale(A::load(g.B, addr), sB);
        }
        __syncthreads();
        if (tid < active) {
            const V* ap_ = As + (size_t)z * TK * TMp + y;
            const V* bp_ = Bs + (size_t)z * TK * TNp + x;
            for (int k = 0; k < TK; k++) {
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

    if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) {
        if (blockIdx.x == 0 && tid == 0) {
            g.meta[g.mc].exp = g.meta[g.ma].exp + max_exponent(g.meta[g.ma].maxbits) + g.meta[g.mb].exp +
                               max_exponent(g.meta[g.mb].maxbits);
        }
    }
    float lmax = 0.0f;
    if (tid < active) {
        const i64 nout = (i64)1 << (g.lb + g.li + g.lj);
        const Planes dst = g.lsplit ? g.P : g.C;
        const i64 base = g.lsplit ? (i64)split * nout : 0;
#pragma unroll
        for (int r = 0; r < RM; r++)
#pragma unroll
            for (int c = 0; c < RN; c++) {
                i64 o = ((((b0 + z) << g.li) | (i0 + y + r * TMt)) << g.lj) | (j0 + x + c * TNt);
                A::store(dst, base + o, acc[r][c]);
                if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) lmax = fmaxf(lmax, acc[r][c]);
            }
    }
    if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) {
        if (!g.lsplit) {
            for (int off = 32; off > 0; off >>= 1) lmax = fmaxf(lmax, __shfl_xor(lmax, off));
            if ((tid & 63) == 0 && lmax > 0.0f) atomicMax(&g.meta[g.mc].maxbits, __float_as_uint(lmax));
        }
    }
}

GemmShape choose_gemm_shape(int dsr, int lb, int li, int lj, int lk, int a_t, int b_t) {
    GemmShape g{};
    g.lb = lb;
    g.li = li;
    g.lj = lj;
    g.lk = lk;
    g.a_t = a_t;
    g.b_t = b_t;
    const int eb = lds_elem_bytes(dsr);
    const int lds_cap = 40 * 1024;
    if (li >= 6 && lj >= 6 && lk >= 4) {
        // contraction-heavy node: 64x64 tile, 4x4 per thread
        g.rm = g.rn = 4;
        g.ti = g.tj = 6;
        g.tb = 0;
        g.tk = lk < 5 ? lk : 5;
        while (g.tk > 0 && (1 << g.tk) * 128 * eb > lds_cap) g.tk--;
    } else {
        g.rm = li >= 1 ? 2 : 1;
        g.rn = lj >= 1 ? 2 : 1;
        const int lr = (g.rm == 2) + (g.rn == 2);
        const int tot = 8 + lr;  // log2 outputs per workgroup
        g.ti = li < 5 ? li : 5;
        g.tj = lj < 5 ? lj : 5;
        while (g.ti + g.tj > tot) {
            if (g.ti >= g.tj && g.ti > (g.rm == 2)) g.ti--;
            else if (g.tj > (g.rn == 2)) g.tj--;
            else g.ti--;
        }
        int rest = tot - g.ti - g.tj;
        g.tb = lb < rest ? lb : rest;
        rest -= g.tb;
        while (rest > 0 && g.ti < li) {
            g.ti++;
            rest--;
        }
        while (rest > 0 && g.tj < lj) {
            g.tj++;
            rest--;
        }
        g.tk = lk < 5 ? lk : 5;
        while (g.tk > 0 && (1ll << (g.tb + g.tk)) * ((1 << g.ti) + (1 << g.tj)) * eb > lds_cap) g.tk--;
        // a tile needs at least RM rows / RN columns per thread
        if ((1 << g.ti) < g.rm) g.rm = 1;
        if ((1 << g.tj) < g.rn) g.rn = 1;
    }
    // split K when there are too few output tiles to fill the chip
    int ltiles = (lb - g.tb) + (li - g.ti) + (lj - g.tj);
    g.lsplit = 0;
    if (ltiles < 9 && lk - g.tk >= 2) {
        int want = 10 - ltiles;
        int room = lk - g.tk - 1;
        g.lsplit = want < room ? want : room;
        if (g.lsplit < 0) g.lsplit = 0;
    }
    return g;
}

bool gemm_shape_valid(int dsr, const GemmShape& g) {
    if (g.tb < 0 || g.ti < 0 || g.tj < 0 || g.tk < 0 || g.lsplit < 0) return false;
    if (g.tb > g.lb || g.ti > g.li || g.tj > g.lj || g.tk + g.lsplit > g.lk) return false;
    if (g.rm != 1 && g.rm != 2 && g.rm != 4) return false;
    if (g.rn != 1 && g.rn != 2 && g.rn != 4) return false;
    if ((1 << g.ti) < g.rm || (1 << g.tj) < g.rn) return false;
    long long threads = (1ll << (g.tb + g.ti + g.tj)) / (g.rm * g.rn);
    if (threads > 256 || threads < 1) return false;
    long long lds = (1ll << (g.tb + g.tk)) * ((1 << g.ti) + 1 + (1 << g.tj) + 1) * lds_elem_bytes(dsr);
    return lds <= 48 * 1024;
}

template <int D, int RM, int RN>
static hipError_t gemm_go(const GemmArgs& a, size_t lds, u64 blocks, hipStream_t s) {
    gemm_kernel<D, RM, RN><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
    return hipGetLastError();
}

template <int D>
static hipError_t gemm_dispatch(const GemmArgs& a, int rm, int rn, size_t lds, u64 blocks, hipStream_t s) {
    if (rm == 1 && rn == 1) return gemm_go<D, 1, 1>(a, lds, blocks, s);
    if (rm == 1 && rn == 2) return gemm_go<D, 1, 2>(a, lds, blocks, s);
    if (rm == 2 && rn == 1) return gemm_go<D, 2, 1>(a, lds, blocks, s);
    if (rm == 2 && rn == 2) return gemm_go<D, 2, 2>(a, lds, blocks, s);
    if (rm == 4 && rn == 4) return gemm_go<D, 4, 4>(a, lds, blocks, s);
    if (rm == 1 && rn == 4) return gemm_go<D, 1, 4>(a, lds, blocks, s);
    if (rm == 4 && rn == 1) return gemm_go<D, 4, 1>(a, lds, blocks, s);
    if (rm == 2 && rn == 4) return gemm_go<D, 2, 4>(a, lds, blocks, s);
    if (rm == 4 && rn == 2) return gemm_go<D, 4, 2>(a, lds, blocks, s);
    return hipErrorInvalidValue;
}

hipError_t launch_gemm(int dsr, Planes Ap, Planes Bp, Planes Cp, Planes part, const GemmShape& g,
                       const AlgebraParams& ap, TensorMeta* meta, int ma, int mb, int mc, hipStream_t s) {
    if (!gemm_shape_valid(dsr, g)) return hipErrorInvalidValue;
    GemmArgs a;
    a.A = Ap;
    a.B = Bp;
    a.C = Cp;
    a.P = part;
    a.lb = g.lb;
    a.li = g.li;
    a.lj = g.lj;
    a.lk = g.lk;
    a.a_t = g.a_t;
    a.b_t = g.b_t;
    a.tb = g.tb;
    a.ti = g.ti;
    a.tj = g.tj;
    a.tk = g.tk;
    a.lsplit = g.lsplit;
    a.ap = ap;
    a.meta = meta;
    a.ma = ma;
    a.mb = mb;
    a.mc = mc;
    const int eb = lds_elem_bytes(dsr);
    const int TMp = (1 << g.ti) + ((1 << g.ti) >= 32 ? 1 : 0), TNp = (1 << g.tj) + ((1 << g.tj) >= 32 ? 1 : 0);
    size_t lds = (size_t)(1 << (g.tb + g.tk)) * (TMp + TNp) * eb;
    u64 blocks = 1ull << ((g.lb - g.tb) + (g.li - g.ti) + (g.lj - g.tj) + g.lsplit);
    switch (dsr) {
    case DSR_TROP_I32: return gemm_dispatch<DSR_TROP_I32>(a, g.rm, g.rn, lds, blocks, s);
    case DSR_TROP_F32: return gemm_dispatch<DSR_TROP_F32>(a, g.rm, g.rn, lds, blocks, s);
    case DSR_CTROP: return gemm_dispatch<DSR_CTROP>(a, g.rm, g.rn, lds, blocks, s);
    case DSR_U64: return gemm_dispatch<DSR_U64>(a, g.rm, g.rn, lds, blocks, s);
    case DSR_MODP: return gemm_dispatch<DSR_MODP>(a, g.rm, g.rn, lds, blocks, s);
    case DSR_Z_F32: return gemm_dispatch<DSR_Z_F32>(a, g.rm, g.rn, lds, blocks, s);
    case DSR_Z_BF16: return gemm_dispatch<DSR_Z_BF16>(a, g.rm, g.rn, lds, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

// --------------------------------------------------------- split reduce --
// C[o] = (+)_s part[s][o].  Large outputs: one thread per entry; small
// outputs: one workgroup per entry with an LDS tree over the splits.
template <int D>
__global__ __launch_bounds__(256) void split_reduce_kernel(Planes part, Planes C, i64 nout, int lsplit,
                                                           AlgebraParams ap, TensorMeta* meta, int mc,
                                                           int per_block) {
    using A = Alg<D>;
    using V = typename A::V;
    const int S = 1 << lsplit;
    float lmax = 0.0f;
    if (!per_block) {
        i64 o = (i64)blockIdx.x * 256 + threadIdx.x;
        if (o < nout) {
            V acc = A::zero(ap);
            for (int s = 0; s < S; s++) acc = A::add(acc, A::load(part, (i64)s * nout + o), ap);
            A::store(C, o, acc);
            if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) lmax = acc;
        }
    } else {
        __shared__ V red[256];
        i64 o = blockIdx.x;
        V acc = A::zero(ap);
        for (int s = threadIdx.x; s < S; s += 256) acc = A::add(acc, A::load(part, (i64)s * nout + o), ap);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = A::add(red[threadIdx.x], red[threadIdx.x + w], ap);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            A::store(C, o, red[0]);
            if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) lmax = red[0];
        }
    }
    if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) {
        for (int off = 32; off > 0; off >>= 1) lmax = fmaxf(lmax, __shfl_xor(lmax, off));
        if ((threadIdx.x & 63) == 0 && lmax > 0.0f) atomicMax(&meta[mc].maxbits, __float_as_uint(lmax));
    }
}

hipError_t launch_split_reduce(int dsr, Planes part, Planes C, i64 nout, int lsplit, const AlgebraParams& ap,
                               TensorMeta* meta, int mc, hipStream_t s) {
    int per_block = nout < 1024 ? 1 : 0;
    unsigned blocks = per_block ? (unsigned)nout : (unsigned)((nout + 255) / 256);
#define TN_SR(D)                                                                                       \
    case D:                                                                                            \
        split_reduce_kernel<D><<<blocks, 256, 0, s>>>(part, C, nout, lsplit, ap, meta, mc, per_block); \
        break;
    switch (dsr) {
        TN_SR(DSR_TROP_I32)
        TN_SR(DSR_TROP_F32)
        TN_SR(DSR_CTROP)
        TN_SR(DSR_U64)
        TN_SR(DSR_MODP)
        TN_SR(DSR_Z_F32)
        TN_SR(DSR_Z_BF16)
    default: return hipErrorInvalidValue;
    }
#undef TN_SR
    return hipGetLastError();
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
__global__ void accumulate_kernel(Planes root, int mroot, TensorMeta* meta, void* acc, int first, AlgebraParams ap) {
    using A = Alg<D>;
    if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) {
        ZAcc* z = (ZAcc*)acc;
        if (first) {
            z->m = 0.0;
            z->e = 0;
        }
        zacc_add(*z, (double)((const float*)root.p0)[0], meta[mroot].exp);
    } else if constexpr (D == DSR_CTROP) {
        CTv v = A::load(root, 0);
        int* n = (int*)acc;
        u64* c = (u64*)((char*)acc + 8);
        CTv a = first ? A::zero(ap) : CTv{*n, *c};
        a = A::add(a, v, ap);
        *n = a.n;
        *c = a.c;
    } else {
        using V = typename A::V;
        V v = A::load(root, 0);
        V* a = (V*)acc;
        *a = first ? v : A::add(*a, v, ap);
    }
}

hipError_t launch_accumulate(int dsr, Planes root, int mroot, TensorMeta* meta, void* acc, int first,
                             const AlgebraParams& ap, hipStream_t s) {
#define TN_AC(D)                                                              \
    case D:                                                                   \
        accumulate_kernel<D><<<1, 1, 0, s>>>(root, mroot, meta, acc, first, ap); \
        break;
    switch (dsr) {
        TN_AC(DSR_TROP_I32)
        TN_AC(DSR_TROP_F32)
        TN_AC(DSR_CTROP)
        TN_AC(DSR_U64)
        TN_AC(DSR_MODP)
        TN_AC(DSR_Z_F32)
        TN_AC(DSR_Z_BF16)
    default: return hipErrorInvalidValue;
    }
#undef TN_AC
    return hipGetLastError();
}

template <int D>
__global__ void set_one_kernel(void* acc, AlgebraParams ap) {
    using A = Alg<D>;
    if constexpr (D == DSR_Z_F32 || D == DSR_Z_BF16) {
        ZAcc* z = (ZAcc*)acc;
        z->m = 1.0;
        z->e = 0;
    } else if constexpr (D == DSR_CTROP) {
        *(int*)acc = 0;
        *(u64*)((char*)acc + 8) = 1ull;
    } else {
        *(typename A::V*)acc = A::one(ap);
    }
}

hipError_t launch_set_one(int dsr, void* acc, const AlgebraParams& ap, hipStream_t s) {
#define TN_SO(D)                                     \
    case D:                                          \
        set_one_kernel<D><<<1, 1, 0, s>>>(acc, ap); \
        break;
    switch (dsr) {
        TN_SO(DSR_TROP_I32)
        TN_SO(DSR_TROP_F32)
        TN_SO(DSR_CTROP)
        TN_SO(DSR_U64)
        TN_SO(DSR_MODP)
        TN_SO(DSR_Z_F32)
        TN_SO(DSR_Z_BF16)
    default: return hipErrorInvalidValue;
    }
#undef TN_SO
    return hipGetLastError();
}

int accumulator_bytes(int) { return 16; }

}  // namespace tn
