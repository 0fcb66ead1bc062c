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

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "kernels_dev.h"

namespace tn {

int plane_bytes(int dsr, int plane) {
    switch (dsr) {
    case DSR_CTROP: return plane == 0 ? 4 : 8;
    case DSR_TOPK: return plane == 0 ? 32 : 0;
    case DSR_TPOLY: return plane == 0 ? 4 : 32;
    default: return plane == 0 ? 4 : 0;
    }
}

static int lds_elem_bytes(int dsr) {
    switch (dsr) {
    case DSR_CTROP: return 16;
    case DSR_TOPK: return 32;
    case DSR_TPOLY: return (int)sizeof(TP4);
    default: return 4;
    }
}

// ----------------------------------------------------- Z dynamic range --
__global__ __launch_bounds__(256) void z_range_kernel(const TensorMeta* meta, int n, void* acc, int first) {
    __shared__ float red[256];
    z_range_block(meta, n, acc, first, red);
}

hipError_t launch_z_range(const TensorMeta* meta, int n, void* acc, int first, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    z_range_kernel<<<1, 256, 0, s>>>(meta, n, acc, first);
    return hipGetLastError();
}

// ------------------------------------------------------------ meta init --
__global__ void meta_init_kernel(TensorMeta* meta, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) meta_set(meta, i, 0, 0u);
}

hipError_t launch_meta_init(TensorMeta* meta, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    meta_init_kernel<<<(n + 255) / 256, 256, 0, s>>>(meta, n);
    return hipGetLastError();
}

// --------------------------------------------------------------- leaves --
template <int D>
__global__ void leaf_kernel(const LeafDev* leaves, int nleaf, const float* w, const int* spos, u64 sid,
                            Planes arena, AlgebraParams ap, TensorMeta* meta) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nleaf) return;
    leaf_dispatch<D>(leaves[l], l, w, spos, sid, arena, ap, meta);
}

hipError_t launch_leaves(int dsr, const LeafDev* leaves, int nleaf, const float* w, const int* spos, u64 sid,
                         Planes arena, const AlgebraParams& ap, TensorMeta* meta, hipStream_t s) {
    if (nleaf <= 0) return hipSuccess;
    dim3 grid((nleaf + 127) / 128), block(128);
#define TN_LF(D)                                                                                 \
    case D:                                                                                      \
        leaf_kernel<D><<<grid, block, 0, s>>>(leaves, nleaf, w, spos, sid, arena, ap, meta); \
        break;
    switch (dsr) {
        TN_LF(DSR_TROP_I32)
        TN_LF(DSR_TROP_F32)
        TN_LF(DSR_CTROP)
        TN_LF(DSR_MODP)
        TN_LF(DSR_Z_F32)
        TN_LF(DSR_Z_BF16)
        TN_LF(DSR_TOPK)
        TN_LF(DSR_TPOLY)
    default: return hipErrorInvalidValue;
    }
#undef TN_LF
    return hipGetLastError();
}

// -------------------------------------------------------------- permute --

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
    const int r = rank;
    const int u = perm_tile_bits(r);
    int inv[64];
    for (int q = 0; q < r; q++) inv[src[q]] = q;
    // tile bits: input bits 0, 1, ... interleaved with the input bits that
    // feed output bits 0, 1, ..., until there are u of them
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
    int posU[64], nu = 0, nvo = 0;
    for (int b = 0; b < r; b++)
        if (inU[b]) {
            posU[b] = nu;
            pp.u[nu++] = (signed char)b;  // read-order bit t <-> input bit b
        }
    for (int q = 0; q < r; q++)
        if (inU[src[q]]) {
            pp.vo[nvo] = (signed char)q;              // write-order bit t <-> output bit q
            pp.ef[nvo++] = (signed char)posU[src[q]];  // fed by read-order bit posU[src[q]]
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

static_assert(kPermTile == 1 << kPermTileBits, "permute tile size");

// one workgroup of 64 threads per permute, one table entry per thread
__global__ __launch_bounds__(64) void expand_perms_kernel(const PermParams* __restrict__ perms,
                                                          PermTables* __restrict__ tables, int n) {
    const int i = blockIdx.x, x = threadIdx.x;
    if (i >= n || x >= 64) return;
    const PermParams& p = perms[i];
    PermTables& t = tables[i];
    long long il, ih, ol, oh;
    int el, eh;
    perm_table_entry(p, x, il, ih, ol, oh, el, eh);
    t.in_lo[x] = il;
    t.in_hi[x] = ih;
    t.out_lo[x] = ol;
    t.out_hi[x] = oh;
    t.e_lo[x] = el;
    t.e_hi[x] = eh;
    if (x < 48) {
        t.tin[x] = p.tin[x];
        t.tout[x] = p.tout[x];
    }
    if (x == 0) {
        t.rank = p.rank;
        t.tile_bits = p.tile_bits;
        t.ntile_bits = p.ntile_bits;
        t.pad = 0;
    }
}

hipError_t launch_expand_perms(const PermParams* perms, PermTables* tables, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    expand_perms_kernel<<<n, 64, 0, s>>>(perms, tables, n);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void permute_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                      const PermTables* __restrict__ pp, i64 ntiles) {
    __shared__ PermLds tabs;
    __shared__ __align__(16) T tile[kPermTile];
    perm_load_tables(&tabs, pp);
    const int u = pp->tile_bits, nt = pp->ntile_bits;
    __syncthreads();
    for (i64 t = blockIdx.x; t < ntiles; t += gridDim.x) permute_tile<T>(in, out, &tabs, tile, u, nt, t);
}

hipError_t launch_permute(int elem_bytes, const void* in, void* out, const PermTables* pp_dev, int rank,
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
template <int D, int RM, int RN>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile<D, RM, RN>(g, blockIdx.x, smem);
}

template <int D, int LTM, int LTN>
__global__ __launch_bounds__(256) void gemm_big_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile_big<D, LTM, LTN>(g, blockIdx.x, smem);
}

template <int D>
__global__ __launch_bounds__(256) void gemm_thin_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile_thin<D>(g, blockIdx.x, smem);
}

template <int D>
__global__ __launch_bounds__(256) void gemm_dot_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile_dot<D>(g, blockIdx.x, smem);
}

template <int D>
static hipError_t gemm_mode_go(const GemmArgs& a, int mode, size_t lds, u64 blocks, hipStream_t s) {
    if (mode == GEMM_THIN)
        gemm_thin_kernel<D><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
    else
        gemm_dot_kernel<D><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
    return hipGetLastError();
}

template <int LTM, int LTN, bool AHEAD>
__global__ __launch_bounds__(256, 2) void gemm_ct_big_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile_ct_big<LTM, LTN, AHEAD>(g, blockIdx.x, smem);
}

static hipError_t gemm_ct_big_go(const GemmArgs& a, size_t lds, u64 blocks, hipStream_t s) {
    const dim3 grid((unsigned)blocks), block(256);
    const bool ahead = ct_ahead_shape(a.ti, a.tj, a.tk);
    if (a.ti == 7 && a.tj == 6 && ahead) gemm_ct_big_kernel<7, 6, true><<<grid, block, lds, s>>>(a);
    else if (a.ti == 6 && a.tj == 7 && ahead) gemm_ct_big_kernel<6, 7, true><<<grid, block, lds, s>>>(a);
    else if (a.ti == 7 && a.tj == 6) gemm_ct_big_kernel<7, 6, false><<<grid, block, lds, s>>>(a);
    else if (a.ti == 6 && a.tj == 7) gemm_ct_big_kernel<6, 7, false><<<grid, block, lds, s>>>(a);
    else if (a.ti == 8 && a.tj == 5) gemm_ct_big_kernel<8, 5, false><<<grid, block, lds, s>>>(a);
    else if (a.ti == 5 && a.tj == 8) gemm_ct_big_kernel<5, 8, false><<<grid, block, lds, s>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int D>
static hipError_t gemm_big_go(const GemmArgs& a, size_t lds, u64 blocks, hipStream_t s) {
    const dim3 grid((unsigned)blocks), block(256);
    if (a.ti == 7 && a.tj == 7) gemm_big_kernel<D, 7, 7><<<grid, block, lds, s>>>(a);
    else if (a.ti == 7 && a.tj == 6) gemm_big_kernel<D, 7, 6><<<grid, block, lds, s>>>(a);
    else if (a.ti == 6 && a.tj == 7) gemm_big_kernel<D, 6, 7><<<grid, block, lds, s>>>(a);
    else if (a.ti == 8 && a.tj == 6) gemm_big_kernel<D, 8, 6><<<grid, block, lds, s>>>(a);
    else if (a.ti == 8 && a.tj == 5) gemm_big_kernel<D, 8, 5><<<grid, block, lds, s>>>(a);
    else if (a.ti == 6 && a.tj == 8) gemm_big_kernel<D, 6, 8><<<grid, block, lds, s>>>(a);
    else if (a.ti == 5 && a.tj == 8) gemm_big_kernel<D, 5, 8><<<grid, block, lds, s>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int D>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile_mfma<D>(g, blockIdx.x, smem);
}

template <int D>
__global__ __launch_bounds__(256) void gemm_mfma128_kernel(GemmArgs g) {
    extern __shared__ __align__(16) unsigned char smem[];
    gemm_tile_mfma128<D>(g, blockIdx.x, smem);
}

// Dynamic LDS of the LDS-staged tile kernel: the A and B tiles of one K step
// (rows padded as the kernel pads them).
static long long tiled_lds_bytes(int dsr, int tb, int ti, int tj, int tk) {
    return (1ll << (tb + tk)) * (pad_dim(1 << ti) + pad_dim(1 << tj)) * lds_elem_bytes(dsr);
}

GemmShape heuristic_gemm_shape(int dsr, int lb, int li, int lj, int lk, int a_t, int b_t, bool mfma128) {
    GemmShape g{};
    g.lb = lb;
    g.li = li;
    g.lj = lj;
    g.lk = lk;
    g.a_t = a_t;
    g.b_t = b_t;
    const int lds_cap = 40 * 1024;
    g.mfma = 0;
    g.mode = GEMM_TILED;
    // 32- and 40-byte entries: LDS-staged tiles, one output per thread
    const bool topk = dsr == DSR_TOPK || dsr == DSR_TPOLY;
    if (!topk && li == 0 && lj == 0 && lk >= 12) {  // one output per batch, long K
        g.mode = GEMM_DOT;
        g.rm = g.rn = 1;
        int ls = 9 - lb;  // about 512 workgroups, each over >= 2^12 of K
        if (ls > lk - 12) ls = lk - 12;
        if (ls > 10) ls = 10;
        g.lsplit = ls < 0 ? 0 : ls;
        return g;
    }
    const int kthin = dsr == DSR_CTROP ? 1 : 2;  // K entries of <= 16 bytes per row
    if (!topk && li >= 10 && lj <= 4 && lk <= kthin && lj + lk <= 5) {  // thin: N * K <= 32
        g.mode = GEMM_THIN;
        g.rm = g.rn = 1;
        g.ti = li < 12 ? li : 12;
        g.tj = lj;
        g.tk = lk;
        return g;
    }
    const bool four_byte_valu = dsr == DSR_TROP_I32 || dsr == DSR_TROP_F32 || dsr == DSR_MODP;
    // register-tiled family: 128 x 128 for large M and N; 256 x 64 / 256 x 32
    // (or mirrored) when one side is large and the other 2^5 or 2^6
    int bti = 0, btj = 0;
    if (li >= 7 && lj >= 7 && lk >= 4) {
        bti = btj = 7;
        // at most 32 output tiles: halve the tile so that two workgroups per
        // CU of a 32-CU chiplet each get one (instead of some CUs two tiles)
        if (lb + (li - 7) + (lj - 7) <= 5) {
            if (lj >= li) btj = 6;
            else bti = 6;
        }
    }
    else if (li >= 8 && (lj == 5 || lj == 6) && lk >= 2) bti = 8, btj = lj;
    else if (lj >= 8 && (li == 5 || li == 6) && lk >= 2) bti = li, btj = 8;
    // counting tropical: 128 x 64 / 64 x 128, or 256 x 32 / 32 x 256
    int cti = 0, ctj = 0;
    if (li >= 7 && lj >= 6 && lk >= 2) cti = 7, ctj = 6;
    else if (li >= 6 && lj >= 7 && lk >= 2) cti = 6, ctj = 7;
    else if (li >= 8 && lj == 5 && lk >= 2) cti = 8, ctj = 5;
    else if (lj >= 8 && li == 5 && lk >= 2) cti = 5, ctj = 8;
    if (topk) {
        cti = 0;
        bti = 0;
    }
    if (dsr == DSR_CTROP && cti) {
        g.rm = g.rn = 8;
        g.ti = cti;
        g.tj = ctj;
        g.tb = 0;
        const int tkmax = (cti == 8 || ctj == 8) ? 3 : 4;  // operand tiles <= 40 KB of LDS
        g.tk = lk < tkmax ? lk : tkmax;
    } else if (four_byte_valu && bti) {
        g.rm = g.rn = 8;
        g.ti = bti;
        g.tj = btj;
        g.tb = 0;
        // K step: 32 for the square tile, 16 for the 256-wide ones, so that
        // four workgroups' operand tiles fit in one CU's LDS
        const int tkmax = (bti == 8 || btj == 8) ? 4 : 5;
        g.tk = lk < tkmax ? lk : tkmax;
    } else if (mfma128 && (dsr == DSR_Z_F32 || dsr == DSR_Z_BF16) && li >= 7 && lj >= 7 &&
               lk >= (dsr == DSR_Z_BF16 ? 5 : 4)) {
        // partition function on the matrix cores, 128 x 128 tiles
        g.rm = g.rn = 4;
        g.ti = g.tj = 7;
        g.tb = 0;
        g.tk = dsr == DSR_Z_BF16 ? 5 : 4;
        g.mfma = 2;
    } else if (!topk && li >= 6 && lj >= 6 && lk >= 4) {
        // contraction-heavy node: 64x64 tile, 4x4 per thread (or one 32x32
        // matrix-core block per wave for the partition function)
        g.rm = g.rn = 4;
        g.ti = g.tj = 6;
        g.tb = 0;
        g.tk = lk < 5 ? lk : 5;
        while (g.tk > 0 && tiled_lds_bytes(dsr, 0, 6, 6, g.tk) > lds_cap) g.tk--;
        g.mfma = (dsr == DSR_Z_F32 || dsr == DSR_Z_BF16) ? 1 : 0;
    } else {
        // little reuse per output (K <= 8) and many outputs: 4 x 4 per
        // thread, 4096 outputs per workgroup, so fewer and larger tiles
        // carry the output traffic (each tile pays one load round trip)
        const bool wide = !topk && lk <= 3 && li >= 2 && lj >= 2 && lb + li + lj >= 14;
        g.rm = topk ? 1 : wide ? 4 : (li >= 1 ? 2 : 1);
        g.rn = topk ? 1 : wide ? 4 : (lj >= 1 ? 2 : 1);
        const int lr = (g.rm == 4 ? 2 : g.rm == 2 ? 1 : 0) + (g.rn == 4 ? 2 : g.rn == 2 ? 1 : 0);
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
        while (g.tk > 0 && tiled_lds_bytes(dsr, g.tb, g.ti, g.tj, g.tk) > lds_cap) g.tk--;
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
    if ((dsr == DSR_TOPK || dsr == DSR_TPOLY) && (g.mode != GEMM_TILED || g.rm != 1 || g.rn != 1 || g.mfma))
        return false;
    if (g.mode == GEMM_DOT)
        return g.li == 0 && g.lj == 0 && g.ti == 0 && g.tj == 0 && g.tb == 0 && !g.mfma && g.lsplit >= 0 &&
               g.lsplit <= 10 && g.lsplit <= g.lk;
    if (g.mode == GEMM_THIN)
        return g.tb == 0 && g.tj == g.lj && g.tk == g.lk && g.lj <= 4 && g.lk <= 2 && g.lj + g.lk <= 5 &&
               g.ti >= 10 && g.ti <= g.li && g.lsplit == 0 && !g.mfma;
    if (g.mode != GEMM_TILED) return false;
    if ((g.rm == 8 || g.rn == 8) && dsr == DSR_CTROP) {  // counting-tropical register tiles
        if (g.rm != 8 || g.rn != 8 || !ct_tile_shape(g.ti, g.tj) || g.tb != 0 || g.mfma) return false;
        if (g.tk < 0 || g.tk > 4 || g.tk + g.lsplit > g.lk || g.li < g.ti || g.lj < g.tj) return false;
        return (size_t)(1 << g.tk) * (((1 << g.ti) + 4) + ((1 << g.tj) + 4)) * 12 <= 40 * 1024;
    }
    if (g.rm == 8 || g.rn == 8) {  // the register-tiled family; ti, tj give the tile
        if (dsr != DSR_TROP_I32 && dsr != DSR_TROP_F32 && dsr != DSR_MODP) return false;
        if (g.rm != 8 || g.rn != 8 || !big_tile_shape(g.ti, g.tj) || g.tb != 0 || g.mfma) return false;
        if (g.tk < 1 || g.tk > 5 || g.tk + g.lsplit > g.lk || g.li < g.ti || g.lj < g.tj) return false;
        return true;
    }
    if (g.mfma == 2) {  // 128 x 128 matrix-core tiles, fixed K step
        if (dsr != DSR_Z_F32 && dsr != DSR_Z_BF16) return false;
        return g.ti == 7 && g.tj == 7 && g.tb == 0 && g.rm == 4 && g.rn == 4 && g.li >= 7 && g.lj >= 7 &&
               g.tk == (dsr == DSR_Z_BF16 ? 5 : 4) && g.lsplit >= 0 && g.tk + g.lsplit <= g.lk;
    }
    if (g.mfma) {
        if (g.mfma != 1 || (dsr != DSR_Z_F32 && dsr != DSR_Z_BF16)) return false;
        if (g.ti != 6 || g.tj != 6 || g.tb != 0) return false;
        if (g.tk < (dsr == DSR_Z_BF16 ? 4 : 1)) return false;
    }
    if (g.tb < 0 || g.ti < 0 || g.tj < 0 || g.tk < 0 || g.lsplit < 0) return false;
    if (g.tb > g.lb || g.ti > g.li || g.tj > g.lj || g.tk + g.lsplit > g.lk) return false;
    if (g.rm != 1 && g.rm != 2 && g.rm != 4) return false;
    if (g.rn != 1 && g.rn != 2 && g.rn != 4) return false;
    if ((1 << g.ti) < g.rm || (1 << g.tj) < g.rn) return false;
    long long threads = (1ll << (g.tb + g.ti + g.tj)) / (g.rm * g.rn);
    if (threads > 256 || threads < 1) return false;
    return tiled_lds_bytes(dsr, g.tb, g.ti, g.tj, g.tk) <= 48 * 1024;
}

size_t gemm_lds_bytes(int dsr, const GemmShape& g) {
    if (g.mode == GEMM_DOT) return 256 * (size_t)lds_elem_bytes(dsr);
    if (g.mfma == 2) return dsr == DSR_Z_BF16 ? Mfma128<DSR_Z_BF16>::LDS : Mfma128<DSR_Z_F32>::LDS;
    if (g.mode == GEMM_THIN) return ((size_t)1 << (g.lk + g.lj)) * lds_elem_bytes(dsr);
    if (g.rm == 8)
        return (size_t)(1 << g.tk) * (((1 << g.ti) + 4) + ((1 << g.tj) + 4)) * (dsr == DSR_CTROP ? 12 : 4);
    return (size_t)tiled_lds_bytes(dsr, g.tb, g.ti, g.tj, g.tk);
}

template <int D, int RM, int RN>
static hipError_t gemm_go(const GemmArgs& a, size_t lds, u64 blocks, hipStream_t s) {
    gemm_kernel<D, RM, RN><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
    return hipGetLastError();
}

template <int D>
static hipError_t gemm_dispatch(const GemmArgs& a, int rm, int rn, size_t lds, u64 blocks, hipStream_t s) {
    if constexpr (D == DSR_TOPK || D == DSR_TPOLY) {  // wide entries: one output per thread
        if (rm == 1 && rn == 1) return gemm_go<D, 1, 1>(a, lds, blocks, s);
        return hipErrorInvalidValue;
    } else {
        if (rm == 1 && rn == 1) return gemm_go<D, 1, 1>(a, lds, blocks, s);
        if (rm == 1 && rn == 2) return gemm_go<D, 1, 2>(a, lds, blocks, s);
        if (rm == 2 && rn == 1) return gemm_go<D, 2, 1>(a, lds, blocks, s);
        if (rm == 2 && rn == 2) return gemm_go<D, 2, 2>(a, lds, blocks, s);
        if (rm == 4 && rn == 4) return gemm_go<D, 4, 4>(a, lds, blocks, s);
        return hipErrorInvalidValue;
    }
}

GemmArgs make_gemm_args(Planes Ap, Planes Bp, Planes Cp, Planes part, const GemmShape& g, const AlgebraParams& ap,
                        TensorMeta* meta, int ma, int mb, int mc) {
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
    return a;
}

hipError_t launch_gemm(int dsr, Planes Ap, Planes Bp, Planes Cp, Planes part, const GemmShape& g,
                       const AlgebraParams& ap, TensorMeta* meta, int ma, int mb, int mc, hipStream_t s) {
    if (!gemm_shape_valid(dsr, g)) return hipErrorInvalidValue;
    GemmArgs a = make_gemm_args(Ap, Bp, Cp, part, g, ap, meta, ma, mb, mc);
    size_t lds = gemm_lds_bytes(dsr, g);
    u64 blocks = 1ull << ((g.lb - g.tb) + (g.li - g.ti) + (g.lj - g.tj) + g.lsplit);
    if (g.mode != GEMM_TILED) {
        switch (dsr) {
        case DSR_TROP_I32: return gemm_mode_go<DSR_TROP_I32>(a, g.mode, lds, blocks, s);
        case DSR_TROP_F32: return gemm_mode_go<DSR_TROP_F32>(a, g.mode, lds, blocks, s);
        case DSR_CTROP: return gemm_mode_go<DSR_CTROP>(a, g.mode, lds, blocks, s);
        case DSR_MODP: return gemm_mode_go<DSR_MODP>(a, g.mode, lds, blocks, s);
        case DSR_Z_F32: return gemm_mode_go<DSR_Z_F32>(a, g.mode, lds, blocks, s);
        case DSR_Z_BF16: return gemm_mode_go<DSR_Z_BF16>(a, g.mode, lds, blocks, s);
        case DSR_TOPK:
        case DSR_TPOLY: return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    }
    if (g.rm == 8) {
        if (dsr == DSR_CTROP) return gemm_ct_big_go(a, lds, blocks, s);
        if (dsr == DSR_TROP_I32) return gemm_big_go<DSR_TROP_I32>(a, lds, blocks, s);
        if (dsr == DSR_TROP_F32) return gemm_big_go<DSR_TROP_F32>(a, lds, blocks, s);
        return gemm_big_go<DSR_MODP>(a, lds, blocks, s);
    }
    if (g.mfma == 2) {
        if (dsr == DSR_Z_F32)
            gemm_mfma128_kernel<DSR_Z_F32><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
        else
            gemm_mfma128_kernel<DSR_Z_BF16><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
        return hipGetLastError();
    }
    if (g.mfma) {
        if (dsr == DSR_Z_F32)
            gemm_mfma_kernel<DSR_Z_F32><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
        else
            gemm_mfma_kernel<DSR_Z_BF16><<<dim3((unsigned)blocks), dim3(256), lds, s>>>(a);
        return hipGetLastError();
    }
#define TN_GM(D) \
    case D: return gemm_dispatch<D>(a, g.rm, g.rn, lds, blocks, s);
    switch (dsr) {
        TN_GM(DSR_TROP_I32)
        TN_GM(DSR_TROP_F32)
        TN_GM(DSR_CTROP)
        TN_GM(DSR_MODP)
        TN_GM(DSR_Z_F32)
        TN_GM(DSR_Z_BF16)
        TN_GM(DSR_TOPK)
        TN_GM(DSR_TPOLY)
    default: return hipErrorInvalidValue;
    }
#undef TN_GM
}

// --------------------------------------------------------- split reduce --
// Large outputs: one thread per entry; small outputs: one workgroup per entry.
template <int D>
__global__ __launch_bounds__(256) void split_reduce_kernel(Planes part, Planes C, i64 nout, int lsplit,
                                                           AlgebraParams ap, TensorMeta* meta, int mc,
                                                           int per_block) {
    using A = Alg<D>;
    using V = typename A::V;
    __shared__ V red[256];
    if (per_block) {
        split_reduce_one<D>(part, C, nout, lsplit, ap, meta, mc, (i64)blockIdx.x, red);
        return;
    }
    const int S = 1 << lsplit;
    float lmax = 0.0f, lmin = INFINITY;
    i64 o = (i64)blockIdx.x * 256 + threadIdx.x;
    if (o < nout) {
        const V acc = split_sum<D>(part, nout, o, S, ap);
        A::store(C, o, acc);
        if constexpr (is_z<D>()) z_track(acc, lmax, lmin);
    }
    if constexpr (is_z<D>()) z_meta_block(meta, mc, lmax, lmin);
}

// ---------------------------------------------------------- back-trace --
// One workgroup walks the tree from the root, one depth level at a time (a
// node's output indices are fixed once its parent is done, and nodes of one
// level sum disjoint index sets, so they are independent).  Within a level
// each wave takes whole nodes: lane 0 reads the node's value at its assigned
// output indices and lists the summed indices, then the 64 lanes scan the
// assignments of the summed indices in increasing order, 64 at a time, for
// the first one whose A + B equals that value.  The GEMM formed the value as
// the maximum of exactly these float sums, so the equality is exact, and the
// first match is the smallest assignment, whatever the waves' timing.
constexpr int kBtWaves = 8;

// the lanes of one wave see each other's LDS writes after this point
__device__ inline void bt_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64 * kBtWaves) void backtrace_kernel(
    const float* arena, const int* g_nodes, int ninner, const int* g_ord_off, const int* g_ord_ids,
    const long long* g_off, const int* g_lvl_off, const int* g_lvl_nodes, int nlevels, int* g_assign, int* status,
    int nn, int nids, int nv, int use_lds) {
    // the tables and the assignment live in LDS when they fit
    extern __shared__ __align__(16) unsigned char bt_lds[];
    const int* nodes = g_nodes;
    const int* ord_off = g_ord_off;
    const int* ord_ids = g_ord_ids;
    const long long* off = g_off;
    const int* lvl_off = g_lvl_off;
    const int* lvl_nodes = g_lvl_nodes;
    int* assign = g_assign;
    if (use_lds) {
        long long* s_off = (long long*)bt_lds;
        int* s_nodes = (int*)(s_off + nn);
        int* s_oo = s_nodes + 3 * ninner;
        int* s_oi = s_oo + nn + 1;
        int* s_lo = s_oi + nids;
        int* s_ln = s_lo + nlevels + 1;
        int* s_as = s_ln + ninner;
        for (int i = threadIdx.x; i < nn; i += blockDim.x) s_off[i] = g_off[i];
        for (int i = threadIdx.x; i < 3 * ninner; i += blockDim.x) s_nodes[i] = g_nodes[i];
        for (int i = threadIdx.x; i <= nn; i += blockDim.x) s_oo[i] = g_ord_off[i];
        for (int i = threadIdx.x; i < nids; i += blockDim.x) s_oi[i] = g_ord_ids[i];
        for (int i = threadIdx.x; i <= nlevels; i += blockDim.x) s_lo[i] = g_lvl_off[i];
        for (int i = threadIdx.x; i < ninner; i += blockDim.x) s_ln[i] = g_lvl_nodes[i];
        for (int i = threadIdx.x; i < nv; i += blockDim.x) s_as[i] = g_assign[i];
        nodes = s_nodes;
        ord_off = s_oo;
        ord_ids = s_oi;
        off = s_off;
        lvl_off = s_lo;
        lvl_nodes = s_ln;
        assign = s_as;
    }
    constexpr int kMaxFree = 30, kMaxRank = 62;
    // per wave: the summed indices of its node, and where each operand index
    // takes its bit from (>= 0: position among the summed indices; < 0:
    // -1 - the fixed value)
    __shared__ int w_free[kBtWaves][kMaxFree];
    __shared__ int w_mapA[kBtWaves][kMaxRank], w_mapB[kBtWaves][kMaxRank];
    __shared__ int w_nfree[kBtWaves], w_rankA[kBtWaves], w_rankB[kBtWaves], w_err[kBtWaves];
    __shared__ long long w_taddr[kBtWaves];
    __shared__ int stop;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    if (threadIdx.x == 0) stop = 0;
    __syncthreads();
    for (int lv = 0; lv < nlevels; lv++) {
        for (int i = lvl_off[lv] + wave; i < lvl_off[lv + 1]; i += kBtWaves) {
            const int t = lvl_nodes[i];
            const int x = nodes[3 * t], a = nodes[3 * t + 1], b = nodes[3 * t + 2];
            if (lane == 0) {
                int err = 0;
                long long addr = 0;
                const int rc = ord_off[x + 1] - ord_off[x];
                if (rc > kMaxRank) err = 2;
                for (int q = 0; q < rc && !err; q++) {
                    const int v = assign[ord_ids[ord_off[x] + q]];
                    if (v < 0) err = 3;  // an output index left unset
                    addr |= (long long)(v & 1) << q;
                }
                w_taddr[wave] = err ? 0 : off[x] + addr;
                int nfree = 0;
                for (int side = 0; side < 2 && !err; side++) {
                    const int y = side ? b : a;
                    int* map = side ? w_mapB[wave] : w_mapA[wave];
                    const int r = ord_off[y + 1] - ord_off[y];
                    if (side) w_rankB[wave] = r;
                    else w_rankA[wave] = r;
                    if (r > kMaxRank) {
                        err = 2;
                        break;
                    }
                    for (int q = 0; q < r; q++) {
                        const int id = ord_ids[ord_off[y] + q];
                        const int cur = assign[id];
                        if (cur >= 0) {
                            map[q] = -1 - (cur & 1);
                            continue;
                        }
                        // a summed index already listed for this node is marked
                        // -2 - position until the node's values are written
                        int pos = cur <= -2 ? -2 - cur : -1;
                        if (pos < 0) {
                            if (nfree == kMaxFree) {
                                err = 2;
                                break;
                            }
                            pos = nfree;
                            w_free[wave][nfree++] = id;
                            assign[id] = -2 - pos;
                        }
                        map[q] = pos;
                    }
                }
                w_nfree[wave] = nfree;
                w_err[wave] = err;
                if (err) {
                    *status = err;
                    stop = err;
                }
            }
            bt_wave_sync();
            if (w_err[wave]) break;
            const int nf = w_nfree[wave], ra = w_rankA[wave], rb = w_rankB[wave];
            const int* mapA = w_mapA[wave];
            const int* mapB = w_mapB[wave];
            const float target = arena[w_taddr[wave]];
            const long long baseA = off[a], baseB = off[b];
            const unsigned long long total = 1ull << nf;
            long long found = -1;
            for (unsigned long long s0 = 0; s0 < total; s0 += 64) {
                const unsigned long long sv = s0 + (unsigned long long)lane;
                bool hit = false;
                if (sv < total) {
                    long long addrA = 0, addrB = 0;
                    for (int q = 0; q < ra; q++) {
                        const int m = mapA[q];
                        addrA |= (long long)(m >= 0 ? (int)((sv >> m) & 1) : -1 - m) << q;
                    }
                    for (int q = 0; q < rb; q++) {
                        const int m = mapB[q];
                        addrB |= (long long)(m >= 0 ? (int)((sv >> m) & 1) : -1 - m) << q;
                    }
                    hit = arena[baseA + addrA] + arena[baseB + addrB] == target;
                }
                const unsigned long long mask = __ballot(hit);
                if (mask) {
                    found = (long long)(s0 + (unsigned long long)__builtin_ctzll(mask));
                    break;
                }
            }
            if (lane == 0) {
                if (found < 0) {
                    *status = 1;
                    stop = 1;
                } else {
                    for (int f = 0; f < nf; f++) assign[w_free[wave][f]] = (int)((found >> f) & 1);
                }
            }
            bt_wave_sync();  // the wave's tables are rewritten for its next node
            if (found < 0) break;
        }
        __syncthreads();
        const int halt = stop;
        __syncthreads();
        if (halt) break;
    }
    if (use_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < nv; i += blockDim.x) g_assign[i] = assign[i];
    }
}

hipError_t launch_backtrace(const float* arena, const int* nodes, int ninner, const int* ord_off, const int* ord_ids,
                            const long long* off, const int* lvl_off, const int* lvl_nodes, int nlevels, int* assign,
                            int* status, int nn, int nids, int nv, hipStream_t s) {
    const size_t bytes = 8 * (size_t)nn + 4 * (3 * (size_t)ninner + (size_t)nn + 1 + (size_t)nids + (size_t)nlevels +
                                               1 + (size_t)ninner + (size_t)nv);
    const int use_lds = bytes <= 40 * 1024 ? 1 : 0;
    backtrace_kernel<<<1, 64 * kBtWaves, use_lds ? bytes : 0, s>>>(arena, nodes, ninner, ord_off, ord_ids, off, lvl_off,
                                                                   lvl_nodes, nlevels, assign, status, nn, nids, nv,
                                                                   use_lds);
    return hipGetLastError();
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
        TN_SR(DSR_MODP)
        TN_SR(DSR_Z_F32)
        TN_SR(DSR_Z_BF16)
        TN_SR(DSR_TOPK)
        TN_SR(DSR_TPOLY)
    default: return hipErrorInvalidValue;
    }
#undef TN_SR
    return hipGetLastError();
}

// ---------------------------------------------------------- accumulate ---
// Entry e of the root (a scalar, or the tensor over the open vertices) is
// folded into accumulator slot e (kAccSlotBytes apart).
template <int D>
__global__ void accumulate_kernel(Planes root, int mroot, TensorMeta* meta, void* acc, int first, AlgebraParams ap,
                                  long long nent) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent) return;
    Planes r;
    r.p0 = (unsigned char*)root.p0 + e * plane_bytes_dev<D>(0);
    r.p1 = plane_bytes_dev<D>(1) ? (unsigned char*)root.p1 + e * plane_bytes_dev<D>(1) : nullptr;
    accumulate_one<D>(r, mroot, meta, (unsigned char*)acc + kAccSlotBytes * e, first, ap);
}

hipError_t launch_accumulate(int dsr, Planes root, int mroot, TensorMeta* meta, void* acc, int first,
                             const AlgebraParams& ap, hipStream_t s, long long nent) {
    if (nent < 1) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((nent + 255) / 256), threads = nent < 256 ? (unsigned)nent : 256u;
#define TN_AC(D)                                                                                        \
    case D:                                                                                             \
        accumulate_kernel<D><<<blocks, threads, 0, s>>>(root, mroot, meta, acc, first, ap, nent); \
        break;
    switch (dsr) {
        TN_AC(DSR_TROP_I32)
        TN_AC(DSR_TROP_F32)
        TN_AC(DSR_CTROP)
        TN_AC(DSR_MODP)
        TN_AC(DSR_Z_F32)
        TN_AC(DSR_Z_BF16)
        TN_AC(DSR_TOPK)
        TN_AC(DSR_TPOLY)
    default: return hipErrorInvalidValue;
    }
#undef TN_AC
    return hipGetLastError();
}

template <int D>
__global__ void set_one_kernel(void* acc, AlgebraParams ap) {
    set_one<D>(acc, ap);
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
        TN_SO(DSR_MODP)
        TN_SO(DSR_Z_F32)
        TN_SO(DSR_Z_BF16)
        TN_SO(DSR_TOPK)
        TN_SO(DSR_TPOLY)
    default: return hipErrorInvalidValue;
    }
#undef TN_SO
    return hipGetLastError();
}

int accumulator_bytes(int) { return 16; }

// ------------------------------------------------------ tuning helpers --
// Seeded operand data for timing and checking candidate launch shapes: a
// SplitMix64-style hash of (seed, index) mapped into each algebra's values
// (small sizes, full 64-bit counts, residues below p, positive reals).
__device__ inline u64 mix64(u64 z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void fill_tune_kernel(int dsr, Planes p, i64 n, u64 seed, unsigned int prime) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const u64 h = mix64(seed ^ mix64((u64)i));
        switch (dsr) {
        case DSR_TROP_I32: ((int*)p.p0)[i] = (int)(h & 15); break;
        case DSR_TROP_F32: ((float*)p.p0)[i] = (float)(h & 255) * 0.0625f; break;
        case DSR_CTROP:
            ((int*)p.p0)[i] = (int)(h & 3);
            ((u64*)p.p1)[i] = mix64(h);
            break;
        case DSR_MODP: ((unsigned int*)p.p0)[i] = (unsigned int)((h >> 16) % prime); break;
        default: ((float*)p.p0)[i] = 0.5f + (float)(h & 0xffff) * (0.5f / 65536.0f); break;
        }
    }
}

hipError_t launch_fill_tune(int dsr, Planes p, i64 n, u64 seed, unsigned int prime, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const i64 blocks = std::min<i64>((n + 255) / 256, 8192);
    fill_tune_kernel<<<(unsigned)blocks, 256, 0, s>>>(dsr, p, n, seed, prime);
    return hipGetLastError();
}

// Entries of x and y that differ: bit patterns for the exact algebras, and
// more than rtol relative for the real ones.
__global__ void compare_tune_kernel(int dsr, Planes x, Planes y, i64 n, float rtol, unsigned long long* bad) {
    unsigned long long local = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        bool diff;
        if (dsr == DSR_Z_F32 || dsr == DSR_Z_BF16) {
            const float a = ((const float*)x.p0)[i], b = ((const float*)y.p0)[i];
            diff = !(fabsf(a - b) <= rtol * fmaxf(fabsf(a), fabsf(b)));
        } else {
            diff = ((const unsigned int*)x.p0)[i] != ((const unsigned int*)y.p0)[i];
            if (dsr == DSR_CTROP) diff = diff || ((const u64*)x.p1)[i] != ((const u64*)y.p1)[i];
        }
        local += diff ? 1 : 0;
    }
    if (local) atomicAdd(bad, local);
}

hipError_t launch_compare_tune(int dsr, Planes x, Planes y, i64 n, float rtol, unsigned long long* bad,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const i64 blocks = std::min<i64>((n + 255) / 256, 8192);
    compare_tune_kernel<<<(unsigned)blocks, 256, 0, s>>>(dsr, x, y, n, rtol, bad);
    return hipGetLastError();
}

}  // namespace tn
