// Host-callable launchers of the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

// Device algebra of one contraction pass.  Exact counting runs one pass per
// prime: DSR_MODP (counts mod p), recombined by CRT on the host.
enum DevSemiring {
    DSR_TROP_I32 = 0,
    DSR_TROP_F32 = 1,
    DSR_CTROP = 2,   // plane 0 int32 size, plane 1 uint64 count
    DSR_MODP = 3,    // Montgomery form, R = 2^32
    DSR_Z_F32 = 4,   // float32 with per-tensor power-of-two exponents
    DSR_Z_BF16 = 5,  // as DSR_Z_F32, GEMM inputs rounded to bfloat16
    DSR_TOPK = 6,    // the eight largest values with multiplicity (32-byte entries)
    DSR_TPOLY = 7,   // truncated polynomial: plane 0 int32 top exponent, plane 1 four uint64 counts
    DSR_COUNT_ = 8
};

// bytes per entry of plane 0 / plane 1 (0 = no such plane)
int plane_bytes(int dsr, int plane);

struct Planes {
    void* p0 = nullptr;
    void* p1 = nullptr;
};

// Per-tensor bookkeeping of the partition-function algebra: the true tensor
// is stored * 2^exp; maxbits is the float bit pattern of max|stored|.
struct TensorMeta {
    long long exp;
    unsigned int maxbits;    // bits of the largest stored entry (a non-negative float)
    unsigned int minnz_inv;  // complement of the bits of the smallest nonzero stored entry; 0: none yet
    float operand_range;     // inner nodes: log2 range of A plus that of B (what a product spans)
    unsigned int pad;
};

struct AlgebraParams {
    uint32_t p = 0, pinv = 0, r1 = 0;  // modulus, -p^{-1} mod 2^32, 2^32 mod p
    uint32_t xv = 0;                   // mod p: the vertex tensor's x (Montgomery form; 1 = r1 counts)
    int fix_off = -1;                  // fixed vertices: w[fix_off + v] = -1 (free), 0 or 1; -1: none
    int pad = 0;
    double beta = 0;
};

// Leaf descriptor on the device (one per leaf tensor, rank <= 2).
struct LeafDev {
    int u, v;          // edge ends (u < v) or u = vertex of a vertex-only leaf, v = -1
    int flags;         // 1: edge factor, 2: W_u, 4: W_v, 8: spin-glass factors
    int jidx;          // spin glass: index of the edge's coupling in the weight array (-1: none)
    int pad;
    int rank;          // unsliced output indices
    int var0, var1;    // vertex at bit 0 / bit 1
    long long off;     // arena offset (entries)
};

// One permute of the bits of a linear offset, compact (see kernels.hip): the
// tile bits (input bit u[t] and output bit vo[t] of tile bit t; ef[t]: the
// read-order bit that feeds output tile bit t) and the bits that enumerate
// tiles.  Built on the host and uploaded; a kernel expands it into
// PermTables once per program.
struct PermParams {
    signed char u[12], vo[12], ef[12];
    signed char tin[48], tout[48];
    int rank, tile_bits, ntile_bits, pad;
};

// The same permute as the permute kernels read it: 64-entry lookup tables of
// six tile bits each (input and output offsets, read-order index) and the
// tile-enumeration bits, device-resident.
struct PermTables {
    long long in_lo[64], in_hi[64];
    long long out_lo[64], out_hi[64];
    int e_lo[64], e_hi[64];
    signed char tin[48], tout[48];
    int rank, tile_bits, ntile_bits, pad;
};

struct GemmShape {
    int lb, li, lj, lk;    // log2 batch, M, N, K
    int a_t, b_t;          // operand transposition flags
    int tb, ti, tj, tk;    // log2 tile (batch, M, N, K-step)
    int rm, rn;            // per-thread micro tile
    int lsplit;            // log2 of K splits (partials then reduce)
    int mfma;              // partition function on matrix cores (64 x 64 tile, 4 waves)
    int mode;              // GEMM_TILED, GEMM_THIN or GEMM_DOT
};

// GEMM kernel modes: LDS-staged tiles (the 4x4 / register-tiled families),
// row streaming for thin nodes (N * K <= 32: each thread owns whole output
// rows, B sits in LDS), and a long-K reduction for nodes with one output per
// batch (M = N = 1).
enum GemmMode { GEMM_TILED = 0, GEMM_THIN = 1, GEMM_DOT = 2 };

// log2 entries of one permute tile for a tensor of the given rank
constexpr int kPermTileBits = 12;
inline int perm_tile_bits(int rank) { return rank < kPermTileBits ? rank : kPermTileBits; }

void build_perm_params(int rank, const int* src, PermParams& pp);

hipError_t launch_meta_init(TensorMeta* meta, int n, hipStream_t s);
hipError_t launch_leaves(int dsr, const LeafDev* leaves, int nleaf, const float* w, const int* slice_pos,
                         unsigned long long slice_id, Planes arena, const AlgebraParams& ap,
                         TensorMeta* meta, hipStream_t s);
// tables[i] = the expansion of perms[i], i < n (device pointers)
hipError_t launch_expand_perms(const PermParams* perms, PermTables* tables, int n, hipStream_t s);
hipError_t launch_permute(int elem_bytes, const void* in, void* out, const PermTables* pp_dev, int rank,
                          int tile_bits, hipStream_t s);
hipError_t launch_gemm(int dsr, Planes A, Planes B, Planes C, Planes part, const GemmShape& g,
                       const AlgebraParams& ap, TensorMeta* meta, int ma, int mb, int mc, hipStream_t s);
hipError_t launch_split_reduce(int dsr, Planes part, Planes C, int64_t nout, int lsplit,
                               const AlgebraParams& ap, TensorMeta* meta, int mc, hipStream_t s);
// acc[e] (+)= root[e] for the nent root entries, kAccSlotBytes apart; first
// != 0 copies.  For the partition function a slot is {double mantissa, int64
// exponent}.
constexpr int kAccSlotBytes = 48;
// The partition function's dynamic range (the largest log2(max / smallest
// nonzero) of a stored tensor, or of the two operands of a product added):
// a float at this byte of the pass's first accumulator slot.
constexpr int kZRangeOffset = 32;
hipError_t launch_z_range(const TensorMeta* meta, int n, void* acc, int first, hipStream_t s);
hipError_t launch_accumulate(int dsr, Planes root, int mroot, TensorMeta* meta, void* acc, int first,
                             const AlgebraParams& ap, hipStream_t s, long long nent = 1);
// The device-side identity element of a whole (empty) network.
hipError_t launch_set_one(int dsr, void* acc, const AlgebraParams& ap, hipStream_t s);
int accumulator_bytes(int dsr);

// Back-trace of a max-plus float32 contraction kept in the dependency-graph
// layout (every tensor at arena + off[x] in its storage order): from the root
// down, each inner node's summed indices are set to the first assignment
// whose A + B reproduces the node's stored value.  nodes: 3 ints (node,
// left, right) per inner node in execution order; the storage order of node
// x is ord_ids[ord_off[x] .. ord_off[x+1]) (index ids = vertex ids).  The
// inner nodes by depth from the root: level l holds lvl_nodes[lvl_off[l] ..
// lvl_off[l+1]) (positions in nodes).  assign (nv ints, -1 = unset) receives
// every index value; status: 0 ok, 1 no matching assignment, 2 too many
// summed indices, 3 an output index unset.  nn: all nodes; nids: entries of
// ord_ids; the tables are staged in LDS when they fit in 40 KB.
hipError_t launch_backtrace(const float* arena, const int* nodes, int ninner, const int* ord_off, const int* ord_ids,
                            const long long* off, const int* lvl_off, const int* lvl_nodes, int nlevels, int* assign,
                            int* status, int nn, int nids, int nv, hipStream_t s);

// Launch shape of a GEMM node.  For a per-node launch over the whole chip:
// the entry of the tuning table for this node shape if there is one
// (tune.cpp), else the fixed heuristic.  For a task of the persistent launch
// (chiplet = true: the node's tiles share one chiplet's 32 CUs with the
// job's other nodes) always the heuristic, without the 128 x 128
// matrix-core tiles, which leave too few tiles to go round there; the table
// was timed over the whole chip and does not apply.  Either way the shape
// depends on the node alone, never on the other work of a launch.
GemmShape choose_gemm_shape(int dsr, int lb, int li, int lj, int lk, int a_t, int b_t, bool chiplet = false);
GemmShape heuristic_gemm_shape(int dsr, int lb, int li, int lj, int lk, int a_t, int b_t, bool mfma128 = true);
bool gemm_shape_valid(int dsr, const GemmShape& g);
size_t gemm_lds_bytes(int dsr, const GemmShape& g);
// Counting-tropical register tiles whose next K step is read into LDS while
// the current one computes (128 x 64 and 64 x 128 tiles, 4 <= TK <= 16).
constexpr bool ct_ahead_shape(int ti, int tj, int tk) {
    return ((ti == 7 && tj == 6) || (ti == 6 && tj == 7)) && tk >= 2 && tk <= 4;
}
// Name of the kernel (template instance) a launch of shape g runs, as in
// profiler listings, e.g. "gemm_ct_big_kernel<7, 6, true>".
const char* gemm_kernel_name(int dsr, const GemmShape& g, char* buf, size_t cap);

// Tuning helpers: seeded operand data for an algebra, and a device-side
// count of the entries where two results differ (bit patterns for the exact
// algebras, relative rtol for the real ones), added to *bad.
hipError_t launch_fill_tune(int dsr, Planes p, int64_t n, unsigned long long seed, unsigned int prime, hipStream_t s);
hipError_t launch_compare_tune(int dsr, Planes x, Planes y, int64_t n, float rtol, unsigned long long* bad,
                               hipStream_t s);

}  // namespace tn
