// Persistent batched kernel: executes a task table of many contraction
// passes in one launch (see batch.h for the task model).
#include <hip/hip_runtime.h>

#include <climits>

#include "batch.h"
#include "kernels_dev.h"

namespace tn {

// bytes of dynamic LDS: the largest GEMM tile, a permute tile of 8-byte
// entries with its tables, or a 256-entry reduction buffer
constexpr size_t kBatchLds = 48 * 1024;

size_t batch_lds_bytes() { return kBatchLds; }
static_assert(((sizeof(PermLds) + 255) & ~(size_t)255) + kPermTile * 8 <= kBatchLds, "permute tile fits");

// All tasks of one job run on the same XCC (the host assigns every job to
// one chiplet's queue and a workgroup serves the queue of the XCC it runs
// on), so producer and consumer share that XCC's L2: a task's results are
// visible to the next task once its stores have reached L2 (vmcnt drained)
// and the consumer's CU has dropped its L1 lines.  The counters themselves
// are device-scope atomics.
//
// Every wait is bounded: a wait longer than `limit` ticks of the constant
// wall clock, or any wait while the launch's abort flag is set, sets the flag
// and gives up; the workgroup then leaves the launch.  Every other workgroup
// either runs its next tasks (their inputs are complete) or reaches a wait
// that sees the flag and leaves too, so the kernel always ends and the host
// reports the launch as failed.  The flag and the clock are read only once a
// counter has been found short, and then every 16th poll, so a dependency
// that is already met costs one load.  The first wave polls with the
// counter's value made wave-uniform, so the loop branches on scalars.
__device__ inline bool wait_one(const int* counters, int d, int need, int* abort_flag, long long limit) {
    if (d < 0) return true;
    auto have = [&] {
        return __builtin_amdgcn_readfirstlane(
                   __hip_atomic_load(&counters[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= need;
    };
    if (have()) return true;
    const long long t0 = wall_clock64();
    for (int poll = 1;; poll++) {
        __builtin_amdgcn_s_sleep(1);
        if (have()) return true;
        if ((poll & 15) == 0 &&
            (__builtin_amdgcn_readfirstlane(__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0 ||
             wall_clock64() - t0 > limit)) {
            if ((threadIdx.x & 63) == 0) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// Returns false on giving up.  Out of line: the task loop keeps its values
// in registers that calls preserve, and inlined there the poll loop reloaded
// spilled values from scratch on every poll.
__attribute__((noinline)) __device__ bool wait_counters(const int* counters, int d0, int n0, int d1, int n1, int* abort_flag,
                                     long long limit) {
    __shared__ int s_ok;
    if (__builtin_amdgcn_readfirstlane(threadIdx.x) < 64) {  // the first wave (a wave-uniform branch)
        // wave-uniform arguments (the call passes them in vector registers)
        d0 = __builtin_amdgcn_readfirstlane(d0), n0 = __builtin_amdgcn_readfirstlane(n0);
        d1 = __builtin_amdgcn_readfirstlane(d1), n1 = __builtin_amdgcn_readfirstlane(n1);
        const bool ok = wait_one(counters, d0, n0, abort_flag, limit) && wait_one(counters, d1, n1, abort_flag, limit);
        if (threadIdx.x == 0) s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    const bool ok = s_ok != 0;
    asm volatile("buffer_inv sc0" ::: "memory");  // this CU's L1: refetch from the XCC's L2
    return ok;
}

__device__ inline void signal_counter(int* counters, int c) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores have reached L2
    __syncthreads();
    if (threadIdx.x == 0 && c >= 0) __hip_atomic_fetch_add(&counters[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int D>
__device__ __attribute__((always_inline)) void run_gemm(const BJob& j, const BNode& nd, i64 tile,
                                                        unsigned char* smem) {
    auto at = [&](int64_t off) {
        Planes r;
        r.p0 = (unsigned char*)j.arena.p0 + off * plane_bytes_dev<D>(0);
        r.p1 = plane_bytes_dev<D>(1) ? (unsigned char*)j.arena.p1 + off * plane_bytes_dev<D>(1) : nullptr;
        return r;
    };
    GemmArgs g;
    g.A = at(nd.a_off);
    g.B = at(nd.b_off);
    g.C = at(nd.c_off);
    g.P.p0 = (unsigned char*)j.part.p0 + nd.part_off * plane_bytes_dev<D>(0);
    g.P.p1 = plane_bytes_dev<D>(1) ? (unsigned char*)j.part.p1 + nd.part_off * plane_bytes_dev<D>(1) : nullptr;
    g.lb = nd.g.lb;
    g.li = nd.g.li;
    g.lj = nd.g.lj;
    g.lk = nd.g.lk;
    g.a_t = nd.g.a_t;
    g.b_t = nd.g.b_t;
    g.tb = nd.g.tb;
    g.ti = nd.g.ti;
    g.tj = nd.g.tj;
    g.tk = nd.g.tk;
    g.lsplit = nd.g.lsplit;
    g.ap = j.ap;
    g.meta = j.meta;
    g.ma = nd.ma;
    g.mb = nd.mb;
    g.mc = nd.mc;
    const int rm = nd.g.rm, rn = nd.g.rn;
    if constexpr (D == DSR_TOPK || D == DSR_TPOLY) {  // wide entries: one output per thread only
        gemm_tile<D, 1, 1>(g, (u64)tile, smem);
    } else {
        if (nd.g.mode == GEMM_THIN) {
            gemm_tile_thin<D>(g, (u64)tile, smem);
            return;
        }
        if (nd.g.mode == GEMM_DOT) {
            gemm_tile_dot<D>(g, (u64)tile, smem);
            return;
        }
        if constexpr (is_z<D>()) {  // 64 x 64 matrix-core tiles only (the host never picks 128 x 128 here)
            if (nd.g.mfma) {
                gemm_tile_mfma<D>(g, (u64)tile, smem);
                return;
            }
        }
        if constexpr (big_tile_ok<D>()) {
            if (rm == 8) {
                gemm_tile_big_any<D>(g, (u64)tile, smem);
                return;
            }
        }
        if constexpr (D == DSR_CTROP) {
            if (rm == 8) {
                gemm_tile_ct_big_any<D>(g, (u64)tile, smem);
                return;
            }
        }
        if (rm == 2 && rn == 2)
            gemm_tile<D, 2, 2>(g, (u64)tile, smem);
        else if (rm == 4 && rn == 4)
            gemm_tile<D, 4, 4>(g, (u64)tile, smem);
        else if (rm == 1 && rn == 2)
            gemm_tile<D, 1, 2>(g, (u64)tile, smem);
        else if (rm == 2 && rn == 1)
            gemm_tile<D, 2, 1>(g, (u64)tile, smem);
        else
            gemm_tile<D, 1, 1>(g, (u64)tile, smem);
    }
}

// stores of this workgroup visible to its own later loads (same CU)
__device__ inline void local_step_sync() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    asm volatile("buffer_inv sc0" ::: "memory");
}

template <int D>
__device__ void run_perm(const BJob& j, const BNode& nd, int side, int plane, i64 first, int count,
                         unsigned char* smem) {
    PermLds* tabs = (PermLds*)smem;
    // the truncated polynomial's count plane moves as 4-byte words of rank + 3
    const bool wide1 = D == DSR_TPOLY && plane == 1;
    perm_load_tables(tabs, wide1 ? nd.pp1[side] : nd.pp[side]);
    __syncthreads();
    const int pb = plane_bytes_dev<D>(plane);
    unsigned char* base = (unsigned char*)(plane ? j.arena.p1 : j.arena.p0);
    unsigned char* tile = smem + ((sizeof(PermLds) + 255) & ~(size_t)255);
    const int rank = wide1 ? nd.prank[side] + 3 : nd.prank[side];
    const int tbits = rank < kPermTileBits ? rank : kPermTileBits;
    const int nt = rank - tbits;
    for (int k = 0; k < count; k++) {
        if (pb == 4 || pb == 32)  // 32-byte entries: their 4-byte words, by the host's widened tables
            permute_tile<unsigned int>((const unsigned int*)(base + nd.psrc[side] * pb),
                                       (unsigned int*)(base + nd.pdst[side] * pb), tabs, (unsigned int*)tile,
                                       tbits, nt, first + k);
        else
            permute_tile<u64>((const u64*)(base + nd.psrc[side] * 8), (u64*)(base + nd.pdst[side] * 8), tabs,
                              (u64*)tile, tbits, nt, first + k);
    }
}

template <int D>
__device__ void run_reduce(const BJob& j, const BNode& nd, i64 first, int count, unsigned char* smem) {
    using A = Alg<D>;
    using V = typename A::V;
    Planes C, P;
    C.p0 = (unsigned char*)j.arena.p0 + nd.c_off * plane_bytes_dev<D>(0);
    C.p1 = plane_bytes_dev<D>(1) ? (unsigned char*)j.arena.p1 + nd.c_off * plane_bytes_dev<D>(1) : nullptr;
    P.p0 = (unsigned char*)j.part.p0 + nd.part_off * plane_bytes_dev<D>(0);
    P.p1 = plane_bytes_dev<D>(1) ? (unsigned char*)j.part.p1 + nd.part_off * plane_bytes_dev<D>(1) : nullptr;
    if (nd.reduce_per_block) {
        for (int k = 0; k < count; k++)
            split_reduce_one<D>(P, C, nd.nout, nd.g.lsplit, j.ap, j.meta, nd.mc, first + k, (V*)smem);
        return;
    }
    const int S = 1 << nd.g.lsplit;
    if constexpr (D == DSR_TOPK || D == DSR_TPOLY) {  // wide entries: one unit at a time
        for (int k = 0; k < count; k++) {
            const i64 o = (first + k) * 256 + threadIdx.x;
            if (o < nd.nout) A::store(C, o, split_sum<D>(P, nd.nout, o, S, j.ap));
        }
        return;
    }
    float lmax = 0.0f, lmin = INFINITY;
    for (int k = 0; k < count; k += 4) {
        // four units per pass: with at most 4 splits all their loads are in
        // flight together (a unit is one output per thread)
        i64 o[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            o[u] = (first + k + u) * 256 + threadIdx.x;
            ok[u] = k + u < count && o[u] < nd.nout;
        }
        V acc[4];
        if (D != DSR_CTROP && S <= 4) {  // counting tropical: registers are tight
            V v[4][4];
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int s = 0; s < 4; s++)
                    if (ok[u] && s < S) v[u][s] = A::load(P, (i64)s * nd.nout + o[u]);
#pragma unroll
            for (int u = 0; u < 4; u++) {
                acc[u] = A::zero(j.ap);
#pragma unroll
                for (int s = 0; s < 4; s++)
                    if (ok[u] && s < S) acc[u] = A::add(acc[u], v[u][s], j.ap);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) acc[u] = ok[u] ? split_sum<D>(P, nd.nout, o[u], S, j.ap) : A::zero(j.ap);
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (ok[u]) {
                A::store(C, o[u], acc[u]);
                if constexpr (is_z<D>()) z_track(acc[u], lmax, lmin);
            }
    }
    if constexpr (is_z<D>()) z_meta_block(j.meta, nd.mc, lmax, lmin);
}

// one inner node, start to end, by this workgroup alone
template <int D>
__device__ void run_node_whole(const BJob& j, const BNode& nd, unsigned char* smem) {
    const int npl = plane_bytes_dev<D>(1) ? 2 : 1;
    bool any = false;
    for (int side = 0; side < 2; side++) {
        if (!nd.pp[side]) continue;
        for (int pl = 0; pl < npl; pl++) {
            const int rank = (D == DSR_TPOLY && pl == 1) ? nd.prank[side] + 3 : nd.prank[side];
            const int ntiles = 1 << (rank - (rank < kPermTileBits ? rank : kPermTileBits));
            run_perm<D>(j, nd, side, pl, 0, ntiles, smem);
        }
        any = true;
    }
    if (any) local_step_sync();
    const int nblocks = 1 << ((nd.g.lb - nd.g.tb) + (nd.g.li - nd.g.ti) + (nd.g.lj - nd.g.tj) + nd.g.lsplit);
    for (int k = 0; k < nblocks; k++) run_gemm<D>(j, nd, k, smem);
    local_step_sync();
    if (nd.g.lsplit > 0) {
        const i64 nred = nd.reduce_per_block ? nd.nout : (nd.nout + 255) / 256;
        run_reduce<D>(j, nd, 0, (int)nred, smem);
        local_step_sync();
    }
}

// One task of an algebra-D job.  Kept out of line, one function per algebra,
// with everything it runs inlined: registers are then allocated per algebra
// (each fits the two-waves-per-SIMD budget; only counting tropical spills a
// few) rather than over the union of all algebras in the task loop, and the call
// costs one register save per task.  (Inlining all algebras into the task
// loop spills heavily; calling a GEMM routine per tile saves registers to
// scratch on every tile.)
template <int D>
__attribute__((noinline)) __device__ void run_task(const BTask& t, const BJob& j, const BNode* nodes,
                                                   const int* subtree, unsigned char* smem) {
    switch (t.kind) {
    case BT_LEAVES: {
        // fresh partition-function bookkeeping for every node, then the leaves
        if (j.meta)
            for (int i = threadIdx.x; i < j.nnode; i += blockDim.x) meta_set(j.meta, i, 0, 0u);
        __syncthreads();
        for (int l = threadIdx.x; l < j.nleaf; l += blockDim.x) leaf_dispatch<D>(j.leaves[l], l, j.w, j.spos, 0ull, j.arena, j.ap, j.meta);
        break;
    }
    case BT_PERM: run_perm<D>(j, nodes[t.node], t.aux >> 1, t.aux & 1, t.tile, t.count, smem); break;
    case BT_GEMM:
        for (int k = 0; k < t.count; k++) run_gemm<D>(j, nodes[t.node], t.tile + k, smem);
        break;
    case BT_REDUCE: run_reduce<D>(j, nodes[t.node], t.tile, t.count, smem); break;
    case BT_SUBTREE:
        for (int k = 0; k < t.aux; k++) run_node_whole<D>(j, nodes[subtree[t.node + k]], smem);
        break;
    case BT_ACCUM: {
        if (threadIdx.x == 0) {
            // the root's tensor sits at the arena offset carried in the tile field
            Planes r;
            int64_t off = t.tile;
            r.p0 = (unsigned char*)j.arena.p0 + off * plane_bytes_dev<D>(0);
            r.p1 = plane_bytes_dev<D>(1) ? (unsigned char*)j.arena.p1 + off * plane_bytes_dev<D>(1) : nullptr;
            accumulate_one<D>(r, j.root, j.meta, j.acc, 1, j.ap);
        }
        if constexpr (is_z<D>()) z_range_block(j.meta, j.nnode, j.acc, 1, (float*)smem);
        break;
    }
    case BT_ONE: {
        if (threadIdx.x == 0) set_one<D>(j.acc, j.ap);
        break;
    }
    default: break;
    }
}

__device__ inline unsigned int hw_xcc_id() {
    unsigned int x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 0xfu;
}

// At least two waves per SIMD (registers capped at 256 per lane): the grid of
// two workgroups per CU is then resident at once.  WIDE selects the algebras
// one instance serves: the 4-byte ones (and counting tropical), or the
// wide-entry ones (eight-lists, truncated polynomials), so that the wide
// algebras' task routines do not enlarge the kernel the common algebras run
// in (that cost the 4-byte launches some 5%).
template <bool WIDE>
__global__ __launch_bounds__(256, 2) void batch_kernel(const BTask* __restrict__ tasks, const int* __restrict__ qbegin,
                                                    const int* __restrict__ qcount, int nq,
                                                    const BJob* __restrict__ jobs, const BNode* __restrict__ nodes,
                                                    const int* __restrict__ subtree, int* counters, int* tickets,
                                                    unsigned long long* trace, long long wait_limit) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_task;
    const int q = (int)(hw_xcc_id() % (unsigned)nq);
    const int qb = qbegin[q], qn = qcount[q];
    int* abort_flag = tickets + nq;  // set when a wait gave up: every workgroup leaves at its next wait
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(&tickets[q], 1);
        __syncthreads();
        // no second barrier: thread 0 writes s_task again only after the
        // task's last barrier, which every wave passes after reading it here
        const int tq = __builtin_amdgcn_readfirstlane(s_task);
        if (tq >= qn) break;  // every workgroup leaves once its queue's tickets run out
        const int ti = qb + tq;
        const unsigned long long t_start = trace ? wall_clock64() : 0ull;
        const BTask t = tasks[ti];
        if (!wait_counters(counters, t.dep0, t.need0, t.dep1, t.need1, abort_flag, wait_limit)) break;
        const unsigned long long t_ready = trace ? wall_clock64() : 0ull;
        const BJob& j = jobs[t.job];
        if constexpr (WIDE) {
            switch (j.dsr) {
            case DSR_TOPK: run_task<DSR_TOPK>(t, j, nodes, subtree, smem); break;
            case DSR_TPOLY: run_task<DSR_TPOLY>(t, j, nodes, subtree, smem); break;
            default: break;
            }
        } else {
            switch (j.dsr) {
            case DSR_TROP_I32: run_task<DSR_TROP_I32>(t, j, nodes, subtree, smem); break;
            case DSR_TROP_F32: run_task<DSR_TROP_F32>(t, j, nodes, subtree, smem); break;
            case DSR_CTROP: run_task<DSR_CTROP>(t, j, nodes, subtree, smem); break;
            case DSR_MODP: run_task<DSR_MODP>(t, j, nodes, subtree, smem); break;
            case DSR_Z_F32: run_task<DSR_Z_F32>(t, j, nodes, subtree, smem); break;
            case DSR_Z_BF16: run_task<DSR_Z_BF16>(t, j, nodes, subtree, smem); break;
            default: break;
            }
        }
        signal_counter(counters, t.signal);
        if (trace && threadIdx.x == 0) {
            trace[4 * (size_t)ti + 0] = t_start;
            trace[4 * (size_t)ti + 1] = t_ready;
            trace[4 * (size_t)ti + 2] = wall_clock64();
            trace[4 * (size_t)ti + 3] = hw_xcc_id();
        }
    }
}

hipError_t launch_batch(const BTask* tasks, const int* qbegin, const int* qcount, int nq, const BJob* jobs,
                        const BNode* nodes, const int* subtree, int* counters, int* tickets, int nworkgroups,
                        unsigned long long* trace, int wide, long long wait_limit, hipStream_t s) {
    if (nworkgroups <= 0) return hipSuccess;
    if (wide)
        batch_kernel<true><<<nworkgroups, 256, kBatchLds, s>>>(tasks, qbegin, qcount, nq, jobs, nodes, subtree,
                                                               counters, tickets, trace, wait_limit);
    else
        batch_kernel<false><<<nworkgroups, 256, kBatchLds, s>>>(tasks, qbegin, qcount, nq, jobs, nodes, subtree,
                                                                counters, tickets, trace, wait_limit);
    return hipGetLastError();
}

}  // namespace tn
