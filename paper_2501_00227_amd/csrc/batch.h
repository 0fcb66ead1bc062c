// Persistent batched executor: many contraction passes (of one or many
// networks) as one task table executed by a single persistent launch.
//
// Tasks are (job, node, tile) units: leaf initialisation, one permute tile,
// one GEMM tile, one split-K reduction unit, root accumulation.  Each task
// waits on at most two completion counters and bumps one.  Every job is
// assigned to one XCC (chiplet) queue; workgroups take tasks of their XCC's
// queue in ticket order; a queue is sorted by dependency level, so every task
// a workgroup waits on holds a smaller ticket of the same queue and is
// already running or done: the launch cannot deadlock, and every workgroup
// leaves the loop once its queue's tickets run out.
#pragma once

#include <cstdint>

#include "kernels.h"

namespace tn {

enum BatchTaskKind { BT_LEAVES = 0, BT_PERM = 1, BT_GEMM = 2, BT_REDUCE = 3, BT_ACCUM = 4, BT_ONE = 5, BT_SUBTREE = 6 };

struct BJob {  // one contraction pass of one network
    int dsr;
    int nleaf;
    int nnode;
    int root;  // node id of the root
    AlgebraParams ap;
    Planes arena, part;
    TensorMeta* meta;
    void* acc;
    const LeafDev* leaves;
    const float* w;
    const int* spos;
};

struct BNode {  // one inner node; jobs of the same plan and algebra share it (offsets are job-relative)
    GemmShape g;
    int64_t a_off, b_off, c_off;  // effective operand offsets (after permutes)
    int ma, mb, mc;
    const PermTables* pp[2];
    // the truncated-polynomial algebra's 32-byte count plane: the same permute
    // over 4-byte words (rank + 3, three lowest bits in place); else null
    const PermTables* pp1[2];
    int64_t psrc[2], pdst[2];
    int prank[2], ptile_bits[2];
    int64_t part_off;     // this node's split-K partials inside the job's partial buffer
    int64_t nout;         // 2^(lb+li+lj)
    int reduce_per_block; // split reduction: one workgroup per output
};

struct BTask {
    // the dependencies first: one aligned 16-byte load on the device
    int dep0, need0;  // wait until counters[dep0] >= need0 (dep0 < 0: none)
    int dep1, need1;
    int kind;
    int job;
    int node;    // index into the BNode table (GEMM/PERM/REDUCE); SUBTREE: offset in the subtree list
    int aux;     // PERM: side*2 + plane; SUBTREE: number of nodes
    int64_t tile;  // first tile (GEMM/PERM) or reduction unit; ACCUM: root arena offset
    int signal;  // counter to bump when done (-1: none)
    int count;   // tiles / units this task runs, from `tile` on
};
static_assert(sizeof(BTask) == 48, "three 16-byte loads per task");

// Tasks are grouped into one queue per XCC (chiplet): queue q holds tasks
// [qbegin[q], qbegin[q] + qcount[q]) in level order, served by the
// workgroups running on XCC q (hardware id modulo nq) with ticket tickets[q].
// trace: NULL, or 4 x ntasks timestamps (start, ready, end, xcc) per task.
// wide: the launch's jobs use the wide-entry algebras (eight-lists,
// truncated polynomials; a launch holds either these or the others only).
// tickets has nq + 1 entries: one per queue, then the abort flag a wait sets
// when it exceeds wait_limit ticks of the constant wall clock.
hipError_t launch_batch(const BTask* tasks, const int* qbegin, const int* qcount, int nq, const BJob* jobs,
                        const BNode* nodes, const int* subtree, int* counters, int* tickets, int nworkgroups,
                        unsigned long long* trace, int wide, long long wait_limit, hipStream_t s);
size_t batch_lds_bytes();

}  // namespace tn
