// Executor: device contexts, per-plan device programs, and single-network
// contraction on one HIP stream.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "kernels.h"
#include "plan.h"

struct tn_net {
    tn::Net net;
};

struct tn_plan {
    tn::Plan plan;
};

namespace tn {

// Host copy of the executor program of one plan for one device algebra.
struct NodeLaunch {
    GemmShape shape;
    int64_t part_entries = 0;  // split-K partial buffer entries (0 if none)
};

// Launch shapes of every node of a plan for one device algebra, with the
// split-K partial sizes they imply.
struct LaunchSet {
    std::vector<NodeLaunch> nodes;
    int64_t part_entries = 0;              // largest node's partials (one node at a time)
    std::vector<int64_t> part_off_dag;     // each split node's own partials (dependency-graph layout)
    int64_t part_entries_dag = 0;          // sum over split nodes
};

// Device-resident constant data of one plan: leaf descriptors, permute
// tables and slice positions.  Uploaded once per (context, plan).
struct DevProgram {  // device tables of one plan (in a buffer that ctx->prog_bufs owns)
    LeafDev* leaves = nullptr;
    PermTables* perms = nullptr;  // indexed by permute slot
    int nperms = 0;
    // the same permutes for 32-byte entries, as 4-byte permutes of rank + 3
    // whose three lowest bits stay in place: built and uploaded (own buffer)
    // the first time an algebra with such entries runs the plan
    PermTables* perms_wide = nullptr;
    void* wide_buf = nullptr;
    size_t wide_bytes = 0;
    int* slice_pos = nullptr;     // nv entries: position in the sliced list or -1
    std::vector<int> perm_slot_a, perm_slot_b;  // per inner node, -1 if none
    // launch shapes per (tuning-table generation, device algebra): a new
    // table makes new entries, so references handed out stay valid
    std::map<int64_t, LaunchSet> launch_sets;
};

struct PendingRec {
    hipEvent_t start, stop;
    tn_kernel_record rec;
};

}  // namespace tn

namespace tn {
struct BatchLaunch;
}

struct tn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tn_allocator alloc{};
    bool has_alloc = false;
    bool profiling = false;
    std::vector<tn::PendingRec> pending;
    std::vector<tn_kernel_record> records;
    std::vector<hipEvent_t> event_pool;
    void* pinned = nullptr;  // host staging (results, weights)
    size_t pinned_bytes = 0;
    std::map<uint64_t, tn::DevProgram> progs;  // keyed by plan uid
    std::vector<std::pair<void*, size_t>> prog_bufs;  // device buffers holding the programs
    int cu_count = 0;
    // grow-only device scratch reused by synchronous persistent launches
    void* batch_dev = nullptr;
    size_t batch_dev_cap = 0, batch_dev_used = 0, batch_dev_peak = 0;
    std::vector<std::pair<void*, size_t>> batch_overflow;
    // pinned staging buffers handed to persistent launches
    struct PinnedBuf {
        void* p;
        size_t bytes;
        bool busy;
    };
    std::vector<PinnedBuf> pinned_pool;
    std::mutex pinned_mu;
    std::vector<tn_task_record> task_trace;  // persistent-launch timelines (profiling)
    double wait_limit_s = 10.0;  // longest dependency wait of a persistent launch
    int wall_khz = 0;            // the device's constant wall-clock rate (cached)
    // the last synchronous persistent launch, kept for an identical next call
    tn::BatchLaunch* batch_cache = nullptr;
    std::vector<uint64_t> batch_cache_key;
};

namespace tn {

void* pinned_acquire(tn_ctx* ctx, size_t bytes);
void pinned_release(tn_ctx* ctx, void* p);
void* dev_alloc(tn_ctx* ctx, size_t bytes);
void dev_free(tn_ctx* ctx, void* p, size_t bytes);
tn_status ensure_pinned(tn_ctx* ctx, size_t bytes);
tn_status get_program(tn_ctx* ctx, const Plan& p, DevProgram*& out);
// Programs of every plan in the list not yet on the device, with one upload.
tn_status get_programs(tn_ctx* ctx, const std::vector<const Plan*>& plans);
// The widened permute tables of a program (no-op once built).
tn_status ensure_wide_perms(tn_ctx* ctx, const Plan& p, DevProgram& dp);
// Launch shapes of every node for one device algebra under the current
// tuning table (cached in dp; the reference stays valid while dp lives).
const LaunchSet& node_launches(DevProgram& dp, const Plan& p, int dsr, bool chiplet);
// Tuning table (tune.cpp): generation (bumped by every change), tuning of a
// plan's nodes, table file I/O.
uint64_t tune_generation();
tn_status tune_plan(tn_ctx* ctx, const Plan& plan, const std::vector<int>& dsrs, double min_log2_ops, int reps,
                    int32_t* ntuned);
tn_status tune_save(const char* path, int32_t* nentries);
tn_status tune_load(const char* path, int32_t* nentries);
void tune_clear();
int32_t tune_records(tn_tune_record* recs, int32_t cap);
tn_status tune_env_load();

// Profiling bracket around one launch (no-op unless profiling is on).
struct ProfScope {
    tn_ctx* ctx;
    PendingRec pr;
    bool on;
    ProfScope(tn_ctx* c, int kind, int node, int sr, const int shape[4], double bytes, double ops,
              const char* kernel = "", bool enable = true);
    ~ProfScope();
};

// Device-memory layout of one solve (bytes from the base of its buffer).
struct SolveLayout {
    size_t o_a0 = 0, o_a1 = 0, o_p0 = 0, o_p1 = 0, o_meta = 0, o_w = 0, o_acc = 0, need = 0, acc_bytes = 0;
    int64_t nent = 1;  // root entries per pass
    int pb0 = 0, pb1 = 0;
};
struct PassSpec;

// tensor: for plans with open vertices, receives the 2^nopen results (entry
// bits = open vertices in the plan's order); res then holds entry 0.
// raw: receives the first pass's accumulator slot (kAccSlotBytes).
tn_status solve_one(tn_ctx* ctx, const Net& net, const Plan& plan, const tn_solve_opts& o, tn_result& res,
                    std::vector<tn_result>* tensor = nullptr, std::vector<unsigned char>* raw = nullptr);

// Device algebras needed for a user algebra, and the lane primes.
struct PassSpec {
    int dsr;
    uint32_t prime;
    uint32_t xval = 1;  // mod p: value of x in the vertex tensors [1, x] (1: counting)
};
// Internal semiring codes (not part of tn_semiring), raw accumulator results:
// the eight largest values (SizeMax(k), k <= 8) and the truncated polynomial
// of the four highest orders (CountingMax(k), k <= 4; per-node executor).
constexpr int kSemiringTop8 = 100;
// residue primes of an exact count (CRT primes plus one check prime)
constexpr int kMaxPrimes = 16;
constexpr int kSemiringTPoly4 = 101;
tn_status make_passes(const Net& net, const tn_solve_opts& o, std::vector<PassSpec>& passes);
AlgebraParams algebra_params(int dsr, uint32_t prime, double beta, uint32_t xval = 1);
// Decode the accumulators of all passes into the result struct.
// out = a (+) b for results of disjoint slice ranges (tn_result_combine).
tn_status combine_results(const tn_result& a, const tn_result& b, tn_result& out);
tn_status decode_result(const tn_solve_opts& o, const std::vector<PassSpec>& passes,
                        const std::vector<std::vector<unsigned char>>& acc, tn_result& res);

// The pieces of solve_one, for callers that bring their own device memory.
// check_solve: plan/network match and the slice range [sb, se).
tn_status check_solve(const Net& net, const Plan& plan, const tn_solve_opts& o, int64_t& sb, int64_t& se);
SolveLayout solve_layout(const Net& net, const Plan& plan, const std::vector<PassSpec>& passes, DevProgram* dp,
                         bool tensor_root);
tn_status run_solve(tn_ctx* ctx, const Net& net, const Plan& plan, const tn_solve_opts& o,
                    const std::vector<PassSpec>& passes, DevProgram* dp, unsigned char* base, const SolveLayout& L,
                    int64_t sb, int64_t se, void* stage, std::vector<unsigned char>& all);
// run_solve on stream s; async: nothing waits (the weights go up from and
// the accumulators come back into stage, in stream order), and the caller
// reads the accumulators from stage once the stream has passed; launches
// are not profiled.  all may be NULL when async.
tn_status run_solve_on(tn_ctx* ctx, hipStream_t s, bool async, const Net& net, const Plan& plan,
                       const tn_solve_opts& o, const std::vector<PassSpec>& passes, DevProgram* dp,
                       unsigned char* base, const SolveLayout& L, int64_t sb, int64_t se, void* stage,
                       std::vector<unsigned char>* all);
tn_status decode_root(const tn_solve_opts& o, const std::vector<PassSpec>& passes, const std::vector<unsigned char>& all,
                      int64_t nent, int64_t addr, tn_result& r);
// Bytes of device memory the program of a plan takes (leaves, slice
// positions, compact and expanded permute tables).
size_t program_bytes(const Plan& p);
// Write the program of a plan into dev (at least program_bytes(p) bytes, 256-
// byte aligned) with copies from pageable host memory on the context stream
// and expand its permute tables there; dp receives pointers into dev.  Waits
// for the copies.  No allocation of device or pinned memory.
tn_status program_into(tn_ctx* ctx, const Plan& p, unsigned char* dev, DevProgram& dp);

// Scratch-free solve (noalloc.hip): the fixed device array is looked up once
// per device at context creation; solve_noalloc runs tn_solve's per-node
// contraction entirely inside it.
void noalloc_init_device(int device);
size_t noalloc_scratch_bytes();
tn_status solve_noalloc(tn_ctx* ctx, const Net& net, const Plan& plan, const tn_solve_opts& o, tn_result& res);

}  // namespace tn
