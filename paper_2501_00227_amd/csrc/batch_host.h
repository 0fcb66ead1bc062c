// Host interface of the persistent batched executor (batch.cpp), used by
// tn_solve (small trees), tn_solve_batch and the server.
#pragma once

#include <array>
#include <functional>
#include <vector>

#include "batch.h"
#include "exec.h"

namespace tn {

struct BatchItem {
    const Net* net;
    const Plan* plan;
    tn_solve_opts opts;
    // explicit passes (their roots are returned raw, not decoded); null: the
    // passes of opts.semiring
    const std::vector<PassSpec>* passes = nullptr;
};

struct ItemState {
    tn_solve_opts opts{};
    std::vector<PassSpec> passes;
    std::vector<int> job_ids;  // one job per pass
    tn_status status = TN_OK;
    bool raw = false;          // explicit passes: no decoding
};

struct DevAllocFn {
    std::function<void*(size_t)> alloc;
    std::function<void(void*, size_t)> free;
};

// Everything one persistent launch owns until it is finished and released.
struct BatchLaunch {
    std::vector<ItemState> items;
    int njobs = 0, ntasks = 0;
    int wide = 0;  // the jobs use the wide-entry algebras (a separate kernel instance)
    void* data = nullptr;    // arenas, partials, meta, accumulators, weights
    size_t data_bytes = 0;
    void* tables = nullptr;  // jobs, nodes, tasks, counters
    size_t table_bytes = 0;
    void* host = nullptr;    // pinned staging: tables, weights, returned accumulators
    size_t host_bytes = 0, o_wstage = 0, wbytes = 0, o_hacc = 0;
    BJob* d_jobs = nullptr;
    BNode* d_nodes = nullptr;
    BTask* d_tasks = nullptr;
    int* d_counters = nullptr;
    int* d_ticket = nullptr;  // one ticket per XCC queue
    int* d_qbegin = nullptr;
    int* d_qcount = nullptr;
    int* d_subtree = nullptr;  // BNode indices of the fused small subtrees
    std::vector<int> subtree_list;
    int nq = 1;
    std::vector<int> qbegin, qcount;
    size_t o_hticket = 0;
    void* d_accs = nullptr;   // the jobs' root accumulator slots, kAccSlotBytes each
    size_t o_reset = 0, reset_bytes = 0;  // counters and tickets within the tables
    bool uploaded = false;    // tables and weights are on the device
    std::vector<void*> job_arena0;  // plane 0 of every job's arena (dependency-graph layout)
    double total_ops = 0, total_bytes = 0;  // algorithmic work of the launch
    unsigned long long* d_trace = nullptr;  // per-task timestamps (profiling)
    std::vector<BTask> host_tasks;          // kept for the trace
    std::function<void(void*, size_t)> free_fn;
    tn_ctx* ctx = nullptr;  // owner of the pinned staging buffer
};

int device_cu_count(tn_ctx* ctx);
long long wait_limit_ticks(tn_ctx* ctx);
// Build and upload nothing yet: lay out memory, allocate, fill the staging.
tn_status batch_prepare(tn_ctx* ctx, std::vector<BatchItem>& items, BatchLaunch& L, const DevAllocFn& alloc);
// Enqueue upload, the persistent kernel and the root read-back on stream s.
tn_status batch_launch(tn_ctx* ctx, BatchLaunch& L, hipStream_t s);
// After the stream has passed the launch: decode every item's result.
tn_status batch_finish(BatchLaunch& L, std::vector<tn_result>& out);
void batch_release(BatchLaunch& L);
void collect_trace(tn_ctx* ctx, BatchLaunch& L);
tn_status solve_batch_sync(tn_ctx* ctx, std::vector<BatchItem>& items, std::vector<tn_result>& out);
// One synchronous persistent launch of explicit passes of one unsliced
// network; accs receives the root accumulator slot of every pass, in order.
tn_status run_passes_sync(tn_ctx* ctx, const Net& net, const Plan& plan, const std::vector<PassSpec>& passes,
                          std::vector<std::array<unsigned char, kAccSlotBytes>>& accs);
// As run_passes_sync, but the launch stays alive (its arenas hold every
// tensor of the contraction) until batch_done.
tn_status run_passes_keep(tn_ctx* ctx, const Net& net, const Plan& plan, const std::vector<PassSpec>& passes,
                          std::vector<std::array<unsigned char, kAccSlotBytes>>& accs, BatchLaunch& L);
void batch_done(tn_ctx* ctx, BatchLaunch& L);
// One maximum configuration (SingleConfigMax): config[v] in {0, 1}.
tn_status single_config_max(tn_ctx* ctx, const Net& net, const Plan& plan, int32_t* config, float* value);
// Independence polynomial (finite-field method); coeffs: (nv + 1) * limbs.
tn_status solve_polynomial(tn_ctx* ctx, const Net& net, const Plan& plan, int limbs, uint32_t* coeffs, int* degree);
// Release the launch a synchronous batch keeps for an identical next call.
void batch_cache_drop(tn_ctx* ctx);
// Route a single unsliced small tree through the persistent launch.
bool use_persistent(const Plan& p);
// The route of a job launched together with others (tn_solve_batch, the
// server): use_persistent, or a mid-size tree in an exact algebra.
bool use_persistent_shared(const Plan& p, int semiring);

}  // namespace tn
