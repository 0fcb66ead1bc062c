// Scratch-free solve: the contraction of tn_solve on per-node launches, with
// every device buffer it needs -- the plan's program tables, the arena of
// live intermediates, split-K partials, partition-function bookkeeping,
// weights and root accumulators -- inside one fixed device array of this
// file, so that a call allocates no device or pinned host memory.
#include <algorithm>
#include <mutex>
#include <string>

#include "exec.h"

namespace tn {

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Look up this device's copy of the array (once per device, with the device
// current).  A failure is kept and reported by the entry point.
void noalloc_init_device(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> g(g_mu);
    if (g_done[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? (unsigned char*)p : nullptr;
    g_done[device] = true;
}

tn_status solve_noalloc(tn_ctx* ctx, const Net& net, const Plan& plan, const tn_solve_opts& o, tn_result& res) {
    const int dev = ctx->device;
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (dev < 0 || dev >= kMaxDevices || !g_done[dev]) return fail(TN_EDEVICE, "scratch not set up for this device");
        if (g_err[dev] != hipSuccess)
            return fail(TN_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                        hipGetErrorString(g_err[dev]));
        base = g_ptr[dev];
    }
    int64_t sb = 0, se = 0;
    tn_status st = check_solve(net, plan, o, sb, se);
    if (st != TN_OK) return st;
    if (!plan.open.empty()) return fail(TN_EINVAL, "plans with open vertices are solved by tn_solve_open");
    std::vector<PassSpec> passes;
    st = make_passes(net, o, passes);
    if (st != TN_OK) return st;
    // scratch: [program tables | solve buffer]
    const size_t prog = align256(program_bytes(plan));
    DevProgram dp;
    DevProgram* dpp = plan.nleaf() > 0 ? &dp : nullptr;
    SolveLayout L = solve_layout(net, plan, passes, dpp, false);
    if (prog + L.need > kScratchBytes)
        return fail(TN_ETOOBIG, "the solve needs " + std::to_string(prog + L.need) + " bytes of device memory, above the " +
                                    std::to_string(kScratchBytes) + "-byte scratch of the scratch-free entry point");
    if (dpp) {
        st = program_into(ctx, plan, base, dp);
        if (st != TN_OK) return st;
        for (auto& ps : passes) node_launches(dp, plan, ps.dsr, false);
    }
    std::vector<unsigned char> stage(std::max<size_t>(L.acc_bytes, sizeof(float) * net.wdev.size()) + 64);
    std::vector<unsigned char> all;
    const bool prof = ctx->profiling;  // profiling records create events: off for this call
    ctx->profiling = false;
    st = run_solve(ctx, net, plan, o, passes, dpp, base + prog, L, sb, se, stage.data(), all);
    ctx->profiling = prof;
    if (st != TN_OK) return st;
    return decode_root(o, passes, all, L.nent, 0, res);
}

}  // namespace tn
