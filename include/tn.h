/*
 * tn.h -- C ABI of the MI355X (gfx950) generic tensor-network library.
 *
 * The library solves the independent-set problem by contracting its tensor
 * network over a semiring, following "Programming guide for solving
 * constraint satisfaction problems with tensor networks" (arXiv 2501.00227):
 *
 *   graph + weights  --tn_net_independent_set-->  network      (Sec. 3.2)
 *   network          --tn_plan_create-->          contraction tree, slicing
 *                                                 (Sec. 4.1 complexity, Sec. 4.2 optimizers)
 *   network + plan   --tn_solve-->                solution-space property
 *                                                 (Sec. 5.1 solve, Sec. 5 property table)
 *
 * plus a batched form (many networks in one persistent launch) and a server
 * form (continuous batching with HBM-budget admission).
 *
 * Conventions for every call:
 *   - Every function that can fail returns tn_status; nothing aborts and no
 *     C++ exception crosses this boundary.  tn_last_error() returns a
 *     thread-local text for the last failure on the calling thread.
 *   - Vertex ids are 0-based (the paper's Julia ids are 1-based).
 *   - Input arrays are owned by the caller and copied during the call.
 *     Handles (tn_ctx, tn_net, tn_plan, tn_server) are owned by the library
 *     until the matching *_destroy.  Results are plain structs written into
 *     caller memory.
 *   - A tn_ctx is used by one thread at a time; tn_server_* calls are
 *     thread-safe.
 *   - Device memory comes from the context's allocator callbacks (for
 *     example PyTorch's caching allocator), or from hipMallocAsync on the
 *     context stream when no allocator is given.
 */
#ifndef TN_H_
#define TN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TN_OK = 0,
    TN_EINVAL = -1,     /* invalid argument (bad graph, options, handle) */
    TN_ENOMEM = -2,     /* host or device allocation failed */
    TN_EDEVICE = -3,    /* a HIP runtime call failed */
    TN_EOVERFLOW = -4,  /* exact count exceeds the CRT range (check residue disagrees) */
    TN_ETOOBIG = -5,    /* plan needs more device memory than allowed */
    TN_EBUSY = -6,      /* server queue full */
    TN_ECANCELED = -7   /* job cancelled or server shut down before it ran */
} tn_status;

/* Element algebra of the contraction (Sec. 5 property table).
 *   TN_TROPICAL_I32      SizeMax     max-plus over int32, -inf = INT32_MIN with
 *                                    saturating add; integer weights only
 *                                    (|w| <= 65536 and sum |w| <= 2^28)
 *   TN_TROPICAL_F32      SizeMax     max-plus over float32, -inf = -INFINITY
 *   TN_COUNTING_TROPICAL CountingMax (int32 size, uint64 count): larger size wins,
 *                                    equal sizes add counts; the count is exact
 *                                    modulo 2^64; integer weights only
 *   TN_COUNT_EXACT       CountingAll: counts modulo primes below 2^30 (one
 *                                    contraction per prime), recombined by CRT
 *                                    into an exact integer and checked modulo
 *                                    one more prime (Z(beta=0) of Sec. 3.1)
 *   TN_PARTITION_F32     PartitionFunction(beta): float32 values, one power-of-two
 *                                    exponent per intermediate tensor
 *   TN_PARTITION_BF16    as above with bfloat16-rounded GEMM inputs, float32
 *                                    accumulation (error reported, not bounded) */
typedef enum {
    TN_TROPICAL_I32 = 0,
    TN_TROPICAL_F32 = 1,
    TN_COUNTING_TROPICAL = 2,
    TN_COUNT_EXACT = 3,
    TN_PARTITION_F32 = 4,
    TN_PARTITION_BF16 = 5
} tn_semiring;

typedef struct tn_ctx tn_ctx;
typedef struct tn_net tn_net;
typedef struct tn_plan tn_plan;
typedef struct tn_server tn_server;

/* Device allocator callbacks.  alloc returns a device pointer (256-byte
 * aligned) or NULL; both are called on the thread that calls the library,
 * with the context stream. */
typedef void* (*tn_alloc_fn)(size_t bytes, void* user, void* stream);
typedef void (*tn_free_fn)(void* ptr, size_t bytes, void* user, void* stream);
typedef struct {
    tn_alloc_fn alloc;
    tn_free_fn free;
    void* user;
} tn_allocator;

/* ------------------------------------------------------------- context --- */

/* Create a context on HIP device `device`.  stream: a hipStream_t to run on
 * (NULL: the context creates its own default-priority stream).  alloc: NULL
 * uses hipMallocAsync/hipFreeAsync on that stream.  Errors: TN_EINVAL for a
 * bad device, TN_EDEVICE if HIP fails. */
tn_status tn_ctx_create(int device, void* stream, const tn_allocator* alloc, tn_ctx** out);
void tn_ctx_destroy(tn_ctx* ctx);
const char* tn_last_error(void);

/* Per-launch profiling.  When enabled, every kernel the context launches is
 * bracketed by HIP events recorded on the stream it runs on; records hold the
 * kernel kind, the tree node, the measured duration and the algorithmic work
 * of that launch (bytes of operands read + result written, and semiring ops
 * = product of the node's index dimensions, Sec. 4.1 tc/rwc).  Records are
 * kept until read or cleared. */
typedef enum {
    TN_K_LEAF = 0,      /* leaf tensor initialisation */
    TN_K_PERMUTE = 1,   /* operand transpose into GEMM layout */
    TN_K_GEMM = 2,      /* batched semiring GEMM (VALU) */
    TN_K_GEMM_MFMA = 3, /* batched GEMM on matrix cores (partition function) */
    TN_K_ACCUM = 4,     /* slice accumulation / root handling */
    TN_K_BATCH = 5,     /* persistent batched launch */
    TN_K_GEMM_BIG = 6,  /* batched semiring GEMM, register-tiled VALU kernels (large M, N) */
    TN_K_GEMM_THIN = 7, /* batched semiring GEMM, row streaming for N * K <= 32 */
    TN_K_GEMM_DOT = 8   /* batched semiring GEMM with M = N = 1: long-K reduction */
} tn_kernel_kind;

typedef struct {
    int32_t kind;       /* tn_kernel_kind */
    int32_t node;       /* inner-node index, -1 if none */
    int32_t semiring;   /* tn_semiring */
    int32_t shape[4];   /* GEMM: log2 batch, M, N, K; permute: rank, 0, 0, 0 */
    float ms;           /* measured duration */
    double alg_bytes;   /* algorithmic bytes of the launch */
    double ops;         /* semiring ops of the launch (GEMM) */
    char kernel[64];    /* the kernel (template instance) launched, as profilers name it,
                           e.g. "gemm_ct_big_kernel<7, 6>" */
} tn_kernel_record;

tn_status tn_ctx_set_profiling(tn_ctx* ctx, int enabled);
/* Copy up to cap records; *n receives the number available.  Synchronises the
 * context stream.  clear != 0 drops the records afterwards. */
tn_status tn_ctx_profile(tn_ctx* ctx, tn_kernel_record* recs, int32_t cap, int32_t* n, int clear);
tn_status tn_ctx_synchronize(tn_ctx* ctx);

/* Per-task timeline of the persistent launches run while profiling was on:
 * for each task its kind (0 leaves, 1 permute tile, 2 GEMM tile, 3 split
 * reduction, 4 root accumulation), job, tree node, the hardware XCC (chiplet)
 * that ran it, and its start (ticket taken), ready (dependencies met) and end
 * times in microseconds since the launch's first ticket.  Copies up to cap
 * records; *n receives the number available.  clear != 0 drops them. */
typedef struct {
    int32_t kind, job, node, xcc;
    float t_start, t_ready, t_end;
} tn_task_record;
tn_status tn_ctx_task_trace(tn_ctx* ctx, tn_task_record* recs, int32_t cap, int32_t* n, int clear);

/* Longest dependency wait of a persistent launch (tn_solve_batch, the
 * persistent executor of tn_solve, the server, and the passes of the
 * polynomial / max-k / configuration calls), default 10 s.  A workgroup whose
 * wait for an input exceeds it sets the launch's abort flag; every workgroup
 * then leaves the launch, the kernel ends, and the call returns TN_EDEVICE
 * for every job of that launch.  Errors: TN_EINVAL (seconds not positive). */
tn_status tn_ctx_set_wait_limit(tn_ctx* ctx, double seconds);

/* ------------------------------------------------------------- network --- */

/* Independent-set network of a graph (Sec. 3.2): one index per vertex, an
 * edge tensor B = [[1,1],[1,0]] per edge and a vertex tensor W = [1, x^w_v]
 * per vertex, where 1 and 0 are the multiplicative and additive identities of
 * the chosen algebra and x^w is w (tropical) or e^{beta w} (real).
 *   nv      number of vertices (>= 0)
 *   ne      number of edges (>= 0); edges: 2*ne vertex ids, pair e = (u, v)
 *   weights nv floats, or NULL for unit weights
 * Duplicate edges are merged (edge ids follow the first occurrence).  Errors: TN_EINVAL for self-loops, ids out of
 * range, non-finite weights, nv > 4096. */
tn_status tn_net_independent_set(int32_t nv, int32_t ne, const int32_t* edges,
                                 const float* weights, tn_net** out);

/* Spin-glass network of a graph (Sec. 2: H(s) = sum_(u,v) J_uv s_u s_v +
 * sum_v h_v s_v, s_v in {-1, 1}; index value n_v = (s_v + 1) / 2): an edge
 * tensor x^(-J_uv s_u s_v) per edge and a vertex tensor x^(-h_v s_v) per
 * vertex.  Every algebra then solves for -H: the tropical ones give
 * max(-H) = -(ground-state energy), counting tropical also the ground-state
 * degeneracy (CountingMin of the Sec. 6.4 buckyball example), the real one
 * Z(beta) = sum_s e^(-beta H), exact counting 2^nv.
 *   J  ne floats in edge order (NULL: all 1, antiferromagnetic unit
 *      coupling); duplicate edges add their couplings
 *   h  nv floats (NULL: all 0)
 * Tropical int32 and counting tropical need integer J and h.  The
 * independence polynomial is not defined for it (TN_EINVAL).  Errors as
 * tn_net_independent_set, plus non-finite J or h. */
tn_status tn_net_spin_glass(int32_t nv, int32_t ne, const int32_t* edges, const float* J, const float* h,
                            tn_net** out);
void tn_net_destroy(tn_net* net);
/* Sizes after de-duplication. */
tn_status tn_net_info(const tn_net* net, int32_t* nv, int32_t* ne);

/* A conditioned copy of a network (the fixed vertices of the Sec. 5 network
 * object): vertices[k] is fixed to values[k] (0 = not in the set / spin
 * down, 1 = in the set / spin up), on top of any fixings src already has.
 * Every leaf tensor that holds a fixed vertex is multiplied by the indicator
 * of its value, so every property (sizes, counts, Z, polynomial, maximum
 * configuration) becomes the property of the configurations that agree with
 * the fixings.  The copy has src's structure: plans of src fit it.  Errors:
 * TN_EINVAL (vertex out of range, value not 0/1, a vertex fixed to both
 * values, NULL arguments).  Release with tn_net_destroy. */
tn_status tn_net_condition(const tn_net* src, int32_t n, const int32_t* vertices, const int32_t* values,
                           tn_net** out);

/* ---------------------------------------------------------------- plan --- */

/* Options of the contraction-order optimizers (Sec. 4.2).
 *   method 0 GreedyMethod: cost size(Ti*Tj) - alpha (size(Ti) + size(Tj));
 *            temperature > 0 samples pairs by e^{-cost/T} (hyper-greedy);
 *            best of nrepeat runs.
 *   method 1 TreeSA: greedy start, then simulated annealing over the four
 *            tree rotations with cost tc + sc_weight * max(0, sc - sc_target)
 *            + rw_weight * rwc (all log2), Metropolis acceptance, inverse
 *            temperatures beta_start:beta_step:beta_stop, niters sweeps per
 *            temperature, best of ntrials (trials run on host threads).
 *   method 2 automatic: the greedy tree; when it needs more than 2^26
 *            semiring ops, TreeSA with the same options as well, and the
 *            tree of lower TreeSA cost is kept (cheap planning for small
 *            networks, annealed trees for the large ones).
 *   nslices  upper bound on sliced indices; indices are sliced (Sec. 4.2)
 *            while sc > sc_target.  0 = never slice.
 *   absorb_vertices  fold each vertex tensor into one incident edge tensor
 *            (same result, fewer leaves).
 *   open     open vertices (the open vertices of the Sec. 5 network object):
 *            never summed, so the root is a tensor over them (at most 16);
 *            they are never sliced.  Such a plan is solved by tn_solve_open
 *            only. */
typedef struct {
    int32_t method;
    double alpha;
    double temperature;
    int32_t nrepeat;
    uint64_t seed;
    double sc_target;
    double sc_weight;
    double rw_weight;
    double beta_start;
    double beta_step;
    double beta_stop;
    int32_t ntrials;
    int32_t niters;
    int32_t nslices;
    int32_t absorb_vertices;
    int32_t nthreads; /* host threads for TreeSA trials; 0 = hardware count */
    int32_t nopen;       /* open vertices: indices the contraction keeps to the root */
    const int32_t* open; /* nopen distinct vertex ids (copied); see tn_solve_open */
} tn_plan_opts;

/* Defaults: greedy alpha 0, T 0, nrepeat 10 (Sec. 4.2.1); TreeSA sc_target 20,
 * betas 0.01:0.05:15, ntrials 10, niters 50, sc_weight 1, rw_weight 0.2
 * (Sec. 4.2.2); no slicing; vertices absorbed. */
void tn_plan_opts_default(tn_plan_opts* opts);

tn_status tn_plan_create(const tn_net* net, const tn_plan_opts* opts, tn_plan** out);

/* A plan from an explicit binary tree (e.g. the tree printed in Sec. 4.1).
 * Leaves 0..nleaf-1 hold the factors fac[fac_off[l] .. fac_off[l+1]) where a
 * code c >= 0 is edge c and c < 0 is the vertex tensor of vertex -c-1; every
 * factor appears exactly once.  Inner node t (id nleaf+t) has children
 * left[t], right[t] with smaller ids; the last node is the root.  Output
 * indices follow the einsum rule (an index stays open while it occurs outside
 * the subtree).  sliced: nsliced vertex ids fixed per slice.  TN_EINVAL if the
 * tree is not a valid binary tree over all factors. */
tn_status tn_plan_from_tree(const tn_net* net, int32_t nleaf, const int32_t* fac_off,
                            const int32_t* fac, int32_t ninner, const int32_t* left,
                            const int32_t* right, int32_t nsliced, const int32_t* sliced,
                            tn_plan** out);

/* Contraction complexity of the plan (Sec. 4.1): tc = log2 of the total
 * number of semiring operations (product of all index dimensions at each
 * binary contraction, times 2^nsliced), sc = log2 of the largest intermediate
 * (entries, per slice), rwc = log2 of the total entries read and written. */
tn_status tn_plan_complexity(const tn_plan* plan, double* tc_log2, double* sc_log2,
                             double* rwc_log2);

typedef struct {
    int32_t nleaf;
    int32_t ninner;
    int32_t nsliced;
    int32_t max_rank;        /* sc as an integer */
    double tc_log2, sc_log2, rwc_log2;
    uint64_t arena_entries;  /* live-entry peak of the memory plan, per slice */
    int32_t npermutes;       /* operand permutes the executor will run per slice */
} tn_plan_info_t;
tn_status tn_plan_info(const tn_plan* plan, tn_plan_info_t* info);

/* Device bytes one tn_solve of this plan needs in the given algebra (arena of
 * live intermediates, permute scratch, leaves and bookkeeping). */
tn_status tn_plan_peak_bytes(const tn_plan* plan, tn_semiring semiring, uint64_t* bytes);

/* The GEMM launch shape of every inner node for one semiring (introspection:
 * which kernel family and tile each contraction step of Sec. 4.1 runs on).
 * One row of TN_SHAPE_ROW int32 per (device algebra, inner node), inner nodes
 * in execution order; one device algebra per semiring.  Row: algebra index, node id, log2 batch / M /
 * N / K, A and B transposition flags, log2 tile batch / M / N / K step, micro
 * tile rows / columns, log2 K splits, kernel kind (tn_kernel_kind), 1 if the
 * shape is one the kernels accept, 0.  Writes at most cap rows (rows may be
 * NULL with cap 0); *nrows receives the full count. */
#define TN_SHAPE_ROW 18
tn_status tn_plan_gemm_shapes(const tn_plan* plan, tn_semiring semiring, int32_t cap, int32_t* rows,
                              int32_t* nrows);

/* Export the tree in the format of tn_plan_from_tree, plus the ordered output
 * indices of every node (leaves first).  Call with NULL arrays to get the
 * sizes: *nfac, *nidx.  idx_off has nleaf+ninner+1 entries. */
tn_status tn_plan_export(const tn_plan* plan, int32_t* nleaf, int32_t* ninner, int32_t* nfac,
                         int32_t* nidx, int32_t* nsliced, int32_t* fac_off, int32_t* fac,
                         int32_t* left, int32_t* right, int32_t* idx_off, int32_t* idx,
                         int32_t* sliced);
void tn_plan_destroy(tn_plan* plan);

/* Complexity of the unordered (flat) einsum of a network: one node over all
 * indices (Sec. 4.1, the EinCode before optimize_code). */
tn_status tn_net_flat_complexity(const tn_net* net, double* tc_log2, double* sc_log2,
                                 double* rwc_log2);

/* --------------------------------------------------------------- solve --- */

typedef struct {
    int32_t semiring;          /* tn_semiring */
    double beta;               /* inverse temperature for TN_PARTITION_* (x = e^beta) */
    int32_t nprimes;           /* TN_COUNT_EXACT: residue primes incl. one check prime,
                                  2..16 (0 = default: enough CRT primes for an
                                  upper bound on the count, at least two, plus
                                  one check; at most 15 CRT primes, range 2^449;
                                  counts above 2^512 are TN_EOVERFLOW) */
    const uint32_t* primes;    /* NULL = default primes (largest primes below 2^30) */
    int64_t slice_begin;       /* run slices [slice_begin, slice_end) only; slice s */
    int64_t slice_end;         /* fixes sliced index k to bit k of s; 0,0 = all */
    int32_t executor;          /* 0 auto: one persistent launch for unsliced trees with
                                  sc <= 22 and at most 2^27 semiring ops per pass
                                  (a persistent launch keeps a job on one chiplet),
                                  per-node stream launches otherwise;
                                  1 per-node stream launches; 2 persistent launch
                                  (unsliced plans only) */
} tn_solve_opts;

void tn_solve_opts_default(tn_solve_opts* opts);

/* Result of one contraction (a 0-dimensional tensor, Sec. 5.1).
 *   Tropical:  size_i32 / size_f32; size_is_neg_inf when no configuration
 *              exists (cannot happen for independent sets, kept for slices).
 *   Counting tropical: size_i32 and count_mod_2_64.
 *   Exact count: count_mod_2_64, residues[] (one per prime), count_limbs
 *              (little-endian 32-bit limbs of the exact integer from CRT,
 *              count_nlimbs of them); TN_EOVERFLOW if the check prime
 *              disagrees with the CRT value.
 *   Partition function: Z = z_mant * 2^z_exp2 (z_mant in [1,2) or 0),
 *              log_z = ln Z, z = Z as a double (inf if above DBL_MAX);
 *              z_range_log2 = the largest, over the contraction tree, of a
 *              tensor's log2(max / smallest nonzero entry) as stored (float32
 *              entries under one power-of-two exponent per tensor, Sec. 3.1
 *              rescaled) and of the sum of a product's two operand ranges
 *              (the span of the products it forms): terms more than about
 *              2^126 below a tensor's maximum flush to zero, so values above
 *              100 mean the result may have lost such terms; 0 for the
 *              other semirings. */
typedef struct {
    int32_t semiring;
    int32_t size_i32;
    float size_f32;
    int32_t size_is_neg_inf;
    uint64_t count_mod_2_64;
    uint32_t residues[16];
    uint32_t primes[16];
    int32_t nresidues;
    uint32_t count_limbs[16];
    int32_t count_nlimbs;
    double z_mant;
    int64_t z_exp2;
    double log_z;
    double z;
    double seconds;            /* wall time of the call */
    double z_range_log2;       /* partition function: dynamic range of the tree's tensors (see above) */
} tn_result;

/* Contract the network along the plan on the context's stream and wait for
 * the root.  Errors: TN_EINVAL (semiring needs integer weights, plan built
 * for another network), TN_ENOMEM (allocator returned NULL), TN_EDEVICE,
 * TN_EOVERFLOW (exact count).  With the environment variable TN_LOG naming a
 * file, each call appends one JSON line to it (status, semiring, executor,
 * the plan's tc/sc/rwc, slice range, wall time and the result's key
 * values). */
tn_status tn_solve(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, const tn_solve_opts* opts,
                   tn_result* out);

/* Checkpoint and resume of sliced contractions (Sec. 4.2: the contraction is
 * the (+)-sum of its slices).  out = a (+) b for two results of one network,
 * plan and options over disjoint slice ranges (tn_solve with
 * opts->slice_begin / slice_end): a long run can store a tn_result (plain
 * bytes, owned by the caller) with the next slice index and continue later.
 * Host-side only; out may alias a or b.  Per semiring: tropical, the larger
 * size; counting tropical, the larger size with its count, the counts added
 * (mod 2^64) when the sizes are equal; exact count, the residues added per
 * prime and the CRT value and its check prime recomputed (TN_EOVERFLOW as in
 * tn_solve); partition function, Z_a + Z_b in float64 mantissa and exponent,
 * z_range_log2 the larger.  seconds: the sum.  TN_EINVAL for NULL pointers,
 * different semirings or primes, or another semiring. */
tn_status tn_result_combine(const tn_result* a, const tn_result* b, tn_result* out);

/* The contraction of tn_solve (per-node launches, opts->executor 0 or 1;
 * sliced plans too, opts->slice_begin/slice_end as there) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Every device buffer of the call
 * (the plan's program tables, the arena of live intermediates, split-K
 * partials, partition-function bookkeeping, weights and root accumulators)
 * lives in one fixed 256 MiB device array of the library, one copy per GPU,
 * held until the process ends; the call makes no device or pinned-host
 * allocation (host-side temporaries only) and no profiling records.  The
 * array keeps the last call's contents; a call sets up everything it reads.
 * Calls that overlap on one GPU (several contexts or threads on the same
 * device) race on the array: the caller serialises them.  Same result as
 * tn_solve with executor 1.  Errors as tn_solve, plus TN_ETOOBIG when the
 * solve needs more than the array (tn_plan_peak_bytes plus the program
 * tables), TN_EINVAL for plans with open vertices or executor 2, TN_EDEVICE
 * when the array could not be located on the device. */
tn_status tn_solve_noalloc(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, const tn_solve_opts* opts,
                           tn_result* out);

/* Many networks in one persistent launch: a device task table of
 * (job, node, tile) entries with dependency counters; workgroups pop ready
 * tiles until every job's root is done.  Jobs with much work run one after
 * the other on per-node launches over the whole chip instead: trees the auto
 * executor of tn_solve sends to per-node launches, except that in the exact
 * algebras (all but the partition function) trees of up to 2^31 semiring ops
 * per pass with intermediates of at most 2^24 entries stay in the shared
 * launch, where several of them fill the chiplets side by side (their
 * results do not depend on the route).  Launch shapes come from the tuning
 * table (or the heuristic) keyed by each node's own shape (see the
 * autotuner below), so a job's result does not depend on the other jobs in
 * the batch.  n jobs; opts and out have n
 * entries.  Jobs must not be sliced.  Per-job failures are reported in
 * out[i].semiring = -1 and the call returns the first failure. */
tn_status tn_solve_batch(tn_ctx* ctx, int32_t n, const tn_net* const* nets,
                         const tn_plan* const* plans, const tn_solve_opts* opts, tn_result* out);

/* Independence polynomial I(G, x) = sum_k c_k x^k, c_k = the number of
 * independent sets of size k: the GraphPolynomial property of the Sec. 5
 * table, computed by the finite-field method of Sec. 6.2.  The network is
 * contracted with vertex tensors [1, t] for t = 0 .. alpha (alpha = the
 * largest independent-set size, from one max-plus contraction) modulo primes
 * below 2^30 whose product exceeds the total count (from one exact-count
 * contraction), every evaluation one mod-p pass of the persistent launch;
 * the values are interpolated mod each prime and the coefficients
 * recombined by CRT, with one more prime as a check.
 *   limbs   32-bit limbs per coefficient (>= 1)
 *   coeffs  caller memory of (nv + 1) * limbs uint32: coefficient k, little
 *           endian, at coeffs[k * limbs]; entries above the degree are 0
 *   degree  receives alpha (NULL allowed)
 * Unit weights only; the plan must not be sliced.  Errors: TN_EINVAL
 * (weighted network, sliced plan, bad arguments), TN_ETOOBIG (nv > 512),
 * TN_EOVERFLOW (a coefficient needs more than limbs limbs, or the check
 * prime disagrees), TN_EDEVICE (device failure, or the coefficients do not
 * sum to the exact count). */
tn_status tn_solve_polynomial(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, int32_t limbs, uint32_t* coeffs,
                              int32_t* degree);

/* The k largest independent-set sizes and their counts (SizeMax(k) and
 * CountingMax(k) of the Sec. 5 table, Sec. 5.3 examples), for unit weights:
 * both are read off the independence polynomial (tn_solve_polynomial).
 *   sizes   k int32: the k largest sizes of independent sets, with
 *           multiplicity, largest first (SizeMax(k); fewer than k sets:
 *           the rest is INT32_MIN)
 *   counts  k * limbs uint32 (NULL allowed): the numbers of independent sets
 *           of sizes alpha, alpha - 1, ..., alpha - k + 1 (CountingMax(k),
 *           the coefficients of the k highest orders; 0 below size 0)
 *   k       1 .. 64
 * Errors as tn_solve_polynomial. */
tn_status tn_solve_max_k(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, int32_t k, int32_t* sizes,
                         int32_t limbs, uint32_t* counts);

/* Solve a plan with open vertices (tn_plan_opts.open): the result is the
 * tensor over the open vertices, one tn_result per assignment (marginals in
 * the chosen algebra: the property of the configurations that agree with
 * that assignment).  out[e] holds the assignment whose bit q is the value of
 * open vertex q in the order given at plan creation; cap >= 2^nopen.  Runs
 * on the stream executor (sliced plans too: open vertices are never
 * sliced); opts.executor 2 (persistent) is refused.  Errors as tn_solve, and
 * TN_EINVAL for cap too small.  A plan without open vertices gives one
 * result. */
tn_status tn_solve_open(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, const tn_solve_opts* opts, int64_t cap,
                        tn_result* out);

/* SizeMax(k) of the Sec. 5 table for any weights (and for spin glasses: the
 * k largest values of -H, i.e. minus the k lowest energies): the k largest
 * total weights over all independent sets, with multiplicity, largest first.
 * Computed in max-plus over sorted lists of the eight largest values (float32
 * weights, 32-byte tensor entries; the (x) of two lists keeps the eight
 * largest pairwise sums).
 *   k         1 .. 8
 *   executor  0 auto: one persistent launch for unsliced trees with
 *             sc <= 14 (a persistent launch runs one job on one chiplet),
 *             per-node launches otherwise; 1 per-node launches (sliced plans
 *             too); 2 persistent (unsliced plans only)
 *   sizes     caller memory of k floats; fewer than k configurations: the
 *             rest is -INFINITY
 * Synchronous.  Errors: TN_EINVAL (k or executor out of range, plan with open
 * vertices or built for another network, executor 2 with a sliced plan),
 * TN_ENOMEM, TN_EDEVICE. */
tn_status tn_solve_size_max_k(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, int32_t k, int32_t executor,
                              float* sizes);

/* CountingMax(k) of the Sec. 5 table for integer weights (and for spin
 * glasses with integer J and h: values of -H): the number of configurations
 * at each of the k values top, top - 1, ..., top - k + 1, where top is the
 * largest value.  Computed in one contraction over truncated polynomials
 * (per tensor entry the four highest-order terms c_d x^(m - d) of the
 * polynomial whose exponents are configuration values; (+) aligns two such
 * lists by their top exponent, (x) adds exponents and convolves the counts).
 * Counts are modulo 2^64 (as TN_COUNTING_TROPICAL); a value in between that
 * no configuration takes has count 0.
 *   k         1 .. 4
 *   executor  as for tn_solve_size_max_k: 0 auto (persistent for unsliced
 *             trees with sc <= 14), 1 per-node launches (sliced plans too),
 *             2 persistent (unsliced plans only)
 *   top       out: the largest value; INT32_MIN if no configuration
 *             satisfies the fixed vertices (then every count is 0)
 *   counts    caller memory of k uint64: counts[d] at value top - d
 * Synchronous.  Errors: TN_EINVAL (k or executor out of range, non-integer
 * weights, plan with open vertices or built for another network, executor 2
 * with a sliced plan), TN_ENOMEM, TN_EDEVICE. */
tn_status tn_solve_counting_max_k(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, int32_t k, int32_t executor,
                                  int32_t* top, uint64_t* counts);

/* One maximum configuration (SingleConfigMax of the Sec. 5 table): an
 * independent set of largest total weight, or for a spin-glass network a
 * ground state (a configuration of smallest energy H, Sec. 2).  The max-plus
 * float32 contraction runs once on the persistent executor with every tensor
 * of the tree kept; a one-workgroup kernel then traces the maximum back from
 * the root (at each inner node the summed indices take the first values whose
 * operand entries add up to the node's entry), and the host sets the
 * vertices that a single leaf sums by itself.
 *   config  caller memory of nv int32: config[v] = 1 if vertex v is in the
 *           set (spin glass: spin s_v = 2 config[v] - 1)
 *   value   receives the float32 maximum: the set's weight, or -H of the
 *           ground state (NULL allowed)
 * Among several maxima any one may be returned.  The plan must not be
 * sliced.  Errors: TN_EINVAL (sliced or foreign plan, no configuration
 * satisfies the fixed vertices, NULL config with
 * nv > 0), TN_ETOOBIG (an inner node sums more than 30 indices, or a tensor
 * of rank > 62), TN_ENOMEM, TN_EDEVICE (device failure, or no assignment
 * reproduces a node's value). */
tn_status tn_solve_single_config_max(tn_ctx* ctx, const tn_net* net, const tn_plan* plan, int32_t* config,
                                     float* value);

/* ----------------------------------------------------------- autotuner --- */

/* Launch shapes (kernel family, tile, K step, K splits) of the batched
 * semiring GEMMs come from a process-wide table keyed by the node's own
 * shape: device algebra, log2 batch / M / N / K and operand orders.  Keys not
 * in the table use a fixed heuristic.  The key holds nothing but the node's
 * shape, so a job runs the same launches alone and in any batch.
 *
 * tn_tune_plan times, for every inner node of the plan with at least
 * 2^min_log2_ops semiring operations whose key is not yet in the table, each
 * candidate shape the kernels accept on seeded operands of the node's size
 * (best of reps launches, split reduction included) and stores the fastest.
 * A candidate whose result differs from the heuristic shape's (any bit in
 * the exact algebras, more than 1e-4 relative per entry for the real one,
 * whose sums change order with the tile) is rejected.
 * Each semiring tunes the device algebras it runs (TN_COUNT_EXACT: the mod-p
 * kernels).  Device memory for the node's operands comes from the context's
 * allocator.  *ntuned receives the number of keys added.  Plans run after
 * the call use the new entries.  Errors: TN_EINVAL (NULL arguments, unknown
 * semiring), TN_ENOMEM, TN_EDEVICE. */
typedef struct {
    int32_t dsr;             /* device algebra: 0 max-plus int32, 1 max-plus float32, 2 counting
                                tropical, 3 counts mod p, 4 real float32, 5 real bfloat16 inputs */
    int32_t lb, li, lj, lk;  /* log2 batch, M, N, K */
    int32_t a_t, b_t;        /* operand orders: A [b][k][i], B [b][j][k] when set */
    int32_t ncand;           /* candidate shapes tried */
    int32_t nrejected;       /* candidates whose result differed */
    float heuristic_ms;      /* the heuristic shape's time */
    float best_ms;           /* the winner's time */
    int32_t shape[10];       /* winner: mode (0 tiled, 1 thin, 2 long-K), log2 tile batch / M / N,
                                log2 K step, rows / columns per thread, log2 K splits, matrix
                                cores, 0 */
} tn_tune_record;

tn_status tn_tune_plan(tn_ctx* ctx, const tn_plan* plan, int32_t semiring, double min_log2_ops, int32_t reps,
                       int32_t* ntuned);
/* Write the table as text (one line per key); *nentries (NULL allowed)
 * receives the entry count.  TN_EINVAL if the file cannot be written. */
tn_status tn_tune_save(const char* path, int32_t* nentries);
/* Merge a table file into the table.  Every line must be an entry the
 * kernels accept for its key, else nothing of the file is taken
 * (TN_EINVAL).  The file named by the environment variable TN_TUNE_FILE is
 * loaded at the first tn_ctx_create of the process. */
tn_status tn_tune_load(const char* path, int32_t* nentries);
/* Empty the table (every node back on the heuristic) and the records. */
void tn_tune_clear(void);
/* Records of the keys tuned since the last clear: copies up to cap; *n
 * receives the number available. */
tn_status tn_tune_records(tn_tune_record* recs, int32_t cap, int32_t* n);

/* -------------------------------------------------------------- server --- */

/* Continuous-batching server on one context.  Jobs are admitted in arrival
 * order while the sum of their device bytes (tn_server_job_bytes) stays
 * within hbm_budget_bytes and fewer than max_slots run; admitted jobs are
 * merged into the next persistent launch (on one of three streams) while
 * earlier launches may still run; a job tn_solve_batch would run on per-node
 * launches (see there) goes out alone on per-node launches, asynchronously on
 * its own stream.  Each job's latency is result-on-host minus submit time.
 * The server owns a scheduler thread. */
tn_status tn_server_create(tn_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_slots,
                           tn_server** out);
/* Thread-safe.  The net and plan must stay alive until the job is done.
 * TN_ETOOBIG if the job alone exceeds the budget. */
tn_status tn_server_submit(tn_server* s, const tn_net* net, const tn_plan* plan,
                           const tn_solve_opts* opts, uint64_t* job_id);
/* Thread-safe.  *done = 1 once the result is on the host. */
tn_status tn_server_poll(tn_server* s, uint64_t job_id, tn_result* out, int32_t* done,
                         double* latency_s);
/* Block until all submitted jobs are done. */
tn_status tn_server_drain(tn_server* s);

/* Device bytes a job takes in a server (the admission measure: every tensor
 * of every pass in its own region, as the persistent launch lays them out);
 * a server refuses a job above its budget.  No device access. */
tn_status tn_server_job_bytes(const tn_net* net, const tn_plan* plan, const tn_solve_opts* opts, uint64_t* bytes);

/* Cancel a job still in the queue: its poll then returns TN_ECANCELED.
 * Errors: TN_EBUSY (the job is already on the device), TN_EINVAL (unknown
 * or finished job).  Thread-safe. */
tn_status tn_server_cancel(tn_server* s, uint64_t job_id);

typedef struct {
    uint64_t submitted, completed, failed, launches;
    uint64_t peak_admitted_bytes;   /* largest sum of admitted jobs' device bytes (never above the budget) */
    int32_t peak_running;           /* most jobs on the device at once */
    int32_t peak_inflight;          /* most persistent launches in flight at once */
    uint64_t peak_pool_bytes;       /* high-water mark of the server's device pool (jobs and task tables) */
    uint64_t rejected;              /* submits refused with TN_ETOOBIG */
    uint64_t canceled;              /* jobs cancelled in the queue */
    uint64_t requeued;              /* admissions put back because the pool could not hold them */
} tn_server_stats_t;
tn_status tn_server_stats(tn_server* s, tn_server_stats_t* st);
tn_status tn_server_destroy(tn_server* s); /* drains first */

#ifdef __cplusplus
}
#endif

#endif /* TN_H_ */
