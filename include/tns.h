/*
 * tns.h -- C ABI of the MI355X (gfx950) tensor-network-states amplitude
 * library.
 *
 * Method: Guo, Zhao, Huang, "Verifying Random Quantum Circuits with Arbitrary
 * Geometry Using Tensor Network States Algorithm" (arXiv:2011.02621).  Given a
 * circuit on a graph G = {V, E} and bitstrings s, the library returns the
 * amplitudes <s|U|0...0> ("two-sided circuit evolution" paragraph):
 *
 *   1. every two-qubit gate, with neighbouring single-qubit gates fused in, is
 *      split by SVD into P and Q (Eq. (2));
 *   2. the first group of cycles is applied to the product state |0...0>
 *      (Eq. (1)) and the second group, transposed and in reverse order, to the
 *      product state <s| (Eqs. (3)-(4)), each gate followed by an SVD bond
 *      compression (Eqs. (5)-(6));
 *   3. the two tensor network states are merged over their physical legs into
 *      one network without open legs (Eq. (8));
 *   4. optional cut bonds split that network into independent sub-networks
 *      ("slices") whose scalars sum to the amplitude (overlap paragraph);
 *   5. each sub-network is contracted pairwise along one linear path
 *      (supplement, Algorithm 1 or a greedy search), every step a permute
 *      followed by a complex GEMM over the shared bonds.
 *
 * Every compute step runs in HIP kernels on the device; the host only plans
 * (graph bookkeeping, bond-dimension bounds, path search, slicing, launch
 * descriptors).
 *
 * Conventions
 *   - Every call returns tns_status; 0 is success.  No C++ exception crosses
 *     this boundary.  On failure tns_last_error() describes the cause.
 *   - Qubit q of bitstring b is bits[b * n_qubits + q] (0 or 1).
 *   - A two-qubit gate matrix is indexed by 2*b(q0) + b(q1); rows are outputs.
 *     Matrices are row-major complex numbers stored as interleaved (re, im)
 *     doubles: 2x2 in m[0..7], 4x4 in m[0..31].
 *   - Amplitudes are returned as complex128 (re, im) pairs whatever the
 *     contraction precision.
 *   - The caller owns every array it passes.  Inputs are copied during the
 *     call, except the bits/amps arrays of tns_submit, which must stay valid
 *     until the request completes.
 *   - Plans are immutable after creation and may be shared between threads.
 *     A context may be used from several threads; calls on one context are
 *     serialised internally.
 */
#ifndef TNS_H
#define TNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TNS_OK = 0,
    TNS_E_INVALID_ARG = -1,    /* null pointer, negative size, bad option value */
    TNS_E_BAD_CIRCUIT = -2,    /* qubit out of range, two-qubit gate on a non-edge,
                                  duplicate edge, matrix not unitary within 1e-8 */
    TNS_E_BAD_PATH = -3,       /* path not a permutation of 0..N-1, bad cut edge,
                                  or the path search found no admissible path */
    TNS_E_OUT_OF_MEMORY = -4,  /* the plan cannot fit the HBM budget */
    TNS_E_ADMISSION = -5,      /* serving: request cannot be admitted */
    TNS_E_DEVICE = -6,         /* a HIP call failed */
    TNS_E_CANCELLED = -7,      /* request cancelled */
    TNS_E_UNSUPPORTED = -8,    /* valid input outside what the kernels support
                                  (e.g. a site with more than TNS_MAX_DEGREE legs) */
    TNS_E_NO_DEVICE = -9       /* compute call on a planning-only context */
} tns_status;

/* Contraction number type.  Gate splitting, evolution and compression always
 * run in complex128 (FP64); so does the final sum over slices. */
typedef enum {
    TNS_C128 = 0,              /* complex128 GEMM on FP64 MFMA */
    TNS_C64 = 1,               /* complex64 GEMM on FP32 MFMA (4 real products) */
    TNS_C64_SPLIT_BF16_3 = 2,  /* complex64 operands split into bf16 hi+lo, 3 products,
                                  FP32 accumulation */
    TNS_C64_SPLIT_BF16_6 = 3   /* hi+mid+lo split, 6 products, FP32 accumulation */
} tns_precision;

typedef enum {
    TNS_PATH_GREEDY = 0,       /* best-first single path by least step cost */
    TNS_PATH_ALGORITHM1 = 1    /* priority-queue search of the supplement (Algorithm 1) */
} tns_path_mode;

#define TNS_MAX_DEGREE 8       /* legs per site the kernels accept */
#define TNS_MAX_QUBITS 128

typedef struct tns_ctx tns_ctx;
typedef struct tns_plan tns_plan;
typedef struct tns_request tns_request;

typedef struct {
    int32_t q0;                /* qubit */
    int32_t q1;                /* second qubit, or -1 for a single-qubit gate */
    int32_t cycle;             /* cycle index; decides the side of the two-sided split */
    int32_t reserved;          /* set to 0 */
    double m[32];              /* row-major complex matrix, interleaved (re, im) */
} tns_gate;

typedef struct {
    int32_t n_qubits;          /* N, 2..TNS_MAX_QUBITS */
    int32_t n_edges;
    const int32_t *edges;      /* [n_edges][2]: the graph G; each pair once */
    int32_t n_gates;
    const tns_gate *gates;     /* in time order */
} tns_circuit_desc;

typedef struct {
    int32_t split_cycle;       /* gates with cycle < split_cycle evolve the ket |0..0>,
                                  the rest evolve the bra <s|; -1 = choose the
                                  split with the least planned contraction cost */
    const int32_t *path;       /* [n_qubits] contraction order, or NULL = search */
    int32_t path_mode;         /* tns_path_mode, used when path == NULL */
    int32_t max_rank;          /* Algorithm 1 rank bound (the paper's M); 0 = auto */
    int32_t path_assumptions;  /* 1 = apply the three assumptions of Algorithm 1,
                                  0 = unrestricted search (exact optimum, small N only) */
    int32_t n_cuts;            /* >= 0 with cut_edges, or -1 = choose cuts automatically */
    const int32_t *cut_edges;  /* [n_cuts] edge ids to slice over */
    uint64_t max_intermediate_elems; /* automatic cuts keep every intermediate at or
                                        below this many elements; 0 = 2^32 */
    double svd_rel_cutoff;     /* in every SVD compression (Eq. (5)), singular values
                                  <= cutoff * sigma_max of that SVD are set to zero
                                  (the planned bond dimension is kept, the dropped
                                  directions carry exact zeros); 0 = 1e-12 */
    int64_t max_search_states; /* Algorithm 1 pop budget; 0 = 4,000,000 */
    tns_precision precision;
    int32_t n_open;            /* 0..20 qubits whose output bit is left open */
    const int32_t *open_qubits;/* [n_open] distinct qubits, or NULL when n_open = 0.
                                  The bra's bit of each open qubit stays a free leg, so
                                  one contraction yields the 2^n_open amplitudes of all
                                  bitstrings that agree outside these qubits (the rest
                                  of the network, and its contraction, is shared). */
    int32_t path_branches;     /* 1 (default) = relax the linear path into a main path with
                                  side branches where that lowers the summed cost (several
                                  main paths, the relaxation of the single main path that the
                                  supplement leaves open); 0 = one linear path */
} tns_plan_opts;

/* Description of a plan.  Pointers refer to plan-owned memory, valid until
 * tns_plan_destroy. */
typedef struct {
    int32_t n_qubits, n_edges, split_cycle, n_steps;
    const int32_t *path;            /* [n_qubits] contraction order */
    const int64_t *step_m;          /* [n_steps] GEMM rows (open legs kept) */
    const int64_t *step_k;          /* [n_steps] shared-bond product */
    const int64_t *step_n;          /* [n_steps] new-leg product */
    const int32_t *step_kernel;     /* [n_steps] 0 MFMA GEMM (real embedding), 1 small,
                                       2 final dot, 3 MFMA GEMM in the three-multiplication
                                       form (complex64 steps with even K >= 128 or even
                                       K <= 64, N >= 64, M >= 64) */
    const int32_t *step_permute;    /* [n_steps] 0 no permute, 1 permute launch, 2 permute done
                                       by the previous step's store (fused; a GEMM, or a
                                       small-bond step with at least 64 rows) */
    const int32_t *bond_ket;        /* [n_edges] ket bond dimensions */
    const int32_t *bond_bra;        /* [n_edges] bra bond dimensions */
    const int32_t *bond_overlap;    /* [n_edges] overlap bond dimensions */
    int32_t n_cuts;
    const int32_t *cut_edges;       /* [n_cuts] */
    int64_t n_slices;
    double flops_per_amp;           /* 8 * sum over slices and steps of M*K*N, the shared
                                       prefix steps counted once */
    double gemm_bytes_per_amp;      /* element bytes * sum (MK + KN + MN) */
    double permute_bytes_per_amp;   /* 2 * element bytes * elements of the permute launches */
    double path_score;              /* sum of M*K*N of one slice (the supplement's score) */
    int64_t peak_elems;             /* largest intermediate of one slice */
    int64_t device_bytes_resident;  /* ket tensors and plan tables */
    int64_t device_bytes_per_unit;  /* workspace of one (bitstring, slice) unit */
    int32_t n_fused_ket, n_fused_bra;
    int32_t search_complete;        /* 1 when every Algorithm 1 search behind the final path
                                       finished within max_search_states (also 1 for a given
                                       or greedy path); 0 when one stopped at the budget, whose
                                       result is then the greedy path */
    int64_t search_states;          /* states popped by those Algorithm 1 searches */
    int32_t max_rank_used;          /* rank bound M used by the search */
    double fidelity;                /* Eq. (9) with the paper's Sycamore error rates */
    double n_samples;               /* (3 / fidelity)^2 */
    tns_precision precision;
    int32_t n_open;                 /* open qubits; each input bitstring yields 2^n_open amplitudes */
    const int32_t *open_qubits;     /* [n_open] */
    int32_t n_branches;             /* side branches of the path (tns_plan_opts.path_branches) */
    const int32_t *branch_windows;  /* [n_branches][2]: positions [a, b) of `path` contracted as
                                       one branch (in path order) and absorbed by the main path
                                       just before it reaches position b */
    const int32_t *step_chain;      /* [n_steps] 0 main path, w + 1 a step of branch w */
    double linear_score;            /* sum of M*K*N of one slice along `path` as a single linear
                                       path (path_score is that of the plan with its branches) */
    int32_t n_prefix_steps;         /* leading entries of step_* whose tensors carry no cut bond
                                       (every slice has the same ones: overlap paragraph,
                                       cutting): computed once per bitstring and copied to each
                                       (bitstring, slice) unit; 0 without cuts or when only the
                                       first tensor would be shared */
    double prefix_flops_per_amp;    /* 8 * sum of M*K*N over those steps (in flops_per_amp once) */
} tns_plan_info;

typedef struct {
    double ms_total;                /* host wall time of the call */
    double ms_bra;                  /* bra evolution (device) */
    double ms_merge;                /* overlap merge (device) */
    double ms_contract;             /* contraction steps and slice sum (device) */
    double flops;                   /* algorithmic contraction flops executed */
    int64_t units;                  /* (bitstring, slice) work units */
    int64_t launches;               /* kernel launches */
    int64_t peak_device_bytes;      /* workspace high-water mark */
    /* per-kernel-class device time, measured with HIP events on the launch
     * stream around every launch of the class (filled when stats != NULL) */
    double ms_gemm;                 /* MFMA complex GEMM launches */
    int64_t gemm_launches;
    double gemm_flops;              /* algorithmic flops of those launches (8 M K N) */
    double gemm_bytes;              /* algorithmic bytes (e * (MK + KN + MN)) */
    double ms_permute;              /* boundary permutes */
    double permute_bytes;           /* bytes read + written by them */
    double ms_small;                /* small-bond and final-dot steps */
    double gemm_mfma_flops;         /* real flops the MFMA instructions of the GEMM launches
                                       execute: 8 M K N for the real-embedded forms, 6 M K N
                                       for the three-multiplication complex64 form, 3x or 6x
                                       8 M K N (BF16) for split-BF16 */
    /* the three-multiplication complex64 GEMM launches alone (step kernel 3),
     * a subset of the GEMM launches above */
    double ms_gemm3m;
    int64_t gemm3m_launches;
    double gemm3m_flops;            /* 8 M K N, the complex product's real flops */
    double gemm3m_mfma_flops;       /* 6 M K N, what its MFMA instructions execute */
    double gemm3m_bytes;            /* e * (MK + KN + MN) */
} tns_stats;

/* --- context ---------------------------------------------------------- */

/* device >= 0 selects a HIP device; device = -1 creates a planning-only
 * context (no GPU use; tns_plan_create works and tns_amplitudes returns
 * TNS_E_NO_DEVICE).  hbm_budget_bytes = 0 uses 90 % of the device's free
 * memory. */
tns_status tns_init(int device, uint64_t hbm_budget_bytes, tns_ctx **out);

/* Install a device allocator (e.g. a framework's caching allocator).  alloc
 * returns NULL on failure.  Must be called before the first plan. */
tns_status tns_set_allocator(tns_ctx *ctx,
                             void *(*alloc)(size_t bytes, void *stream, void *user),
                             void (*free_)(void *ptr, void *stream, void *user),
                             void *user);

/* Stops the serving workers and frees the context.  Plans created on a
 * device context hold its device memory: tns_finalize fails with
 * TNS_E_INVALID_ARG while any of them is alive (destroy them first). */
tns_status tns_finalize(tns_ctx *ctx);

/* --- plans ------------------------------------------------------------ */

void tns_plan_opts_default(tns_plan_opts *opts);

/* Validate the circuit, fuse single-qubit gates into their two-qubit
 * neighbours, split every fused gate by SVD (Eq. (2)), evolve the ket side
 * on the device (kept resident), bound every bond dimension, choose cuts and
 * a contraction path, and compile the step list.  Inputs are copied. */
tns_status tns_plan_create(tns_ctx *ctx, const tns_circuit_desc *desc,
                           const tns_plan_opts *opts, tns_plan **out);
tns_status tns_plan_info_get(const tns_plan *plan, tns_plan_info *out);
/* Waits for the serving requests submitted on the plan to complete, then
 * frees it. */
tns_status tns_plan_destroy(tns_plan *plan);

/* --- amplitudes ------------------------------------------------------- */

/* amps[2*b], amps[2*b+1] = <s_b|U|0...0> for b < n.  bits and amps are host
 * arrays; amps is written only on TNS_OK.  hip_stream = NULL uses the
 * context's stream.  stats may be NULL.  Blocks until the results are on the
 * host.  With open qubits amps holds [n][2^n_open] complex values: entry
 * (b, x) is the amplitude of s_b with its open bits replaced by the bits of x,
 * the first open qubit being the most significant bit of x; the bits given
 * for open qubits are ignored. */
tns_status tns_amplitudes(tns_ctx *ctx, const tns_plan *plan, int64_t n,
                          const uint8_t *bits, double *amps, void *hip_stream,
                          tns_stats *stats);

/* Partial amplitudes over the slices [slice_begin, slice_end) of the plan's
 * cut bonds: amps[b] = sum over those slices of the sub-network scalars
 * (overlap paragraph: every slice of the cut network yields one scalar and
 * the scalars add up to the amplitude).  Partial sums over disjoint ranges
 * covering [0, n_slices) add up to the amplitudes of tns_amplitudes, so the
 * slices of one amplitude can be split over calls, streams or devices.
 * 0 <= slice_begin < slice_end <= n_slices, else TNS_E_INVALID_ARG. */
tns_status tns_amplitudes_sliced(tns_ctx *ctx, const tns_plan *plan, int64_t n,
                                 const uint8_t *bits, int64_t slice_begin, int64_t slice_end,
                                 double *amps, void *hip_stream, tns_stats *stats);

/* Allocation-free variant of tns_amplitudes, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It computes the same amplitudes as
 * tns_amplitudes (same kernels), with every intermediate -- bra tensors,
 * merged site tensors, boundary tensors, GEMM operands, per-slice partial
 * sums -- placed in a static device array of TNS_NOALLOC_SCRATCH_BYTES per
 * GPU that exists from library load to process end; the call allocates and
 * frees nothing and does not synchronise: it only enqueues work on
 * hip_stream (NULL = the context's stream) and returns.
 *   bits_dev  device array [n][n_qubits], bit = byte & 1; read in place.
 *   amps_dev  device array [n][2^n_open] of complex128 (re, im) pairs,
 *             written in place; valid once the stream reaches that point.
 * Both stay owned by the caller and must stay valid until the stream has
 * run the work.  The plan must have been created on ctx (plan creation
 * itself allocates).  Errors: TNS_E_INVALID_ARG as tns_amplitudes;
 * TNS_E_OUT_OF_MEMORY, before any launch, when the plan's workspace for one
 * bitstring does not fit the static array (larger batches are split into
 * batches that fit).  Every call on one GPU shares that GPU's array, and
 * the array keeps the last call's contents: calls whose work overlaps on the
 * device race (two streams, or two contexts on one GPU); order them on one
 * stream or synchronise between them. */
#define TNS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tns_status tns_amplitudes_noalloc(tns_ctx *ctx, const tns_plan *plan, int64_t n,
                                  const uint8_t *bits_dev, double *amps_dev, void *hip_stream);

/* Frugal rejection sampling from correlated batches.  The tensor network's
 * advantage over a state vector includes simulating measurements
 * (introduction); with open qubits (tns_plan_opts.open_qubits, k of them)
 * one contraction yields the 2^k amplitudes of a batch, and each of them is
 * accepted or rejected on the device by the published frugal rule: candidate
 * x of batch b is accepted when 2^N |amp(b, x)|^2 / m_bound > uniforms[b][x],
 * i.e. with probability min(1, 2^N p / m_bound).  When m_bound bounds
 * 2^N p for every candidate, the accepted bitstrings are distributed as p
 * (with uniformly random fixed bits); for random circuits p follows the
 * Porter-Thomas law and about 1 / m_bound of the candidates are accepted.
 *   fixed_bits  [n_batches][N] 0/1, host; bits of open qubits are ignored.
 *   uniforms    [n_batches][2^k] in [0, 1), host, supplied by the caller.
 *   accepted    [n_batches][2^k] 0/1 out, host; candidate x of batch b is
 *               fixed_bits[b] with its open bits set from x (first open qubit
 *               most significant, as in tns_amplitudes).
 *   amps        [n_batches][2^k] complex out (as tns_amplitudes).
 * Errors: TNS_E_INVALID_ARG for NULL arrays or m_bound <= 0, plus those of
 * tns_amplitudes.  A plan without open qubits gives one candidate per batch. */
tns_status tns_sample_frugal(tns_ctx *ctx, const tns_plan *plan, int64_t n_batches,
                             const uint8_t *fixed_bits, const double *uniforms, double m_bound,
                             uint8_t *accepted, double *amps, void *hip_stream,
                             tns_stats *stats);

/* --- serving ---------------------------------------------------------- */

/* Asynchronous request (continuous batching).  A request is cut into work
 * items, each a range of bitstrings times a range of slices (a block of the
 * independent (bitstring, slice) units of the overlap paragraph's cutting),
 * shaped at submission to about 4e13 contraction flops each and to fit
 * memory.  The context's worker threads, one HIP stream and workspace each,
 * take the next item of the active request with the least planned work left
 * (shortest remaining work first), so requests that arrive while others run
 * are admitted as workers and memory free up, short requests are not held
 * behind long ones, and items of several requests overlap on the device.  Memory: the first tns_submit starts the
 * workers; a quarter of the context's HBM budget stays with synchronous
 * calls on the same context (a larger cached synchronous workspace is
 * released) and the rest is a pool the workers share; an item starts only
 * when its workspace fits the pool beside the other workers' reservations,
 * and while items wait for memory, idle workers return their cached
 * workspace.  The partial sums of a request's slice ranges are added per
 * bitstring in slice-range order, so a result does not depend on what else
 * was served beside it.  bits and amps must stay valid until done.  A
 * request of which one (bitstring, slice) unit does not fit the pool fails
 * with TNS_E_ADMISSION. */

/* Serving knobs, before the first tns_submit on ctx: n_workers (1..16, 0 =
 * 3) and the contraction flops per work item (0 = 4e13; a small value cuts
 * every request into single (bitstring, slice) units). */
tns_status tns_serving_configure(tns_ctx *ctx, int32_t n_workers, double item_flops);

tns_status tns_submit(tns_ctx *ctx, const tns_plan *plan, int64_t n,
                      const uint8_t *bits, double *amps, tns_request **out);
tns_status tns_poll(tns_request *req, int *done);   /* *done = 1 when finished */
tns_status tns_wait(tns_request *req);              /* returns the request's status */
tns_status tns_cancel(tns_request *req);
tns_status tns_request_free(tns_request *req);      /* waits for completion first */
/* Request timing: arrival-to-completion and admission-to-completion, ms. */
tns_status tns_request_latency(const tns_request *req, double *ms_total, double *ms_run);

/* --- planning helpers (host only) ------------------------------------ */

/* Linear contraction path over an arbitrary graph with bond dimensions
 * dims[e] (supplement, path section).  mode: tns_path_mode.  assumptions: as
 * in tns_plan_opts.  path_out[n] receives the order, score_out the summed
 * step cost (product of the dimensions of every bond carried by either
 * operand).  max_intermediate > 0 (Algorithm 1 only): a size-aware bound
 * beside the rank bound -- no intermediate may exceed that many elements
 * (0 = no bound).  Fails with TNS_E_BAD_PATH when no admissible path
 * exists. */
tns_status tns_path_search(int32_t n, int32_t n_edges, const int32_t *edges,
                           const double *dims, int32_t mode, int32_t max_rank,
                           int32_t assumptions, int64_t max_states, double max_intermediate,
                           int32_t *path_out, double *score_out);

/* Thread-local description of the last failure on this thread. */
const char *tns_last_error(void);
const char *tns_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TNS_H */
