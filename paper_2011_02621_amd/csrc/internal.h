// Internal declarations of the tensor-network-states amplitude library.
// Host planning structures, device launch descriptors and the launcher
// prototypes shared by the host code and the HIP kernels.
#pragma once

#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tns.h"

namespace tns {

// ----------------------------------------------------------------------------
// errors

struct Error : std::runtime_error {
    tns_status code;
    Error(tns_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(tns_status code, const std::string &msg);
void set_last_error(const std::string &msg);

// ----------------------------------------------------------------------------
// limits

constexpr int kMaxDeg = TNS_MAX_DEGREE;   // legs per site
constexpr int kMaxGatherDims = 24;        // axes of one strided gather / permute
constexpr int kMaxChi = 4;                // two-qubit operator Schmidt rank

// ----------------------------------------------------------------------------
// device launch descriptors (passed by value to kernels)

// Shape of a site tensor during the evolution: n axes, axis 0 the physical
// leg (2), then the site's bonds in edge-id order.
struct SiteShape {
    int32_t n;
    int32_t d[kMaxDeg + 1];
};

// Strided gather: out[i] = in[base + sum_a idx_a(i) * stride[a]] with i the
// row-major index over size[0..n).  Used for permutes, the initial boundary
// tensor and the B operand of each step.
struct Gather {
    int32_t n;
    int64_t size[kMaxGatherDims];
    int64_t stride[kMaxGatherDims];
};

// Offset of one slice inside a site tensor: the slice index is a mixed-radix
// number over the cut bonds (last cut fastest); only the cut bonds that touch
// the site contribute, each with its stride in the site tensor.
constexpr int kMaxCuts = 24;
struct SliceMap {
    int32_t n;
    int64_t div[kMaxCuts];
    int64_t dim[kMaxCuts];
    int64_t stride[kMaxCuts];
};

// One fused two-qubit operation for the fuse/split kernel.
struct FuseDesc {
    int32_t gate;        // base two-qubit gate (index into the circuit's gates)
    int32_t pre0, pre1;  // chains applied before the gate on q0 / q1 (-1: none)
    int32_t post0, post1;// chains applied after the gate (-1: none)
    int32_t transpose;   // split the transpose (bra side)
    int32_t chi;         // number of singular triplets to keep
    int32_t pad;
};

// ----------------------------------------------------------------------------
// host planning structures

struct Graph {
    int n = 0;
    std::vector<std::pair<int, int>> edges;
    std::vector<std::vector<int>> legs;   // per site, incident edge ids ascending
    std::map<std::pair<int, int>, int> index;
    int edge_id(int a, int b) const {
        auto it = index.find({a < b ? a : b, a < b ? b : a});
        return it == index.end() ? -1 : it->second;
    }
    int leg_of(int site, int edge) const {
        for (size_t i = 0; i < legs[site].size(); ++i)
            if (legs[site][i] == edge) return (int)i;
        return -1;
    }
};

// A fused two-qubit operation as applied on one side of the evolution.
struct EvoOp {
    int fused;           // index into the fuse descriptors (P/Q storage slot)
    int q0, q1, edge, chi;
    int leg0, leg1;      // position of `edge` among the bonds of q0 / q1
    SiteShape s0, s1;    // shapes of the two sites before the op
    int d_before, d_grown, d_after;
    int comp;            // -1: no compression; 0: SVD on q0, absorb into q1; 1: reverse
};

struct SideEvolution {
    std::vector<EvoOp> ops;              // in application order
    std::vector<int> bond;               // final bond dims per edge
    std::vector<int64_t> cap;            // per-site buffer capacity (elements)
    std::vector<SiteShape> final_shape;  // per-site shape at the end
};

// One pairwise contraction step (supplement, Eq. for C^{i_1..i_m}).
// Store layout of a GEMM whose result goes straight into the order the next
// step multiplies in (that step's boundary permute fused into the store):
// complex element (m, n) of a unit lands at fa[m >> shift] + fb[m & mask] +
// fg[n].  A pure axis permutation is additive over the digits of m and n, and
// with power-of-two dimensions over the high and low bits of m, so three
// small tables describe it exactly.
struct ScatterStore {
    const int64_t *fa = nullptr, *fb = nullptr, *fg = nullptr;
    int shift = 0;
    int mfast = 0;   // 1: consecutive rows are consecutive in the target, 0: columns
};

// LDS of the row-tiled small-step kernel, sized per launch: rows of A
// (padded by one complex) in at most kSmallRowsA bytes, at least 8 of them,
// and B^T (N x K, padded likewise) in at most kSmallRowsB.
constexpr int64_t kSmallRowsA = 32768, kSmallRowsB = 32768;
inline int64_t small_rows_block(int64_t K, int64_t csize) {
    const int64_t rb = kSmallRowsA / ((K + 1) * csize);
    return rb < 256 ? rb : 256;
}
// csize: bytes per complex element (8 for complex64, 16 for complex128)
// complex64 MFMA steps that take the three-multiplication GEMM (kernel
// class 3) and at least 64 complex columns: even K of at least 128 (its
// block is 128 x 64; measured with fused stores: +12 % from K = 256 up,
// +2-7 % at K = 128, a loss of 3-10 % at K = 64), or even K of at most 64,
// where a kernel that keeps A in registers and walks the columns (the
// output-bound short-K steps) takes them (gemm_3m_short_k)
// Split K (launch::gemm, three-multiplication form): a small output over a
// very long K, with the destination's unit slot large enough to hold the S
// partial products past the M N outputs
inline int64_t splitk_parts(int64_t K) {
    const int64_t S = std::min<int64_t>(512, (K + 255) / 256);
    const int64_t kc = ((K + S - 1) / S + 31) / 32 * 32;
    return (K + kc - 1) / kc;
}
inline bool gemm_3m_splitk(int64_t M, int64_t K, int64_t N, int64_t units, int64_t sC) {
    return M <= 64 && N <= 64 && K >= 4096 && units <= 64 && sC >= (splitk_parts(K) + 1) * M * N;
}
inline bool gemm_3m_short_k(int64_t K) { return K <= 64; }
inline bool gemm_3m_fits(int64_t M, int64_t K, int64_t N) {
    return K % 2 == 0 && (K >= 128 || K <= 64) && N >= 64 && M >= 64;
}
inline bool small_rows_fits(int64_t M, int64_t K, int64_t N, int64_t csize) {
    return M >= 64 && small_rows_block(K, csize) >= 8 && N * (K + 1) * csize <= kSmallRowsB;
}

struct Step {
    int chain = 0;                       // 0: the main path; w + 1: branch w
    bool start = false;                  // the chain's first tensor, gathered from `site`
    int site = -1;                       // site tensor absorbed (i_{m+1}), or the start site
    int branch = -1;                     // >= 0: absorbs that branch's tensor instead of a site
    int prev = -1;                       // step that produced this step's A operand
    std::vector<int> t_legs;             // boundary legs before the step (storage order)
    bool permute = false;
    bool permute_fused = false;          // done by the previous step's GEMM store
    Gather perm;                         // boundary permute (t_legs -> m_legs ++ k_legs)
    bool store_fused = false;            // this step's GEMM stores in the next step's order
    std::vector<int64_t> sc_tab;         // host tables fa ++ fb ++ fg
    int64_t sc_na = 0, sc_nb = 0;        // entries of fa and fb (fg: N entries)
    int sc_shift = 0, sc_mfast = 0;
    std::vector<int> m_legs, k_legs, n_legs;
    int64_t M = 1, K = 1, N = 1;
    int kernel = 0;                      // 0 MFMA GEMM, 1 small, 2 final dot, 3 MFMA GEMM (3 products)
    Gather bgather;                      // site tensor -> B[n][k] (k fastest)
    int64_t out_elems = 0;               // M * N
};

struct Plan;

// ----------------------------------------------------------------------------
// host planner entry points (planner.cpp)

struct Circuit {
    int n = 0;
    Graph g;                       // real couplers first, then one dangling leg per open qubit
    std::vector<tns_gate> gates;
    int max_cycle = 0;
    int n_real_edges = 0;
    int n_open = 0;
    std::vector<int> open_qubits;  // the bra's output bit of these qubits stays an open leg
};

void validate_and_build(const tns_circuit_desc *desc, Circuit &c);
void add_open_legs(Circuit &c, const tns_plan_opts &opts);
int operator_schmidt_rank(const double *m32);

struct PathResult {
    std::vector<int> order;
    double score = 0;
    double peak = 0;
    int max_rank = 0;
    int64_t states = 0;
    bool complete = true;
};

// max_size > 0: Algorithm 1 admits no intermediate above max_size elements
// (the size-aware bound beside the rank bound M)
PathResult path_search(int n, const std::vector<std::pair<int, int>> &edges,
                       const std::vector<double> &dims, int mode, int max_rank,
                       bool assumptions, int64_t max_states, double max_size = 0);
double path_score(int n, const std::vector<std::pair<int, int>> &edges,
                  const std::vector<double> &dims, const std::vector<int> &order,
                  double *peak, int *max_rank);

void plan_host(const Circuit &c, const tns_plan_opts &opts, Plan &p);
std::vector<std::pair<int, int>> choose_branches(const Circuit &c, const std::vector<double> &d,
                                                 const std::vector<int> &order, double log2_limit,
                                                 double log2_branch_limit, double *score_out);
// branch tensors stay below this many elements (their buffer is a third
// boundary buffer of each work unit)
constexpr int64_t kBranchPeakElems = (int64_t)1 << 28;

// ----------------------------------------------------------------------------
// the plan

struct DeviceBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Ctx;

struct Plan {
    // inputs
    Circuit circ;
    tns_plan_opts opts{};
    int split = 0;
    int precision = TNS_C128;

    // fusion
    std::vector<FuseDesc> fuse;          // ket ops first, then bra ops
    std::vector<int32_t> chain_flat;     // gate indices
    std::vector<int32_t> chain_off, chain_len;
    std::vector<int32_t> ket_init_chain, bra_final_chain;  // per qubit, -1: identity
    int n_fused_ket = 0, n_fused_bra = 0;

    SideEvolution ket, bra;
    std::vector<int> bond_overlap;

    // slicing
    std::vector<int> cuts;
    int64_t n_slices = 1;
    std::vector<int64_t> slice_radix;    // dims of the cut bonds

    // overlap site tensors: physical layout = bonds in edge-id order
    std::vector<std::vector<int64_t>> site_dims;   // per site, overlap dims per bond
    std::vector<int64_t> site_elems;

    // path and steps
    PathResult path;
    // branches (several main paths): windows [a, b) of path.order contracted
    // by their own linear path and absorbed whole by the main path
    std::vector<std::pair<int, int>> branches;
    double linear_score = 0;             // sum of M K N of the single linear path
    // Algorithm 1 searches that built the final path: all finished within
    // their state budget, and the states they popped
    bool search_complete = true;
    int64_t search_states = 0;
    std::vector<Step> steps;
    int64_t peak_elems = 0;
    int64_t branch_peak_elems = 0;       // largest tensor of a branch
    int64_t unit_stride = 0;             // boundary buffer stride per unit (peak, 32-aligned)
    int64_t branch_stride = 0;           // branch buffer stride per unit (32-aligned)
    int64_t max_b_elems = 0;             // largest B operand (complex elements)
    // Slice prefix: steps [0, prefix_steps) are on the main path and carry no
    // cut bond, so every slice computes the same tensors there; they run once
    // per bitstring and their result (prefix_elems per bitstring) is copied to
    // each (bitstring, slice) unit.  0 when there is nothing to share.
    int prefix_steps = 0;
    int64_t prefix_elems = 0;
    double prefix_flops = 0;             // 8 M K N summed over the prefix steps
    double flops_per_amp = 0, gemm_bytes_per_amp = 0, permute_bytes_per_amp = 0;
    double path_score = 0;

    // per-site slice offsets of the cut bonds
    std::vector<SliceMap> slice_map;
    int64_t out_per_unit = 1;            // 2^(open qubits): values per (bitstring, slice)
    Gather final_perm{};                 // open legs of the last tensor -> output order

    // info arrays exposed through tns_plan_info
    std::vector<int64_t> info_m, info_k, info_n;
    std::vector<int32_t> info_kernel, info_permute, info_path, info_chain, info_branch_windows;
    double fidelity = 0, n_samples = 0;

    // device state
    Ctx *ctx = nullptr;
    bool on_device = false;
    DeviceBuf d_mats, d_chain, d_chain_off, d_chain_len, d_fuse, d_pq;
    DeviceBuf d_ket_vec, d_bra_mat;
    std::vector<DeviceBuf> ket_site;     // resident ket tensors (complex128)
    std::vector<DeviceBuf> d_scatter;    // per step: fused-store tables (empty if none)
    std::vector<ScatterStore> scatter;   // per step: device view of d_scatter
    int64_t resident_bytes = 0;
    int64_t bytes_per_unit = 0;
    int64_t bytes_per_bitstring = 0;
    int64_t bra_scratch_elems = 0;       // V' scratch per bitstring (complex128)
    mutable std::atomic<int> serving_in_flight{0};   // submitted requests not yet complete
};

// ----------------------------------------------------------------------------
// runtime context

struct Ctx;

// Workspace buffers owned by one executor (the synchronous path or one
// serving stream); grown on demand, reused across calls.
// In arena mode (arena != nullptr) the slots are carved once, in order, out
// of a caller-provided device region of arena_cap bytes, and nothing is
// allocated or freed: a slot that would not fit fails with
// TNS_E_OUT_OF_MEMORY.
struct Workspace {
    std::vector<DeviceBuf> bufs;
    int64_t bytes = 0;
    char *arena = nullptr;
    size_t arena_cap = 0, arena_top = 0;
    void *get(Ctx *ctx, int slot, size_t bytes, void *stream);
    void release(Ctx *ctx, void *stream);
};

// Device address of the static workspace of tns_amplitudes_noalloc on one
// device (scratch.hip).  scratch_setup looks it up once per device and must
// run with that device current; scratch_device_ptr returns the stored address
// (nullptr before setup).
constexpr size_t kNoAllocScratchBytes = TNS_NOALLOC_SCRATCH_BYTES;
void scratch_setup(int device);
void *scratch_device_ptr(int device);

struct Server;

struct Ctx {
    int device = -1;
    uint64_t budget = 0;
    void *stream = nullptr;              // hipStream_t
    void *(*alloc_fn)(size_t, void *, void *) = nullptr;
    void (*free_fn)(void *, void *, void *) = nullptr;
    void *alloc_user = nullptr;
    std::mutex mu;                       // serialises synchronous calls
    std::mutex mu_stats;
    Workspace ws;                        // workspace of synchronous calls
    int64_t peak_bytes = 0;
    Server *server = nullptr;
    int serving_workers = 0;             // 0: three
    double serving_item_flops = 0;       // 0: the default work per item
    std::atomic<int> live_plans{0};      // plans holding device memory of this context
};

void *dev_alloc(Ctx *ctx, size_t bytes, void *stream);
void dev_free(Ctx *ctx, void *p, void *stream);

void plan_device_setup(Ctx *ctx, Plan &p);
void plan_device_release(Plan &p);

struct RunStats {
    double ms_bra = 0, ms_merge = 0, ms_contract = 0;
    double flops = 0;
    int64_t units = 0, launches = 0;
    bool profile = false;            // time kernel classes with events
    double ms_gemm = 0, gemm_flops = 0, gemm_bytes = 0, gemm_mfma_flops = 0;
    int64_t gemm_launches = 0;
    double ms_permute = 0, permute_bytes = 0, ms_small = 0;
    double ms_gemm3m = 0, gemm3m_flops = 0, gemm3m_mfma_flops = 0, gemm3m_bytes = 0;
    int64_t gemm3m_launches = 0;
};

// Frugal rejection on the device amplitudes: value j is accepted when
// |amp_j|^2 * scale > uniforms[j]; flags (0/1) go to the host.
struct FrugalAccept {
    const double *uniforms = nullptr;   // host, one per amplitude
    double scale = 0;                   // 2^N / M
    uint8_t *flags = nullptr;           // host, one per amplitude
};

// Amplitudes of bitstrings [0, n) into host amps (complex128 pairs), using at
// most `budget` bytes of workspace beyond the plan's resident tensors.
// With bits_dev / amps_dev (device arrays of the same layouts) the bits are
// read in place and the amplitudes written in place, without host copies or
// a final synchronisation (the call only enqueues); bits_host / amps_host
// are then unused.
void run_amplitudes(Ctx *ctx, const Plan &p, int64_t n, const uint8_t *bits_host,
                    double *amps_host, void *stream, Workspace &ws, RunStats &st,
                    const std::atomic<int> *cancel, uint64_t budget, int64_t slice_begin = 0,
                    int64_t slice_end = -1, const FrugalAccept *frugal = nullptr,
                    const uint8_t *bits_dev = nullptr, double *amps_dev = nullptr);
int64_t max_bitstrings_per_batch(const Ctx *ctx, const Plan &p, uint64_t budget, int64_t n_sl);
// Workspace bytes a fresh workspace holds after run_amplitudes(n bitstrings,
// n_sl slices) under `budget`.
uint64_t call_workspace_bytes(const Plan &p, int64_t n, int64_t n_sl, uint64_t budget);

// ----------------------------------------------------------------------------
// kernel launchers (kernels_*.hip).  All take a hipStream_t as void*.

namespace launch {
void fuse_split(const double *mats, const int32_t *chain, const int32_t *chain_off,
                const int32_t *chain_len, const FuseDesc *fuse, int n_fuse,
                double *pq, int n_qubits, const int32_t *ket_chain,
                const int32_t *bra_chain, double *ket_vec, double *bra_mat, void *stream);
void init_ket(const double *ket_vec, int q, double *site, void *stream);
void init_bra(const uint8_t *bits, int n_qubits, int64_t nb, int q, const double *bra_mat,
              double *site, int64_t stride, int open, void *stream);
void gate_apply(const double *in, double *out, int64_t nb, int64_t in_stride,
                int64_t out_stride, SiteShape s, int leg, int chi, const double *g,
                void *stream);
void svd_compress(const double *in, double *out_site, double *vp, int64_t nb,
                  int64_t in_stride, int64_t out_stride, int64_t vp_stride, SiteShape s,
                  int leg, double cutoff, void *stream);
void absorb(const double *in, const double *vp, double *out, int64_t nb, int64_t in_stride,
            int64_t vp_stride, int64_t out_stride, SiteShape s, int leg, int r,
            void *stream);
void merge(const double *ket, const double *bra, void *out, int64_t nb, int64_t bra_stride,
           int64_t out_stride, SiteShape sk, SiteShape sb, int c64, void *stream);

void gather(const void *in, void *out, int64_t units, int64_t in_unit_stride,
            int64_t out_unit_stride, const Gather &g, int elem_bytes, void *stream);
void gather_site(const void *site, void *out, int64_t units, int64_t u0, int64_t n_slices,
                 int64_t slice0, int64_t site_stride, const SliceMap &sm, int64_t out_unit_stride,
                 const Gather &g, int elem_bytes, void *stream);
void build_b(const void *site, void *out, int64_t units, int64_t u0, int64_t n_slices,
             int64_t slice0, int64_t site_stride, const SliceMap &sm, const Gather &g, int64_t K,
             int64_t N, int c64, int embed, void *stream);
// out[u][i] = pre[(u0 + u) / nper][i], i < elems (unit stride out_us): each
// (bitstring, slice) unit starts from its bitstring's slice-prefix tensor.
void expand_prefix(const void *pre, void *out, int64_t units, int64_t u0, int64_t nper, int64_t elems,
                   int64_t out_us, int elem_bytes, void *stream);
// sc: when non-null, C is stored through the fused-store tables (the row
// index includes every row of the unit, C is the unit's base).  mode 4 (the
// three-multiplication form) takes Bt as the plain complex [N][K].
void gemm(const void *A, const void *Bt, void *C, int64_t units, int64_t M, int64_t K,
          int64_t N, int64_t sA, int64_t sB, int64_t sC, int mode, void *stream,
          const ScatterStore *sc = nullptr);
// Steps with a small bond (K or N < 16, or M < 16).  With many rows and a
// small B (small_rows_fits) a block stages whole rows of A and all of B in
// LDS and may store through fused-store tables (sc); otherwise one thread per
// output element, plain stores only.
void small_contract(const void *A, const void *Bt, void *C, int64_t units, int64_t M,
                    int64_t K, int64_t N, int64_t sA, int64_t sB, int64_t sC, int c64,
                    void *stream, const ScatterStore *sc = nullptr);
void final_dot(const void *A, const void *Bt, double *partial, int64_t units, int64_t K,
               int64_t sA, int64_t sB, int c64, void *stream);
void frugal_accept(const double *amps, const double *uniforms, double scale, uint8_t *flags,
                   int64_t n, void *stream);
void slice_sum(const double *partial, double *amps, int64_t nb, int64_t n_slices, int64_t per,
               void *stream);
void finalize(const void *T, double *partial, int64_t units, int64_t t_us, int64_t per,
              const Gather &g, int c64, void *stream);
}  // namespace launch

}  // namespace tns
