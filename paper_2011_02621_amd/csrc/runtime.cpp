// Device runtime: allocation, plan upload, the resident ket evolution and the
// batched amplitude executor.  Host code only orders launches; every
// arithmetic step is a kernel (kernels_evolve.hip, kernels_contract.hip).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdio>

#include "internal.h"

namespace tns {

static void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(TNS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void *dev_alloc(Ctx *ctx, size_t bytes, void *stream) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (ctx->alloc_fn) {
        p = ctx->alloc_fn(bytes, stream, ctx->alloc_user);
        if (!p) fail(TNS_E_OUT_OF_MEMORY, "device allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(TNS_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    return p;
}

void dev_free(Ctx *ctx, void *p, void *stream) {
    if (!p) return;
    if (ctx->alloc_fn) ctx->free_fn(p, stream, ctx->alloc_user);
    else (void)hipFree(p);
}

void *Workspace::get(Ctx *ctx, int slot, size_t need, void *stream) {
    if ((int)bufs.size() <= slot) bufs.resize(slot + 1);
    DeviceBuf &b = bufs[slot];
    if (arena) {
        if (b.ptr) {
            if (b.bytes < need) fail(TNS_E_OUT_OF_MEMORY, "static workspace slot cannot grow");
            return b.ptr;
        }
        const size_t len = (std::max(need, (size_t)256) + 255) & ~(size_t)255;
        if (len > arena_cap - arena_top)
            fail(TNS_E_OUT_OF_MEMORY, "the call needs more than the " + std::to_string(arena_cap) +
                                      " bytes of the static workspace (" + std::to_string(arena_top) +
                                      " in use, " + std::to_string(len) + " more asked)");
        b.ptr = arena + arena_top;
        b.bytes = len;
        arena_top += len;
        bytes += len;
        return b.ptr;
    }
    if (b.bytes < need) {
        if (b.ptr) {
            hip_check(hipStreamSynchronize((hipStream_t)stream), "workspace sync");
            dev_free(ctx, b.ptr, stream);
            bytes -= b.bytes;
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t grow = std::max(need, (size_t)256);
        b.ptr = dev_alloc(ctx, grow, stream);
        b.bytes = grow;
        bytes += grow;
        std::lock_guard<std::mutex> lk(ctx->mu_stats);
        ctx->peak_bytes = std::max<int64_t>(ctx->peak_bytes, bytes);
    }
    return b.ptr;
}

void Workspace::release(Ctx *ctx, void *stream) {
    if (arena) {
        bufs.clear();
        bytes = 0;
        arena_top = 0;
        return;
    }
    if (!bufs.empty()) (void)hipStreamSynchronize((hipStream_t)stream);
    for (auto &b : bufs) dev_free(ctx, b.ptr, stream);
    bufs.clear();
    bytes = 0;
}

static DeviceBuf upload(Ctx *ctx, const void *host, size_t bytes, void *stream) {
    DeviceBuf b;
    b.bytes = std::max<size_t>(bytes, 8);
    b.ptr = dev_alloc(ctx, b.bytes, stream);
    if (bytes)
        hip_check(hipMemcpyAsync(b.ptr, host, bytes, hipMemcpyHostToDevice, (hipStream_t)stream),
                  "upload");
    return b;
}

// ----------------------------------------------------------------------------
// one side of the evolution on `nb` copies (Eqs. (3)-(6))

struct SideBuffers {
    std::vector<double *> buf[2];   // per site, ping-pong
    std::vector<int> cur;
    std::vector<int64_t> stride;    // per site, complex elements per copy
};

static void run_side(const Plan &p, const SideEvolution &side, SideBuffers &sb, int64_t nb,
                     double *vp, int64_t vp_stride, void *stream, int64_t &launches) {
    const double *pq = (const double *)p.d_pq.ptr;
    for (const EvoOp &op : side.ops) {
        const double *P = pq + 64 * (int64_t)op.fused;
        const double *Q = P + 32;
        const int q0 = op.q0, q1 = op.q1;
        launch::gate_apply(sb.buf[sb.cur[q0]][q0], sb.buf[1 - sb.cur[q0]][q0], nb, sb.stride[q0],
                           sb.stride[q0], op.s0, op.leg0, op.chi, P, stream);
        sb.cur[q0] ^= 1;
        launch::gate_apply(sb.buf[sb.cur[q1]][q1], sb.buf[1 - sb.cur[q1]][q1], nb, sb.stride[q1],
                           sb.stride[q1], op.s1, op.leg1, op.chi, Q, stream);
        sb.cur[q1] ^= 1;
        launches += 2;
        if (op.comp < 0) continue;
        const int k = op.comp == 0 ? q0 : q1, l = op.comp == 0 ? q1 : q0;
        SiteShape sk = op.comp == 0 ? op.s0 : op.s1, sl = op.comp == 0 ? op.s1 : op.s0;
        const int legk = op.comp == 0 ? op.leg0 : op.leg1, legl = op.comp == 0 ? op.leg1 : op.leg0;
        sk.d[1 + legk] = op.d_grown;
        sl.d[1 + legl] = op.d_grown;
        launch::svd_compress(sb.buf[sb.cur[k]][k], sb.buf[1 - sb.cur[k]][k], vp, nb, sb.stride[k],
                             sb.stride[k], vp_stride, sk, legk,
                             p.opts.svd_rel_cutoff > 0 ? p.opts.svd_rel_cutoff : 1e-12, stream);
        sb.cur[k] ^= 1;
        launch::absorb(sb.buf[sb.cur[l]][l], vp, sb.buf[1 - sb.cur[l]][l], nb, sb.stride[l], vp_stride,
                       sb.stride[l], sl, legl, op.d_after, stream);
        sb.cur[l] ^= 1;
        launches += 2;
    }
}

// ----------------------------------------------------------------------------
// plan setup: gate fusion + split on the device, resident ket

void plan_device_setup(Ctx *ctx, Plan &p) {
    void *st = ctx->stream;
    const Circuit &c = p.circ;
    std::vector<double> mats(c.gates.size() * 32);
    for (size_t i = 0; i < c.gates.size(); ++i)
        std::memcpy(&mats[32 * i], c.gates[i].m, 32 * sizeof(double));
    p.d_mats = upload(ctx, mats.data(), mats.size() * 8, st);
    p.d_chain = upload(ctx, p.chain_flat.data(), p.chain_flat.size() * 4, st);
    p.d_chain_off = upload(ctx, p.chain_off.data(), p.chain_off.size() * 4, st);
    p.d_chain_len = upload(ctx, p.chain_len.data(), p.chain_len.size() * 4, st);
    p.d_fuse = upload(ctx, p.fuse.data(), p.fuse.size() * sizeof(FuseDesc), st);
    DeviceBuf kc = upload(ctx, p.ket_init_chain.data(), p.ket_init_chain.size() * 4, st);
    DeviceBuf bc = upload(ctx, p.bra_final_chain.data(), p.bra_final_chain.size() * 4, st);
    p.d_pq.bytes = std::max<size_t>(p.fuse.size() * 64 * 8, 8);
    p.d_pq.ptr = dev_alloc(ctx, p.d_pq.bytes, st);
    p.d_ket_vec.bytes = c.n * 4 * 8;
    p.d_ket_vec.ptr = dev_alloc(ctx, p.d_ket_vec.bytes, st);
    p.d_bra_mat.bytes = c.n * 8 * 8;
    p.d_bra_mat.ptr = dev_alloc(ctx, p.d_bra_mat.bytes, st);
    launch::fuse_split((const double *)p.d_mats.ptr, (const int32_t *)p.d_chain.ptr,
                       (const int32_t *)p.d_chain_off.ptr, (const int32_t *)p.d_chain_len.ptr,
                       (const FuseDesc *)p.d_fuse.ptr, (int)p.fuse.size(), (double *)p.d_pq.ptr, c.n,
                       (const int32_t *)kc.ptr, (const int32_t *)bc.ptr, (double *)p.d_ket_vec.ptr,
                       (double *)p.d_bra_mat.ptr, st);

    // ket evolution from |0...0> (with its leading single-qubit products)
    SideBuffers sb;
    sb.buf[0].resize(c.n);
    sb.buf[1].resize(c.n);
    sb.cur.assign(c.n, 0);
    sb.stride.assign(p.ket.cap.begin(), p.ket.cap.end());
    std::vector<DeviceBuf> bufs(2 * c.n);
    for (int q = 0; q < c.n; ++q)
        for (int h = 0; h < 2; ++h) {
            bufs[2 * q + h].bytes = p.ket.cap[q] * 16;
            bufs[2 * q + h].ptr = dev_alloc(ctx, bufs[2 * q + h].bytes, st);
            sb.buf[h][q] = (double *)bufs[2 * q + h].ptr;
        }
    for (int q = 0; q < c.n; ++q) launch::init_ket((const double *)p.d_ket_vec.ptr, q, sb.buf[0][q], st);
    DeviceBuf vp;
    vp.bytes = std::max<int64_t>(p.bra_scratch_elems, 1) * 16;
    vp.ptr = dev_alloc(ctx, vp.bytes, st);
    int64_t launches = 0;
    run_side(p, p.ket, sb, 1, (double *)vp.ptr, p.bra_scratch_elems, st, launches);
    hip_check(hipStreamSynchronize((hipStream_t)st), "ket evolution");
    p.ket_site.resize(c.n);
    p.resident_bytes = 0;
    for (int q = 0; q < c.n; ++q) {
        p.ket_site[q] = bufs[2 * q + sb.cur[q]];
        dev_free(ctx, bufs[2 * q + 1 - sb.cur[q]].ptr, st);
        p.resident_bytes += p.ket_site[q].bytes;
    }
    dev_free(ctx, vp.ptr, st);
    dev_free(ctx, kc.ptr, st);
    dev_free(ctx, bc.ptr, st);

    p.resident_bytes += p.d_mats.bytes + p.d_pq.bytes + p.d_fuse.bytes + p.d_chain.bytes;
    // fused-store tables of the GEMM steps that write in the next step's order
    p.d_scatter.assign(p.steps.size(), DeviceBuf{});
    p.scatter.assign(p.steps.size(), ScatterStore{});
    for (size_t m = 0; m < p.steps.size(); ++m) {
        const Step &s = p.steps[m];
        if (!s.store_fused) continue;
        p.d_scatter[m] = upload(ctx, s.sc_tab.data(), s.sc_tab.size() * sizeof(int64_t), st);
        const int64_t *t = (const int64_t *)p.d_scatter[m].ptr;
        p.scatter[m] = ScatterStore{t, t + s.sc_na, t + s.sc_na + s.sc_nb, s.sc_shift, s.sc_mfast};
        p.resident_bytes += p.d_scatter[m].bytes;
    }
    hip_check(hipStreamSynchronize((hipStream_t)st), "plan upload");
    p.ctx = ctx;
    p.on_device = true;
}

void plan_device_release(Plan &p) {
    if (!p.on_device || !p.ctx) return;
    Ctx *ctx = p.ctx;
    void *st = ctx->stream;
    (void)hipDeviceSynchronize();
    for (DeviceBuf *b : {&p.d_mats, &p.d_chain, &p.d_chain_off, &p.d_chain_len, &p.d_fuse, &p.d_pq,
                         &p.d_ket_vec, &p.d_bra_mat}) {
        dev_free(ctx, b->ptr, st);
        b->ptr = nullptr;
    }
    for (auto &b : p.ket_site) dev_free(ctx, b.ptr, st);
    p.ket_site.clear();
    for (auto &b : p.d_scatter) dev_free(ctx, b.ptr, st);
    p.d_scatter.clear();
    p.scatter.clear();
    p.on_device = false;
}

// ----------------------------------------------------------------------------
// executor

int64_t max_bitstrings_per_batch(const Ctx *, const Plan &p, uint64_t budget, int64_t n_sl) {
    // half of the budget for per-bitstring tensors, the rest for work units
    int64_t per = p.bytes_per_bitstring + p.n_slices * 16 * p.out_per_unit + 32;
    int64_t nb = (int64_t)(budget / 2) / std::max<int64_t>(per, 1);
    nb = std::max<int64_t>(1, std::min<int64_t>(nb, 4096));
    // a shared slice prefix: as many bitstrings as an eighth of the budget
    // holds prefix tensors for (none fits: the prefix is recomputed per unit)
    if (p.prefix_steps > 0 && n_sl > 1) {
        const int64_t pb = p.prefix_elems * (p.precision != TNS_C128 ? 8 : 16);
        const int64_t cap = (int64_t)(budget / 8) / std::max<int64_t>(pb, 1);
        if (cap >= 1) nb = std::min(nb, cap);
    }
    return nb;
}

enum Slot { S_BITS = 0, S_BRA, S_VP, S_SITES, S_PARTIAL, S_AMPS, S_TX, S_TY, S_B, S_TZ, S_PRE, S_COUNT };

// The slice prefix is shared when several slices of a bitstring run in the
// call and the batch's prefix tensors take at most an eighth of the budget
// (a prefix as large as the biggest intermediates -- 2^32 elements at 104
// qubits -- is recomputed per unit instead of holding a third boundary-sized
// buffer).
static bool share_prefix(const Plan &p, int64_t nb, int64_t n_sl, uint64_t budget) {
    const int64_t elem = p.precision != TNS_C128 ? 8 : 16;
    return p.prefix_steps > 0 && n_sl > 1 && (uint64_t)(nb * p.prefix_elems * elem) <= budget / 8;
}

uint64_t call_workspace_bytes(const Plan &p, int64_t n, int64_t n_sl, uint64_t budget) {
    // mirrors the slot sizes run_amplitudes takes from a fresh workspace
    // (the first batch is the largest), in the workspace's own byte count
    if (n <= 0) return 0;
    const Circuit &c = p.circ;
    const int64_t elem = p.precision != TNS_C128 ? 8 : 16;
    const int64_t opu = p.out_per_unit;
    // the arena rounds every slot up to 256 bytes
    auto slot = [](int64_t b) { return ((uint64_t)std::max<int64_t>(b, 256) + 255) & ~(uint64_t)255; };
    int64_t bra_total = 0, site_total = 0;
    for (int q = 0; q < c.n; ++q) {
        bra_total += 2 * p.bra.cap[q];
        site_total += p.site_elems[q];
    }
    const int64_t nb = std::min<int64_t>(n, max_bitstrings_per_batch(nullptr, p, budget, n_sl));
    const int64_t units = nb * n_sl;
    uint64_t used = slot(n * opu * 16) + slot(nb * c.n) + slot(bra_total * nb * 16) +
                    slot(std::max<int64_t>(p.bra_scratch_elems, 1) * nb * 16) +
                    slot(site_total * nb * elem) + slot(units * opu * 16);
    if (share_prefix(p, nb, n_sl, budget)) used += slot(nb * p.prefix_elems * elem);
    const uint64_t left = budget > used ? budget - used : 0;
    int64_t G = (int64_t)(left / std::max<int64_t>(p.bytes_per_unit, 1));
    const int64_t fill = std::max<int64_t>(1, ((int64_t)1 << 30) / std::max<int64_t>(p.unit_stride, 1));
    G = std::max<int64_t>(1, std::min<int64_t>(std::min(G, fill), units));
    used += 2 * slot(G * p.unit_stride * elem) + slot(G * p.max_b_elems * 2 * elem);
    if (p.branch_stride) used += slot(G * p.branch_stride * elem);
    return used;
}

namespace {
struct Timer {
    hipEvent_t e[2];
    void *st;
    bool on;
    Timer(void *s, bool enable) : st(s), on(enable) {
        if (on) {
            (void)hipEventCreate(&e[0]);
            (void)hipEventCreate(&e[1]);
            (void)hipEventRecord(e[0], (hipStream_t)st);
        }
    }
    double stop() {
        if (!on) return 0;
        (void)hipEventRecord(e[1], (hipStream_t)st);
        (void)hipEventSynchronize(e[1]);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e[0], e[1]);
        (void)hipEventDestroy(e[0]);
        (void)hipEventDestroy(e[1]);
        return ms;
    }
};
}  // namespace

void run_amplitudes(Ctx *ctx, const Plan &p, int64_t n, const uint8_t *bits_host,
                    double *amps_host, void *stream, Workspace &ws, RunStats &st,
                    const std::atomic<int> *cancel, uint64_t budget, int64_t slice_begin,
                    int64_t slice_end, const FrugalAccept *frugal, const uint8_t *bits_dev_in,
                    double *amps_dev_out) {
    const Circuit &c = p.circ;
    if (slice_end < 0) slice_end = p.n_slices;
    const int64_t n_sl = slice_end - slice_begin;   // slices computed per bitstring
    const bool c64 = p.precision != TNS_C128;
    const int elem = c64 ? 8 : 16;
    const int64_t nb_max = std::min<int64_t>(n, max_bitstrings_per_batch(ctx, p, budget, n_sl));
    // phase timing syncs the host on events: only when stats are asked for
    const bool timing = st.profile;

    const int64_t opu = p.out_per_unit;   // amplitudes per bitstring (open qubits)
    double *amps_dev = amps_dev_out ? amps_dev_out
                                    : (double *)ws.get(ctx, S_AMPS, (size_t)n * opu * 16, stream);
    std::vector<char> is_open(c.n, 0);
    for (int q : c.open_qubits) is_open[q] = 1;
    int64_t bra_total = 0, site_total = 0;
    for (int q = 0; q < c.n; ++q) {
        bra_total += 2 * p.bra.cap[q];
        site_total += p.site_elems[q];
    }
    for (int64_t b0 = 0; b0 < n; b0 += nb_max) {
        if (cancel && cancel->load(std::memory_order_relaxed)) fail(TNS_E_CANCELLED, "request cancelled");
        const int64_t nb = std::min(nb_max, n - b0);
        const int64_t units = nb * n_sl;
        // every workspace slot of the batch is taken before its first launch
        uint8_t *bits_dev = bits_dev_in ? (uint8_t *)bits_dev_in + b0 * c.n
                                        : (uint8_t *)ws.get(ctx, S_BITS, (size_t)nb * c.n, stream);
        double *bra = (double *)ws.get(ctx, S_BRA, (size_t)bra_total * nb * 16, stream);
        double *vp = (double *)ws.get(ctx, S_VP, (size_t)std::max<int64_t>(p.bra_scratch_elems, 1) * nb * 16, stream);
        char *sites = (char *)ws.get(ctx, S_SITES, (size_t)site_total * nb * elem, stream);
        double *partial = (double *)ws.get(ctx, S_PARTIAL, (size_t)units * opu * 16, stream);
        // slice prefix: computed once per bitstring when several slices run
        const bool share = share_prefix(p, nb, n_sl, budget);
        char *pre = share ? (char *)ws.get(ctx, S_PRE, (size_t)nb * p.prefix_elems * elem, stream) : nullptr;
        const uint64_t used = ws.bytes;
        const uint64_t left = budget > used ? budget - used : 0;
        int64_t G = (int64_t)(left / std::max<int64_t>(p.bytes_per_unit, 1));
        // units per launch up to 2^30 boundary elements (measured on the
        // 25-qubit workload, 4 -> 32 units per launch: +4.8 %, from shorter
        // launch tails and fewer launches); the budget bounds it as well
        const int64_t fill = std::max<int64_t>(1, ((int64_t)1 << 30) / std::max<int64_t>(p.unit_stride, 1));
        G = std::max<int64_t>(1, std::min<int64_t>(std::min(G, fill), units));
        const int64_t peak = p.unit_stride;
        char *X = (char *)ws.get(ctx, S_TX, (size_t)G * peak * elem, stream);
        char *Y = (char *)ws.get(ctx, S_TY, (size_t)G * peak * elem, stream);
        char *Bb = (char *)ws.get(ctx, S_B, (size_t)G * p.max_b_elems * 2 * elem, stream);
        char *Z = p.branch_stride ? (char *)ws.get(ctx, S_TZ, (size_t)G * p.branch_stride * elem, stream) : nullptr;
        if (!bits_dev_in)
            hip_check(hipMemcpyAsync(bits_dev, bits_host + b0 * c.n, (size_t)nb * c.n,
                                     hipMemcpyHostToDevice, (hipStream_t)stream), "bits upload");

        // ---- bra evolution, batched over bitstrings
        Timer tb(stream, timing);
        SideBuffers sb;
        sb.buf[0].resize(c.n);
        sb.buf[1].resize(c.n);
        sb.cur.assign(c.n, 0);
        sb.stride.assign(p.bra.cap.begin(), p.bra.cap.end());
        {
            int64_t off = 0;
            for (int q = 0; q < c.n; ++q)
                for (int h = 0; h < 2; ++h) {
                    sb.buf[h][q] = bra + 2 * off;
                    off += p.bra.cap[q] * nb;
                }
        }
        for (int q = 0; q < c.n; ++q)
            launch::init_bra(bits_dev, c.n, nb, q, (const double *)p.d_bra_mat.ptr, sb.buf[0][q],
                             p.bra.cap[q], is_open[q], stream);
        st.launches += c.n;
        run_side(p, p.bra, sb, nb, vp, p.bra_scratch_elems, stream, st.launches);
        st.ms_bra += tb.stop();

        // ---- overlap merge (Eq. (8))
        Timer tm(stream, timing);
        std::vector<char *> site_ptr(c.n);
        {
            int64_t off = 0;
            for (int q = 0; q < c.n; ++q) {
                site_ptr[q] = sites + off * elem;
                off += p.site_elems[q] * nb;
            }
        }
        for (int q = 0; q < c.n; ++q)
            launch::merge((const double *)p.ket_site[q].ptr, sb.buf[sb.cur[q]][q], site_ptr[q], nb,
                          p.bra.cap[q], p.site_elems[q], p.ket.final_shape[q], p.bra.final_shape[q],
                          c64 ? 1 : 0, stream);
        st.launches += c.n;
        st.ms_merge += tm.stop();

        // ---- contraction of every (bitstring, slice) unit along the path
        Timer tc(stream, timing);
        // optional per-class timing: events recorded around launches on this stream
        struct Ev { hipEvent_t a, b; int cls; double flops, bytes, mfma; };
        std::vector<Ev> evs;
        auto ev_begin = [&](int cls, double fl, double by, double mfma = 0) {
            if (!st.profile) return;
            Ev e{};
            (void)hipEventCreate(&e.a);
            (void)hipEventCreate(&e.b);
            e.cls = cls; e.flops = fl; e.bytes = by; e.mfma = mfma;
            (void)hipEventRecord(e.a, (hipStream_t)stream);
            evs.push_back(e);
        };
        auto ev_end = [&]() {
            if (!st.profile) return;
            (void)hipEventRecord(evs.back().b, (hipStream_t)stream);
        };
        // Boundary buffers: X and Y hold the main path's tensor (ping-pong);
        // a branch's tensors alternate between Z and whichever of X / Y the
        // main path is not using.  An absorbed branch tensor is first copied
        // into the B operand, so its buffer is free again before the step's
        // permute and GEMM write.
        struct Buf { char *p; int64_t us; };
        const Buf bx{X, peak}, by{Y, peak}, bz{Z, p.branch_stride};
        // Steps [m0, m1) on g units: unit u is bitstring (u0 + u) / nper of
        // the batch and slice s0 + (u0 + u) % nper; cur_main holds the main
        // tensor when m0 > 0; last (if set) receives the output of step m1 - 1.
        auto run_steps = [&](size_t m0, size_t m1, int64_t g, int64_t u0, int64_t nper, int64_t s0,
                             Buf cur_main, const Buf *last) {
            Buf cur_br{nullptr, 0};
            auto free_main = [&]() { return cur_main.p == X ? by : bx; };
            for (size_t m = m0; m < m1; ++m) {
                const Step &s = p.steps[m];
                const bool main = s.chain == 0;
                if (s.start) {
                    const Buf to = main ? bx : bz;
                    launch::gather_site(site_ptr[s.site], to.p, g, u0, nper, s0, p.site_elems[s.site],
                                        p.slice_map[s.site], to.us, s.bgather, elem, stream);
                    (main ? cur_main : cur_br) = to;
                    st.launches += 1;
                    continue;
                }
                // B[n][k] from the absorbed tensor: the real-embedded GEMM takes its
                // real embedding, the three-multiplication GEMM and the small kernels
                // the plain complex matrix
                if (s.branch < 0)
                    launch::build_b(site_ptr[s.site], Bb, g, u0, nper, s0, p.site_elems[s.site],
                                    p.slice_map[s.site], s.bgather, s.K, s.N, c64 ? 1 : 0,
                                    s.kernel == 0 ? 1 : 0, stream);
                else
                    launch::build_b(cur_br.p, Bb, g, 0, 1, 0, cur_br.us, SliceMap{}, s.bgather, s.K, s.N,
                                    c64 ? 1 : 0, s.kernel == 0 ? 1 : 0, stream);
                const Buf cur = main ? cur_main : cur_br;
                auto other_of = [&](const Buf &b) {
                    if (main) return b.p == X ? by : bx;
                    return b.p == Z ? free_main() : bz;
                };
                Buf src = cur;
                if (s.permute && !s.permute_fused) {
                    int64_t te = 1;
                    for (int a = 0; a < s.perm.n; ++a) te *= s.perm.size[a];
                    const Buf o = other_of(cur);
                    ev_begin(1, 0, 2.0 * elem * te * g);
                    launch::gather(cur.p, o.p, g, cur.us, o.us, s.perm, elem, stream);
                    ev_end();
                    src = o;
                    st.launches += 1;
                }
                const Buf dst = (last && m + 1 == m1) ? *last : other_of(src);
                const double mkn = (double)s.M * s.K * s.N * g;
                const double bytes = (double)elem * ((double)s.M * s.K + (double)s.K * s.N + (double)s.M * s.N) * g;
                const bool is_gemm = s.kernel == 0 || s.kernel == 3;
                // real flops the MFMA instructions execute: 8 M K N for the real
                // embedding, 6 M K N for the three-multiplication form, times the
                // number of products of a split-BF16 form; class 3 is k_gemm_3m
                // (the short-K and split-K steps count with the other GEMMs)
                const double prod = p.precision == TNS_C64_SPLIT_BF16_3 ? 3.0
                                    : p.precision == TNS_C64_SPLIT_BF16_6 ? 6.0 : 1.0;
                const bool k3m = s.kernel == 3 && !gemm_3m_short_k(s.K) && !gemm_3m_splitk(s.M, s.K, s.N, g, dst.us);
                ev_begin(k3m ? 3 : is_gemm ? 0 : 2, 8.0 * mkn, bytes,
                         (s.kernel == 3 && !gemm_3m_splitk(s.M, s.K, s.N, g, dst.us) ? 6.0 : 8.0 * prod) * mkn);
                if (s.kernel == 0)
                    launch::gemm(src.p, Bb, dst.p, g, s.M, s.K, s.N, src.us, s.K * s.N, dst.us, p.precision,
                                 stream, s.store_fused ? &p.scatter[m] : nullptr);
                else if (s.kernel == 3)
                    launch::gemm(src.p, Bb, dst.p, g, s.M, s.K, s.N, src.us, s.K * s.N, dst.us, 4, stream,
                                 s.store_fused ? &p.scatter[m] : nullptr);
                else if (s.kernel == 1)
                    launch::small_contract(src.p, Bb, dst.p, g, s.M, s.K, s.N, src.us, s.K * s.N, dst.us,
                                           c64 ? 1 : 0, stream, s.store_fused ? &p.scatter[m] : nullptr);
                else
                    launch::final_dot(src.p, Bb, partial + 2 * u0, g, s.K, src.us, s.K, c64 ? 1 : 0, stream);
                ev_end();
                if (m + 1 == p.steps.size() && s.kernel != 2) {
                    // open legs: the last tensor holds this unit's 2^open values
                    launch::finalize(dst.p, partial + 2 * u0 * opu, g, dst.us, opu, p.final_perm,
                                     c64 ? 1 : 0, stream);
                    st.launches += 1;
                }
                st.launches += 2;
                (main ? cur_main : cur_br) = dst;
            }
        };
        // the slice prefix, once per bitstring of the batch (G at a time)
        const size_t P = share ? (size_t)p.prefix_steps : 0;
        for (int64_t pb0 = 0; share && pb0 < nb; pb0 += G) {
            if (cancel && cancel->load(std::memory_order_relaxed)) fail(TNS_E_CANCELLED, "request cancelled");
            const int64_t g = std::min(G, nb - pb0);
            const Buf out{pre + (size_t)pb0 * p.prefix_elems * elem, p.prefix_elems};
            run_steps(0, P, g, pb0, 1, 0, Buf{nullptr, 0}, &out);
        }
        for (int64_t ug0 = 0; ug0 < units; ug0 += G) {
            if (cancel && cancel->load(std::memory_order_relaxed)) fail(TNS_E_CANCELLED, "request cancelled");
            const int64_t g = std::min(G, units - ug0);
            Buf start{nullptr, 0};
            if (share) {
                // every unit starts from its bitstring's prefix tensor
                launch::expand_prefix(pre, X, g, ug0, n_sl, p.prefix_elems, peak, elem, stream);
                st.launches += 1;
                start = bx;
            }
            run_steps(P, p.steps.size(), g, ug0, n_sl, slice_begin, start, nullptr);
        }
        launch::slice_sum(partial, amps_dev + 2 * b0 * opu, nb, n_sl, opu, stream);
        st.launches += 1;
        st.ms_contract += tc.stop();
        for (Ev &e : evs) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e.a, e.b);
            if (e.cls == 3) {
                st.ms_gemm3m += ms;
                st.gemm3m_flops += e.flops;
                st.gemm3m_bytes += e.bytes;
                st.gemm3m_mfma_flops += e.mfma;
                st.gemm3m_launches++;
            }
            if (e.cls == 0 || e.cls == 3) {
                st.ms_gemm += ms;
                st.gemm_flops += e.flops;
                st.gemm_bytes += e.bytes;
                st.gemm_mfma_flops += e.mfma;
                st.gemm_launches++;
            }
            else if (e.cls == 1) { st.ms_permute += ms; st.permute_bytes += e.bytes; }
            else st.ms_small += ms;
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        st.units += units;
        st.flops += p.flops_per_amp * nb * ((double)n_sl / (double)p.n_slices);
    }
    if (frugal) {
        const int64_t na = n * opu;
        double *u_dev = (double *)ws.get(ctx, S_BITS, (size_t)na * 9, stream);
        uint8_t *f_dev = (uint8_t *)(u_dev + na);
        hip_check(hipMemcpyAsync(u_dev, frugal->uniforms, (size_t)na * 8, hipMemcpyHostToDevice,
                                 (hipStream_t)stream), "uniforms upload");
        launch::frugal_accept(amps_dev, u_dev, frugal->scale, f_dev, na, stream);
        hip_check(hipMemcpyAsync(frugal->flags, f_dev, (size_t)na, hipMemcpyDeviceToHost,
                                 (hipStream_t)stream), "flags download");
    }
    if (amps_dev_out) return;   // results stay on the device, ordered on `stream`
    hip_check(hipMemcpyAsync(amps_host, amps_dev, (size_t)n * opu * 16, hipMemcpyDeviceToHost,
                             (hipStream_t)stream), "amplitude download");
    hip_check(hipStreamSynchronize((hipStream_t)stream), "amplitudes");
}

}  // namespace tns
