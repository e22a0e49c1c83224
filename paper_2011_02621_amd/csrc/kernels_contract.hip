// Contraction-side kernels (supplement: C^{i_1..i_{m+1}} = contract(C^{i_1..i_m},
// C^{i_{m+1}}), one pairwise step at a time):
//   gather / gather_site -- strided copies: boundary permutes, the starting
//                           tensor, slice selection of cut bonds
//   build_b              -- the site tensor as B[n][k] (k fastest), either plain
//                           complex or as the real embedding of a complex matrix
//   gemm                 -- complex GEMM T'[M,N] = T[M,K] B[K,N] as one real GEMM
//                           [M,2K] x [2K,2N] on the MFMA cores (4 real products):
//                           complex64 on FP32 MFMA, complex128 on FP64 MFMA
//   small_contract       -- thread-per-output contraction for small K or N
//   final_dot            -- last step (scalar): widened to FP64
//   slice_sum            -- FP64 sum of the slices of each bitstring (overlap
//                           paragraph: the sub-network scalars add up)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace tns {
namespace {

inline unsigned grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 65536 * 4) g = 65536 * 4;
    if (g < 1) g = 1;
    return (unsigned)g;
}

inline void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(TNS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

__device__ __forceinline__ int64_t slice_offset(const SliceMap &sm, int64_t s) {
    int64_t off = 0;
    for (int c = 0; c < sm.n; ++c) off += ((s / sm.div[c]) % sm.dim[c]) * sm.stride[c];
    return off;
}

__device__ __forceinline__ int64_t gather_offset(const Gather &g, int64_t i) {
    int64_t off = 0;
    for (int a = g.n - 1; a >= 0; --a) {
        const int64_t s = g.size[a];
        const int64_t q = i / s;
        off += (i - q * s) * g.stride[a];
        i = q;
    }
    return off;
}

// ---------------------------------------------------------------------------
// strided gathers.  E is the complex element (float2 or double2).

template <typename E>
__global__ void k_gather(const E *__restrict__ in, E *__restrict__ out, int64_t units,
                         int64_t in_us, int64_t out_us, Gather g, int64_t per) {
    const int64_t total = per * units;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / per, i = t - u * per;
        out[u * out_us + i] = in[u * in_us + gather_offset(g, i)];
    }
}

// Strided gather with 32-bit index arithmetic (64-bit integer division is a
// long instruction sequence on CDNA), valid when one unit holds fewer than
// 2^31 elements (the launcher checks).  Units come from blockIdx.y.  With
// VEC = 2 (complex64, output-fastest axis contiguous in the input and of even
// size) each copy moves two elements with one 16-byte load and store; every
// thread keeps four copies in flight.
template <typename E, int VEC>
__global__ __launch_bounds__(256) void k_gather32(const E *__restrict__ in, E *__restrict__ out,
                                                   int64_t in_us, int64_t out_us, Gather g,
                                                   uint32_t per) {
    using V = typename std::conditional<VEC == 2, float4, E>::type;
    const int n = g.n;
    const E *src = in + blockIdx.y * in_us;
    E *dst = out + blockIdx.y * out_us;
    const uint32_t nv = per / VEC;
    const uint32_t step = gridDim.x * blockDim.x;
    for (uint32_t v0 = blockIdx.x * blockDim.x + threadIdx.x; v0 < nv; v0 += 4 * step) {
        V val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t v = v0 + u * step;
            if (v < nv) {
                uint32_t r = v * VEC, off = 0;
                for (int a = n - 1; a >= 0; --a) {
                    const uint32_t sz = (uint32_t)g.size[a];
                    const uint32_t q = r / sz;
                    off += (r - q * sz) * (uint32_t)g.stride[a];
                    r = q;
                }
                val[u] = *reinterpret_cast<const V *>(src + off);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t v = v0 + u * step;
            if (v < nv) *reinterpret_cast<V *>(dst + (size_t)v * VEC) = val[u];
        }
    }
}

// LDS-tiled permute.  The output is row-major over g.size; g.stride gives
// each output axis's input stride.  Axis ai is the input-contiguous axis
// (input stride 1) and axis ao the output-contiguous one (the last output
// axis); a tile covers up to 64 x 64 (ai, ao) positions and is read along ai
// (coalesced reads), staged in LDS and written along ao (coalesced writes).
// Every other axis, and the unit, is one coordinate of the tile index.
struct PermTile {
    int32_t n;                 // axes
    int32_t ai, ao;            // input- and output-contiguous axes
    int32_t ti, to;            // tile extents along ai and ao
    int64_t size[kMaxGatherDims];
    int64_t in_stride[kMaxGatherDims];
    int64_t out_stride[kMaxGatherDims];
    int64_t tiles_i, tiles_o;  // tiles along ai and ao
    int64_t tiles_per_unit;
};

template <typename E>
__global__ __launch_bounds__(256) void k_permute_tiled(const E *__restrict__ in, E *__restrict__ out,
                                                        int64_t units, int64_t in_us, int64_t out_us,
                                                        PermTile pt) {
    __shared__ E tile[64 * 65];
    const int64_t total = pt.tiles_per_unit * units;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int64_t u = t / pt.tiles_per_unit;
        int64_t r = t - u * pt.tiles_per_unit;
        const int64_t tio = r % pt.tiles_o; r /= pt.tiles_o;
        const int64_t tii = r % pt.tiles_i; r /= pt.tiles_i;
        int64_t base_in = u * in_us, base_out = u * out_us;
        for (int a = pt.n - 1; a >= 0; --a) {
            if (a == pt.ai || a == pt.ao) continue;
            const int64_t c = r % pt.size[a];
            r /= pt.size[a];
            base_in += c * pt.in_stride[a];
            base_out += c * pt.out_stride[a];
        }
        const int64_t i0 = tii * pt.ti, o0 = tio * pt.to;
        const int ni = (int)min<int64_t>(pt.ti, pt.size[pt.ai] - i0);
        const int no = (int)min<int64_t>(pt.to, pt.size[pt.ao] - o0);
        __syncthreads();
        for (int e = threadIdx.x; e < ni * no; e += 256) {
            const int o = e / ni, i = e - o * ni;
            tile[o * 65 + i] = in[base_in + (i0 + i) + (o0 + o) * pt.in_stride[pt.ao]];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ni * no; e += 256) {
            const int i = e / no, o = e - i * no;
            out[base_out + (o0 + o) + (i0 + i) * pt.out_stride[pt.ai]] = tile[o * 65 + i];
        }
    }
}

// unit u of this launch is global unit ug = u0 + u = bitstring * n_slices + j,
// computing slice slice0 + j
// the slice prefix of a unit's bitstring copied into the unit's buffer
template <typename E>
__global__ void k_expand_prefix(const E *__restrict__ pre, E *__restrict__ out, int64_t units, int64_t u0,
                                int64_t nper, int64_t elems, int64_t out_us) {
    const int64_t total = units * elems;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / elems, i = t - u * elems;
        out[u * out_us + i] = pre[((u0 + u) / nper) * elems + i];
    }
}

template <typename E>
__global__ void k_gather_site(const E *__restrict__ site, E *__restrict__ out, int64_t units,
                              int64_t u0, int64_t n_slices, int64_t slice0, int64_t site_stride,
                              SliceMap sm, int64_t out_us, Gather g,
                              int64_t per) {
    const int64_t total = per * units;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / per, i = t - u * per;
        const int64_t ug = u0 + u;
        const int64_t b = ug / n_slices, s = slice0 + ug - b * n_slices;
        const int64_t base = b * site_stride + slice_offset(sm, s);
        out[u * out_us + i] = site[base + gather_offset(g, i)];
    }
}

// B[n][k] from the site tensor; with embed, the real matrix Bt[2N][2K]
// (k fastest) whose product with the interleaved [M][2K] view of T yields the
// interleaved complex result [M][2N]:
//   Bt[2n][2k] = Re b, Bt[2n][2k+1] = -Im b, Bt[2n+1][2k] = Im b, Bt[2n+1][2k+1] = Re b.
template <typename R>
__global__ void k_build_b(const R *__restrict__ site, R *__restrict__ out, int64_t units,
                          int64_t u0, int64_t n_slices, int64_t slice0, int64_t site_stride,
                          SliceMap sm, Gather g, int64_t K, int64_t N,
                          int embed) {
    const int64_t per = K * N;
    const int64_t total = per * units;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / per, i = t - u * per;
        const int64_t ug = u0 + u;
        const int64_t b = ug / n_slices, s = slice0 + ug - b * n_slices;
        const int64_t src = b * site_stride + slice_offset(sm, s) + gather_offset(g, i);
        const R re = site[2 * src], im = site[2 * src + 1];
        if (!embed) {
            out[2 * (u * per + i)] = re;
            out[2 * (u * per + i) + 1] = im;
        } else {
            const int64_t n = i / K, k = i - n * K;
            R *o = out + u * 4 * per;
            const int64_t ld = 2 * K;
            o[(2 * n) * ld + 2 * k] = re;
            o[(2 * n) * ld + 2 * k + 1] = -im;
            o[(2 * n + 1) * ld + 2 * k] = im;
            o[(2 * n + 1) * ld + 2 * k + 1] = re;
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 MFMA GEMM: C[M][Nr] = A[M][Kr] * Bt[Nr][Kr]^T, all row-major, Kr % 4 == 0.
// 256 threads, tile 128 x 128, k-step 32.  Four waves in a 2 x 2 layout, each
// owning 64 x 64 as 2 x 2 blocks of v_mfma_f32_32x32x2f32.  The two k-slots
// of one MFMA (lanes 0-31 / 32-63) are mapped to k = 4*slot + t for the four
// MFMAs t = 0..3 of an 8-wide k group, so each lane reads its four A (and B)
// values with one 16-byte LDS load.

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// Tile order: consecutive workgroup ids are dispatched round-robin over the
// 8 XCDs, each with its own L2.  Remap so that each XCD receives a contiguous
// run of logical tiles (row-major over (tile_m, tile_n)), i.e. the tiles that
// share rows of A, and so their A reads, stay on one XCD.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t ntiles) {
    const int64_t per = ntiles / 8;
    if (per == 0) return b;
    const int64_t main = per * 8;
    if (b >= main) return b;
    return (b & 7) * per + (b >> 3);
}

// Split-BF16: each FP32 operand x is split by round-to-nearest-even into bf16
// parts, x = hi + mid (+ lo), and the product is summed from the significant
// part products on the BF16 MFMA cores with FP32 accumulation:
//   NSPLIT = 2: hi*hi + hi*mid + mid*hi                          (3 products)
//   NSPLIT = 3: the same plus hi*lo + mid*mid + lo*hi            (6 products)
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <int NSPLIT>
__device__ __forceinline__ void split_store(__bf16 *dst, int part_stride, v4f v) {
    bf16x4 h, m, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float x = v[e];
        const __bf16 a = (__bf16)x;
        const float r1 = x - (float)a;
        const __bf16 b = (__bf16)r1;
        h[e] = a;
        m[e] = b;
        if (NSPLIT == 3) l[e] = (__bf16)(r1 - (float)b);
    }
    *reinterpret_cast<bf16x4 *>(dst) = h;
    *reinterpret_cast<bf16x4 *>(dst + part_stride) = m;
    if (NSPLIT == 3) *reinterpret_cast<bf16x4 *>(dst + 2 * part_stride) = l;
}

// Orders one wave's LDS stores before its own later LDS loads (and the loads
// before its next stores): the staging area of the fused store is private to
// the wave, so no block barrier is needed.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Target offsets of a block's fused store, read from the tables once and
// kept in LDS: ofs_r[i] for row rb0 + i of the launch (-1 past M), ofs_c[c]
// for complex column cb0 + c (-1 past N).  Called by all 256 threads before
// the k-loop, whose barriers publish it.  The store loops then read offsets
// from LDS only: a table read from global memory between two stores waits
// on the vector-memory counter, which also counts the wave's stores still in
// flight, and so would hold every store until the previous ones completed.
__device__ __forceinline__ void fused_offsets(int64_t *ofs_r, int nr, int64_t *ofs_c, int nc,
                                              const ScatterStore &sc, int64_t row0, int64_t rb0, int64_t M,
                                              int64_t cb0, int64_t N, int tid) {
    const int64_t mask = ((int64_t)1 << sc.shift) - 1;
    for (int i = tid; i < nr; i += 256) {
        const int64_t row = rb0 + i;
        int64_t v = -1;
        if (row < M) {
            const int64_t gr = row0 + row;
            v = sc.fa[gr >> sc.shift] + sc.fb[gr & mask];
        }
        ofs_r[i] = v;
    }
    for (int c = tid; c < nc; c += 256) {
        const int64_t col = cb0 + c;
        ofs_c[c] = col < N ? sc.fg[col] : -1;
    }
}

// Fused store of one wave's tile (WR rows, BJ slices of CW complex columns),
// staged through LDS: stage(j) writes slice j into stg (row stride SLD
// reals), then each lane stores whole complex values V in the order in
// which the target is contiguous (rows when mfast, else columns).  ofs_r
// and ofs_c (fused_offsets, in LDS) start at the wave's first row and first
// complex column.  64 is a multiple of WR and of CW, so a lane keeps one row
// (row order) or one column (column order) across its stores.
template <typename V, int WR, int CW, int SLD, int BJ, typename R, typename Stage>
__device__ __forceinline__ void fused_store_wave(R *__restrict__ C, R *stg, int mfast, const int64_t *ofs_r,
                                                 const int64_t *ofs_c, int lane, Stage stage) {
    static_assert(64 % WR == 0 && 64 % CW == 0, "lane-invariant row or column");
    constexpr int PER = WR * CW / 64;   // stores per lane and slice
    if (mfast) {
        const int lr = lane % WR;
        const int64_t ro = ofs_r[lr];
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            stage(j);
            wave_sync();
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int lc = lane / WR + k * (64 / WR);
                const int64_t co = ofs_c[j * CW + lc];
                if (ro >= 0 && co >= 0)
                    *reinterpret_cast<V *>(C + 2 * (ro + co)) = *reinterpret_cast<const V *>(&stg[lr * SLD + 2 * lc]);
            }
            wave_sync();
        }
    } else {
        const int lc = lane % CW;
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            stage(j);
            wave_sync();
            const int64_t co = ofs_c[j * CW + lc];
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const int lr = lane / CW + k * (64 / CW);
                const int64_t ro = ofs_r[lr];
                if (ro >= 0 && co >= 0)
                    *reinterpret_cast<V *>(C + 2 * (ro + co)) = *reinterpret_cast<const V *>(&stg[lr * SLD + 2 * lc]);
            }
            wave_sync();
        }
    }
}

// C[M][Nr] = A[M][Kr] * Bt[Nr][Kr]^T, row-major, Kr % 4 == 0.  256 threads =
// 4 waves in a WGM x WGN layout; each wave owns BI x BJ blocks of 32 x 32, so
// the tile is (WGM*BI*32) x (WGN*BJ*32), k-step BK reals.  The next k-tile is
// fetched into registers while the current one is multiplied out of LDS.
// NSTAGE = 2 keeps two LDS k-tiles, so the next one is stored half-way
// through the current one and a k-step needs one barrier; it doubles the LDS
// of a block, which pays where two blocks still fit on a CU (the 128 x 128
// tile) and costs occupancy on the narrow tiles, which keep NSTAGE = 1.
// MODE 1: FP32 operands, v_mfma_f32_32x32x2f32; the two k-slots of an MFMA
// (lanes 0-31 / 32-63) take k = 4*slot + t for the four MFMAs t of an
// 8-wide k group, so each lane reads its values with one 16-byte LDS load.
// MODE 2 / 3: split-BF16 with 3 / 6 products, v_mfma_f32_32x32x16_bf16, a
// lane supplying 8 consecutive k of its row (A) and of its column (B).
// SCAT: the result is stored through fused-store tables (ScatterStore): the
// complex element (row0 + row, col / 2) of the unit goes to
// fa[r >> shift] + fb[r & mask] + fg[col / 2], the next step's order.
template <int BI, int BJ, int WGM, int WGN, int MODE, int NSTAGE, int BK, bool SCAT>
__global__ __launch_bounds__(256) void k_gemm_c64(const float *__restrict__ A,
                                                   const float *__restrict__ Bt,
                                                   float *__restrict__ C, int64_t M, int Kr, int Nr,
                                                   int64_t sA, int64_t sB, int64_t sC, int tiles_n,
                                                   ScatterStore sc, int64_t row0) {
    static_assert(WGM * WGN == 4, "four waves");
    constexpr int BM = WGM * BI * 32, BN = WGN * BJ * 32;
    constexpr int NSPLIT = MODE == 1 ? 1 : MODE;          // 1, 2 or 3 parts
    static_assert(BK == 16 || BK == 32, "k-step of 16 or 32 reals");
    constexpr int LD = MODE == 1 ? BK + 4 : BK + 8;   // padded row (elements)
    using ET = typename std::conditional<MODE == 1, float, __bf16>::type;
    constexpr int APART = BM * LD, BPART = BN * LD;
    static_assert(NSTAGE == 1 || NSTAGE == 2, "one or two LDS stages");
    // one LDS array: the A stages, then the B stages (the fused store stages
    // its output through all of it after the k-loop)
    constexpr int SMEM = NSTAGE * NSPLIT * (APART + BPART);
    __shared__ ET smem[SMEM];
    __shared__ int64_t fofs[SCAT ? BM + BN / 2 : 1];   // fused-store offsets: rows, then complex columns
    auto As = [&](int st) { return smem + st * NSPLIT * APART; };
    auto Bs = [&](int st) { return smem + NSTAGE * NSPLIT * APART + st * NSPLIT * BPART; };
    // a k-tile row is BK/4 float4; 256 threads cover RPP rows per pass;
    // float4 loads per thread, a B tile narrower than one pass leaving the
    // threads with lrow >= BN idle
    constexpr int TPR = BK / 4, RPP = 256 / TPR;
    constexpr int AV = BM / RPP, BV = (BN + RPP - 1) / RPP;
    constexpr bool BPART_PASS = BN % RPP != 0;
    const int64_t u = blockIdx.y;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / tiles_n, tn = tile - tm * tiles_n;
    const int64_t m0 = tm * BM;
    const int n0 = (int)tn * BN;
    A += u * sA;
    Bt += u * sB;
    C += u * sC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    if constexpr (SCAT) fused_offsets(fofs, BM, fofs + BM, BN / 2, sc, row0, m0, M, n0 / 2, Nr / 2, tid);
    v16f acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int lrow = tid / TPR, lcol = (tid % TPR) * 4;
    v4f ra[AV], rb[BV];
    // Row pointers clamped into the operands: a row past M (or Nr) loads the
    // last valid row, whose products are never stored, so a full k-tile is
    // fetched without guards or branches; only a partial last k-tile checks k
    // (the two-stage tiles).
    const float *ap[AV], *bp[BV];
#pragma unroll
    for (int i = 0; i < AV; ++i) ap[i] = A + std::min<int64_t>(m0 + lrow + RPP * i, M - 1) * Kr + lcol;
#pragma unroll
    for (int i = 0; i < BV; ++i) bp[i] = Bt + (int64_t)std::min(n0 + lrow + RPP * i, Nr - 1) * Kr + lcol;
    auto fetch = [&](int k0) {
        if (k0 + BK <= Kr) {
#pragma unroll
            for (int i = 0; i < AV; ++i) ra[i] = *reinterpret_cast<const v4f *>(ap[i] + k0);
#pragma unroll
            for (int i = 0; i < BV; ++i) rb[i] = *reinterpret_cast<const v4f *>(bp[i] + k0);
        } else {
            const bool in = k0 + lcol < Kr;
#pragma unroll
            for (int i = 0; i < AV; ++i) ra[i] = in ? *reinterpret_cast<const v4f *>(ap[i] + k0) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < BV; ++i) rb[i] = in ? *reinterpret_cast<const v4f *>(bp[i] + k0) : v4f{0.f, 0.f, 0.f, 0.f};
        }
    };
    // the single-stage narrow tiles keep per-row guards (measured faster there)
    auto fetch_guarded = [&](int k0) {
        const int gk = k0 + lcol;
#pragma unroll
        for (int i = 0; i < AV; ++i) {
            const int64_t gm = m0 + lrow + RPP * i;
            ra[i] = v4f{0.f, 0.f, 0.f, 0.f};
            if (gm < M && gk < Kr) ra[i] = *reinterpret_cast<const v4f *>(A + gm * Kr + gk);
        }
#pragma unroll
        for (int i = 0; i < BV; ++i) {
            const int gn = n0 + lrow + RPP * i;
            rb[i] = v4f{0.f, 0.f, 0.f, 0.f};
            if (gn < Nr && gk < Kr && (!BPART_PASS || lrow + RPP * i < BN))
                rb[i] = *reinterpret_cast<const v4f *>(Bt + (int64_t)gn * Kr + gk);
        }
    };
    auto stash = [&](int stage) {
#pragma unroll
        for (int i = 0; i < AV; ++i) {
            ET *dst = As(stage) + (lrow + RPP * i) * LD + lcol;
            if constexpr (MODE == 1) *reinterpret_cast<v4f *>(dst) = ra[i];
            else split_store<NSPLIT>(dst, APART, ra[i]);
        }
#pragma unroll
        for (int i = 0; i < BV; ++i) {
            if (BPART_PASS && lrow + RPP * i >= BN) continue;
            ET *dst = Bs(stage) + (lrow + RPP * i) * LD + lcol;
            if constexpr (MODE == 1) *reinterpret_cast<v4f *>(dst) = rb[i];
            else split_store<NSPLIT>(dst, BPART, rb[i]);
        }
    };
    // Fragments of one k-group (8 reals for MODE 1, 16 for MODE 2 / 3); the
    // two-stage tiles keep two register sets, so the next group's LDS reads
    // are in flight during the current group's MFMAs.
    constexpr int KG = MODE == 1 ? 8 : 16, NG = BK / KG;
    using FT = typename std::conditional<MODE == 1, v4f, bf16x8>::type;
    FT fa[2][BI][NSPLIT], fb[2][BJ][NSPLIT];
    const int arow = (wm * BI * 32 + (lane & 31)) * LD + (KG / 2) * (lane >> 5);
    const int brow = (wn * BJ * 32 + (lane & 31)) * LD + (KG / 2) * (lane >> 5);
    auto frags = [&](int buf, const ET *Ac, const ET *Bc, int kk) {
#pragma unroll
        for (int p = 0; p < NSPLIT; ++p) {
#pragma unroll
            for (int i = 0; i < BI; ++i)
                fa[buf][i][p] = *reinterpret_cast<const FT *>(&Ac[p * APART + arow + i * 32 * LD + kk]);
#pragma unroll
            for (int j = 0; j < BJ; ++j)
                fb[buf][j][p] = *reinterpret_cast<const FT *>(&Bc[p * BPART + brow + j * 32 * LD + kk]);
        }
    };
    auto mfma_group = [&](int buf) {
        if constexpr (MODE == 1) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < BI; ++i)
#pragma unroll
                    for (int j = 0; j < BJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[buf][i][0][t], fb[buf][j][0][t], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int i = 0; i < BI; ++i)
#pragma unroll
                for (int j = 0; j < BJ; ++j) {
                    // smallest terms first
                    if constexpr (NSPLIT == 3) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][i][2], fb[buf][j][0], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][i][1], fb[buf][j][1], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][i][0], fb[buf][j][2], acc[i][j], 0, 0, 0);
                    }
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][i][1], fb[buf][j][0], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][i][0], fb[buf][j][1], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[buf][i][0], fb[buf][j][0], acc[i][j], 0, 0, 0);
                }
        }
    };
    if constexpr (NSTAGE == 2) {
        // Two LDS stages and two register k-tiles in flight: tile t+1 is
        // already in registers when tile t starts; half-way through tile t it
        // goes to the other stage (last read in tile t-1, before the previous
        // barrier) and the fetch of tile t+2 is issued, so global latency
        // spans a whole tile and the barrier at the end waits on no store.
        constexpr int MID = NG > 1 ? NG / 2 - 1 : 0;
        fetch(0);
        stash(0);
        if (BK < Kr) fetch(BK);
        __syncthreads();
        int stage = 0;
        for (int k0 = 0; k0 < Kr; k0 += BK) {
            const bool more = k0 + BK < Kr, more2 = k0 + 2 * BK < Kr;
            // compiler strategy that interleaves the MFMAs with the LDS reads:
            // measured +1.3-1.6 % on the 128 x 256 FP32 tile, no gain or a
            // loss on the other tiles and modes
            if constexpr (MODE == 1 && BJ == 4) __builtin_amdgcn_iglp_opt(1);
            const ET *Ac = As(stage), *Bc = Bs(stage);
            frags(0, Ac, Bc, 0);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (g + 1 < NG) frags((g + 1) & 1, Ac, Bc, (g + 1) * KG);
                mfma_group(g & 1);
                if (g == MID && more) {
                    stash(stage ^ 1);
                    if (more2) fetch(k0 + 2 * BK);
                }
            }
            __syncthreads();
            stage ^= 1;
        }
    } else {
        fetch_guarded(0);
        stash(0);
        __syncthreads();
        for (int k0 = 0; k0 < Kr; k0 += BK) {
            const bool more = k0 + BK < Kr;
            if (more) fetch_guarded(k0 + BK);
            const ET *Ac = As(0), *Bc = Bs(0);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                frags(0, Ac, Bc, g * KG);
                mfma_group(0);
            }
            __syncthreads();
            if (more) {
                stash(0);
                __syncthreads();
            }
        }
    }
    // 32x32 accumulator layout: lane holds column lane%32 and rows
    // 8*(r/4) + 4*(lane/32) + r%4 for its 16 values r.
    if constexpr (!SCAT) {
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = m0 + wm * BI * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int col = n0 + wn * BJ * 32 + j * 32 + (lane & 31);
                    if (row < M && col < Nr) C[row * Nr + col] = acc[i][j][r];
                }
    } else {
        // Fused store, staged per wave through LDS (the operand stages are
        // free after the k-loop's last barrier): each 32-column slice of the
        // wave's tile is written in the accumulator layout and read back one
        // complex value per lane in the order in which the target is
        // contiguous (rows when sc.mfast, else columns).
        constexpr int WR = BI * 32;   // rows of the wave's tile
        constexpr int CW = 16;        // complex columns of a slice
        constexpr int SLD = 34;       // staging row: 32 floats + 2 (keeps float2 alignment)
        static_assert(4 * WR * SLD * sizeof(float) <= SMEM * sizeof(ET), "staging fits in the stages");
        float *stg = reinterpret_cast<float *>(smem) + wave * WR * SLD;
        fused_store_wave<float2, WR, CW, SLD, BJ>(
            C, stg, sc.mfast, fofs + wm * WR, fofs + BM + wn * BJ * 16, lane, [&](int j) {
#pragma unroll
                for (int i = 0; i < BI; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        stg[(i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * SLD + (lane & 31)] = acc[i][j][r];
            });
    }
}

// Complex64 GEMM in the three-multiplication form on FP32 MFMA:
// C[M][N] = A[M][K] B[N][K]^T with A, B, C complex (interleaved re, im) and
//   T0 = Ar Br^T, T1 = Ai Bi^T, T2 = (Ar + Ai)(Br + Bi)^T,
//   Re C = T0 - T1, Im C = T2 - T0 - T1,
// three real products of M x K x N instead of the four that the real
// embedding of the other kernels multiplies (6 M K N flops instead of 8).
// Loads read interleaved complex pairs; the LDS store writes two planes (re,
// im) of A and of B, and the (re + im) operands are formed in registers
// right before the MFMAs that take them (a third of the LDS traffic and 36 KB
// of LDS per block instead of 55 KB; +1.7 % on the 53-qubit depth-12 slices,
// results unchanged: the same FP32 sum, formed later).  Four waves in 2 x 2,
// each owning 64 rows x 32 BJ complex columns (2 BJ blocks of 32 x 32 per
// product), so the block is 128 x 64 BJ complex; k-step 8 complex; two LDS
// stages with the next tile in registers and the tile after it fetched right
// behind, one barrier per tile, and one set of fragments in registers, which
// keeps a wave under 168 VGPRs: three waves per SIMD (three blocks per CU)
// hide each other's barrier and LDS waits.  K is even (pairs never straddle
// the end of K).
constexpr int M3_BKC = 8, M3_LD = M3_BKC + 4;   // complex k per tile, floats per plane row
template <bool SCAT, bool FULLK, int BJ>
__global__ __launch_bounds__(256, BJ == 1 ? 3 : 1) void k_gemm_3m(const float *__restrict__ A, const float *__restrict__ B,
                                                 float *__restrict__ C, int64_t M, int K, int N,
                                                 int64_t sA, int64_t sB, int64_t sC, int tiles_n,
                                                 ScatterStore sc, int64_t row0) {
    constexpr int BI = 2, BM = 128, BN = 64 * BJ, LD = M3_LD;
    constexpr int APL = BM * LD, BPL = BN * LD, STG = 2 * (APL + BPL);
    __shared__ float smem[2 * STG];
    __shared__ int64_t fofs[SCAT ? BM + BN : 1];   // fused-store offsets: rows, then columns
    auto As = [&](int st, int p) { return smem + st * STG + p * APL; };
    auto Bs = [&](int st, int p) { return smem + st * STG + 2 * APL + p * BPL; };
    // a row's k-tile is 8 complex = 4 float4; 256 threads cover 64 rows per pass
    constexpr int TPR = M3_BKC / 2, RPP = 256 / TPR, AV = BM / RPP, BV = BN / RPP;
    const int64_t u = blockIdx.y;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / tiles_n, tn = tile - tm * tiles_n;
    const int64_t m0 = tm * BM;
    const int n0 = (int)tn * BN;
    A += 2 * u * sA;
    B += 2 * u * sB;
    C += 2 * u * sC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    if constexpr (SCAT) fused_offsets(fofs, BM, fofs + BM, BN, sc, row0, m0, M, n0, N, tid);
    v16f acc[3][BI][BJ];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[p][i][j][r] = 0.0f;
    const int lrow = tid / TPR, lk = (tid % TPR) * 2;   // this thread's complex pair in the k-tile
    // rows clamped into the operands (rows past M or N are never stored)
    const float *ap[AV], *bp[BV];
#pragma unroll
    for (int i = 0; i < AV; ++i) ap[i] = A + 2 * (std::min<int64_t>(m0 + lrow + RPP * i, M - 1) * K + lk);
#pragma unroll
    for (int i = 0; i < BV; ++i) bp[i] = B + 2 * ((int64_t)std::min(n0 + lrow + RPP * i, N - 1) * K + lk);
    v4f ra[AV], rb[BV];
    auto fetch = [&](int k0) {
        // FULLK (K a multiple of the k-step): no guard and no branch, which
        // keeps the loads in the MFMAs' basic block (measured +10 %)
        if (FULLK || k0 + M3_BKC <= K) {
#pragma unroll
            for (int i = 0; i < AV; ++i) ra[i] = *reinterpret_cast<const v4f *>(ap[i] + 2 * k0);
#pragma unroll
            for (int i = 0; i < BV; ++i) rb[i] = *reinterpret_cast<const v4f *>(bp[i] + 2 * k0);
        } else {
            const bool in = k0 + lk < K;   // K even: the pair is whole or absent
#pragma unroll
            for (int i = 0; i < AV; ++i) ra[i] = in ? *reinterpret_cast<const v4f *>(ap[i] + 2 * k0) : v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < BV; ++i) rb[i] = in ? *reinterpret_cast<const v4f *>(bp[i] + 2 * k0) : v4f{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto planes = [&](float *p0, float *p1, int o, v4f x) {
        *reinterpret_cast<v2f *>(p0 + o) = v2f{x[0], x[2]};
        *reinterpret_cast<v2f *>(p1 + o) = v2f{x[1], x[3]};
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int i = 0; i < AV; ++i) planes(As(st, 0), As(st, 1), (lrow + RPP * i) * LD + lk, ra[i]);
#pragma unroll
        for (int i = 0; i < BV; ++i) planes(Bs(st, 0), Bs(st, 1), (lrow + RPP * i) * LD + lk, rb[i]);
    };
    // lanes 0-31 / 32-63 take k-slots 0 / 1 of an MFMA: k = 4 * slot + q for
    // the four MFMAs q of the tile, one 16-byte LDS read per plane and block
    const int arow = (wm * BI * 32 + (lane & 31)) * LD + 4 * (lane >> 5);
    const int brow = (wn * BJ * 32 + (lane & 31)) * LD + 4 * (lane >> 5);
    v4f fa[2][BI], fb[2][BJ];   // re and im planes of the tile's fragments
    auto frags = [&](int st) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int i = 0; i < BI; ++i) fa[p][i] = *reinterpret_cast<const v4f *>(As(st, p) + arow + i * 32 * LD);
#pragma unroll
            for (int j = 0; j < BJ; ++j) fb[p][j] = *reinterpret_cast<const v4f *>(Bs(st, p) + brow + j * 32 * LD);
        }
    };
    auto mfmas = [&](int q) {
        float sa[BI], sb[BJ];
#pragma unroll
        for (int i = 0; i < BI; ++i) sa[i] = fa[0][i][q] + fa[1][i][q];
#pragma unroll
        for (int j = 0; j < BJ; ++j) sb[j] = fb[0][j][q] + fb[1][j][q];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int i = 0; i < BI; ++i)
#pragma unroll
                for (int j = 0; j < BJ; ++j)
                    acc[p][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[p][i][q], fb[p][j][q], acc[p][i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j)
                acc[2][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[i], sb[j], acc[2][i][j], 0, 0, 0);
    };
    const int nt = (K + M3_BKC - 1) / M3_BKC;
    fetch(0);
    stash(0);
    if (nt > 1) fetch(M3_BKC);
    __syncthreads();
    frags(0);
    // Tile t (fragments in registers): its MFMAs with tile t+1 written from
    // registers into the other stage (last read for tile t-1, before the
    // previous barrier) and tile t+2 fetched among them, then the barrier and
    // tile t+1's fragments.  The fetch past the last tile reads the last tile
    // again, so the body has no branch.
    for (int t = 0; t + 1 < nt; ++t) {
        const int st = t & 1;
        mfmas(0);
        mfmas(1);
        stash(st ^ 1);
        fetch(std::min(t + 2, nt - 1) * M3_BKC);
        mfmas(2);
        mfmas(3);
        __syncthreads();
        frags(st ^ 1);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) mfmas(q);
    __syncthreads();   // the stages are reused for the store
    // 32x32 accumulator layout: lane holds complex column lane%32 of its block
    // and rows 8*(r/4) + 4*(lane/32) + r%4 for its 16 values r
    if constexpr (!SCAT) {
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = m0 + wm * BI * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int col = n0 + wn * BJ * 32 + j * 32 + (lane & 31);
                    const float t0 = acc[0][i][j][r], t1 = acc[1][i][j][r], t2 = acc[2][i][j][r];
                    if (row < M && col < N)
                        *reinterpret_cast<v2f *>(C + 2 * (row * N + col)) = v2f{t0 - t1, t2 - t0 - t1};
                }
    } else {
        // fused store staged per wave through LDS (free after the last
        // barrier), in 2 BJ slices of 16 complex columns: lanes whose column
        // falls in slice j stage their values, then every lane stores whole
        // complex values in the order in which the target is contiguous
        constexpr int WR = BI * 32, SLD = 34;
        static_assert(4 * WR * SLD <= 2 * STG, "staging fits in the stages");
        float *stg = smem + wave * WR * SLD;
        const int hc = lane & 31, half = hc >> 4;
        fused_store_wave<float2, WR, 16, SLD, 2 * BJ>(
            C, stg, sc.mfast, fofs + wm * WR, fofs + BM + wn * BJ * 32, lane, [&](int s) {
                if (half != (s & 1)) return;
                const int jb = s >> 1;
#pragma unroll
                for (int j = 0; j < BJ; ++j) {
                    if (j != jb) continue;
#pragma unroll
                    for (int i = 0; i < BI; ++i)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float t0 = acc[0][i][j][r], t1 = acc[1][i][j][r], t2 = acc[2][i][j][r];
                            *reinterpret_cast<v2f *>(
                                &stg[(i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * SLD + 2 * (hc - 16 * (s & 1))]) =
                                v2f{t0 - t1, t2 - t0 - t1};
                        }
                }
            });
    }
}

// The three-multiplication form for short K (even K <= 64 complex): steps
// whose output is many times their operands (K = 16 to 64 against N of
// hundreds to thousands), so that the time goes to writing the output, or
// too short for the k-loop of k_gemm_3m to hide its prologue and store.  A
// block owns 128 rows (32 per wave) and a chunk of S3_NT column tiles of 32
// complex; each wave keeps the re, im and (re + im) fragments of its rows,
// all of K, in registers for the whole chunk, and the block walks the column
// tiles with the next tile's B loaded during the current one's MFMAs (two
// LDS stages of re and im planes, one barrier per tile).  Each tile's
// product is stored as soon as it is formed, so the stores of one tile drain
// while the MFMAs of the next run (and while other waves on the SIMD
// compute).  G k-groups of 8 complex cover K (a tail group is zero-filled).
constexpr int S3_NT = 8;
template <bool SCAT, int G>
__global__ __launch_bounds__(256, G > 4 ? 2 : (SCAT || G > 2 ? 3 : 4)) void k_gemm_3m_short(const float *__restrict__ A,
                                                                       const float *__restrict__ B,
                                                                       float *__restrict__ C, int64_t M, int K, int N,
                                                                       int64_t sA, int64_t sB, int64_t sC, int chunks_n,
                                                                       ScatterStore sc, int64_t row0) {
    constexpr int KP = 8 * G;          // k (complex) covered by the groups
    constexpr int BLD = KP + 4;        // floats per plane row: 16-byte aligned, rows on distinct banks
    constexpr int BPL = 32 * BLD;      // one plane of one stage
    constexpr int WR = 32, SLD = 34;   // output staging of a wave: 32 rows of 32 floats + 2
    constexpr int NF4 = 16 * KP;       // float4 (two complex) in one B tile
    constexpr int PB = (NF4 + 255) / 256;
    __shared__ float bs[2 * 2 * BPL];  // [stage][plane re / im]
    __shared__ float stg_all[4 * WR * SLD];
    __shared__ int64_t fofs[SCAT ? 128 + 32 * S3_NT : 1];   // fused-store offsets: rows, then columns
    const int64_t u = blockIdx.y;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / chunks_n, tc = tile - tm * chunks_n;
    const int64_t m0 = tm * 128;
    const int c0 = (int)tc * (32 * S3_NT);
    const int ntile = min(S3_NT, (N - c0 + 31) / 32);
    A += 2 * u * sA;
    B += 2 * u * sB;
    C += 2 * u * sC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, slot = lane >> 5;
    if constexpr (SCAT) fused_offsets(fofs, 128, fofs + 128, 32 * S3_NT, sc, row0, m0, M, c0, N, tid);
    // A fragments: lane (r, slot) holds k = 8 g + 4 slot + t (t = 0..3) of
    // row m0 + 32 wave + r, the k of the t-th MFMA of group g; rows past M
    // read the last row (never stored), k past K reads zero.  The (re + im)
    // fragments are formed per tile (four adds against twelve MFMAs), which
    // keeps the kernel at three waves per SIMD.
    v4f ar[G], ai[G];
    {
        const float *ap = A + 2 * std::min<int64_t>(m0 + 32 * wave + r, M - 1) * K;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int k = 8 * g + 4 * slot;
            v4f x0 = v4f{0.f, 0.f, 0.f, 0.f}, x1 = v4f{0.f, 0.f, 0.f, 0.f};
            if (k + 2 <= K) x0 = *reinterpret_cast<const v4f *>(ap + 2 * k);
            if (k + 4 <= K) x1 = *reinterpret_cast<const v4f *>(ap + 2 * k + 4);
            ar[g] = v4f{x0[0], x0[2], x1[0], x1[2]};
            ai[g] = v4f{x0[1], x0[3], x1[1], x1[3]};
        }
    }
    // B tile j: columns c0 + 32 j .. + 31, float4 f = column (f / (KP/2)),
    // complex pair (f % (KP/2)); columns past N read the last column
    v4f rb[PB];
    auto fetch = [&](int j) {
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int f = tid + 256 * i;
            const int cc = f / (KP / 2), k = 2 * (f % (KP / 2));
            const int col = std::min(c0 + 32 * j + cc, N - 1);
            rb[i] = (f < NF4 && k < K) ? *reinterpret_cast<const v4f *>(B + 2 * ((int64_t)col * K + k))
                                       : v4f{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int f = tid + 256 * i;
            if (f >= NF4) continue;
            const int cc = f / (KP / 2), k = 2 * (f % (KP / 2));
            float *p0 = bs + st * 2 * BPL + cc * BLD + k;
            *reinterpret_cast<v2f *>(p0) = v2f{rb[i][0], rb[i][2]};
            *reinterpret_cast<v2f *>(p0 + BPL) = v2f{rb[i][1], rb[i][3]};
        }
    };
    float *stg = stg_all + wave * WR * SLD;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int j = 0; j < ntile; ++j) {
        const int st = j & 1;
        if (j + 1 < ntile) fetch(j + 1);
        v16f t0, t1, t2;
#pragma unroll
        for (int e = 0; e < 16; ++e) t0[e] = t1[e] = t2[e] = 0.0f;
        const float *bre = bs + st * 2 * BPL + r * BLD + 4 * slot;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const v4f br = *reinterpret_cast<const v4f *>(bre + 8 * g);
            const v4f bi = *reinterpret_cast<const v4f *>(bre + BPL + 8 * g);
            const v4f bsum = br + bi, asum = ar[g] + ai[g];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                t0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[g][t], br[t], t0, 0, 0, 0);
                t1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[g][t], bi[t], t1, 0, 0, 0);
                t2 = __builtin_amdgcn_mfma_f32_32x32x2f32(asum[t], bsum[t], t2, 0, 0, 0);
            }
        }
        if (j + 1 < ntile) stash(st ^ 1);
        // Re = T0 - T1 into t0, Im = T2 - T0 - T1 into t1 (t2 is then free)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float a = t0[e], b = t1[e];
            t0[e] = a - b;
            t1[e] = t2[e] - a - b;
        }
        const int cj = c0 + 32 * j;
        // accumulator layout: lane holds complex column cj + r and rows
        // 8 (e / 4) + 4 slot + e % 4 of the wave's 32
        if constexpr (!SCAT) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = m0 + 32 * wave + 8 * (e >> 2) + 4 * slot + (e & 3);
                const int col = cj + r;
                if (row < M && col < N) *reinterpret_cast<v2f *>(C + 2 * (row * N + col)) = v2f{t0[e], t1[e]};
            }
        } else if (!sc.mfast) {
            // columns contiguous in the target: the accumulator layout is
            // already in store order (32 lanes, 32 consecutive columns of a
            // row), so the values go out directly, offsets read from LDS
            const int64_t co = fofs[128 + 32 * j + r];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t ro = fofs[32 * wave + 8 * (e >> 2) + 4 * slot + (e & 3)];
                if (ro >= 0 && co >= 0) *reinterpret_cast<v2f *>(C + 2 * (ro + co)) = v2f{t0[e], t1[e]};
            }
        } else {
            const int half = r >> 4;
            fused_store_wave<float2, WR, 16, SLD, 2>(
                C, stg, sc.mfast, fofs + 32 * wave, fofs + 128 + 32 * j, lane, [&](int s) {
                    if (half != s) return;
#pragma unroll
                    for (int e = 0; e < 16; ++e)
                        *reinterpret_cast<v2f *>(&stg[(8 * (e >> 2) + 4 * slot + (e & 3)) * SLD + 2 * (r - 16 * s)]) =
                            v2f{t0[e], t1[e]};
                });
        }
        __syncthreads();
    }
}

// Split K for steps with a small output and a very long K (M, N <= 64,
// K >= 4096: near the end of a path, where one output tile would run as one
// block per unit).  Block (s, u) forms the complex64 partial product of unit
// u over k in [s kc, (s + 1) kc) -- complex multiply-adds in FP32, A and B
// staged through LDS 32 k at a time, each thread 16 outputs -- and writes it
// to P[u][s][M][N]; k_splitk_sum then adds the S partials of each output in
// order s = 0..S-1 (deterministic) and stores the sum, through the
// fused-store tables when given.
constexpr int SK_KT = 32;
__global__ __launch_bounds__(256) void k_splitk_part(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                     float2 *__restrict__ P, int M, int K, int N, int kc,
                                                     int64_t sA, int64_t sB, int64_t sP) {
    __shared__ float2 As[64][SK_KT + 1], Bs[64][SK_KT + 1];
    const int s = blockIdx.x;
    const int64_t u = blockIdx.y;
    A += u * sA;
    B += u * sB;
    P += u * sP + (int64_t)s * M * N;
    const int tid = threadIdx.x;
    const int m = tid >> 2, n0 = (tid & 3) * 16;   // rows 0..63, 16 columns each
    float re[16], im[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) re[j] = im[j] = 0.f;
    const int kb = s * kc, ke = min(K, kb + kc);
    for (int k0 = kb; k0 < ke; k0 += SK_KT) {
        // 64 rows x 32 k of A and of B: 2048 complex each, 8 per thread
        for (int i = tid; i < 64 * SK_KT; i += 256) {
            const int r = i / SK_KT, kk = i % SK_KT, k = k0 + kk;
            const bool in = k < ke;
            As[r][kk] = (r < M && in) ? A[(int64_t)r * K + k] : float2{0.f, 0.f};
            Bs[r][kk] = (r < N && in) ? B[(int64_t)r * K + k] : float2{0.f, 0.f};
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < SK_KT; ++kk) {
            const float2 a = As[m][kk];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float2 b = Bs[n0 + j][kk];
                re[j] += a.x * b.x - a.y * b.y;
                im[j] += a.x * b.y + a.y * b.x;
            }
        }
        __syncthreads();
    }
    if (m < M) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (n0 + j < N) P[m * N + n0 + j] = float2{re[j], im[j]};
    }
}

template <bool SCAT>
__global__ void k_splitk_sum(const float2 *__restrict__ P, float2 *__restrict__ C, int M, int N, int S,
                             int64_t sP, int64_t sC, ScatterStore sc) {
    const int64_t u = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    const float2 *p = P + u * sP + i;
    float re = 0.f, im = 0.f;
    for (int s = 0; s < S; ++s) {
        const float2 v = p[(int64_t)s * M * N];
        re += v.x;
        im += v.y;
    }
    const int m = i / N, n = i - m * N;
    float2 *c = C + u * sC;
    if constexpr (SCAT) {
        const int64_t mask = ((int64_t)1 << sc.shift) - 1;
        c[sc.fa[m >> sc.shift] + sc.fb[m & mask] + sc.fg[n]] = float2{re, im};
    } else {
        c[(int64_t)m * N + n] = float2{re, im};
    }
}

// FP64 MFMA GEMM with v_mfma_f64_16x16x4f64: four waves in 2 x 2, each
// owning BI x BJ blocks of 16 x 16, so the tile is (32*BI) x (32*BJ), k-step
// 16.  The four k-slots (lanes 16*slot .. 16*slot+15) map to k = 4*slot + t
// for the four MFMAs t of a 16-wide k group.  The next k-tile is fetched into
// registers during the current one's MFMAs; NSTAGE = 2 keeps two LDS stages
// (one barrier per k-step, the next tile stored half-way through the current
// one) as in the FP32 kernel.
constexpr int F64_BK = 16, F64_LD = F64_BK + 2;

template <int BI, int BJ, int NSTAGE, bool SCAT>
__global__ __launch_bounds__(256) void k_gemm_f64(const double *__restrict__ A,
                                                   const double *__restrict__ Bt,
                                                   double *__restrict__ C, int64_t M, int Kr,
                                                   int Nr, int64_t sA, int64_t sB, int64_t sC,
                                                   int tiles_n, ScatterStore sc, int64_t row0) {
    constexpr int BM = 32 * BI, BN = 32 * BJ;
    constexpr int AP = BM / 64, BP = BN / 64;   // 64-row load passes per operand
    static_assert(BM % 64 == 0 && BN % 64 == 0, "tile edges are multiples of 64");
    __shared__ double As[NSTAGE][BM * F64_LD];
    __shared__ double Bs[NSTAGE][BN * F64_LD];
    __shared__ int64_t fofs[SCAT ? BM + BN / 2 : 1];   // fused-store offsets: rows, then complex columns
    const int64_t u = blockIdx.y;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tm = tile / tiles_n, tn = tile - tm * tiles_n;
    const int64_t m0 = tm * BM;
    const int n0 = (int)tn * BN;
    A += u * sA;
    Bt += u * sB;
    C += u * sC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    if constexpr (SCAT) fused_offsets(fofs, BM, fofs + BM, BN / 2, sc, row0, m0, M, n0 / 2, Nr / 2, tid);
    v4d acc[BI][BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
    const int lrow = tid >> 2, lcol = (tid & 3) * 4;
    v2d ra[AP][2], rb[BP][2];
    // row pointers clamped into the operands, as in the FP32 kernel: a full
    // k-tile is fetched without guards, a partial last one checks k
    const double *ap[AP], *bp[BP];
#pragma unroll
    for (int p = 0; p < AP; ++p) ap[p] = A + std::min<int64_t>(m0 + lrow + 64 * p, M - 1) * Kr + lcol;
#pragma unroll
    for (int p = 0; p < BP; ++p) bp[p] = Bt + (int64_t)std::min(n0 + lrow + 64 * p, Nr - 1) * Kr + lcol;
    auto fetch = [&](int k0) {
        const bool full = k0 + F64_BK <= Kr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bool in = full || k0 + lcol + 2 * h < Kr;
#pragma unroll
            for (int p = 0; p < AP; ++p)
                ra[p][h] = in ? *reinterpret_cast<const v2d *>(ap[p] + k0 + 2 * h) : v2d{0.0, 0.0};
#pragma unroll
            for (int p = 0; p < BP; ++p)
                rb[p][h] = in ? *reinterpret_cast<const v2d *>(bp[p] + k0 + 2 * h) : v2d{0.0, 0.0};
        }
    };
    auto stash = [&](int stage) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int p = 0; p < AP; ++p)
                *reinterpret_cast<v2d *>(&As[stage][(lrow + 64 * p) * F64_LD + lcol + 2 * h]) = ra[p][h];
#pragma unroll
            for (int p = 0; p < BP; ++p)
                *reinterpret_cast<v2d *>(&Bs[stage][(lrow + 64 * p) * F64_LD + lcol + 2 * h]) = rb[p][h];
        }
    };
    const int kofs = 4 * (lane >> 4);
    auto mfmas = [&](const v4d *a, const v4d *b, int t0, int t1) {
#pragma unroll
        for (int t = t0; t < t1; ++t)
#pragma unroll
            for (int i = 0; i < BI; ++i)
#pragma unroll
                for (int j = 0; j < BJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][t], b[j][t], acc[i][j], 0, 0, 0);
    };
    auto frags = [&](v4d *a, v4d *b, const double *Ac, const double *Bc) {
#pragma unroll
        for (int i = 0; i < BI; ++i) {
            const double *q = &Ac[(wm * BI * 16 + i * 16 + (lane & 15)) * F64_LD + kofs];
            a[i] = v4d{q[0], q[1], q[2], q[3]};
        }
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            const double *q = &Bc[(wn * BJ * 16 + j * 16 + (lane & 15)) * F64_LD + kofs];
            b[j] = v4d{q[0], q[1], q[2], q[3]};
        }
    };
    if constexpr (NSTAGE == 2) {
        // tile t+1 waits in registers; half-way through tile t it goes to the
        // other stage and the fetch of tile t+2 is issued (as in the FP32 kernel)
        fetch(0);
        stash(0);
        if (F64_BK < Kr) fetch(F64_BK);
        __syncthreads();
        int stage = 0;
        for (int k0 = 0; k0 < Kr; k0 += F64_BK) {
            const bool more = k0 + F64_BK < Kr, more2 = k0 + 2 * F64_BK < Kr;
            // MFMA / LDS-read interleaving strategy of the compiler: measured
            // +1.8-2.4 % on the 128 x 128 tile
            if constexpr (BI == 4 && BJ == 4) __builtin_amdgcn_iglp_opt(1);
            v4d a[BI], b[BJ];
            frags(a, b, As[stage], Bs[stage]);
            mfmas(a, b, 0, 2);
            if (more) {
                stash(stage ^ 1);
                if (more2) fetch(k0 + 2 * F64_BK);
            }
            mfmas(a, b, 2, 4);
            __syncthreads();
            stage ^= 1;
        }
    } else {
        fetch(0);
        stash(0);
        __syncthreads();
        for (int k0 = 0; k0 < Kr; k0 += F64_BK) {
            const bool more = k0 + F64_BK < Kr;
            if (more) fetch(k0 + F64_BK);
            v4d a[BI], b[BJ];
            frags(a, b, As[0], Bs[0]);
            mfmas(a, b, 0, 4);
            __syncthreads();
            if (more) {
                stash(0);
                __syncthreads();
            }
        }
    }
    // 16x16 f64 accumulator layout: lane holds column lane%16 and rows lane/16 + 4*r.
    if constexpr (!SCAT) {
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + wm * BI * 16 + i * 16 + (lane >> 4) + 4 * r;
                    const int col = n0 + wn * BJ * 16 + j * 16 + (lane & 15);
                    if (row < M && col < Nr) C[row * Nr + col] = acc[i][j][r];
                }
    } else {
        // fused store, direct: each lane already writes 8-byte values and the
        // re/im halves of a complex value sit in neighbouring lanes, so
        // (measured) staging through LDS does not pay here; the offsets come
        // from LDS (fused_offsets)
        int64_t cofs[BJ];
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            const int col = wn * BJ * 16 + j * 16 + (lane & 15);   // within the block
            const int64_t co = fofs[BM + (col >> 1)];
            cofs[j] = co >= 0 ? 2 * co + (col & 1) : -1;
        }
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t ro = fofs[wm * BI * 16 + i * 16 + (lane >> 4) + 4 * r];
                if (ro < 0) continue;
#pragma unroll
                for (int j = 0; j < BJ; ++j)
                    if (cofs[j] >= 0) C[2 * ro + cofs[j]] = acc[i][j][r];
            }
    }
}

// ---------------------------------------------------------------------------
// small steps, C[u][m][n] = sum_k A[u][m][k] B[u][n][k] with a small K or N.
// k_small_rows: a block copies RB consecutive rows of A (one unit, contiguous)
// and all of B into LDS (sized per launch) with coalesced complex loads (rows
// padded by one complex against bank conflicts), then its threads produce the
// RB x N outputs from LDS.  Outputs are stored row-major (consecutive threads,
// consecutive addresses) or through the fused-store tables in the order in
// which the target is contiguous.  HBM traffic: A and C once.
template <typename R, bool SCAT>
__global__ __launch_bounds__(256) void k_small_rows(const R *__restrict__ A, const R *__restrict__ Bt,
                                                    R *__restrict__ C, int64_t M, int K, int N, int RB,
                                                    int64_t sA, int64_t sB, int64_t sC, ScatterStore sc) {
    using C2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    extern __shared__ __align__(16) unsigned char small_lds[];
    const int ld = K + 1;
    C2 *As = reinterpret_cast<C2 *>(small_lds);   // RB x ld
    C2 *Bs = As + (int64_t)RB * ld;               // N x ld
    const int64_t u = blockIdx.y;
    const int64_t m0 = (int64_t)blockIdx.x * RB;
    const int rows = (int)(M - m0 < RB ? M - m0 : RB);
    const int tid = threadIdx.x;
    const C2 *a = reinterpret_cast<const C2 *>(A) + u * sA + m0 * K;
    const C2 *b = reinterpret_cast<const C2 *>(Bt) + u * sB;
    const int na = rows * K, nb = N * K;
    for (int i = tid; i < na; i += 256) {
        const int r = i / K;
        As[r * ld + (i - r * K)] = a[i];
    }
    for (int i = tid; i < nb; i += 256) {
        const int n = i / K;
        Bs[n * ld + (i - n * K)] = b[i];
    }
    __syncthreads();
    C2 *c = reinterpret_cast<C2 *>(C) + u * sC;
    const bool rfast = SCAT && sc.mfast;
    const int64_t mask = ((int64_t)1 << sc.shift) - 1;
    const int nout = rows * N;
    for (int o = tid; o < nout; o += 256) {
        int r, n;
        if (rfast) {
            n = o / rows;
            r = o - n * rows;
        } else {
            r = o / N;
            n = o - r * N;
        }
        const C2 *ar = As + r * ld, *bn = Bs + n * ld;
        R re = 0, im = 0;
        for (int k = 0; k < K; ++k) {
            const C2 x = ar[k], y = bn[k];
            re += x.x * y.x - x.y * y.y;
            im += x.x * y.y + x.y * y.x;
        }
        C2 v;
        v.x = re;
        v.y = im;
        const int64_t row = m0 + r;
        if constexpr (SCAT)
            c[sc.fa[row >> sc.shift] + sc.fb[row & mask] + sc.fg[n]] = v;
        else
            c[row * N + n] = v;
    }
}

// Fixed small K x N (8 x 8: the steps that absorb a site through two bonds
// of dimension 8 on either side), one row per thread: a block stages 256
// consecutive rows of A (one unit, contiguous) in LDS with 16-byte loads,
// every thread keeps its row in registers, reads B^T (broadcast, all lanes
// the same address) and writes its N outputs -- row-major, or through the
// fused-store tables, where consecutive rows (lanes) are contiguous in the
// target when sc.mfast.  Same arithmetic and order as k_small_rows.
template <typename R, int KK, int NN, bool SCAT>
__global__ __launch_bounds__(256) void k_small_fixed(const R *__restrict__ A, const R *__restrict__ Bt,
                                                     R *__restrict__ C, int64_t M, int64_t sA, int64_t sB,
                                                     int64_t sC, ScatterStore sc) {
    using C2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    constexpr int LD = KK + 1;
    __shared__ C2 As[256 * LD];
    __shared__ C2 Bs[NN * KK];
    // the column parts of the fused-store offsets, read once per block: a
    // table read between two stores would wait for the stores in flight
    __shared__ int64_t fgs[SCAT ? NN : 1];
    const int64_t u = blockIdx.y;
    const int64_t m0 = (int64_t)blockIdx.x * 256;
    const int rows = (int)(M - m0 < 256 ? M - m0 : 256);
    const int tid = threadIdx.x;
    const C2 *a = reinterpret_cast<const C2 *>(A) + u * sA + m0 * KK;
    const C2 *b = reinterpret_cast<const C2 *>(Bt) + u * sB;
    for (int i = tid; i < NN * KK; i += 256) Bs[i] = b[i];
    if constexpr (SCAT)
        if (tid < NN) fgs[tid] = sc.fg[tid];
    if constexpr (sizeof(R) == 4 && KK % 2 == 0) {
        // two complex64 values per 16-byte load (the chunk starts 16-byte aligned)
        const float4 *a4 = reinterpret_cast<const float4 *>(a);
        for (int i = tid; i < rows * KK / 2; i += 256) {
            const float4 v = a4[i];
            const int r = (2 * i) / KK, k = 2 * i - r * KK;
            As[r * LD + k] = C2{v.x, v.y};
            As[r * LD + k + 1] = C2{v.z, v.w};
        }
    } else {
        for (int i = tid; i < rows * KK; i += 256) {
            const int r = i / KK;
            As[r * LD + (i - r * KK)] = a[i];
        }
    }
    __syncthreads();
    if (tid >= rows) return;
    C2 x[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) x[k] = As[tid * LD + k];
    const int64_t row = m0 + tid;
    C2 *c = reinterpret_cast<C2 *>(C) + u * sC;
    int64_t base;
    if constexpr (SCAT) base = sc.fa[row >> sc.shift] + sc.fb[row & (((int64_t)1 << sc.shift) - 1)];
    else base = row * NN;
#pragma unroll
    for (int n = 0; n < NN; ++n) {
        R re = 0, im = 0;
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            const C2 y = Bs[n * KK + k];
            re += x[k].x * y.x - x[k].y * y.y;
            im += x[k].x * y.y + x[k].y * y.x;
        }
        C2 v;
        v.x = re;
        v.y = im;
        if constexpr (SCAT) c[base + fgs[n]] = v;
        else c[base + n] = v;
    }
}

// the general case: one thread per output element

template <typename R, typename Acc>
__global__ void k_small(const R *__restrict__ A, const R *__restrict__ Bt, R *__restrict__ C,
                        int64_t units, int64_t M, int64_t K, int64_t N, int64_t sA, int64_t sB,
                        int64_t sC) {
    const int64_t per = M * N;
    const int64_t total = per * units;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / per, i = t - u * per;
        const int64_t m = i / N, n = i - m * N;
        const R *a = A + 2 * (u * sA + m * K);
        const R *b = Bt + 2 * (u * sB + n * K);
        Acc re = 0, im = 0;
        for (int64_t k = 0; k < K; ++k) {
            const Acc ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
            re += ar * br - ai * bi;
            im += ar * bi + ai * br;
        }
        C[2 * (u * sC + i)] = (R)re;
        C[2 * (u * sC + i) + 1] = (R)im;
    }
}

// last step: one workgroup per unit, sum_k A[k] B[k] accumulated in FP64
template <typename R>
__global__ __launch_bounds__(256) void k_final_dot(const R *__restrict__ A,
                                                    const R *__restrict__ Bt,
                                                    double *__restrict__ partial, int64_t K,
                                                    int64_t sA, int64_t sB) {
    using C2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    __shared__ double wre[4], wim[4];
    const int64_t u = blockIdx.x;
    const C2 *a = reinterpret_cast<const C2 *>(A) + u * sA;
    const C2 *b = reinterpret_cast<const C2 *>(Bt) + u * sB;
    double re = 0, im = 0;
    for (int64_t k = threadIdx.x; k < K; k += 256) {
        const C2 x = a[k], y = b[k];
        const double ar = x.x, ai = x.y, br = y.x, bi = y.y;
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
    }
    // wave64 butterfly: every lane ends with its wave's sum (fixed order)
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        re += __shfl_xor(re, m, 64);
        im += __shfl_xor(im, m, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        wre[wave] = re;
        wim[wave] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * u] = (wre[0] + wre[1]) + (wre[2] + wre[3]);
        partial[2 * u + 1] = (wim[0] + wim[1]) + (wim[2] + wim[3]);
    }
}

// Last tensor of a unit with open legs -> its row of partial results, in
// output order and widened to complex128.
template <typename R>
__global__ void k_finalize(const R *__restrict__ T, double *__restrict__ partial, int64_t units,
                           int64_t t_us, int64_t per, Gather g) {
    const int64_t total = units * per;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = t / per, i = t - u * per;
        const R *src = T + 2 * (u * t_us + gather_offset(g, i));
        partial[2 * t] = (double)src[0];
        partial[2 * t + 1] = (double)src[1];
    }
}

// Pairwise (binary-counter) summation of the slices of each (bitstring,
// output) pair: a fixed tree, so the result does not depend on launch
// configuration.  partial is [bitstring][slice][per].
__global__ void k_slice_sum(const double *__restrict__ partial, double *__restrict__ amps,
                            int64_t nb, int64_t n_slices, int64_t per) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nb * per) return;
    const int64_t b = t / per, o = t - b * per;
    double sr[64], si[64];
    int lv[64];
    int top = 0;
    const double *x = partial + 2 * (b * n_slices * per + o);
    for (int64_t i = 0; i < n_slices; ++i) {
        double vr = x[2 * i * per], vi = x[2 * i * per + 1];
        int l = 0;
        while (top > 0 && lv[top - 1] == l) {
            vr = sr[top - 1] + vr;
            vi = si[top - 1] + vi;
            --top;
            ++l;
        }
        sr[top] = vr;
        si[top] = vi;
        lv[top] = l;
        ++top;
    }
    double rr = 0, ri = 0;
    if (top > 0) {
        rr = sr[top - 1];
        ri = si[top - 1];
        for (int j = top - 2; j >= 0; --j) {
            rr = sr[j] + rr;
            ri = si[j] + ri;
        }
    }
    amps[2 * t] = rr;
    amps[2 * t + 1] = ri;
}

}  // namespace

namespace launch {

void gather(const void *in, void *out, int64_t units, int64_t in_unit_stride,
            int64_t out_unit_stride, const Gather &g, int elem_bytes, void *stream) {
    int64_t per = 1;
    for (int a = 0; a < g.n; ++a) per *= g.size[a];
    const int64_t total = per * units;
    // tiled transpose when the input- and output-contiguous axes differ
    int ai = -1;
    for (int a = 0; a < g.n; ++a)
        if (g.stride[a] == 1 && g.size[a] > 1) ai = a;
    const int ao = g.n - 1;
    if (ai >= 0 && ai != ao && g.size[ai] >= 8 && g.size[ao] >= 8) {
        PermTile pt{};
        pt.n = g.n;
        pt.ai = ai;
        pt.ao = ao;
        int64_t os = 1;
        for (int a = g.n - 1; a >= 0; --a) {
            pt.size[a] = g.size[a];
            pt.in_stride[a] = g.stride[a];
            pt.out_stride[a] = os;
            os *= g.size[a];
        }
        pt.ti = (int)std::min<int64_t>(64, g.size[ai]);
        pt.to = (int)std::min<int64_t>(64, g.size[ao]);
        pt.tiles_i = (g.size[ai] + pt.ti - 1) / pt.ti;
        pt.tiles_o = (g.size[ao] + pt.to - 1) / pt.to;
        pt.tiles_per_unit = per / (g.size[ai] * g.size[ao]) * pt.tiles_i * pt.tiles_o;
        const int64_t tiles = pt.tiles_per_unit * units;
        const unsigned blocks = (unsigned)std::min<int64_t>(tiles, 65536 * 8);
        if (elem_bytes == 8)
            hipLaunchKernelGGL(k_permute_tiled<float2>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                               (const float2 *)in, (float2 *)out, units, in_unit_stride,
                               out_unit_stride, pt);
        else
            hipLaunchKernelGGL(k_permute_tiled<double2>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                               (const double2 *)in, (double2 *)out, units, in_unit_stride,
                               out_unit_stride, pt);
        check_launch("permute");
        return;
    }
    constexpr int64_t k31 = (int64_t)1 << 31;
    if (per >= k31 && g.n >= 2) {
        // Peel leading output axes until one launch covers < 2^31 elements:
        // the last peeled axis becomes the launch's unit dimension, the ones
        // before it and the units are host loops; each piece then takes the
        // 32-bit kernel below.
        int p = 0;
        int64_t rest = per;
        while (p < g.n - 1 && rest >= k31) rest /= g.size[p++];
        if (rest < k31 && g.size[p - 1] <= 65535) {
            Gather inner{};
            inner.n = g.n - p;
            for (int a = p; a < g.n; ++a) {
                inner.size[a - p] = g.size[a];
                inner.stride[a - p] = g.stride[a];
            }
            int64_t outer = 1;
            for (int a = 0; a < p - 1; ++a) outer *= g.size[a];
            const int64_t lead = g.size[p - 1];
            for (int64_t u = 0; u < units; ++u)
                for (int64_t o = 0; o < outer; ++o) {
                    int64_t in_off = u * in_unit_stride, r = o;
                    for (int a = p - 2; a >= 0; --a) {
                        in_off += (r % g.size[a]) * g.stride[a];
                        r /= g.size[a];
                    }
                    const int64_t out_off = u * out_unit_stride + o * lead * rest;
                    gather((const char *)in + in_off * elem_bytes, (char *)out + out_off * elem_bytes,
                           lead, g.stride[p - 1], rest, inner, elem_bytes, stream);
                }
            return;
        }
    }
    if (per < k31 && units <= 65535) {
        const bool vec = elem_bytes == 8 && g.stride[g.n - 1] == 1 && g.size[g.n - 1] % 2 == 0;
        const int64_t work = vec ? per / 2 : per;
        const unsigned bx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 1023) / 1024, 65536));
        const dim3 grid(bx, (unsigned)units);
        if (elem_bytes == 8 && vec)
            hipLaunchKernelGGL((k_gather32<float2, 2>), grid, dim3(256), 0, (hipStream_t)stream,
                               (const float2 *)in, (float2 *)out, in_unit_stride, out_unit_stride, g,
                               (uint32_t)per);
        else if (elem_bytes == 8)
            hipLaunchKernelGGL((k_gather32<float2, 1>), grid, dim3(256), 0, (hipStream_t)stream,
                               (const float2 *)in, (float2 *)out, in_unit_stride, out_unit_stride, g,
                               (uint32_t)per);
        else
            hipLaunchKernelGGL((k_gather32<double2, 1>), grid, dim3(256), 0, (hipStream_t)stream,
                               (const double2 *)in, (double2 *)out, in_unit_stride, out_unit_stride, g,
                               (uint32_t)per);
        check_launch("gather32");
        return;
    }

    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather<float2>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const float2 *)in, (float2 *)out, units,
                           in_unit_stride, out_unit_stride, g, per);
    else
        hipLaunchKernelGGL(k_gather<double2>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const double2 *)in, (double2 *)out, units,
                           in_unit_stride, out_unit_stride, g, per);
    check_launch("gather");
}

void expand_prefix(const void *pre, void *out, int64_t units, int64_t u0, int64_t nper, int64_t elems,
                   int64_t out_us, int elem_bytes, void *stream) {
    const int64_t total = units * elems;
    if (total <= 0) return;
    const dim3 grid(grid_for(total, 256));
    if (elem_bytes == 8)
        hipLaunchKernelGGL((k_expand_prefix<float2>), grid, dim3(256), 0, (hipStream_t)stream,
                           (const float2 *)pre, (float2 *)out, units, u0, nper, elems, out_us);
    else
        hipLaunchKernelGGL((k_expand_prefix<double2>), grid, dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)pre, (double2 *)out, units, u0, nper, elems, out_us);
    check_launch("expand_prefix");
}

void gather_site(const void *site, void *out, int64_t units, int64_t u0, int64_t n_slices,
                 int64_t slice0, int64_t site_stride, const SliceMap &sm, int64_t out_unit_stride,
                 const Gather &g, int elem_bytes, void *stream) {
    int64_t per = 1;
    for (int a = 0; a < g.n; ++a) per *= g.size[a];
    const int64_t total = per * units;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_gather_site<float2>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const float2 *)site, (float2 *)out, units, u0,
                           n_slices, slice0, site_stride, sm, out_unit_stride, g, per);
    else
        hipLaunchKernelGGL(k_gather_site<double2>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const double2 *)site, (double2 *)out, units, u0,
                           n_slices, slice0, site_stride, sm, out_unit_stride, g, per);
    check_launch("gather_site");
}

void build_b(const void *site, void *out, int64_t units, int64_t u0, int64_t n_slices,
             int64_t slice0, int64_t site_stride, const SliceMap &sm, const Gather &g, int64_t K,
             int64_t N, int c64, int embed, void *stream) {
    const int64_t total = K * N * units;
    if (c64)
        hipLaunchKernelGGL(k_build_b<float>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const float *)site, (float *)out, units, u0,
                           n_slices, slice0, site_stride, sm, g, K, N, embed);
    else
        hipLaunchKernelGGL(k_build_b<double>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const double *)site, (double *)out, units, u0,
                           n_slices, slice0, site_stride, sm, g, K, N, embed);
    check_launch("build_b");
}

// NSTAGE: two LDS stages on the 128 x 128 tile (k-step 32: 73.7 KB FP32,
// 81.9 KB 3-product BF16; k-step 16 for short k-loops and for the 6-product
// form, 40.9 / 49.2 / 61.4 KB), so two blocks fit on a CU; one stage on the
// narrow tiles.
template <int BI, int BJ, int WGM, int WGN, bool SCAT>
static void launch_c64(int mode, dim3 grid, hipStream_t st, const float *A, const float *B, float *C,
                       int64_t M, int Kr, int Nr, int64_t sA, int64_t sB, int64_t sC, int tiles_n,
                       const ScatterStore &sc, int64_t row0) {
    constexpr int S = WGN == 2 ? 2 : 1;
    if constexpr (BJ == 4) {
        // 128 x 256 (FP32 and split-BF16 x3): k-step 16, since two stages at
        // k-step 32 would leave one block per CU
        if (mode == 1)
            hipLaunchKernelGGL((k_gemm_c64<BI, BJ, WGM, WGN, 1, 2, 16, SCAT>), grid, dim3(256), 0, st, A, B, C, M,
                               Kr, Nr, sA, sB, sC, tiles_n, sc, row0);
        else if (mode == 2)
            hipLaunchKernelGGL((k_gemm_c64<BI, BJ, WGM, WGN, 2, 2, 16, SCAT>), grid, dim3(256), 0, st, A, B, C, M,
                               Kr, Nr, sA, sB, sC, tiles_n, sc, row0);
        else
            fail(TNS_E_UNSUPPORTED, "internal: no 128 x 256 tile for split-BF16 x6");
    } else {
        // measured: on the 128 x 128 FP32 tile a k-step of 16 pays for short
        // k-loops (2K < 1024), a k-step of 32 for long ones; split-BF16 x3
        // measured best at 32 throughout
        if constexpr (S == 2) {
            if (Kr < 1024 && mode == 1) {
                hipLaunchKernelGGL((k_gemm_c64<BI, BJ, WGM, WGN, 1, S, 16, SCAT>), grid, dim3(256), 0, st, A, B, C, M,
                                   Kr, Nr, sA, sB, sC, tiles_n, sc, row0);
                return;
            }
        }
        if (mode == 1)
            hipLaunchKernelGGL((k_gemm_c64<BI, BJ, WGM, WGN, 1, S, 32, SCAT>), grid, dim3(256), 0, st, A, B, C, M, Kr, Nr,
                               sA, sB, sC, tiles_n, sc, row0);
        else if (mode == 2)
            hipLaunchKernelGGL((k_gemm_c64<BI, BJ, WGM, WGN, 2, S, 32, SCAT>), grid, dim3(256), 0, st, A, B, C, M, Kr, Nr,
                               sA, sB, sC, tiles_n, sc, row0);
        else
            hipLaunchKernelGGL((k_gemm_c64<BI, BJ, WGM, WGN, 3, S, (S == 2 ? 16 : 32), SCAT>), grid, dim3(256), 0, st, A,
                               B, C, M, Kr, Nr, sA, sB, sC, tiles_n, sc, row0);
    }
}

template <int BI, int BJ, int WGM, int WGN>
static void launch_c64(int mode, dim3 grid, hipStream_t st, const float *A, const float *B, float *C,
                       int64_t M, int Kr, int Nr, int64_t sA, int64_t sB, int64_t sC, int tiles_n,
                       const ScatterStore *sc, int64_t row0) {
    if (sc) launch_c64<BI, BJ, WGM, WGN, true>(mode, grid, st, A, B, C, M, Kr, Nr, sA, sB, sC, tiles_n, *sc, row0);
    else launch_c64<BI, BJ, WGM, WGN, false>(mode, grid, st, A, B, C, M, Kr, Nr, sA, sB, sC, tiles_n, ScatterStore{}, 0);
}

template <int BI, int BJ>
static void launch_f64(dim3 grid, hipStream_t st, const double *A, const double *B, double *C, int64_t M, int Kr,
                       int Nr, int64_t sA, int64_t sB, int64_t sC, int tiles_n, const ScatterStore *sc,
                       int64_t row0) {
    if (sc)
        hipLaunchKernelGGL((k_gemm_f64<BI, BJ, 2, true>), grid, dim3(256), 0, st, A, B, C, M, Kr, Nr, sA, sB, sC,
                           tiles_n, *sc, row0);
    else
        hipLaunchKernelGGL((k_gemm_f64<BI, BJ, 2, false>), grid, dim3(256), 0, st, A, B, C, M, Kr, Nr, sA, sB, sC,
                           tiles_n, ScatterStore{}, (int64_t)0);
}

// Three-multiplication launches: BJ column blocks of 32 complex per wave (a
// block of 128 x 64 BJ complex), chunked so that one launch holds at most 2^30
// tiles per unit row range and 65535 units.
template <int BJ>
void launch_3m(const float *A, const float *Bt, float *C, int64_t units, int64_t M, int64_t K, int64_t N,
               int64_t sA, int64_t sB, int64_t sC, hipStream_t st, const ScatterStore *sc) {
    constexpr int BN = 64 * BJ;
    const int tiles_n = (int)((N + BN - 1) / BN);
    const int64_t rows_per = (((int64_t)1 << 30) / tiles_n) * 128;
    const bool full = K % M3_BKC == 0;
    const ScatterStore none{};
    for (int64_t u0 = 0; u0 < units; u0 += 65535) {
        const int64_t nu = std::min<int64_t>(65535, units - u0);
        for (int64_t r0 = 0; r0 < M; r0 += rows_per) {
            const int64_t mr = std::min<int64_t>(rows_per, M - r0);
            const dim3 grid((unsigned)(((mr + 127) / 128) * tiles_n), (unsigned)nu);
            const int64_t crow = sc ? 0 : r0;
            const float *a = A + 2 * (u0 * sA + r0 * K);
            const float *b = Bt + 2 * u0 * sB;
            float *c = C + 2 * (u0 * sC + crow * N);
            if (sc && full)
                hipLaunchKernelGGL((k_gemm_3m<true, true, BJ>), grid, dim3(256), 0, st, a, b, c, mr, (int)K, (int)N,
                                   sA, sB, sC, tiles_n, *sc, r0);
            else if (sc)
                hipLaunchKernelGGL((k_gemm_3m<true, false, BJ>), grid, dim3(256), 0, st, a, b, c, mr, (int)K, (int)N,
                                   sA, sB, sC, tiles_n, *sc, r0);
            else if (full)
                hipLaunchKernelGGL((k_gemm_3m<false, true, BJ>), grid, dim3(256), 0, st, a, b, c, mr, (int)K, (int)N,
                                   sA, sB, sC, tiles_n, none, (int64_t)0);
            else
                hipLaunchKernelGGL((k_gemm_3m<false, false, BJ>), grid, dim3(256), 0, st, a, b, c, mr, (int)K, (int)N,
                                   sA, sB, sC, tiles_n, none, (int64_t)0);
            check_launch("gemm_3m");
        }
    }
}

template <int G>
void launch_3m_short(const float *A, const float *Bt, float *C, int64_t units, int64_t M, int64_t K, int64_t N,
                     int64_t sA, int64_t sB, int64_t sC, hipStream_t st, const ScatterStore *sc) {
    const int chunks_n = (int)((N + 32 * S3_NT - 1) / (32 * S3_NT));
    const int64_t rows_per = (((int64_t)1 << 30) / chunks_n) * 128;
    const ScatterStore none{};
    for (int64_t u0 = 0; u0 < units; u0 += 65535) {
        const int64_t nu = std::min<int64_t>(65535, units - u0);
        for (int64_t r0 = 0; r0 < M; r0 += rows_per) {
            const int64_t mr = std::min<int64_t>(rows_per, M - r0);
            const dim3 grid((unsigned)(((mr + 127) / 128) * chunks_n), (unsigned)nu);
            const int64_t crow = sc ? 0 : r0;
            const float *a = A + 2 * (u0 * sA + r0 * K);
            const float *b = Bt + 2 * u0 * sB;
            float *c = C + 2 * (u0 * sC + crow * N);
            if (sc)
                hipLaunchKernelGGL((k_gemm_3m_short<true, G>), grid, dim3(256), 0, st, a, b, c, mr, (int)K, (int)N,
                                   sA, sB, sC, chunks_n, *sc, r0);
            else
                hipLaunchKernelGGL((k_gemm_3m_short<false, G>), grid, dim3(256), 0, st, a, b, c, mr, (int)K, (int)N,
                                   sA, sB, sC, chunks_n, none, (int64_t)0);
            check_launch("gemm_3m_short");
        }
    }
}

void gemm(const void *A, const void *Bt, void *C, int64_t units, int64_t M, int64_t K,
          int64_t N, int64_t sA, int64_t sB, int64_t sC, int mode, void *stream,
          const ScatterStore *sc) {
    // mode: 0 complex128 (FP64 MFMA), 1 complex64 (FP32 MFMA), 2 / 3 complex64 on
    // split-BF16 MFMA with 3 / 6 products, 4 complex64 in the three-
    // multiplication form (FP32 MFMA; Bt is then the plain complex [N][K], not
    // its real embedding; K <= 64 takes the short-K kernel).  Strides arrive
    // in complex elements; the kernels index reals.
    const hipStream_t st = (hipStream_t)stream;
    if (mode == 4) {
        if (K % 2 != 0) fail(TNS_E_UNSUPPORTED, "three-multiplication GEMM needs an even K");
        if (units <= 0 || M <= 0 || N <= 0) return;
        if (gemm_3m_splitk(M, K, N, units, sC)) {
            // split K: the partials go to the unit's own output slot past its
            // M N outputs (the slot holds the path's largest intermediate)
            const int64_t Sn = splitk_parts(K);
            const int64_t kc = (K + Sn - 1) / Sn;
            const float2 *a = (const float2 *)A, *b = (const float2 *)Bt;
            float2 *c = (float2 *)C;
            hipLaunchKernelGGL(k_splitk_part, dim3((unsigned)Sn, (unsigned)units), dim3(256), 0, st, a, b,
                               c + M * N, (int)M, (int)K, (int)N, (int)kc, sA, sB, sC);
            check_launch("splitk_part");
            const dim3 g2((unsigned)((M * N + 255) / 256), (unsigned)units);
            const ScatterStore none{};
            if (sc)
                hipLaunchKernelGGL((k_splitk_sum<true>), g2, dim3(256), 0, st, c + M * N, c, (int)M, (int)N,
                                   (int)Sn, sC, sC, *sc);
            else
                hipLaunchKernelGGL((k_splitk_sum<false>), g2, dim3(256), 0, st, c + M * N, c, (int)M, (int)N,
                                   (int)Sn, sC, sC, none);
            check_launch("splitk_sum");
            return;
        }
        if (gemm_3m_short_k(K)) {
            // short K: A stays in registers (K = 16: 2 groups of 8, 32: 4, 64: 8)
            if (K <= 16) launch_3m_short<2>((const float *)A, (const float *)Bt, (float *)C, units, M, K, N, sA, sB, sC, st, sc);
            else if (K <= 32) launch_3m_short<4>((const float *)A, (const float *)Bt, (float *)C, units, M, K, N, sA, sB, sC, st, sc);
            else launch_3m_short<8>((const float *)A, (const float *)Bt, (float *)C, units, M, K, N, sA, sB, sC, st, sc);
            return;
        }
        // BJ = 2 (128 x 128 complex, one wave per SIMD) measured level with or
        // up to 10 % behind BJ = 1 (two waves per SIMD) on every step shape
        launch_3m<1>((const float *)A, (const float *)Bt, (float *)C, units, M, K, N, sA, sB, sC, st, sc);
        return;
    }
    const int c64 = mode != 0;
    const int Kr = (int)(2 * K), Nr = (int)(2 * N);
    if (c64 && (Kr % 4) != 0) fail(TNS_E_UNSUPPORTED, "FP32 GEMM needs an even K");
    // tile shape: complex64 256 x 32 for N <= 16 complex, 256 x 64 for N <= 32,
    // else 128 x 128, or 128 x 256 for split-BF16 x3 with N >= 128 complex
    // (+5-8 %) and for FP32 with N >= 256 and 2K >= 1024 (+0.5-1 %; split-BF16
    // x6 loses there, its fragments leave one block per CU); complex128
    // 128 x 128 for N >= 128 complex and M >= 4096, else 64 x 64 (measured: the
    // large tiles lose on narrow and short shapes)
    const bool f64_big = Nr >= 256 && M >= 4096;
    const bool wide = (mode == 2 && Nr >= 256) || (mode == 1 && Nr >= 512 && Kr >= 1024);
    const int shape = !c64 ? (f64_big ? 4 : 0) : (Nr <= 32 ? 1 : (Nr <= 64 ? 2 : (wide ? 5 : 3)));
    const int BM = shape == 0 ? 64 : (shape == 3 || shape == 4 || shape == 5 ? 128 : 256);
    const int BN = shape == 0 ? 64 : (shape == 1 ? 32 : (shape == 2 ? 64 : (shape == 5 ? 256 : 128)));
    const int tiles_n = (Nr + BN - 1) / BN;
    // rows per launch so that the grid stays below 2^31 blocks
    const int64_t max_tiles_m = ((int64_t)1 << 30) / tiles_n;
    const int64_t rows_per = max_tiles_m * BM;
    for (int64_t u0 = 0; u0 < units; u0 += 65535) {
        const int64_t nu = std::min<int64_t>(65535, units - u0);
        for (int64_t r0 = 0; r0 < M; r0 += rows_per) {
            const int64_t mr = std::min<int64_t>(rows_per, M - r0);
            const int64_t tiles_m = (mr + BM - 1) / BM;
            const dim3 grid((unsigned)(tiles_m * tiles_n), (unsigned)nu);
            // with a fused store the row offset goes to the tables, not to C
            const int64_t crow = sc ? 0 : r0;
            if (c64) {
                const float *a = (const float *)A + 2 * (u0 * sA + r0 * K);
                const float *b = (const float *)Bt + 4 * u0 * sB;
                float *c = (float *)C + 2 * (u0 * sC + crow * N);
                if (shape == 1) launch_c64<2, 1, 4, 1>(mode, grid, st, a, b, c, mr, Kr, Nr, 2 * sA, 4 * sB, 2 * sC, tiles_n, sc, r0);
                else if (shape == 2) launch_c64<2, 2, 4, 1>(mode, grid, st, a, b, c, mr, Kr, Nr, 2 * sA, 4 * sB, 2 * sC, tiles_n, sc, r0);
                else if (shape == 3) launch_c64<2, 2, 2, 2>(mode, grid, st, a, b, c, mr, Kr, Nr, 2 * sA, 4 * sB, 2 * sC, tiles_n, sc, r0);
                else launch_c64<2, 4, 2, 2>(mode, grid, st, a, b, c, mr, Kr, Nr, 2 * sA, 4 * sB, 2 * sC, tiles_n, sc, r0);
            } else {
                const double *a = (const double *)A + 2 * (u0 * sA + r0 * K);
                const double *b = (const double *)Bt + 4 * u0 * sB;
                double *c = (double *)C + 2 * (u0 * sC + crow * N);
                if (shape == 4) launch_f64<4, 4>(grid, st, a, b, c, mr, Kr, Nr, 2 * sA, 4 * sB, 2 * sC, tiles_n, sc, r0);
                else launch_f64<2, 2>(grid, st, a, b, c, mr, Kr, Nr, 2 * sA, 4 * sB, 2 * sC, tiles_n, sc, r0);
            }
            check_launch("gemm");
        }
    }
}

void small_contract(const void *A, const void *Bt, void *C, int64_t units, int64_t M,
                    int64_t K, int64_t N, int64_t sA, int64_t sB, int64_t sC, int c64,
                    void *stream, const ScatterStore *sc) {
    const int64_t csize = c64 ? 8 : 16;
    const hipStream_t st = (hipStream_t)stream;
    if (units <= 0 || M <= 0 || N <= 0) return;
    if (K == 8 && N == 8 && M >= 256) {
        const int64_t blocks = (M + 255) / 256;
        if (blocks >= ((int64_t)1 << 31)) fail(TNS_E_UNSUPPORTED, "small step with too many rows");
        const ScatterStore none{};
        for (int64_t u0 = 0; u0 < units; u0 += 65535) {
            const int64_t nu = std::min<int64_t>(65535, units - u0);
            const dim3 grid((unsigned)blocks, (unsigned)nu);
            if (c64) {
                const float *a = (const float *)A + 2 * u0 * sA, *b = (const float *)Bt + 2 * u0 * sB;
                float *c = (float *)C + 2 * u0 * sC;
                if (sc) hipLaunchKernelGGL((k_small_fixed<float, 8, 8, true>), grid, dim3(256), 0, st, a, b, c, M,
                                           sA, sB, sC, *sc);
                else hipLaunchKernelGGL((k_small_fixed<float, 8, 8, false>), grid, dim3(256), 0, st, a, b, c, M,
                                        sA, sB, sC, none);
            } else {
                const double *a = (const double *)A + 2 * u0 * sA, *b = (const double *)Bt + 2 * u0 * sB;
                double *c = (double *)C + 2 * u0 * sC;
                if (sc) hipLaunchKernelGGL((k_small_fixed<double, 8, 8, true>), grid, dim3(256), 0, st, a, b, c, M,
                                           sA, sB, sC, *sc);
                else hipLaunchKernelGGL((k_small_fixed<double, 8, 8, false>), grid, dim3(256), 0, st, a, b, c, M,
                                        sA, sB, sC, none);
            }
            check_launch("small_fixed");
        }
        return;
    }
    if (small_rows_fits(M, K, N, csize)) {
        const int RB = (int)small_rows_block(K, csize);
        const int64_t blocks = (M + RB - 1) / RB;
        const size_t lds = (size_t)(RB + N) * (K + 1) * csize;   // <= 64 KiB
        if (blocks >= ((int64_t)1 << 31)) fail(TNS_E_UNSUPPORTED, "small step with too many rows");
        const ScatterStore none{};
        for (int64_t u0 = 0; u0 < units; u0 += 65535) {
            const int64_t nu = std::min<int64_t>(65535, units - u0);
            const dim3 grid((unsigned)blocks, (unsigned)nu);
            if (c64) {
                const float *a = (const float *)A + 2 * u0 * sA, *b = (const float *)Bt + 2 * u0 * sB;
                float *c = (float *)C + 2 * u0 * sC;
                if (sc) hipLaunchKernelGGL((k_small_rows<float, true>), grid, dim3(256), lds, st, a, b, c, M, (int)K,
                                           (int)N, RB, sA, sB, sC, *sc);
                else hipLaunchKernelGGL((k_small_rows<float, false>), grid, dim3(256), lds, st, a, b, c, M, (int)K,
                                        (int)N, RB, sA, sB, sC, none);
            } else {
                const double *a = (const double *)A + 2 * u0 * sA, *b = (const double *)Bt + 2 * u0 * sB;
                double *c = (double *)C + 2 * u0 * sC;
                if (sc) hipLaunchKernelGGL((k_small_rows<double, true>), grid, dim3(256), lds, st, a, b, c, M, (int)K,
                                           (int)N, RB, sA, sB, sC, *sc);
                else hipLaunchKernelGGL((k_small_rows<double, false>), grid, dim3(256), lds, st, a, b, c, M, (int)K,
                                        (int)N, RB, sA, sB, sC, none);
            }
            check_launch("small_contract");
        }
        return;
    }
    if (sc) fail(TNS_E_UNSUPPORTED, "internal: fused store on a small step outside the row kernel");
    const int64_t total = M * N * units;
    if (c64)
        hipLaunchKernelGGL((k_small<float, float>), dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const float *)A, (const float *)Bt, (float *)C,
                           units, M, K, N, sA, sB, sC);
    else
        hipLaunchKernelGGL((k_small<double, double>), dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const double *)A, (const double *)Bt, (double *)C,
                           units, M, K, N, sA, sB, sC);
    check_launch("small_contract");
}

void final_dot(const void *A, const void *Bt, double *partial, int64_t units, int64_t K,
               int64_t sA, int64_t sB, int c64, void *stream) {
    for (int64_t u0 = 0; u0 < units; u0 += 1 << 30) {
        const int64_t nu = std::min<int64_t>(1 << 30, units - u0);
        if (c64)
            hipLaunchKernelGGL(k_final_dot<float>, dim3((unsigned)nu), dim3(256), 0,
                               (hipStream_t)stream, (const float *)A + 2 * u0 * sA,
                               (const float *)Bt + 2 * u0 * sB, partial + 2 * u0, K, sA, sB);
        else
            hipLaunchKernelGGL(k_final_dot<double>, dim3((unsigned)nu), dim3(256), 0,
                               (hipStream_t)stream, (const double *)A + 2 * u0 * sA,
                               (const double *)Bt + 2 * u0 * sB, partial + 2 * u0, K, sA, sB);
        check_launch("final_dot");
    }
}

void slice_sum(const double *partial, double *amps, int64_t nb, int64_t n_slices, int64_t per,
               void *stream) {
    hipLaunchKernelGGL(k_slice_sum, dim3((unsigned)((nb * per + 63) / 64)), dim3(64), 0,
                       (hipStream_t)stream, partial, amps, nb, n_slices, per);
    check_launch("slice_sum");
}

void finalize(const void *T, double *partial, int64_t units, int64_t t_us, int64_t per,
              const Gather &g, int c64, void *stream) {
    const int64_t total = units * per;
    if (c64)
        hipLaunchKernelGGL(k_finalize<float>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const float *)T, partial, units, t_us, per, g);
    else
        hipLaunchKernelGGL(k_finalize<double>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, (const double *)T, partial, units, t_us, per, g);
    check_launch("finalize");
}

}  // namespace launch
}  // namespace tns
