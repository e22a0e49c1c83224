// Evolution-side kernels, all complex128 (FP64):
//   fuse/split   -- fused two-qubit gate and its SVD split into P, Q (Eq. (2))
//   init         -- product-state site tensors (Eq. (1) and the bra <s|)
//   gate_apply   -- P or Q applied to one site, widening one bond by chi
//                   (Eqs. (3)-(4))
//   svd_compress -- one-sided Jacobi SVD of the widened site, keeping the
//                   planned rank (Eq. (5)); singular values below the
//                   relative cutoff are set to zero
//   absorb       -- S V folded into the neighbouring site (Eq. (6))
//   merge        -- overlap site tensors C = sum_sigma A^sigma B^sigma (Eq. (8))
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace tns {
namespace {

struct cdbl {
    double x, y;
};
__device__ __forceinline__ cdbl cmul(cdbl a, cdbl b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cdbl cadd(cdbl a, cdbl b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cdbl cconj(cdbl a) { return {a.x, -a.y}; }
__device__ __forceinline__ cdbl cscale(cdbl a, double s) { return {a.x * s, a.y * s}; }

// Jacobi rotation that orthogonalises two rows x, y with Gram entries
// alpha = |x|^2, beta = |y|^2, gamma = <x, y> = sum x conj(y).  With
// gamma = |gamma| e^{i phi}, the Hermitian 2x2 Gram matrix is diagonalised by
// G = diag(1, e^{-i phi}) [[c, s], [-s, c]] (the real symmetric Schur
// rotation of Golub & Van Loan).  New rows: x' = c x - s e^{i phi} y,
// y' = s x + c e^{i phi} y; accumulated left factor columns:
// J_p' = c J_p - s e^{-i phi} J_q, J_q' = s J_p + c e^{-i phi} J_q.
struct Rot {
    double c, s;
    cdbl ph;   // e^{i phi}
};
// floor: rows whose squared norm is at or below it count as zero and are not
// rotated.  Rows left over from exact cancellations can be as small as
// 1e-150 of the matrix scale; their Gram entries are then denormal, the
// phase gamma / |gamma| loses its unit modulus and the rotation stops being
// unitary, which breaks the factorisation A = J W the compression relies on.
// Not rotating such a pair is the identity, which is always exact.  The
// threshold is formed as sqrt(alpha) sqrt(beta) (alpha * beta can underflow)
// and the phase is renormalised.
__device__ __forceinline__ bool make_rot(double alpha, double beta, cdbl gamma, double tol,
                                         double floor, Rot &r) {
    if (!(alpha > floor) || !(beta > floor)) return false;
    double g = sqrt(gamma.x * gamma.x + gamma.y * gamma.y);
    if (!(g > tol * sqrt(alpha) * sqrt(beta))) return false;
    r.ph = {gamma.x / g, gamma.y / g};
    const double pn = sqrt(r.ph.x * r.ph.x + r.ph.y * r.ph.y);
    r.ph = {r.ph.x / pn, r.ph.y / pn};
    double zeta = (beta - alpha) / (2.0 * g);
    double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    r.c = 1.0 / sqrt(1.0 + t * t);
    r.s = r.c * t;
    return true;
}
__device__ __forceinline__ void rot_rows(cdbl &x, cdbl &y, const Rot &r) {
    cdbl py = cmul(r.ph, y);
    cdbl nx = {r.c * x.x - r.s * py.x, r.c * x.y - r.s * py.y};
    cdbl ny = {r.s * x.x + r.c * py.x, r.s * x.y + r.c * py.y};
    x = nx;
    y = ny;
}
__device__ __forceinline__ void rot_cols(cdbl &jp, cdbl &jq, const Rot &r) {
    cdbl pq = cmul(cconj(r.ph), jq);
    cdbl np = {r.c * jp.x - r.s * pq.x, r.c * jp.y - r.s * pq.y};
    cdbl nq = {r.s * jp.x + r.c * pq.x, r.s * jp.y + r.c * pq.y};
    jp = np;
    jq = nq;
}

constexpr double kJacobiTol = 1e-14;
constexpr int kMaxSweeps = 40;
// zero-row floor of the Jacobi rotations, relative to the largest squared
// row norm of the matrix, with an absolute floor above the denormal range
__device__ __forceinline__ double jacobi_floor(double max_row2) { return fmax(1e-200 * max_row2, 1e-290); }

// ---------------------------------------------------------------------------
// fuse + split: one thread per fused gate, one per qubit boundary chain

__device__ void chain_product(const double *mats, const int32_t *chain, const int32_t *off,
                              const int32_t *len, int id, cdbl out[2][2]) {
    out[0][0] = {1, 0}; out[0][1] = {0, 0}; out[1][0] = {0, 0}; out[1][1] = {1, 0};
    if (id < 0) return;
    for (int t = 0; t < len[id]; ++t) {
        const double *g = mats + 32 * (int64_t)chain[off[id] + t];
        cdbl m[2][2] = {{{g[0], g[1]}, {g[2], g[3]}}, {{g[4], g[5]}, {g[6], g[7]}}};
        cdbl r[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) r[i][j] = cadd(cmul(m[i][0], out[0][j]), cmul(m[i][1], out[1][j]));
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) out[i][j] = r[i][j];
    }
}

__global__ void k_fuse_split(const double *__restrict__ mats, const int32_t *chain,
                             const int32_t *chain_off, const int32_t *chain_len,
                             const FuseDesc *fuse, int n_fuse, double *__restrict__ pq,
                             int n_qubits, const int32_t *ket_chain, const int32_t *bra_chain,
                             double *ket_vec, double *bra_mat) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_fuse) {
        const int q = t - n_fuse;
        if (q >= n_qubits) return;
        cdbl g[2][2];
        chain_product(mats, chain, chain_off, chain_len, ket_chain[q], g);
        // initial ket site: G |0> (first column)
        ket_vec[4 * q + 0] = g[0][0].x; ket_vec[4 * q + 1] = g[0][0].y;
        ket_vec[4 * q + 2] = g[1][0].x; ket_vec[4 * q + 3] = g[1][0].y;
        chain_product(mats, chain, chain_off, chain_len, bra_chain[q], g);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                bra_mat[8 * q + 2 * (2 * i + j)] = g[i][j].x;
                bra_mat[8 * q + 2 * (2 * i + j) + 1] = g[i][j].y;
            }
        return;
    }
    const FuseDesc f = fuse[t];
    const double *gb = mats + 32 * (int64_t)f.gate;
    cdbl O[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) O[r][c] = {gb[2 * (4 * r + c)], gb[2 * (4 * r + c) + 1]};
    cdbl A0[2][2], A1[2][2], B0[2][2], B1[2][2];
    chain_product(mats, chain, chain_off, chain_len, f.pre0, A0);
    chain_product(mats, chain, chain_off, chain_len, f.pre1, A1);
    chain_product(mats, chain, chain_off, chain_len, f.post0, B0);
    chain_product(mats, chain, chain_off, chain_len, f.post1, B1);
    // O' = (B0 (x) B1) O (A0 (x) A1);  (X (x) Y)[(a b), (c d)] = X[a][c] Y[b][d]
    cdbl T[4][4], F[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            cdbl acc = {0, 0};
            for (int k = 0; k < 4; ++k)
                acc = cadd(acc, cmul(O[r][k], cmul(A0[k >> 1][c >> 1], A1[k & 1][c & 1])));
            T[r][c] = acc;
        }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            cdbl acc = {0, 0};
            for (int k = 0; k < 4; ++k)
                acc = cadd(acc, cmul(cmul(B0[r >> 1][k >> 1], B1[r & 1][k & 1]), T[k][c]));
            F[r][c] = acc;
        }
    // the bra side applies the transpose (no conjugation) to <s|
    if (f.transpose)
        for (int r = 0; r < 4; ++r)
            for (int c = r + 1; c < 4; ++c) {
                cdbl tmp = F[r][c]; F[r][c] = F[c][r]; F[c][r] = tmp;
            }
    // Eq. (2): M[(s0' s0), (s1' s1)] = O'[(s0' s1'), (s0 s1)] = sum_s P[s0',s0,s] Q[s1',s1,s]
    cdbl W[4][4], J[4][4];
    for (int a0p = 0; a0p < 2; ++a0p)
        for (int a0 = 0; a0 < 2; ++a0)
            for (int b0p = 0; b0p < 2; ++b0p)
                for (int b0 = 0; b0 < 2; ++b0)
                    W[2 * a0p + a0][2 * b0p + b0] = F[2 * a0p + b0p][2 * a0 + b0];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) J[r][c] = {r == c ? 1.0 : 0.0, 0.0};
    double max_row2 = 0;
    for (int r = 0; r < 4; ++r) {
        double a = 0;
        for (int c = 0; c < 4; ++c) a += W[r][c].x * W[r][c].x + W[r][c].y * W[r][c].y;
        max_row2 = fmax(max_row2, a);
    }
    const double floor4 = jacobi_floor(max_row2);
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        bool changed = false;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                double al = 0, be = 0;
                cdbl ga = {0, 0};
                for (int c = 0; c < 4; ++c) {
                    al += W[p][c].x * W[p][c].x + W[p][c].y * W[p][c].y;
                    be += W[q][c].x * W[q][c].x + W[q][c].y * W[q][c].y;
                    ga = cadd(ga, cmul(W[p][c], cconj(W[q][c])));
                }
                Rot r;
                if (!make_rot(al, be, ga, kJacobiTol, floor4, r)) continue;
                changed = true;
                for (int c = 0; c < 4; ++c) rot_rows(W[p][c], W[q][c], r);
                for (int c = 0; c < 4; ++c) rot_cols(J[c][p], J[c][q], r);
            }
        if (!changed) break;
    }
    double sig[4];
    int idx[4] = {0, 1, 2, 3};
    for (int s = 0; s < 4; ++s) {
        double a = 0;
        for (int c = 0; c < 4; ++c) a += W[s][c].x * W[s][c].x + W[s][c].y * W[s][c].y;
        sig[s] = sqrt(a);
    }
    for (int i = 0; i < 4; ++i)   // descending order of singular values
        for (int j = i + 1; j < 4; ++j)
            if (sig[idx[j]] > sig[idx[i]]) { int tmp = idx[i]; idx[i] = idx[j]; idx[j] = tmp; }
    double *P = pq + 64 * (int64_t)t;   // [2 s'][2 s][4 chi] complex
    double *Q = P + 32;
    for (int s = 0; s < 4; ++s) {
        const int k = idx[s];
        const bool keep = s < f.chi && sig[k] > 0.0;
        const double rt = keep ? sqrt(sig[k]) : 0.0;
        for (int a = 0; a < 4; ++a) {
            // a = 2 * s' + s  (row of M for P, column of M for Q)
            cdbl pv = keep ? cscale(J[a][k], rt) : cdbl{0, 0};
            cdbl qv = keep ? cscale(W[k][a], 1.0 / rt) : cdbl{0, 0};
            P[2 * (4 * a + s)] = pv.x; P[2 * (4 * a + s) + 1] = pv.y;
            Q[2 * (4 * a + s)] = qv.x; Q[2 * (4 * a + s) + 1] = qv.y;
        }
    }
}

// ---------------------------------------------------------------------------
// product-state initialisation

__global__ void k_init_ket(const double *ket_vec, int q, double *site) {
    if (threadIdx.x < 4) site[threadIdx.x] = ket_vec[4 * q + threadIdx.x];
}

// <s| H: row s_q of the trailing single-qubit product H.  For an open qubit
// the output bit stays free: B[sigma][o] = H[o][sigma], an extra leg of size 2.
__global__ void k_init_bra(const uint8_t *bits, int n_qubits, int64_t nb, int q,
                           const double *bra_mat, double *site, int64_t stride, int open) {
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double *o = site + 2 * b * stride;
    if (open) {
        const double *h = bra_mat + 8 * q;   // H[r][c] at 2 * (2 r + c)
        for (int sg = 0; sg < 2; ++sg)
            for (int ob = 0; ob < 2; ++ob) {
                o[2 * (2 * sg + ob)] = h[2 * (2 * ob + sg)];
                o[2 * (2 * sg + ob) + 1] = h[2 * (2 * ob + sg) + 1];
            }
        return;
    }
    const int s = bits[b * n_qubits + q] & 1;
    const double *h = bra_mat + 8 * q + 4 * s;
    o[0] = h[0]; o[1] = h[1]; o[2] = h[2]; o[3] = h[3];
}

// ---------------------------------------------------------------------------
// Eqs. (3)-(4): A'[s', .., (a_m chi_idx), ..] = sum_s G[s', s, chi_idx] A[s, .., a_m, ..]

struct LegSplit {
    int64_t outer;   // product of axes strictly between the physical axis and the leg
    int64_t D;       // leg dimension
    int64_t inner;   // product of axes after the leg
};
__host__ __device__ inline LegSplit leg_split(const SiteShape &s, int leg) {
    LegSplit r{1, s.d[1 + leg], 1};
    for (int a = 1; a < 1 + leg; ++a) r.outer *= s.d[a];
    for (int a = 2 + leg; a < s.n; ++a) r.inner *= s.d[a];
    return r;
}

__global__ void k_gate_apply(const double *__restrict__ in, double *__restrict__ out, int64_t nb,
                             int64_t in_stride, int64_t out_stride, LegSplit ls, int chi,
                             const double *__restrict__ g) {
    const int64_t per = 2 * ls.outer * ls.D * chi * ls.inner;
    const int64_t total = per * nb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / per;
        int64_t i = t - b * per;
        const int64_t inner = i % ls.inner; i /= ls.inner;
        const int s = (int)(i % chi); i /= chi;
        const int64_t a = i % ls.D; i /= ls.D;
        const int64_t o = i % ls.outer; i /= ls.outer;
        const int sp = (int)i;
        const double *src = in + 2 * b * in_stride;
        cdbl acc = {0, 0};
        for (int sg = 0; sg < 2; ++sg) {
            const int64_t off = ((sg * ls.outer + o) * ls.D + a) * ls.inner + inner;
            cdbl v = {src[2 * off], src[2 * off + 1]};
            const double *gg = g + 2 * (4 * (2 * sp + sg) + s);
            acc = cadd(acc, cmul(cdbl{gg[0], gg[1]}, v));
        }
        double *dst = out + 2 * (b * out_stride + (t - b * per));
        dst[0] = acc.x;
        dst[1] = acc.y;
    }
}

// ---------------------------------------------------------------------------
// Eq. (5): one-sided (Hestenes) Jacobi SVD of the widened site tensor viewed
// as M[(s', other bonds)][leg], R rows < C columns.  The R rows are rotated
// until mutually orthogonal (parallel round-robin ordering, n/2 disjoint pairs
// per round); the accumulated rotations J are the left singular vectors and
// the rotated rows are S V.  All R singular triplets are kept (the planned
// rank), sorted by decreasing singular value: the new site tensor is J and
// V' = S V goes to the neighbour (Eq. (6)).  One workgroup per matrix, the
// matrix and J held in LDS.

constexpr int kSvdThreads = 256;

// cut2: a kept row of S V whose squared norm is at most cut2 times the
// largest is written as exact zeros (a singular value below the relative
// cutoff counts as zero; the planned shape is unchanged)
__global__ __launch_bounds__(kSvdThreads) void k_svd_rows(
    const double *__restrict__ in, double *__restrict__ out_site, double *__restrict__ vp,
    int64_t in_stride, int64_t out_stride, int64_t vp_stride, LegSplit ls, int R, double cut2) {
    extern __shared__ double lds[];
    const int C = (int)ls.D;
    cdbl *W = reinterpret_cast<cdbl *>(lds);          // [R][C]
    cdbl *J = W + (int64_t)R * C;                      // [R][R]
    double *nrm = reinterpret_cast<double *>(J + (int64_t)R * R);   // [R]
    int *perm = reinterpret_cast<int *>(nrm + R);      // [R]
    __shared__ int changed;
    __shared__ double wmax[kSvdThreads / 64];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const double *src = in + 2 * b * in_stride;
    // gather rows: row rho = (outer index incl. physical axis, inner index)
    for (int e = tid; e < R * C; e += kSvdThreads) {
        const int rho = e / C, c = e % C;
        const int64_t o = rho / ls.inner, inr = rho % ls.inner;
        const int64_t off = (o * ls.D + c) * ls.inner + inr;
        W[e] = {src[2 * off], src[2 * off + 1]};
    }
    for (int e = tid; e < R * R; e += kSvdThreads) J[e] = {(e / R) == (e % R) ? 1.0 : 0.0, 0.0};
    __syncthreads();
    // largest squared row norm: the scale of the zero-row floor
    double mx0 = 0;
    for (int s = tid; s < R; s += kSvdThreads) {
        double a = 0;
        for (int c = 0; c < C; ++c) a += W[s * C + c].x * W[s * C + c].x + W[s * C + c].y * W[s * C + c].y;
        mx0 = fmax(mx0, a);
    }
    for (int m = 32; m > 0; m >>= 1) mx0 = fmax(mx0, __shfl_xor(mx0, m, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = mx0;
    __syncthreads();
    double scale0 = 0;
    for (int w = 0; w < kSvdThreads / 64; ++w) scale0 = fmax(scale0, wmax[w]);
    const double zfloor = jacobi_floor(scale0);
    __syncthreads();   // wmax is reused below

    const int Rp = R + (R & 1);
    const int npairs = Rp / 2;
    int G = 64;
    while (G > 1 && G * npairs > kSvdThreads) G >>= 1;
    const int pi = tid / G, gl = tid % G;
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) changed = 0;
        __syncthreads();
        for (int round = 0; round < Rp - 1; ++round) {
            int p = -1, q = -1;
            if (pi < npairs) {
                // circle method: position 0 fixed, others rotate each round
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (Rp - 1)) + 1; };
                p = player(pi);
                q = player(Rp - 1 - pi);
                if (p > q) { int tmp = p; p = q; q = tmp; }
            }
            const bool active = pi < npairs && q < R;
            double al = 0, be = 0;
            cdbl ga = {0, 0};
            if (active) {
                for (int c = gl; c < C; c += G) {
                    cdbl x = W[p * C + c], y = W[q * C + c];
                    al += x.x * x.x + x.y * x.y;
                    be += y.x * y.x + y.y * y.y;
                    ga = cadd(ga, cmul(x, cconj(y)));
                }
            }
            for (int m = 1; m < G; m <<= 1) {
                al += __shfl_xor(al, m, 64);
                be += __shfl_xor(be, m, 64);
                ga.x += __shfl_xor(ga.x, m, 64);
                ga.y += __shfl_xor(ga.y, m, 64);
            }
            Rot r;
            if (active && make_rot(al, be, ga, kJacobiTol, zfloor, r)) {
                for (int c = gl; c < C; c += G) rot_rows(W[p * C + c], W[q * C + c], r);
                for (int rr = gl; rr < R; rr += G) rot_cols(J[rr * R + p], J[rr * R + q], r);
                if (gl == 0) changed = 1;
            }
            __syncthreads();
        }
        if (!changed) break;
        __syncthreads();
    }
    // singular values and their descending order
    double mx = 0;
    for (int s = tid; s < R; s += kSvdThreads) {
        double a = 0;
        for (int c = 0; c < C; ++c) a += W[s * C + c].x * W[s * C + c].x + W[s * C + c].y * W[s * C + c].y;
        nrm[s] = a;
        mx = fmax(mx, a);
    }
    for (int m = 32; m > 0; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = mx;
    __syncthreads();
    double smax = 0;
    for (int w = 0; w < kSvdThreads / 64; ++w) smax = fmax(smax, wmax[w]);
    const double zero_below = cut2 * smax;
    for (int s = tid; s < R; s += kSvdThreads) {
        int rank = 0;
        for (int t = 0; t < R; ++t) rank += (nrm[t] > nrm[s]) || (nrm[t] == nrm[s] && t < s);
        perm[rank] = s;
    }
    __syncthreads();
    double *dst = out_site + 2 * b * out_stride;
    for (int e = tid; e < R * R; e += kSvdThreads) {
        const int rho = e / R, sp = e % R;
        const int64_t o = rho / ls.inner, inr = rho % ls.inner;
        const int64_t off = (o * R + sp) * ls.inner + inr;
        cdbl v = J[rho * R + perm[sp]];
        dst[2 * off] = v.x;
        dst[2 * off + 1] = v.y;
    }
    double *vd = vp + 2 * b * vp_stride;
    for (int e = tid; e < R * C; e += kSvdThreads) {
        const int sp = e / C, c = e % C;
        const bool zero = nrm[perm[sp]] <= zero_below;
        cdbl v = zero ? cdbl{0.0, 0.0} : W[perm[sp] * C + c];
        vd[2 * e] = v.x;
        vd[2 * e + 1] = v.y;
    }
}

// Eq. (6): A^l[.., s', ..] = sum_c A^l[.., c, ..] V'[s', c]
__global__ void k_absorb(const double *__restrict__ in, const double *__restrict__ vp,
                         double *__restrict__ out, int64_t nb, int64_t in_stride,
                         int64_t vp_stride, int64_t out_stride, LegSplit ls, int r) {
    const int64_t per = ls.outer * r * ls.inner;   // ls.outer includes the physical axis
    const int64_t total = per * nb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / per;
        int64_t i = t - b * per;
        const int64_t inner = i % ls.inner; i /= ls.inner;
        const int sp = (int)(i % r); i /= r;
        const int64_t o = i;   // includes the physical axis
        const double *src = in + 2 * b * in_stride;
        const double *v = vp + 2 * (b * vp_stride + (int64_t)sp * ls.D);
        cdbl acc = {0, 0};
        for (int64_t c = 0; c < ls.D; ++c) {
            const int64_t off = (o * ls.D + c) * ls.inner + inner;
            acc = cadd(acc, cmul(cdbl{src[2 * off], src[2 * off + 1]}, cdbl{v[2 * c], v[2 * c + 1]}));
        }
        double *dst = out + 2 * (b * out_stride + (t - b * per));
        dst[0] = acc.x;
        dst[1] = acc.y;
    }
}

// ---------------------------------------------------------------------------
// Eq. (8): C[(a_1 b_1), ..] = sum_sigma A[sigma, a_1, ..] B[sigma, b_1, ..]
// (no complex conjugation: the bra side already carries <s| U_2)

struct MergeShape {
    int32_t n;                  // bonds
    int32_t da[kMaxDeg], db[kMaxDeg];
    int64_t ket_half, bra_half; // elements per physical value
};

template <typename OutT>
__global__ void k_merge(const double *__restrict__ ket, const double *__restrict__ bra,
                        OutT *__restrict__ out, int64_t nb, int64_t bra_stride,
                        int64_t out_stride, MergeShape ms) {
    int64_t per = 1;
    for (int i = 0; i < ms.n; ++i) per *= (int64_t)ms.da[i] * ms.db[i];
    const int64_t total = per * nb;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / per;
        int64_t i = t - b * per;
        int64_t ka = 0, kb = 0, sa = 1, sb = 1;
        for (int l = ms.n - 1; l >= 0; --l) {
            const int64_t dd = (int64_t)ms.da[l] * ms.db[l];
            const int64_t cidx = i % dd;
            i /= dd;
            ka += (cidx / ms.db[l]) * sa;
            kb += (cidx % ms.db[l]) * sb;
            sa *= ms.da[l];
            sb *= ms.db[l];
        }
        const double *br = bra + 2 * b * bra_stride;
        cdbl a0 = {ket[2 * ka], ket[2 * ka + 1]};
        cdbl a1 = {ket[2 * (ka + ms.ket_half)], ket[2 * (ka + ms.ket_half) + 1]};
        cdbl b0 = {br[2 * kb], br[2 * kb + 1]};
        cdbl b1 = {br[2 * (kb + ms.bra_half)], br[2 * (kb + ms.bra_half) + 1]};
        cdbl v = cadd(cmul(a0, b0), cmul(a1, b1));
        OutT *o = out + 2 * (b * out_stride + (t - b * per));
        o[0] = (OutT)v.x;
        o[1] = (OutT)v.y;
    }
}

inline unsigned grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

inline void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(TNS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace launch {

void fuse_split(const double *mats, const int32_t *chain, const int32_t *chain_off,
                const int32_t *chain_len, const FuseDesc *fuse, int n_fuse, double *pq,
                int n_qubits, const int32_t *ket_chain, const int32_t *bra_chain,
                double *ket_vec, double *bra_mat, void *stream) {
    const int total = n_fuse + n_qubits;
    hipLaunchKernelGGL(k_fuse_split, dim3((total + 63) / 64), dim3(64), 0, (hipStream_t)stream,
                       mats, chain, chain_off, chain_len, fuse, n_fuse, pq, n_qubits, ket_chain,
                       bra_chain, ket_vec, bra_mat);
    check_launch("fuse_split");
}

void init_ket(const double *ket_vec, int q, double *site, void *stream) {
    hipLaunchKernelGGL(k_init_ket, dim3(1), dim3(64), 0, (hipStream_t)stream, ket_vec, q, site);
    check_launch("init_ket");
}

void init_bra(const uint8_t *bits, int n_qubits, int64_t nb, int q, const double *bra_mat,
              double *site, int64_t stride, int open, void *stream) {
    hipLaunchKernelGGL(k_init_bra, dim3(grid_for(nb, 256)), dim3(256), 0, (hipStream_t)stream,
                       bits, n_qubits, nb, q, bra_mat, site, stride, open);
    check_launch("init_bra");
}

void gate_apply(const double *in, double *out, int64_t nb, int64_t in_stride,
                int64_t out_stride, SiteShape s, int leg, int chi, const double *g,
                void *stream) {
    LegSplit ls = leg_split(s, leg);
    const int64_t total = 2 * ls.outer * ls.D * chi * ls.inner * nb;
    hipLaunchKernelGGL(k_gate_apply, dim3(grid_for(total, 256)), dim3(256), 0,
                       (hipStream_t)stream, in, out, nb, in_stride, out_stride, ls, chi, g);
    check_launch("gate_apply");
}

size_t svd_lds_bytes(int R, int C) {
    return (size_t)R * C * 16 + (size_t)R * R * 16 + (size_t)R * 8 + (size_t)R * 4;
}

void svd_compress(const double *in, double *out_site, double *vp, int64_t nb,
                  int64_t in_stride, int64_t out_stride, int64_t vp_stride, SiteShape s,
                  int leg, double cutoff, void *stream) {
    LegSplit ls = leg_split(s, leg);
    const int64_t rows = 2 * ls.outer * ls.inner;
    const size_t lds = svd_lds_bytes((int)rows, (int)ls.D);
    if (rows >= ls.D || rows > 512 || lds > 160 * 1024)
        fail(TNS_E_UNSUPPORTED, "SVD block too large for one workgroup (" + std::to_string(rows) +
                                    " x " + std::to_string(ls.D) + ")");
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_svd_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    // the physical axis folds into "outer" for row indexing
    LegSplit rs = ls;
    rs.outer = 2 * ls.outer;
    hipLaunchKernelGGL(k_svd_rows, dim3((unsigned)nb), dim3(kSvdThreads), lds, (hipStream_t)stream,
                       in, out_site, vp, in_stride, out_stride, vp_stride, rs, (int)rows, cutoff * cutoff);
    check_launch("svd_compress");
}

void absorb(const double *in, const double *vp, double *out, int64_t nb, int64_t in_stride,
            int64_t vp_stride, int64_t out_stride, SiteShape s, int leg, int r, void *stream) {
    LegSplit ls = leg_split(s, leg);
    LegSplit rs = ls;
    rs.outer = 2 * ls.outer;
    const int64_t total = 2 * ls.outer * r * ls.inner * nb;
    hipLaunchKernelGGL(k_absorb, dim3(grid_for(total, 256)), dim3(256), 0, (hipStream_t)stream,
                       in, vp, out, nb, in_stride, vp_stride, out_stride, rs, r);
    check_launch("absorb");
}

void merge(const double *ket, const double *bra, void *out, int64_t nb, int64_t bra_stride,
           int64_t out_stride, SiteShape sk, SiteShape sb, int c64, void *stream) {
    MergeShape ms{};
    ms.n = sk.n - 1;
    int64_t per = 1, kh = 1, bh = 1;
    for (int i = 0; i < ms.n; ++i) {
        ms.da[i] = sk.d[1 + i];
        ms.db[i] = sb.d[1 + i];
        per *= (int64_t)ms.da[i] * ms.db[i];
        kh *= ms.da[i];
        bh *= ms.db[i];
    }
    ms.ket_half = kh;
    ms.bra_half = bh;
    const int64_t total = per * nb;
    if (c64)
        hipLaunchKernelGGL(k_merge<float>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, ket, bra, (float *)out, nb, bra_stride, out_stride, ms);
    else
        hipLaunchKernelGGL(k_merge<double>, dim3(grid_for(total, 256)), dim3(256), 0,
                           (hipStream_t)stream, ket, bra, (double *)out, nb, bra_stride, out_stride, ms);
    check_launch("merge");
}

}  // namespace launch
}  // namespace tns
