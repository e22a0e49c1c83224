/*
 * CPU oracle (test infrastructure only): dense state-vector simulation in
 * complex128.
 *
 * What it computes is the plain definition of an output amplitude that the
 * paper's method reaches exactly: amp(s) = <s_1 ... s_N| U |0 ... 0>, with U the
 * time-ordered product of the circuit's explicit gate matrices (the paper's
 * problem statement for computing amplitudes, "two-sided circuit evolution"
 * paragraph, and the state of Eq. (1)).  None of the tensor-network steps
 * (gate splitting, SVD compression, overlap, cutting, contraction order) is
 * used here.
 *
 * Conventions: the dense index of bitstring s is sum_q s_q 2^(N-1-q); a
 * two-qubit matrix is indexed by 2*b(q0) + b(q1), rows = output.
 * Gate matrices are row-major complex numbers stored as interleaved
 * (re, im) doubles: 8 doubles for 2x2, 32 for 4x4.
 *
 * This file shares no code with the GPU library.  Only tests/, the smoke entry
 * point and the benchmark's CPU-baseline leg may load it.
 */
#include <stdint.h>
#include <string.h>
#include <omp.h>

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) {
    cplx r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}
static inline cplx cadd(cplx a, cplx b) { cplx r = { a.re + b.re, a.im + b.im }; return r; }

/* Insert a zero bit at position p (counted from the least significant bit). */
static inline uint64_t insert_zero(uint64_t x, int p) {
    uint64_t low = x & ((1ULL << p) - 1ULL);
    return ((x >> p) << (p + 1)) | low;
}

static void apply1(cplx *psi, int n, int q, const double *m) {
    const int p = n - 1 - q;
    const uint64_t half = 1ULL << (n - 1);
    cplx g[4];
    for (int i = 0; i < 4; ++i) { g[i].re = m[2 * i]; g[i].im = m[2 * i + 1]; }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)half; ++t) {
        uint64_t i0 = insert_zero((uint64_t)t, p);
        uint64_t i1 = i0 | (1ULL << p);
        cplx a = psi[i0], b = psi[i1];
        psi[i0] = cadd(cmul(g[0], a), cmul(g[1], b));
        psi[i1] = cadd(cmul(g[2], a), cmul(g[3], b));
    }
}

static void apply2(cplx *psi, int n, int q0, int q1, const double *m) {
    const int p0 = n - 1 - q0, p1 = n - 1 - q1;
    const int plo = p0 < p1 ? p0 : p1, phi = p0 < p1 ? p1 : p0;
    const uint64_t quarter = 1ULL << (n - 2);
    cplx g[16];
    for (int i = 0; i < 16; ++i) { g[i].re = m[2 * i]; g[i].im = m[2 * i + 1]; }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)quarter; ++t) {
        uint64_t base = insert_zero(insert_zero((uint64_t)t, plo), phi);
        uint64_t idx[4];
        /* basis index 2*b(q0) + b(q1) */
        idx[0] = base;
        idx[1] = base | (1ULL << p1);
        idx[2] = base | (1ULL << p0);
        idx[3] = base | (1ULL << p0) | (1ULL << p1);
        cplx in[4];
        for (int k = 0; k < 4; ++k) in[k] = psi[idx[k]];
        for (int r = 0; r < 4; ++r) {
            cplx acc = { 0.0, 0.0 };
            for (int c = 0; c < 4; ++c) acc = cadd(acc, cmul(g[4 * r + c], in[c]));
            psi[idx[r]] = acc;
        }
    }
}

/* psi must hold 2^n complex numbers (2^(n+1) doubles).  Returns 0 on success,
 * -1 on a bad argument.  The state starts as |0...0>. */
int oracle_sv_run(int n, double *psi_out, int n_gates, const int32_t *q0,
                  const int32_t *q1, const double *mats, int n_threads) {
    if (n < 2 || n > 40 || !psi_out) return -1;
    if (n_threads > 0) omp_set_num_threads(n_threads);
    cplx *psi = (cplx *)psi_out;
    const uint64_t dim = 1ULL << n;
    memset(psi, 0, dim * sizeof(cplx));
    psi[0].re = 1.0;
    for (int g = 0; g < n_gates; ++g) {
        if (q0[g] < 0 || q0[g] >= n) return -1;
        if (q1[g] < 0) {
            apply1(psi, n, q0[g], mats + 32 * (int64_t)g);
        } else {
            if (q1[g] >= n || q1[g] == q0[g]) return -1;
            apply2(psi, n, q0[g], q1[g], mats + 32 * (int64_t)g);
        }
    }
    return 0;
}

/* Gather amplitudes of bitstrings bits[b*n + q] from a computed state. */
void oracle_sv_gather(int n, const double *psi, int64_t n_bits, const uint8_t *bits,
                      double *amps) {
    for (int64_t b = 0; b < n_bits; ++b) {
        uint64_t idx = 0;
        for (int q = 0; q < n; ++q) idx = (idx << 1) | (bits[b * n + q] & 1u);
        amps[2 * b] = psi[2 * idx];
        amps[2 * b + 1] = psi[2 * idx + 1];
    }
}

int oracle_sv_max_threads(void) { return omp_get_max_threads(); }
