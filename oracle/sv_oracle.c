/*
 * Test oracle -- NOT part of the simulator.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load this file's library.
 *
 * A plain FP64 gate-by-gate state-vector simulator, written from the paper's
 * background section:
 *   - an n-qubit state is 2^n complex amplitudes (state definition);
 *   - a k-qubit gate is a 2^k x 2^k unitary U and maps psi -> U psi;
 *   - the one-qubit update (the equation following the state definition)
 *     pairs amplitude f(i) with f(i) + 2^q, f(i) = 2^(q+1) floor(i/2^q) + (i mod 2^q),
 *     so qubit q is bit q of the amplitude index.
 * Multi-qubit gates generalise the pairing: for each base index b whose bits
 * at the gate's qubits are zero, the 2^k amplitudes b + sum_j r_j 2^(q_j)
 * (r in [0, 2^k), bit j of r <-> the j-th listed qubit) form the vector that
 * U multiplies.  Gates are applied in sequence order.
 *
 * Gate matrices follow the OpenQASM 2 conventions (the paper defines none).
 * Nothing here is shared with the GPU library.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t kind, nq, q[3], flags;
    double p[3];
} og_gate;

enum { G_H, G_X, G_Y, G_Z, G_S, G_T, G_RX, G_RY, G_RZ, G_P, G_U3,
       G_CX, G_CZ, G_CP, G_RZZ, G_SWAP, G_NUM };

static const int arity[G_NUM] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2};

/* Row-major 2^nq x 2^nq matrix of gate g.  Returns nq, or -1 if unknown. */
int oracle_gate_matrix(const og_gate *g, double complex *U)
{
    if (g->kind >= G_NUM) return -1;
    int k = arity[g->kind];
    int d = 1 << k;
    for (int i = 0; i < d * d; ++i) U[i] = 0;
    double t = g->p[0];
    double c = cos(t / 2), s = sin(t / 2);
    switch (g->kind) {
    case G_H:  U[0] = U[1] = U[2] = 1 / sqrt(2.0); U[3] = -1 / sqrt(2.0); break;
    case G_X:  U[1] = U[2] = 1; break;
    case G_Y:  U[1] = -I; U[2] = I; break;
    case G_Z:  U[0] = 1; U[3] = -1; break;
    case G_S:  U[0] = 1; U[3] = I; break;
    case G_T:  U[0] = 1; U[3] = cexp(I * M_PI / 4); break;
    case G_RX: U[0] = c; U[1] = -I * s; U[2] = -I * s; U[3] = c; break;
    case G_RY: U[0] = c; U[1] = -s; U[2] = s; U[3] = c; break;
    case G_RZ: U[0] = cexp(-I * t / 2); U[3] = cexp(I * t / 2); break;
    case G_P:  U[0] = 1; U[3] = cexp(I * t); break;
    case G_U3: {
        double ph = g->p[1], la = g->p[2];
        U[0] = c;
        U[1] = -cexp(I * la) * s;
        U[2] = cexp(I * ph) * s;
        U[3] = cexp(I * (ph + la)) * c;
        break;
    }
    /* two-qubit: matrix index r = b0 + 2 b1, b0 <-> q[0], b1 <-> q[1] */
    case G_CX:  /* flips q[1] when q[0] = 1: |1> <-> |3> */
        U[0 * 4 + 0] = 1; U[2 * 4 + 2] = 1; U[3 * 4 + 1] = 1; U[1 * 4 + 3] = 1; break;
    case G_CZ:
        U[0] = 1; U[5] = 1; U[10] = 1; U[15] = -1; break;
    case G_CP:
        U[0] = 1; U[5] = 1; U[10] = 1; U[15] = cexp(I * t); break;
    case G_RZZ:  /* exp(-i t/2 Z(x)Z): even parity -> e^{-it/2}, odd -> e^{+it/2} */
        U[0] = cexp(-I * t / 2); U[5] = cexp(I * t / 2);
        U[10] = cexp(I * t / 2); U[15] = cexp(-I * t / 2); break;
    case G_SWAP:
        U[0] = 1; U[2 * 4 + 1] = 1; U[1 * 4 + 2] = 1; U[15] = 1; break;
    }
    return k;
}

/* Insert a zero bit at position pos of x. */
static inline uint64_t insert_zero(uint64_t x, int pos)
{
    uint64_t lo = x & ((1ull << pos) - 1);
    return ((x >> pos) << (pos + 1)) | lo;
}

/* Apply one gate: psi is 2^n complex128 values (interleaved re, im). */
int oracle_apply_gate(int n, double complex *psi, const og_gate *g)
{
    double complex U[64];
    int k = oracle_gate_matrix(g, U);
    if (k < 0 || (int)g->nq != k) return -1;
    for (int j = 0; j < k; ++j) {
        if ((int)g->q[j] >= n) return -1;
        for (int i = 0; i < j; ++i) if (g->q[i] == g->q[j]) return -1;
    }
    int d = 1 << k;
    /* qubits sorted ascending, for building base indices */
    int srt[3];
    for (int j = 0; j < k; ++j) srt[j] = (int)g->q[j];
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (srt[b] < srt[a]) { int tmp = srt[a]; srt[a] = srt[b]; srt[b] = tmp; }
    uint64_t offs[8];
    for (int r = 0; r < d; ++r) {
        uint64_t o = 0;
        for (int j = 0; j < k; ++j) if ((r >> j) & 1) o |= 1ull << g->q[j];
        offs[r] = o;
    }
    int64_t nbase = (int64_t)1 << (n - k);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nbase; ++i) {
        uint64_t b = (uint64_t)i;
        for (int j = 0; j < k; ++j) b = insert_zero(b, srt[j]);
        double complex v[8], w[8];
        for (int r = 0; r < d; ++r) v[r] = psi[b + offs[r]];
        for (int r = 0; r < d; ++r) {
            double complex acc = 0;
            for (int c = 0; c < d; ++c) acc += U[r * d + c] * v[c];
            w[r] = acc;
        }
        for (int r = 0; r < d; ++r) psi[b + offs[r]] = w[r];
    }
    return 0;
}

/* Apply gates[0..count) in order.  Returns 0, or -1-(index of a bad gate). */
int64_t oracle_run(int n, double *psi, const og_gate *gates, int64_t count)
{
    for (int64_t i = 0; i < count; ++i)
        if (oracle_apply_gate(n, (double complex *)psi, &gates[i]) != 0) return -1 - i;
    return 0;
}

/* Plain FP64 inner product <a|b> = sum conj(a_i) b_i, sequential order. */
void oracle_inner(const double *a, const double *b, int64_t N, double out[2])
{
    double re = 0, im = 0;
    for (int64_t i = 0; i < N; ++i) {
        double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
    out[0] = re; out[1] = im;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later parallel loops (1 = a single core). */
void oracle_set_threads(int t)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
