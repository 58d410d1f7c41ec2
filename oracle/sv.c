/*
 * Dense state-vector simulation in complex128, plain C.  TEST INFRASTRUCTURE
 * (part of the oracle; nothing in the GPU library uses it).
 *
 * The amplitude of bitstring b is <b|psi> with psi = U_G ... U_1 |0...0>
 * (Supplementary Information, Sec. II).  The state is 2^n complex numbers,
 * entry i holding the amplitude of the bitstring whose qubit q is bit q of i.
 * Each gate is applied in place, in circuit order:
 *   one-qubit gate U on q:  for every i with bit q clear,
 *     (psi[i], psi[i + 2^q]) <- U (psi[i], psi[i + 2^q]);
 *   two-qubit gate G on (a, b), basis |q_a q_b> with index 2 q_a + q_b:
 *     for every i with bits a and b clear, the four entries
 *     i + x_a 2^a + x_b 2^b (x = 2 x_a + x_b) are multiplied by G.
 * Memory: 16 * 2^n bytes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t insert_zero(uint64_t i, int pos) {
  const uint64_t low = i & ((1ULL << pos) - 1);
  return ((i >> pos) << (pos + 1)) | low;
}

static void apply1(double *psi, int n, int q, const double *u) {
  const int64_t half = (int64_t)1 << (n - 1);
  const uint64_t step = 1ULL << q;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < half; ++i) {
    const uint64_t i0 = insert_zero((uint64_t)i, q), i1 = i0 | step;
    const double ar = psi[2 * i0], ai = psi[2 * i0 + 1];
    const double br = psi[2 * i1], bi = psi[2 * i1 + 1];
    psi[2 * i0] = u[0] * ar - u[1] * ai + u[2] * br - u[3] * bi;
    psi[2 * i0 + 1] = u[0] * ai + u[1] * ar + u[2] * bi + u[3] * br;
    psi[2 * i1] = u[4] * ar - u[5] * ai + u[6] * br - u[7] * bi;
    psi[2 * i1 + 1] = u[4] * ai + u[5] * ar + u[6] * bi + u[7] * br;
  }
}

static void apply2(double *psi, int n, int a, int b, const double *g) {
  const int64_t quarter = (int64_t)1 << (n - 2);
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  const uint64_t sa = 1ULL << a, sb = 1ULL << b;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < quarter; ++i) {
    const uint64_t base = insert_zero(insert_zero((uint64_t)i, lo), hi);
    uint64_t idx[4];
    double vr[4], vi[4];
    for (int x = 0; x < 4; ++x) {
      idx[x] = base | ((x >> 1) ? sa : 0) | ((x & 1) ? sb : 0);
      vr[x] = psi[2 * idx[x]];
      vi[x] = psi[2 * idx[x] + 1];
    }
    for (int r = 0; r < 4; ++r) {
      double sr = 0.0, si = 0.0;
      for (int c = 0; c < 4; ++c) {
        const double gr = g[2 * (4 * r + c)], gi = g[2 * (4 * r + c) + 1];
        sr += gr * vr[c] - gi * vi[c];
        si += gr * vi[c] + gi * vr[c];
      }
      psi[2 * idx[r]] = sr;
      psi[2 * idx[r] + 1] = si;
    }
  }
}

/*
 * gates: kind[g] = 1 or 2; qa[g], qb[g] the qubits; mats holds 32 doubles
 * per gate (a 2x2 gate uses the first 8: row-major, interleaved re/im).
 * words[k]: bitstrings (bit q = qubit q); out: 2*k doubles.
 * Returns 0, or -1 if the state does not fit in memory.
 */
int sv_amplitudes(int n, int n_gates, const int *kind, const int *qa, const int *qb, const double *mats,
                  int64_t k, const uint64_t *words, double *out) {
  const size_t N = (size_t)1 << n;
  double *psi = (double *)malloc(2 * N * sizeof(double));
  if (!psi) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)(2 * N); ++i) psi[i] = 0.0;
  psi[0] = 1.0;
  for (int g = 0; g < n_gates; ++g) {
    if (kind[g] == 1)
      apply1(psi, n, qa[g], mats + 32 * (size_t)g);
    else
      apply2(psi, n, qa[g], qb[g], mats + 32 * (size_t)g);
  }
  for (int64_t i = 0; i < k; ++i) {
    out[2 * i] = psi[2 * words[i]];
    out[2 * i + 1] = psi[2 * words[i] + 1];
  }
  free(psi);
  return 0;
}
