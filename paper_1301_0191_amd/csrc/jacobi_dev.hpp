// Cyclic two-sided Jacobi eigensolver for one small symmetric matrix held
// in LDS, run by a whole workgroup.  Parallel round-robin ordering: in every
// round the n indices form n/2 disjoint pairs (p, q); their rotations commute,
// so A <- J^T A J is applied as independent 2x2-block updates
// [A_pp' A_pq'; A_qp' A_qq'] <- R_k1^T [..] R_k2 for every pair of pairs
// (k1, k2), with one barrier per round.
#pragma once
#include <hip/hip_runtime.h>

namespace ambddc {

// A: n x n (ld = n) symmetric, overwritten (diagonal -> eigenvalues).
// V: n x n (ld = n) receives the eigenvectors (columns).
// rot: scratch of 4 * (n/2 + 1) doubles; red: 16 doubles.  n <= 128.
__device__ inline void jacobi_lds(double* A, double* V, int n, double* rot, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n * n; i += nt) V[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
  __syncthreads();
  if (n <= 1) return;
  const int np = (n + 1) & ~1;   // even player count (a dummy when n is odd)
  const int half = np / 2;
  const int m = np - 1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = tid; i < n * n; i += nt) {
      const int r = i % n, c = i / n;
      const double v = A[i] * A[i];
      if (r == c) dia += v; else off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dia += __shfl_xor(dia, o);
    }
    if ((tid & 63) == 0) { red[2 * (tid >> 6)] = off; red[2 * (tid >> 6) + 1] = dia; }
    __syncthreads();
    off = 0.0; dia = 0.0;
    for (int w = 0; w < (nt + 63) / 64; ++w) { off += red[2 * w]; dia += red[2 * w + 1]; }
    __syncthreads();
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int r = 0; r < m; ++r) {
      if (tid < half) {
        int p, q;
        if (tid == 0) { p = r; q = np - 1; }
        else { p = (r + tid) % m; q = (r - tid + m) % m; }
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p + q * n];
          if (apq != 0.0) {
            const double app = A[p + p * n], aqq = A[q + q * n];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        rot[4 * tid] = c;
        rot[4 * tid + 1] = s;
        rot[4 * tid + 2] = p;
        rot[4 * tid + 3] = (q < n) ? q : -1;
      }
      __syncthreads();
      for (int i = tid; i < half * half; i += nt) {
        const int k1 = i % half, k2 = i / half;
        const double c1 = rot[4 * k1], s1 = rot[4 * k1 + 1];
        const double c2 = rot[4 * k2], s2 = rot[4 * k2 + 1];
        const int p1 = int(rot[4 * k1 + 2]), q1 = int(rot[4 * k1 + 3]);
        const int p2 = int(rot[4 * k2 + 2]), q2 = int(rot[4 * k2 + 3]);
        const double a = A[p1 + p2 * n];
        const double b = q2 >= 0 ? A[p1 + q2 * n] : 0.0;
        const double cc = q1 >= 0 ? A[q1 + p2 * n] : 0.0;
        const double d = (q1 >= 0 && q2 >= 0) ? A[q1 + q2 * n] : 0.0;
        // rows: p' = c1 p - s1 q, q' = s1 p + c1 q; columns the same with (c2, s2)
        const double ra = c1 * a - s1 * cc, rb = c1 * b - s1 * d;
        const double rc = s1 * a + c1 * cc, rd = s1 * b + c1 * d;
        A[p1 + p2 * n] = c2 * ra - s2 * rb;
        if (q2 >= 0) A[p1 + q2 * n] = s2 * ra + c2 * rb;
        if (q1 >= 0) A[q1 + p2 * n] = c2 * rc - s2 * rd;
        if (q1 >= 0 && q2 >= 0) A[q1 + q2 * n] = s2 * rc + c2 * rd;
      }
      for (int i = tid; i < half * n; i += nt) {
        const int k = i / n, row = i % n;
        const int q = int(rot[4 * k + 3]);
        if (q < 0) continue;
        const int p = int(rot[4 * k + 2]);
        const double c = rot[4 * k], s = rot[4 * k + 1];
        const double vp = V[row + p * n], vq = V[row + q * n];
        V[row + p * n] = c * vp - s * vq;
        V[row + q * n] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

// Descending order of the diagonal of A (n <= 128): perm[r] = index of the
// r-th largest eigenvalue.  Ties are broken by index.
__device__ inline void sort_desc_lds(const double* A, int n, int* perm) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) {
    const double v = A[i + i * n];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double w = A[j + j * n];
      rank += (w > v) || (w == v && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
}

}  // namespace ambddc
