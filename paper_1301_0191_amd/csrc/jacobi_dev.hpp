// Cyclic two-sided Jacobi eigensolver for one small symmetric matrix held
// in LDS, run by a whole workgroup (parallel round-robin ordering: in every
// round n/2 disjoint rotations are computed and applied together).
#pragma once
#include <hip/hip_runtime.h>

namespace ambddc {

// A: n x n (ld = n) symmetric, overwritten (diagonal -> eigenvalues).
// V: n x n (ld = n) receives the eigenvectors (columns).
// rot: scratch of 4 * ((n+1)/2) doubles.  n <= 128.
__device__ inline void jacobi_lds(double* A, double* V, int n, double* rot, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n * n; i += nt) V[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
  __syncthreads();
  if (n <= 1) return;
  const int np = (n + 1) & ~1;   // even player count (a dummy when n is odd)
  const int half = np / 2;
  const int m = np - 1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test on the off-diagonal mass
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
      // rows: A <- J^T A
      for (int i = tid; i < half * n; i += nt) {
        const int k = i / n, col = i % n;
        const int q = int(rot[4 * k + 3]);
        if (q < 0) continue;
        const int p = int(rot[4 * k + 2]);
        const double c = rot[4 * k], s = rot[4 * k + 1];
        const double ap = A[p + col * n], aq = A[q + col * n];
        A[p + col * n] = c * ap - s * aq;
        A[q + col * n] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int i = tid; i < half * n; i += nt) {
        const int k = i / n, row = i % n;
        const int q = int(rot[4 * k + 3]);
        if (q < 0) continue;
        const int p = int(rot[4 * k + 2]);
        const double c = rot[4 * k], s = rot[4 * k + 1];
        const double ap = A[row + p * n], aq = A[row + q * n];
        A[row + p * n] = c * ap - s * aq;
        A[row + q * n] = s * ap + c * aq;
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
