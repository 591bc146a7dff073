// Cyclic two-sided Jacobi eigensolver for one small symmetric matrix held
// in LDS, run by a workgroup of 32 * TPP threads.
//
// Parallel round-robin ordering: in every round the n indices form n/2
// disjoint pairs (p, q) whose rotations commute.  Thread t works for pair
// k = t / TPP and block b = t % TPP of rows (columns) b, b + TPP, ..., so
// the TPP threads of a pair are neighbouring lanes of one wave.  A round is:
// each thread computes its pair's rotation from A_pp, A_qq, A_pq; the column
// rotations of A and of the eigenvector matrix V on its rows (a wave reads
// those three entries before it writes the columns, and no other wave
// touches them); a barrier; the row rotations of A on its columns, which set
// the annihilated entries to zero; a barrier.
#pragma once
#include <hip/hip_runtime.h>

namespace ambddc {

constexpr int JAC_MAXN = 64;
constexpr int JAC_WORK = 32;   // doubles

// pair k of round rr (np even player count, mm = np - 1 rounds per sweep);
// q = -1 when the partner is the dummy player of an odd n
__device__ inline void jac_pair(int k, int rr, int np, int mm, int n, int& p, int& q) {
  if (k == 0) {
    p = rr;
    q = np - 1;
  } else {
    p = rr + k;
    if (p >= mm) p -= mm;
    q = rr - k;
    if (q < 0) q += mm;
  }
  if (p > q) { const int t = p; p = q; q = t; }
  if (q >= n) q = -1;
}

// A: n x n (ld lda) symmetric, overwritten (diagonal -> eigenvalues).
// V: n x n (ld ldv) receives the eigenvectors (columns).  Odd lda and ldv
// keep the LDS accesses free of bank conflicts.  work: JAC_WORK doubles.
// n <= JAC_MAXN, blockDim = 32 * TPP, TPP in {8, 16, 32}.
template <int TPP>
__device__ inline void jacobi_lds(double* A, int lda, double* V, int ldv, int n, double* work) {
  constexpr int RPT = JAC_MAXN / TPP;   // rows (columns) per thread
  constexpr int NW = TPP / 2;           // waves
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = tid / TPP, blk = tid % TPP;
  double* red = work;   // [2 * NW]: (off, diag) partial sums per wave
  for (int idx = tid; idx < n * n; idx += 32 * TPP) {
    const int i = idx % n, j = idx / n;
    V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n <= 1) return;
  const int np = (n + 1) & ~1, half = np / 2, mm = np - 1;
  for (int g = 0;; ++g) {
    const int rr = g % mm, sweep = g / mm;
    if (sweep >= 40) break;
    const bool acc = (rr == 0);
    int p = -1, q = -1;
    if (k < half) jac_pair(k, rr, np, mm, n, p, q);
    double c = 1.0, s = 0.0;
    double off = 0.0, dia = 0.0;
    if (q >= 0) {
      const double apq = A[p + q * lda];
      if (apq != 0.0) {
        // the smaller rotation angle annihilating A_pq, d = A_qq - A_pp:
        // cos 2theta = |d| rho with rho = (d^2 + 4 A_pq^2)^{-1/2}, so
        // c = sqrt(h), h = (1 + |d| rho) / 2, and s = sgn(d) A_pq rho / c
        // (two reciprocal square roots; c^2 + s^2 = 1 holds exactly in exact
        // arithmetic)
        const double d = A[q + q * lda] - A[p + p * lda];
        const double rho = rsqrt(d * d + 4.0 * apq * apq);
        const double h = 0.5 + 0.5 * fabs(d) * rho;
        const double ic = rsqrt(h);
        c = h * ic;
        s = (d >= 0.0 ? 1.0 : -1.0) * apq * rho * ic;
      }
      // column pass: new col p = c col_p - s col_q, new col q = s col_p + c col_q
      double a[RPT], b[RPT];
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = blk + TPP * u;
        if (i < n) {
          a[u] = A[i + p * lda];
          b[u] = A[i + q * lda];
        }
      }
      if (acc) {
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const int i = blk + TPP * u;
          if (i < n) {
            const double a2 = a[u] * a[u], b2 = b[u] * b[u];
            dia += (i == p ? a2 : 0.0) + (i == q ? b2 : 0.0);
            off += (i == p ? 0.0 : a2) + (i == q ? 0.0 : b2);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = blk + TPP * u;
        if (i < n) {
          A[i + p * lda] = c * a[u] - s * b[u];
          A[i + q * lda] = s * a[u] + c * b[u];
        }
      }
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = blk + TPP * u;
        if (i < n) {
          a[u] = V[i + p * ldv];
          b[u] = V[i + q * ldv];
        }
      }
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = blk + TPP * u;
        if (i < n) {
          V[i + p * ldv] = c * a[u] - s * b[u];
          V[i + q * ldv] = s * a[u] + c * b[u];
        }
      }
    } else if (acc && p >= 0) {
      // paired with the dummy: column p is only read, for the norms
      for (int u = 0; u < RPT; ++u) {
        const int i = blk + TPP * u;
        if (i < n) {
          const double a2 = A[i + p * lda] * A[i + p * lda];
          dia += (i == p) ? a2 : 0.0;
          off += (i == p) ? 0.0 : a2;
        }
      }
    }
    if (acc) {
      for (int o = 32; o > 0; o >>= 1) {
        off += __shfl_xor(off, o);
        dia += __shfl_xor(dia, o);
      }
      if (lane == 0) {
        red[2 * wave] = off;
        red[2 * wave + 1] = dia;
      }
    }
    __syncthreads();
    // row pass, with the annihilated entries set to zero
    if (q >= 0) {
      double a[RPT], b[RPT];
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int j = blk + TPP * u;
        if (j < n) {
          a[u] = A[p + j * lda];
          b[u] = A[q + j * lda];
        }
      }
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int j = blk + TPP * u;
        if (j < n) {
          A[p + j * lda] = (j == q) ? 0.0 : c * a[u] - s * b[u];
          A[q + j * lda] = (j == p) ? 0.0 : s * a[u] + c * b[u];
        }
      }
    }
    bool stop = false;
    if (acc) {
      double to = 0.0, td = 0.0;
      for (int w = 0; w < NW; ++w) { to += red[2 * w]; td += red[2 * w + 1]; }
      stop = (to <= 1e-30 * td || to == 0.0);
    }
    __syncthreads();
    if (stop) break;
  }
}

// Descending order of the diagonal of A (ld lda, n <= JAC_MAXN): perm[r] =
// index of the r-th largest eigenvalue.  Ties are broken by index.
__device__ inline void sort_desc_lds(const double* A, int lda, int n, int* perm) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) {
    const double v = A[i + i * lda];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double w = A[j + j * lda];
      rank += (w > v) || (w == v && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
}

}  // namespace ambddc
