// Pair kernels of the batched LOBPCG (one workgroup per face pair).
//
// Pair vectors live on [Gamma^s; Gamma^t].  With pair weights
// d_s = K^s_jj / (K^s_jj + K^t_jj), d_t = 1 - d_s on a shared DOF j, the
// operator I - E^st acts on the two copies (w_s, w_t) as
//   (I-E)w = (d_t (w_s - w_t), d_s (w_t - w_s)),
//   (I-E)^T y = (d_t y_s - d_s y_t, -d_t y_s + d_s y_t),
// and is zero off the shared DOFs (E^st is the identity there, Section 7).
// Pi is the orthogonal projection onto null(D), D = [C^s_sh, -C^t_sh]; the
// rows of D have disjoint supports, so Pi = I - sum_r d_r d_r^T / |d_r|^2.
#include <algorithm>
#include <cmath>

#include "rr_eig.hpp"
#include "lobpcg.hpp"

namespace ambddc {

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  __syncthreads();
  return t;
}

__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// X block: uniform(-1, 1) from a counter-based hash of (seed, pair, entry).
__global__ __launch_bounds__(256) void k_random(const PairDev* P, double* V, int m, uint64_t seed) {
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  double* X = V + p.v_off;
  for (int i = threadIdx.x; i < n * m; i += blockDim.x) {
    const uint64_t h = mix64(seed ^ mix64((uint64_t(blockIdx.x) << 32) + uint64_t(i)));
    X[i] = (double(h >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
  }
}

void lp_random(const PairDev* P, int np, double* V, int m, uint64_t seed, hipStream_t st) {
  if (np == 0) return;
  k_random<<<np, 256, 0, st>>>(P, V, m, seed);
  AMB_LAUNCH_CHECK();
}

// v <- Pi v (and, when deflating, remove the orthonormal pair rigid modes).
// Each row of D = [C^s_sh, -C^t_sh] is supported on the DOFs of one shared
// corner or edge only; its entries are listed in dr (pair-vector index and
// position of the coefficient in the constraint buffer; t-side entries carry
// the minus sign).  Rows have disjoint supports, so Pi subtracts each row's
// component independently: a group of 16 lanes per (row, column) gathers the
// row's support in parallel, sums with DPP inside the group, and updates the
// support, with no barrier.  The rigid-mode deflation needs whole columns and
// starts after a barrier.
constexpr int DEFL_RB = 6;     // rigid modes of a pair (3D elasticity)
constexpr int DEFL_COLS = 6;   // columns per workgroup: ceil(m / PAIR_COL_GROUPS), m <= 21

__device__ void pair_project(const PairDev& p, double* v, int ldv, int ncol, const double* C,
                             const DRows dr, const double* rb, bool deflate, double* sm) {
  const int n = p.nGs + p.nGt;
  const int nd = p.dr1 - p.dr0;
  const int tid = threadIdx.x, nt = blockDim.x;
  // the 16 lanes of a group share idx, so a group is active or idle as a
  // whole and the row reduction only reads active lanes
  const int sub = tid & 15;
  for (int idx = tid >> 4; idx < nd * ncol; idx += nt >> 4) {
    const int r = idx / ncol, c = idx % ncol;
    double* vc = v + (size_t)c * ldv;
    const int q0 = dr.ptr[p.dr0 + r], q1 = dr.ptr[p.dr0 + r + 1];
    double dot = 0.0, nrm = 0.0;
    for (int q = q0 + sub; q < q1; q += 16) {
      const int i = dr.idx[q];
      const double a = (i < p.nGs ? 1.0 : -1.0) * C[dr.cpos[q]];
      dot += a * vc[i];
      nrm += a * a;
    }
    dot = row16_sum(dot);
    nrm = row16_sum(nrm);
    const double coef = nrm > 0.0 ? dot / nrm : 0.0;
    for (int q = q0 + sub; q < q1; q += 16) {
      const int i = dr.idx[q];
      vc[i] -= coef * (i < p.nGs ? 1.0 : -1.0) * C[dr.cpos[q]];
    }
  }
  if (deflate && p.nrb > 0) {
    __syncthreads();
    double* coef = sm;   // [nrb * ncol]
    const double* R = rb + p.rb_off;
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    if (p.nrb <= DEFL_RB && ncol <= DEFL_COLS) {
      // one pass over the rows: every thread accumulates all nrb x ncol
      // products of its rows, so R and v are each read once per phase
      double acc[DEFL_RB][DEFL_COLS];
#pragma unroll
      for (int r = 0; r < DEFL_RB; ++r)
#pragma unroll
        for (int c = 0; c < DEFL_COLS; ++c) acc[r][c] = 0.0;
      for (int i = tid; i < n; i += nt) {
        double vi[DEFL_COLS];
#pragma unroll
        for (int c = 0; c < DEFL_COLS; ++c) vi[c] = c < ncol ? v[i + (size_t)c * ldv] : 0.0;
#pragma unroll
        for (int r = 0; r < DEFL_RB; ++r) {
          if (r >= p.nrb) break;
          const double ri = R[i + (size_t)r * n];
#pragma unroll
          for (int c = 0; c < DEFL_COLS; ++c) acc[r][c] += ri * vi[c];
        }
      }
      // wave sums, then the waves' partial sums in a fixed order
      double* part = sm + DEFL_RB * DEFL_COLS;   // [nw][DEFL_RB * DEFL_COLS]
#pragma unroll
      for (int r = 0; r < DEFL_RB; ++r)
#pragma unroll
        for (int c = 0; c < DEFL_COLS; ++c) {
          const double t = wave_sum(acc[r][c]);
          if (lane == 0) part[wave * DEFL_RB * DEFL_COLS + r * DEFL_COLS + c] = t;
        }
      __syncthreads();
      if (tid < DEFL_RB * DEFL_COLS) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += part[w * DEFL_RB * DEFL_COLS + tid];
        coef[tid] = t;   // coef[r * DEFL_COLS + c]
      }
      __syncthreads();
      for (int i = tid; i < n; i += nt) {
        double corr[DEFL_COLS];
#pragma unroll
        for (int c = 0; c < DEFL_COLS; ++c) corr[c] = 0.0;
#pragma unroll
        for (int r = 0; r < DEFL_RB; ++r) {
          if (r >= p.nrb) break;
          const double ri = R[i + (size_t)r * n];
#pragma unroll
          for (int c = 0; c < DEFL_COLS; ++c) corr[c] += coef[r * DEFL_COLS + c] * ri;
        }
#pragma unroll
        for (int c = 0; c < DEFL_COLS; ++c)
          if (c < ncol) v[i + (size_t)c * ldv] -= corr[c];
      }
      return;
    }
    for (int idx = wave; idx < p.nrb * ncol; idx += nw) {
      const int r = idx / ncol, c = idx % ncol;
      const double* vc = v + (size_t)c * ldv;
      const double* rr = R + (size_t)r * n;
      double dot = 0.0;
      for (int i = lane; i < n; i += 64) dot += rr[i] * vc[i];
      dot = wave_sum(dot);
      if (lane == 0) coef[idx] = dot;
    }
    __syncthreads();
    for (int idx = tid; idx < n * ncol; idx += nt) {
      const int i = idx % n, c = idx / n;
      double corr = 0.0;
      for (int r = 0; r < p.nrb; ++r) corr += coef[r * ncol + c] * R[i + (size_t)r * n];
      v[i + (size_t)c * ldv] -= corr;
    }
  }
}

// Columns [c0, c1) of the m-column block handled by this workgroup: the pair
// kernels below run on a grid of (pairs, PAIR_COL_GROUPS) workgroups.
__device__ inline void col_range(int m, int& c0, int& c1) {
  const int per = (m + (int)gridDim.y - 1) / (int)gridDim.y;
  c0 = (int)blockIdx.y * per;
  c1 = min(m, c0 + per);
}

__global__ __launch_bounds__(256) void k_project(const PairDev* P, double* V, int m, int col,
                                                 const double* C, const DRows dr,
                                                 const double* rb, const int* active, bool deflate) {
  __shared__ double sm[64 * 16];
  if (active && !active[blockIdx.x]) return;
  int c0, c1;
  col_range(m, c0, c1);
  if (c0 >= c1) return;
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  pair_project(p, V + p.v_off + (size_t)(col * m + c0) * n, n, c1 - c0, C, dr, rb, deflate, sm);
}

void lp_project(const PairDev* P, int np, double* V, int m, int col, const double* C,
                const DRows dr, const double* rb, const int* active, bool deflate,
                hipStream_t st) {
  if (np == 0) return;
  k_project<<<dim3(np, PAIR_COL_GROUPS), 256, 0, st>>>(P, V, m, col, C, dr, rb, active, deflate);
  AMB_LAUNCH_CHECK();
}

__device__ inline double pair_ds(const PairDev& p, const double* diagG, int is, int it) {
  const double a = diagG[p.gs_off + is], b = diagG[p.gt_off + it];
  return a / (a + b);
}

// Copy the column block `col` of V into the pair's slots of U^s and U^t;
// with_ie also writes (I-E) of the block into the next m slot columns.
__global__ __launch_bounds__(256) void k_to_slab(const PairDev* P, const double* V, int m, int col,
                                                 bool with_ie, const double* diagG, const int* sh_s,
                                                 const int* sh_t, double* U, float* U32,
                                                 const int* active) {
  if (active && !active[blockIdx.x]) return;
  // pairs in the FP32 phase also get the slot in FP32 (the operand of the
  // FP32 products)
  if (U32 && !(active && active[blockIdx.x] == 1)) U32 = nullptr;
  int c0, c1;
  col_range(m, c0, c1);
  if (c0 >= c1) return;
  const int nc = c1 - c0;
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  const double* v = V + p.v_off + (size_t)(col * m + c0) * n;
  double* us = U + p.us_off + (size_t)c0 * p.nGs;
  double* ut = U + p.ut_off + (size_t)c0 * p.nGt;
  float* us32 = U32 ? U32 + p.us_off + (size_t)c0 * p.nGs : nullptr;
  float* ut32 = U32 ? U32 + p.ut_off + (size_t)c0 * p.nGt : nullptr;
  for (int idx = threadIdx.x; idx < n * nc; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    const double x = v[idx];
    const size_t e = i < p.nGs ? i + (size_t)c * p.nGs : (i - p.nGs) + (size_t)c * p.nGt;
    if (i < p.nGs) us[e] = x;
    else ut[e] = x;
    if (us32) (i < p.nGs ? us32 : ut32)[e] = static_cast<float>(x);
  }
  if (!with_ie) return;
  // (I-E) of column c goes to slot column m + c
  for (int idx = threadIdx.x; idx < p.nGs * nc; idx += blockDim.x) {
    us[(size_t)m * p.nGs + idx] = 0.0;
    if (us32) us32[(size_t)m * p.nGs + idx] = 0.f;
  }
  for (int idx = threadIdx.x; idx < p.nGt * nc; idx += blockDim.x) {
    ut[(size_t)m * p.nGt + idx] = 0.0;
    if (ut32) ut32[(size_t)m * p.nGt + idx] = 0.f;
  }
  __syncthreads();
  const int nsh = p.sh1 - p.sh0;
  for (int idx = threadIdx.x; idx < nsh * nc; idx += blockDim.x) {
    const int q = idx % nsh, c = idx / nsh;
    const int is = sh_s[p.sh0 + q], it = sh_t[p.sh0 + q];
    const double ds = pair_ds(p, diagG, is, it), dt = 1.0 - ds;
    const double ws = v[is + (size_t)c * n], wt = v[p.nGs + it + (size_t)c * n];
    const double a = dt * (ws - wt), b = ds * (wt - ws);
    us[(size_t)(m + c) * p.nGs + is] = a;
    ut[(size_t)(m + c) * p.nGt + it] = b;
    if (us32) {
      us32[(size_t)(m + c) * p.nGs + is] = static_cast<float>(a);
      ut32[(size_t)(m + c) * p.nGt + it] = static_cast<float>(b);
    }
  }
}

void lp_to_slab(const PairDev* P, int np, const double* V, int m, int col, bool with_ie,
                const double* diagG, const int* sh_s, const int* sh_t, double* U, float* U32,
                const int* active, hipStream_t st) {
  if (np == 0) return;
  k_to_slab<<<dim3(np, PAIR_COL_GROUPS), 256, 0, st>>>(P, V, m, col, with_ie, diagG, sh_s, sh_t,
                                                       U, U32, active);
  AMB_LAUNCH_CHECK();
}

// BV = Pi (S w),  AV = Pi (I-E)^T (S (I-E) w)   from the slots of Y^s, Y^t.
__global__ __launch_bounds__(256) void k_from_slab_ab(const PairDev* P, const double* Y, int m,
                                                      int col, double* AV, double* BV,
                                                      const double* diagG, const int* sh_s,
                                                      const int* sh_t, const double* C,
                                                      const DRows dr, const int* active) {
  if (active && !active[blockIdx.x]) return;
  int c0, c1;
  col_range(m, c0, c1);
  if (c0 >= c1) return;
  const int nc = c1 - c0;
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  const double* ys = Y + p.ys_off + (size_t)c0 * p.nls;
  const double* yt = Y + p.yt_off + (size_t)c0 * p.nlt;
  double* bv = BV + p.v_off + (size_t)(col * m + c0) * n;
  double* av = AV + p.v_off + (size_t)(col * m + c0) * n;
  for (int idx = threadIdx.x; idx < n * nc; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    bv[idx] = (i < p.nGs) ? ys[i + (size_t)c * p.nls] : yt[(i - p.nGs) + (size_t)c * p.nlt];
    av[idx] = 0.0;
  }
  __syncthreads();
  const int nsh = p.sh1 - p.sh0;
  for (int idx = threadIdx.x; idx < nsh * nc; idx += blockDim.x) {
    const int q = idx % nsh, c = idx / nsh;
    const int is = sh_s[p.sh0 + q], it = sh_t[p.sh0 + q];
    const double ds = pair_ds(p, diagG, is, it), dt = 1.0 - ds;
    const double a = ys[is + (size_t)(m + c) * p.nls];
    const double b = yt[it + (size_t)(m + c) * p.nlt];
    av[is + (size_t)c * n] = dt * a - ds * b;
    av[p.nGs + it + (size_t)c * n] = -dt * a + ds * b;
  }
  __syncthreads();
  pair_project(p, bv, n, nc, C, dr, nullptr, false, nullptr);
  pair_project(p, av, n, nc, C, dr, nullptr, false, nullptr);
}

void lp_from_slab_ab(const PairDev* P, int np, const double* Y, int m, int col, double* AV,
                     double* BV, const double* diagG, const int* sh_s, const int* sh_t,
                     const double* C, const DRows dr, const int* active, hipStream_t st) {
  if (np == 0) return;
  k_from_slab_ab<<<dim3(np, PAIR_COL_GROUPS), 256, 0, st>>>(P, Y, m, col, AV, BV, diagG, sh_s,
                                                            sh_t, C, dr, active);
  AMB_LAUNCH_CHECK();
}

// Pair coarse correction: y_c = Psi^T u (from -Y rows nG..nl of both
// subdomains, summed over shared coarse DOFs), z_c = K_p^+ y_c, written to
// the coarse slabs of s and t.
__global__ __launch_bounds__(256) void k_coarse(const PairDev* P, const double* Y, int m,
                                                const double* Kp, const int* pc_s, const int* pc_t,
                                                double* Zc, const int* active) {
  extern __shared__ double sm[];   // yc, zc: ncp_max x m each
  if (active && !active[blockIdx.x]) return;
  const PairDev p = P[blockIdx.x];
  const int ncp = p.ncp;
  double* yc = sm;
  double* zc = sm + (size_t)ncp * m;
  for (int i = threadIdx.x; i < ncp * m; i += blockDim.x) yc[i] = 0.0;
  __syncthreads();
  for (int idx = threadIdx.x; idx < p.ncs * m; idx += blockDim.x) {
    const int r = idx % p.ncs, c = idx / p.ncs;
    yc[pc_s[p.pcs0 + r] + c * ncp] -= Y[p.ys_off + p.nGs + r + (size_t)c * p.nls];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < p.nct * m; idx += blockDim.x) {
    const int r = idx % p.nct, c = idx / p.nct;
    yc[pc_t[p.pct0 + r] + c * ncp] -= Y[p.yt_off + p.nGt + r + (size_t)c * p.nlt];
  }
  __syncthreads();
  const double* K = Kp + p.kp_off;
  for (int idx = threadIdx.x; idx < ncp * m; idx += blockDim.x) {
    const int i = idx % ncp, c = idx / ncp;
    double v = 0.0;
    for (int j = 0; j < ncp; ++j) v += K[i + (size_t)j * ncp] * yc[j + c * ncp];
    zc[idx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < p.ncs * m; idx += blockDim.x) {
    const int r = idx % p.ncs, c = idx / p.ncs;
    Zc[p.zs_off + r + (size_t)c * p.ncs] = zc[pc_s[p.pcs0 + r] + c * ncp];
  }
  for (int idx = threadIdx.x; idx < p.nct * m; idx += blockDim.x) {
    const int r = idx % p.nct, c = idx / p.nct;
    Zc[p.zt_off + r + (size_t)c * p.nct] = zc[pc_t[p.pct0 + r] + c * ncp];
  }
}

void lp_coarse(const PairDev* P, int np, const double* Y, int m, const double* Kp,
               const int* pc_s, const int* pc_t, double* Zc, int ncp_max, const int* active,
               hipStream_t st) {
  if (np == 0) return;
  const size_t sm = sizeof(double) * 2 * size_t(std::max(ncp_max, 1)) * m;
  k_coarse<<<np, 256, sm, st>>>(P, Y, m, Kp, pc_s, pc_t, Zc, active);
  AMB_LAUNCH_CHECK();
}

// W = -(Y rows 0..nG of s and t)  (the slab holds -(Z u + Psi z_c))
__global__ __launch_bounds__(256) void k_from_slab_w(const PairDev* P, const double* Y, int m,
                                                     double* V, const int* active) {
  if (active && !active[blockIdx.x]) return;
  int c0, c1;
  col_range(m, c0, c1);
  if (c0 >= c1) return;
  const int nc = c1 - c0;
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  double* w = V + p.v_off + (size_t)(m + c0) * n;
  const double* ys = Y + p.ys_off + (size_t)c0 * p.nls;
  const double* yt = Y + p.yt_off + (size_t)c0 * p.nlt;
  for (int idx = threadIdx.x; idx < n * nc; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    w[idx] = -((i < p.nGs) ? ys[i + (size_t)c * p.nls] : yt[(i - p.nGs) + (size_t)c * p.nlt]);
  }
}

void lp_from_slab_w(const PairDev* P, int np, const double* Y, int m, double* V, const int* active,
                    hipStream_t st) {
  if (np == 0) return;
  k_from_slab_w<<<dim3(np, PAIR_COL_GROUPS), 256, 0, st>>>(P, Y, m, V, active);
  AMB_LAUNCH_CHECK();
}

// R = AX - BX diag(lam) into the W block; per-column relative residuals.
// active[p] is the pair's phase: 2 = FP64 products (a pair stays active
// until its first nconv columns have converged to tol; converged columns are
// soft-locked), 1 = FP32 products (no column converges or locks; the pair
// moves to phase 2 once the largest residual of its first nconv columns is
// <= tol32, or has made no new best at least twice below the previous best
// for three iterations: the FP32 products stall there).  hist: 4 doubles per
// pair (best residual, iterations since it halved, -, iterations).  One wave per column
// (wave reductions, no barrier inside a column).
constexpr int RES_THREADS = 1024;

__global__ __launch_bounds__(RES_THREADS) void k_residual(const PairDev* P, double* V,
                                                          const double* AV, const double* BV,
                                                          const double* lam, int m, int nconv,
                                                          double tol, double tol32, int* active,
                                                          double* resn, double* hist) {
  __shared__ int n_bad;
  __shared__ double relc[32];
  const int mode = active[blockIdx.x];
  if (!mode) return;
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  const double* l = lam + (size_t)blockIdx.x * m;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x == 0) n_bad = 0;
  __syncthreads();
  for (int c = wave; c < m; c += RES_THREADS / 64) {
    const double* ax = AV + p.v_off + (size_t)c * n;
    const double* bx = BV + p.v_off + (size_t)c * n;
    double* w = V + p.v_off + (size_t)(m + c) * n;
    const double lc = l[c];
    double rr = 0.0, aa = 0.0, bb = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double a = ax[i], b = bx[i];
      const double r = a - lc * b;
      w[i] = r;
      rr += r * r;
      aa += a * a;
      bb += b * b;
    }
    for (int o = 32; o > 0; o >>= 1) {
      rr += __shfl_xor(rr, o);
      aa += __shfl_xor(aa, o);
      bb += __shfl_xor(bb, o);
    }
    // eigenvalues far below the pair's largest (the exact zeros of a pair with
    // few shared DOFs) are measured against 1e-6 lambda_1 instead of |lambda|
    const double den = sqrt(aa) + fmax(fabs(lc), 1e-6 * fabs(l[0])) * sqrt(bb);
    const double rel = den > 0.0 ? sqrt(rr) / den : 0.0;
    if (lane == 0) {
      resn[(size_t)blockIdx.x * m + c] = rel;
      if (c < 32) relc[c] = rel;
      if (mode == 2 && c < nconv && !(rel <= tol)) atomicAdd(&n_bad, 1);
    }
    // soft locking: a converged column contributes no search direction
    if (mode == 2 && rel <= tol)
      for (int i = lane; i < n; i += 64) w[i] = 0.0;
  }
  __shared__ int to_fp64;
  __syncthreads();
  if (mode == 2) {
    if (threadIdx.x == 0 && n_bad == 0) active[blockIdx.x] = 0;
    return;
  }
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int c = 0; c < min(nconv, 32); ++c) r = fmax(r, relc[c]);
    // stalled: no new best residual at least twice below the previous best
    // for three iterations (robust to the oscillation of a rounding floor)
    double* h = hist + 4 * (size_t)blockIdx.x;
    if (h[3] == 0.0 || r < 0.5 * h[0]) {
      h[0] = r;
      h[1] = 0.0;
    } else {
      h[1] += 1.0;
    }
    h[3] += 1.0;
    to_fp64 = (r <= tol32 || h[1] >= 3.0 || !(r == r)) ? 1 : 0;
    if (to_fp64) active[blockIdx.x] = 2;
  }
  __syncthreads();
  // entering the FP64 phase restarts the search history: the P block, built
  // from FP32 products, is dropped (the next Rayleigh-Ritz runs on [X W]),
  // and columns already at tol are soft-locked as in phase 2 (a residual at
  // the rounding level gives a search direction of pure noise)
  if (to_fp64) {
    double* pb = V + p.v_off + (size_t)(2 * m) * n;
    for (int i = threadIdx.x; i < m * n; i += RES_THREADS) pb[i] = 0.0;
    for (int c = wave; c < min(m, 32); c += RES_THREADS / 64) {
      if (!(relc[c] <= tol)) continue;
      double* w = V + p.v_off + (size_t)(m + c) * n;
      for (int i = lane; i < n; i += 64) w[i] = 0.0;
    }
  }
}

void lp_residual(const PairDev* P, int np, double* V, const double* AV, const double* BV,
                 const double* lam, int m, int nconv, double tol, double tol32, int* active,
                 double* resn, double* hist, hipStream_t st) {
  if (np == 0) return;
  k_residual<<<np, RES_THREADS, 0, st>>>(P, V, AV, BV, lam, m, nconv, tol, tol32, active, resn,
                                         hist);
  AMB_LAUNCH_CHECK();
}

// Rayleigh-Ritz on span(V).  With D = diag(GB)^{-1/2}, the scaled Gram
// matrix B = D GB D is reduced by a diagonally pivoted elimination: step j
// picks the remaining index p with the largest diagonal entry of the current
// B (stopping below 1e-8: numerically dependent directions are dropped) and
// eliminates column p from the remaining rows, B <- B - b_p b_p^T / b_pp,
// while the same row operations are accumulated in F (F <- E F, starting
// from I; stopping below the drop level, see k_rr).  With the pivot rows of
// F scaled by b_pp^{-1/2} and by D,
// Fc (r x nb) satisfies Fc GB Fc^T = I, and A_r = Fc GA Fc^T (two small
// products) gives its m largest eigenpairs (Y, descending) by tridiagonal
// reduction, multisection and inverse iteration (rr_eig.hpp), which only
// computes the vectors that are kept.  The Ritz coefficients are Fc^T Y;
// Cf2 (ld 3m) holds the first m of them (columns
// 0..m-1) and the same with the X rows zeroed (columns m..2m-1, giving the
// new P).
//
// Elimination: lanes are rows, each of RR_EW waves owns a fixed set of
// columns, one barrier per step (the other waves only take the pivot
// maximum, to leave the loop at the same step).  A row of F that is not yet a pivot is nonzero only in
// the columns of earlier pivots and its own, so only those are updated;
// pivot rows are never touched again (their scaling is applied at the end).
// The next pivot is the largest key (diagonal value with its low 6 bits
// replaced by 63 - index; a positive double whose order is that of the
// values, ties broken by index): every row's key sits in an LDS array, double
// buffered across steps, and every wave takes the maximum with DPP.
constexpr int RR_THREADS = 1024;   // 16 waves
constexpr int RR_MAXNB = 64;       // order of the reduced problem (3m, m <= 21)
constexpr int RR_COLS = 4;         // columns per wave when all 16 waves share nb <= 64 columns
constexpr int RR_EW = 8;           // waves that eliminate (the others only follow the pivots)
constexpr int RR_ECOLS = 8;        // columns per eliminating wave

__device__ inline double rr_key(double v, int i) {
  if (!(v > 0.0)) return 0.0;
  return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(v) & ~63ull) |
                                          (unsigned long long)(63 - i)));
}

__global__ __launch_bounds__(RR_THREADS) void k_rr(const double* GA, const double* GB, int nb, int m,
                                            double* Cf2, double* lam, const int* active) {
  extern __shared__ double sm[];
  if (active && !active[blockIdx.x]) return;
  // a direction is dropped when the scaled B-norm^2 it keeps after the
  // elimination is this small: its reduced entries are then the Gram
  // matrices' rounding errors divided by it, and kept directions of that
  // kind give Ritz vectors whose residuals stall far above the tolerance.
  // 1e-8 for FP64 products, 1e-4 while the pair's products are FP32 (Gram
  // errors near 1e-7 of the entries)
  const double drop = (active && active[blockIdx.x] == 1) ? 1e-4 : 1e-8;
  const int M3 = 3 * m;
  const int ld = nb | 1;          // odd: row walks are free of bank conflicts
  const double* ga = GA + (size_t)blockIdx.x * M3 * M3;
  const double* gb = GB + (size_t)blockIdx.x * M3 * M3;
  double* A = sm;                 // sym(GA), nb x nb (ld); later A_r (r x r, ld r|1)
  double* B = A + nb * ld;        // scaled GB; later Fc (r x nb, ld)
  double* F = B + nb * ld;        // F (nb x nb, ld); later GA Fc^T, then Y
  double* dsc = F + nb * ld;      // nb
  double* rs = dsc + nb;          // nb
  double* eigws = rs + nb;        // EIG_WS
  double* elam = eigws + EIG_WS;  // EIG_MAXN
  double* key = elam + EIG_MAXN;  // 2 x 64: row keys, double buffered
  double* pinv = key + 128;       // nb: 1 / pivot, in pivot order
  int* piv = reinterpret_cast<int*>(pinv + nb);   // nb
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, nw = nt >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int i = tid; i < nb; i += nt) {
    const double d = gb[i + (size_t)i * nb];
    dsc[i] = d > 1e-300 ? 1.0 / sqrt(d) : 0.0;
  }
  for (int idx = tid; idx < nb * nb; idx += nt) {
    const int i = idx % nb, k = idx / nb;
    A[i + k * ld] = ga[idx];
    B[i + k * ld] = gb[idx];
    F[i + k * ld] = (i == k) ? 1.0 : 0.0;
  }
  __syncthreads();
  // symmetrise (A) and scale (B): columns owned by waves, lanes = rows; read
  // into registers, then written after a barrier
  double sa[RR_COLS], sb[RR_COLS];
  {
    int u = 0;
    for (int k = wave; k < nb; k += nw, ++u) {
      const int i = lane;
      if (i < nb) {
        sa[u] = 0.5 * (A[i + k * ld] + A[k + i * ld]);
        sb[u] = 0.5 * (B[i + k * ld] + B[k + i * ld]) * dsc[i] * dsc[k];
      }
    }
  }
  __syncthreads();
  {
    int u = 0;
    for (int k = wave; k < nb; k += nw, ++u) {
      const int i = lane;
      if (i < nb) {
        A[i + k * ld] = sa[u];
        B[i + k * ld] = sb[u];
        if (i == k) key[i] = rr_key(sb[u], i);
      }
    }
  }
  __syncthreads();
  uint64_t done = 0;
  int r = 0;
  for (int j = 0; j < nb; ++j) {
    const double* kcur = key + 64 * (j & 1);
    double* knext = key + 64 * ((j + 1) & 1);
    const double kd = wave_max(lane < nb ? kcur[lane] : 0.0);   // the same for every lane
    const unsigned long long kj = (unsigned long long)__double_as_longlong(kd);
    const double vj = __longlong_as_double((long long)(kj & ~63ull));
    if (kj == 0ull || !(vj > drop)) break;
    const int p = 63 - (int)(kj & 63ull);
    if (wave < RR_EW) {
      const int i = lane, ic = i < nb ? i : nb - 1;
      const double bpp = B[p + p * ld];
      const double bip = B[ic + p * ld];
      // this wave's columns, batched: B columns not yet eliminated get the
      // Schur update, F columns of earlier pivots and of p the row operation
      double x[RR_ECOLS], y[RR_ECOLS];
#pragma unroll
      for (int u = 0; u < RR_ECOLS; ++u) {
        const int k = wave + u * RR_EW;
        if (k < nb) {
          const double* M = (k == p || ((done >> k) & 1ull)) ? F : B;
          y[u] = M[p + k * ld];
          x[u] = M[ic + k * ld];
        }
      }
      const double inv = 1.0 / bpp;
      const bool row = i < nb && i != p && !((done >> i) & 1ull);
      const double gi = bip * inv;
      double dnew = 0.0;
      if (row) {
#pragma unroll
        for (int u = 0; u < RR_ECOLS; ++u) {
          const int k = wave + u * RR_EW;
          if (k < nb) {
            double* M = (k == p || ((done >> k) & 1ull)) ? F : B;
            const double v = x[u] - gi * y[u];
            M[i + k * ld] = v;
            if (k == i) dnew = v;
          }
        }
      }
      // the owner of column i publishes row i's key for the next step
      if (i < nb && i % RR_EW == wave) knext[i] = row ? rr_key(dnew, i) : 0.0;
      if (tid == 0) { piv[j] = p; pinv[j] = inv; }
    }
    done |= 1ull << p;
    r = j + 1;
    __syncthreads();
  }
  for (int l = tid; l < r; l += nt) rs[piv[l]] = sqrt(pinv[l]);
  __syncthreads();
  // Fc[l, k] = rs_p dsc_k F[p, k], p = piv[l] (column-major, ld)
  double* Fc = B;
  for (int idx = tid; idx < r * nb; idx += nt) {
    const int l = idx % r, k = idx / r;
    const int pl = piv[l];
    Fc[l + k * ld] = rs[pl] * dsc[k] * F[pl + k * ld];
  }
  __syncthreads();
  // W = sym(GA) Fc^T (nb x r, ld) over F, 2 x 2 outputs per thread
  double* Wt = F;
  const int tx = tid & 31, ty = tid >> 5;
  {
    double acc[2][2] = {};
    for (int k = 0; k < nb; ++k) {
      double x[2], y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ii = tx + 32 * a, c = ty + 32 * a;
        x[a] = ii < nb ? A[ii + k * ld] : 0.0;
        y[a] = c < r ? Fc[c + k * ld] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] += x[a] * y[b];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int ii = tx + 32 * a, c = ty + 32 * b;
        if (ii < nb && c < r) Wt[ii + c * ld] = acc[a][b];
      }
  }
  __syncthreads();
  // A_r = Fc W (r x r, ld lr) over A
  const int lr = r | 1;
  double* J = A;
  {
    double acc[2][2] = {};
    for (int k = 0; k < nb; ++k) {
      double x[2], y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ii = tx + 32 * a, c = ty + 32 * a;
        x[a] = ii < r ? Fc[ii + k * ld] : 0.0;
        y[a] = c < r ? Wt[k + c * ld] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] += x[a] * y[b];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int ii = tx + 32 * a, c = ty + 32 * b;
        if (ii < r && c < r) J[ii + c * lr] = acc[a][b];
      }
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += nt) {
    const int ii = idx % r, c = idx / r;
    if (ii > c) {
      const double s = 0.5 * (J[ii + c * lr] + J[c + ii * lr]);
      J[ii + c * lr] = s;
      J[c + ii * lr] = s;
    }
  }
  __syncthreads();
  double* Y = F;
  const int ly = r | 1;
  const int mm = min(m, r);
  sym_top_eig<RR_THREADS>(J, lr, r, mm, Y, ly, elam, eigws);
  double* cf = Cf2 + (size_t)blockIdx.x * M3 * 2 * m;
  for (int idx = tid; idx < nb * m; idx += nt) {
    const int ii = idx % nb, c = idx / nb;
    double v = 0.0;
    if (c < mm) {
      const double* y = Y + c * ly;
      for (int l = 0; l < r; ++l) v += Fc[l + ii * ld] * y[l];
    }
    cf[ii + (size_t)c * M3] = v;
    cf[ii + (size_t)(c + m) * M3] = (ii < m) ? 0.0 : v;
  }
  for (int c = tid; c < m; c += nt)
    lam[(size_t)blockIdx.x * m + c] = c < mm ? elam[c] : 0.0;
}

size_t rr_smem(int nb) {
  const int ld = nb | 1;
  return sizeof(double) * (3 * nb * ld + 3 * nb + EIG_WS + EIG_MAXN + 128) + sizeof(int) * nb;
}

void lp_rr(const PairDev* P, int np, const double* GA, const double* GB, int nb, int m,
           double* Cf, double* lam, const int* active, hipStream_t st) {
  (void)P;
  if (np == 0) return;
  if (nb > RR_MAXNB || nb < 1) throw Error(1, "Rayleigh-Ritz block larger than 64");
  const size_t sm = rr_smem(nb);
  if (sm > 64 * 1024) {
    // more than the default LDS of a workgroup (up to 96 KB for nb = 63):
    // gfx950 has 160 KB per CU; ask for it once and fail cleanly if refused
    static size_t granted = 0;
    if (sm > granted) {
      int dev = 0, lim = 0;
      AMB_HIP(hipGetDevice(&dev));
      AMB_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      if (size_t(lim) < sm)
        throw Error(1, "Rayleigh-Ritz of order " + std::to_string(nb) + " needs " +
                           std::to_string(sm) + " bytes of LDS; the device allows " +
                           std::to_string(lim));
      AMB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rr),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(sm)));
      granted = sm;
    }
  }
  k_rr<<<np, RR_THREADS, sm, st>>>(GA, GB, nb, m, Cf, lam, active);
  AMB_LAUNCH_CHECK();
}

// X <- T[:, 0:m], P <- T[:, m:2m] for V (and AV, BV unless only_v); the T
// blocks are n x 2m per operand, stored consecutively from 2 * v_off.
__global__ __launch_bounds__(256) void k_commit(const PairDev* P, double* V, double* AV,
                                                double* BV, const double* T, int m, bool with_p,
                                                bool only_v, const int* active) {
  if (active && !active[blockIdx.x]) return;
  int c0, c1;
  col_range(m, c0, c1);
  if (c0 >= c1) return;
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  // T layout per pair: [TV | TAV | TBV], each n x 2m, at offset v_off (same 3m*n footprint x2)
  const double* t = T + 2 * p.v_off;
  double* dst[3] = {V + p.v_off, AV + p.v_off, BV + p.v_off};
  const size_t e0 = (size_t)c0 * n, e1 = (size_t)c1 * n;
  for (int o = 0; o < (only_v ? 1 : 3); ++o) {
    const double* src = t + (size_t)o * n * 2 * m;
    for (size_t idx = e0 + threadIdx.x; idx < e1; idx += blockDim.x) {
      dst[o][idx] = src[idx];
      if (with_p) dst[o][(size_t)2 * m * n + idx] = src[(size_t)m * n + idx];
    }
  }
}

void lp_commit(const PairDev* P, int np, double* V, double* AV, double* BV, const double* T,
               int m, bool with_p, bool only_v, const int* active, hipStream_t st) {
  if (np == 0) return;
  k_commit<<<dim3(np, PAIR_COL_GROUPS), 256, 0, st>>>(P, V, AV, BV, T, m, with_p, only_v, active);
  AMB_LAUNCH_CHECK();
}

// Pair coarse matrix Psi^T S^st Psi = R_c^s^T K_c^s R_c^s + R_c^t^T K_c^t R_c^t.
__global__ __launch_bounds__(256) void k_pair_coarse(const PairDev* P, const double* kc,
                                                     const int64_t* kc_off, const int* pc_s,
                                                     const int* pc_t, double* Kp) {
  const PairDev p = P[blockIdx.x];
  double* K = Kp + p.kp_off;
  const int ncp = p.ncp;
  for (int i = threadIdx.x; i < ncp * ncp; i += blockDim.x) K[i] = 0.0;
  __syncthreads();
  const double* ks = kc + kc_off[p.s];
  for (int idx = threadIdx.x; idx < p.ncs * p.ncs; idx += blockDim.x) {
    const int a = idx % p.ncs, b = idx / p.ncs;
    K[pc_s[p.pcs0 + a] + pc_s[p.pcs0 + b] * ncp] += ks[idx];
  }
  __syncthreads();
  const double* kt = kc + kc_off[p.t];
  for (int idx = threadIdx.x; idx < p.nct * p.nct; idx += blockDim.x) {
    const int a = idx % p.nct, b = idx / p.nct;
    K[pc_t[p.pct0 + a] + pc_t[p.pct0 + b] * ncp] += kt[idx];
  }
}

void lp_pair_coarse(const PairDev* P, int np, const double* kc, const int64_t* kc_off,
                    const int* pc_s, const int* pc_t, double* Kp, hipStream_t st) {
  if (np == 0) return;
  k_pair_coarse<<<np, 256, 0, st>>>(P, kc, kc_off, pc_s, pc_t, Kp);
  AMB_LAUNCH_CHECK();
}

// Generalised inverse of the pair coarse matrix K = Psi^T S^st Psi (Section 5
// drops the near-null part of its eigendecomposition).  K is scaled to unit
// diagonal, Kt = D^{-1/2} K D^{-1/2}; when both subdomains float, its null
// space is spanned by the coarse values of the nrb pair rigid modes
// (N = C^s, C^t applied to them), so with Nt = orthonormal basis of
// D^{1/2} N the pseudo-inverse is Kt^+ = (Kt + Nt Nt^T)^{-1} - Nt Nt^T, and
// G = D^{-1/2} Kt^+ D^{-1/2} satisfies K G K = K; otherwise K is
// nonsingular (Assumption 1) and G = K^{-1}.  The inverse comes from a
// batched signed LDL^T of [[Kt + Nt Nt^T, I], [I, 0]]: a non-positive pivot
// means K has more null vectors than rigid modes, i.e. Assumption 1 fails.
//
// Step 1: Nt (ncp x nrb, stored at kp_off of Nb) for every pair with nrb > 0.
__global__ __launch_bounds__(256) void k_pair_null(const PairDev* P, const double* C,
                                                   const int* pc_s, const int* pc_t,
                                                   const double* Kp, const double* rb,
                                                   double* Nb) {
  __shared__ double red[8];
  const PairDev p = P[blockIdx.x];
  if (p.nrb == 0) return;
  const int ncp = p.ncp, n = p.nGs + p.nGt;
  double* N = Nb + p.kp_off;
  const double* K = Kp + p.kp_off;
  const double* R = rb + p.rb_off;
  for (int idx = threadIdx.x; idx < p.ncs * p.nrb; idx += blockDim.x) {
    const int r = idx % p.ncs, j = idx / p.ncs;
    double v = 0.0;
    for (int i = 0; i < p.nGs; ++i) v += C[p.cs_off + r + (int64_t)i * p.ncs] * R[i + (size_t)j * n];
    N[pc_s[p.pcs0 + r] + (size_t)j * ncp] = v;
  }
  __syncthreads();
  // t writes its coarse DOFs afterwards (shared ones carry the same values)
  for (int idx = threadIdx.x; idx < p.nct * p.nrb; idx += blockDim.x) {
    const int r = idx % p.nct, j = idx / p.nct;
    double v = 0.0;
    for (int i = 0; i < p.nGt; ++i)
      v += C[p.ct_off + r + (int64_t)i * p.nct] * R[p.nGs + i + (size_t)j * n];
    N[pc_t[p.pct0 + r] + (size_t)j * ncp] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < ncp * p.nrb; idx += blockDim.x) {
    const int i = idx % ncp;
    const double d = K[i + (size_t)i * ncp];
    N[idx] *= d > 0.0 ? sqrt(d) : 1.0;
  }
  __syncthreads();
  // modified Gram-Schmidt, twice
  for (int j = 0; j < p.nrb; ++j) {
    double* nj = N + (size_t)j * ncp;
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < j; ++q) {
        const double* nq = N + (size_t)q * ncp;
        double dot = 0.0;
        for (int i = threadIdx.x; i < ncp; i += blockDim.x) dot += nq[i] * nj[i];
        dot = block_sum(dot, red);
        for (int i = threadIdx.x; i < ncp; i += blockDim.x) nj[i] -= dot * nq[i];
        __syncthreads();
      }
    }
    double nrm = 0.0;
    for (int i = threadIdx.x; i < ncp; i += blockDim.x) nrm += nj[i] * nj[i];
    nrm = block_sum(nrm, red);
    const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
    for (int i = threadIdx.x; i < ncp; i += blockDim.x) nj[i] *= inv;
    __syncthreads();
  }
}

// Step 2: the augmented matrices [[Kt + Nt Nt^T, I], [I, 0]] (order 2 ncp,
// at 4 kp_off of Aug).
__global__ __launch_bounds__(256) void k_pinv_fill(const PairDev* P, const double* Kp,
                                                   const double* Nb, double* Aug) {
  const PairDev p = P[blockIdx.x];
  const int ncp = p.ncp, N2 = 2 * ncp;
  const double* K = Kp + p.kp_off;
  const double* Nt = Nb + p.kp_off;
  double* A = Aug + 4 * p.kp_off;
  for (int idx = threadIdx.x; idx < N2 * N2; idx += blockDim.x) {
    const int i = idx % N2, k = idx / N2;
    double v = 0.0;
    if (i < ncp && k < ncp) {
      const double di = K[i + (size_t)i * ncp], dk = K[k + (size_t)k * ncp];
      const double si = di > 0.0 ? 1.0 / sqrt(di) : 1.0, sk = dk > 0.0 ? 1.0 / sqrt(dk) : 1.0;
      v = 0.5 * (K[i + (size_t)k * ncp] + K[k + (size_t)i * ncp]) * si * sk;
      for (int j = 0; j < p.nrb; ++j) v += Nt[i + (size_t)j * ncp] * Nt[k + (size_t)j * ncp];
    } else if (i == k + ncp || k == i + ncp) {
      v = 1.0;
    }
    A[idx] = v;
  }
}

// Step 3 (after the factorisation, whose trailing block is -(Kt + Nt Nt^T)^{-1}):
// G = D^{-1/2} (-T - Nt Nt^T) D^{-1/2} over K.
__global__ __launch_bounds__(256) void k_pinv_extract(const PairDev* P, const double* Aug,
                                                      const double* Nb, double* Kp, int* nsmall) {
  __shared__ double sc[PAIR_COARSE_MAX];
  __shared__ int cnt;
  const PairDev p = P[blockIdx.x];
  const int ncp = p.ncp, N2 = 2 * ncp;
  double* K = Kp + p.kp_off;
  const double* Nt = Nb + p.kp_off;
  const double* A = Aug + 4 * p.kp_off;
  const double* T = A + ncp + (size_t)ncp * N2;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < ncp; i += blockDim.x) {
    const double d = K[i + (size_t)i * ncp];
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
    // the factor's diagonal holds the square roots of the pivots of the
    // unit-diagonal matrix Kt + Nt Nt^T; a tiny pivot is a null vector
    // beyond the rigid modes
    const double l = A[i + (size_t)i * N2];
    if (!(l * l > 1e-10)) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) nsmall[blockIdx.x] = cnt;
  for (int idx = threadIdx.x; idx < ncp * ncp; idx += blockDim.x) {
    const int i = idx % ncp, k = idx / ncp;
    double v = -0.5 * (T[i + (size_t)k * N2] + T[k + (size_t)i * N2]);
    for (int j = 0; j < p.nrb; ++j) v -= Nt[i + (size_t)j * ncp] * Nt[k + (size_t)j * ncp];
    K[idx] = v * sc[i] * sc[k];
  }
}

void lp_pair_null(const PairDev* P, int np, const double* C, const int* pc_s, const int* pc_t,
                  const double* Kp, const double* rb, double* Nb, hipStream_t st) {
  if (np == 0) return;
  k_pair_null<<<np, 256, 0, st>>>(P, C, pc_s, pc_t, Kp, rb, Nb);
  AMB_LAUNCH_CHECK();
}

void lp_pinv_fill(const PairDev* P, int np, const double* Kp, const double* Nb, double* Aug,
                  hipStream_t st) {
  if (np == 0) return;
  k_pinv_fill<<<np, 256, 0, st>>>(P, Kp, Nb, Aug);
  AMB_LAUNCH_CHECK();
}

void lp_pinv_extract(const PairDev* P, int np, const double* Aug, const double* Nb, double* Kp,
                     int* nsmall, hipStream_t st) {
  if (np == 0) return;
  k_pinv_extract<<<np, 256, 0, st>>>(P, Aug, Nb, Kp, nsmall);
  AMB_LAUNCH_CHECK();
}

// Orthonormal pair-continuous rigid modes on [Gamma^s; Gamma^t] (pairs whose
// two subdomains float); modified Gram-Schmidt applied twice.
__global__ __launch_bounds__(256) void k_rigid(const PairDev* P, const double* rigid, int nrbl,
                                               int ndof, const int* gdof, double* rb) {
  __shared__ double red[8];
  const PairDev p = P[blockIdx.x];
  if (p.nrb == 0) return;
  const int n = p.nGs + p.nGt;
  double* R = rb + p.rb_off;
  for (int idx = threadIdx.x; idx < n * p.nrb; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    const int j = (i < p.nGs) ? gdof[p.gs_off + i] : gdof[p.gt_off + i - p.nGs];
    R[idx] = rigid[j + (size_t)c * ndof];
  }
  __syncthreads();
  for (int c = 0; c < p.nrb; ++c) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < c; ++q) {
        double d = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) d += R[i + (size_t)q * n] * R[i + (size_t)c * n];
        d = block_sum(d, red);
        for (int i = threadIdx.x; i < n; i += blockDim.x) R[i + (size_t)c * n] -= d * R[i + (size_t)q * n];
        __syncthreads();
      }
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += R[i + (size_t)c * n] * R[i + (size_t)c * n];
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) R[i + (size_t)c * n] *= inv;
    __syncthreads();
  }
}

void lp_rigid(const PairDev* P, int np, const double* rigid, int ndof, const int* gdof,
              double* rb, hipStream_t st) {
  if (np == 0) return;
  k_rigid<<<np, 256, 0, st>>>(P, rigid, 0, ndof, gdof, rb);
  AMB_LAUNCH_CHECK();
}

// Selection (Alg. 2) and constraint rows: k = #{lambda_j > tau, j < nev_max}
// (or k = fixed when fixed > 0); c_l = (A w_l) restricted to the support of
// the rows in s (the face DOFs, edge and corner entries dropped, or all
// shared DOFs), orthonormalised by Gram-Schmidt (twice) with the rank test
// |R_jj| > 1e-10 max |R_jj|; rows stored row-major (nev_max x nface).
__global__ __launch_bounds__(256) void k_select(const PairDev* P, const double* AV,
                                                const double* lam, int m, int nev_max, double tau,
                                                int fixed, const int* face_s, double* fc, int* kout,
                                                double* lam_next) {
  extern __shared__ double sm[];
  __shared__ double red[8];
  __shared__ double rdiag[32];
  const PairDev p = P[blockIdx.x];
  const int n = p.nGs + p.nGt;
  const double* l = lam + (size_t)blockIdx.x * m;
  const int cap = min(nev_max, m);
  int k = 0;
  // with a fixed count, eigenvalues that are zero up to rounding (their
  // c = A w vanishes) are never taken
  const double zero = 1e-9 * fmax(1.0, l[0]);
  if (fixed > 0) while (k < min(cap, fixed) && l[k] > zero) ++k;
  else while (k < cap && l[k] > tau) ++k;
  if (threadIdx.x == 0) lam_next[blockIdx.x] = (k < m) ? l[k] : 0.0;
  const int nf = p.nface;
  double* Q = sm;   // k x nf (row-major)
  for (int idx = threadIdx.x; idx < k * nf; idx += blockDim.x) {
    const int j = idx / nf, q = idx % nf;
    Q[idx] = AV[p.v_off + face_s[p.face0 + q] + (size_t)j * n];
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < j; ++i) {
        double d = 0.0;
        for (int q = threadIdx.x; q < nf; q += blockDim.x) d += Q[i * nf + q] * Q[j * nf + q];
        d = block_sum(d, red);
        for (int q = threadIdx.x; q < nf; q += blockDim.x) Q[j * nf + q] -= d * Q[i * nf + q];
        __syncthreads();
      }
    }
    double s = 0.0;
    for (int q = threadIdx.x; q < nf; q += blockDim.x) s += Q[j * nf + q] * Q[j * nf + q];
    s = sqrt(block_sum(s, red));
    if (threadIdx.x == 0) rdiag[j] = s;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int q = threadIdx.x; q < nf; q += blockDim.x) Q[j * nf + q] *= inv;
    __syncthreads();
  }
  double rmax = 0.0;
  for (int j = 0; j < k; ++j) rmax = fmax(rmax, rdiag[j]);
  // canonical sign (the span is what the method fixes): the entry of largest
  // magnitude, first on ties, is made positive
  __shared__ double sgn;
  int kk = 0;
  for (int j = 0; j < k; ++j) {
    if (!(rdiag[j] > 1e-10 * rmax)) continue;
    if (threadIdx.x == 0) {
      double best = -1.0, v = 1.0;
      for (int q = 0; q < nf; ++q) {
        const double a = fabs(Q[j * nf + q]);
        if (a > best) { best = a; v = Q[j * nf + q]; }
      }
      sgn = v < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nf; q += blockDim.x)
      fc[p.fc_off + (size_t)kk * nf + q] = sgn * Q[j * nf + q];
    __syncthreads();
    ++kk;
  }
  if (threadIdx.x == 0) kout[blockIdx.x] = kk;
}

void lp_select(const PairDev* P, int np, const double* AV, const double* lam, int m, int nev_max,
               double tau, int fixed, const int* face_s, int nface_max, double* fc, int* kout,
               double* lam_next, hipStream_t st) {
  if (np == 0) return;
  const size_t sm = sizeof(double) * size_t(std::min(nev_max, m)) * nface_max;
  if (sm > 64 * 1024) {
    // rows of many constraints on large faces: up to the 160 KB of a gfx950 CU
    static size_t granted = 0;
    if (sm > granted) {
      int dev = 0, lim = 0;
      AMB_HIP(hipGetDevice(&dev));
      AMB_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      if (size_t(lim) < sm + 1024)
        throw Error(1, "constraint rows of a face need " + std::to_string(sm) +
                           " bytes of LDS; the device allows " + std::to_string(lim));
      AMB_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_select),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(sm)));
      granted = sm;
    }
  }
  k_select<<<np, 256, sm, st>>>(P, AV, lam, m, nev_max, tau, fixed, face_s, fc, kout, lam_next);
  AMB_LAUNCH_CHECK();
}

}  // namespace ambddc
