// Kernels of the BDDC structures (weights, constraint and Neumann matrices,
// coarse element matrices) and of the preconditioner application and PCG.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace ambddc {

__global__ void k_aug_identity(const int64_t* off, const int* ld, const int* nid, const int* col0,
                               const int* row0, double* A) {
  const int s = blockIdx.y;
  const int n = nid[s];
  double* a = A + off[s];
  const int l = ld[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int r = row0[s] + i, c = col0[s] + i;
    a[r + (size_t)c * l] = 1.0;
    a[c + (size_t)r * l] = 1.0;
  }
}

void launch_aug_identity(int nsub, const int64_t* off, const int* ld, const int* nrow_id,
                         const int* col0, const int* row0, hipStream_t st, double* A) {
  if (nsub == 0) return;
  dim3 g(8, nsub);
  k_aug_identity<<<g, 256, 0, st>>>(off, ld, nrow_id, col0, row0, A);
  AMB_LAUNCH_CHECK();
}

__global__ void k_gather(int n, const int64_t* idx, const double* src, int64_t lds, double* dst,
                         int64_t ldd, int nrhs, double scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t j = idx[k];
  for (int r = 0; r < nrhs; ++r) dst[k + r * ldd] = scale * src[j + r * lds];
}

void launch_gather(int n, const int64_t* idx, const double* src, int64_t lds, double* dst,
                   int64_t ldd, int nrhs, double scale, hipStream_t st) {
  if (n == 0) return;
  k_gather<<<ceil_div(n, 256), 256, 0, st>>>(n, idx, src, lds, dst, ldd, nrhs, scale);
  AMB_LAUNCH_CHECK();
}

__global__ void k_scatter(int n, const int64_t* idx, const double* src, int64_t lds, double* dst,
                          int64_t ldd, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t j = idx[k];
  for (int r = 0; r < nrhs; ++r) dst[j + r * ldd] = src[k + r * lds];
}

void launch_scatter(int n, const int64_t* idx, const double* src, int64_t lds, double* dst,
                    int64_t ldd, int nrhs, hipStream_t st) {
  if (n == 0) return;
  k_scatter<<<ceil_div(n, 256), 256, 0, st>>>(n, idx, src, lds, dst, ldd, nrhs);
  AMB_LAUNCH_CHECK();
}

// stiffness scaling: delta^s_j = K^s_jj / sum_r K^r_jj over the copies of DOF j
__global__ void k_weights(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                          const double* diag, double* delta) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nG) return;
  const int j = gdof[k];
  double s = 0.0;
  for (int q = inc_ptr[j]; q < inc_ptr[j + 1]; ++q) s += diag[inc_pos[q]];
  delta[k] = diag[k] / s;
}

void launch_weights(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                    const double* diag, double* delta, hipStream_t st) {
  if (nG == 0) return;
  k_weights<<<ceil_div(nG, 256), 256, 0, st>>>(nG, gdof, inc_ptr, inc_pos, diag, delta);
  AMB_LAUNCH_CHECK();
}

__global__ void k_iface_res(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                            const int64_t* g2y, const double* delta, const double* r, int64_t ldr,
                            const double* y, int64_t ldy, double* out, int64_t ldo, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nG) return;
  const int j = gdof[k];
  const double d = delta[k];
  for (int c = 0; c < nrhs; ++c) {
    double v = r[j + c * ldr];
    if (y)
      for (int q = inc_ptr[j]; q < inc_ptr[j + 1]; ++q) v += y[g2y[inc_pos[q]] + c * ldy];
    out[k + c * ldo] = d * v;
  }
}

void launch_interface_residual(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                               const int64_t* g2y, const double* delta, const double* r,
                               int64_t ldr, const double* y, int64_t ldy, double* out,
                               int64_t ldo, int nrhs, hipStream_t st) {
  if (nG == 0) return;
  k_iface_res<<<ceil_div(nG, 256), 256, 0, st>>>(nG, gdof, inc_ptr, inc_pos, g2y, delta, r, ldr, y,
                                                 ldy, out, ldo, nrhs);
  AMB_LAUNCH_CHECK();
}

__global__ void k_average(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                          const int64_t* g2w, const double* delta, const double* w, int64_t ldw,
                          double* out, int64_t ldo, double* dst, int64_t ldd, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nG) return;
  const int j = gdof[k];
  const int q0 = inc_ptr[j], q1 = inc_ptr[j + 1];
  const bool first = inc_pos[q0] == k;
  for (int c = 0; c < nrhs; ++c) {
    double v = 0.0;
    for (int q = q0; q < q1; ++q) {
      const int kk = inc_pos[q];
      v += delta[kk] * w[g2w[kk] + c * ldw];
    }
    out[k + c * ldo] = v;
    if (first && dst) dst[j + c * ldd] = v;
  }
}

void launch_average(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                    const int64_t* g2w, const double* delta, const double* w, int64_t ldw,
                    double* out, int64_t ldo, double* dst, int64_t ldd, int nrhs, hipStream_t st) {
  if (nG == 0) return;
  k_average<<<ceil_div(nG, 256), 256, 0, st>>>(nG, gdof, inc_ptr, inc_pos, g2w, delta, w, ldw, out,
                                               ldo, dst, ldd, nrhs);
  AMB_LAUNCH_CHECK();
}

__global__ void k_segsum(int n, const int* ptr, const int64_t* pos, const double* src, int64_t lds,
                         double* dst, int64_t ldd, int nrhs, double scale) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int r = 0; r < nrhs; ++r) {
    double v = 0.0;
    for (int q = ptr[c]; q < ptr[c + 1]; ++q) v += src[pos[q] + r * lds];
    dst[c + r * ldd] = scale * v;
  }
}

void launch_segment_sum(int n, const int* ptr, const int64_t* pos, const double* src, int64_t lds,
                        double* dst, int64_t ldd, int nrhs, double scale, hipStream_t st) {
  if (n == 0) return;
  k_segsum<<<ceil_div(n, 256), 256, 0, st>>>(n, ptr, pos, src, lds, dst, ldd, nrhs, scale);
  AMB_LAUNCH_CHECK();
}

__global__ void k_fill_values(int n, const int64_t* pos, const double* val, double* dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[pos[k]] = val[k];
}

void launch_fill_values(int n, const int64_t* pos, const double* val, double* dst, hipStream_t st) {
  if (n == 0) return;
  k_fill_values<<<ceil_div(n, 256), 256, 0, st>>>(n, pos, val, dst);
  AMB_LAUNCH_CHECK();
}

// Adaptive rows of C: one wave per row copies the pair's face row from fc to
// the row's interface positions (amap: local index of every face DOF).
__global__ void k_fill_adaptive(int nrows, const AdaptRow* __restrict__ rows,
                                const int* __restrict__ amap, const double* __restrict__ fc,
                                double* C) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (w >= nrows) return;
  const AdaptRow a = rows[w];
  for (int q = lane; q < a.nf; q += 64) C[a.dst + int64_t(amap[a.map + q]) * a.ldc] = fc[a.src + q];
}

void launch_fill_adaptive(int nrows, const AdaptRow* rows, const int* amap, const double* fc,
                          double* C, hipStream_t st) {
  if (nrows == 0) return;
  k_fill_adaptive<<<ceil_div(nrows, 4), 256, 0, st>>>(nrows, rows, amap, fc, C);
  AMB_LAUNCH_CHECK();
}

// Leading (nG+nc) block of [[S + rho C^T C, C^T, I, 0], [C, 0, 0, I], [I, 0, 0, 0], [0, I, 0, 0]]
// one workgroup per column of the leading block; the identity coupling is
// written by the same workgroup.
__global__ __launch_bounds__(256) void k_neumann_fill(const NeuDesc* __restrict__ d, int nd) {
  const int wg = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].col_start <= wg) lo = mid; else hi = mid - 1;
  }
  const NeuDesc g = d[lo];
  const int j = wg - g.col_start;
  const int nG = g.nG, nc = g.nc, nl = nG + nc;
  double* col = g.A + (size_t)j * g.lda;
  for (int i = threadIdx.x; i < nl; i += blockDim.x) {
    double v = 0.0;
    if (i < nG && j < nG) {
      v = g.S[i + (size_t)j * g.lds];   // rho C^T C is added afterwards by a GEMM
    } else if (i >= nG && j < nG) {
      v = g.C[(i - nG) + (size_t)j * nc];
    } else if (i < nG && j >= nG) {
      v = g.C[(j - nG) + (size_t)i * nc];
    }
    col[i] = v;
  }
  if (threadIdx.x == 0) {
    g.A[(nl + j) + (size_t)j * g.lda] = 1.0;
    g.A[j + (size_t)(nl + j) * g.lda] = 1.0;
  }
}

// dst = sqrt(scale[s]) src on the entries [off[s], off[s] + cnt[s]) of every s
__global__ __launch_bounds__(256) void k_scale_sqrt_sub(const int64_t* __restrict__ off,
                                                        const int64_t* __restrict__ cnt,
                                                        const double* __restrict__ scale,
                                                        const double* __restrict__ src,
                                                        double* __restrict__ dst) {
  const int s = blockIdx.y;
  const double f = sqrt(scale[s]);
  const int64_t o = off[s], n = cnt[s];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[o + i] = f * src[o + i];
}

void launch_scale_sqrt_sub(int nsub, const int64_t* off, const int64_t* cnt, const double* scale,
                           const double* src, double* dst, hipStream_t st) {
  if (nsub == 0) return;
  k_scale_sqrt_sub<<<dim3(16, nsub), 256, 0, st>>>(off, cnt, scale, src, dst);
  AMB_LAUNCH_CHECK();
}

void launch_neumann_fill(const NeuDesc* d, int nd, int ncols, hipStream_t st) {
  if (ncols == 0) return;
  k_neumann_fill<<<ncols, 256, 0, st>>>(d, nd);
  AMB_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_diag_mean(const int64_t* off, const int* ld, const int* n0,
                                                   const int* n, const double* A, double* out) {
  const int s = blockIdx.x;
  const double* a = A + off[s];
  const int l = ld[s], b = n0[s], m = n[s];
  double v = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) v += a[(b + i) + (size_t)(b + i) * l];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    out[s] = m > 0 ? t / m : 1.0;
  }
}

void launch_diag_mean(int nsub, const int64_t* off, const int* ld, const int* n0, const int* n,
                      const double* A, double* out, hipStream_t st) {
  if (nsub == 0) return;
  k_diag_mean<<<nsub, 256, 0, st>>>(off, ld, n0, n, A, out);
  AMB_LAUNCH_CHECK();
}

__global__ void k_extract_kc(const int64_t* naug_off, const int* naug_ld, const int* nG,
                             const int* nc, const int64_t* kc_off, const double* rho,
                             const int* nrho, const double* naug, double* kc) {
  const int s = blockIdx.y;
  const int m = nc[s];
  const int mr = nrho ? nrho[s] : m;
  const int base = nG[s] + m + nG[s];
  const double* a = naug + naug_off[s];
  const int l = naug_ld[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m * m; i += gridDim.x * blockDim.x) {
    const int r = i % m, c = i / m;
    kc[kc_off[s] + i] = a[(base + r) + (size_t)(base + c) * l] - (r == c && r < mr ? rho[s] : 0.0);
  }
}

void launch_extract_kc(int nsub, const int64_t* naug_off, const int* naug_ld, const int* nG,
                       const int* nc, const int64_t* kc_off, const double* rho, const int* nrho,
                       const double* naug, double* kc, hipStream_t st) {
  if (nsub == 0) return;
  dim3 g(4, nsub);
  k_extract_kc<<<g, 256, 0, st>>>(naug_off, naug_ld, nG, nc, kc_off, rho, nrho, naug, kc);
  AMB_LAUNCH_CHECK();
}

// Border of the bordered inverse: T[0:nl, nl:nl+k] = -W, T[nl:, 0:nl] = -W^T,
// T[nl:, nl:] = -Tsc (one descriptor per matrix, blockIdx.y).
__global__ void k_border_fill(const BorderDesc* d) {
  const BorderDesc g = d[blockIdx.y];
  const int nl = g.nl, k = g.k;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl * k; i += gridDim.x * blockDim.x) {
    const int r = i % nl, j = i / nl;
    const double v = -g.W[r + (size_t)j * g.ldw];
    g.T[r + (size_t)(nl + j) * g.ldt] = v;
    g.T[(nl + j) + (size_t)r * g.ldt] = v;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k * k; i += gridDim.x * blockDim.x) {
    const int r = i % k, j = i / k;
    g.T[(nl + r) + (size_t)(nl + j) * g.ldt] = -g.Tsc[r + (size_t)j * g.lds];
  }
}

void launch_border_fill(const BorderDesc* d, int n, hipStream_t st) {
  if (n == 0) return;
  dim3 g(16, n);
  k_border_fill<<<g, 256, 0, st>>>(d);
  AMB_LAUNCH_CHECK();
}

__global__ void k_copy_block(const int64_t* src_off, const int* src_ld, const int* r0,
                             const int* rows, const int* cols, const int64_t* dst_off,
                             const int* dst_ld, const double* src, double* dst) {
  const int s = blockIdx.y;
  const int m = rows[s], n = cols[s];
  const double* a = src + src_off[s];
  double* b = dst + dst_off[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m * n; i += gridDim.x * blockDim.x) {
    const int r = i % m, c = i / m;
    b[r + (size_t)c * dst_ld[s]] = a[(r0[s] + r) + (size_t)(r0[s] + c) * src_ld[s]];
  }
}

void launch_copy_block(int nsub, const int64_t* src_off, const int* src_ld, const int* r0,
                       const int* rows, const int* cols, const int64_t* dst_off, const int* dst_ld,
                       const double* src, double* dst, hipStream_t st) {
  if (nsub == 0) return;
  dim3 g(16, nsub);
  k_copy_block<<<g, 256, 0, st>>>(src_off, src_ld, r0, rows, cols, dst_off, dst_ld, src, dst);
  AMB_LAUNCH_CHECK();
}

__global__ void k_diag_copy(int n, const int64_t* pos, const double* A, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = A[pos[k]];
}

void launch_diag_copy(int n, const int64_t* pos, const double* A, double* out, hipStream_t st) {
  if (n == 0) return;
  k_diag_copy<<<ceil_div(n, 256), 256, 0, st>>>(n, pos, A, out);
  AMB_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Krylov helpers
// ---------------------------------------------------------------------------

constexpr int DOT_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_dot_part(int n, const double* a, const double* b,
                                                  double* part) {
  const int r = blockIdx.y;
  const double* x = a + (size_t)r * n;
  const double* y = b + (size_t)r * n;
  double v = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    v += x[i] * y[i];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x + r * gridDim.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_dot_final(int nb, const double* part, double* out) {
  const int r = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) v += part[i + r * nb];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[r] = red[0] + red[1] + red[2] + red[3];
}

// One-launch column dots: every block writes its partial and releases it
// (device scope) before counting itself in at the column's counter; the
// block that arrives last acquires the partials, sums them in block order
// and resets the counter for the next call.  Blocks of at least DOT_MIN
// entries, at most DOT_BLOCKS of them: on short vectors the cache
// write-backs of the release would cost more than the partial sums.
__global__ __launch_bounds__(256) void k_dot_fin(int n, const double* a, const double* b,
                                                 double* part, int* cnt, double* out) {
  const int r = blockIdx.y;
  const int nb = gridDim.x;
  const double* x = a + (size_t)r * n;
  const double* y = b + (size_t)r * n;
  double v = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    v += x[i] * y[i];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __shared__ double red[4];
  __shared__ int last;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x + r * nb] = red[0] + red[1] + red[2] + red[3];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    last = atomicAdd(&cnt[r], 1) == nb - 1;
  }
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  v = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    v += part[i + r * nb];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    out[r] = red[0] + red[1] + red[2] + red[3];
    cnt[r] = 0;
  }
}

// part: DOT_BLOCKS * nrhs doubles; cnt: nrhs ints, zero between calls.
void launch_dot_cols_fin(int n, int nrhs, const double* a, const double* b, double* part,
                         int* cnt, double* out, hipStream_t st) {
  constexpr int DOT_MIN = 512;
  dim3 g(std::max(1, std::min(DOT_BLOCKS, n / DOT_MIN)), nrhs);
  k_dot_fin<<<g, 256, 0, st>>>(n, a, b, part, cnt, out);
  AMB_LAUNCH_CHECK();
}

// Deterministic two-stage column dots: part needs DOT_BLOCKS * nrhs doubles.
void launch_dot_cols(int n, int nrhs, const double* a, const double* b, double* part, double* out,
                     hipStream_t st) {
  dim3 g(DOT_BLOCKS, nrhs);
  k_dot_part<<<g, 256, 0, st>>>(n, a, b, part);
  k_dot_final<<<nrhs, 256, 0, st>>>(DOT_BLOCKS, part, out);
  AMB_LAUNCH_CHECK();
}

__global__ void k_pcg_xr(int n, int nrhs, const double* rz, const double* pq, const int* active,
                         double* x, double* r, const double* p, const double* q, double* ahist,
                         const int* itp, int maxit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const int it = *itp;
  // a zero direction (a residual that is exactly zero) takes no step
  const double a = active[c] && pq[c] != 0.0 ? rz[c] / pq[c] : 0.0;
  if (i == 0 && active[c]) ahist[it + (size_t)c * maxit] = a;
  if (i >= n) return;
  const size_t k = i + (size_t)c * n;
  x[k] += a * p[k];
  r[k] -= a * q[k];
}

void launch_pcg_update_x_r(int n, int nrhs, const double* rz, const double* pq, const int* active,
                           double* x, double* r, const double* p, const double* q, double* alpha_hist,
                           const int* itp, int maxit, hipStream_t st) {
  dim3 g(ceil_div(n, 256), nrhs);
  k_pcg_xr<<<g, 256, 0, st>>>(n, nrhs, rz, pq, active, x, r, p, q, alpha_hist, itp, maxit);
  AMB_LAUNCH_CHECK();
}

// beta = rz_new / rz; 0 for a column whose residual was just replaced by
// the true one (restart: p = z), whose repl flag is cleared here.  Closes
// the iteration: the device iteration counter *itp advances.
__global__ void k_pcg_beta(int nrhs, const double* rz_new, double* rz, double* beta,
                           const int* active, int* repl, double* bhist, int* itp, int maxit) {
  const int c = threadIdx.x;
  const int it = *itp;
  if (c < nrhs) {
    const bool restart = repl && repl[c];
    if (restart) repl[c] = 0;
    const double b = active[c] && !restart && rz[c] != 0.0 ? rz_new[c] / rz[c] : 0.0;
    beta[c] = b;
    if (active[c]) {
      bhist[it + (size_t)c * maxit] = b;
      rz[c] = rz_new[c];
    }
  }
  __syncthreads();
  if (c == 0) *itp = it + 1;
}

__global__ void k_pcg_p(int n, const double* beta, const int* active, double* p, const double* z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || !active[c]) return;
  const size_t k = i + (size_t)c * n;
  p[k] = z[k] + beta[c] * p[k];
}

// beta = rz_new / rz (stored after rz_new in the same array: rz_new[nrhs..2nrhs) used as scratch)
void launch_pcg_update_p(int n, int nrhs, const double* rz_new, double* rz, const int* active,
                         int* restart, double* p, const double* z, double* beta_hist, int* itp,
                         int maxit, hipStream_t st) {
  double* beta = rz + nrhs;   // scratch right after rz
  k_pcg_beta<<<1, 64, 0, st>>>(nrhs, rz_new, rz, beta, active, restart, beta_hist, itp, maxit);
  dim3 g(ceil_div(n, 256), nrhs);
  k_pcg_p<<<g, 256, 0, st>>>(n, beta, active, p, z);
  AMB_LAUNCH_CHECK();
}

// PCG column flags, kept on the device (one thread per column, nrhs <= 64).
// cnt[0]: columns whose recursive residual met rtol in this iteration,
// cnt[1]: active columns, cnt[2]: residual replacements of this check.
__global__ void k_pcg_init_flags(int nrhs, const double* ff, int* act, int* nal, int* repl,
                                 int* stall, double* tprev, int* cnt) {
  const int c = threadIdx.x;
  if (c < nrhs) {
    act[c] = ff[c] > 0.0 ? 1 : 0;
    nal[c] = 0;
    repl[c] = 0;
    stall[c] = 0;
    tprev[c] = 0.0;
  }
  __syncthreads();
  if (c == 0) {
    int a = 0;
    for (int k = 0; k < nrhs; ++k) a += act[k];
    cnt[0] = 0;
    cnt[1] = a;
    cnt[2] = 0;
    cnt[3] = 0;
    cnt[4] = 0;   // iteration counter
  }
  if (c < nrhs) cnt[8 + c] = 0;   // one-launch dot counters
}

void launch_pcg_init_flags(int nrhs, const double* ff, int* act, int* nal, int* repl, int* stall,
                           double* tprev, int* cnt, hipStream_t st) {
  k_pcg_init_flags<<<1, 64, 0, st>>>(nrhs, ff, act, nal, repl, stall, tprev, cnt);
  AMB_LAUNCH_CHECK();
}

// After iteration `it`: every active column has taken it + 1 steps; meets[c]
// says its recursive residual rr[c] <= rtol^2 ff[c].
__global__ void k_pcg_meets(int nrhs, const double* rr, const double* ff, double rtol2,
                            const int* act, int* nal, int* meets, int* cnt, const int* itp) {
  const int c = threadIdx.x;
  const int it = *itp;
  if (c < nrhs) {
    const int m = act[c] && rr[c] <= rtol2 * ff[c];
    meets[c] = m;
    if (act[c]) nal[c] = it + 1;
  }
  __syncthreads();
  if (c == 0) {
    int k = 0;
    for (int j = 0; j < nrhs; ++j) k += meets[j];
    cnt[0] = k;
  }
}

void launch_pcg_meets(int nrhs, const double* rr, const double* ff, double rtol2, const int* act,
                      int* nal, int* meets, int* cnt, const int* itp, hipStream_t st) {
  k_pcg_meets<<<1, 64, 0, st>>>(nrhs, rr, ff, rtol2, act, nal, meets, cnt, itp);
  AMB_LAUNCH_CHECK();
}

// For the columns in meets, with their true residuals tt: the column stops
// (act = 0) if tt <= rtol^2 ff; it stops as stalled (stall = 1) if the true
// residual fell by less than half since the column's previous check (tprev:
// the rounding floor of f - K x in FP64 is reached above rtol); otherwise it
// is marked for residual replacement (repl = 1, which also restarts its
// search direction).  cnt[3] counts stalled columns.
__global__ void k_pcg_true(int nrhs, const double* tt, const double* ff, double rtol2, int* act,
                           const int* meets, int* repl, int* stall, double* tprev, int* cnt) {
  const int c = threadIdx.x;
  if (c < nrhs && meets[c]) {
    const double t = tt[c];
    if (t <= rtol2 * ff[c]) {
      act[c] = 0;
    } else if (tprev[c] > 0.0 && t > 0.25 * tprev[c]) {
      act[c] = 0;
      stall[c] = 1;
    } else {
      repl[c] = 1;
      tprev[c] = t;
    }
  }
  __syncthreads();
  if (c == 0) {
    int a = 0, r = 0, sl = 0;
    for (int j = 0; j < nrhs; ++j) {
      a += act[j];
      r += repl[j];
      sl += stall[j];
    }
    cnt[1] = a;
    cnt[2] = r;
    cnt[3] = sl;
  }
}

void launch_pcg_true(int nrhs, const double* tt, const double* ff, double rtol2, int* act,
                     const int* meets, int* repl, int* stall, double* tprev, int* cnt,
                     hipStream_t st) {
  k_pcg_true<<<1, 64, 0, st>>>(nrhs, tt, ff, rtol2, act, meets, repl, stall, tprev, cnt);
  AMB_LAUNCH_CHECK();
}

// Extreme eigenvalues of the CG Lanczos tridiagonal by Sturm bisection.
__device__ inline int sturm_count(const double* d, const double* e2, int k, double x) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0) ++cnt;
  for (int j = 1; j < k; ++j) {
    if (q == 0.0) q = 1e-300;
    q = d[j] - x - e2[j - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// Extreme eigenvalues by parallel multisection: every thread evaluates the
// Sturm count at one point of the current bracket, which shrinks by the
// block size per pass.
__device__ inline double multisect(const double* d, const double* e2, int k, double lo, double hi,
                                   int target, int* cnt) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int pass = 0; pass < 12; ++pass) {
    const double h = (hi - lo) / (nt + 1);
    cnt[tid] = sturm_count(d, e2, k, lo + (tid + 1) * h);
    __syncthreads();
    int first = nt;
    for (int t = 0; t < nt; ++t)
      if (cnt[t] >= target) { first = t; break; }
    __syncthreads();
    const double nlo = lo + first * h;
    hi = lo + (first + 1) * h;
    lo = nlo;
  }
  return 0.5 * (lo + hi);
}

__global__ __launch_bounds__(256) void k_lanczos(int nrhs, const int* nalpha, const double* alpha,
                                                 const double* beta, int maxit, double* out,
                                                 double* work) {
  __shared__ int cnt[256];
  __shared__ double bounds[2];
  const int c = blockIdx.x;
  const int k = nalpha[c];
  if (k <= 0) {
    if (threadIdx.x == 0) { out[c] = 1.0; out[nrhs + c] = 1.0; out[2 * nrhs + c] = 1.0; }
    return;
  }
  const double* a = alpha + (size_t)c * maxit;
  const double* b = beta + (size_t)c * maxit;
  double* d = work + (size_t)c * 2 * maxit;
  double* e2 = d + maxit;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    d[j] = (j == 0) ? 1.0 / a[0] : 1.0 / a[j] + b[j - 1] / a[j - 1];
    if (j > 0) {
      const double e = sqrt(b[j - 1]) / a[j - 1];
      e2[j - 1] = e * e;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lo = 1e300, hi = -1e300;
    for (int j = 0; j < k; ++j) {
      double rr = 0.0;
      if (j > 0) rr += sqrt(e2[j - 1]);
      if (j < k - 1) rr += sqrt(e2[j]);
      lo = fmin(lo, d[j] - rr);
      hi = fmax(hi, d[j] + rr);
    }
    bounds[0] = lo;
    bounds[1] = hi;
  }
  __syncthreads();
  const double lmin = multisect(d, e2, k, bounds[0], bounds[1], 1, cnt);
  const double lmax = multisect(d, e2, k, bounds[0], bounds[1], k, cnt);
  if (threadIdx.x == 0) {
    out[c] = lmax / lmin;
    out[nrhs + c] = lmin;
    out[2 * nrhs + c] = lmax;
  }
}

// out[0:nrhs] = cond, out[nrhs:2nrhs] = lambda_min, out[2nrhs:3nrhs] = lambda_max.
// `out` must hold 3*nrhs + 2*maxit*nrhs doubles (the tail is scratch).
void launch_lanczos_cond(int nrhs, const int* nalpha, const double* alpha, const double* beta,
                         int maxit, double* out, hipStream_t st) {
  k_lanczos<<<nrhs, 256, 0, st>>>(nrhs, nalpha, alpha, beta, maxit, out, out + 3 * nrhs);
  AMB_LAUNCH_CHECK();
}

__global__ void k_fill(double* p, size_t n, double v) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill(double* p, size_t n, double v, hipStream_t st) {
  if (n == 0) return;
  k_fill<<<ceil_div(int64_t(n), 256), 256, 0, st>>>(p, n, v);
  AMB_LAUNCH_CHECK();
}

__global__ void k_copy(double* dst, const double* src, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

void launch_copy(double* dst, const double* src, size_t n, hipStream_t st) {
  if (n == 0) return;
  k_copy<<<ceil_div(int64_t(n), 256), 256, 0, st>>>(dst, src, n);
  AMB_LAUNCH_CHECK();
}

// out = 10^theta elementwise (coefficients from log10-coefficients)
__global__ void k_pow10(size_t n, const double* theta, double* out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = exp10(theta[i]);
}

void launch_pow10(size_t n, const double* theta, double* out, hipStream_t st) {
  if (n == 0) return;
  k_pow10<<<ceil_div(int64_t(n), 256), 256, 0, st>>>(n, theta, out);
  AMB_LAUNCH_CHECK();
}

// dst[:, c] = src[:, c] for the columns c with mask[c] != 0 (residual
// replacement of the PCG columns whose true residual lags the recursive one)
__global__ void k_copy_cols(int n, const double* src, double* dst, const int* mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || !mask[c]) return;
  dst[i + (size_t)c * n] = src[i + (size_t)c * n];
}

void launch_copy_cols(int n, int nrhs, const double* src, double* dst, const int* mask,
                      hipStream_t st) {
  if (n == 0 || nrhs == 0) return;
  dim3 g(ceil_div(n, 256), nrhs);
  k_copy_cols<<<g, 256, 0, st>>>(n, src, dst, mask);
  AMB_LAUNCH_CHECK();
}

// Input check of the element data: bad[0] = 1 + the first element whose
// coefficient is not a finite number (0 if none), bad[1] the same for a
// Poisson ratio outside (-1, 1/2) or not finite (nu may be null).
__global__ void k_check_coeff(int n, const double* coeff, const double* nu, int* bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c = coeff[i];
  if (!(fabs(c) <= 1.7976931348623157e308)) atomicMin(&bad[0], i + 1);
  if (nu) {
    const double v = nu[i];
    if (!(v > -1.0 && v < 0.5)) atomicMin(&bad[1], i + 1);
  }
}

void launch_check_coeff(int n, const double* coeff, const double* nu, int* bad, hipStream_t st) {
  if (n == 0) return;
  k_check_coeff<<<ceil_div(n, 256), 256, 0, st>>>(n, coeff, nu, bad);
  AMB_LAUNCH_CHECK();
}

// out = a - b elementwise
__global__ void k_sub(size_t n, const double* a, const double* b, double* out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

void launch_sub(size_t n, const double* a, const double* b, double* out, hipStream_t st) {
  if (n == 0) return;
  k_sub<<<ceil_div(int64_t(n), 256), 256, 0, st>>>(n, a, b, out);
  AMB_LAUNCH_CHECK();
}

}  // namespace ambddc

namespace ambddc {

__global__ void k_move(int n, const int64_t* sidx, const double* src, int64_t lds,
                       const int64_t* didx, double* dst, int64_t ldd, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t a = sidx[k], b = didx[k];
  for (int r = 0; r < nrhs; ++r) dst[b + r * ldd] = src[a + r * lds];
}

void launch_move(int n, const int64_t* sidx, const double* src, int64_t lds, const int64_t* didx,
                 double* dst, int64_t ldd, int nrhs, hipStream_t st) {
  if (n == 0) return;
  k_move<<<ceil_div(n, 256), 256, 0, st>>>(n, sidx, src, lds, didx, dst, ldd, nrhs);
  AMB_LAUNCH_CHECK();
}

// dst[idx[k], r] = 0 for every column (mask null) or the columns with mask[r].
__global__ void k_zero_rows(int n, const int64_t* idx, double* dst, int64_t ldd, int nrhs,
                            const int* mask) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t b = idx[k];
  for (int r = 0; r < nrhs; ++r)
    if (!mask || mask[r]) dst[b + r * ldd] = 0.0;
}

void launch_zero_rows(int n, const int64_t* idx, double* dst, int64_t ldd, int nrhs,
                      const int* mask, hipStream_t st) {
  if (n == 0) return;
  k_zero_rows<<<ceil_div(n, 256), 256, 0, st>>>(n, idx, dst, ldd, nrhs, mask);
  AMB_LAUNCH_CHECK();
}

// dst[didx[k], r] += src[sidx[k], r] for the columns r with mask[r] != 0.
__global__ void k_move_add_masked(int n, const int64_t* sidx, const double* src, int64_t lds,
                                  const int64_t* didx, double* dst, int64_t ldd, int nrhs,
                                  const int* mask) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t a = sidx[k], b = didx[k];
  for (int r = 0; r < nrhs; ++r)
    if (mask[r]) dst[b + r * ldd] += src[a + r * lds];
}

void launch_move_add_masked(int n, const int64_t* sidx, const double* src, int64_t lds,
                            const int64_t* didx, double* dst, int64_t ldd, int nrhs,
                            const int* mask, hipStream_t st) {
  if (n == 0) return;
  k_move_add_masked<<<ceil_div(n, 256), 256, 0, st>>>(n, sidx, src, lds, didx, dst, ldd, nrhs,
                                                      mask);
  AMB_LAUNCH_CHECK();
}

// Rigid-body modes at level-1 free DOFs: Poisson the constant; elasticity
// three translations and three rotations about the origin.
__global__ void k_rigid1(int n_nodes, int dof, const double* coords, const int* free_of_full,
                         int ndof, double* rigid) {
  const int nd = blockIdx.x * blockDim.x + threadIdx.x;
  if (nd >= n_nodes) return;
  const double x = coords[3 * nd], y = coords[3 * nd + 1], z = coords[3 * nd + 2];
  for (int q = 0; q < dof; ++q) {
    const int f = free_of_full[(size_t)nd * dof + q];
    if (f < 0) continue;
    if (dof == 1) { rigid[f] = 1.0; continue; }
    double v[6] = {0, 0, 0, 0, 0, 0};
    v[q] = 1.0;
    if (q == 0) { v[4] = z; v[5] = -y; }
    if (q == 1) { v[3] = -z; v[5] = x; }
    if (q == 2) { v[3] = y; v[4] = -x; }
    for (int c = 0; c < 6; ++c) rigid[f + (size_t)c * ndof] = v[c];
  }
}

void launch_rigid_level1(int n_nodes, int dof, const double* coords, const int* free_of_full,
                         int ndof, double* rigid, hipStream_t st) {
  if (n_nodes == 0) return;
  k_rigid1<<<ceil_div(n_nodes, 256), 256, 0, st>>>(n_nodes, dof, coords, free_of_full, ndof, rigid);
  AMB_LAUNCH_CHECK();
}

// Coarse values of rigid modes: rigid2[k, c] = C^s_r . rigid1[Gamma^s, c] for
// the first (s, r) carrying coarse DOF k.
__global__ void k_coarse_rigid(int n2, int nrb, const int* sub_of, const int* row_of,
                               const int64_t* c_off, const int* nc, const int* nG,
                               const int64_t* Goff, const int* Gdof, const double* C,
                               const double* rigid1, int n1, double* rigid2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n2) return;
  const int s = sub_of[k], r = row_of[k];
  for (int c = 0; c < nrb; ++c) {
    double v = 0.0;
    for (int i = 0; i < nG[s]; ++i)
      v += C[c_off[s] + r + (size_t)i * nc[s]] * rigid1[Gdof[Goff[s] + i] + (size_t)c * n1];
    rigid2[k + (size_t)c * n2] = v;
  }
}

void launch_coarse_rigid(int n2, int nrb, const int* sub_of, const int* row_of, const int64_t* c_off,
                         const int* nc, const int* nG, const int64_t* Goff, const int* Gdof,
                         const double* C, const double* rigid1, int n1, double* rigid2,
                         hipStream_t st) {
  if (n2 == 0) return;
  k_coarse_rigid<<<ceil_div(n2, 256), 256, 0, st>>>(n2, nrb, sub_of, row_of, c_off, nc, nG, Goff,
                                                    Gdof, C, rigid1, n1, rigid2);
  AMB_LAUNCH_CHECK();
}

}  // namespace ambddc
