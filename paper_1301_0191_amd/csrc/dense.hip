// Batched dense kernels on uneven batches (see dense.hpp).
#include <algorithm>
#include <cmath>

#include "dense.hpp"
#include "mfma_tile.hpp"

namespace ambddc {

__device__ __forceinline__ int ceil_div_dev(int a, int b) { return (a + b - 1) / b; }

// --------------------------------------------------------------------------
// GEMM
// --------------------------------------------------------------------------

// Column-slot test of a tile: does any slot in [c0, c1] belong to an item
// whose flags meet the mask?
__device__ __forceinline__ bool slots_live(const GemmDesc& g, int c0, int c1, const int* act,
                                           int mask, int excl) {
  bool any = false, veto = false;
  for (int j = c0 / g.scols; j <= c1 / g.scols; ++j) {
    const int a = act[g.spair[j]];
    any = any || (a & mask) != 0;
    veto = veto || (a & excl) != 0;
  }
  return any && !veto;
}

template <int WM, int WN, typename TBe>
__global__ __launch_bounds__(256) void k_gemm_f32(const GemmDesc* __restrict__ d, int nd,
                                                  double alpha, double beta,
                                                  const int* __restrict__ act, int mask,
                                                  int excl) {
  __shared__ TileSmem32<WM, WN> sm;
  const int tile = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmDesc g = d[lo];
  if (g.flag && *g.flag == 0) return;
  const int lt = tile - g.tile_start;
  const int tm = lt % g.tiles_m, tn = lt / g.tiles_m;
  if (g.scols > 0 &&
      !slots_live(g, tn * 32 * WN, min(g.N, (tn + 1) * 32 * WN) - 1, act, mask, excl))
    return;
  mfma_tile_f32<WM, WN, TBe>(static_cast<const float*>(g.A), g.lda,
                             reinterpret_cast<const TBe*>(g.B), g.ldb, g.C, g.ldc, g.M, g.N, g.K,
                             tm * 32 * WM, tn * 32 * WN, alpha, beta, sm);
}

template <bool TA, bool TB, int WM, int WN, typename TAe>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(const GemmDesc* __restrict__ d, int nd, double alpha,
                                              double beta, const int* __restrict__ act, int mask,
                                              int excl) {
  __shared__ TileSmem<WM, WN> sm;
  const int tile = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmDesc g = d[lo];
  if (g.flag && *g.flag == 0) return;
  const int lt = tile - g.tile_start;
  const int tm = lt % g.tiles_m, tn = lt / g.tiles_m;
  if (g.scols > 0) {
    const int c0 = tn * TileShape<WM, WN>::TN;
    const int c1 = min(g.N, c0 + TileShape<WM, WN>::TN) - 1;
    if (!slots_live(g, c0, c1, act, mask, excl)) return;
  }
  mfma_tile<TA, TB, WM, WN>(static_cast<const TAe*>(g.A), g.lda, g.B, g.ldb, g.C, g.ldc, g.M, g.N,
                            g.K, tm * TileShape<WM, WN>::TM, tn * TileShape<WM, WN>::TN, alpha,
                            beta, -1, sm);
}

// C = alpha sum_s P_s + beta C for every split product, one workgroup each.
__global__ __launch_bounds__(256) void k_split_sum(const SplitDesc* __restrict__ d,
                                                   const double* __restrict__ part, double alpha,
                                                   double beta) {
  const SplitDesc g = d[blockIdx.x];
  if (g.flag && *g.flag == 0) return;
  const int mn = g.M * g.N;
  const double* p = part + g.poff;
  for (int e = threadIdx.x; e < mn; e += 256) {
    double v = 0.0;
    for (int s = 0; s < g.S; ++s) v += p[(size_t)s * mn + e];
    double* c = g.C + (e % g.M) + (size_t)(e / g.M) * g.ldc;
    *c = alpha * v + (beta != 0.0 ? beta * (*c) : 0.0);
  }
}

void GemmOp::finalize(hipStream_t st) {
  const int TM = narrow ? 128 : 64, TN = narrow ? 32 : 64;
  hs.clear();
  if (ksplit != 1 && !h.empty() && !f32) {
    int t0 = 0, kmin = 1 << 30;
    for (const auto& g : h) {
      if (g.scols > 0) throw Error(1, "GemmOp: split-K with column slots");
      t0 += ceil_div(g.M, TM) * ceil_div(g.N, TN);
      kmin = std::min(kmin, g.K);
    }
    int S = ksplit > 1 ? ksplit : std::max(1, std::min(8, SPLIT_TARGET / std::max(t0, 1)));
    while (S > 1 && kmin / S < 64) --S;
    if (S > 1) {
      std::vector<GemmDesc> hp;
      std::vector<int64_t> eoff;   // partial block of every piece
      int64_t poff = 0;
      for (const auto& g : h) {
        hs.push_back(SplitDesc{g.C, g.ldc, g.M, g.N, g.flag, poff, S});
        for (int q = 0; q < S; ++q) {
          const int k0 = int(int64_t(g.K) * q / S), k1 = int(int64_t(g.K) * (q + 1) / S);
          GemmDesc e = g;
          const size_t ao = ta ? size_t(k0) : size_t(k0) * g.lda;
          const size_t bo = tb ? size_t(k0) * g.ldb : size_t(k0);
          e.A = static_cast<const double*>(g.A) + ao;
          e.B = g.B + bo;
          e.K = k1 - k0;
          e.C = nullptr;   // set below, once the partial buffer exists
          e.ldc = g.M;
          eoff.push_back(poff + int64_t(q) * g.M * g.N);
          hp.push_back(e);
        }
        poff += int64_t(S) * g.M * g.N;
      }
      if (a32) throw Error(1, "GemmOp: split-K with FP32 operands");
      part.alloc(size_t(poff));
      for (size_t i = 0; i < hp.size(); ++i) hp[i].C = part.p + eoff[i];
      h.swap(hp);
      ds.upload(hs, st);
    }
  }
  tiles = 0;
  for (auto& g : h) {
    if (g.scols > 0 && !act) throw Error(1, "GemmOp: column slots without item flags");
    g.tiles_m = ceil_div(g.M, TM);
    g.tile_start = tiles;
    tiles += g.tiles_m * ceil_div(g.N, TN);
  }
  d.upload(h, st);
}

template <bool TA, bool TB, typename TAe>
static void gemm_dispatch(const GemmOp& op, double alpha, double beta, hipStream_t st) {
  if (op.narrow)
    k_gemm<TA, TB, 4, 1, TAe><<<op.tiles, 256, 0, st>>>(op.d.p, int(op.h.size()), alpha, beta,
                                                        op.act, op.act_mask, op.act_excl);
  else
    k_gemm<TA, TB, 2, 2, TAe><<<op.tiles, 256, 0, st>>>(op.d.p, int(op.h.size()), alpha, beta,
                                                        op.act, op.act_mask, op.act_excl);
}

template <typename TAe>
static void gemm_run(const GemmOp& op, double alpha, double beta, hipStream_t st) {
  if (!op.ta && !op.tb) gemm_dispatch<false, false, TAe>(op, alpha, beta, st);
  else if (op.ta && !op.tb) gemm_dispatch<true, false, TAe>(op, alpha, beta, st);
  else if (!op.ta && op.tb) gemm_dispatch<false, true, TAe>(op, alpha, beta, st);
  else gemm_dispatch<true, true, TAe>(op, alpha, beta, st);
}

void GemmOp::run(double alpha, double beta, hipStream_t st) const {
  if (h.empty() || tiles == 0) return;
  if (f32) {
    if (ta || tb || !hs.empty()) throw Error(1, "GemmOp: FP32 products are not transposed or split");
    if (narrow && b32)
      k_gemm_f32<4, 1, float><<<tiles, 256, 0, st>>>(d.p, int(h.size()), alpha, beta, act,
                                                     act_mask, act_excl);
    else if (narrow)
      k_gemm_f32<4, 1, double><<<tiles, 256, 0, st>>>(d.p, int(h.size()), alpha, beta, act,
                                                      act_mask, act_excl);
    else if (b32)
      k_gemm_f32<2, 2, float><<<tiles, 256, 0, st>>>(d.p, int(h.size()), alpha, beta, act,
                                                     act_mask, act_excl);
    else
      k_gemm_f32<2, 2, double><<<tiles, 256, 0, st>>>(d.p, int(h.size()), alpha, beta, act,
                                                      act_mask, act_excl);
    AMB_LAUNCH_CHECK();
    return;
  }
  if (a32 && ta) throw Error(1, "GemmOp: FP32 operands are panel-packed, not transposed");
  if (!hs.empty()) {
    gemm_run<double>(*this, 1.0, 0.0, st);   // partial products
    AMB_LAUNCH_CHECK();
    k_split_sum<<<int(hs.size()), 256, 0, st>>>(ds.p, part.p, alpha, beta);
    AMB_LAUNCH_CHECK();
    return;
  }
  if (a32) gemm_run<float>(*this, alpha, beta, st);
  else gemm_run<double>(*this, alpha, beta, st);
  AMB_LAUNCH_CHECK();
}

void TunedGemm::drop_events() {
  for (auto& e : ev) {
    for (hipEvent_t x : e) (void)hipEventDestroy(x);
    e.clear();
  }
}

void TunedGemm::run(double alpha, double beta, hipStream_t st) {
  if (follow) {
    v[*follow >= 0 ? *follow : 0].run(alpha, beta, st);
    return;
  }
  if (!choice || *choice >= 0) {
    v[choice ? *choice : 0].run(alpha, beta, st);
    return;
  }
  const int k = calls & 1;
  hipEvent_t a, b;
  AMB_HIP(hipEventCreate(&a));
  AMB_HIP(hipEventCreate(&b));
  AMB_HIP(hipEventRecord(a, st));
  v[k].run(alpha, beta, st);
  AMB_HIP(hipEventRecord(b, st));
  ev[k].push_back(a);
  ev[k].push_back(b);
  if (++calls < 2 * TUNE_CALLS) return;
  AMB_HIP(hipEventSynchronize(b));
  float t[2] = {0.0f, 0.0f};
  for (int q = 0; q < 2; ++q)
    for (size_t i = 0; i + 1 < ev[q].size(); i += 2) {
      float ms = 0.0f;
      AMB_HIP(hipEventElapsedTime(&ms, ev[q][i], ev[q][i + 1]));
      t[q] += ms;
    }
  *choice = t[1] < t[0] ? 1 : 0;
  drop_events();
}

// --------------------------------------------------------------------------
// FP32 copies of dense blocks (one workgroup per 4096 entries)
// --------------------------------------------------------------------------

constexpr int CVT_PER_WG = 4096;

__global__ __launch_bounds__(256) void k_cvt_f32(const CvtDesc* __restrict__ d, int nd) {
  const int wg = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  const CvtDesc g = d[lo];
  const int64_t n = int64_t(g.rows) * g.cols;
  const int64_t e0 = int64_t(wg - g.wg_start) * CVT_PER_WG;
  for (int64_t e = e0 + threadIdx.x; e < min(n, e0 + CVT_PER_WG); e += 256) {
    const int64_t r = e % g.rows, c = e / g.rows;
    g.dst[r + c * g.ldd] = static_cast<float>(g.src[r + c * g.lds]);
  }
}

void convert_blocks_f32(const std::vector<CvtDesc>& blocks, hipStream_t st) {
  std::vector<CvtDesc> h;
  int wgs = 0;
  for (CvtDesc b : blocks) {
    const int64_t n = int64_t(b.rows) * b.cols;
    if (n <= 0) continue;
    b.wg_start = wgs;
    wgs += ceil_div(n, CVT_PER_WG);
    h.push_back(b);
  }
  if (h.empty()) return;
  DBuf<CvtDesc> d;
  d.upload(h, st);
  k_cvt_f32<<<wgs, 256, 0, st>>>(d.p, int(h.size()));
  AMB_LAUNCH_CHECK();
}

// --------------------------------------------------------------------------
// GEMV (transposed, several right-hand sides): one wave per output column
// --------------------------------------------------------------------------

// The column is read in 16-byte pairs (after one leading element when the
// column starts on an odd double), U pairs per lane in flight, so the wave
// keeps 4 KB of loads outstanding instead of waiting on every 512 bytes.
template <int R>
__global__ __launch_bounds__(256) void k_gemv_t(const GemvDesc* __restrict__ d, int nd, double alpha,
                                                double beta) {
  constexpr int U = 4;
  const int wg = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  const GemvDesc g = d[lo];
  const int col = (wg - g.wg_start) * 4 + (threadIdx.x >> 6);
  if (col >= g.M) return;
  const int lane = threadIdx.x & 63;
  const double* __restrict__ a = static_cast<const double*>(g.A) + (size_t)col * g.lda;
  const double* __restrict__ x = g.X;
  const size_t ldx = g.ldx;
  const int K = g.K;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const int head = (K > 0 && ((reinterpret_cast<uintptr_t>(a) >> 3) & 1)) ? 1 : 0;
  if (head && lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += a[0] * x[r * ldx];
  }
  const double2* __restrict__ a2 = reinterpret_cast<const double2*>(a + head);
  const double* __restrict__ xh = x + head;
  const int n2 = (K - head) >> 1;
  int p = lane;
  for (; p + 64 * (U - 1) < n2; p += 64 * U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = a2[p + 64 * u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = 2 * (p + 64 * u);
#pragma unroll
      for (int r = 0; r < R; ++r)
        acc[r] += v[u].x * xh[i + r * ldx] + v[u].y * xh[i + 1 + r * ldx];
    }
  }
  for (; p < n2; p += 64) {
    const double2 v = a2[p];
    const int i = 2 * p;
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += v.x * xh[i + r * ldx] + v.y * xh[i + 1 + r * ldx];
  }
  if (lane == 0 && ((K - head) & 1)) {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += a[K - 1] * x[K - 1 + r * ldx];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = acc[r];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    acc[r] = v;
  }
  if (lane < R) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r == lane) v = acc[r];
    double* y = g.Y + col + (size_t)lane * g.ldy;
    *y = alpha * v + (beta != 0.0 ? beta * (*y) : 0.0);
  }
}

// Short columns (K <= SHORT_K): a group of 16 lanes per output column, 16
// columns per workgroup; no lane leaves before the group reductions.
template <int R>
__global__ __launch_bounds__(256) void k_gemv_t16(const GemvDesc* __restrict__ d, int nd,
                                                  double alpha, double beta) {
  constexpr int G = 16;
  const int wg = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  const GemvDesc g = d[lo];
  const int col = (wg - g.wg_start) * (256 / G) + int(threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const bool ok = col < g.M;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  if (ok) {
    const double* __restrict__ a = static_cast<const double*>(g.A) + (size_t)col * g.lda;
    for (int i = lane; i < g.K; i += G) {
      const double av = a[i];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += av * g.X[i + (size_t)r * g.ldx];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = acc[r];
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    acc[r] = v;
  }
  if (ok && lane < R) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r == lane) v = acc[r];
    double* y = g.Y + col + (size_t)lane * g.ldy;
    *y = alpha * v + (beta != 0.0 ? beta * (*y) : 0.0);
  }
}

// --------------------------------------------------------------------------
// Symmetric GEMV from the tiles on or below the diagonal
// --------------------------------------------------------------------------

// Partials of one descriptor: tile (J, I), I >= J, at tri(J, I) = J nb -
// J (J - 1) / 2 + (I - J) holds A_IJ x_J (A_JJ x_J for I = J); the column
// sums sum_{I > J} A_IJ^T x_I follow at tri count + J.  Each is 3 x 64.
__device__ __forceinline__ int64_t symv_tri(int nb, int J, int I) {
  return int64_t(J) * nb - int64_t(J) * (J - 1) / 2 + (I - J);
}

// One workgroup per (descriptor, block column J); wave w owns the 16 columns
// J*64 + 16w.., lane l the row I*64 + l of every tile I >= J.
template <int R>
__global__ __launch_bounds__(256) void k_symv_part(const SymvDesc* __restrict__ d,
                                                   const int2* __restrict__ work,
                                                   double* __restrict__ part) {
  __shared__ double red[2][4][R][64];
  __shared__ double xs[R][64];   // x at the block column (zero past n)
  const int2 wk = work[blockIdx.x];
  const SymvDesc g = d[wk.x];
  const int J = wk.y, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c0 = J * 64 + w * 16;
  const double* __restrict__ x = g.X;
  const size_t ldx = g.ldx;
  if (w < R) xs[w][lane] = (J * 64 + lane < g.n) ? x[J * 64 + lane + w * ldx] : 0.0;
  __syncthreads();
  double cs[16][R];
#pragma unroll
  for (int k = 0; k < 16; ++k)
#pragma unroll
    for (int r = 0; r < R; ++r) cs[k][r] = 0.0;
  double* P = part + g.part_off;
  const int tri_n = g.nb * (g.nb + 1) / 2;
  const int kmax = min(16, max(0, g.n - c0));   // valid columns of this wave
  for (int I = J; I < g.nb; ++I) {
    const int row = I * 64 + lane;
    const bool rv = row < g.n;
    double z[16];
    const double* __restrict__ a = g.A + row + (size_t)c0 * g.lda;
#pragma unroll
    for (int k = 0; k < 16; ++k) z[k] = (rv && k < kmax) ? a[(size_t)k * g.lda] : 0.0;
    double rp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) v += z[k] * xs[r][w * 16 + k];
      rp[r] = v;
    }
    if (I > J) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double xr = rv ? x[row + r * ldx] : 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) cs[k][r] += z[k] * xr;
      }
    }
    const int b = I & 1;
#pragma unroll
    for (int r = 0; r < R; ++r) red[b][w][r][lane] = rp[r];
    __syncthreads();
    // one wave adds the four column groups' partial rows of this tile; the
    // buffer is written again two tiles later, after the next barrier
    if (w == (I & 3)) {
      double* t = P + symv_tri(g.nb, J, I) * (3 * 64);
#pragma unroll
      for (int r = 0; r < R; ++r)
        t[r * 64 + lane] =
            (red[b][0][r][lane] + red[b][1][r][lane]) + (red[b][2][r][lane] + red[b][3][r][lane]);
    }
  }
  // column sums of this wave's 16 columns: reduce over the 64 rows
  double* t = P + (int64_t(tri_n) + J) * (3 * 64);
#pragma unroll
  for (int k = 0; k < 16; ++k)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double v = cs[k][r];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == k) t[r * 64 + w * 16 + k] = v;
    }
}

// y_i = alpha (colsum_J(i) + sum_{J <= I} tile (J, I)) + beta y_i, I = i / 64.
template <int R>
__global__ __launch_bounds__(256) void k_symv_sum(const SymvDesc* __restrict__ d, int nd, int rows,
                                                  const double* __restrict__ part, double alpha,
                                                  double beta) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= rows) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].row_start <= gi) lo = mid; else hi = mid - 1;
  }
  const SymvDesc g = d[lo];
  const int i = gi - g.row_start;
  const int I = i >> 6, l = i & 63;
  const double* P = part + g.part_off;
  const int tri_n = g.nb * (g.nb + 1) / 2;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = P[(int64_t(tri_n) + I) * (3 * 64) + r * 64 + l];
    for (int J = 0; J <= I; ++J) v += P[symv_tri(g.nb, J, I) * (3 * 64) + r * 64 + l];
    double* y = g.Y + i + (size_t)r * g.ldy;
    *y = alpha * v + (beta != 0.0 ? beta * (*y) : 0.0);
  }
}

void SymvOp::finalize(hipStream_t st) {
  std::vector<int2> wk;
  int64_t off = 0;
  rows = 0;
  for (size_t q = 0; q < h.size(); ++q) {
    SymvDesc& g = h[q];
    g.nb = ceil_div(g.n, 64);
    g.row_start = rows;
    g.part_off = off;
    rows += g.n;
    off += (int64_t(g.nb) * (g.nb + 1) / 2 + g.nb) * 3 * 64;
    for (int J = 0; J < g.nb; ++J) wk.push_back(make_int2(int(q), J));
  }
  // the longest block columns first, so that the short ones fill the tail
  std::stable_sort(wk.begin(), wk.end(), [&](const int2& a, const int2& b) {
    return h[a.x].nb - a.y > h[b.x].nb - b.y;
  });
  nwork = int(wk.size());
  d.upload(h, st);
  work.upload(wk, st);
  part.alloc(size_t(std::max<int64_t>(off, 1)));
}

void SymvOp::run(double alpha, double beta, int nrhs, hipStream_t st) const {
  if (h.empty()) return;
  if (nrhs < 1 || nrhs > MAX_RHS) throw Error(1, "SymvOp: nrhs must be in 1..3");
  const int nd = int(h.size());
  switch (nrhs) {
#define AMB_CASE(R)                                                                       \
  case R:                                                                                 \
    k_symv_part<R><<<nwork, 256, 0, st>>>(d.p, work.p, part.p);                           \
    AMB_LAUNCH_CHECK();                                                                   \
    k_symv_sum<R><<<ceil_div(rows, 256), 256, 0, st>>>(d.p, nd, rows, part.p, alpha, beta); \
    break;
    AMB_CASE(1) AMB_CASE(2) AMB_CASE(3)
#undef AMB_CASE
  }
  AMB_LAUNCH_CHECK();
}

// --------------------------------------------------------------------------
// FP32 operator copies, stored transposed in row panels: A' = A^T (M x K) is
// cut into panels of PANEL_ROWS rows, each panel stored column by column
// (element (m, k) at (m / 128) * 128 K + 128 k + m % 128; rows past M are
// zero).  A GEMM tile of 128 rows then reads one contiguous block per K
// chunk, and the GEMV reads runs of 512 bytes.
// --------------------------------------------------------------------------

struct PackTDesc {
  const double* src;   // K x M, leading dimension lds
  int64_t lds;
  int K, M;
  float* dst;          // ceil(M / 128) panels of 128 x K
  int tiles_k, tile_start;
};

// One 64 x 64 tile per workgroup, transposed through LDS: reads run along K
// of the source, writes along M of the copy.
__global__ __launch_bounds__(256) void k_pack_t_f32(const PackTDesc* __restrict__ d, int nd) {
  __shared__ float t[64][65];
  const int tile = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_start <= tile) lo = mid; else hi = mid - 1;
  }
  const PackTDesc g = d[lo];
  const int lt = tile - g.tile_start;
  const int k0 = (lt % g.tiles_k) * 64, m0 = (lt / g.tiles_k) * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int kk = e & 63, mm = e >> 6;
    const int k = k0 + kk, m = m0 + mm;
    t[mm][kk] = (k < g.K && m < g.M) ? static_cast<float>(g.src[k + (size_t)m * g.lds]) : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int mm = e & 63, kk = e >> 6;
    const int k = k0 + kk, m = m0 + mm;   // m < ceil(M / 128) * 128 by the tile count
    if (k < g.K) g.dst[panel_index(m, k, g.K)] = t[mm][kk];
  }
}

// Y = alpha A' X + beta Y for 1..3 right-hand sides: a workgroup owns 256
// rows of A' (a float4 of rows per lane); its four waves take every fourth
// column of A' and their partial sums meet in LDS.
constexpr int GN_ROWS = 256;

template <int R>
__global__ __launch_bounds__(256) void k_gemv_n32(const GemvDesc* __restrict__ d, int nd,
                                                  double alpha, double beta) {
  __shared__ double red[3][GN_ROWS * R];
  const int wg = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  const GemvDesc g = d[lo];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lrow = 4 * lane;
  const int row0 = (wg - g.wg_start) * GN_ROWS + lrow;
  // this lane's float4 of rows inside its panel, column 0
  const float* A = static_cast<const float*>(g.A) + panel_index(row0, 0, g.K);
  double acc[4][R];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[u][r] = 0.0;
  if (row0 < g.M) {
#pragma unroll 4
    for (int k = wave; k < g.K; k += 4) {
      const float4 a = *reinterpret_cast<const float4*>(A + (size_t)k * PANEL_ROWS);
      const double a4[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double x = g.X[k + (size_t)r * g.ldx];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u][r] += a4[u] * x;
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) red[wave - 1][(lrow + u) * R + r] = acc[u][r];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = row0 + u;
      if (row >= g.M) break;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = (lrow + u) * R + r;
        const double v = acc[u][r] + red[0][e] + red[1][e] + red[2][e];
        double* y = g.Y + row + (size_t)r * g.ldy;
        *y = alpha * v + (beta != 0.0 ? beta * (*y) : 0.0);
      }
    }
  }
}

void GemvOp::pack_a_f32(DBuf<float>& store, hipStream_t st) {
  if (a32) throw Error(1, "GemvOp::pack_a_f32 called twice");
  if (!by_nrhs.empty()) throw Error(1, "GemvOp::pack_a_f32 after run");
  std::vector<PackTDesc> pd;
  std::vector<int64_t> off;
  int64_t total = 0;
  int tiles = 0;
  for (const auto& g : h) {
    const int panels = ceil_div(g.M, PANEL_ROWS);
    PackTDesc p{static_cast<const double*>(g.A), g.lda, g.K, g.M, nullptr, ceil_div(g.K, 64),
                tiles};
    tiles += p.tiles_k * panels * (PANEL_ROWS / 64);
    off.push_back(total);
    total += int64_t(panels) * PANEL_ROWS * g.K;
    pd.push_back(p);
  }
  store.alloc(size_t(std::max<int64_t>(total, 4)));
  for (size_t i = 0; i < pd.size(); ++i) pd[i].dst = store.p + off[i];
  if (tiles > 0) {
    DBuf<PackTDesc> dd;
    dd.upload(pd, st);
    k_pack_t_f32<<<tiles, 256, 0, st>>>(dd.p, int(pd.size()));
    AMB_LAUNCH_CHECK();
  }
  for (size_t i = 0; i < h.size(); ++i) {
    h[i].A = pd[i].dst;
    h[i].lda = PANEL_ROWS;   // the panel height; element (m, k) at panel_index(m, k, K)
  }
  a32 = true;
}

void GemvOp::finalize(hipStream_t st) {
  int kmax = 0;
  for (const auto& g : h) kmax = std::max(kmax, g.K);
  short_k = !a32 && kmax <= SHORT_K;
  wgs = 0;
  for (auto& g : h) {
    g.wg_start = wgs;
    wgs += a32 ? ceil_div(g.M, GN_ROWS) : short_k ? ceil_div(g.M, 16) : ceil_div(g.M, 4);
  }
  d.upload(h, st);
}

void GemvOp::run(double alpha, double beta, int nrhs, hipStream_t st) const {
  if (h.empty() || wgs == 0) return;
  if (nrhs >= GEMM_FROM && nrhs <= 16) {
    if (by_nrhs.size() < 17) by_nrhs.resize(17);
    if (!by_nrhs[nrhs]) {
      auto g = std::make_unique<GemmOp>();
      g->ta = !a32;   // the FP32 copy is stored transposed
      g->narrow = true;
      g->a32 = a32;
      for (const auto& v : h)
        g->h.push_back(
            GemmDesc{v.A, v.X, v.Y, v.lda, v.ldx, v.ldy, v.M, nrhs, v.K, 0, 0, nullptr, nullptr, 0});
      g->finalize(st);
      by_nrhs[nrhs] = std::move(g);
    }
    by_nrhs[nrhs]->run(alpha, beta, st);
    return;
  }
  const int nd = int(h.size());
  if (a32) {
    switch (nrhs) {
      case 1: k_gemv_n32<1><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
      case 2: k_gemv_n32<2><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
      case 3: k_gemv_n32<3><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
      default: throw Error(1, "GemvOp: nrhs must be in 1..16");
    }
    AMB_LAUNCH_CHECK();
    return;
  }
  if (short_k) {
    switch (nrhs) {
      case 1: k_gemv_t16<1><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
      case 2: k_gemv_t16<2><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
      case 3: k_gemv_t16<3><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
      default: throw Error(1, "GemvOp: nrhs must be in 1..16");
    }
    AMB_LAUNCH_CHECK();
    return;
  }
  switch (nrhs) {
#define AMB_CASE(R) case R: k_gemv_t<R><<<wgs, 256, 0, st>>>(d.p, nd, alpha, beta); break;
    AMB_CASE(1) AMB_CASE(2) AMB_CASE(3) AMB_CASE(4) AMB_CASE(5) AMB_CASE(6) AMB_CASE(7)
    AMB_CASE(8) AMB_CASE(9) AMB_CASE(10) AMB_CASE(11) AMB_CASE(12) AMB_CASE(13) AMB_CASE(14)
    AMB_CASE(15) AMB_CASE(16)
#undef AMB_CASE
    default: throw Error(1, "GemvOp: nrhs must be in 1..16");
  }
  AMB_LAUNCH_CHECK();
}

// --------------------------------------------------------------------------
// Signed partial LDL^T, right-looking, panel width NB
// --------------------------------------------------------------------------

__device__ __forceinline__ int find_active(const int* pre, int n, int x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Factor the NB x NB diagonal block of every active matrix in place.
__global__ __launch_bounds__(256) void k_ldlt_diag(const LdltDesc* __restrict__ d,
                                                   const int* __restrict__ act, int k0, int* info) {
  constexpr int NB = LdltOp::NB;
  __shared__ double L[NB][NB + 1];
  const LdltDesc g = d[act[blockIdx.x]];
  const int kb = min(NB, g.p - k0);
  const int tid = threadIdx.x;
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i % NB, c = i / NB;
    L[r][c] = (r < kb && c < kb) ? g.A[(k0 + r) + (size_t)(k0 + c) * g.lda] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    const double sg = (k0 + j < g.q) ? 1.0 : -1.0;
    const double dj = L[j][j] * sg;
    const bool bad = !(dj > 0.0);
    const double piv = bad ? 1.0 : sqrt(dj);
    __syncthreads();
    if (tid == 0) {
      if (bad) atomicCAS(info, 0, act[blockIdx.x] + 1);
      L[j][j] = piv;
    }
    for (int i = j + 1 + tid; i < kb; i += 256) L[i][j] /= (sg * piv);
    __syncthreads();
    const int rem = kb - j - 1;
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int i = j + 1 + idx % rem, l = j + 1 + idx / rem;
      if (l <= i) L[i][l] -= sg * L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  for (int i = tid; i < kb * kb; i += 256) {
    const int r = i % kb, c = i / kb;
    if (r >= c) g.A[(k0 + r) + (size_t)(k0 + c) * g.lda] = L[r][c];
  }
}

// Panel: rows below the diagonal block, L_i = A_i (L_kk D)^{-T}.
__global__ __launch_bounds__(256) void k_ldlt_panel(const LdltDesc* __restrict__ d,
                                                    const int* __restrict__ act,
                                                    const int* __restrict__ pre, int nact, int k0) {
  constexpr int NB = LdltOp::NB;
  __shared__ double L[NB][NB + 1];
  const int a = find_active(pre, nact, blockIdx.x);
  const LdltDesc g = d[act[a]];
  const int chunk = blockIdx.x - pre[a];
  const int kb = min(NB, g.p - k0);
  const int tid = threadIdx.x;
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i % NB, c = i / NB;
    L[r][c] = (r < kb && c < kb && r >= c) ? g.A[(k0 + r) + (size_t)(k0 + c) * g.lda] : 0.0;
  }
  __syncthreads();
  const int row = k0 + kb + chunk * LdltOp::ROWS + tid;
  if (row >= g.N) return;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = (j < kb) ? g.A[row + (size_t)(k0 + j) * g.lda] : 0.0;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < kb) {
      double v = x[j];
#pragma unroll
      for (int p = 0; p < j; ++p) {
        const double sp = (k0 + p < g.q) ? 1.0 : -1.0;
        v -= x[p] * sp * L[j][p];
      }
      const double sj = (k0 + j < g.q) ? 1.0 : -1.0;
      x[j] = v / (sj * L[j][j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (j < kb) g.A[row + (size_t)(k0 + j) * g.lda] = x[j];
}

// Update of the rest of the outer block after the inner step at k0:
// A[r, c] -= sum_p L[r, p] sigma_p L[c, p] (p = panel columns k0..k0+kb) for
// columns c in [k0+kb, c1), c1 = end of the outer block, rows r >= c.
__global__ __launch_bounds__(256) void k_ldlt_strip(const LdltDesc* __restrict__ d,
                                                    const int* __restrict__ act,
                                                    const int* __restrict__ pre, int nact, int k0,
                                                    int outer) {
  __shared__ TileSmem<2, 2> sm;
  const int a = find_active(pre, nact, blockIdx.x);
  const LdltDesc g = d[act[a]];
  int l = blockIdx.x - pre[a];
  const int kb = min(LdltOp::NB, g.p - k0);
  const int r0 = k0 + kb;
  const int c1 = min(outer + LdltOp::OB, g.p);
  const int nrt = (g.N - r0 + LdltOp::TILE - 1) / LdltOp::TILE;
  int tc = 0;
  while (l >= nrt - tc) { l -= nrt - tc; ++tc; }
  const int tr = tc + l;
  const double* P = g.A + (size_t)k0 * g.lda;
  mfma_tile<false, true, 2, 2>(P, g.lda, P, g.lda, g.A, g.lda, g.N, c1, kb, r0 + tr * LdltOp::TILE,
                               r0 + tc * LdltOp::TILE, -1.0, 1.0, max(g.q - k0, 0), sm);
}

// Trailing update after the outer block starting at `outer`: lower tiles of
// A[c1:, c1:] -= L D L^T over the block's columns outer..c1.  Panel column p
// is a negative pivot when outer + p >= q (clamped: all negative when q <= outer).
__global__ __launch_bounds__(256) void k_ldlt_update(const LdltDesc* __restrict__ d,
                                                     const int* __restrict__ act,
                                                     const int* __restrict__ pre, int nact,
                                                     int outer) {
  __shared__ TileSmem<2, 2> sm;
  const int a = find_active(pre, nact, blockIdx.x);
  const LdltDesc g = d[act[a]];
  const int l = blockIdx.x - pre[a];
  int ti2 = int((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
  while ((ti2 + 1) * (ti2 + 2) / 2 <= l) ++ti2;
  while (ti2 * (ti2 + 1) / 2 > l) --ti2;
  const int tj = l - ti2 * (ti2 + 1) / 2;
  const int c1 = min(outer + LdltOp::OB, g.p);
  const int m0 = c1 + ti2 * LdltOp::TILE, n0 = c1 + tj * LdltOp::TILE;
  const double* P = g.A + (size_t)outer * g.lda;
  mfma_tile<false, true, 2, 2>(P, g.lda, P, g.lda, g.A, g.lda, g.N, g.N, c1 - outer, m0, n0, -1.0,
                               1.0, max(g.q - outer, 0), sm);
}

void LdltOp::finalize(hipStream_t st) {
  int maxp = 0;
  for (auto& g : h) maxp = std::max(maxp, g.p);
  ph.clear();
  std::vector<int> a, pp_all, up_all;
  for (int outer = 0; outer < maxp; outer += OB) {
    for (int k0 = outer; k0 < std::min(outer + OB, maxp); k0 += NB) {
      Phase f{0, k0, outer, int(a.size()), 0, 0, 0};
      for (size_t i = 0; i < h.size(); ++i) {
        const auto& g = h[i];
        if (g.p <= k0) continue;
        const int kb = std::min(NB, g.p - k0);
        const int rows = g.N - k0 - kb;
        const int c1 = std::min(outer + OB, g.p);
        const int w = c1 - (k0 + kb);
        a.push_back(int(i));
        pp_all.push_back(f.pan_total);
        up_all.push_back(f.upd_total);
        f.pan_total += rows > 0 ? ceil_div(rows, ROWS) : 0;
        if (w > 0 && rows > 0) {
          const int nct = ceil_div(w, TILE), nrt = ceil_div(rows, TILE);
          f.upd_total += nct * nrt - nct * (nct - 1) / 2;
        }
        ++f.nact;
      }
      ph.push_back(f);
    }
    Phase f{1, outer, outer, int(a.size()), 0, 0, 0};
    for (size_t i = 0; i < h.size(); ++i) {
      const auto& g = h[i];
      if (g.p <= outer) continue;
      const int c1 = std::min(outer + OB, g.p);
      const int rows = g.N - c1;
      if (rows <= 0) continue;
      a.push_back(int(i));
      pp_all.push_back(0);
      up_all.push_back(f.upd_total);
      const int nt = ceil_div(rows, TILE);
      f.upd_total += nt * (nt + 1) / 2;
      ++f.nact;
    }
    ph.push_back(f);
  }
  d.upload(h, st);
  act.upload(a, st);
  pan_pre.upload(pp_all, st);
  upd_pre.upload(up_all, st);
  info.alloc(1);
}

void LdltOp::run(hipStream_t st) {
  if (h.empty()) return;
  info.zero(st);
  for (const Phase& f : ph) {
    if (f.nact == 0) continue;
    if (!f.big) {
      k_ldlt_diag<<<f.nact, 256, 0, st>>>(d.p, act.p + f.off, f.k0, info.p);
      if (f.pan_total > 0)
        k_ldlt_panel<<<f.pan_total, 256, 0, st>>>(d.p, act.p + f.off, pan_pre.p + f.off, f.nact,
                                                  f.k0);
      if (f.upd_total > 0)
        k_ldlt_strip<<<f.upd_total, 256, 0, st>>>(d.p, act.p + f.off, upd_pre.p + f.off, f.nact,
                                                  f.k0, f.outer);
    } else if (f.upd_total > 0) {
      k_ldlt_update<<<f.upd_total, 256, 0, st>>>(d.p, act.p + f.off, upd_pre.p + f.off, f.nact,
                                                 f.outer);
    }
  }
  AMB_LAUNCH_CHECK();
}

int LdltOp::failed(hipStream_t st) {
  int v = 0;
  AMB_HIP(hipMemcpyAsync(&v, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  AMB_HIP(hipStreamSynchronize(st));
  return v - 1;
}

// --------------------------------------------------------------------------
// Right-side triangular solve X L = B (TrsmOp)
// --------------------------------------------------------------------------

// Record lookup of a launch: the last record whose first workgroup is at or
// before this one.
__device__ __forceinline__ int find_rec(const TrsmOp::Rec* __restrict__ r, int n, int wg) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (r[mid].start <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// B[:, c0:c0+w] -= X[:, kb:ke] L[kb:ke, c0:c0+w] (X = the solved columns of
// B), one 64 x 64 MFMA tile per workgroup.
__global__ __launch_bounds__(256) void k_trsm_update(const TrsmDesc* __restrict__ d,
                                                     const TrsmOp::Rec* __restrict__ recs, int n) {
  __shared__ TileSmem<2, 2> sm;
  const TrsmOp::Rec r = recs[find_rec(recs, n, blockIdx.x)];
  const TrsmDesc g = d[r.m];
  const int l = blockIdx.x - r.start;
  const int tiles_m = (g.nG + 63) / 64;
  const int tm = l % tiles_m, tn = l / tiles_m;
  const int c = r.c0 + tn * 64, w = min(64, r.c0 + r.w - c);
  double* B = g.A + g.nI;                       // rows nI.., column 0
  mfma_tile<false, false, 2, 2>(B + (size_t)r.kb * g.lda, g.lda, g.A + r.kb + (size_t)c * g.lda,
                                g.lda, B + (size_t)c * g.lda, g.lda, g.nG, w, r.ke - r.kb, tm * 64,
                                0, -1.0, 1.0, -1, sm);
}

// Every row x of B[:, c0:c0+w] (w <= TB) solves x L[c0:c0+w, c0:c0+w] = b
// (back substitution over the block's columns); L's block and the
// reciprocals of its diagonal in LDS, the row in registers.
__global__ __launch_bounds__(256) void k_trsm_solve(const TrsmDesc* __restrict__ d,
                                                    const TrsmOp::Rec* __restrict__ recs, int n) {
  constexpr int TB = TrsmOp::TB;
  __shared__ double Ld[TB][TB + 1];
  __shared__ double dinv[TB];
  const TrsmOp::Rec rc = recs[find_rec(recs, n, blockIdx.x)];
  const TrsmDesc g = d[rc.m];
  const int chunk = blockIdx.x - rc.start;
  const int c0 = rc.c0, w = rc.w;
  for (int i = threadIdx.x; i < TB * TB; i += 256) {
    const int r = i % TB, c = i / TB;
    Ld[r][c] = (r < w && c < w && r >= c) ? g.A[(c0 + r) + (size_t)(c0 + c) * g.lda] : 0.0;
  }
  if (threadIdx.x < TB)
    dinv[threadIdx.x] =
        threadIdx.x < w ? 1.0 / g.A[(c0 + threadIdx.x) + (size_t)(c0 + threadIdx.x) * g.lda] : 0.0;
  __syncthreads();
  const int row = chunk * 256 + threadIdx.x;
  if (row >= g.nG) return;
  double* b = g.A + g.nI + row + (size_t)c0 * g.lda;
  double x[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) x[j] = j < w ? b[(size_t)j * g.lda] : 0.0;
#pragma unroll
  for (int k = TB - 1; k >= 0; --k) {
    if (k < w) {
      double v = x[k];
#pragma unroll
      for (int i = k + 1; i < TB; ++i) v -= x[i] * Ld[i][k];
      x[k] = v * dinv[k];
    }
  }
#pragma unroll
  for (int j = 0; j < TB; ++j)
    if (j < w) b[(size_t)j * g.lda] = x[j];
}

// Columns are taken from the right in groups of GB blocks of TB: the group
// first takes all solved columns to its right in one wide update, then its
// blocks, right to left, take the solved blocks of the group (a narrow
// update) and are solved.  Matrices run in lockstep by group and sub-step.
void TrsmOp::finalize(hipStream_t st) {
  launches.clear();
  std::vector<Rec> all;
  int maxg = 0;
  for (const auto& g : h) maxg = std::max(maxg, ceil_div(ceil_div(g.nI, TB), GB));
  auto open = [&](bool solve) {
    launches.push_back(Launch{solve, int(all.size()), 0, 0});
  };
  auto push = [&](int m, int c0, int w, int kb, int ke, bool solve) {
    Launch& L = launches.back();
    const auto& g = h[m];
    const int wgs = solve ? ceil_div(g.nG, 256) : ceil_div(g.nG, 64) * ceil_div(w, 64);
    all.push_back(Rec{m, c0, w, kb, ke, L.wgs});
    L.wgs += wgs;
    ++L.n;
  };
  for (int og = 0; og < maxg; ++og) {
    // wide update of the group with everything solved to its right
    open(false);
    for (size_t m = 0; m < h.size(); ++m) {
      const auto& g = h[m];
      const int nb = ceil_div(g.nI, TB), ng = ceil_div(nb, GB);
      if (og >= ng) continue;
      const int jhi = nb - 1 - og * GB, jlo = std::max(0, jhi - GB + 1);
      const int c0 = jlo * TB, c1 = std::min(g.nI, (jhi + 1) * TB);
      if (c1 < g.nI) push(int(m), c0, c1 - c0, c1, g.nI, false);
    }
    for (int i = 0; i < GB; ++i) {
      // block jhi - i: narrow update with the group's solved blocks, solve
      open(false);
      for (size_t m = 0; m < h.size(); ++m) {
        const auto& g = h[m];
        const int nb = ceil_div(g.nI, TB), ng = ceil_div(nb, GB);
        if (og >= ng) continue;
        const int jhi = nb - 1 - og * GB, j = jhi - i;
        if (j < 0 || i == 0) continue;
        const int c0 = j * TB, c1 = std::min(g.nI, (jhi + 1) * TB);
        push(int(m), c0, TB, c0 + TB, c1, false);
      }
      open(true);
      for (size_t m = 0; m < h.size(); ++m) {
        const auto& g = h[m];
        const int nb = ceil_div(g.nI, TB), ng = ceil_div(nb, GB);
        if (og >= ng) continue;
        const int j = nb - 1 - og * GB - i;
        if (j < 0) continue;
        push(int(m), j * TB, std::min(TB, g.nI - j * TB), 0, 0, true);
      }
    }
  }
  // drop empty launches
  std::vector<Launch> keep;
  for (const auto& L : launches)
    if (L.n > 0) keep.push_back(L);
  launches.swap(keep);
  d.upload(h, st);
  recs.upload(all, st);
}

void TrsmOp::run(hipStream_t st) const {
  for (const Launch& L : launches) {
    if (L.solve)
      k_trsm_solve<<<L.wgs, 256, 0, st>>>(d.p, recs.p + L.off, L.n);
    else
      k_trsm_update<<<L.wgs, 256, 0, st>>>(d.p, recs.p + L.off, L.n);
  }
  AMB_LAUNCH_CHECK();
}

// --------------------------------------------------------------------------
// x <- K_II^{-1} x with the partial Cholesky factor (forward, then backward)
// --------------------------------------------------------------------------

constexpr int TRSV_THREADS = 1024;

// v of lane l (l uniform across the wave).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), l));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Diagonal block ob of TrsvOp::OB rows (counted from the top in the forward
// pass, from the bottom in the backward pass) of every matrix, one workgroup
// per matrix, all R right-hand sides together; the rows outside the block
// already hold the contributions of the blocks solved before (k_trsv_panel).
// Inner block q of 64 rows: the 16 waves take every 16th solved column of the
// outer block (lanes = the inner block's rows, eight columns in flight per
// wave) and meet in LDS; wave 0 then solves the 64 x 64 diagonal block, one
// lane per row.
template <int R>
__global__ __launch_bounds__(TRSV_THREADS) void k_trsv_chol(const TrsvDesc* __restrict__ d,
                                                            int pass, int ob) {
  constexpr int B = 64, NW = TRSV_THREADS / 64, U = 8, OB = TrsvOp::OB;
  __shared__ double Ld[B][B + 1];
  __shared__ double part[2][NW][B];   // one right-hand side at a time, double buffered
  __shared__ double zb[R][B];
  const TrsvDesc g = d[blockIdx.x];
  double* x = g.x;
  const int64_t ldx = g.ldx;
  const int n = g.nI, lda = g.lda;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nob = (n + OB - 1) / OB;
  if (ob >= nob) return;
  const int bo = pass == 0 ? ob : nob - 1 - ob;
  const int o0 = bo * OB, o1 = min(n, o0 + OB);
  const int qb = o0 / B, nq = (o1 - o0 + B - 1) / B;
  {
    for (int qq = 0; qq < nq; ++qq) {
      // forward: inner block qq from the top, L[r0.., c] for the solved
      // o0 <= c < r0; backward: from the bottom, L^T[r0.., c] = L[c, r0..]
      // (the upper triangle holds L^T) for the solved r0 + w <= c < o1
      const int jb = qb + (pass == 0 ? qq : nq - 1 - qq);
      const int r0 = jb * B, w = min(B, n - r0);
      const int ca = pass == 0 ? o0 : r0 + w, cb = pass == 0 ? r0 : o1;
      double acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = 0.0;
      const double* arow = g.A + r0 + min(lane, w - 1);
      int c = ca + wave;
      for (; c + (U - 1) * NW < cb; c += U * NW) {
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = arow[(size_t)(c + u * NW) * lda];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double* xr = x + (size_t)r * ldx + c;
          double t = 0.0;
#pragma unroll
          for (int u = 0; u < U; ++u) t += a[u] * xr[u * NW];
          acc[r] += t;
        }
      }
      for (; c < cb; c += NW) {
        const double a = arow[(size_t)c * lda];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += a * x[(size_t)r * ldx + c];
      }
      for (int i = threadIdx.x; i < B * B; i += TRSV_THREADS) {
        const int rr = i % B, cc = i / B;
        Ld[rr][cc] = (rr < w && cc < w && rr >= cc) ? g.A[(r0 + rr) + (size_t)(r0 + cc) * lda] : 0.0;
      }
      // the waves' partial sums, one right-hand side per round: wave r % NW
      // adds them up (in wave order) while the others write the next round
#pragma unroll
      for (int r = 0; r < R; ++r) {
        part[r & 1][wave][lane] = acc[r];
        __syncthreads();
        if (wave == r % NW) {
          double t = 0.0;
          for (int k = 0; k < NW; ++k) t += part[r & 1][k][lane];
          zb[r][lane] = t;
        }
      }
      __syncthreads();
      // diagonal block: L y = z (forward) or L^T y = z (backward); waves
      // 0..R-1 take one right-hand side each, one lane per row
      // (each lane holds the reciprocal of its diagonal entry; the solved
      // value of row k is read from lane k by v_readlane)
      if (wave < R) {
        const int r = wave;
        double z = 0.0;
        const double dinv = lane < w ? 1.0 / Ld[lane][lane] : 0.0;
        if (lane < w) z = x[(size_t)r * ldx + r0 + lane] - zb[r][lane];
        // the next step's entry of L is loaded one step ahead
        if (pass == 0) {
          double ln = Ld[lane][0];
          for (int k = 0; k < w; ++k) {
            const double lk = ln;
            if (k + 1 < w) ln = Ld[lane][k + 1];
            const double yk = readlane_f64(z * dinv, k);
            if (lane > k && lane < w) z -= lk * yk;
            if (lane == k) z = yk;
          }
        } else {
          double ln = Ld[w - 1][lane];
          for (int k = w - 1; k >= 0; --k) {
            const double lk = ln;
            if (k > 0) ln = Ld[k - 1][lane];
            const double yk = readlane_f64(z * dinv, k);
            if (lane < k) z -= lk * yk;
            if (lane == k) z = yk;
          }
        }
        if (lane < w) x[(size_t)r * ldx + r0 + lane] = z;
      }
      __syncthreads();
    }
  }
}

// After diagonal block ob: the rows below it (forward, L) or above it
// (backward, L^T from the upper triangle) subtract the block's columns times
// its solved values.  One thread per row and right-hand sides, PANEL_ROWS
// rows per workgroup (pre: first workgroup of every matrix); lanes read
// consecutive rows of one column.
template <int R>
__global__ __launch_bounds__(256) void k_trsv_panel(const TrsvDesc* __restrict__ d,
                                                    const int* __restrict__ pre, int nd, int pass,
                                                    int ob) {
  constexpr int OB = TrsvOp::OB, U = 8;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= int(blockIdx.x)) lo = mid; else hi = mid - 1;
  }
  const TrsvDesc g = d[lo];
  const int n = g.nI;
  const int nob = (n + OB - 1) / OB;
  if (ob >= nob) return;
  const int bo = pass == 0 ? ob : nob - 1 - ob;
  const int o0 = bo * OB, o1 = min(n, o0 + OB);
  const int ra = pass == 0 ? o1 : 0, rb = pass == 0 ? n : o0;
  const int r = ra + (int(blockIdx.x) - pre[lo]) * 256 + int(threadIdx.x);
  if (r >= rb) return;
  double* x = g.x;
  const int64_t ldx = g.ldx;
  const double* __restrict__ a = g.A + r;
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  int c = o0;
  for (; c + U <= o1; c += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = a[(size_t)(c + u) * g.lda];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double t = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) t += v[u] * x[c + u + q * ldx];
      acc[q] += t;
    }
  }
  for (; c < o1; ++c) {
    const double v = a[(size_t)c * g.lda];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] += v * x[c + q * ldx];
  }
#pragma unroll
  for (int q = 0; q < R; ++q) x[r + q * ldx] -= acc[q];
}

void TrsvOp::finalize(hipStream_t st) {
  std::vector<int> p;
  nob = 0;
  pwgs = 0;
  for (const auto& g : h) {
    p.push_back(pwgs);
    pwgs += ceil_div(g.nI, 256);
    nob = std::max(nob, ceil_div(g.nI, OB));
  }
  d.upload(h, st);
  pre.upload(p, st);
}

template <int R>
static void trsv_run(const TrsvOp& op, const TrsvDesc* d, const int* pre, int nd, int nob,
                     int pwgs, hipStream_t st) {
  for (int pass = 0; pass < 2; ++pass)
    for (int ob = 0; ob < nob; ++ob) {
      k_trsv_chol<R><<<nd, TRSV_THREADS, 0, st>>>(d, pass, ob);
      if (ob + 1 < nob) k_trsv_panel<R><<<pwgs, 256, 0, st>>>(d, pre, nd, pass, ob);
    }
  (void)op;
}

void TrsvOp::run(int nrhs, hipStream_t st) const {
  if (h.empty() || nrhs == 0) return;
  const int nd = int(h.size());
  switch (nrhs) {
#define AMB_CASE(R) case R: trsv_run<R>(*this, d.p, pre.p, nd, nob, pwgs, st); break;
    AMB_CASE(1) AMB_CASE(2) AMB_CASE(3) AMB_CASE(4) AMB_CASE(5) AMB_CASE(6) AMB_CASE(7)
    AMB_CASE(8) AMB_CASE(9) AMB_CASE(10) AMB_CASE(11) AMB_CASE(12) AMB_CASE(13) AMB_CASE(14)
    AMB_CASE(15) AMB_CASE(16)
#undef AMB_CASE
    default: throw Error(1, "trsv: nrhs must be in 1..16");
  }
  AMB_LAUNCH_CHECK();
}

// --------------------------------------------------------------------------
// lower -> upper copy on a square block [n0, n0+n)^2
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_sym(const SymOp::Desc* __restrict__ d, int nd) {
  const int blk = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].start <= blk) lo = mid; else hi = mid - 1;
  }
  const SymOp::Desc g = d[lo];
  const int nt = ceil_div_dev(g.n, 32);
  const int l = blk - g.start;
  const int bi = l % nt, bj = l / nt;   // tile (bi, bj) of the upper triangle, bi <= bj
  if (bi > bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    const int r = bi * 32 + tx, c = bj * 32 + yy;   // upper entry (r < c)
    if (r < g.n && c < g.n && r < c)
      g.A[(g.n0 + r) + (size_t)(g.n0 + c) * g.lda] = g.A[(g.n0 + c) + (size_t)(g.n0 + r) * g.lda];
  }
}

void SymOp::finalize(hipStream_t st) {
  tiles = 0;
  for (auto& g : h) {
    g.start = tiles;
    const int nt = ceil_div(g.n, 32);
    tiles += nt * nt;
  }
  d.upload(h, st);
}

void SymOp::run(hipStream_t st) const {
  if (h.empty() || tiles == 0) return;
  k_sym<<<tiles, 256, 0, st>>>(d.p, int(h.size()));
  AMB_LAUNCH_CHECK();
}

}  // namespace ambddc
