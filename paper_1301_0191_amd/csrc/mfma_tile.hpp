// One workgroup tile of C = alpha * op(A) * diag(sigma) * op(B) + beta * C on
// CDNA MFMA (v_mfma_f64_16x16x4f64), FP64.  64 WM WN threads = WM x WN waves;
// every wave owns a 32x32 sub-tile (2x2 MFMA blocks).  K is staged
// through LDS in chunks of KC so that global reads are coalesced for either
// operand orientation; the staging is double-buffered: the next chunk is
// loaded into registers while the current one feeds the MFMAs, then stored
// to the other LDS buffer, with one barrier per chunk.
//
// MFMA 16x16x4 operand layout (per wave of 64 lanes):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, element r holds D[4 * r + l / 16][l % 16]   (FP64 variant)
#pragma once
#include <hip/hip_runtime.h>

namespace ambddc {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// FP32 operands are stored in row panels: element (m, k) of an M x K matrix
// at (m / PANEL_ROWS) * PANEL_ROWS * K + PANEL_ROWS * k + m % PANEL_ROWS.
constexpr int PANEL_ROWS = 128;
__host__ __device__ __forceinline__ size_t panel_index(int m, int k, int K) {
  return (size_t)(m / PANEL_ROWS) * PANEL_ROWS * K + (size_t)k * PANEL_ROWS + (m % PANEL_ROWS);
}

// Loads through global-address-space pointers: the compiler then emits
// global loads, which only count in vmcnt, so waiting for LDS reads does not
// also wait for the next chunk's loads still in flight (flat loads count in
// both counters).
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  typedef const __attribute__((address_space(1))) T* gptr;
  return *(gptr)p;
}

template <int WM, int WN>
struct TileShape {
  static constexpr int TM = 32 * WM;
  static constexpr int TN = 32 * WN;
  static constexpr int KC = 16;
  static constexpr int PAD = 4;
};

template <int WM, int WN>
struct TileSmem {
  double As[2][TileShape<WM, WN>::KC][TileShape<WM, WN>::TM + TileShape<WM, WN>::PAD];
  double Bs[2][TileShape<WM, WN>::KC][TileShape<WM, WN>::TN + TileShape<WM, WN>::PAD];
};

// op(A)(m, k) = TA ? A[k + m*lda] : A[m + k*lda]
// op(B)(k, n) = TB ? B[n + k*ldb] : B[k + n*ldb]
// sign_split >= 0: column k of op(A) is scaled by +1 if k < sign_split, else -1.
// TAe is the element type of A in memory: double, or float widened on load.
// A float A is not transposed (TA false) and stored in row panels
// (panel_index); lda is then unused.
template <bool TA, bool TB, int WM, int WN, typename TAe>
__device__ __forceinline__ void mfma_tile(const TAe* __restrict__ A, int lda,
                                          const double* __restrict__ B, int ldb, double* C, int ldc,
                                          int M, int N, int K, int m0, int n0, double alpha,
                                          double beta, int sign_split, TileSmem<WM, WN>& sm) {
  using S = TileShape<WM, WN>;
  constexpr int TM = S::TM, TN = S::TN, KC = S::KC;
  constexpr int NT = 64 * WM * WN;                       // threads: one wave per 32 x 32
  constexpr int NA = KC * TM / NT, NB = KC * TN / NT;   // staged values per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  TAe ra[NA];      // raw A values: converted and sign-flipped when stored to LDS
  double rb[NB];
  // global -> registers for the chunk starting at k0
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + u * NT;
      int m, k;
      if (!TA) { m = idx % TM; k = idx / TM; }
      else { k = idx % KC; m = idx / KC; }
      const int gm = m0 + m, gk = k0 + k;
      TAe v = TAe(0);
      if (gm < M && gk < K) {
        if constexpr (sizeof(TAe) == 4)
          v = gld(A + panel_index(gm, gk, K));
        else
          v = gld(TA ? A + gk + (size_t)gm * lda : A + gm + (size_t)gk * lda);
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + u * NT;
      int n, k;
      if (TB) { n = idx % TN; k = idx / TN; }
      else { k = idx % KC; n = idx / KC; }
      const int gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < N && gk < K) v = gld(TB ? B + gn + (size_t)gk * ldb : B + gk + (size_t)gn * ldb);
      rb[u] = v;
    }
  };
  // registers (chunk starting at k0) -> LDS buffer
  auto sstore = [&](int buf, int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + u * NT;
      int m, k;
      if (!TA) { m = idx % TM; k = idx / TM; }
      else { k = idx % KC; m = idx / KC; }
      double v = static_cast<double>(ra[u]);
      if (sign_split >= 0 && k0 + k >= sign_split) v = -v;
      sm.As[buf][k][m] = v;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + u * NT;
      int n, k;
      if (TB) { n = idx % TN; k = idx / TN; }
      else { k = idx % KC; n = idx / KC; }
      sm.Bs[buf][k][n] = rb[u];
    }
  };
  if (K > 0) {
    gload(0);
    sstore(0, 0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += KC) {
    const bool more = k0 + KC < K;
    if (more) gload(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sm.As[buf][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sm.Bs[buf][kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1, k0 + KC);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 32 + i * 16 + 4 * r + (lane >> 4);
        const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          double* c = C + gm + (size_t)gn * ldc;
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * (*c);
          *c = v;
        }
      }
}

}  // namespace ambddc

namespace ambddc {

// ---------------------------------------------------------------------------
// FP32 variant: C = alpha * A * B + beta * C with A FP32 (column-major, lda),
// B FP32, or FP64 rounded to FP32 as it is staged, products and sums on
// v_mfma_f32_16x16x4f32 (FP32 accumulation), C FP64.  Same tiling as the
// FP64 tile: 4 waves of 32 x 32 (2 x 2 MFMA blocks of 16 x 16), K staged
// through LDS in chunks of KC32, double buffered, one barrier per chunk.
// MFMA 16x16x4 f32 operands: A lane l holds A[l % 16][l / 16], B lane l
// holds B[l / 16][l % 16]; D lane l, element r holds D[4 (l / 16) + r][l % 16].
// ---------------------------------------------------------------------------
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int KC32 = 32;

template <int WM, int WN>
struct TileSmem32 {
  float As[2][KC32][32 * WM + 4];
  float Bs[2][KC32][32 * WN + 4];
};

template <int WM, int WN, typename TBe>
__device__ __forceinline__ void mfma_tile_f32(const float* __restrict__ A, int lda,
                                              const TBe* __restrict__ B, int ldb, double* C,
                                              int ldc, int M, int N, int K, int m0, int n0,
                                              double alpha, double beta, TileSmem32<WM, WN>& sm) {
  constexpr int TM = 32 * WM, TN = 32 * WN, KC = KC32;
  constexpr int NA = KC * TM / 256, NB = KC * TN / 256;   // staged values per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  flt4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  float ra[NA];
  TBe rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + u * 256;
      const int m = idx % TM, k = idx / TM;
      const int gm = m0 + m, gk = k0 + k;
      ra[u] = (gm < M && gk < K) ? gld(A + gm + (size_t)gk * lda) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + u * 256;
      const int k = idx % KC, n = idx / KC;
      const int gn = n0 + n, gk = k0 + k;
      rb[u] = (gn < N && gk < K) ? gld(B + gk + (size_t)gn * ldb) : TBe(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int idx = tid + u * 256;
      sm.As[buf][idx / TM][idx % TM] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = tid + u * 256;
      sm.Bs[buf][idx % KC][idx / KC] = static_cast<float>(rb[u]);
    }
  };
  if (K > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += KC) {
    const bool more = k0 + KC < K;
    if (more) gload(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kr = kk + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sm.As[buf][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sm.Bs[buf][kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          double* c = C + gm + (size_t)gn * ldc;
          double v = alpha * static_cast<double>(acc[i][j][r]);
          if (beta != 0.0) v += beta * (*c);
          *c = v;
        }
      }
}

}  // namespace ambddc
