// Batched dense linear algebra on uneven batches (FP64), gfx950.
//   GemmOp : C_b = alpha op(A_b) op(B_b) + beta C_b on MFMA 16x16x4 tiles
//   GemvOp : Y_b = alpha A_b^T X_b + beta Y_b for a few right-hand sides
//   LdltOp : signed partial LDL^T (Cholesky with fixed pivot signs), the
//            trailing block becomes the Schur complement
//   SymOp  : copy the lower triangle of a square block to the upper one
// GemvOp can keep its operators as FP32 copies (pack_a_f32): they are
// rounded once and widened to FP64 as they are loaded, so the products still
// accumulate in FP64 while the HBM traffic for the operators halves.
#pragma once
#include <memory>

#include "common.hpp"

namespace ambddc {

struct GemmDesc {
  const void* A;    // const double*, or const float* when the op's a32 is set
  const double* B;
  double* C;
  int lda, ldb, ldc;
  int M, N, K;
  int tiles_m, tile_start;
  const int* flag;  // optional: skip the product when *flag == 0
  // optional column slots: columns [j scols, (j+1) scols) belong to item
  // spair[j]; a tile whose slots all have act[item] == 0 (GemmOp::act) is
  // skipped
  const int* spair;
  int scols;
};

// Reduction of split-K partial products: C = alpha sum_s P_s + beta C.
struct SplitDesc {
  double* C;
  int ldc, M, N;
  const int* flag;
  int64_t poff;     // first partial block (M x N, ld M) in GemmOp::part
  int S;            // number of partial blocks
};

class GemmOp {
 public:
  bool ta = false, tb = false, narrow = false;  // narrow: 128x32 tiles (N <= 32)
  bool a32 = false;                             // A operands are FP32 (GemvOp copies)
  // f32: A operands are plain column-major FP32 (lda), B is rounded to FP32
  // as it is staged, and the products accumulate in FP32 on FP32 MFMA; C
  // stays FP64.  Not transposed, no split-K.
  bool f32 = false;
  bool b32 = false;                             // with f32: B operands are FP32 as well
  const int* act = nullptr;                     // item flags for column-slot skipping
  int act_mask = ~0;                            // a slot counts when (act[item] & act_mask) != 0
  int act_excl = 0;                             // ... and a tile is skipped when any of its
                                                // slots has (act[item] & act_excl) != 0
  // Split-K: 0 = chosen at finalize (products with few tiles and long K are
  // split so that the launch has about SPLIT_TARGET workgroups), 1 = never.
  // Each product's K range is cut into S pieces whose partial products go to
  // `part`; a second kernel sums them in a fixed order (deterministic).
  static constexpr int SPLIT_TARGET = 4096;
  int ksplit = 1;
  std::vector<GemmDesc> h;
  DBuf<GemmDesc> d;
  int tiles = 0;
  std::vector<SplitDesc> hs;
  DBuf<SplitDesc> ds;
  DBuf<double> part;
  void add(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int M, int N,
           int K, const int* flag = nullptr, const int* spair = nullptr, int scols = 0) {
    if (M <= 0 || N <= 0) return;
    h.push_back(GemmDesc{A, B, C, lda, ldb, ldc, M, N, K, 0, 0, flag, spair, scols});
  }
  void finalize(hipStream_t st);
  void run(double alpha, double beta, hipStream_t st) const;
  bool empty() const { return h.empty(); }
};

// One batched product in two tile shapes, 64 x 64 (v[0]) and 128 x 32
// (v[1]).  The shapes only change which workgroup computes which outputs;
// every output is summed over K in the same order, so both give the same
// results.  While *choice < 0, runs alternate the shapes under HIP events;
// after TUNE_CALLS runs of each, the faster one is written to *choice (which
// outlives the op, so later set-ups reuse it) and used from then on.
class TunedGemm {
 public:
  static constexpr int TUNE_CALLS = 3;
  GemmOp v[2];
  int* choice = nullptr;   // -1: still measuring; null: always v[0]
  // follow: take the shape another op has chosen (v[0] until it has) and
  // never measure (for an op whose early calls have no work to time)
  const int* follow = nullptr;
  TunedGemm() { v[1].narrow = true; }
  TunedGemm(const TunedGemm&) = delete;
  TunedGemm& operator=(const TunedGemm&) = delete;
  ~TunedGemm() { drop_events(); }
  void reset() {           // empty both shapes, keep the choice and follow pointers
    drop_events();
    v[0] = GemmOp();
    v[1] = GemmOp();
    v[1].narrow = true;
    calls = 0;
  }
  void set_act(const int* a, int mask = ~0, int excl = 0) {
    v[0].act = v[1].act = a;
    v[0].act_mask = v[1].act_mask = mask;
    v[0].act_excl = v[1].act_excl = excl;
  }
  void set_f32(bool b32 = false) {
    v[0].f32 = v[1].f32 = true;
    v[0].b32 = v[1].b32 = b32;
  }
  void add(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int M, int N,
           int K, const int* flag = nullptr, const int* spair = nullptr, int scols = 0) {
    for (auto& g : v) g.add(A, lda, B, ldb, C, ldc, M, N, K, flag, spair, scols);
  }
  void finalize(hipStream_t st) {
    v[0].finalize(st);
    if (choice || follow) v[1].finalize(st);
  }
  void run(double alpha, double beta, hipStream_t st);

 private:
  int calls = 0;
  std::vector<hipEvent_t> ev[2];
  void drop_events();
};

struct GemvDesc {
  const void* A;    // K x M double block, column-major; after pack_a_f32 the
                    // transposed M x K float copy in row panels
  int lda, K, M;
  const double* X;  // K x nrhs
  int ldx;
  double* Y;        // M x nrhs
  int ldy;
  int wg_start;
};

class GemvOp {
 public:
  // from this many right-hand sides on, the product runs as an MFMA GEMM
  // (the operator is read once and the right-hand sides are staged in LDS)
  static constexpr int GEMM_FROM = 4;
  // FP64 operators whose columns are all at most this long take 16 lanes per
  // column instead of a wave
  static constexpr int SHORT_K = 128;
  bool a32 = false;                 // A blocks are FP32 (pack_a_f32)
  bool short_k = false;
  std::vector<GemvDesc> h;
  DBuf<GemvDesc> d;
  int wgs = 0;
  mutable std::vector<std::unique_ptr<GemmOp>> by_nrhs;   // built on first use
  void add(const double* A, int lda, int K, int M, const double* X, int ldx, double* Y, int ldy) {
    if (M <= 0) return;
    h.push_back(GemvDesc{A, lda, K, M, X, ldx, Y, ldy, 0});
  }
  void finalize(hipStream_t st);
  // Round every A block to FP32 into one buffer owned by `store`, stored
  // transposed (M x K) in row panels of PANEL_ROWS rows (see mfma_tile.hpp)
  // so that both the GEMV and the GEMM read it in contiguous runs, and point
  // the descriptors at it.  Call after the last add() and before finalize();
  // the FP64 source must hold its final values.
  void pack_a_f32(DBuf<float>& store, hipStream_t st);
  // Y = alpha A^T X + beta Y, nrhs in 1..16
  void run(double alpha, double beta, int nrhs, hipStream_t st) const;
  bool empty() const { return h.empty(); }
};

// y = alpha A x + beta y for symmetric n x n blocks (column-major, stored
// whole), reading only the 64 x 64 tiles on or below the diagonal: each
// workgroup takes one block column J, forms A_IJ x_J for the tiles I >= J as
// partial rows and A_IJ^T x_I for I > J as its own column sums, and a second
// pass adds the partials of every row in a fixed order.  Half the bytes of a
// GEMV over the whole block; 1..3 right-hand sides.
struct SymvDesc {
  const double* A;
  int lda, n;
  const double* X;
  int ldx;
  double* Y;
  int ldy;
  int nb;             // ceil(n / 64)
  int row_start;      // first row of this block in the rows of the sum pass
  int64_t part_off;   // partials: nb (nb + 1) / 2 tiles + nb column sums, 3 x 64 each
};

class SymvOp {
 public:
  static constexpr int MAX_RHS = 3;
  std::vector<SymvDesc> h;
  void add(const double* A, int lda, int n, const double* X, int ldx, double* Y, int ldy) {
    if (n <= 0) return;
    h.push_back(SymvDesc{A, lda, n, X, ldx, Y, ldy, 0, 0, 0});
  }
  void finalize(hipStream_t st);
  void run(double alpha, double beta, int nrhs, hipStream_t st) const;
  bool empty() const { return h.empty(); }

 private:
  DBuf<SymvDesc> d;
  DBuf<int2> work;     // (descriptor, block column), most tiles first
  DBuf<double> part;
  int nwork = 0, rows = 0;
};

// FP32 copies of dense blocks: dst (ld ldd) = src (ld lds), rows x cols.
struct CvtDesc {
  const double* src;
  int64_t lds;
  int rows, cols;
  float* dst;
  int64_t ldd;
  int wg_start;
};
void convert_blocks_f32(const std::vector<CvtDesc>& blocks, hipStream_t st);

struct LdltDesc {
  double* A;
  int lda, N, p, q;  // eliminate p pivots; pivots < q positive, the rest negative
};

class LdltOp {
 public:
  static constexpr int NB = 32;     // panel width
  static constexpr int OB = 256;    // outer block: columns per full trailing update
  static constexpr int TILE = 64;   // trailing update tile
  static constexpr int ROWS = 256;  // panel rows per workgroup
  std::vector<LdltDesc> h;
  DBuf<LdltDesc> d;
  // Phases in order: for every outer block of OB columns, its NB-wide inner
  // steps (diagonal block, panel, update of the rest of the outer block),
  // then one update of the whole trailing matrix with the OB panel columns.
  struct Phase {
    int big;       // 0: inner step at column k0; 1: trailing update of the block at k0
    int k0, outer; // k0 and the outer block's first column
    int off, nact, pan_total, upd_total;
  };
  std::vector<Phase> ph;
  DBuf<int> act, pan_pre, upd_pre;  // per phase: matrix ids, prefix sums of work items
  DBuf<int> info;                   // first failing matrix + 1 (0 = ok)
  void add(double* A, int lda, int N, int p, int q) { h.push_back(LdltDesc{A, lda, N, p, q}); }
  void finalize(hipStream_t st);
  void run(hipStream_t st);
  int failed(hipStream_t st);       // returns failing matrix index or -1
};

// In-place right-side triangular solve X L = B for a batch of matrices
// after their partial Cholesky: L (nI x nI, lower, in the leading block of
// A) and B (nG x nI, the block rows nI..nI+nG, columns 0..nI of A, i.e.
// K_GI L^{-T}) are overwritten by X = B L^{-1} = K_GI K_II^{-1}.  Columns from
// the right in groups of GB blocks of TB: a group first subtracts the product
// of all solved columns to its right in one MFMA GEMM (K up to nI), then each
// of its blocks, right to left, subtracts the group's solved blocks (K up to
// (GB - 1) TB) and is solved with its TB x TB diagonal block of L (one thread
// per row).
struct TrsmDesc {
  double* A;
  int lda, nI, nG;
};

class TrsmOp {
 public:
  static constexpr int TB = 64;   // columns per row solve
  static constexpr int GB = 4;    // row-solve blocks per group (one wide update each)
  std::vector<TrsmDesc> h;
  // one launch: block updates (B[:, c0:c0+w] -= X[:, kb:ke] L[kb:ke, c0:c0+w],
  // 64 x 64 tiles) or row solves (x L[c0:c0+w, c0:c0+w] = b, 256 rows per
  // workgroup) of the matrices that have such a step
  struct Rec {
    int m, c0, w, kb, ke, start;   // matrix, columns, K range, first workgroup
  };
  struct Launch {
    bool solve;
    int off, n, wgs;   // records [off, off + n) of recs
  };
  std::vector<Launch> launches;
  DBuf<TrsmDesc> d;
  DBuf<Rec> recs;
  void add(double* A, int lda, int nI, int nG) {
    if (nI > 0 && nG > 0) h.push_back(TrsmDesc{A, lda, nI, nG});
  }
  void finalize(hipStream_t st);
  void run(hipStream_t st) const;
};

// Batched x <- K_II^{-1} x with the partial Cholesky factor of every matrix
// (L lower in the leading nI x nI block of A and L^T in its upper triangle),
// all (up to 16) right-hand sides together: forward then backward
// substitution by diagonal blocks of OB rows, each solved by one workgroup per
// matrix in blocks of 64 rows, and after each block one wide launch that
// updates the remaining rows of every matrix with the block's solution.
struct TrsvDesc {
  const double* A;
  int lda, nI;
  double* x;        // nI x nrhs, leading dimension ldx
  int64_t ldx;
};

class TrsvOp {
 public:
  static constexpr int OB = 512;
  std::vector<TrsvDesc> h;
  void add(const double* A, int lda, int nI, double* x, int64_t ldx) {
    if (nI > 0) h.push_back(TrsvDesc{A, lda, nI, x, ldx});
  }
  void finalize(hipStream_t st);
  void run(int nrhs, hipStream_t st) const;
  bool empty() const { return h.empty(); }

 private:
  DBuf<TrsvDesc> d;
  DBuf<int> pre;   // first panel workgroup of every matrix
  int nob = 0, pwgs = 0;
};

class SymOp {
 public:
  struct Desc { double* A; int lda, n0, n; int start; };
  std::vector<Desc> h;
  DBuf<Desc> d;
  int tiles = 0;
  void add(double* A, int lda, int n0, int n) { if (n > 0) h.push_back(Desc{A, lda, n0, n, 0}); }
  void finalize(hipStream_t st);
  void run(hipStream_t st) const;
};

}  // namespace ambddc
