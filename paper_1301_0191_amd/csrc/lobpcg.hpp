// Batched LOBPCG over all face pairs of a level (pair eigenproblem of
// eq. eig-matrix, preconditioner of eq. bddc_pair) and the adaptive
// constraint construction.
#pragma once
#include "common.hpp"

namespace ambddc {

constexpr int PAIR_COARSE_MAX = 256;   // pair coarse DOFs (LDS of the coarse correction)
// The column-parallel pair kernels (slab copies, projection, commit) split a
// pair's m-column block over this many workgroups.
constexpr int PAIR_COL_GROUPS = 4;

struct PairDev {
  int s, t, nGs, nGt;
  int64_t gs_off, gt_off;      // stacked interface offsets of s and t
  int64_t v_off;               // offset of the pair's (n_p x 3m) blocks
  int64_t us_off, ut_off;      // first column of the pair's slot in U^s / U^t (ld nGs / nGt)
  int64_t ys_off, yt_off;      // same in Y^s / Y^t (ld nls / nlt)
  int nls, nlt;                // nG + nc
  int64_t zs_off, zt_off;      // in the coarse-slab Zc^s / Zc^t (ld nc)
  int ncs, nct;
  int sh0, sh1;                // shared interface DOFs
  int dr0, dr1;                // rows of D (shared initial coarse DOFs)
  int64_t cs_off, ct_off;      // C^s, C^t in the constraint buffer (ld nc)
  int pcs0, pct0;              // pair-coarse index ranges (length ncs, nct)
  int ncp;
  int64_t kp_off;              // pair coarse matrix / pseudo-inverse (ncp x ncp)
  int face0, nface;
  int64_t rb_off;              // orthonormal pair rigid modes (n_p x nrb), nrb = 0 if none
  int nrb;
  int64_t fc_off;              // face constraint rows (nev_max x nface, row-major)
};

struct PairIdx {               // flat index arrays referenced by PairDev ranges
  DBuf<int> sh_s, sh_t, pc_s, pc_t, face_s;
  DBuf<int> dptr, didx;        // entries of the rows of D (global row ids dr0..dr1 per pair)
  DBuf<int64_t> dcpos;
};

struct DRows {                 // device view of the sparse rows of D
  const int* ptr;
  const int* idx;
  const int64_t* cpos;
};

// Launchers (lobpcg.hip).  `m` is the block size, `col` selects a column
// block of V (0 = X, 1 = W, 2 = P), ncol columns.
void lp_random(const PairDev* P, int np, double* V, int m, uint64_t seed, hipStream_t st);
void lp_project(const PairDev* P, int np, double* V, int m, int col, const double* C,
                const DRows dr, const double* rb, const int* active, bool deflate,
                hipStream_t st);
// U32 (may be null): the slots of pairs in the FP32 phase are also written
// in FP32 there (same layout as U)
void lp_to_slab(const PairDev* P, int np, const double* V, int m, int col, bool with_ie,
                const double* diagG, const int* sh_s, const int* sh_t, double* U, float* U32,
                const int* active, hipStream_t st);
void lp_from_slab_ab(const PairDev* P, int np, const double* Y, int m, int col, double* AV,
                     double* BV, const double* diagG, const int* sh_s, const int* sh_t,
                     const double* C, const DRows dr, const int* active, hipStream_t st);
void lp_coarse(const PairDev* P, int np, const double* Y, int m, const double* Kp,
               const int* pc_s, const int* pc_t, double* Zc, int ncp_max, const int* active,
               hipStream_t st);
void lp_from_slab_w(const PairDev* P, int np, const double* Y, int m, double* V, const int* active,
                    hipStream_t st);
// active[p]: 0 converged, 1 FP32 products, 2 FP64 products (see lobpcg.hip)
void lp_residual(const PairDev* P, int np, double* V, const double* AV, const double* BV,
                 const double* lam, int m, int nconv, double tol, double tol32, int* active,
                 double* resn, double* hist, hipStream_t st);
void lp_rr(const PairDev* P, int np, const double* GA, const double* GB, int nb, int m,
           double* Cf, double* lam, const int* active, hipStream_t st);
void lp_commit(const PairDev* P, int np, double* V, double* AV, double* BV, const double* T,
               int m, bool with_p, bool only_v, const int* active, hipStream_t st);
void lp_pair_coarse(const PairDev* P, int np, const double* kc, const int64_t* kc_off,
                    const int* pc_s, const int* pc_t, double* Kp, hipStream_t st);
// Pair coarse pseudo-inverse (at most PAIR_COARSE_MAX pair coarse DOFs):
// null-space basis, augmented matrices, and the result after the batched
// factorisation of the augmented matrices (see lobpcg.hip).
void lp_pair_null(const PairDev* P, int np, const double* C, const int* pc_s, const int* pc_t,
                  const double* Kp, const double* rb, double* Nb, hipStream_t st);
void lp_pinv_fill(const PairDev* P, int np, const double* Kp, const double* Nb, double* Aug,
                  hipStream_t st);
void lp_pinv_extract(const PairDev* P, int np, const double* Aug, const double* Nb, double* Kp,
                     int* nsmall, hipStream_t st);
void lp_rigid(const PairDev* P, int np, const double* rigid, int ndof, const int* gdof,
              double* rb, hipStream_t st);
void lp_select(const PairDev* P, int np, const double* AV, const double* lam, int m, int nev_max,
               double tau, int fixed, const int* face_s, int nface_max, double* fc, int* kout,
               double* lam_next, hipStream_t st);

}  // namespace ambddc
