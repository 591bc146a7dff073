// Device-resident state of one substructuring level and of the top coarse
// problem.
#pragma once
#include "kernels.hpp"
#include "lobpcg.hpp"
#include "plan.hpp"

namespace ambddc {

struct Level {
  LevelPlan plan;
  int nsub = 0, ndof = 0, nrb = 1;
  std::vector<int> nI, nG, ns, augN;
  int augN_max = 0;   // largest augN
  std::vector<int64_t> aug_off, Ioff, Goff, y1off;
  int64_t aug_total = 0, nI_tot = 0, nG_tot = 0, y1_tot = 0;
  DBuf<double> aug, diagG, delta, rho, rigid;
  DBuf<int64_t> d_aug_off, diagpos, Imap, I2y1, g2y1, g2y2;
  DBuf<int> d_augN, d_nI, d_nG, d_ns, Gdof, incptr, incpos;
  AssemblyMaps am;
  const double* emat = nullptr;
  LdltOp ldl_aug;
  SymOp sym_aug;
  GemvOp g1, g4;
  // plain: the level-1 block is [[K_II, K_IG], [K_GI, K_GG]] without the
  // identity augmentation; after the factorisation its Gamma x I block holds
  // K_GI K_II^{-1} (trsm) and the interior block L and L^T (sym_L), and
  // interior solves are triangular solves (trsv) instead of the dense K_II^{-1}
  bool plain = false;
  TrsmOp trsm;
  SymOp sym_L;
  TrsvOp trsv;
  DBuf<int64_t> Iiota;

  // constraint-dependent part
  std::vector<int> nc, nl, naugN;
  std::vector<int64_t> c_off, naug_off, kc_off, y2off, cloff;
  int64_t c_total = 0, naug_total = 0, kc_total = 0, y2_tot = 0, cl_tot = 0;
  int ncoarse = 0;
  DBuf<double> C, naug, kc;
  DBuf<int64_t> d_naug_off, d_kc_off, cpos, clmap, cfill_pos;
  DBuf<double> cfill_val;
  DBuf<AdaptRow> cadapt_rows;   // adaptive rows of C and their face DOF maps
  DBuf<int> cadapt_map;
  DBuf<int> d_nc, d_nl, d_naugN, cptr;
  DBuf<NeuDesc> neu;
  int neu_cols = 0;
  LdltOp ldl_naug;
  SymOp sym_naug;
  GemvOp g2, g3;
  // FP64, 1..3 right-hand sides: g2 as the symmetric Z (tiles on or below the
  // diagonal) plus a GEMV over the coarse columns
  SymvOp g2z;
  GemvOp g2c;
  DBuf<double> Cs;                // sqrt(rho_s) C^s
  DBuf<int64_t> d_c_off, d_c_cnt;
  GemmOp gcc;                     // rho C^T C added to the (1,1) Neumann block

  // FP32 copies of the g1..g4 operators (precision 1)
  DBuf<float> g1_32, g2_32, g3_32, g4_32;

  // workspace of the preconditioner application
  int nrhs_cap = 0;
  DBuf<double> w_xI, w_y1, w_rBs, w_y2, w_rc, w_uc, w_ucl, w_uBs;

  // adaptive results
  int m = 0;
  std::vector<double> pair_lam, pair_lnext, pair_res;
  std::vector<int> pair_k, pair_conv, pair_nnull;
  std::vector<int> face_nf;
  std::vector<int64_t> fc_off;
  DBuf<double> fc;
  double omega = 0.0;
  int lobpcg_its = 0, n_unconv = 0, n_added = 0;
  int lobpcg_its32 = 0;   // iterations in which some pair ran FP32 products
};

struct Top {
  int n = 0;
  DBuf<double> aug, Kc;  // [[K_C, I], [I, 0]] of order 2n; Kc copy before factorisation
  AssemblyMaps am;
  DBuf<int64_t> d_off;
  DBuf<int> d_ld;
  LdltOp ldl;
  SymOp sym;
  GemvOp solve;
};

}  // namespace ambddc
