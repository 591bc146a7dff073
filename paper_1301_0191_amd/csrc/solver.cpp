// Set-up (Alg. 3), Multilevel BDDC application (Alg. 1), PCG, and the C ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <memory>
#include <numeric>
#include <string>

#include "../../include/ambddc.h"
#include "level.hpp"

using namespace ambddc;

namespace {

thread_local std::string g_err;

// Position of dof in the ascending range [b, e), or -1.
int find_sorted(const int* b, const int* e, int dof) {
  const int* it = std::lower_bound(b, e, dof);
  return (it != e && *it == dof) ? int(it - b) : -1;
}

struct LocalIndex {   // sorted (dof, local) pairs of one subdomain
  std::vector<std::pair<int, int>> v;
  void build(const std::vector<int>& dofs) {
    v.resize(dofs.size());
    for (size_t i = 0; i < dofs.size(); ++i) v[i] = {dofs[i], int(i)};
    std::sort(v.begin(), v.end());
  }
  int find(int dof) const {
    auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(dof, -1));
    return (it != v.end() && it->first == dof) ? it->second : -1;
  }
};

// Column-incidence maps: element matrices -> dense blocks of `ntgt` targets.
void build_assembly(AssemblyMaps& am, int nelem, const std::vector<int>& elem_tgt,
                    const std::vector<int64_t>& edptr, const std::vector<int>& edofs,
                    const std::vector<int64_t>& emat_off, const std::vector<LocalIndex>& loc,
                    const std::vector<int>& tgt_ncols, hipStream_t st) {
  const int ntgt = int(tgt_ncols.size());
  std::vector<int64_t> colbase(ntgt + 1, 0);
  for (int s = 0; s < ntgt; ++s) colbase[s + 1] = colbase[s] + tgt_ncols[s];
  const int64_t ncols = colbase[ntgt];
  std::vector<int> eloc(edofs.size(), -1);
  std::vector<int64_t> eloc_off(nelem + 1), cnt(ncols + 1, 0);
  std::vector<int> ene(nelem);
  for (int e = 0; e < nelem; ++e) {
    eloc_off[e] = edptr[e];
    ene[e] = int(edptr[e + 1] - edptr[e]);
    const int s = elem_tgt[e];
    for (int64_t p = edptr[e]; p < edptr[e + 1]; ++p) {
      if (edofs[p] < 0) continue;
      const int j = loc[s].find(edofs[p]);
      if (j < 0) throw Error(AMBDDC_E_INVALID_ARG, "element DOF missing from its subdomain");
      eloc[p] = j;
      cnt[colbase[s] + j + 1]++;
    }
  }
  eloc_off[nelem] = edptr[nelem];
  for (int64_t c = 0; c < ncols; ++c) cnt[c + 1] += cnt[c];
  std::vector<int> inc_e(cnt[ncols]), inc_a(cnt[ncols]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int e = 0; e < nelem; ++e) {
    const int s = elem_tgt[e];
    for (int64_t p = edptr[e]; p < edptr[e + 1]; ++p) {
      if (eloc[p] < 0) continue;
      const int64_t c = colbase[s] + eloc[p];
      inc_e[fill[c]] = e;
      inc_a[fill[c]] = int(p - edptr[e]);
      fill[c]++;
    }
  }
  std::vector<int> col_sub(ncols), col_j(ncols);
  for (int s = 0; s < ntgt; ++s)
    for (int j = 0; j < tgt_ncols[s]; ++j) {
      col_sub[colbase[s] + j] = s;
      col_j[colbase[s] + j] = j;
    }
  am.ncols = int(ncols);
  am.max_ne = nelem ? *std::max_element(ene.begin(), ene.end()) : 0;
  am.col_sub.upload(col_sub, st);
  am.col_j.upload(col_j, st);
  am.inc_ptr.upload(cnt, st);
  am.inc_e.upload(inc_e, st);
  am.inc_a.upload(inc_a, st);
  am.emat_off.upload(emat_off, st);
  am.elem_ne.upload(ene, st);
  am.eloc_off.upload(eloc_off, st);
  am.eloc.upload(eloc, st);
}

}  // namespace

struct ambddc_ctx {
  hipStream_t st = nullptr;
  ambddc_options opt{};
  int n_nodes = 0, n_elems = 0, dof = 1, levels = 2;
  std::vector<int> free_of_full;
  std::vector<std::vector<int>> parents;
  LevelPlan plan0;
  DBuf<double> coords;
  DBuf<int> en, edofs;
  CsrMaps csr;
  DBuf<double> csr_vals, Ke;
  DBuf<unsigned char> imask;   // level-1 interior rows of the global vectors
  std::vector<std::unique_ptr<Level>> L;
  Top top;
  bool ready = false;
  ambddc_stats stats{};
  KTimer kt;   // optional per-class kernel timing
  std::map<std::string, int> tune;   // tile-shape choices of tuned products (-1: measuring)
  DBuf<double> coeff_buf, mis_part, mis_out;   // log10 set-up and misfit workspace
  // PCG workspace of ambddc_solve (carved into a PcgWork)
  int pcg_cap = 0, pcg_maxit = 0;
  DBuf<double> pwd;
  DBuf<int> pwi;
  int pcg_repl = 0;   // residual replacements in the last solve
  double last_res[16] = {};   // true relative residuals of the last solve
  int n_last_res = 0;
  // pinned host copy of the PCG counters and the event that follows its copy
  int* hcnt = nullptr;
  hipEvent_t ev_cnt = nullptr;
  // PCG iteration graphs: captured on cap_st, launched on st; valid for one
  // set-up (setup_epoch) and one set of solve arguments (pcg_gkey)
  int setup_epoch = 0, pcg_gepoch = -1;
  hipStream_t cap_st = nullptr;
  int graphs = 0;   // ambddc_set_graphs flags
  hipGraphExec_t pcg_g1 = nullptr, pcg_g2 = nullptr;
  const void* pcg_gkey[5] = {};
  double pcg_grtol = 0.0;
  void drop_pcg_graphs() {
    if (pcg_g1) (void)hipGraphExecDestroy(pcg_g1);
    if (pcg_g2) (void)hipGraphExecDestroy(pcg_g2);
    pcg_g1 = pcg_g2 = nullptr;
    pcg_gepoch = -1;
  }
  ~ambddc_ctx() {
    drop_pcg_graphs();
    if (cap_st) (void)hipStreamDestroy(cap_st);
    if (ev_cnt) (void)hipEventDestroy(ev_cnt);
    if (hcnt) (void)hipHostFree(hcnt);
  }
};

namespace {

// Residual at which a pair's LOBPCG leaves FP32 products for FP64 ones
// (precision 2), unless it stalls earlier.
constexpr double LOBPCG_TOL32 = 1e-5;

// Most adaptive constraints one face can receive: nev_max under Alg. 2, or
// the fixed count per face.
int nsel_max(const ambddc_options& o) { return o.fixed_per_face > 0 ? o.fixed_per_face : o.nev_max; }

// ---------------------------------------------------------------------------
// level structure
// ---------------------------------------------------------------------------

void build_level_maps(ambddc_ctx& c, Level& L, const double* emat,
                      const std::vector<int64_t>& emat_off, bool plain) {
  hipStream_t st = c.st;
  const LevelPlan& P = L.plan;
  L.plain = plain;
  L.nsub = P.in.n_sub;
  L.ndof = P.in.n_dof;
  L.nrb = P.in.n_rb;
  const int ns = L.nsub;
  L.nI.resize(ns); L.nG.resize(ns); L.ns.resize(ns); L.augN.resize(ns);
  L.aug_off.assign(ns + 1, 0); L.Ioff.assign(ns + 1, 0); L.Goff.assign(ns + 1, 0);
  L.y1off.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    L.nI[s] = P.subs[s].nI;
    L.nG[s] = P.subs[s].nG;
    L.ns[s] = L.nI[s] + L.nG[s];
    L.augN[s] = plain ? L.ns[s] : L.ns[s] + L.nI[s];
    L.aug_off[s + 1] = L.aug_off[s] + int64_t(L.augN[s]) * L.augN[s];
    L.Ioff[s + 1] = L.Ioff[s] + L.nI[s];
    L.Goff[s + 1] = L.Goff[s] + L.nG[s];
    L.y1off[s + 1] = L.y1off[s] + L.nG[s] + L.nI[s];
  }
  L.aug_total = L.aug_off[ns];
  L.augN_max = ns ? *std::max_element(L.augN.begin(), L.augN.end()) : 0;
  L.nI_tot = L.Ioff[ns];
  L.nG_tot = L.Goff[ns];
  L.y1_tot = L.y1off[ns];
  L.aug.alloc(size_t(L.aug_total));
  L.d_aug_off.upload(std::vector<int64_t>(L.aug_off.begin(), L.aug_off.end() - 1), st);
  L.d_augN.upload(L.augN, st);
  L.d_nI.upload(L.nI, st);
  L.d_nG.upload(L.nG, st);
  L.d_ns.upload(L.ns, st);
  // assembly: elements of this level into the leading blocks of Aug^s
  std::vector<LocalIndex> loc(ns);
  for (int s = 0; s < ns; ++s) loc[s].build(P.subs[s].dofs);
  build_assembly(L.am, P.in.n_elem, P.in.elem_sub, P.in.elem_dof_ptr, P.in.elem_dofs, emat_off, loc,
                 L.ns, st);
  L.emat = emat;
  // stacked maps
  std::vector<int64_t> Imap(L.nI_tot), I2y1(L.nI_tot), g2y1(L.nG_tot), g2y2(L.nG_tot),
      diagpos(L.nG_tot);
  std::vector<int> Gdof(L.nG_tot);
  std::vector<int> incptr(L.ndof + 1, 0);
  for (int s = 0; s < ns; ++s) {
    const auto& d = P.subs[s].dofs;
    for (int i = 0; i < L.nI[s]; ++i) {
      Imap[L.Ioff[s] + i] = d[i];
      I2y1[L.Ioff[s] + i] = L.y1off[s] + L.nG[s] + i;
    }
    for (int i = 0; i < L.nG[s]; ++i) {
      const int64_t k = L.Goff[s] + i;
      Gdof[k] = d[L.nI[s] + i];
      g2y1[k] = L.y1off[s] + i;
      diagpos[k] = L.aug_off[s] + (L.nI[s] + i) + int64_t(L.nI[s] + i) * L.augN[s];
      incptr[Gdof[k] + 1]++;
    }
  }
  for (int j = 0; j < L.ndof; ++j) incptr[j + 1] += incptr[j];
  std::vector<int> incpos(L.nG_tot);
  {
    std::vector<int> f(incptr.begin(), incptr.end() - 1);
    for (int64_t k = 0; k < L.nG_tot; ++k) incpos[f[Gdof[k]]++] = int(k);
  }
  L.Imap.upload(Imap, st);
  L.I2y1.upload(I2y1, st);
  L.g2y1.upload(g2y1, st);
  L.diagpos.upload(diagpos, st);
  L.Gdof.upload(Gdof, st);
  L.incptr.upload(incptr, st);
  L.incpos.upload(incpos, st);
  L.diagG.alloc(L.nG_tot);
  L.delta.alloc(L.nG_tot);
  L.rho.alloc(ns);
  (void)g2y2;
  // batched partial factorisation of Aug^s = [[K, I_I^T], [I_I, 0]] (or of
  // K alone on a plain level): nI positive pivots
  L.ldl_aug = LdltOp();
  L.sym_aug = SymOp();
  L.trsm = TrsmOp();
  L.sym_L = SymOp();
  L.g1 = GemvOp();
  L.g4 = GemvOp();
  for (int s = 0; s < ns; ++s) {
    double* A = L.aug.p + L.aug_off[s];
    const int N = L.augN[s];
    L.ldl_aug.add(A, N, N, L.nI[s], L.nI[s]);
    L.sym_aug.add(A, N, L.nI[s], plain ? L.nG[s] : L.nG[s] + L.nI[s]);
    if (plain) {
      L.trsm.add(A, N, L.nI[s], L.nG[s]);
      L.sym_L.add(A, N, 0, L.nI[s]);
    }
  }
  L.ldl_aug.finalize(st);
  L.sym_aug.finalize(st);
  if (plain) {
    L.trsm.finalize(st);
    L.sym_L.finalize(st);
    std::vector<int64_t> iota(std::max<int64_t>(L.nI_tot, 1));
    for (int64_t i = 0; i < int64_t(iota.size()); ++i) iota[i] = i;
    L.Iiota.upload(iota, st);
  }
}

void alloc_workspace(Level& L, int nrhs) {
  if (L.nrhs_cap >= nrhs) return;
  L.nrhs_cap = nrhs;
  L.w_xI.alloc(size_t(std::max<int64_t>(L.nI_tot, 1)) * nrhs);
  L.w_y1.alloc(size_t(std::max<int64_t>(L.y1_tot, 1)) * nrhs);
  L.w_rBs.alloc(size_t(std::max<int64_t>(L.nG_tot, 1)) * nrhs);
  L.w_uBs.alloc(size_t(std::max<int64_t>(L.nG_tot, 1)) * nrhs);
}

void alloc_coarse_workspace(Level& L, int nrhs) {
  L.w_y2.alloc(size_t(std::max<int64_t>(L.y2_tot, 1)) * nrhs);
  L.w_rc.alloc(size_t(std::max(L.ncoarse, 1)) * nrhs);
  L.w_uc.alloc(size_t(std::max(L.ncoarse, 1)) * nrhs);
  L.w_ucl.alloc(size_t(std::max<int64_t>(L.cl_tot, 1)) * nrhs);
}

// GEMV descriptors of the preconditioner (depend on workspace pointers)
void build_apply_ops(ambddc_ctx& c, Level& L) {
  hipStream_t st = c.st;
  L.g1 = GemvOp();
  L.g2 = GemvOp();
  L.g2z = SymvOp();
  L.g2c = GemvOp();
  L.g3 = GemvOp();
  L.g4 = GemvOp();
  L.trsv = TrsvOp();
  for (int s = 0; s < L.nsub; ++s) {
    const int N = L.augN[s], nI = L.nI[s], nG = L.nG[s], nsl = L.ns[s];
    double* A = L.aug.p + L.aug_off[s];
    if (L.plain) {
      // interior solves by the factor; K_II^{-1} K_IG u_B = (Aug[nI:nI+nG, 0:nI])^T u_B
      L.trsv.add(A, N, nI, L.w_xI.p + L.Ioff[s], L.nI_tot);
      L.g4.add(A + nI, N, nG, nI, L.w_uBs.p + L.Goff[s], int(L.nG_tot),
               L.w_y1.p + L.y1off[s] + nG, int(L.y1_tot));
    } else {
      // [g; -K_II^{-1} r_I] = M^T r_I,  M = Aug[ns:ns+nI, nI:nI+nG+nI]
      L.g1.add(A + nsl + int64_t(nI) * N, N, nI, nG + nI, L.w_xI.p + L.Ioff[s], int(L.nI_tot),
               L.w_y1.p + L.y1off[s], int(L.y1_tot));
      // interior:  Tr[nG:, 0:nG] u_B = (Aug[nI:nI+nG, ns:ns+nI])^T u_B = -K_II^{-1} K_IG u_B
      L.g4.add(A + nI + int64_t(nsl) * N, N, nG, nI, L.w_uBs.p + L.Goff[s], int(L.nG_tot),
               L.w_y1.p + L.y1off[s] + nG, int(L.y1_tot));
    }
    const int nl = L.nl[s], NN = L.naugN[s];
    double* B = L.naug.p + L.naug_off[s];
    // [-Z r; -Psi^T r] = (Trn[0:nG, 0:nl])^T r
    L.g2.add(B + nl + int64_t(nl) * NN, NN, nG, nl, L.w_rBs.p + L.Goff[s], int(L.nG_tot),
             L.w_y2.p + L.y2off[s], int(L.y2_tot));
    if (c.opt.precision == 0) {
      // Trn[0:nG, 0:nG] = -Z is symmetric
      L.g2z.add(B + nl + int64_t(nl) * NN, NN, nG, L.w_rBs.p + L.Goff[s], int(L.nG_tot),
                L.w_y2.p + L.y2off[s], int(L.y2_tot));
      L.g2c.add(B + nl + int64_t(nl + nG) * NN, NN, nG, nl - nG, L.w_rBs.p + L.Goff[s],
                int(L.nG_tot), L.w_y2.p + L.y2off[s] + nG, int(L.y2_tot));
    }
    // -Psi u_c = (Trn[nG:nl, 0:nG])^T u_c
    L.g3.add(B + nl + nG + int64_t(nl) * NN, NN, L.nc[s], nG, L.w_ucl.p + L.cloff[s],
             int(std::max<int64_t>(L.cl_tot, 1)), L.w_y2.p + L.y2off[s], int(L.y2_tot));
  }
  if (L.plain) L.trsv.finalize(st);
  if (c.opt.precision >= 1) {
    // Alg. 1's dense operators are only read by the preconditioner: keep them
    // in FP32 (the FP64 blocks stay for the Schur complements and set-up).
    // On level 1 the PCG iterates in the discrete harmonic space, which the
    // interior solves of x0 and the interior post-correction (g4) must keep
    // to FP64 rounding: a residual component on the interiors is never
    // corrected there, so those stay FP64.
    const bool level1 = &L == c.L[0].get();
    if (!level1 && !L.plain) L.g1.pack_a_f32(L.g1_32, st);
    L.g2.pack_a_f32(L.g2_32, st);
    L.g3.pack_a_f32(L.g3_32, st);
    if (!level1) L.g4.pack_a_f32(L.g4_32, st);
  }
  L.g1.finalize(st);
  L.g2.finalize(st);
  L.g2z.finalize(st);
  L.g2c.finalize(st);
  L.g3.finalize(st);
  L.g4.finalize(st);
}

// constraint-dependent structures (sizes from plan.subs[s].cons)
void build_constraint_maps(ambddc_ctx& c, Level& L) {
  hipStream_t st = c.st;
  const LevelPlan& P = L.plan;
  const int ns = L.nsub;
  L.ncoarse = int(P.cons.size());
  L.nc.resize(ns); L.nl.resize(ns); L.naugN.resize(ns);
  L.c_off.assign(ns + 1, 0); L.naug_off.assign(ns + 1, 0); L.kc_off.assign(ns + 1, 0);
  L.y2off.assign(ns + 1, 0); L.cloff.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    L.nc[s] = int(P.subs[s].cons.size());
    L.nl[s] = L.nG[s] + L.nc[s];
    L.naugN[s] = 2 * L.nl[s];
    L.c_off[s + 1] = L.c_off[s] + int64_t(L.nc[s]) * L.nG[s];
    L.naug_off[s + 1] = L.naug_off[s] + int64_t(L.naugN[s]) * L.naugN[s];
    L.kc_off[s + 1] = L.kc_off[s] + int64_t(L.nc[s]) * L.nc[s];
    L.y2off[s + 1] = L.y2off[s] + L.nl[s];
    L.cloff[s + 1] = L.cloff[s] + L.nc[s];
  }
  L.c_total = L.c_off[ns];
  L.naug_total = L.naug_off[ns];
  L.kc_total = L.kc_off[ns];
  L.y2_tot = L.y2off[ns];
  L.cl_tot = L.cloff[ns];
  L.C.alloc(std::max<int64_t>(L.c_total, 1));
  L.naug.alloc(std::max<int64_t>(L.naug_total, 1));
  L.kc.alloc(std::max<int64_t>(L.kc_total, 1));
  L.d_naug_off.upload(std::vector<int64_t>(L.naug_off.begin(), L.naug_off.end() - 1), st);
  L.d_kc_off.upload(std::vector<int64_t>(L.kc_off.begin(), L.kc_off.end() - 1), st);
  L.d_nc.upload(L.nc, st);
  L.d_nl.upload(L.nl, st);
  L.d_naugN.upload(L.naugN, st);
  // C entries: initial constraints get 1 or 1/m; adaptive rows copy their
  // pair's face row from fc (every row of a pair has the pair's face DOFs,
  // whose local indices are looked up once per subdomain and pair)
  std::vector<int64_t> fpos;
  std::vector<double> fval;
  std::vector<AdaptRow> arows;
  std::vector<int> amap;
  std::vector<int64_t> g2y2(L.nG_tot);
  for (int s = 0; s < ns; ++s)
    for (int i = 0; i < L.nG[s]; ++i) g2y2[L.Goff[s] + i] = L.y2off[s] + i;
  std::vector<int> cptr(L.ncoarse + 1, 0);
  for (int s = 0; s < ns; ++s) {
    const auto& cs = P.subs[s].cons;
    const int* G0 = P.subs[s].dofs.data() + L.nI[s];   // interface DOFs, ascending
    const int* G1 = G0 + L.nG[s];
    auto local = [&](int dof) {
      const int i = find_sorted(G0, G1, dof);
      if (i < 0) throw Error(AMBDDC_E_INVALID_ARG, "constraint DOF outside the interface");
      return i;
    };
    std::vector<std::pair<int, int64_t>> pair_map;   // (pair, offset in amap)
    for (int r = 0; r < L.nc[s]; ++r) {
      const Constraint& K = P.cons[cs[r]];
      cptr[cs[r] + 1]++;
      if (K.kind == CONS_ADAPT) {
        int64_t off = -1;
        for (const auto& pm : pair_map)
          if (pm.first == K.pair) off = pm.second;
        if (off < 0) {
          off = int64_t(amap.size());
          for (int d : K.dofs) amap.push_back(local(d));
          pair_map.push_back({K.pair, off});
        }
        arows.push_back(AdaptRow{L.c_off[s] + r,
                                 L.fc_off[K.pair] + int64_t(K.row) * L.face_nf[K.pair], off,
                                 L.nc[s], int(K.dofs.size())});
      } else {
        const double v = K.kind == CONS_UNIT ? 1.0 : 1.0 / double(K.dofs.size());
        for (int d : K.dofs) {
          fpos.push_back(L.c_off[s] + r + int64_t(local(d)) * L.nc[s]);
          fval.push_back(v);
        }
      }
    }
  }
  for (int k = 0; k < L.ncoarse; ++k) cptr[k + 1] += cptr[k];
  std::vector<int64_t> cpos(cptr[L.ncoarse]), clmap(L.cl_tot);
  {
    std::vector<int> f(cptr.begin(), cptr.end() - 1);
    for (int s = 0; s < ns; ++s) {
      const auto& cs = P.subs[s].cons;
      for (int r = 0; r < L.nc[s]; ++r) {
        cpos[f[cs[r]]++] = L.y2off[s] + L.nG[s] + r;
        clmap[L.cloff[s] + r] = cs[r];
      }
    }
  }
  L.cfill_pos.upload(fpos, st);
  L.cfill_val.upload(fval, st);
  L.cadapt_rows.upload(arows, st);
  L.cadapt_map.upload(amap, st);
  L.cptr.upload(cptr, st);
  L.cpos.upload(cpos, st);
  L.clmap.upload(clmap, st);
  L.g2y2.upload(g2y2, st);
  // Neumann augmented matrices and their factorisation
  std::vector<NeuDesc> nd(ns);
  L.neu_cols = 0;
  L.ldl_naug = LdltOp();
  L.sym_naug = SymOp();
  for (int s = 0; s < ns; ++s) {
    const int N = L.augN[s];
    nd[s].S = L.aug.p + L.aug_off[s] + L.nI[s] + int64_t(L.nI[s]) * N;
    nd[s].lds = N;
    nd[s].C = L.C.p + L.c_off[s];
    nd[s].nc = L.nc[s];
    nd[s].A = L.naug.p + L.naug_off[s];
    nd[s].lda = L.naugN[s];
    nd[s].nG = L.nG[s];
    nd[s].rho = L.rho.p + s;
    nd[s].col_start = L.neu_cols;
    L.neu_cols += L.nl[s];
    L.ldl_naug.add(nd[s].A, L.naugN[s], L.naugN[s], L.nl[s], L.nG[s]);
    L.sym_naug.add(nd[s].A, L.naugN[s], L.nl[s], L.nl[s]);
  }
  L.neu.upload(nd, st);
  L.ldl_naug.finalize(st);
  L.sym_naug.finalize(st);
  // rho_s C^T C = (sqrt(rho_s) C)^T (sqrt(rho_s) C) on MFMA, added to S in place
  L.Cs.alloc(size_t(std::max<int64_t>(L.c_total, 1)));
  {
    std::vector<int64_t> co(ns), cn(ns);
    for (int s = 0; s < ns; ++s) {
      co[s] = L.c_off[s];
      cn[s] = int64_t(L.nc[s]) * L.nG[s];
    }
    L.d_c_off.upload(co, st);
    L.d_c_cnt.upload(cn, st);
  }
  L.gcc = GemmOp();
  L.gcc.ta = true;
  for (int s = 0; s < ns; ++s) {
    if (L.nc[s] == 0) continue;
    const double* cs = L.Cs.p + L.c_off[s];
    L.gcc.add(cs, L.nc[s], cs, L.nc[s], L.naug.p + L.naug_off[s], L.naugN[s], L.nG[s], L.nG[s],
              L.nc[s]);
  }
  L.gcc.finalize(st);
  alloc_coarse_workspace(L, std::max(L.nrhs_cap, 1));
}

void check_ldlt(LdltOp& op, hipStream_t st, const char* what, int level) {
  const int f = op.failed(st);
  if (f >= 0)
    throw Error(AMBDDC_E_NOT_SPD, std::string(what) + ": non-positive pivot in matrix " +
                                      std::to_string(f) + " on level " + std::to_string(level + 1));
}

// assemble K^s, weights, Schur complements (Section 2, Section 7)
void numeric_schur(ambddc_ctx& c, Level& L, int li) {
  hipStream_t st = c.st;
  if (L.plain && L.augN_max <= 8192 && L.am.max_ne <= 64) {
    // every column of the ns x ns blocks is assembled whole
    launch_assemble_cols(L.am, L.augN_max, L.emat, L.d_aug_off.p, L.d_augN.p, L.aug.p, st);
  } else {
    L.aug.zero(st);
    launch_assemble(L.am, L.emat, L.d_aug_off.p, L.d_augN.p, L.aug.p, st);
  }
  // identity coupling Aug[ns + i, i] = Aug[i, ns + i] = 1, i < nI
  if (!L.plain) {
    std::vector<int> zero(L.nsub, 0);
    DBuf<int> dz;
    dz.upload(zero, st);
    launch_aug_identity(L.nsub, L.d_aug_off.p, L.d_augN.p, L.d_nI.p, dz.p, L.d_ns.p, st, L.aug.p);
  }
  launch_diag_copy(int(L.nG_tot), L.diagpos.p, L.aug.p, L.diagG.p, st);
  launch_weights(int(L.nG_tot), L.Gdof.p, L.incptr.p, L.incpos.p, L.diagG.p, L.delta.p, st);
  {
    double f = 0.0, b = 0.0;
    for (int s = 0; s < L.nsub; ++s) {
      const double nI = L.nI[s], nG = L.nG[s];
      f += nI * nI * nI / 3.0 + nI * nI * nG + nI * nG * nG;
      if (L.plain) f += nI * nI * nG;   // K_GI K_II^{-1} by the triangular solve
      b += 8.0 * (nI + nG) * (nI + nG);
    }
    c.kt.begin("schur", st);
    L.ldl_aug.run(st);
    if (L.plain) L.trsm.run(st);   // K_GI K_II^{-1} from the factor
    c.kt.end("schur", st, f, b);
  }
  check_ldlt(L.ldl_aug, st, "interior factorisation", li);
  L.sym_aug.run(st);
  if (L.plain) L.sym_L.run(st);
  // rho_s = mean diag(S^s)
  {
    std::vector<int> n0(L.nsub);
    for (int s = 0; s < L.nsub; ++s) n0[s] = L.nI[s];
    DBuf<int> dn0;
    dn0.upload(n0, st);
    launch_diag_mean(L.nsub, L.d_aug_off.p, L.d_augN.p, dn0.p, L.d_nG.p, L.aug.p, L.rho.p, st);
  }
}

// constraint matrices, constrained Neumann operators, coarse basis (Section 5)
// C^s: initial rows 1 or 1/m, adaptive rows from the face constraint rows
void fill_constraints(Level& L, hipStream_t st) {
  L.C.zero(st);
  launch_fill_values(int(L.cfill_pos.n), L.cfill_pos.p, L.cfill_val.p, L.C.p, st);
  launch_fill_adaptive(int(L.cadapt_rows.n), L.cadapt_rows.p, L.cadapt_map.p, L.fc.p, L.C.p, st);
}

void numeric_neumann(ambddc_ctx& c, Level& L, int li) {
  hipStream_t st = c.st;
  fill_constraints(L, st);
  L.naug.zero(st);
  launch_neumann_fill(L.neu.p, L.nsub, L.neu_cols, st);
  launch_scale_sqrt_sub(L.nsub, L.d_c_off.p, L.d_c_cnt.p, L.rho.p, L.C.p, L.Cs.p, st);
  L.gcc.run(1.0, 1.0, st);
  L.ldl_naug.run(st);
  check_ldlt(L.ldl_naug, st, "constrained Neumann factorisation", li);
  L.sym_naug.run(st);
  launch_extract_kc(L.nsub, L.d_naug_off.p, L.d_naugN.p, L.d_nG.p, L.d_nc.p, L.d_kc_off.p, L.rho.p,
                    nullptr, L.naug.p, L.kc.p, st);
}

// The constrained Neumann inverses of a level before its adaptive rows are
// added (the trailing blocks T = -X^{-1} of the augmented matrices), kept to
// border them with the new rows.
struct NeumannPrev {
  DBuf<double> naug;
  std::vector<int> nc, nl;
  std::vector<int64_t> naug_off;
};

NeumannPrev keep_neumann(Level& L) {
  NeumannPrev o;
  o.naug = std::move(L.naug);
  o.nc = L.nc;
  o.nl = L.nl;
  o.naug_off = L.naug_off;
  return o;
}

// Constrained Neumann inverses after adaptive rows C_a (k per subdomain,
// appended after the existing rows) are added, by bordering the previous
// ones instead of factorising again.  With X the previous saddle-point
// matrix [[S + rho C^T C, C^T], [C, 0]] and b = [C_a^T; 0], the new matrix
// is [[X, b], [b^T, 0]]; with Y = X^{-1} b and the SPD k x k matrix
// S_c = b^T Y, its inverse is [[X^{-1} - Y S_c^{-1} Y^T, Y S_c^{-1}],
// [S_c^{-1} Y^T, -S_c^{-1}]].  The rho term then acts on the previous rows
// only: Z and Psi (the displacement rows of the inverse) do not depend on
// it, and K_c takes the rho correction on those rows only.  Work per
// subdomain about 2 n_l^2 k instead of a factorisation of order 2 n_l.
void neumann_bordered(ambddc_ctx& c, Level& L, int li, NeumannPrev& old) {
  hipStream_t st = c.st;
  const int ns = L.nsub;
  fill_constraints(L, st);
  std::vector<int64_t> src_off(ns), dst_off(ns), yoff(ns + 1, 0), aoff(ns + 1, 0);
  std::vector<int> src_ld(ns), r0(ns), rows(ns), dst_ld(ns);
  for (int s = 0; s < ns; ++s) {
    const int k = L.nc[s] - old.nc[s], nl = old.nl[s], nl2 = L.nl[s];
    if (k < 0 || nl2 != nl + k) throw Error(AMBDDC_E_INVALID_ARG, "constraint rows removed");
    src_off[s] = old.naug_off[s];
    src_ld[s] = 2 * nl;
    r0[s] = nl;
    rows[s] = nl;
    dst_off[s] = L.naug_off[s] + nl2 + int64_t(nl2) * (2 * nl2);
    dst_ld[s] = 2 * nl2;
    yoff[s + 1] = yoff[s] + int64_t(nl) * k;
    aoff[s + 1] = aoff[s] + int64_t(2 * k) * (2 * k);
  }
  {
    DBuf<int64_t> so, dof;
    DBuf<int> sl, rr, nr, dl;
    so.upload(src_off, st);
    dof.upload(dst_off, st);
    sl.upload(src_ld, st);
    rr.upload(r0, st);
    nr.upload(rows, st);
    dl.upload(dst_ld, st);
    launch_copy_block(ns, so.p, sl.p, rr.p, nr.p, nr.p, dof.p, dl.p, old.naug.p, L.naug.p, st);
  }
  DBuf<double> Y, Wm, Sa;
  Y.alloc(size_t(std::max<int64_t>(yoff[ns], 1)));
  Wm.alloc(size_t(std::max<int64_t>(yoff[ns], 1)));
  Sa.alloc(size_t(std::max<int64_t>(aoff[ns], 1)));
  Sa.zero(st);
  GemmOp gy, gs, gw, gt;
  gy.tb = true;
  gt.tb = true;
  LdltOp lsc;
  SymOp ssc;
  std::vector<BorderDesc> bd;
  std::vector<int64_t> ioff;
  std::vector<int> ild, ik, izero;
  for (int s = 0; s < ns; ++s) {
    const int k = L.nc[s] - old.nc[s], nl = old.nl[s], nl2 = L.nl[s], nG = L.nG[s];
    if (k == 0) continue;
    const double* Told = old.naug.p + old.naug_off[s] + nl + int64_t(nl) * (2 * nl);
    const double* Ca = L.C.p + L.c_off[s] + old.nc[s];
    double* Ys = Y.p + yoff[s];
    double* Ws = Wm.p + yoff[s];
    double* Ss = Sa.p + aoff[s];
    double* Tsc = Ss + k + int64_t(k) * (2 * k);
    double* Tn = L.naug.p + dst_off[s];
    gy.add(Told, 2 * nl, Ca, L.nc[s], Ys, nl, nl, k, nG);        // Y = -T[:, :nG] C_a^T
    gs.add(Ca, L.nc[s], Ys, nl, Ss, 2 * k, k, k, nG);            // S_c = C_a Y[:nG]
    lsc.add(Ss, 2 * k, 2 * k, k, k);                             // [[S_c, I], [I, 0]] -> -S_c^{-1}
    ssc.add(Ss, 2 * k, k, k);
    gw.add(Ys, nl, Tsc, 2 * k, Ws, nl, nl, k, k);                // W = -Y (-S_c^{-1})
    gt.add(Ws, nl, Ys, nl, Tn, 2 * nl2, nl, nl, k);              // T += W Y^T
    bd.push_back(BorderDesc{Tn, Ws, Tsc, 2 * nl2, nl, 2 * k, nl, k});
    ioff.push_back(aoff[s]);
    ild.push_back(2 * k);
    ik.push_back(k);
    izero.push_back(0);
  }
  if (!bd.empty()) {
    gy.finalize(st);
    gs.finalize(st);
    gw.finalize(st);
    gt.finalize(st);
    lsc.finalize(st);
    ssc.finalize(st);
    DBuf<int64_t> io;
    DBuf<int> il, ikk, iz;
    DBuf<BorderDesc> db;
    io.upload(ioff, st);
    il.upload(ild, st);
    ikk.upload(ik, st);
    iz.upload(izero, st);
    db.upload(bd, st);
    gy.run(-1.0, 0.0, st);
    gs.run(1.0, 0.0, st);
    launch_aug_identity(int(bd.size()), io.p, il.p, ikk.p, iz.p, ikk.p, st, Sa.p);
    lsc.run(st);
    check_ldlt(lsc, st, "constrained Neumann border (new constraint rows)", li);
    ssc.run(st);
    gw.run(-1.0, 0.0, st);
    gt.run(1.0, 1.0, st);
    launch_border_fill(db.p, int(bd.size()), st);
  }
  DBuf<int> nrho;
  nrho.upload(old.nc, st);
  launch_extract_kc(ns, L.d_naug_off.p, L.d_naugN.p, L.d_nG.p, L.d_nc.p, L.d_kc_off.p, L.rho.p,
                    nrho.p, L.naug.p, L.kc.p, st);
  AMB_HIP(hipStreamSynchronize(st));
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// adaptive selection on one level: batched LOBPCG over all face pairs
// ---------------------------------------------------------------------------

struct PairWork {
  int np = 0, m = 0, ncp_max = 0, nface_max = 0;
  std::vector<PairDev> hp;
  DBuf<PairDev> dp;
  PairIdx idx;
  DBuf<double> V, AV, BV, T, GA, GB, Cf, lam, resn, U, Y, Zc, Kp, rb, lnext, Cxw, Nb, Aug;
  DBuf<int> active, kout, nnull, slot_pair;
  DBuf<double> hist;        // per pair: residual history of the FP32 phase
  TunedGemm gS, gM1, gM2;   // grouped per-subdomain products, tile shape tuned
  // the same products on FP32 copies of S^s and the Neumann inverse with FP32
  // accumulation, for pairs in the FP32 phase (precision 2)
  TunedGemm gS32, gM1_32, gM2_32;
  bool lo = false;          // some pairs start in the FP32 phase
  DBuf<float> S32, T32, U32;
  GemmOp gram[3], upd_v[3], orth_c, orth_u, orthp_c, orthp_u;   // gram: V^T AV and V^T BV in one launch
  KTimer* kt = nullptr;
  std::vector<int> act;                          // host copy of the active flags
  std::vector<int> h_slot_off, h_slot_pair;      // pair of every subdomain slot
};

// Pinned host copy of the active flags, read back through an event so that
// the stream keeps working while the host waits for it.
struct FlagReadback {
  int* h = nullptr;
  hipEvent_t ev = nullptr;
  int n = 0;
  explicit FlagReadback(int np) : n(np) {
    AMB_HIP(hipHostMalloc((void**)&h, sizeof(int) * std::max(np, 1), hipHostMallocDefault));
    AMB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  FlagReadback(const FlagReadback&) = delete;
  FlagReadback& operator=(const FlagReadback&) = delete;
  ~FlagReadback() {
    if (ev) (void)hipEventSynchronize(ev);
    if (ev) (void)hipEventDestroy(ev);
    if (h) (void)hipHostFree(h);
  }
  void fetch(const int* d, hipStream_t st) {
    AMB_HIP(hipMemcpyAsync(h, d, sizeof(int) * n, hipMemcpyDeviceToHost, st));
    AMB_HIP(hipEventRecord(ev, st));
  }
  std::vector<int> wait() const {
    AMB_HIP(hipEventSynchronize(ev));
    return std::vector<int>(h, h + n);
  }
};

void build_pair_work(ambddc_ctx& c, Level& L, int li, PairWork& W) {
  hipStream_t st = c.st;
  const LevelPlan& P = L.plan;
  const int m = W.m;
  W.np = int(P.pairs.size());
  std::vector<int64_t> Uoff(L.nsub + 1, 0), Yoff(L.nsub + 1, 0), Zoff(L.nsub + 1, 0);
  for (int s = 0; s < L.nsub; ++s) {
    const int64_t cols = int64_t(P.sub_npairs[s]) * 2 * m;
    Uoff[s + 1] = Uoff[s] + cols * L.nG[s];
    Yoff[s + 1] = Yoff[s] + cols * L.nl[s];
    Zoff[s + 1] = Zoff[s] + cols * L.nc[s];
  }
  std::vector<int> sh_s, sh_t, pc_s, pc_t, face_s, dptr{0}, didx;
  std::vector<int64_t> dcpos;
  // local interface index of a DOF (the interface DOFs are ascending)
  auto gfind = [&](int s, int dof) {
    const int* G0 = P.subs[s].dofs.data() + L.nI[s];
    return find_sorted(G0, G0 + L.nG[s], dof);
  };
  int64_t voff = 0, kpoff = 0, rboff = 0, fcoff = 0;
  W.hp.resize(W.np);
  L.fc_off.assign(W.np, 0);
  L.face_nf.assign(W.np, 0);
  for (int p = 0; p < W.np; ++p) {
    const Pair& Q = P.pairs[p];
    PairDev d{};
    d.s = Q.s;
    d.t = Q.t;
    d.nGs = L.nG[Q.s];
    d.nGt = L.nG[Q.t];
    d.gs_off = L.Goff[Q.s];
    d.gt_off = L.Goff[Q.t];
    const int n = d.nGs + d.nGt;
    d.v_off = voff;
    voff += int64_t(n) * 3 * m;
    d.us_off = Uoff[Q.s] + int64_t(Q.slot_s) * 2 * m * d.nGs;
    d.ut_off = Uoff[Q.t] + int64_t(Q.slot_t) * 2 * m * d.nGt;
    d.nls = L.nl[Q.s];
    d.nlt = L.nl[Q.t];
    d.ys_off = Yoff[Q.s] + int64_t(Q.slot_s) * 2 * m * d.nls;
    d.yt_off = Yoff[Q.t] + int64_t(Q.slot_t) * 2 * m * d.nlt;
    d.ncs = L.nc[Q.s];
    d.nct = L.nc[Q.t];
    d.zs_off = Zoff[Q.s] + int64_t(Q.slot_s) * 2 * m * d.ncs;
    d.zt_off = Zoff[Q.t] + int64_t(Q.slot_t) * 2 * m * d.nct;
    d.sh0 = int(sh_s.size());
    sh_s.insert(sh_s.end(), Q.sh_s.begin(), Q.sh_s.end());
    sh_t.insert(sh_t.end(), Q.sh_t.begin(), Q.sh_t.end());
    d.sh1 = int(sh_s.size());
    // rows of D: one per shared initial coarse DOF, supported on its glob's DOFs
    d.dr0 = int(dptr.size()) - 1;
    for (size_t r = 0; r < Q.dr_s.size(); ++r) {
      const Constraint& K = P.cons[P.subs[Q.s].cons[Q.dr_s[r]]];
      for (int j : K.dofs) {
        const int is = gfind(Q.s, j), it = gfind(Q.t, j);
        if (is < 0 || it < 0) throw Error(AMBDDC_E_INVALID_ARG, "shared constraint outside a pair");
        didx.push_back(is);
        dcpos.push_back(L.c_off[Q.s] + Q.dr_s[r] + int64_t(is) * L.nc[Q.s]);
        didx.push_back(d.nGs + it);
        dcpos.push_back(L.c_off[Q.t] + Q.dr_t[r] + int64_t(it) * L.nc[Q.t]);
      }
      dptr.push_back(int(didx.size()));
    }
    d.dr1 = int(dptr.size()) - 1;
    d.cs_off = L.c_off[Q.s];
    d.ct_off = L.c_off[Q.t];
    d.pcs0 = int(pc_s.size());
    pc_s.insert(pc_s.end(), Q.pc_s.begin(), Q.pc_s.end());
    d.pct0 = int(pc_t.size());
    pc_t.insert(pc_t.end(), Q.pc_t.begin(), Q.pc_t.end());
    d.ncp = Q.n_cp;
    d.kp_off = kpoff;
    kpoff += int64_t(Q.n_cp) * Q.n_cp;
    W.ncp_max = std::max(W.ncp_max, Q.n_cp);
    d.face0 = int(face_s.size());
    face_s.insert(face_s.end(), Q.face_s.begin(), Q.face_s.end());
    d.nface = int(Q.face_s.size());
    W.nface_max = std::max(W.nface_max, d.nface);
    d.nrb = Q.both_floating ? L.nrb : 0;
    d.rb_off = rboff;
    rboff += int64_t(n) * d.nrb;
    d.fc_off = fcoff;
    L.fc_off[p] = fcoff;
    L.face_nf[p] = d.nface;
    fcoff += int64_t(nsel_max(c.opt)) * d.nface;
    W.hp[p] = d;
  }
  if (W.ncp_max > PAIR_COARSE_MAX)
    throw Error(AMBDDC_E_INVALID_ARG, "pair coarse space larger than " +
                                          std::to_string(PAIR_COARSE_MAX) + " is not supported");
  W.dp.upload(W.hp, st);
  W.idx.sh_s.upload(sh_s, st);
  W.idx.sh_t.upload(sh_t, st);
  W.idx.dptr.upload(dptr, st);
  W.idx.didx.upload(didx, st);
  W.idx.dcpos.upload(dcpos, st);
  W.idx.pc_s.upload(pc_s, st);
  W.idx.pc_t.upload(pc_t, st);
  W.idx.face_s.upload(face_s, st);
  W.V.alloc(voff); W.AV.alloc(voff); W.BV.alloc(voff); W.T.alloc(2 * voff);
  W.V.zero(st); W.AV.zero(st); W.BV.zero(st);
  W.GA.alloc(size_t(W.np) * 9 * m * m);
  W.GB.alloc(size_t(W.np) * 9 * m * m);
  W.Cf.alloc(size_t(W.np) * 3 * m * 2 * m);
  W.Cxw.alloc(size_t(W.np) * m * m);
  W.lam.alloc(size_t(W.np) * m);
  W.lam.zero(st);
  W.resn.alloc(size_t(W.np) * m);
  W.U.alloc(std::max<int64_t>(Uoff[L.nsub], 1));
  W.Y.alloc(std::max<int64_t>(Yoff[L.nsub], 1));
  W.Zc.alloc(std::max<int64_t>(Zoff[L.nsub], 1));
  W.U.zero(st); W.Y.zero(st); W.Zc.zero(st);
  W.Kp.alloc(std::max<int64_t>(kpoff, 1));
  W.rb.alloc(std::max<int64_t>(rboff, 1));
  W.lnext.alloc(W.np);
  W.active.alloc(W.np);
  W.hist.alloc(size_t(4) * W.np);
  W.hist.zero(st);
  W.kout.alloc(W.np);
  W.nnull.alloc(W.np);
  L.fc.alloc(std::max<int64_t>(fcoff, 1));
  L.fc.zero(st);
  // grouped S / Z / Psi products: one GEMM per subdomain over all its pair
  // slots; a tile whose slots all belong to converged pairs is skipped
  std::vector<int> slot_off(L.nsub + 1, 0), slot_pair;
  for (int s = 0; s < L.nsub; ++s) slot_off[s + 1] = slot_off[s] + P.sub_npairs[s];
  slot_pair.assign(std::max(slot_off[L.nsub], 1), 0);
  for (int p = 0; p < W.np; ++p) {
    slot_pair[slot_off[P.pairs[p].s] + P.pairs[p].slot_s] = p;
    slot_pair[slot_off[P.pairs[p].t] + P.pairs[p].slot_t] = p;
  }
  W.slot_pair.upload(slot_pair, st);
  W.h_slot_off = slot_off;
  W.h_slot_pair = slot_pair;
  // tile shapes: measured on the first set-up of the handle, then reused
  const std::string lk = "L" + std::to_string(li) + ".";
  W.gS.reset(); W.gM1.reset(); W.gM2.reset();
  if (W.lo) {
    // the FP64 products have no work until pairs leave the FP32 phase: they
    // take the tile shapes the FP32 products measure
    W.gS.follow = &c.tune.emplace(lk + "S32", -1).first->second;
    W.gM1.follow = &c.tune.emplace(lk + "Z32", -1).first->second;
    W.gM2.follow = &c.tune.emplace(lk + "Psi32", -1).first->second;
  } else {
    W.gS.choice = &c.tune.emplace(lk + "S", -1).first->second;
    W.gM1.choice = &c.tune.emplace(lk + "Z", -1).first->second;
    W.gM2.choice = &c.tune.emplace(lk + "Psi", -1).first->second;
  }
  // phases (active[p]): 1 = FP32 products, 2 = FP64 products.  An FP64
  // product that overwrites (beta 0) runs after the FP32 one on every tile
  // with an FP64-phase slot; the accumulating Psi product runs each tile once
  // (in FP32 if any of its slots is in the FP32 phase: it is part of the
  // preconditioner, which only steers the search).
  W.gS.set_act(W.active.p, 2);
  W.gM1.set_act(W.active.p, 2);
  W.gM2.set_act(W.active.p, 2, W.lo ? 1 : 0);
  for (int s = 0; s < L.nsub; ++s) {
    const int cols = P.sub_npairs[s] * 2 * m;
    if (cols == 0) continue;
    const int N = L.augN[s], nI = L.nI[s], nG = L.nG[s], nl = L.nl[s], NN = L.naugN[s];
    const double* S = L.aug.p + L.aug_off[s] + nI + int64_t(nI) * N;
    const double* Tn = L.naug.p + L.naug_off[s] + nl + int64_t(nl) * NN;
    const int* sp = W.slot_pair.p + slot_off[s];
    W.gS.add(S, N, W.U.p + Uoff[s], nG, W.Y.p + Yoff[s], nl, nG, cols, nG, nullptr, sp, 2 * m);
    W.gM1.add(Tn, NN, W.U.p + Uoff[s], nG, W.Y.p + Yoff[s], nl, nl, cols, nG, nullptr, sp, 2 * m);
    if (L.nc[s] > 0)
      W.gM2.add(Tn + int64_t(nG) * NN, NN, W.Zc.p + Zoff[s], L.nc[s], W.Y.p + Yoff[s], nl, nG, cols,
                L.nc[s], nullptr, sp, 2 * m);
  }
  W.gS.finalize(st);
  W.gM1.finalize(st);
  W.gM2.finalize(st);
  if (W.lo) {
    // FP32 copies: S^s (nG x nG) and the Neumann inverse block (nl x nl)
    std::vector<int64_t> so(L.nsub + 1, 0), to(L.nsub + 1, 0);
    for (int s = 0; s < L.nsub; ++s) {
      const bool used = P.sub_npairs[s] > 0;
      so[s + 1] = so[s] + (used ? int64_t(L.nG[s]) * L.nG[s] : 0);
      to[s + 1] = to[s] + (used ? int64_t(L.nl[s]) * L.nl[s] : 0);
    }
    W.S32.alloc(size_t(std::max<int64_t>(so[L.nsub], 1)));
    W.T32.alloc(size_t(std::max<int64_t>(to[L.nsub], 1)));
    std::vector<CvtDesc> cv;
    for (int s = 0; s < L.nsub; ++s) {
      if (P.sub_npairs[s] == 0) continue;
      const int N = L.augN[s], nI = L.nI[s], nG = L.nG[s], nl = L.nl[s], NN = L.naugN[s];
      cv.push_back(CvtDesc{L.aug.p + L.aug_off[s] + nI + int64_t(nI) * N, N, nG, nG,
                           W.S32.p + so[s], nG, 0});
      cv.push_back(CvtDesc{L.naug.p + L.naug_off[s] + nl + int64_t(nl) * NN, NN, nl, nl,
                           W.T32.p + to[s], nl, 0});
    }
    convert_blocks_f32(cv, st);
    W.gS32.reset(); W.gM1_32.reset(); W.gM2_32.reset();
    W.gS32.choice = &c.tune.emplace(lk + "S32", -1).first->second;
    W.gM1_32.choice = &c.tune.emplace(lk + "Z32", -1).first->second;
    W.gM2_32.choice = &c.tune.emplace(lk + "Psi32", -1).first->second;
    W.U32.alloc(std::max<int64_t>(Uoff[L.nsub], 1));
    W.U32.zero(st);
    W.gS32.set_f32(true);       // S^s (FP32) times the FP32 slots
    W.gM1_32.set_f32(true);
    W.gM2_32.set_f32(false);    // the coarse slab stays FP64
    for (TunedGemm* g : {&W.gS32, &W.gM1_32, &W.gM2_32}) g->set_act(W.active.p, 1);
    for (int s = 0; s < L.nsub; ++s) {
      const int cols = P.sub_npairs[s] * 2 * m;
      if (cols == 0) continue;
      const int nG = L.nG[s], nl = L.nl[s];
      const float* S = W.S32.p + so[s];
      const float* Tn = W.T32.p + to[s];
      const int* sp = W.slot_pair.p + slot_off[s];
      // the FP32 GEMM reads A as plain column-major: the pointers carry floats
      const double* U32s = reinterpret_cast<const double*>(W.U32.p + Uoff[s]);
      W.gS32.add(reinterpret_cast<const double*>(S), nG, U32s, nG, W.Y.p + Yoff[s], nl, nG, cols,
                 nG, nullptr, sp, 2 * m);
      W.gM1_32.add(reinterpret_cast<const double*>(Tn), nl, U32s, nG, W.Y.p + Yoff[s], nl, nl,
                   cols, nG, nullptr, sp, 2 * m);
      if (L.nc[s] > 0)
        W.gM2_32.add(reinterpret_cast<const double*>(Tn + int64_t(nG) * nl), nl,
                     W.Zc.p + Zoff[s], L.nc[s], W.Y.p + Yoff[s], nl, nG, cols, L.nc[s], nullptr,
                     sp, 2 * m);
    }
    W.gS32.finalize(st);
    W.gM1_32.finalize(st);
    W.gM2_32.finalize(st);
  }
  // W <- W - X (BX^T W): B-orthogonalise the search directions against X
  W.orth_c = GemmOp();
  W.orth_u = GemmOp();
  W.orth_c.ta = true;
  W.orth_c.ksplit = 0;
  W.orth_u.narrow = (m <= 32);
  for (int p = 0; p < W.np; ++p) {
    const PairDev& d = W.hp[p];
    const int n = d.nGs + d.nGt;
    const int* fl = W.active.p + p;
    double* cx = W.Cxw.p + size_t(p) * m * m;
    W.orth_c.add(W.BV.p + d.v_off, n, W.V.p + d.v_off + int64_t(m) * n, n, cx, m, m, m, n, fl);
    W.orth_u.add(W.V.p + d.v_off, n, cx, m, W.V.p + d.v_off + int64_t(m) * n, n, n, m, m, fl);
  }
  W.orth_c.finalize(st);
  W.orth_u.finalize(st);
  // P <- P - X (BX^T P): keeps the P block from collapsing onto X near convergence
  W.orthp_c = GemmOp();
  W.orthp_u = GemmOp();
  W.orthp_c.ta = true;
  W.orthp_c.ksplit = 0;
  W.orthp_u.narrow = (m <= 32);
  for (int p = 0; p < W.np; ++p) {
    const PairDev& d = W.hp[p];
    const int n = d.nGs + d.nGt;
    const int* fl = W.active.p + p;
    double* cx = W.Cxw.p + size_t(p) * m * m;
    W.orthp_c.add(W.BV.p + d.v_off, n, W.V.p + d.v_off + int64_t(2 * m) * n, n, cx, m, m, m, n, fl);
    W.orthp_u.add(W.V.p + d.v_off, n, cx, m, W.V.p + d.v_off + int64_t(2 * m) * n, n, n, m, m, fl);
  }
  W.orthp_c.finalize(st);
  W.orthp_u.finalize(st);
  for (int v = 0; v < 3; ++v) {
    const int nb = (v + 1) * m;
    W.gram[v] = GemmOp();
    W.upd_v[v] = GemmOp();
    W.gram[v].ta = true;
    W.gram[v].ksplit = 0;
    W.upd_v[v].narrow = (2 * m <= 32);
    for (int p = 0; p < W.np; ++p) {
      const PairDev& d = W.hp[p];
      const int n = d.nGs + d.nGt;
      const int* fl = W.active.p + p;
      W.gram[v].add(W.V.p + d.v_off, n, W.AV.p + d.v_off, n, W.GA.p + size_t(p) * 9 * m * m, nb,
                    nb, nb, n, fl);
      W.gram[v].add(W.V.p + d.v_off, n, W.BV.p + d.v_off, n, W.GB.p + size_t(p) * 9 * m * m, nb,
                    nb, nb, n, fl);
      const double* cf = W.Cf.p + size_t(p) * 3 * m * 2 * m;
      double* t = W.T.p + 2 * d.v_off;
      W.upd_v[v].add(W.V.p + d.v_off, n, cf, 3 * m, t, n, n, 2 * m, nb, fl);
    }
    W.gram[v].finalize(st);
    W.upd_v[v].finalize(st);
  }
}

// Pseudo-inverses of the pair coarse matrices (see lobpcg.hip): null-space
// basis, augmented matrices, one batched factorisation, extraction.
void pair_pinv(ambddc_ctx& c, Level& L, PairWork& W, int li) {
  hipStream_t st = c.st;
  const size_t kp = W.Kp.n;
  W.Nb.alloc(kp);
  W.Nb.zero(st);
  W.Aug.alloc(4 * kp);
  lp_pair_null(W.dp.p, W.np, L.C.p, W.idx.pc_s.p, W.idx.pc_t.p, W.Kp.p, W.rb.p, W.Nb.p, st);
  lp_pinv_fill(W.dp.p, W.np, W.Kp.p, W.Nb.p, W.Aug.p, st);
  LdltOp ldl;
  SymOp sym;
  std::vector<int> of_desc;
  for (int p = 0; p < W.np; ++p) {
    const int n = W.hp[p].ncp;
    if (n == 0) continue;
    double* A = W.Aug.p + 4 * W.hp[p].kp_off;
    ldl.add(A, 2 * n, 2 * n, n, n);
    sym.add(A, 2 * n, n, n);
    of_desc.push_back(p);
  }
  auto fail = [&](int p, const std::string& why) {
    return Error(AMBDDC_E_ASSUMPTION, "Assumption 1 fails on level " + std::to_string(li + 1) +
                                          " pair (" + std::to_string(W.hp[p].s) + "," +
                                          std::to_string(W.hp[p].t) + "): " + why);
  };
  if (!of_desc.empty()) {
    ldl.finalize(st);
    sym.finalize(st);
    ldl.run(st);
    const int f = ldl.failed(st);
    if (f >= 0) throw fail(of_desc[f], "the pair coarse matrix has null vectors beyond the " +
                                           std::to_string(W.hp[of_desc[f]].nrb) + " rigid modes");
    sym.run(st);
  }
  lp_pinv_extract(W.dp.p, W.np, W.Aug.p, W.Nb.p, W.Kp.p, W.nnull.p, st);
  const std::vector<int> small = W.nnull.download(st);
  L.pair_nnull.assign(W.np, 0);
  for (int p = 0; p < W.np; ++p) {
    if (small[p] > 0)
      throw fail(p, std::to_string(small[p]) + " near-zero pivots beyond the " +
                        std::to_string(W.hp[p].nrb) + " rigid modes");
    L.pair_nnull[p] = W.hp[p].nrb;
  }
  W.Aug.release();
}

// Algorithmic work of S^s applied to the slots of the active pairs (W.act).
void apply_work(const Level& L, const PairWork& W, double& fl, double& by) {
  fl = 0.0;
  by = 0.0;
  for (int s = 0; s < L.nsub; ++s) {
    int na = 0;
    for (int j = W.h_slot_off[s]; j < W.h_slot_off[s + 1]; ++j)
      na += (W.act.empty() || W.act[W.h_slot_pair[j]]) ? 1 : 0;
    if (na == 0) continue;
    const double nG = L.nG[s], c = 2.0 * W.m * na;
    fl += 2.0 * nG * nG * c;
    by += 8.0 * (nG * nG + 2.0 * nG * c);
  }
}

void apply_ab(Level& L, PairWork& W, int col, hipStream_t st) {
  lp_to_slab(W.dp.p, W.np, W.V.p, W.m, col, true, L.diagG.p, W.idx.sh_s.p, W.idx.sh_t.p, W.U.p,
             W.lo ? W.U32.p : nullptr, W.active.p, st);
  if (W.kt->any()) {
    double fl, by;
    apply_work(L, W, fl, by);
    W.kt->begin("pair_apply", st);
    if (W.lo) W.gS32.run(1.0, 0.0, st);
    W.gS.run(1.0, 0.0, st);
    W.kt->end("pair_apply", st, fl, by);
  } else {
    if (W.lo) W.gS32.run(1.0, 0.0, st);
    W.gS.run(1.0, 0.0, st);
  }
  lp_from_slab_ab(W.dp.p, W.np, W.Y.p, W.m, col, W.AV.p, W.BV.p, L.diagG.p, W.idx.sh_s.p,
                  W.idx.sh_t.p, L.C.p, DRows{W.idx.dptr.p, W.idx.didx.p, W.idx.dcpos.p}, W.active.p,
                  st);
}

// Rayleigh-Ritz on span(V) and the new X, P (the products AV, BV are always
// recomputed explicitly from the current blocks, never updated implicitly:
// with coefficient jumps the implicit updates drift out of the factor space).
void rayleigh_ritz(Level& L, PairWork& W, int v, bool with_p, hipStream_t st) {
  const int nb = (v + 1) * W.m;
  if (W.kt->any()) {
    double fg = 0.0, bg = 0.0, nact = 0.0;
    for (int p = 0; p < W.np; ++p) {
      if (!W.act.empty() && !W.act[p]) continue;
      const double n = W.hp[p].nGs + W.hp[p].nGt;
      fg += 2.0 * 2.0 * n * nb * nb;
      bg += 2.0 * 8.0 * (2.0 * n * nb + double(nb) * nb);
      nact += 1.0;
    }
    const double b3 = double(nb) * nb * nb;
    const double frr = nact * (9.0 * b3 + 4.0 / 3.0 * b3 + 2.0 * double(nb) * nb * W.m);
    const double brr = nact * 8.0 * (2.0 * double(nb) * nb + 2.0 * double(nb) * W.m);
    W.kt->begin("pair_gram", st);
    W.gram[v].run(1.0, 0.0, st);
    W.kt->end("pair_gram", st, fg, bg);
    W.kt->begin("pair_rr", st);
    lp_rr(W.dp.p, W.np, W.GA.p, W.GB.p, nb, W.m, W.Cf.p, W.lam.p, W.active.p, st);
    W.kt->end("pair_rr", st, frr, brr);
  } else {
    W.gram[v].run(1.0, 0.0, st);
    lp_rr(W.dp.p, W.np, W.GA.p, W.GB.p, nb, W.m, W.Cf.p, W.lam.p, W.active.p, st);
  }
  W.upd_v[v].run(1.0, 0.0, st);
  lp_commit(W.dp.p, W.np, W.V.p, W.AV.p, W.BV.p, W.T.p, W.m, with_p, true, W.active.p, st);
  lp_project(W.dp.p, W.np, W.V.p, W.m, 0, L.C.p, DRows{W.idx.dptr.p, W.idx.didx.p, W.idx.dcpos.p}, W.rb.p, W.active.p,
             true, st);
  if (with_p)
    lp_project(W.dp.p, W.np, W.V.p, W.m, 2, L.C.p, DRows{W.idx.dptr.p, W.idx.didx.p, W.idx.dcpos.p}, W.rb.p,
               W.active.p, true, st);
}

int count_active(PairWork& W, hipStream_t st) {
  W.act = W.active.download(st);
  int n = 0;
  for (int x : W.act) n += x != 0;
  return n;
}

void adaptive_level(ambddc_ctx& c, Level& L, int li) {
  hipStream_t st = c.st;
  PairWork W;
  const int nev = nsel_max(c.opt);
  W.m = std::max(c.opt.lobpcg_block, nev + 1);
  if (W.m > 21)
    throw Error(AMBDDC_E_INVALID_ARG,
                "LOBPCG block (max(lobpcg_block, constraints per face + 1)) above 21 is not "
                "supported");
  L.m = W.m;
  W.kt = &c.kt;
  W.lo = c.opt.precision == 2;
  build_pair_work(c, L, li, W);
  if (W.np == 0) {
    L.omega = 0.0;
    return;
  }
  // pair rigid modes and pair coarse pseudo-inverses
  lp_pair_coarse(W.dp.p, W.np, L.kc.p, L.d_kc_off.p, W.idx.pc_s.p, W.idx.pc_t.p, W.Kp.p, st);
  lp_rigid(W.dp.p, W.np, L.rigid.p, L.ndof, L.Gdof.p, W.rb.p, st);
  pair_pinv(c, L, W, li);
  const int m = W.m;
  const int nconv = std::min(nev + 1, m);
  std::vector<int> ones(W.np, W.lo ? 1 : 2);
  W.active.upload(ones, st);
  W.act = ones;
  L.lobpcg_its32 = 0;
  // start block, projected; first Rayleigh-Ritz on X alone
  lp_random(W.dp.p, W.np, W.V.p, m, c.opt.seed + uint64_t(li) * 7919u, st);
  lp_project(W.dp.p, W.np, W.V.p, m, 0, L.C.p, DRows{W.idx.dptr.p, W.idx.didx.p, W.idx.dcpos.p}, W.rb.p, nullptr, true, st);
  apply_ab(L, W, 0, st);
  rayleigh_ritz(L, W, 0, false, st);
  FlagReadback flags(W.np);
  int it = 0;
  for (it = 1; it <= c.opt.lobpcg_maxit; ++it) {
    apply_ab(L, W, 0, st);
    if (it >= 2) {
      W.orthp_c.run(1.0, 0.0, st);
      W.orthp_u.run(-1.0, 1.0, st);
      apply_ab(L, W, 2, st);
    }
    lp_residual(W.dp.p, W.np, W.V.p, W.AV.p, W.BV.p, W.lam.p, m, nconv, c.opt.lobpcg_tol,
                LOBPCG_TOL32, W.active.p, W.resn.p, W.hist.p, st);
    // The new flags travel to the host while the stream already runs the
    // next block: every kernel and product below skips converged pairs on
    // the device, so when no pair is left the block is launches without work.
    flags.fetch(W.active.p, st);
    // W = M R  (eq. bddc_pair: Z^st R + Psi (Psi^T S Psi)^+ Psi^T R, then Pi and deflation)
    lp_to_slab(W.dp.p, W.np, W.V.p, m, 1, false, L.diagG.p, W.idx.sh_s.p, W.idx.sh_t.p, W.U.p,
               W.lo ? W.U32.p : nullptr, W.active.p, st);
    if (W.lo) W.gM1_32.run(1.0, 0.0, st);
    W.gM1.run(1.0, 0.0, st);
    lp_coarse(W.dp.p, W.np, W.Y.p, m, W.Kp.p, W.idx.pc_s.p, W.idx.pc_t.p, W.Zc.p, W.ncp_max,
              W.active.p, st);
    if (W.lo) W.gM2_32.run(1.0, 1.0, st);
    W.gM2.run(1.0, 1.0, st);
    lp_from_slab_w(W.dp.p, W.np, W.Y.p, m, W.V.p, W.active.p, st);
    lp_project(W.dp.p, W.np, W.V.p, m, 1, L.C.p, DRows{W.idx.dptr.p, W.idx.didx.p, W.idx.dcpos.p}, W.rb.p, W.active.p,
               true, st);
    W.orth_c.run(1.0, 0.0, st);
    W.orth_u.run(-1.0, 1.0, st);
    double fl0 = 0.0, by0 = 0.0, fl1 = 0.0, by1 = 0.0;
    if (W.kt->any()) apply_work(L, W, fl0, by0);   // what apply_ab records (previous flags)
    apply_ab(L, W, 1, st);
    W.act = flags.wait();
    if (W.kt->any()) {
      apply_work(L, W, fl1, by1);
      W.kt->amend("pair_apply", fl1 - fl0, by1 - by0);
    }
    int nact = 0, n32 = 0;
    for (int x : W.act) {
      nact += x != 0;
      n32 += x == 1;
    }
    if (n32 > 0) ++L.lobpcg_its32;
    if (nact == 0) break;
    rayleigh_ritz(L, W, it == 1 ? 1 : 2, true, st);
  }
  if (it > c.opt.lobpcg_maxit) apply_ab(L, W, 0, st);   // products of the final X
  L.lobpcg_its = std::min(it, c.opt.lobpcg_maxit);
  L.n_unconv = count_active(W, st);
  lp_select(W.dp.p, W.np, W.AV.p, W.lam.p, m, nev, c.opt.tau, c.opt.fixed_per_face,
            W.idx.face_s.p, W.nface_max, L.fc.p,
            W.kout.p, W.lnext.p, st);
  L.pair_k = W.kout.download(st);
  L.pair_lnext = W.lnext.download(st);
  L.pair_lam = W.lam.download(st);
  L.pair_res = W.resn.download(st);
  std::vector<int> act = W.active.download(st);
  L.pair_conv.resize(W.np);
  for (int p = 0; p < W.np; ++p) L.pair_conv[p] = act[p] == 0;
  L.omega = 0.0;
  L.n_added = 0;
  for (int p = 0; p < W.np; ++p) {
    L.omega = std::max(L.omega, L.pair_lnext[p]);
    L.n_added += L.pair_k[p];
  }
}

// ---------------------------------------------------------------------------
// next level, top coarse problem, preconditioner application
// ---------------------------------------------------------------------------

void build_top(ambddc_ctx& c) {
  hipStream_t st = c.st;
  Level& L = *c.L.back();
  Top& T = c.top;
  T = Top();
  T.n = L.ncoarse;
  if (T.n == 0) return;
  const int n = T.n, N = 2 * n;
  T.aug.alloc(size_t(N) * N);
  T.aug.zero(st);
  std::vector<int64_t> edptr(L.nsub + 1, 0);
  std::vector<int> edofs;
  for (int s = 0; s < L.nsub; ++s) {
    const auto& cs = L.plan.subs[s].cons;
    edofs.insert(edofs.end(), cs.begin(), cs.end());
    edptr[s + 1] = int64_t(edofs.size());
  }
  std::vector<int> tgt(L.nsub, 0);
  std::vector<LocalIndex> loc(1);
  std::vector<int> ident(n);
  std::iota(ident.begin(), ident.end(), 0);
  loc[0].build(ident);
  std::vector<int64_t> koff(L.kc_off.begin(), L.kc_off.end() - 1);
  build_assembly(T.am, L.nsub, tgt, edptr, edofs, koff, loc, {n}, st);
  T.d_off.upload(std::vector<int64_t>{0}, st);
  T.d_ld.upload(std::vector<int>{N}, st);
  launch_assemble(T.am, L.kc.p, T.d_off.p, T.d_ld.p, T.aug.p, st);
  if (n <= 4096) {
    T.Kc.alloc(size_t(n) * n);
    DBuf<int64_t> so, dof;
    DBuf<int> sl, r0, rr, dl;
    so.upload(std::vector<int64_t>{0}, st);
    dof.upload(std::vector<int64_t>{0}, st);
    sl.upload(std::vector<int>{N}, st);
    r0.upload(std::vector<int>{0}, st);
    rr.upload(std::vector<int>{n}, st);
    dl.upload(std::vector<int>{n}, st);
    launch_copy_block(1, so.p, sl.p, r0.p, rr.p, rr.p, dof.p, dl.p, T.aug.p, T.Kc.p, st);
  }
  {
    DBuf<int> nid, c0, r0;
    nid.upload(std::vector<int>{n}, st);
    c0.upload(std::vector<int>{0}, st);
    r0.upload(std::vector<int>{n}, st);
    launch_aug_identity(1, T.d_off.p, T.d_ld.p, nid.p, c0.p, r0.p, st, T.aug.p);
  }
  T.ldl.add(T.aug.p, N, N, n, n);
  T.ldl.finalize(st);
  T.sym.add(T.aug.p, N, n, n);
  T.sym.finalize(st);
  T.ldl.run(st);
  check_ldlt(T.ldl, st, "coarsest factorisation", int(c.L.size()));
  T.sym.run(st);
}

void build_top_solve(ambddc_ctx& c) {
  Top& T = c.top;
  if (T.n == 0) return;
  Level& L = *c.L.back();
  const int n = T.n, N = 2 * n;
  T.solve = GemvOp();
  T.solve.add(T.aug.p + n + int64_t(n) * N, N, n, n, L.w_rc.p, n, L.w_uc.p, n);
  T.solve.finalize(c.st);
}

void ensure_workspace(ambddc_ctx& c, int nrhs) {
  bool changed = false;
  for (auto& lp : c.L) {
    Level& L = *lp;
    if (L.nrhs_cap < nrhs) {
      alloc_workspace(L, nrhs);
      alloc_coarse_workspace(L, nrhs);
      changed = true;
    }
  }
  if (changed) {
    for (auto& lp : c.L) build_apply_ops(c, *lp);
    build_top_solve(c);
  }
}

// Alg. 1 on level li: r (ld ldr) -> u (ld ldu).  harmonic: r is zero on the
// level's interior DOFs (every residual of the PCG below, which starts from
// the interior solution), so the interior pre-correction u_I and the part of
// the post-correction it feeds are exactly zero and are not computed.
void apply_level(ambddc_ctx& c, int li, const double* r, int64_t ldr, double* u, int64_t ldu,
                 int nrhs, bool harmonic = false) {
  hipStream_t st = c.st;
  Level& L = *c.L[li];
  // interior pre-correction and updated residual on the interface
  if (!harmonic) {
    launch_gather(int(L.nI_tot), L.Imap.p, r, ldr, L.w_xI.p, L.nI_tot, nrhs, 1.0, st);
    L.g1.run(1.0, 0.0, nrhs, st);
  }
  launch_interface_residual(int(L.nG_tot), L.Gdof.p, L.incptr.p, L.incpos.p, L.g2y1.p, L.delta.p,
                            r, ldr, harmonic ? nullptr : L.w_y1.p, L.y1_tot, L.w_rBs.p, L.nG_tot,
                            nrhs, st);
  // substructure corrections and coarse right-hand side
  if (!L.g2z.empty() && nrhs <= SymvOp::MAX_RHS) {
    L.g2z.run(1.0, 0.0, nrhs, st);
    L.g2c.run(1.0, 0.0, nrhs, st);
  } else {
    L.g2.run(1.0, 0.0, nrhs, st);
  }
  if (L.ncoarse > 0) {
    launch_segment_sum(L.ncoarse, L.cptr.p, L.cpos.p, L.w_y2.p, L.y2_tot, L.w_rc.p, L.ncoarse, nrhs,
                       -1.0, st);
    if (li + 1 == int(c.L.size())) c.top.solve.run(-1.0, 0.0, nrhs, st);
    else apply_level(c, li + 1, L.w_rc.p, L.ncoarse, L.w_uc.p, L.ncoarse, nrhs);
    launch_gather(int(L.cl_tot), L.clmap.p, L.w_uc.p, L.ncoarse, L.w_ucl.p, L.cl_tot, nrhs, 1.0, st);
  }
  L.g3.run(-1.0, -1.0, nrhs, st);
  // averaging, interior post-correction, combination
  launch_average(int(L.nG_tot), L.Gdof.p, L.incptr.p, L.incpos.p, L.g2y2.p, L.delta.p, L.w_y2.p,
                 L.y2_tot, L.w_uBs.p, L.nG_tot, u, ldu, nrhs, st);
  if (L.plain && !harmonic) throw Error(AMBDDC_E_STATE, "interior pre-correction on a plain level");
  L.g4.run(L.plain ? -1.0 : 1.0, harmonic ? 0.0 : -1.0, nrhs, st);
  launch_move(int(L.nI_tot), L.I2y1.p, L.w_y1.p, L.y1_tot, L.Imap.p, u, ldu, nrhs, st);
}

// x = [K_II^{-1} f_I; 0] on level 0 (every subdomain's interior solve, the
// rows of y1 that the pre-correction writes): f - K x is zero on the
// interiors up to rounding.
void interior_solve(ambddc_ctx& c, const double* f, double* x, int nrhs) {
  hipStream_t st = c.st;
  Level& L = *c.L[0];
  const int64_t n = L.ndof;
  launch_fill(x, size_t(n) * nrhs, 0.0, st);
  launch_gather(int(L.nI_tot), L.Imap.p, f, n, L.w_xI.p, L.nI_tot, nrhs, 1.0, st);
  if (L.plain) {
    L.trsv.run(nrhs, st);
    launch_move(int(L.nI_tot), L.Iiota.p, L.w_xI.p, L.nI_tot, L.Imap.p, x, n, nrhs, st);
    return;
  }
  L.g1.run(-1.0, 0.0, nrhs, st);
  launch_move(int(L.nI_tot), L.I2y1.p, L.w_y1.p, L.y1_tot, L.Imap.p, x, n, nrhs, st);
}

// x_I += K_II^{-1} r_I on level 0 for the columns with mask != 0.
void interior_correct(ambddc_ctx& c, const double* r, double* x, int nrhs, const int* mask) {
  hipStream_t st = c.st;
  Level& L = *c.L[0];
  const int64_t n = L.ndof;
  launch_gather(int(L.nI_tot), L.Imap.p, r, n, L.w_xI.p, L.nI_tot, nrhs, 1.0, st);
  if (L.plain) {
    L.trsv.run(nrhs, st);
    launch_move_add_masked(int(L.nI_tot), L.Iiota.p, L.w_xI.p, L.nI_tot, L.Imap.p, x, n, nrhs,
                           mask, st);
    return;
  }
  L.g1.run(-1.0, 0.0, nrhs, st);
  launch_move_add_masked(int(L.nI_tot), L.I2y1.p, L.w_y1.p, L.y1_tot, L.Imap.p, x, n, nrhs, mask,
                         st);
}

void next_level(ambddc_ctx& c, int li) {
  hipStream_t st = c.st;
  Level& L = *c.L[li];
  auto N = std::make_unique<Level>();
  std::string e = next_level_input(L.plan, c.parents[li], N->plan.in);
  if (!e.empty()) throw Error(AMBDDC_E_INVALID_ARG, e);
  e = build_level_plan(N->plan, c.opt.initial_constraints, c.opt.keep_edges != 0);
  if (!e.empty()) throw Error(AMBDDC_E_INVALID_ARG, e);
  std::vector<int64_t> koff(L.kc_off.begin(), L.kc_off.end() - 1);
  build_level_maps(c, *N, L.kc.p, koff, false);
  // coarse values of the level-li rigid modes
  N->rigid.alloc(size_t(N->ndof) * N->nrb);
  {
    std::vector<int> sub_of(N->ndof, -1), row_of(N->ndof, -1);
    for (int s = 0; s < L.nsub; ++s) {
      const auto& cs = L.plan.subs[s].cons;
      for (int r = 0; r < int(cs.size()); ++r)
        if (sub_of[cs[r]] < 0) { sub_of[cs[r]] = s; row_of[cs[r]] = r; }
    }
    DBuf<int> ds, dr, dnc;
    DBuf<int64_t> dco, dgo;
    ds.upload(sub_of, st);
    dr.upload(row_of, st);
    dnc.upload(L.nc, st);
    dco.upload(std::vector<int64_t>(L.c_off.begin(), L.c_off.end() - 1), st);
    dgo.upload(std::vector<int64_t>(L.Goff.begin(), L.Goff.end() - 1), st);
    launch_coarse_rigid(N->ndof, N->nrb, ds.p, dr.p, dco.p, dnc.p, L.d_nG.p, dgo.p, L.Gdof.p, L.C.p,
                        L.rigid.p, L.ndof, N->rigid.p, st);
  }
  c.L.push_back(std::move(N));
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void setup_impl(ambddc_ctx& c, const double* coeff, const double* nu) {
  hipStream_t st = c.st;
  const double t0 = now_s();
  c.ready = false;
  ++c.setup_epoch;   // the operators the PCG graphs point at are rebuilt
  std::memset(&c.stats, 0, sizeof(c.stats));
  {
    const int big = std::numeric_limits<int>::max();
    DBuf<int> bad;
    bad.upload(std::vector<int>{big, big}, st);
    launch_check_coeff(c.n_elems, coeff, c.dof == 3 ? nu : nullptr, bad.p, st);
    const std::vector<int> b = bad.download(st);
    if (b[0] != big)
      throw Error(AMBDDC_E_INVALID_ARG,
                  "coefficient of element " + std::to_string(b[0] - 1) + " is not a finite number");
    if (b[1] != big)
      throw Error(AMBDDC_E_INVALID_ARG, "Poisson ratio of element " + std::to_string(b[1] - 1) +
                                            " is not in (-1, 1/2)");
  }
  const int ne = 8 * c.dof;
  launch_element_matrices(c.coords.p, c.en.p, coeff, nu, c.n_elems, c.dof, c.Ke.p, st);
  launch_csr_values(c.csr, c.edofs.p, ne, c.Ke.p, c.csr_vals.p, st);
  c.L.resize(1);
  Level& L0 = *c.L[0];
  L0.plan = c.plan0;
  L0.nrhs_cap = 0;
  const bool adaptive = (c.opt.tau > 0.0 && std::isfinite(c.opt.tau)) || c.opt.fixed_per_face > 0;
  double tph[8] = {0};
  for (int li = 0; li < c.levels - 1; ++li) {
    if (li > 0) next_level(c, li - 1);
    Level& L = *c.L[li];
    AMB_HIP(hipStreamSynchronize(st));
    double ta = now_s();
    numeric_schur(c, L, li);
    AMB_HIP(hipStreamSynchronize(st));
    double tb = now_s();
    tph[0] += tb - ta;
    build_constraint_maps(c, L);
    numeric_neumann(c, L, li);
    AMB_HIP(hipStreamSynchronize(st));
    double tcc = now_s();
    tph[1] += tcc - tb;
    if (adaptive) {
      adaptive_level(c, L, li);
      AMB_HIP(hipStreamSynchronize(st));
      double td = now_s();
      tph[2] += td - tcc;
      NeumannPrev prev = keep_neumann(L);
      add_adaptive_constraints(L.plan, L.pair_k);
      build_constraint_maps(c, L);
      neumann_bordered(c, L, li, prev);
      AMB_HIP(hipStreamSynchronize(st));
      tph[4] += now_s() - td;
    }
  }
  double te = now_s();
  build_top(c);
  AMB_HIP(hipStreamSynchronize(st));
  tph[5] += now_s() - te;
  for (auto& lp : c.L) lp->nrhs_cap = 0;
  ensure_workspace(c, 1);
  AMB_HIP(hipStreamSynchronize(st));
  c.stats.levels = int(c.L.size());
  c.stats.n_free = c.L[0]->ndof;
  for (int i = 0; i < int(c.L.size()) && i < 8; ++i) {
    const Level& L = *c.L[i];
    c.stats.n_sub[i] = L.nsub;
    c.stats.n_pairs[i] = int(L.plan.pairs.size());
    c.stats.n_coarse[i] = L.ncoarse;
    c.stats.n_adaptive[i] = L.n_added;
    c.stats.lobpcg_iters[i] = L.lobpcg_its;
    c.stats.lobpcg_iters_fp32[i] = L.lobpcg_its32;
    c.stats.n_unconverged[i] = L.n_unconv;
    c.stats.omega_tilde[i] = L.omega;
  }
  for (int k = 0; k < 6; ++k) c.stats.t_phase[k] = tph[k];
  c.stats.t_phase[6] = now_s() - t0;
  c.ready = true;
}

// ---------------------------------------------------------------------------
// PCG
// ---------------------------------------------------------------------------

// Device memory of one PCG solve (all pointers on the device): the columns
// r, z, p, q (n x nrhs each), the dot products, reduction partials, the
// coefficient histories of the Lanczos estimate and the column flags.
struct PcgWork {
  double *r, *z, *p, *q;
  double* dot;     // 8 nrhs: rz, beta, pq, rr, rzn, ff
  double* part;    // 256 nrhs reduction partials
  double *ah, *bh; // ldh x nrhs coefficient histories
  double* lz;      // 3 nrhs + 2 ldh nrhs: condition estimates and Sturm workspace
  double* tprev;   // nrhs: true residual at the column's last check
  int *act, *nal, *meets, *repl, *stall, *cnt;   // nrhs each; cnt: 8 + nrhs (cnt[4]: iteration,
                                                 // cnt[8..]: one-launch dot counters)
  int ldh;
};

// Doubles and ints one PcgWork needs.
void pcg_work_size(int64_t n, int nrhs, int ldh, int64_t& nd, int64_t& ni) {
  nd = 4 * n * nrhs + 8 * int64_t(nrhs) + 256 * int64_t(nrhs) + 2 * int64_t(ldh) * nrhs +
       3 * int64_t(nrhs) + 2 * int64_t(ldh) * nrhs + int64_t(nrhs);
  ni = 6 * int64_t(nrhs) + 8;
}

// Carve a PcgWork out of nd doubles at d and ni ints at ip.
PcgWork pcg_work_carve(double* d, int* ip, int64_t n, int nrhs, int ldh) {
  PcgWork w{};
  const size_t nn = size_t(n) * nrhs;
  w.r = d; d += nn;
  w.z = d; d += nn;
  w.p = d; d += nn;
  w.q = d; d += nn;
  w.dot = d; d += 8 * nrhs;
  w.part = d; d += 256 * nrhs;
  w.ah = d; d += size_t(ldh) * nrhs;
  w.bh = d; d += size_t(ldh) * nrhs;
  w.lz = d; d += 3 * size_t(nrhs) + 2 * size_t(ldh) * nrhs;
  w.tprev = d;
  w.act = ip; ip += nrhs;
  w.nal = ip; ip += nrhs;
  w.meets = ip; ip += nrhs;
  w.repl = ip; ip += nrhs;
  w.stall = ip; ip += nrhs;
  w.cnt = ip;
  w.ldh = ldh;
  return w;
}

// PCG (x0 = [K_II^{-1} f_I; 0]) with Alg. 1 as preconditioner, columns in lockstep, flags on
// the device; the host reads four counters per iteration.  A column whose
// recursive residual meets rtol is checked against its recomputed true
// residual f - K x: it stops if that meets rtol too; otherwise the true
// residual replaces the recursive one and the column restarts from it
// (p = z: the old direction is not conjugate to the new residual), unless
// the true residual fell by less than half since its previous check, when
// the column stops as stalled at the FP64 floor of f - K x.  Allocates
// nothing when `timed` is false (the preconditioner's workspace for nrhs
// columns must exist).  Returns the number of columns that did not converge
// (stalled or still active at maxit).
int pcg_core(ambddc_ctx& c, const PcgWork& w, const double* f, int nrhs, double rtol, int maxit,
             double* x, int* its, double* cond, bool timed) {
  hipStream_t st = c.st;
  const double t0 = now_s();
  const int n = c.L[0]->ndof;
  const size_t nn = size_t(n) * nrhs;
  const double rtol2 = rtol * rtol;
  double* rz = w.dot;                 // rz[0:nrhs], beta scratch rz[nrhs:2nrhs]
  double* pq = w.dot + 2 * nrhs;
  double* rr = w.dot + 3 * nrhs;
  double* rzn = w.dot + 4 * nrhs;
  double* ff = w.dot + 5 * nrhs;
  int* hc = c.hcnt;   // pinned: the copy runs in stream order without a staging sync
  auto fetch_cnt = [&]() {
    AMB_HIP(hipMemcpyAsync(hc, w.cnt, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    AMB_HIP(hipEventRecord(c.ev_cnt, st));
  };
  auto read_cnt = [&]() {
    fetch_cnt();
    AMB_HIP(hipEventSynchronize(c.ev_cnt));
  };
  // x0 = the interior solution, so that every residual of the iteration is
  // zero on the level-1 interiors (discrete harmonic iterates: PCG on the
  // interface problem of the Schur complement, which is the problem the
  // BDDC preconditioner is built for)
  // The recursive residual keeps its interior part exactly zero (K p of a
  // harmonic p is zero there in exact arithmetic; its rounding, about eps
  // kappa(K_II), is dropped): it is the interface residual.  The true
  // residual, interiors included, is what stops a column.
  Level& L1 = *c.L[0];
  interior_solve(c, f, x, nrhs);
  launch_spmv(c.csr, c.csr_vals.p, x, w.r, nrhs, st);
  launch_sub(nn, f, w.r, w.r, st);
  launch_zero_rows(int(L1.nI_tot), L1.Imap.p, w.r, n, nrhs, nullptr, st);
  launch_dot_cols(n, nrhs, f, f, w.part, ff, st);
  launch_pcg_init_flags(nrhs, ff, w.act, w.nal, w.repl, w.stall, w.tprev, w.cnt, st);
  // algorithmic work of one preconditioner application (timing only)
  double apf = 0.0, apb = 0.0;
  const bool kt = timed && c.kt.any();
  if (kt) {
    // level 1 reads K_II^{-1} K_IG (FP64 in every precision), Z and Psi (no
    // pre-correction: harmonic residuals); deeper levels also K_II^{-1} and
    // K_GI K_II^{-1}
    const double esz = c.opt.precision >= 1 ? 4.0 : 8.0;
    double ent = 0.0, byt = 0.0;
    for (size_t li = 0; li < c.L.size(); ++li) {
      const Level& Lv = *c.L[li];
      for (int s = 0; s < Lv.nsub; ++s) {
        const double nI = Lv.nI[s], nG = Lv.nG[s], ncs = Lv.nc[s];
        const double pre = li == 0 ? 0.0 : nI * nI + nI * nG;
        // Z is symmetric: the FP64 path for up to 3 right-hand sides reads
        // its lower triangle
        const double zent = (c.opt.precision == 0 && nrhs <= SymvOp::MAX_RHS)
                                ? nG * (nG + 1.0) / 2.0 : nG * nG;
        const double post = nI * nG, sub = nG * nG + 2.0 * nG * ncs;
        ent += pre + post + sub;
        byt += esz * (pre + sub - nG * nG + zent) + (li == 0 ? 8.0 : esz) * post;
      }
    }
    const double top = double(c.top.n) * c.top.n;   // the coarsest inverse stays FP64
    apf = 2.0 * (ent + top) * nrhs;
    apb = byt + 8.0 * top + 48.0 * double(n) * nrhs;
  }
  auto precondition = [&]() {
    if (kt) c.kt.begin("bddc_apply", st);
    apply_level(c, 0, w.r, n, w.z, n, nrhs, true);
    if (kt) c.kt.end("bddc_apply", st, apf, apb);
  };
  precondition();
  launch_dot_cols(n, nrhs, w.r, w.z, w.part, rz, st);
  launch_copy(w.p, w.z, nn, st);
  read_cnt();
  int* itp = w.cnt + 4;   // device iteration counter (the history slot of the step)
  // one step's mat-vec through the convergence flags, the counters copied
  // back at its end; then the preconditioner of the new residual
  // The step's dot products in one launch each for up to 3 columns; with
  // more, the blocks' cache write-backs cost more than the second launch.
  int* dcnt = w.cnt + 8;
  auto dots = [&](const double* a, const double* b, double* out, hipStream_t s) {
    if (nrhs <= 3) launch_dot_cols_fin(n, nrhs, a, b, w.part, dcnt, out, s);
    else launch_dot_cols(n, nrhs, a, b, w.part, out, s);
  };
  auto step1 = [&](hipStream_t s) {
    launch_spmv(c.csr, c.csr_vals.p, w.p, w.q, nrhs, s, c.imask.p);   // interior rows zero
    dots(w.p, w.q, pq, s);
    launch_pcg_update_x_r(n, nrhs, rz, pq, w.act, x, w.r, w.p, w.q, w.ah, itp, w.ldh, s);
    dots(w.r, w.r, rr, s);
    launch_pcg_meets(nrhs, rr, ff, rtol2, w.act, w.nal, w.meets, w.cnt, itp, s);
    AMB_HIP(hipMemcpyAsync(hc, w.cnt, sizeof(int) * 4, hipMemcpyDeviceToHost, s));
  };
  auto step2 = [&](hipStream_t s) {
    apply_level(c, 0, w.r, n, w.z, n, nrhs, true);   // on c.st, which is s here
    dots(w.r, w.z, rzn, s);
  };
  // When switched on, without kernel-class timing (whose events cannot sit
  // in a graph) and for up to 3 right-hand sides (no product builds anything
  // on first use), the two parts run as HIP graphs from the second step on:
  // captured once per set-up and solve arguments, replayed every step.
  const bool use_graph = (c.graphs & 1) && timed && !c.kt.any() && nrhs <= SymvOp::MAX_RHS;
  const void* key[5] = {f, x, w.r, w.cnt, reinterpret_cast<const void*>(intptr_t(nrhs))};
  auto capture = [&](auto&& fn) {
    hipStream_t cs = c.cap_st;
    hipStream_t saved = c.st;
    AMB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    c.st = cs;
    hipGraph_t g = nullptr;
    try {
      fn(cs);
    } catch (...) {
      c.st = saved;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    c.st = saved;
    AMB_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    AMB_HIP(err);
    return e;
  };
  auto graphs_ready = [&]() {
    if (c.pcg_g1 && c.pcg_gepoch == c.setup_epoch && c.pcg_grtol == rtol &&
        std::equal(key, key + 5, c.pcg_gkey))
      return;
    c.drop_pcg_graphs();
    if (!c.cap_st) AMB_HIP(hipStreamCreateWithFlags(&c.cap_st, hipStreamNonBlocking));
    c.pcg_g1 = capture(step1);
    c.pcg_g2 = capture(step2);
    std::copy(key, key + 5, c.pcg_gkey);
    c.pcg_grtol = rtol;
    c.pcg_gepoch = c.setup_epoch;
  };
  int nact = hc[1];
  int repl = 0;
  for (int it = 0; it < maxit && nact > 0; ++it) {
    // The counters travel back while the preconditioner of this residual is
    // already queued: it stays valid unless a check below replaces columns of r.
    if (use_graph && it > 0) {
      graphs_ready();
      AMB_HIP(hipGraphLaunch(c.pcg_g1, st));
      AMB_HIP(hipEventRecord(c.ev_cnt, st));
      AMB_HIP(hipGraphLaunch(c.pcg_g2, st));
    } else {
      step1(st);
      AMB_HIP(hipEventRecord(c.ev_cnt, st));
      if (kt) c.kt.begin("bddc_apply", st);
      step2(st);
      if (kt) c.kt.end("bddc_apply", st, apf, apb);
    }
    AMB_HIP(hipEventSynchronize(c.ev_cnt));
    if (hc[0] > 0) {
      // The recursive residual drifts from f - K x by rounding (most on
      // ill-conditioned problems): recompute the true residual (q is free
      // here) and stop only the columns it confirms.
      // The iteration never corrects the interiors (harmonic residuals), so
      // the rounding of the interior updates accumulates there (about eps
      // kappa(K_II) per step): the checked columns first re-solve their
      // interiors from the true residual, x_I += K_II^{-1} (f - K x)_I.
      launch_spmv(c.csr, c.csr_vals.p, x, w.q, nrhs, st);
      launch_sub(nn, f, w.q, w.q, st);
      interior_correct(c, w.q, x, nrhs, w.meets);
      launch_spmv(c.csr, c.csr_vals.p, x, w.q, nrhs, st);
      launch_sub(nn, f, w.q, w.q, st);
      launch_dot_cols(n, nrhs, w.q, w.q, w.part, rr, st);
      launch_pcg_true(nrhs, rr, ff, rtol2, w.act, w.meets, w.repl, w.stall, w.tprev, w.cnt, st);
      launch_copy_cols(n, nrhs, w.q, w.r, w.repl, st);
      launch_zero_rows(int(L1.nI_tot), L1.Imap.p, w.r, n, nrhs, w.repl, st);
      read_cnt();
      nact = hc[1];
      repl += hc[2];
      if (nact == 0) break;
      if (hc[2] > 0) {   // replaced residual columns: precondition them again
        precondition();
        launch_dot_cols(n, nrhs, w.r, w.z, w.part, rzn, st);
      }
    }
    launch_pcg_update_p(n, nrhs, rzn, rz, w.act, w.repl, w.p, w.z, w.bh, itp, w.ldh, st);
  }
  // iterations per column and the true residuals ||f - K x|| / ||f||
  int hnal[16];
  double htt[16], hff[16];
  launch_spmv(c.csr, c.csr_vals.p, x, w.q, nrhs, st);
  launch_sub(nn, f, w.q, w.q, st);
  launch_dot_cols(n, nrhs, w.q, w.q, w.part, rr, st);
  AMB_HIP(hipMemcpyAsync(hnal, w.nal, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
  AMB_HIP(hipMemcpyAsync(htt, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  AMB_HIP(hipMemcpyAsync(hff, ff, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  if (cond) {
    launch_lanczos_cond(nrhs, w.nal, w.ah, w.bh, w.ldh, w.lz, st);
    AMB_HIP(hipMemcpyAsync(cond, w.lz, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  }
  AMB_HIP(hipStreamSynchronize(st));
  c.n_last_res = nrhs;
  for (int k = 0; k < nrhs; ++k) {
    its[k] = hnal[k];
    c.last_res[k] = hff[k] > 0.0 ? std::sqrt(htt[k] / hff[k]) : 0.0;
  }
  c.pcg_repl = repl;
  c.stats.t_phase[7] = now_s() - t0;
  c.stats.pcg_replacements = repl;
  c.stats.pcg_stalled = hc[3];
  return nact + hc[3];
}

int pcg_impl(ambddc_ctx& c, const double* f, int nrhs, double rtol, int maxit, double* x,
             int* its, double* cond) {
  ensure_workspace(c, nrhs);
  const int n = c.L[0]->ndof;
  if (c.pcg_cap < nrhs || c.pcg_maxit < maxit) {
    c.pcg_cap = std::max(c.pcg_cap, nrhs);
    c.pcg_maxit = std::max(c.pcg_maxit, maxit);
    int64_t nd, ni;
    pcg_work_size(n, c.pcg_cap, c.pcg_maxit, nd, ni);
    c.pwd.alloc(size_t(nd));
    c.pwi.alloc(size_t(ni));
  }
  const PcgWork w = pcg_work_carve(c.pwd.p, c.pwi.p, n, nrhs, c.pcg_maxit);
  return pcg_core(c, w, f, nrhs, rtol, maxit, x, its, cond, true);
}

// ---------------------------------------------------------------------------
// PCG scratch of ambddc_solve_noalloc: one fixed device array per GPU
// ---------------------------------------------------------------------------

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) double scratch[NOALLOC_BYTES / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};   // device address of `scratch` per device id

// The device address of this device's copy of `scratch`, looked up once per
// device (the array's name in host code is only a stand-in for it).
void* scratch_address() {
  int dev = 0;
  AMB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(AMBDDC_E_DEVICE, "device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(AMBDDC_E_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

int pcg_noalloc(ambddc_ctx& c, const double* f, int nrhs, double rtol, int maxit, double* x,
                int* its, double* cond) {
  if (nrhs > 3)
    throw Error(AMBDDC_E_INVALID_ARG, "ambddc_solve_noalloc takes 1 to 3 right-hand sides");
  for (auto& lp : c.L)
    if (lp->nrhs_cap < nrhs)
      throw Error(AMBDDC_E_INVALID_ARG,
                  "the preconditioner's workspace holds " + std::to_string(lp->nrhs_cap) +
                      " right-hand side(s); run ambddc_solve once with " + std::to_string(nrhs) +
                      " to prepare it");
  const int n = c.L[0]->ndof;
  int64_t nd, ni;
  pcg_work_size(n, nrhs, maxit, nd, ni);
  const size_t dbytes = (size_t(nd) * sizeof(double) + 255) / 256 * 256;
  const size_t need = dbytes + size_t(ni) * sizeof(int);
  if (need > NOALLOC_BYTES)
    throw Error(AMBDDC_E_INVALID_ARG,
                "solve needs " + std::to_string(need) + " bytes of scratch (n_free " +
                    std::to_string(n) + ", nrhs " + std::to_string(nrhs) + ", maxit " +
                    std::to_string(maxit) + "); the fixed array holds " +
                    std::to_string(NOALLOC_BYTES));
  char* base = static_cast<char*>(scratch_address());
  const PcgWork w = pcg_work_carve(reinterpret_cast<double*>(base),
                                   reinterpret_cast<int*>(base + dbytes), n, nrhs, maxit);
  return pcg_core(c, w, f, nrhs, rtol, maxit, x, its, cond, false);
}

std::string noconv_message(const ambddc_ctx& c, int left) {
  double worst = 0.0;
  for (int k = 0; k < c.n_last_res; ++k) worst = std::max(worst, c.last_res[k]);
  std::string m = std::to_string(left) + " right-hand side(s) did not reach rtol: ";
  if (c.stats.pcg_stalled > 0)
    m += std::to_string(c.stats.pcg_stalled) +
         " stalled (the true residual stopped falling above rtol: the FP64 rounding floor of "
         "f - K x on this system)";
  else
    m += "maxit reached";
  char buf[64];
  std::snprintf(buf, sizeof(buf), "; largest true residual %.3e", worst);
  return m + buf;
}

int guard(const std::function<void()>& fn) {
  try {
    fn();
    g_err.clear();
    return AMBDDC_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_err = e.what();
    return AMBDDC_E_DEVICE;
  }
}

// Entry points on a handle: device memory is cached for the handle's stream.
int hguard(ambddc_handle h, const std::function<void()>& fn) {
  DevStreamScope ds(h ? h->st : nullptr);
  return guard(fn);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void ambddc_default_options(ambddc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tau = 10.0;
  o->nev_max = 10;
  o->lobpcg_maxit = 100;
  o->lobpcg_block = 16;
  o->lobpcg_tol = 1e-7;
  o->precision = 0;
  o->initial_constraints = AMBDDC_INIT_CE;
  o->keep_edges = 0;
  o->fixed_per_face = 0;
  o->seed = 12345;
  o->stream = nullptr;
}

const char* ambddc_last_error(void) { return g_err.c_str(); }

ambddc_status ambddc_analyze(const ambddc_mesh* mesh, const ambddc_decomp* dec,
                             int32_t initial_constraints, ambddc_analysis* out, int32_t* sizes,
                             int32_t n_sub_cap) {
  return ambddc_status(guard([&] {
    if (!mesh || !dec || !out || !mesh->elem_nodes || !mesh->dirichlet || !dec->elem_to_sub)
      throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (mesh->dof_per_node != 1 && mesh->dof_per_node != 3)
      throw Error(AMBDDC_E_INVALID_ARG, "dof_per_node must be 1 or 3");
    LevelPlan P;
    std::vector<int> fof;
    std::string e = level1_input(mesh->n_nodes, mesh->n_elems, mesh->dof_per_node, mesh->elem_nodes,
                                 mesh->dirichlet, dec->elem_to_sub, P.in, fof);
    if (!e.empty()) throw Error(AMBDDC_E_INVALID_ARG, e);
    e = build_level_plan(P, initial_constraints, false);
    if (!e.empty()) throw Error(AMBDDC_E_INVALID_ARG, e);
    std::memset(out, 0, sizeof(*out));
    out->n_free = P.in.n_dof;
    out->n_sub = P.in.n_sub;
    for (const auto& g : P.globs) {
      out->n_interface += int(g.dofs.size());
      if (g.type == GLOB_FACE) out->n_faces++;
      else if (g.type == GLOB_EDGE) out->n_edges++;
      else out->n_corners++;
    }
    out->n_coarse_initial = P.n_cons_initial;
    out->n_pairs = int(P.pairs.size());
    if (sizes) {
      if (n_sub_cap < P.in.n_sub) throw Error(AMBDDC_E_INVALID_ARG, "sub_sizes too small");
      for (int s = 0; s < P.in.n_sub; ++s) {
        sizes[2 * s] = P.subs[s].nI;
        sizes[2 * s + 1] = P.subs[s].nG;
      }
    }
  }));
}

ambddc_status ambddc_create(const ambddc_mesh* mesh, const ambddc_decomp* dec,
                            const ambddc_options* opt, ambddc_handle* out) {
  return ambddc_status(guard([&] {
    if (!mesh || !dec || !opt || !out) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (mesh->dof_per_node != 1 && mesh->dof_per_node != 3)
      throw Error(AMBDDC_E_INVALID_ARG, "dof_per_node must be 1 or 3");
    if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || !mesh->coords || !mesh->elem_nodes ||
        !mesh->dirichlet)
      throw Error(AMBDDC_E_INVALID_ARG, "empty or missing mesh arrays");
    if (dec->levels < 2 || dec->levels > 8 || !dec->elem_to_sub)
      throw Error(AMBDDC_E_INVALID_ARG, "levels must be in 2..8 with an element map");
    if (dec->levels > 2 && !dec->parents) throw Error(AMBDDC_E_INVALID_ARG, "missing parent maps");
    if (opt->precision < 0 || opt->precision > 2)
      throw Error(AMBDDC_E_INVALID_ARG, "precision must be 0, 1 or 2");
    if (opt->nev_max < 0 || opt->lobpcg_maxit < 1 || opt->lobpcg_tol <= 0.0 ||
        opt->fixed_per_face < 0)
      throw Error(AMBDDC_E_INVALID_ARG, "bad LOBPCG options");
    if (opt->initial_constraints < 0 || opt->initial_constraints > 2)
      throw Error(AMBDDC_E_INVALID_ARG, "initial_constraints must be AMBDDC_INIT_CE, _CEF or _C");
    DevStreamScope ds(static_cast<hipStream_t>(opt->stream));
    auto c = std::make_unique<ambddc_ctx>();
    c->opt = *opt;
    c->st = static_cast<hipStream_t>(opt->stream);
    AMB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->hcnt), 4 * sizeof(int),
                          hipHostMallocDefault));
    AMB_HIP(hipEventCreateWithFlags(&c->ev_cnt, hipEventDisableTiming));
    c->n_nodes = mesh->n_nodes;
    c->n_elems = mesh->n_elems;
    c->dof = mesh->dof_per_node;
    c->levels = dec->levels;
    std::string e = level1_input(mesh->n_nodes, mesh->n_elems, mesh->dof_per_node, mesh->elem_nodes,
                                 mesh->dirichlet, dec->elem_to_sub, c->plan0.in, c->free_of_full);
    if (!e.empty()) throw Error(AMBDDC_E_INVALID_ARG, e);
    e = build_level_plan(c->plan0, opt->initial_constraints, opt->keep_edges != 0);
    if (!e.empty()) throw Error(AMBDDC_E_INVALID_ARG, e);
    // parent maps, checked level by level
    int nsub = c->plan0.in.n_sub;
    for (int i = 0; i < dec->levels - 2; ++i) {
      if (!dec->parents[i]) throw Error(AMBDDC_E_INVALID_ARG, "null parent map");
      std::vector<int> p(dec->parents[i], dec->parents[i] + nsub);
      int np = 0;
      for (int v : p) {
        if (v < 0) throw Error(AMBDDC_E_INVALID_ARG, "negative parent id");
        np = std::max(np, v + 1);
      }
      c->parents.push_back(p);
      nsub = np;
    }
    hipStream_t st = c->st;
    std::vector<double> xy(mesh->coords, mesh->coords + size_t(mesh->n_nodes) * 3);
    c->coords.upload(xy, st);
    std::vector<int> en(mesh->elem_nodes, mesh->elem_nodes + size_t(mesh->n_elems) * 8);
    c->en.upload(en, st);
    c->edofs.upload(c->plan0.in.elem_dofs, st);
    const int ne = 8 * c->dof;
    c->Ke.alloc(size_t(mesh->n_elems) * ne * ne);
    // global CSR pattern of the free DOFs and row incidences
    {
      const int nn = mesh->n_nodes, d = c->dof;
      std::vector<int> nptr(nn + 1, 0);
      for (int e2 = 0; e2 < mesh->n_elems; ++e2)
        for (int a = 0; a < 8; ++a) nptr[en[size_t(e2) * 8 + a] + 1]++;
      for (int i = 0; i < nn; ++i) nptr[i + 1] += nptr[i];
      std::vector<int> nel(nptr[nn]), nla(nptr[nn]);
      {
        std::vector<int> f(nptr.begin(), nptr.end() - 1);
        for (int e2 = 0; e2 < mesh->n_elems; ++e2)
          for (int a = 0; a < 8; ++a) {
            const int nd = en[size_t(e2) * 8 + a];
            nel[f[nd]] = e2;
            nla[f[nd]++] = a;
          }
      }
      const int nf = c->plan0.in.n_dof;
      std::vector<int> rowptr(nf + 1, 0), cols;
      std::vector<int64_t> incp(nf + 1, 0);
      std::vector<int> ie, ia;
      std::vector<int> row_of_free(nf);
      for (int nd = 0; nd < nn; ++nd)
        for (int q = 0; q < d; ++q) {
          const int fi = c->free_of_full[size_t(nd) * d + q];
          if (fi < 0) continue;
          std::vector<int> cc;
          for (int k = nptr[nd]; k < nptr[nd + 1]; ++k) {
            const int e2 = nel[k];
            for (int b = 0; b < ne; ++b) {
              const int cj = c->plan0.in.elem_dofs[size_t(e2) * ne + b];
              if (cj >= 0) cc.push_back(cj);
            }
            ie.push_back(e2);
            ia.push_back(nla[k] * d + q);
          }
          std::sort(cc.begin(), cc.end());
          cc.erase(std::unique(cc.begin(), cc.end()), cc.end());
          cols.insert(cols.end(), cc.begin(), cc.end());
          rowptr[fi + 1] = int(cols.size());
          incp[fi + 1] = int64_t(ie.size());
        }
      c->csr.n = nf;
      c->csr.nnz = int64_t(cols.size());
      for (int i = 0; i < nf; ++i)
        c->csr.maxrow = std::max(c->csr.maxrow, rowptr[i + 1] - rowptr[i]);
      c->csr.rowptr.upload(rowptr, st);
      c->csr.cols.upload(cols, st);
      c->csr.inc_ptr.upload(incp, st);
      c->csr.inc_e.upload(ie, st);
      c->csr.inc_a.upload(ia, st);
      c->csr_vals.alloc(cols.size());
    }
    // level-1 structures that do not depend on the coefficients or constraints
    auto L0 = std::make_unique<Level>();
    L0->plan = c->plan0;
    std::vector<int64_t> eoff(mesh->n_elems);
    for (int e2 = 0; e2 < mesh->n_elems; ++e2) eoff[e2] = int64_t(e2) * ne * ne;
    build_level_maps(*c, *L0, c->Ke.p, eoff, true);
    // rows of the level-1 interiors, which the PCG mat-vec writes as zero
    c->imask.alloc(size_t(std::max(L0->ndof, 1)));
    c->imask.zero(st);
    launch_mark_rows(int(L0->nI_tot), L0->Imap.p, c->imask.p, st);
    L0->rigid.alloc(size_t(L0->ndof) * L0->nrb);
    {
      DBuf<int> fof;
      fof.upload(c->free_of_full, st);
      launch_rigid_level1(mesh->n_nodes, c->dof, c->coords.p, fof.p, L0->ndof, L0->rigid.p, st);
      AMB_HIP(hipStreamSynchronize(st));
    }
    c->L.push_back(std::move(L0));
    dev_stream_acquire(c->st);
    *out = c.release();
  }));
}

ambddc_status ambddc_setup(ambddc_handle h, const double* coeff, const double* nu) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !coeff) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (h->dof == 3 && !nu) throw Error(AMBDDC_E_INVALID_ARG, "elasticity needs nu");
    setup_impl(*h, coeff, nu);
  }));
}

ambddc_status ambddc_setup_log10(ambddc_handle h, const double* theta, const double* nu) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !theta) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (h->dof == 3 && !nu) throw Error(AMBDDC_E_INVALID_ARG, "elasticity needs nu");
    if (h->coeff_buf.n != size_t(h->n_elems)) h->coeff_buf.alloc(h->n_elems);
    launch_pow10(size_t(h->n_elems), theta, h->coeff_buf.p, h->st);
    setup_impl(*h, h->coeff_buf.p, nu);
  }));
}

ambddc_status ambddc_misfit(ambddc_handle h, const double* X, const double* Xobs, int32_t nrhs,
                            double* R, double* J) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !X || !Xobs || !R) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (h->L.empty()) throw Error(AMBDDC_E_STATE, "misfit needs a created handle");
    if (nrhs < 1 || nrhs > 16) throw Error(AMBDDC_E_INVALID_ARG, "nrhs must be in 1..16");
    const int n = h->L[0]->ndof;
    launch_sub(size_t(n) * nrhs, X, Xobs, R, h->st);
    if (J) {
      if (h->mis_part.n < size_t(256) * 16) h->mis_part.alloc(size_t(256) * 16);
      if (h->mis_out.n < 16) h->mis_out.alloc(16);
      launch_dot_cols(n, nrhs, R, R, h->mis_part.p, h->mis_out.p, h->st);
      std::vector<double> v = h->mis_out.download(h->st);
      double s = 0.0;
      for (int k = 0; k < nrhs; ++k) s += v[k];
      *J = 0.5 * s;
    } else {
      AMB_HIP(hipStreamSynchronize(h->st));
    }
  }));
}

ambddc_status ambddc_solve(ambddc_handle h, const double* rhs, int32_t nrhs, double rtol,
                           int32_t maxit, double* x, int32_t* iterations, double* cond) {
  int code = guard([&] {
    if (!h || !rhs || !x) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (!h->ready) throw Error(AMBDDC_E_STATE, "solve called before a successful setup");
    if (nrhs < 1 || nrhs > 16) throw Error(AMBDDC_E_INVALID_ARG, "nrhs must be in 1..16");
    if (maxit < 1 || !(rtol > 0.0)) throw Error(AMBDDC_E_INVALID_ARG, "bad rtol or maxit");
    std::vector<int> its(nrhs, 0);
    std::vector<double> cd(nrhs, 0.0);
    const int left = pcg_impl(*h, rhs, nrhs, rtol, maxit, x, its.data(), cd.data());
    if (iterations) std::copy(its.begin(), its.end(), iterations);
    if (cond) std::copy(cd.begin(), cd.end(), cond);
    if (left > 0) throw Error(AMBDDC_E_NO_CONVERGENCE, noconv_message(*h, left));
  });
  return ambddc_status(code);
}

ambddc_status ambddc_solve_noalloc(ambddc_handle h, const double* rhs, int32_t nrhs, double rtol,
                                   int32_t maxit, double* x, int32_t* iterations, double* cond) {
  int code = guard([&] {
    if (!h || !rhs || !x) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (!h->ready) throw Error(AMBDDC_E_STATE, "solve called before a successful setup");
    if (nrhs < 1) throw Error(AMBDDC_E_INVALID_ARG, "nrhs must be >= 1");
    if (maxit < 1 || !(rtol > 0.0)) throw Error(AMBDDC_E_INVALID_ARG, "bad rtol or maxit");
    int its[16] = {};
    double cd[16] = {};
    const int left = pcg_noalloc(*h, rhs, nrhs, rtol, maxit, x, its, cd);
    if (iterations) std::copy(its, its + nrhs, iterations);
    if (cond) std::copy(cd, cd + nrhs, cond);
    if (left > 0) throw Error(AMBDDC_E_NO_CONVERGENCE, noconv_message(*h, left));
  });
  return ambddc_status(code);
}

ambddc_status ambddc_element_gradient(ambddc_handle h, const double* X, const double* Lam,
                                      int32_t nrhs, double* grad) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !X || !Lam || !grad) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (!h->ready) throw Error(AMBDDC_E_STATE, "gradient needs a setup");
    launch_element_gradient(h->n_elems, 8 * h->dof, h->L[0]->ndof, nrhs, h->edofs.p, h->Ke.p, X, Lam,
                            grad, h->st);
    AMB_HIP(hipStreamSynchronize(h->st));
  }));
}

ambddc_status ambddc_last_residual(ambddc_handle h, int32_t nrhs, double* res) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !res) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (nrhs != h->n_last_res)
      throw Error(AMBDDC_E_STATE, "nrhs differs from the last solve (" +
                                      std::to_string(h->n_last_res) + ")");
    std::copy(h->last_res, h->last_res + nrhs, res);
  }));
}

ambddc_status ambddc_get_stats(ambddc_handle h, ambddc_stats* out) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !out) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    *out = h->stats;
  }));
}

static const char* const kTimingClasses[] = {"pair_rr", "pair_apply", "pair_gram", "schur",
                                             "bddc_apply"};

static bool known_class(const std::string& name) {
  for (const char* k : kTimingClasses)
    if (name == k) return true;
  return false;
}

ambddc_status ambddc_timing_enable(ambddc_handle h, const char* classes) {
  return ambddc_status(hguard(h, [&] {
    if (!h) throw Error(AMBDDC_E_INVALID_ARG, "null handle");
    const std::string list = classes ? classes : "";
    size_t a = 0;
    while (a < list.size()) {
      size_t b = list.find(',', a);
      if (b == std::string::npos) b = list.size();
      const std::string name = list.substr(a, b - a);
      if (!name.empty() && !known_class(name))
        throw Error(AMBDDC_E_INVALID_ARG, "unknown timing class '" + name + "'");
      a = b + 1;
    }
    h->kt.enable(list);
  }));
}

ambddc_status ambddc_set_graphs(ambddc_handle h, int32_t flags) {
  return ambddc_status(hguard(h, [&] {
    if (!h) throw Error(AMBDDC_E_INVALID_ARG, "null handle");
    if (flags & ~1) throw Error(AMBDDC_E_INVALID_ARG, "unknown graph flags");
    h->graphs = flags;
    if (!(flags & 1)) h->drop_pcg_graphs();
  }));
}

ambddc_status ambddc_timing_read(ambddc_handle h, const char* cls, int32_t* launches,
                                 double* total_ms, double* flops, double* bytes) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !cls) throw Error(AMBDDC_E_INVALID_ARG, "null argument");
    if (!known_class(cls)) throw Error(AMBDDC_E_INVALID_ARG, std::string("unknown timing class '") + cls + "'");
    h->kt.collect();
    const int i = h->kt.find(cls);
    KTimer::Acc a;
    if (i >= 0) a = h->kt.acc[i];
    if (launches) *launches = a.launches;
    if (total_ms) *total_ms = a.ms;
    if (flops) *flops = a.flops;
    if (bytes) *bytes = a.bytes;
  }));
}

ambddc_status ambddc_level_info(ambddc_handle h, int32_t level, int32_t* n_dof, int32_t* n_sub,
                                int32_t* n_pairs, int32_t* n_coarse) {
  return ambddc_status(hguard(h, [&] {
    if (!h || level < 0 || level >= int(h->L.size()))
      throw Error(AMBDDC_E_INVALID_ARG, "bad handle or level");
    const Level& L = *h->L[level];
    if (n_dof) *n_dof = L.ndof;
    if (n_sub) *n_sub = L.nsub;
    if (n_pairs) *n_pairs = int(L.plan.pairs.size());
    if (n_coarse) *n_coarse = L.ncoarse;
  }));
}

ambddc_status ambddc_sub_dofs(ambddc_handle h, int32_t level, int32_t sub, int32_t* dofs,
                              int32_t* n_I, int32_t* n_G) {
  return ambddc_status(hguard(h, [&] {
    if (!h || level < 0 || level >= int(h->L.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad level");
    const Level& L = *h->L[level];
    if (sub < 0 || sub >= L.nsub) throw Error(AMBDDC_E_INVALID_ARG, "bad subdomain");
    const Sub& S = L.plan.subs[sub];
    if (n_I) *n_I = S.nI;
    if (n_G) *n_G = S.nG;
    if (dofs) std::copy(S.dofs.begin(), S.dofs.end(), dofs);
  }));
}

ambddc_status ambddc_get_schur(ambddc_handle h, int32_t level, int32_t sub, double* S) {
  return ambddc_status(hguard(h, [&] {
    if (!h || !S || level < 0 || level >= int(h->L.size()))
      throw Error(AMBDDC_E_INVALID_ARG, "bad argument");
    const Level& L = *h->L[level];
    if (sub < 0 || sub >= L.nsub || !L.aug.p) throw Error(AMBDDC_E_INVALID_ARG, "bad subdomain");
    const int nG = L.nG[sub], nI = L.nI[sub], N = L.augN[sub];
    AMB_HIP(hipMemcpy2DAsync(S, sizeof(double) * nG,
                             L.aug.p + L.aug_off[sub] + nI + int64_t(nI) * N, sizeof(double) * N,
                             sizeof(double) * nG, nG, hipMemcpyDeviceToHost, h->st));
    AMB_HIP(hipStreamSynchronize(h->st));
  }));
}

ambddc_status ambddc_pair_info(ambddc_handle h, int32_t level, int32_t pair, int32_t* s, int32_t* t,
                               int32_t* n_face) {
  return ambddc_status(hguard(h, [&] {
    if (!h || level < 0 || level >= int(h->L.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad level");
    const Level& L = *h->L[level];
    if (pair < 0 || pair >= int(L.plan.pairs.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad pair");
    const Pair& P = L.plan.pairs[pair];
    if (s) *s = P.s;
    if (t) *t = P.t;
    if (n_face) *n_face = int(P.face_dofs.size());
  }));
}

ambddc_status ambddc_get_pair_result(ambddc_handle h, int32_t level, int32_t pair, int32_t cap,
                                     int32_t* block, double* lam, double* resid, int32_t* k,
                                     double* lam_next, int32_t* iters, int32_t* converged) {
  return ambddc_status(hguard(h, [&] {
    if (!h || level < 0 || level >= int(h->L.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad level");
    const Level& L = *h->L[level];
    if (pair < 0 || pair >= int(L.plan.pairs.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad pair");
    if (L.pair_k.empty()) throw Error(AMBDDC_E_STATE, "no adaptive results on this level");
    if (block) *block = L.m;
    if ((lam || resid) && cap < L.m)
      throw Error(AMBDDC_E_INVALID_ARG, "result arrays hold " + std::to_string(cap) +
                                            " entries; the block has " + std::to_string(L.m));
    if (lam) std::copy(L.pair_lam.begin() + size_t(pair) * L.m,
                       L.pair_lam.begin() + size_t(pair + 1) * L.m, lam);
    if (resid) std::copy(L.pair_res.begin() + size_t(pair) * L.m,
                         L.pair_res.begin() + size_t(pair + 1) * L.m, resid);
    if (k) *k = L.pair_k[pair];
    if (lam_next) *lam_next = L.pair_lnext[pair];
    if (iters) *iters = L.lobpcg_its;
    if (converged) *converged = L.pair_conv[pair];
  }));
}

ambddc_status ambddc_get_face_constraints(ambddc_handle h, int32_t level, int32_t pair, double* rows,
                                          int32_t* face_dofs) {
  return ambddc_status(hguard(h, [&] {
    if (!h || level < 0 || level >= int(h->L.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad level");
    const Level& L = *h->L[level];
    if (pair < 0 || pair >= int(L.plan.pairs.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad pair");
    const Pair& P = L.plan.pairs[pair];
    if (face_dofs) std::copy(P.face_dofs.begin(), P.face_dofs.end(), face_dofs);
    if (rows && !L.pair_k.empty() && L.pair_k[pair] > 0) {
      const size_t cnt = size_t(L.pair_k[pair]) * P.face_dofs.size();
      AMB_HIP(hipMemcpyAsync(rows, L.fc.p + L.fc_off[pair], sizeof(double) * cnt,
                             hipMemcpyDeviceToHost, h->st));
      AMB_HIP(hipStreamSynchronize(h->st));
    }
  }));
}

ambddc_status ambddc_get_coarse_element(ambddc_handle h, int32_t level, int32_t sub, double* Kc,
                                        int32_t* nc) {
  return ambddc_status(hguard(h, [&] {
    if (!h || level < 0 || level >= int(h->L.size())) throw Error(AMBDDC_E_INVALID_ARG, "bad level");
    const Level& L = *h->L[level];
    if (sub < 0 || sub >= L.nsub || L.nc.empty()) throw Error(AMBDDC_E_INVALID_ARG, "bad subdomain");
    if (nc) *nc = L.nc[sub];
    if (Kc && L.nc[sub] > 0) {
      AMB_HIP(hipMemcpyAsync(Kc, L.kc.p + L.kc_off[sub], sizeof(double) * L.nc[sub] * L.nc[sub],
                             hipMemcpyDeviceToHost, h->st));
      AMB_HIP(hipStreamSynchronize(h->st));
    }
  }));
}

ambddc_status ambddc_get_top_coarse(ambddc_handle h, double* Kc, int32_t* n) {
  return ambddc_status(hguard(h, [&] {
    if (!h) throw Error(AMBDDC_E_INVALID_ARG, "null handle");
    if (n) *n = h->top.n;
    if (Kc && h->top.n > 0) {
      if (!h->top.Kc.p) throw Error(AMBDDC_E_STATE, "coarse matrix too large to keep a copy");
      AMB_HIP(hipMemcpyAsync(Kc, h->top.Kc.p, sizeof(double) * h->top.Kc.n, hipMemcpyDeviceToHost,
                             h->st));
      AMB_HIP(hipStreamSynchronize(h->st));
    }
  }));
}

void ambddc_destroy(ambddc_handle h) {
  if (!h) return;
  hipStream_t st = h->st;
  {
    DevStreamScope ds(st);
    (void)hipStreamSynchronize(st);
    delete h;
  }
  dev_stream_release(st);
}

}  // extern "C"
