// Launchers of the HIP kernels used by the set-up and solve drivers.
#pragma once
#include "common.hpp"
#include "dense.hpp"

namespace ambddc {

// Column-gather assembly of dense subdomain blocks from element matrices.
struct AssemblyMaps {
  int ncols = 0;
  int max_ne = 0;                  // largest element matrix order
  DBuf<int> col_sub, col_j;        // per assembled column: subdomain, local column
  DBuf<int64_t> inc_ptr;           // per column: incident (element, local index)
  DBuf<int> inc_e, inc_a;
  DBuf<int64_t> emat_off;          // per element: offset of its matrix
  DBuf<int> elem_ne;               // per element: matrix order
  DBuf<int64_t> eloc_off;          // per element: offset into eloc
  DBuf<int> eloc;                  // element DOF -> local row in its subdomain (-1 fixed)
};

struct CsrMaps {
  int n = 0;
  int maxrow = 0;   // longest row
  int64_t nnz = 0;
  DBuf<int> rowptr, cols;
  DBuf<int64_t> inc_ptr;
  DBuf<int> inc_e, inc_a;
};

void launch_element_matrices(const double* coords, const int* en, const double* coeff,
                             const double* nu, int n_elem, int dof, double* Ke, hipStream_t st);
void launch_assemble(const AssemblyMaps& m, const double* emat, const int64_t* tgt_off,
                     const int* tgt_ld, double* tgt, hipStream_t st);
// Every column of the target blocks written whole (zeros included): the
// blocks need no fill beforehand; tgt_ld[s] <= ldmax <= 8192, elements of at
// most 64 DOFs.
void launch_assemble_cols(const AssemblyMaps& m, int ldmax, const double* emat,
                          const int64_t* tgt_off, const int* tgt_ld, double* tgt, hipStream_t st);
void launch_csr_values(const CsrMaps& m, const int* edofs, int ne, const double* Ke, double* vals,
                       hipStream_t st);
// zmask (optional, n bytes): rows with a nonzero byte are written as zero
void launch_spmv(const CsrMaps& m, const double* vals, const double* x, double* y, int nrhs,
                 hipStream_t st, const unsigned char* zmask = nullptr);
// mask[pos[i]] = 1 for i < n
void launch_mark_rows(int n, const int64_t* pos, unsigned char* mask, hipStream_t st);
void launch_element_gradient(int n_elem, int ne, int n, int nrhs, const int* edofs, const double* Ke,
                             const double* X, const double* L, double* grad, hipStream_t st);

// ---- level structures (bddc.hip) ----

// identity blocks of the augmented subdomain matrices [[K, I_I^T],[I_I, 0]]
void launch_aug_identity(int nsub, const int64_t* off, const int* ld, const int* nrow_id,
                         const int* col0, const int* row0, hipStream_t st, double* A);
// stacked copies: dst[k] = src[idx[k]] (per column r, strides ldd / lds)
void launch_gather(int n, const int64_t* idx, const double* src, int64_t lds, double* dst,
                   int64_t ldd, int nrhs, double scale, hipStream_t st);
void launch_scatter(int n, const int64_t* idx, const double* src, int64_t lds, double* dst,
                    int64_t ldd, int nrhs, hipStream_t st);
// weights: delta[k] = diag[k] / sum over copies of the DOF
void launch_weights(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                    const double* diag, double* delta, hipStream_t st);
// r_B restricted and weighted: out[k] = delta[k] * (r[gdof[k]] + sum_{copies} y[g2y[c]])
// (y may be null: a residual that is zero on the interiors needs no correction)
void launch_interface_residual(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                               const int64_t* g2y, const double* delta, const double* r,
                               int64_t ldr, const double* y, int64_t ldy, double* out,
                               int64_t ldo, int nrhs, hipStream_t st);
// averaging: out[k] = sum_{copies c of gdof[k]} delta[c] * w[g2w[c]]; dst[gdof] too
void launch_average(int nG, const int* gdof, const int* inc_ptr, const int* inc_pos,
                    const int64_t* g2w, const double* delta, const double* w, int64_t ldw,
                    double* out, int64_t ldo, double* dst, int64_t ldd, int nrhs, hipStream_t st);
// sum of stacked entries into coarse DOFs: rc[c] = scale * sum_{q in ptr[c]} src[pos[q]]
void launch_segment_sum(int n, const int* ptr, const int64_t* pos, const double* src, int64_t lds,
                        double* dst, int64_t ldd, int nrhs, double scale, hipStream_t st);
// dense constraint matrices from entry lists
// One adaptive row of C^s: C[dst + amap[map + q] * ldc] = fc[src + q], q < nf.
struct AdaptRow {
  int64_t dst, src, map;
  int ldc, nf;
};
void launch_fill_adaptive(int nrows, const AdaptRow* rows, const int* amap, const double* fc,
                          double* C, hipStream_t st);
void launch_fill_values(int n, const int64_t* pos, const double* val, double* dst, hipStream_t st);
// Neumann augmented matrices
struct NeuDesc {
  const double* S;  int lds;   // S^s (ld lds)
  const double* C;  int nc;    // C^s (nc x nG, ld nc)
  double* A;        int lda;   // augmented matrix of order 2(nG+nc)
  int nG;
  const double* rho;           // scalar on device (unused by the fill)
  int col_start;
};
// Fills [[S, C^T, I, 0], [C, 0, 0, I], [I, 0, 0, 0], [0, I, 0, 0]] (the
// rho C^T C term of the (1,1) block is added separately).
void launch_neumann_fill(const NeuDesc* d, int nd, int ncols, hipStream_t st);
// dst = sqrt(scale[s]) src on the entries [off[s], off[s] + cnt[s]) of every s
void launch_scale_sqrt_sub(int nsub, const int64_t* off, const int64_t* cnt, const double* scale,
                           const double* src, double* dst, hipStream_t st);
void launch_diag_mean(int nsub, const int64_t* off, const int* ld, const int* n0, const int* n,
                      const double* A, double* out, hipStream_t st);
// K_c^s = trailing(n_G: , n_G:) - rho E  copied compact, E the identity on
// the first nrho[s] constraint rows (all rows when nrho is null)
void launch_extract_kc(int nsub, const int64_t* naug_off, const int* naug_ld, const int* nG,
                       const int* nc, const int64_t* kc_off, const double* rho, const int* nrho,
                       const double* naug, double* kc, hipStream_t st);
// The border of a bordered symmetric inverse T (ld ldt) of order nl + k:
// T[0:nl, nl:] = -W, T[nl:, 0:nl] = -W^T, T[nl:, nl:] = -Tsc.
struct BorderDesc {
  double* T;
  const double* W;
  const double* Tsc;
  int ldt, ldw, lds, nl, k;
};
void launch_border_fill(const BorderDesc* d, int n, hipStream_t st);
void launch_copy_block(int nsub, const int64_t* src_off, const int* src_ld, const int* r0,
                       const int* rows, const int* cols, const int64_t* dst_off, const int* dst_ld,
                       const double* src, double* dst, hipStream_t st);
void launch_diag_copy(int n, const int64_t* pos, const double* A, double* out, hipStream_t st);

// ---- Krylov helpers ----
void launch_dot_cols(int n, int nrhs, const double* a, const double* b, double* part, double* out,
                     hipStream_t st);
// one launch; cnt: nrhs ints that are zero between calls (left zero)
void launch_dot_cols_fin(int n, int nrhs, const double* a, const double* b, double* part,
                         int* cnt, double* out, hipStream_t st);
void launch_pcg_update_x_r(int n, int nrhs, const double* rz, const double* pq, const int* active,
                           double* x, double* r, const double* p, const double* q, double* alpha_hist,
                           const int* itp, int maxit, hipStream_t st);
void launch_pcg_update_p(int n, int nrhs, const double* rz_new, double* rz, const int* active,
                         int* restart, double* p, const double* z, double* beta_hist, int* itp,
                         int maxit, hipStream_t st);
void launch_lanczos_cond(int nrhs, const int* nalpha, const double* alpha, const double* beta,
                         int maxit, double* out, hipStream_t st);
// cnt: 8 + nrhs ints (meets, active, replaced, stalled counts, iteration
// counter, 3 spare, then the counters of launch_dot_cols_fin, zeroed here)
void launch_pcg_init_flags(int nrhs, const double* ff, int* act, int* nal, int* repl, int* stall,
                           double* tprev, int* cnt, hipStream_t st);
void launch_pcg_meets(int nrhs, const double* rr, const double* ff, double rtol2, const int* act,
                      int* nal, int* meets, int* cnt, const int* itp, hipStream_t st);
void launch_pcg_true(int nrhs, const double* tt, const double* ff, double rtol2, int* act,
                     const int* meets, int* repl, int* stall, double* tprev, int* cnt,
                     hipStream_t st);
void launch_fill(double* p, size_t n, double v, hipStream_t st);
void launch_move(int n, const int64_t* sidx, const double* src, int64_t lds, const int64_t* didx,
                 double* dst, int64_t ldd, int nrhs, hipStream_t st);
// dst[idx[k], r] = 0 for every column (mask null) or the columns with mask[r] != 0
void launch_zero_rows(int n, const int64_t* idx, double* dst, int64_t ldd, int nrhs,
                      const int* mask, hipStream_t st);
// dst[didx[k], r] += src[sidx[k], r] for the columns with mask[r] != 0
void launch_move_add_masked(int n, const int64_t* sidx, const double* src, int64_t lds,
                            const int64_t* didx, double* dst, int64_t ldd, int nrhs,
                            const int* mask, hipStream_t st);
void launch_rigid_level1(int n_nodes, int dof, const double* coords, const int* free_of_full,
                         int ndof, double* rigid, hipStream_t st);
void launch_coarse_rigid(int n2, int nrb, const int* sub_of, const int* row_of, const int64_t* c_off,
                         const int* nc, const int* nG, const int64_t* Goff, const int* Gdof,
                         const double* C, const double* rigid1, int n1, double* rigid2,
                         hipStream_t st);
void launch_copy(double* dst, const double* src, size_t n, hipStream_t st);
void launch_pow10(size_t n, const double* theta, double* out, hipStream_t st);
void launch_sub(size_t n, const double* a, const double* b, double* out, hipStream_t st);
void launch_copy_cols(int n, int nrhs, const double* src, double* dst, const int* mask,
                      hipStream_t st);
void launch_check_coeff(int n, const double* coeff, const double* nu, int* bad, hipStream_t st);

}  // namespace ambddc
