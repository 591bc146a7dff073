// Q1 element matrices, dense subdomain assembly, global CSR values and
// matrix-vector product, element gradient.
#include "kernels.hpp"

namespace ambddc {

// Trilinear hexahedron, 2x2x2 Gauss.  Local node a + 2b + 4c sits at the
// reference corner ((-1)^{a+1}, (-1)^{b+1}, (-1)^{c+1}).
__device__ inline void q1_grads(const double* xe, double gx, double gy, double gz,
                                double (&G)[8][3], double& det) {
  double dN[8][3];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const double rx = (n & 1) ? 1.0 : -1.0;
    const double ry = (n & 2) ? 1.0 : -1.0;
    const double rz = (n & 4) ? 1.0 : -1.0;
    const double fx = 1.0 + rx * gx, fy = 1.0 + ry * gy, fz = 1.0 + rz * gz;
    dN[n][0] = 0.125 * rx * fy * fz;
    dN[n][1] = 0.125 * fx * ry * fz;
    dN[n][2] = 0.125 * fx * fy * rz;
  }
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // J[i][j] = dx_j / dxi_i
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) J[i][j] += dN[n][i] * xe[3 * n + j];
  det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double id = 1.0 / det;
  double Ji[3][3];
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  // grad_x N = J^{-1} grad_xi N
#pragma unroll
  for (int n = 0; n < 8; ++n)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      G[n][j] = Ji[j][0] * dN[n][0] + Ji[j][1] * dN[n][1] + Ji[j][2] * dN[n][2];
}

// One workgroup of 64 threads per element; thread t owns matrix entries t, t+64, ...
__global__ __launch_bounds__(64) void k_elem_poisson(const double* __restrict__ coords,
                                                     const int* __restrict__ en,
                                                     const double* __restrict__ kappa, double* Ke) {
  const int e = blockIdx.x;
  __shared__ double xe[24];
  __shared__ double Gs[8][8][3];
  __shared__ double dets[8];
  const int t = threadIdx.x;
  if (t < 24) xe[t] = coords[3 * en[8 * e + t / 3] + t % 3];
  __syncthreads();
  if (t < 8) {
    const double g = 0.57735026918962576451;
    const double gx = (t & 1) ? g : -g, gy = (t & 2) ? g : -g, gz = (t & 4) ? g : -g;
    double G[8][3], det;
    q1_grads(xe, gx, gy, gz, G, det);
    for (int n = 0; n < 8; ++n)
      for (int j = 0; j < 3; ++j) Gs[t][n][j] = G[n][j];
    dets[t] = det;
  }
  __syncthreads();
  const int a = t % 8, b = t / 8;
  double v = 0.0;
  for (int q = 0; q < 8; ++q)
    v += dets[q] * (Gs[q][a][0] * Gs[q][b][0] + Gs[q][a][1] * Gs[q][b][1] + Gs[q][a][2] * Gs[q][b][2]);
  Ke[(size_t)e * 64 + t] = kappa[e] * v;
}

// Isotropic elasticity: 24x24, DOF order 3*node + component; Voigt strain
// (xx, yy, zz, yz, xz, xy), D = lambda m m^T + mu diag(2,2,2,1,1,1).
__global__ __launch_bounds__(256) void k_elem_elastic(const double* __restrict__ coords,
                                                      const int* __restrict__ en,
                                                      const double* __restrict__ E,
                                                      const double* __restrict__ nu, double* Ke) {
  const int e = blockIdx.x;
  __shared__ double xe[24];
  __shared__ double Gs[8][8][3];
  __shared__ double dets[8];
  const int t = threadIdx.x;
  if (t < 24) xe[t] = coords[3 * en[8 * e + t / 3] + t % 3];
  __syncthreads();
  if (t < 8) {
    const double g = 0.57735026918962576451;
    const double gx = (t & 1) ? g : -g, gy = (t & 2) ? g : -g, gz = (t & 4) ? g : -g;
    double G[8][3], det;
    q1_grads(xe, gx, gy, gz, G, det);
    for (int n = 0; n < 8; ++n)
      for (int j = 0; j < 3; ++j) Gs[t][n][j] = G[n][j];
    dets[t] = det;
  }
  __syncthreads();
  const double Ee = E[e], ne = nu[e];
  const double lam = Ee * ne / ((1.0 + ne) * (1.0 - 2.0 * ne));
  const double mu = Ee / (2.0 * (1.0 + ne));
  for (int idx = t; idx < 576; idx += 256) {
    const int r = idx % 24, c = idx / 24;
    const int a = r / 3, i = r % 3, b = c / 3, j = c % 3;
    double v = 0.0;
    for (int q = 0; q < 8; ++q) {
      const double* ga = Gs[q][a];
      const double* gb = Gs[q][b];
      // u_a e_i, u_b e_j:  lam (da_i)(db_j) + mu [ (ga.gb) delta_ij + da_j db_i ]
      double s = lam * ga[i] * gb[j] + mu * ga[j] * gb[i];
      if (i == j) s += mu * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
      v += dets[q] * s;
    }
    Ke[(size_t)e * 576 + idx] = v;
  }
}

void launch_element_matrices(const double* coords, const int* en, const double* coeff,
                             const double* nu, int n_elem, int dof, double* Ke, hipStream_t st) {
  if (n_elem == 0) return;
  if (dof == 1) k_elem_poisson<<<n_elem, 64, 0, st>>>(coords, en, coeff, Ke);
  else k_elem_elastic<<<n_elem, 256, 0, st>>>(coords, en, coeff, nu, Ke);
  AMB_LAUNCH_CHECK();
}

// Column-gather assembly: thread per (subdomain, local column j).  Every
// element containing the column's DOF adds its column into the dense
// subdomain block; each thread writes only its own column (no atomics,
// fixed summation order).
__global__ __launch_bounds__(256) void k_assemble(int ncols, const int* __restrict__ col_sub,
                                                  const int* __restrict__ col_j,
                                                  const int64_t* __restrict__ inc_ptr,
                                                  const int* __restrict__ inc_e,
                                                  const int* __restrict__ inc_a,
                                                  const int64_t* __restrict__ emat_off,
                                                  const int* __restrict__ elem_ne,
                                                  const int64_t* __restrict__ eloc_off,
                                                  const int* __restrict__ eloc,
                                                  const double* __restrict__ emat,
                                                  const int64_t* __restrict__ tgt_off,
                                                  const int* __restrict__ tgt_ld, double* tgt) {
  const int gc = blockIdx.x * blockDim.x + threadIdx.x;
  if (gc >= ncols) return;
  const int s = col_sub[gc], j = col_j[gc];
  double* col = tgt + tgt_off[s] + (int64_t)j * tgt_ld[s];
  for (int64_t q = inc_ptr[gc]; q < inc_ptr[gc + 1]; ++q) {
    const int e = inc_e[q], a = inc_a[q];
    const int ne = elem_ne[e];
    const double* ke = emat + emat_off[e] + (int64_t)a * ne;
    const int* loc = eloc + eloc_off[e];
    for (int b = 0; b < ne; ++b) {
      const int r = loc[b];
      if (r >= 0) col[r] += ke[b];
    }
  }
}

void launch_assemble(const AssemblyMaps& m, const double* emat, const int64_t* tgt_off,
                     const int* tgt_ld, double* tgt, hipStream_t st) {
  if (m.ncols == 0) return;
  k_assemble<<<ceil_div(m.ncols, 256), 256, 0, st>>>(
      m.ncols, m.col_sub.p, m.col_j.p, m.inc_ptr.p, m.inc_e.p, m.inc_a.p, m.emat_off.p,
      m.elem_ne.p, m.eloc_off.p, m.eloc.p, emat, tgt_off, tgt_ld, tgt);
  AMB_LAUNCH_CHECK();
}

// Lanes of one wave that hand LDS values to each other between steps: a
// wave's LDS accesses complete in program order, and the fences keep the
// compiler from moving them across the step boundary.
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Whole-column assembly: one wave per (subdomain, local column j).  The
// column is built in LDS, zeros plus every incident element's column in the
// fixed incidence order, and written out whole (leading dimension rows), so
// the dense block needs no separate zero fill and takes no read-modify-write
// traffic.  The metadata of up to 8 incidences is loaded by 8 lanes at once
// and their element entries are in flight together before the LDS adds; one
// element's DOFs are distinct rows.  Elements of at most 64 DOFs.
__global__ __launch_bounds__(256) void k_assemble_cols(int ncols, int ldmax,
                                                       const int* __restrict__ col_sub,
                                                       const int* __restrict__ col_j,
                                                       const int64_t* __restrict__ inc_ptr,
                                                       const int* __restrict__ inc_e,
                                                       const int* __restrict__ inc_a,
                                                       const int64_t* __restrict__ emat_off,
                                                       const int* __restrict__ elem_ne,
                                                       const int64_t* __restrict__ eloc_off,
                                                       const int* __restrict__ eloc,
                                                       const double* __restrict__ emat,
                                                       const int64_t* __restrict__ tgt_off,
                                                       const int* __restrict__ tgt_ld, double* tgt) {
  constexpr int QC = 8;
  extern __shared__ double asm_col[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gc = blockIdx.x * (blockDim.x >> 6) + w;
  if (gc >= ncols) return;   // whole waves leave together
  double* cs = asm_col + (size_t)w * ldmax;
  const int s = col_sub[gc], j = col_j[gc];
  const int ld = tgt_ld[s];
  for (int r = lane; r < ld; r += 64) cs[r] = 0.0;
  const int64_t qa = inc_ptr[gc], qb = inc_ptr[gc + 1];
  for (int64_t q0 = qa; q0 < qb; q0 += QC) {
    const int nq = int(min<int64_t>(QC, qb - q0));
    int ne_t = 0, eo_lo = 0, eo_hi = 0, lo_lo = 0, lo_hi = 0;
    if (lane < nq) {
      const int e = inc_e[q0 + lane], a = inc_a[q0 + lane];
      ne_t = elem_ne[e];
      const int64_t eo = emat_off[e] + (int64_t)a * ne_t, lo = eloc_off[e];
      eo_lo = int(uint32_t(eo)); eo_hi = int(uint64_t(eo) >> 32);
      lo_lo = int(uint32_t(lo)); lo_hi = int(uint64_t(lo) >> 32);
    }
    int rr[QC];
    double vv[QC];
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int neu = __shfl(ne_t, u);
      const int64_t eo = int64_t((uint64_t(uint32_t(__shfl(eo_hi, u))) << 32) |
                                 uint32_t(__shfl(eo_lo, u)));
      const int64_t lo = int64_t((uint64_t(uint32_t(__shfl(lo_hi, u))) << 32) |
                                 uint32_t(__shfl(lo_lo, u)));
      rr[u] = -1;
      vv[u] = 0.0;
      if (u < nq && lane < neu) {
        rr[u] = eloc[lo + lane];
        vv[u] = emat[eo + lane];
      }
    }
    group_sync();   // the zeros (first chunk) or the previous chunk's adds
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      if (rr[u] >= 0) cs[rr[u]] += vv[u];
      group_sync();
    }
  }
  group_sync();
  double* col = tgt + tgt_off[s] + (int64_t)j * ld;
  for (int r = lane; r < ld; r += 64) col[r] = cs[r];
}

void launch_assemble_cols(const AssemblyMaps& m, int ldmax, const double* emat,
                          const int64_t* tgt_off, const int* tgt_ld, double* tgt, hipStream_t st) {
  if (m.ncols == 0) return;
  if (m.max_ne > 64) throw Error(1, "assemble_cols: elements of more than 64 DOFs");
  const size_t per_col = size_t(ldmax) * sizeof(double);
  if (per_col > 64 * 1024) throw Error(1, "assemble_cols: column longer than the LDS staging allows");
  int waves = 4;
  while (waves > 1 && size_t(waves) * per_col > 64 * 1024) --waves;
  k_assemble_cols<<<ceil_div(m.ncols, waves), 64 * waves, waves * per_col, st>>>(
      m.ncols, ldmax, m.col_sub.p, m.col_j.p, m.inc_ptr.p, m.inc_e.p, m.inc_a.p, m.emat_off.p,
      m.elem_ne.p, m.eloc_off.p, m.eloc.p, emat, tgt_off, tgt_ld, tgt);
  AMB_LAUNCH_CHECK();
}

// Global CSR values: a group of G lanes per row (G >= DOFs per element).  The
// row's column indices are staged in LDS beside one accumulator per entry;
// for every element incident to the row, lane b adds the element-matrix entry
// of the element's DOF b at the position found by binary search over the
// staged indices.  One element's DOFs are distinct columns, and the elements
// are taken in the fixed incidence order, so the sums are deterministic.  A
// group lives inside one wave (group_sync).
template <int G>
__global__ __launch_bounds__(256) void k_csr_values(int n, int maxrow,
                                                    const int* __restrict__ rowptr,
                                                    const int* __restrict__ cols,
                                                    const int64_t* __restrict__ inc_ptr,
                                                    const int* __restrict__ inc_e,
                                                    const int* __restrict__ inc_a,
                                                    const int* __restrict__ edofs, int ne,
                                                    const double* __restrict__ Ke, double* vals) {
  extern __shared__ double csr_sm[];
  const int rpb = blockDim.x / G;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  double* acc = csr_sm + (size_t)grp * maxrow;
  int* cl = reinterpret_cast<int*>(csr_sm + (size_t)rpb * maxrow) + (size_t)grp * maxrow;
  const int i = blockIdx.x * rpb + grp;
  if (i >= n) return;   // whole groups leave together
  const int r0 = rowptr[i], len = rowptr[i + 1] - r0;
  for (int k = lane; k < len; k += G) {
    acc[k] = 0.0;
    cl[k] = cols[r0 + k];
  }
  group_sync();
  const int64_t q1 = inc_ptr[i + 1];
  for (int64_t q = inc_ptr[i]; q < q1; ++q) {
    const int e = inc_e[q], a = inc_a[q];
    if (lane < ne) {
      const int c = edofs[(size_t)e * ne + lane];
      if (c >= 0) {
        int lo = 0, hi = len - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (cl[mid] < c) lo = mid + 1; else hi = mid;
        }
        acc[lo] += Ke[(size_t)e * ne * ne + (size_t)a * ne + lane];
      }
    }
    group_sync();
  }
  for (int k = lane; k < len; k += G) vals[r0 + k] = acc[k];
}

void launch_csr_values(const CsrMaps& m, const int* edofs, int ne, const double* Ke, double* vals,
                       hipStream_t st) {
  if (m.n == 0) return;
  const int G = ne <= 8 ? 8 : ne <= 16 ? 16 : ne <= 32 ? 32 : 64;
  if (ne > 64) throw Error(1, "csr values: more than 64 DOFs per element");
  const size_t per_row = size_t(m.maxrow) * (sizeof(double) + sizeof(int));
  int rpb = 256 / G;
  while (rpb > 1 && size_t(rpb) * per_row > 64 * 1024) rpb >>= 1;
  if (size_t(rpb) * per_row > 64 * 1024)
    throw Error(1, "csr values: row longer than the LDS staging allows");
  const size_t lds = size_t(rpb) * per_row;
  const int blocks = ceil_div(m.n, rpb);
  switch (G) {
#define AMB_CASE(GG)                                                                          \
  case GG:                                                                                    \
    k_csr_values<GG><<<blocks, rpb * GG, lds, st>>>(m.n, m.maxrow, m.rowptr.p, m.cols.p,      \
                                                    m.inc_ptr.p, m.inc_e.p, m.inc_a.p, edofs, \
                                                    ne, Ke, vals);                            \
    break;
    AMB_CASE(8) AMB_CASE(16) AMB_CASE(32) AMB_CASE(64)
#undef AMB_CASE
  }
  AMB_LAUNCH_CHECK();
}

// y = K x for any number of right-hand sides (ld = n): one thread per row.
__global__ __launch_bounds__(256) void k_spmv_any(int n, int nrhs, const int* __restrict__ rowptr,
                                                  const int* __restrict__ cols,
                                                  const double* __restrict__ vals,
                                                  const double* __restrict__ x, double* y,
                                                  const unsigned char* __restrict__ zmask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool z = zmask && zmask[i];
  for (int r = 0; r < nrhs; ++r) {
    double acc = 0.0;
    if (!z)
      for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += vals[k] * x[cols[k] + (size_t)r * n];
    y[i + (size_t)r * n] = acc;
  }
}

// y = K x with G lanes per row (G divides 64, rows aligned to groups of G
// lanes): the lanes read consecutive entries of the row, so a wave's loads of
// the values and column indices are contiguous, and the group sums with
// shuffles.  Used for rows of more than a few entries (27 for Poisson, 81 for
// elasticity).
template <int R, int G>
__global__ __launch_bounds__(256) void k_spmv_g(int n, const int* __restrict__ rowptr,
                                                const int* __restrict__ cols,
                                                const double* __restrict__ vals,
                                                const double* __restrict__ x, double* y,
                                                const unsigned char* __restrict__ zmask) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / G, lane = t % G;
  if (i >= n) return;   // whole groups leave together
  if (zmask && zmask[i]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane == r % G) y[i + (size_t)r * n] = 0.0;
    return;
  }
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const int k1 = rowptr[i + 1];
  for (int k = rowptr[i] + lane; k < k1; k += G) {
    const double v = vals[k];
    const int c = cols[k];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += v * x[c + (size_t)r * n];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += __shfl_xor(acc[r], o);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane == r % G) y[i + (size_t)r * n] = acc[r];
}

template <int G>
static void spmv_g(const CsrMaps& m, const double* vals, const double* x, double* y, int nrhs,
                   hipStream_t st, const unsigned char* zm) {
  const int g = ceil_div(m.n, 256 / G);
  switch (nrhs) {
    case 1: k_spmv_g<1, G><<<g, 256, 0, st>>>(m.n, m.rowptr.p, m.cols.p, vals, x, y, zm); break;
    case 2: k_spmv_g<2, G><<<g, 256, 0, st>>>(m.n, m.rowptr.p, m.cols.p, vals, x, y, zm); break;
    case 4: k_spmv_g<4, G><<<g, 256, 0, st>>>(m.n, m.rowptr.p, m.cols.p, vals, x, y, zm); break;
    case 8: k_spmv_g<8, G><<<g, 256, 0, st>>>(m.n, m.rowptr.p, m.cols.p, vals, x, y, zm); break;
    case 16: k_spmv_g<16, G><<<g, 256, 0, st>>>(m.n, m.rowptr.p, m.cols.p, vals, x, y, zm); break;
    default:
      k_spmv_any<<<ceil_div(m.n, 256), 256, 0, st>>>(m.n, nrhs, m.rowptr.p, m.cols.p, vals, x, y,
                                                     zm);
  }
}

void launch_spmv(const CsrMaps& m, const double* vals, const double* x, double* y, int nrhs,
                 hipStream_t st, const unsigned char* zmask) {
  if (m.n == 0) return;
  // lanes per row from the mean row length
  const double avg = double(m.nnz) / m.n;
  if (avg > 48.0) spmv_g<32>(m, vals, x, y, nrhs, st, zmask);
  else if (avg > 12.0) spmv_g<16>(m, vals, x, y, nrhs, st, zmask);
  else spmv_g<4>(m, vals, x, y, nrhs, st, zmask);
  AMB_LAUNCH_CHECK();
}

__global__ void k_mark_rows(int n, const int64_t* __restrict__ pos, unsigned char* mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) mask[pos[i]] = 1;
}

void launch_mark_rows(int n, const int64_t* pos, unsigned char* mask, hipStream_t st) {
  if (n == 0) return;
  k_mark_rows<<<ceil_div(n, 256), 256, 0, st>>>(n, pos, mask);
  AMB_LAUNCH_CHECK();
}

// grad[e] = -ln(10) sum_k lam_k,e^T K_e x_k,e  (element DOFs, fixed DOFs = 0)
__global__ __launch_bounds__(256) void k_elem_grad(int n_elem, int ne, int n, int nrhs,
                                                   const int* __restrict__ edofs,
                                                   const double* __restrict__ Ke,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ L, double* grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  const int* ed = edofs + (size_t)e * ne;
  const double* ke = Ke + (size_t)e * ne * ne;
  double g = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    const double* x = X + (size_t)r * n;
    const double* l = L + (size_t)r * n;
    for (int b = 0; b < ne; ++b) {
      const int cb = ed[b];
      if (cb < 0) continue;
      double kx = 0.0;
      for (int a = 0; a < ne; ++a) {
        const int ca = ed[a];
        if (ca >= 0) kx += ke[b + (size_t)a * ne] * x[ca];
      }
      g += l[cb] * kx;
    }
  }
  grad[e] = -2.302585092994045684 * g;
}

void launch_element_gradient(int n_elem, int ne, int n, int nrhs, const int* edofs, const double* Ke,
                             const double* X, const double* L, double* grad, hipStream_t st) {
  if (n_elem == 0) return;
  k_elem_grad<<<ceil_div(n_elem, 256), 256, 0, st>>>(n_elem, ne, n, nrhs, edofs, Ke, X, L, grad);
  AMB_LAUNCH_CHECK();
}

}  // namespace ambddc
