// Largest eigenpairs of one small symmetric matrix held in LDS, computed by
// one workgroup of NT threads (NT / 64 >= the number of eigenpairs wanted).
//
// 1. Householder reduction to tridiagonal form T = Q^T A Q: for k = 0..n-3 the
//    reflector H_k = I - tau_k u_k u_k^T (u_k[0] = 1) annihilates A[k+2:, k];
//    with p = tau A22 u and w = p - (tau/2)(u.p) u the trailing block becomes
//    A22 - u w^T - w u^T.  u_k is kept in A[k+1:, k].  Two barriers a step.
// 2. The mm largest eigenvalues of T by multisection: a group of EIG_MSP
//    lanes per eigenvalue evaluates Sturm counts (negative pivots of the
//    LDL^T of T - xI, with a Newton-refined hardware reciprocal) at EIG_MSP
//    interior points of the current interval, and the ballot of
//    "count >= target" picks the sub-interval (a factor EIG_MSP + 1 a pass),
//    down to a width of 2 eps ||T||: the reduction to tridiagonal form is
//    backward stable at that absolute level, so more is not resolved.
//    d and e^2 sit one entry per lane and are read with readlane.
// 3. Their eigenvectors of T by inverse iteration, one wave per eigenvalue,
//    all at once (LU of T - lambda I with partial pivoting, row i of the
//    factors kept by lane i; two solves).  After each solve the vectors of
//    every cluster (eigenvalues closer than EIG_CTOL ||T||) are orthonormalised
//    by modified Gram-Schmidt in eigenvalue order; the step count is the
//    largest cluster size, all clusters proceed together.
// 4. The back-transformation y = H_0 H_1 ... H_{n-3} z, one wave per vector.
// Wave reductions use DPP row operations and one readlane.
#pragma once
#include <hip/hip_runtime.h>

namespace ambddc {

constexpr int EIG_MAXN = 64;
constexpr int EIG_MSP = 16;          // multisection points per eigenvalue
constexpr double EIG_CTOL = 1e-5;     // cluster gap, relative to ||T||
// LDS scratch in doubles: d, e, e^2, tau, p
constexpr int EIG_WS = 5 * EIG_MAXN;

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_add(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffff), hi = (int)(b >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, false);
  return x + __longlong_as_double(((long long)(unsigned)rhi << 32) | (unsigned)rlo);
}
// sum over each aligned group of 16 lanes, in every lane of the group
__device__ __forceinline__ double row16_sum(double x) {
  x = dpp_add<0xb1, 0xf>(x);
  x = dpp_add<0x4e, 0xf>(x);
  x = dpp_add<0x141, 0xf>(x);
  return dpp_add<0x140, 0xf>(x);
}
// sum over the wave, returned in every lane
__device__ __forceinline__ double wave_sum(double x) {
  x = row16_sum(x);
  x = dpp_add<0x142, 0xa>(x);
  x = dpp_add<0x143, 0xc>(x);
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_max(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffff), hi = (int)(b >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false);
  return fmax(x, __longlong_as_double(((long long)(unsigned)rhi << 32) | (unsigned)rlo));
}
// maximum over the wave, returned in every lane (no NaN inputs)
__device__ __forceinline__ double wave_max(double x) {
  x = dpp_max<0xb1, 0xf>(x);
  x = dpp_max<0x4e, 0xf>(x);
  x = dpp_max<0x141, 0xf>(x);
  x = dpp_max<0x140, 0xf>(x);
  x = dpp_max<0x142, 0xa>(x);
  x = dpp_max<0x143, 0xc>(x);
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double rl(double v, int i) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), i);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
// 1 / q from the hardware reciprocal and one Newton step
__device__ __forceinline__ double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  return r * (2.0 - q * r);
}

// A: n x n symmetric (ld lda), destroyed.  Y: n x mm eigenvectors (ld ldy),
// lam: mm eigenvalues, descending, mm = min(m, n).  ws: EIG_WS doubles.
// n <= EIG_MAXN, m <= 4 NT / 64 (the eigenvectors are computed by the NT / 64
// waves in passes of NT / 64).
template <int NT>
__device__ inline void sym_top_eig(double* A, int lda, int n, int m, double* Y, int ldy,
                                   double* lam, double* ws) {
  static_assert(NT % 64 == 0 && NT / 16 >= EIG_MAXN, "sym_top_eig: thread count");
  constexpr double EPS = 2.220446049250313e-16;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* d = ws;
  double* e = ws + EIG_MAXN;
  double* e2 = ws + 2 * EIG_MAXN;
  double* tau = ws + 3 * EIG_MAXN;
  double* p = ws + 4 * EIG_MAXN;
  const int mm = min(m, n);
  if (n <= 0) return;

  // 1. tridiagonal reduction.  The reflector of column k + 1 is built by
  // wave 0 right after it has updated that column (the first elements of the
  // rank-2 update are column k + 1, all in wave 0), so a step needs two
  // barriers.  reflect(): x holds A[k+1+l, k] in lane l (0 from nk on).
  auto reflect = [&](int k, int nk, double x) {
    const double s = wave_sum((lane >= 1 && lane < nk) ? x * x : 0.0);
    const double alpha = rl(x, 0);
    double t = 0.0, beta = alpha, scale = 0.0;
    if (s > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    double* col = A + (k + 1) + (size_t)k * lda;
    if (lane < nk) col[lane] = (lane == 0) ? 1.0 : x * scale;
    if (lane == 0) {
      e[k] = beta;
      tau[k] = t;
    }
  };
  if (n > 2) {
    if (wave == 0) reflect(0, n - 1, lane < n - 1 ? A[1 + lane] : 0.0);
    __syncthreads();
  }
  for (int k = 0; k + 2 < n; ++k) {
    const int nk = n - k - 1;
    const double* col = A + (k + 1) + (size_t)k * lda;
    const bool next = k + 3 < n;   // column k + 1 gets a reflector too
    const double tk = tau[k];
    if (tk != 0.0) {
      // p = tau A22 u with 16 lanes per row (A22 symmetric, read by columns)
      const int g = tid >> 4, l16 = tid & 15;
      if (g < nk) {
        const double* arow = A + (k + 1) + (size_t)(k + 1 + g) * lda;
        double acc = 0.0;
        for (int j = l16; j < nk; j += 16) acc += arow[j] * col[j];
        acc = row16_sum(acc);
        if (l16 == 0) p[g] = tk * acc;
      }
      __syncthreads();
      const double K = 0.5 * tk * wave_sum(lane < nk ? col[lane] * p[lane] : 0.0);
      auto update = [&](int idx) {
        const int i = idx % nk, j = idx / nk;
        const double ui = col[i], uj = col[j];
        const double wi = p[i] - K * ui, wj = p[j] - K * uj;
        double* a = A + (k + 1 + i) + (size_t)(k + 1 + j) * lda;
        const double v = *a - (ui * wj + wi * uj);
        *a = v;
        return v;
      };
      // lanes i < nk of wave 0 hold the new A[k+1+i, k+1] in v0
      const double v0 = tid < nk * nk ? update(tid) : 0.0;
      if (wave == 0 && next) {
        const double xn = __shfl_down(v0, 1);
        reflect(k + 1, nk - 1, lane + 1 < nk ? xn : 0.0);
      }
      for (int idx = tid + NT; idx < nk * nk; idx += NT) update(idx);
    } else if (wave == 0 && next) {
      reflect(k + 1, nk - 1, lane + 1 < nk ? A[(k + 2 + lane) + (size_t)(k + 1) * lda] : 0.0);
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) d[i] = A[i + (size_t)i * lda];
  if (tid == 0 && n >= 2) e[n - 2] = A[(n - 1) + (size_t)(n - 2) * lda];
  __syncthreads();
  for (int i = tid; i + 1 < n; i += NT) e2[i] = e[i] * e[i];
  __syncthreads();

  // bounds of the spectrum (Gershgorin), computed by every wave
  double lo_i = 1e300, hi_i = -1e300, ee = 0.0;
  if (lane < n) {
    const double r = (lane > 0 ? fabs(e[lane - 1]) : 0.0) + (lane + 1 < n ? fabs(e[lane]) : 0.0);
    lo_i = d[lane] - r;
    hi_i = d[lane] + r;
    ee = lane + 1 < n ? e2[lane] : 0.0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo_i = fmin(lo_i, __shfl_xor(lo_i, o));
    hi_i = fmax(hi_i, __shfl_xor(hi_i, o));
    ee = fmax(ee, __shfl_xor(ee, o));
  }
  const double lo = lo_i, hi = hi_i;
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = 1e-280 * fmax(1.0, ee);

  // d, e, e^2 of T spread over the lanes (lane i holds entry i)
  const double dl = lane < n ? d[lane] : 0.0;
  const double el = lane + 1 < n ? e[lane] : 0.0;
  const double e2l = lane + 1 < n ? e2[lane] : 0.0;
  // 2. eigenvalues by multisection: EIG_MSP points per eigenvalue, 64 / EIG_MSP
  // eigenvalues per wave; lane group g of wave w finds eigenvalue
  // w (64 / EIG_MSP) + g (0 = largest)
  {
    constexpr int G = 64 / EIG_MSP;
    const int grp = lane / EIG_MSP, pl = lane % EIG_MSP;
    const int ev = wave * G + grp;
    if (wave * G < mm) {
      const int target = n - ev;   // Sturm count >= target  <=>  x > lambda_ev
      double a = lo, b = hi;
      for (int it = 0; it < 64; ++it) {
        const bool open = ev < mm && b - a > 2.0 * EPS * fmax(fmax(fabs(a), fabs(b)), tnorm);
        if (!__ballot(open)) break;
        const double x = a + (b - a) * double(pl + 1) / double(EIG_MSP + 1);
        double q = rl(dl, 0) - x;
        if (fabs(q) < pivmin) q = -pivmin;
        int cnt = q < 0.0;
#pragma unroll 8
        for (int i = 1; i < n; ++i) {
          q = rl(dl, i) - x - rl(e2l, i - 1) * rcp_nr(q);
          if (fabs(q) < pivmin) q = -pivmin;
          cnt += q < 0.0;
        }
        const unsigned long long ball = __ballot(cnt >= target);
        const unsigned long long gm = EIG_MSP == 64 ? ~0ull : ((1ull << EIG_MSP) - 1);
        const unsigned long long mine = (ball >> (grp * EIG_MSP)) & gm;
        const int l = mine ? __ffsll((long long)mine) - 1 : EIG_MSP;
        const double na = l > 0 ? a + (b - a) * double(l) / double(EIG_MSP + 1) : a;
        const double nb = l < EIG_MSP ? a + (b - a) * double(l + 1) / double(EIG_MSP + 1) : b;
        if (open) {
          a = na;
          b = nb;
        }
      }
      if (pl == 0 && ev < mm) lam[ev] = 0.5 * (a + b);
    }
  }
  __syncthreads();

  // 3. inverse iteration, one wave per wanted eigenvalue, all at once
  const double ctol = EIG_CTOL * tnorm;
  const double tiny = EPS * fmax(tnorm, 1e-300);
  constexpr int NW = NT / 64;
  // Pass q computes the eigenvectors j = q NW + wave.  Members of a cluster
  // that fall in earlier passes are final by then, so the Gram-Schmidt
  // rounds of a pass also remove their components.
  for (int j0 = 0; j0 < mm; j0 += NW) {
  // rank of this wave's member in its cluster and the cluster's first member
  int rank = 0, cs = 0, rounds = 1;
  const int j = j0 + wave;
  {
    int rk = 0, start = 0;
    for (int i = 0; i < min(mm, j0 + NW); ++i) {
      if (i > 0 && lam[i - 1] - lam[i] <= ctol) rk += 1;
      else { rk = 0; start = i; }
      if (i >= j0) rounds = max(rounds, rk + 1);
      if (i == j) { rank = rk; cs = start; }
    }
  }
  const bool member = j < mm;
  // LU of T - lam_j I with partial pivoting: a chain that every lane runs
  // alike; lane i keeps row i (reciprocal pivot, the two entries right of
  // it, multiplier, row swap)
  double myDi = 0.0, myU1 = 0.0, myU2 = 0.0, myL = 0.0;
  int mySw = 0;
  double yv = 0.0;
  if (member) {
    const double lj = lam[j];
    double diag = rl(dl, 0) - lj, sup = n > 1 ? rl(el, 0) : 0.0;
    for (int i = 0; i + 1 < n; ++i) {
      const double sub_ = rl(el, i), nd = rl(dl, i + 1) - lj;
      const double nsup = (i + 2 < n) ? rl(el, i + 1) : 0.0;
      double Di, U1i, U2i, Li;
      int sw = 0;
      if (fabs(diag) >= fabs(sub_)) {
        Di = fabs(diag) >= tiny ? diag : (diag >= 0.0 ? tiny : -tiny);
        Li = sub_ * rcp_nr(Di);
        U1i = sup;
        U2i = 0.0;
        diag = nd - Li * sup;
        sup = nsup;
      } else {
        Di = sub_;
        Li = diag * rcp_nr(sub_);
        U1i = nd;
        U2i = nsup;
        sw = 1;
        diag = sup - Li * nd;
        sup = -Li * nsup;
      }
      if (lane == i) {
        myDi = rcp_nr(Di);
        myU1 = U1i;
        myU2 = U2i;
        myL = Li;
        mySw = sw;
      }
    }
    if (lane == n - 1) myDi = rcp_nr(fabs(diag) >= tiny ? diag : (diag >= 0.0 ? tiny : -tiny));
    // start vector: positive, different for every member (members of a
    // multiple eigenvalue must not start from the same direction)
    yv = lane < n ? 1.0 + double((lane * 37 + j * 11) % 17) / 17.0 : 0.0;
    yv *= rsqrt(wave_sum(yv * yv));
  }
  for (int it = 0; it < 2; ++it) {
    if (member) {
      // forward elimination of the right-hand side; lane i keeps x_i
      double xi = rl(yv, 0);
      for (int i = 0; i + 1 < n; ++i) {
        double xn = rl(yv, i + 1);
        if (__builtin_amdgcn_readlane(mySw, i)) {
          const double t = xi;
          xi = xn;
          xn = t;
        }
        if (lane == i) yv = xi;
        xi = xn - rl(myL, i) * xi;
      }
      if (lane == n - 1) yv = xi;
      // back substitution
      double z1 = 0.0, z2 = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        const double z = (rl(yv, i) - rl(myU1, i) * z1 - rl(myU2, i) * z2) * rl(myDi, i);
        if (lane == i) yv = z;
        z2 = z1;
        z1 = z;
      }
      // scale to unit norm before the Gram-Schmidt products
      yv *= rsqrt(wave_sum(yv * yv));
    }
    // modified Gram-Schmidt inside every cluster, all clusters at once: in
    // step r the member of rank r is normalised and published, then every
    // later member of its cluster removes its component
    for (int r = 0; r < rounds; ++r) {
      if (member && rank == r) {
        yv *= rsqrt(wave_sum(yv * yv));
        if (lane < n) Y[lane + (size_t)j * ldy] = yv;
      }
      __syncthreads();
      if (member && rank > r) {
        const double yi = lane < n ? Y[lane + (size_t)(cs + r) * ldy] : 0.0;
        yv -= wave_sum(yi * yv) * yi;
      }
    }
  }
  __syncthreads();
  }

  // 4. back-transformation by the reflectors
  for (int jv = wave; jv < mm; jv += NW) {
    double* y = Y + (size_t)jv * ldy;
    for (int k = n - 3; k >= 0; --k) {
      const double tk = tau[k];
      if (tk == 0.0) continue;
      const int nk = n - k - 1;
      const double* u = A + (k + 1) + (size_t)k * lda;
      const double ul = lane < nk ? u[lane] : 0.0;
      const double s = tk * wave_sum(lane < nk ? ul * y[k + 1 + lane] : 0.0);
      if (lane < nk) y[k + 1 + lane] -= s * ul;
    }
  }
  __syncthreads();
}

}  // namespace ambddc
