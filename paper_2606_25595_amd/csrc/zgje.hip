// Batched FP64 Gauss-Jordan inversion with partial pivoting for gfx950.
//
// Block Gaussian elimination needs the explicit inverse of every Schur
// complement (Section IV-A; its stability is governed by the condition number,
// Eq. 6).  Inversion always runs in FP64.
//
// Algorithm (blocked, in place, implicit row pivoting):
//   for each column panel K = [k0, k0+nb):
//     1. panel kernel (one workgroup per matrix, panel held in registers):
//        for every column c of the panel, choose as pivot the row p with the
//        largest |re|+|im| among the rows not yet used (lowest row on ties),
//        scale row p by 1/pivot and eliminate column c from every other row,
//        all restricted to the panel's columns.  Rows are never swapped; the
//        pivot row of every step is recorded.  The eliminated panel W holds the
//        panel columns of the accumulated transform.
//     2. trailing update, a complex GEMM on the matrix cores:
//        X[:, j] += (W - E_p) * X[p_K, j] for every column j outside the panel,
//        where E_p has a unit entry at (pivot row of step k, k) and X[p_K, :] are
//        the panel's pivot rows before the update (copied to Tp, zero in the
//        panel's columns, so the GEMM leaves the panel untouched).
//   After all panels, X = T Pi with T A = Pi (Pi e_k = e_{pivot(k)}), so
//   A^-1 = Pi^T X Pi^T, i.e. A^-1[r][c] = X[pivot(r)][pivot^-1(c)], which the
//   unscramble kernel gathers into the output.
#include "qtx_internal.h"

namespace qtx {

namespace {

constexpr int PT = 512;   // threads of the panel kernel (8 waves)

template <int NB, int RPT>
__global__ __launch_bounds__(PT) void gje_panel_kernel(int n, int k0, double2* X, int64_t sX,
                                                       GjeWork w, int32_t* status) {
  const int z = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nbw = min(NB, n - k0);
  double2* __restrict__ Xz = X + (int64_t)z * sX;
  int32_t* __restrict__ prow = w.prow + (int64_t)z * n;
  int32_t* __restrict__ used = w.used + (int64_t)z * n;

  __shared__ double red_mag[2][PT / 64];
  __shared__ int red_idx[2][PT / 64];
  __shared__ double2 piv_row[2][NB];
  __shared__ int piv_of[NB];
  __shared__ int singular;

  if (tid == 0) singular = 0;

  double2 v[RPT][NB];
  bool u[RPT];
  int pivcol[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = tid + PT * j;
    pivcol[j] = -1;
    u[j] = (r >= n) || (used[r] != 0);
#pragma unroll
    for (int k = 0; k < NB; ++k)
      v[j][k] = (r < n && k < nbw) ? Xz[(int64_t)r * n + k0 + k] : cmk(0.0, 0.0);
  }

  // The column loop stays rolled; every register access uses a compile-time
  // index (the current column is selected with compares), so the panel never
  // leaves the register file.
  for (int k = 0; k < nbw; ++k) {
    const int buf = k & 1;
    double2 ck[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      ck[j] = cmk(0.0, 0.0);
#pragma unroll
      for (int kk = 0; kk < NB; ++kk)
        if (kk == k) ck[j] = v[j][kk];
    }
    // local arg-max over my unused rows (rows increase with j: strict > keeps the lowest)
    double bm = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int r = tid + PT * j;
      if (!u[j]) {
        double mag = fabs(ck[j].x) + fabs(ck[j].y);
        if (mag != mag) mag = __builtin_huge_val();   // a NaN row is taken (its NaN propagates)
        if (mag > bm) { bm = mag; bi = r; }
      }
    }
    // wave reduction: larger magnitude wins, lower row on ties
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double om = __shfl_xor(bm, off);
      const int oi = __shfl_xor(bi, off);
      if (om > bm || (om == bm && oi < bi)) { bm = om; bi = oi; }
    }
    if (lane == 0) { red_mag[buf][wave] = bm; red_idx[buf][wave] = bi; }
    __syncthreads();
    double pm = red_mag[buf][0];
    int p = red_idx[buf][0];
#pragma unroll
    for (int q = 1; q < PT / 64; ++q) {
      const double om = red_mag[buf][q];
      const int oi = red_idx[buf][q];
      if (om > pm || (om == pm && oi < p)) { pm = om; p = oi; }
    }
    // p is an unused row (one always exists while k0 + k < n and every candidate
    // has a magnitude >= 0); pm == 0 means singular.  Defensive clamp only.
    if ((unsigned)p >= (unsigned)n) p = 0;
    const int owner = p % PT, oj = p / PT;
    if (tid == owner) {
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (j == oj) {
#pragma unroll
          for (int kk = 0; kk < NB; ++kk) piv_row[buf][kk] = v[j][kk];
          u[j] = true;
          pivcol[j] = k;
        }
    }
    if (tid == 0) {
      piv_of[k] = p;
      prow[k0 + k] = p;
      if (!(pm > 0.0)) singular = 1;
    }
    __syncthreads();
    const double2 pv = piv_row[buf][k];
    const double2 dinv = (pv.x == 0.0 && pv.y == 0.0) ? cmk(1.0, 0.0) : cinv(pv);
    // Branch-free update (both forms are evaluated and selected per element, so
    // the pivot row's thread does not split the live ranges of the panel).
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const bool isp = (tid + PT * j) == p;
      const double2 fd = cmul(ck[j], dinv);
      const double2 newk = isp ? dinv : cmk(-fd.x, -fd.y);
#pragma unroll
      for (int k8 = 0; k8 < NB; k8 += 8) {
        double2 pr[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) pr[q] = piv_row[buf][k8 + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          // the pivot row becomes pr*dinv, every other row v - fd*pr; the column
          // being eliminated is replaced by the transform entry newk
          const double2 m = isp ? dinv : fd;
          const double2 t = cmul(m, isp ? v[j][k8 + q] : pr[q]);
          double2 nv;
          nv.x = isp ? t.x : v[j][k8 + q].x - t.x;
          nv.y = isp ? t.y : v[j][k8 + q].y - t.y;
          const bool col = (k8 + q == k);
          v[j][k8 + q].x = col ? newk.x : nv.x;
          v[j][k8 + q].y = col ? newk.y : nv.y;
        }
        asm volatile("" ::: "memory");
      }
    }
  }
  __syncthreads();

  // write back the panel, the shifted transform Wp and the usage flags
  double2* __restrict__ Wp = w.Wp + (int64_t)z * n * NB;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = tid + PT * j;
    if (r < n) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k < nbw) Xz[(int64_t)r * n + k0 + k] = v[j][k];
        double2 wv = (k < nbw) ? v[j][k] : cmk(0.0, 0.0);
        if (k == pivcol[j]) wv.x -= 1.0;
        Wp[(int64_t)r * NB + k] = wv;
      }
      if (pivcol[j] >= 0) used[r] = 1;
    }
  }
  // pivot rows of this panel (pre-update values outside the panel), panel columns zeroed
  double2* __restrict__ Tp = w.Tp + (int64_t)z * NB * n;
  for (int idx = tid; idx < NB * n; idx += PT) {
    const int k = idx / n, c = idx - k * n;
    double2 val = cmk(0.0, 0.0);
    if (k < nbw && (c < k0 || c >= k0 + nbw)) val = Xz[(int64_t)piv_of[k] * n + c];
    Tp[idx] = val;
  }
  if (tid == 0 && singular && status) status[z] = 5;   // QTX_ERR_SINGULAR
}

// ---- 32-column panel (n <= 512) --------------------------------------------
// Same elimination as gje_panel_kernel, organised for a short pivot step:
//  * 512 threads; the half h = tid / 256 holds columns 16h .. 16h+15 of rows l and
//    l + 256 (l = tid % 256): 32 complex values per thread stay in VGPRs with two
//    waves per SIMD (two rows of all 32 columns per thread would not fit the 256
//    VGPRs and move through AGPRs at every step);
//  * the column loop is 2 rolled halves of 16 unrolled columns, so the current column
//    and the pivot-column test are compile-time, and only the half that holds the
//    column (wave-uniform) searches it;
//  * every row is updated with one formula, v <- v - m pr (four FMAs per complex
//    value), where m = v_k / pivot, and m = -1/pivot for the pivot row, whose values
//    are set to zero when it is posted (so it turns into pr / pivot); the pivot
//    column then takes the transform entry (1/pivot, resp. -v_k / pivot);
//  * the searching half reduces (|re| + |im|, row) over each thread's rows, then
//    within 16-lane groups with DPP moves and selects (no branches), and posts each
//    group's candidate (magnitude, row and column-k value) and every row's column-k
//    value; after a barrier every thread picks the best of the 16 candidates, the two
//    threads that hold the pivot row (one per half) post their halves of it while
//    every thread forms the pivot's reciprocal and its rows' multipliers, and after a
//    second barrier every thread updates its 16 columns.
template <int CTRL>
__device__ inline void argmax_dpp(double& m, int& i) {
  const int2 mb = __builtin_bit_cast(int2, m);
  int2 ob;
  ob.x = __builtin_amdgcn_mov_dpp(mb.x, CTRL, 0xF, 0xF, true);
  ob.y = __builtin_amdgcn_mov_dpp(mb.y, CTRL, 0xF, 0xF, true);
  const int oi = __builtin_amdgcn_mov_dpp(i, CTRL, 0xF, 0xF, true);
  const double om = __builtin_bit_cast(double, ob);
  const bool take = (om > m) | ((om == m) & (oi < i));
  m = take ? om : m;
  i = take ? oi : i;
}
__device__ inline void argmax_row16(double& m, int& i) {
  argmax_dpp<0xB1>(m, i);    // quad_perm [1,0,3,2]
  argmax_dpp<0x4E>(m, i);    // quad_perm [2,3,0,1]
  argmax_dpp<0x141>(m, i);   // row_half_mirror
  argmax_dpp<0x140>(m, i);   // row_mirror
}

constexpr int PT32 = 512;   // threads of the 32-column panel kernel

__global__ __launch_bounds__(PT32) void gje_panel32_kernel(int n, int k0, double2* X, int64_t sX, GjeWork w,
                                                           int32_t* status) {
  constexpr int NB = 32, HB = 16, RPT = 2, NG = 16;
  const int z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int h = tid >> 8, l = tid & 255;
  const int nbw = min(NB, n - k0);
  double2* __restrict__ Xz = X + (int64_t)z * sX;
  int32_t* __restrict__ prow = w.prow + (int64_t)z * n;
  int32_t* __restrict__ used = w.used + (int64_t)z * n;

  __shared__ double cand_mag[2][NG];
  __shared__ int cand_idx[2][NG];
  __shared__ double2 cand_val[2][NG];       // each candidate's column-k value
  __shared__ double2 piv_row[2][2][HB];     // each half's columns of the pivot row
  __shared__ double2 colk[2][RPT * 256];    // column k of every row
  __shared__ int piv_of[NB];
  // One half of the panel (16 columns of every row, pitch 17 so that the threads of a
  // wave, one row each, read distinct banks): the panel moves between HBM and the
  // threads' registers through it, 16 lanes per row (256 contiguous bytes), instead of
  // one row per lane (16 bytes of 64 rows per load).
  constexpr int SP = HB + 1;
  __shared__ double2 stage[RPT * 256 * SP];
  const int tot = n * HB;   // staged elements per half

  bool u[RPT];
  int pivcol[RPT];
  double2 v[RPT][HB];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = l + 256 * j;
    u[j] = (r >= n) || (used[r] != 0);
    pivcol[j] = -1;
  }
  for (int hh = 0; hh < 2; ++hh) {
    for (int e0 = 0; e0 < tot; e0 += PT32 * 4) {
      double2 t[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + PT32 * q + tid, row = e >> 4, gc = HB * hh + (e & 15);
        t[q] = (e < tot && gc < nbw) ? Xz[(int64_t)row * n + k0 + gc] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + PT32 * q + tid;
        if (e < tot) stage[(e >> 4) * SP + (e & 15)] = t[q];
      }
    }
    __syncthreads();
    if (h == hh) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = l + 256 * j;
#pragma unroll
        for (int c = 0; c < HB; ++c) v[j][c] = (r < n) ? stage[r * SP + c] : cmk(0.0, 0.0);
      }
    }
    __syncthreads();
  }
  bool singular = false;

  for (int hk = 0; hk < 2; ++hk) {
    const bool srch = (h == hk);   // wave-uniform: this half holds the current column
#pragma unroll
    for (int kc = 0; kc < HB; ++kc) {
      const int k = HB * hk + kc;
      if (k < nbw) {   // uniform
        const int buf = k & 1;
        if (srch) {
          double mag = -1.0;
          int idx = 0x7fffffff;
#pragma unroll
          for (int j = 0; j < RPT; ++j) {
            const double2 ck = v[j][kc];
            colk[buf][l + 256 * j] = ck;
            double mg = fabs(ck.x) + fabs(ck.y);
            mg = (mg != mg) ? __builtin_huge_val() : mg;   // a NaN row is taken (its NaN propagates)
            const bool take = !u[j] && mg > mag;           // rows increase with j: strict > keeps the lower
            mag = take ? mg : mag;
            idx = take ? l + 256 * j : idx;
          }
          argmax_row16(mag, idx);
          const int grp = l >> 4;
          if ((lane & 15) == 0) { cand_mag[buf][grp] = mag; cand_idx[buf][grp] = idx; }
#pragma unroll
          for (int j = 0; j < RPT; ++j)
            if (idx == l + 256 * j) cand_val[buf][grp] = v[j][kc];
        }
        __syncthreads();
        double pm = cand_mag[buf][lane & (NG - 1)];
        int p = cand_idx[buf][lane & (NG - 1)];
        argmax_row16(pm, p);
        // p is an unused row while k0 + k < n; pm == 0 means singular.  Defensive clamp only.
        if ((unsigned)p >= (unsigned)n) p = 0;
        const int pl = p & 255, pj = p >> 8;
        const double2 pv = cand_val[buf][pl >> 4];   // the pivot (the winning candidate's value)
        double2 ck[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) ck[j] = colk[buf][l + 256 * j];
        if (l == pl) {
#pragma unroll
          for (int j = 0; j < RPT; ++j)
            if (j == pj) {
#pragma unroll
              for (int c = 0; c < HB; ++c) {
                piv_row[buf][h][c] = v[j][c];
                v[j][c] = cmk(0.0, 0.0);
              }
            }
        }
        // The reciprocal of the pivot and every row's multiplier (column k was posted
        // before the first barrier) are formed while the pivot row is being posted.
        const double2 dinv = (pv.x == 0.0 && pv.y == 0.0) ? cmk(1.0, 0.0) : cinv(pv);
        double2 m[RPT], newk[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          const bool isp = (l + 256 * j == p);
          const double2 fd = cmul(ck[j], dinv);
          m[j] = isp ? cmk(-dinv.x, -dinv.y) : fd;
          newk[j] = isp ? dinv : cmk(-fd.x, -fd.y);
          u[j] = u[j] || isp;
          pivcol[j] = isp ? k : pivcol[j];
        }
        __syncthreads();
        const double2* __restrict__ prs = &piv_row[buf][h][0];
#pragma unroll
        for (int c8 = 0; c8 < HB; c8 += 8) {
          double2 pr[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) pr[q] = prs[c8 + q];
#pragma unroll
          for (int j = 0; j < RPT; ++j)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int c = c8 + q;
              double2 nv;
              nv.x = fma(-m[j].x, pr[q].x, fma(m[j].y, pr[q].y, v[j][c].x));
              nv.y = fma(-m[j].x, pr[q].y, fma(-m[j].y, pr[q].x, v[j][c].y));
              if (c == kc && srch) nv = newk[j];
              v[j][c] = nv;
            }
        }
        if (tid == 0) {
          piv_of[k] = p;
          prow[k0 + k] = p;
        }
        singular = singular || !(pm > 0.0);
      }
    }
  }
  __syncthreads();

  // write back the panel columns and the shifted transform Wp (the panel minus a unit at
  // each pivot: row piv_of[k] of column k), one half at a time through the stage, and the
  // usage flags
  double2* __restrict__ Wp = w.Wp + (int64_t)z * n * NB;
  for (int hh = 0; hh < 2; ++hh) {
    if (h == hh) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = l + 256 * j;
        if (r < n) {
#pragma unroll
          for (int c = 0; c < HB; ++c) stage[r * SP + c] = v[j][c];
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < tot; e += PT32) {
      const int row = e >> 4, gc = HB * hh + (e & 15);
      const double2 val = stage[row * SP + (e & 15)];
      double2 wv = cmk(0.0, 0.0);
      if (gc < nbw) {
        Xz[(int64_t)row * n + k0 + gc] = val;
        wv = val;
        if (piv_of[gc] == row) wv.x -= 1.0;
      }
      Wp[(int64_t)row * NB + gc] = wv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = l + 256 * j;
    if (r < n && h == 0 && pivcol[j] >= 0) used[r] = 1;
  }
  // pivot rows of this panel (pre-update values outside the panel), panel columns zeroed
  double2* __restrict__ Tp = w.Tp + (int64_t)z * NB * n;
  for (int base = 0; base < NB * n; base += PT32 * 8) {
    double2 val[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = base + PT32 * q + tid;
      const int k = idx / n, c = idx - k * n;
      val[q] = cmk(0.0, 0.0);
      if (idx < NB * n && k < nbw && (c < k0 || c >= k0 + nbw)) val[q] = Xz[(int64_t)piv_of[k] * n + c];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = base + PT32 * q + tid;
      if (idx < NB * n) Tp[idx] = val[q];
    }
  }
  if (tid == 0 && singular && status) status[z] = 5;   // QTX_ERR_SINGULAR
}

__global__ void gje_reset_kernel(int n, int batch, int32_t* used) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)n * batch) used[i] = 0;
}

// Out[r][c] = X[pivot(r)][pivot^-1(c)]; NaN for singular matrices.
__global__ __launch_bounds__(256) void gje_unscramble_kernel(int n, const double2* X, int64_t sX,
                                                             double2* Out, int64_t sOut,
                                                             double2* const* tOut,
                                                             const int32_t* prow_all,
                                                             const int32_t* status) {
  extern __shared__ int perm[];   // [2n]: pivot, inverse pivot
  const int z = blockIdx.y;
  const int32_t* prow = prow_all + (int64_t)z * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int q = prow[i];
    perm[i] = ((unsigned)q < (unsigned)n) ? q : 0;
    perm[n + i] = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) perm[n + perm[i]] = i;
  __syncthreads();
  const bool bad = status && status[z] == 5;
  const double nan = __builtin_nan("");
  const double2* Xz = X + (int64_t)z * sX;
  double2* Oz = tOut ? tOut[z] : Out + (int64_t)z * sOut;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n), c = (int)(e - (int64_t)r * n);
    double2 val = Xz[(int64_t)perm[r] * n + perm[n + c]];
    if (bad) val = cmk(nan, nan);
    Oz[e] = val;
  }
}

}  // namespace

int gje_panel_width(int n) {
  if (n <= 512) return 32;
  return 16;   // n <= 1024
}

size_t gje_work_bytes(int n, int batch) {
  const int nb = gje_panel_width(n);
  size_t bytes = 0;
  bytes += (size_t)batch * n * nb * sizeof(double2);   // Wp
  bytes += (size_t)batch * nb * n * sizeof(double2);   // Tp
  bytes += (size_t)batch * n * sizeof(int32_t) * 2;     // prow, used
  return bytes + 1024;
}

GjeWork gje_carve(void* base, int n, int batch) {
  const int nb = gje_panel_width(n);
  GjeWork w;
  char* p = (char*)base;
  w.Wp = (double2*)p; p += (size_t)batch * n * nb * sizeof(double2);
  w.Tp = (double2*)p; p += (size_t)batch * nb * n * sizeof(double2);
  w.prow = (int32_t*)p; p += (size_t)batch * n * sizeof(int32_t);
  w.used = (int32_t*)p;
  return w;
}

hipError_t launch_gje_invert(int n, double2* X, int64_t sX, double2* Out, int64_t sOut, int batch,
                             const GjeWork& w, int32_t* status, hipStream_t s, double2* const* tOut) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  if (n > 1024 || !X || (!Out && !tOut)) return hipErrorInvalidValue;
  const int nb = gje_panel_width(n);
  {
    const int64_t tot = (int64_t)n * batch;
    hipLaunchKernelGGL(gje_reset_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, batch, w.used);
  }
  for (int k0 = 0; k0 < n; k0 += nb) {
    if (nb == 32) hipLaunchKernelGGL(gje_panel32_kernel, dim3(batch), dim3(PT32), 0, s, n, k0, X, sX, w, status);
    else hipLaunchKernelGGL((gje_panel_kernel<16, 2>), dim3(batch), dim3(PT), 0, s, n, k0, X, sX, w, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int kw = (n - k0 < nb) ? n - k0 : nb;
    if (kw == n) continue;   // a single panel covers the matrix: nothing outside it
    // X += Wp * Tp  (the panel's trailing update, FP64 matrix cores)
    GemmDesc d;
    d.M = n; d.N = n; d.K = kw;
    d.opA = OP_N; d.opB = OP_N;
    d.A = w.Wp; d.lda = nb; d.sA = (int64_t)n * nb;
    d.B = w.Tp; d.ldb = n; d.sB = (int64_t)nb * n;
    d.C = X; d.ldc = n; d.sC = sX;
    d.alpha = cmk(1.0, 0.0);
    d.add[0].X = X; d.add[0].ld = n; d.add[0].stride = sX; d.add[0].coef = cmk(1.0, 0.0);
    d.batch = batch;
    d.skip_c0 = k0; d.skip_c1 = k0 + kw;   // Tp is zero in the panel's columns
    e = launch_zgemm_f64(d, s, GEMM_INV_UPDATE);
    if (e != hipSuccess) return e;
  }
  const int64_t nn = (int64_t)n * n;
  unsigned gx = (unsigned)((nn + 256 * 4 - 1) / (256 * 4));
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(gje_unscramble_kernel, dim3(gx, batch), dim3(256), 2 * n * sizeof(int), s, n, X, sX, Out, sOut,
                     tOut, w.prow, status);
  return hipGetLastError();
}

}  // namespace qtx
