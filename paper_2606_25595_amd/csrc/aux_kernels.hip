// Small HBM-bound helper kernels: status handling, NaN fill of failed energies,
// and the per-energy transport observables (traces of block products).
#include "qtx_internal.h"

namespace qtx {

namespace {

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Deterministic pseudo-random complex values in [-1, 1) x [-1, 1) (an integer
// hash of the index and seed; synthetic operands for timing runs).
__device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}
__global__ void fill_hash_kernel(double2* p, int64_t n, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t h = mix32((uint32_t)i ^ mix32(seed ^ (uint32_t)(i >> 32)));
  const uint32_t g = mix32(h ^ 0x9e3779b9U);
  p[i] = make_double2((double)(h >> 8) * (1.0 / 8388608.0) - 1.0, (double)(g >> 8) * (1.0 / 8388608.0) - 1.0);
}

// Fill the per_batch elements of batch entry z with NaN when status[z] != 0.
__global__ void nan_fill_kernel(double2* X, int64_t per_batch, int64_t stride, const int32_t* status) {
  const int z = blockIdx.y;
  if (status[z] == 0) return;
  const double nan = __builtin_nan("");
  double2* Xz = X + (int64_t)z * stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_batch; i += (int64_t)gridDim.x * blockDim.x)
    Xz[i] = cmk(nan, nan);
}

// status[z] = NONFINITE if any of the per_batch elements of entry z is NaN/Inf
// (only a status that is still OK is changed).
__global__ void check_finite_kernel(const double2* X, int64_t per_batch, int64_t stride, int32_t* status) {
  const int z = blockIdx.y;
  const double2* Xz = X + (int64_t)z * stride;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_batch; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = Xz[i];
    bad |= !(isfinite(v.x) && isfinite(v.y));
  }
  bad = __syncthreads_or(bad);
  if (bad && threadIdx.x == 0) atomicCAS(status + z, 0, 6);   // QTX_ERR_NONFINITE
}

__global__ void check_finite_entries_kernel(const double2* const* t, int64_t count, int32_t* status) {
  const int z = blockIdx.y;
  const double2* Xz = t[z];
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = Xz[i];
    bad |= !(isfinite(v.x) && isfinite(v.y));
  }
  bad = __syncthreads_or(bad);
  if (bad && threadIdx.x == 0) atomicCAS(status + z, 0, 6);   // QTX_ERR_NONFINITE
}

__global__ void nan_fill_entries_kernel(double2* const* t, const int64_t* counts, const int32_t* status) {
  const int z = blockIdx.y;
  if (status[z] == 0) return;
  const double nan = __builtin_nan("");
  double2* Xz = t[z];
  const int64_t n = counts[z];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Xz[i] = cmk(nan, nan);
}

// Top half of a split energy (part[z] >= 0) takes its bottom half's failure.  Only
// top halves are written and only bottom halves are read.
__global__ void status_merge_kernel(int32_t* st, const int32_t* part, int n) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < n && part[z] >= 0 && st[z] == 0) st[z] = st[part[z]];
}

// X <- -X^H in place for each b x b block t[m]: one workgroup per pair of 32 x 32
// tiles (ti <= tj), both staged in LDS before either is written.
__global__ __launch_bounds__(256) void neg_ctrans_kernel(double2* const* t, int b, int count) {
  __shared__ double2 ta[32][33], tb[32][33];
  const int nt = (b + 31) / 32;
  int q = blockIdx.x, ti = 0;
  while (q >= nt - ti) { q -= nt - ti; ++ti; }
  const int tj = ti + q;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int m = blockIdx.y; m < count; m += gridDim.y) {
    double2* X = t[m];
    for (int k = ty; k < 32; k += 8) {
      int r = ti * 32 + k, c = tj * 32 + tx;
      if (r < b && c < b) ta[k][tx] = X[(int64_t)r * b + c];
      r = tj * 32 + k; c = ti * 32 + tx;
      if (r < b && c < b) tb[k][tx] = X[(int64_t)r * b + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      int r = ti * 32 + k, c = tj * 32 + tx;
      if (r < b && c < b) { const double2 v = tb[tx][k]; X[(int64_t)r * b + c] = cmk(-v.x, v.y); }
      r = tj * 32 + k; c = ti * 32 + tx;
      if (r < b && c < b) { const double2 v = ta[tx][k]; X[(int64_t)r * b + c] = cmk(-v.x, v.y); }
    }
    __syncthreads();
  }
}

// dst[m] = -src[m]^H for `count` b x b blocks: one workgroup per 32 x 32 tile of dst,
// the source tile staged in LDS.
__global__ __launch_bounds__(256) void neg_ctrans_copy_kernel(const double2* const* src, double2* const* dst, int b,
                                                              int count) {
  __shared__ double2 tl[32][33];
  const int nt = (b + 31) / 32;
  const int ti = blockIdx.x % nt, tj = blockIdx.x / nt;   // dst tile (ti, tj) <- src tile (tj, ti)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int m = blockIdx.y; m < count; m += gridDim.y) {
    const double2* S = src[m];
    double2* D = dst[m];
    for (int k = ty; k < 32; k += 8) {
      const int r = tj * 32 + k, c = ti * 32 + tx;
      if (r < b && c < b) tl[k][tx] = S[(int64_t)r * b + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int r = ti * 32 + k, c = tj * 32 + tx;
      if (r < b && c < b) { const double2 v = tl[tx][k]; D[(int64_t)r * b + c] = cmk(-v.x, v.y); }
    }
    __syncthreads();
  }
}

__global__ void scatter_status_kernel(const int32_t* st, int32_t* const* dst, int n) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < n && dst[z]) *dst[z] = st[z];
}

// Per energy e (one workgroup): with M1 = Gamma G, M2 = Gamma G^H,
//   Tr[Gamma A] = Re(i (Tr M1 - Tr M2)),   Tr[Gamma G Gamma G^H] = Tr[M1 M2],
//   T = Tr[Gamma A] - Re Tr[M1 M2],  j = Re(i Tr[Gamma G^<]) + f Tr[Gamma A].
// Fixed-order FP64 reduction (deterministic).
__global__ __launch_bounds__(256) void observables_kernel(int b, const double2* GL, int64_t sG,
                                                          const double2* M1, const double2* M2,
                                                          const double2* gam, const double* fL,
                                                          double* T, double* jout) {
  const int e = blockIdx.x;
  const double2* m1 = M1 + (int64_t)e * b * b;
  const double2* m2 = M2 + (int64_t)e * b * b;
  const double2* gl = GL + (int64_t)e * sG;
  double acc[6] = {0, 0, 0, 0, 0, 0};   // Tr M1M2 (re), Im Tr M1, Im Tr M2, Tr Gamma G^< (re, im), unused
  const int64_t bb = (int64_t)b * b;
  for (int64_t idx = threadIdx.x; idx < bb; idx += blockDim.x) {
    const int i = (int)(idx / b), j = (int)(idx - (int64_t)i * b);
    const double2 p = cmul(m1[idx], m2[(int64_t)j * b + i]);
    acc[0] += p.x;
    const double2 q = cmul(gam[idx], gl[(int64_t)j * b + i]);
    acc[3] += q.x;
    acc[4] += q.y;
    if (i == j) { acc[1] += m1[idx].y; acc[2] += m2[idx].y; }
  }
  __shared__ double sh[5][256];
  for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double trGA = -(sh[1][0] - sh[2][0]);      // Re(i z) = -Im z
    T[e] = trGA - sh[0][0];
    jout[e] = -sh[4][0] + fL[e] * trGA;
  }
}

// Bond current of energy e = blockIdx.y across bond i = blockIdx.x (Section II-B uses the
// current and its conservation as the accuracy criterion):
//   J = 2 Re Tr[(H_{i,i+1} - E S_{i,i+1}) G^<_{i+1,i}],   G^<_{i+1,i} = -(G^<_{i,i+1})^H,
// so J = -2 sum_jk Re(c_jk conj(g_jk)) with c the coupling and g = G^<_{i,i+1}.
// Fixed-order FP64 reduction (deterministic).
__global__ __launch_bounds__(256) void bond_current_kernel(int b, int nbond, const double2* Hu, const double2* Su,
                                                           const double* E, const double2* GLu, int64_t sGu,
                                                           double* J) {
  const int i = blockIdx.x, e = blockIdx.y;
  const int64_t bb = (int64_t)b * b;
  const double2* h = Hu + (int64_t)i * bb;
  const double2* sm = Su ? Su + (int64_t)i * bb : nullptr;
  const double2* g = GLu + (int64_t)e * sGu + (int64_t)i * bb;
  const double en = E[e];
  double acc = 0.0;
  for (int64_t idx = threadIdx.x; idx < bb; idx += blockDim.x) {
    double2 c = h[idx];
    if (sm) { c.x = fma(-en, sm[idx].x, c.x); c.y = fma(-en, sm[idx].y, c.y); }
    const double2 v = g[idx];
    acc = fma(c.x, v.x, fma(c.y, v.y, acc));
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[(int64_t)e * nbond + i] = -2.0 * sh[0];
}

}  // namespace

hipError_t launch_bond_currents(int b, int n_b, int n_e, const double2* Hu, const double2* Su, const double* E,
                                const double2* GLu, int64_t sGu, double* J, hipStream_t s) {
  if (n_b < 2 || n_e <= 0) return hipSuccess;
  hipLaunchKernelGGL(bond_current_kernel, dim3(n_b - 1, n_e), dim3(256), 0, s, b, n_b - 1, Hu, Su, E, GLu, sGu, J);
  return hipGetLastError();
}

hipError_t launch_fill_hash(double2* p, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_hash_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_nan_fill_failed(double2* X, int64_t per_batch, int64_t stride, int batch,
                                  const int32_t* status, hipStream_t s) {
  if (per_batch <= 0 || batch <= 0) return hipSuccess;
  int64_t g = (per_batch + 1023) / 1024;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(nan_fill_kernel, dim3((unsigned)g, batch), dim3(256), 0, s, X, per_batch, stride, status);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double2* X, int64_t per_batch, int64_t stride, int batch,
                               int32_t* status, hipStream_t s) {
  if (per_batch <= 0 || batch <= 0) return hipSuccess;
  int64_t g = (per_batch + 1023) / 1024;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)g, batch), dim3(256), 0, s, X, per_batch, stride, status);
  return hipGetLastError();
}

hipError_t launch_check_finite_entries(const double2* const* t, int64_t count, int batch, int32_t* status,
                                       hipStream_t s) {
  if (count <= 0 || batch <= 0) return hipSuccess;
  if (!t) return hipErrorInvalidValue;
  int64_t g = (count + 1023) / 1024;
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(check_finite_entries_kernel, dim3((unsigned)g, batch), dim3(256), 0, s, t, count, status);
  return hipGetLastError();
}

hipError_t launch_nan_fill_entries(double2* const* t, const int64_t* counts, int batch, const int32_t* status,
                                   hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (!t) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nan_fill_entries_kernel, dim3(256, batch), dim3(256), 0, s, t, counts, status);
  return hipGetLastError();
}

hipError_t launch_status_merge(int32_t* st, const int32_t* part, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(status_merge_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, st, part, batch);
  return hipGetLastError();
}

hipError_t launch_neg_ctrans_entries(double2* const* t, int b, int count, hipStream_t s) {
  if (count <= 0 || b <= 0) return hipSuccess;
  if (!t) return hipErrorInvalidValue;
  const int nt = (b + 31) / 32;
  const int gy = count < 65535 ? count : 65535;
  hipLaunchKernelGGL(neg_ctrans_kernel, dim3((unsigned)(nt * (nt + 1) / 2), gy), dim3(256), 0, s, t, b, count);
  return hipGetLastError();
}

hipError_t launch_neg_ctrans_copy(const double2* const* src, double2* const* dst, int b, int count, hipStream_t s) {
  if (count <= 0 || b <= 0) return hipSuccess;
  if (!src || !dst) return hipErrorInvalidValue;
  const int nt = (b + 31) / 32;
  const int gy = count < 65535 ? count : 65535;
  hipLaunchKernelGGL(neg_ctrans_copy_kernel, dim3((unsigned)(nt * nt), gy), dim3(256), 0, s, src, dst, b, count);
  return hipGetLastError();
}

hipError_t launch_scatter_status(const int32_t* st, int32_t* const* dst, int batch, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_status_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, st, dst, batch);
  return hipGetLastError();
}

hipError_t launch_observables(int b, int n_e, const double2* G, const double2* GL, int64_t sG,
                              const double2* M1, const double2* M2, const double2* gam,
                              const double* fL, double* T, double* j, hipStream_t s) {
  (void)G;
  if (n_e <= 0) return hipSuccess;
  hipLaunchKernelGGL(observables_kernel, dim3(n_e), dim3(256), 0, s, b, GL, sG, M1, M2, gam, fL, T, j);
  return hipGetLastError();
}

}  // namespace qtx
