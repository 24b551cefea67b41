// Per-mode factorization and solve drivers (Section 6: LU per mode, further
// right-hand sides reuse the factors), with the complex64-LU + complex128
// iterative-refinement variant: x <- x + LU32^{-1} (b - A x), the residual in
// complex128 with the complex128 matrix, until ||b - A x|| <= tol ||b||.
//
// Right-hand sides arrive unweighted; the stored matrices are the L^2-weighted
// ones (A~ = W^{1/2} A W^{-1/2}), so b~ = W^{1/2} b and x = W^{-1/2} x~.
// Negative modes reuse the factors of |m| through A_{-m} = D A_m D,
// D = diag(1, -1, -1, 1) per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "msv_internal.h"

struct msv_plan;  // defined in plan.hip; accessed through the helpers below

namespace msv {
namespace {

__device__ __forceinline__ double parity(int m, int row) {
  if (m >= 0) return 1.0;
  int c = row & 3;
  return (c == 1 || c == 2) ? -1.0 : 1.0;
}

// xw[i][q][row] = D(m_i) sqrt(w[row/4]) rhs[i][q][row]
__global__ void prep_rhs(const double2* rhs, double2* xw, const double* sqw, int n, int nrhs, int m_lo) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t tot = (size_t)gridDim.y * nrhs * n;
  (void)tot;
  int i = blockIdx.y;
  if (e >= (size_t)nrhs * n) return;
  int row = (int)(e % n);
  double s = parity(m_lo + i, row) * sqw[row >> 2];
  double2 v = rhs[(size_t)i * nrhs * n + e];
  xw[(size_t)i * nrhs * n + e] = make_double2(s * v.x, s * v.y);
}

// x[i][q][row] = D(m_i) xw[i][q][row] / sqrt(w[row/4])
__global__ void finish_x(const double2* xw, double2* x, const double* sqw, int n, int nrhs, int m_lo) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (e >= (size_t)nrhs * n) return;
  int row = (int)(e % n);
  double s = parity(m_lo + i, row) / sqw[row >> 2];
  double2 v = xw[(size_t)i * nrhs * n + e];
  x[(size_t)i * nrhs * n + e] = make_double2(s * v.x, s * v.y);
}

// Elementwise kernels walk their range in strides of the whole grid: a
// dispatch counts its work-items in 32 bits, so one work-item per element
// would wrap for the 8.7e9 elements of 129 matrices of order 8192.
__global__ void to_c64(const double2* a, float2* b, size_t count) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += step) {
    double2 v = a[e];
    b[e] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void add_c64(double2* x, const float2* d, size_t count) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += step) {
    double2 v = x[e];
    float2 u = d[e];
    x[e] = make_double2(v.x + (double)u.x, v.y + (double)u.y);
  }
}

__global__ void fill_zero(double2* x, size_t count) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += step)
    x[e] = make_double2(0.0, 0.0);
}

// ratio[i*nrhs+q] = max|r| / max|b| over the vector
__global__ __launch_bounds__(256) void ratio_inf(const double2* r, const double2* b, double* out, int n) {
  const size_t v = blockIdx.x;
  __shared__ double sr[256], sb[256];
  double mr = 0, mb = 0;
  for (int j = threadIdx.x; j < n; j += 256) {
    double2 a = r[v * n + j], c = b[v * n + j];
    mr = fmax(mr, fabs(a.x) + fabs(a.y));
    mb = fmax(mb, fabs(c.x) + fabs(c.y));
  }
  sr[threadIdx.x] = mr;
  sb[threadIdx.x] = mb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + s]);
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sb[0] > 0 ? sr[0] / sb[0] : 0.0;
}

// out[0] = max of r[0 .. count)
__global__ __launch_bounds__(256) void max_reduce(const double* r, int count, double* out) {
  __shared__ double sm[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) v = fmax(v, r[i]);
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// The vectors of a solve over modes m_lo .. m_lo+nm-1 (n_rhs each), grouped
// by the factor f = |m| - fac_lo they use: for each f the vectors of mode -a,
// then of +a (a = fac_lo + f), right-hand sides in order, kVB to a batch.
// Record b is built by thread b; entries past a batch's count are 0, a valid
// offset.
__device__ __forceinline__ int modes_of(int a, int m_lo, int nm, int* idx) {
  int k = 0;
  const int i0 = -a - m_lo, i1 = a - m_lo;
  if (i0 >= 0 && i0 < nm) idx[k++] = i0;
  if (a != 0 && i1 >= 0 && i1 < nm) idx[k++] = i1;
  return k;
}

__global__ void vec_batches(VecBatch* vb, int nvb, int m_lo, int nm, int n_rhs, int fac_lo, int nfac) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nvb) return;
  int first = 0;
  for (int f = 0; f < nfac; ++f) {
    int idx[2];
    const int cnt = modes_of(fac_lo + f, m_lo, nm, idx) * n_rhs;
    const int nbf = (cnt + kVB - 1) / kVB;
    if (b < first + nbf) {
      const int j = b - first;
      VecBatch r;
      r.fac = f;
      r.nv = min(kVB, cnt - j * kVB);
      for (int v = 0; v < kVB; ++v) {
        const int g = j * kVB + v;
        r.off[v] = v < r.nv ? idx[g / n_rhs] * n_rhs + g % n_rhs : 0;
      }
      vb[b] = r;
      return;
    }
    first += nbf;
  }
}

// 256-thread workgroups, at most 2^20 of them (2^28 work-items; the kernels
// loop over the rest)
inline dim3 grid1(size_t count) { return dim3((unsigned)std::min<size_t>((count + 255) / 256, (size_t)1 << 20)); }

}  // namespace

int count_vec_batches(int m_lo, int nm, int n_rhs, int fac_lo, int nfac) {
  int nvb = 0;
  for (int f = 0; f < nfac; ++f) {
    const int a = fac_lo + f, i0 = -a - m_lo, i1 = a - m_lo;
    const int k = (i0 >= 0 && i0 < nm) + (a != 0 && i1 >= 0 && i1 < nm);
    nvb += (k * n_rhs + kVB - 1) / kVB;
  }
  return nvb;
}
hipError_t build_vec_batches(VecBatch* vb, int nvb, int m_lo, int nm, int n_rhs, int fac_lo, int nfac,
                             hipStream_t s) {
  hipLaunchKernelGGL(vec_batches, dim3((nvb + 63) / 64), dim3(64), 0, s, vb, nvb, m_lo, nm, n_rhs, fac_lo, nfac);
  return hipGetLastError();
}

hipError_t solve_prep(const double2* rhs, double2* xw, const double* sqw, int n, int nrhs, int nm, int m_lo,
                      hipStream_t s) {
  dim3 g((unsigned)(((size_t)nrhs * n + 255) / 256), nm);
  hipLaunchKernelGGL(prep_rhs, g, dim3(256), 0, s, rhs, xw, sqw, n, nrhs, m_lo);
  return hipGetLastError();
}
hipError_t solve_finish(const double2* xw, double2* x, const double* sqw, int n, int nrhs, int nm, int m_lo,
                        hipStream_t s) {
  dim3 g((unsigned)(((size_t)nrhs * n + 255) / 256), nm);
  hipLaunchKernelGGL(finish_x, g, dim3(256), 0, s, xw, x, sqw, n, nrhs, m_lo);
  return hipGetLastError();
}
hipError_t conv_c64(const double2* a, float2* b, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(to_c64, grid1(count), dim3(256), 0, s, a, b, count);
  return hipGetLastError();
}
hipError_t accum_c64(double2* x, const float2* d, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(add_c64, grid1(count), dim3(256), 0, s, x, d, count);
  return hipGetLastError();
}
hipError_t zero_c128(double2* x, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero, grid1(count), dim3(256), 0, s, x, count);
  return hipGetLastError();
}
hipError_t ratios(const double2* r, const double2* b, double* out, int n, int nvec, hipStream_t s) {
  hipLaunchKernelGGL(ratio_inf, dim3(nvec), dim3(256), 0, s, r, b, out, n);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  hipLaunchKernelGGL(max_reduce, dim3(1), dim3(256), 0, s, out, nvec, out + nvec);
  return hipGetLastError();
}

}  // namespace msv
