// Triangular solves with the per-mode LU factors and the complex128 residual
// of the refinement loop (Section 6: further right-hand sides reuse the
// factors of each mode).
//
// Right-hand sides are grouped into vector batches: up to kVB = 16 vectors
// that use the same factors (a mode m and its mirror -m share them, since
// A_{-m} = D A_m D and the D's are applied when the right-hand sides are
// prepared).  One pass over a factor then serves every vector of the batch,
// and every product below is a 16-row x 16-vector MFMA tile.
//
// Solve = gather by the pivot permutation, then one launch per 64-row block
// for the forward (unit L) and backward (U) sweeps.  The inverses of the
// 64 x 64 diagonal blocks of L and U are formed once per factorization, so a
// launch for block i is two dense products: every workgroup forms
// x_i = inv(T_ii) b_i from the current b_i (redundantly; the block sits in
// L2), workgroup 0 stores x_i in the output array, and each workgroup
// subtracts T[c, i] x_i from one 64-row chunk c of the rows not yet solved.
// Input and output arrays differ, so no workgroup reads a row another one
// writes in the same launch.
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };

template <typename T>
__device__ __forceinline__ T cfms(T acc, T a, T b) {  // acc - a b
  acc.x -= a.x * b.x - a.y * b.y;
  acc.y -= a.x * b.y + a.y * b.x;
  return acc;
}

// 16x16x4 MFMA per real type.  Operands: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element i of lane l is C[row(l, i)][l % 16].
template <typename R> struct Mf;
template <> struct Mf<double> {
  using C4 = __attribute__((ext_vector_type(4))) double;
  static __device__ __forceinline__ C4 op(double a, double b, C4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <> struct Mf<float> {
  using C4 = __attribute__((ext_vector_type(4))) float;
  static __device__ __forceinline__ C4 op(float a, float b, C4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// (cr, ci) += A[16 rows x 64 cols] * B[64 x 16], complex: the wave's 16 rows
// start at Arow (leading dimension ld), only columns < kmax and rows with
// row_ok are read; B is a [64][kVB] tile in LDS.
template <typename R>
__device__ __forceinline__ void tile_mma(const typename C2<R>::T* Arow, size_t ld, bool row_ok, int kmax,
                                         const typename C2<R>::T (*B)[kVB], typename Mf<R>::C4& cr,
                                         typename Mf<R>::C4& ci) {
  using T = typename C2<R>::T;
  const int lane = threadIdx.x & 63;
  const T* ap = Arow + (size_t)(lane & 15) * ld + (lane >> 4);
  T a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int k = 4 * s + (lane >> 4);
    a[s] = (row_ok && k < kmax) ? ap[4 * s] : T{0, 0};
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const T b = B[4 * s + (lane >> 4)][lane & 15];
    cr = Mf<R>::op(a[s].x, b.x, cr);
    cr = Mf<R>::op(-a[s].y, b.y, cr);
    ci = Mf<R>::op(a[s].x, b.y, ci);
    ci = Mf<R>::op(a[s].y, b.x, ci);
  }
}

// Inverses of the 64 x 64 diagonal blocks of the unit-lower L and upper U
// (zero beyond the matrix order), inv[f][blk][0] = L^-1, inv[f][blk][1] = U^-1.
// Thread j forms column j by substitution; columns live in LDS.
template <typename R>
__global__ __launch_bounds__(64) void inv_diag(const typename C2<R>::T* LU, long long stride, int n,
                                               typename C2<R>::T* inv) {
  using T = typename C2<R>::T;
  __shared__ T D[64][65];
  __shared__ T Y[64][64];
  const int blk = blockIdx.x, f = blockIdx.y, j = threadIdx.x;
  const int nblk = (n + 63) / 64;
  const int rb = blk * 64;
  const int h = min(64, n - rb);
  const T* M = LU + (size_t)f * stride;
  const T zero = {0, 0};
  for (int r = 0; r < 64; ++r) D[r][j] = load_or_zero(M + (size_t)(rb + r) * n + rb + j, r < h && j < h);
  __syncthreads();
  T* out = inv + ((size_t)f * nblk + blk) * 2 * 64 * 64;
  // L^-1 column j: y_r = [r == j] - sum_{j <= k < r} L[r][k] y_k
  for (int r = 0; r < 64; ++r) {
    T y = (r == j && r < h) ? T{1, 0} : zero;
    if (r < h && r > j)
      for (int k = j; k < r; ++k) y = cfms(y, D[r][k], Y[k][j]);
    Y[r][j] = y;
  }
  for (int r = 0; r < 64; ++r) out[r * 64 + j] = Y[r][j];
  // U^-1 column j: y_r = ([r == j] - sum_{r < k <= j} U[r][k] y_k) / U[r][r]
  for (int r = 63; r >= 0; --r) {
    T y = zero;
    if (r < h && r <= j && j < h) {
      y = (r == j) ? T{1, 0} : zero;
      for (int k = r + 1; k <= j; ++k) y = cfms(y, D[r][k], Y[k][j]);
      const T d = D[r][r];
      const R den = d.x * d.x + d.y * d.y;
      T q;
      q.x = (y.x * d.x + y.y * d.y) / den;
      q.y = (y.y * d.x - y.x * d.y) / den;
      y = q;
    }
    Y[r][j] = y;
  }
  for (int r = 0; r < 64; ++r) out[64 * 64 + r * 64 + j] = Y[r][j];
}

// perm[f][i]: source row of row i after the LAPACK-style interchanges ipiv[f]
// (row k swapped with ipiv[k], k ascending).  One workgroup per factor.
__global__ __launch_bounds__(256) void build_perm(const int32_t* ipiv, int32_t* perm, int n) {
  extern __shared__ int32_t idx[];
  const int32_t* piv = ipiv + (size_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) idx[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < n; ++k) {
      int p = piv[k];
      if (p != k) {
        int t = idx[k];
        idx[k] = idx[p];
        idx[p] = t;
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) perm[(size_t)blockIdx.x * n + i] = idx[i];
}

// out[v][i] = in[v][perm[fac(v)][i]] (optionally rounded to complex64)
template <typename TO>
__global__ __launch_bounds__(256) void gather_perm(const double2* in, TO* out, const int32_t* perm,
                                                   const VecBatch* vb, int n) {
  const VecBatch& b = vb[blockIdx.y];
  const int32_t* pm = perm + (size_t)b.fac * n;
  for (int v = 0; v < b.nv; ++v) {
    const size_t o = (size_t)b.off[v] * n;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
      double2 a = in[o + pm[i]];
      TO t;
      t.x = a.x;
      t.y = a.y;
      out[o + i] = t;
    }
  }
}

template <typename R, bool FWD>
__global__ __launch_bounds__(256) void tri_step(const typename C2<R>::T* LU, const typename C2<R>::T* inv,
                                                long long stride, int n, const VecBatch* vb,
                                                typename C2<R>::T* X, typename C2<R>::T* Y, int blk) {
  using T = typename C2<R>::T;
  using C4 = typename Mf<R>::C4;
  __shared__ T xb[64][kVB];  // b_i
  __shared__ T xi[64][kVB];  // x_i
  __shared__ int s_off[kVB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const VecBatch& b = vb[blockIdx.y];
  const int nv = b.nv;
  if (tid < kVB) s_off[tid] = tid < nv ? b.off[tid] : 0;
  __syncthreads();
  const int nblk = (n + 63) / 64;
  const int rb = blk * 64;
  const int h = min(64, n - rb);
  for (int e = tid; e < kVB * 64; e += 256) {
    const int v = e >> 6, k = e & 63;
    xb[k][v] = load_or_zero(X + (size_t)s_off[v] * n + rb + k, v < nv && k < h);
  }
  __syncthreads();
  // x_i = inv(T_ii) b_i, wave w: rows 16w .. 16w+15
  const T* Inv = inv + (((size_t)b.fac * nblk + blk) * 2 + (FWD ? 0 : 1)) * 64 * 64;
  C4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  tile_mma<R>(Inv + (size_t)(16 * w) * 64, 64, true, 64, xb, cr, ci);
#pragma unroll
  for (int i = 0; i < 4; ++i) xi[16 * w + Mf<R>::row(lane, i)][lane & 15] = T{cr[i], ci[i]};
  __syncthreads();
  if (blockIdx.x == 0)
    for (int e = tid; e < kVB * 64; e += 256) {
      const int v = e >> 6, k = e & 63;
      if (v < nv && k < h) Y[(size_t)s_off[v] * n + rb + k] = xi[k][v];
    }
  const int c = FWD ? blk + 1 + (int)blockIdx.x : (int)blockIdx.x;
  if (FWD ? (c >= nblk) : (c >= blk)) return;
  const int cb = c * 64;
  const int hc = min(64, n - cb);
  const T* M = LU + (size_t)b.fac * stride;
  cr = C4{0, 0, 0, 0};
  ci = C4{0, 0, 0, 0};
  const int r0 = 16 * w;
  tile_mma<R>(M + (size_t)(cb + r0) * n + rb, n, r0 + (lane & 15) < hc, h, xi, cr, ci);
  const int v = lane & 15;
  if (v < nv)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + Mf<R>::row(lane, i);
      if (r < hc) {
        T* xp = X + (size_t)s_off[v] * n + cb + r;
        T o = *xp;
        o.x -= cr[i];
        o.y -= ci[i];
        *xp = o;
      }
    }
}

// r_v = b_v - A[fac] x_v (complex128).  Workgroup: 64 rows (16 per wave);
// x is staged in 64-column tiles.
__global__ __launch_bounds__(256) void residual_b(const double2* A, long long stride, int n,
                                                  const VecBatch* vb, const double2* bv,
                                                  const double2* x, double2* r) {
  using C4 = Mf<double>::C4;
  __shared__ double2 xt[64][kVB];
  __shared__ int s_off[kVB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const VecBatch& b = vb[blockIdx.y];
  const int nv = b.nv;
  if (tid < kVB) s_off[tid] = tid < nv ? b.off[tid] : 0;
  const double2* M = A + (size_t)b.fac * stride;
  const int r0 = blockIdx.x * 64 + 16 * w;
  const bool row_ok = r0 + (lane & 15) < n;
  C4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += 64) {
    __syncthreads();
    for (int e = tid; e < kVB * 64; e += 256) {
      const int v = e >> 6, k = e & 63;
      xt[k][v] = (v < nv && k0 + k < n) ? x[(size_t)s_off[v] * n + k0 + k] : double2{0, 0};
    }
    __syncthreads();
    tile_mma<double>(M + (size_t)r0 * n + k0, n, row_ok, n - k0, xt, cr, ci);
  }
  const int v = lane & 15;
  if (v < nv)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = r0 + Mf<double>::row(lane, i);
      if (row < n) {
        const size_t o = (size_t)s_off[v] * n + row;
        const double2 bb = bv[o];
        r[o] = double2{bb.x - cr[i], bb.y - ci[i]};
      }
    }
}

template <typename R>
hipError_t solve_batches(const typename C2<R>::T* LU, const typename C2<R>::T* inv, long long stride, int n,
                         const VecBatch* d_vb, int nvb, typename C2<R>::T* X, typename C2<R>::T* Y,
                         hipStream_t s) {
  const int nblk = (n + 63) / 64;
  for (int i = 0; i < nblk; ++i) {
    const int chunks = nblk - i - 1;
    hipLaunchKernelGGL((tri_step<R, true>), dim3(chunks > 0 ? chunks : 1, nvb), dim3(256), 0, s, LU, inv, stride,
                       n, d_vb, X, Y, i);
  }
  for (int i = nblk - 1; i >= 0; --i) {
    const int chunks = i;
    hipLaunchKernelGGL((tri_step<R, false>), dim3(chunks > 0 ? chunks : 1, nvb), dim3(256), 0, s, LU, inv,
                       stride, n, d_vb, Y, X, i);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t lu_perm(const int32_t* ipiv, int32_t* perm, int n, int nfac, hipStream_t s) {
  hipLaunchKernelGGL(build_perm, dim3(nfac), dim3(256), sizeof(int32_t) * n, s, ipiv, perm, n);
  return hipGetLastError();
}

hipError_t gather_z(const double2* in, double2* out, const int32_t* perm, const VecBatch* d_vb, int nvb, int n,
                    hipStream_t s) {
  hipLaunchKernelGGL(gather_perm<double2>, dim3((n + 255) / 256, nvb), dim3(256), 0, s, in, out, perm, d_vb, n);
  return hipGetLastError();
}

hipError_t gather_c(const double2* in, float2* out, const int32_t* perm, const VecBatch* d_vb, int nvb, int n,
                    hipStream_t s) {
  hipLaunchKernelGGL(gather_perm<float2>, dim3((n + 255) / 256, nvb), dim3(256), 0, s, in, out, perm, d_vb, n);
  return hipGetLastError();
}

hipError_t lu_inv_diag_z(const double2* LU, long long stride, int n, int nfac, double2* inv, hipStream_t s) {
  hipLaunchKernelGGL(inv_diag<double>, dim3((n + 63) / 64, nfac), dim3(64), 0, s, LU, stride, n, inv);
  return hipGetLastError();
}
hipError_t lu_inv_diag_c(const float2* LU, long long stride, int n, int nfac, float2* inv, hipStream_t s) {
  hipLaunchKernelGGL(inv_diag<float>, dim3((n + 63) / 64, nfac), dim3(64), 0, s, LU, stride, n, inv);
  return hipGetLastError();
}

// X holds P b on entry; on return X holds A^{-1} b and Y is scratch.
hipError_t trsv_z(const double2* LU, const double2* inv, long long stride, int n, const VecBatch* d_vb, int nvb,
                  double2* X, double2* Y, hipStream_t s) {
  return solve_batches<double>(LU, inv, stride, n, d_vb, nvb, X, Y, s);
}
hipError_t trsv_c(const float2* LU, const float2* inv, long long stride, int n, const VecBatch* d_vb, int nvb,
                  float2* X, float2* Y, hipStream_t s) {
  return solve_batches<float>(LU, inv, stride, n, d_vb, nvb, X, Y, s);
}

hipError_t residual_batches(const double2* A, long long stride, int n, const VecBatch* d_vb, int nvb,
                            const double2* b, const double2* x, double2* r, hipStream_t s) {
  hipLaunchKernelGGL(residual_b, dim3((n + 63) / 64, nvb), dim3(256), 0, s, A, stride, n, d_vb, b, x, r);
  return hipGetLastError();
}

}  // namespace msv
