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
// 64 x 64 diagonal blocks of L and U are formed once per factorization.  The
// launch for block i subtracts T[c, i] x_i from every 64-row chunk c not yet
// solved (one workgroup per chunk); the workgroup of the next chunk then
// forms that block's solution x = inv(T_cc) b_c from its updated b_c and
// stores it, so the next launch reads it instead of recomputing it (only the
// first launch of a sweep forms its x_i itself, in every workgroup).  Input
// and output arrays differ, so no workgroup reads a row another one writes
// in the same launch.
//
// Operand layout of the 16x16x4 MFMA products here: lane group q = lane / 16
// takes k = 16 q + s at step s, so each lane reads 16 consecutive elements of
// its matrix row; LDS vector tiles keep k at row 4 (k % 16) + k / 16, so the
// four lane groups of a step read distinct banks.
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };

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

// LDS row of element k of a 64 x kVB vector tile.
__device__ __forceinline__ int pk(int k) { return 4 * (k & 15) + (k >> 4); }

// A 64 x kVB vector tile xs[pk(k)][v] = V[off_v n + rb + k] (vectors v < nv,
// k < h; zero elsewhere) staged by 256 threads in two steps, so that other
// loads can be issued between them: load_vectors issues the thread's four
// loads (element k = lane of the vectors v = wave + 4 i, whose offsets the
// caller passes in offs, 0 past nv), store_vectors zeroes what lies outside
// and writes the tile.
template <typename T>
__device__ __forceinline__ void load_vectors(T (&t)[4], const T* V, const int (&offs)[4], int n, int rb, int h) {
  const int k = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) t[i] = V[(size_t)offs[i] * n + rb + (k < h ? k : 0)];
}
template <typename T>
__device__ __forceinline__ void store_vectors(T (*xs)[kVB], T (&t)[4], int nv, int h) {
  const int k = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!(w + 4 * i < nv && k < h)) t[i].x = t[i].y = 0;
    xs[pk(k)][w + 4 * i] = t[i];
  }
}
// offs[i] = offset of vector w + 4 i of the batch (0 past nv); w is uniform
// over the wave, so these are scalar loads
__device__ __forceinline__ void batch_offsets(const VecBatch& b, int nv, int w, int (&offs)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = b.off[w + 4 * i];
    offs[i] = w + 4 * i < nv ? o : 0;
  }
}

// a[s] = p[s], s < 16, with 16-byte loads (p 16-byte aligned).
__device__ __forceinline__ void load_row16(const float2* p, float2 (&a)[16]) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float4 t = q[j];
    a[2 * j] = float2{t.x, t.y};
    a[2 * j + 1] = float2{t.z, t.w};
  }
}
__device__ __forceinline__ void load_row16(const double2* p, double2 (&a)[16]) {
#pragma unroll
  for (int j = 0; j < 16; ++j) a[j] = p[j];
}

// (cr, ci) += A[16 rows x 64 cols] * B[64 x 16], complex: the wave's 16 rows
// start at Arow (leading dimension ld, 16-byte aligned rows), only columns
// < kmax and rows with row_ok are read; B is a [64][kVB] tile in LDS with k at
// row pk(k).
// The lane's 16 operands of a 16 x 64 tile of A (rows Arow + li ld, columns
// 16 q .. 16 q + 15), zero past kmax or where !row_ok.
template <typename R>
__device__ __forceinline__ void tile_load(const typename C2<R>::T* Arow, size_t ld, bool row_ok, int kmax,
                                          typename C2<R>::T (&a)[16]) {
  using T = typename C2<R>::T;
  const int lane = threadIdx.x & 63, li = lane & 15, q = lane >> 4;
  const T* ap = Arow + (size_t)li * ld + 16 * q;
  if (row_ok && 16 * q + 16 <= kmax) {
    load_row16(ap, a);
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) a[s] = load_or_zero(ap + s, row_ok && 16 * q + s < kmax);
  }
}

// (cr, ci) += A B for the tile loaded by tile_load and the vector tile B
template <typename R>
__device__ __forceinline__ void tile_mul(const typename C2<R>::T (&a)[16], const typename C2<R>::T (*B)[kVB],
                                         typename Mf<R>::C4& cr, typename Mf<R>::C4& ci) {
  using T = typename C2<R>::T;
  using C4 = typename Mf<R>::C4;
  const int lane = threadIdx.x & 63, li = lane & 15, q = lane >> 4;
  // three real products per complex one: t1 = Ar Br, t2 = Ai Bi,
  // t3 = (Ar + Ai)(Br + Bi); Re = t1 - t2, Im = t3 - t1 - t2
  C4 t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const T b0 = B[4 * s + q][li];
    t1 = Mf<R>::op(a[s].x, b0.x, t1);
    t2 = Mf<R>::op(a[s].y, b0.y, t2);
    t3 = Mf<R>::op(a[s].x + a[s].y, b0.x + b0.y, t3);
  }
  cr += t1 - t2;
  ci += t3 - t1 - t2;
}

template <typename R>
__device__ __forceinline__ void tile_mma(const typename C2<R>::T* Arow, size_t ld, bool row_ok, int kmax,
                                         const typename C2<R>::T (*B)[kVB], typename Mf<R>::C4& cr,
                                         typename Mf<R>::C4& ci) {
  typename C2<R>::T a[16];
  tile_load<R>(Arow, ld, row_ok, kmax, a);
  tile_mul<R>(a, B, cr, ci);
}

// Inverses of the 64 x 64 diagonal blocks of the unit-lower L and upper U
// (zero beyond the matrix order), inv[f][blk][0] = L^-1, inv[f][blk][1] = U^-1.
// Column j by the 16 lanes 16j .. 16j + 15 of one wave: lane t sums the terms
// k = t (mod 16) of the substitution (at most four), four DPP steps add the
// 16 partial sums and lane t = 0 stores y, which the lanes read in later rows
// (LDS accesses of a wave complete in order).  Terms outside the sum read a
// known element of the column times zero, so a row's loads issue together.
template <typename R>
__global__ __launch_bounds__(1024) void inv_diag(const typename C2<R>::T* LU, long long stride, int n,
                                                 typename C2<R>::T* inv) {
  using T = typename C2<R>::T;
  __shared__ T D[64][65];
  __shared__ T Y[64][65];
  const int blk = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  const int j = tid >> 4, t = tid & 15;
  const int nblk = (n + 63) / 64;
  const int rb = blk * 64;
  const int h = min(64, n - rb);
  const T* M = LU + (size_t)f * stride;
  {
    // four loads per thread issued together; elements outside the block read
    // its corner and are zeroed afterwards
    T v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 1024 * i, r = e >> 6, c = e & 63;
      v[i] = M[(size_t)rb * n + rb + (r < h && c < h ? (size_t)r * n + c : 0)];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 1024 * i, r = e >> 6, c = e & 63;
      if (!(r < h && c < h)) v[i].x = v[i].y = 0;
      D[r][c] = v[i];
    }
  }
  __syncthreads();
  T* out = inv + ((size_t)f * nblk + blk) * 2 * 64 * 64;
  // L^-1 column j: y_r = [r == j] - sum_{j <= k < r} L[r][k] y_k
  for (int r = 0; r < 64; ++r) {
    R sx = 0, sy = 0;
    if (r > j && r < h) {
      T l[4], y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = j + t + 16 * i;
        const int kc = k < r ? k : j;
        l[i] = D[r][kc];
        y[i] = Y[kc][j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const R m = j + t + 16 * i < r ? (R)1 : (R)0;
        sx += m * (l[i].x * y[i].x - l[i].y * y[i].y);
        sy += m * (l[i].x * y[i].y + l[i].y * y[i].x);
      }
    }
    sx = row_sum(sx);
    sy = row_sum(sy);
    if (t == 0) {
      T y;
      y.x = r == j && r < h ? (R)1 : (r > j && r < h ? -sx : (R)0);
      y.y = r > j && r < h ? -sy : (R)0;
      Y[r][j] = y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 1024) out[e] = Y[e >> 6][e & 63];
  __syncthreads();
  // U^-1 column j: y_r = ([r == j] - sum_{r < k <= j} U[r][k] y_k) / U[r][r];
  // every Y element holds a finite value from the pass above when first read
  for (int r = 63; r >= 0; --r) {
    R sx = 0, sy = 0;
    const bool live = r < h && r <= j && j < h;
    if (live) {
      T u[4], y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = r + 1 + t + 16 * i;
        const int kc = k <= j ? k : j;
        u[i] = D[r][kc];
        y[i] = Y[kc][j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const R m = r + 1 + t + 16 * i <= j ? (R)1 : (R)0;
        sx += m * (u[i].x * y[i].x - u[i].y * y[i].y);
        sy += m * (u[i].x * y[i].y + u[i].y * y[i].x);
      }
    }
    sx = row_sum(sx);
    sy = row_sum(sy);
    if (t == 0) {
      T y = {0, 0};
      if (live) {
        const R bx = (r == j ? (R)1 : (R)0) - sx, by = -sy;
        const T d = D[r][r];
        const R den = d.x * d.x + d.y * d.y;
        y.x = (bx * d.x + by * d.y) / den;
        y.y = (by * d.x - bx * d.y) / den;
      }
      Y[r][j] = y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 1024) out[64 * 64 + e] = Y[e >> 6][e & 63];
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
                                                typename C2<R>::T* X, typename C2<R>::T* Y, int blk, int first) {
  using T = typename C2<R>::T;
  using C4 = typename Mf<R>::C4;
  __shared__ T xt[64][kVB];  // x_blk
  __shared__ T xn[64][kVB];  // a right-hand-side block
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int v = lane & 15, q = lane >> 4;
  const VecBatch& b = vb[blockIdx.y];
  const int nv = b.nv;
  int offs[4];
  batch_offsets(b, nv, w, offs);
  const int nblk = n / 64;
  const int rb = blk * 64;
  const size_t inv_blk = 2 * 64 * 64;
  const T* inv_f = inv + (size_t)b.fac * nblk * inv_blk + (FWD ? 0 : 64 * 64);
  // Every load that does not wait on another is issued up front: the lane's
  // vector offset, x_blk (the previous launch's result), this workgroup's
  // tile of the factor, its entries of X, and, in workgroup 0, the inverse of
  // the next diagonal block.  A workgroup past the last chunk (only when
  // there is a single block) reads block blk instead.
  const int lo = b.off[v];
  T t[4];
  load_vectors(t, first ? X : Y, offs, n, rb, 64);
  const int chunks = FWD ? nblk - 1 - blk : blk;
  const bool active = (int)blockIdx.x < chunks;
  const bool next = blockIdx.x == 0;  // chunk c is the next block to solve
  const int c = active ? (FWD ? blk + 1 + (int)blockIdx.x : blk - 1 - (int)blockIdx.x) : blk;
  const int cb = c * 64;
  const int r0 = 16 * w;
  const T* M = LU + (size_t)b.fac * stride;
  T a[16], ai[16];
  load_row16(M + (size_t)(cb + r0 + v) * n + rb + 16 * q, a);
  // (complex64 only: with complex128 operands the preloaded inverse would
  // leave one wave per SIMD)
  constexpr bool kPreInv = sizeof(R) == 4;
  if (kPreInv && next) load_row16(inv_f + c * inv_blk + (size_t)(r0 + v) * 64 + 16 * q, ai);
  const size_t vo = (size_t)(v < nv ? lo : 0) * n;
  T o[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = X[vo + cb + r0 + Mf<R>::row(lane, i)];
  if (first) {
    // x_blk = inv(T_blk,blk) b_blk, in every workgroup; workgroup 0 stores it
    T ab[16];
    load_row16(inv_f + blk * inv_blk + (size_t)(r0 + v) * 64 + 16 * q, ab);
    store_vectors(xn, t, nv, 64);
    __syncthreads();
    C4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    tile_mul<R>(ab, xn, cr, ci);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + Mf<R>::row(lane, i);
      xt[pk(r)][v] = T{cr[i], ci[i]};
      if (next && v < nv) Y[vo + rb + r] = T{cr[i], ci[i]};
    }
  } else {
    store_vectors(xt, t, nv, 64);
  }
  __syncthreads();
  if (!active) return;
  C4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  tile_mul<R>(a, xt, cr, ci);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + Mf<R>::row(lane, i);
    T y;
    y.x = v < nv ? o[i].x - cr[i] : (R)0;
    y.y = v < nv ? o[i].y - ci[i] : (R)0;
    if (v < nv) X[vo + cb + r] = y;
    if (next) xn[pk(r)][v] = y;
  }
  if (!next) return;
  __syncthreads();
  // x_c = inv(T_cc) b_c
  cr = C4{0, 0, 0, 0};
  ci = C4{0, 0, 0, 0};
  if (!kPreInv) load_row16(inv_f + c * inv_blk + (size_t)(r0 + v) * 64 + 16 * q, ai);
  tile_mul<R>(ai, xn, cr, ci);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + Mf<R>::row(lane, i);
    if (v < nv) Y[vo + cb + r] = T{cr[i], ci[i]};
  }
}

// r_v = b_v - A[fac] x_v (complex128).  Workgroup: 64 rows (16 per wave);
// x is staged in LDS in 64-column tiles.  n is a multiple of 64.
__global__ __launch_bounds__(256) void residual_b(const double2* A, long long stride, int n,
                                                  const VecBatch* vb, const double2* bv,
                                                  const double2* x, double2* r) {
  using C4 = Mf<double>::C4;
  __shared__ double2 xt[64][kVB];
  __shared__ int s_off[kVB];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const VecBatch& b = vb[blockIdx.y];
  const int nv = b.nv;
  if (tid < kVB) s_off[tid] = tid < nv ? b.off[tid] : 0;
  int offs[4];
  batch_offsets(b, nv, w, offs);
  const double2* M = A + (size_t)b.fac * stride;
  const int r0 = blockIdx.x * 64 + 16 * w;
  const bool row_ok = r0 + (lane & 15) < n;
  C4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += 64) {
    __syncthreads();
    double2 t[4];
    load_vectors(t, x, offs, n, k0, 64);
    store_vectors(xt, t, nv, 64);
    __syncthreads();
    tile_mma<double>(M + (size_t)r0 * n + k0, n, row_ok, 64, xt, cr, ci);
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
  if (n % 64 != 0) return hipErrorInvalidValue;
  const int nblk = n / 64;
  // launch i updates the blocks after i and solves block i + 1 (forward);
  // the last block is solved by the launch before it
  const int nfwd = nblk > 1 ? nblk - 1 : 1;
  for (int i = 0; i < nfwd; ++i) {
    const int chunks = nblk - 1 - i;
    hipLaunchKernelGGL((tri_step<R, true>), dim3(chunks > 0 ? chunks : 1, nvb), dim3(256), 0, s, LU, inv, stride,
                       n, d_vb, X, Y, i, i == 0 ? 1 : 0);
  }
  const int last = nblk > 1 ? 1 : 0;
  for (int i = nblk - 1; i >= last; --i) {
    const int chunks = i;
    hipLaunchKernelGGL((tri_step<R, false>), dim3(chunks > 0 ? chunks : 1, nvb), dim3(256), 0, s, LU, inv,
                       stride, n, d_vb, Y, X, i, i == nblk - 1 ? 1 : 0);
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
  hipLaunchKernelGGL(inv_diag<double>, dim3((n + 63) / 64, nfac), dim3(1024), 0, s, LU, stride, n, inv);
  return hipGetLastError();
}
hipError_t lu_inv_diag_c(const float2* LU, long long stride, int n, int nfac, float2* inv, hipStream_t s) {
  hipLaunchKernelGGL(inv_diag<float>, dim3((n + 63) / 64, nfac), dim3(1024), 0, s, LU, stride, n, inv);
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
