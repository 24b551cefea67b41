// Batched dense complex LU with partial pivoting and triangular solves on
// gfx950, for the per-mode Mueller systems (one matrix per azimuthal mode; the
// paper factors each mode with LAPACK, Section 6).
//
// Storage: row-major.  A batch is either uniform (`nb` matrices of order n,
// `stride` elements apart) or a list of matrices of different orders (the
// batching form: modes of several bodies factored by the same launches).
// Kernels take the matrix from blockIdx.z; extents given as -1 run to the
// matrix's own order, and a matrix whose order a step lies beyond does
// nothing in that step.
//
// Factorization (right-looking, recursive panels):
//   for each outer panel of NB = 128 columns:
//     factor the (n-k) x NB panel recursively: halves down to 8-column strips
//       factored by one workgroup per matrix with the strip in registers,
//       the right half updated by swaps + TRSM + GEMM
//     apply the panel's swaps left and right of it, TRSM the row block,
//     and update the trailing matrix with an MFMA GEMM.
// The GEMM computes C -= A B in complex arithmetic from four real MFMA
// products per k-step (f64 16x16x4 for complex128, f32 16x16x4 for complex64).
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

// A batch of matrices, uniform or listed (see msv_internal.h, LuMat).
template <typename T>
struct Mats {
  T* A;             // uniform: matrix z at A + z * stride
  int32_t* ipiv;    // uniform: [nb][n]
  int32_t* info;    // uniform: [nb]
  long long stride;
  int n;
  const LuMat* list;  // non-null: matrix z is list[z]
};
template <typename T>
struct Mz {
  T* a;
  int32_t* piv;
  int32_t* info;
  int n;
};
template <typename T>
__device__ __forceinline__ Mz<T> mat_at(const Mats<T>& B, int z) {
  if (B.list) {
    const LuMat& m = B.list[z];
    return Mz<T>{global_ptr(static_cast<T*>(m.a)), global_ptr(m.ipiv), global_ptr(m.info), m.n};
  }
  return Mz<T>{global_ptr(B.A + (size_t)z * B.stride), global_ptr(B.ipiv + (size_t)z * B.n),
               global_ptr(B.info + z), B.n};
}

constexpr int kPanelThreads = 1024;
constexpr int kMaxRowsPerThread = 12;  // n <= kPanelThreads * kMaxRowsPerThread

// One row of a strip, columns [0, W) of rowp with w valid: loaded without a
// condition (row and column indices clamped by the caller and here) and
// masked afterwards, so the loads of all rows are in flight together;
// complex64 pairs as 16-byte loads (w even).
template <int W>
__device__ __forceinline__ void strip_load(const float2* rowp, int w, bool rok, float2 (&o)[W]) {
#pragma unroll
  for (int q = 0; q < W / 2; ++q) {
    const bool ok = rok && 2 * q + 1 < w;
    const float4 t = reinterpret_cast<const float4*>(rowp)[2 * q + 1 < w ? q : 0];
    o[2 * q] = make_float2(ok ? t.x : 0.f, ok ? t.y : 0.f);
    o[2 * q + 1] = make_float2(ok ? t.z : 0.f, ok ? t.w : 0.f);
  }
}
template <int W>
__device__ __forceinline__ void strip_load(const double2* rowp, int w, bool rok, double2 (&o)[W]) {
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const double2 t = rowp[c < w ? c : 0];
    const bool ok = rok && c < w;
    o[c] = make_double2(ok ? t.x : 0.0, ok ? t.y : 0.0);
  }
}
template <int W>
__device__ __forceinline__ void strip_store(float2* rowp, int w, const float2 (&o)[W]) {
  if ((w & 1) == 0) {
#pragma unroll
    for (int q = 0; q < W / 2; ++q)
      if (2 * q + 1 < w)
        reinterpret_cast<float4*>(rowp)[q] = make_float4(o[2 * q].x, o[2 * q].y, o[2 * q + 1].x, o[2 * q + 1].y);
  } else {
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (c < w) rowp[c] = o[c];
  }
}
template <int W>
__device__ __forceinline__ void strip_store(double2* rowp, int w, const double2 (&o)[W]) {
#pragma unroll
  for (int c = 0; c < W; ++c)
    if (c < w) rowp[c] = o[c];
}

// ---------------------------------------------------------------------------
// base panel: rows [c0, n) x columns [c0, c0 + w), w <= kBaseW, pivoting in column.
// Thread tid owns rows c0 + tid + i * kPanelThreads, i < kRowsPerThread; the
// column loop is unrolled so the strip is indexed with constants.
// ---------------------------------------------------------------------------
// Largest 64-bit key over the wave, returned to every lane: DPP within each
// row of 16 lanes (quad swaps, half-row and row mirrors), then the four row
// results read as scalars.  (A shuffle ladder goes through the LDS crossbar,
// about a hundred cycles per dependent step.)
template <int kCtrl>
__device__ __forceinline__ unsigned long long dpp_max_u64(unsigned long long x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), kCtrl, 0xf, 0xf, false);
  const unsigned long long y = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  return y > x ? y : x;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
  k = dpp_max_u64<0xb1>(k);   // quad_perm [1, 0, 3, 2]
  k = dpp_max_u64<0x4e>(k);   // quad_perm [2, 3, 0, 1]
  k = dpp_max_u64<0x141>(k);  // row_half_mirror
  k = dpp_max_u64<0x140>(k);  // row_mirror
  unsigned long long r = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)k, 16 * q);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k >> 32), 16 * q);
    const unsigned long long y = ((unsigned long long)hi << 32) | lo;
    r = y > r ? y : r;
  }
  return r;
}

//
// kLeft: the strip is the right half of a node of width 2 kBaseW whose left
// strip [c0 - kBaseW, c0) has just been factored, and this kernel also does
// that node's steps between the two strips: the left strip's interchanges
// (composed, so that each row is loaded once from where it ends up coming
// from), U12 = L11^{-1} A12 for rows [c0 - kBaseW, c0), and A22 -= L21 U12
// for the rows below, before the strip is factored.
template <typename R, int kRowsPerThread, int kBaseW, bool kLeft>
__global__ __launch_bounds__(kPanelThreads) void base_panel(Mats<typename V2<R>::T> B, int c0, int w) {
  using T = typename V2<R>::T;
  const Mz<T> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (c0 >= n) return;
  T* M = mz.a;
  int32_t* piv = mz.piv;
  // per column (two sets, by column parity): each wave's best key and the
  // row it names, and row j as it was
  __shared__ unsigned long long red_k[2][kPanelThreads / 64];
  __shared__ T red_row[2][kPanelThreads / 64][kBaseW];
  __shared__ T oldj[2][kBaseW];
  const int tid = threadIdx.x;
  const int rows = n - c0;
  // rows owned: r = c0 + tid + i * kPanelThreads
  T v[kRowsPerThread][kBaseW];
  // Global stores wait out at the next barrier (the workgroup release waits
  // for them), so the pivots and U12 are stored after the column loop: thread
  // j keeps column j's pivot row.
  int my_piv = 0;
  T my_u12 = {0, 0};  // kLeft: entry (tid / W, tid % W) of U12, tid < W^2
  if constexpr (kLeft) {
    __shared__ T u12[kBaseW][kBaseW];  // rows [cl, c0) of the strip, then U12
    __shared__ T l11[kBaseW][kBaseW];
    const int cl = c0 - kBaseW;
    // after the interchanges (cl + k <-> pk[k], k = 0, 1, ...) row g holds
    // what row sigma(g) held: sigma applies them in reverse order
    int pk[kBaseW];
#pragma unroll
    for (int k = 0; k < kBaseW; ++k) pk[k] = piv[cl + k];
    auto sigma = [&](int g) {
#pragma unroll
      for (int k = kBaseW - 1; k >= 0; --k) g = g == cl + k ? pk[k] : (g == pk[k] ? cl + k : g);
      return g;
    };
    // L21 rows (the left strip's columns) of the thread's rows, loaded with
    // the strip (the registers allow it at 2 rows per thread; at 4 rows per
    // thread loading them a column at a time was slower than the separate
    // launches this replaces)
    static_assert(kRowsPerThread <= 2, "the fused strip holds L21 in registers");
    T l21[kRowsPerThread][kBaseW];
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
      const int r = tid + i * kPanelThreads;
      const bool rok = r < rows;
      strip_load(M + (size_t)(rok ? sigma(c0 + r) : c0) * n + c0, kBaseW, rok, v[i]);
      strip_load(M + (size_t)(c0 + (rok ? r : 0)) * n + cl, kBaseW, rok, l21[i]);
    }
    if (tid < kBaseW * kBaseW) {
      const int r = tid / kBaseW, c = tid % kBaseW;
      u12[r][c] = M[(size_t)sigma(cl + r) * n + c0 + c];
      l11[r][c] = M[(size_t)(cl + r) * n + cl + c];
    }
    __syncthreads();
    if (tid < kBaseW) {  // column tid of U12 by substitution
#pragma unroll
      for (int r = 1; r < kBaseW; ++r) {
        T acc = u12[r][tid];
#pragma unroll
        for (int q = 0; q < r; ++q) {
          const T l = l11[r][q], u = u12[q][tid];
          acc.x -= l.x * u.x - l.y * u.y;
          acc.y -= l.x * u.y + l.y * u.x;
        }
        u12[r][tid] = acc;
      }
    }
    __syncthreads();
    if (tid < kBaseW * kBaseW) my_u12 = u12[tid / kBaseW][tid % kBaseW];
    // A22 -= L21 U12 one row q of U12 at a time (a loop the compiler keeps,
    // so that only one row of U12 is in registers)
#pragma unroll 1
    for (int q = 0; q < kBaseW; ++q) {
      T u[kBaseW];
#pragma unroll
      for (int c = 0; c < kBaseW; ++c) u[c] = u12[q][c];
#pragma unroll
      for (int i = 0; i < kRowsPerThread; ++i) {
        T l = l21[i][0];
#pragma unroll
        for (int t = 1; t < kBaseW; ++t) l = q == t ? l21[i][t] : l;
#pragma unroll
        for (int c = 0; c < kBaseW; ++c) {
          v[i][c].x -= l.x * u[c].x - l.y * u[c].y;
          v[i][c].y -= l.x * u[c].y + l.y * u[c].x;
        }
      }
    }
  } else if (sizeof(T) == 8 && (w & 1)) {
    // odd width (not produced by the blocking used here): element loads
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
      const int r = tid + i * kPanelThreads;
#pragma unroll
      for (int c = 0; c < kBaseW; ++c) v[i][c] = load_or_zero(M + (size_t)(c0 + r) * n + c0 + c, r < rows && c < w);
    }
  } else {
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
      const int r = tid + i * kPanelThreads;
      const bool rok = r < rows;
      strip_load(M + (size_t)(c0 + (rok ? r : 0)) * n + c0, w, rok, v[i]);
    }
  }
#pragma unroll
  for (int j = 0; j < kBaseW; ++j) {
    if (j >= w) break;
    // pivot search over local rows >= j on keys that order candidates by
    // |re| + |im| (as float), then by the smaller row: no key is 0, the key
    // of "no candidate"; all comparisons are branch-free maxima
    unsigned long long best = 0;
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
      const int r = tid + i * kPanelThreads;
      const float a = (float)(fabs(v[i][j].x) + fabs(v[i][j].y));
      const unsigned long long key =
          ((unsigned long long)__float_as_uint(a) << 32) | (unsigned)(0x7fffffff - r);
      best = (r >= j && r < rows && key > best) ? key : best;
    }
    best = wave_max_u64(best);
    // publish, before the one barrier of the column: the wave's best key,
    // the row it names (from the lane that holds it), and row j (thread j
    // holds it: j < kBaseW <= kPanelThreads)
    const int pb = j & 1;
    {
      const int rb = 0x7fffffff - (int)(unsigned)(best & 0xffffffffu);
#pragma unroll
      for (int i = 0; i < kRowsPerThread; ++i)
        if (best != 0 && tid + i * kPanelThreads == rb) {
#pragma unroll
          for (int c = 0; c < kBaseW; ++c) red_row[pb][tid >> 6][c] = v[i][c];
        }
    }
    if ((tid & 63) == 0) red_k[pb][tid >> 6] = best;
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < kBaseW; ++c) oldj[pb][c] = v[0][c];
    }
    // The sets alternate by column parity: a thread writes column j + 1's set
    // only after this barrier, which every thread passes only once done with
    // column j - 1's reads of that set.
    __syncthreads();
    // every thread picks the pivot from the per-wave keys
    unsigned long long kq[kPanelThreads / 64];
#pragma unroll
    for (int q = 0; q < kPanelThreads / 64; ++q) kq[q] = red_k[pb][q];
#pragma unroll
    for (int h = kPanelThreads / 128; h > 0; h >>= 1)  // tree: depth 4, not a chain of 16
#pragma unroll
      for (int q = 0; q < h; ++q) kq[q] = kq[q + h] > kq[q] ? kq[q + h] : kq[q];
    best = kq[0];
    int p = 0x7fffffff - (int)(unsigned)(best & 0xffffffffu);
    const int qb = (p % kPanelThreads) >> 6;  // the wave that holds row p
    const bool none = (best >> 32) == 0 || p >= rows;  // no candidate, or a zero column
    if (none) {
      if (tid == 0 && *mz.info == 0) *mz.info = c0 + j + 1;
      p = j;
    }
    if (tid == j) my_piv = c0 + p;
    T prow[kBaseW];
#pragma unroll
    for (int c = 0; c < kBaseW; ++c) prow[c] = none ? oldj[pb][c] : red_row[pb][qb][c];
    // the interchange: the holder of row p takes row j, thread j takes row p
    if (p != j) {
      const int op = p % kPanelThreads, ip = p / kPanelThreads;
      if (tid == op) {
#pragma unroll
        for (int i = 0; i < kRowsPerThread; ++i)
          if (i == ip) {
#pragma unroll
            for (int c = 0; c < kBaseW; ++c) v[i][c] = oldj[pb][c];
          }
      }
      if (tid == j) {
#pragma unroll
        for (int c = 0; c < kBaseW; ++c) v[0][c] = prow[c];
      }
    }
    // pivot and multipliers
    T pv = prow[j];
    const R den = pv.x * pv.x + pv.y * pv.y;
    const R rden = den != 0 ? (R)1 / den : (R)0;
    T inv;
    inv.x = pv.x * rden;
    inv.y = -pv.y * rden;
#pragma unroll
    for (int i = 0; i < kRowsPerThread; ++i) {
      int r = tid + i * kPanelThreads;
      if (r > j && r < rows) {
        T a = v[i][j];
        T l;
        l.x = a.x * inv.x - a.y * inv.y;
        l.y = a.x * inv.y + a.y * inv.x;
        v[i][j] = l;
#pragma unroll
        for (int c = 0; c < kBaseW; ++c)
          if (c > j && c < w) {
            T u = prow[c];
            v[i][c].x -= l.x * u.x - l.y * u.y;
            v[i][c].y -= l.x * u.y + l.y * u.x;
          }
      }
    }
  }
  if (tid < w) piv[c0 + tid] = my_piv;
  if constexpr (kLeft) {
    // the rows of U12 (every row of the strip was loaded before the first
    // barrier, so they may be overwritten)
    if (tid < kBaseW * kBaseW) {
      const int r = tid / kBaseW, c = tid % kBaseW;
      M[(size_t)(c0 - kBaseW + r) * n + c0 + c] = my_u12;
    }
  }
#pragma unroll
  for (int i = 0; i < kRowsPerThread; ++i) {
    const int r = tid + i * kPanelThreads;
    if (r < rows) strip_store(M + (size_t)(c0 + r) * n + c0, w, v[i]);
  }
}

// ---------------------------------------------------------------------------
// row interchanges for pivots [k1, k2) applied to columns [cb, ce)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void laswp(Mats<T> B, int k1, int k2, int cb, int ce) {
  const Mz<T> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (k1 >= n) return;
  if (ce < 0) ce = n;
  T* M = mz.a;
  const int32_t* piv = mz.piv;
  int c = cb + blockIdx.x * 256 + threadIdx.x;
  if (c >= ce) return;
  // groups of 8 interchanges: the group's pivots are read together, so only
  // the interchanges actually made (p != k; most pivots lie on the diagonal)
  // wait on memory, not every pivot read; a shorter rest goes one at a time
  int k0 = k1;
  for (; k0 + 8 <= k2; k0 += 8) {
    int p[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) p[j] = piv[k0 + j];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (p[j] != k0 + j) {
        const size_t rk = (size_t)(k0 + j) * n + c, rp = (size_t)p[j] * n + c;
        const T a = M[rk], bb = M[rp];
        M[rk] = bb;
        M[rp] = a;
      }
    }
  }
  for (int k = k0; k < k2; ++k) {
    const int p = piv[k];
    if (p != k) {
      T a = M[(size_t)k * n + c];
      M[(size_t)k * n + c] = M[(size_t)p * n + c];
      M[(size_t)p * n + c] = a;
    }
  }
}


// ---------------------------------------------------------------------------
// X <- L^{-1} X, L = unit lower A[k:k+h, k:k+h] (h <= 64), X = A[k:k+h, cb:ce]:
// linv_block forms L^{-1} (identity-padded to 64 x 64) once per matrix, then
// trsm_inv multiplies each 64-column tile of X by it on MFMA, in place (a
// workgroup reads its whole tile into LDS before writing it back).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(1024) void linv_block(Mats<typename V2<R>::T> B, int k, int h,
                                                   typename V2<R>::T* linv, int slot) {
  using T = typename V2<R>::T;
  __shared__ T Ls[64][65];
  __shared__ T Y[64][65];
  const Mz<T> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (k >= n) return;
  const T* M = mz.a;
  const int tid = threadIdx.x;
  // the four loads of a thread are issued together (elements outside the
  // block read the corner element and are zeroed afterwards)
  T v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 1024 * i, r = e >> 6, c = e & 63;
    v[i] = M[(size_t)k * n + k + (r < h && c < h ? (size_t)r * n + c : 0)];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 1024 * i, r = e >> 6, c = e & 63;
    if (!(r < h && c < h)) v[i].x = v[i].y = 0;
    Ls[r][c] = v[i];
  }
  __syncthreads();
  // column j by the 16 lanes 16j .. 16j + 15 of one wave: lane t sums the
  // terms q = j + t + 16i (i < 4) of y_rj = [r == j] - sum_{j <= q < r}
  // L[r][q] y_qj, four DPP steps add the 16 partial sums, and lane t = 0
  // stores y_rj, which the lanes read in later rows (LDS accesses of a wave
  // complete in order).  Terms past r read a column element already known
  // (y_jj) times zero, so the four loads of a row are issued together.
  const int j = tid >> 4, t = tid & 15;
  for (int r = 0; r < 64; ++r) {
    R sx = 0, sy = 0;
    if (r > j && r < h) {
      T l[4], x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = j + t + 16 * i;
        const int qc = q < r ? q : j;
        l[i] = Ls[r][qc];
        x[i] = Y[qc][j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const R m = j + t + 16 * i < r ? (R)1 : (R)0;
        sx -= m * (l[i].x * x[i].x - l[i].y * x[i].y);
        sy -= m * (l[i].x * x[i].y + l[i].y * x[i].x);
      }
    }
    sx = row_sum(sx);
    sy = row_sum(sy);
    if (t == 0) {
      T y;
      y.x = r == j ? (R)1 : (r > j && r < h ? sx : (R)0);
      y.y = r > j && r < h ? sy : (R)0;
      Y[r][j] = y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  T* out = linv + ((size_t)blockIdx.z * kLinvSlots + slot) * 64 * 64;
  for (int e = tid; e < 64 * 64; e += 1024) out[e] = Y[e >> 6][e & 63];
}

// In-panel TRSM (at most 64 columns right of a block of h = 4..64 rows):
// 64 columns x 4 threads; thread t of a column keeps rows j = t (mod 4) in
// registers and row i's dot product is split over the four threads.
template <typename R, int H>
__global__ __launch_bounds__(256) void trsm_small(Mats<typename V2<R>::T> B, int k, int cb, int ce) {
  using T = typename V2<R>::T;
  constexpr int Q = H / 4;
  __shared__ T Ls[H][H + 1];
  const Mz<T> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (k >= n) return;
  if (ce < 0) ce = n;
  T* M = mz.a;
  for (int e = threadIdx.x; e < H * H; e += 256) {
    const int i = e / H, j = e % H;
    Ls[i][j] = M[(size_t)(k + i) * n + k + j];
  }
  __syncthreads();
  const int t = threadIdx.x & 3;
  const int c = cb + blockIdx.x * 64 + (threadIdx.x >> 2);
  const bool ok = c < ce;
  T x[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    x[q] = load_or_zero(M + (size_t)(k + 4 * q + t) * n + c, ok);
  }
#pragma unroll
  for (int i = 1; i < H; ++i) {
    R sr = 0, si = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (4 * q + t < i) {
        const T l = Ls[i][4 * q + t];
        sr += l.x * x[q].x - l.y * x[q].y;
        si += l.x * x[q].y + l.y * x[q].x;
      }
    sr = quad_sum(sr);
    si = quad_sum(si);
    if ((i & 3) == t) {
      x[i >> 2].x -= sr;
      x[i >> 2].y -= si;
    }
  }
  if (ok)
#pragma unroll
    for (int q = 0; q < Q; ++q) M[(size_t)(k + 4 * q + t) * n + c] = x[q];
}

template <typename R> struct Mfma;

template <typename R>
__global__ __launch_bounds__(256) void trsm_inv(Mats<typename V2<R>::T> B, int k, int h, int cb, int ce,
                                                const typename V2<R>::T* linv, int slot) {
  using T = typename V2<R>::T;
  using C4 = typename Mfma<R>::C4;
  __shared__ T Xs[64][65];  // [row][col]
  const Mz<T> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (k >= n) return;
  if (ce < 0) ce = n;
  T* M = mz.a;
  const T* Li = linv + ((size_t)blockIdx.z * kLinvSlots + slot) * 64 * 64;
  const int c0 = cb + blockIdx.x * 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // the tile's 16 loads per thread and the 16 inverse elements of the
  // thread's MFMA operands are all issued before the first wait (tile
  // elements outside the block read its first element and are zeroed)
  T v[16], a[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = tid + 256 * i, r = e >> 6, c = e & 63;
    v[i] = M[(size_t)k * n + c0 + (r < h && c0 + c < ce ? (size_t)r * n + c : 0)];
  }
  const T* Lrow = Li + (size_t)(16 * wave + (lane & 15)) * 64 + (lane >> 4);
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = Lrow[4 * s];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = tid + 256 * i, r = e >> 6, c = e & 63;
    if (!(r < h && c0 + c < ce)) v[i].x = v[i].y = 0;
    Xs[r][c] = v[i];
  }
  __syncthreads();
  if (16 * wave >= h) return;
  C4 cr[4], ci[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    cr[j] = C4{0, 0, 0, 0};
    ci[j] = C4{0, 0, 0, 0};
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int kk = 4 * s + (lane >> 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T bb = Xs[kk][16 * j + (lane & 15)];
      cr[j] = Mfma<R>::op(a[s].x, bb.x, cr[j]);
      cr[j] = Mfma<R>::op(-a[s].y, bb.y, cr[j]);
      ci[j] = Mfma<R>::op(a[s].x, bb.y, ci[j]);
      ci[j] = Mfma<R>::op(a[s].y, bb.x, ci[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * wave + Mfma<R>::row(lane, i);
      const int c = c0 + 16 * j + (lane & 15);
      if (r < h && c < ce) {
        T v;
        v.x = cr[j][i];
        v.y = ci[j][i];
        M[(size_t)(k + r) * n + c] = v;
      }
    }
}

// ---------------------------------------------------------------------------
// C[r0:r0+Mr, c0:c0+Nc] -= A[r0:, k0:k0+K] * A[k0:k0+K, c0:] on MFMA
// Workgroup: 256 threads = 4 waves (2 x 2), tile 64 x 64, K chunk 16.
// ---------------------------------------------------------------------------
constexpr int kGT = 64, kGK = 16;

// Operand layout (both): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// Accumulator layout (measured on gfx950): column l % 16 in both; row
// 4 * i + l / 16 for f64, 4 * (l / 16) + i for f32, i = register 0..3.
template <> struct Mfma<double> {
  using C4 = __attribute__((ext_vector_type(4))) double;
  static __device__ __forceinline__ C4 op(double a, double b, C4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <> struct Mfma<float> {
  using C4 = __attribute__((ext_vector_type(4))) float;
  static __device__ __forceinline__ C4 op(float a, float b, C4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <typename R>
__global__ __launch_bounds__(256) void gemm_update(Mats<typename V2<R>::T> B, int r0, int rend, int c0, int cend,
                                                   int k0, int K) {
  using T = typename V2<R>::T;
  using C4 = typename Mfma<R>::C4;
  // A as [row][k] with stride kGK + 1, B as [k][col] with stride kGT + 16:
  // both the transposing stores and the MFMA operand reads of a wave then
  // fall in distinct LDS banks
  __shared__ R As_re[kGT][kGK + 1], As_im[kGT][kGK + 1];
  __shared__ R Bs_re[kGK][kGT + 16], Bs_im[kGK][kGT + 16];
  const Mz<T> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (rend < 0) rend = n;
  if (cend < 0) cend = n;
  const int tr = r0 + blockIdx.y * kGT;
  const int tc = c0 + blockIdx.x * kGT;
  if (k0 >= n || tr >= rend || tc >= cend) return;
  T* M = mz.a;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  C4 cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = C4{0, 0, 0, 0};
      cim[a][b] = C4{0, 0, 0, 0};
    }
  const int kend = k0 + K;
  // A tile [64 rows][16 k] and B tile [16 k][64 cols], four elements of each
  // per thread, loaded one chunk ahead without a condition (an out-of-range
  // element reads M[0]) and masked where they are stored to LDS
  constexpr int kQ = kGT * kGK / 256;
  T ra[kQ], rb[kQ];
  bool oka[kQ], okb[kQ];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + 256 * q;
      const int rr = e / kGK, kk = e % kGK;
      const int gr = tr + rr, gk = kc + kk;
      oka[q] = gr < rend && gk < kend;
      ra[q] = M[oka[q] ? (size_t)gr * n + gk : 0];
      const int kb = e / kGT, cc = e % kGT;
      const int gkb = kc + kb, gc = tc + cc;
      okb[q] = gkb < kend && gc < cend;
      rb[q] = M[okb[q] ? (size_t)gkb * n + gc : 0];
    }
  };
  fetch(k0);
  for (int kc = k0; kc < kend; kc += kGK) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + 256 * q;
      const int rr = e / kGK, kk = e % kGK;
      As_re[rr][kk] = oka[q] ? -ra[q].x : (R)0;
      As_im[rr][kk] = oka[q] ? ra[q].y : (R)0;
      const int kb = e / kGT, cc = e % kGT;
      Bs_re[kb][cc] = okb[q] ? rb[q].x : (R)0;
      Bs_im[kb][cc] = okb[q] ? rb[q].y : (R)0;
    }
    __syncthreads();
    if (kc + kGK < kend) fetch(kc + kGK);
#pragma unroll
    for (int k4 = 0; k4 < kGK; k4 += 4) {
      const int kk = k4 + (lane >> 4);
      const int li = lane & 15;
      R are[2], aim[2], bre[2], bim[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        are[a] = As_re[wr + 16 * a + li][kk];  // = -Re A
        aim[a] = As_im[wr + 16 * a + li][kk];  // = +Im A
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bre[b] = Bs_re[kk][wc + 16 * b + li];
        bim[b] = Bs_im[kk][wc + 16 * b + li];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // C -= A B:  Re += (-Ar) Br + Ai Bi,  Im += (-Ar) Bi + (-Ai) Br
          cre[a][b] = Mfma<R>::op(are[a], bre[b], cre[a][b]);
          cre[a][b] = Mfma<R>::op(aim[a], bim[b], cre[a][b]);
          cim[a][b] = Mfma<R>::op(are[a], bim[b], cim[a][b]);
          cim[a][b] = Mfma<R>::op(-aim[a], bre[b], cim[a][b]);
        }
    }
    __syncthreads();
  }
  // accumulate into C (accumulator layout per Mfma<R>::row); all loads are
  // issued before the first add
  T cv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + Mfma<R>::row(lane, i);
        const int gc = tc + wc + 16 * b + (lane & 15);
        cv[a][b][i] = M[(gr < rend && gc < cend) ? (size_t)gr * n + gc : 0];
      }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + Mfma<R>::row(lane, i);
        const int gc = tc + wc + 16 * b + (lane & 15);
        if (gr < rend && gc < cend) {
          T v = cv[a][b][i];
          v.x += cre[a][b][i];
          v.y += cim[a][b][i];
          M[(size_t)gr * n + gc] = v;
        }
      }
}

// complex64 trailing update.  The tiles are staged in LDS as they lie in
// memory (complex interleaved, row-major), written with 16-byte stores.  The
// MFMA k-slot of lane group q at step s holds k = 4q + s of the 16-k chunk, so
// that a lane's A values for the four steps are four consecutive complex
// numbers (two 16-byte LDS reads) and its B value per step one complex (one
// 8-byte read).  Row strides of 18 (A) and 68 (B) complex keep the reads and
// the writes of a wave free of bank conflicts.  The next chunk's global
// loads are issued before the current chunk's MFMAs.
constexpr int kAS = kGK + 2, kBS = kGT + 4;
__global__ __launch_bounds__(256) void gemm_update_c(Mats<float2> B, int r0, int rend, int c0, int cend, int k0,
                                                     int K) {
  using C4 = Mfma<float>::C4;
  __shared__ float4 As4[kGT * kAS / 2];  // [row][k] complex, 16-byte aligned
  __shared__ float4 Bs4[kGK * kBS / 2];  // [k][col] complex
  float2* As = reinterpret_cast<float2*>(As4);
  float2* Bs = reinterpret_cast<float2*>(Bs4);
  const Mz<float2> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (rend < 0) rend = n;
  if (cend < 0) cend = n;
  const int tr = r0 + blockIdx.y * kGT;
  const int tc = c0 + blockIdx.x * kGT;
  if (k0 >= n || tr >= rend || tc >= cend) return;
  float2* M = mz.a;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lq = lane >> 4;
  // A B by three real products: t1 = Ar Br, t2 = Ai Bi, t3 = (Ar + Ai)(Br + Bi);
  // Re = t1 - t2, Im = t3 - t1 - t2
  C4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = C4{0, 0, 0, 0};
      t2[a][b] = C4{0, 0, 0, 0};
      t3[a][b] = C4{0, 0, 0, 0};
    }
  const int kend = k0 + K;
  // thread -> pair of complex: A tile 64 rows x 8 pairs, B tile 16 rows x 32
  // pairs (columns start at even offsets; n and all extents are multiples of
  // 4).  The loads are unconditional (an out-of-range element reads M[0])
  // and masked where they are stored to LDS.
  float4 ra[2], rb[2];
  bool oka[2], okb[2];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 3, kp = (e & 7) * 2;
      const int gr = tr + rr, gk = kc + kp;
      oka[q] = gr < rend && gk < kend;
      ra[q] = *reinterpret_cast<const float4*>(M + (oka[q] ? (size_t)gr * n + gk : 0));
      const int kb = e >> 5, cp = (e & 31) * 2;
      const int gkb = kc + kb, gc = tc + cp;
      okb[q] = gkb < kend && gc < cend;
      rb[q] = *reinterpret_cast<const float4*>(M + (okb[q] ? (size_t)gkb * n + gc : 0));
    }
  };
  // component-wise, so that no address is selected (which would put the
  // prefetch registers in scratch memory)
  auto masked = [](const float4& r, bool ok) {
    return make_float4(ok ? r.x : 0.f, ok ? r.y : 0.f, ok ? r.z : 0.f, ok ? r.w : 0.f);
  };
  fetch(k0);
  // the tile's block of C, loaded with the first chunk (it lies outside the
  // operands, and the tile is this workgroup's alone): one round trip less
  float2 cv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + Mfma<float>::row(lane, i);
        const int gc = tc + wc + 16 * b + li;
        const bool ok = gr < rend && gc < cend;
        cv[a][b][i] = M[ok ? (size_t)gr * n + gc : 0];
      }
  for (int kc = k0; kc < kend; kc += kGK) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + 256 * q;
      const int rr = e >> 3, kp = (e & 7) * 2;
      *reinterpret_cast<float4*>(As + rr * kAS + kp) = masked(ra[q], oka[q]);
      const int kb = e >> 5, cp = (e & 31) * 2;
      *reinterpret_cast<float4*>(Bs + kb * kBS + cp) = masked(rb[q], okb[q]);
    }
    __syncthreads();
    if (kc + kGK < kend) fetch(kc + kGK);
    float4 av[2][2];  // [a][half]: complex k = 4 lq + 0..3 of row wr + 16 a + li
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const float4* pa = reinterpret_cast<const float4*>(As + (wr + 16 * a + li) * kAS + 4 * lq);
      av[a][0] = pa[0];
      av[a][1] = pa[1];
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      float are[2], aim[2], bre[2], bim[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float4 h = av[a][st >> 1];
        are[a] = (st & 1) ? h.z : h.x;
        aim[a] = (st & 1) ? h.w : h.y;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float2 v = Bs[(4 * lq + st) * kBS + wc + 16 * b + li];
        bre[b] = v.x;
        bim[b] = v.y;
      }
      float sa[2], sb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) sa[a] = are[a] + aim[a];
#pragma unroll
      for (int b = 0; b < 2; ++b) sb[b] = bre[b] + bim[b];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          t1[a][b] = Mfma<float>::op(are[a], bre[b], t1[a][b]);
          t2[a][b] = Mfma<float>::op(aim[a], bim[b], t2[a][b]);
          t3[a][b] = Mfma<float>::op(sa[a], sb[b], t3[a][b]);
        }
    }
    __syncthreads();
  }
  // C -= A B
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + Mfma<float>::row(lane, i);
        const int gc = tc + wc + 16 * b + li;
        if (gr < rend && gc < cend) {
          float2 v = cv[a][b][i];
          v.x -= t1[a][b][i] - t2[a][b][i];
          v.y -= t3[a][b][i] - t1[a][b][i] - t2[a][b][i];
          M[(size_t)gr * n + gc] = v;
        }
      }
}

// complex64 trailing update on bf16 MFMA.  Every fp32 operand x is split as
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (|x - hi - lo| <=
// 2^-17 |x|), and each real product is formed as hi hi + hi lo + lo hi in fp32
// accumulators: about 16 bits of the product, against 24 of fp32.  With the
// three real products of 3M (Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)) that is 9 bf16
// MFMAs per complex product, at 16 times the fp32 MFMA rate.  The factors
// only precondition the complex128 refinement, whose residual removes the
// difference.
//
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16], t < 8, and holds C[4 (l / 16) + i][l % 16].
// Both tiles are staged in LDS as six bf16 planes (re, im, re + im; hi, lo) of
// [64][kBP] with k contiguous (B transposed), so each operand is one 16-byte
// read.  Rows are padded from 32 to 48 elements (96 bytes): measured on the
// 128 x 128 kernel at K = 256, strides of 36 and 44 run at half the rate of
// 40 and 48 (16-byte reads that straddle a 16-byte boundary), and 48 is a
// little ahead of 40.  K chunk 32, K a multiple of 32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kBK = 32, kBP = 48;

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 h = (__bf16)x[t];
    hi[t] = h;
    lo[t] = (__bf16)(x[t] - (float)h);
  }
}

__global__ __launch_bounds__(256) void gemm_update_bf(Mats<float2> B, int r0, int rend, int c0, int cend, int k0,
                                                      int K) {
  using C4 = Mfma<float>::C4;
  __shared__ __attribute__((aligned(16))) __bf16 As[6][kGT][kBP];  // re hi, re lo, im hi, im lo, s hi, s lo
  __shared__ __attribute__((aligned(16))) __bf16 Bs[6][kGT][kBP];  // [col][k]
  const Mz<float2> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (rend < 0) rend = n;
  if (cend < 0) cend = n;
  const int tr = r0 + blockIdx.y * kGT;
  const int tc = c0 + blockIdx.x * kGT;
  if (k0 >= n || tr >= rend || tc >= cend) return;
  float2* M = mz.a;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lq = lane >> 4;
  C4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = C4{0, 0, 0, 0};
      t2[a][b] = C4{0, 0, 0, 0};
      t3[a][b] = C4{0, 0, 0, 0};
    }
  const int kend = k0 + K;
  // staging: thread -> (row or column rc, k range 8 kq .. 8 kq + 7); loads are
  // unconditional (an out-of-range row or column reads row or column 0 of the
  // tile's matrix) and masked when converted
  const int rc = tid & 63, kq = tid >> 6;
  const bool oka = tr + rc < rend, okb = tc + rc < cend;
  const float2* pa = M + (size_t)(oka ? tr + rc : 0) * n + 8 * kq;
  const float2* pb = M + (size_t)(8 * kq) * n + (okb ? tc + rc : 0);
  float4 ra[4];
  float2 rb[8];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = reinterpret_cast<const float4*>(pa + kc)[q];
#pragma unroll
    for (int t = 0; t < 8; ++t) rb[t] = pb[(size_t)(kc + t) * n];
  };
  fetch(k0);
  // the tile's block of C, loaded with the first chunk (it lies outside the
  // operands, and the tile is this workgroup's alone): one round trip less
  float2 cv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + 4 * lq + i;
        const int gc = tc + wc + 16 * b + li;
        const bool ok = gr < rend && gc < cend;
        cv[a][b][i] = M[ok ? (size_t)gr * n + gc : 0];
      }
  for (int kc = k0; kc < kend; kc += kBK) {
    {
      float re[8], im[8], sm[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        re[2 * q] = oka ? ra[q].x : 0.f;
        im[2 * q] = oka ? ra[q].y : 0.f;
        re[2 * q + 1] = oka ? ra[q].z : 0.f;
        im[2 * q + 1] = oka ? ra[q].w : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) sm[t] = re[t] + im[t];
      bf16x8 h, l;
      split8(re, h, l);
      *reinterpret_cast<bf16x8*>(&As[0][rc][8 * kq]) = h;
      *reinterpret_cast<bf16x8*>(&As[1][rc][8 * kq]) = l;
      split8(im, h, l);
      *reinterpret_cast<bf16x8*>(&As[2][rc][8 * kq]) = h;
      *reinterpret_cast<bf16x8*>(&As[3][rc][8 * kq]) = l;
      split8(sm, h, l);
      *reinterpret_cast<bf16x8*>(&As[4][rc][8 * kq]) = h;
      *reinterpret_cast<bf16x8*>(&As[5][rc][8 * kq]) = l;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        re[t] = okb ? rb[t].x : 0.f;
        im[t] = okb ? rb[t].y : 0.f;
        sm[t] = re[t] + im[t];
      }
      split8(re, h, l);
      *reinterpret_cast<bf16x8*>(&Bs[0][rc][8 * kq]) = h;
      *reinterpret_cast<bf16x8*>(&Bs[1][rc][8 * kq]) = l;
      split8(im, h, l);
      *reinterpret_cast<bf16x8*>(&Bs[2][rc][8 * kq]) = h;
      *reinterpret_cast<bf16x8*>(&Bs[3][rc][8 * kq]) = l;
      split8(sm, h, l);
      *reinterpret_cast<bf16x8*>(&Bs[4][rc][8 * kq]) = h;
      *reinterpret_cast<bf16x8*>(&Bs[5][rc][8 * kq]) = l;
    }
    __syncthreads();
    if (kc + kBK < kend) fetch(kc + kBK);
    // the three real products; plane pairs (0, 1) re, (2, 3) im, (4, 5) re + im
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ah[a] = *reinterpret_cast<const bf16x8*>(&As[2 * pr][wr + 16 * a + li][8 * lq]);
        al[a] = *reinterpret_cast<const bf16x8*>(&As[2 * pr + 1][wr + 16 * a + li][8 * lq]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bh[b] = *reinterpret_cast<const bf16x8*>(&Bs[2 * pr][wc + 16 * b + li][8 * lq]);
        bl[b] = *reinterpret_cast<const bf16x8*>(&Bs[2 * pr + 1][wc + 16 * b + li][8 * lq]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          C4& t = pr == 0 ? t1[a][b] : pr == 1 ? t2[a][b] : t3[a][b];
          t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], t, 0, 0, 0);
          t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], t, 0, 0, 0);
          t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], t, 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // C -= A B
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + 4 * lq + i;
        const int gc = tc + wc + 16 * b + li;
        if (gr < rend && gc < cend) {
          float2 v = cv[a][b][i];
          v.x -= t1[a][b][i] - t2[a][b][i];
          v.y -= t3[a][b][i] - t1[a][b][i] - t2[a][b][i];
          M[(size_t)gr * n + gc] = v;
        }
      }
}

// The large trailing updates on 128 x 128 tiles, fed from operands split
// once per update instead of once per tile.  split_planes writes
// A = M[r0:rend, k0:k0+K] and B = M[k0:k0+K, c0:cend] as four bf16 planes
// each (re hi, re lo, im hi, im lo): P[c][p][i][t] is plane p of element
// 32 c + t of row i of A, or of column i of B, with rows (columns) past the
// block zero up to RA (RB), multiples of 128.  Per matrix the planes of A take
// 4 RA K elements, those of B the next 4 RB K; matrices are ws_stride
// elements apart.
constexpr int kPlanes = 4;
__global__ __launch_bounds__(256) void split_planes(Mats<float2> B, int r0, int rend, int c0, int cend, int k0,
                                                    int K, __bf16* ws, size_t ws_stride, int RA, int RB) {
  const Mz<float2> mz = mat_at(B, blockIdx.z);
  const int n = mz.n;
  if (rend < 0) rend = n;
  if (cend < 0) cend = n;
  const int c = blockIdx.y;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const bool live = k0 < n;
  __bf16* w = global_ptr(ws + blockIdx.z * ws_stride);
  float re[8], im[8];
  bf16x8 h, l;
  if (g < 4 * RA) {
    // A: 4 threads per row, 8 consecutive k each (a row's 64 bytes per plane
    // from 4 neighbouring lanes)
    const int i = g >> 2, q = g & 3;
    const bool ok = live && r0 + i < rend;
    const float4* src =
        reinterpret_cast<const float4*>(mz.a + (ok ? (size_t)(r0 + i) * n + k0 + 32 * c + 8 * q : 0));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float4 v = src[t];
      re[2 * t] = ok ? v.x : 0.f;
      im[2 * t] = ok ? v.y : 0.f;
      re[2 * t + 1] = ok ? v.z : 0.f;
      im[2 * t + 1] = ok ? v.w : 0.f;
    }
    __bf16* out = w + ((size_t)c * kPlanes * RA + i) * 32 + 8 * q;
    const size_t ps = (size_t)RA * 32;
    split8(re, h, l);
    *reinterpret_cast<bf16x8*>(out) = h;
    *reinterpret_cast<bf16x8*>(out + ps) = l;
    split8(im, h, l);
    *reinterpret_cast<bf16x8*>(out + 2 * ps) = h;
    *reinterpret_cast<bf16x8*>(out + 3 * ps) = l;
  } else if (g < 4 * (RA + RB)) {
    // B: 4 threads per column, 8 consecutive k each; a wave takes 64
    // consecutive columns at one k quarter (512-byte row segments read, the
    // 16-byte quarter q of 64 consecutive 64-byte rows written per plane)
    const int gb = g - 4 * RA;
    const int q = (gb >> 6) & 3;
    const int j = ((gb >> 8) << 6) + (gb & 63);
    const bool ok = live && c0 + j < cend;
    const float2* src = mz.a + (size_t)(k0 + 32 * c + 8 * q) * n + (ok ? c0 + j : 0);
    __bf16* out = w + (size_t)kPlanes * RA * K + ((size_t)c * kPlanes * RB + j) * 32 + 8 * q;
    const size_t ps = (size_t)RB * 32;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float2 v = ok ? src[(size_t)t * n] : make_float2(0.f, 0.f);
      re[t] = v.x;
      im[t] = v.y;
    }
    split8(re, h, l);
    *reinterpret_cast<bf16x8*>(out) = h;
    *reinterpret_cast<bf16x8*>(out + ps) = l;
    split8(im, h, l);
    *reinterpret_cast<bf16x8*>(out + 2 * ps) = h;
    *reinterpret_cast<bf16x8*>(out + 3 * ps) = l;
  }
}

// C -= A B on 128 x 128 tiles from the planes, with the four real products
// of the complex product (re = Ar Br - Ai Bi, im = Ar Bi + Ai Br; the minus
// sign flips the sign bits of the Bi operands) and each as hi hi + hi lo +
// lo hi: 12 bf16 MFMAs per complex product, into two accumulators instead of
// the three of 3M.  512 threads: wave w computes rows 64 (w / 4) .. + 64 and
// columns 32 (w % 4) .. + 32 of the tile (4 x 2 MFMA blocks), so two waves
// share each SIMD and one's MFMAs issue while the other waits on LDS.  K
// chunks of 32 go through two LDS buffers, each 4 planes of A and 4 of B as
// [128][32] bf16 rows with the 16-byte quarters of row r permuted as
// q ^ (r >> 1 & 3).  The chunks move from memory straight into LDS
// (global_load_lds_dwordx4, one 1 KB block of 16 rows per wave instruction,
// each lane fetching the quarter that belongs at its slot), so no register
// holds a chunk in flight: chunk c + 1 is issued before chunk c's products and
// waited for after them, one barrier per chunk.  A wave reads its A rows and
// B columns of a chunk from LDS once, every operand of the chunk's 96 MFMAs in
// registers together.  128 KB of dynamic LDS; one workgroup per CU.
constexpr int kBT = 128;
constexpr int kChunkElems = 2 * kPlanes * kBT * 32;  // one LDS buffer: A then B
constexpr size_t kBfLds = 2 * kChunkElems * sizeof(__bf16);

// Workgroup -> (column tile x, row tile y, matrix z) of a 1-D grid of
// nb TY TX tiles.  The hardware hands workgroups to the 8 XCDs round-robin
// (id mod 8); each XCD instead takes a contiguous range of tiles, walked down
// a group of kGY row tiles, then across the columns.  The workgroups resident
// on one XCD then share a few row tiles of A and column tiles of B in its L2,
// where round-robin order spreads every tile over all eight.
constexpr int kGY = 2;
__device__ __forceinline__ void update_tile(int TX, int TY, int& x, int& y, int& z) {
  const int T = (int)gridDim.x, L = (int)blockIdx.x;
  const int base = T >> 3, rem = T & 7, xcd = L & 7;
  const int id = xcd * base + (xcd < rem ? xcd : rem) + (L >> 3);
  const int per = TX * TY;
  z = id / per;
  const int l = id - z * per;
  const int y0 = l / (kGY * TX) * kGY;
  const int gh = TY - y0 < kGY ? TY - y0 : kGY;
  const int r = l - y0 * TX;
  y = y0 + r % gh;
  x = r / gh;
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 v) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

__global__ __launch_bounds__(512) void gemm_update_planes(Mats<float2> B, int r0, int rend, int c0, int cend,
                                                           int k0, int K, const __bf16* ws, size_t ws_stride,
                                                           int RA, int RB) {
  using C4 = Mfma<float>::C4;
  extern __shared__ __attribute__((aligned(16))) __bf16 lds_bf[];
  int bx, by, bz;
  update_tile(RB / kBT, RA / kBT, bx, by, bz);
  const Mz<float2> mz = mat_at(B, bz);
  const int n = mz.n;
  if (rend < 0) rend = n;
  if (cend < 0) cend = n;
  const int tr = r0 + by * kBT;
  const int tc = c0 + bx * kBT;
  if (k0 >= n || tr >= rend || tc >= cend) return;
  float2* M = mz.a;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 2) * 64, wc = (wave & 3) * 32;
  const int li = lane & 15, lq = lane >> 4;
  C4 tre[4][2], tim[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      tre[a][b] = C4{0, 0, 0, 0};
      tim[a][b] = C4{0, 0, 0, 0};
    }
  const __bf16* wa = global_ptr(ws + bz * ws_stride) + (size_t)by * kBT * 32;
  const __bf16* wb = global_ptr(ws + bz * ws_stride) + (size_t)kPlanes * RA * K + (size_t)bx * kBT * 32;
  const int rd_ofs = li * 32 + 8 * (lq ^ ((li >> 1) & 3));
  auto products = [&](int buf) {
    const __bf16* xa = lds_bf + buf * kChunkElems + rd_ofs + wr * 32;
    const __bf16* xb = lds_bf + buf * kChunkElems + kPlanes * kBT * 32 + rd_ofs + wc * 32;
    bf16x8 arh[4], arl[4], aih[4], ail[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      arh[a] = *reinterpret_cast<const bf16x8*>(xa + (0 * kBT + 16 * a) * 32);
      arl[a] = *reinterpret_cast<const bf16x8*>(xa + (1 * kBT + 16 * a) * 32);
      aih[a] = *reinterpret_cast<const bf16x8*>(xa + (2 * kBT + 16 * a) * 32);
      ail[a] = *reinterpret_cast<const bf16x8*>(xa + (3 * kBT + 16 * a) * 32);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const bf16x8 brh = *reinterpret_cast<const bf16x8*>(xb + (0 * kBT + 16 * b) * 32);
      const bf16x8 brl = *reinterpret_cast<const bf16x8*>(xb + (1 * kBT + 16 * b) * 32);
      const bf16x8 bih = *reinterpret_cast<const bf16x8*>(xb + (2 * kBT + 16 * b) * 32);
      const bf16x8 bil = *reinterpret_cast<const bf16x8*>(xb + (3 * kBT + 16 * b) * 32);
      const bf16x8 nih = neg8(bih), nil = neg8(bil);
#pragma unroll
      for (int a = 0; a < 4; ++a) tre[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], brh, tre[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tim[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], bih, tim[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tre[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], brl, tre[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tim[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh[a], bil, tim[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tre[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl[a], brh, tre[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tim[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl[a], bih, tim[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tim[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[a], brh, tim[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tre[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[a], nih, tre[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tim[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[a], brl, tim[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tre[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih[a], nil, tre[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tim[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail[a], brh, tim[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) tre[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail[a], nih, tre[a][b], 0, 0, 0);
    }
  };
  // wave w moves rows 16 w .. 16 w + 15 of every plane of a chunk from memory
  // straight into LDS: lane l writes the 16 bytes at row 16 w + l / 4, slot
  // l % 4, which hold the row's quarter (l % 4) ^ swizzle
  const int dr = 16 * wave + (lane >> 2), dsl = lane & 3;
  const unsigned dofs = (unsigned)(dr * 32 + 8 * (dsl ^ ((dr >> 1) & 3)));
  auto issue = [&](int c, int buf) {
    __bf16* base = lds_bf + buf * kChunkElems + 16 * wave * 32;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const __bf16* pa = wa + (size_t)(kPlanes * c + v) * RA * 32 + dofs;
      const __bf16* pb = wb + (size_t)(kPlanes * c + v) * RB * 32 + dofs;
      __builtin_amdgcn_global_load_lds(pa, base + v * kBT * 32, 16, 0, 0);
      __builtin_amdgcn_global_load_lds(pb, base + (kPlanes + v) * kBT * 32, 16, 0, 0);
    }
  };
  const int nc = K / kBK;
  float2 cv[4][2][4];
  issue(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    if (c + 1 < nc) issue(c + 1, (c + 1) & 1);
    if (c == nc - 1) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int gr = tr + wr + 16 * a + 4 * lq + i;
            const int gc = tc + wc + 16 * b + li;
            const bool ok = gr < rend && gc < cend;
            cv[a][b][i] = M[ok ? (size_t)gr * n + gc : 0];
          }
    }
    products(c & 1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = tr + wr + 16 * a + 4 * lq + i;
        const int gc = tc + wc + 16 * b + li;
        if (gr < rend && gc < cend) {
          float2 v = cv[a][b][i];
          v.x -= tre[a][b][i];
          v.y -= tim[a][b][i];
          M[(size_t)gr * n + gc] = v;
        }
      }
}

// Host view of a batch: the device descriptor plus its count and the
// largest order (which sizes the grids).
template <typename T>
struct Batch {
  Mats<T> d;
  int nb;
  int nmax;
  T* linv;  // [nb][kLinvSlots][64][64] diagonal-block inverses
  __bf16* planes = nullptr;  // bf16 operand planes of the large complex64 updates
  size_t planes_stride = 0;  // elements per matrix
  // complex64 updates of at least plane_min rows and columns take the
  // 128 x 128-tile planes kernel, smaller ones the 64 x 64-tile kernels
  int plane_min = 2 * kBT;
};

// Workspace split: diagonal-block inverses, then (complex64) room for the
// planes of one trailing update per matrix, 4 (RA + RB) K <= 8 R 512 with R
// the largest order rounded up to 128.
size_t linv_bytes(int nb, size_t elem) { return ((size_t)nb * kLinvSlots * 64 * 64 * elem + 255) / 256 * 256; }
size_t planes_per_matrix(int n) { return (size_t)2 * kPlanes * ((n + kBT - 1) / kBT * kBT) * 512; }

template <typename T>
Batch<T> make_batch(const Mats<T>& d, int nb, int nmax, void* work) {
  Batch<T> bt{d, nb, nmax, static_cast<T*>(work)};
  if constexpr (sizeof(T) == 8) {
    bt.planes = reinterpret_cast<__bf16*>(static_cast<char*>(work) + linv_bytes(nb, sizeof(T)));
    bt.planes_stride = planes_per_matrix(nmax);
  }
  return bt;
}

// C[r0:rend, c0:cend] -= A[r0:rend, k0:k0+K] * A[k0:k0+K, c0:cend]; rend or
// cend -1 = the matrix order.  The grid covers the largest order.
template <typename R>
hipError_t gemm(const Batch<typename V2<R>::T>& b, int r0, int rend, int c0, int cend, int k0, int K,
                hipStream_t s) {
  const int Mr = (rend < 0 ? b.nmax : rend) - r0, Nc = (cend < 0 ? b.nmax : cend) - c0;
  if (Mr <= 0 || Nc <= 0 || K <= 0) return hipSuccess;
  dim3 g((Nc + kGT - 1) / kGT, (Mr + kGT - 1) / kGT, b.nb);
  if constexpr (sizeof(R) == 4) {
    const int RA = (Mr + kBT - 1) / kBT * kBT, RB = (Nc + kBT - 1) / kBT * kBT;
    if (K % kBK == 0 && Mr >= b.plane_min && Nc >= b.plane_min && b.planes &&
        (size_t)kPlanes * (RA + RB) * K <= b.planes_stride) {
      static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_update_planes),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBfLds);
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL(split_planes, dim3((4 * (RA + RB) + 255) / 256, K / kBK, b.nb), dim3(256), 0, s, b.d, r0, rend, c0,
                         cend, k0, K, b.planes, b.planes_stride, RA, RB);
      hipLaunchKernelGGL(gemm_update_planes, dim3((RB / kBT) * (RA / kBT) * b.nb), dim3(512), kBfLds, s, b.d, r0,
                         rend, c0, cend, k0, K, b.planes, b.planes_stride, RA, RB);
    } else if (K % kBK == 0)
      hipLaunchKernelGGL(gemm_update_bf, g, dim3(256), 0, s, b.d, r0, rend, c0, cend, k0, K);
    else
      hipLaunchKernelGGL(gemm_update_c, g, dim3(256), 0, s, b.d, r0, rend, c0, cend, k0, K);
  } else
    hipLaunchKernelGGL(gemm_update<R>, g, dim3(256), 0, s, b.d, r0, rend, c0, cend, k0, K);
  return hipGetLastError();
}

template <typename R>
hipError_t swaps(const Batch<typename V2<R>::T>& b, int k1, int k2, int cb, int ce, hipStream_t s) {
  const int cmax = ce < 0 ? b.nmax : ce;
  if (cmax <= cb || k2 <= k1) return hipSuccess;
  dim3 g((cmax - cb + 255) / 256, 1, b.nb);
  hipLaunchKernelGGL(laswp<typename V2<R>::T>, g, dim3(256), 0, s, b.d, k1, k2, cb, ce);
  return hipGetLastError();
}

#define MSV_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

// X = A[k:k+h, cb:ce] <- L^{-1} X with L the unit-lower A[k:k+h, k:k+h]; ce -1
// = the matrix order.  Blocks of 64 rows and more (64-aligned from the outer
// panel start k0), and every row block of an outer step, are halved down to
// 64-row pieces, with a GEMM update of the lower half by the upper one in
// between; each piece is multiplied by the inverse of its diagonal block
// (formed when its 64-column sub-panel was finished, or here for a shorter
// last piece).  Shorter in-panel blocks are solved by register substitution.
template <typename R>
hipError_t trsm(const Batch<typename V2<R>::T>& b, int k, int h, int cb, int ce, int k0, hipStream_t s) {
  const int cmax = ce < 0 ? b.nmax : ce;
  if (cmax <= cb || h <= 0) return hipSuccess;
  if (h >= 64 || ce < 0) {
    if ((k - k0) % 64 != 0 || k + h - k0 > 64 * kLinvSlots) return hipErrorInvalidValue;
    if (h > 64) {
      // halves (the upper one a multiple of 64): solve the upper rows, update
      // the lower ones with them, solve the lower rows -- the rows of the
      // block pass through a product about log2(h / 64) times
      const int h1 = (h / 2 + 63) / 64 * 64;
      MSV_TRY(trsm<R>(b, k, h1, cb, ce, k0, s));
      MSV_TRY(gemm<R>(b, k + h1, k + h, cb, ce, k, h1, s));
      return trsm<R>(b, k + h1, h - h1, cb, ce, k0, s);
    }
    const int slot = (k - k0) / 64;
    if (h < 64) hipLaunchKernelGGL(linv_block<R>, dim3(1, 1, b.nb), dim3(1024), 0, s, b.d, k, h, b.linv, slot);
    hipLaunchKernelGGL(trsm_inv<R>, dim3((cmax - cb + 63) / 64, 1, b.nb), dim3(256), 0, s, b.d, k, h, cb, ce, b.linv,
                       slot);
    return hipGetLastError();
  }
  dim3 g((ce - cb + 63) / 64, 1, b.nb);
  switch (h) {
    case 4: hipLaunchKernelGGL((trsm_small<R, 4>), g, dim3(256), 0, s, b.d, k, cb, ce); break;
    case 8: hipLaunchKernelGGL((trsm_small<R, 8>), g, dim3(256), 0, s, b.d, k, cb, ce); break;
    case 16: hipLaunchKernelGGL((trsm_small<R, 16>), g, dim3(256), 0, s, b.d, k, cb, ce); break;
    case 32: hipLaunchKernelGGL((trsm_small<R, 32>), g, dim3(256), 0, s, b.d, k, cb, ce); break;
    default: return hipErrorInvalidValue;  // panel halves are powers of two
  }
  return hipGetLastError();
}

// Recursive factorization of the panel rows [c0, n) x columns [c0, c0 + w).
template <typename R>
hipError_t panel_rec(const Batch<typename V2<R>::T>& b, int c0, int w, int k0, hipStream_t s) {
  // strips of 8 columns while they fit the registers (complex64 up to 4 rows
  // per thread, complex128 up to 2), else 4; every width <= 4 is a base case.
  // (16 columns fit at 2 rows per thread but ran slower: the unrolled column
  // loop grows past what the instruction cache holds)
  const int rows = b.nmax - c0;  // the strip's rows, spread over the workgroup
  const dim3 g(1, 1, b.nb), t(kPanelThreads);
  if constexpr (sizeof(R) == 4) {
    if (rows <= 2 * kPanelThreads && w <= 8) {
      hipLaunchKernelGGL((base_panel<R, 2, 8, false>), g, t, 0, s, b.d, c0, w);
      return hipGetLastError();
    }
    if (rows > 2 * kPanelThreads && rows <= 4 * kPanelThreads && w <= 8) {
      hipLaunchKernelGGL((base_panel<R, 4, 8, false>), g, t, 0, s, b.d, c0, w);
      return hipGetLastError();
    }
    if (rows > 4 * kPanelThreads && w <= 4) {
      if (rows <= 8 * kPanelThreads)
        hipLaunchKernelGGL((base_panel<R, 8, 4, false>), g, t, 0, s, b.d, c0, w);
      else
        hipLaunchKernelGGL((base_panel<R, kMaxRowsPerThread, 4, false>), g, t, 0, s, b.d, c0, w);
      return hipGetLastError();
    }
  } else {
    if (rows <= 2 * kPanelThreads && w <= 8) {
      hipLaunchKernelGGL((base_panel<R, 2, 8, false>), g, t, 0, s, b.d, c0, w);
      return hipGetLastError();
    }
    if (rows > 2 * kPanelThreads && w <= 4) {
      if (rows <= 4 * kPanelThreads)
        hipLaunchKernelGGL((base_panel<R, 4, 4, false>), g, t, 0, s, b.d, c0, w);
      else if (rows <= 8 * kPanelThreads)
        hipLaunchKernelGGL((base_panel<R, 8, 4, false>), g, t, 0, s, b.d, c0, w);
      else
        hipLaunchKernelGGL((base_panel<R, kMaxRowsPerThread, 4, false>), g, t, 0, s, b.d, c0, w);
      return hipGetLastError();
    }
  }
  int h = w / 2;
  MSV_TRY(panel_rec<R>(b, c0, h, k0, s));
  if constexpr (sizeof(R) == 4) {
    // two 8-column base strips of at most 2048 rows: the right strip's kernel
    // also applies the left strip's interchanges, U12 and the update of its
    // rows (one launch in place of four)
    if (w == 16 && h == 8 && rows <= 2 * kPanelThreads) {
      hipLaunchKernelGGL((base_panel<R, 2, 8, true>), g, t, 0, s, b.d, c0 + h, h);
      MSV_TRY(hipGetLastError());
      return swaps<R>(b, c0 + h, c0 + w, c0, c0 + h, s);
    }
  }
  MSV_TRY(swaps<R>(b, c0, c0 + h, c0 + h, c0 + w, s));
  MSV_TRY(trsm<R>(b, c0, h, c0 + h, c0 + w, k0, s));
  MSV_TRY(gemm<R>(b, c0 + h, -1, c0 + h, c0 + w, c0, h, s));
  MSV_TRY(panel_rec<R>(b, c0 + h, w - h, k0, s));
  // swaps of the right half also apply to the left half of the panel
  MSV_TRY(swaps<R>(b, c0 + h, c0 + w, c0, c0 + h, s));
  if (w == 64 && (c0 - k0) % 64 == 0) {
    // a finished 64-wide sub-panel: keep the inverse of its unit-lower block
    hipLaunchKernelGGL(linv_block<R>, dim3(1, 1, b.nb), dim3(1024), 0, s, b.d, c0, 64, b.linv, (c0 - k0) / 64);
    MSV_TRY(hipGetLastError());
  }
  return hipSuccess;
}

template <typename T>
__global__ void zero_info(Mats<T> B, int nb) {
  for (int i = threadIdx.x; i < nb; i += blockDim.x) *mat_at(B, i).info = 0;
}

// Outer panels of NB = 64, 128, 256 or 512 columns (complex64 alone: 512,
// complex128: 256).  In a listed batch every order
// below the largest must be a multiple of NB, so that a panel is never cut
// short for one matrix and not for another.
template <typename R>
hipError_t factor(const Batch<typename V2<R>::T>& b, int NB, hipStream_t s) {
  const int n = b.nmax;
  if (n > kPanelThreads * kMaxRowsPerThread) return hipErrorInvalidValue;
  if (NB != 64 && NB != 128 && NB != 256 && NB != 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_info<typename V2<R>::T>, dim3(1), dim3(256), 0, s, b.d, b.nb);
  MSV_TRY(hipGetLastError());
  for (int k = 0; k < n; ) {
    // panel widths are powers of two (the recursive panel halves them down to
    // the register strips): the largest one not above what is left
    int w = n - k < NB ? n - k : NB;
    while (w & (w - 1)) w &= w - 1;
    MSV_TRY(panel_rec<R>(b, k, w, k, s));
    MSV_TRY(swaps<R>(b, k, k + w, 0, k, s));
    MSV_TRY(swaps<R>(b, k, k + w, k + w, -1, s));
    // U12 = L11^{-1} A12 by 64-row pieces, then A22
    MSV_TRY(trsm<R>(b, k, w, k + w, -1, k, s));
    MSV_TRY(gemm<R>(b, k + w, -1, k + w, -1, k, w, s));
    k += w;
  }
  return hipSuccess;
}

// G batches of the same order, batch g factored on stream st[g], each one
// panel phase behind the one before.  A panel factorization runs one
// workgroup per matrix and is bound by the latency of its column steps,
// while a trailing update fills the chip's MFMA units; with every panel of
// batch g waiting for the same panel of batch g - 1, the panels of one batch
// run while the updates of others do.  The batches share no memory.  ev:
// kStaggerEvents events, all on the device of the streams.
template <typename R>
hipError_t factor_staggered(const Batch<typename V2<R>::T>* bt, int G, int NB, const hipStream_t* st,
                            hipEvent_t* ev) {
  using T = typename V2<R>::T;
  const int n = bt[0].nmax;
  if (G < 2 || G > kStaggerMax || n > kPanelThreads * kMaxRowsPerThread) return hipErrorInvalidValue;
  for (int g = 1; g < G; ++g)
    if (bt[g].nmax != n) return hipErrorInvalidValue;
  if (NB != 64 && NB != 128 && NB != 256 && NB != 512) return hipErrorInvalidValue;
  // ev[0]: the fork; ev[g], 0 < g < G: batch g done; then G - 1 per step.
  // Steps: n / NB full panels plus at most log2(NB) narrower ones at the end.
  if (G + (n / NB + 10) * (G - 1) > kStaggerEvents) return hipErrorInvalidValue;
  MSV_TRY(hipEventRecord(ev[0], st[0]));  // the other streams start after the work queued on st[0]
  for (int g = 0; g < G; ++g) {
    if (g) MSV_TRY(hipStreamWaitEvent(st[g], ev[0], 0));
    hipLaunchKernelGGL(zero_info<T>, dim3(1), dim3(256), 0, st[g], bt[g].d, bt[g].nb);
    MSV_TRY(hipGetLastError());
  }
  hipEvent_t* step_ev = ev + G;
  for (int k = 0; k < n; step_ev += G - 1) {
    int w = n - k < NB ? n - k : NB;
    while (w & (w - 1)) w &= w - 1;
    for (int g = 0; g < G; ++g) {
      if (g) MSV_TRY(hipStreamWaitEvent(st[g], step_ev[g - 1], 0));
      MSV_TRY(panel_rec<R>(bt[g], k, w, k, st[g]));
      if (g + 1 < G) MSV_TRY(hipEventRecord(step_ev[g], st[g]));
    }
    for (int g = 0; g < G; ++g) {
      MSV_TRY(swaps<R>(bt[g], k, k + w, 0, k, st[g]));
      MSV_TRY(swaps<R>(bt[g], k, k + w, k + w, -1, st[g]));
      MSV_TRY(trsm<R>(bt[g], k, w, k + w, -1, k, st[g]));
      MSV_TRY(gemm<R>(bt[g], k + w, -1, k + w, -1, k, w, st[g]));
    }
    k += w;
  }
  for (int g = 1; g < G; ++g) {  // st[0] continues after every batch
    MSV_TRY(hipEventRecord(ev[g], st[g]));
    MSV_TRY(hipStreamWaitEvent(st[0], ev[g], 0));
  }
  return hipSuccess;
}

// A strided batch cut into G consecutive groups (the first nb mod G one
// matrix larger), each with its part of the workspace, and factored by
// factor_staggered.
template <typename R>
hipError_t factor_groups_staggered(typename V2<R>::T* A, int32_t* ipiv, int32_t* info, const LuBatch& lb,
                                   void* work, int G, int NB, const hipStream_t* st, hipEvent_t* ev) {
  using T = typename V2<R>::T;
  if (G < 2 || G > kStaggerMax) return hipErrorInvalidValue;
  Batch<T> bt[kStaggerMax];
  int off = 0;
  char* w = static_cast<char*>(work);
  for (int g = 0; g < G; ++g) {
    const int cnt = lb.nb / G + (g < lb.nb % G ? 1 : 0);
    bt[g] = make_batch(Mats<T>{A + off * lb.stride, ipiv + (size_t)off * lb.n, info + off, lb.stride, lb.n, nullptr},
                       cnt, lb.n, w);
    off += cnt;
    w += lu_work_bytes(lb.n, cnt, sizeof(T) == 16);
  }
  return factor_staggered<R>(bt, G, NB, st, ev);
}

}  // namespace

size_t lu_work_bytes(int n, int nb, bool c128) {
  return c128 ? linv_bytes(nb, sizeof(double2)) : linv_bytes(nb, sizeof(float2)) + nb * planes_per_matrix(n) * 2;
}
hipError_t lu_factor_z(double2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, hipStream_t s) {
  return factor<double>(make_batch(Mats<double2>{A, ipiv, info, b.stride, b.n, nullptr}, b.nb, b.n, work), 256, s);
}
hipError_t lu_factor_c(float2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, hipStream_t s) {
  return factor<float>(make_batch(Mats<float2>{A, ipiv, info, b.stride, b.n, nullptr}, b.nb, b.n, work), 512, s);
}
hipError_t lu_factor_staggered_z(double2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, int G,
                                 const hipStream_t* st, hipEvent_t* ev) {
  if (G > b.nb) G = b.nb;
  if (G < 2) return lu_factor_z(A, ipiv, info, b, work, st[0]);
  return factor_groups_staggered<double>(A, ipiv, info, b, work, G, 256, st, ev);
}
hipError_t lu_factor_staggered_c(float2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, int G,
                                 const hipStream_t* st, hipEvent_t* ev) {
  if (G > b.nb) G = b.nb;
  if (G < 2) return lu_factor_c(A, ipiv, info, b, work, st[0]);
  return factor_groups_staggered<float>(A, ipiv, info, b, work, G, 512, st, ev);
}
hipError_t lu_factor_list_c(const LuMat* d_list, int nb, int nmax, int panel, int plane_min, void* work,
                            hipStream_t s) {
  if (plane_min < 2 * kBT) return hipErrorInvalidValue;
  Batch<float2> bt = make_batch(Mats<float2>{nullptr, nullptr, nullptr, 0, nmax, d_list}, nb, nmax, work);
  bt.plane_min = plane_min;
  return factor<float>(bt, panel, s);
}
}  // namespace msv
