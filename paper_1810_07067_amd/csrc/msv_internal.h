// Internal declarations shared by the host plan and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msv.h"

namespace msv {

constexpr int kOrder = 16;
constexpr int kTypes = 9;

// Pair classes of the modal-kernel table.
enum : uint8_t { kFar = 0, kNear = 1, kZero = 2 };

// Parameters of the modal-kernel tabulation, identical for every pair of a body.
struct TabParams {
  int N;        // curve nodes
  int S;        // support slots per target
  int NS;       // N + S: row length of the table
  int M2;       // modes stored: 0 .. M+1
  int L;        // azimuthal FFT length
  int Mq;       // L/2 - 1: band limit of the singular spectra
  int fwd_n;    // forward Q recurrence iff acosh(chi) * fwd_n <= fwd_lim
  double fwd_lim;
  double miller_extra;  // Miller start: fwd_n + ceil(miller_extra / acosh chi)
  double k0;            // real
  double k1r, k1i;      // complex interior wavenumber
  const double* r;      // [N] node r
  const double* z;      // [N] node z
  const double* sup;    // [N][S][kSupFields]
  const uint8_t* cls;   // [N][NS]
  const int2* near;     // near pairs (t, source column), sorted by t
  int n_near;
  // row block: targets t0 .. t0+nt-1, their near pairs near[near_lo .. near_hi)
  int t0, nt, near_lo, near_hi;
  double2* out;         // [M2][9][nt][NS]
  // scratch for the Legendre-Q spectra of up to spec_cap near pairs at a
  // time: [spec_cap][L/2 + 1] complex (X1_n, X3_n)
  double2* spec;
  int spec_cap;
  // azimuth tables of the transforms, N = L/2: [N] e^{-2 pi i k / 2N}, then
  // [N/2 + 1] (cos, sin)(pi j / N), then [N + 2] sin^2(pi j / 2N) (doubles)
  const double2* tabs;
};
// doubles in the azimuth tables for FFT length L
inline size_t tab_doubles(int L) {
  const size_t N = L / 2;
  return 2 * N + 2 * (N / 2 + 1) + (N + 2);
}
// near pairs whose spectra the scratch holds at once, and its size in bytes
constexpr int kSpecCap = 262144;  // a launch of this many threads keeps 16 waves on each CU
inline size_t spec_bytes(int L, int n_near) {
  const size_t cap = (size_t)(n_near < kSpecCap ? n_near : kSpecCap);
  return (cap + 63) / 64 * 64 * (size_t)(L / 2 + 1) * sizeof(double2);  // pairs in groups of 64
}

// Support-slot record (doubles): offset from the target, the source geometry
// needed by the assembly, and the quadrature weight (0 = unused slot).
enum { kSupDr = 0, kSupDz, kSupR, kSupTr, kSupTz, kSupW, kSupFields };

struct AsmParams {
  int N, S, NS, M2, npan, n_self, n_adj, m_lo, m_hi;
  int t0, nt;           // equations of targets t0 .. t0+nt-1; kern holds their rows
  double k0, k1r, k1i, omega;
  double eps0r, eps0i, mu0r, mu0i, eps1r, eps1i, mu1r, mu1i;
  int formulation;      // 0: eq. mullerrep, 1: eq. dualmullrep
  const double* r;      // [N]
  const double* tr;     // [N] unit tangent r' = -nz
  const double* tz;     // [N] unit tangent z' = nr
  const double* w;      // [N] arclength weights
  const double* sqw;    // [N] sqrt(w)
  const double* sup;    // [N][S][kSupFields]
  const int* left;      // [npan]
  const int* right;     // [npan]
  const double* lag_self;  // [16][n_self][16]
  const double* lag_adj;   // [n_adj][16]
  const double2* kern;  // table rows of the block: [M2][9][nt][NS]
  double2* A;           // [m_hi-m_lo+1][4N][4N]
};

hipError_t launch_tabulate(const TabParams& p, hipStream_t s);
hipError_t launch_assemble(const AsmParams& p, hipStream_t s);

// Off-surface evaluation (fields.hip): the currents of nvec solves synthesized
// on the N x T surface grid, then one reduction per (vector, direction or point).
struct FieldParams {
  int N, T, nm, m_lo, nvec;
  const double* r;      // [N]
  const double* z;      // [N]
  const double* tr;     // [N] r'
  const double* tz;     // [N] z'
  const double* w;      // [N] arclength weights
  const double2* x;     // [nm][nvec][4N] modes m_lo .. m_lo + nm - 1 of the currents
  double2* tw;          // [T] (cos, sin)(2 pi j / T)
  double2* grid;        // [nvec][N][T][4] J^1, J^2, M^1, M^2 times the area weight
  int npts;
  const double* pts;    // [npts][3] unit directions (far field) or points
  double k0, kr, ki, omega, mu0;
  double2 aE, bE, aH, bH;  // E = aE ccS J + bE cS M, H = aH ccS M + bH cS J
  double2* out;         // [nvec][npts][3]: E_inf, or E
  double2* out2;        // [nvec][npts][3]: H
};
hipError_t launch_surface_grid(const FieldParams& p, hipStream_t s);
// current modes [nmv][4N] at U sub-panels of 16 nodes per panel: [nmv][4NU]
hipError_t launch_interp_currents(const double2* x, double2* xf, const double* L, int N, int U, int nmv,
                                  hipStream_t s);
hipError_t launch_far_field(const FieldParams& p, hipStream_t s);
hipError_t launch_fields(const FieldParams& p, hipStream_t s);

// Batched dense LU / solve (row-major, complex), see lu.hip.
// Inverses of 64 x 64 unit-lower diagonal blocks kept per matrix by the LU:
// one slot per 64-row piece of a 512-column outer panel.  The LU workspace
// passed to lu_factor_* holds them and, for complex64, the bf16 planes of the
// large trailing updates: lu_work_bytes(largest order, nb, complex128?).
constexpr int kLinvSlots = 8;
size_t lu_work_bytes(int n, int nb, bool c128);

struct LuBatch {
  int n;           // matrix order
  int nb;          // number of matrices
  long long ld;    // leading dimension (= n)
  long long stride;  // elements between matrices
};
// One matrix of a listed batch (matrices of different orders factored by the
// same launches): row-major storage of order n, its pivots [n] and info flag.
// A device pointer that the compiler is told lies in global memory.  Pointers
// read from memory (a list of matrices) or from a struct argument are generic
// to it; loads through them become flat loads, which also count against the
// LDS wait counter and so stall every LDS wait until they return.  On gfx9 a
// generic address of global memory is the global address itself.
template <typename T>
__device__ __forceinline__ T* global_ptr(T* p) {
  return (T*)(T __attribute__((address_space(1)))*)(size_t)p;
}

// *p where ok, else zero (a two-component vector type).  Written as a branch
// around the load so that the compiler does not pick between the address of
// p and the address of a local zero and load through a flat pointer.
template <typename T>
__device__ __forceinline__ T load_or_zero(const T* p, bool ok) {
  T v;
  v.x = 0;
  v.y = 0;
  if (ok) v = *p;
  return v;
}

// Sum over the 4 lanes of a quad, returned to each, in the order of a
// butterfly (x_t + x_t^1) + (x_t^2 + x_t^3): two DPP quad permutations in
// place of two LDS-permute shuffles.
template <int kCtrl>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xf, 0xf, false));
}
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename R>
__device__ __forceinline__ R quad_sum(R x) {
  x += dpp_move<0xb1>(x);  // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4e>(x);  // quad_perm [2, 3, 0, 1]
  return x;
}
// Sum over the 16 lanes of a DPP row, returned to each: the quad sums, then
// quads paired by the half-row mirror and halves by the row mirror.
template <typename R>
__device__ __forceinline__ R row_sum(R x) {
  x = quad_sum(x);
  x += dpp_move<0x141>(x);  // row_half_mirror
  x += dpp_move<0x140>(x);  // row_mirror
  return x;
}

struct LuMat {
  void* a;
  int32_t* ipiv;
  int32_t* info;
  int32_t n;
  int32_t pad;
};
// work: lu_work_bytes(n, nb, complex128?) bytes
hipError_t lu_factor_z(double2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, hipStream_t s);
hipError_t lu_factor_c(float2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, hipStream_t s);
// The same factorizations with the batch cut into G <= kStaggerMax
// consecutive groups (fewer if nb < G), group g on stream st[g], whose
// panels each wait for the same panel of group g - 1 (one group's panel
// factorization overlaps the others' trailing updates).  st[1..] wait for
// the work queued on st[0] before the call, and st[0] for all of their
// launches after it.  ev: kStaggerEvents events on the device.
constexpr int kStaggerMax = 4;
constexpr int kStaggerEvents = 256;
#ifndef MSV_LU_GROUPS
#define MSV_LU_GROUPS 2
#endif
constexpr int kLuGroups = MSV_LU_GROUPS;  // groups of a plan's own factorization
// A plan staggers its factorization only above this order: at 8192 it gains
// 8%, at 4096 nothing, and below that the extra waits cost more than the
// overlap saves (orders 512..2048 factored one body at a time: 1.5x slower).
constexpr int kStaggerMinOrder = 4097;
static_assert(kLuGroups >= 1 && kLuGroups <= kStaggerMax, "1 to kStaggerMax groups");
hipError_t lu_factor_staggered_z(double2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, int G,
                                 const hipStream_t* st, hipEvent_t* ev);
hipError_t lu_factor_staggered_c(float2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, void* work, int G,
                                 const hipStream_t* st, hipEvent_t* ev);
// complex64 factorization of a listed batch (d_list on the device) with outer
// panels of `panel` = 64, 128, 256 or 512 columns; nmax is the largest order, every
// other order a multiple of `panel`.  Trailing updates of at least plane_min
// (>= 256) rows and columns use 128 x 128 tiles, smaller ones 64 x 64.
hipError_t lu_factor_list_c(const LuMat* d_list, int nb, int nmax, int panel, int plane_min, void* work,
                            hipStream_t s);

// Right-hand-side batches for the solves (trsv.hip): up to kVB vectors that
// use factor `fac`; vector v is stored at element off[v] * n of the work
// arrays ([modes][nrhs][n]).
constexpr int kVB = 16;
struct VecBatch {
  int fac;
  int nv;
  int off[kVB];
};
// The batches of a solve over modes m_lo .. m_lo+nm-1 with n_rhs vectors each,
// against factors of modes fac_lo .. fac_lo+nfac-1 (|m| selects the factor):
// their number, and the table itself, written on the device in stream order.
int count_vec_batches(int m_lo, int nm, int n_rhs, int fac_lo, int nfac);
hipError_t build_vec_batches(VecBatch* vb, int nvb, int m_lo, int nm, int n_rhs, int fac_lo, int nfac,
                             hipStream_t s);
// perm[f][i] = source row of row i under the interchanges ipiv[f]
hipError_t lu_perm(const int32_t* ipiv, int32_t* perm, int n, int nfac, hipStream_t s);
// out = P in for every vector of the batches (complex128 or rounded to complex64)
hipError_t gather_z(const double2* in, double2* out, const int32_t* perm, const VecBatch* d_vb, int nvb, int n,
                    hipStream_t s);
hipError_t gather_c(const double2* in, float2* out, const int32_t* perm, const VecBatch* d_vb, int nvb, int n,
                    hipStream_t s);
// inverses of the 64 x 64 diagonal blocks of L and U: [nfac][ceil(n/64)][2][64][64]
hipError_t lu_inv_diag_z(const double2* LU, long long stride, int n, int nfac, double2* inv, hipStream_t s);
hipError_t lu_inv_diag_c(const float2* LU, long long stride, int n, int nfac, float2* inv, hipStream_t s);
// X <- U^{-1} L^{-1} X (X already permuted); Y is scratch of the same layout
hipError_t trsv_z(const double2* LU, const double2* inv, long long stride, int n, const VecBatch* d_vb, int nvb,
                  double2* X, double2* Y, hipStream_t s);
hipError_t trsv_c(const float2* LU, const float2* inv, long long stride, int n, const VecBatch* d_vb, int nvb,
                  float2* X, float2* Y, hipStream_t s);
// r = b - A[fac] x per vector, complex128
hipError_t residual_batches(const double2* A, long long stride, int n, const VecBatch* d_vb, int nvb,
                            const double2* b, const double2* x, double2* r, hipStream_t s);

// solve-side helpers (solve.hip)
hipError_t solve_prep(const double2* rhs, double2* xw, const double* sqw, int n, int nrhs, int nm,
                      int m_lo, hipStream_t s);
hipError_t solve_finish(const double2* xw, double2* x, const double* sqw, int n, int nrhs, int nm,
                        int m_lo, hipStream_t s);
hipError_t conv_c64(const double2* a, float2* b, size_t count, hipStream_t s);
hipError_t accum_c64(double2* x, const float2* d, size_t count, hipStream_t s);
hipError_t zero_c128(double2* x, size_t count, hipStream_t s);
// out[v] = ||r_v||_inf / ||b_v||_inf for v < nvec, and out[nvec] = their maximum
hipError_t ratios(const double2* r, const double2* b, double* out, int n, int nvec, hipStream_t s);

}  // namespace msv
