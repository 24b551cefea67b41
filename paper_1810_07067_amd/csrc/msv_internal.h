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
  double2* out;         // [M2][9][N][NS]
};

// Support-slot record (doubles): offset from the target, the source geometry
// needed by the assembly, and the quadrature weight (0 = unused slot).
enum { kSupDr = 0, kSupDz, kSupR, kSupTr, kSupTz, kSupW, kSupFields };

struct AsmParams {
  int N, S, NS, M2, npan, n_self, n_adj, m_lo, m_hi;
  double k0, k1r, k1i, omega;
  double eps0r, eps0i, mu0r, mu0i, eps1r, eps1i, mu1r, mu1i;
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
  const double2* kern;  // table
  double2* A;           // [m_hi-m_lo+1][4N][4N]
};

hipError_t launch_tabulate(const TabParams& p, hipStream_t s);
hipError_t launch_assemble(const AsmParams& p, hipStream_t s);

// Batched dense LU / solve (row-major, complex), see lu.hip.
struct LuBatch {
  int n;           // matrix order
  int nb;          // number of matrices
  long long ld;    // leading dimension (= n)
  long long stride;  // elements between matrices
};
hipError_t lu_factor_z(double2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, hipStream_t s);
hipError_t lu_factor_c(float2* A, int32_t* ipiv, int32_t* info, const LuBatch& b, hipStream_t s);
// x <- A^{-1} x for nrhs right-hand sides stored [nvec][nrhs][n]; batch entry
// i uses matrix map[i] of the factored batch (LuBatch::nb = nvec here).
hipError_t lu_solve_z(const double2* LU, const int32_t* ipiv, const int* map, double2* X, int nrhs,
                      const LuBatch& b, hipStream_t s);
hipError_t lu_solve_c(const float2* LU, const int32_t* ipiv, const int* map, float2* X, int nrhs,
                      const LuBatch& b, hipStream_t s);

// solve-side helpers (solve.hip)
hipError_t solve_prep(const double2* rhs, double2* xw, const double* sqw, int n, int nrhs, int nm,
                      int m_lo, hipStream_t s);
hipError_t solve_finish(const double2* xw, double2* x, const double* sqw, int n, int nrhs, int nm,
                        int m_lo, hipStream_t s);
hipError_t conv_c64(const double2* a, float2* b, size_t count, hipStream_t s);
hipError_t accum_c64(double2* x, const float2* d, size_t count, hipStream_t s);
hipError_t zero_c128(double2* x, size_t count, hipStream_t s);
hipError_t residual_z(const double2* A, const int* map, const double2* b, const double2* x, double2* r,
                      int n, int nrhs, int nm, hipStream_t s);
hipError_t ratios(const double2* r, const double2* b, double* out, int n, int nvec, hipStream_t s);

}  // namespace msv
