// Fields off the surface and the far-field pattern from the modal currents
// (Section 2.1: eqs. exteriorfield, interiorfield; Section 2.2: eq.
// interior_dual; Section 6: eq. farfieldform).
//
// The currents J = J^1 t + J^2 e_theta, M likewise, of one solve are given by
// their azimuthal modes.  They are first synthesized on a surface grid: the
// N nodes of the generating curve times T equispaced azimuths theta_t =
// 2 pi t / T, each point weighted by its share of the area element
// w_n r_n (2 pi / T) (Gauss-Legendre along the curve, trapezoid in theta).
// The mode sum at (n, t) reads e^{i m theta_t} from a table by the exact
// index (m t) mod T.  Every field value is then one sum over the grid,
// reduced by one workgroup:
//
//   far field:  Jt = sum e^{-i k0 xhat.y} J da,  Mt likewise,
//               E_inf = (1/(4 pi)) [i k0 xhat x Mt - i omega mu0 xhat x (xhat x Jt)];
//   off-surface point x, wavenumber k of its region, G = e^{i k R}/(4 pi R):
//               curl S V      = sum grad_x G x V da,
//               curl curl S V = sum [(grad grad G) V + k^2 G V] da,
//   with grad_x G = G (i k - 1/R) R_vec / R and
//   d_a d_b G = G [(3 - 3 i k R - k^2 R^2) R_a R_b / R^4 + (i k R - 1) delta_ab / R^2],
//   and E = aE curl curl S J + bE curl S M, H = aH curl curl S M + bH curl S J
//   with the coefficients of the region's representation.
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

constexpr int kFieldThreads = 256;

struct cz {
  double re, im;
};
__device__ __forceinline__ cz cmk(double r, double i) { return cz{r, i}; }
__device__ __forceinline__ cz operator+(cz a, cz b) { return cmk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cz operator-(cz a, cz b) { return cmk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cz operator*(cz a, cz b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cz operator*(double s, cz a) { return cmk(s * a.re, s * a.im); }
__device__ __forceinline__ cz from2(double2 v) { return cmk(v.x, v.y); }

__global__ __launch_bounds__(kFieldThreads) void twiddles(double2* tw, int T) {
  const int j = blockIdx.x * kFieldThreads + threadIdx.x;
  if (j >= T) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)T, &s, &c);
  tw[j] = make_double2(c, s);
}

// One workgroup per (vector v, node n); threads over the azimuths.
__global__ __launch_bounds__(kFieldThreads) void surface_grid(FieldParams P) {
  const int vn = blockIdx.x;
  const int v = vn / P.N, n = vn - v * P.N;
  const int T = P.T;
  const double da = P.w[n] * P.r[n] * (2.0 * M_PI / T);
  for (int t = threadIdx.x; t < T; t += kFieldThreads) {
    long long i0 = ((long long)P.m_lo * t) % T;
    if (i0 < 0) i0 += T;
    int idx = (int)i0;
    cz acc[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};
    const double2* xs = P.x + (size_t)v * 4 * P.N + 4 * n;
    const size_t mstride = (size_t)P.nvec * 4 * P.N;
    for (int k = 0; k < P.nm; ++k) {
      const cz e = from2(P.tw[idx]);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = acc[c] + from2(xs[c]) * e;
      xs += mstride;
      idx += t;  // t < T: one wrap at most
      if (idx >= T) idx -= T;
    }
    double2* g = P.grid + (((size_t)v * P.N + n) * T + t) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = make_double2(da * acc[c].re, da * acc[c].im);
  }
}

// Sum NV doubles over the workgroup; the result is valid in thread 0.
template <int NV>
__device__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kFieldThreads / 64; ++w)
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] += red[w * NV + i];
}

// Cartesian components of a1 t + a2 e_theta at azimuth (c, s) = (cos, sin).
__device__ __forceinline__ void to_cart(cz a1, cz a2, double trn, double tzn, double c, double s, cz (&V)[3]) {
  V[0] = (trn * c) * a1 - s * a2;
  V[1] = (trn * s) * a1 + c * a2;
  V[2] = tzn * a1;
}

// One workgroup per (direction d, vector v): blockIdx.x = v * ndirs + d.
__global__ __launch_bounds__(kFieldThreads) void far_field(FieldParams P) {
  __shared__ double red[kFieldThreads / 64 * 12];
  const int v = blockIdx.x / P.npts, d = blockIdx.x - v * P.npts;
  const double xh[3] = {P.pts[3 * d], P.pts[3 * d + 1], P.pts[3 * d + 2]};
  double acc[12] = {};  // Jt (re, im) x 3, then Mt
  const int T = P.T;
  for (int n = 0; n < P.N; ++n) {
    const double rn = P.r[n], zn = P.z[n], trn = P.tr[n], tzn = P.tz[n];
    const double2* g = P.grid + ((size_t)v * P.N + n) * T * 4;
    for (int t = threadIdx.x; t < T; t += kFieldThreads) {
      const double2 cs = P.tw[t];
      const double ph = -P.k0 * (xh[0] * rn * cs.x + xh[1] * rn * cs.y + xh[2] * zn);
      double sn, cn;
      sincos(ph, &sn, &cn);
      const cz e = cmk(cn, sn);
      cz J[3], M[3];
      to_cart(from2(g[4 * t]), from2(g[4 * t + 1]), trn, tzn, cs.x, cs.y, J);
      to_cart(from2(g[4 * t + 2]), from2(g[4 * t + 3]), trn, tzn, cs.x, cs.y, M);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cz a = e * J[c], b = e * M[c];
        acc[2 * c] += a.re;
        acc[2 * c + 1] += a.im;
        acc[6 + 2 * c] += b.re;
        acc[6 + 2 * c + 1] += b.im;
      }
    }
  }
  block_sum<12>(acc, red);
  if (threadIdx.x != 0) return;
  cz Jt[3], Mt[3];
  for (int c = 0; c < 3; ++c) {
    Jt[c] = cmk(acc[2 * c], acc[2 * c + 1]);
    Mt[c] = cmk(acc[6 + 2 * c], acc[6 + 2 * c + 1]);
  }
  // xhat x Mt, xhat x (xhat x Jt) = xhat (xhat . Jt) - Jt
  cz xM[3], xxJ[3];
  xM[0] = xh[1] * Mt[2] - xh[2] * Mt[1];
  xM[1] = xh[2] * Mt[0] - xh[0] * Mt[2];
  xM[2] = xh[0] * Mt[1] - xh[1] * Mt[0];
  const cz xJ = xh[0] * Jt[0] + xh[1] * Jt[1] + xh[2] * Jt[2];
  for (int c = 0; c < 3; ++c) xxJ[c] = xh[c] * xJ - Jt[c];
  const double s4 = 1.0 / (4.0 * M_PI);
  double2* out = P.out + ((size_t)v * P.npts + d) * 3;
  for (int c = 0; c < 3; ++c) {
    // (1/4 pi) [i k0 xM - i omega mu0 xxJ]
    const cz a = P.k0 * xM[c] - (P.omega * P.mu0) * xxJ[c];
    out[c] = make_double2(-s4 * a.im, s4 * a.re);
  }
}

// One workgroup per (point p, vector v): blockIdx.x = v * npts + p.
__global__ __launch_bounds__(kFieldThreads) void near_fields(FieldParams P) {
  __shared__ double red[kFieldThreads / 64 * 24];
  const int v = blockIdx.x / P.npts, p = blockIdx.x - v * P.npts;
  const double x0 = P.pts[3 * p], x1 = P.pts[3 * p + 1], x2 = P.pts[3 * p + 2];
  const cz k = cmk(P.kr, P.ki);
  const cz ik = cmk(-P.ki, P.kr), k2 = k * k;
  // curl S J, curl curl S J, curl S M, curl curl S M: 4 x 3 complex
  double acc[24] = {};
  const int T = P.T;
  for (int n = 0; n < P.N; ++n) {
    const double rn = P.r[n], zn = P.z[n], trn = P.tr[n], tzn = P.tz[n];
    const double2* g = P.grid + ((size_t)v * P.N + n) * T * 4;
    for (int t = threadIdx.x; t < T; t += kFieldThreads) {
      const double2 cs = P.tw[t];
      const double R[3] = {x0 - rn * cs.x, x1 - rn * cs.y, x2 - zn};
      const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      const double r = sqrt(r2), ir = 1.0 / r, ir2 = ir * ir;
      double sn, cn;
      sincos(P.kr * r, &sn, &cn);
      const double dmp = exp(-P.ki * r) * ir * (0.25 / M_PI);
      const cz G = cmk(dmp * cn, dmp * sn);
      const cz ikr = r * ik;
      const cz g1 = (ir * G) * (ik - cmk(ir, 0.0));                            // grad G = g1 R
      const cz f1 = (ir2 * ir2) * G * (cmk(3.0, 0.0) - 3.0 * ikr - r2 * k2);   // coefficient of R_a R_b
      const cz f2 = ir2 * G * (ikr - cmk(1.0, 0.0)) + k2 * G;                  // of delta_ab, plus k^2 G
      cz V[2][3];
      to_cart(from2(g[4 * t]), from2(g[4 * t + 1]), trn, tzn, cs.x, cs.y, V[0]);
      to_cart(from2(g[4 * t + 2]), from2(g[4 * t + 3]), trn, tzn, cs.x, cs.y, V[1]);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const cz* W = V[q];
        const cz cr[3] = {R[1] * W[2] - R[2] * W[1], R[2] * W[0] - R[0] * W[2], R[0] * W[1] - R[1] * W[0]};
        const cz RW = R[0] * W[0] + R[1] * W[1] + R[2] * W[2];
        const cz f1RW = f1 * RW;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cz a = g1 * cr[c];
          const cz b = R[c] * f1RW + f2 * W[c];
          acc[12 * q + 2 * c] += a.re;
          acc[12 * q + 2 * c + 1] += a.im;
          acc[12 * q + 6 + 2 * c] += b.re;
          acc[12 * q + 6 + 2 * c + 1] += b.im;
        }
      }
    }
  }
  block_sum<24>(acc, red);
  if (threadIdx.x != 0) return;
  const cz aE = from2(P.aE), bE = from2(P.bE), aH = from2(P.aH), bH = from2(P.bH);
  double2* E = P.out + ((size_t)v * P.npts + p) * 3;
  double2* H = P.out2 + ((size_t)v * P.npts + p) * 3;
  for (int c = 0; c < 3; ++c) {
    const cz cJ = cmk(acc[2 * c], acc[2 * c + 1]), ccJ = cmk(acc[6 + 2 * c], acc[6 + 2 * c + 1]);
    const cz cM = cmk(acc[12 + 2 * c], acc[12 + 2 * c + 1]), ccM = cmk(acc[18 + 2 * c], acc[18 + 2 * c + 1]);
    const cz e = aE * ccJ + bE * cM, h = aH * ccM + bH * cJ;
    E[c] = make_double2(e.re, e.im);
    H[c] = make_double2(h.re, h.im);
  }
}

// Current modes at the sub-panel nodes: xf[kv][4 nf + c] = sum_j L[f][j]
// x[kv][4 (16 p + j) + c] for fine node nf = 16 U p + f (L: [16 U][16]).
__global__ __launch_bounds__(kFieldThreads) void interp_currents(const double2* __restrict__ x,
                                                                 double2* __restrict__ xf, const double* L, int N,
                                                                 int U, long long total) {
  const int NU = N * U, F = 16 * U;
  for (long long i = (long long)blockIdx.x * kFieldThreads + threadIdx.x; i < total;
       i += (long long)gridDim.x * kFieldThreads) {
    const int c = (int)(i & 3);
    const long long q = i >> 2;
    const long long kv = q / NU;
    const int nf = (int)(q - kv * NU);
    const int p = nf / F, f = nf - p * F;
    const double2* src = x + kv * 4 * N + 4 * 16 * p + c;
    const double* l = L + 16 * f;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double2 v = src[4 * j];
      re = fma(l[j], v.x, re);
      im = fma(l[j], v.y, im);
    }
    xf[i] = make_double2(re, im);
  }
}

}  // namespace

hipError_t launch_interp_currents(const double2* x, double2* xf, const double* L, int N, int U, int nmv,
                                  hipStream_t s) {
  const long long total = (long long)nmv * N * U * 4;
  const long long blocks = (total + kFieldThreads - 1) / kFieldThreads;
  hipLaunchKernelGGL(interp_currents, dim3((unsigned)(blocks < (1 << 20) ? blocks : (1 << 20))),
                     dim3(kFieldThreads), 0, s, x, xf, L, N, U, total);
  return hipGetLastError();
}

hipError_t launch_surface_grid(const FieldParams& P, hipStream_t s) {
  if (P.T < 1 || P.N < 1 || P.nvec < 1 || P.nm < 1) return hipErrorInvalidValue;
  if ((long long)P.nvec * P.N >= (1LL << 31) / kFieldThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL(twiddles, dim3((P.T + kFieldThreads - 1) / kFieldThreads), dim3(kFieldThreads), 0, s, P.tw, P.T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(surface_grid, dim3(P.nvec * P.N), dim3(kFieldThreads), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_far_field(const FieldParams& P, hipStream_t s) {
  if ((long long)P.nvec * P.npts >= (1LL << 31) / kFieldThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL(far_field, dim3(P.nvec * P.npts), dim3(kFieldThreads), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_fields(const FieldParams& P, hipStream_t s) {
  if ((long long)P.nvec * P.npts >= (1LL << 31) / kFieldThreads) return hipErrorInvalidValue;
  hipLaunchKernelGGL(near_fields, dim3(P.nvec * P.npts), dim3(kFieldThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace msv
