// Per-mode Mueller-Nystrom matrices on gfx950.
//
// For target node t and a source point y the 4x4 block couples the unknowns
// (J^1, J^2, M^1, M^2)(y) to the magnetic (rows 0,1) and electric (rows 2,3)
// equations of eq. mullerrep at t:
//
//   rows 0,1:  -i w (mu0 N^{k0} - mu1 N^{k1}) on J,   -(K^{k0} - K^{k1}) on M
//   rows 2,3:   (K^{k0} - K^{k1}) on J,   -i w (eps0 N^{k0} - eps1 N^{k1}) on M
//
// or, for the indirect system (eq. dualmullrep, Section 2.2), the same
// operators with the materials exchanged and other weights:
//
//   rows 0,1:  -i w (eps0 N^{k0} - eps1 N^{k1}) on J,  -(eps0/mu0)(K^{k0} - K^{k1}) on M
//   rows 2,3:   (mu0/eps0)(K^{k0} - K^{k1}) on J,   -i w (mu0 N^{k0} - mu1 N^{k1}) on M
//
// with jump terms -(i w/2)(eps0 + eps1) on J and -(i w/2)(mu0 + mu1) on M.
//
// The table holds g^{k0} and g^{k0} - g^{k1} (with derivatives), so
// mu N^{k0} - mu' N^{k1} = (mu - mu') N^{k0} + mu' (N^{k0} - N^{k1}) and the
// k^2 terms of K are (k0^2 - k1^2) c(g^{k0}) + k1^2 c(g^{k0} - g^{k1}).
//
// with N and K in mode m from the coefficients c^1, c^2, c^3 of Lemma 1 and the
// expansions of Section 3 (e_theta components taken with the sign that
// n x V = V_theta t - (r' V_r + z' V_z) e_theta gives for n = z' e_r - r' e_z).
// g^2_m = (g_{m+1} + g_{m-1})/2, g^3_m = (g_{m-1} - g_{m+1})/2 (from green21,
// green31).  The identity terms (i w/2)(mu0 + mu1), (i w/2)(eps0 + eps1) sit on
// the diagonal.  Quadrature (eqs. disequ, eq_nyslike2): far panels w_j B(t, x_j);
// the target's panel and its neighbours through the support nodes,
// sum_q W_q B(t, y_q) l_k(y_q).  Stored is the L^2-weighted matrix
// sqrt(w_t / w_j) A_tj, row-major.
//
// Two kernels write disjoint entries: `far` one thread per (t, node j) off the
// near panels, coalesced along j; `near` one workgroup per (t, m) for the
// 3 x 16 near columns, contracting support-node blocks held in LDS.
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

struct cd {
  double re, im;
};
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return mk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cd operator-(cd a, cd b) { return mk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cd operator-(cd a) { return mk(-a.re, -a.im); }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cd operator*(double s, cd a) { return mk(s * a.re, s * a.im); }
__device__ __forceinline__ cd ld(const double2* p) {
  double2 v = *p;
  return mk(v.x, v.y);
}
__device__ __forceinline__ cd mul_i(cd a) { return mk(-a.im, a.re); }  // i a

struct Consts {
  cd k12, kd2;      // k1^2, k0^2 - k1^2
  cd cJ0, cJ1;      // J block of rows 0,1: cJ0 N^{k0} + cJ1 (N^{k0} - N^{k1})
  cd cM0, cM1;      // M block of rows 2,3 likewise
  cd kJM, kMJ;      // K^{k0} - K^{k1} weights: rows 0,1 on M, rows 2,3 on J
  cd jJ, jM;        // jump terms on J (rows 0,1) and M (rows 2,3)
};

__device__ __forceinline__ cd cdiv(cd a, cd b) {
  const double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

__device__ Consts make_consts(const AsmParams& P) {
  Consts c;
  cd k1 = mk(P.k1r, P.k1i);
  c.k12 = k1 * k1;
  c.kd2 = mk(P.k0 * P.k0, 0) - c.k12;
  const cd miw = mk(0, -P.omega), hiw = mk(0, 0.5 * P.omega);
  const cd e0 = mk(P.eps0r, P.eps0i), m0 = mk(P.mu0r, P.mu0i);
  const cd e1 = mk(P.eps1r, P.eps1i), m1 = mk(P.mu1r, P.mu1i);
  // the J equations weigh N by mu (direct) or eps (indirect), the M equations
  // by the other material
  const cd a0 = P.formulation ? e0 : m0, a1 = P.formulation ? e1 : m1;
  const cd b0 = P.formulation ? m0 : e0, b1 = P.formulation ? m1 : e1;
  c.cJ0 = miw * (a0 - a1);
  c.cJ1 = miw * a1;
  c.cM0 = miw * (b0 - b1);
  c.cM1 = miw * b1;
  if (P.formulation) {
    c.kJM = -cdiv(e0, m0);
    c.kMJ = cdiv(m0, e0);
    c.jJ = -(hiw * (e0 + e1));
    c.jM = -(hiw * (m0 + m1));
  } else {
    c.kJM = mk(-1.0, 0.0);
    c.kMJ = mk(1.0, 0.0);
    c.jJ = hiw * (m0 + m1);
    c.jM = hiw * (e0 + e1);
  }
  return c;
}

// c^1, c^2, c^3 of Lemma 1 for a unit density in component beta (0: t, 1: theta)
// from one kernel family (G1 = g_m, G2 = g^2_m, G3 = g^3_m).
struct Cv {
  cd c1[2], c2[2], c3[2];
};
__device__ __forceinline__ Cv cvals(cd G1, cd G2, cd G3, double rs, double trs, double tzs) {
  Cv v;
  v.c1[0] = (rs * trs) * G2;
  v.c1[1] = -(rs * mul_i(G3));
  v.c2[0] = (rs * trs) * mul_i(G3);
  v.c2[1] = rs * G2;
  v.c3[0] = (rs * tzs) * G1;
  v.c3[1] = mk(0, 0);
  return v;
}

// 4x4 block for one (target, source point) pair; T[j][ty] holds modes
// m-1, m, m+1 (j = 0, 1, 2) of the nine tabulated types.
__device__ void block4(const cd T[3][kTypes], int m, double rt, double trt, double tzt, double rs,
                       double trs, double tzs, const Consts& C, cd B[4][4]) {
  cd G1[kTypes], G2[kTypes], G3[kTypes];
#pragma unroll
  for (int ty = 0; ty < kTypes; ++ty) {
    G1[ty] = T[1][ty];
    G2[ty] = 0.5 * (T[2][ty] + T[0][ty]);
    G3[ty] = 0.5 * (T[0][ty] - T[2][ty]);
  }
  const double irt = 1.0 / rt;
  const cd im_ = mk(0, (double)m);
  const cd im_r = mk(0, m * irt);
  const cd im_r2 = mk(0, m * irt * irt);
  const double m2_r2 = (double)m * m * irt * irt;
  cd N[2][2][2];  // [k][alpha][beta]
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int b = 3 * kk;
    Cv g = cvals(G1[b], G2[b], G3[b], rs, trs, tzs);
    Cv gr = cvals(G1[b + 1], G2[b + 1], G3[b + 1], rs, trs, tzs);
    Cv gz = cvals(G1[b + 2], G2[b + 2], G3[b + 2], rs, trs, tzs);
#pragma unroll
    for (int be = 0; be < 2; ++be) {
      N[kk][0][be] = gz.c1[be] - gr.c3[be];
      cd inner = (tzt * irt) * (g.c2[be] + rt * gr.c2[be] - im_ * g.c1[be]) +
                 trt * (im_r * g.c3[be] - gz.c2[be]);
      N[kk][1][be] = -inner;
    }
  }
  // K^{k0} - K^{k1} from the difference family (types 3..5)
  Cv d = cvals(G1[3], G2[3], G3[3], rs, trs, tzs);
  Cv dr = cvals(G1[4], G2[4], G3[4], rs, trs, tzs);
  Cv dz = cvals(G1[5], G2[5], G3[5], rs, trs, tzs);
  Cv rr = cvals(G1[6], G2[6], G3[6], rs, trs, tzs);
  Cv rz = cvals(G1[7], G2[7], G3[7], rs, trs, tzs);
  Cv zz = cvals(G1[8], G2[8], G3[8], rs, trs, tzs);
  Cv g0 = cvals(G1[0], G2[0], G3[0], rs, trs, tzs);
  cd K[2][2];
#pragma unroll
  for (int be = 0; be < 2; ++be) {
    cd Kt = C.kd2 * g0.c2[be] + C.k12 * d.c2[be] + im_r2 * d.c1[be] + im_r * dr.c1[be] -
            m2_r2 * d.c2[be] + im_r * dz.c3[be];
    cd dzD = irt * dz.c1[be] + rz.c1[be] + im_r * dz.c2[be] + zz.c3[be];
    cd drD = -(irt * irt) * d.c1[be] + irt * dr.c1[be] + rr.c1[be] - im_r2 * d.c2[be] +
             im_r * dr.c2[be] + rz.c3[be];
    cd kk = C.kd2 * (tzt * g0.c3[be] + trt * g0.c1[be]) + C.k12 * (tzt * d.c3[be] + trt * d.c1[be]);
    K[0][be] = Kt;
    K[1][be] = -(kk + tzt * dzD + trt * drD);
  }
#pragma unroll
  for (int al = 0; al < 2; ++al)
#pragma unroll
    for (int be = 0; be < 2; ++be) {
      // N[0] = N^{k0}, N[1] = N^{k0} - N^{k1}
      B[al][be] = C.cJ0 * N[0][al][be] + C.cJ1 * N[1][al][be];
      B[al][2 + be] = C.kJM * K[al][be];
      B[2 + al][be] = C.kMJ * K[al][be];
      B[2 + al][2 + be] = C.cM0 * N[0][al][be] + C.cM1 * N[1][al][be];
    }
}

__device__ __forceinline__ void load_T(const AsmParams& P, int m, int t, int col, cd T[3][kTypes]) {
  const int ms[3] = {m > 0 ? m - 1 : 1, m, m + 1};
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int ty = 0; ty < kTypes; ++ty)
      T[j][ty] = ld(P.kern + (((size_t)ms[j] * kTypes + ty) * P.nt + (t - P.t0)) * P.NS + col);
}

__device__ __forceinline__ bool near_panel(const AsmParams& P, int pt, int ps) {
  return ps == pt || ps == P.left[pt] || ps == P.right[pt];
}

constexpr int kFarThreads = 64;

// Work items (mode, source block, target), mode fastest.  Workgroups are
// dealt to the 8 XCDs round-robin, so the linear workgroup id is remapped to
// give each XCD one contiguous range of items: the three modes that read a
// table slice (m - 1, m, m + 1) then run back to back on one XCD and find the
// slice in its L2, instead of reading it from HBM three times.
__global__ __launch_bounds__(kFarThreads, 3) void assemble_far(AsmParams P, int n_items) {
  const int per = (n_items + 7) / 8;
  const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (item >= n_items) return;
  const int nm = P.m_hi - P.m_lo + 1;
  const int njb = (P.N + kFarThreads - 1) / kFarThreads;
  const int mi = item % nm;
  const int jb = (item / nm) % njb;
  const int t = P.t0 + item / nm / njb;
  const int j0 = jb * kFarThreads, j = j0 + threadIdx.x;
  const int m = P.m_lo + mi;
  const int pt = t / kOrder;
  const bool mine = j < P.N && !near_panel(P, pt, j / kOrder);
  cd B[4][4];
  double sc = 0.0;
  if (mine) {
    const Consts C = make_consts(P);
    cd T[3][kTypes];
    load_T(P, m, t, j, T);
    block4(T, m, P.r[t], P.tr[t], P.tz[t], P.r[j], P.tr[j], P.tz[j], C, B);
    sc = P.sqw[t] * P.sqw[j];  // w_j * sqrt(w_t / w_j)
  }
  // each row of the blocks goes out through LDS, so that a store instruction
  // writes 64 consecutive entries of the row (1 KB) instead of 16 bytes
  // every 64 (the workgroup is one wave)
  __shared__ double2 S[4 * kFarThreads];
  const size_t n = 4 * (size_t)P.N;
  double2* A = P.A + (size_t)mi * n * n;
#pragma unroll
  for (int al = 0; al < 4; ++al) {
    if (mine)
#pragma unroll
      for (int be = 0; be < 4; ++be) S[4 * threadIdx.x + be] = make_double2(sc * B[al][be].re, sc * B[al][be].im);
    __syncthreads();
    double2* row = A + (4 * (size_t)t + al) * n + 4 * (size_t)j0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = v * kFarThreads + threadIdx.x;  // entry 4 (j - j0) + beta
      const int je = j0 + (e >> 2);
      if (je < P.N && !near_panel(P, pt, je / kOrder)) row[e] = S[e];
    }
    __syncthreads();
  }
}

constexpr int kNearThreads = 256;

// Work items (mode, target), mode fastest, each XCD a contiguous range (as
// for the far blocks): the three modes that read a support slice of the table
// run back to back on one XCD.
__global__ __launch_bounds__(kNearThreads) void assemble_near(AsmParams P, int n_items) {
  extern __shared__ double smem[];
  const int per = (n_items + 7) / 8;
  const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (item >= n_items) return;
  const int nm = P.m_hi - P.m_lo + 1;
  const int mi = item % nm;
  const int t = P.t0 + item / nm;
  const int m = P.m_lo + mi;
  const int S = P.S;
  double2* Bw = reinterpret_cast<double2*>(smem);  // [S][16]
  // the Lagrange rows this target uses: its own panel's row kt, then the
  // adjacent panels' rows ([n][16] each), read from LDS in the contraction
  double* Ls = smem + 2 * 16 * (size_t)S;
  const int pt = t / kOrder, kt = t % kOrder;
  for (int e = threadIdx.x; e < P.n_self * kOrder; e += kNearThreads)
    Ls[e] = P.lag_self[(size_t)kt * P.n_self * kOrder + e];
  for (int e = threadIdx.x; e < P.n_adj * kOrder; e += kNearThreads) Ls[P.n_self * kOrder + e] = P.lag_adj[e];
  const Consts C = make_consts(P);
  const double rt = P.r[t], trt = P.tr[t], tzt = P.tz[t];
  for (int s = threadIdx.x; s < S; s += kNearThreads) {
    const double* sp = P.sup + ((size_t)t * S + s) * kSupFields;
    double wq = sp[kSupW];
    if (wq == 0.0) {
      for (int e = 0; e < 16; ++e) Bw[s * 16 + e] = make_double2(0, 0);
      continue;
    }
    cd T[3][kTypes];
    load_T(P, m, t, P.N + s, T);
    cd B[4][4];
    block4(T, m, rt, trt, tzt, sp[kSupR], sp[kSupTr], sp[kSupTz], C, B);
#pragma unroll
    for (int al = 0; al < 4; ++al)
#pragma unroll
      for (int be = 0; be < 4; ++be)
        Bw[s * 16 + al * 4 + be] = make_double2(wq * B[al][be].re, wq * B[al][be].im);
  }
  __syncthreads();
  const int panels[3] = {pt, P.left[pt], P.right[pt]};
  const int s0[3] = {0, P.n_self, P.n_self + P.n_adj};
  const int ns[3] = {P.n_self, P.n_adj, P.n_adj};
  const size_t n = 4 * (size_t)P.N;
  double2* A = P.A + (size_t)mi * n * n;
  const double sqt = P.sqw[t];
  // output e = (panel, alpha, node k, beta): consecutive threads -> consecutive
  // (k, beta) so each row segment of 64 complex is written contiguously
  for (int e = threadIdx.x; e < 3 * 4 * kOrder * 4; e += kNearThreads) {
    const int be = e & 3;
    const int k = (e >> 2) & (kOrder - 1);
    const int al = (e >> 6) & 3;
    const int pi = e >> 8;
    const int ps = panels[pi];
    if (ps < 0) continue;
    const double* lag = (pi == 0) ? Ls : Ls + P.n_self * kOrder;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < ns[pi]; ++q) {
      double l = lag[q * kOrder + k];
      double2 b = Bw[(s0[pi] + q) * 16 + al * 4 + be];
      re = fma(l, b.x, re);
      im = fma(l, b.y, im);
    }
    const int j = ps * kOrder + k;
    const double sc = sqt / P.sqw[j];
    re *= sc;
    im *= sc;
    if (j == t && al == be) {  // identity term, unchanged by the weighting
      const cd jt = (al < 2) ? C.jJ : C.jM;
      re += jt.re;
      im += jt.im;
    }
    A[(4 * (size_t)t + al) * n + 4 * (size_t)j + be] = make_double2(re, im);
  }
}

}  // namespace

hipError_t launch_assemble(const AsmParams& P, hipStream_t s) {
  const int nm = P.m_hi - P.m_lo + 1;
  if (P.nt <= 0) return hipSuccess;
  const long long items = (long long)nm * ((P.N + kFarThreads - 1) / kFarThreads) * P.nt;
  // a dispatch counts work-items in 32 bits
  if (items * kFarThreads >= (1LL << 32)) return hipErrorInvalidValue;
  const int n_items = (int)items;
  hipLaunchKernelGGL(assemble_far, dim3(8 * ((n_items + 7) / 8)), dim3(kFarThreads), 0, s, P, n_items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t lds = sizeof(double2) * 16 * (size_t)P.S + sizeof(double) * kOrder * (size_t)(P.n_self + P.n_adj);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&assemble_near), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  const int n_near = nm * P.nt;
  hipLaunchKernelGGL(assemble_near, dim3(8 * ((n_near + 7) / 8)), dim3(kNearThreads), lds, s, P, n_near);
  return hipGetLastError();
}

}  // namespace msv
