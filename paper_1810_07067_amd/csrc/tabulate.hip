// Modal-kernel tabulation on gfx950 (Section 4 of Lai & O'Neil).
//
// For each (target, source) pair the nine modal quantities are the azimuthal
// Fourier coefficients, m = 0..M+1, of integrands that are even in phi.  Each
// integrand is sampled on phi_j = 2 pi j / L (j = 0..L/2 by evenness) and
// transformed with the real-even (cosine) form of the L-point DFT.  Integrands
// are split as sum(analytic factor x X) + analytic part, X in {1/rho,
// 1/rho^3}; for well separated ("far") pairs X is exact, for near pairs X is
// replaced by its band-limited series sum_{|n|<=M_q} X_n e^{i n phi}/(2 pi)
// with X_n from the half-odd Legendre recurrences (eqs. lm, recurform, pm and
// Lemma A.2), which turns the L-point sum into the discrete convolution of
// eq. discA.
//
// Work decomposition: a 256-thread workgroup owns TP pairs.  The folded sample
// index j in [0, L/4] pairs phi_j with pi - phi_j, so even modes need
// f(phi_j) + f(pi - phi_j) and odd modes f(phi_j) - f(pi - phi_j).  Samples are
// produced chunk by chunk into LDS (one thread per (pair, folded j)), then each
// thread accumulates 18 real sequences x MB modes of one parity for one pair
// in registers.  Outputs go to HBM once, coalesced along the source index.
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

constexpr int kThreads = 256;
constexpr int kSeq = 2 * kTypes;  // 18 real sequences
// LDS stride of one pair's folded samples: one double of padding puts the
// pairs a wave reads at distinct banks
constexpr int kEO = 2 * kSeq + 1;
constexpr int kNSer = 13;  // |x| <= 2: the 13th term is below 1e-17 of the first

struct SeriesCoef {
  double sinc[kNSer], y3[kNSer], wt[kNSer], ut[kNSer], v5[kNSer], ct[kNSer];
};

constexpr double cfact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

constexpr SeriesCoef make_coef() {
  // Taylor coefficients in y = x^2 of
  //   sinc x, Y3 = (x cos x - sin x)/x^3, Wt = (cos x + x sin x - 1)/x^2,
  //   Ut = (3 cos x - x^2 cos x + 3 x sin x - 3)/x^2,
  //   V5 = (3 sin x - x^2 sin x - 3 x cos x)/x^5, Ct = (cos x - 1)/x^2.
  SeriesCoef c{};
  for (int i = 0; i < kNSer; ++i) {
    double sg = (i % 2 == 0) ? 1.0 : -1.0;
    c.sinc[i] = sg / cfact(2 * i + 1);
    c.y3[i] = -sg * 2.0 * (i + 1) / cfact(2 * i + 3);
    c.wt[i] = sg * (2.0 * i + 1) / cfact(2 * i + 2);
    c.ut[i] = -sg * (2.0 * i + 1) * (2.0 * i - 1) / cfact(2 * i + 2);
    c.v5[i] = sg * 4.0 * (i + 2) * (i + 1) / cfact(2 * i + 5);
    c.ct[i] = -sg / cfact(2 * i + 2);
  }
  return c;
}

__constant__ SeriesCoef kCoef = make_coef();

struct cd {
  double re, im;
};
__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return mk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ cd operator-(cd a, cd b) { return mk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ cd operator*(double s, cd a) { return mk(s * a.re, s * a.im); }
__device__ __forceinline__ cd cinv(cd a) {
  double d = 1.0 / (a.re * a.re + a.im * a.im);
  return mk(a.re * d, -a.im * d);
}

// Analytic factors of x = k rho (Section 4; small-rho Taylor branch).
struct FacR {
  double c, sinc, W, Y3, Wt, Ut, V5, Ct;
};
struct FacC {
  cd c, sinc, W, Y3, Wt, Ut, V5, Ct;
};

__device__ __forceinline__ FacR factors(double x) {
  FacR f;
  double s, c;
  sincos(x, &s, &c);
  double y = x * x;
  f.c = c;
  if (fabs(x) <= 2.0) {
    double a0 = kCoef.sinc[kNSer - 1], a1 = kCoef.y3[kNSer - 1], a2 = kCoef.wt[kNSer - 1];
    double a3 = kCoef.ut[kNSer - 1], a4 = kCoef.v5[kNSer - 1], a5 = kCoef.ct[kNSer - 1];
#pragma unroll
    for (int i = kNSer - 2; i >= 0; --i) {
      a0 = fma(a0, y, kCoef.sinc[i]);
      a1 = fma(a1, y, kCoef.y3[i]);
      a2 = fma(a2, y, kCoef.wt[i]);
      a3 = fma(a3, y, kCoef.ut[i]);
      a4 = fma(a4, y, kCoef.v5[i]);
      a5 = fma(a5, y, kCoef.ct[i]);
    }
    f.sinc = a0;
    f.Y3 = a1;
    f.Wt = a2;
    f.Ut = a3;
    f.V5 = a4;
    f.Ct = a5;
  } else {
    double ix = 1.0 / x;
    double iy = ix * ix;
    f.sinc = s * ix;
    f.Y3 = (x * c - s) * ix * iy;
    f.Wt = (c + x * s - 1.0) * iy;
    f.Ut = (3.0 * c - y * c + 3.0 * x * s - 3.0) * iy;
    f.V5 = (3.0 * s - y * s - 3.0 * x * c) * iy * iy * ix;
    f.Ct = (c - 1.0) * iy;
  }
  f.W = 1.0 + y * f.Wt;
  return f;
}

__device__ __forceinline__ FacC factors(cd x) {
  FacC f;
  double sa, ca;
  sincos(x.re, &sa, &ca);
  double ch = cosh(x.im), sh = sinh(x.im);
  cd c = mk(ca * ch, -sa * sh);
  cd s = mk(sa * ch, ca * sh);
  cd y = x * x;
  f.c = c;
  if (x.re * x.re + x.im * x.im <= 4.0) {
    cd a0 = mk(kCoef.sinc[kNSer - 1], 0), a1 = mk(kCoef.y3[kNSer - 1], 0);
    cd a2 = mk(kCoef.wt[kNSer - 1], 0), a3 = mk(kCoef.ut[kNSer - 1], 0);
    cd a4 = mk(kCoef.v5[kNSer - 1], 0), a5 = mk(kCoef.ct[kNSer - 1], 0);
#pragma unroll
    for (int i = kNSer - 2; i >= 0; --i) {
      a0 = a0 * y + mk(kCoef.sinc[i], 0);
      a1 = a1 * y + mk(kCoef.y3[i], 0);
      a2 = a2 * y + mk(kCoef.wt[i], 0);
      a3 = a3 * y + mk(kCoef.ut[i], 0);
      a4 = a4 * y + mk(kCoef.v5[i], 0);
      a5 = a5 * y + mk(kCoef.ct[i], 0);
    }
    f.sinc = a0;
    f.Y3 = a1;
    f.Wt = a2;
    f.Ut = a3;
    f.V5 = a4;
    f.Ct = a5;
  } else {
    cd ix = cinv(x);
    cd iy = ix * ix;
    cd xs = x * s, xc = x * c, yc = y * c, ys = y * s;
    f.sinc = s * ix;
    f.Y3 = (xc - s) * ix * iy;
    f.Wt = (c + xs - mk(1.0, 0)) * iy;
    f.Ut = (3.0 * c - yc + 3.0 * xs - mk(3.0, 0)) * iy;
    f.V5 = (3.0 * s - ys - 3.0 * xc) * iy * iy * ix;
    f.Ct = (c - mk(1.0, 0)) * iy;
  }
  f.W = mk(1.0, 0) + y * f.Wt;
  return f;
}

// Pair geometry, target-relative.
struct Pair {
  double rt, rs, dr, dz, d2, a, inv2rt;
};

__device__ __forceinline__ Pair make_pair(double rt, double dr, double dz) {
  Pair p;
  p.rt = rt;
  p.dr = dr;
  p.dz = dz;
  p.rs = rt + dr;
  p.d2 = dr * dr + dz * dz;
  p.a = -dr * (2.0 * rt + dr) - dz * dz;  // r_t^2 - r_s^2 - z_d^2
  p.inv2rt = 0.5 / rt;
  return p;
}

// The nine integrands (times 4 pi) at one azimuth: o[2*type + {re, im}].
// NEAR: X1, X3 are band-limited and r_d/rho^3, r_d^2/rho^3 go through
// r_d = (rho^2 + a)/(2 r_t); far pairs have exact X and use r_d directly (the
// identity cancels badly when r_t is small and rho is not).
template <bool NEAR, bool K1C>
__device__ __forceinline__ void sample(const Pair& g, double s2, double cphi, double X1, double X3,
                                       double k0, cd k1, double* o) {
  double rho2 = g.d2 + 4.0 * g.rt * g.rs * s2;
  double rho = sqrt(rho2);
  double rd = g.rt - g.rs * cphi;
  double zd = -g.dz;
  double Xa, Xaa;  // r_d / rho^3, r_d^2 / rho^3
  if (NEAR) {
    Xa = (X1 + g.a * X3) * g.inv2rt;
    Xaa = (rho2 * X1 + 2.0 * g.a * X1 + g.a * g.a * X3) * (g.inv2rt * g.inv2rt);
  } else {
    Xa = rd * X3;
    Xaa = rd * rd * X3;
  }
  FacR f0 = factors(k0 * rho);
  double k02 = k0 * k0, k03 = k02 * k0, k05 = k03 * k02;
  o[0] = f0.c * X1;
  o[1] = k0 * f0.sinc;
  o[2] = -f0.W * Xa;
  o[3] = k03 * f0.Y3 * rd;
  o[4] = -zd * f0.W * X3;
  o[5] = zd * k03 * f0.Y3;
  // interior family as k0 - k1 differences:
  //   dg = rho^2 Cd X1 + i Sd,  d_r dg = r_d F,  d_z dg = z_d F,  F = -Wd X1 + i Y3d
  cd P, Wd, V5d, Y3d, Cd, Sd;
  if (!K1C) {
    double k1r = k1.re;
    FacR f1 = factors(k1r * rho);
    double k12 = k1r * k1r, k13 = k12 * k1r, k15 = k13 * k12;
    P = mk(k02 * f0.Ut - k12 * f1.Ut, 0);
    Wd = mk(k02 * f0.Wt - k12 * f1.Wt, 0);
    V5d = mk(k05 * f0.V5 - k15 * f1.V5, 0);
    Y3d = mk(k03 * f0.Y3 - k13 * f1.Y3, 0);
    Cd = mk(k02 * f0.Ct - k12 * f1.Ct, 0);
    Sd = mk(k0 * f0.sinc - k1r * f1.sinc, 0);
  } else {
    FacC f1 = factors(rho * k1);
    cd k12 = k1 * k1, k13 = k12 * k1, k15 = k13 * k12;
    P = mk(k02 * f0.Ut, 0) - k12 * f1.Ut;
    Wd = mk(k02 * f0.Wt, 0) - k12 * f1.Wt;
    V5d = mk(k05 * f0.V5, 0) - k15 * f1.V5;
    Y3d = mk(k03 * f0.Y3, 0) - k13 * f1.Y3;
    Cd = mk(k02 * f0.Ct, 0) - k12 * f1.Ct;
    Sd = mk(k0 * f0.sinc, 0) - k1 * f1.sinc;
  }
  {
    const cd dg = (rho2 * X1) * Cd + mk(-Sd.im, Sd.re);
    const cd F = mk(-Y3d.im - X1 * Wd.re, Y3d.re - X1 * Wd.im);
    o[6] = dg.re;
    o[7] = dg.im;
    o[8] = rd * F.re;
    o[9] = rd * F.im;
    o[10] = zd * F.re;
    o[11] = zd * F.im;
  }
  // i * (V5d rd^2 + Y3d) etc.
  cd t_rr = V5d * mk(rd * rd, 0) + Y3d;
  cd t_rz = V5d * mk(rd * zd, 0);
  cd t_zz = V5d * mk(zd * zd, 0) + Y3d;
  cd rr = Xaa * P - X1 * Wd + mk(-t_rr.im, t_rr.re);
  cd rz = (zd * Xa) * P + mk(-t_rz.im, t_rz.re);
  cd zz = (zd * zd * X3) * P - X1 * Wd + mk(-t_zz.im, t_zz.re);
  o[12] = rr.re;
  o[13] = rr.im;
  o[14] = rz.re;
  o[15] = rz.im;
  o[16] = zz.re;
  o[17] = zz.im;
}

// Complete elliptic integrals K, E of modulus k given k'^2, by the AGM from
// (1, k'), accurate as k' -> 0.
__device__ void elliptic_ke(double kp2, double& K, double& E) {
  double a = 1.0, b = sqrt(kp2);
  double s = 0.5 * (1.0 - kp2), p = 0.5;
  for (int it = 0; it < 40; ++it) {
    double c = 0.5 * (a - b);
    double an = 0.5 * (a + b);
    b = sqrt(a * b);
    a = an;
    p *= 2.0;
    s += p * c * c;
    if (c == 0.0 || fabs(c) <= 1e-17 * a) break;
  }
  K = M_PI / (2.0 * a);
  E = K * (1.0 - s);
}

// Spectra X1_n, X3_n (n = 0..Mq) of 1/rho and 1/rho^3 for one near pair.
// Written to x1[n], x3[n] (LDS).
__device__ void near_spectra(const Pair& g, const TabParams& P, double* x1, double* x3) {
  const int Mq = P.Mq;
  double eta = g.d2 / (2.0 * g.rt * g.rs);
  double chi = 1.0 + eta;
  double acs = log1p(eta + sqrt(eta * (2.0 + eta)));
  double K, E;
  elliptic_ke(eta / (2.0 + eta), K, E);
  double q0 = sqrt(2.0 / (2.0 + eta)) * K;
  double tail = sqrt(2.0 * (2.0 + eta)) * E;  // chi Q_{-1/2} - Q_{1/2}
  double c1 = 2.0 / sqrt(g.rt * g.rs);
  double c3 = sqrt(8.0) / (eta * (2.0 + eta)) / ((2.0 * g.rt * g.rs) * sqrt(2.0 * g.rt * g.rs));
  if (acs * P.fwd_n <= P.fwd_lim) {
    // Forward recurrence on D_n = Q_{n-1/2} - Q_{n-3/2}:
    //   (n + 1/2) D_{n+1} = (n - 1/2) D_n + 2 n eta Q_{n-1/2}
    double Q = q0;
    double D = eta * q0 - tail;
    x1[0] = c1 * Q;
    x3[0] = c3 * tail;
    for (int n = 1; n <= Mq; ++n) {
      Q = Q + D;
      double num = D + eta * Q;
      x1[n] = c1 * Q;
      x3[n] = c3 * (1.0 - 2.0 * n) * num;
      D = ((n - 0.5) * D + 2.0 * n * eta * Q) / (n + 0.5);
    }
  } else {
    // Miller's backward recurrence from n_start, normalized by Q_{-1/2}.
    int ns = P.fwd_n + (int)ceil(P.miller_extra / acs);
    if (ns < Mq + 2) ns = Mq + 2;
    double fhi = 0.0, f = 1.0;
    for (int n = ns; n >= 1; --n) {
      double flo = (2.0 * n * chi * f - (n + 0.5) * fhi) / (n - 0.5);
      fhi = f;
      f = flo;
      if (n - 1 <= Mq) x1[n - 1] = f;
      if (fabs(f) > 1e250) {
        fhi *= 1e-250;
        f *= 1e-250;
        for (int i = n - 1; i <= Mq; ++i) x1[i] *= 1e-250;
      }
    }
    double sc = q0 / x1[0];
    // num_n = chi Q_n - Q_{n-1}; go downward so Q_{n-1} is still raw
    for (int n = Mq; n >= 1; --n) {
      double Qn = x1[n] * sc, Qm = x1[n - 1] * sc;
      x3[n] = c3 * (1.0 - 2.0 * n) * (chi * Qn - Qm);
    }
    x3[0] = c3 * tail;
    for (int n = 0; n <= Mq; ++n) x1[n] = c1 * (x1[n] * sc);
  }
}

template <bool NEAR, bool K1C, int MB>
__global__ __launch_bounds__(kThreads) void tabulate_kernel(TabParams P, int TP, int JC, int Q) {
  extern __shared__ double smem[];
  const int L = P.L;
  const int Lq = L / 4;
  const int Mq = P.Mq;
  double* cos_tab = smem;                 // [L]
  double* s2_tab = cos_tab + L;           // [L/2 + 1]
  double* geo = s2_tab + (L / 2 + 2);     // [TP][4]: rt, dr, dz, valid flag
  double* EO = geo + 4 * TP;              // [JC][TP][kEO]: 2 x 18 folded samples
  double* Xh = EO + (size_t)JC * TP * kEO;  // NEAR: [TP][2][Mq+1]
  int* tgt = reinterpret_cast<int*>(NEAR ? Xh + (size_t)TP * 2 * (Mq + 1) : Xh);  // [TP] t, [TP] src
  int* srcs = tgt + TP;

  const int tid = threadIdx.x;
  for (int i = tid; i < L; i += kThreads) cos_tab[i] = cospi(2.0 * i / L);
  for (int i = tid; i <= L / 2; i += kThreads) {
    double s = sinpi((double)i / L);
    s2_tab[i] = s * s;
  }
  // pairs of this tile
  if (tid < TP) {
    int t, src;
    bool ok;
    if (NEAR) {
      long long idx = (long long)P.near_lo + (long long)blockIdx.x * TP + tid;
      ok = idx < P.near_hi;
      int2 pr = ok ? P.near[idx] : make_int2(P.t0, 0);
      t = pr.x;
      src = pr.y;
    } else {
      t = P.t0 + blockIdx.y;
      src = blockIdx.x * TP + tid;
      ok = src < P.NS;
    }
    uint8_t cl = ok ? P.cls[(size_t)t * P.NS + src] : kZero;
    double rt = P.r[t], dr = 0.0, dz = 0.0;
    if (ok) {
      if (src < P.N) {
        dr = P.r[src] - rt;
        dz = P.z[src] - P.z[t];
      } else {
        const double* sp = P.sup + ((size_t)t * P.S + (src - P.N)) * kSupFields;
        dr = sp[kSupDr];
        dz = sp[kSupDz];
      }
    }
    geo[4 * tid + 0] = rt;
    geo[4 * tid + 1] = dr;
    geo[4 * tid + 2] = dz;
    // valid (compute) flag: far kernel computes class kFar, near kernel kNear;
    // 2 marks a kZero pair to be written as zeros by the far kernel.
    double flag = 0.0;
    if (ok) {
      if (NEAR) flag = (cl == kNear) ? 1.0 : 0.0;
      else flag = (cl == kFar) ? 1.0 : (cl == kZero ? 2.0 : 0.0);
    }
    geo[4 * tid + 3] = flag;
    tgt[tid] = t;
    srcs[tid] = src;
  }
  __syncthreads();
  if (!NEAR) {
    // skip tiles without work; write zeros for kZero pairs
    bool any = false;
    for (int p = 0; p < TP; ++p) any |= (geo[4 * p + 3] != 0.0);
    if (!any) return;
  }
  if (NEAR && tid < TP && geo[4 * tid + 3] == 1.0) {
    Pair g = make_pair(geo[4 * tid], geo[4 * tid + 1], geo[4 * tid + 2]);
    near_spectra(g, P, Xh + (size_t)tid * 2 * (Mq + 1), Xh + (size_t)tid * 2 * (Mq + 1) + (Mq + 1));
  }
  __syncthreads();

  // accumulator role
  const int q = tid / TP;      // 0 .. Q-1 (tid >= Q*TP: idle in accumulation)
  const int pp = tid % TP;
  const int par = q & 1;
  const int grp = q >> 1;
  const bool acc_active = q < Q;
  double acc[kSeq][MB];
#pragma unroll
  for (int k = 0; k < kSeq; ++k)
#pragma unroll
    for (int i = 0; i < MB; ++i) acc[k][i] = 0.0;

  const double k0 = P.k0;
  const cd k1 = mk(P.k1r, P.k1i);
  const int nchunks = (Lq + 1 + JC - 1) / JC;
  for (int ch = 0; ch < nchunks; ++ch) {
    // sampling: task = jj * TP + p
    for (int task = tid; task < JC * TP; task += kThreads) {
      int p = task % TP, jj = task / TP;
      int j = ch * JC + jj;
      double* eo = EO + ((size_t)jj * TP + p) * kEO;
      bool live = (j <= Lq) && (geo[4 * p + 3] == 1.0);
      if (!live) {
        for (int k = 0; k < 2 * kSeq; ++k) eo[k] = 0.0;
        continue;
      }
      Pair g = make_pair(geo[4 * p], geo[4 * p + 1], geo[4 * p + 2]);
      int jb = L / 2 - j;  // mirror index: phi_jb = pi - phi_j
      double X1a, X3a, X1b, X3b;
      if (NEAR) {
        const double* x1 = Xh + (size_t)p * 2 * (Mq + 1);
        const double* x3 = x1 + (Mq + 1);
        double e1 = x1[0], o1 = 0.0, e3 = x3[0], o3 = 0.0;
        for (int n = 1; n <= Mq; ++n) {
          double cs = 2.0 * cos_tab[(n * j) & (L - 1)];
          if (n & 1) {
            o1 = fma(x1[n], cs, o1);
            o3 = fma(x3[n], cs, o3);
          } else {
            e1 = fma(x1[n], cs, e1);
            e3 = fma(x3[n], cs, e3);
          }
        }
        const double i2pi = 0.15915494309189535;  // 1/(2 pi)
        X1a = (e1 + o1) * i2pi;
        X1b = (e1 - o1) * i2pi;
        X3a = (e3 + o3) * i2pi;
        X3b = (e3 - o3) * i2pi;
      } else {
        double ra = sqrt(g.d2 + 4.0 * g.rt * g.rs * s2_tab[j]);
        double rb = sqrt(g.d2 + 4.0 * g.rt * g.rs * s2_tab[jb]);
        X1a = 1.0 / ra;
        X3a = X1a * X1a * X1a;
        X1b = 1.0 / rb;
        X3b = X1b * X1b * X1b;
      }
      double fa[kSeq], fb[kSeq];
      sample<NEAR, K1C>(g, s2_tab[j], cos_tab[j], X1a, X3a, k0, k1, fa);
      if (j == Lq) {
#pragma unroll
        for (int k = 0; k < kSeq; ++k) {
          eo[k] = 2.0 * fa[k];
          eo[kSeq + k] = 0.0;
        }
      } else {
        sample<NEAR, K1C>(g, s2_tab[jb], cos_tab[jb], X1b, X3b, k0, k1, fb);
        double w = (j == 0) ? 1.0 : 2.0;
#pragma unroll
        for (int k = 0; k < kSeq; ++k) {
          eo[k] = w * (fa[k] + fb[k]);
          eo[kSeq + k] = w * (fa[k] - fb[k]);
        }
      }
    }
    __syncthreads();
    if (acc_active) {
      int jmax = min(JC, Lq + 1 - ch * JC);
      for (int jj = 0; jj < jmax; ++jj) {
        int j = ch * JC + jj;
        const double* v = EO + ((size_t)jj * TP + pp) * kEO + par * kSeq;
        double cs[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
          int m = par + 2 * (grp * MB + i);
          cs[i] = cos_tab[(m * j) & (L - 1)];
        }
#pragma unroll
        for (int k = 0; k < kSeq; ++k) {
          double vk = v[k];
#pragma unroll
          for (int i = 0; i < MB; ++i) acc[k][i] = fma(vk, cs[i], acc[k][i]);
        }
      }
    }
    __syncthreads();
  }

  if (!acc_active) return;
  double flag = geo[4 * pp + 3];
  if (flag == 0.0) return;
  const int t = tgt[pp], src = srcs[pp];
  const double scale = (flag == 1.0) ? 1.0 / (2.0 * L) : 0.0;  // (2pi/L)/(4pi)
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    int m = par + 2 * (grp * MB + i);
    if (m >= P.M2) continue;
#pragma unroll
    for (int ty = 0; ty < kTypes; ++ty) {
      size_t off = (((size_t)m * kTypes + ty) * P.nt + (t - P.t0)) * P.NS + src;
      P.out[off] = make_double2(acc[2 * ty][i] * scale, acc[2 * ty + 1][i] * scale);
    }
  }
}

template <bool NEAR, bool K1C, int MB>
hipError_t launch_one(const TabParams& P, hipStream_t s) {
  const int NM = P.M2;
  const int neven = (NM + 1) / 2;
  const int G = (neven + MB - 1) / MB;
  const int Q = 2 * G;
  const int Mq = P.Mq;
  auto lds_of = [&](int tp) {
    const int jc = kThreads / tp;
    return sizeof(double) * ((size_t)P.L + (P.L / 2 + 2) + 4 * tp + (size_t)jc * tp * kEO +
                             (NEAR ? (size_t)tp * 2 * (Mq + 1) : 0)) +
           sizeof(int) * 2 * tp;
  };
  // pairs per workgroup: all Q accumulator groups busy, LDS within 112 KB
  // (threads beyond TP * Q only sample)
  int TP = kThreads / Q;
  while (TP > 8 && lds_of(TP) > 112 * 1024) TP /= 2;
  const int JC = kThreads / TP;
  const size_t lds = lds_of(TP);
  if (lds > 112 * 1024) return hipErrorInvalidValue;
  dim3 grid;
  if (NEAR) {
    const int cnt = P.near_hi - P.near_lo;
    if (cnt <= 0) return hipSuccess;
    grid = dim3((cnt + TP - 1) / TP, 1, 1);
  } else {
    grid = dim3((P.NS + TP - 1) / TP, P.nt, 1);
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&tabulate_kernel<NEAR, K1C, MB>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tabulate_kernel<NEAR, K1C, MB>), grid, dim3(kThreads), lds, s, P, TP, JC, Q);
  return hipGetLastError();
}

template <bool K1C, int MB>
hipError_t launch_pair(const TabParams& P, hipStream_t s) {
  hipError_t e = launch_one<false, K1C, MB>(P, s);
  if (e != hipSuccess) return e;
  return launch_one<true, K1C, MB>(P, s);
}

}  // namespace

// Three modes per accumulating thread: with the file compiled without
// machine-level loop-invariant hoisting (which otherwise keeps the series and
// sincos constants live in registers across the chunk loop) the real-k1
// kernels fit 256 registers, two waves per SIMD.
hipError_t launch_tabulate(const TabParams& P, hipStream_t s) {
  if (P.k1i != 0.0) return launch_pair<true, 3>(P, s);
  return launch_pair<false, 3>(P, s);
}

}  // namespace msv
