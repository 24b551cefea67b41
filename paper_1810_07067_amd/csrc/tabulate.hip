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
// Work decomposition: a 256-thread workgroup owns TP = max(1, 256 / (L/2))
// pairs and keeps all L/2 + 1 azimuth samples of their nine integrands in LDS.
// Near pairs first synthesize their band-limited 1/rho, 1/rho^3 from the
// spectra with one real-even FFT; then every pair's samples are transformed
// with nine real-even FFTs (see the transform section below) and modes
// m = 0..M+1 go to HBM, consecutive threads writing consecutive sources.
#include <hip/hip_runtime.h>

#include "msv_internal.h"

namespace msv {
namespace {

constexpr int kSeq = 2 * kTypes;  // 18 real sequences
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

// LDS position of element i of a transform sequence: one element of padding
// per 32 spreads the bit-reversed stores of the transforms (indices that
// differ only in their high bits) over distinct banks.
__device__ __forceinline__ int lpos(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int seq_stride(int N) { return N + 1 + ((N + 1) >> 5) + 1; }

// Spectra X1_n, X3_n (n = 0..Mq) of 1/rho and 1/rho^3 for one near pair:
// xs(n) = (X1_n, X3_n) for n <= Mq, xs(Mq + 1) = 0 (xs(n) returns a reference).
template <class At>
__device__ void near_spectra(const Pair& g, const TabParams& P, At xs) {
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
    xs(0) = make_double2(c1 * Q, c3 * tail);
    for (int n = 1; n <= Mq; ++n) {
      Q = Q + D;
      double num = D + eta * Q;
      xs(n) = make_double2(c1 * Q, c3 * (1.0 - 2.0 * n) * num);
      D = ((n - 0.5) * D + 2.0 * n * eta * Q) / (n + 0.5);
    }
  } else {
    // Miller's backward recurrence from n_start, normalized by Q_{-1/2}; the
    // raw values are kept in the .x slots until the normalization is known.
    int ns = P.fwd_n + (int)ceil(P.miller_extra / acs);
    if (ns < Mq + 2) ns = Mq + 2;
    double fhi = 0.0, f = 1.0;
    for (int n = ns; n >= 1; --n) {
      double flo = (2.0 * n * chi * f - (n + 0.5) * fhi) / (n - 0.5);
      fhi = f;
      f = flo;
      if (n - 1 <= Mq) xs(n - 1).x = f;
      if (fabs(f) > 1e250) {
        fhi *= 1e-250;
        f *= 1e-250;
        for (int i = n - 1; i <= Mq; ++i) xs(i).x *= 1e-250;
      }
    }
    double sc = q0 / xs(0).x;
    // num_n = chi Q_n - Q_{n-1}; go downward so Q_{n-1} is still raw
    for (int n = Mq; n >= 1; --n) {
      double Qn = xs(n).x * sc, Qm = xs(n - 1).x * sc;
      xs(n).y = c3 * (1.0 - 2.0 * n) * (chi * Qn - Qm);
    }
    xs(0).y = c3 * tail;
    for (int n = 0; n <= Mq; ++n) xs(n).x = c1 * (xs(n).x * sc);
  }
  xs(Mq + 1) = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Real-even transforms (the discrete convolution of eq. discA).
//
// Every sequence here is even with period L = 2N, so only x_0 .. x_N are held,
// and its length-L DFT is the type-I cosine transform
//   F_m = x_0 + (-1)^m x_N + 2 sum_{j=1}^{N-1} x_j cos(pi m j / N),  m = 0..N.
// With u_j = x_j + x_{N-j}, v_j = x_j - x_{N-j} and y_j = u_j - 2 sin(pi j/N) v_j
// (j = 0..N-1, x_{N-0} = x_N) and Y = FFT_N(y):
//   F_{2k}   = (Y_k + Y_{N-k}) / 2,
//   F_{2k+1} = F_{2k-1} + i (Y_k - Y_{N-k}) / 2,   F_1 = sum_j cos(pi j/N) v_j,
// for complex x as well (the real and imaginary parts are two real even
// sequences and every step is linear with real coefficients), so one complex
// FFT of length N transforms the real and imaginary parts of one kernel type.
// The odd outputs come from a running sum started at F_1, so each carries an
// absolute error of a few ulps of |F_1|: harmless for the modal coefficients,
// but the band-limited 1/rho, 1/rho^3 of a near-singular pair fall by many
// orders of magnitude from phi = 0 to pi.  Those are therefore synthesized
// from their spectra with a complex FFT of the full length 2N of the even
// extension, which needs no running sum (the two real spectra share it).
// All of it runs on the workgroup's LDS; the FFT is an in-place radix-2
// decimation in time on bit-reversed input, two stages per pass through LDS.
// ---------------------------------------------------------------------------
struct Seqs {
  double2* base;  // sequence s at base + s * stride, element i at lpos(i)
  int stride;
  int nseq;
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// pre-pass: y in bit-reversed order, F_1 per sequence into f1[s].  One wave
// per sequence; every lane loads before any lane stores.
constexpr int kMaxR = 5;  // (N/2 + 1) / 64 rounded up, N <= 512
__device__ void dct_pre(const Seqs& q, int logN, const double2* cs, double2* f1, int wave, int lane, int nwaves) {
  const int N = 1 << logN, H = N / 2;
  for (int s = wave; s < q.nseq; s += nwaves) {
    double2* x = q.base + (size_t)s * q.stride;
    double2 xa[kMaxR], xb[kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int j = lane + 64 * r;
      const int jc = j <= H ? j : H;  // lanes past N/2 load a valid element and drop it
      xa[r] = x[lpos(jc)];
      xb[r] = x[lpos(N - jc)];
      if (j > H) xa[r] = xb[r] = make_double2(0, 0);
    }
    double2 acc = make_double2(0, 0);
    double2 ya[kMaxR], yb[kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int j = lane + 64 * r;
      const double2 u = cadd(xa[r], xb[r]), v = csub(xa[r], xb[r]);
      const double c = (j <= H) ? cs[j].x : 0.0, sn = (j <= H) ? cs[j].y : 0.0;
      // F_1 = v_0 + 2 sum_{0<j<N/2} cos(pi j/N) v_j (the pairs j, N-j)
      const double wgt = (j == 0) ? 1.0 : (j < H ? 2.0 * c : 0.0);
      acc = make_double2(fma(wgt, v.x, acc.x), fma(wgt, v.y, acc.y));
      ya[r] = make_double2(fma(-2.0 * sn, v.x, u.x), fma(-2.0 * sn, v.y, u.y));
      yb[r] = make_double2(fma(2.0 * sn, v.x, u.x), fma(2.0 * sn, v.y, u.y));
    }
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int j = lane + 64 * r;
      if (j > H) continue;
      const unsigned rj = __brev((unsigned)j) >> (32 - logN);
      x[lpos((int)rj)] = ya[r];
      if (j != 0 && j != H) {
        const unsigned rk = __brev((unsigned)(N - j)) >> (32 - logN);
        x[lpos((int)rk)] = yb[r];
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
    }
    if (lane == 0) f1[s] = acc;
  }
}

// Twiddle idx of a table holding hq entries: entry hq + k is -i times entry
// k, which holds when the hq entries span a quarter turn (tables that span
// more are never indexed past hq).
__device__ __forceinline__ double2 twid(const double2* tw, int idx, int hq) {
  if (idx < hq) return tw[idx];
  const double2 w = tw[idx - hq];
  return make_double2(w.y, -w.x);
}

// in-place FFT of length N = 2^logN of every sequence (bit-reversed input,
// natural output); twiddle ts * k = e^{-2 pi i k / N}, k < N/2, from a table
// of hq entries (twid).  Ends with a barrier.
__device__ void dct_fft(const Seqs& q, int logN, const double2* tw, int ts, int hq, int tid, int nthreads) {
  const int N = 1 << logN;
  int h = 1, lh = 0;
  for (; 4 * h <= N; h *= 4, lh += 2) {
    const int lG = logN - 2;  // N/4 butterfly groups per sequence
    const int total = q.nseq << lG;
    for (int g = tid; g < total; g += nthreads) {
      const int s = g >> lG, r = g & ((1 << lG) - 1);
      const int p = r & (h - 1), b = r >> lh;
      double2* x = q.base + (size_t)s * q.stride;
      const int i0 = b * 4 * h + p;
      double2 a0 = x[lpos(i0)], a1 = x[lpos(i0 + h)], a2 = x[lpos(i0 + 2 * h)], a3 = x[lpos(i0 + 3 * h)];
      const double2 w1 = twid(tw, ts * p * (N / (2 * h)), hq);
      double2 t = cmul(w1, a1);
      a1 = csub(a0, t);
      a0 = cadd(a0, t);
      t = cmul(w1, a3);
      a3 = csub(a2, t);
      a2 = cadd(a2, t);
      const double2 w2 = twid(tw, ts * p * (N / (4 * h)), hq), w3 = twid(tw, ts * (p + h) * (N / (4 * h)), hq);
      t = cmul(w2, a2);
      a2 = csub(a0, t);
      a0 = cadd(a0, t);
      t = cmul(w3, a3);
      a3 = csub(a1, t);
      a1 = cadd(a1, t);
      x[lpos(i0)] = a0;
      x[lpos(i0 + h)] = a1;
      x[lpos(i0 + 2 * h)] = a2;
      x[lpos(i0 + 3 * h)] = a3;
    }
    __syncthreads();
  }
  if (h < N) {  // one radix-2 stage left: half size h = N/2
    const int total = q.nseq << lh;
    for (int g = tid; g < total; g += nthreads) {
      const int s = g >> lh, p = g & (h - 1);
      double2* x = q.base + (size_t)s * q.stride;
      const double2 a0 = x[lpos(p)], t = cmul(twid(tw, ts * p, hq), x[lpos(p + h)]);
      x[lpos(p + h)] = csub(a0, t);
      x[lpos(p)] = cadd(a0, t);
    }
    __syncthreads();
  }
}

// post-pass: outputs F_m * scale for m < mout, in place at lpos(m).  One wave
// per sequence; each lane owns consecutive k and every lane loads before any
// lane stores.
__device__ void dct_post(const Seqs& q, int logN, int mout, double scale, const double2* f1, int wave, int lane,
                         int nwaves) {
  const int N = 1 << logN;
  const int kmax = (mout - 1) / 2;  // F_{2k} or F_{2k+1} below mout for k <= kmax
  const int R = (kmax + 64) / 64;   // <= kMaxR
  for (int s = wave; s < q.nseq; s += nwaves) {
    double2* x = q.base + (size_t)s * q.stride;
    double2 yk[kMaxR], yn[kMaxR];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int k = lane * R + r;
      const bool ok = r < R && k <= kmax;
      const int kc = ok ? k : 0;  // lanes without a k load element 0 and drop it
      yk[r] = x[lpos(kc)];
      yn[r] = x[lpos((N - kc) & (N - 1))];
      if (!ok) yk[r] = yn[r] = make_double2(0, 0);
    }
    // odd outputs: prefix sums of D_k = i (Y_k - Y_{N-k}) / 2, D_0 = 0
    double2 pre[kMaxR];
    double2 run = make_double2(0, 0);
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int k = lane * R + r;
      if (r < R && k >= 1) {
        run.x += -0.5 * (yk[r].y - yn[r].y);
        run.y += 0.5 * (yk[r].x - yn[r].x);
      }
      pre[r] = run;
    }
    // exclusive scan of the lane totals across the wave
    double2 inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double ux = __shfl_up(inc.x, o, 64), uy = __shfl_up(inc.y, o, 64);
      if (lane >= o) {
        inc.x += ux;
        inc.y += uy;
      }
    }
    const double2 base1 = cadd(f1[s], csub(inc, run));
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int k = lane * R + r;
      if (r >= R || k > kmax) continue;
      if (2 * k < mout) x[lpos(2 * k)] = cscale(0.5 * scale, cadd(yk[r], yn[r]));
      if (2 * k + 1 < mout) x[lpos(2 * k + 1)] = cscale(scale, cadd(base1, pre[r]));
    }
  }
}

constexpr int kThreads = 256;
constexpr int kMaxTask = 3;  // samples per thread: TP (N + 1) <= 3 * 256 for N <= 512

// The Legendre-Q spectra of near pairs near[near_lo .. near_hi), one thread
// per pair, into spec[idx - near_lo][n], n = 0..N (N = L/2; the recurrences are
// serial in n).  The exponent e that scales the 1/rho^3 spectrum to the size
// of the 1/rho one (their transform is shared; see below) is stored in place
// of the zero entry n = N.
// Entry n of pair i (counted from the chunk's first pair) in the spectra
// scratch: pairs in groups of 64, [i / 64][n][i % 64], so that the 64 pairs
// of a wave, one per thread, store and load each n as one contiguous 1 KB
// (with a pair's N + 1 entries kept together, every such instruction touched
// 64 lines).  A workgroup reading one pair's spectrum takes lines that the
// workgroups of its neighbouring pairs, resident on the same XCD, read too.
__device__ __forceinline__ size_t spec_at(long long i, int n, int N) {
  return ((size_t)(i >> 6) * (size_t)(N + 1) + (size_t)n) * 64 + (size_t)(i & 63);
}

__global__ __launch_bounds__(kThreads) void near_spectra_kernel(TabParams P) {
  const long long idx = (long long)P.near_lo + (long long)blockIdx.x * kThreads + threadIdx.x;
  if (idx >= P.near_hi) return;
  const int N = P.L / 2;
  const int2 pr = P.near[idx];
  const int t = pr.x, src = pr.y;
  const double rt = P.r[t];
  double dr, dz;
  if (src < P.N) {
    dr = P.r[src] - rt;
    dz = P.z[src] - P.z[t];
  } else {
    const double* sp = P.sup + ((size_t)t * P.S + (src - P.N)) * kSupFields;
    dr = sp[kSupDr];
    dz = sp[kSupDz];
  }
  const Pair g = make_pair(rt, dr, dz);
  double2* spec = P.spec;
  const long long i = idx - P.near_lo;
  near_spectra(g, P, [spec, i, N](int n) -> double2& { return spec[spec_at(i, n, N)]; });
  double m1 = 0.0, m3 = 0.0;
  for (int n = 0; n < N; ++n) {
    const double2 v = spec[spec_at(i, n, N)];
    m1 = fmax(m1, fabs(v.x));
    m3 = fmax(m3, fabs(v.y));
  }
  int e = 0;
  if (m1 > 0.0 && m3 > 0.0) e = ilogb(m1) - ilogb(m3);
  spec[spec_at(i, N, N)] = make_double2((double)e, 0.0);
}

// One workgroup = TP pairs (TP = max(1, 256 / N)), all L/2 + 1 = N + 1
// azimuth samples of their nine integrands resident in LDS.
template <bool NEAR, bool K1C>
__global__ __launch_bounds__(kThreads) void tabulate_kernel(TabParams P, int logTP, int logN, int n_items, int ntile) {
  const int TP = 1 << logTP;
  extern __shared__ double2 smem2[];
  const int N = 1 << logN, H = N / 2, L = 2 * N;
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD one
  // contiguous range of tiles, so neighbouring sources are written from one L2
  const int per = (n_items + 7) / 8;
  const int item = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (item >= n_items) return;
  const int stride = seq_stride(N), stride2 = seq_stride(2 * N);
  // Azimuth tables.  N/2 twiddles live in LDS: near workgroups hold the
  // quarter turn of e^{-2 pi i k / 2N} (the 2N-point synthesis, and every
  // second entry for the N-point transforms; twid derives the rest), far
  // ones the N/2 of e^{-2 pi i k / N}.  cs [N/2 + 1] = (cos, sin)(pi j / N)
  // and s2 [N + 1] = sin^2(pi j / 2N) are read from the plan's copy in global
  // memory (a few KB, cache-resident).  With the near pairs' band-limited
  // samples sharing the LDS of the sequences (below), four workgroups of
  // either kind fit a CU at L = 512.
  double2* tw = smem2;
  const double2* cs = P.tabs + N;
  const double* s2 = reinterpret_cast<const double*>(P.tabs + N + H + 1);
  double2* geo2 = tw + H;  // [TP][3]: (rt, dr), (dz, flag), (1/sigma, -)
  double2* f1 = geo2 + 3 * TP;         // [9 TP]
  double2* S = f1 + 10 * TP;           // [TP][9][stride]
  double2* XS = S;                     // NEAR: [TP][stride2], in the sequences' LDS until sampled
  int* tgt = reinterpret_cast<int*>(S + (size_t)TP * kTypes * stride);  // [TP] t, [TP] src
  int* srcs = tgt + TP;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kThreads / 64;
  for (int i = tid; i < H; i += kThreads) tw[i] = P.tabs[NEAR ? i : 2 * i];
  if (tid < TP) {
    int t, src;
    bool ok;
    if (NEAR) {
      const long long idx = (long long)P.near_lo + (long long)item * TP + tid;
      ok = idx < P.near_hi;
      const int2 pr = ok ? P.near[idx] : make_int2(P.t0, 0);
      t = pr.x;
      src = pr.y;
    } else {
      t = P.t0 + item / ntile;
      src = (item % ntile) * TP + tid;
      ok = src < P.NS;
    }
    const uint8_t cl = ok ? P.cls[(size_t)t * P.NS + src] : kZero;
    const double rt = P.r[t];
    double dr = 0.0, dz = 0.0;
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
    // flag 1: this kernel computes the pair; 2: a zero pair the far kernel
    // writes as zeros; 0: nothing to write here
    double flag = 0.0;
    if (ok) {
      if (NEAR) flag = (cl == kNear) ? 1.0 : 0.0;
      else flag = (cl == kFar) ? 1.0 : (cl == kZero ? 2.0 : 0.0);
    }
    geo2[3 * tid] = make_double2(rt, dr);
    geo2[3 * tid + 1] = make_double2(dz, flag);
    // near pairs: 1/(2 pi) for the synthesized 1/rho and 1/(2 pi sigma) for
    // 1/rho^3, sigma = 2^e the scaling applied before the shared transform
    double isig = 0.15915494309189535;
    if (NEAR && flag == 1.0) {
      const long long idx = (long long)P.near_lo + (long long)item * TP + tid;
      isig = ldexp(isig, -(int)P.spec[spec_at(idx - P.near_lo, N, N)].x);
    }
    geo2[3 * tid + 2] = make_double2(isig, 0.0);
    tgt[tid] = t;
    srcs[tid] = src;
  }
  __syncthreads();
  bool any = false;
  for (int p = 0; p < TP; ++p) any |= (geo2[3 * p + 1].y != 0.0);
  if (!any) return;  // uniform: every thread read the same flags

  if (NEAR) {
    // band-limited 1/rho, 1/rho^3 at every azimuth sample: the cosine series
    // of their Legendre-Q spectra (scratch, written by near_spectra_kernel),
    // one transform of the even extension of length 2N per pair.  The two
    // spectra share it; next to a source the 1/rho^3 spectrum is 1e9 or more
    // times the 1/rho one, and its rounding would swamp the latter, so it
    // enters scaled to the same size by a power of two (exact).
    for (int e = tid; e < (TP << (logN + 1)); e += kThreads) {
      const int p = e >> (logN + 1), j = e & (2 * N - 1);
      const int n = j <= N ? j : 2 * N - j;
      const long long i = (long long)item * TP + p;
      double2 v = make_double2(0.0, 0.0);
      if (n < N && geo2[3 * p + 1].y == 1.0) {
        v = P.spec[spec_at(i, n, N)];
        v.y = ldexp(v.y, (int)P.spec[spec_at(i, N, N)].x);
      }
      const unsigned rj = __brev((unsigned)j) >> (31 - logN);
      XS[(size_t)p * stride2 + lpos((int)rj)] = v;
    }
    __syncthreads();
    dct_fft(Seqs{XS, stride2, TP}, logN + 1, tw, 1, H, tid, kThreads);
  }

  // samples: one thread per (pair, azimuth j = 0..N); phi_j and pi - phi_j
  // share the tables (cos(pi - phi) = -cos phi)
  const double k0 = P.k0;
  const cd k1 = mk(P.k1r, P.k1i);
  const int ntask = TP * (N + 1);  // at most kMaxTask per thread
  // near pairs: every thread takes its band-limited samples into registers
  // before any integrand is written over them
  double xn1[kMaxTask], xn3[kMaxTask];
  if constexpr (NEAR) {
#pragma unroll
    for (int r = 0; r < kMaxTask; ++r) {
      const int task = tid + r * kThreads;
      xn1[r] = xn3[r] = 0.0;
      if (task < ntask) {
        const int p = task / (N + 1), j = task - p * (N + 1);
        const double2 xl = XS[(size_t)p * stride2 + lpos(j)];
        xn1[r] = xl.x * 0.15915494309189535;  // 1/(2 pi)
        xn3[r] = xl.y * geo2[3 * p + 2].x;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < kMaxTask; ++r) {
    const int task = tid + r * kThreads;
    if (task >= ntask) continue;
    const int p = task / (N + 1), j = task - p * (N + 1);
    if (geo2[3 * p + 1].y != 1.0) continue;
    const Pair g = make_pair(geo2[3 * p].x, geo2[3 * p].y, geo2[3 * p + 1].x);
    double X1, X3;
    if (NEAR) {
      X1 = xn1[r];
      X3 = xn3[r];
    } else {
      const double rho = sqrt(g.d2 + 4.0 * g.rt * g.rs * s2[j]);
      X1 = 1.0 / rho;
      X3 = X1 * X1 * X1;
    }
    const double cphi = j <= H ? cs[j].x : -cs[N - j].x;
    double f[kSeq];
    sample<NEAR, K1C>(g, s2[j], cphi, X1, X3, k0, k1, f);
    double2* seq = S + (size_t)p * kTypes * stride;
#pragma unroll
    for (int ty = 0; ty < kTypes; ++ty) seq[ty * stride + lpos(j)] = make_double2(f[2 * ty], f[2 * ty + 1]);
  }
  __syncthreads();
  const Seqs qs{S, stride, kTypes * TP};
  dct_pre(qs, logN, cs, f1, wave, lane, nwaves);
  __syncthreads();
  dct_fft(qs, logN, tw, NEAR ? 2 : 1, H, tid, kThreads);
  const double scale = 1.0 / (2.0 * L);  // (2 pi / L) / (4 pi)
  dct_post(qs, logN, P.M2, scale, f1, wave, lane, nwaves);
  __syncthreads();
  // out[m][type][t][src]: consecutive threads take consecutive pairs
  const int nout = P.M2 * kTypes * TP;
  for (int e = tid; e < nout; e += kThreads) {
    const int p = e & (TP - 1), rest = e >> logTP;
    const int ty = rest % kTypes, m = rest / kTypes;
    const double flag = geo2[3 * p + 1].y;
    if (flag == 0.0) continue;
    const double2 v = (flag == 1.0) ? S[((size_t)p * kTypes + ty) * stride + lpos(m)] : make_double2(0.0, 0.0);
    P.out[(((size_t)m * kTypes + ty) * P.nt + (tgt[p] - P.t0)) * P.NS + srcs[p]] = v;
  }
}

template <bool NEAR, bool K1C>
hipError_t launch_one(const TabParams& P, hipStream_t s) {
  const int N = P.L / 2;
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  if ((1 << logN) != N || N < 4 || N > 512) return hipErrorInvalidValue;
  if (P.M2 > N + 1) return hipErrorInvalidValue;
  const int TP = N >= 256 ? 1 : 256 / N;
  int logTP = 0;
  while ((1 << logTP) < TP) ++logTP;
  const int stride = seq_stride(N);
  // the near samples [TP][stride2] share the sequences' [TP][9][stride]
  if (seq_stride(2 * N) > kTypes * stride || TP * (N + 1) > kMaxTask * kThreads) return hipErrorInvalidValue;
  const size_t lds = sizeof(double2) * ((size_t)N / 2 + 3 * TP + 10 * TP + (size_t)TP * kTypes * stride) +
                     sizeof(int) * 2 * TP;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&tabulate_kernel<NEAR, K1C>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (!NEAR) {
    const int ntile = (P.NS + TP - 1) / TP;
    const long long items = (long long)ntile * P.nt;
    // a dispatch counts work-items in 32 bits
    if ((items + 7) / 8 * 8 * kThreads >= (1LL << 32)) return hipErrorInvalidValue;
    const int n_items = (int)items;
    hipLaunchKernelGGL((tabulate_kernel<NEAR, K1C>), dim3(8 * ((n_items + 7) / 8)), dim3(kThreads), lds, s, P,
                       logTP, logN, n_items, ntile);
    return hipGetLastError();
  }
  // near pairs in chunks that the spectra scratch holds (a multiple of TP)
  if (P.near_hi <= P.near_lo) return hipSuccess;
  if (!P.spec || P.spec_cap < TP) return hipErrorInvalidValue;
  const int chunk = P.spec_cap / TP * TP;
  for (int c0 = P.near_lo; c0 < P.near_hi; c0 += chunk) {
    TabParams Q = P;
    Q.near_lo = c0;
    Q.near_hi = c0 + chunk < P.near_hi ? c0 + chunk : P.near_hi;
    const int cnt = Q.near_hi - Q.near_lo;
    hipLaunchKernelGGL(near_spectra_kernel, dim3((cnt + kThreads - 1) / kThreads), dim3(kThreads), 0, s, Q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int n_items = (cnt + TP - 1) / TP;
    hipLaunchKernelGGL((tabulate_kernel<NEAR, K1C>), dim3(8 * ((n_items + 7) / 8)), dim3(kThreads), lds, s, Q,
                       logTP, logN, n_items, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool K1C>
hipError_t launch_pair(const TabParams& P, hipStream_t s) {
  hipError_t e = launch_one<false, K1C>(P, s);
  if (e != hipSuccess) return e;
  return launch_one<true, K1C>(P, s);
}

}  // namespace

hipError_t launch_tabulate(const TabParams& P, hipStream_t s) {
  if (P.k1i != 0.0) return launch_pair<true>(P, s);
  return launch_pair<false>(P, s);
}

}  // namespace msv
