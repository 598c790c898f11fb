// Device-side building blocks of the Tersoff kernels (gfx950, wave64).
//
//  * scalar types: double (FP64 path), float (mixed path), and Dual<B>, a
//    forward-mode dual number (value + one tangent) used by the adjoint;
//  * math on those types (exp, log, log1p, sqrt, sin, cos, reciprocal);
//  * the per-entry kernel parameter record derived from the 14-field table;
//  * wave-level reductions (the paper's in-register reductions, Section V-A)
//    and hardware FP64 atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __device__ __forceinline__

namespace ters {

constexpr int kWave = 64;
constexpr int kNField = 14;
enum Field {
  FM = 0, FGAMMA, FLAM3, FC, FD, FH, FN, FBETA, FLAM2, FB, FR, FDC, FLAM1, FA
};

// ---------------------------------------------------------------------------
// dual numbers
// ---------------------------------------------------------------------------
template <class B>
struct Dual {
  B v, d;
  Dual() = default;
  DEV Dual(B a) : v(a), d(B(0)) {}
  DEV Dual(B a, B b) : v(a), d(b) {}
};

template <class T> struct Base { using type = T; };
template <class B> struct Base<Dual<B>> { using type = B; };
template <class T> using base_t = typename Base<T>::type;
template <class T> struct IsDual { static constexpr bool value = false; };
template <class B> struct IsDual<Dual<B>> { static constexpr bool value = true; };

DEV double val(double a) { return a; }
DEV float val(float a) { return a; }
template <class B> DEV B val(const Dual<B> &a) { return a.v; }
DEV double tan_of(double) { return 0.0; }
DEV float tan_of(float) { return 0.0f; }
template <class B> DEV B tan_of(const Dual<B> &a) { return a.d; }

template <class B> DEV Dual<B> operator+(Dual<B> a, Dual<B> b) { return {a.v + b.v, a.d + b.d}; }
template <class B> DEV Dual<B> operator-(Dual<B> a, Dual<B> b) { return {a.v - b.v, a.d - b.d}; }
template <class B> DEV Dual<B> operator*(Dual<B> a, Dual<B> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class B> DEV Dual<B> operator-(Dual<B> a) { return {-a.v, -a.d}; }
template <class B> DEV Dual<B> operator+(Dual<B> a, B b) { return {a.v + b, a.d}; }
template <class B> DEV Dual<B> operator+(B b, Dual<B> a) { return {a.v + b, a.d}; }
template <class B> DEV Dual<B> operator-(Dual<B> a, B b) { return {a.v - b, a.d}; }
template <class B> DEV Dual<B> operator-(B b, Dual<B> a) { return {b - a.v, -a.d}; }
template <class B> DEV Dual<B> operator*(Dual<B> a, B b) { return {a.v * b, a.d * b}; }
template <class B> DEV Dual<B> operator*(B b, Dual<B> a) { return {a.v * b, a.d * b}; }
template <class B> DEV Dual<B> &operator+=(Dual<B> &a, Dual<B> b) { a.v += b.v; a.d += b.d; return a; }
template <class B> DEV Dual<B> &operator-=(Dual<B> &a, Dual<B> b) { a.v -= b.v; a.d -= b.d; return a; }

// reciprocal: FP64 uses IEEE division; FP32 refines the hardware reciprocal
// (1 ulp) by one Newton step, so that its error is a rounding error (below
// half an ulp but for a tiny fraction) with no systematic sign: the mixed
// path's energy sums millions of such values.  a must be finite and non-zero.
DEV double rcp(double a) { return 1.0 / a; }
DEV float rcp(float a) {
  const float r = __builtin_amdgcn_rcpf(a);
  return fmaf(r, fmaf(-a, r, 1.0f), r);
}
template <class B> DEV Dual<B> rcp(Dual<B> a) { B r = rcp(a.v); return {r, -a.d * r * r}; }
template <class B> DEV Dual<B> operator/(Dual<B> a, Dual<B> b) { return a * rcp(b); }
template <class B> DEV Dual<B> operator/(Dual<B> a, B b) { return {a.v / b, a.d / b}; }

// ---------------------------------------------------------------------------
// Elementary functions on the ranges the kernels need, written out from their
// series (host and device).  The general-purpose library versions carry
// range reductions and special cases these arguments never need: FP64 log
// and log1p and FP32 log1p cost about a hundred instructions each, sin and
// cos over a hundred with their large-argument reduction.
// ---------------------------------------------------------------------------
#define HDEV __host__ __device__ __forceinline__

// ln 2 split so that k * kLn2Hi is exact for |k| < 2^21 (Cody and Waite)
constexpr double kLn2Hi = 0.6931471803691238;
constexpr double kLn2Lo = 1.9082149292705877e-10;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kLog2e = 1.4426950408889634;
constexpr double kSqrtHalf = 0.7071067811865476;
constexpr double kSqrt2m1 = 0.41421356237309503;

// e^x (FP64): x = k ln 2 + f with |f| <= ln(2)/2, e^f from its Taylor series
// to f^13/13! (truncation below 5e-18 relative), then scaled by 2^k.
// Arguments beyond the FP64 range give 0 or infinity.
HDEV double exp_d(double x) {
  x = fmin(fmax(x, -746.0), 710.0);
  const double k = rint(x * kLog2e);
  double f = fma(-k, kLn2Hi, x);
  f = fma(-k, kLn2Lo, f);
  double p = 1.0 / 6227020800.0;       // 1/13!
  p = fma(p, f, 1.0 / 479001600.0);    // 1/12!
  p = fma(p, f, 1.0 / 39916800.0);
  p = fma(p, f, 1.0 / 3628800.0);
  p = fma(p, f, 1.0 / 362880.0);
  p = fma(p, f, 1.0 / 40320.0);
  p = fma(p, f, 1.0 / 5040.0);
  p = fma(p, f, 1.0 / 720.0);
  p = fma(p, f, 1.0 / 120.0);
  p = fma(p, f, 1.0 / 24.0);
  p = fma(p, f, 1.0 / 6.0);
  p = fma(p, f, 0.5);
  p = fma(p, f, 1.0);
  p = fma(p, f, 1.0);
  return ldexp(p, (int)k);
}

// 2 atanh(s) = ln((1 + s)/(1 - s)) for |s| <= 3 - 2 sqrt(2) (about 0.1716):
// 2 (s + s^3/3 + ... + s^21/21), truncation below 1e-18 relative (FP64);
// to s^9/9 in FP32 (below 3e-9 relative)
HDEV double two_atanh_d(double s) {
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = s + s;
  return fma(s2 * z, p, s2);
}
HDEV float two_atanh_f(float s) {
  const float z = s * s;
  float p = 1.0f / 9.0f;
  p = fmaf(p, z, 1.0f / 7.0f);
  p = fmaf(p, z, 1.0f / 5.0f);
  p = fmaf(p, z, 1.0f / 3.0f);
  const float s2 = s + s;
  return fmaf(s2 * z, p, s2);
}

// ln x (FP64) for finite x > 0 (normal): x = m 2^e with m in [1/sqrt(2), sqrt(2)),
// ln m = 2 atanh((m - 1)/(m + 1)), ln x = e ln 2 + ln m
HDEV double log_d(double x) {
  int e;
  double m = frexp(x, &e);  // [0.5, 1)
  if (m < kSqrtHalf) {
    m += m;
    e -= 1;
  }
  const double t = two_atanh_d((m - 1.0) / (m + 1.0));
  const double de = (double)e;
  return fma(de, kLn2Hi, fma(de, kLn2Lo, t));
}

// ln(1 + y) for 0 <= y <= 1 from y itself (1 + y is never rounded): below
// sqrt(2) - 1, 2 atanh(y / (2 + y)); above, ln 2 + 2 atanh((y - 1)/(y + 3))
HDEV double log1p01_d(double y) {
  const bool big = y > kSqrt2m1;
  const double num = big ? y - 1.0 : y;
  const double den = big ? y + 3.0 : y + 2.0;
  return (big ? kLn2 : 0.0) + two_atanh_d(num / den);
}

// sin w for 0 <= w <= pi/2 from its Taylor series: to w^21/21! in FP64
// (truncation below 2e-18), to w^13/13! in FP32 (below 7e-10)
HDEV double sin_q_d(double w) {
  const double z = w * w;
  double p = -1.0 / 51090942171709440000.0;  // -1/21!
  p = fma(p, z, 1.0 / 121645100408832000.0);  // 1/19!
  p = fma(p, z, -1.0 / 355687428096000.0);    // -1/17!
  p = fma(p, z, 1.0 / 1307674368000.0);       // 1/15!
  p = fma(p, z, -1.0 / 6227020800.0);         // -1/13!
  p = fma(p, z, 1.0 / 39916800.0);            // 1/11!
  p = fma(p, z, -1.0 / 362880.0);             // -1/9!
  p = fma(p, z, 1.0 / 5040.0);                // 1/7!
  p = fma(p, z, -1.0 / 120.0);                // -1/5!
  p = fma(p, z, 1.0 / 6.0);                   // 1/3!... with the sign below
  // p now holds 1/3! - z/5! + ...; sin w = w - w z p
  return fma(-w * z, p, w);
}
HDEV float sin_q_f(float w) {
  const float z = w * w;
  float p = -1.0f / 6227020800.0f;          // -1/13!
  p = fmaf(p, z, 1.0f / 39916800.0f);       // 1/11!
  p = fmaf(p, z, -1.0f / 362880.0f);        // -1/9!
  p = fmaf(p, z, 1.0f / 5040.0f);           // 1/7!
  p = fmaf(p, z, -1.0f / 120.0f);           // -1/5!
  p = fmaf(p, z, 1.0f / 6.0f);              // 1/3!
  return fmaf(-w * z, p, w);
}

DEV double t_exp(double a) { return exp_d(a); }
DEV float t_exp(float a) { return expf(a); }
DEV double t_log(double a) { return log_d(a); }
DEV float t_log(float a) { return logf(a); }
// ln(1 + y), 0 <= y <= 1
DEV double t_log1p01(double y) { return log1p01_d(y); }
DEV float t_log1p01(float y) {
  const bool big = y > (float)kSqrt2m1;
  const float num = big ? y - 1.0f : y;
  const float den = big ? y + 3.0f : y + 2.0f;
  return (big ? (float)kLn2 : 0.0f) + two_atanh_f(num * rcp(den));
}
DEV double t_sqrt(double a) { return sqrt(a); }
DEV float t_sqrt(float a) { return sqrtf(a); }
DEV double t_sin_q(double w) { return sin_q_d(w); }
DEV float t_sin_q(float w) { return sin_q_f(w); }

template <class B> DEV Dual<B> t_exp(Dual<B> a) { B e = t_exp(a.v); return {e, a.d * e}; }
template <class B> DEV Dual<B> t_log(Dual<B> a) { return {t_log(a.v), a.d * rcp(a.v)}; }
template <class B> DEV Dual<B> t_log1p01(Dual<B> a) { return {t_log1p01(a.v), a.d * rcp(B(1) + a.v)}; }
template <class B> DEV Dual<B> t_sqrt(Dual<B> a) { B s = t_sqrt(a.v); return {s, a.d * B(0.5) * rcp(s)}; }

// conversion of an FP64 value (with optional FP64 tangent) to the compute type
template <class T> struct Conv;
template <> struct Conv<double> { static DEV double from(double v, double) { return v; } };
template <> struct Conv<float> { static DEV float from(double v, double) { return (float)v; } };
template <class B> struct Conv<Dual<B>> {
  static DEV Dual<B> from(double v, double d) { return {(B)v, (B)d}; }
};

// widen to FP64 accumulators
template <class T> struct Acc { using type = double; };
template <class B> struct Acc<Dual<B>> { using type = Dual<double>; };
template <class T> using acc_t = typename Acc<T>::type;
DEV double widen(double a) { return a; }
DEV double widen(float a) { return (double)a; }
template <class B> DEV Dual<double> widen(Dual<B> a) { return {(double)a.v, (double)a.d}; }

// ---------------------------------------------------------------------------
// kernel parameter record (derived once per table entry on the host)
// ---------------------------------------------------------------------------
// Compensation of FP32-rounded constants.  A constant c kept as c_hi + c_lo
// (c_lo what rounding to FP32 dropped) enters a product as one FMA,
// c_hi * x + (c_lo * x), so that the correction is added to the exact product
// and survives the single rounding; added after the rounding of c_hi * x it
// would be lost whenever it is below half an ulp, always in the same
// direction, and every pair of a species pair would carry the same relative
// bias of up to 6e-8.  The FP64 path has no residuals (c_lo = 0) and takes
// the plain product.
DEV double fma_lo(double a, double x, double) { return a * x; }
DEV float fma_lo(float a, float x, float c) { return fmaf(a, x, c); }
template <class B> DEV Dual<B> fma_lo(B a, Dual<B> x, Dual<B> c) {
  return {fma_lo(a, x.v, c.v), a * x.d + c.d};
}
template <class T, class B> DEV T mul_lo(B hi, B lo, T x) { return fma_lo(hi, x, lo * x); }
// (x - lo)^2 for x = v - c_hi and a constant c = c_hi + c_lo: x^2 - 2 lo x in
// one FMA (FP64: lo = 0)
DEV double sq_lo(double x, double) { return x * x; }
DEV float sq_lo(float x, float lo) { return fmaf(x, x, x * (-2.0f * lo)); }
template <class B> DEV Dual<B> sq_lo(Dual<B> x, B lo) { return {sq_lo(x.v, lo), B(2) * x.v * x.d}; }
// x + lo for a residual lo (FP64: lo = 0, nothing added)
DEV double add_lo(double x, double) { return x; }
DEV float add_lo(float x, float lo) { return x + lo; }
template <class B> DEV Dual<B> add_lo(Dual<B> x, B lo) { return {add_lo(x.v, lo), x.d}; }

template <class B>
struct KParam {
  // cutoff of the distance this entry is used for: R +- D, pi/(2D), pi/(4D)
  B R, D, rcut, rin, pi2d, pi4d;
  // pair part (valid for entries [ti][tj][tj]); *_lo hold what rounding the
  // FP64 value to B dropped (0 for FP64), so FP32 exponentials stay unbiased
  B A, lam1, Bc, lam2, beta, n, inv2n;
  B A_lo, lam1_lo, B_lo, lam2_lo, R_lo, h_lo;
  // three-body part: gamma, c^2, d^2, h, gamma c^2, c^2/d^2, lambda3, c, d
  B gamma, c2, d2, h, gc2, c2d2, lam3, c, d;
  // further residuals of FP32 rounding (0 for FP64 and in the single mode):
  // n, 1/(2n), gamma, c^2/d^2, d^2, lambda3, pi/(2D), and ln(beta) - ln(beta_hi)
  B n_lo, inv2n_lo, gamma_lo, c2d2_lo, d2_lo, lam3_lo, pi2d_lo, lbeta_lo;
  int32_t m3;   // 1 when m == 3, 0 when m == 1
  int32_t pad;
};

// c * exp(-lam * r) with c = c_hi + c_lo and lam = lam_hi + lam_lo.  In FP32 the
// rounding of lam to single precision would shift every exponent by lam*r*eps
// (r ~ 2.4 A, lam*r ~ 8): a systematic bias of the pair energy.  The product
// lam*r is therefore formed exactly (fma residual plus the lo part) and the
// residual applied to first order.
// r = r_hi + r_lo likewise carries the FP64 distance into the FP32 path.
DEV double scaled_exp(double c, double, double lam, double, double r, double) {
  return c * exp(-lam * r);
}
DEV float scaled_exp(float c, float c_lo, float lam, float lam_lo, float r, float r_lo) {
  float p = lam * r;
  float corr = fmaf(lam, r, -p) + (lam_lo * r + lam * r_lo);
  float e = expf(-p);
  return fmaf(e, c, e * (c_lo - c * corr));  // e c exact, the correction added before rounding
}
// The same in FP64, for the mixed path's pair energy: c = c_hi + c_lo,
// lam = lam_hi + lam_lo and r = r_hi + r_lo (the FP32 distance and the
// residual of the FP64 one) widened exactly.  Each FP32 pair exponential
// carries ~0.6 ulp of rounding; in disordered cells, where the repulsive and
// attractive parts nearly cancel, that rounding would set the energy error,
// so the mixed path evaluates the two exponentials of a pair once in FP64
// (the forces use them rounded to FP32).
DEV double exp64(float c, float c_lo, float lam, float lam_lo, float r, float r_lo) {
  const double rr = (double)r + (double)r_lo;
  return ((double)c + (double)c_lo) * exp(-((double)lam + (double)lam_lo) * rr);
}

template <class B>
DEV Dual<B> scaled_exp(B c, B c_lo, B lam, B lam_lo, Dual<B> r, B r_lo) {
  B v = scaled_exp(c, c_lo, lam, lam_lo, r.v, r_lo);
  return {v, -(lam + lam_lo) * v * r.d};
}

// replace the value part of a scalar (keeps a dual number's tangent)
DEV void set_val(double &a, double v) { a = v; }
DEV void set_val(float &a, double v) { a = (float)v; }
template <class B> DEV void set_val(Dual<B> &a, double v) { a.v = (B)v; }

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------
DEV int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
DEV float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
DEV Dual<double> wave_sum(Dual<double> v) { return {wave_sum(v.v), wave_sum(v.d)}; }

// Workgroups of a launch are dealt to the GPU's eight XCDs in turn
// (workgroup b runs on XCD b mod 8), and each XCD has its own L2.  This
// bijection of [0, G) gives every XCD one contiguous range of logical block
// ids instead, so spatially close atoms (cell order) and the neighbour data
// they share stay in one L2.
DEV int xcd_block(int b, int G) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, q = G / kXcd, r = G % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// Sum in FP64, in slot order, of the force slots [s0, s1) (3 values each); the
// slots are fetched four at a time so that their loads are in flight together.
template <class S>
DEV void sum_slots(const S *__restrict__ fslot, int s0, int s1, double &fx, double &fy,
                   double &fz) {
  for (int s = s0; s < s1; s += 4) {
    S v[12];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = 3 * (int64_t)min(s + u, s1 - 1);
      v[3 * u] = fslot[q];
      v[3 * u + 1] = fslot[q + 1];
      v[3 * u + 2] = fslot[q + 2];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (s + u < s1) {
        fx += (double)v[3 * u];
        fy += (double)v[3 * u + 1];
        fz += (double)v[3 * u + 2];
      }
    }
  }
}

// Species of atom i, used as an index into the parameter table: a value
// outside [0, nt) (which the list build reports as an error) reads entry 0
// instead of memory outside the table.
DEV int species(const int32_t *__restrict__ type, int64_t i, int nt) {
  const int t = type[i];
  return (unsigned)t < (unsigned)nt ? t : 0;
}

// hardware FP64 atomic add to global memory (global_atomic_add_f64)
DEV void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

}  // namespace ters
