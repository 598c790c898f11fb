// The Tersoff functions on the scalar types of the kernels (double, float,
// dual numbers): cutoff switch, bond order, the three-body term and its
// gradients, and the parameter partials used by the adjoint.
//
//   f_C(r)      = 1 below R-D, 0 above R+D, 1/2 - 1/2 sin(pi (r-R) / (2D)) between
//   b(zeta)     = (1 + (beta zeta)^n)^(-1/(2n))
//   zeta(i,j,k) = f_C(r_ik) g(cos theta_ijk) exp(lambda3^m (r_ij - r_ik)^m)
//   g(cos)      = gamma (1 + c^2 t^2 / (d^2 (d^2 + t^2))),  t = cos - h
// (the paper, Section III, Eqs. ters-2 and ters-3, with Tersoff's forms).
#pragma once
#include "ters_device.h"

namespace ters {

template <class T> struct Zero { static DEV T get() { return T(base_t<T>(0)); } };

// The switch between R - D and R + D, written with w = pi (R + D - r) / (4D)
// and v = pi (r - R + D) / (4D) (w + v = pi/2, both in [0, pi/2]):
//   f_C = 1/2 - 1/2 sin(pi (r - R) / (2D)) = sin^2 w,
//   f_C' = -pi/(4D) cos(pi (r - R) / (2D)) = -pi/(2D) sin w sin v,
// each sine taken near its own zero, so f_C keeps its relative accuracy up
// to R + D and f_C' up to R - D.  arg = pi (r - R) / (2D) is given.
template <class B> DEV void switch_of(B arg, B pi4d, B &fc, B &dfc) {
  const B q = B(0.78539816339744831);  // pi/4
  const B sw = t_sin_q(q - B(0.5) * arg), sv = t_sin_q(q + B(0.5) * arg);
  fc = sw * sw;
  dfc = -B(2) * pi4d * (sw * sv);
}
template <class B> DEV void switch_of(Dual<B> arg, B pi4d, Dual<B> &fc, Dual<B> &dfc) {
  B f, df;
  switch_of(arg.v, pi4d, f, df);
  // d f_C / d arg = -1/2 cos(arg) = df / (2 pi4d); d f_C' / d arg = pi4d sin(arg)
  const B q = B(0.78539816339744831);
  const B sw = t_sin_q(q - B(0.5) * arg.v), sv = t_sin_q(q + B(0.5) * arg.v);
  fc = {f, arg.d * df * (B(0.5) / pi4d)};
  dfc = {df, arg.d * pi4d * (sv * sv - sw * sw)};
}

// f_C and f_C' (sine switch from 1 at R-D to 0 at R+D)
template <class T, class B>
DEV void fcut(const KParam<B> &p, T r, T &fc, T &dfc) {
  B rv = val(r);
  if (rv <= p.rin) {
    fc = T(B(1));
    dfc = T(B(0));
  } else if (rv >= p.rcut) {
    fc = T(B(0));
    dfc = T(B(0));
  } else {
    T arg = mul_lo(p.pi2d, p.pi2d_lo, (r - p.R) - p.R_lo);
    switch_of(arg, p.pi4d, fc, dfc);
  }
}

// the same, with the FP64 distance at hand: the switch argument is formed in
// FP64 before rounding (keeps the FP32 path unbiased in the transition region)
template <class T, class B>
DEV void fcut64(const KParam<B> &p, T r, double r64, T &fc, T &dfc) {
  B rv = val(r);
  if (rv <= p.rin) {
    fc = T(B(1));
    dfc = T(B(0));
  } else if (rv >= p.rcut) {
    fc = T(B(0));
    dfc = T(B(0));
  } else {
    T arg = r * p.pi2d;  // tangent part
    set_val(arg, (r64 - (double)p.R - (double)p.R_lo) * ((double)p.pi2d + (double)p.pi2d_lo));
    switch_of(arg, p.pi4d, fc, dfc);
  }
}

// b(zeta) = (1 + (beta zeta)^n)^(-1/(2n)) and db/dzeta, in a form that cannot
// overflow: with s = n ln(beta zeta), ln(1 + e^s) = s + ln(1 + e^-s) for s > 0.
// Also d b / d beta and d b / d n for the parameter gradient.
template <class T, class B, bool PG>
DEV void bond(const KParam<B> &p, T z, T &b, T &db, T &dbeta, T &dn) {
  if (val(z) <= B(0)) {
    b = T(B(1));
    db = T(B(0));
    dbeta = T(B(0));
    dn = T(B(0));
    return;
  }
  // s = n ln(beta zeta), with the residuals of n and beta entering in one FMA
  T lz = t_log(p.beta * z);
  T s = fma_lo(p.n, lz, p.n * p.lbeta_lo + p.n_lo * lz);
  // y = e^s: with e = e^-|s| (in (0, 1]), ln(1 + y) = max(s, 0) + ln(1 + e) and
  // y / (1 + y) = (s > 0 ? 1 : e) / (1 + e); one path for every lane
  const bool pos = val(s) > B(0);
  const T em = t_exp(pos ? -s : s);
  const T l1p = (pos ? s : Zero<T>::get()) + t_log1p01(em);
  const T ri = rcp(B(1) + em);
  const T w = pos ? ri : em * ri;  // ln(1 + y), y / (1 + y)
  b = t_exp(-mul_lo(p.inv2n, p.inv2n_lo, l1p));
  T bw = b * w;
  db = -B(0.5) * bw * rcp(z);
  if (PG) {
    dbeta = -B(0.5) * bw * rcp(T(p.beta));
    dn = b * p.inv2n * (l1p * rcp(T(p.n)) - w * add_lo(lz, p.lbeta_lo));
  } else {
    dbeta = T(B(0));
    dn = T(B(0));
  }
}

// b(zeta) in FP64 from the FP32 parameter record's hi/lo pairs, for the
// energy of the mixed path: the FP32 evaluation above (a logarithm and two
// exponentials of FP32 arguments, then a power) errs by a few parts in 1e7
// of b, and in disordered cells the attractive and repulsive parts of the
// energy are each about ten times the energy itself, so that error would
// reach the energy at 1e-7 per atom; zeta is then the FP64 sum of the same
// FP32 terms.  Same steps as bond(): s = n ln(beta zeta), ln(1 + e^s) =
// max(s, 0) + ln(1 + e^-|s|), b = e^(-ln(1 + e^s)/(2n)).
DEV double bond_value_d(const KParam<float> &p, double z) {
  if (z <= 0.0) return 1.0;
  const double lz = log_d((double)p.beta * z) + (double)p.lbeta_lo;
  const double s = ((double)p.n + (double)p.n_lo) * lz;
  const double em = exp_d(-fabs(s));
  const double l1p = fmax(s, 0.0) + log1p01_d(em);
  return exp_d(-((double)p.inv2n + (double)p.inv2n_lo) * l1p);
}

// zeta(i,j,k) alone (the first K loop of Algorithm 2 needs only the value).
template <class T, class B>
DEV T zeta_value(const KParam<B> &p, T rij, const T *u, T rik, const T *v, T fck) {
  T cs = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
  T t2 = sq_lo(cs - p.h, p.h_lo);  // (cos - h)^2
  T q = t2 * rcp(add_lo(t2, p.d2_lo) + p.d2);
  T g = mul_lo(p.gamma, p.gamma_lo, B(1) + mul_lo(p.c2d2, p.c2d2_lo, q));
  if (p.lam3 == B(0)) return fck * g;
  T uu = mul_lo(p.lam3, p.lam3_lo, rij - rik);
  T arg = p.m3 ? uu * uu * uu : uu;
  return fck * g * t_exp(arg);
}

// zeta(i,j,k) = f_C(r_ik) g(cos) exp(lambda3^m (r_ij - r_ik)^m) and its
// gradients wrt x_j and x_k (the one wrt x_i is minus their sum).  With PG,
// also the partials wrt gamma, c, d, h, lambda3, m, R, D of this entry.
template <class T, class B, bool PG>
DEV T zeta_term(const KParam<B> &p, T rij, T rinv_ij, const T *u, T rik, T rinv_ik, const T *v,
                T fck, T dfck, T *gj, T *gk, T *dpar) {
  T cs = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
  T x = cs - p.h;
  T t = x - p.h_lo;     // cos - h
  T t2 = sq_lo(x, p.h_lo);
  T iden = rcp(add_lo(t2, p.d2_lo) + p.d2);
  T gn = B(1) + mul_lo(p.c2d2, p.c2d2_lo, t2 * iden);  // g / gamma
  T g = mul_lo(p.gamma, p.gamma_lo, gn);
  T dg = B(2) * p.gc2 * t * iden * iden;
  T e, de;  // exponential factor and its derivative wrt dr = r_ij - r_ik
  T dr = rij - rik;
  T uu = mul_lo(p.lam3, p.lam3_lo, dr);
  T arg;
  if (p.lam3 == B(0)) {  // exponential factor is exactly 1 (e.g. the Si/C sets)
    e = T(B(1));
    de = T(B(0));
    arg = T(B(0));
  } else if (p.m3) {
    arg = uu * uu * uu;
    e = t_exp(arg);
    de = B(3) * p.lam3 * uu * uu * e;
  } else {
    arg = uu;
    e = t_exp(arg);
    de = p.lam3 * e;
  }
  T fge = fck * g;
  T z = fge * e;
  T s1 = fck * dg * e;
  T s2 = fge * de;
  T s3 = dfck * g * e;
  T s32 = s3 - s2;
  // with d cos / d x_j = (v - cos u) / r_ij and d cos / d x_k = (u - cos v) / r_ik:
  //   gj = s1 (v - cos u) / r_ij + s2 u = a1 v + b1 u,
  //   gk = s1 (u - cos v) / r_ik + s32 v = a2 u + b2 v
  const T a1 = s1 * rinv_ij, a2 = s1 * rinv_ik;
  const T b1 = s2 - a1 * cs, b2 = s32 - a2 * cs;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gj[c] = a1 * v[c] + b1 * u[c];
    gk[c] = a2 * u[c] + b2 * v[c];
  }
  if (PG) {
    T fe = fck * e;
    T ge = g * e;
    dpar[0] = fe * gn;                                            // gamma
    dpar[1] = fe * (B(2) * p.gamma * p.c * t2 * iden / p.d2);     // c
    dpar[2] = fe * (B(2) * p.gc2 * (p.d * iden * iden - B(1) / (p.d2 * p.d)));  // d
    dpar[3] = -fe * dg;                                           // h
    if (p.m3) dpar[4] = fge * e * (B(3) * uu * uu * dr);          // lambda3
    else dpar[4] = fge * e * dr;
    B au = val(uu) < B(0) ? -val(uu) : val(uu);
    if (p.lam3 == B(0) || au == B(0)) {
      dpar[5] = T(B(0));                                          // m
    } else {
      T lu = val(uu) < B(0) ? t_log(-uu) : t_log(uu);
      dpar[5] = fge * e * arg * lu;
    }
    dpar[6] = -ge * dfck;                                         // R (of r_ik)
    dpar[7] = -ge * dfck * (rik - p.R) * (B(1) / p.D);            // D (of r_ik)
  }
  return z;
}

// ---------------------------------------------------------------------------
// output combination: forward writes values; the adjoint writes
// e_bar * value - tangent (parameter gradient) and its negative (x gradient)
// ---------------------------------------------------------------------------
DEV double out_of(double c, double) { return c; }
DEV double out_of(const Dual<double> &c, double ebar) { return ebar * c.v - c.d; }


struct GradSlots {  // field index of each parameter partial
  static constexpr int three[8] = {FGAMMA, FC, FD, FH, FLAM3, FM, FR, FDC};
  static constexpr int pair[8] = {FA, FLAM1, FB, FLAM2, FBETA, FN, FR, FDC};
};

}  // namespace ters
