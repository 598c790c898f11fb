// Tersoff energy / forces / virial kernel (and its dual-number adjoint).
//
// One workgroup takes a run of atoms in cell order (spatially compact).  Inside
// the workgroup, work is spread over lanes at the level where it is dense
// (the paper's "filter" and "computational" split, Section IV-B):
//
//  1 filter   lanes over (atom, list slot): FP64 minimum-image distance and
//             the cutoff test; the in-cutoff neighbours of each atom are
//             compacted in list order with a wave ballot (Section IV-D: the
//             test uses, for each species pair, the largest cutoff in which
//             that pair can take part, so nothing that contributes is lost)
//  2 pairs    lanes over in-cutoff pairs (i, m): r, 1/r, f_C, f_C' staged in LDS
//  3 zeta     lane per pair (i, j): the first k loop of the paper's Algorithm 3
//             accumulates zeta_ij and dzeta/dx_j in registers and stores
//             dzeta/dx_k for up to k_max neighbours in LDS; then the pair term
//             V(i, j, zeta_ij), its forces and dV/dzeta
//  4 gather   lane per pair slot (i, m): collects, in a fixed order, the force
//             that all terms rooted at i exert on m (pair term, m as j, and m as
//             k: dV/dzeta_ij * dzeta_ijm/dx_m, read from LDS or recomputed
//             beyond k_max as in the fallback of Algorithm 3), adds the virial
//             d_im (x) f_im, and scatters f_im to atom m with one FP64 atomic
//             per component
//  5 own      lane per atom: the force on i is minus the sum of its f_im
//             (every term's forces sum to zero), per-atom energy
//
// Scalar type T: double (FP64 path), float (mixed path: FP32 arithmetic, FP64
// displacements and accumulators), Dual<double> / Dual<float> (adjoint: the
// same computation in forward-mode dual numbers along the direction f_bar,
// which yields the Hessian-vector product and the mixed parameter derivative).
#include "ters_device.h"
#include "ters_internal.h"
#include "ters_math.h"

#include <type_traits>

namespace ters {

namespace {

constexpr int kNMax = 32;  // most in-cutoff neighbours of one atom

template <class T, bool NT1, bool PG, int AMAX, int BS, int PCAP, int TCAP>
__global__ __launch_bounds__(BS) void k_force(FwdArgs a, int A) {
  using B = base_t<T>;
  using KP = KParam<B>;
  using AT = acc_t<T>;
  constexpr bool DUAL = IsDual<T>::value;
  constexpr int NTL = 27;  // parameter entries cached in LDS (ntypes <= 3)
  static_assert(AMAX <= kWave, "sub-chunk planning runs on one wave");
  static_assert(BS % kWave == 0, "whole waves");

  // s_atom: cell-order position (list row); s_aid: its atom (per-atom arrays)
  __shared__ int s_atom[AMAX], s_aid[AMAX], s_type[AMAX], s_lcnt[AMAX], s_cnt[AMAX], s_kmx[AMAX];
  __shared__ int s_pst[AMAX], s_tst[AMAX], s_conf[AMAX];
  __shared__ int s_stage[AMAX * kNMax];
  __shared__ unsigned char s_slot[AMAX * kNMax];  // list slot of each staged neighbour
  __shared__ int s_sub[AMAX + 1];
  __shared__ int s_nsub;
  __shared__ unsigned char s_pa[PCAP], s_pq[PCAP];
  __shared__ int s_j[PCAP], s_tj[PCAP];
  __shared__ T s_dx[PCAP], s_dy[PCAP], s_dz[PCAP], s_r[PCAP], s_ri[PCAP], s_fc[PCAP],
      s_dfc[PCAP], s_dzeta[PCAP];
  __shared__ B s_rlo[PCAP];  // FP64 distance minus its rounding to B (0 for FP64)
  __shared__ AT s_fx[PCAP], s_fy[PCAP], s_fz[PCAP];
  __shared__ double s_ev[PCAP];
  __shared__ T s_gkx[TCAP > 0 ? TCAP : 1], s_gky[TCAP > 0 ? TCAP : 1], s_gkz[TCAP > 0 ? TCAP : 1];
  __shared__ KP s_kp[NT1 ? 1 : NTL];
  __shared__ double s_g[PG && !NT1 ? NTL * kNField : 1];
  __shared__ double s_red[BS / kWave][8];

  const int tid = threadIdx.x;
  // molecular dynamics: the list kernels of this step have read the rebuild
  // flag; it is cleared here and set again by the drift of the next step
  if (a.clear_flag && blockIdx.x == 0 && tid == 0) *a.clear_flag = 0;
  const int lane = lane_id();
  const int nt = a.ntypes;
  const int64_t first = (int64_t)xcd_block(blockIdx.x, gridDim.x) * A;
  const int na = (int)min((int64_t)A, (int64_t)a.n - first);
  if (na <= 0) return;

  const KP *P;
  if (NT1) {
    P = (const KP *)a.kparam;
  } else if (nt * nt * nt <= NTL) {
    for (int e = tid; e < nt * nt * nt; e += BS) s_kp[e] = ((const KP *)a.kparam)[e];
    P = s_kp;
  } else {
    P = (const KP *)a.kparam;
  }
  // one species: the record is read once into registers (uniform, scalar
  // loads) instead of from memory in the inner loops
  KP kp0;
  if (NT1) kp0 = P[0];
  auto param = [&](int ti, int tj, int tk) -> const KP & {
    return NT1 ? kp0 : P[(ti * nt + tj) * nt + tk];
  };
  const double *filt2 = (const double *)a.filt2;

  double gacc[NT1 && PG ? kNField : 1];
  if (NT1 && PG) {
#pragma unroll
    for (int f = 0; f < kNField; ++f) gacc[f] = 0.0;
  }
  if (PG && !NT1)
    for (int e = tid; e < NTL * kNField; e += BS) s_g[e] = 0.0;
  const bool grad_in_lds = nt * nt * nt <= NTL;
  auto add_grad = [&](int ti, int tj, int tk, int field, double v) {
    if (NT1) {
      gacc[field] += v;  // field is a compile-time constant after unrolling
    } else if (grad_in_lds) {
      unsafeAtomicAdd(&s_g[((ti * nt + tj) * nt + tk) * kNField + field], v);
    } else {
      atomic_add(&a.pgrad[((ti * nt + tj) * nt + tk) * kNField + field], v);
    }
  };

  // ---- 0: atoms of this workgroup ----------------------------------------
  for (int at = tid; at < na; at += BS) {
    const int i = (int)(first + at);
    const int ia = a.order[i];
    s_atom[at] = i;
    s_aid[at] = ia;
    s_type[at] = NT1 ? 0 : species(a.type, ia, a.ntypes);
    s_lcnt[at] = min(a.count[i], a.cap);
    s_conf[at] = a.conf_of ? a.conf_of[ia] : 0;
  }
  __syncthreads();

  // ---- 1: filter and compact in-cutoff neighbours ---------------------------
  {
    const int cap = a.cap;  // power of two <= 64: an atom's slots never straddle a wave
    const int lsh = __ffs(cap) - 1;
    const uint64_t segbits = cap == 64 ? ~0ull : ((1ull << cap) - 1ull);
    const int total = na * cap;
    for (int base = 0; base < total; base += BS) {
      int t = base + tid;
      int at = t >> lsh;
      int s = t & (cap - 1);
      bool pass = false;
      int j = 0;
      if (at < na && s < s_lcnt[at]) {
        const int i = s_aid[at];
        j = a.list[(int64_t)s_atom[at] * cap + s];  // neighbour's atom
        const ConfDesc &cf = a.conf[s_conf[at]];
        double dx = a.x[3 * j] - a.x[3 * i];
        double dy = a.x[3 * j + 1] - a.x[3 * i + 1];
        double dz = a.x[3 * j + 2] - a.x[3 * i + 2];
        dx -= cf.box[0] * rint(dx * cf.inv_box[0]);
        dy -= cf.box[1] * rint(dy * cf.inv_box[1]);
        dz -= cf.box[2] * rint(dz * cf.inv_box[2]);
        double r2 = dx * dx + dy * dy + dz * dz;
        int tj = NT1 ? 0 : species(a.type, j, a.ntypes);
        pass = r2 < filt2[NT1 ? 0 : s_type[at] * nt + tj];
      }
      uint64_t m = __ballot(pass);
      int seg0 = lane & ~(cap - 1);
      uint64_t seg = segbits << seg0;
      uint64_t below = m & seg & ((1ull << lane) - 1ull);
      int pos = __popcll(below);
      if (pass) {
        if (pos < kNMax) {
          s_stage[at * kNMax + pos] = j;
          s_slot[at * kNMax + pos] = (unsigned char)s;
        } else {
          atomicOr(a.err, kErrTooManyInCutoff);
        }
      } else if (a.fslot && at < na && s < s_lcnt[at]) {
        const int r = a.rev[(int64_t)s_atom[at] * cap + s];
        if (r >= 0) {
          B *fs = (B *)a.fslot + 3 * (int64_t)r;  // slots hold the base type
          fs[0] = B(0);
          fs[1] = B(0);
          fs[2] = B(0);
        }
      }
      if (at < na && s == cap - 1) s_cnt[at] = min(__popcll(m & seg), kNMax);
    }
  }
  __syncthreads();

  // ---- 1b: split into sub-chunks whose pairs and stored triplets fit LDS ----
  if (tid < kWave) {
    int nA = tid < na ? s_cnt[tid] : 0;
    int km = 0;
    if (TCAP > 0 && nA > 1) {
      km = min(nA - 1, a.kmax);
      km = min(km, TCAP / nA);
    }
    int tA = nA * km;
    int pinc = nA, tinc = tA;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      int u1 = __shfl_up(pinc, o, kWave), u2 = __shfl_up(tinc, o, kWave);
      if (lane >= o) {
        pinc += u1;
        tinc += u2;
      }
    }
    int ptot = __shfl(pinc, kWave - 1, kWave), ttot = __shfl(tinc, kWave - 1, kWave);
    if (tid < na) s_kmx[tid] = km;
    if (ptot <= PCAP && ttot <= (TCAP > 0 ? TCAP : 0)) {
      if (tid < na) {
        s_pst[tid] = pinc - nA;
        s_tst[tid] = tinc - tA;
      }
      if (tid == 0) {
        s_nsub = 1;
        s_sub[0] = 0;
        s_sub[1] = na;
      }
    } else if (tid == 0) {
      int ns = 0, pp = 0, tt = 0;
      s_sub[0] = 0;
      for (int at = 0; at < na; ++at) {
        int n1 = s_cnt[at];
        int k1 = 0;
        if (TCAP > 0 && n1 > 1) k1 = min(min(n1 - 1, a.kmax), TCAP / n1);
        int t1 = n1 * k1;
        if (at > 0 && (pp + n1 > PCAP || tt + t1 > TCAP)) {
          s_sub[++ns] = at;
          pp = 0;
          tt = 0;
        }
        s_pst[at] = pp;
        s_tst[at] = tt;
        pp += n1;
        tt += t1;
      }
      s_sub[++ns] = na;
      s_nsub = ns;
    }
  }
  __syncthreads();

  double eacc = 0.0, wacc[6] = {0, 0, 0, 0, 0, 0};
  // batch: a workgroup whose atoms span two configurations attributes its
  // energy and virial per pair with atomics instead of one block sum
  const bool straddle = a.conf_of != nullptr && s_conf[0] != s_conf[na - 1];
  const uint32_t flags = a.flags;
  const bool want_f = DUAL ? (a.xgrad != nullptr) : ((flags & TERS_FORCES) && a.forces);
  const bool want_w = !DUAL && (flags & TERS_VIRIAL);
  const bool want_ea = !DUAL && (flags & TERS_PER_ATOM_E) && a.e_atom;
  // mixed path with a two-species table: the energy takes b from an FP64 sum
  // of the FP32 zeta terms, evaluated in FP64 (bond_value_d), when an energy
  // is asked for (disordered two-species cells cancel their repulsive and
  // attractive parts to a few per cent; single-species cells keep the FP32
  // bond order, as in the wavefront kernel)
  constexpr bool kE64 = std::is_same<T, float>::value && !NT1;
  const bool want_e = !DUAL && (a.partials != nullptr || want_ea);

  const int nsub = s_nsub;
  for (int sc = 0; sc < nsub; ++sc) {
    const int a0 = s_sub[sc], a1 = s_sub[sc + 1];
    const int np = s_pst[a1 - 1] + s_cnt[a1 - 1];

    // ---- 2: pair map and pair staging ---------------------------------------
    for (int at = a0 + tid; at < a1; at += BS) {
      int b = s_pst[at];
      for (int q = 0; q < s_cnt[at]; ++q) {
        s_pa[b + q] = (unsigned char)at;
        s_pq[b + q] = (unsigned char)q;
      }
    }
    __syncthreads();
    for (int p = tid; p < np; p += BS) {
      int at = s_pa[p], q = s_pq[p];
      int i = s_aid[at];
      int j = s_stage[at * kNMax + q];
      int ti = s_type[at];
      int tj = NT1 ? 0 : species(a.type, j, a.ntypes);
      const ConfDesc &cf = a.conf[s_conf[at]];
      double d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double dd = a.x[3 * j + c] - a.x[3 * i + c];
        d[c] = dd - cf.box[c] * rint(dd * cf.inv_box[c]);
      }
      T dT[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        dT[c] = Conv<T>::from(d[c], DUAL ? (a.fbar[3 * j + c] - a.fbar[3 * i + c]) : 0.0);
      const double r64 = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      T r = t_sqrt(dT[0] * dT[0] + dT[1] * dT[1] + dT[2] * dT[2]);
      set_val(r, r64);
      T fc, dfc;
      fcut64(param(ti, tj, tj), r, r64, fc, dfc);
      s_rlo[p] = (B)(r64 - (double)val(r));
      s_j[p] = j;
      s_tj[p] = tj;
      s_dx[p] = dT[0];
      s_dy[p] = dT[1];
      s_dz[p] = dT[2];
      s_r[p] = r;
      s_ri[p] = rcp(r);
      s_fc[p] = fc;
      s_dfc[p] = dfc;
    }
    __syncthreads();

    // ---- 3: zeta pass and pair term (lane per pair) ---------------------------
    for (int p = tid; p < np; p += BS) {
      const int at = s_pa[p], q = s_pq[p];
      const int nA = s_cnt[at], base = s_pst[at], kmx = s_kmx[at];
      const int tb = s_tst[at] + q * kmx;
      const int ti = s_type[at], tj = s_tj[p];
      const KP &pp = param(ti, tj, tj);
      const T rij = s_r[p];
      AT f0 = Zero<AT>::get(), f1 = Zero<AT>::get(), f2 = Zero<AT>::get();
      T dzeta = Zero<T>::get();
      double ev = 0.0;
      if (val(rij) < pp.rcut) {
        const T rinv = s_ri[p];
        const T u[3] = {s_dx[p] * rinv, s_dy[p] * rinv, s_dz[p] * rinv};
        T zeta = Zero<T>::get();
        double zeta64 = 0.0;  // kE64: the same terms summed in FP64
        T gj[3] = {Zero<T>::get(), Zero<T>::get(), Zero<T>::get()};
        int kk = 0;
        for (int kq = 0; kq < nA; ++kq) {
          if (kq == q) continue;
          const int kp = base + kq;
          const KP &pk = param(ti, tj, s_tj[kp]);
          const T rik = s_r[kp];
          if (val(rik) < pk.rcut) {
            T fck, dfck;
            if (a.cut_consistent) {
              fck = s_fc[kp];
              dfck = s_dfc[kp];
            } else {
              fcut(pk, rik, fck, dfck);
            }
            const T rki = s_ri[kp];
            const T v[3] = {s_dx[kp] * rki, s_dy[kp] * rki, s_dz[kp] * rki};
            T gjt[3], gkt[3];
            T z = zeta_term<T, B, false>(pk, rij, rinv, u, rik, rki, v, fck, dfck, gjt, gkt, nullptr);
            zeta += z;
            if constexpr (kE64) zeta64 += (double)z;
            gj[0] += gjt[0];
            gj[1] += gjt[1];
            gj[2] += gjt[2];
            if (TCAP > 0 && kk < kmx) {
              s_gkx[tb + kk] = gkt[0];
              s_gky[tb + kk] = gkt[1];
              s_gkz[tb + kk] = gkt[2];
            }
          }
          ++kk;
        }
        // pair term V(i, j, zeta_ij)
        const B rlo = s_rlo[p];
        T fr, fa;
        AT fre, fae;  // the same for the energy
        if constexpr (std::is_same<T, float>::value) {  // mixed: FP64 exponentials
          const double e1 = exp64(pp.A, pp.A_lo, pp.lam1, pp.lam1_lo, rij, rlo);
          const double e2 = exp64(pp.Bc, pp.B_lo, pp.lam2, pp.lam2_lo, rij, rlo);
          fr = (float)e1;
          fa = -(float)e2;
          fre = e1;
          fae = -e2;
        } else {
          fr = scaled_exp(pp.A, pp.A_lo, pp.lam1, pp.lam1_lo, rij, rlo);
          fa = -scaled_exp(pp.Bc, pp.B_lo, pp.lam2, pp.lam2_lo, rij, rlo);
          fre = widen(fr);
          fae = widen(fa);
        }
        T b, db, dbb, dbn;
        bond<T, B, PG>(pp, zeta, b, db, dbb, dbn);
        const T fcij = s_fc[p], dfcij = s_dfc[p];
        const T vr = fr + b * fa;
        // the energy itself is assembled in FP64 from the factors (the FP32
        // path's large repulsive and attractive parts cancel at close contacts)
        AT bE = widen(b);
        if constexpr (kE64) {
          if (want_e) bE = bond_value_d(pp, zeta64);
        }
        const AT V = widen(fcij) * (fre + bE * fae);
        const T dVdr = dfcij * vr + fcij * (-pp.lam1 * fr - pp.lam2 * b * fa);
        dzeta = B(0.5) * fcij * fa * db;
        const T hp = B(0.5) * dVdr;
        f0 = widen(-(hp * u[0]) - dzeta * gj[0]);
        f1 = widen(-(hp * u[1]) - dzeta * gj[1]);
        f2 = widen(-(hp * u[2]) - dzeta * gj[2]);
        ev = 0.5 * val(V);
        if (!DUAL && straddle && a.partials) atomic_add(&a.partials[(int64_t)s_conf[at] * 8], ev);
        else eacc += ev;
        if (PG) {
          const double eb = DUAL ? (a.ebar_conf ? a.ebar_conf[s_conf[at]] : a.ebar) : 1.0;
          const T h = T(B(0.5)) * fcij;
          T dp[8];
          dp[0] = h * fr * (B(1) / pp.A);
          dp[1] = -h * rij * fr;
          dp[2] = h * b * fa * (B(1) / pp.Bc);
          dp[3] = -h * b * rij * fa;
          dp[4] = h * fa * dbb;
          dp[5] = h * fa * dbn;
          dp[6] = -B(0.5) * dfcij * vr;
          dp[7] = -B(0.5) * dfcij * (rij - pp.R) * (B(1) / pp.D) * vr;
#pragma unroll
          for (int f = 0; f < 8; ++f) add_grad(ti, tj, tj, GradSlots::pair[f], out_of(widen(dp[f]), eb));
        }
      }
      s_dzeta[p] = dzeta;
      s_fx[p] = f0;
      s_fy[p] = f1;
      s_fz[p] = f2;
      s_ev[p] = ev;
    }
    __syncthreads();

    // ---- 4: gather f_im for every pair slot, virial, scatter to m ------------
    for (int p = tid; p < np; p += BS) {
      const int at = s_pa[p], m = s_pq[p];
      const int nA = s_cnt[at], base = s_pst[at], kmx = s_kmx[at];
      const int ti = s_type[at], tm = s_tj[p];
      AT f[3] = {s_fx[p], s_fy[p], s_fz[p]};
      const T rim = s_r[p];
      const T rmi = s_ri[p];
      const T v[3] = {s_dx[p] * rmi, s_dy[p] * rmi, s_dz[p] * rmi};
      const double eb = DUAL ? (a.ebar_conf ? a.ebar_conf[s_conf[at]] : a.ebar) : 1.0;
      for (int jq = 0; jq < nA; ++jq) {
        if (jq == m) continue;
        const int jp = base + jq;
        const T dzj = s_dzeta[jp];
        if (val(dzj) == B(0)) continue;
        const int tj = s_tj[jp];
        const KP &pk = param(ti, tj, tm);
        if (val(rim) >= pk.rcut) continue;
        const int kk = m < jq ? m : m - 1;
        T gk[3];
        if (TCAP > 0 && kk < kmx) {
          const int idx = s_tst[at] + jq * kmx + kk;
          gk[0] = s_gkx[idx];
          gk[1] = s_gky[idx];
          gk[2] = s_gkz[idx];
        } else {
          T fck, dfck;
          if (a.cut_consistent) {
            fck = s_fc[p];
            dfck = s_dfc[p];
          } else {
            fcut(pk, rim, fck, dfck);
          }
          const T rij = s_r[jp], rji = s_ri[jp];
          const T u[3] = {s_dx[jp] * rji, s_dy[jp] * rji, s_dz[jp] * rji};
          T gj[3], dp[8];
          zeta_term<T, B, PG>(pk, rij, rji, u, rim, rmi, v, fck, dfck, gj, gk, dp);
          if (PG) {
#pragma unroll
            for (int fl = 0; fl < 8; ++fl)
              add_grad(ti, tj, tm, GradSlots::three[fl], out_of(widen(dzj * dp[fl]), eb));
          }
        }
        f[0] -= widen(dzj * gk[0]);
        f[1] -= widen(dzj * gk[1]);
        f[2] -= widen(dzj * gk[2]);
      }
      if (want_w) {
        const double dx = val(widen(s_dx[p])), dy = val(widen(s_dy[p])), dz = val(widen(s_dz[p]));
        const double fx = val(f[0]), fy = val(f[1]), fz = val(f[2]);
        const double wv[6] = {dx * fx, dy * fy, dz * fz, dx * fy, dx * fz, dy * fz};
        if (straddle) {
          if (a.partials)
            for (int k = 0; k < 6; ++k) atomic_add(&a.partials[(int64_t)s_conf[at] * 8 + 1 + k], wv[k]);
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k) wacc[k] += wv[k];
        }
      }
      if (want_f) {
        const int j = s_j[p];
        const double o0 = DUAL ? -out_of(f[0], eb) : val(f[0]);
        const double o1 = DUAL ? -out_of(f[1], eb) : val(f[1]);
        const double o2 = DUAL ? -out_of(f[2], eb) : val(f[2]);
        if (!DUAL && a.fslot) {
          // i's own force below sums the slot values as stored, so that the
          // forces of every term cancel exactly in the gathered total
          set_val(f[0], (double)(B)o0);
          set_val(f[1], (double)(B)o1);
          set_val(f[2], (double)(B)o2);
        }
        if (a.fslot) {
          const int r = a.rev[(int64_t)s_atom[at] * a.cap + s_slot[at * kNMax + m]];
          if (r >= 0) {
            B *fs = (B *)a.fslot + 3 * (int64_t)r;
            fs[0] = (B)o0;
            fs[1] = (B)o1;
            fs[2] = (B)o2;
          }
        } else {
          double *dst = DUAL ? a.xgrad : a.forces;
          atomic_add(&dst[3 * (int64_t)j + 0], o0);
          atomic_add(&dst[3 * (int64_t)j + 1], o1);
          atomic_add(&dst[3 * (int64_t)j + 2], o2);
        }
      }
      s_fx[p] = f[0];
      s_fy[p] = f[1];
      s_fz[p] = f[2];
    }
    __syncthreads();

    // ---- 5: own force of each atom, per-atom energy --------------------------
    for (int at = a0 + tid; at < a1; at += BS) {
      const int b = s_pst[at], nA = s_cnt[at];
      AT fx = Zero<AT>::get(), fy = Zero<AT>::get(), fz = Zero<AT>::get();
      double e = 0.0;
      for (int q = 0; q < nA; ++q) {
        fx -= s_fx[b + q];
        fy -= s_fy[b + q];
        fz -= s_fz[b + q];
        e += s_ev[b + q];
      }
      const int i = s_aid[at];
      if (want_f) {
        const double eb = DUAL ? (a.ebar_conf ? a.ebar_conf[s_conf[at]] : a.ebar) : 1.0;
        const double o0 = DUAL ? -out_of(fx, eb) : val(fx);
        const double o1 = DUAL ? -out_of(fy, eb) : val(fy);
        const double o2 = DUAL ? -out_of(fz, eb) : val(fz);
        if (a.fown) {  // indexed by atom
          double *fo = a.fown + 3 * (int64_t)i;
          fo[0] = o0;
          fo[1] = o1;
          fo[2] = o2;
        } else {
          double *dst = DUAL ? a.xgrad : a.forces;
          atomic_add(&dst[3 * (int64_t)i + 0], o0);
          atomic_add(&dst[3 * (int64_t)i + 1], o1);
          atomic_add(&dst[3 * (int64_t)i + 2], o2);
        }
      }
      if (want_ea) {
        if (flags & TERS_ACCUMULATE) a.e_atom[i] += e;
        else a.e_atom[i] = e;
      }
    }
    __syncthreads();
  }

  // ---- block reductions ------------------------------------------------------
  const int w = tid / kWave;
  if (!DUAL && a.partials) {
    double vals[7] = {eacc, wacc[0], wacc[1], wacc[2], wacc[3], wacc[4], wacc[5]};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      double s = wave_sum(vals[k]);
      if (lane == 0) s_red[w][k] = s;
    }
    __syncthreads();
    if (tid < 7) {
      double s = 0.0;
      for (int q = 0; q < BS / kWave; ++q) s += s_red[q][tid];
      if (a.conf_of) {
        // batch: per-configuration energy / virial; a workgroup whose atoms
        // span configurations falls back to per-atom attribution below
        if (!straddle) atomic_add(&a.partials[(int64_t)s_conf[0] * 8 + tid], s);
      } else {
        a.partials[(int64_t)blockIdx.x * 8 + tid] = s;
      }
    }
  }
  if (PG) {
    if (NT1) {
#pragma unroll
      for (int f = 0; f < kNField; ++f) {
        double s = wave_sum(gacc[f]);
        if (lane == 0) atomic_add(&a.pgrad[f], s);
      }
    } else if (grad_in_lds) {
      __syncthreads();
      for (int e = tid; e < nt * nt * nt * kNField; e += BS)
        if (s_g[e] != 0.0) atomic_add(&a.pgrad[e], s_g[e]);
    }
  }
}

// Fixed-order sum of the per-workgroup partials.  With a trace, the energy is
// also stored at trace[*step] and the device step counter advanced (keeps a
// captured molecular-dynamics step replayable).
constexpr int kRedBS = 1024;
template <int NK>
__global__ __launch_bounds__(kRedBS) void k_reduce_partials(const double *partials, int nblocks,
                                                            int stride, double *energy,
                                                            double *virial, int accumulate,
                                                            double *trace, int32_t *step) {
  // one workgroup; thread t sums records t, t + 1024, ... (contiguous across
  // the threads, fetched CH at a time so that the loads overlap), then a fixed
  // tree over the workgroup: the order of the sum is fixed
  constexpr int CH = NK == 1 ? 16 : 4;
  __shared__ double red[kRedBS / kWave][NK];
  double acc[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[k] = 0.0;
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += CH * kRedBS) {
    double v[CH][NK];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int b = b0 + c * kRedBS;
#pragma unroll
      for (int k = 0; k < NK; ++k) v[c][k] = b < nblocks ? partials[(int64_t)b * stride + k] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int k = 0; k < NK; ++k) acc[k] += v[c][k];
  }
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane_id() == 0) red[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < NK) {
    const int k = threadIdx.x;
    double tot = 0.0;
    for (int q = 0; q < kRedBS / kWave; ++q) tot += red[q][k];
    double *dst = k == 0 ? energy : virial + (k - 1);
    if (dst) *dst = accumulate ? *dst + tot : tot;
    if (k == 0 && trace) {
      trace[*step] = tot;
      *step += 1;
    }
  }
}

// schedule constants per scalar type
template <class T> struct Sched;
template <> struct Sched<double> { static constexpr int AMAX = 64, BS = 256, PCAP = 256, TCAP = 512; };
template <> struct Sched<float> { static constexpr int AMAX = 64, BS = 256, PCAP = 256, TCAP = 1024; };
template <> struct Sched<Dual<double>> { static constexpr int AMAX = 32, BS = 128, PCAP = 160, TCAP = 0; };
template <> struct Sched<Dual<float>> { static constexpr int AMAX = 32, BS = 128, PCAP = 160, TCAP = 0; };

template <class T, bool PG>
void launch_t(const FwdArgs &a, int A, hipStream_t s) {
  using S = Sched<T>;
  if (A <= 0 || A > S::AMAX) A = S::AMAX;
  int nb = (a.n + A - 1) / A;
  if (nb == 0) return;
  if (a.ntypes == 1)
    k_force<T, true, PG, S::AMAX, S::BS, S::PCAP, S::TCAP><<<nb, S::BS, 0, s>>>(a, A);
  else
    k_force<T, false, PG, S::AMAX, S::BS, S::PCAP, S::TCAP><<<nb, S::BS, 0, s>>>(a, A);
}

}  // namespace

int forward_blocks(int n, int A) { return (n + A - 1) / A; }

void launch_forward(const FwdArgs &a, int precision, int A, int nblocks_out[1], hipStream_t s) {
  const bool pg = (a.flags & TERS_PARAM_GRAD) && a.pgrad;
  if (precision == TERS_FP64) {
    if (A <= 0 || A > Sched<double>::AMAX) A = Sched<double>::AMAX;
    if (pg) launch_t<double, true>(a, A, s);
    else launch_t<double, false>(a, A, s);
  } else {
    if (A <= 0 || A > Sched<float>::AMAX) A = Sched<float>::AMAX;
    if (pg) launch_t<float, true>(a, A, s);
    else launch_t<float, false>(a, A, s);
  }
  nblocks_out[0] = forward_blocks(a.n, A);
}

void launch_adjoint(const FwdArgs &a, int precision, int A, hipStream_t s) {
  if (precision == TERS_FP64) launch_t<Dual<double>, true>(a, A, s);
  else launch_t<Dual<float>, true>(a, A, s);
}

void launch_reduce_partials(const double *partials, int nblocks, int stride, double *energy,
                            double *virial, int accumulate, hipStream_t s, double *trace,
                            int32_t *step) {
  if (virial)
    k_reduce_partials<7><<<1, kRedBS, 0, s>>>(partials, nblocks, stride, energy, virial,
                                              accumulate, trace, step);
  else
    k_reduce_partials<1><<<1, kRedBS, 0, s>>>(partials, nblocks, stride, energy, virial,
                                              accumulate, trace, step);
}

}  // namespace ters
