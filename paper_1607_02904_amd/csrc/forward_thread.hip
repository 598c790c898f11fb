// Tersoff force kernel, thread-per-atom schedule: the paper's mapping scheme
// (c) of Section IV-B (atoms over threads, neighbours j and k walked one after
// the other by the thread), as its GPU back end runs it.  Kept as a baseline
// for the measurements of the other two schedules.
//
// Thread t takes the atom at cell-order position t and walks its list row:
// entries outside the largest cutoff are skipped (the filter, in line), for
// each in-cutoff j the first K loop sums zeta_ij, the pair term gives dV/dzeta
// and the second K loop evaluates dzeta(i,j,k)/dx (Algorithm 2, nothing
// stored between the loops).  Forces on j and k go out by FP64 atomic adds,
// the force on i as one atomic add of minus their sum at the end; there is no
// owner-gather form of this schedule.  Precision handling follows the other
// schedules (FP64, or FP32 arithmetic with FP64 displacements, distances and
// accumulators).
#include "ters_device.h"
#include "ters_internal.h"
#include "ters_math.h"

#include <type_traits>

namespace ters {

namespace {

constexpr int kTBS = 256;

template <class T, bool NT1>
__global__ __launch_bounds__(kTBS) void k_force_thread(FwdArgs a) {
  using B = base_t<T>;
  using KP = KParam<B>;
  using AT = acc_t<T>;
  const int nt = a.ntypes;
  const KP *P = (const KP *)a.kparam;
  auto param = [&](int ti, int tj, int tk) -> const KP & {
    return P[NT1 ? 0 : (ti * nt + tj) * nt + tk];
  };
  const double *filt2 = (const double *)a.filt2;
  const uint32_t flags = a.flags;
  const bool want_f = (flags & TERS_FORCES) && a.forces;
  const bool want_w = (flags & TERS_VIRIAL) != 0;
  const bool want_ea = (flags & TERS_PER_ATOM_E) && a.e_atom;
  // mixed path with a two-species table: the energy takes b from an FP64 sum
  // of the FP32 zeta terms, evaluated in FP64 (bond_value_d), when an energy
  // is asked for (disordered two-species cells cancel their repulsive and
  // attractive parts to a few per cent; single-species cells keep the FP32
  // bond order, as in the wavefront kernel)
  constexpr bool kE64 = std::is_same<T, float>::value && !NT1;
  const bool want_e = a.partials != nullptr || want_ea;

  double eacc = 0.0, wacc[6] = {0, 0, 0, 0, 0, 0};
  const int t = blockIdx.x * kTBS + threadIdx.x;
  if (t < a.n) {
    const int i = a.order[t];
    const int ti = NT1 ? 0 : species(a.type, i, a.ntypes);
    const int cf = a.conf_of ? a.conf_of[i] : 0;
    const ConfDesc &c = a.conf[cf];
    const int cnt = min(a.count[t], a.cap);
    const int32_t *row = a.list + (int64_t)t * a.cap;
    double xi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) xi[k] = a.x[3 * (int64_t)i + k];

    // displacement to neighbour j (minimum image, FP64), its rounding to T,
    // distance, switch; false when j is outside the filter radius
    struct Nb {
      T d[3], r, ri, fc, dfc;
      B rlo;
      double d64[3];
    };
    auto neighbour = [&](int j, int tj, const KP &pc, Nb &o) -> bool {
      double d[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double dd = a.x[3 * (int64_t)j + k] - xi[k];
        d[k] = dd - c.box[k] * rint(dd * c.inv_box[k]);
      }
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (!(r2 < filt2[NT1 ? 0 : ti * nt + tj])) return false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        o.d64[k] = d[k];
        o.d[k] = Conv<T>::from(d[k], 0.0);
      }
      const double r64 = sqrt(r2);
      o.r = t_sqrt(o.d[0] * o.d[0] + o.d[1] * o.d[1] + o.d[2] * o.d[2]);
      set_val(o.r, r64);
      o.ri = rcp(o.r);
      fcut64(pc, o.r, r64, o.fc, o.dfc);
      o.rlo = (B)(r64 - (double)val(o.r));
      return true;
    };

    AT fi[3] = {AT(0), AT(0), AT(0)};
    double ei = 0.0;
    for (int s = 0; s < cnt; ++s) {
      const int j = row[s];
      const int tj = NT1 ? 0 : species(a.type, j, a.ntypes);
      const KP &pp = param(ti, tj, tj);
      Nb nj;
      if (!neighbour(j, tj, pp, nj)) continue;
      if (!(val(nj.r) < pp.rcut)) continue;
      const T u[3] = {nj.d[0] * nj.ri, nj.d[1] * nj.ri, nj.d[2] * nj.ri};

      // first K loop: zeta_ij
      T zeta = T(B(0));
      double zeta64 = 0.0;  // kE64: the same terms summed in FP64
      for (int s2 = 0; s2 < cnt; ++s2) {
        if (s2 == s) continue;
        const int k = row[s2];
        const int tk = NT1 ? 0 : species(a.type, k, a.ntypes);
        Nb nk;
        if (!neighbour(k, tk, param(ti, tk, tk), nk)) continue;
        const KP &pk = param(ti, tj, tk);
        if (!(val(nk.r) < pk.rcut)) continue;
        T fck = nk.fc, dfck = nk.dfc;
        if (!a.cut_consistent) fcut(pk, nk.r, fck, dfck);
        const T v[3] = {nk.d[0] * nk.ri, nk.d[1] * nk.ri, nk.d[2] * nk.ri};
        const T zt = zeta_value<T, B>(pk, nj.r, u, nk.r, v, fck);
        zeta += zt;
        if constexpr (kE64) zeta64 += (double)zt;
      }

      // pair term
      T fr, fa;
      AT fre, fae;  // the same for the energy
      if constexpr (std::is_same<T, float>::value) {  // mixed: FP64 exponentials
        const double e1 = exp64(pp.A, pp.A_lo, pp.lam1, pp.lam1_lo, nj.r, nj.rlo);
        const double e2 = exp64(pp.Bc, pp.B_lo, pp.lam2, pp.lam2_lo, nj.r, nj.rlo);
        fr = (float)e1;
        fa = -(float)e2;
        fre = e1;
        fae = -e2;
      } else {
        fr = scaled_exp(pp.A, pp.A_lo, pp.lam1, pp.lam1_lo, nj.r, nj.rlo);
        fa = -scaled_exp(pp.Bc, pp.B_lo, pp.lam2, pp.lam2_lo, nj.r, nj.rlo);
        fre = widen(fr);
        fae = widen(fa);
      }
      T b, db, dbb, dbn;
      bond<T, B, false>(pp, zeta, b, db, dbb, dbn);
      const T vr = fr + b * fa;
      AT bE = widen(b);
      if constexpr (kE64) {
        if (want_e) bE = bond_value_d(pp, zeta64);
      }
      const AT V = widen(nj.fc) * (fre + bE * fae);
      const T dVdr = nj.dfc * vr + nj.fc * (-pp.lam1 * fr - pp.lam2 * b * fa);
      const T dzeta = B(0.5) * nj.fc * fa * db;
      const T hp = B(0.5) * dVdr;
      ei += 0.5 * val(V);
      AT fj[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) fj[q] = widen(-(hp * u[q]));

      // second K loop: dzeta/dx_j and dzeta/dx_k
      for (int s2 = 0; s2 < cnt && val(dzeta) != B(0); ++s2) {
        if (s2 == s) continue;
        const int k = row[s2];
        const int tk = NT1 ? 0 : species(a.type, k, a.ntypes);
        Nb nk;
        if (!neighbour(k, tk, param(ti, tk, tk), nk)) continue;
        const KP &pk = param(ti, tj, tk);
        if (!(val(nk.r) < pk.rcut)) continue;
        T fck = nk.fc, dfck = nk.dfc;
        if (!a.cut_consistent) fcut(pk, nk.r, fck, dfck);
        const T v[3] = {nk.d[0] * nk.ri, nk.d[1] * nk.ri, nk.d[2] * nk.ri};
        T gj[3], gk[3], dp[8];
        zeta_term<T, B, false>(pk, nj.r, nj.ri, u, nk.r, nk.ri, v, fck, dfck, gj, gk, dp);
        AT fk[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          fj[q] -= widen(dzeta * gj[q]);
          fk[q] = widen(-(dzeta * gk[q]));
          fi[q] -= fk[q];
        }
        if (want_f)
#pragma unroll
          for (int q = 0; q < 3; ++q) atomic_add(&a.forces[3 * (int64_t)k + q], val(fk[q]));
        if (want_w) {
          const double fx = val(fk[0]), fy = val(fk[1]), fz = val(fk[2]);
          wacc[0] += nk.d64[0] * fx;
          wacc[1] += nk.d64[1] * fy;
          wacc[2] += nk.d64[2] * fz;
          wacc[3] += nk.d64[0] * fy;
          wacc[4] += nk.d64[0] * fz;
          wacc[5] += nk.d64[1] * fz;
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) fi[q] -= fj[q];
      if (want_f)
#pragma unroll
        for (int q = 0; q < 3; ++q) atomic_add(&a.forces[3 * (int64_t)j + q], val(fj[q]));
      if (want_w) {
        const double fx = val(fj[0]), fy = val(fj[1]), fz = val(fj[2]);
        wacc[0] += nj.d64[0] * fx;
        wacc[1] += nj.d64[1] * fy;
        wacc[2] += nj.d64[2] * fz;
        wacc[3] += nj.d64[0] * fy;
        wacc[4] += nj.d64[0] * fz;
        wacc[5] += nj.d64[1] * fz;
      }
    }
    if (want_f)
#pragma unroll
      for (int q = 0; q < 3; ++q) atomic_add(&a.forces[3 * (int64_t)i + q], val(fi[q]));
    if (want_ea) {
      if (flags & TERS_ACCUMULATE) a.e_atom[i] += ei;
      else a.e_atom[i] = ei;
    }
    eacc = ei;
    if (a.conf_of && a.partials) {  // batches: per-configuration energy and virial
      atomic_add(&a.partials[(int64_t)cf * 8], eacc);
      for (int k = 0; k < 6; ++k) atomic_add(&a.partials[(int64_t)cf * 8 + 1 + k], wacc[k]);
    }
  }

  // workgroup reduction of energy and virial into this workgroup's record
  if (a.partials && !a.conf_of) {
    __shared__ double s_red[kTBS / kWave][7];
    const int w = threadIdx.x / kWave, lane = lane_id();
    double vals[7] = {eacc, wacc[0], wacc[1], wacc[2], wacc[3], wacc[4], wacc[5]};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const double sum = wave_sum(vals[k]);
      if (lane == 0) s_red[w][k] = sum;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
      double sum = 0.0;
      for (int q = 0; q < kTBS / kWave; ++q) sum += s_red[q][threadIdx.x];
      a.partials[(int64_t)blockIdx.x * 8 + threadIdx.x] = sum;
    }
  }
}

template <class T>
void launch_thread_t(const FwdArgs &a, hipStream_t s) {
  const int nb = thread_blocks(a.n);
  if (nb == 0) return;
  if (a.ntypes == 1) k_force_thread<T, true><<<nb, kTBS, 0, s>>>(a);
  else k_force_thread<T, false><<<nb, kTBS, 0, s>>>(a);
}

}  // namespace

int thread_blocks(int n) { return (n + kTBS - 1) / kTBS; }

void launch_forward_thread(const FwdArgs &a, int precision, hipStream_t s) {
  if (precision == TERS_FP64) launch_thread_t<double>(a, s);
  else launch_thread_t<float>(a, s);
}

}  // namespace ters
