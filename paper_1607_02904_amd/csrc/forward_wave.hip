// Tersoff force kernel, wavefront schedule.
//
// Every wavefront works alone (no workgroup barriers) on a run of atoms in
// cell order.  Its lanes hold one in-cutoff pair (i, j) each; the neighbours
// of an atom occupy consecutive lanes.  The data of neighbour k that the pair
// (i, j) needs in its K loops is read from lane (i, k) with a cross-lane
// permute, so per-pair data stays in registers.  The two K loops follow the
// paper's Algorithms 2 and 3: the first accumulates zeta_ij (and, without the
// parameter gradient, already evaluates dzeta(i,j,k)/dx_j and /dx_k, keeping
// the x_k part of the first few k in LDS as Algorithm 3 stores it), the pair
// term gives dV/dzeta, the second distributes the forces (evaluating the
// three-body term again for k beyond the stored ones, as Algorithm 2 does).
// In the second loop the lanes of one atom walk their neighbours cyclically
// (lane q visits k = q + s mod n in step s), so the force that pair (i, j)
// produces for atom k in step s is exactly what lane (i, k) pulls from lane
// (i, k - s) in that step: every pair slot gathers all contributions of atom
// i's terms to its atom in a fixed order, without atomics in LDS.
//
// The wavefront's list rows are contiguous (rows by cell-order position); the
// filter batches its list, reverse-map and position loads over several
// windows so that they are in flight together.
//
// Scalar types and precision handling are those of the workgroup schedule
// (FP64, mixed FP32 with FP64 displacements/accumulators, dual numbers), plus
// the all-FP32 single mode (SP).
#include "ters_device.h"
#include "ters_internal.h"
#include "ters_math.h"

#include <algorithm>
#include <type_traits>

namespace ters {

namespace {

constexpr int kNMax = 32;  // most in-cutoff neighbours of one atom
constexpr int kAMax = 32;  // most atoms per wavefront
constexpr int kBatch = 4;  // filter windows whose loads are issued together

// Wavefronts per workgroup.  One: the wavefronts share nothing, so each starts
// and retires on its own instead of holding its workgroup's registers until
// the slowest of several has finished.  The parameter-gradient kernels keep
// four, so that their LDS gradient table is flushed with a quarter of the
// atomics.
template <bool PG> constexpr int waves_per_group() { return PG ? 4 : 1; }

// Register budget of the forward kernels: three wavefronts per SIMD for FP64
// (at most 168 VGPRs), four for FP32 (128); the others take what they need.
template <class T, bool PG> struct WavesPerEu { static constexpr int value = 1; };
template <> struct WavesPerEu<double, false> { static constexpr int value = 3; };
template <> struct WavesPerEu<float, false> { static constexpr int value = 4; };

// --- cross-lane reads (ds_bpermute); every lane of the wave must take part --
DEV int lane_read(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
DEV float lane_read(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
DEV double lane_read(double v, int src) {
  int2 u = *reinterpret_cast<int2 *>(&v);
  u.x = __builtin_amdgcn_ds_bpermute(src << 2, u.x);
  u.y = __builtin_amdgcn_ds_bpermute(src << 2, u.y);
  return *reinterpret_cast<double *>(&u);
}
template <class B> DEV Dual<B> lane_read(const Dual<B> &v, int src) {
  return {lane_read(v.v, src), lane_read(v.d, src)};
}

DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SP: the single-precision mode (T = float): positions rounded to FP32 before
// the displacement, no hi/lo compensation (the parameter record passed in has
// zero residuals), and every accumulator in FP32 as well; the per-wavefront
// sums leave the kernel as FP64 partials.
// PERSIST: the persistent form (chunks from work queues, a.items set);
// otherwise one chunk per wavefront.
template <class T, bool NT1, bool PG, bool SP = false, bool PERSIST = false>
__global__ __launch_bounds__(waves_per_group<PG>() * kWave)
__attribute__((amdgpu_waves_per_eu(WavesPerEu<T, PG>::value))) void k_force_wave(FwdArgs a, int A) {
  static_assert(!SP || (std::is_same<T, float>::value && !PG), "single precision: forward FP32 only");
  constexpr int kWPB = waves_per_group<PG>();
  using B = base_t<T>;
  using KP = KParam<B>;
  using AT = typename std::conditional<SP, float, acc_t<T>>::type;
  // energy, virial and own-force accumulators
  using EA = typename std::conditional<SP, float, double>::type;
  auto wide = [](const T &v) -> AT {
    if constexpr (SP) return v;
    else return widen(v);
  };
  // x_j - x_i (in FP32 from FP32-rounded positions in the single mode)
  auto sp_sub = [](double xj, double xi) -> double {
    if constexpr (SP) return (double)((float)xj - (float)xi);
    else return xj - xi;
  };
  // the force of atom i's terms on one neighbour (a sum of a few terms, stored
  // in one slot) is accumulated in the kernel's arithmetic type in the mixed
  // path, in FP64 otherwise; atom forces, energy and virial stay FP64 (FP32 in
  // the single-precision mode)
  using FA = typename std::conditional<std::is_same<T, float>::value, float, AT>::type;
  auto to_fa = [](const auto &v) -> FA { return (FA)v; };
  constexpr bool DUAL = IsDual<T>::value;
  constexpr int NTL = 27;

  // per-wavefront scratch (no sharing between wavefronts)
  __shared__ int s_stage[kWPB][kAMax * kNMax];
  __shared__ unsigned char s_slot[kWPB][kAMax * kNMax];  // list slot of each staged neighbour
  __shared__ unsigned short s_map[kWPB][kBatch * kWave];  // filter: (atom << 8) | slot
  __shared__ KP s_kp[NT1 ? 1 : NTL];
  // parameter gradient with a multi-species table: kGCopies copies of the
  // accumulator (lane l adds to copy l % kGCopies), so that the lanes of a
  // wavefront adding to the entry of one species triple rarely meet on the
  // same LDS word; summed over the copies at the end
  constexpr int kGCopies = 8;
  // (one species: each wavefront's sums, added over the workgroup at the end)
  __shared__ double s_g[PG ? (NT1 ? kWPB * kNField : kGCopies * NTL * kNField) : 1];
  __shared__ double s_red[kWPB][8];
  // Without the parameter gradient the first K loop already evaluates the
  // whole three-body term (value and both gradients); the gradient wrt x_k of
  // the first kKeep steps waits here, per lane, for dV/dzeta, and the one wrt
  // x_j is summed over k.  Later steps (atoms with more neighbours) evaluate
  // the term again in the second loop.
  constexpr bool kOnePass = !PG && !DUAL;
  constexpr int kKeep = 4;
  __shared__ T s_gk[kOnePass ? kWPB : 1][kOnePass ? kKeep : 1][3][kWave];

  const int tid = threadIdx.x;
  // molecular dynamics: the list kernels of this step have read the rebuild
  // flag; it is cleared here and set again by the drift of the next step
  if (a.clear_flag && blockIdx.x == 0 && tid == 0) *a.clear_flag = 0;
  const int w = tid / kWave;
  const int lane = lane_id();
  const int nt = a.ntypes;

  const KP *P;
  if (NT1) {
    P = (const KP *)a.kparam;
  } else if (nt * nt * nt <= NTL) {
    for (int e = tid; e < nt * nt * nt; e += kWPB * kWave) s_kp[e] = ((const KP *)a.kparam)[e];
    P = s_kp;
  } else {
    P = (const KP *)a.kparam;
  }
  const bool grad_in_lds = !NT1 && PG && nt * nt * nt <= NTL;
  if (grad_in_lds)
    for (int e = tid; e < kGCopies * NTL * kNField; e += kWPB * kWave) s_g[e] = 0.0;
  if (!NT1) __syncthreads();  // the only workgroup barrier before the final reductions

  // one species: the record is read once into registers (uniform, scalar
  // loads) instead of from memory inside the K loops
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
  auto add_grad = [&](int ti, int tj, int tk, int field, double v) {
    if (NT1) gacc[field] += v;
    else if (grad_in_lds)
      unsafeAtomicAdd(&s_g[((lane % kGCopies) * NTL + (ti * nt + tj) * nt + tk) * kNField + field], v);
    else atomic_add(&a.pgrad[((ti * nt + tj) * nt + tk) * kNField + field], v);
  };

  EA eacc = 0, wacc[6] = {0, 0, 0, 0, 0, 0};
  const uint32_t flags = a.flags;
  const bool want_f = DUAL ? (a.xgrad != nullptr) : ((flags & TERS_FORCES) && a.forces);
  const bool want_w = !DUAL && (flags & TERS_VIRIAL);
  const bool want_ea = !DUAL && (flags & TERS_PER_ATOM_E) && a.e_atom;
  // mixed path with a two-species table: the energy takes b from an FP64 sum
  // of the FP32 zeta terms, evaluated in FP64 (bond_value_d), when an energy
  // is asked for.  Disordered two-species cells (SiC) cancel their repulsive
  // and attractive parts to a few per cent, so the FP32 bond order's error
  // (a few parts in 1e7 of b) would reach 1e-7 of the energy per atom.  The
  // single-species kernel holds its parameter record in registers, where the
  // FP64 evaluation would push values out to scratch memory; single-species
  // cells keep the FP32 bond order.
  constexpr bool kE64 = std::is_same<T, float>::value && !SP && !NT1;
  const bool want_e = !DUAL && (a.partials != nullptr || want_ea);

  // periodic box: one record for a single system (uniform, read once),
  // the configuration's own record per lane for a batch
  double box0[3], ibox0[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    box0[k] = a.conf[0].box[k];
    ibox0[k] = a.conf[0].inv_box[k];
  }
  const bool one_conf = a.conf_of == nullptr;
  // d <- minimum image of d in configuration cf
  auto min_image = [&](double *d, int cf) {
    if constexpr (SP) {  // FP32 positions, FP32 displacement and image shift
      const ConfDesc &c = a.conf[one_conf ? 0 : cf];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float df = (float)d[k];
        d[k] = (double)(df - (float)c.box[k] * rintf(df * (float)c.inv_box[k]));
      }
      return;
    }
    if (one_conf) {
#pragma unroll
      for (int k = 0; k < 3; ++k) d[k] -= box0[k] * rint(d[k] * ibox0[k]);
    } else {
      const ConfDesc &c = a.conf[cf];
#pragma unroll
      for (int k = 0; k < 3; ++k) d[k] -= c.box[k] * rint(d[k] * c.inv_box[k]);
    }
  };
  const double filt2_0 = ((const double *)a.filt2)[0];

  // Chunks of atoms (consecutive cell-order positions): one per wavefront
  // from its workgroup id, or, in the persistent form (a.items set), items
  // (first position, count) from eight work queues, one per XCD (each a
  // contiguous range of the items, so that neighbouring chunks share an L2).
  // A wavefront takes a.grab items at a time with one atomic add, from its
  // own XCD's queue first and then from the others'; a.grab = 0 instead
  // deals each XCD's range to its wavefronts in turn (no atomics).
  const int home = (int)(blockIdx.x % 8u);
  const int xwave = (int)(blockIdx.x / 8u) * kWPB + w;  // wavefront within its XCD
  const int xwaves = (int)((gridDim.x + 7u - (unsigned)home) / 8u) * kWPB;
  int item = 0, run_end = 0, taken = 0;  // current item, end of the run taken
  auto next_run = [&]() -> bool {  // the next run of items [item, run_end); false when done
    if (a.grab == 0) {  // this XCD's range, every xwaves-th item from xwave on
      const int cand = a.qbound[home] + xwave + taken * xwaves;
      ++taken;
      item = cand;
      run_end = cand + 1;
      return cand < a.qbound[home + 1];
    }
    int v = -1, cnt = 0;
    if (lane == 0) {
      for (int k = 0; k < 8; ++k) {
        const int xq = (home + k) & 7;
        const int len = a.qbound[xq + 1] - a.qbound[xq];
        // a queue already used up is skipped on a plain read: the counters are
        // a few words that every wavefront of the launch comes back to, and
        // adds to one word serialise
        if (len <= 0 ||
            __hip_atomic_load(&a.queue[xq], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len)
          continue;
        const int got = atomicAdd(&a.queue[xq], a.grab);
        if (got < len) {
          v = a.qbound[xq] + got;
          cnt = min(a.grab, len - got);
          break;
        }
      }
    }
    v = __shfl(v, 0, kWave);
    cnt = __shfl(cnt, 0, kWave);
    item = v;
    run_end = v + cnt;
    return v >= 0;
  };
  // chunk of this pass: positions [first, first + na)
  int64_t first = 0;
  int na = 0;
  if constexpr (PERSIST) {
    if (!next_run()) goto done;
    first = a.items[item].x;
    na = a.items[item].y;
  } else {
    first = ((int64_t)xcd_block(blockIdx.x, gridDim.x) * kWPB + w) * A;
    na = (int)max((int64_t)0, min((int64_t)A, (int64_t)a.n - first));
  }
again:
  {
    // chunk atoms: lane `lane` < na holds atom `lane` of the chunk (A <= 64)
    int my_i = 0, my_a = 0, my_t = 0, my_lc = 0, my_cf = 0;  // position, atom
    double my_x[3] = {0.0, 0.0, 0.0};  // position of the lane's atom
    if (lane < na) {
      my_i = (int)(first + lane);  // cell-order position: list row
      my_a = a.order[my_i];        // the atom: per-atom arrays
      my_t = NT1 ? 0 : species(a.type, my_a, a.ntypes);
      my_lc = min(a.count[my_i], a.cap);
      my_cf = a.conf_of ? a.conf_of[my_a] : 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) my_x[k] = a.x[3 * (int64_t)my_a + k];
    }
    // ---- filter: compact the in-cutoff neighbours of every atom of the chunk --
    // The chunk's list entries are numbered without the row padding (atom a's
    // entries follow those of atoms 0..a-1) and visited a wavefront at a time.
    int my_e = my_lc;  // exclusive prefix of the list counts, below
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(my_e, o, kWave);
      if (lane >= o) my_e += u;
    }
    const int total = __shfl(my_e, kWave - 1, kWave);
    my_e -= my_lc;
    int my_cnt = 0;  // in-cutoff neighbours found so far (atom lanes)
    // Windows are taken kBatch at a time: the list entries of all windows of a
    // batch are loaded first, then the neighbours' positions, so that a
    // wavefront has all these loads in flight at once; the tests follow window
    // by window (the staging position of a pass depends on the earlier ones).
    for (int base0 = 0; base0 < total; base0 += kBatch * kWave) {
      // entry -> (atom, slot), written by the atoms' lanes
      {
        const int lo = max(my_e, base0), hi = min(my_e + my_lc, base0 + kBatch * kWave);
        for (int t = lo; t < hi; ++t) s_map[w][t - base0] = (unsigned short)((lane << 8) | (t - my_e));
      }
      wave_sync();
      int cw[kBatch], jw[kBatch], rw[kBatch];  // entry code, neighbour's atom, reverse slot
      double xw[kBatch][3];
      // (no branches around the loads: lanes past the end read entry 0 and
      // atom 0 and discard them, so that the loads issue back to back)
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const bool valid = base0 + u * kWave + lane < total;
        cw[u] = valid ? (int)s_map[w][u * kWave + lane] : -1;
        const int at = valid ? cw[u] >> 8 : 0;
        const int i = lane_read(my_i, at);
        const int64_t e = valid ? (int64_t)i * a.cap + (cw[u] & 0xff) : 0;
        const int jl = a.list[e];
        const int rl = a.rev[e];  // the reverse map exists in both force modes
        jw[u] = valid ? jl : 0;
        rw[u] = (valid && a.fslot) ? rl : -1;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xw[u][k] = a.x[3 * (int64_t)jw[u] + k];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int base = base0 + u * kWave;
        if (base >= total) break;  // uniform
        const bool valid = cw[u] >= 0;
        const int at = valid ? cw[u] >> 8 : 0, s = cw[u] & 0xff;
        const int ti = lane_read(my_t, at), cf = lane_read(my_cf, at);
        const int e_at = lane_read(my_e, at), c_at = lane_read(my_cnt, at);
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = sp_sub(xw[u][k], lane_read(my_x[k], at));
        bool pass = false;
        const int j = jw[u];
        if (valid) {
          min_image(d, cf);
          const int tj = NT1 ? 0 : species(a.type, j, a.ntypes);
          const double f2 = NT1 ? filt2_0 : filt2[ti * nt + tj];
          if constexpr (SP)
            pass = (float)d[0] * (float)d[0] + (float)d[1] * (float)d[1] + (float)d[2] * (float)d[2] <
                   (float)f2;
          else
            pass = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < f2;
          pass = pass || a.no_filter;  // without the filter every entry takes a lane
        }
        const uint64_t m = __ballot(pass);
        // passes of the same atom in lower lanes of this window (e_at <= base + lane)
        const int lo_lane = max(e_at - base, 0);
        const uint64_t below = ((1ull << lane) - 1ull) & ~((1ull << lo_lane) - 1ull);
        const int pos = c_at + __popcll(m & below);
        if (pass) {
          if (pos < kNMax) {
            s_stage[w][at * kNMax + pos] = j;
            s_slot[w][at * kNMax + pos] = (unsigned char)s;
          } else {
            atomicOr(a.err, kErrTooManyInCutoff);
          }
        } else if (valid && rw[u] >= 0) {
          B *fs = (B *)a.fslot + 3 * (int64_t)rw[u];  // slots hold the base type
          fs[0] = B(0);
          fs[1] = B(0);
          fs[2] = B(0);
        }
        const int lo = max(my_e, base), hi = min(my_e + my_lc, base + kWave);
        if (hi > lo) {
          const int l0 = lo - base, l1 = hi - base;  // this atom's lanes [l0, l1)
          const uint64_t mine = (l1 == kWave ? ~0ull : (1ull << l1) - 1ull) & ~((1ull << l0) - 1ull);
          my_cnt += __popcll(m & mine);
        }
      }
      wave_sync();  // s_map is rewritten by the next batch
    }
    const int my_n = lane < na ? min(my_cnt, kNMax) : 0;
    int incl = my_n;  // inclusive prefix of pair counts over the chunk's atoms
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += u;
    }

    // ---- rounds: consecutive atoms whose pairs fill at most one wavefront ------
    int a0 = 0;
    while (a0 < na) {
      const int base = a0 > 0 ? __shfl(incl, a0 - 1, kWave) : 0;
      const uint64_t fits = __ballot(lane >= a0 && lane < na && incl - base <= kWave);
      const int a1 = a0 + __popcll(fits);  // >= a0 + 1: one atom has at most 32 pairs
      const int np = __shfl(incl, a1 - 1, kWave) - base;
      // pair map of this round: an atom's pairs occupy the slots from its start
      // on, so the atom of slot p is the last one starting at or before p; each
      // atom marks its start with (start << 8 | atom + 1) and a prefix maximum
      // over the slots recovers both
      s_map[w][lane] = 0;
      wave_sync();
      if (lane >= a0 && lane < a1 && my_n > 0) {
        const int b = incl - my_n - base;
        s_map[w][b] = (unsigned short)((b << 8) | (lane + 1));
      }
      wave_sync();
      int pm = s_map[w][lane];
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(pm, o, kWave);
        if (lane >= o) pm = max(pm, u);
      }
      wave_sync();  // s_map is rewritten in the next round
      const bool act = lane < np;
      const int at = act ? (pm & 0xff) - 1 : a0;
      const int q = act ? lane - (pm >> 8) : 0;
      const int n_i = lane_read(my_n, at);
      const int seg0 = lane - q;  // first lane of this atom's pairs
      const int i = lane_read(my_i, at), ti = lane_read(my_t, at), cf = lane_read(my_cf, at);
      const int ia = lane_read(my_a, at);  // atom of position i
      const int j = act ? s_stage[w][at * kNMax + q] : ia;  // neighbour's atom
      const int tj = NT1 ? 0 : (act ? species(a.type, j, a.ntypes) : 0);
      // incoming slot at j for this pair's force on j, fetched now so that the
      // load is complete when the force is stored
      const int r_out = a.rev[act ? (int64_t)i * a.cap + s_slot[w][at * kNMax + q] : 0];

      // pair data in registers: the unit vector u = d / r, r, 1/r, f_C, f_C'
      // (what the lanes of the other pairs of the atom read in their K loops)
      T ux, uy, uz, r, ri, fc, dfc;
      B rlo;
      {
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = lane_read(my_x[k], at);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = sp_sub(a.x[3 * (int64_t)j + k], d[k]);
        min_image(d, cf);
        if (!act) {
          d[0] = 1.0;
          d[1] = 0.0;
          d[2] = 0.0;
        }
        T dT[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          dT[k] = Conv<T>::from(d[k], (DUAL && act) ? (a.fbar[3 * j + k] - a.fbar[3 * ia + k]) : 0.0);
        if constexpr (SP) {
          r = t_sqrt(dT[0] * dT[0] + dT[1] * dT[1] + dT[2] * dT[2]);
          ri = rcp(r);
          fcut(param(ti, tj, tj), r, fc, dfc);
          rlo = B(0);
        } else if constexpr (std::is_same<T, float>::value) {
          // mixed: the FP64 distance from the hardware FP32 square root and
          // one Newton step in FP64 (relative error ~1e-14, far below what
          // the FP32 arithmetic downstream resolves)
          const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          const float r32 = __builtin_amdgcn_sqrtf((float)r2);
          const double rr = (double)r32;
          const double r64 = fma(fma(-rr, rr, r2), (double)(0.5f * __builtin_amdgcn_rcpf(r32)), rr);
          r = (float)r64;
          ri = rcp(r);
          fcut64(param(ti, tj, tj), r, r64, fc, dfc);
          rlo = (B)(r64 - (double)r);
        } else {
          r = t_sqrt(dT[0] * dT[0] + dT[1] * dT[1] + dT[2] * dT[2]);
          const double r64 = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          set_val(r, r64);
          ri = rcp(r);
          fcut64(param(ti, tj, tj), r, r64, fc, dfc);
          rlo = (B)(r64 - (double)val(r));
        }
        ux = dT[0] * ri;
        uy = dT[1] * ri;
        uz = dT[2] * ri;
      }
      const T u[3] = {ux, uy, uz};
      // largest neighbour count in this round (uniform loop bound)
      int nmax = n_i;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, kWave));

      // ---- first K loop: zeta_ij -----------------------------------------------
      const KP &pp = param(ti, tj, tj);
      const bool in_pair = act && val(r) < pp.rcut;
      T zeta = Zero<T>::get();
      double zeta64 = 0.0;  // kE64: the same terms summed in FP64
      T gs[3] = {Zero<T>::get(), Zero<T>::get(), Zero<T>::get()};  // sum over kept k of dzeta/dx_j
      for (int s = 1; s < nmax; ++s) {
        const bool keep = kOnePass && s <= kKeep;  // uniform
        const int kq = q + s < n_i ? q + s : q + s - n_i;
        const int src = act && s < n_i ? seg0 + kq : lane;
        const T v[3] = {lane_read(ux, src), lane_read(uy, src), lane_read(uz, src)};
        const T kr = lane_read(r, src), kri = lane_read(ri, src);
        const T kfc = lane_read(fc, src), kdfc = lane_read(dfc, src);
        const int tk = NT1 ? 0 : lane_read(tj, src);
        T gk[3] = {Zero<T>::get(), Zero<T>::get(), Zero<T>::get()};
        if (in_pair && s < n_i) {
          const KP &pk = param(ti, tj, tk);
          if (val(kr) < pk.rcut) {
            T fck = kfc, dfck = kdfc;
            if (!a.cut_consistent) fcut(pk, kr, fck, dfck);
            T zt;
            if (keep) {
              T gj[3], dp[8];
              zt = zeta_term<T, B, false>(pk, r, ri, u, kr, kri, v, fck, dfck, gj, gk, dp);
#pragma unroll
              for (int c = 0; c < 3; ++c) gs[c] += gj[c];
            } else {
              zt = zeta_value<T, B>(pk, r, u, kr, v, fck);
            }
            zeta += zt;
            if constexpr (kE64) zeta64 += (double)zt;
          }
        }
        if (keep) {
#pragma unroll
          for (int c = 0; c < 3; ++c) s_gk[kOnePass ? w : 0][keep ? s - 1 : 0][c][lane] = gk[c];
        }
      }
      // pair term V(i, j, zeta)
      T dzeta = Zero<T>::get();
      FA f0 = Zero<FA>::get(), f1 = Zero<FA>::get(), f2 = Zero<FA>::get();
      EA ev = 0;
      double e_cfa = 0.0;  // kE64: 0.5 f_C f_A and the FP32 b, for the energy's
      float e_b32 = 0.f;   // correction to the FP64 bond order after the K loops
      const double eb = DUAL ? (a.ebar_conf ? a.ebar_conf[cf] : a.ebar) : 1.0;
      if (in_pair) {
        T fr, fa;
        AT fre, fae;  // the same for the energy
        if constexpr (std::is_same<T, float>::value && !SP) {  // mixed: FP64 exponentials
          const double e1 = exp64(pp.A, pp.A_lo, pp.lam1, pp.lam1_lo, r, rlo);
          const double e2 = exp64(pp.Bc, pp.B_lo, pp.lam2, pp.lam2_lo, r, rlo);
          fr = (float)e1;
          fa = -(float)e2;
          fre = e1;
          fae = -e2;
        } else {
          fr = scaled_exp(pp.A, pp.A_lo, pp.lam1, pp.lam1_lo, r, rlo);
          fa = -scaled_exp(pp.Bc, pp.B_lo, pp.lam2, pp.lam2_lo, r, rlo);
          fre = wide(fr);
          fae = wide(fa);
        }
        T b, db, dbb, dbn;
        bond<T, B, PG>(pp, zeta, b, db, dbb, dbn);
        const T vr = fr + b * fa;
        const AT V = wide(fc) * (fre + wide(b) * fae);
        const T dVdr = dfc * vr + fc * (-pp.lam1 * fr - pp.lam2 * b * fa);
        dzeta = B(0.5) * fc * fa * db;
        const T hp = B(0.5) * dVdr;
        f0 = to_fa(wide(-(hp * u[0])));
        f1 = to_fa(wide(-(hp * u[1])));
        f2 = to_fa(wide(-(hp * u[2])));
        if (kOnePass) {
          f0 -= to_fa(wide(dzeta * gs[0]));
          f1 -= to_fa(wide(dzeta * gs[1]));
          f2 -= to_fa(wide(dzeta * gs[2]));
        }
        ev = 0.5 * val(V);
        if constexpr (kE64) {
          e_cfa = 0.5 * wide(fc) * fae;
          e_b32 = b;
        }
        if (PG) {
          const T h = T(B(0.5)) * fc;
          T dp[8];
          dp[0] = h * fr * (B(1) / pp.A);
          dp[1] = -h * r * fr;
          dp[2] = h * b * fa * (B(1) / pp.Bc);
          dp[3] = -h * b * r * fa;
          dp[4] = h * fa * dbb;
          dp[5] = h * fa * dbn;
          dp[6] = -B(0.5) * dfc * vr;
          dp[7] = -B(0.5) * dfc * (r - pp.R) * (B(1) / pp.D) * vr;
#pragma unroll
          for (int f = 0; f < 8; ++f) add_grad(ti, tj, tj, GradSlots::pair[f], out_of(wide(dp[f]), eb));
        }
      }
      // ---- second K loop: dzeta/dx, forces on j (kept) and on k (sent) -----------
      for (int s = 1; s < nmax; ++s) {
        const bool live = act && s < n_i;
        const int kq = q + s < n_i ? q + s : q + s - n_i;      // k this lane treats
        const int bq = q - s >= 0 ? q - s : q - s + n_i;       // lane whose k is me
        const int src = live ? seg0 + kq : lane;
        const int bsrc = live ? seg0 + bq : lane;
        T cx = Zero<T>::get(), cy = Zero<T>::get(), cz = Zero<T>::get();  // force sent to k
        if (kOnePass && s <= kKeep) {  // uniform: the term was evaluated in the first loop
          if (live && in_pair && val(dzeta) != B(0)) {
            const int sk = kOnePass && s <= kKeep ? s - 1 : 0;
            cx = -(dzeta * s_gk[kOnePass ? w : 0][sk][0][lane]);
            cy = -(dzeta * s_gk[kOnePass ? w : 0][sk][1][lane]);
            cz = -(dzeta * s_gk[kOnePass ? w : 0][sk][2][lane]);
          }
        } else {
        const T v[3] = {lane_read(ux, src), lane_read(uy, src), lane_read(uz, src)};
        const T kr = lane_read(r, src), kri = lane_read(ri, src);
        const T kfc = lane_read(fc, src), kdfc = lane_read(dfc, src);
        const int tk = NT1 ? 0 : lane_read(tj, src);
        if (live && in_pair && val(dzeta) != B(0)) {
          const KP &pk = param(ti, tj, tk);
          if (val(kr) < pk.rcut) {
            T fck = kfc, dfck = kdfc;
            if (!a.cut_consistent) fcut(pk, kr, fck, dfck);
            T gj[3], gk[3], dp[8];
            zeta_term<T, B, PG>(pk, r, ri, u, kr, kri, v, fck, dfck, gj, gk, dp);
            f0 -= to_fa(wide(dzeta * gj[0]));
            f1 -= to_fa(wide(dzeta * gj[1]));
            f2 -= to_fa(wide(dzeta * gj[2]));
            cx = -(dzeta * gk[0]);
            cy = -(dzeta * gk[1]);
            cz = -(dzeta * gk[2]);
            if (PG) {
#pragma unroll
              for (int fl = 0; fl < 8; ++fl)
                add_grad(ti, tj, tk, GradSlots::three[fl], out_of(wide(dzeta * dp[fl]), eb));
            }
          }
        }
        }
        // pull the force that lane (i, bq) computed for my atom in this step
        const T rx = lane_read(cx, bsrc), ry = lane_read(cy, bsrc), rz = lane_read(cz, bsrc);
        if (live) {
          f0 += to_fa(wide(rx));
          f1 += to_fa(wide(ry));
          f2 += to_fa(wide(rz));
        }
      }

      // mixed path: the energy's bond order in FP64, evaluated here, where the
      // K loops' registers are free: ev += 0.5 f_C f_A (b64 - b32)
      if constexpr (kE64) {
        if (want_e && in_pair) ev += e_cfa * (bond_value_d(pp, zeta64) - (double)e_b32);
      }

      // ---- f_im complete: virial, scatter to j, own force of i ------------------
      if (!DUAL && a.partials) {
        EA wv[7] = {ev, 0, 0, 0, 0, 0, 0};
        if (act && want_w) {
          const EA ddx = val(wide(ux * r)), ddy = val(wide(uy * r)), ddz = val(wide(uz * r));
          const EA fx = val(f0), fy = val(f1), fz = val(f2);
          wv[1] = ddx * fx;
          wv[2] = ddy * fy;
          wv[3] = ddz * fz;
          wv[4] = ddx * fy;
          wv[5] = ddx * fz;
          wv[6] = ddy * fz;
        }
        if (a.conf_of && !PERSIST) {
          // batches: per-configuration energy and virial; one atomic per value
          // when the round belongs to one configuration, per lane otherwise
          // (the persistent form sums a chunk, which lies in one configuration,
          // and adds it when the chunk is done)
          const int cf0 = __shfl(cf, 0, kWave);
          if (__ballot(act && cf != cf0) == 0ull) {
#pragma unroll
            for (int k = 0; k < 7; ++k) {
              const double sum = wave_sum(wv[k]);
              if (lane == 0) atomic_add(&a.partials[(int64_t)cf0 * 8 + k], (double)sum);
            }
          } else if (act) {
#pragma unroll
            for (int k = 0; k < 7; ++k) atomic_add(&a.partials[(int64_t)cf * 8 + k], wv[k]);
          }
        } else {
          eacc += wv[0];
#pragma unroll
          for (int k = 0; k < 6; ++k) wacc[k] += wv[k + 1];
        }
      }
      // the force this slot hands to j as stored (rounded to the slot type in
      // owner-gather mode); i's own force is minus the sum of these, so the
      // forces of every term cancel exactly in the gathered total
      double o0 = 0.0, o1 = 0.0, o2 = 0.0;
      if (act && want_f) {
        o0 = DUAL ? -out_of(f0, eb) : val(f0);
        o1 = DUAL ? -out_of(f1, eb) : val(f1);
        o2 = DUAL ? -out_of(f2, eb) : val(f2);
        if (a.fslot) {
          o0 = (double)(B)o0;
          o1 = (double)(B)o1;
          o2 = (double)(B)o2;
          if (r_out >= 0) {
            B *fs = (B *)a.fslot + 3 * (int64_t)r_out;
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
      // own force of i (minus the sum of its slot forces; segmented sum over the
      // atom's lanes) and per-atom energy, taken by the atom's first lane
      // (slot values rounded to FP32 travel as FP32: one permute each)
      const bool o32 = std::is_same<B, float>::value && !DUAL && a.fslot != nullptr;
      EA sx = (EA)o0, sy = (EA)o1, sz = (EA)o2, se = ev;
      for (int s = 1; s < nmax && (want_f || want_ea); ++s) {
        const int src = (act && s < n_i) ? seg0 + s : lane;
        EA tx = 0, ty = 0, tz = 0, te = 0;
        if (want_f && o32) {
          tx = (EA)lane_read((float)o0, src);
          ty = (EA)lane_read((float)o1, src);
          tz = (EA)lane_read((float)o2, src);
        } else if (want_f) {
          tx = lane_read((EA)o0, src);
          ty = lane_read((EA)o1, src);
          tz = lane_read((EA)o2, src);
        }
        if (want_ea) te = lane_read(ev, src);
        if (act && q == 0 && s < n_i) {
          sx += tx;
          sy += ty;
          sz += tz;
          se += te;
        }
      }
      if (act && q == 0) {
        if (want_f) {
          if (a.fown) {  // indexed by atom
            double *fo = a.fown + 3 * (int64_t)ia;
            fo[0] = -sx;
            fo[1] = -sy;
            fo[2] = -sz;
          } else {
            double *dst = DUAL ? a.xgrad : a.forces;
            atomic_add(&dst[3 * (int64_t)ia + 0], -sx);
            atomic_add(&dst[3 * (int64_t)ia + 1], -sy);
            atomic_add(&dst[3 * (int64_t)ia + 2], -sz);
          }
        }
        if (want_ea) {
          if (flags & TERS_ACCUMULATE) a.e_atom[ia] += se;
          else a.e_atom[ia] = se;
        }
      }
      // atoms of the chunk without any in-cutoff neighbour: zero per-atom energy
      // and, in owner-gather mode, zero own force
      if (lane >= a0 && lane < a1 && my_n == 0) {
        if (want_ea && !(flags & TERS_ACCUMULATE)) a.e_atom[my_a] = 0.0;
        if (want_f && a.fown) {
          double *fo = a.fown + 3 * (int64_t)my_a;
          fo[0] = 0.0;
          fo[1] = 0.0;
          fo[2] = 0.0;
        }
      }
      wave_sync();
      a0 = a1;
    }
  }
  if constexpr (PERSIST) {  // the next chunk, if any
    if (!DUAL && a.partials && a.conf_of) {
      // the chunk's energy and virial to its configuration: one atomic per value
      const int cfc = a.conf_of[a.order[first]];
      EA vals[7] = {eacc, wacc[0], wacc[1], wacc[2], wacc[3], wacc[4], wacc[5]};
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const double sum = wave_sum(vals[k]);
        if (lane == 0) atomic_add(&a.partials[(int64_t)cfc * 8 + k], sum);
      }
      eacc = 0;
#pragma unroll
      for (int k = 0; k < 6; ++k) wacc[k] = 0;
    }
    ++item;
    if (item >= run_end && !next_run()) goto done;
    first = a.items[item].x;
    na = a.items[item].y;
    goto again;
  }
done:

  // ---- workgroup reductions ------------------------------------------------------
  if (!DUAL && a.partials && !a.conf_of) {
    EA vals[7] = {eacc, wacc[0], wacc[1], wacc[2], wacc[3], wacc[4], wacc[5]};
    if (kWPB == 1) {
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const double sum = wave_sum(vals[k]);  // every lane holds the sum
        if (lane == k) a.partials[(int64_t)blockIdx.x * 8 + k] = sum;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        double sum = wave_sum(vals[k]);
        if (lane == 0) s_red[w][k] = sum;
      }
      __syncthreads();
      if (tid < 7) {
        double sum = 0.0;
        for (int q2 = 0; q2 < kWPB; ++q2) sum += s_red[q2][tid];
        a.partials[(int64_t)blockIdx.x * 8 + tid] = sum;
      }
    }
  }
  if (PG) {
    if (NT1) {
      // the workgroup's sum, one atomic per field: every workgroup adds to the
      // same 14 words, and adds to one word serialise
#pragma unroll
      for (int f = 0; f < kNField; ++f) {
        double sum = wave_sum(gacc[f]);
        if (lane == 0) s_g[w * kNField + f] = sum;
      }
      __syncthreads();
      if (tid < kNField) {
        double sum = 0.0;
        for (int q = 0; q < kWPB; ++q) sum += s_g[q * kNField + tid];
        if (sum != 0.0) atomic_add(&a.pgrad[tid], sum);
      }
    } else if (grad_in_lds) {
      __syncthreads();
      for (int e = tid; e < nt * nt * nt * kNField; e += kWPB * kWave) {
        double sum = 0.0;
        for (int c = 0; c < kGCopies; ++c) sum += s_g[c * NTL * kNField + e];
        if (sum != 0.0) atomic_add(&a.pgrad[e], sum);
      }
    }
  }
}

template <class T, bool PG, bool SP = false>
void launch_wave_t(const FwdArgs &a, int A, hipStream_t s) {
  constexpr int kWPB = waves_per_group<PG>();
  if (A <= 0 || A > kAMax) A = 16;
  const int64_t per_block = (int64_t)kWPB * A;
  const int nb = a.items ? wave_persistent_launch(a.grid, a.nitems, a.grab, PG)
                         : (int)((a.n + per_block - 1) / per_block);
  if (nb <= 0 || a.n == 0) return;
  if (a.items) {
    if (a.ntypes == 1)
      k_force_wave<T, true, PG, SP, true><<<nb, kWPB * kWave, 0, s>>>(a, A);
    else
      k_force_wave<T, false, PG, SP, true><<<nb, kWPB * kWave, 0, s>>>(a, A);
  } else if (a.ntypes == 1) {
    k_force_wave<T, true, PG, SP><<<nb, kWPB * kWave, 0, s>>>(a, A);
  } else {
    k_force_wave<T, false, PG, SP><<<nb, kWPB * kWave, 0, s>>>(a, A);
  }
}

// workgroups of one kernel resident on the whole device at once
template <class T, bool PG>
int resident_grid(bool nt1) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const auto kern = nt1 ? reinterpret_cast<const void *>(&k_force_wave<T, true, PG, false, true>)
                        : reinterpret_cast<const void *>(&k_force_wave<T, false, PG, false, true>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, waves_per_group<PG>() * kWave, 0) !=
      hipSuccess)
    return 0;
  return ncu * std::max(per_cu, 1);
}

}  // namespace

int wave_persistent_grid(int precision, bool adjoint, bool multi_species) {
  const bool nt1 = !multi_species;
  if (adjoint)
    return precision == TERS_FP64 ? resident_grid<Dual<double>, true>(nt1)
                                  : resident_grid<Dual<float>, true>(nt1);
  return precision == TERS_FP64 ? resident_grid<double, false>(nt1) : resident_grid<float, false>(nt1);
}

int wave_persistent_launch(int grid, int nitems, int grab, bool pg) {
  if (nitems <= 0) return grid;
  // no more workgroups than take a run of items each at the start (at least
  // one per XCD queue): the others would only find the queues empty
  const int wpb = pg ? waves_per_group<true>() : waves_per_group<false>();
  const int64_t runs = (nitems + std::max(grab, 1) - 1) / std::max(grab, 1);
  return (int)std::min<int64_t>(grid, std::max<int64_t>(8, (runs + wpb - 1) / wpb));
}

int wave_blocks(int n, int A, bool pg) {
  if (A <= 0 || A > kAMax) A = 16;
  const int64_t per_block = (int64_t)(pg ? waves_per_group<true>() : waves_per_group<false>()) * A;
  return (int)((n + per_block - 1) / per_block);
}

void launch_forward_wave(const FwdArgs &a, int precision, int A, hipStream_t s) {
  const bool pg = (a.flags & TERS_PARAM_GRAD) && a.pgrad;
  if (precision == TERS_SINGLE) {
    launch_wave_t<float, false, true>(a, A, s);  // no parameter gradient in this mode
  } else if (precision == TERS_FP64) {
    if (pg) launch_wave_t<double, true>(a, A, s);
    else launch_wave_t<double, false>(a, A, s);
  } else {
    if (pg) launch_wave_t<float, true>(a, A, s);
    else launch_wave_t<float, false>(a, A, s);
  }
}

void launch_adjoint_wave(const FwdArgs &a, int precision, int A, hipStream_t s) {
  if (precision == TERS_FP64) launch_wave_t<Dual<double>, true>(a, A, s);
  else launch_wave_t<Dual<float>, true>(a, A, s);
}

}  // namespace ters
