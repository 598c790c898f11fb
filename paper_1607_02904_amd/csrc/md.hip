// Velocity-Verlet integration (metal units) with the list-rebuild test folded
// into the position update, so that one molecular-dynamics step needs no host
// synchronisation and can be captured in a graph.
#include "ters_device.h"
#include "ters_internal.h"

#include <algorithm>

namespace ters {

namespace {

// eV/(Angstrom amu) -> Angstrom/ps^2: elementary charge over atomic mass
// constant (CODATA 2018), 1.602176634e-19 / 1.66053906660e-27 * 1e-4
constexpr double kFtm2v = 9648.533215665328;
constexpr int kBS = 256;

// v += dt/2 F/m; x += dt v (each a fused multiply-add, in every MD kernel,
// so that the rounding does not depend on the compiler's contraction
// choices); F = 0 when the force kernel accumulates into it
// (atomic scatter); flag = 1 if any atom moved more than skin/2 since the last
// list build (FP64, minimum image)
__global__ void k_vv_first(int n, double *__restrict__ x, double *__restrict__ v,
                           double *__restrict__ f, const int32_t *__restrict__ type,
                           const double *__restrict__ mass, int nt, double dt,
                           const double *__restrict__ xref, const ConfDesc *__restrict__ conf,
                           double lim2, int32_t *flag, int zero_f) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool over = false;
  if (i < n) {
    const double s = 0.5 * dt * kFtm2v / mass[species(type, i, nt)];
    const ConfDesc &c = conf[0];
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double vv = fma(s, f[3 * i + a], v[3 * i + a]);
      double xx = fma(dt, vv, x[3 * i + a]);
      v[3 * i + a] = vv;
      x[3 * i + a] = xx;
      if (zero_f) f[3 * i + a] = 0.0;
      double d = xx - xref[3 * i + a];
      d -= c.box[a] * rint(d * c.inv_box[a]);
      r2 += d * d;
    }
    over = !(r2 <= lim2);
  }
  if (__ballot(over) != 0ull && lane_id() == 0) *flag = 1;
}

// v += dt/2 F/m; the rebuild flag is cleared for the next step
__global__ void k_vv_second(int n, double *__restrict__ v, const double *__restrict__ f,
                            const int32_t *__restrict__ type, const double *__restrict__ mass,
                            int nt, double dt, int32_t *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && flag) *flag = 0;
  if (i >= n) return;
  const double s = 0.5 * dt * kFtm2v / mass[species(type, i, nt)];
  v[3 * i + 0] = fma(s, f[3 * i + 0], v[3 * i + 0]);
  v[3 * i + 1] = fma(s, f[3 * i + 1], v[3 * i + 1]);
  v[3 * i + 2] = fma(s, f[3 * i + 2], v[3 * i + 2]);
}


// Energy partials of the force kernel summed by the first kRedBlocks
// workgroups: workgroup b sums slice b (fixed order) into esum[b]; the last of
// them to finish (a counter, no waiting) adds esum[0..kRedBlocks) in index
// order, stores the energy at energy and trace[*step], advances *step and
// resets the counter.  The result does not depend on which workgroup is last.
constexpr int kRedBlocks = 16;
DEV void reduce_energy(const double *__restrict__ partials, int nblocks, double *esum,
                       int32_t *count, double *energy, double *trace, int32_t *step) {
  __shared__ double red[kBS / kWave];
  __shared__ int s_last;
  const int b = blockIdx.x;
  const int per = (nblocks + kRedBlocks - 1) / kRedBlocks;
  const int lo = b * per, hi = min(nblocks, lo + per);
  double acc = 0.0;
  for (int k = lo + (int)threadIdx.x; k < hi; k += kBS) acc += partials[(int64_t)k * 8];
  acc = wave_sum(acc);
  if (lane_id() == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < kBS / kWave; ++w) tot += red[w];
    __hip_atomic_store(&esum[b], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    s_last = atomicAdd(count, 1) == kRedBlocks - 1;
    if (s_last) {
      __threadfence();
      double e = 0.0;
      for (int k = 0; k < kRedBlocks; ++k)
        e += __hip_atomic_load(&esum[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *energy = e;
      trace[*step] = e;
      *step += 1;
      *count = 0;
    }
  }
}

// Owner gather of the forces (FP64 sums, in slot order, of the incoming
// slots of the atom, [soff[i], soff[i + 1]) kept in srange_a[i]), the second half
// kick of this step and, with NEXT, the first half kick, drift and rebuild
// test of the next one (the operations of k_vv_first, in the same order).
// The forces are stored in F only on the last step (without NEXT): the
// steps in between use them in registers.  Thread per atom: every load of
// the atom is issued before the arithmetic and its stores go out back to
// back, so that each thread waits for memory once and writes whole lines at
// a time.  With a trace, the first workgroups also sum the force kernel's
// energy partials.
template <class S, bool NEXT>
__global__ void k_vv_gather_kick_drift(int n, const int2 *__restrict__ srange_a,
                                       const S *__restrict__ fslot,
                                       const double *__restrict__ fown, double *__restrict__ F,
                                       double *__restrict__ v, double *__restrict__ x,
                                       const int32_t *__restrict__ type,
                                       const double *__restrict__ mass, int nt, double dt,
                                       const double *__restrict__ xref,
                                       const ConfDesc *__restrict__ conf, double lim2,
                                       int32_t *flag, const double *__restrict__ partials,
                                       int nblocks, double *esum, int32_t *count, double *energy,
                                       double *trace, int32_t *step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool over = false;
  if (i < n) {
    const int2 rg = srange_a[i];
    double fv[3], vv[3], xx[3], xr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      fv[a] = fown[3 * i + a];
      vv[a] = v[3 * i + a];
      if (NEXT) {
        xx[a] = x[3 * i + a];
        xr[a] = xref[3 * i + a];
      }
    }
    const double s = 0.5 * dt * kFtm2v / mass[species(type, i, nt)];
    sum_slots(fslot, rg.x, rg.y, fv[0], fv[1], fv[2]);
    const ConfDesc &c = conf[0];
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vv[a] = fma(s, fv[a], vv[a]);
      if (NEXT) {
        vv[a] = fma(s, fv[a], vv[a]);
        xx[a] = fma(dt, vv[a], xx[a]);
        double d = xx[a] - xr[a];
        d -= c.box[a] * rint(d * c.inv_box[a]);
        r2 += d * d;
      }
    }
    if (!NEXT) {
#pragma unroll
      for (int a = 0; a < 3; ++a) F[3 * i + a] = fv[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) v[3 * i + a] = vv[a];
    if (NEXT) {
#pragma unroll
      for (int a = 0; a < 3; ++a) x[3 * i + a] = xx[a];
    }
    over = NEXT && !(r2 <= lim2);  // NaN counts as moved
  }
  if (__ballot(over) != 0ull && lane_id() == 0) *flag = 1;
  if (blockIdx.x < kRedBlocks && trace)
    reduce_energy(partials, nblocks, esum, count, energy, trace, step);
}

}  // namespace

void launch_vv_gather_kick_drift(const NList &nl, double *x, double *v, double *F,
                                 const void *fslot, bool slot_f32, const double *fown,
                                 const int32_t *type, const double *mass, int nt, double dt,
                                 int32_t *flag, int do_next, const double *partials, int nblocks,
                                 double *energy, double *trace, int32_t *step, hipStream_t s) {
  const int n = nl.n;
  const int g = std::max((std::max(n, 1) + kBS - 1) / kBS, kRedBlocks);
  const double half = 0.5 * nl.skin;
  double *esum = energy + 8;  // the energy scratch holds 8 + kRedBlocks doubles
  int32_t *count = (int32_t *)(energy + 8 + kRedBlocks);
  auto launch = [&](auto kern, auto slots) {
    kern<<<g, kBS, 0, s>>>(n, nl.srange_a.as<int2>(), slots, fown, F, v, x, type, mass, nt, dt,
                           nl.xref.as<double>(), nl.conf.as<ConfDesc>(), half * half, flag,
                           partials, nblocks, esum, count, energy, trace, step);
  };
  if (slot_f32) {
    const float *fs = (const float *)fslot;
    if (do_next) launch(k_vv_gather_kick_drift<float, true>, fs);
    else launch(k_vv_gather_kick_drift<float, false>, fs);
  } else {
    const double *fs = (const double *)fslot;
    if (do_next) launch(k_vv_gather_kick_drift<double, true>, fs);
    else launch(k_vv_gather_kick_drift<double, false>, fs);
  }
}

void launch_vv_first(int n, double *x, double *v, double *f, const int32_t *type,
                     const double *mass, int nt, double dt, const NList &nl, int32_t *flag, int zero_f,
                     hipStream_t s) {
  if (n <= 0) return;
  const double half = 0.5 * nl.skin;
  k_vv_first<<<(n + kBS - 1) / kBS, kBS, 0, s>>>(n, x, v, f, type, mass, nt, dt, nl.xref.as<double>(),
                                                 nl.conf.as<ConfDesc>(), half * half, flag,
                                                 zero_f);
}

void launch_vv_second(int n, double *v, const double *f, const int32_t *type, const double *mass,
                      int nt, double dt, int32_t *flag, hipStream_t s) {
  k_vv_second<<<(std::max(n, 1) + kBS - 1) / kBS, kBS, 0, s>>>(n, v, f, type, mass, nt, dt, flag);
}

}  // namespace ters
