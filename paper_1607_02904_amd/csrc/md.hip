// Velocity-Verlet integration (metal units) with the list-rebuild test folded
// into the position update, so that one molecular-dynamics step needs no host
// synchronisation and can be captured in a graph.
#include "ters_device.h"
#include "ters_internal.h"

#include <algorithm>

namespace ters {

namespace {

constexpr double kFtm2v = 9648.533212331;  // eV/(Angstrom amu) -> Angstrom/ps^2
constexpr int kBS = 256;

// v += dt/2 F/m; x += dt v; F = 0 when the force kernel accumulates into it
// (atomic scatter); flag = 1 if any atom moved more than skin/2 since the last
// list build (FP64, minimum image)
__global__ void k_vv_first(int n, double *__restrict__ x, double *__restrict__ v,
                           double *__restrict__ f, const int32_t *__restrict__ type,
                           const double *__restrict__ mass, double dt,
                           const double *__restrict__ xref, const ConfDesc *__restrict__ conf,
                           double lim2, int32_t *flag, int zero_f) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool over = false;
  if (i < n) {
    const double s = 0.5 * dt * kFtm2v / mass[type[i]];
    const ConfDesc &c = conf[0];
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double vv = v[3 * i + a] + s * f[3 * i + a];
      double xx = x[3 * i + a] + dt * vv;
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
                            double dt, int32_t *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && flag) *flag = 0;
  if (i >= n) return;
  const double s = 0.5 * dt * kFtm2v / mass[type[i]];
  v[3 * i + 0] += s * f[3 * i + 0];
  v[3 * i + 1] += s * f[3 * i + 1];
  v[3 * i + 2] += s * f[3 * i + 2];
}


// owner gather of the forces into F (fixed order), then v += dt/2 F/m; the
// rebuild flag is cleared for the next step
__global__ void k_vv_second_gather(int n, int cap, const int32_t *__restrict__ count,
                                   const double *__restrict__ fslot,
                                   const double *__restrict__ fown, double *__restrict__ F,
                                   double *__restrict__ v, const int32_t *__restrict__ type,
                                   const double *__restrict__ mass, double dt, int32_t *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && flag) *flag = 0;
  if (i >= n) return;
  double fx = fown[3 * i], fy = fown[3 * i + 1], fz = fown[3 * i + 2];
  const int ci = min(count[i], cap);
  const double *in = fslot + 3 * (int64_t)i * cap;
  for (int s = 0; s < ci; ++s) {
    fx += in[3 * s];
    fy += in[3 * s + 1];
    fz += in[3 * s + 2];
  }
  F[3 * i] = fx;
  F[3 * i + 1] = fy;
  F[3 * i + 2] = fz;
  const double s = 0.5 * dt * kFtm2v / mass[type[i]];
  v[3 * i + 0] += s * fx;
  v[3 * i + 1] += s * fy;
  v[3 * i + 2] += s * fz;
}

}  // namespace

void launch_vv_second_gather(const NList &nl, double *v, double *F, const double *fslot,
                             const double *fown, const int32_t *type, const double *mass,
                             double dt, int32_t *flag, hipStream_t s) {
  const int n = nl.n;
  k_vv_second_gather<<<(std::max(n, 1) + kBS - 1) / kBS, kBS, 0, s>>>(
      n, nl.cap, nl.count.as<int32_t>(), fslot, fown, F, v, type, mass, dt, flag);
}

void launch_vv_first(int n, double *x, double *v, double *f, const int32_t *type,
                     const double *mass, double dt, const NList &nl, int32_t *flag, int zero_f,
                     hipStream_t s) {
  if (n <= 0) return;
  const double half = 0.5 * nl.skin;
  k_vv_first<<<(n + kBS - 1) / kBS, kBS, 0, s>>>(n, x, v, f, type, mass, dt, nl.xref.as<double>(),
                                                 nl.conf.as<ConfDesc>(), half * half, flag,
                                                 zero_f);
}

void launch_vv_second(int n, double *v, const double *f, const int32_t *type, const double *mass,
                      double dt, int32_t *flag, hipStream_t s) {
  k_vv_second<<<(std::max(n, 1) + kBS - 1) / kBS, kBS, 0, s>>>(n, v, f, type, mass, dt, flag);
}

}  // namespace ters
