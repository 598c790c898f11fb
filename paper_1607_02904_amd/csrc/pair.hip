// A pair potential on the same machinery: the paper's Algorithm 1 (Section
// II), E = 1/2 sum_i sum_{j in N_i} V(r_ij), here with the truncated
// Lennard-Jones V(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6) for r < r_c.
//
// It runs over the Tersoff context's device neighbour list (rows by cell-order
// position, full list: j in i's row and i in j's).  One thread per atom in
// cell order walks its row and sums the forces on its own atom, so every atom's
// force is written once, without atomics; the energy and virial halves of a
// pair are counted from both ends.  The row is taken eight entries at a time:
// their indices (two 16-byte loads; rows are 16-byte aligned, cap being a
// multiple of 8), then all eight neighbours' positions, then the arithmetic,
// so that a thread has one round of dependent loads per eight neighbours.  The list's radius must be at least r_c
// (entries beyond r_c are skipped, as the filter of Section IV-B does).
// Precision: FP64, or FP32 arithmetic with FP64 displacements, distances and
// accumulators.
#include "ters_device.h"
#include "ters_internal.h"

namespace ters {

namespace {

constexpr int kPBS = 256;

template <class T>
__global__ __launch_bounds__(kPBS) void k_pair_lj(PairArgs p) {
  double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
  const int t = blockIdx.x * kPBS + threadIdx.x;
  if (t < p.n) {
    const int i = p.order[t];
    const ConfDesc &c = p.conf[0];
    const int cnt = min(p.count[t], p.cap);
    const int32_t *row = p.list + (int64_t)t * p.cap;
    double xi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) xi[k] = p.x[3 * (int64_t)i + k];
    const T eps4 = (T)(4.0 * p.eps), eps24 = (T)(24.0 * p.eps), sig2 = (T)(p.sigma * p.sigma);
    double fi[3] = {0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < cnt; s0 += 8) {
      const int4 ja = *reinterpret_cast<const int4 *>(row + s0);
      const int4 jb = *reinterpret_cast<const int4 *>(row + s0 + 4);
      const int jj[8] = {ja.x, ja.y, ja.z, ja.w, jb.x, jb.y, jb.z, jb.w};
      double xj[8][3];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = s0 + u < cnt ? jj[u] : i;  // entries past the row's end: the atom itself
#pragma unroll
        for (int k = 0; k < 3; ++k) xj[u][k] = p.x[3 * (int64_t)j + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
      if (s0 + u >= cnt) break;
      double d[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double dd = xj[u][k] - xi[k];
        d[k] = dd - c.box[k] * rint(dd * c.inv_box[k]);
      }
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (!(r2 < p.rc2)) continue;
      const T ir2 = T(1) / (T)r2;
      const T s2 = sig2 * ir2;
      const T s6 = s2 * s2 * s2;
      const T v = eps4 * (s6 * s6 - s6);
      const double g = (double)(eps24 * (T(2) * s6 * s6 - s6) * ir2);  // -V'(r) / r
      e += 0.5 * (double)v;
      // force on j from the pair is g d; on i, -g d
#pragma unroll
      for (int k = 0; k < 3; ++k) fi[k] -= g * d[k];
      w[0] += 0.5 * g * d[0] * d[0];
      w[1] += 0.5 * g * d[1] * d[1];
      w[2] += 0.5 * g * d[2] * d[2];
      w[3] += 0.5 * g * d[0] * d[1];
      w[4] += 0.5 * g * d[0] * d[2];
      w[5] += 0.5 * g * d[1] * d[2];
      }
    }
    if (p.forces) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (p.accumulate) p.forces[3 * (int64_t)i + k] += fi[k];
        else p.forces[3 * (int64_t)i + k] = fi[k];
      }
    }
  }
  // workgroup sums of energy and virial
  __shared__ double s_red[kPBS / kWave][7];
  const int wv = threadIdx.x / kWave, lane = lane_id();
  double vals[7] = {e, w[0], w[1], w[2], w[3], w[4], w[5]};
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double sum = wave_sum(vals[k]);
    if (lane == 0) s_red[wv][k] = sum;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    double sum = 0.0;
    for (int q = 0; q < kPBS / kWave; ++q) sum += s_red[q][threadIdx.x];
    p.partials[(int64_t)blockIdx.x * 8 + threadIdx.x] = sum;
  }
}

}  // namespace

int pair_blocks(int n) { return (n + kPBS - 1) / kPBS; }

void launch_pair_lj(const PairArgs &p, int precision, hipStream_t s) {
  const int nb = pair_blocks(p.n);
  if (nb == 0) return;
  if (precision == TERS_FP64) k_pair_lj<double><<<nb, kPBS, 0, s>>>(p);
  else k_pair_lj<float><<<nb, kPBS, 0, s>>>(p);
}

}  // namespace ters
