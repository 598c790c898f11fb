// Neighbour-list construction by cell binning (the paper, Section II Eq. neigh
// and Section III skin list S_i), for one configuration or a batch of them.
//
//   bin     atom -> cell of side >= r_list in its own configuration's grid,
//           count atoms per cell
//   scan    exclusive prefix sum of the cell counts (cell_start)
//   place   counting-sort the atoms into cells; keep a cell-ordered copy of
//           the positions and the reference positions of the rebuild check
//   sort    order atoms inside each cell by index (run-to-run determinism)
//   build   for each atom scan the 27 surrounding cells (1 along an axis that
//           holds fewer than 3 cells) and keep j != i with minimum-image
//           r_ij <= r_list, in a padded row of `cap` entries
//
// Every kernel takes an optional device flag: when it is non-null and zero the
// kernel returns at once, so a molecular-dynamics step can keep the rebuild
// on the device and be captured in a graph.
#include "ters_device.h"
#include "ters_internal.h"

namespace ters {

namespace {

constexpr int kBS = 256;

DEV bool skip(const int32_t *cond) { return cond != nullptr && *cond == 0; }
DEV int conf_index(const int32_t *conf_of, int i) { return conf_of ? conf_of[i] : 0; }

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n, const int32_t *cond) {
  if (skip(cond)) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// zero the cell counts and the longest-row register in one launch
__global__ void k_zero_cells(int32_t *cell_count, int64_t m, int32_t *maxcount, const int32_t *cond) {
  if (skip(cond)) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) *maxcount = 0;
  for (; i < m; i += (int64_t)gridDim.x * blockDim.x) cell_count[i] = 0;
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

DEV void bin_one(int i, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                 const int32_t *__restrict__ conf_of, int32_t *__restrict__ cell_of,
                 int32_t *__restrict__ cell_count, uint32_t *err);

__global__ void k_bin(int n, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                      const int32_t *__restrict__ conf_of, int32_t *__restrict__ cell_of,
                      int32_t *__restrict__ cell_count, int32_t *__restrict__ maxcount,
                      const int32_t *cond, uint32_t *err) {
  if (skip(cond)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *maxcount = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    bin_one(i, x, conf, conf_of, cell_of, cell_count, err);
}

DEV void bin_one(int i, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                 const int32_t *__restrict__ conf_of, int32_t *__restrict__ cell_of,
                 int32_t *__restrict__ cell_count, uint32_t *err) {
  const ConfDesc &c = conf[conf_index(conf_of, i)];
  int q[3];
  bool finite = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double xv = x[3 * i + a];
    finite = finite && isfinite(xv);
    double s = xv * c.inv_box[a];
    s -= floor(s);
    int k = (int)(s * c.nc[a]);
    k = k < 0 ? 0 : (k >= c.nc[a] ? c.nc[a] - 1 : k);
    q[a] = finite ? k : 0;
  }
  if (!finite) atomicOr(err, kErrNotFinite);
  int cell = c.cell_off + (q[2] * c.nc[1] + q[1]) * c.nc[0] + q[0];
  cell_of[i] = cell;
  atomicAdd(&cell_count[cell], 1);
}

// ---- exclusive scan of int32 (tiles of 1024, then tile sums, then add) ----
constexpr int kScanPer = 4;
constexpr int kScanTile = kBS * kScanPer;

DEV int wave_incl_scan(int v) {
  int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive block scan of one value per thread (blockDim == kBS)
DEV int block_excl_scan(int v, int *total) {
  __shared__ int wsum[kBS / kWave];
  int lane = lane_id(), w = threadIdx.x / kWave;
  int inc = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBS / kWave; ++k) {
    if (k < w) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  if (total) *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(kBS) void k_scan_tiles(const int32_t *__restrict__ in,
                                                    int32_t *__restrict__ out, int64_t m,
                                                    int32_t *__restrict__ tile_sum,
                                                    const int32_t *cond) {
  if (skip(cond)) return;
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
  int v[kScanPer];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < m) ? in[base + k] : 0;
    s += v[k];
  }
  int tot;
  int off = block_excl_scan(s, &tot);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < m) out[base + k] = off;
    off += v[k];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// one workgroup per tile: adds the sum of all earlier tiles (summed here, so
// no separate pass over the tile sums) and clears the counts (they become
// the placement cursors)
__global__ __launch_bounds__(kBS) void k_scan_add(int32_t *out, int64_t m,
                                                  const int32_t *tile_sum, int32_t *counts,
                                                  const int32_t *cond) {
  if (skip(cond)) return;
  __shared__ int wsum[kBS / kWave];
  int part = 0;
  for (int t = threadIdx.x; t < (int)blockIdx.x; t += kBS) part += tile_sum[t];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
  if (lane_id() == 0) wsum[threadIdx.x / kWave] = part;
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int w = 0; w < kBS / kWave; ++w) off += wsum[w];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kBS) {
    const int64_t i = base + k;
    if (i < m) {
      out[i] += off;
      counts[i] = 0;
    }
  }
}

// whole exclusive scan in one workgroup (used when the cell count is moderate):
// contiguous chunks per thread, one block scan of the chunk sums; the counts
// are cleared on the way (they become the placement cursors)
constexpr int kScan1Max = 8192;  // above this the three-kernel parallel scan wins
__global__ __launch_bounds__(kBS) void k_scan_single(int32_t *__restrict__ counts,
                                                     int32_t *__restrict__ out, int64_t m,
                                                     const int32_t *cond) {
  if (skip(cond)) return;
  const int64_t per = (m + kBS - 1) / kBS;
  const int64_t b = threadIdx.x * per;
  const int64_t e = b + per < m ? b + per : m;
  int s = 0;
  for (int64_t i = b; i < e; ++i) s += counts[i];
  int tot;
  int off = block_excl_scan(s, &tot);
  for (int64_t i = b; i < e; ++i) {
    int c = counts[i];
    out[i] = off;
    off += c;
    counts[i] = 0;
  }
}

__global__ void k_place(int n, const double *__restrict__ x, const int32_t *__restrict__ cell_of,
                        const int32_t *__restrict__ cell_start, int32_t *__restrict__ cursor,
                        int32_t *__restrict__ order, double *__restrict__ xref,
                        const int32_t *cond) {
  if (skip(cond)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int c = cell_of[i];
    int pos = cell_start[c] + atomicAdd(&cursor[c], 1);
    order[pos] = i;
    xref[3 * i + 0] = x[3 * i + 0];
    xref[3 * i + 1] = x[3 * i + 1];
    xref[3 * i + 2] = x[3 * i + 2];
  }
}

// order atoms inside each cell by index; the counts (used as placement
// cursors) are cleared for the next build
__global__ void k_sort_cells(int64_t ncell, const int32_t *__restrict__ cell_start,
                             int32_t *__restrict__ order, int32_t *__restrict__ counts,
                             const int32_t *cond) {
  if (skip(cond)) return;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * blockDim.x) {
    int b = cell_start[c], e = cell_start[c + 1];
    for (int p = b + 1; p < e; ++p) {
      int v = order[p];
      int q = p - 1;
      while (q >= b && order[q] > v) {
        order[q + 1] = order[q];
        --q;
      }
      order[q + 1] = v;
    }
    counts[c] = 0;
  }
}

__global__ __launch_bounds__(kBS) void k_build(int n, const double *__restrict__ x,
                                               const ConfDesc *__restrict__ conf,
                                               const int32_t *__restrict__ conf_of,
                                               const int32_t *__restrict__ order,
                                               const int32_t *__restrict__ cell_of,
                                               const int32_t *__restrict__ cell_start,
                                               double rl2, int cap, int32_t *__restrict__ count,
                                               int32_t *__restrict__ list,
                                               int32_t *__restrict__ maxcount,
                                               const int32_t *cond, uint32_t *err,
                                               int64_t *rebuilds) {
  if (skip(cond)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0 && rebuilds) *rebuilds += 1;
  int worst = 0;
  // grid-stride over atoms in cell order (each XCD takes one contiguous range
  // per pass, so neighbouring cells share its L2); every lane runs the same
  // number of iterations so the wave reduction below sees all lanes
  const int stride = gridDim.x * blockDim.x;
  const int iters = (n + stride - 1) / stride;
  for (int it = 0; it < iters; ++it) {
  const int t = it * stride + xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (t < n) {
    int i = order[t];
    const ConfDesc &c = conf[conf_index(conf_of, i)];
    double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
    int lc = cell_of[i] - c.cell_off;
    int cx = lc % c.nc[0], cy = (lc / c.nc[0]) % c.nc[1], cz = lc / (c.nc[0] * c.nc[1]);
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = c.nc[a] >= 3 ? -1 : 0;
      hi[a] = c.nc[a] >= 3 ? 1 : 0;
    }
    int32_t *row = list + (int64_t)i * cap;
    for (int oz = lo[2]; oz <= hi[2]; ++oz) {
      int qz = cz + oz;
      qz += (qz < 0) ? c.nc[2] : 0;
      qz -= (qz >= c.nc[2]) ? c.nc[2] : 0;
      for (int oy = lo[1]; oy <= hi[1]; ++oy) {
        int qy = cy + oy;
        qy += (qy < 0) ? c.nc[1] : 0;
        qy -= (qy >= c.nc[1]) ? c.nc[1] : 0;
        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
          int qx = cx + ox;
          qx += (qx < 0) ? c.nc[0] : 0;
          qx -= (qx >= c.nc[0]) ? c.nc[0] : 0;
          int cell = c.cell_off + (qz * c.nc[1] + qy) * c.nc[0] + qx;
          int b = cell_start[cell], e = cell_start[cell + 1];
          for (int p = b; p < e; ++p) {
            int j = order[p];
            if (j == i) continue;
            double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
            dx -= c.box[0] * rint(dx * c.inv_box[0]);
            dy -= c.box[1] * rint(dy * c.inv_box[1]);
            dz -= c.box[2] * rint(dz * c.inv_box[2]);
            if (dx * dx + dy * dy + dz * dz <= rl2) {
              if (cnt < cap) row[cnt] = j;
              ++cnt;
            }
          }
        }
      }
    }
    count[i] = cnt;
  }
  worst = max(worst, cnt);
  }
  // largest row, one atomic per wave
  int m = worst;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
  if (lane_id() == 0 && m > 0) {
    atomicMax(maxcount, m);
    if (m > cap) atomicOr(err, kErrNlistOverflow);
  }
}

// rev[i*cap + s] = slot of i in the row of j = list[i*cap + s].  The list is
// symmetric by construction (r_ij and r_ji are computed from exactly negated
// displacements), so the slot exists; a missing one is latched as an error.
__global__ void k_reverse(int n, int cap, const int32_t *__restrict__ count,
                          const int32_t *__restrict__ list, int32_t *__restrict__ rev,
                          const int32_t *cond, uint32_t *err) {
  if (skip(cond)) return;
  for (int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < n;
       i += gridDim.x * blockDim.x) {
  const int ci = min(count[i], cap);
  for (int s = 0; s < ci; ++s) {
    const int j = list[(int64_t)i * cap + s];
    const int cj = min(count[j], cap);
    int found = -1;
    for (int t = 0; t < cj; ++t)
      if (list[(int64_t)j * cap + t] == i) {
        found = t;
        break;
      }
    if (found < 0) atomicOr(err, kErrListAsymmetric);
    rev[(int64_t)i * cap + s] = found < 0 ? -1 : j * cap + found;
  }
  }
}

// owner gather: fixed-order sum of the forces that every neighbour's terms put
// on atom a (its incoming slots, contiguous), plus a's own part
__global__ void k_gather(int n, int cap, const int32_t *__restrict__ count,
                         const double *__restrict__ fslot, const double *__restrict__ fown,
                         double *__restrict__ F, int accumulate) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double fx = fown[3 * a], fy = fown[3 * a + 1], fz = fown[3 * a + 2];
  const int ca = min(count[a], cap);
  const double *in = fslot + 3 * (int64_t)a * cap;
  for (int s = 0; s < ca; ++s) {
    fx += in[3 * s];
    fy += in[3 * s + 1];
    fz += in[3 * s + 2];
  }
  if (accumulate) {
    F[3 * a] += fx;
    F[3 * a + 1] += fy;
    F[3 * a + 2] += fz;
  } else {
    F[3 * a] = fx;
    F[3 * a + 1] = fy;
    F[3 * a + 2] = fz;
  }
}

__global__ void k_check(int n, const double *__restrict__ x, const double *__restrict__ xref,
                        const ConfDesc *__restrict__ conf, const int32_t *__restrict__ conf_of,
                        double lim2, int32_t *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool over = false;
  if (i < n) {
    const ConfDesc &c = conf[conf_index(conf_of, i)];
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double d = x[3 * i + a] - xref[3 * i + a];
      d -= c.box[a] * rint(d * c.inv_box[a]);
      r2 += d * d;
    }
    over = !(r2 <= lim2);  // NaN counts as moved
  }
  if (__ballot(over) != 0ull && lane_id() == 0) *flag = 1;
}

inline int grid_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, const int32_t *cond, hipStream_t s) {
  if (n <= 0) return;
  int g = grid_for(n, kBS);
  if (g > 4096) g = 4096;
  k_fill_i32<<<g, kBS, 0, s>>>(p, v, n, cond);
}

void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int g = grid_for(n, kBS);
  if (g > 4096) g = 4096;
  k_fill_f64<<<g, kBS, 0, s>>>(p, v, n);
}

// Build the list for the configuration set described by nl (geometry already
// filled in by the caller).  cond: device flag (may be null); when non-null
// and zero every kernel returns immediately.
void nlist_build(NList &nl, const double *x, const int32_t *cond, uint32_t *err, hipStream_t s,
                 int64_t *rebuild_counter) {
  const int n = nl.n;
  const int64_t ncell = nl.ncell;
  int32_t *cell_count = nl.cell_count.as<int32_t>();
  int32_t *cell_start = nl.cell_start.as<int32_t>();
  const ConfDesc *conf = nl.conf.as<ConfDesc>();
  const int32_t *conf_of = nl.nconf > 1 ? nl.conf_of.as<int32_t>() : nullptr;
  const int64_t m = ncell + 1;
  // Cell counts are zero between builds (the sort step clears them); a build
  // started from the host clears them once more, since the buffer may be new.
  if (cond == nullptr) {
    int g = grid_for(m, kBS);
    k_zero_cells<<<g > 4096 ? 4096 : g, kBS, 0, s>>>(cell_count, m, nl.maxcount.as<int32_t>(), cond);
  }
  // grids are capped (grid-stride loops): a skipped rebuild then costs one
  // short dispatch per kernel
  const int gcap = 1024;
  auto grid = [&](int64_t work) {
    int g = grid_for(work, kBS);
    return g < 1 ? 1 : (g > gcap ? gcap : g);
  };
  if (n > 0)
    k_bin<<<grid(n), kBS, 0, s>>>(n, x, conf, conf_of, nl.cell_of.as<int32_t>(), cell_count,
                                  nl.maxcount.as<int32_t>(), cond, err);
  if (m <= kScan1Max) {
    k_scan_single<<<1, kBS, 0, s>>>(cell_count, cell_start, m, cond);
  } else {
    const int ntile = grid_for(m, kScanTile);
    k_scan_tiles<<<ntile, kBS, 0, s>>>(cell_count, cell_start, m, nl.scan_tmp.as<int32_t>(), cond);
    k_scan_add<<<ntile, kBS, 0, s>>>(cell_start, m, nl.scan_tmp.as<int32_t>(), cell_count, cond);
  }
  if (n > 0) {
    k_place<<<grid(n), kBS, 0, s>>>(n, x, nl.cell_of.as<int32_t>(), cell_start, cell_count,
                                    nl.order.as<int32_t>(), nl.xref.as<double>(), cond);
    k_sort_cells<<<grid(ncell), kBS, 0, s>>>(ncell, cell_start, nl.order.as<int32_t>(), cell_count,
                                             cond);
    k_build<<<grid(n), kBS, 0, s>>>(n, x, conf, conf_of, nl.order.as<int32_t>(),
                                             nl.cell_of.as<int32_t>(), cell_start,
                                             nl.rlist * nl.rlist, nl.cap, nl.count.as<int32_t>(),
                                             nl.list.as<int32_t>(), nl.maxcount.as<int32_t>(),
                                             cond, err, rebuild_counter);
    if (nl.rev.p)
      k_reverse<<<grid(n), kBS, 0, s>>>(n, nl.cap, nl.count.as<int32_t>(),
                                                 nl.list.as<int32_t>(), nl.rev.as<int32_t>(), cond,
                                                 err);
  }
}

void launch_gather(const NList &nl, const double *fslot, const double *fown, double *F,
                   int accumulate, hipStream_t s) {
  if (nl.n <= 0) return;
  k_gather<<<grid_for(nl.n, kBS), kBS, 0, s>>>(nl.n, nl.cap, nl.count.as<int32_t>(), fslot, fown,
                                               F, accumulate);
}

void nlist_check(const NList &nl, const double *x, int32_t *flag, hipStream_t s) {
  if (nl.n <= 0) return;
  const double half = 0.5 * nl.skin;
  k_check<<<grid_for(nl.n, kBS), kBS, 0, s>>>(nl.n, x, nl.xref.as<double>(),
                                              nl.conf.as<ConfDesc>(),
                                              nl.nconf > 1 ? nl.conf_of.as<int32_t>() : nullptr,
                                              half * half, flag);
}

}  // namespace ters
