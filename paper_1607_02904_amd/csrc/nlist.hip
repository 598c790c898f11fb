// Neighbour-list construction by cell binning (the paper, Section II Eq. neigh
// and Section III skin list S_i), for one configuration or a batch of them.
//
//   bin     atom -> cell of side >= r_list in its own configuration's grid,
//           count atoms per cell
//   scan    exclusive prefix sum of the cell counts (cell_start)
//   place   counting-sort the atoms into cells; keep the reference positions
//           of the rebuild check
//   sort    order atoms inside each cell by index (run-to-run determinism)
//           and keep a cell-ordered copy of the positions
//   build   for each atom scan the 27 surrounding cells (1 along an axis that
//           holds fewer than 3 cells) and keep j != i with minimum-image
//           r_ij <= r_list, in a padded row of `cap` entries; hand out each
//           atom's range of incoming force slots (compact, no row padding)
//   reverse for every row entry (i, j), the slot of i's force on j among j's
//           incoming slots
//
// Every kernel takes an optional device flag: when it is non-null and zero the
// kernel returns at once, so a molecular-dynamics step can keep the rebuild
// on the device and be captured in a graph.
#include "ters_device.h"
#include "ters_internal.h"

#include <algorithm>
#include <cmath>

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

// also checks every species against [0, ntypes) when type is given
__global__ void k_bin(int n, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                      const int32_t *__restrict__ conf_of, int32_t *__restrict__ cell_of,
                      int32_t *__restrict__ cell_count, const int32_t *__restrict__ type,
                      int ntypes, const int32_t *cond, uint32_t *err) {
  if (skip(cond)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    bin_one(i, x, conf, conf_of, cell_of, cell_count, err);
    if (type && (unsigned)type[i] >= (unsigned)ntypes) atomicOr(err, kErrBadType);
  }
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

// exclusive block scan of one value per thread (blockDim == BS)
template <int BS>
DEV int block_excl_scan_t(int v, int *total) {
  __shared__ int wsum[BS / kWave];
  int lane = lane_id(), w = threadIdx.x / kWave;
  int inc = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < BS / kWave; ++k) {
    if (k < w) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  if (total) *total = tot;
  return off + inc - v;
}
DEV int block_excl_scan(int v, int *total) { return block_excl_scan_t<kBS>(v, total); }

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
constexpr int kScan1BS = 1024;
constexpr int64_t kScan1Max = 8192;  // above this the two-launch parallel scan wins
__global__ __launch_bounds__(kScan1BS) void k_scan_single(int32_t *__restrict__ counts,
                                                          int32_t *__restrict__ out, int64_t m,
                                                          const int32_t *cond) {
  if (skip(cond)) return;
  const int64_t per = (m + kScan1BS - 1) / kScan1BS;
  const int64_t b = threadIdx.x * per;
  const int64_t e = b + per < m ? b + per : m;
  int s = 0;
#pragma unroll 8
  for (int64_t i = b; i < e; ++i) s += counts[i];
  int tot;
  int off = block_excl_scan_t<kScan1BS>(s, &tot);
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

// order atoms inside each cell by index, record each atom's position in the
// cell order (pos, the inverse of order) and copy the positions in that order
// for the build (xs: FP32, wrapped into the configuration's box; the build's
// distance test allows for that rounding); the counts (used as placement
// cursors) are cleared for
// the next build
__global__ void k_sort_cells(int64_t ncell, const int32_t *__restrict__ cell_start,
                             int32_t *__restrict__ order, int32_t *__restrict__ counts,
                             const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                             const int32_t *__restrict__ conf_of, float4 *__restrict__ xs,
                             int32_t *__restrict__ pos, const int32_t *cond) {
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
    for (int p = b; p < e; ++p) {
      const int i = order[p];
      pos[i] = p;
      const ConfDesc &cf = conf[conf_index(conf_of, i)];
      float w[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double v = x[3 * i + a];
        w[a] = (float)(v - cf.box[a] * floor(v * cf.inv_box[a]));
      }
      xs[p] = make_float4(w[0], w[1], w[2], 0.f);
    }
    counts[c] = 0;
  }
}

DEV int wrap_cell(int q, int nc) { return q < 0 ? q + nc : (q >= nc ? q - nc : q); }

// Seven atoms per wavefront (cell order), nine lanes per atom: lane r of an
// atom takes the row (oz, oy) = (r / 3 - 1, r % 3 - 1) of neighbour cells
// (z-major, the order the rows of the list keep; one offset along an axis with
// fewer than 3 cells).  The cells ox = -1, 0, +1 of a row are consecutive cell
// indices except across the periodic seam, so their atoms form at most two
// runs of the cell-ordered position copy xs.  A first pass counts each lane's
// hits (the first 64 also as a bit mask), an exclusive scan over the atom's
// nine lanes gives every lane its first position in the row, and a second pass
// writes the hits there.
//
// Rows and counts are indexed by cell-order position: row t lists the
// neighbours (atom indices) of the atom at position t, so that the rows of a
// run of atoms that a force wavefront takes are contiguous.
//
// Incoming force slots (min(count, cap) per atom) are laid out without row
// padding: each workgroup numbers its atoms' slots from 0 in processing order
// (loff, packed with the workgroup's id) and leaves its total and its longest
// row in bsum; k_reverse turns these into global offsets.  No atomics.
constexpr int kRows = 9;
constexpr int kAtomsPerWave = kWave / kRows;  // 7
constexpr int kBuildMaxBlocks = 4096;         // bsum holds 2 ints per block
constexpr int kLoffBits = 19;                 // slots numbered within a workgroup
__global__ __launch_bounds__(kBS) void k_build(int n, const float4 *__restrict__ xs,
                                               const ConfDesc *__restrict__ conf,
                                               const int32_t *__restrict__ conf_of,
                                               const int32_t *__restrict__ order,
                                               const int32_t *__restrict__ cell_of,
                                               const int32_t *__restrict__ cell_start,
                                               float rl2, int cap, int32_t *__restrict__ count,
                                               int32_t *__restrict__ list,
                                               int32_t *__restrict__ loff,
                                               int32_t *__restrict__ bsum, const int32_t *cond,
                                               uint32_t *err, int64_t *rebuilds) {
  if (skip(cond)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0 && rebuilds) *rebuilds += 1;
  __shared__ int s_wmax[kBS / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int la = lane / kRows, r = lane - kRows * la;  // atom of the wave (7 = idle lane), row
  const int last = min(kRows * la + kRows - 1, kWave - 1);  // the atom's row-8 lane
  constexpr int kWPB = kBS / kWave;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t ngroups = (n + kAtomsPerWave - 1) / kAtomsPerWave;
  // each workgroup takes one contiguous range of groups of atoms in cell order
  // (so slot numbers, and off, increase along the cell order, and each XCD
  // works on one contiguous range whose neighbour cells share its L2); every
  // lane runs the same number of passes (workgroup scan below)
  const int64_t per_blk = (ngroups + gridDim.x - 1) / gridDim.x;
  const int iters = (int)((per_blk + kWPB - 1) / kWPB);
  const int64_t gend = min((int64_t)(blk + 1) * per_blk, ngroups);
  int worst = 0, run = 0;  // longest row; slots numbered so far in this workgroup
  for (int it = 0; it < iters; ++it) {
    const int64_t g = (int64_t)blk * per_blk + (int64_t)it * kWPB + w;
    const int64_t t64 = g * kAtomsPerWave + la;
    const bool act = g < gend && la < kAtomsPerWave && t64 < n;
    const int t = act ? (int)t64 : -1;
    int i = 0, b0 = 0, e0 = 0, b1 = 0, e1 = 0;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    const ConfDesc *c = conf;
    if (act) {
      i = order[t];
      c = conf + conf_index(conf_of, i);
      const float4 q = xs[t];
      xi = q.x;
      yi = q.y;
      zi = q.z;
      const int lc = cell_of[i] - c->cell_off;
      const int nx = c->nc[0], ny = c->nc[1], nz = c->nc[2];
      const int cx = lc % nx, cy = (lc / nx) % ny, cz = lc / (nx * ny);
      const int oz = r / 3 - 1, oy = r % 3 - 1;
      if ((nz >= 3 || oz == 0) && (ny >= 3 || oy == 0)) {
        const int rc = c->cell_off + (wrap_cell(cz + oz, nz) * ny + wrap_cell(cy + oy, ny)) * nx;
        int c0, c1, c2 = 0, c3 = 0;  // runs [c0, c1) and [c2, c3) of cells
        if (nx < 3) {
          c0 = rc + cx;
          c1 = c0 + 1;
        } else if (cx == 0) {
          c0 = rc + nx - 1;
          c1 = rc + nx;
          c2 = rc;
          c3 = rc + 2;
        } else if (cx == nx - 1) {
          c0 = rc + cx - 1;
          c1 = rc + nx;
          c2 = rc;
          c3 = rc + 1;
        } else {
          c0 = rc + cx - 1;
          c1 = rc + cx + 2;
        }
        b0 = cell_start[c0];
        e0 = cell_start[c1];
        if (c3 > c2) {
          b1 = cell_start[c2];
          e1 = cell_start[c3];
        }
      }
    }
    const int len0 = e0 - b0, len = len0 + (e1 - b1);
    const float bx = (float)c->box[0], by = (float)c->box[1], bz = (float)c->box[2];
    const float ibx = (float)c->inv_box[0], iby = (float)c->inv_box[1], ibz = (float)c->inv_box[2];
    // minimum image in FP32 (the squared radius carries a margin for the
    // rounding, so the list is a superset of the exact one); exactly negated
    // for (j, i), so the list is symmetric
    auto within_at = [&](int p, float px, float py, float pz) {
      float dx = px - xi, dy = py - yi, dz = pz - zi;
      dx -= bx * rintf(dx * ibx);
      dy -= by * rintf(dy * iby);
      dz -= bz * rintf(dz * ibz);
      return p != t && dx * dx + dy * dy + dz * dz <= rl2;
    };
    auto within = [&](int p) {
      const float4 q = xs[p];
      return within_at(p, q.x, q.y, q.z);
    };
    // pass 1: count (the first 64 hits of the runs also as a mask); the
    // positions of four candidates are fetched before any is tested
    int nhit = 0;
    uint64_t mask = 0;
    for (int k0 = 0; k0 < len; k0 += 4) {
      float4 q[4];
      int pp[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = min(k0 + u, len - 1);
        pp[u] = k < len0 ? b0 + k : b1 + (k - len0);
        q[u] = xs[pp[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u;
        if (k < len && within_at(pp[u], q[u].x, q[u].y, q[u].z)) {
          ++nhit;
          if (k < 64) mask |= 1ull << k;
        }
      }
    }
    // exclusive scan over the atom's nine lanes
    int incl = nhit;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int u = __shfl_up(incl, o, kWave);
      if (r >= o) incl += u;
    }
    const int total = __shfl(incl, last, kWave);
    // pass 2: write the hits from the row position of this lane on
    if (act) {
      int32_t *row = list + (int64_t)t * cap;
      int pos = incl - nhit;
      while (mask) {
        const int k = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1ull;
        const int p = k < len0 ? b0 + k : b1 + (k - len0);
        if (pos < cap) row[pos] = order[p];
        ++pos;
      }
      for (int k = 64; k < len; ++k) {  // rows of more than 64 candidates
        const int p = k < len0 ? b0 + k : b1 + (k - len0);
        if (within(p)) {
          if (pos < cap) row[pos] = order[p];
          ++pos;
        }
      }
    }
    const bool owner = act && r == kRows - 1;
    if (owner) {
      count[t] = total;
      if (total > cap) atomicOr(err, kErrNlistOverflow);
    }
    worst = max(worst, owner ? total : 0);
    // slots of this pass, numbered after those of the earlier passes
    int tot;
    const int ex = block_excl_scan(owner ? min(total, cap) : 0, &tot);
    if (owner) loff[t] = (int32_t)(((uint32_t)blk << kLoffBits) | (uint32_t)(run + ex));
    run += tot;
  }
  // the workgroup's slot total and longest row
  int m = worst;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
  if (lane == 0) s_wmax[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int bm = 0;
    for (int k = 0; k < kWPB; ++k) bm = max(bm, s_wmax[k]);
    bsum[2 * blk] = run;
    bsum[2 * blk + 1] = bm;
  }
}

// Global slot offsets and the reverse map (rows, counts and slot records are
// indexed by cell-order position, row entries are atoms).  Every workgroup
// first scans the build's per-workgroup slot totals (nb <= kBuildMaxBlocks,
// in LDS), so the first slot of the atom at position t is off(t) = (slots of
// earlier build workgroups) + (t's number within its own); workgroup 0 also
// stores the longest row.  Then, per position t: soff[t] = off(t) (slots
// increase along the cell order, so t's are [soff[t], soff[t + 1])), and
// rev[t*cap + s] = incoming force slot at atom j = list[t*cap + s] that holds
// the force of t's terms on j: off(pos[j]) + (place of order[t] in row pos[j]).  The list
// is symmetric by construction (r_ij and r_ji are computed from exactly
// negated displacements), so the position exists; a missing one is latched as
// an error.  The rows of 4 neighbours are searched together with 16-byte
// loads (rows start 16-byte aligned: cap is a multiple of 4).
__global__ __launch_bounds__(kBS) void k_reverse(int n, int cap, const int32_t *__restrict__ order,
                                                 const int32_t *__restrict__ pos,
                                                 const int32_t *__restrict__ count,
                                                 const int32_t *__restrict__ list,
                                                 const int32_t *__restrict__ loff,
                                                 const int32_t *__restrict__ bsum, int nb,
                                                 int32_t *__restrict__ soff,
                                                 int32_t *__restrict__ rev,
                                                 int32_t *__restrict__ maxcount, const int32_t *cond,
                                                 uint32_t *err) {
  if (skip(cond)) return;
  __shared__ int s_pre[kBuildMaxBlocks];
  {
    constexpr int kPer = kBuildMaxBlocks / kBS;
    const int b0 = threadIdx.x * kPer;
    int v[kPer];
    int sum = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const bool in = b0 + k < nb;
      v[k] = in ? bsum[2 * (b0 + k)] : 0;
      mx = max(mx, in ? bsum[2 * (b0 + k) + 1] : 0);
      sum += v[k];
    }
    int tot;
    int run = block_excl_scan(sum, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      s_pre[b0 + k] = run;
      run += v[k];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, kWave));
    __shared__ int s_mx[kBS / kWave];
    if (lane_id() == 0) s_mx[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      int m = 0;
      for (int k = 0; k < kBS / kWave; ++k) m = max(m, s_mx[k]);
      *maxcount = m;
    }
  }
  auto offset_of = [&](int a) {
    const uint32_t v = (uint32_t)loff[a];
    return s_pre[v >> kLoffBits] + (int)(v & ((1u << kLoffBits) - 1u));
  };
  for (int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; t < n;
       t += gridDim.x * blockDim.x) {
    const int i = order[t];  // the atom, as it appears in its neighbours' rows
    const int ci = min(count[t], cap);
    const int oi = offset_of(t);
    soff[t] = oi;  // slots of the atom at position t: [soff[t], soff[t + 1])
    if (t == n - 1) soff[n] = oi + ci;
    const int32_t *row_i = list + (int64_t)t * cap;
    for (int s0 = 0; s0 < ci; s0 += 4) {
      int j[4], cj[4], oj[4], found[4];  // j: neighbour's row (its position)
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = s0 + u < ci ? row_i[s0 + u] : i;
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = pos[j[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool live = s0 + u < ci;
        cj[u] = live ? min(count[j[u]], cap) : 0;
        oj[u] = live ? offset_of(j[u]) : 0;
        found[u] = -1;
      }
      for (int k = 0; k < cap; k += 4) {
        int4 v[4];
        bool any = false;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (found[u] < 0 && k < cj[u]) {
            v[u] = *reinterpret_cast<const int4 *>(list + (int64_t)j[u] * cap + k);
            any = true;
          }
        }
        if (!any) break;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (found[u] < 0 && k < cj[u]) {
            if (v[u].x == i) found[u] = k;
            else if (k + 1 < cj[u] && v[u].y == i) found[u] = k + 1;
            else if (k + 2 < cj[u] && v[u].z == i) found[u] = k + 2;
            else if (k + 3 < cj[u] && v[u].w == i) found[u] = k + 3;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (s0 + u < ci) {
          if (found[u] < 0) atomicOr(err, kErrListAsymmetric);
          rev[(int64_t)t * cap + s0 + u] = found[u] < 0 ? -1 : oj[u] + found[u];
        }
      }
    }
  }
}

// owner gather: fixed-order sum of the forces that every neighbour's terms put
// on atom a (its incoming slots [soff[t], soff[t + 1]) for t = pos[a], the
// position of a in cell order; FP32 in the mixed path), plus a's own part, in
// FP64.  Thread per atom: the outputs are written contiguously.
template <class S>
__global__ void k_gather(int n, const int32_t *__restrict__ pos,
                         const int32_t *__restrict__ soff, const S *__restrict__ fslot,
                         const double *__restrict__ fown, double *__restrict__ F, int accumulate) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int t = pos[a];
  const int s0 = soff[t], s1 = soff[t + 1];
  double fx = fown[3 * t], fy = fown[3 * t + 1], fz = fown[3 * t + 2];
  sum_slots(fslot, s0, s1, fx, fy, fz);
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
void nlist_build(NList &nl, const double *x, const int32_t *type, int ntypes, const int32_t *cond,
                 uint32_t *err, hipStream_t s, int64_t *rebuild_counter) {
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
    k_bin<<<grid(n), kBS, 0, s>>>(n, x, conf, conf_of, nl.cell_of.as<int32_t>(), cell_count, type,
                                  ntypes, cond, err);
  if (m <= kScan1Max) {
    k_scan_single<<<1, kScan1BS, 0, s>>>(cell_count, cell_start, m, cond);
  } else {
    const int ntile = grid_for(m, kScanTile);
    k_scan_tiles<<<ntile, kBS, 0, s>>>(cell_count, cell_start, m, nl.scan_tmp.as<int32_t>(), cond);
    k_scan_add<<<ntile, kBS, 0, s>>>(cell_start, m, nl.scan_tmp.as<int32_t>(), cell_count, cond);
  }
  if (n > 0) {
    k_place<<<grid(n), kBS, 0, s>>>(n, x, nl.cell_of.as<int32_t>(), cell_start, cell_count,
                                    nl.order.as<int32_t>(), nl.xref.as<double>(), cond);
    k_sort_cells<<<grid(ncell), kBS, 0, s>>>(ncell, cell_start, nl.order.as<int32_t>(), cell_count,
                                             x, conf, conf_of, nl.xs.as<float4>(),
                                             nl.pos.as<int32_t>(), cond);
    // the list build is latency-bound: a larger grid than the other kernels
    const int64_t groups = (n + kAtomsPerWave - 1) / kAtomsPerWave;
    const int gb = (int)std::min<int64_t>(
        std::max<int64_t>((groups + kBS / kWave - 1) / (kBS / kWave), 1), kBuildMaxBlocks);
    // FP32 distance test on positions wrapped into the box: a coordinate is
    // rounded by at most 2^-24 of the longest side, a squared distance by a
    // few units in the last place; the radius grows by a bound of both, so no
    // pair within r_list is missed (the filter applies the exact cutoffs)
    const double lmax = nl.box_max;
    const double rl = nl.rlist + 8.0 * std::ldexp(lmax, -24) + std::ldexp(nl.rlist, -18);
    k_build<<<gb, kBS, 0, s>>>(n, nl.xs.as<float4>(), conf, conf_of, nl.order.as<int32_t>(),
                               nl.cell_of.as<int32_t>(), cell_start, (float)(rl * rl), nl.cap,
                               nl.count.as<int32_t>(), nl.list.as<int32_t>(), nl.loff.as<int32_t>(),
                               nl.bsum.as<int32_t>(), cond, err, rebuild_counter);
    k_reverse<<<grid(n), kBS, 0, s>>>(n, nl.cap, nl.order.as<int32_t>(), nl.pos.as<int32_t>(),
                                      nl.count.as<int32_t>(),
                                      nl.list.as<int32_t>(), nl.loff.as<int32_t>(),
                                      nl.bsum.as<int32_t>(), gb, nl.soff.as<int32_t>(),
                                      nl.rev.as<int32_t>(), nl.maxcount.as<int32_t>(), cond, err);
  }
}

void launch_gather(const NList &nl, const void *fslot, bool slot_f32, const double *fown,
                   double *F, int accumulate, hipStream_t s) {
  if (nl.n <= 0) return;
  if (slot_f32)
    k_gather<float><<<grid_for(nl.n, kBS), kBS, 0, s>>>(
        nl.n, nl.pos.as<int32_t>(), nl.soff.as<int32_t>(), (const float *)fslot, fown, F,
        accumulate);
  else
    k_gather<double><<<grid_for(nl.n, kBS), kBS, 0, s>>>(
        nl.n, nl.pos.as<int32_t>(), nl.soff.as<int32_t>(), (const double *)fslot, fown, F,
        accumulate);
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
