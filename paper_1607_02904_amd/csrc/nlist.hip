// Neighbour-list construction by cell binning (the paper, Section II Eq. neigh
// and Section III skin list S_i), for one configuration or a batch of them.
//
//   bin     atom -> cell of side >= r_list in its own configuration's grid,
//           a place in its cell's bucket (or overflow list)
//   cells   one pass over the cells: read each bucket, exclusive prefix sum of
//           the cell sizes (cell_start, one-pass scan), each atom placed at
//           its rank by index among its cell's atoms (run-to-run
//           determinism), with the reference positions of the rebuild check
//           and a cell-ordered copy of the positions
//   build   for each atom scan the 27 surrounding cells (1 along an axis that
//           holds fewer than 3 cells) and keep j != i with minimum-image
//           r_ij <= r_list, in a padded row of `cap` entries
//   slots   each atom's range of incoming force slots (compact, no row
//           padding): a one-pass scan of the row lengths
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
#include <type_traits>

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

// empty every cell (zero counts, empty overflow lists) and zero the
// longest-row register in one launch
__global__ void k_clear_cells(int32_t *cell_count, int32_t *cell_head, int64_t m,
                              int32_t *maxcount, const int32_t *cond) {
  if (skip(cond)) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) *maxcount = 0;
  for (; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    cell_count[i] = 0;
    cell_head[i] = -1;
  }
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

DEV int cell_of_atom(int i, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                     const int32_t *__restrict__ conf_of, uint32_t *err);

// Each atom takes a place in its cell (a counter per cell): the first
// kCellReg atoms of a cell go to the cell's bucket of kCellReg entries, any
// further one is linked into the cell's overflow list (cell_head[c] -> atom ->
// next[atom] -> ... -> -1).  The order the places are taken in does not
// matter: the cell pass ranks each cell's atoms by index.  Also checks every
// species against [0, ntypes) when type is given, and clears the state of
// the current list build's one-pass scans (tickets, tile flags, the longest-row register).
constexpr int kCellReg = 8;
__global__ void k_bin(int n, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                      const int32_t *__restrict__ conf_of, int32_t *__restrict__ cell_count,
                      int32_t *__restrict__ bucket, int32_t *__restrict__ cell_head,
                      int32_t *__restrict__ next, const int32_t *__restrict__ type,
                      int ntypes, unsigned long long *__restrict__ lb, int64_t nlb,
                      int32_t *__restrict__ maxcount, const int32_t *cond, uint32_t *err) {
  if (skip(cond)) return;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nlb;
       k += (int64_t)gridDim.x * blockDim.x)
    lb[k] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) *maxcount = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = cell_of_atom(i, x, conf, conf_of, err);
    const int slot = atomicAdd(&cell_count[c], 1);
    if (slot < kCellReg) bucket[(int64_t)c * kCellReg + slot] = i;
    else next[i] = atomicExch(&cell_head[c], i);
    if (type && (unsigned)type[i] >= (unsigned)ntypes) atomicOr(err, kErrBadType);
  }
}

DEV int cell_of_atom(int i, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
                     const int32_t *__restrict__ conf_of, uint32_t *err) {
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
  return c.cell_off + (q[2] * c.nc[1] + q[1]) * c.nc[0] + q[0];
}

// ---- exclusive scans of int32 ----

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

DEV int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}

// One-pass exclusive scan (decoupled look-back).  Workgroups take tiles of
// kLbTile values in the order of a ticket counter, so every tile a
// workgroup waits for belongs to a workgroup that is already running: the
// waits end whatever the number of resident workgroups.  Each tile publishes
// its sum (status 1) as soon as it is known and, once the sum of all earlier
// tiles is found by walking back over their flags, its inclusive prefix
// (status 2); a flag holds the status in bits 62-63 and the value in the low
// 32 bits.  The flags and the ticket are cleared by the binning pass of the
// same build.
constexpr unsigned long long kLbSum = 1ull << 62, kLbPrefix = 2ull << 62;
constexpr int kScanBS = 1024;              // workgroup size of the one-pass scans (few
                                           // workgroups: one ticket each)
constexpr int kLbPer = 4;                  // values per thread of the slot scan
constexpr int kLbTile = kScanBS * kLbPer;  // values per tile of the slot scan

DEV int scan_ticket(int32_t *ticket) {
  __shared__ int s_tile;
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1);
  __syncthreads();
  return s_tile;
}

// The sum of the tiles before this one, found by the whole workgroup: lane l
// of wavefront w reads the flag of tile top - 64 w - l (BS earlier tiles per
// round, their loads in flight together: a flag read goes out to memory, so
// the walk costs one memory latency per round); the nearest inclusive prefix
// among them ends the walk, and the sums of the tiles in between are added
// to it.  While a tile in the walk has not published, the walk resumes at the
// wavefront window that holds it.  Every thread of the workgroup calls it;
// the result is valid in all of them.
template <int BS>
DEV int scan_lookback(unsigned long long *flags, int tile, int sum) {
  constexpr int kNW = BS / kWave;
  __shared__ int s_first[kNW], s_sum[kNW], s_open[kNW];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  auto put = [&](unsigned long long v) {
    if (threadIdx.x == 0)
      __hip_atomic_store(&flags[tile], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  if (tile == 0) {
    put(kLbPrefix | (unsigned)sum);
    return 0;
  }
  put(kLbSum | (unsigned)sum);
  int excl = 0;
  for (int top = tile - 1;;) {
    const int idx = top - w * kWave - lane;
    // below tile 0: a zero prefix (never reached past tile 0's own prefix)
    const unsigned long long f =
        idx >= 0 ? __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 : kLbPrefix;
    const unsigned long long st = f & (3ull << 62);
    const uint64_t pre = __ballot(st == kLbPrefix), none = __ballot(st == 0ull);
    const int first = pre ? __builtin_ctzll(pre) : kWave;  // nearest prefix of the window
    const uint64_t upto = first >= kWave - 1 ? ~0ull : (2ull << first) - 1ull;
    int v = lane <= first ? (int)(unsigned)(f & 0xffffffffull) : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0) {
      s_first[w] = first;
      s_sum[w] = v;
      s_open[w] = (none & upto) != 0ull;  // a tile of the walk has not published yet
    }
    __syncthreads();
    // windows in order of distance: add the complete ones up to the first
    // prefix; stop at a window that is still open
    int acc = 0, stop = kNW;
    bool found = false;
    for (int u = 0; u < kNW; ++u) {
      if (s_open[u]) {
        stop = u;
        break;
      }
      acc += s_sum[u];
      if (s_first[u] < kWave) {
        found = true;
        break;
      }
    }
    __syncthreads();  // the next round rewrites the window results
    excl += acc;
    if (found) break;
    top -= stop * kWave;
    if (stop < kNW) __builtin_amdgcn_s_sleep(1);  // resume at the open window
  }
  put(kLbPrefix | (unsigned)(excl + sum));
  return excl;
}

// The atom placed at position t of the cell order: its index (order, and pos
// for the inverse), the reference position of the rebuild test (xref), and
// the copy of its position that the build reads (xs: FP32, wrapped into the
// configuration's box, with the atom index in the fourth word; the build's
// distance test allows for that rounding) together with the cell coordinates
// of the position (cell_at, packed by pack_cell).
DEV int pack_cell(int64_t c, const ConfDesc &cf) {  // x | y << 11 | z << 22 in the grid
  const int lc = (int)(c - cf.cell_off), nx = cf.nc[0], ny = cf.nc[1];
  return (lc % nx) | ((lc / nx) % ny) << 11 | (lc / (nx * ny)) << 22;
}
DEV void place_atom(int i, int t, int packed, int32_t *__restrict__ order,
                    int32_t *__restrict__ pos, const double *__restrict__ x,
                    const ConfDesc *__restrict__ conf, const int32_t *__restrict__ conf_of,
                    float4 *__restrict__ xs, int32_t *__restrict__ cell_at,
                    double *__restrict__ xref) {
  order[t] = i;
  pos[i] = t;
  const ConfDesc &cf = conf[conf_index(conf_of, i)];
  float w[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double v = x[3 * i + a];
    xref[3 * i + a] = v;
    w[a] = (float)(v - cf.box[a] * floor(v * cf.inv_box[a]));
  }
  xs[t] = make_float4(w[0], w[1], w[2], __int_as_float(i));
  cell_at[t] = packed;
}

// Counting sort of the atoms into cells, canonical inside each cell, in one
// pass over the cells: a thread per cell, workgroups of kScanBS threads taking
// tiles of kScanBS cells in ticket order.  Each thread reads its cell's count
// and bucket (two 16-byte loads) and empties the cell for the next build; the
// counts are scanned (block scan, then the one-pass look-back over the
// earlier tiles) into cell_start (m = cells + 1 values, the last one the
// total); each atom of the cell goes to position start + (number of the
// cell's atoms with a smaller index), so the order depends only on which
// atoms share a cell.  Cells of up to kCellReg atoms are ranked in registers
// by their thread and staged in LDS by position within the tile, and the
// workgroup then places them a thread per position (every lane busy, however
// unevenly the atoms fill the cells); larger cells are copied to order_u
// (bucket, then overflow list) and ranked by the whole workgroup, a thread
// per atom, so that a crowded cell costs its size per atom, not its square on
// one thread.
constexpr int kStage = 4096;  // positions staged per round
__global__ __launch_bounds__(kScanBS) void k_cells(
    int64_t m, int32_t *__restrict__ cell_count, const int32_t *__restrict__ bucket,
    int32_t *__restrict__ cell_head, const int32_t *__restrict__ next,
    int32_t *__restrict__ cell_start, int32_t *__restrict__ order_u, int32_t *__restrict__ order,
    int32_t *__restrict__ pos, const double *__restrict__ x, const ConfDesc *__restrict__ conf,
    const int32_t *__restrict__ conf_of, float4 *__restrict__ xs, int32_t *__restrict__ cell_at,
    double *__restrict__ xref, int32_t *ticket, unsigned long long *flags, const int32_t *cond) {
  if (skip(cond)) return;
  constexpr int BS = kScanBS;
  __shared__ int s_nq;                        // crowded cells of the tile
  __shared__ int s_q[BS];                     // their threads
  __shared__ int s_b[BS], s_k[BS];            // first position and size, by thread
  __shared__ int s_pack[BS];                  // packed cell coordinates, by thread
  __shared__ int s_at[kStage];                // staged atoms by position in the tile
  __shared__ unsigned short s_cl[kStage];     // and the thread of their cell
  if (threadIdx.x == 0) s_nq = 0;
  const int tile = scan_ticket(ticket);  // (its barrier also publishes s_nq)
  const int64_t c = (int64_t)tile * BS + threadIdx.x;
  const int k = c < m - 1 ? cell_count[c] : 0;
  int a[kCellReg], r[kCellReg];
  {
    static_assert(kCellReg == 8, "two 16-byte loads per bucket");
    int4 q0 = make_int4(-1, -1, -1, -1), q1 = q0;
    if (k > 0) {
      const int4 *bk = reinterpret_cast<const int4 *>(bucket + c * kCellReg);
      q0 = bk[0];
      if (k > 4) q1 = bk[1];
    }
    const int raw[kCellReg] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int u = 0; u < kCellReg; ++u) a[u] = u < k ? raw[u] : -1;
  }
#pragma unroll
  for (int u = 0; u < kCellReg; ++u) {
    r[u] = 0;  // empty registers hold -1, above every index as unsigned
#pragma unroll
    for (int v = 0; v < kCellReg; ++v) r[u] += (unsigned)a[v] < (unsigned)a[u];
  }
  if (k > 0) s_pack[threadIdx.x] = pack_cell(c, conf[conf_index(conf_of, a[0])]);
  int tot;
  const int off = block_excl_scan_t<BS>(k, &tot);
  const int base = scan_lookback<BS>(flags, tile, tot);  // first position of the tile
  const int b = base + off;
  if (c < m) cell_start[c] = b;
  if (c < m - 1) cell_count[c] = 0;
  const bool crowded = k > kCellReg;
  if (crowded) {
#pragma unroll
    for (int u = 0; u < kCellReg; ++u) order_u[b + u] = a[u];
    int j = b + kCellReg;
    for (int q = cell_head[c]; q >= 0; q = next[q]) order_u[j++] = q;
    cell_head[c] = -1;
    s_b[threadIdx.x] = b;
    s_k[threadIdx.x] = k;
    s_q[atomicAdd(&s_nq, 1)] = threadIdx.x;
  }
  for (int lo = 0; lo < tot; lo += kStage) {  // (tot is the same in every thread)
    if (crowded) {  // its positions are left to the workgroup pass below
      for (int rel = max(off - lo, 0); rel < min(off + k - lo, kStage); ++rel) s_at[rel] = -1;
    } else {
#pragma unroll
      for (int u = 0; u < kCellReg; ++u) {
        const int rel = off + r[u] - lo;
        if (u < k && rel >= 0 && rel < kStage) {
          s_at[rel] = a[u];
          s_cl[rel] = (unsigned short)threadIdx.x;
        }
      }
    }
    __syncthreads();
    const int cnt = min(kStage, tot - lo);
    for (int j = threadIdx.x; j < cnt; j += BS) {
      const int i = s_at[j];
      if (i >= 0)
        place_atom(i, base + lo + j, s_pack[s_cl[j]], order, pos, x, conf, conf_of, xs, cell_at,
                   xref);
    }
    __syncthreads();
  }
  // crowded cells (a tile with one has atoms, so the rounds above ordered
  // these reads after the copies to order_u and after every s_nq update)
  const int nq = s_nq;
  for (int e = 0; e < nq; ++e) {
    const int tq = s_q[e];
    const int bq = s_b[tq], kq = s_k[tq], pk = s_pack[tq];
    for (int idx = threadIdx.x; idx < kq; idx += BS) {
      const int i = order_u[bq + idx];
      int rk = 0;
      for (int q = 0; q < kq; ++q) rk += order_u[bq + q] < i;
      place_atom(i, bq + rk, pk, order, pos, x, conf, conf_of, xs, cell_at, xref);
    }
  }
}

// One thread per atom, taken in cell order; workgroups are dealt to the XCDs
// in contiguous ranges of the cell order.  For each row (oz, oy) of neighbour
// cells, walked in z-major order (one offset along an axis with fewer than 3
// cells), the atom's candidates form a near run (the cells ox = -1, 0, +1 of
// its own column that lie on the same side of the periodic seam, consecutive
// in the cell-ordered position copy xs, whose fourth word holds the atom
// index) and, next to the seam, a far run (the cell across it).  Consecutive
// threads share most of their candidates, so the fetches of a wavefront fall
// on a few cache lines.
//
// With at least 3 cells along every axis, the periodic image of a candidate
// is fixed by its cell: the displacement is (x_k - x_i) + s with s = 0 or
// +-box per axis, taken from the row (y, z) and the run (x); with fewer cells
// along some axis (MINIMG: some configuration of the set has such an axis)
// the minimum image is taken per candidate.  Either form is exactly negated
// for the pair (k, i), so the list is symmetric.
//
// Hits are taken in the order (row, near run, far run, position): the
// neighbour's atom index goes to the list row and its position to the plist
// row.  With LDSOUT (list capacity up to 32) the rows are collected in LDS and
// copied out with 16-byte stores (workgroups of BS = 256 threads for a
// capacity of 16, 128 for 32: 32 KB of LDS either way); otherwise each entry
// is stored as found.
//
// Rows and counts are indexed by cell-order position: row t lists the
// neighbours (atom indices) of the atom at position t, so that the rows of a
// run of atoms that a force wavefront takes are contiguous.  The incoming
// force slots are numbered afterwards by a scan of the row lengths (k_slots).
DEV int wrap_cell(int q, int nc) { return q < 0 ? q + nc : (q >= nc ? q - nc : q); }

template <bool LDSOUT, bool MINIMG, int BS>
__global__ __launch_bounds__(BS) void k_build(int n, const float4 *__restrict__ xs,
                                               const int32_t *__restrict__ cell_at,
                                               const ConfDesc *__restrict__ conf,
                                               const int32_t *__restrict__ conf_of,
                                               const int32_t *__restrict__ cell_start,
                                               float rl2, int cap, int32_t *__restrict__ count,
                                               int32_t *__restrict__ list,
                                               int32_t *__restrict__ plist, const int32_t *cond,
                                               uint32_t *err, int64_t *rebuilds) {
  if (skip(cond)) return;
  extern __shared__ int4 obuf4[];  // LDSOUT: [wave][2][64 * cap] int32: atom indices, positions
  if (blockIdx.x == 0 && threadIdx.x == 0 && rebuilds) *rebuilds += 1;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int64_t wbase = (int64_t)xcd_block(blockIdx.x, gridDim.x) * BS + w * kWave;
  const bool act = wbase + lane < n;
  const int t = act ? (int)(wbase + lane) : n - 1;  // idle lanes shadow the last atom, store nothing
  const float4 qi = xs[t];
  const int packed = cell_at[t];
  const ConfDesc &c = conf[conf_index(conf_of, __float_as_int(qi.w))];
  const int nx = c.nc[0], ny = c.nc[1], nz = c.nc[2];
  const int cx = packed & 2047, cy = (packed >> 11) & 2047, cz = packed >> 22;
  const float bx = (float)c.box[0], by = (float)c.box[1], bz = (float)c.box[2];
  const float ibx = (float)c.inv_box[0], iby = (float)c.inv_box[1], ibz = (float)c.inv_box[2];
  const bool fixed = nx >= 3 && ny >= 3 && nz >= 3;  // image fixed by the cell
  const bool kind_a = nx >= 3 && cx == nx - 1, kind_b = nx >= 3 && cx == 0;
  const float sfx = kind_b ? -bx : (kind_a ? bx : 0.f);  // image shift of the far run
  int nb[9], ne[9], fb[9], fe[9];  // near and far runs of positions
  float sy[9], sz[9];              // image shifts of the row
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int oz = r / 3 - 1, oy = r % 3 - 1;
    nb[r] = ne[r] = fb[r] = fe[r] = 0;
    sy[r] = cy + oy < 0 ? -by : (cy + oy >= ny ? by : 0.f);
    sz[r] = cz + oz < 0 ? -bz : (cz + oz >= nz ? bz : 0.f);
    if ((nz >= 3 || oz == 0) && (ny >= 3 || oy == 0)) {
      const int rc = c.cell_off + (wrap_cell(cz + oz, nz) * ny + wrap_cell(cy + oy, ny)) * nx;
      int c0, c1, c2 = 0, c3 = 0;  // near cells [c0, c1), far cells [c2, c3)
      if (nx < 3) {
        c0 = rc + cx;
        c1 = c0 + 1;
      } else if (kind_b) {
        c0 = rc;
        c1 = rc + 2;
        c2 = rc + nx - 1;
        c3 = rc + nx;
      } else if (kind_a) {
        c0 = rc + cx - 1;
        c1 = rc + nx;
        c2 = rc;
        c3 = rc + 1;
      } else {
        c0 = rc + cx - 1;
        c1 = rc + cx + 2;
      }
      nb[r] = cell_start[c0];
      ne[r] = cell_start[c1];
      if (c3 > c2) {
        fb[r] = cell_start[c2];
        fe[r] = cell_start[c3];
      }
    }
  }

  int32_t *oid = reinterpret_cast<int32_t *>(obuf4) + (size_t)w * 2 * kWave * cap;
  int32_t *opos = oid + kWave * cap;
  int32_t *row = list + (int64_t)t * cap;
  int32_t *prow = plist + (int64_t)t * cap;
  int cnt = 0;
  // candidates are fetched U at a time from xs[k0 ..]: xs carries U - 1
  // padding entries past n, and entries at or past the run's end are not
  // taken.  Image shifts that are zero are not added (adding zero changes no
  // distance, so the pair (k, i) still sees the negated displacement): the
  // x shift exists only on far runs, the y and z shifts only in the rows of a
  // wavefront that touch the box's faces.  Only the near run of the middle
  // row holds the atom itself.
  constexpr int U = 4;
  // MI: the minimum image per candidate; a wavefront whose atoms all lie in
  // configurations of at least three cells per axis takes the cell's fixed
  // image instead (the same arithmetic as the MI form gives them)
  auto walk = [&](auto far_c, auto yz_c, auto mid_c, auto mi_c, int r, int b, int e)
                  __attribute__((always_inline)) {
    constexpr bool FAR = decltype(far_c)::value, YZ = decltype(yz_c)::value;
    constexpr bool MID = decltype(mid_c)::value, MI = decltype(mi_c)::value;
    for (int k0 = b; k0 < e; k0 += U) {
      float4 q[U];
      const float4 *src = xs + k0;
#pragma unroll
      for (int u = 0; u < U; ++u) q[u] = src[u];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float dx = q[u].x - qi.x, dy = q[u].y - qi.y, dz = q[u].z - qi.z;
        if (!MI) {
          if (FAR) dx += sfx;
          if (YZ) {
            dy += sy[r];
            dz += sz[r];
          }
        } else {  // the form is a property of the configuration, the same for (k, i)
          dx = fixed ? dx + (FAR ? sfx : 0.f) : dx - bx * rintf(dx * ibx);
          dy = fixed ? dy + sy[r] : dy - by * rintf(dy * iby);
          dz = fixed ? dz + sz[r] : dz - bz * rintf(dz * ibz);
        }
        const int p = k0 + u;
        if (p < e && (!MID || p != t) && dx * dx + dy * dy + dz * dz <= rl2) {
          if (LDSOUT && cnt < cap) {
            oid[lane * cap + cnt] = __float_as_int(q[u].w);
            opos[lane * cap + cnt] = p;
          } else if (!LDSOUT && act && cnt < cap) {
            row[cnt] = __float_as_int(q[u].w);
            prow[cnt] = p;
          }
          ++cnt;
        }
      }
    }
  };
  using TT = std::true_type;
  using FF = std::false_type;
  auto walk_rows = [&](auto mi_c) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const bool yz = __ballot(sy[r] != 0.f || sz[r] != 0.f) != 0ull;  // uniform
      if (r == 4) {
        if (yz) walk(FF(), TT(), TT(), mi_c, r, nb[r], ne[r]);
        else walk(FF(), FF(), TT(), mi_c, r, nb[r], ne[r]);
      } else {
        if (yz) walk(FF(), TT(), FF(), mi_c, r, nb[r], ne[r]);
        else walk(FF(), FF(), FF(), mi_c, r, nb[r], ne[r]);
      }
      if (__ballot(fe[r] > fb[r]) != 0ull) walk(TT(), TT(), FF(), mi_c, r, fb[r], fe[r]);
    }
  };
  if constexpr (!MINIMG) {
    walk_rows(FF());
  } else if (__ballot(act && !fixed) == 0ull) {  // uniform: every atom's image is fixed
    walk_rows(FF());
  } else {
    walk_rows(TT());
  }
  if (act) {
    count[t] = cnt;
    if (cnt > cap) atomicOr(err, kErrNlistOverflow);
  }
  if (!LDSOUT) return;
  __syncthreads();
  // copy the wavefront's rows out: rows wbase .. wbase + 63 are contiguous
  const int rows = (int)min<int64_t>(kWave, n - wbase);
  const int q4 = cap / 4;  // 16-byte pieces per row
  int4 *gl = reinterpret_cast<int4 *>(list + wbase * cap);
  int4 *gp = reinterpret_cast<int4 *>(plist + wbase * cap);
  const int4 *li = reinterpret_cast<const int4 *>(oid);
  const int4 *lp = reinterpret_cast<const int4 *>(opos);
  for (int k = lane; k < rows * q4; k += kWave) {
    gl[k] = li[k];
    gp[k] = lp[k];
  }
}

// Incoming force slots, numbered along the atom order without row padding:
// atom a owns [soff[a], soff[a + 1]) with soff[a] = sum of min(count, cap)
// over the rows of earlier atoms, so that the gathers (a thread per atom) read
// the slots of consecutive atoms from consecutive addresses; the pair
// (soff[a], soff[a + 1]) is also kept as one 8-byte word per atom (srange_a,
// for the gathers) and per cell-order position (srange, for the reverse map).
// One pass (the one-pass scan above) over atoms 0 .. n, atom n adding zero so
// that soff[n] is the total; a row longer than cap raises maxcount to its
// length (only such rows touch it, so the register is not contended).
__global__ __launch_bounds__(kScanBS) void k_slots(const int32_t *__restrict__ count, int cap, int n,
                                               const int32_t *__restrict__ pos,
                                               int32_t *__restrict__ soff, int2 *__restrict__ srange,
                                               int2 *__restrict__ srange_a,
                                               int32_t *__restrict__ maxcount, int32_t *ticket,
                                               unsigned long long *flags, const int32_t *cond) {
  if (skip(cond)) return;
  const int tile = scan_ticket(ticket);
  const int64_t base = (int64_t)tile * kLbTile + threadIdx.x * kLbPer;
  int v[kLbPer], p[kLbPer];
  int sum = 0, mx = 0;
#pragma unroll
  for (int k = 0; k < kLbPer; ++k) p[k] = (base + k < n) ? pos[base + k] : 0;
#pragma unroll
  for (int k = 0; k < kLbPer; ++k) {  // atom n closes the scan with a zero
    const int c = (base + k < n) ? count[p[k]] : 0;
    mx = max(mx, c);
    v[k] = min(c, cap);
    sum += v[k];
  }
  int tot;
  int off = block_excl_scan_t<kScanBS>(sum, &tot);
  off += scan_lookback<kScanBS>(flags, tile, tot);
  mx = wave_max_i(mx);
  if (lane_id() == 0 && mx > cap) atomicMax(maxcount, mx);  // only rows that overflowed
#pragma unroll
  for (int k = 0; k < kLbPer; ++k) {
    const int64_t i = base + k;
    if (i <= n) soff[i] = off;
    if (i < n) {
      const int2 rg = make_int2(off, off + v[k]);
      srange_a[i] = rg;
      srange[p[k]] = rg;
    }
    off += v[k];
  }
}

// The reverse map: for row entry (t, s) with neighbour j = list[t*cap + s] at
// position p = plist[t*cap + s], rev[t*cap + s] = the incoming force slot at j
// that holds the force of t's terms on j: soff[p] + (place of the atom at t in
// row p).  The list is symmetric by construction (r_ij and r_ji are computed
// from exactly negated displacements), so the place exists; a missing one is
// latched as an error.  One thread per row, eight entries at a time: their
// positions and slot ranges, then the entries of each of their rows four at a
// time (16-byte loads; rows start 16-byte aligned, cap being a multiple of 8),
// the loads of all eight rows in flight together.
__global__ __launch_bounds__(kBS) void k_reverse(int n, int cap, const float4 *__restrict__ xs,
                                                 const int2 *__restrict__ srange,
                                                 const int32_t *__restrict__ list,
                                                 const int32_t *__restrict__ plist,
                                                 int32_t *__restrict__ rev, const int32_t *cond,
                                                 uint32_t *err) {
  if (skip(cond)) return;
  const int64_t t64 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBS + threadIdx.x;
  if (t64 >= n) return;
  const int t = (int)t64;
  const int i = __float_as_int(xs[t].w);  // the atom, as it appears in its neighbours' rows
  const int2 rt = srange[t];
  const int ci = rt.y - rt.x;
  const int32_t *prow = plist + (int64_t)t * cap;
  int32_t *rrow = rev + (int64_t)t * cap;
  for (int s0 = 0; s0 < ci; s0 += 8) {
    int p[8], cj[8], oj[8], found[8];
    const int4 pa = *reinterpret_cast<const int4 *>(prow + s0);
    const int4 pb = *reinterpret_cast<const int4 *>(prow + s0 + 4);
    p[0] = pa.x, p[1] = pa.y, p[2] = pa.z, p[3] = pa.w;
    p[4] = pb.x, p[5] = pb.y, p[6] = pb.z, p[7] = pb.w;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool live = s0 + u < ci;
      if (!live) p[u] = t;  // entries past the row's end are never written
      const int2 rg = srange[p[u]];
      oj[u] = rg.x;
      cj[u] = live ? rg.y - rg.x : 0;
      found[u] = -1;
    }
    // four entries of each searched row at a time; the next four only for
    // the entries not found yet
    for (int k = 0; k < cap; k += 4) {
      int4 v[8];
      bool any = false;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (found[u] < 0 && k < cj[u]) {
          v[u] = *reinterpret_cast<const int4 *>(list + (int64_t)p[u] * cap + k);
          any = true;
        }
      }
      if (!any) break;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (found[u] < 0 && k < cj[u]) {
          if (v[u].x == i) found[u] = k;
          else if (k + 1 < cj[u] && v[u].y == i) found[u] = k + 1;
          else if (k + 2 < cj[u] && v[u].z == i) found[u] = k + 2;
          else if (k + 3 < cj[u] && v[u].w == i) found[u] = k + 3;
        }
      }
    }
    int o[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (s0 + u < ci && found[u] < 0) atomicOr(err, kErrListAsymmetric);
      o[u] = found[u] < 0 ? -1 : oj[u] + found[u];
    }
    // entries past the row's end (set to -1 or junk) are never read
    *reinterpret_cast<int4 *>(rrow + s0) = make_int4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<int4 *>(rrow + s0 + 4) = make_int4(o[4], o[5], o[6], o[7]);
  }
}

// owner gather: fixed-order sum of the forces that every neighbour's terms put
// on atom a (its incoming slots [soff[a], soff[a + 1]); FP32 in the mixed
// path), plus a's own part, in FP64.  Thread per atom: slots, own forces and
// outputs of consecutive atoms are contiguous.
template <class S>
__global__ void k_gather(int n, const int2 *__restrict__ srange_a, const S *__restrict__ fslot,
                         const double *__restrict__ fown, double *__restrict__ F, int accumulate) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int2 rg = srange_a[a];
  double fx = fown[3 * a], fy = fown[3 * a + 1], fz = fown[3 * a + 2];
  sum_slots(fslot, rg.x, rg.y, fx, fy, fz);
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

// flag <- 1 when an atom moved farther than sqrt(lim2) (minimum image) since
// the last build; with type set also when a species lies outside [0, ntypes),
// and with maxcount set when the last build overflowed a row (so that the
// build runs again and reports it)
__global__ void k_check(int n, const double *__restrict__ x, const double *__restrict__ xref,
                        const ConfDesc *__restrict__ conf, const int32_t *__restrict__ conf_of,
                        double lim2, int32_t *flag, const int32_t *__restrict__ type, int ntypes,
                        const int32_t *maxcount) {
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
    if (type && (unsigned)type[i] >= (unsigned)ntypes) over = true;
  }
  if (maxcount && i == 0 && *maxcount > 0) over = true;
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
  int32_t *cell_head = nl.cell_head.as<int32_t>();
  int32_t *bucket = nl.cell_bucket.as<int32_t>();
  int32_t *cell_start = nl.cell_start.as<int32_t>();
  const ConfDesc *conf = nl.conf.as<ConfDesc>();
  const int32_t *conf_of = nl.nconf > 1 ? nl.conf_of.as<int32_t>() : nullptr;
  const int64_t m = ncell + 1;
  // Cells are empty between builds (the cell pass empties them); a build
  // started from the host empties them once more, since the buffers may be new.
  if (cond == nullptr) {
    int g = grid_for(m, kBS);
    k_clear_cells<<<g > 4096 ? 4096 : g, kBS, 0, s>>>(cell_count, cell_head, m,
                                                       nl.maxcount.as<int32_t>(), cond);
  }
  // grids are capped (grid-stride loops): a skipped rebuild then costs one
  // short dispatch per kernel
  const int gcap = 1024;
  auto grid = [&](int64_t work) {
    int g = grid_for(work, kBS);
    return g < 1 ? 1 : (g > gcap ? gcap : g);
  };
  if (n <= 0) return;  // nothing reads the cells of an empty set
  // one-pass scan state: two tickets, then the tile flags of the cell pass and
  // of the slot scan
  static_assert(kCellTile == kScanBS && kSlotTile == kLbTile, "tile sizes of the one-pass scans");
  const int ntc = grid_for(m, kCellTile), nts = grid_for((int64_t)n + 1, kSlotTile);
  unsigned long long *lb = nl.lbstate.as<unsigned long long>();
  int32_t *tickets = reinterpret_cast<int32_t *>(lb);
  static_assert(kCellReg == kCellBucket, "bucket size");
  k_bin<<<grid(n), kBS, 0, s>>>(n, x, conf, conf_of, cell_count, bucket, cell_head,
                                nl.cell_next.as<int32_t>(), type, ntypes, lb, lb_words(m, n),
                                nl.maxcount.as<int32_t>(), cond, err);
  k_cells<<<ntc, kScanBS, 0, s>>>(m, cell_count, bucket, cell_head, nl.cell_next.as<int32_t>(), cell_start,
                              nl.order_u.as<int32_t>(), nl.order.as<int32_t>(),
                              nl.pos.as<int32_t>(), x, conf, conf_of, nl.xs.as<float4>(),
                              nl.cell_at.as<int32_t>(), nl.xref.as<double>(), tickets, lb + 1,
                              cond);
  {
    // FP32 distance test on positions wrapped into the box: a coordinate is
    // rounded by at most 2^-24 of the longest side, a squared distance by a
    // few units in the last place; the radius grows by a bound of both, so no
    // pair within r_list is missed (the filter applies the exact cutoffs)
    const double lmax = nl.box_max;
    const double rl = nl.rlist + 8.0 * std::ldexp(lmax, -24) + std::ldexp(nl.rlist, -18);
    const int gt = grid_for(n, kBS);  // one thread per atom
    // the workgroup size of the launch is the kernel's BS: rows collected in
    // LDS (32 KB per workgroup) with 256 threads up to a capacity of 16 and
    // 128 up to 32; beyond that stored as found, 256 threads
    const bool minimg = nl.small_axis;
    void (*kern)(int, const float4 *, const int32_t *, const ConfDesc *, const int32_t *,
                 const int32_t *, float, int, int32_t *, int32_t *, int32_t *, const int32_t *,
                 uint32_t *, int64_t *);
    int bs;
    size_t obytes;
    if (nl.cap <= 16) {
      kern = minimg ? k_build<true, true, kBS> : k_build<true, false, kBS>;
      bs = kBS;
      obytes = sizeof(int32_t) * 2 * kBS * nl.cap;
    } else if (nl.cap <= 32) {
      kern = minimg ? k_build<true, true, kBS / 2> : k_build<true, false, kBS / 2>;
      bs = kBS / 2;
      obytes = sizeof(int32_t) * 2 * (kBS / 2) * nl.cap;
    } else {
      kern = minimg ? k_build<false, true, kBS> : k_build<false, false, kBS>;
      bs = kBS;
      obytes = 0;
    }
    kern<<<grid_for(n, bs), bs, obytes, s>>>(n, nl.xs.as<float4>(), nl.cell_at.as<int32_t>(), conf, conf_of,
                                 cell_start, (float)(rl * rl), nl.cap, nl.count.as<int32_t>(),
                                 nl.list.as<int32_t>(), nl.plist.as<int32_t>(), cond, err,
                                 rebuild_counter);
    k_slots<<<nts, kScanBS, 0, s>>>(nl.count.as<int32_t>(), nl.cap, n, nl.pos.as<int32_t>(),
                                nl.soff.as<int32_t>(), nl.srange.as<int2>(),
                                nl.srange_a.as<int2>(), nl.maxcount.as<int32_t>(), tickets + 1,
                                lb + 1 + ntc, cond);
    k_reverse<<<gt, kBS, 0, s>>>(n, nl.cap, nl.xs.as<float4>(), nl.srange.as<int2>(),
                                 nl.list.as<int32_t>(), nl.plist.as<int32_t>(),
                                 nl.rev.as<int32_t>(), cond, err);
  }
}

void launch_gather(const NList &nl, const void *fslot, bool slot_f32, const double *fown,
                   double *F, int accumulate, hipStream_t s) {
  if (nl.n <= 0) return;
  if (slot_f32)
    k_gather<float><<<grid_for(nl.n, kBS), kBS, 0, s>>>(
        nl.n, nl.srange_a.as<int2>(), (const float *)fslot, fown, F,
        accumulate);
  else
    k_gather<double><<<grid_for(nl.n, kBS), kBS, 0, s>>>(
        nl.n, nl.srange_a.as<int2>(), (const double *)fslot, fown, F,
        accumulate);
}

void nlist_check(const NList &nl, const double *x, int32_t *flag, hipStream_t s) {
  if (nl.n <= 0) return;
  const double half = 0.5 * nl.skin;
  k_check<<<grid_for(nl.n, kBS), kBS, 0, s>>>(nl.n, x, nl.xref.as<double>(),
                                              nl.conf.as<ConfDesc>(),
                                              nl.nconf > 1 ? nl.conf_of.as<int32_t>() : nullptr,
                                              half * half, flag, nullptr, 0, nullptr);
}

void nlist_check_moved(const NList &nl, const double *x, const int32_t *type, int ntypes,
                       int32_t *flag, hipStream_t s) {
  if (nl.n <= 0) return;
  k_check<<<grid_for(nl.n, kBS), kBS, 0, s>>>(nl.n, x, nl.xref.as<double>(),
                                              nl.conf.as<ConfDesc>(),
                                              nl.nconf > 1 ? nl.conf_of.as<int32_t>() : nullptr,
                                              0.0, flag, type, ntypes, nl.maxcount.as<int32_t>());
}

}  // namespace ters
